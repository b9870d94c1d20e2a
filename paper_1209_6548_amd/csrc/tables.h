// Host-side constants: velocity sets, per-problem parameters, fast division.
#pragma once

#include <stdint.h>

#include <vector>

#include "params.h"

namespace esbgk {

struct HostLattice {
  int velset = 0, D = 0, Q = 0, N = 0, P = 0;
  double r = 0;
  std::vector<int> e;     // Q x 3
  std::vector<double> w;  // Q
};

// Derived once per process; null if the derivation failed.
const HostLattice* host_lattice(int velset);

// The n-point Gauss-Hermite product set of the paper's own scheme (n = 4, 6
// or 8: D2Q16, D2Q36, D2Q64): positive roots xi[0..n/2-1] of He_n
// (ascending), and per velocity (in the order of GHSet<n>) the abscissae
// c[a][2] and weights w[a]. Derived once per process and set; null if the
// derivation failed or n is not one of those.
struct HostGH {
  int n, Q, P, N;
  double xi[4];
  double c[64][2];
  double w[64];
};
const HostGH* host_gh(int n);

// The 3-D cube of the 6-point rule, D3Q216: positive roots xi[0..2], and
// per velocity (in the order of D3Q216GH) c[a][3] and w[a].
struct HostGH3 {
  double xi[3];
  double c[216][3];
  double w[216];
};
const HostGH3* host_gh3();

// S(T, u)/w - 1 at velocity a (eq. feq0, rho = 1, order N of the lattice).
double shat_minus_one(const HostLattice& lat, int a, double T, const double u[3]);
// The same at an arbitrary velocity c[D], truncated at order N.
double shat_minus_one_at(int D, int N, const double* c, double T, const double u[3]);

// FP64 version of ProbParams.
struct HostProblem {
  double dt, hs, hsdt, xcoef, omv, invPr, b;
  double g[3];
  int force;
  double Em1[2][QMAX];
  double Ehat[2][QMAX];
  double K0[2], invden[2];
  double gam[2];
  int specular;
};

HostProblem make_problem(const HostLattice& lat, int n_ref, int scheme, double Kn, double Pr, double varpi,
                         const double g[3], const double Tw[2], const double uw[2][3], const double gam[2]);

template <typename C>
void pack_params(const HostProblem& h, int Q, ProbParams<C>& d);
template <typename C>
void pack_lattice(const HostLattice& lat, LatConsts<C>& d);

FastDiv make_fastdiv(uint32_t d);

// Geometry of an nx x ny x nz lattice of Q velocities (D = 2: nz = 1) stored
// in elements of ss bytes. sliced: the slice-blocked population layout of the
// single-lattice path, pstride = ipad and sstride = Q ipad + SLICE_PAD;
// otherwise plain SoA. Returns false if the slot count or a slice block's
// byte size does not fit 32 bits.
constexpr uint32_t SLICE_PAD = 256;   // elements between consecutive slice blocks
bool make_geometry(int D, int Q, uint32_t nx, uint32_t ny, uint32_t nz, bool walls, bool sliced, size_t ss,
                   Geometry& g);


}  // namespace esbgk
