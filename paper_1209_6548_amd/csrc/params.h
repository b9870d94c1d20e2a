// Parameter blocks shared by the host runtime and the kernels.
//
// LatConsts and ProbParams live in device memory (inside the caller's
// workspace) and are read by the kernels through uniform pointers, so they
// arrive in scalar registers and a captured HIP graph stays valid when the
// gas, wall or force parameters change.
#pragma once

#include <stdint.h>

namespace esbgk {

constexpr int QMAX = 39;

// Lattice constants: quadrature weights and the velocity scale c = r e.
template <typename C>
struct LatConsts {
  C w[QMAX];
  C r;
};

// Per-problem constants of one step (derived on the host in FP64).
//   dt      time step dx/r
//   hs      half shift: dt/2 (trapezoid) or 0 (Euler)
//   hsdt    hs/dt
//   xcoef   dt Pr / Kn, so that dt/tau = xcoef rho T^(1-varpi)
//   omv     1 - varpi
//   invPr   1/Pr
//   b       1 - 1/Pr
//   g       body force
//   force   g != 0
// Walls (side 0 low, 1 high), Ehat = S(T_w, u_w)/w at every velocity:
//   Em1     Ehat - 1
//   Ehat    Ehat
//   K0      (sum_{alpha leaving} |e_n| w_alpha)/den - 1
//   invden  1/den, den = sum_{alpha entering} |e_n| w_alpha Ehat_alpha
// so that rho_W - 1 = K0 + invden * (sum of the partial sums of w h over the
// populations that leave through the wall).
//   gam       accommodation gamma of each wall (Maxwell's model, Sec. 3.2):
//             the fraction re-emitted diffusely; 1 - gamma is reflected
//             specularly
//   specular  some wall has gamma < 1
template <typename C>
struct ProbParams {
  C dt, hs, hsdt, xcoef, omv, invPr, b;
  C g[3];
  int force;
  C Em1[2][QMAX];
  C Ehat[2][QMAX];
  C K0[2], invden[2];
  C gam[2];
  int specular;
};

// Unsteady boundary heating (Sec. 4.2): wall temperatures
// T_W(t) = T[side] + amp[side] sin(freq[side] t). Before a step from stored
// level n the device rebuilds the wall tables of ProbParams (Em1, Ehat, K0,
// invden) at t = (n + 1/2) dt, the midpoint of that step's streaming.
struct WallProgram {
  double T[2], amp[2], freq[2];
  double u[2][3];
  double dt;
};

// Division by a run-time constant d for n < 2^31: q = (umulhi(n, m) + n) >> l
// with l = ceil(log2 d) and m = floor(2^32 (2^l - d) / d) + 1.
struct FastDiv {
  uint32_t m, l;
};

// Geometry of one lattice (kernel argument, fixed for a handle's life).
//
// Cells are grouped in slices along the last axis (y in 2-D, z in 3-D; the
// wall axis when there are walls): slice s holds the `inner` cells with that
// last coordinate, numbered i = x (2-D) or i = y nx + x (3-D), and the dense
// cell index is s * inner + i. Population alpha of cell (s, i) is element
// s * sstride + alpha * pstride + i of a population buffer: plain SoA is
// pstride = ncells, sstride = inner; the slice-blocked layout of the
// single-lattice path is pstride >= inner, sstride >= Q * pstride.
struct Geometry {
  uint32_t nx, ny, nz;       // extents
  uint32_t ncells;           // nx*ny*nz
  uint32_t ncols;            // cells of one layer across the wall axis (= inner)
  uint32_t walls;            // 1: diffuse walls across the last axis
  uint32_t nxy;              // nx*ny
  FastDiv div_nx, div_ny;    // division by nx and by ny
  uint32_t inner;            // cells per slice
  uint32_t nslices;          // slices (ny in 2-D, nz in 3-D)
  uint32_t pstride;          // elements between the planes of two velocities in a slice
  uint32_t sstride;          // elements between two consecutive slices
  uint32_t ipad;             // inner rounded up to a multiple of 64: thread slots per slice
  FastDiv div_ipad;          // division by ipad
  uint32_t window_ok;        // 7 slice blocks span < 4 GiB (32-bit offsets of the wave pull)
};

// FP64 reduction slots: mass, energy, momentum x/y/z, sum |u - u_prev|^2,
// sum |u|^2, number of invalid cells.
constexpr int NRED = 8;

// Fields per cell returned by the moments kernel: rho, u[D], T, sigma, q[D].
constexpr int nfields(int D) { return D == 2 ? 9 : 14; }

}  // namespace esbgk
