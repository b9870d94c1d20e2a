// The paper's 3-D velocity set (Sec. 2.2): the tensor cube of the 6-point
// Gauss-Hermite rule of eq. weight, D3Q216 (exact to degree 11 along each
// axis, carrying the N = 4 expansion), for the forward-Euler TVD scheme of
// Sec. 3.1. The paper's validation runs use this set (D = 3).
//
// Velocity order (shared with the population I/O): the 108 representatives
// (first component positive) sorted by |c|^2 and then by descending tuple of
// root indices, then their opposites at alpha + 108. Ranks and order are
// compile-time; root values and weights come from the host.
//
// 216 populations do not fit a register-resident cell: the kernels stream a
// cell's populations once to accumulate its moments (Moments3) and once more
// velocity pair by velocity pair to apply the collision and the fluxes.
#pragma once

#include "gh.h"

namespace esbgk {

template <int NPTS>
struct GHCube {
  static_assert(NPTS == 6, "the paper's 6-point rule");
  static constexpr int n = NPTS;
  static constexpr int H = NPTS / 2;
  static constexpr int D = 3;
  static constexpr int Q = NPTS * NPTS * NPTS;
  static constexpr int P = Q / 2;
  static constexpr int N = 4;
  struct Ranks {
    int K[P][3];
  };
  static constexpr int index(int k) { return k > 0 ? H + k - 1 : H + k; }
  static constexpr Ranks make_ranks() {
    Ranks t{};
    double r[H + 1] = {};
    for (int m = 1; m <= H; ++m) r[m] = gh_root(n, m);
    int cnt = 0;
    for (int k1 = 1; k1 <= H; ++k1)
      for (int k2 = -H; k2 <= H; ++k2)
        for (int k3 = -H; k3 <= H; ++k3)
          if (k2 != 0 && k3 != 0) {
            t.K[cnt][0] = k1;
            t.K[cnt][1] = k2;
            t.K[cnt][2] = k3;
            ++cnt;
          }
    // |c|^2 summed over the sorted squares, so that permuted tuples tie
    // exactly and the root-index rule orders them
    auto c2 = [&r](const int* k) {
      double q[3] = {};
      for (int i = 0; i < 3; ++i) {
        const double a = r[k[i] < 0 ? -k[i] : k[i]];
        q[i] = a * a;
      }
      for (int i = 1; i < 3; ++i)
        for (int j = i; j > 0 && q[j] < q[j - 1]; --j) {
          const double t = q[j];
          q[j] = q[j - 1];
          q[j - 1] = t;
        }
      return (q[0] + q[1]) + q[2];
    };
    auto before = [&](const int* u, const int* v) {
      const double cu = c2(u), cv = c2(v);
      if (cu != cv) return cu < cv;
      for (int i = 0; i < 3; ++i)
        if (index(u[i]) != index(v[i])) return index(u[i]) > index(v[i]);
      return false;
    };
    for (int i = 1; i < P; ++i)
      for (int j = i; j > 0 && before(t.K[j], t.K[j - 1]); --j)
        for (int d = 0; d < 3; ++d) {
          const int a = t.K[j][d];
          t.K[j][d] = t.K[j - 1][d];
          t.K[j - 1][d] = a;
        }
    return t;
  }
  static constexpr Ranks ranks = make_ranks();
};

using D3Q216GH = GHCube<6>;

// The monomials c_i c_j ... of degree 1 to 4 of a 3-D velocity, one per
// sorted index tuple: x y z | xx xy xz yy yz zz | 10 cubic | 15 quartic.
// mult is the number of orderings of the tuple (its weight when a symmetric
// tensor is contracted with the velocity).
constexpr int GH3_MONO = 34;
struct Mono3Table {
  int deg[GH3_MONO];
  int idx[GH3_MONO][4];
  int mult[GH3_MONO];
  int zdeg[GH3_MONO];   // the power of c_z
};
constexpr Mono3Table make_mono3() {
  Mono3Table t{};
  int m = 0;
  const int fact[5] = {1, 1, 2, 6, 24};
  for (int d = 1; d <= 4; ++d) {
    int lim = 1;
    for (int k = 0; k < d; ++k) lim *= 3;
    for (int a = 0; a < lim; ++a) {        // digit strings of length d, lexicographic
      int id[4] = {0, 0, 0, 0}, v = a;
      for (int k = d - 1; k >= 0; --k) {
        id[k] = v % 3;
        v /= 3;
      }
      bool sorted = true;
      for (int k = 1; k < d; ++k)
        if (id[k] < id[k - 1]) sorted = false;
      if (!sorted) continue;
      int cnt[3] = {0, 0, 0};
      for (int k = 0; k < d; ++k) {
        t.idx[m][k] = id[k];
        ++cnt[id[k]];
      }
      t.deg[m] = d;
      t.mult[m] = fact[d] / (fact[cnt[0]] * fact[cnt[1]] * fact[cnt[2]]);
      t.zdeg[m] = cnt[2];
      ++m;
    }
  }
  return t;
}
constexpr Mono3Table MONO3 = make_mono3();
static_assert(MONO3.deg[2] == 1 && MONO3.deg[3] == 2 && MONO3.deg[9] == 3 && MONO3.deg[19] == 4 &&
                  MONO3.deg[33] == 4 && MONO3.mult[7] == 2 && MONO3.mult[13] == 6 && MONO3.mult[23] == 12,
              "monomial table of degree 1..4 in three variables");

// Per-set constants (device memory, built on the host) for the 108
// representatives: weight, the 34 monomials, Courant numbers nu = c dt/dx
// per axis and nk = |nu| (1 - |nu|) / 2.
// The representatives fall into 18 groups of six that share (c_x, c_y)
// (c_x > 0: 3 values, c_y: 6) and differ in c_z (6 values). For a cell, the
// collision polynomial of a group is a polynomial in c_z alone, formed once
// per group.
constexpr int GH3_GROUPS = 18, GH3_GROUP = 6;

template <typename C>
struct GH3Consts {
  C w[D3Q216GH::P];
  C mono[D3Q216GH::P][GH3_MONO];
  C nu[D3Q216GH::P][3];
  C nk[D3Q216GH::P][3];
  int order[D3Q216GH::P];        // the pair visited j-th: group by group
  C cz[D3Q216GH::P];             // its c_z
  C gxy[GH3_GROUPS][GH3_MONO];   // c_x^i c_y^j of monomial t for group g
};

// Running sums of the raw moments sum w h (1, c, cc, ccc) over velocity
// pairs (alpha, alpha + P), from the pair sum ws = w (h_a + h_a+P) and
// difference wd = w (h_a - h_a+P); the third moments only when requested.
template <typename C>
struct Moments3 {
  C drho, J[3], S2[6], S3[10];
};

template <typename C>
__device__ __forceinline__ void moments3_zero(Moments3<C>& a) {
  a.drho = C(0);
#pragma unroll
  for (int i = 0; i < 3; ++i) a.J[i] = C(0);
#pragma unroll
  for (int i = 0; i < 6; ++i) a.S2[i] = C(0);
#pragma unroll
  for (int i = 0; i < 10; ++i) a.S3[i] = C(0);
}

template <typename C>
__device__ __forceinline__ void moments3_add(Moments3<C>& a, C w, const C* __restrict__ mo, C hp, C hm, bool third) {
  const C ws = w * (hp + hm), wd = w * (hp - hm);
  a.drho += ws;
#pragma unroll
  for (int i = 0; i < 3; ++i) a.J[i] = fmac(wd, mo[i], a.J[i]);
#pragma unroll
  for (int i = 0; i < 6; ++i) a.S2[i] = fmac(ws, mo[3 + i], a.S2[i]);
  if (third) {
#pragma unroll
    for (int i = 0; i < 10; ++i) a.S3[i] = fmac(wd, mo[9 + i], a.S3[i]);
  }
}

// The symmetric tensors of RawMoments from the running sums.
template <typename C>
__device__ __forceinline__ void moments3_finish(const Moments3<C>& a, RawMoments<D3Q216GH, C>& m) {
  m.drho = a.drho;
#pragma unroll
  for (int i = 0; i < 3; ++i) m.J[i] = a.J[i];
#pragma unroll
  for (int t = 0; t < 6; ++t) {
    const int i = MONO3.idx[3 + t][0], j = MONO3.idx[3 + t][1];
    m.S2[i][j] = m.S2[j][i] = a.S2[t];
  }
#pragma unroll
  for (int t = 0; t < 10; ++t) {
    const int i = MONO3.idx[9 + t][0], j = MONO3.idx[9 + t][1], k = MONO3.idx[9 + t][2];
    const C v = a.S3[t];
    m.S3[i][j][k] = m.S3[i][k][j] = m.S3[j][i][k] = v;
    m.S3[j][k][i] = m.S3[k][i][j] = m.S3[k][j][i] = v;
  }
}

// Collision of Sec. 3.1 (forward Euler, Sec. 2.2 coefficients) as per-cell
// polynomial coefficients per monomial, multiplicities folded in.
template <typename C>
struct GH3Collision {
  C K0, k[GH3_MONO], omw;
};

template <typename C>
__device__ __forceinline__ void collision_gh3(const Moments3<C>& acc, const LatConsts<C>* __restrict__ lc,
                                              const ProbParams<C>* __restrict__ pp, GH3Collision<C>& k) {
  using L = D3Q216GH;
  RawMoments<L, C> m;
  moments3_finish<C>(acc, m);
  CellState<L, C> s;
  reconstruct<L, C>(m, lc, pp, s);
  C K0, K1[3], K2[3][3], K3[3][3][3], K4[3][3][3][3];
  poly_coeffs<L, C>(m, s, lc, pp, K0, K1, K2, K3, K4);
  k.K0 = K0;
#pragma unroll
  for (int t = 0; t < GH3_MONO; ++t) {
    const int* id = MONO3.idx[t];
    const C mult = C(MONO3.mult[t]);
    C v;
    if (MONO3.deg[t] == 1) v = K1[id[0]];
    else if (MONO3.deg[t] == 2) v = K2[id[0]][id[1]];
    else if (MONO3.deg[t] == 3) v = K3[id[0]][id[1]][id[2]];
    else v = K4[id[0]][id[1]][id[2]][id[3]];
    k.k[t] = mult * v;
  }
  k.omw = C(1) - s.omega;
}

// The collision polynomial of one group as polynomials in c_z: e (even
// total degree, powers 0..4) and o (odd total degree, powers 0..3).
template <typename C>
struct GH3Group {
  C e[5], o[4];
};

template <typename C>
__device__ __forceinline__ void group_poly(const GH3Collision<C>& k, const C* __restrict__ gxy, GH3Group<C>& g) {
  g.e[0] = k.K0;
#pragma unroll
  for (int n = 1; n < 5; ++n) g.e[n] = C(0);
#pragma unroll
  for (int n = 0; n < 4; ++n) g.o[n] = C(0);
#pragma unroll
  for (int t = 0; t < GH3_MONO; ++t) {
    const int z = MONO3.zdeg[t];
    if (MONO3.deg[t] % 2) g.o[z] = fmac(k.k[t], gxy[t], g.o[z]);
    else g.e[z] = fmac(k.k[t], gxy[t], g.e[z]);
  }
}

// Post-collision values of the pair (c, -c) of a group from their
// pre-collision values, by Horner in c_z: even part shared, odd part
// changes sign.
template <typename C>
__device__ __forceinline__ void collide_pair_group(const GH3Group<C>& g, C omw, C cz, C hp, C hm, C& outp, C& outm) {
  const C E = fmac(fmac(fmac(fmac(g.e[4], cz, g.e[3]), cz, g.e[2]), cz, g.e[1]), cz, g.e[0]);
  const C O = fmac(fmac(fmac(g.o[3], cz, g.o[2]), cz, g.o[1]), cz, g.o[0]);
  outp = fmac(omw, hp, E + O);
  outm = fmac(omw, hm, E - O);
}

// Post-collision values of the pair (p, p + P) from their pre-collision
// values: even monomials shared, odd ones change sign.
template <typename C>
__device__ __forceinline__ void collide_pair_gh3(const GH3Collision<C>& k, const C* __restrict__ mo, C hp, C hm,
                                                 C& outp, C& outm) {
  C E = k.K0, O = C(0);
#pragma unroll
  for (int t = 0; t < GH3_MONO; ++t) {
    if (MONO3.deg[t] % 2) O = fmac(k.k[t], mo[t], O);
    else E = fmac(k.k[t], mo[t], E);
  }
  outp = fmac(k.omw, hp, E + O);
  outm = fmac(k.omw, hm, E - O);
}

}  // namespace esbgk
