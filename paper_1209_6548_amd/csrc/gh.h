// The paper's own velocity sets and scheme (Sec. 2.2, Sec. 3.1): tensor
// products of the n-point Gauss-Hermite rule of eq. weight (exact to degree
// 2n - 1 along each axis), with forward Euler in time and TVD minmod
// finite-volume fluxes in space. The paper's set is n = 6 (degree 11,
// carrying the N = 4 expansion); n = 4 (degree 7, N = 3) and n = 8 (degree
// 15, N = 4) bracket it for velocity-set convergence studies.
//
// The abscissae are off the lattice. Velocity alpha of a 2-D set is
// (xi_{kx}, xi_{ky}) with signed root ranks k in +-1..+-n/2 (xi_{+-1} the
// positive and negative roots nearest zero). The root values and weights are
// derived on the host at start-up; here only the ranks and their order are
// compile-time.
//
// Velocity order (shared with the population I/O): the representatives
// (first component positive) sorted by |c|^2 and then by descending tuple of
// root indices (root index = position of the root in ascending order), then
// their opposites at alpha + P.
#pragma once

#include "cell.h"

namespace esbgk {

// He_n(x) by the three-term recurrence He_{k+1} = x He_k - k He_{k-1}.
constexpr double gh_he(int n, double x) {
  double a = 1.0, b = x;
  if (n == 0) return a;
  for (int k = 1; k < n; ++k) {
    const double c = x * b - double(k) * a;
    a = b;
    b = c;
  }
  return b;
}

// The m-th positive root of He_n (m = 1..n/2, ascending), by a sign scan from
// 0 and bisection: accurate enough to order the velocities (|c|^2 of
// distinct shells differ by more than 0.1 for n <= 8).
constexpr double gh_root(int n, int m) {
  const double step = 1.0 / 64;
  double x = 0.0, fx = gh_he(n, 0.0);
  int found = 0;
  for (int i = 0; i < 64 * 8; ++i) {
    const double y = x + step, fy = gh_he(n, y);
    if ((fx < 0) != (fy < 0) && ++found == m) {
      double lo = x, hi = y;
      for (int it = 0; it < 60; ++it) {
        const double mid = 0.5 * (lo + hi);
        if ((gh_he(n, mid) < 0) == (fx < 0)) lo = mid;
        else hi = mid;
      }
      return 0.5 * (lo + hi);
    }
    x = y;
    fx = fy;
  }
  return -1.0;
}

// The tensor product of the n-point rule in 2-D.
template <int NPTS>
struct GHSet {
  static_assert(NPTS % 2 == 0 && NPTS >= 4 && NPTS <= 8, "even rules of 4 to 8 points");
  static constexpr int n = NPTS;
  static constexpr int H = NPTS / 2;           // positive roots per axis
  static constexpr int D = 2;
  static constexpr int Q = NPTS * NPTS;
  static constexpr int P = Q / 2;
  static constexpr int N = NPTS >= 6 ? 4 : 3;  // Hermite order the set carries (2N + 1 <= 2n - 1)
  struct Ranks {
    int K[P][2];
  };
  // root index of signed rank k: 0..n-1 in ascending root order
  static constexpr int index(int k) { return k > 0 ? H + k - 1 : H + k; }
  static constexpr Ranks make_ranks() {
    Ranks t{};
    double r[H + 1] = {};
    for (int m = 1; m <= H; ++m) r[m] = gh_root(NPTS, m);
    int cnt = 0;
    for (int k1 = 1; k1 <= H; ++k1)
      for (int k2 = -H; k2 <= H; ++k2)
        if (k2 != 0) {
          t.K[cnt][0] = k1;
          t.K[cnt][1] = k2;
          ++cnt;
        }
    auto c2 = [&r](const int* k) {
      const double a = r[k[0] < 0 ? -k[0] : k[0]], b = r[k[1] < 0 ? -k[1] : k[1]];
      return a * a + b * b;
    };
    auto before = [&](const int* u, const int* v) {
      const double cu = c2(u), cv = c2(v);
      if (cu != cv) return cu < cv;
      if (index(u[0]) != index(v[0])) return index(u[0]) > index(v[0]);
      return index(u[1]) > index(v[1]);
    };
    for (int i = 1; i < P; ++i)          // insertion sort
      for (int j = i; j > 0 && before(t.K[j], t.K[j - 1]); --j) {
        const int a0 = t.K[j][0], a1 = t.K[j][1];
        t.K[j][0] = t.K[j - 1][0];
        t.K[j][1] = t.K[j - 1][1];
        t.K[j - 1][0] = a0;
        t.K[j - 1][1] = a1;
      }
    return t;
  }
  static constexpr Ranks ranks = make_ranks();
};

using D2Q16GH = GHSet<4>;
using D2Q36GH = GHSet<6>;
using D2Q64GH = GHSet<8>;

// Sign of component i of velocity alpha of set L.
template <class L>
__host__ __device__ constexpr int gh_sign(int alpha, int i) {
  return (alpha < L::P ? 1 : -1) * (L::ranks.K[alpha % L::P][i] > 0 ? 1 : -1);
}

// Number of monomials c^n, n = 1..4, of a 2-D velocity: x y | xx xy yy |
// xxx xxy xyy yyy | xxxx xxxy xxyy xyyy yyyy.
constexpr int GH_MONO = 14;
constexpr int GH_PMAX = 32;   // representatives of the largest set

// Per-set constants of the scheme (device memory, built on the host), for
// the representatives p < P of the set:
//   w     weight of representative p (its opposite has the same weight)
//   mono  the 14 monomials of representative p (the opposite's odd ones
//         change sign)
//   nu    c dt / dx of representative p along x and y (Courant numbers;
//         the opposite velocity has -nu)
//   nk    |nu| (1 - |nu|) / 2, the weight of the limited slopes in the
//         flux difference (the same for the opposite velocity)
template <typename C>
struct GHConsts {
  C w[GH_PMAX];
  C mono[GH_PMAX][GH_MONO];
  C nu[GH_PMAX][2];
  C nk[GH_PMAX][2];
};

// Raw moments sum w h (1, c, cc, ccc) of the deviational h over the set,
// from the (alpha, alpha + P) pair sums and differences.
template <class L, typename C>
__device__ __forceinline__ void raw_moments_gh(const C (&h)[L::Q], const GHConsts<C>* __restrict__ g,
                                               bool third, RawMoments<L, C>& m) {
  constexpr int P = L::P;
  m.drho = C(0);
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    m.J[i] = C(0);
#pragma unroll
    for (int j = 0; j < 3; ++j) {
      m.S2[i][j] = C(0);
#pragma unroll
      for (int k = 0; k < 3; ++k) m.S3[i][j][k] = C(0);
    }
  }
  C s111 = C(0), s112 = C(0), s122 = C(0), s222 = C(0);
#pragma unroll
  for (int p = 0; p < P; ++p) {
    const C* mo = g->mono[p];
    const C ws = g->w[p] * (h[p] + h[p + P]);
    const C wd = g->w[p] * (h[p] - h[p + P]);
    m.drho += ws;
    m.J[0] = fmac(wd, mo[0], m.J[0]);
    m.J[1] = fmac(wd, mo[1], m.J[1]);
    m.S2[0][0] = fmac(ws, mo[2], m.S2[0][0]);
    m.S2[0][1] = fmac(ws, mo[3], m.S2[0][1]);
    m.S2[1][1] = fmac(ws, mo[4], m.S2[1][1]);
    if (third) {
      s111 = fmac(wd, mo[5], s111);
      s112 = fmac(wd, mo[6], s112);
      s122 = fmac(wd, mo[7], s122);
      s222 = fmac(wd, mo[8], s222);
    }
  }
  m.S2[1][0] = m.S2[0][1];
  // written on both paths (zero without `third`): a store under the
  // condition alone leaves the compiler a store through a selected pointer,
  // which keeps these fields in scratch memory
  m.S3[0][0][0] = s111;
  m.S3[0][0][1] = m.S3[0][1][0] = m.S3[1][0][0] = s112;
  m.S3[0][1][1] = m.S3[1][0][1] = m.S3[1][1][0] = s122;
  m.S3[1][1][1] = s222;
}

// Forward-Euler collision and force of the scheme (Sec. 3.1):
// h* = h - omega (h - h_ES) + dt F/w, with omega = dt/tau and the ES and
// force coefficients of Sec. 2.2 from the moments of h. lc carries r = 1
// (the velocities are the abscissae themselves); pp has hs = hsdt = 0.
// h_ES + dt F/w is a polynomial of degree 4 in c; GHCollision holds its
// coefficients per monomial (multiplicities folded in) and 1 - omega, so
// that the pair (p, p + P) follows from its even and odd parts.
template <typename C>
struct GHCollision {
  C K0, K1[2], k2[3], k3[4], k4[5], omw;
};

template <class L, typename C>
__device__ __forceinline__ void collision_gh(const C (&h)[L::Q], const GHConsts<C>* __restrict__ g,
                                             const LatConsts<C>* __restrict__ lc,
                                             const ProbParams<C>* __restrict__ pp, GHCollision<C>& k) {
  RawMoments<L, C> m;
  raw_moments_gh<L, C>(h, g, pp->force != 0 && L::N >= 4, m);
  CellState<L, C> s;
  reconstruct<L, C>(m, lc, pp, s);
  C K0, K1[3], K2[3][3], K3[3][3][3], K4[3][3][3][3];
  poly_coeffs<L, C>(m, s, lc, pp, K0, K1, K2, K3, K4);
  k.K0 = K0;
  k.K1[0] = K1[0];
  k.K1[1] = K1[1];
  k.k2[0] = K2[0][0];
  k.k2[1] = C(2) * K2[0][1];
  k.k2[2] = K2[1][1];
  k.k3[0] = K3[0][0][0];
  k.k3[1] = C(3) * K3[0][0][1];
  k.k3[2] = C(3) * K3[0][1][1];
  k.k3[3] = K3[1][1][1];
  if constexpr (L::N >= 4) {
    k.k4[0] = K4[0][0][0][0];
    k.k4[1] = C(4) * K4[0][0][0][1];
    k.k4[2] = C(6) * K4[0][0][1][1];
    k.k4[3] = C(4) * K4[0][1][1][1];
    k.k4[4] = K4[1][1][1][1];
  } else {
#pragma unroll
    for (int j = 0; j < 5; ++j) k.k4[j] = C(0);
  }
  k.omw = C(1) - s.omega;
}

// Post-collision values of the pair (p, p + P) from their pre-collision
// values hp, hm (the quartic terms only for a set carrying N = 4).
template <class L, typename C>
__device__ __forceinline__ void collide_pair_gh(const GHCollision<C>& k, const C* __restrict__ mo, C hp, C hm,
                                                C& outp, C& outm) {
  C E = k.K0, O = C(0);
  O = fmac(k.K1[0], mo[0], O);
  O = fmac(k.K1[1], mo[1], O);
#pragma unroll
  for (int j = 0; j < 3; ++j) E = fmac(k.k2[j], mo[2 + j], E);
#pragma unroll
  for (int j = 0; j < 4; ++j) O = fmac(k.k3[j], mo[5 + j], O);
  if constexpr (L::N >= 4) {
#pragma unroll
    for (int j = 0; j < 5; ++j) E = fmac(k.k4[j], mo[9 + j], E);
  }
  outp = fmac(k.omw, hp, E + O);
  outm = fmac(k.omw, hm, E - O);
}

// The collision of every velocity in place.
template <class L, typename C>
__device__ __forceinline__ void collide_gh(C (&h)[L::Q], const GHConsts<C>* __restrict__ g,
                                           const LatConsts<C>* __restrict__ lc,
                                           const ProbParams<C>* __restrict__ pp) {
  constexpr int P = L::P;
  GHCollision<C> k;
  collision_gh<L, C>(h, g, lc, pp, k);
#pragma unroll
  for (int p = 0; p < P; ++p) collide_pair_gh<L, C>(k, g->mono[p], h[p], h[p + P], h[p], h[p + P]);
}

// rho, u[2], T, sigma (xx, xy, yy), q[2] of the stored (physical) f.
// rho, u[D], T, sigma (i <= j), q[D] from the raw moments of the stored
// (physical) f.
template <class L, typename C>
__device__ __forceinline__ void fields_from_moments(const RawMoments<L, C>& m, const LatConsts<C>* __restrict__ lc,
                                                    const ProbParams<C>* __restrict__ pp, double* out) {
  constexpr int D = L::D;
  CellState<L, C> s;
  reconstruct<L, C>(m, lc, pp, s);
  C A3[3][3][3], a2[3][3], a3[3][3][3];
  es3_and_a2<L, C>(s, A3, a2);
  physical_a3<L, C>(m, s, A3, a2, lc->r, pp->hs, pp->g, pp->force != 0, a3);
  int f = 0;
  out[f++] = 1.0 + double(s.drho);
#pragma unroll
  for (int i = 0; i < D; ++i) out[f++] = double(s.u[i]);
  out[f++] = 1.0 + double(s.theta);
#pragma unroll
  for (int i = 0; i < D; ++i)
#pragma unroll
    for (int j = i; j < D; ++j) out[f++] = double(s.sigma[i][j]);
  C uu = C(0), tra2 = C(0);
#pragma unroll
  for (int i = 0; i < D; ++i) { uu += s.u[i] * s.u[i]; tra2 += a2[i][i]; }
#pragma unroll
  for (int i = 0; i < D; ++i) {
    C t3 = C(0), au = C(0);
#pragma unroll
    for (int j = 0; j < D; ++j) { t3 += a3[i][j][j]; au += a2[i][j] * s.u[j]; }
    out[f++] = double(C(0.5) * (t3 - s.u[i] * tra2 - C(2) * au + C(2) * s.rho * s.u[i] * uu));
  }
}

template <class L, typename C>
__device__ __forceinline__ void cell_fields_gh(const C (&h)[L::Q], const GHConsts<C>* __restrict__ g,
                                               const LatConsts<C>* __restrict__ lc,
                                               const ProbParams<C>* __restrict__ pp, double* out) {
  RawMoments<L, C> m;
  raw_moments_gh<L, C>(h, g, true, m);
  fields_from_moments<L, C>(m, lc, pp, out);
}

// minmod(a, b): 0 unless a and b share a sign, else the one smaller in
// magnitude; equals a Psi(b / a) with the limiter Psi of Sec. 3.1 and the
// median of (a, b, 0), which is one instruction (v_med3_f32) in FP32.
__device__ __forceinline__ float minmod(float a, float b) { return __builtin_amdgcn_fmed3f(a, b, 0.0f); }
__device__ __forceinline__ double minmod(double a, double b) {
  return fmax(fmin(a, b), fmin(fmax(a, b), 0.0));
}

// Value of lane i - 1 (shr) or i + 1 (shl) of the wavefront; the lane
// whose source is off the wavefront (lane 0, lane 63) keeps its `old`.
__device__ __forceinline__ int dpp_shift(int old, int v, bool right) {
  return right ? __builtin_amdgcn_update_dpp(old, v, 0x138, 0xf, 0xf, false)    // wave_shr:1
               : __builtin_amdgcn_update_dpp(old, v, 0x130, 0xf, 0xf, false);   // wave_shl:1
}
__device__ __forceinline__ float lane_shift(float old, float v, bool right) {
  return __builtin_bit_cast(float, dpp_shift(__builtin_bit_cast(int, old), __builtin_bit_cast(int, v), right));
}
__device__ __forceinline__ double lane_shift(double old, double v, bool right) {
  const uint64_t o = __builtin_bit_cast(uint64_t, old), w = __builtin_bit_cast(uint64_t, v);
  const uint32_t lo = uint32_t(dpp_shift(int(uint32_t(o)), int(uint32_t(w)), right));
  const uint32_t hi = uint32_t(dpp_shift(int(uint32_t(o >> 32)), int(uint32_t(w >> 32)), right));
  return __builtin_bit_cast(double, (uint64_t(hi) << 32) | lo);
}

// Cache policy of the TVD kernels' population stores: non-temporal (2) when
// a cell's Q populations take 144 bytes or more, else the default (0). The
// stencil re-reads of the neighbouring rows are served by L2, and keeping the
// stores out of it leaves more room for them. Measured on MI355X at 1024^2
// (and 128^3 for D3Q216): 1-5 % faster for D2Q36 FP32, D2Q64 FP32, D2Q36
// FP64 and D3Q216 FP32; 3 % slower for D2Q36 FP16 (72 B) and 17 % slower for
// D2Q16 FP32 (64 B).
template <typename S>
constexpr int tvd_store_policy(int Q) {
  return Q * int(sizeof(S)) >= 144 ? 2 : 0;
}

// The flux difference nu (F_{i+1/2} - F_{i-1/2}) of one velocity along one
// axis (Sec. 3.1) is nu d + nk m, with nk = |nu| (1 - |nu|) / 2, d the
// upwind difference (f_i - f_{i-1} for nu > 0, f_{i+1} - f_i for nu < 0)
// and m the difference of the limited slopes at the right and left faces
// (for nu < 0 the paper's formula mirrored). The stencil is the four
// upwind-biased values: f2 = f_{i-2} for nu > 0, f2 = f_{i+2} for nu < 0.
template <typename C>
__device__ __forceinline__ void tvd_terms(bool positive, C f2, C fm1, C f0, C fp1, C& d, C& m) {
  if (positive) {
    const C dm = fm1 - f2, d0 = f0 - fm1, dp = fp1 - f0;
    d = d0;
    m = minmod(dp, d0) - minmod(d0, dm);
  } else {
    const C dm = f0 - fm1, d0 = fp1 - f0, dp = f2 - fp1;
    d = d0;
    m = minmod(d0, dp) - minmod(dm, d0);
  }
}

// tvd_terms without a branch on the direction, for loops whose velocity is
// not a compile-time constant: the same differences and limited slopes (the
// minmod is symmetric and -(x - y) rounds as y - x), chosen by selects.
template <typename C>
__device__ __forceinline__ void tvd_terms_sel(bool positive, C f2, C fm1, C f0, C fp1, C& d, C& m) {
  const C back = f0 - fm1, fwd = fp1 - f0;
  const C d2 = positive ? fm1 - f2 : f2 - fp1;   // the difference one cell further upwind
  d = positive ? back : fwd;
  const C t = minmod(fwd, back) - minmod(d, d2);
  m = positive ? t : -t;
}

}  // namespace esbgk
