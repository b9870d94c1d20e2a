// Per-cell arithmetic of the lattice ES-BGK step (device code).
//
// A cell holds its populations as deviations h_alpha = f_alpha/w_alpha - 1.
// With c_alpha = r e_alpha and the quadrature identities sum w = 1,
// sum w c = 0, sum w c c = delta, sum w c c c = 0 the raw moments of fbar are
//     rho - 1 = sum w h,  j = r sum w h e,  Mbar2 - delta = r^2 sum w h e e,
//     Mbar3 = r^3 sum w h e e e,
// all small numbers, which keeps FP32 arithmetic accurate. The moments are
// accumulated over (e, -e) pairs: even moments from w (h_e + h_-e), odd ones
// from w (h_e - h_-e).
//
// Reconstruction (physical moments of f at the current level) and collision:
//   rho u   = j + hs rho g
//   D rho (T - 1) = tr(Mbar2 - rho delta) + 2 hs rho g.u - rho u^2
//   dt/tau  = x = (dt Pr / Kn) rho T^(1 - varpi)        (tau of Sec. 2.2)
//   xh = x hs/dt, omega = x/(1 + xh), phi = 1 - omega hs/dt
//   sigma   = traceless(Mbar2 - rho u u + hs rho (g u + u g)) / (1 + xh/Pr)
//   Lambda  = lambda - delta = (T - 1) delta + b sigma / rho   (eq. cfeq)
//   a_ES^n  closed forms of Sec. 2.2 written with Lambda
//   a_F^n   = n sym(g (x) a^(n-1)) of the physical f (force expansion, Sec. 2.2)
//   h*_alpha = (1 - omega) h_alpha + sum_n (1/n!) c^(n) : chi^(n)(c_alpha) - omega,
//   c^(n) = omega a_ES^(n) + phi dt a_F^(n).
// The Hermite sum is rewritten once per cell as a polynomial in c (constant,
// linear, ... quartic coefficients K0..K4), then evaluated for each pair as
// its even part E and odd part O with the integer e as compile-time
// constants: h*_e = (1-omega) h_e + E + O, h*_-e = (1-omega) h_-e + E - O.
#pragma once

#include <hip/hip_runtime.h>

#include "lattice.h"
#include "params.h"

namespace esbgk {

// ---- small helpers ---------------------------------------------------------

// Fused multiply-add in the compute type (no promotion of float to double).
__device__ __forceinline__ float fmac(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
__device__ __forceinline__ double fmac(double a, double b, double c) { return __builtin_fma(a, b, c); }

// 1/x: the hardware reciprocal (1 ulp) in FP32, a correctly rounded division
// in FP64.
__device__ __forceinline__ float recip(float x) { return __builtin_amdgcn_rcpf(x); }
__device__ __forceinline__ double recip(double x) { return 1.0 / x; }

// acc + k x for an integer k known at compile time after unrolling; zero terms
// vanish without relying on fast-math.
template <typename C>
__device__ __forceinline__ C addk(C acc, C x, int k) {
  if (k == 0) return acc;
  if (k == 1) return acc + x;
  if (k == -1) return acc - x;
  return fmac(x, C(k), acc);
}

__device__ __forceinline__ constexpr int fact(int n) { return n <= 1 ? 1 : n * fact(n - 1); }

// Number of distinct orderings of a sorted index tuple (multinomial factor).
__device__ __forceinline__ constexpr int mult2(int i, int j) { return i == j ? 1 : 2; }
__device__ __forceinline__ constexpr int mult3(int i, int j, int k) {
  return (i == j && j == k) ? 1 : ((i == j || j == k || i == k) ? 3 : 6);
}
__device__ __forceinline__ constexpr int mult4(int i, int j, int k, int l) {
  // i <= j <= k <= l
  int c[3] = {0, 0, 0};
  c[i]++; c[j]++; c[k]++; c[l]++;
  return 24 / (fact(c[0]) * fact(c[1]) * fact(c[2]));
}

template <typename C> __device__ __forceinline__ C pow_pos(C x, C y);
template <> __device__ __forceinline__ float pow_pos<float>(float x, float y) {
  // x > 0; hardware log2/exp2 (about 1 ulp each)
  return __builtin_amdgcn_exp2f(y * __builtin_amdgcn_logf(x));
}
template <> __device__ __forceinline__ double pow_pos<double>(double x, double y) {
  return pow(x, y);
}

// Storage conversions.
template <typename C, typename S> __device__ __forceinline__ C widen(S v) { return C(v); }
template <typename S, typename C> __device__ __forceinline__ S narrow(C v) { return S(v); }
// FP32 -> FP16 storage: the FP32 value is rounded on its own (round to
// nearest even). The empty asm keeps the compiler from folding the
// conversion into the FMA that produced the value (a single rounding of the
// exact result), which it would do in some kernels and not in others:
// every path then stores the same bits.
template <> __device__ __forceinline__ _Float16 narrow<_Float16, float>(float v) {
  asm("" : "+v"(v));
  return _Float16(v);
}

// ---- raw moments -------------------------------------------------------------

template <class L, typename C>
struct RawMoments {
  C drho;                  // rho - 1
  C J[3];                  // sum w h e
  C S2[3][3];              // sum w h e e
  C S3[3][3][3];           // sum w h e e e (filled on request)
};

template <class L, typename C>
__device__ __forceinline__ void raw_moments(const C (&h)[L::Q], const LatConsts<C>* __restrict__ lc,
                                            bool third, RawMoments<L, C>& m) {
  constexpr int D = L::D, P = L::P;
  m.drho = lc->w[0] * h[0];
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
#pragma unroll
  for (int p = 1; p <= P; ++p) {
    const C wp = lc->w[p];
    const C ws = wp * (h[p] + h[p + P]);
    const C wd = wp * (h[p] - h[p + P]);
    m.drho += ws;
#pragma unroll
    for (int i = 0; i < D; ++i) m.J[i] = addk(m.J[i], wd, L::E[p - 1][i]);
#pragma unroll
    for (int i = 0; i < D; ++i)
#pragma unroll
      for (int j = i; j < D; ++j) m.S2[i][j] = addk(m.S2[i][j], ws, L::E[p - 1][i] * L::E[p - 1][j]);
  }
  if (third) {
#pragma unroll
    for (int p = 1; p <= P; ++p) {
      const C wd = lc->w[p] * (h[p] - h[p + P]);
#pragma unroll
      for (int i = 0; i < D; ++i)
#pragma unroll
        for (int j = i; j < D; ++j)
#pragma unroll
          for (int k = j; k < D; ++k)
            m.S3[i][j][k] = addk(m.S3[i][j][k], wd, L::E[p - 1][i] * L::E[p - 1][j] * L::E[p - 1][k]);
    }
  }
  // mirror the symmetric entries
#pragma unroll
  for (int i = 0; i < D; ++i)
#pragma unroll
    for (int j = 0; j < i; ++j) m.S2[i][j] = m.S2[j][i];
  if (third) {
#pragma unroll
    for (int i = 0; i < D; ++i)
#pragma unroll
      for (int j = i; j < D; ++j)
#pragma unroll
        for (int k = j; k < D; ++k) {
          const C v = m.S3[i][j][k];
          m.S3[i][k][j] = v; m.S3[j][i][k] = v; m.S3[j][k][i] = v;
          m.S3[k][i][j] = v; m.S3[k][j][i] = v;
        }
  }
}

// ---- reconstruction of the physical state ------------------------------------

template <class L, typename C>
struct CellState {
  C rho, irho, drho, theta;   // theta = T - 1
  C u[3], j[3];
  C sigma[3][3], Lam[3][3];
  C omega, phi, xh;
};

template <class L, typename C>
__device__ __forceinline__ void reconstruct(const RawMoments<L, C>& m, const LatConsts<C>* __restrict__ lc,
                                            const ProbParams<C>* __restrict__ pp, CellState<L, C>& s) {
  constexpr int D = L::D;
  const C r = lc->r, r2 = r * r;
  const C hs = pp->hs;
  s.drho = m.drho;
  s.rho = C(1) + m.drho;
  s.irho = recip(s.rho);
  C uu = C(0), gu = C(0);
#pragma unroll
  for (int i = 0; i < D; ++i) {
    s.j[i] = r * m.J[i];
    s.u[i] = s.j[i] * s.irho + hs * pp->g[i];
    uu += s.u[i] * s.u[i];
    gu += pp->g[i] * s.u[i];
  }
  // Mbar2 - rho delta
  C a2b[3][3];
  C tr = C(0);
#pragma unroll
  for (int i = 0; i < D; ++i)
#pragma unroll
    for (int j = 0; j < D; ++j) a2b[i][j] = r2 * m.S2[i][j] - (i == j ? m.drho : C(0));
#pragma unroll
  for (int i = 0; i < D; ++i) tr += a2b[i][i];
  s.theta = (tr + C(2) * hs * s.rho * gu - s.rho * uu) * s.irho * C(1.0 / D);
  const C T = C(1) + s.theta;
  const C x = pp->xcoef * s.rho * pow_pos<C>(T, pp->omv);
  s.xh = x * pp->hsdt;
  s.omega = x * recip(C(1) + s.xh);
  s.phi = C(1) - s.omega * pp->hsdt;
  const C kap = recip(C(1) + s.xh * pp->invPr);
  C Sg[3][3];
  C trS = C(0);
  // symmetric tensors: the upper entries, mirrored (the lower ones would be
  // the same values in another rounding order)
#pragma unroll
  for (int i = 0; i < D; ++i)
#pragma unroll
    for (int j = i; j < D; ++j) {
      Sg[i][j] = a2b[i][j] - s.rho * s.u[i] * s.u[j] + hs * s.rho * (pp->g[i] * s.u[j] + s.u[i] * pp->g[j]);
      Sg[j][i] = Sg[i][j];
    }
#pragma unroll
  for (int i = 0; i < D; ++i) trS += Sg[i][i];
  const C b = pp->b;
#pragma unroll
  for (int i = 0; i < D; ++i)
#pragma unroll
    for (int j = i; j < D; ++j) {
      s.sigma[i][j] = kap * (Sg[i][j] - (i == j ? trS * C(1.0 / D) : C(0)));
      s.Lam[i][j] = (i == j ? s.theta : C(0)) + b * s.sigma[i][j] * s.irho;
      s.sigma[j][i] = s.sigma[i][j];
      s.Lam[j][i] = s.Lam[i][j];
    }
}

// a_ES^(3) of the anisotropic Gaussian (Sec. 2.2) and the physical a^(2).
template <class L, typename C>
__device__ __forceinline__ void es3_and_a2(const CellState<L, C>& s, C (&A3)[3][3][3], C (&a2)[3][3]) {
  constexpr int D = L::D;
#pragma unroll
  for (int i = 0; i < D; ++i)
#pragma unroll
    for (int j = i; j < D; ++j) {
      a2[i][j] = s.rho * s.u[i] * s.u[j] + (i == j ? s.rho * s.theta : C(0)) + s.sigma[i][j];
      a2[j][i] = a2[i][j];
    }
#pragma unroll
  for (int i = 0; i < D; ++i)
#pragma unroll
    for (int j = i; j < D; ++j)
#pragma unroll
      for (int k = j; k < D; ++k) {
        const C v = s.rho * (s.u[i] * s.u[j] * s.u[k] + s.Lam[i][j] * s.u[k] + s.Lam[i][k] * s.u[j] +
                             s.Lam[j][k] * s.u[i]);
        A3[i][j][k] = v; A3[i][k][j] = v; A3[j][i][k] = v;
        A3[j][k][i] = v; A3[k][i][j] = v; A3[k][j][i] = v;
      }
}

// Physical third Hermite coefficient a^(3) of f:
//   a3 = [abar3 + xh a_ES^(3) + hs 3 sym(g (x) a2)] / (1 + xh),
//   abar3 = Mbar3 - 3 sym(j (x) delta).
template <class L, typename C>
__device__ __forceinline__ void physical_a3(const RawMoments<L, C>& m, const CellState<L, C>& s,
                                            const C (&A3)[3][3][3], const C (&a2)[3][3], C r, C hs,
                                            const C* g, bool force, C (&a3)[3][3][3]) {
  constexpr int D = L::D;
  const C r3 = r * r * r;
  const C inv = recip(C(1) + s.xh);
#pragma unroll
  for (int i = 0; i < D; ++i)
#pragma unroll
    for (int j = 0; j < D; ++j)
#pragma unroll
      for (int k = 0; k < D; ++k) {
        C ab = r3 * m.S3[i][j][k] - ((j == k ? s.j[i] : C(0)) + (i == k ? s.j[j] : C(0)) +
                                      (i == j ? s.j[k] : C(0)));
        C v = ab + s.xh * A3[i][j][k];
        if (force) v += hs * (g[i] * a2[j][k] + g[j] * a2[i][k] + g[k] * a2[i][j]);
        a3[i][j][k] = v * inv;
      }
}

// ---- collision -----------------------------------------------------------

// Polynomial coefficients of the post-collision update: with
// c^(n) = omega a_ES^(n) + phi dt a_F^(n) (Sec. 2.2), the relaxation adds
//   w_alpha sum_n c^(n) : chi^(n)(c_alpha) / n!
// which, expanded in powers of e = c / r, is K0 + K1.e + K2:ee + K3:eee +
// K4:eeee (for the deviational h, c^(0) - omega is omega (rho - 1)).
template <class L, typename C>
__device__ __forceinline__ void poly_coeffs(const RawMoments<L, C>& m, const CellState<L, C>& s,
                                            const LatConsts<C>* __restrict__ lc,
                                            const ProbParams<C>* __restrict__ pp, C& K0, C (&K1)[3], C (&K2)[3][3],
                                            C (&K3)[3][3][3], C (&K4)[3][3][3][3]) {
  constexpr int D = L::D, N = L::N;
  const bool force = pp->force != 0;

  const C om = s.omega;
  const C cf = s.phi * pp->dt;   // weight of the force coefficients
  const C* g = pp->g;
  const C rho = s.rho;

  // c^(n) = omega a_ES^(n) + phi dt a_F^(n); c^(0) - omega = omega (rho - 1)
  C c1[3], c2[3][3], c3[3][3][3];
  C c4[3][3][3][3];
  C A3[3][3][3], a2[3][3];
  es3_and_a2<L, C>(s, A3, a2);
#pragma unroll
  for (int i = 0; i < D; ++i) {
    c1[i] = om * rho * s.u[i];
    if (force) c1[i] += cf * rho * g[i];
  }
#pragma unroll
  for (int i = 0; i < D; ++i)
#pragma unroll
    for (int j = 0; j < D; ++j) {
      c2[i][j] = om * rho * (s.u[i] * s.u[j] + s.Lam[i][j]);
      if (force) c2[i][j] += cf * rho * (g[i] * s.u[j] + g[j] * s.u[i]);
    }
#pragma unroll
  for (int i = 0; i < D; ++i)
#pragma unroll
    for (int j = 0; j < D; ++j)
#pragma unroll
      for (int k = 0; k < D; ++k) {
        c3[i][j][k] = om * A3[i][j][k];
        if (force) c3[i][j][k] += cf * (g[i] * a2[j][k] + g[j] * a2[i][k] + g[k] * a2[i][j]);
      }
  if constexpr (N >= 4) {
    C a3[3][3][3];
    if (force) physical_a3<L, C>(m, s, A3, a2, lc->r, pp->hs, g, true, a3);
#pragma unroll
    for (int i = 0; i < D; ++i)
#pragma unroll
      for (int j = i; j < D; ++j)
#pragma unroll
        for (int k = j; k < D; ++k)
#pragma unroll
          for (int l = k; l < D; ++l) {
            const C* u = s.u;
            C v = u[i] * u[j] * u[k] * u[l] + s.Lam[i][j] * u[k] * u[l] + s.Lam[i][k] * u[j] * u[l] +
                  s.Lam[i][l] * u[j] * u[k] + s.Lam[j][k] * u[i] * u[l] + s.Lam[j][l] * u[i] * u[k] +
                  s.Lam[k][l] * u[i] * u[j] + s.Lam[i][j] * s.Lam[k][l] + s.Lam[i][k] * s.Lam[j][l] +
                  s.Lam[i][l] * s.Lam[j][k];
            v = om * rho * v;
            if (force) v += cf * (g[i] * a3[j][k][l] + g[j] * a3[i][k][l] + g[k] * a3[i][j][l] + g[l] * a3[i][j][k]);
            // store every permutation
            const int id[4] = {i, j, k, l};
#pragma unroll
            for (int p0 = 0; p0 < 4; ++p0)
#pragma unroll
              for (int p1 = 0; p1 < 4; ++p1)
#pragma unroll
                for (int p2 = 0; p2 < 4; ++p2) {
                  const int p3 = 6 - p0 - p1 - p2;
                  if (p0 != p1 && p0 != p2 && p1 != p2 && p3 >= 0 && p3 < 4 && p3 != p0 && p3 != p1 && p3 != p2)
                    c4[id[p0]][id[p1]][id[p2]][id[p3]] = v;
                }
          }
  }

  // polynomial coefficients in e (c = r e)
  const C r = lc->r, r2 = r * r, r3 = r2 * r, r4 = r2 * r2;
  K0 = om * s.drho;
  {
    C tr2 = C(0);
#pragma unroll
    for (int i = 0; i < D; ++i) tr2 += c2[i][i];
    K0 -= C(0.5) * tr2;
  }
#pragma unroll
  for (int i = 0; i < D; ++i) {
    C t = C(0);
#pragma unroll
    for (int j = 0; j < D; ++j) t += j < i ? c3[j][j][i] : c3[i][j][j];   // c3 is symmetric: sorted indices
    K1[i] = r * (c1[i] - C(0.5) * t);
  }
#pragma unroll
  for (int i = 0; i < D; ++i)
#pragma unroll
    for (int j = 0; j < D; ++j) K2[i][j] = r2 * C(0.5) * c2[i][j];
  if constexpr (N >= 4) {
    C t4 = C(0);
#pragma unroll
    for (int i = 0; i < D; ++i)
#pragma unroll
      for (int j = 0; j < D; ++j) t4 += c4[i][i][j][j];
    K0 += C(0.125) * t4;
#pragma unroll
    for (int i = 0; i < D; ++i)
#pragma unroll
      for (int j = 0; j < D; ++j) {
        C t = C(0);
#pragma unroll
        for (int k = 0; k < D; ++k) t += c4[i][j][k][k];
        K2[i][j] -= r2 * C(0.25) * t;
      }
  }
#pragma unroll
  for (int i = 0; i < D; ++i)
#pragma unroll
    for (int j = 0; j < D; ++j)
#pragma unroll
      for (int k = 0; k < D; ++k) K3[i][j][k] = r3 * C(1.0 / 6.0) * c3[i][j][k];

  if constexpr (N >= 4) {
#pragma unroll
    for (int i = 0; i < D; ++i)
#pragma unroll
      for (int j = i; j < D; ++j)
#pragma unroll
        for (int k = j; k < D; ++k)
#pragma unroll
          for (int l = k; l < D; ++l) K4[i][j][k][l] = r4 * C(1.0 / 24.0) * c4[i][j][k][l];
  }

}

// The relaxed population (1 - omega) h + poly rounded to the storage type:
// in the compute type one FMA, then the conversion; for FP16 storage one
// mixed-precision FMA that rounds the FP32 operands' exact result once to
// FP16 (v_fma_mixlo_f16), the same in every kernel.
template <typename S, typename C>
__device__ __forceinline__ S relax_store(C omw, C h, C poly) {
  return narrow<S, C>(fmac(omw, h, poly));
}
template <>
__device__ __forceinline__ _Float16 relax_store<_Float16, float>(float omw, float h, float poly) {
  unsigned int d;
  asm("v_fma_mixlo_f16 %0, %1, %2, %3 op_sel_hi:[0,0,0]" : "=v"(d) : "v"(omw), "v"(h), "v"(poly));
  return __builtin_bit_cast(_Float16, static_cast<unsigned short>(d & 0xffffu));
}

// Collision of one cell: h holds the pre-collision populations (compute
// type); out receives the post-collision populations in the storage type S.
template <class L, typename C, typename S>
__device__ __forceinline__ void collide_to(const C (&h)[L::Q], S (&out)[L::Q], const LatConsts<C>* __restrict__ lc,
                                           const ProbParams<C>* __restrict__ pp, CellState<L, C>& s);

template <class L, typename C>
__device__ __forceinline__ void collide(C (&h)[L::Q], const LatConsts<C>* __restrict__ lc,
                                        const ProbParams<C>* __restrict__ pp, CellState<L, C>& s) {
  collide_to<L, C, C>(h, h, lc, pp, s);
}

template <class L, typename C, typename S>
__device__ __forceinline__ void collide_to(const C (&h)[L::Q], S (&out)[L::Q], const LatConsts<C>* __restrict__ lc,
                                           const ProbParams<C>* __restrict__ pp, CellState<L, C>& s) {
  constexpr int D = L::D, P = L::P, N = L::N;
  const bool force = pp->force != 0;
  RawMoments<L, C> m;
  raw_moments<L, C>(h, lc, N >= 4 && force, m);
  reconstruct<L, C>(m, lc, pp, s);
  C K0, K1[3], K2[3][3], K3[3][3][3], K4[3][3][3][3];
  poly_coeffs<L, C>(m, s, lc, pp, K0, K1, K2, K3, K4);
  const C om = s.omega;
  const C omw = C(1) - om;
  out[0] = relax_store<S, C>(omw, h[0], K0);
#pragma unroll
  for (int p = 1; p <= P; ++p) {
    const int e[3] = {L::E[p - 1][0], L::E[p - 1][1], L::E[p - 1][2]};
    C E = K0, O = C(0);
#pragma unroll
    for (int i = 0; i < D; ++i) O = addk(O, K1[i], e[i]);
#pragma unroll
    for (int i = 0; i < D; ++i)
#pragma unroll
      for (int j = i; j < D; ++j) E = addk(E, K2[i][j], mult2(i, j) * e[i] * e[j]);
#pragma unroll
    for (int i = 0; i < D; ++i)
#pragma unroll
      for (int j = i; j < D; ++j)
#pragma unroll
        for (int k = j; k < D; ++k) O = addk(O, K3[i][j][k], mult3(i, j, k) * e[i] * e[j] * e[k]);
    if constexpr (N >= 4) {
#pragma unroll
      for (int i = 0; i < D; ++i)
#pragma unroll
        for (int j = i; j < D; ++j)
#pragma unroll
          for (int k = j; k < D; ++k)
#pragma unroll
            for (int l = k; l < D; ++l)
              E = addk(E, K4[i][j][k][l], mult4(i, j, k, l) * e[i] * e[j] * e[k] * e[l]);
    }
    const S hp = relax_store<S, C>(omw, h[p], E + O);
    const S hm = relax_store<S, C>(omw, h[p + P], E - O);
    out[p] = hp;
    out[p + P] = hm;
  }
}

// ---- macroscopic output ------------------------------------------------------

// rho, u[D], T, sigma (unique components), q[D] of the physical f at the
// current level; q_i = 1/2 [a3_ijj - u_i tr a2 - 2 a2_ij u_j + 2 rho u_i u^2].
template <class L, typename C>
__device__ __forceinline__ void cell_fields(const C (&h)[L::Q], const LatConsts<C>* __restrict__ lc,
                                            const ProbParams<C>* __restrict__ pp, double* out) {
  constexpr int D = L::D;
  RawMoments<L, C> m;
  raw_moments<L, C>(h, lc, true, m);
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

}  // namespace esbgk
