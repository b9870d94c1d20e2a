// Kernels of the paper's own scheme (Sec. 3.1) on its 3-D set D3Q216: per
// cell the forward-Euler ES-BGK collision and force (Sec. 2.2) from the
// cell's own populations, and per velocity the TVD minmod flux differences
// along x, y and z from the five-cell stencils of the stored level:
//   h^{n+1} = h^n - omega (h^n - h_ES) + dt F/w - sum_axes nu [...].
// Periodic in x and y; in z periodic or bounded by the diffuse walls of
// Sec. 3.2 (ghost slices copy the wall slice; k_tvd3_walls re-emits after
// each step). Populations use the slice layout of Geometry (slice = z
// plane, in-slice index y nx + x).
//
// A cell's 216 populations are streamed twice: once pair by pair into the
// running moment sums, once more pair by pair (from L1/L2) to apply the
// collision and the fluxes; nothing larger than a velocity pair is held.

#include <hip/hip_runtime.h>

#include "gh3.h"
#include "stream.h"
#include "tvd.h"

namespace esbgk {

namespace {

constexpr uint32_t BLOCK3 = 512;
constexpr uint32_t Z3 = BLOCK3 / 64;   // slices per workgroup of the step kernel

}  // namespace

// Eight waves per SIMD (the most a SIMD holds) for FP32 compute: 64 VGPRs,
// 67 more spilled to scratch. The pair loop is latency-bound, and the extra
// waves hide more of it than the scratch reloads cost (128^3 FP32: 2.24 ms
// against 2.63 at six waves and 3.21 at four).
template <typename S>
__global__ void __launch_bounds__(BLOCK3, (sizeof(S) == 8 ? 1 : 8))
k_tvd3(Geometry geo, const S* __restrict__ src, S* __restrict__ dst,
       const GH3Consts<typename StepT<S>::type>* __restrict__ gc,
       const LatConsts<typename StepT<S>::type>* __restrict__ lc,
       const ProbParams<typename StepT<S>::type>* __restrict__ pp) {
  using C = typename StepT<S>::type;
  using L = D3Q216GH;
  constexpr int P = L::P;
  constexpr uint32_t ss = sizeof(S);
  // a workgroup takes one 64-cell chunk of the slice in Z3 = 8 consecutive
  // slices (one wavefront each), chunks fastest: its wavefronts read each
  // other's populations as z-neighbours at about the same velocity pair,
  // and the y-neighbours are chunks started at about the same time (measured
  // at 128^3 FP32: 2.63 ms against 2.68 for 4 slices and 2.76 for 4 chunks
  // of one slice)
  const uint32_t blk = xcd_block(blockIdx.x, gridDim.x);
  const uint32_t nchunks = geo.ipad >> 6;
  const uint32_t band = blk / nchunks, chunk = blk - band * nchunks;
  const uint32_t s = band * Z3 + __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  if (s >= geo.nslices) return;
  const uint32_t i0 = chunk * 64u;
  if (i0 >= geo.inner) return;                       // the slice's padding slots
  const uint32_t lane = threadIdx.x & 63u;
  // lanes past the end of the slice compute its last cell again and store
  // into their own padding slots (i0 + 64 <= ipad)
  const uint32_t i = min(i0 + lane, geo.inner - 1);
  const int nx = int(geo.nx), ny = int(geo.ny), ns = int(geo.nslices);
  const int y = int(fdiv(i, geo.div_nx)), x = int(i) - y * nx;
  uint32_t xo[5], yo[5];
#pragma unroll
  for (int k = -2; k <= 2; ++k) {
    xo[k + 2] = uint32_t(y * nx + wrapc(x + k, nx)) * ss;
    yo[k + 2] = uint32_t(wrapc(y + k, ny) * nx + x) * ss;
  }
  const uint32_t so = (i0 + lane) * ss;
  const uint32_t bb = geo.sstride * ss, pb = geo.pstride * ss;
  Rsrc row[5];
#pragma unroll
  for (int k = -2; k <= 2; ++k) {
    const int r = geo.walls ? min(max(int(s) + k, 0), ns - 1) : wrapc(int(s) + k, ns);
    row[k + 2] = block_rsrc(reinterpret_cast<const char*>(src) + size_t(r) * bb, bb);
  }
  const Rsrc out = block_rsrc(reinterpret_cast<char*>(dst) + size_t(s) * bb, bb);

  // pass 1: moments
  Moments3<C> acc;
  moments3_zero<C>(acc);
  const bool third = pp->force != 0;
#pragma unroll 4
  for (int p = 0; p < P; ++p) {
    const C hp = widen<C, S>(buf_ld<S>(row[2], xo[2], uint32_t(p) * pb));
    const C hm = widen<C, S>(buf_ld<S>(row[2], xo[2], uint32_t(p + P) * pb));
    moments3_add<C>(acc, gc->w[p], gc->mono[p], hp, hm, third);
  }
  GH3Collision<C> k;
  collision_gh3<C>(acc, lc, pp, k);

  // pass 2: collision and fluxes, pair by pair, in the reverse of pass 1's
  // order, so that it starts on the populations pass 1 read last (the pairs
  // are independent: the order changes no result)
#pragma unroll 1
  for (int p = P - 1; p >= 0; --p) {
    const uint32_t pop = uint32_t(p) * pb;
    C hc[2];
    hc[0] = widen<C, S>(buf_ld<S>(row[2], xo[2], pop));
    hc[1] = widen<C, S>(buf_ld<S>(row[2], xo[2], pop + uint32_t(P) * pb));
    C hs[2];
    collide_pair_gh3<C>(k, gc->mono[p], hc[0], hc[1], hs[0], hs[1]);
#pragma unroll
    for (int side = 0; side < 2; ++side) {
      const uint32_t po = pop + uint32_t(side * P) * pb;
      const C sg = side == 0 ? C(1) : C(-1);
      const C f0 = hc[side];
      C t = C(0);
#pragma unroll
      for (int ax = 0; ax < 3; ++ax) {
        const C nu = sg * gc->nu[p][ax];
        const bool pos = nu > C(0);
        C fm1, fp1, f2;
        if (ax == 0) {
          fm1 = widen<C, S>(buf_ld<S>(row[2], xo[1], po));
          fp1 = widen<C, S>(buf_ld<S>(row[2], xo[3], po));
          f2 = widen<C, S>(buf_ld<S>(row[2], pos ? xo[0] : xo[4], po));
        } else if (ax == 1) {
          fm1 = widen<C, S>(buf_ld<S>(row[2], yo[1], po));
          fp1 = widen<C, S>(buf_ld<S>(row[2], yo[3], po));
          f2 = widen<C, S>(buf_ld<S>(row[2], pos ? yo[0] : yo[4], po));
        } else {
          fm1 = widen<C, S>(buf_ld<S>(row[1], xo[2], po));
          fp1 = widen<C, S>(buf_ld<S>(row[3], xo[2], po));
          f2 = widen<C, S>(buf_ld<S>(pos ? row[0] : row[4], xo[2], po));
        }
        C d, m;
        tvd_terms<C>(pos, f2, fm1, f0, fp1, d, m);
        t = fmac(nu, d, t);
        t = fmac(gc->nk[p][ax], m, t);
      }
      buf_st<S, tvd_store_policy<S>(L::Q)>(narrow<S, C>(hs[side] - t), out, so, po);
    }
  }
}

// Re-emission at the z walls (Sec. 3.2) after a step, per in-slice column
// i and wall side = blockIdx.y (see k_tvd_walls).
template <typename S>
__global__ void __launch_bounds__(BLOCK3)
k_tvd3_walls(Geometry geo, S* __restrict__ pop, const TVDWalls3<typename StepT<S>::type>* __restrict__ w) {
  using C = typename StepT<S>::type;
  using L = D3Q216GH;
  const uint32_t i = blockIdx.x * BLOCK3 + threadIdx.x;
  const int side = int(blockIdx.y);
  if (i >= geo.inner) return;
  const uint32_t jw = side ? geo.nslices - 1 : 0, ji = side ? geo.nslices - 2 : 1;
  const size_t ew = size_t(jw) * geo.sstride + i, ei = size_t(ji) * geo.sstride + i;
  C rho = w->k0[side];
#pragma unroll
  for (int a = 0; a < L::Q; ++a) {
    const int sz = gh_sign<L>(a, 2);
    const bool toward = side == 0 ? sz < 0 : sz > 0;
    if (toward) rho = fmac(w->kin[side][a], widen<C, S>(pop[size_t(a) * geo.pstride + ei]), rho);
  }
#pragma unroll
  for (int a = 0; a < L::Q; ++a) {
    const int sz = gh_sign<L>(a, 2);
    const bool into_gas = side == 0 ? sz > 0 : sz < 0;
    if (into_gas) pop[size_t(a) * geo.pstride + ew] = narrow<S, C>(rho * w->sw[side][a] - C(1));
  }
}

// h = rho S(T, u)/w (1 + amp xi) - 1 (eq. feq0 at N = 4, D = 3) for cells
// [c0, c0 + count); c[Q][3]; fields [count] / [3][count] / [Q][count] or
// null.
template <typename S>
__global__ void __launch_bounds__(BLOCK3)
k_tvd3_init(Geometry geo, S* __restrict__ dst, const double* __restrict__ c, const double* __restrict__ rho,
            const double* __restrict__ u, const double* __restrict__ T, const double* __restrict__ noise,
            double amp, uint32_t c0, uint32_t count) {
  const uint32_t j = blockIdx.x * BLOCK3 + threadIdx.x;
  if (j >= count) return;
  const uint32_t cell = c0 + j;
  const uint32_t s = cell / geo.inner, i = cell - s * geo.inner;
  const size_t elem = size_t(s) * geo.sstride + i;
  const double drho = rho ? rho[j] - 1.0 : 0.0;
  double uv[3];
  for (int d = 0; d < 3; ++d) uv[d] = u ? u[size_t(d) * count + j] : 0.0;
  const double th = T ? T[j] - 1.0 : 0.0;
  const double uu = uv[0] * uv[0] + uv[1] * uv[1] + uv[2] * uv[2];
  constexpr double D = 3.0;
  for (int a = 0; a < D3Q216GH::Q; ++a) {
    const double cx = c[3 * a], cy = c[3 * a + 1], cz = c[3 * a + 2];
    const double cu = cx * uv[0] + cy * uv[1] + cz * uv[2], cc = cx * cx + cy * cy + cz * cz;
    double sm1 = cu + 0.5 * (cu * cu - uu + th * (cc - D)) + cu / 6.0 * (cu * cu - 3.0 * uu + 3.0 * th * (cc - D - 2));
    sm1 += (cu * cu * cu * cu - 6.0 * cu * cu * uu + 3.0 * uu * uu) / 24.0 +
           th / 4.0 * ((cc - D - 2) * (cu * cu - uu) - 2.0 * cu * cu) +
           th * th / 8.0 * (cc * cc - 2.0 * (D + 2) * cc + D * (D + 2));
    double hv = drho * (1.0 + sm1) + sm1;
    if (noise) hv += (1.0 + hv) * amp * noise[size_t(a) * count + j];
    dst[size_t(a) * geo.pstride + elem] = S(hv);
  }
}

// The 14 fields rho, u[3], T, sigma (xx xy xz yy yz zz), q[3] of cells
// [c0, c0 + count) in FP64, written as [14][count].
template <typename S>
__global__ void __launch_bounds__(BLOCK3)
k_tvd3_moments(Geometry geo, const S* __restrict__ src, const GH3Consts<double>* __restrict__ gc,
               const LatConsts<double>* __restrict__ lc, const ProbParams<double>* __restrict__ pp, uint32_t c0,
               uint32_t count, double* __restrict__ out) {
  using L = D3Q216GH;
  const uint32_t j = blockIdx.x * BLOCK3 + threadIdx.x;
  if (j >= count) return;
  const uint32_t cell = c0 + j;
  const uint32_t s = cell / geo.inner, i = cell - s * geo.inner;
  const size_t elem = size_t(s) * geo.sstride + i;
  Moments3<double> acc;
  moments3_zero<double>(acc);
  for (int p = 0; p < L::P; ++p) {
    const double hp = double(src[size_t(p) * geo.pstride + elem]);
    const double hm = double(src[size_t(p + L::P) * geo.pstride + elem]);
    moments3_add<double>(acc, gc->w[p], gc->mono[p], hp, hm, true);
  }
  RawMoments<L, double> m;
  moments3_finish<double>(acc, m);
  double f[14];
  fields_from_moments<L, double>(m, lc, pp, f);
  for (int k = 0; k < 14; ++k) out[size_t(k) * count + j] = f[k];
}

#define ESBGK_TVD3_DISPATCH(storage, CALL)                 \
  do {                                                     \
    if (storage == 0) { using S = double; return CALL; }   \
    if (storage == 1) { using S = float; return CALL; }    \
    if (storage == 2) { using S = _Float16; return CALL; } \
    return hipErrorInvalidValue;                           \
  } while (0)

template <typename S>
static hipError_t tvd3_step_t(const TVDArgs& a) {
  using C = typename StepT<S>::type;
  const uint32_t nb = (a.geo.ipad >> 6) * ((a.geo.nslices + Z3 - 1) / Z3);
  hipLaunchKernelGGL(k_tvd3<S>, dim3(nb), dim3(BLOCK3), 0, a.stream, a.geo, static_cast<const S*>(a.src),
                     static_cast<S*>(a.dst), static_cast<const GH3Consts<C>*>(a.gc),
                     static_cast<const LatConsts<C>*>(a.lc), static_cast<const ProbParams<C>*>(a.pp));
  return hipGetLastError();
}

template <typename S>
static hipError_t tvd3_walls_t(const TVDArgs& a, const void* walls) {
  using C = typename StepT<S>::type;
  const dim3 grid((a.geo.inner + BLOCK3 - 1) / BLOCK3, 2);
  hipLaunchKernelGGL(k_tvd3_walls<S>, grid, dim3(BLOCK3), 0, a.stream, a.geo, static_cast<S*>(a.dst),
                     static_cast<const TVDWalls3<C>*>(walls));
  return hipGetLastError();
}

template <typename S>
static hipError_t tvd3_init_t(const TVDArgs& a, const double* c, const double* rho, const double* u,
                              const double* T, const double* noise, double amp, uint32_t c0, uint32_t count) {
  const uint32_t nb = (count + BLOCK3 - 1) / BLOCK3;
  hipLaunchKernelGGL(k_tvd3_init<S>, dim3(nb), dim3(BLOCK3), 0, a.stream, a.geo, static_cast<S*>(a.dst), c, rho, u,
                     T, noise, amp, c0, count);
  return hipGetLastError();
}

template <typename S>
static hipError_t tvd3_moments_t(const TVDArgs& a, uint32_t c0, uint32_t count, double* out) {
  const uint32_t nb = (count + BLOCK3 - 1) / BLOCK3;
  hipLaunchKernelGGL(k_tvd3_moments<S>, dim3(nb), dim3(BLOCK3), 0, a.stream, a.geo, static_cast<const S*>(a.src),
                     static_cast<const GH3Consts<double>*>(a.gc64), static_cast<const LatConsts<double>*>(a.lc64),
                     static_cast<const ProbParams<double>*>(a.pp64), c0, count, out);
  return hipGetLastError();
}

hipError_t launch_tvd3_step(int storage, const TVDArgs& a) { ESBGK_TVD3_DISPATCH(storage, tvd3_step_t<S>(a)); }

hipError_t launch_tvd3_walls(int storage, const TVDArgs& a, const void* walls) {
  ESBGK_TVD3_DISPATCH(storage, (tvd3_walls_t<S>(a, walls)));
}

hipError_t launch_tvd3_init(int storage, const TVDArgs& a, const double* c, const double* rho, const double* u,
                            const double* T, const double* noise, double amp, uint32_t c0, uint32_t count) {
  ESBGK_TVD3_DISPATCH(storage, (tvd3_init_t<S>(a, c, rho, u, T, noise, amp, c0, count)));
}

hipError_t launch_tvd3_moments(int storage, const TVDArgs& a, uint32_t c0, uint32_t count, double* out) {
  ESBGK_TVD3_DISPATCH(storage, (tvd3_moments_t<S>(a, c0, count, out)));
}

}  // namespace esbgk
