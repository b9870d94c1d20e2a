// Kernels of the paper's own scheme (Sec. 3.1) on the n-point Gauss-Hermite
// product sets (D2Q16, D2Q36, D2Q64): one fused launch per step computes, per cell and
// velocity, the TVD minmod flux difference along x and y from the five-cell
// stencil of the stored level and the forward-Euler ES-BGK collision and
// force from the cell's own populations, and writes
//   h^{n+1} = h^n - omega (h^n - h_ES) + dt F/w - nu_x [...] - nu_y [...].
// Periodic in x; in y periodic or bounded by the diffuse walls of Sec. 3.2
// (ghost rows copy the wall row; a second small kernel re-emits at the
// walls after each step). Populations use the slice layout of Geometry
// (slice = row y); a wavefront shares its row, so the rows y-2..y+2 are
// scalar buffer resources and only the x offsets are per lane.

#include <hip/hip_runtime.h>

#include "gh.h"
#include "stream.h"
#include "tvd.h"

namespace esbgk {

namespace {

constexpr uint32_t BLOCK = 256;

}  // namespace

__device__ __forceinline__ int posmod(int v, int n) { return ((v % n) + n) % n; }

// The advection and collision of every velocity of one cell, writing
// h* - nu_x [...] - nu_y [...]. h holds the cell's level-n populations.
// Lane i of the wavefront holds cell (x0 + i) mod nx of its row, so the x
// neighbours of lanes 1..62 are the neighbouring lanes' registers; the
// halo load of each velocity brings (x0 - 1, x0 - 2, x0 + 65, x0 + 64)
// mod nx into lanes (0, 1, 62, 63) for the rest.
template <class L, typename S, typename C>
__device__ __forceinline__ void tvd_cell(const C (&h)[L::Q], const GHCollision<C>& k,
                                         const GHConsts<C>* __restrict__ gc, const Rsrc (&row)[5], uint32_t xo,
                                         uint32_t hoff, uint32_t so, uint32_t pb, const Rsrc out) {
  constexpr int P = L::P;
  constexpr int G = 3;   // velocity pairs per scheduling group
#pragma unroll
  for (int p0 = 0; p0 < P; p0 += G) {
    __builtin_amdgcn_sched_barrier(0);
    // the plane offsets a pb are formed in each group rather than all at
    // once up front (36 of them would spill out of the scalar registers)
    asm volatile("" : "+s"(pb));
#pragma unroll
    for (int p = p0; p < p0 + G && p < P; ++p) {
      C hs[2];
      collide_pair_gh<L, C>(k, gc->mono[p], h[p], h[p + P], hs[0], hs[1]);
#pragma unroll
      for (int side = 0; side < 2; ++side) {
        const int a = p + side * P;
        const uint32_t po = uint32_t(a) * pb;
        const bool px = gh_sign<L>(a, 0) > 0, py = gh_sign<L>(a, 1) > 0;
        const C sg = side == 0 ? C(1) : C(-1);
        const C f0 = h[a];
        const C H = widen<C, S>(buf_ld<S>(row[2], hoff, po));
        const C xm1 = lane_shift(H, f0, true);
        const C xp1 = lane_shift(H, f0, false);
        const C x2 = px ? lane_shift(lane_shift(H, H, false), xm1, true)     // lane 0 takes x0 - 2
                        : lane_shift(lane_shift(H, H, true), xp1, false);    // lane 63 takes x0 + 65
        const C ym1 = widen<C, S>(buf_ld<S>(row[1], xo, po));
        const C yp1 = widen<C, S>(buf_ld<S>(row[3], xo, po));
        const C y2 = widen<C, S>(buf_ld<S>(py ? row[0] : row[4], xo, po));
        C dx, mx, dy, my;
        tvd_terms<C>(px, x2, xm1, f0, xp1, dx, mx);
        tvd_terms<C>(py, y2, ym1, f0, yp1, dy, my);
        C t = (sg * gc->nu[p][0]) * dx;
        t = fmac(sg * gc->nu[p][1], dy, t);
        t = fmac(gc->nk[p][0], mx, t);
        t = fmac(gc->nk[p][1], my, t);
        buf_st<S, tvd_store_policy<S>(L::Q)>(narrow<S, C>(hs[side] - t), out, so, po);
      }
    }
  }
}

template <class L, typename S>
__global__ void __launch_bounds__(BLOCK)
k_tvd(Geometry geo, const S* __restrict__ src, S* __restrict__ dst,
      const GHConsts<typename StepT<S>::type>* __restrict__ gc,
      const LatConsts<typename StepT<S>::type>* __restrict__ lc,
      const ProbParams<typename StepT<S>::type>* __restrict__ pp) {
  using C = typename StepT<S>::type;
  constexpr int Q = L::Q;
  constexpr uint32_t ss = sizeof(S);
  const uint32_t blk = xcd_block(blockIdx.x, gridDim.x);
  const uint32_t wave0 = blk * BLOCK + (__builtin_amdgcn_readfirstlane(threadIdx.x) & ~63u);
  const uint32_t s = __builtin_amdgcn_readfirstlane(fdiv(wave0, geo.div_ipad));
  if (s >= geo.nslices) return;
  const int nx = int(geo.nx), ns = int(geo.nslices);
  const int x0 = int(__builtin_amdgcn_readfirstlane(wave0 - s * geo.ipad));
  if (x0 >= nx) return;                                // the row's padding slots
  const int lane = int(threadIdx.x & 63u);
  // lanes past the end of the row compute the cells of its start again
  // (periodic) and store them into their own padding slots of the row
  // (x0 + 64 <= ipad), which nothing reads: no lane's store is masked
  const int xc = x0 + lane < nx ? x0 + lane : posmod(x0 + lane, nx);
  // the other lanes of the halo load repeat an address of lanes 0 or 63, so
  // that it touches only the lines beside the wavefront's own
  int hx = lane < 32 ? posmod(x0 - 1, nx) : posmod(x0 + 64, nx);
  if (lane == 1) hx = posmod(x0 - 2, nx);
  if (lane == 62) hx = posmod(x0 + 65, nx);
  const uint32_t xo = uint32_t(xc) * ss, hoff = uint32_t(hx) * ss, so = uint32_t(x0 + lane) * ss;
  const uint32_t bb = geo.sstride * ss, pb = geo.pstride * ss;
  // rows y-2..y+2: periodic images, or (walls) ghost rows that copy the
  // wall row (Sec. 3.2)
  Rsrc row[5];
#pragma unroll
  for (int k = -2; k <= 2; ++k) {
    const int r = geo.walls ? min(max(int(s) + k, 0), ns - 1) : wrapc(int(s) + k, ns);
    row[k + 2] = block_rsrc(reinterpret_cast<const char*>(src) + size_t(r) * bb, bb);
  }

  // level n of the cell stays in registers: the collision and the x
  // neighbours of the advection are both taken from it
  C h[Q];
#pragma unroll
  for (int a = 0; a < Q; ++a) h[a] = widen<C, S>(buf_ld<S>(row[2], xo, uint32_t(a) * pb));
  GHCollision<C> k;
  collision_gh<L, C>(h, gc, lc, pp, k);
  const Rsrc out = block_rsrc(reinterpret_cast<char*>(dst) + size_t(s) * bb, bb);
  tvd_cell<L, S, C>(h, k, gc, row, xo, hoff, so, pb, out);
}

// Re-emission at the walls (Sec. 3.2) after a step: for column x of wall
// side = blockIdx.y, rho_W from the populations moving toward the wall at
// the first node off it, then h = rho_W S/w - 1 for the wall node's
// populations moving into the gas.
template <class L, typename S>
__global__ void __launch_bounds__(BLOCK)
k_tvd_walls(Geometry geo, S* __restrict__ pop, const TVDWalls<typename StepT<S>::type>* __restrict__ w) {
  using C = typename StepT<S>::type;
  const uint32_t x = blockIdx.x * BLOCK + threadIdx.x;
  const int side = int(blockIdx.y);
  if (x >= geo.inner) return;
  const uint32_t jw = side ? geo.nslices - 1 : 0, ji = side ? geo.nslices - 2 : 1;
  const size_t ew = size_t(jw) * geo.sstride + x, ei = size_t(ji) * geo.sstride + x;
  C rho = w->k0[side];
#pragma unroll
  for (int a = 0; a < L::Q; ++a) {
    const bool toward = side == 0 ? gh_sign<L>(a, 1) < 0 : gh_sign<L>(a, 1) > 0;
    if (toward) rho = fmac(w->kin[side][a], widen<C, S>(pop[size_t(a) * geo.pstride + ei]), rho);
  }
#pragma unroll
  for (int a = 0; a < L::Q; ++a) {
    const bool into_gas = side == 0 ? gh_sign<L>(a, 1) > 0 : gh_sign<L>(a, 1) < 0;
    if (into_gas) pop[size_t(a) * geo.pstride + ew] = narrow<S, C>(rho * w->sw[side][a] - C(1));
  }
}

// h = rho S(T, u)/w (1 + amp xi) - 1 for cells [c0, c0 + count) (eq. feq0 at
// the set's order N with the abscissae c[Q][2]); fields [count] / [2][count]
// / [Q][count] or null.
template <class L, typename S>
__global__ void __launch_bounds__(BLOCK)
k_tvd_init(Geometry geo, S* __restrict__ dst, const double* __restrict__ c, const double* __restrict__ rho,
           const double* __restrict__ u, const double* __restrict__ T, const double* __restrict__ noise, double amp,
           uint32_t c0, uint32_t count) {
  const uint32_t i = blockIdx.x * BLOCK + threadIdx.x;
  if (i >= count) return;
  const uint32_t cell = c0 + i;
  const uint32_t y = cell / geo.nx, x = cell - y * geo.nx;
  const size_t elem = size_t(y) * geo.sstride + x;
  const double drho = rho ? rho[i] - 1.0 : 0.0;
  const double ux = u ? u[i] : 0.0, uy = u ? u[size_t(count) + i] : 0.0;
  const double th = T ? T[i] - 1.0 : 0.0;
  const double uu = ux * ux + uy * uy;
  for (int a = 0; a < L::Q; ++a) {
    const double cx = c[2 * a], cy = c[2 * a + 1];
    const double cu = cx * ux + cy * uy, cc = cx * cx + cy * cy;
    double sm1 = cu + 0.5 * (cu * cu - uu + th * (cc - 2.0)) + cu / 6.0 * (cu * cu - 3.0 * uu + 3.0 * th * (cc - 4.0));
    if constexpr (L::N >= 4)
      sm1 += (cu * cu * cu * cu - 6.0 * cu * cu * uu + 3.0 * uu * uu) / 24.0 +
             th / 4.0 * ((cc - 4.0) * (cu * cu - uu) - 2.0 * cu * cu) + th * th / 8.0 * (cc * cc - 8.0 * cc + 8.0);
    double hv = drho * (1.0 + sm1) + sm1;
    if (noise) hv += (1.0 + hv) * amp * noise[size_t(a) * count + i];
    dst[size_t(a) * geo.pstride + elem] = S(hv);
  }
}

// Fields of cells [c0, c0 + count) from their own stored populations (FP64
// arithmetic), written as [9][count].
template <class L, typename S>
__global__ void __launch_bounds__(BLOCK)
k_tvd_moments(Geometry geo, const S* __restrict__ src, const GHConsts<double>* __restrict__ gc,
              const LatConsts<double>* __restrict__ lc, const ProbParams<double>* __restrict__ pp, uint32_t c0,
              uint32_t count, double* __restrict__ out) {
  const uint32_t i = blockIdx.x * BLOCK + threadIdx.x;
  if (i >= count) return;
  const uint32_t cell = c0 + i;
  const uint32_t y = cell / geo.nx, x = cell - y * geo.nx;
  const size_t elem = size_t(y) * geo.sstride + x;
  double h[L::Q];
  for (int a = 0; a < L::Q; ++a) h[a] = double(src[size_t(a) * geo.pstride + elem]);
  double f[9];
  cell_fields_gh<L, double>(h, gc, lc, pp, f);
  for (int k = 0; k < 9; ++k) out[size_t(k) * count + i] = f[k];
}

// Dispatch over the set (velset 4: D2Q16, 3: D2Q36, 5: D2Q64) and the
// storage (0: double, 1: float, 2: _Float16).
#define ESBGK_TVD_DISPATCH(velset, storage, CALL)                        \
  do {                                                                   \
    if (velset == 4) { using L = D2Q16GH; ESBGK_TVD_STORAGE(storage, CALL); } \
    if (velset == 3) { using L = D2Q36GH; ESBGK_TVD_STORAGE(storage, CALL); } \
    if (velset == 5) { using L = D2Q64GH; ESBGK_TVD_STORAGE(storage, CALL); } \
    return hipErrorInvalidValue;                                         \
  } while (0)
#define ESBGK_TVD_STORAGE(storage, CALL)                   \
  do {                                                     \
    if (storage == 0) { using S = double; return CALL; }   \
    if (storage == 1) { using S = float; return CALL; }    \
    if (storage == 2) { using S = _Float16; return CALL; } \
    return hipErrorInvalidValue;                           \
  } while (0)

template <class L, typename S>
static hipError_t tvd_step_t(const TVDArgs& a) {
  using C = typename StepT<S>::type;
  const uint32_t nb = uint32_t((uint64_t(a.geo.nslices) * a.geo.ipad + BLOCK - 1) / BLOCK);
  hipLaunchKernelGGL((k_tvd<L, S>), dim3(nb), dim3(BLOCK), 0, a.stream, a.geo, static_cast<const S*>(a.src),
                     static_cast<S*>(a.dst), static_cast<const GHConsts<C>*>(a.gc),
                     static_cast<const LatConsts<C>*>(a.lc), static_cast<const ProbParams<C>*>(a.pp));
  return hipGetLastError();
}

template <class L, typename S>
static hipError_t tvd_walls_t(const TVDArgs& a, const void* walls) {
  using C = typename StepT<S>::type;
  const dim3 grid((a.geo.inner + BLOCK - 1) / BLOCK, 2);
  hipLaunchKernelGGL((k_tvd_walls<L, S>), grid, dim3(BLOCK), 0, a.stream, a.geo, static_cast<S*>(a.dst),
                     static_cast<const TVDWalls<C>*>(walls));
  return hipGetLastError();
}

template <class L, typename S>
static hipError_t tvd_init_t(const TVDArgs& a, const double* c, const double* rho, const double* u,
                             const double* T, const double* noise, double amp, uint32_t c0, uint32_t count) {
  const uint32_t nb = (count + BLOCK - 1) / BLOCK;
  hipLaunchKernelGGL((k_tvd_init<L, S>), dim3(nb), dim3(BLOCK), 0, a.stream, a.geo, static_cast<S*>(a.dst), c, rho,
                     u, T, noise, amp, c0, count);
  return hipGetLastError();
}

template <class L, typename S>
static hipError_t tvd_moments_t(const TVDArgs& a, uint32_t c0, uint32_t count, double* out) {
  const uint32_t nb = (count + BLOCK - 1) / BLOCK;
  hipLaunchKernelGGL((k_tvd_moments<L, S>), dim3(nb), dim3(BLOCK), 0, a.stream, a.geo, static_cast<const S*>(a.src),
                     static_cast<const GHConsts<double>*>(a.gc64), static_cast<const LatConsts<double>*>(a.lc64),
                     static_cast<const ProbParams<double>*>(a.pp64), c0, count, out);
  return hipGetLastError();
}

hipError_t launch_tvd_step(int velset, int storage, const TVDArgs& a) {
  ESBGK_TVD_DISPATCH(velset, storage, (tvd_step_t<L, S>(a)));
}

hipError_t launch_tvd_walls(int velset, int storage, const TVDArgs& a, const void* walls) {
  ESBGK_TVD_DISPATCH(velset, storage, (tvd_walls_t<L, S>(a, walls)));
}

hipError_t launch_tvd_init(int velset, int storage, const TVDArgs& a, const double* c, const double* rho,
                           const double* u, const double* T, const double* noise, double amp, uint32_t c0,
                           uint32_t count) {
  ESBGK_TVD_DISPATCH(velset, storage, (tvd_init_t<L, S>(a, c, rho, u, T, noise, amp, c0, count)));
}

hipError_t launch_tvd_moments(int velset, int storage, const TVDArgs& a, uint32_t c0, uint32_t count, double* out) {
  ESBGK_TVD_DISPATCH(velset, storage, (tvd_moments_t<L, S>(a, c0, count, out)));
}

}  // namespace esbgk
