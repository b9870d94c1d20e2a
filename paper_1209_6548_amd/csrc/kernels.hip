// HIP kernels of the lattice ES-BGK step for gfx950, and their launchers.
//
// One thread updates one cell per step (pull scheme): it gathers the Q
// populations that stream into the cell from buffer A, collides them
// (cell.h) and writes the cell's Q post-collision populations to buffer B.
// Populations are structure-of-arrays, [alpha][z][y][x], x fastest, so every
// load and store of a wavefront covers 64 consecutive cells of one velocity.
//
// Streaming. For a wavefront whose cells are at least 3 cells away from every
// edge, the source of velocity alpha is cell - shift_alpha with one shift per
// velocity; the kernel folds that shift into the (uniform) base address of
// the velocity plane, so all Q loads share one per-lane offset. Wavefronts
// that touch an edge use per-lane wrapped coordinates and, across a wall, the
// re-emitted populations of the diffuse wall (Sec. 3.2).
//
// Diffuse walls. rho_W of a wall-parallel column is the flux balance of
// Sec. 3.2: the populations that cross the wall in one step (a population
// with |e_n| = k crosses from the k layers next to the wall) over the matching
// flux of S(T_w, u_w). Each step writes, for the cells of the three layers
// next to a wall, the partial sums sum w h over the populations of that cell
// that will cross the wall on the next step, computed from the values as
// stored; the next step sums the three layers of a column. A population that
// streams in from beyond the wall takes rho_W(source column) S(T_w, u_w).
//
// Reductions. The REDUCE variant also accumulates per cell, in FP64, the mass,
// energy, momentum and the residual sums of the pre-collision state, reduces
// them over the workgroup (wavefront shuffles, then LDS) and writes one
// partial per workgroup; k_reduce_finalize sums the partials in a fixed order.

#include <hip/hip_runtime.h>

#include <mutex>

#include "kernels.h"
#include "reduce.h"
#include "stream.h"

namespace esbgk {

constexpr int BLOCK = 256;

// ---- FP64 reductions ---------------------------------------------------------

// Sum NRED values over the workgroup (fixed order) and write them to out.
__device__ __forceinline__ void block_reduce_write(double (&v)[NRED], double* __restrict__ out) {
  __shared__ double lds[BLOCK / 64][NRED];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
  for (int k = 0; k < NRED; ++k) {
    const double s = wave_sum(v[k]);
    if (lane == 0) lds[wave][k] = s;
  }
  __syncthreads();
  if (threadIdx.x < NRED) {
    double s = 0.0;
#pragma unroll
    for (int w = 0; w < BLOCK / 64; ++w) s += lds[w][threadIdx.x];
    out[threadIdx.x] = s;
  }
}

// ---- kernels ---------------------------------------------------------------

// Thread slot -> cell of the step and reduction kernels: slot t is in-slice
// index i = t mod ipad of slice s = t / ipad, active when i < inner and
// s < nslices. ipad is a multiple of 64, so the lanes of a wavefront share
// their slice, which the kernels use as a scalar.
struct Slot {
  uint32_t s, i;
  bool active;
};

__device__ __forceinline__ Slot slot_of(uint32_t blk, const Geometry& geo) {
  const uint32_t wave0 = blk * BLOCK + (__builtin_amdgcn_readfirstlane(threadIdx.x) & ~63u);
  const uint32_t s = __builtin_amdgcn_readfirstlane(fdiv(wave0, geo.div_ipad));
  const uint32_t i = blk * BLOCK + threadIdx.x - s * geo.ipad;
  return {s, i, s < geo.nslices && i < geo.inner};
}

// One time step: pull, collide, store, wall partial sums (and, when REDUCE,
// the FP64 reductions of the pre-collision state).
template <class L, typename S, bool REDUCE>
__global__ void __launch_bounds__(BLOCK)
k_step(Geometry geo, const S* __restrict__ src, S* __restrict__ dst, const typename StepT<S>::type* __restrict__ wp_src,
       typename StepT<S>::type* __restrict__ wp_dst, const LatConsts<typename StepT<S>::type>* __restrict__ lc,
       const ProbParams<typename StepT<S>::type>* __restrict__ pp, typename StepT<S>::type* __restrict__ uprev,
       int have_prev, double* __restrict__ red_part, int rev) {
  using C = typename StepT<S>::type;
  const uint32_t blk = tile_of(blockIdx.x, gridDim.x, rev);
  const Slot sl = slot_of(blk, geo);
  double v[NRED];
  if (REDUCE) {
#pragma unroll
    for (int k = 0; k < NRED; ++k) v[k] = 0.0;
  }
  if (sl.active) {
    const CellPos p = slice_pos<L>(sl.s, sl.i, geo);
    const PullMode mode = pull_mode_wave<L>(sl.s, p, geo);
    C h[L::Q];
    gather_wave<L, S, C, C>(h, src, geo, sl.s, sl.i, p, wp_src, pp, mode);
    CellState<L, C> st;
    S hs[L::Q];
    collide_to<L, C, S>(h, hs, lc, pp, st);
    const uint32_t bb = geo.sstride * uint32_t(sizeof(S)), pb = geo.pstride * uint32_t(sizeof(S));
    const Rsrc out = block_rsrc(reinterpret_cast<char*>(dst) + size_t(sl.s) * bb, bb);
#pragma unroll
    for (int a = 0; a < L::Q; ++a) buf_st<S>(hs[a], out, sl.i * uint32_t(sizeof(S)), uint32_t(a) * pb);
    if (geo.walls) write_wall_partials<L, S, C>([&](int a) { return hs[a]; }, p, geo, lc, wp_dst);
    if (REDUCE) cell_contrib<L, C, C>(st, uprev, sl.s * geo.inner + sl.i, geo.ncells, have_prev, v);
  }
  if (REDUCE) block_reduce_write(v, red_part + size_t(blk) * NRED);
}

// One step of the in-place pair (the layout is described in stream.h): PHASE
// 1 pulls from the buffer and pushes to the opposite planes of the forward
// neighbours; PHASE 2 reads its own cell's opposite planes and writes its own
// planes. The cell arithmetic (collision, wall partial sums, reductions) is
// k_step's, so the pair gives the same bits as two steps through two
// buffers. Only for fully diffuse (or no) walls: a specular image would need
// the values pushed across a wall.
template <class L, typename S, int PHASE, bool REDUCE>
__global__ void __launch_bounds__(BLOCK)
k_pair(Geometry geo, S* buf, const typename StepT<S>::type* __restrict__ wp_src,
       typename StepT<S>::type* __restrict__ wp_dst, const LatConsts<typename StepT<S>::type>* __restrict__ lc,
       const ProbParams<typename StepT<S>::type>* __restrict__ pp, typename StepT<S>::type* __restrict__ uprev,
       int have_prev, double* __restrict__ red_part, int rev) {
  using C = typename StepT<S>::type;
  const uint32_t blk = tile_of(blockIdx.x, gridDim.x, rev);
  const Slot sl = slot_of(blk, geo);
  double v[NRED];
  if (REDUCE) {
#pragma unroll
    for (int k = 0; k < NRED; ++k) v[k] = 0.0;
  }
  if (sl.active) {
    const CellPos p = slice_pos<L>(sl.s, sl.i, geo);
    C h[L::Q];
    PullMode mode = PULL_EDGE;
    if (PHASE == 1) {
      mode = pull_mode_wave<L>(sl.s, p, geo);
      gather_wave<L, S, C, C>(h, buf, geo, sl.s, sl.i, p, wp_src, pp, mode);
    } else {
      gather_local<L, S, C, C>(h, buf, geo, sl.s, sl.i, p, wp_src, pp);
    }
    CellState<L, C> st;
    S hs[L::Q];
    collide_to<L, C, S>(h, hs, lc, pp, st);
    if (PHASE == 1) {
      scatter_wave<L, S>(hs, buf, geo, sl.s, sl.i, p, mode);
    } else {
      const uint32_t bb = geo.sstride * uint32_t(sizeof(S)), pb = geo.pstride * uint32_t(sizeof(S));
      const Rsrc out = block_rsrc(reinterpret_cast<char*>(buf) + size_t(sl.s) * bb, bb);
#pragma unroll
      for (int a = 0; a < L::Q; ++a) buf_st<S>(hs[a], out, sl.i * uint32_t(sizeof(S)), uint32_t(a) * pb);
    }
    if (geo.walls) write_wall_partials<L, S, C>([&](int a) { return hs[a]; }, p, geo, lc, wp_dst);
    if (REDUCE) cell_contrib<L, C, C>(st, uprev, sl.s * geo.inner + sl.i, geo.ncells, have_prev, v);
  }
  if (REDUCE) block_reduce_write(v, red_part + size_t(blk) * NRED);
}

// Reductions of the current level without stepping (FP64 arithmetic), over
// the same slots and workgroups as the fused reductions of the step kernel.
template <class L, typename S>
__global__ void __launch_bounds__(BLOCK)
k_reduce(Geometry geo, const S* __restrict__ src, const typename StepT<S>::type* __restrict__ wp,
         const LatConsts<double>* __restrict__ lc, const ProbParams<double>* __restrict__ pp,
         typename StepT<S>::type* __restrict__ uprev, int have_prev, double* __restrict__ red_part) {
  using P = typename StepT<S>::type;
  const uint32_t blk = xcd_block(blockIdx.x, gridDim.x);
  const Slot sl = slot_of(blk, geo);
  double v[NRED];
#pragma unroll
  for (int k = 0; k < NRED; ++k) v[k] = 0.0;
  if (sl.active) {
    const CellPos p = slice_pos<L>(sl.s, sl.i, geo);
    const PullMode mode = pull_mode_wave<L>(sl.s, p, geo);
    double h[L::Q];
    gather_wave<L, S, double, P>(h, src, geo, sl.s, sl.i, p, wp, pp, mode);
    RawMoments<L, double> m;
    raw_moments<L, double>(h, lc, false, m);
    CellState<L, double> st;
    reconstruct<L, double>(m, lc, pp, st);
    cell_contrib<L, double, P>(st, uprev, sl.s * geo.inner + sl.i, geo.ncells, have_prev, v);
  }
  block_reduce_write(v, red_part + size_t(blk) * NRED);
}

// The same reductions folded onto at most gridDim.x workgroups: workgroup g
// adds the cells of slot blocks g, g + gridDim.x, ... in that order, so the
// partials need room for gridDim.x workgroups whatever the lattice size.
template <class L, typename S>
__global__ void __launch_bounds__(BLOCK)
k_reduce_fold(Geometry geo, const S* __restrict__ src, const typename StepT<S>::type* __restrict__ wp,
              const LatConsts<double>* __restrict__ lc, const ProbParams<double>* __restrict__ pp,
              typename StepT<S>::type* __restrict__ uprev, int have_prev, uint32_t nblocks,
              double* __restrict__ part) {
  using P = typename StepT<S>::type;
  double acc[NRED];
#pragma unroll
  for (int k = 0; k < NRED; ++k) acc[k] = 0.0;
  for (uint32_t blk = blockIdx.x; blk < nblocks; blk += gridDim.x) {
    const Slot sl = slot_of(blk, geo);
    if (!sl.active) continue;
    const CellPos p = slice_pos<L>(sl.s, sl.i, geo);
    const PullMode mode = pull_mode_wave<L>(sl.s, p, geo);
    double h[L::Q];
    gather_wave<L, S, double, P>(h, src, geo, sl.s, sl.i, p, wp, pp, mode);
    RawMoments<L, double> m;
    raw_moments<L, double>(h, lc, false, m);
    CellState<L, double> st;
    reconstruct<L, double>(m, lc, pp, st);
    double v[NRED];
    cell_contrib<L, double, P>(st, uprev, sl.s * geo.inner + sl.i, geo.ncells, have_prev, v);
#pragma unroll
    for (int k = 0; k < NRED; ++k) acc[k] += v[k];
  }
  block_reduce_write(acc, part + size_t(blockIdx.x) * NRED);
}

__global__ void __launch_bounds__(BLOCK) k_reduce_finalize(const double* __restrict__ part, uint32_t nparts,
                                                           double* __restrict__ out) {
  __shared__ double lds[BLOCK][NRED];
  double v[NRED];
#pragma unroll
  for (int k = 0; k < NRED; ++k) v[k] = 0.0;
  for (uint32_t b = threadIdx.x; b < nparts; b += BLOCK) {
#pragma unroll
    for (int k = 0; k < NRED; ++k) v[k] += part[size_t(b) * NRED + k];
  }
#pragma unroll
  for (int k = 0; k < NRED; ++k) lds[threadIdx.x][k] = v[k];
  __syncthreads();
  for (int stride = BLOCK / 2; stride > 0; stride >>= 1) {
    if (int(threadIdx.x) < stride) {
#pragma unroll
      for (int k = 0; k < NRED; ++k) lds[threadIdx.x][k] += lds[threadIdx.x + stride][k];
    }
    __syncthreads();
  }
  if (threadIdx.x < NRED) out[threadIdx.x] = lds[0][threadIdx.x];
}

// Macroscopic fields of cells [c0, c0 + count), FP64 arithmetic from the
// stored state, written as [F][count].
template <class L, typename S>
__global__ void __launch_bounds__(BLOCK)
k_moments(Geometry geo, const S* __restrict__ src, const typename StepT<S>::type* __restrict__ wp,
          const LatConsts<double>* __restrict__ lc, const ProbParams<double>* __restrict__ pp, uint32_t c0,
          uint32_t count, double* __restrict__ out) {
  using P = typename StepT<S>::type;
  const uint32_t i = blockIdx.x * BLOCK + threadIdx.x;
  if (i >= count) return;
  const CellPos p = cell_pos(c0 + i, geo);
  double h[L::Q];
  gather_lane<L, S, double, P, size_t>(h, src, geo, p, wp, pp);
  double f[nfields(L::D)];
  cell_fields<L, double>(h, lc, pp, f);
#pragma unroll
  for (int k = 0; k < nfields(L::D); ++k) out[size_t(k) * count + i] = f[k];
}

// S(T, u)/w - 1 at velocity alpha (eq. feq0 at the order N of the lattice).
template <class L>
__device__ __forceinline__ double shat_m1(int a, double r, const double* u, double th) {
  constexpr int D = L::D;
  double cu = 0.0, uu = 0.0, cc = 0.0;
#pragma unroll
  for (int i = 0; i < D; ++i) {
    const double ci = r * ecomp<L>(a, i);
    cu += ci * u[i];
    uu += u[i] * u[i];
    cc += ci * ci;
  }
  double s = cu + 0.5 * (cu * cu - uu + th * (cc - D)) + cu / 6.0 * (cu * cu - 3.0 * uu + 3.0 * th * (cc - D - 2));
  if (L::N >= 4) {
    s += (cu * cu * cu * cu - 6.0 * cu * cu * uu + 3.0 * uu * uu) / 24.0 +
         th / 4.0 * ((cc - D - 2) * (cu * cu - uu) - 2.0 * cu * cu) +
         th * th / 8.0 * (cc * cc - 2.0 * (D + 2) * cc + D * (D + 2));
  }
  return s;
}

// Wall tables for the step from stored level *level (unsteady heating): one
// workgroup, thread a evaluates S(T_W, u_W)/w - 1 at velocity a for both
// walls, thread 0 sums the flux terms in velocity order and, if advance,
// moves the level on.
template <class L>
__global__ void __launch_bounds__(64)
k_wall_tables(const WallProgram* __restrict__ prog, const LatConsts<double>* __restrict__ lc,
              ProbParams<double>* __restrict__ pp64, ProbParams<float>* __restrict__ pp32,
              int64_t* __restrict__ level, int advance) {
  constexpr int Q = L::Q, W = L::D - 1;
  __shared__ double em1[2][Q];
  const int a = int(threadIdx.x);
  const double t = (double(*level) + 0.5) * prog->dt;
  if (a < Q) {
#pragma unroll
    for (int side = 0; side < 2; ++side) {
      const double th = prog->T[side] + prog->amp[side] * sin(prog->freq[side] * t) - 1.0;
      const double v = shat_m1<L>(a, lc->r, prog->u[side], th);
      em1[side][a] = v;
      pp64->Em1[side][a] = v;
      pp64->Ehat[side][a] = 1.0 + v;
      if (pp32) {
        pp32->Em1[side][a] = float(v);
        pp32->Ehat[side][a] = float(1.0 + v);
      }
    }
  }
  __syncthreads();
  if (a == 0) {
    for (int side = 0; side < 2; ++side) {
      double leave = 0.0, den = 0.0;
      for (int b = 0; b < Q; ++b) {
        const int en = ecomp<L>(b, W);
        const bool out = side == 0 ? en < 0 : en > 0;
        const bool in = side == 0 ? en > 0 : en < 0;
        const double k = double(en < 0 ? -en : en);
        if (out) leave += k * lc->w[b];
        if (in) den += k * lc->w[b] * (1.0 + em1[side][b]);
      }
      pp64->K0[side] = leave / den - 1.0;
      pp64->invden[side] = 1.0 / den;
      if (pp32) {
        pp32->K0[side] = float(leave / den - 1.0);
        pp32->invden[side] = float(1.0 / den);
      }
    }
    if (advance) *level += 1;
  }
}

// Equilibrium initial state h = rho Shat (1 + amp xi) - 1 for cells
// [c0, c0 + count); fields are [count] / [D][count] / [Q][count] or null.
template <class L, typename S>
__global__ void __launch_bounds__(BLOCK)
k_init(Geometry geo, S* __restrict__ dst, double r, const double* __restrict__ rho, const double* __restrict__ u,
       const double* __restrict__ T, const double* __restrict__ noise, double amp, uint32_t c0, uint32_t count) {
  const uint32_t i = blockIdx.x * BLOCK + threadIdx.x;
  if (i >= count) return;
  const size_t elem = cell_elem<L>(cell_pos(c0 + i, geo), geo);
  const double drho = rho ? rho[i] - 1.0 : 0.0;
  double uc[3] = {0.0, 0.0, 0.0};
  if (u) {
#pragma unroll
    for (int d = 0; d < L::D; ++d) uc[d] = u[size_t(d) * count + i];
  }
  const double th = T ? T[i] - 1.0 : 0.0;
#pragma unroll
  for (int a = 0; a < L::Q; ++a) {
    const double sm1 = shat_m1<L>(a, r, uc, th);
    // rho Shat - 1 = drho Shat + (Shat - 1)
    double hv = drho * (1.0 + sm1) + sm1;
    if (noise) hv += (1.0 + hv) * amp * noise[size_t(a) * count + i];
    dst[size_t(a) * geo.pstride + elem] = S(hv);
  }
}

// Wall partial sums of the stored state (after the state was set); the same
// arithmetic as the step kernel's, so a restart is bit-identical.
template <class L, typename S>
__global__ void __launch_bounds__(BLOCK)
k_wall_partials(Geometry geo, const S* __restrict__ src, const LatConsts<typename StepT<S>::type>* __restrict__ lc,
                typename StepT<S>::type* __restrict__ wp_dst) {
  using P = typename StepT<S>::type;
  const uint32_t i = blockIdx.x * BLOCK + threadIdx.x;
  if (i >= 6u * geo.ncols) return;
  const uint32_t col = i % geo.ncols;
  const uint32_t sk = i / geo.ncols;       // side * 3 + k
  const int side = int(sk / 3), k = int(sk % 3);
  const int nw = int(geo.nslices);
  const int cw = side == 0 ? k : nw - 1 - k;
  const size_t elem = size_t(cw) * geo.sstride + col;   // the wall axis is the slice axis
  const CrossSums<L, S, P> cs =
      cross_sums<L, S, P>([&](int a) { return src[size_t(a) * geo.pstride + elem]; }, lc);
  wp_dst[sk * geo.ncols + col] = side == 0 ? layer_partial(cs.lo, k) : layer_partial(cs.hi, k);
}

// ---- launchers -----------------------------------------------------------------

// Workgroups of the step and reduction kernels: nslices * ipad thread slots.
uint32_t slot_blocks(const Geometry& g) { return uint32_t((uint64_t(g.nslices) * g.ipad + BLOCK - 1) / BLOCK); }

template <class L, typename S>
static hipError_t step_t(const StepArgs& a) {
  using C = typename StepT<S>::type;
  const uint32_t nb = slot_blocks(a.geo);
  if (a.reduce) {
    hipLaunchKernelGGL((k_step<L, S, true>), dim3(nb), dim3(BLOCK), 0, a.stream, a.geo, static_cast<const S*>(a.src),
                       static_cast<S*>(a.dst), static_cast<const C*>(a.wp_src), static_cast<C*>(a.wp_dst),
                       static_cast<const LatConsts<C>*>(a.lc), static_cast<const ProbParams<C>*>(a.pp),
                       static_cast<C*>(a.uprev), a.have_prev, a.red_part, a.rev);
  } else {
    hipLaunchKernelGGL((k_step<L, S, false>), dim3(nb), dim3(BLOCK), 0, a.stream, a.geo,
                       static_cast<const S*>(a.src), static_cast<S*>(a.dst), static_cast<const C*>(a.wp_src),
                       static_cast<C*>(a.wp_dst), static_cast<const LatConsts<C>*>(a.lc),
                       static_cast<const ProbParams<C>*>(a.pp), static_cast<C*>(a.uprev), a.have_prev, a.red_part,
                       a.rev);
  }
  return hipGetLastError();
}

template <class L, typename S, int PHASE>
static hipError_t pair_t(const StepArgs& a) {
  using C = typename StepT<S>::type;
  const uint32_t nb = slot_blocks(a.geo);
  S* buf = static_cast<S*>(a.dst);
  if (a.reduce) {
    hipLaunchKernelGGL((k_pair<L, S, PHASE, true>), dim3(nb), dim3(BLOCK), 0, a.stream, a.geo, buf,
                       static_cast<const C*>(a.wp_src), static_cast<C*>(a.wp_dst),
                       static_cast<const LatConsts<C>*>(a.lc), static_cast<const ProbParams<C>*>(a.pp),
                       static_cast<C*>(a.uprev), a.have_prev, a.red_part, a.rev);
  } else {
    hipLaunchKernelGGL((k_pair<L, S, PHASE, false>), dim3(nb), dim3(BLOCK), 0, a.stream, a.geo, buf,
                       static_cast<const C*>(a.wp_src), static_cast<C*>(a.wp_dst),
                       static_cast<const LatConsts<C>*>(a.lc), static_cast<const ProbParams<C>*>(a.pp),
                       static_cast<C*>(a.uprev), a.have_prev, a.red_part, a.rev);
  }
  return hipGetLastError();
}

template <class L, typename S>
static hipError_t reduce_t(const StepArgs& a) {
  using C = typename StepT<S>::type;
  const uint32_t nb = slot_blocks(a.geo);
  hipLaunchKernelGGL((k_reduce<L, S>), dim3(nb), dim3(BLOCK), 0, a.stream, a.geo, static_cast<const S*>(a.src),
                     static_cast<const C*>(a.wp_src), static_cast<const LatConsts<double>*>(a.lc64),
                     static_cast<const ProbParams<double>*>(a.pp64), static_cast<C*>(a.uprev), a.have_prev,
                     a.red_part);
  return hipGetLastError();
}

template <class L, typename S>
static hipError_t moments_t(const StepArgs& a, uint32_t c0, uint32_t count, double* out) {
  using C = typename StepT<S>::type;
  const uint32_t nb = (count + BLOCK - 1) / BLOCK;
  hipLaunchKernelGGL((k_moments<L, S>), dim3(nb), dim3(BLOCK), 0, a.stream, a.geo, static_cast<const S*>(a.src),
                     static_cast<const C*>(a.wp_src), static_cast<const LatConsts<double>*>(a.lc64),
                     static_cast<const ProbParams<double>*>(a.pp64), c0, count, out);
  return hipGetLastError();
}

template <class L, typename S>
static hipError_t init_t(const StepArgs& a, double r, const double* rho, const double* u, const double* T,
                         const double* noise, double amp, uint32_t c0, uint32_t count) {
  const uint32_t nb = (count + BLOCK - 1) / BLOCK;
  hipLaunchKernelGGL((k_init<L, S>), dim3(nb), dim3(BLOCK), 0, a.stream, a.geo, static_cast<S*>(a.dst), r, rho, u,
                     T, noise, amp, c0, count);
  return hipGetLastError();
}

template <class L, typename S>
static hipError_t partials_t(const StepArgs& a) {
  using C = typename StepT<S>::type;
  const uint32_t n = 6u * a.geo.ncols;
  const uint32_t nb = (n + BLOCK - 1) / BLOCK;
  hipLaunchKernelGGL((k_wall_partials<L, S>), dim3(nb), dim3(BLOCK), 0, a.stream, a.geo,
                     static_cast<const S*>(a.src), static_cast<const LatConsts<C>*>(a.lc), static_cast<C*>(a.wp_dst));
  return hipGetLastError();
}

#define ESBGK_DISPATCH(velset, storage, CALL)             \
  do {                                                    \
    if (velset == 1) {                                    \
      using L = D2Q37;                                    \
      if (storage == 0) { using S = double; return CALL; }   \
      if (storage == 1) { using S = float; return CALL; }    \
      if (storage == 2) { using S = _Float16; return CALL; } \
    } else if (velset == 2) {                             \
      using L = D3Q39;                                    \
      if (storage == 0) { using S = double; return CALL; }   \
      if (storage == 1) { using S = float; return CALL; }    \
      if (storage == 2) { using S = _Float16; return CALL; } \
    }                                                     \
    return hipErrorInvalidValue;                          \
  } while (0)

hipError_t launch_step(int velset, int storage, const StepArgs& a) {
  ESBGK_DISPATCH(velset, storage, (step_t<L, S>(a)));
}

hipError_t launch_pair_step(int velset, int storage, int phase, const StepArgs& a) {
  if (phase == 1) ESBGK_DISPATCH(velset, storage, (pair_t<L, S, 1>(a)));
  ESBGK_DISPATCH(velset, storage, (pair_t<L, S, 2>(a)));
}

hipError_t launch_reduce(int velset, int storage, const StepArgs& a) {
  ESBGK_DISPATCH(velset, storage, (reduce_t<L, S>(a)));
}

// ---- reductions without a workspace ----------------------------------------

// Device memory of the workspace-free reduction: the partials of at most
// NOALLOC_PARTS workgroups, then the NRED final sums. One copy per GPU,
// shared by every call on that GPU, for the life of the process.
static __device__ __align__(256) double scratch[NOALLOC_PARTS * NRED + NRED];

namespace {
constexpr int MAX_DEVICES = 64;
std::mutex g_scratch_mu;
double* g_scratch[MAX_DEVICES] = {};
}  // namespace

hipError_t noalloc_scratch(int device, double** out) {
  *out = nullptr;
  if (device < 0 || device >= MAX_DEVICES) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch[device]) {
    int cur = -1;
    hipError_t e = hipGetDevice(&cur);
    if (e != hipSuccess) return e;
    if (cur != device && (e = hipSetDevice(device)) != hipSuccess) return e;
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (cur != device) {
      const hipError_t r = hipSetDevice(cur);
      if (e == hipSuccess) e = r;
    }
    if (e != hipSuccess) return e;
    if (!p) return hipErrorInvalidSymbol;
    g_scratch[device] = static_cast<double*>(p);
  }
  *out = g_scratch[device];
  return hipSuccess;
}

template <class L, typename S>
static hipError_t reduce_fold_t(const StepArgs& a, double* scr) {
  using C = typename StepT<S>::type;
  const uint32_t nb = slot_blocks(a.geo);
  const uint32_t parts = nb < uint32_t(NOALLOC_PARTS) ? nb : uint32_t(NOALLOC_PARTS);
  hipLaunchKernelGGL((k_reduce_fold<L, S>), dim3(parts), dim3(BLOCK), 0, a.stream, a.geo,
                     static_cast<const S*>(a.src), static_cast<const C*>(a.wp_src),
                     static_cast<const LatConsts<double>*>(a.lc64), static_cast<const ProbParams<double>*>(a.pp64),
                     static_cast<C*>(a.uprev), a.have_prev, nb, scr);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_reduce_finalize, dim3(1), dim3(BLOCK), 0, a.stream, scr, parts,
                     scr + size_t(NOALLOC_PARTS) * NRED);
  return hipGetLastError();
}

hipError_t launch_reduce_noalloc(int velset, int storage, const StepArgs& a, double* scr) {
  ESBGK_DISPATCH(velset, storage, (reduce_fold_t<L, S>(a, scr)));
}

hipError_t launch_reduce_finalize(const double* part, uint32_t nparts, double* out, hipStream_t stream) {
  hipLaunchKernelGGL(k_reduce_finalize, dim3(1), dim3(BLOCK), 0, stream, part, nparts, out);
  return hipGetLastError();
}

hipError_t launch_moments(int velset, int storage, const StepArgs& a, uint32_t c0, uint32_t count, double* out) {
  ESBGK_DISPATCH(velset, storage, (moments_t<L, S>(a, c0, count, out)));
}

hipError_t launch_init(int velset, int storage, const StepArgs& a, double r, const double* rho, const double* u,
                       const double* T, const double* noise, double amp, uint32_t c0, uint32_t count) {
  ESBGK_DISPATCH(velset, storage, (init_t<L, S>(a, r, rho, u, T, noise, amp, c0, count)));
}

hipError_t launch_wall_partials(int velset, int storage, const StepArgs& a) {
  ESBGK_DISPATCH(velset, storage, (partials_t<L, S>(a)));
}

template <class L>
static hipError_t wall_tables_t(const WallProgram* prog, const void* lc64, void* pp64, void* pp32, int64_t* level,
                                int advance, hipStream_t stream) {
  hipLaunchKernelGGL(k_wall_tables<L>, dim3(1), dim3(64), 0, stream, prog,
                     static_cast<const LatConsts<double>*>(lc64), static_cast<ProbParams<double>*>(pp64),
                     static_cast<ProbParams<float>*>(pp32), level, advance);
  return hipGetLastError();
}

hipError_t launch_wall_tables(int velset, const WallProgram* prog, const void* lc64, void* pp64, void* pp32,
                              int64_t* level, int advance, hipStream_t stream) {
  if (velset == 1) return wall_tables_t<D2Q37>(prog, lc64, pp64, pp32, level, advance, stream);
  if (velset == 2) return wall_tables_t<D3Q39>(prog, lc64, pp64, pp32, level, advance, stream);
  return hipErrorInvalidValue;
}

}  // namespace esbgk
