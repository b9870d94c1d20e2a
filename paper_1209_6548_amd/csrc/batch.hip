// Persistent kernel for batches of independent channel problems.
//
// The host packs the problems into bins of roughly equal cell count (longest
// problem first, each into the currently lightest bin); one workgroup owns one
// bin for the whole launch. Within a step every wavefront takes 64 slots of
// the bin in turn (slots -> problem through a prefix table in LDS, problems
// starting on multiples of 64 slots), and each lane pulls, collides
// and stores exactly as the single-lattice kernel does, with the problem's
// own geometry and parameter block; a workgroup barrier separates steps, so
// the bin advances n steps in one launch with no host round trip. The
// barrier's workgroup-scope release/acquire makes the global-memory writes of
// one step visible to every wave of the workgroup in the next.
//
// FP64 reductions. A step from a level that is one less than a multiple of R
// also sums, per problem, the FP64 contributions of its cells' reconstructed
// state (mass, energy, momentum, residual terms): each wavefront reduces its
// 64-cell chunk with a butterfly and writes the chunk's partial; after the
// step's barrier one thread per problem adds the problem's chunk partials in
// chunk order. Every problem belongs to one workgroup, so the sums need no
// atomics and do not depend on the scheduling: they are deterministic.
//
// Split problems. A batch of few large problems would leave most compute
// units idle, so the host can cut problems into pieces of whole 64-cell
// chunks and spread them over the bins. A step then needs every piece of a
// problem done before the next one starts: each launch advances one step,
// and k_batch_sum adds the chunk partials of every problem afterwards, in
// the same chunk order (the same bits as whole problems).

#include <hip/hip_runtime.h>

#include "batch.h"
#include "reduce.h"
#include "stream.h"

namespace esbgk {

template <class L, typename S, typename C>
__device__ __forceinline__ void batch_cell(const BatchProblem& bp, uint32_t cell, const S* __restrict__ srcb,
                                           S* __restrict__ dstb, const C* __restrict__ wpsb, C* __restrict__ wpdb,
                                           const LatConsts<C>* __restrict__ lc,
                                           const ProbParams<C>* __restrict__ pp, CellState<L, C>& st) {
  const Geometry& geo = bp.geo;
  const S* src = srcb + bp.pop_off;
  S* dst = dstb + bp.pop_off;
  const C* wps = wpsb + bp.wp_off;
  C* wpd = wpdb + bp.wp_off;
  const CellPos p = cell_pos(cell, geo);
  C h[L::Q];
  gather_lane<L, S, C, C, uint32_t>(h, src, geo, p, wps, pp);
  S hs[L::Q];
  collide_to<L, C, S>(h, hs, lc, pp, st);
  const uint32_t elem = uint32_t(cell_elem<L>(p, geo));
#pragma unroll
  for (int a = 0; a < L::Q; ++a) dst[a * geo.pstride + elem] = hs[a];
  write_wall_partials<L, S, C>([&](int a) { return hs[a]; }, p, geo, lc, wpd);
}

// Bin bookkeeping shared by the step and reduction kernels: the pieces of
// the workgroup's bin, their first thread slots (multiples of 64) and their
// first cells.
struct BinTable {
  uint32_t cum[BATCH_MAX_PER_BIN + 1];
  uint32_t pid[BATCH_MAX_PER_BIN];
  uint32_t c0[BATCH_MAX_PER_BIN];
};

__device__ __forceinline__ uint32_t load_bin(BinTable& bt, const uint32_t* __restrict__ bin_first,
                                             const uint32_t* __restrict__ order,
                                             const uint32_t* __restrict__ piece_c0,
                                             const uint32_t* __restrict__ piece_n) {
  const uint32_t p0 = bin_first[blockIdx.x], p1 = bin_first[blockIdx.x + 1];
  const uint32_t np = p1 - p0;
  if (threadIdx.x == 0) {
    uint32_t acc = 0;
    for (uint32_t k = 0; k < np; ++k) {
      bt.pid[k] = order[p0 + k];
      bt.c0[k] = piece_c0[p0 + k];
      bt.cum[k] = acc;
      acc += (piece_n[p0 + k] + 63u) & ~63u;
    }
    bt.cum[np] = acc;
  }
  __syncthreads();
  return np;
}

// Index k of the bin's piece whose slots hold t0 (cum[k] <= t0 < cum[k+1]);
// t0 is wavefront-uniform, so the search runs on scalars.
__device__ __forceinline__ uint32_t find_problem(const BinTable& bt, uint32_t np, uint32_t t0) {
  uint32_t k = 0, hi = np;
  while (hi - k > 1) {
    const uint32_t mid = (k + hi) >> 1;
    if (uint32_t(__builtin_amdgcn_readfirstlane(bt.cum[mid])) <= t0) k = mid;
    else hi = mid;
  }
  return k;
}

// Butterfly over the wavefront; lane 0 writes the chunk's NRED partials.
__device__ __forceinline__ void write_chunk(double (&v)[NRED], double* __restrict__ dst) {
#pragma unroll
  for (int k = 0; k < NRED; ++k) v[k] = wave_sum(v[k]);
  if ((threadIdx.x & 63u) == 0) {
#pragma unroll
    for (int k = 0; k < NRED; ++k) dst[k] = v[k];
  }
}

// The chunk partials of problem id added in chunk order.
__device__ __forceinline__ void sum_problem(uint32_t id, const BatchProblem* __restrict__ probs, const BatchRed& red,
                                            int64_t level) {
  const BatchProblem& bp = probs[id];
  const uint32_t nch = (bp.geo.ncells + 63u) >> 6;
  double acc[NRED];
#pragma unroll
  for (int k = 0; k < NRED; ++k) acc[k] = 0.0;
  for (uint32_t c = 0; c < nch; ++c) {
    const double* q = red.chunks + size_t(bp.chunk_off + c) * NRED;
#pragma unroll
    for (int k = 0; k < NRED; ++k) acc[k] += q[k];
  }
#pragma unroll
  for (int k = 0; k < NRED; ++k) red.out[size_t(id) * NRED + k] = acc[k];
  red.red_level[id] = level;
}

// After the barrier that follows the chunk writes (whole problems): thread
// k < np adds the chunk partials of the bin's k-th problem.
__device__ __forceinline__ void sum_problems(const BinTable& bt, uint32_t np, const BatchProblem* __restrict__ probs,
                                             const BatchRed& red, int64_t level) {
  if (threadIdx.x < np) sum_problem(bt.pid[threadIdx.x], probs, red, level);
}

// Split problems: after the step launch from level *red.level (or, with
// fixed >= 0, the explicit reduction at that level), thread i adds problem
// i's chunk partials when that step carried a reduction.
__global__ void __launch_bounds__(256)
k_batch_sum(const BatchProblem* __restrict__ probs, BatchRed red, uint32_t nprob, int64_t fixed) {
  const uint32_t i = blockIdx.x * 256u + threadIdx.x;
  if (i >= nprob) return;
  if (fixed >= 0) {
    sum_problem(i, probs, red, fixed);
    return;
  }
  const int64_t lev = *red.level;
  if (red.R > 0 && (lev + 1) % red.R == 0) sum_problem(i, probs, red, lev);
}

template <class L, typename S, typename C, int MAXT>
__global__ void __launch_bounds__(MAXT)
k_batch(const BatchProblem* __restrict__ probs, const ProbParams<C>* __restrict__ pps,
        const uint32_t* __restrict__ bin_first, const uint32_t* __restrict__ order,
        const uint32_t* __restrict__ piece_c0, const uint32_t* __restrict__ piece_n, int split, S* __restrict__ bufA,
        S* __restrict__ bufB, C* __restrict__ wpA, C* __restrict__ wpB, const LatConsts<C>* __restrict__ lc,
        int64_t nsteps, BatchRed red) {
  __shared__ BinTable bt;
  const uint32_t np = load_bin(bt, bin_first, order, piece_c0, piece_n);
  const uint32_t total = bt.cum[np];
  const uint32_t lane = threadIdx.x & 63u;
  const int64_t level0 = *red.level;
  C* uprev = static_cast<C*>(red.uprev);
  for (int64_t s = 0; s < nsteps; ++s) {
    const int64_t lev = level0 + s;
    const bool odd = (lev & 1) != 0;
    const bool rstep = red.R > 0 && (lev + 1) % red.R == 0;
    const S* src = odd ? bufB : bufA;
    S* dst = odd ? bufA : bufB;
    const C* wps = odd ? wpB : wpA;
    C* wpd = odd ? wpA : wpB;
    for (uint32_t t0 = __builtin_amdgcn_readfirstlane(threadIdx.x & ~63u); t0 < total; t0 += blockDim.x) {
      const uint32_t k = find_problem(bt, np, t0);
      const uint32_t id = __builtin_amdgcn_readfirstlane(bt.pid[k]);
      const uint32_t first = __builtin_amdgcn_readfirstlane(bt.cum[k]);
      // the piece's cells are whole 64-cell chunks but for a problem's last
      // piece, whose slots past the problem's end stay idle
      const uint32_t chunk0 = __builtin_amdgcn_readfirstlane(bt.c0[k]) + (t0 - first);
      const uint32_t cell = chunk0 + lane;
      const BatchProblem& bp = probs[id];
      double v[NRED];
#pragma unroll
      for (int q = 0; q < NRED; ++q) v[q] = 0.0;
      if (cell < bp.geo.ncells) {
        CellState<L, C> st;
        batch_cell<L, S, C>(bp, cell, src, dst, wps, wpd, lc, pps + id, st);
        if (rstep)
          cell_contrib<L, C, C>(st, uprev + size_t(L::D) * bp.cell_off, cell, bp.geo.ncells,
                                red.red_level[id] >= 0, v);
      }
      if (rstep) write_chunk(v, red.chunks + size_t(bp.chunk_off + (chunk0 >> 6)) * NRED);
    }
    __syncthreads();
    if (rstep && !split) {
      sum_problems(bt, np, probs, red, lev);
      __syncthreads();
    }
  }
}

// FP64 reductions of the stored state of level `level` (no step): FP64
// pull and reconstruction, as the single-lattice read-out kernels.
template <class L, typename S, typename P, int MAXT>
__global__ void __launch_bounds__(MAXT)
k_batch_reduce(const BatchProblem* __restrict__ probs, const ProbParams<double>* __restrict__ pps,
               const uint32_t* __restrict__ bin_first, const uint32_t* __restrict__ order,
               const uint32_t* __restrict__ piece_c0, const uint32_t* __restrict__ piece_n, int split,
               const S* __restrict__ bufA, const S* __restrict__ bufB, const P* __restrict__ wpA,
               const P* __restrict__ wpB, const LatConsts<double>* __restrict__ lc, BatchRed red, int64_t level) {
  __shared__ BinTable bt;
  const uint32_t np = load_bin(bt, bin_first, order, piece_c0, piece_n);
  const uint32_t total = bt.cum[np];
  const uint32_t lane = threadIdx.x & 63u;
  const bool odd = (level & 1) != 0;
  const S* srcb = odd ? bufB : bufA;
  const P* wpsb = odd ? wpB : wpA;
  P* uprev = static_cast<P*>(red.uprev);
  for (uint32_t t0 = __builtin_amdgcn_readfirstlane(threadIdx.x & ~63u); t0 < total; t0 += blockDim.x) {
    const uint32_t k = find_problem(bt, np, t0);
    const uint32_t id = __builtin_amdgcn_readfirstlane(bt.pid[k]);
    const uint32_t first = __builtin_amdgcn_readfirstlane(bt.cum[k]);
    const uint32_t chunk0 = __builtin_amdgcn_readfirstlane(bt.c0[k]) + (t0 - first);
    const uint32_t cell = chunk0 + lane;
    const BatchProblem& bp = probs[id];
    double v[NRED];
#pragma unroll
    for (int q = 0; q < NRED; ++q) v[q] = 0.0;
    if (cell < bp.geo.ncells) {
      const CellPos p = cell_pos(cell, bp.geo);
      double h[L::Q];
      gather_lane<L, S, double, P, uint32_t>(h, srcb + bp.pop_off, bp.geo, p, wpsb + bp.wp_off, pps + id);
      RawMoments<L, double> m;
      raw_moments<L, double>(h, lc, false, m);
      CellState<L, double> st;
      reconstruct<L, double>(m, lc, pps + id, st);
      cell_contrib<L, double, P>(st, uprev + size_t(L::D) * bp.cell_off, cell, bp.geo.ncells,
                                 red.red_level[id] >= 0, v);
    }
    write_chunk(v, red.chunks + size_t(bp.chunk_off + (chunk0 >> 6)) * NRED);
  }
  if (split) return;   // k_batch_sum adds them
  __syncthreads();
  sum_problems(bt, np, probs, red, level);
}

// Move the device level on by n after a launch (one thread).
__global__ void k_batch_advance(int64_t* __restrict__ level, int64_t n) {
  if (threadIdx.x == 0 && blockIdx.x == 0) *level += n;
}

template <class L, typename S, typename C>
static hipError_t batch_t(const BatchLaunch& a) {
  constexpr int MAXT = batch_max_threads(sizeof(S));
  if (a.threads > uint32_t(MAXT) || a.threads % 64) return hipErrorInvalidValue;
  if (a.split && a.nsteps != 1) return hipErrorInvalidValue;   // split problems: one step per launch
  hipLaunchKernelGGL((k_batch<L, S, C, MAXT>), dim3(a.nbins), dim3(a.threads), 0, a.stream, a.probs,
                     static_cast<const ProbParams<C>*>(a.pps), a.bin_first, a.order, a.piece_c0, a.piece_n,
                     a.split, static_cast<S*>(a.bufA), static_cast<S*>(a.bufB), static_cast<C*>(a.wpA),
                     static_cast<C*>(a.wpB), static_cast<const LatConsts<C>*>(a.lc), a.nsteps, a.red);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  if (a.split && a.red.R > 0) {
    hipLaunchKernelGGL(k_batch_sum, dim3((a.nprob + 255) / 256), dim3(256), 0, a.stream, a.probs, a.red, a.nprob,
                       int64_t(-1));
    e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  hipLaunchKernelGGL(k_batch_advance, dim3(1), dim3(64), 0, a.stream, const_cast<int64_t*>(a.red.level), a.nsteps);
  return hipGetLastError();
}

// The reduction kernel runs FP64 arithmetic: workgroups of 256 threads keep
// it free of scratch (any workgroup size covers a bin).
constexpr int BATCH_REDUCE_THREADS = 256;

template <class L, typename S, typename C>
static hipError_t batch_reduce_t(const BatchLaunch& a, const void* pps64, const void* lc64, int64_t level) {
  constexpr int T = BATCH_REDUCE_THREADS;
  static_assert(T >= BATCH_MAX_PER_BIN, "one thread per problem of a bin sums its chunks");
  hipLaunchKernelGGL((k_batch_reduce<L, S, C, T>), dim3(a.nbins), dim3(T), 0, a.stream, a.probs,
                     static_cast<const ProbParams<double>*>(pps64), a.bin_first, a.order, a.piece_c0, a.piece_n,
                     a.split, static_cast<const S*>(a.bufA), static_cast<const S*>(a.bufB),
                     static_cast<const C*>(a.wpA), static_cast<const C*>(a.wpB),
                     static_cast<const LatConsts<double>*>(lc64), a.red, level);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess || !a.split) return e;
  hipLaunchKernelGGL(k_batch_sum, dim3((a.nprob + 255) / 256), dim3(256), 0, a.stream, a.probs, a.red, a.nprob,
                     level);
  return hipGetLastError();
}

hipError_t launch_batch(int velset, int storage, const BatchLaunch& a) {
  if (velset == 1) {
    if (storage == 0) return batch_t<D2Q37, double, double>(a);
    if (storage == 1) return batch_t<D2Q37, float, float>(a);
    if (storage == 2) return batch_t<D2Q37, _Float16, float>(a);
  } else if (velset == 2) {
    if (storage == 0) return batch_t<D3Q39, double, double>(a);
    if (storage == 1) return batch_t<D3Q39, float, float>(a);
    if (storage == 2) return batch_t<D3Q39, _Float16, float>(a);
  }
  return hipErrorInvalidValue;
}

hipError_t launch_batch_reduce(int velset, int storage, const BatchLaunch& a, const void* pps64, const void* lc64,
                               int64_t level) {
  if (velset == 1) {
    if (storage == 0) return batch_reduce_t<D2Q37, double, double>(a, pps64, lc64, level);
    if (storage == 1) return batch_reduce_t<D2Q37, float, float>(a, pps64, lc64, level);
    if (storage == 2) return batch_reduce_t<D2Q37, _Float16, float>(a, pps64, lc64, level);
  } else if (velset == 2) {
    if (storage == 0) return batch_reduce_t<D3Q39, double, double>(a, pps64, lc64, level);
    if (storage == 1) return batch_reduce_t<D3Q39, float, float>(a, pps64, lc64, level);
    if (storage == 2) return batch_reduce_t<D3Q39, _Float16, float>(a, pps64, lc64, level);
  }
  return hipErrorInvalidValue;
}

}  // namespace esbgk
