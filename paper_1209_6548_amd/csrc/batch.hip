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

#include <hip/hip_runtime.h>

#include "batch.h"
#include "stream.h"

namespace esbgk {

template <class L, typename S, typename C>
__device__ __forceinline__ void batch_cell(const BatchProblem& bp, uint32_t cell, const S* __restrict__ srcb,
                                           S* __restrict__ dstb, const C* __restrict__ wpsb, C* __restrict__ wpdb,
                                           const LatConsts<C>* __restrict__ lc,
                                           const ProbParams<C>* __restrict__ pp) {
  const Geometry& geo = bp.geo;
  const S* src = srcb + bp.pop_off;
  S* dst = dstb + bp.pop_off;
  const C* wps = wpsb + bp.wp_off;
  C* wpd = wpdb + bp.wp_off;
  const CellPos p = cell_pos(cell, geo);
  C h[L::Q];
  gather_lane<L, S, C, C, uint32_t>(h, src, geo, p, wps, pp);
  CellState<L, C> st;
  collide<L, C>(h, lc, pp, st);
  const uint32_t elem = uint32_t(cell_elem<L>(p, geo));
#pragma unroll
  for (int a = 0; a < L::Q; ++a) dst[a * geo.pstride + elem] = narrow<S, C>(h[a]);
  write_wall_partials<L, S, C>([&](int a) { return narrow<S, C>(h[a]); }, p, geo, lc, wpd);
}

template <class L, typename S, typename C, int MAXT>
__global__ void __launch_bounds__(MAXT)
k_batch(const BatchProblem* __restrict__ probs, const ProbParams<C>* __restrict__ pps,
        const uint32_t* __restrict__ bin_first, const uint32_t* __restrict__ order, S* __restrict__ bufA,
        S* __restrict__ bufB, C* __restrict__ wpA, C* __restrict__ wpB, const LatConsts<C>* __restrict__ lc,
        int64_t nsteps, int parity) {
  __shared__ uint32_t cum[BATCH_MAX_PER_BIN + 1];
  __shared__ uint32_t pid[BATCH_MAX_PER_BIN];
  const uint32_t p0 = bin_first[blockIdx.x], p1 = bin_first[blockIdx.x + 1];
  const uint32_t np = p1 - p0;
  // slots of the bin: each problem's cells start on a multiple of 64, so that
  // every wavefront's 64 slots lie in one problem, whose descriptor and
  // parameter block the wavefront then reads as scalars
  if (threadIdx.x == 0) {
    uint32_t acc = 0;
    for (uint32_t k = 0; k < np; ++k) {
      const uint32_t id = order[p0 + k];
      pid[k] = id;
      cum[k] = acc;
      acc += (probs[id].geo.ncells + 63u) & ~63u;
    }
    cum[np] = acc;
  }
  __syncthreads();
  const uint32_t total = cum[np];
  const uint32_t lane = threadIdx.x & 63u;
  for (int64_t s = 0; s < nsteps; ++s) {
    const bool odd = ((s + parity) & 1) != 0;
    const S* src = odd ? bufB : bufA;
    S* dst = odd ? bufA : bufB;
    const C* wps = odd ? wpB : wpA;
    C* wpd = odd ? wpA : wpB;
    for (uint32_t t0 = __builtin_amdgcn_readfirstlane(threadIdx.x & ~63u); t0 < total; t0 += blockDim.x) {
      uint32_t k = 0, hi = np;   // cum[k] <= t0 < cum[k + 1]
      while (hi - k > 1) {
        const uint32_t mid = (k + hi) >> 1;
        if (__builtin_amdgcn_readfirstlane(cum[mid]) <= t0) k = mid;
        else hi = mid;
      }
      const uint32_t id = __builtin_amdgcn_readfirstlane(pid[k]);
      const uint32_t cell = t0 - __builtin_amdgcn_readfirstlane(cum[k]) + lane;
      if (cell < probs[id].geo.ncells) batch_cell<L, S, C>(probs[id], cell, src, dst, wps, wpd, lc, pps + id);
    }
    __syncthreads();
  }
}

template <class L, typename S, typename C>
static hipError_t batch_t(const BatchLaunch& a) {
  constexpr int MAXT = batch_max_threads(sizeof(S));
  if (a.threads > uint32_t(MAXT) || a.threads % 64) return hipErrorInvalidValue;
  hipLaunchKernelGGL((k_batch<L, S, C, MAXT>), dim3(a.nbins), dim3(a.threads), 0, a.stream, a.probs,
                     static_cast<const ProbParams<C>*>(a.pps), a.bin_first, a.order, static_cast<S*>(a.bufA),
                     static_cast<S*>(a.bufB), static_cast<C*>(a.wpA), static_cast<C*>(a.wpB),
                     static_cast<const LatConsts<C>*>(a.lc), a.nsteps, a.parity);
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

}  // namespace esbgk
