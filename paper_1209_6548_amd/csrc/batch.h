// Batched channels: per-problem descriptors and the persistent-kernel launcher.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "params.h"

namespace esbgk {

// Largest workgroup of the persistent kernel: FP32 and FP16 storage fit
// 1024 threads (128 VGPRs; three values outside the per-cell work spill to
// scratch), FP64 256.
constexpr int batch_max_threads(size_t storage_bytes) {
  return storage_bytes == 8 ? 256 : 1024;
}
constexpr int BATCH_MAX_PER_BIN = 64;

struct BatchProblem {
  Geometry geo;
  uint64_t pop_off;    // element offset of the problem's [Q][cells] block
  uint64_t cell_off;   // first cell of the problem in the batch's cell numbering (u_prev: [D][cells] from D*cell_off)
  uint32_t wp_off;     // element offset of its wall partial sums [2][3][ncols]
  uint32_t chunk_off;  // first 64-cell chunk of the problem (reduction partials)
};

// FP64 reductions of the batch (per problem, NRED sums each):
//   level      device step counter: the level the next launch starts from
//   R          fuse the reductions into the steps from levels R-1, 2R-1, ...
//              (0: never)
//   uprev      [D][cells] per problem (compute type): u of the problem's
//              previous reduction, for the residual
//   chunks     [chunks][NRED]: wavefront partials of 64-cell chunks
//   out        [problems][NRED]: sums of the latest reduction
//   red_level  [problems]: level of the latest reduction (-1: none since the
//              state was set)
struct BatchRed {
  const int64_t* level;
  int64_t R;
  void* uprev;
  double* chunks;
  double* out;
  int64_t* red_level;
};

// A bin holds pieces: piece j of the bin table is problem order[j], cells
// [piece_c0[j], piece_c0[j] + piece_n[j]) (piece_c0 a multiple of 64). With
// whole problems (split = 0) every piece is a whole problem and one launch
// advances nsteps steps; with split problems (split = 1) a problem's pieces
// may lie in several bins, so a launch advances one step and the
// per-problem sums of a reduction are added by k_batch_sum afterwards.
struct BatchLaunch {
  const BatchProblem* probs;
  const void* pps;            // ProbParams<C>[n]
  const uint32_t* bin_first;  // [nbins + 1] into order
  const uint32_t* order;      // problem id of each piece, grouped by bin
  const uint32_t* piece_c0;   // first cell of each piece
  const uint32_t* piece_n;    // cells of each piece
  int split;
  uint32_t nprob;
  void* bufA;                 // the state of an even level is in A, of an odd level in B
  void* bufB;
  void* wpA;
  void* wpB;
  const void* lc;
  int64_t nsteps;
  BatchRed red;
  uint32_t nbins, threads;
  hipStream_t stream;
};

// The persistent step kernel (nsteps steps from level *red.level; one with
// split problems), the per-problem reduction sums when split, then the level
// advanced by nsteps.
hipError_t launch_batch(int velset, int storage, const BatchLaunch& a);
// FP64 reductions of every problem at the current level (*red.level) from the
// stored state (no step), recorded as at level `level`; pps/lc are the FP64
// parameter blocks.
hipError_t launch_batch_reduce(int velset, int storage, const BatchLaunch& a, const void* pps64,
                               const void* lc64, int64_t level);

}  // namespace esbgk
