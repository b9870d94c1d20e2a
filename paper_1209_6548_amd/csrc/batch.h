// Batched channels: per-problem descriptors and the persistent-kernel launcher.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "params.h"

namespace esbgk {

// Largest workgroup of the persistent kernel, chosen so that the kernel needs
// no scratch: FP32 and FP16 storage fit 1024 threads (at most 128 VGPRs),
// FP64 256.
constexpr int batch_max_threads(size_t storage_bytes) {
  return storage_bytes == 8 ? 256 : 1024;
}
constexpr int BATCH_MAX_PER_BIN = 64;

struct BatchProblem {
  Geometry geo;
  uint64_t pop_off;   // element offset of the problem's [Q][cells] block
  uint32_t wp_off;    // element offset of its wall partial sums [2][3][ncols]
  uint32_t pad;
};

struct BatchLaunch {
  const BatchProblem* probs;
  const void* pps;            // ProbParams<C>[n]
  const uint32_t* bin_first;  // [nbins + 1] into order
  const uint32_t* order;      // problem ids grouped by bin
  void* bufA;
  void* bufB;
  void* wpA;
  void* wpB;
  const void* lc;
  int64_t nsteps;
  int parity;                 // 0: the current state is in A; 1: in B
  uint32_t nbins, threads;
  hipStream_t stream;
};

hipError_t launch_batch(int velset, int storage, const BatchLaunch& a);

}  // namespace esbgk
