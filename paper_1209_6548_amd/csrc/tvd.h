// Launchers of the kernels of the paper's own scheme (Sec. 3.1) on the 6-point
// Gauss-Hermite product set (internal interface between tvd.hip and
// tvd_api.cpp).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "params.h"

namespace esbgk {

struct TVDArgs {
  Geometry geo;
  const void* src;   // populations read (storage type, slice layout)
  void* dst;         // populations written
  const void* gc;    // GHConsts<C>*    of the compute type
  const void* lc;    // LatConsts<C>*   (w, r = 1)
  const void* pp;    // ProbParams<C>*  (Euler: hs = hsdt = 0)
  const void* gc64;  // FP64 blocks for the read-out and init kernels
  const void* lc64;
  const void* pp64;
  hipStream_t stream;
};

hipError_t launch_tvd_step(int storage, const TVDArgs& a);
hipError_t launch_tvd_init(int storage, const TVDArgs& a, const double* c, const double* rho, const double* u,
                           const double* T, const double* noise, double amp, uint32_t c0, uint32_t count);
hipError_t launch_tvd_moments(int storage, const TVDArgs& a, uint32_t c0, uint32_t count, double* out);

}  // namespace esbgk
