// FP64 reductions of a cell's reconstructed state, shared by the
// single-lattice kernels and the batched persistent kernel.
//
// Each cell contributes, in FP64, its mass rho, its energy
// 1/2 rho (u^2 + D T) (the trace of the physical second moment), its momentum
// rho u, the residual terms |u - u_prev|^2 and |u|^2, and a flag for an
// invalid cell. Sums are formed in a fixed order: a wavefront butterfly, then
// fixed-order passes over the wavefront partials, so that the result does
// not depend on the scheduling of the workgroups.
#pragma once

#include <hip/hip_runtime.h>

#include "cell.h"

namespace esbgk {

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// Per-cell contributions: mass, energy, momentum (3), |u - u_prev|^2, |u|^2,
// invalid-cell count. rho and T are formed in FP64 from their deviations.
template <class L, typename C, typename U>
__device__ __forceinline__ void cell_contrib(const CellState<L, C>& s, U* __restrict__ uprev, uint32_t cell,
                                             uint32_t ncells, int have_prev, double (&v)[NRED]) {
  constexpr int D = L::D;
  const double rho = 1.0 + double(s.drho);
  const double T = 1.0 + double(s.theta);
  double uu = 0.0, du = 0.0;
  v[0] = rho;
#pragma unroll
  for (int i = 0; i < 3; ++i) v[2 + i] = 0.0;
#pragma unroll
  for (int i = 0; i < D; ++i) {
    const double ui = double(s.u[i]);
    v[2 + i] = rho * ui;
    uu += ui * ui;
    if (uprev) {
      const double up = have_prev ? double(uprev[size_t(i) * ncells + cell]) : ui;
      du += (ui - up) * (ui - up);
      uprev[size_t(i) * ncells + cell] = U(ui);
    }
  }
  v[1] = 0.5 * (rho * uu + rho * D * T);
  v[5] = du;
  v[6] = uu;
  const bool bad = !(rho > 0.0) || !(T > 0.0) || !(uu < 1e300) || !(v[1] < 1e300);
  v[7] = bad ? 1.0 : 0.0;
}

}  // namespace esbgk
