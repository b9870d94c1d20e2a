// Launchers of the HIP kernels (internal interface between the C ABI runtime
// and kernels.hip / batch.hip).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "params.h"

namespace esbgk {

struct StepArgs {
  Geometry geo;
  const void* src;      // populations read (storage type)
  void* dst;            // populations written
  const void* wp_src;   // wall partial sums read   [2 sides][3 layers][ncols]
  void* wp_dst;         // wall partial sums written
  const void* lc;       // LatConsts<C>*  of the step's compute type (device)
  const void* pp;       // ProbParams<C>* of the step's compute type (device)
  const void* lc64;     // LatConsts<double>*  (moments and explicit reductions)
  const void* pp64;     // ProbParams<double>*
  void* uprev;          // [D][ncells] velocity of the previous reduction (compute type)
  int have_prev;
  int reduce;           // step kernel: fuse the reductions
  int rev;              // step kernel: walk the tiles in reverse order
  double* red_part;     // [workgroups][NRED]
  hipStream_t stream;
};

// Workgroups of the step and reduction kernels (one FP64 partial each in
// red_part).
uint32_t slot_blocks(const Geometry& g);
hipError_t launch_step(int velset, int storage, const StepArgs& a);
// Step `phase` (1 or 2) of the in-place pair on the buffer a.dst (a.src is
// not used); wall partial sums from a.wp_src to a.wp_dst as launch_step.
hipError_t launch_pair_step(int velset, int storage, int phase, const StepArgs& a);
hipError_t launch_reduce(int velset, int storage, const StepArgs& a);
hipError_t launch_reduce_finalize(const double* part, uint32_t nparts, double* out, hipStream_t stream);
hipError_t launch_moments(int velset, int storage, const StepArgs& a, uint32_t c0, uint32_t count, double* out);
hipError_t launch_init(int velset, int storage, const StepArgs& a, double r, const double* rho, const double* u,
                       const double* T, const double* noise, double amp, uint32_t c0, uint32_t count);
hipError_t launch_wall_partials(int velset, int storage, const StepArgs& a);

// Reductions that use no workspace: the partials of at most NOALLOC_PARTS
// workgroups and the NRED sums live in a static device array of
// kernels.hip (one per GPU). noalloc_scratch gives that GPU's address
// (looked up once per device with the device current); the sums land at
// scr + NOALLOC_PARTS * NRED.
constexpr int NOALLOC_PARTS = 1024;
hipError_t noalloc_scratch(int device, double** scr);
hipError_t launch_reduce_noalloc(int velset, int storage, const StepArgs& a, double* scr);
// Rebuild the wall tables of pp64 (and of pp32 when not null) for the step
// from the level held in *level; advance: then increment *level.
hipError_t launch_wall_tables(int velset, const WallProgram* prog, const void* lc64, void* pp64, void* pp32,
                              int64_t* level, int advance, hipStream_t stream);

}  // namespace esbgk
