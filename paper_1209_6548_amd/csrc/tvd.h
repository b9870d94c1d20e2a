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
  const void* gc;    // GHConsts<C>*    of the compute type (the set's P entries used)
  const void* lc;    // LatConsts<C>*   (w, r = 1)
  const void* pp;    // ProbParams<C>*  (Euler: hs = hsdt = 0)
  const void* gc64;  // FP64 blocks for the read-out and init kernels
  const void* lc64;
  const void* pp64;
  const void* msrc;  // D3Q216: raw moment sums of src (compute type, [MOM3][nslices * ipad])
  void* mdst;        // D3Q216: raw moment sums of dst, written by the step and the walls
  hipStream_t stream;
};

// Diffuse walls of the TVD scheme (Sec. 3.2) on the first (side 0, inward
// normal +y) and last (side 1, normal -y) node rows:
//   kin[s][a]  |c.n| w_a / sum_{c.n>0} |c.n| S_a for the velocities moving
//              toward wall s (c.n < 0), 0 for the others
//   k0[s]      the sum of kin[s][.], so that rho_W = k0 + sum_a kin h_a
//              over the first node off the wall
//   sw[s][a]   S_a(T_W, u_W) / w_a for the velocities moving into the gas
//              (the wall node's new h_a is rho_W sw - 1), 0 for the others
template <typename C>
struct TVDWalls {
  C kin[2][64];
  C k0[2];
  C sw[2][64];
};

// velset: ESBGK_D2Q16GH / ESBGK_D2Q36GH / ESBGK_D2Q64GH; storage: 0 FP64,
// 1 FP32, 2 FP16.
hipError_t launch_tvd_step(int velset, int storage, const TVDArgs& a);
// Re-emission at both walls into a.dst (the level just written by the step).
hipError_t launch_tvd_walls(int velset, int storage, const TVDArgs& a, const void* walls);
hipError_t launch_tvd_init(int velset, int storage, const TVDArgs& a, const double* c, const double* rho,
                           const double* u, const double* T, const double* noise, double amp, uint32_t c0,
                           uint32_t count);
hipError_t launch_tvd_moments(int velset, int storage, const TVDArgs& a, uint32_t c0, uint32_t count, double* out);

// The 3-D set D3Q216 (walls across z); as TVDWalls with 216 velocities.
template <typename C>
struct TVDWalls3 {
  C kin[2][216];
  C k0[2];
  C sw[2][216];
};

// Raw moment sums stored per cell beside each D3Q216 level (see Moments3):
// drho, J[3], S2[6], S3[10], as [MOM3][nslices * ipad] of the compute type.
constexpr int MOM3 = 20;

// One step from a.src (moments a.msrc) into a.dst (moments a.mdst).
hipError_t launch_tvd3_step(int storage, const TVDArgs& a);
// Re-emission at both walls into a.dst, and the wall cells' moments into a.mdst.
hipError_t launch_tvd3_walls(int storage, const TVDArgs& a, const void* walls);
// The moment sums of the level pop into mom (after the level was set from outside).
hipError_t launch_tvd3_rawmom(int storage, const TVDArgs& a, const void* pop, void* mom);
// c[216][3]; u is [3][count]; noise [216][count].
hipError_t launch_tvd3_init(int storage, const TVDArgs& a, const double* c, const double* rho, const double* u,
                            const double* T, const double* noise, double amp, uint32_t c0, uint32_t count);
// writes [14][count]
hipError_t launch_tvd3_moments(int storage, const TVDArgs& a, uint32_t c0, uint32_t count, double* out);

}  // namespace esbgk
