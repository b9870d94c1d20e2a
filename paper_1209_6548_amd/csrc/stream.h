// Streaming (pull) with periodic wrap and diffuse-wall re-emission, shared by
// the single-lattice kernels and the batched persistent kernel.
//
// Diffuse walls (Sec. 3.2). rho_W of a wall-parallel column is the flux
// balance of the paper: the populations that cross the wall in one step
// (a population with |e_n| = k leaves from the k layers next to the wall)
// over the matching flux of S(T_w, u_w). A step writes, for every cell of the
// three layers next to a wall, the partial sum sum w h over its populations
// that cross the wall on the next step, from the values as stored; the next
// step adds the three layers of a column. A population that streams in from
// beyond a wall takes rho_W(source column) S(T_w, u_w).
#pragma once

#include <hip/hip_runtime.h>

#include "cell.h"

namespace esbgk {

__device__ __forceinline__ uint32_t fdiv(uint32_t n, FastDiv d) { return (__umulhi(n, d.m) + n) >> d.l; }

// Load / store element boff / sizeof(S) of a velocity plane. The plane base is
// uniform across the wavefront and boff is a 32-bit byte offset (planes are
// smaller than 4 GiB), so the access is a scalar-base + vector-offset
// instruction with no per-lane 64-bit address arithmetic. FP64 populations
// are stored non-temporally (measured 6% faster for FP64 on MI355X; slower
// for the narrower types, which keep the default policy).
template <typename S>
__device__ __forceinline__ S ld_plane(const S* __restrict__ plane, uint32_t boff) {
  return *reinterpret_cast<const S*>(reinterpret_cast<const char*>(plane) + boff);
}
template <typename S>
__device__ __forceinline__ void st_plane(S* __restrict__ plane, uint32_t boff, S v) {
  S* p = reinterpret_cast<S*>(reinterpret_cast<char*>(plane) + boff);
  if constexpr (sizeof(S) == 8) __builtin_nontemporal_store(v, p);
  else *p = v;
}

__device__ __forceinline__ int wrapc(int v, int n) {
  // v in [-3, n + 2], n >= 1
  if (v < 0) v += n;
  if (v < 0) v += n;
  if (v < 0) v += n;
  if (v >= n) v -= n;
  if (v >= n) v -= n;
  if (v >= n) v -= n;
  return v;
}

struct CellPos {
  int x, y, z;
};

__device__ __forceinline__ CellPos cell_pos(uint32_t cell, const Geometry& geo) {
  const uint32_t yz = fdiv(cell, geo.div_nx);
  const uint32_t x = cell - yz * geo.nx;
  const uint32_t z = fdiv(yz, geo.div_ny);
  const uint32_t y = yz - z * geo.ny;
  return {int(x), int(y), int(z)};
}

// At least 3 cells from every edge: no wrap and no wall within reach.
template <class L>
__device__ __forceinline__ bool interior(const CellPos& p, const Geometry& geo) {
  bool ok = p.x >= 3 && p.x < int(geo.nx) - 3 && p.y >= 3 && p.y < int(geo.ny) - 3;
  if (L::D == 3) ok = ok && p.z >= 3 && p.z < int(geo.nz) - 3;
  return ok;
}

// At least 3 layers from both walls (always true without walls).
template <class L>
__device__ __forceinline__ bool off_walls(const CellPos& p, const Geometry& geo) {
  if (!geo.walls) return true;
  const int cw = L::D == 2 ? p.y : p.z;
  const int nw = L::D == 2 ? int(geo.ny) : int(geo.nz);
  return cw >= 3 && cw < nw - 3;
}

// How a wavefront pulls: every lane interior (shifted plane bases, no
// per-velocity arithmetic); some lane at a periodic edge but none near a wall
// (per-lane wrapped offsets); some lane near a wall (wrapped offsets plus wall
// ghosts).
enum PullMode { PULL_FAST = 0, PULL_WRAP = 1, PULL_WALL = 2 };

template <class L>
__device__ __forceinline__ PullMode pull_mode(const CellPos& p, const Geometry& geo) {
  if (__all(interior<L>(p, geo))) return PULL_FAST;
  return __all(off_walls<L>(p, geo)) ? PULL_WRAP : PULL_WALL;
}

// Pull the Q populations that stream into cell p. P is the type of the wall
// partial sums, C the compute type.
template <class L, typename S, typename C, typename P>
__device__ __forceinline__ void gather(C (&h)[L::Q], const S* __restrict__ src, const Geometry& geo,
                                       uint32_t cell, const CellPos& p, const P* __restrict__ wp,
                                       const ProbParams<C>* __restrict__ pp, PullMode mode) {
  constexpr int D = L::D, Q = L::Q;
  if (mode == PULL_FAST) {
#pragma unroll
    for (int a = 0; a < Q; ++a) {
      const long shift = long(ecomp<L>(a, 2)) * long(geo.nxy) + long(ecomp<L>(a, 1)) * long(geo.nx) +
                         long(ecomp<L>(a, 0));
      const S* plane = src + size_t(a) * geo.ncells - shift;
      h[a] = widen<C, S>(ld_plane(plane, cell * uint32_t(sizeof(S))));
    }
    return;
  }
  // wrapped coordinates of the source for shifts -3..3, pre-scaled to element
  // offsets; along the wall axis they are left unwrapped (out of range = beyond
  // a wall)
  const int nx = int(geo.nx), ny = int(geo.ny), nz = int(geo.nz);
  const bool walls = geo.walls != 0;
  int xo[7], yo[7], zo[7];
#pragma unroll
  for (int s = -3; s <= 3; ++s) {
    xo[s + 3] = wrapc(p.x - s, nx);
    yo[s + 3] = ((D == 2 && walls) ? p.y - s : wrapc(p.y - s, ny)) * nx;
    zo[s + 3] = (D == 3) ? ((walls ? p.z - s : wrapc(p.z - s, nz)) * int(geo.nxy)) : 0;
  }
  if (mode == PULL_WRAP) {
#pragma unroll
    for (int a = 0; a < Q; ++a) {
      const uint32_t off = uint32_t(xo[ecomp<L>(a, 0) + 3] + yo[ecomp<L>(a, 1) + 3] + zo[ecomp<L>(a, 2) + 3]);
      h[a] = widen<C, S>(ld_plane(src + size_t(a) * geo.ncells, off * uint32_t(sizeof(S))));
    }
    return;
  }
  const int cw = D == 2 ? p.y : p.z;
  const int nw = D == 2 ? ny : nz;
#pragma unroll
  for (int a = 0; a < Q; ++a) {
    const int ex = ecomp<L>(a, 0), ey = ecomp<L>(a, 1), ez = ecomp<L>(a, 2);
    const int sw = cw - (D == 2 ? ey : ez);
    if (walls && (sw < 0 || sw >= nw)) {
      const int side = sw < 0 ? 0 : 1;
      const uint32_t col = uint32_t(xo[ex + 3] + (D == 2 ? 0 : yo[ey + 3]));
      const P* q = wp + uint32_t(side) * 3u * geo.ncols + col;
      const C part = C(q[0]) + C(q[geo.ncols]) + C(q[2u * geo.ncols]);
      const C drw = (side ? pp->K0[1] : pp->K0[0]) + (side ? pp->invden[1] : pp->invden[0]) * part;
      const C em1 = side ? pp->Em1[1][a] : pp->Em1[0][a];
      const C eh = side ? pp->Ehat[1][a] : pp->Ehat[0][a];
      h[a] = em1 + eh * drw;
    } else {
      const uint32_t off = uint32_t(xo[ex + 3] + yo[ey + 3] + zo[ez + 3]);
      h[a] = widen<C, S>(ld_plane(src + size_t(a) * geo.ncells, off * uint32_t(sizeof(S))));
    }
  }
}

// Sums of w h over the populations of one cell grouped by how many layers
// they cross: lo[k-1] for e_n = -k (low wall), hi[k-1] for e_n = +k. The
// values are taken as stored (S), summed in P, in velocity order.
template <class L, typename S, typename P>
struct CrossSums {
  P lo[3], hi[3];
};

template <class L, typename S, typename P, typename GetS>
__device__ __forceinline__ CrossSums<L, S, P> cross_sums(GetS stored, const LatConsts<P>* __restrict__ lw) {
  constexpr int D = L::D, Q = L::Q;
  CrossSums<L, S, P> cs;
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    cs.lo[k] = P(0);
    cs.hi[k] = P(0);
  }
#pragma unroll
  for (int a = 1; a < Q; ++a) {
    const int en = ecomp<L>(a, D - 1);
    if (en == 0) continue;
    const P v = lw->w[a] * P(stored(a));
    if (en < 0) cs.lo[-en - 1] += v;
    else cs.hi[en - 1] += v;
  }
  return cs;
}

// Partial sum of layer k (0 = next to the wall): populations with |e_n| > k.
template <typename P>
__device__ __forceinline__ P layer_partial(const P (&g)[3], int k) {
  return k == 0 ? (g[0] + g[1]) + g[2] : (k == 1 ? g[1] + g[2] : g[2]);
}

// Write the partial sums of a wall-layer cell (no-op elsewhere).
template <class L, typename S, typename P, typename GetS>
__device__ __forceinline__ void write_wall_partials(GetS stored, const CellPos& p, const Geometry& geo,
                                                    const LatConsts<P>* __restrict__ lw, P* __restrict__ wp_dst) {
  constexpr int D = L::D;
  const int cw = D == 2 ? p.y : p.z;
  const int nw = D == 2 ? int(geo.ny) : int(geo.nz);
  if (!(cw < 3 || cw >= nw - 3)) return;
  const CrossSums<L, S, P> cs = cross_sums<L, S, P>(stored, lw);
  const uint32_t col = D == 2 ? uint32_t(p.x) : uint32_t(p.y) * geo.nx + uint32_t(p.x);
  if (cw < 3) wp_dst[uint32_t(cw) * geo.ncols + col] = layer_partial(cs.lo, cw);
  if (cw >= nw - 3) {
    const int k = nw - 1 - cw;
    wp_dst[uint32_t(3 + k) * geo.ncols + col] = layer_partial(cs.hi, k);
  }
}

}  // namespace esbgk
