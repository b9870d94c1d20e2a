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
//
// Addressing follows the slice layout of Geometry: population alpha of the
// cell (slice s, in-slice index i) is element s sstride + alpha pstride + i.
// The wall axis, when there are walls, is the slice axis.
#pragma once

#include <hip/hip_runtime.h>

#include "cell.h"

namespace esbgk {

__device__ __forceinline__ uint32_t fdiv(uint32_t n, FastDiv d) { return (__umulhi(n, d.m) + n) >> d.l; }

// Compute type of a storage type: FP64 storage computes in FP64, FP32 and
// FP16 storage in FP32.
template <typename S>
struct StepT {
  using type = float;
};
template <>
struct StepT<double> {
  using type = double;
};

// Workgroups are dispatched round-robin over the 8 XCDs (each with its own
// L2). Give each XCD a contiguous range of tiles so that neighbouring tiles,
// which share cache lines at their edges, are served by the same L2.
__device__ __forceinline__ uint32_t xcd_block(uint32_t b, uint32_t nb) {
  const uint32_t per = nb >> 3;
  if (b < (per << 3)) return (b & 7u) * per + (b >> 3);
  return b;
}

// Tile of workgroup b for a launch that walks the tiles forward (rev = 0) or
// backward (rev = 1). Consecutive steps of a ping-pong pair alternate: the
// tiles a step wrote last are then the first its successor reads, while they
// are still held by the memory-side cache (256 MB on MI355X) - the reuse
// distance of the populations a step writes falls from a whole step's
// traffic to twice what remains of it after the tile.
__device__ __forceinline__ uint32_t tile_of(uint32_t b, uint32_t nb, int rev) {
  const uint32_t t = xcd_block(b, nb);
  return rev ? nb - 1u - t : t;
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

// Position of in-slice index i of slice s.
template <class L>
__device__ __forceinline__ CellPos slice_pos(uint32_t s, uint32_t i, const Geometry& geo) {
  if (L::D == 2) return {int(i), int(s), 0};
  const uint32_t y = fdiv(i, geo.div_nx);
  return {int(i - y * geo.nx), int(y), int(s)};
}

template <class L>
__device__ __forceinline__ int slice_of(const CellPos& p) { return L::D == 2 ? p.y : p.z; }
template <class L>
__device__ __forceinline__ uint32_t inslice_of(const CellPos& p, const Geometry& geo) {
  return L::D == 2 ? uint32_t(p.x) : uint32_t(p.y) * geo.nx + uint32_t(p.x);
}
// Element offset of a cell within one velocity plane of the layout.
template <class L>
__device__ __forceinline__ size_t cell_elem(const CellPos& p, const Geometry& geo) {
  return size_t(slice_of<L>(p)) * geo.sstride + inslice_of<L>(p, geo);
}

// At least 3 cells from every in-slice edge (no in-slice wrap within reach).
template <class L>
__device__ __forceinline__ bool inslice_interior(const CellPos& p, const Geometry& geo) {
  bool ok = p.x >= 3 && p.x < int(geo.nx) - 3;
  if (L::D == 3) ok = ok && p.y >= 3 && p.y < int(geo.ny) - 3;
  return ok;
}

// Ghost value beyond wall `side` for velocity a, from the three partial
// sums q of the source column (Sec. 3.2: rho_W(col) S_alpha(T_w, u_w),
// deviational).
template <class L, typename C, typename P>
__device__ __forceinline__ C wall_ghost_from(int a, int side, const P (&q)[3], const ProbParams<C>* __restrict__ pp) {
  const C part = C(q[0]) + C(q[1]) + C(q[2]);
  const C drw = (side ? pp->K0[1] : pp->K0[0]) + (side ? pp->invden[1] : pp->invden[0]) * part;
  const C em1 = side ? pp->Em1[1][a] : pp->Em1[0][a];
  const C eh = side ? pp->Ehat[1][a] : pp->Ehat[0][a];
  return em1 + eh * drw;
}

// The same from the partial sums of source column col in memory
// (P wp[2 sides][3 layers][ncols], layer 0 next to the wall).
template <class L, typename C, typename P>
__device__ __forceinline__ C wall_ghost(int a, int side, uint32_t col, const Geometry& geo,
                                        const P* __restrict__ wp, const ProbParams<C>* __restrict__ pp) {
  const P* q = wp + uint32_t(side) * 3u * geo.ncols + col;
  const P v[3] = {q[0], q[geo.ncols], q[2u * geo.ncols]};
  return wall_ghost_from<L, C, P>(a, side, v, pp);
}

// Source columns of the wall ghosts: used[side][cx][cy] when some velocity
// pulls across wall `side` from the column at in-slice shift (cx - 3, cy - 3)
// (cy = 3 in 2-D, where the column is the x position), and reach[.] the
// largest number of layers such a velocity crosses (a cell in layer d of
// that wall needs the column when reach > d). A constexpr variable, so that
// it is evaluated by the compiler.
template <class L>
struct GhostColumns {
  bool used[2][7][7];
  int reach[2][7][7];
  constexpr GhostColumns() : used{}, reach{} {
    for (int a = 0; a < L::Q; ++a) {
      const int es = ecomp<L>(a, L::D - 1);
      if (es == 0) continue;
      const int side = es > 0 ? 0 : 1, cx = ecomp<L>(a, 0) + 3, cy = L::D == 3 ? ecomp<L>(a, 1) + 3 : 3;
      used[side][cx][cy] = true;
      const int r = es > 0 ? es : -es;
      if (r > reach[side][cx][cy]) reach[side][cx][cy] = r;
    }
  }
};
template <class L>
inline constexpr GhostColumns<L> ghost_columns{};

// Population alpha pulled from beyond wall `side` (Sec. 3.2, Maxwell's
// model): gamma times the diffuse ghost plus 1 - gamma times the specular
// image, velocity mirror(alpha) leaving the mirrored layer of the same source
// column (a particle that flew into the wall, reflected in its plane).
// image() loads that stored value; it is not called for fully diffuse walls.
template <class L, typename C, typename P, typename Image>
__device__ __forceinline__ C wall_pull(int a, int side, uint32_t col, const Geometry& geo, const P* __restrict__ wp,
                                       const ProbParams<C>* __restrict__ pp, Image image) {
  const C hd = wall_ghost<L, C, P>(a, side, col, geo, wp, pp);
  if (!pp->specular) return hd;
  const C gam = side ? pp->gam[1] : pp->gam[0];
  return gam * hd + (C(1) - gam) * image();
}

// Layer of the specular image of a pull from slice s2 beyond a wall (the
// reflection in the plane half a cell outside the first or last layer).
__device__ __forceinline__ int mirror_layer(int s2, int ns) { return s2 < 0 ? -1 - s2 : 2 * ns - 1 - s2; }

// In-slice source offsets for shifts -3..3 (periodic in-slice axes).
template <class L>
__device__ __forceinline__ void inslice_offsets(const CellPos& p, const Geometry& geo, int (&xo)[7], int (&yo)[7]) {
  const int nx = int(geo.nx), ny = int(geo.ny);
#pragma unroll
  for (int k = -3; k <= 3; ++k) {
    xo[k + 3] = wrapc(p.x - k, nx);
    yo[k + 3] = L::D == 3 ? wrapc(p.y - k, ny) * nx : 0;
  }
}

// Raw buffer resource over one slice block: base address, no stride,
// num_records = the block's bytes (an access beyond it reads zero and writes
// nothing), 32-bit untyped data.
using Rsrc = __amdgpu_buffer_rsrc_t;
__device__ __forceinline__ Rsrc block_rsrc(const void* base, uint32_t bytes) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(base), short(0), int(bytes), 0x00020000);
}

// Load / store one storage element at byte voff (per lane) + soff (uniform)
// of a slice block. POL is the store's cache policy: 2 (non-temporal) or 0.
// The default stores FP64 populations non-temporally (the step kernel:
// measured faster for FP64 on MI355X, slower for the narrower types).
template <typename S>
__device__ __forceinline__ S buf_ld(Rsrc r, uint32_t voff, uint32_t soff) {
  if constexpr (sizeof(S) == 8) {
    return __builtin_bit_cast(S, __builtin_amdgcn_raw_buffer_load_b64(r, int(voff), int(soff), 0));
  } else if constexpr (sizeof(S) == 4) {
    return __builtin_bit_cast(S, __builtin_amdgcn_raw_buffer_load_b32(r, int(voff), int(soff), 0));
  } else {
    return __builtin_bit_cast(S, __builtin_amdgcn_raw_buffer_load_b16(r, int(voff), int(soff), 0));
  }
}
template <typename S, int POL = (sizeof(S) == 8 ? 2 : 0)>
__device__ __forceinline__ void buf_st(S v, Rsrc r, uint32_t voff, uint32_t soff) {
  if constexpr (sizeof(S) == 8) {
    typedef unsigned int u2 __attribute__((ext_vector_type(2)));
    __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u2, v), r, int(voff), int(soff), POL);
  } else if constexpr (sizeof(S) == 4) {
    __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned int, v), r, int(voff), int(soff), POL);
  } else {
    __builtin_amdgcn_raw_buffer_store_b16(__builtin_bit_cast(unsigned short, v), r, int(voff), int(soff), POL);
  }
}

// The wall ghosts of a wavefront's cells in slice s (wave-uniform) next to
// diffuse wall SIDE: the three partial sums of each source column that the
// wall's velocities pull across from are loaded through a resource that is
// empty unless the slice's layer needs that column, so that the loads are
// in flight together (a branch per velocity would wait for each in turn);
// the ghosts then replace the pulled values where the source lies beyond.
template <class L, typename C, typename P, int SIDE>
__device__ __forceinline__ void side_ghosts(C (&h)[L::Q], uint32_t s, const int (&xo)[7], const int (&yo)[7],
                                            const Geometry& geo, const P* __restrict__ wp,
                                            const ProbParams<C>* __restrict__ pp) {
  constexpr int D = L::D, Q = L::Q;
  constexpr uint32_t ps = sizeof(P);
  const int ns = int(geo.nslices);
  const int depth = SIDE == 0 ? int(s) : ns - 1 - int(s);   // the slice's layer from this wall
  P part[7][7][3];
#pragma unroll
  for (int cx = 0; cx < 7; ++cx)
#pragma unroll
    for (int cy = 0; cy < 7; ++cy) {
      if (!ghost_columns<L>.used[SIDE][cx][cy]) continue;
      const bool need = ghost_columns<L>.reach[SIDE][cx][cy] > depth;
      const Rsrc wr = block_rsrc(wp + uint32_t(SIDE) * 3u * geo.ncols, need ? 3u * geo.ncols * ps : 0u);
      const uint32_t col = uint32_t(xo[cx] + yo[cy]);
#pragma unroll
      for (int k = 0; k < 3; ++k) part[cx][cy][k] = buf_ld<P>(wr, col * ps, uint32_t(k) * geo.ncols * ps);
    }
#pragma unroll
  for (int a = 0; a < Q; ++a) {
    const int es = ecomp<L>(a, D - 1);
    if (es == 0 || (es > 0) != (SIDE == 0)) continue;
    const bool beyond = (es > 0 ? es : -es) > depth;
    const C g = wall_ghost_from<L, C, P>(a, SIDE, part[ecomp<L>(a, 0) + 3][D == 3 ? ecomp<L>(a, 1) + 3 : 3], pp);
    h[a] = beyond ? g : h[a];
  }
}

// Within three layers of diffuse walls: the populations whose source lies
// beyond a wall become the wall ghosts (a slice of a lattice thinner than
// six slices can be within reach of both walls).
template <class L, typename C, typename P>
__device__ __forceinline__ void diffuse_ghosts(C (&h)[L::Q], uint32_t s, const int (&xo)[7], const int (&yo)[7],
                                               const Geometry& geo, const P* __restrict__ wp,
                                               const ProbParams<C>* __restrict__ pp) {
  if (s < 3u) side_ghosts<L, C, P, 0>(h, s, xo, yo, geo, wp, pp);
  if (s + 3u >= geo.nslices) side_ghosts<L, C, P, 1>(h, s, xo, yo, geo, wp, pp);
}

// How a wavefront whose lanes share slice s pulls: the seven slices s-3..s+3
// inside the lattice and every lane far from the in-slice edges (PULL_FAST:
// one scalar offset per velocity); the seven slices inside but some lane at
// an in-slice edge (PULL_WRAP: per-lane wrapped in-slice offsets); slice s
// within 3 of the slice-axis ends (PULL_EDGE: the periodic wrap or the wall
// ghosts of that axis, one slice block per velocity).
enum PullMode { PULL_FAST = 0, PULL_WRAP = 1, PULL_EDGE = 2 };

template <class L>
__device__ __forceinline__ PullMode pull_mode_wave(uint32_t s, const CellPos& p, const Geometry& geo) {
  const bool s_inner = s >= 3u && s + 3u < geo.nslices && geo.window_ok;
  if (!s_inner) return PULL_EDGE;
  return __all(inslice_interior<L>(p, geo)) ? PULL_FAST : PULL_WRAP;
}

// Pull the Q populations that stream into the cells of a wavefront whose
// lanes all lie in slice s (s wave-uniform; i = in-slice index of the lane,
// p its position). In the FAST and WRAP modes one buffer resource spans the
// slice blocks s-3..s+3 and a velocity's source is a scalar offset (its slice
// block and plane, less the in-slice shift in FAST mode) plus a per-lane
// offset. P is the type of the wall partial sums, C the compute type.
template <class L, typename S, typename C, typename P>
__device__ __forceinline__ void gather_wave(C (&h)[L::Q], const S* __restrict__ src, const Geometry& geo,
                                            uint32_t s, uint32_t i, const CellPos& p, const P* __restrict__ wp,
                                            const ProbParams<C>* __restrict__ pp, PullMode mode) {
  constexpr int D = L::D, Q = L::Q;
  constexpr uint32_t ss = sizeof(S);
  const uint32_t bb = geo.sstride * ss;         // bytes of one slice block
  const uint32_t pb = geo.pstride * ss;         // bytes of one velocity plane segment
  if (mode == PULL_EDGE) {
    // source slice s - e_s is wave-uniform: one slice block (wrapped along a
    // periodic slice axis), or a ghost beyond a wall. Every velocity is
    // loaded first (a source beyond a wall reads the wavefront's own slice,
    // a value the ghost then replaces), so that all Q loads are in flight
    // together: a load and its widening inside a branch would be waited for
    // before the next velocity's load is issued.
    int xo[7], yo[7];
    inslice_offsets<L>(p, geo, xo, yo);
    const int ns = int(geo.nslices);
    S raw[Q];
#pragma unroll
    for (int a = 0; a < Q; ++a) {
      const int ex = ecomp<L>(a, 0), ey = ecomp<L>(a, 1), es = ecomp<L>(a, D - 1);
      const uint32_t col = uint32_t(xo[ex + 3] + yo[ey + 3]);
      const int s2 = int(s) - es;
      const int sl = (s2 < 0 || s2 >= ns) ? (geo.walls ? int(s) : wrapc(s2, ns)) : s2;
      const Rsrc blk = block_rsrc(reinterpret_cast<const char*>(src) + size_t(sl) * bb, bb);
      raw[a] = buf_ld<S>(blk, col * ss, uint32_t(a) * pb);
    }
#pragma unroll
    for (int a = 0; a < Q; ++a) h[a] = widen<C, S>(raw[a]);
    if (geo.walls && (s < 3u || s + 3u >= geo.nslices) && !pp->specular) {
      diffuse_ghosts<L, C, P>(h, s, xo, yo, geo, wp, pp);
    } else if (geo.walls && (s < 3u || s + 3u >= geo.nslices)) {
#pragma unroll
      for (int a = 0; a < Q; ++a) {
        const int ex = ecomp<L>(a, 0), ey = ecomp<L>(a, 1), es = ecomp<L>(a, D - 1);
        const int s2 = int(s) - es;
        if (s2 >= 0 && s2 < ns) continue;
        const uint32_t col = uint32_t(xo[ex + 3] + yo[ey + 3]);
        const int m = mirror_layer(s2, ns);
        h[a] = wall_pull<L, C, P>(a, s2 < 0 ? 0 : 1, col, geo, wp, pp, [&]() {
          const Rsrc img = block_rsrc(reinterpret_cast<const char*>(src) + size_t(m) * bb, bb);
          return widen<C, S>(buf_ld<S>(img, col * ss, uint32_t(mirror<L>(a)) * pb));
        });
      }
    }
    return;
  }
  const Rsrc win = block_rsrc(reinterpret_cast<const char*>(src) + size_t(s - 3u) * bb, 7u * bb);
  if (mode == PULL_FAST) {
    const uint32_t nxb = geo.nx * ss;
    const uint32_t voff = i * ss;
#pragma unroll
    for (int a = 0; a < Q; ++a) {
      const int ex = ecomp<L>(a, 0), ey = ecomp<L>(a, 1), es = ecomp<L>(a, D - 1);
      const uint32_t soff = uint32_t(3 - es) * bb + uint32_t(a) * pb - uint32_t(int(ss) * ex) -
                            (D == 3 ? uint32_t(ey) * nxb : 0u);
      h[a] = widen<C, S>(buf_ld<S>(win, voff, soff));
    }
    return;
  }
  int xo[7], yo[7];
  inslice_offsets<L>(p, geo, xo, yo);
#pragma unroll
  for (int a = 0; a < Q; ++a) {
    const int ex = ecomp<L>(a, 0), ey = ecomp<L>(a, 1), es = ecomp<L>(a, D - 1);
    const uint32_t off = uint32_t(xo[ex + 3] + yo[ey + 3]) * ss;
    h[a] = widen<C, S>(buf_ld<S>(win, off, uint32_t(3 - es) * bb + uint32_t(a) * pb));
  }
}

// ---- the in-place step pair ----------------------------------------------
//
// Two consecutive steps can share one population buffer. Step one pulls as
// gather_wave does (the buffer holds each cell's post-collision values in
// their own planes) and pushes its post-collision value of velocity b to the
// plane of -e_b at the cell x + e_b: exactly the slot from which the cell
// pulled velocity -e_b, so no other cell reads or writes it. The buffer then
// holds, at plane -e_b of every cell y, the value that streams into y along
// e_b. Step two reads those planes at its own cell, collides, and writes
// every velocity to its own plane at its own cell, which restores the layout
// of step one's input. Populations streaming in from beyond a diffuse wall
// are the wall ghosts in both steps (no cell pushed them), and a push that
// crosses a wall is dropped (the wall partial sums carry it).

// Push the post-collision populations (storage type) of a wavefront's cells (slice s,
// in-slice index i, position p): velocity b to the plane of -e_b at the cell
// x + e_b. Pull modes as gather_wave's: FAST and WRAP use the window of
// slice blocks s-3..s+3, EDGE one slice block per velocity (the periodic
// wrap, or no store across a wall).
template <class L, typename S>
__device__ __forceinline__ void scatter_wave(const S (&h)[L::Q], S* buf, const Geometry& geo, uint32_t s,
                                             uint32_t i, const CellPos& p, PullMode mode) {
  constexpr int D = L::D, Q = L::Q;
  constexpr uint32_t ss = sizeof(S);
  const uint32_t bb = geo.sstride * ss;
  const uint32_t pb = geo.pstride * ss;
  if (mode == PULL_EDGE) {
    int xo[7], yo[7];
    inslice_offsets<L>(p, geo, xo, yo);          // xo[k + 3] = x - k wrapped
    const int ns = int(geo.nslices);
#pragma unroll
    for (int b = 0; b < Q; ++b) {
      const int ex = ecomp<L>(b, 0), ey = ecomp<L>(b, 1), es = ecomp<L>(b, D - 1);
      int s2 = int(s) + es;
      if (geo.walls && (s2 < 0 || s2 >= ns)) continue;
      s2 = wrapc(s2, ns);
      const uint32_t col = uint32_t(xo[3 - ex] + yo[3 - ey]);
      const Rsrc blk = block_rsrc(reinterpret_cast<char*>(buf) + size_t(s2) * bb, bb);
      buf_st<S>(h[b], blk, col * ss, uint32_t(opposite<L>(b)) * pb);
    }
    return;
  }
  const Rsrc win = block_rsrc(reinterpret_cast<char*>(buf) + size_t(s - 3u) * bb, 7u * bb);
  if (mode == PULL_FAST) {
    const uint32_t nxb = geo.nx * ss;
    const uint32_t voff = i * ss;
#pragma unroll
    for (int b = 0; b < Q; ++b) {
      const int ex = ecomp<L>(b, 0), ey = ecomp<L>(b, 1), es = ecomp<L>(b, D - 1);
      const uint32_t soff = uint32_t(3 + es) * bb + uint32_t(opposite<L>(b)) * pb + uint32_t(int(ss) * ex) +
                            (D == 3 ? uint32_t(ey) * nxb : 0u);
      buf_st<S>(h[b], win, voff, soff);
    }
    return;
  }
  int xo[7], yo[7];
  inslice_offsets<L>(p, geo, xo, yo);
#pragma unroll
  for (int b = 0; b < Q; ++b) {
    const int ex = ecomp<L>(b, 0), ey = ecomp<L>(b, 1), es = ecomp<L>(b, D - 1);
    const uint32_t off = uint32_t(xo[3 - ex] + yo[3 - ey]) * ss;
    buf_st<S>(h[b], win, off, uint32_t(3 + es) * bb + uint32_t(opposite<L>(b)) * pb);
  }
}

// Step two's read: velocity a of the wavefront's cells from the plane of -e_a
// at the cell itself; within three layers of a diffuse wall, a population
// whose source lies beyond the wall is the wall ghost.
template <class L, typename S, typename C, typename P>
__device__ __forceinline__ void gather_local(C (&h)[L::Q], const S* buf, const Geometry& geo, uint32_t s,
                                             uint32_t i, const CellPos& p, const P* __restrict__ wp,
                                             const ProbParams<C>* __restrict__ pp) {
  constexpr int D = L::D, Q = L::Q;
  constexpr uint32_t ss = sizeof(S);
  const uint32_t bb = geo.sstride * ss;
  const uint32_t pb = geo.pstride * ss;
  const Rsrc blk = block_rsrc(reinterpret_cast<const char*>(buf) + size_t(s) * bb, bb);
  // every plane is read (all loads in flight together), then the ghosts
  // replace the populations whose source lies beyond a wall
  S raw[Q];
#pragma unroll
  for (int a = 0; a < Q; ++a) raw[a] = buf_ld<S>(blk, i * ss, uint32_t(opposite<L>(a)) * pb);
#pragma unroll
  for (int a = 0; a < Q; ++a) h[a] = widen<C, S>(raw[a]);
  if (geo.walls && (s < 3u || s + 3u >= geo.nslices)) {
    int xo[7], yo[7];
    inslice_offsets<L>(p, geo, xo, yo);
    diffuse_ghosts<L, C, P>(h, s, xo, yo, geo, wp, pp);
  }
}

// The wall ghosts of wall SIDE for lanes at arbitrary cells (slice s per
// lane): the three partial sums of each source column the wall's velocities
// pull across from, loaded for every lane (the lane's own column, an address
// inside the sums) and all before any is used; the ghosts then replace the
// pulled values of the lanes whose source lies beyond the wall.
template <class L, typename C, typename P, int SIDE>
__device__ __forceinline__ void lane_side_ghosts(C (&h)[L::Q], int s, const int (&xo)[7], const int (&yo)[7],
                                                 const Geometry& geo, const P* __restrict__ wp,
                                                 const ProbParams<C>* __restrict__ pp) {
  constexpr int D = L::D, Q = L::Q;
  const int ns = int(geo.nslices);
  const int depth = SIDE == 0 ? s : ns - 1 - s;   // the lane's layer from this wall
  P part[7][7][3];
#pragma unroll
  for (int cx = 0; cx < 7; ++cx)
#pragma unroll
    for (int cy = 0; cy < 7; ++cy) {
      if (!ghost_columns<L>.used[SIDE][cx][cy]) continue;
      const P* q = wp + uint32_t(SIDE) * 3u * geo.ncols + uint32_t(xo[cx] + yo[cy]);
#pragma unroll
      for (int k = 0; k < 3; ++k) part[cx][cy][k] = q[uint32_t(k) * geo.ncols];
    }
#pragma unroll
  for (int a = 0; a < Q; ++a) {
    const int es = ecomp<L>(a, D - 1);
    if (es == 0 || (es > 0) != (SIDE == 0)) continue;
    const bool beyond = (es > 0 ? es : -es) > depth;
    const C g = wall_ghost_from<L, C, P>(a, SIDE, part[ecomp<L>(a, 0) + 3][D == 3 ? ecomp<L>(a, 1) + 3 : 3], pp);
    h[a] = beyond ? g : h[a];
  }
}

// Pull for a lane at an arbitrary cell (no wavefront structure assumed).
// OffT is the element-offset type: 32-bit for buffers below 4 GiB. As in the
// wavefront pulls, all Q loads are issued before any is used (a source
// beyond a wall reads the lane's own slice), and the lanes within three
// layers of a wall then replace those populations by the wall ghosts.
template <class L, typename S, typename C, typename P, typename OffT>
__device__ __forceinline__ void gather_lane(C (&h)[L::Q], const S* __restrict__ src, const Geometry& geo,
                                            const CellPos& p, const P* __restrict__ wp,
                                            const ProbParams<C>* __restrict__ pp) {
  constexpr int D = L::D, Q = L::Q;
  const int ns = int(geo.nslices), s = slice_of<L>(p);
  const bool walls = geo.walls != 0;
  S raw[Q];
  {
    int xo[7], yo[7];
    inslice_offsets<L>(p, geo, xo, yo);
#pragma unroll
  for (int a = 0; a < Q; ++a) {
    const int ex = ecomp<L>(a, 0), ey = ecomp<L>(a, 1), es = ecomp<L>(a, D - 1);
    const uint32_t off = uint32_t(xo[ex + 3] + yo[ey + 3]);
    const int s2 = s - es;
    const int sl = (s2 < 0 || s2 >= ns) ? (walls ? s : wrapc(s2, ns)) : s2;
    raw[a] = src[OffT(sl) * OffT(geo.sstride) + OffT(a) * OffT(geo.pstride) + OffT(off)];
  }
  }
#pragma unroll
  for (int a = 0; a < Q; ++a) h[a] = widen<C, S>(raw[a]);
  const bool edge = walls && (s < 3 || s + 3 >= ns);
  if (walls && !pp->specular && __any(edge)) {
    // diffuse walls: wall by wall, the three partial sums of every source
    // column that some lane next to that wall needs are loaded once per
    // wavefront (each lane at its own column, an address inside the sums),
    // all before any is used; a branch per velocity and lane would wait for
    // each load in turn
    int xo[7], yo[7];
    inslice_offsets<L>(p, geo, xo, yo);
    if (__any(s < 3)) lane_side_ghosts<L, C, P, 0>(h, s, xo, yo, geo, wp, pp);
    if (__any(s + 3 >= ns)) lane_side_ghosts<L, C, P, 1>(h, s, xo, yo, geo, wp, pp);
  } else if (edge) {
    int xo[7], yo[7];
    inslice_offsets<L>(p, geo, xo, yo);
#pragma unroll
    for (int a = 0; a < Q; ++a) {
      const int ex = ecomp<L>(a, 0), ey = ecomp<L>(a, 1), es = ecomp<L>(a, D - 1);
      const int s2 = s - es;
      if (s2 >= 0 && s2 < ns) continue;
      const uint32_t off = uint32_t(xo[ex + 3] + yo[ey + 3]);
      const int m = mirror_layer(s2, ns);
      h[a] = wall_pull<L, C, P>(a, s2 < 0 ? 0 : 1, off, geo, wp, pp, [&]() {
        // the image velocity by the run-time search, not the table: with the
        // table this branch is scheduled as straight-line code that the
        // 3-D batch kernel (128 registers) spills (28-32 values against 3)
        const OffT e = OffT(m) * OffT(geo.sstride) + OffT(mirror_search<L>(a)) * OffT(geo.pstride) + OffT(off);
        return widen<C, S>(src[e]);
      });
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
  const int cw = slice_of<L>(p);
  const int nw = int(geo.nslices);
  if (!(cw < 3 || cw >= nw - 3)) return;
  const CrossSums<L, S, P> cs = cross_sums<L, S, P>(stored, lw);
  const uint32_t col = inslice_of<L>(p, geo);
  if (cw < 3) wp_dst[uint32_t(cw) * geo.ncols + col] = layer_partial(cs.lo, cw);
  if (cw >= nw - 3) {
    const int k = nw - 1 - cw;
    wp_dst[uint32_t(3 + k) * geo.ncols + col] = layer_partial(cs.hi, k);
  }
}

}  // namespace esbgk
