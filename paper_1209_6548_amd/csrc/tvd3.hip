// Kernels of the paper's own scheme (Sec. 3.1) on its 3-D set D3Q216: per
// cell the forward-Euler ES-BGK collision and force (Sec. 2.2) from the
// cell's own populations, and per velocity the TVD minmod flux differences
// along x, y and z from the five-cell stencils of the stored level:
//   h^{n+1} = h^n - omega (h^n - h_ES) + dt F/w - sum_axes nu [...].
// Periodic in x and y; in z periodic or bounded by the diffuse walls of
// Sec. 3.2 (ghost slices copy the wall slice; k_tvd3_walls re-emits after
// each step). Populations use the slice layout of Geometry (slice = z
// plane, in-slice index y nx + x).
//
// The collision needs the moments of a cell's 216 populations before the
// first of them is updated. Each level therefore carries its cells' raw
// moment sums (Moments3, MOM3 values per cell): the step reads them for
// level n, and while it writes level n + 1 pair by pair it sums the values it
// stores into the moments of level n + 1. A level set from outside gets its
// sums from k_tvd3_rawmom, and the walls kernel re-sums the wall cells it
// re-emits. A cell's populations are thus read once per step (plus the
// stencil neighbours), and the sums of every level are formed in the same
// velocity order from the stored values, whichever kernel forms them.

#include <hip/hip_runtime.h>

#include "gh3.h"
#include "stream.h"
#include "tvd.h"

namespace esbgk {

namespace {

constexpr uint32_t BLOCK3 = 512;
constexpr uint32_t Z3 = 8;               // slices per workgroup of the step kernel (one wavefront each)
constexpr uint32_t STEP3 = 64 * Z3;      // its threads

}  // namespace

// Moment sums of one cell, slot e of the [MOM3][mstride] buffer.
template <typename C>
__device__ __forceinline__ void mom3_load(Moments3<C>& m, const C* __restrict__ mom, size_t mstride, size_t e) {
  m.drho = mom[e];
#pragma unroll
  for (int t = 0; t < 3; ++t) m.J[t] = mom[size_t(1 + t) * mstride + e];
#pragma unroll
  for (int t = 0; t < 6; ++t) m.S2[t] = mom[size_t(4 + t) * mstride + e];
#pragma unroll
  for (int t = 0; t < 10; ++t) m.S3[t] = mom[size_t(10 + t) * mstride + e];
}

template <typename C>
__device__ __forceinline__ void mom3_store(const Moments3<C>& m, C* __restrict__ mom, size_t mstride, size_t e) {
  mom[e] = m.drho;
#pragma unroll
  for (int t = 0; t < 3; ++t) mom[size_t(1 + t) * mstride + e] = m.J[t];
#pragma unroll
  for (int t = 0; t < 6; ++t) mom[size_t(4 + t) * mstride + e] = m.S2[t];
#pragma unroll
  for (int t = 0; t < 10; ++t) mom[size_t(10 + t) * mstride + e] = m.S3[t];
}

// Waves per SIMD of the step kernel: FP32 compute holds the cell's
// collision coefficients (36) and the running sums of the new level (20) in
// registers, 128 VGPRs at four waves per SIMD; FP64 needs two registers a
// value.
template <typename S>
constexpr int tvd3_waves() { return sizeof(S) == 8 ? 1 : 4; }

// FP32 storage: a workgroup barrier (no memory fence) after every 8 pairs
// keeps the stacked wavefronts, which read each other's populations as z
// neighbours, within a few pairs of one another (128^3: 1.43 against 1.53 ms;
// every 4 or 16 pairs: 1.43 ms, every 32: 1.46 ms). FP16 and FP64 ran slower
// with it.
template <typename S>
constexpr int tvd3_pace() { return sizeof(S) == 4 ? 4 : 0; }

// FP64: the pairs visited group by group, each group's collision polynomial
// formed once as polynomials in c_z (3.13 against 3.29 ms at 128^3). FP32
// and FP16 keep the monomial sum per pair in velocity order: grouped, they
// ran at 1.86 against 1.33 ms (FP32) and 1.71 against 1.16 ms (FP16).
template <typename S>
constexpr bool tvd3_grouped() { return sizeof(S) == 8; }

template <typename S, bool XD>
__global__ void __launch_bounds__(STEP3, tvd3_waves<S>())
k_tvd3(Geometry geo, const S* __restrict__ src, S* __restrict__ dst,
       const typename StepT<S>::type* __restrict__ msrc, typename StepT<S>::type* __restrict__ mdst,
       const GH3Consts<typename StepT<S>::type>* __restrict__ gc,
       const LatConsts<typename StepT<S>::type>* __restrict__ lc,
       const ProbParams<typename StepT<S>::type>* __restrict__ pp, uint32_t G) {
  using C = typename StepT<S>::type;
  using L = D3Q216GH;
  constexpr int P = L::P;
  constexpr uint32_t ss = sizeof(S);
  // a workgroup takes one 64-cell chunk of the slice in Z3 = 8 consecutive
  // slices (one wavefront each): its wavefronts read each other's
  // populations as z-neighbours at about the same velocity pair (measured at
  // 128^3 FP32: 2.63 ms against 2.68 for 4 slices and 2.76 for 4 chunks of
  // one slice, in an earlier two-pass build).
  // Tiles in groups of G consecutive chunks through all bands, band by
  // band. With more than 8 bands, G = ceil(chunks / 8): each XCD (a
  // contiguous eighth of the tiles) walks a slab of the slice plane through
  // the slices, and the resident workgroups of neighbouring slabs move
  // through the slices together, so the z-neighbours of a band were read
  // shortly before and the y-neighbours at a slab edge at about the same
  // time by the next XCD (128^3: FP32 1.38 against 1.43 ms for plain
  // band-major order, FP64 3.54 against 3.76 ms; same bits). With 8 bands
  // or fewer, G = all chunks: band-major, each XCD within one band, and
  // the XCDs of neighbouring bands move through the plane together
  // (256 x 256 x 64: 2.95 against 3.04 ms for slabs).
  const uint32_t blk = xcd_block(blockIdx.x, gridDim.x);
  const uint32_t nchunks = geo.ipad >> 6, nbands = (geo.nslices + Z3 - 1) / Z3;
  const uint32_t full = nchunks / G, span = G * nbands, sg = blk / span;
  const uint32_t g = sg < full ? G : nchunks - full * G;   // the last group may be narrower
  const uint32_t r = blk - sg * span;
  const uint32_t band = r / g, chunk = sg * G + (r - band * g);
  const uint32_t i0 = chunk * 64u;
  if (i0 >= geo.inner) return;                       // the slice's padding slots (the whole workgroup)
  // a wavefront beyond the last slice (the last band of a lattice whose
  // slice count is not a multiple of Z3) runs the loop on the last slice
  // and stores nothing, so that every wavefront meets every barrier
  const uint32_t sw = band * Z3 + __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const bool live = sw < geo.nslices;
  const uint32_t s = live ? sw : geo.nslices - 1;
  const uint32_t lane = threadIdx.x & 63u;
  // lanes past the end of the slice compute its last cell again and store
  // into their own padding slots (i0 + 64 <= ipad)
  const uint32_t i = min(i0 + lane, geo.inner - 1);
  const int nx = int(geo.nx), ny = int(geo.ny), ns = int(geo.nslices);
  const int y = int(fdiv(i, geo.div_nx)), x = int(i) - y * nx;
  uint32_t xo[5], yo[5];
#pragma unroll
  for (int k = -2; k <= 2; ++k) {
    xo[k + 2] = uint32_t(y * nx + wrapc(x + k, nx)) * ss;
    yo[k + 2] = uint32_t(wrapc(y + k, ny) * nx + x) * ss;
  }
  // XD (nx a multiple of 64): the chunk lies in one row, and the x
  // neighbours come from the neighbouring lanes by wavefront shifts; one
  // halo load per velocity brings x0 - 2, x0 - 1 (lanes 1, 0..31) and
  // x0 + 64, x0 + 65 (lanes 32..63, 62) of the chunk's row
  uint32_t hoff = 0;
  if constexpr (XD) {
    const int x0 = x - int(lane);
    int hx = lane < 32u ? wrapc(x0 - 1, nx) : wrapc(x0 + 64, nx);
    if (lane == 1u) hx = wrapc(x0 - 2, nx);
    if (lane == 62u) hx = wrapc(x0 + 65, nx);
    hoff = uint32_t(y * nx + hx) * ss;
  }
  const uint32_t so = (i0 + lane) * ss;
  const uint32_t bb = geo.sstride * ss, pb = geo.pstride * ss;
  Rsrc row[5];
#pragma unroll
  for (int k = -2; k <= 2; ++k) {
    const int r = geo.walls ? min(max(int(s) + k, 0), ns - 1) : wrapc(int(s) + k, ns);
    row[k + 2] = block_rsrc(reinterpret_cast<const char*>(src) + size_t(r) * bb, bb);
  }
  const Rsrc out = block_rsrc(reinterpret_cast<char*>(dst) + size_t(s) * bb, live ? bb : 0u);
  const size_t mstride = size_t(geo.nslices) * geo.ipad;

  // the collision from the moments of the stored level (the third moments
  // only with a body force)
  GH3Collision<C> k;
  {
    Moments3<C> acc;
    mom3_load<C>(acc, msrc, mstride, size_t(s) * geo.ipad + i);
    if (pp->force == 0) {
#pragma unroll
      for (int t = 0; t < 10; ++t) acc.S3[t] = C(0);
    }
    collision_gh3<C>(acc, lc, pp, k);
  }

  // collision and fluxes pair by pair (FP64: group by group, the collision
  // polynomial of a group of six pairs that share c_x and c_y formed once,
  // as polynomials in c_z); the stored values of the new level go into its
  // moment sums in this visiting order. The 20 loads of pair p + 1
  // are issued before pair p is computed and stored (the compiler may not
  // move loads through a buffer resource past the stores through another),
  // so that one pair's memory latency overlaps the other's arithmetic.
  auto load_pair = [&](int j, S (&v)[2][10]) {
    const int p = tvd3_grouped<S>() ? gc->order[j] : j;
#pragma unroll
    for (int side = 0; side < 2; ++side) {
      const uint32_t po = uint32_t(p + side * P) * pb;
      const C sg = side == 0 ? C(1) : C(-1);
      v[side][0] = buf_ld<S>(row[2], xo[2], po);
#pragma unroll
      for (int ax = 0; ax < 3; ++ax) {
        const bool pos = sg * gc->nu[p][ax] > C(0);
        if (ax == 0) {
          if constexpr (XD) {
            v[side][1] = buf_ld<S>(row[2], hoff, po);
          } else {
            v[side][1] = buf_ld<S>(row[2], xo[1], po);
            v[side][2] = buf_ld<S>(row[2], xo[3], po);
            v[side][3] = buf_ld<S>(row[2], pos ? xo[0] : xo[4], po);
          }
        } else if (ax == 1) {
          v[side][4] = buf_ld<S>(row[2], yo[1], po);
          v[side][5] = buf_ld<S>(row[2], yo[3], po);
          v[side][6] = buf_ld<S>(row[2], pos ? yo[0] : yo[4], po);
        } else {
          v[side][7] = buf_ld<S>(row[1], xo[2], po);
          v[side][8] = buf_ld<S>(row[3], xo[2], po);
          v[side][9] = buf_ld<S>(pos ? row[0] : row[4], xo[2], po);
        }
      }
    }
  };
  Moments3<C> nxt;
  moments3_zero<C>(nxt);
  GH3Group<C> grp;
  auto do_pair = [&](int j, const S (&cur)[2][10]) {
    const int p = tvd3_grouped<S>() ? gc->order[j] : j;
    const uint32_t pop = uint32_t(p) * pb;
    C hs[2];
    if constexpr (tvd3_grouped<S>())
      collide_pair_group<C>(grp, k.omw, gc->cz[j], widen<C, S>(cur[0][0]), widen<C, S>(cur[1][0]), hs[0], hs[1]);
    else
      collide_pair_gh3<C>(k, gc->mono[p], widen<C, S>(cur[0][0]), widen<C, S>(cur[1][0]), hs[0], hs[1]);
    C v[2];
#pragma unroll
    for (int side = 0; side < 2; ++side) {
      const uint32_t po = pop + uint32_t(side * P) * pb;
      const C sg = side == 0 ? C(1) : C(-1);
      const C f0 = widen<C, S>(cur[side][0]);
      C t = C(0);
#pragma unroll
      for (int ax = 0; ax < 3; ++ax) {
        const C nu = sg * gc->nu[p][ax];
        const bool pos = nu > C(0);
        C fm1, fp1, f2;
        if (XD && ax == 0) {
          const C H = widen<C, S>(cur[side][1]);
          fm1 = lane_shift(H, f0, true);
          fp1 = lane_shift(H, f0, false);
          f2 = pos ? lane_shift(lane_shift(H, H, false), fm1, true)     // lane 0 takes x0 - 2
                   : lane_shift(lane_shift(H, H, true), fp1, false);    // lane 63 takes x0 + 65
        } else {
          fm1 = widen<C, S>(cur[side][3 * ax + 1]);
          fp1 = widen<C, S>(cur[side][3 * ax + 2]);
          f2 = widen<C, S>(cur[side][3 * ax + 3]);
        }
        C d, m;
        // FP64: selects instead of a branch on the direction, 3.73 against
        // 3.95 ms at 128^3; FP32 and FP16 keep the branch (1.43 against 1.98
        // ms and 1.22 against 1.55 ms with selects)
        if constexpr (sizeof(C) == 8)
          tvd_terms_sel<C>(pos, f2, fm1, f0, fp1, d, m);
        else
          tvd_terms<C>(pos, f2, fm1, f0, fp1, d, m);
        t = fmac(nu, d, t);
        t = fmac(gc->nk[p][ax], m, t);
      }
      const S o = narrow<S, C>(hs[side] - t);
      buf_st<S, tvd_store_policy<S>(L::Q)>(o, out, so, po);
      v[side] = widen<C, S>(o);
    }
    moments3_add<C>(nxt, gc->w[p], gc->mono[p], v[0], v[1], true);
  };
  // two register sets in turn (P is even): the loads of the next pair go
  // out before the current pair is computed
  static_assert(P % 2 == 0, "pairs in twos");
  S b0[2][10], b1[2][10];
  static_assert(GH3_GROUP % 2 == 0 && GH3_GROUPS * GH3_GROUP == P, "groups of whole pairs of pairs");
  load_pair(0, b0);
#pragma unroll 1
  for (int p = 0; p < P; p += 2) {
    load_pair(p + 1, b1);
    if constexpr (tvd3_grouped<S>())
      if (p % GH3_GROUP == 0) group_poly<C>(k, gc->gxy[p / GH3_GROUP], grp);   // pairs p, p + 1 share a group
    do_pair(p, b0);
    load_pair(p + 2 < P ? p + 2 : p + 1, b0);   // the last round loads pair P - 1 again
    do_pair(p + 1, b1);
    // every wavefront of the workgroup runs the same pairs
    if constexpr (tvd3_pace<S>() > 0)
      if ((p >> 1) % tvd3_pace<S>() == tvd3_pace<S>() - 1) __builtin_amdgcn_s_barrier();
  }
  if (live) mom3_store<C>(nxt, mdst, mstride, size_t(s) * geo.ipad + i0 + lane);
}

// Moment sums of a level set from outside, one thread per slot of the
// [MOM3][nslices * ipad] buffer (padding slots take the slice's last cell).
template <typename S>
__global__ void __launch_bounds__(BLOCK3)
k_tvd3_rawmom(Geometry geo, const S* __restrict__ pop, typename StepT<S>::type* __restrict__ mom,
              const GH3Consts<typename StepT<S>::type>* __restrict__ gc) {
  using C = typename StepT<S>::type;
  using L = D3Q216GH;
  const uint32_t j = blockIdx.x * BLOCK3 + threadIdx.x;
  const size_t mstride = size_t(geo.nslices) * geo.ipad;
  if (j >= mstride) return;
  const uint32_t s = fdiv(j, geo.div_ipad), slot = j - s * geo.ipad;
  const uint32_t i = min(slot, geo.inner - 1);
  const size_t elem = size_t(s) * geo.sstride + i;
  Moments3<C> acc;
  moments3_zero<C>(acc);
  // in the step's visiting order, so that the sums are the step's bits
#pragma unroll 4
  for (int q = 0; q < L::P; ++q) {
    const int p = tvd3_grouped<S>() ? gc->order[q] : q;
    const C hp = widen<C, S>(pop[size_t(p) * geo.pstride + elem]);
    const C hm = widen<C, S>(pop[size_t(p + L::P) * geo.pstride + elem]);
    moments3_add<C>(acc, gc->w[p], gc->mono[p], hp, hm, true);
  }
  mom3_store<C>(acc, mom, mstride, j);
}

// Re-emission at the z walls (Sec. 3.2) after a step, per in-slice column
// i and wall side = blockIdx.y (see k_tvd_walls); the wall cell's moment
// sums are then formed again from its stored values.
template <typename S>
__global__ void __launch_bounds__(BLOCK3)
k_tvd3_walls(Geometry geo, S* __restrict__ pop, const TVDWalls3<typename StepT<S>::type>* __restrict__ w,
             typename StepT<S>::type* __restrict__ mom, const GH3Consts<typename StepT<S>::type>* __restrict__ gc) {
  using C = typename StepT<S>::type;
  using L = D3Q216GH;
  const uint32_t i = blockIdx.x * BLOCK3 + threadIdx.x;
  const int side = int(blockIdx.y);
  if (i >= geo.inner) return;
  const uint32_t jw = side ? geo.nslices - 1 : 0, ji = side ? geo.nslices - 2 : 1;
  const size_t ew = size_t(jw) * geo.sstride + i, ei = size_t(ji) * geo.sstride + i;
  C rho = w->k0[side];
#pragma unroll
  for (int a = 0; a < L::Q; ++a) {
    const int sz = gh_sign<L>(a, 2);
    const bool toward = side == 0 ? sz < 0 : sz > 0;
    if (toward) rho = fmac(w->kin[side][a], widen<C, S>(pop[size_t(a) * geo.pstride + ei]), rho);
  }
  // velocity p + h P moves into the gas when the sign of its z component
  // (that of the Courant number nu[p][2], negated for h = 1) points away
  // from the wall
  Moments3<C> acc;
  moments3_zero<C>(acc);
#pragma unroll 1
  for (int q = 0; q < L::P; ++q) {   // in the step's visiting order
    const int p = tvd3_grouped<S>() ? gc->order[q] : q;
    const bool up = gc->nu[p][2] > C(0);
    C v[2];
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const int a = p + h * L::P;
      const bool into_gas = (up != (h == 1)) == (side == 0);
      S* e = pop + size_t(a) * geo.pstride + ew;
      if (into_gas) {
        const S o = narrow<S, C>(rho * w->sw[side][a] - C(1));
        *e = o;
        v[h] = widen<C, S>(o);
      } else {
        v[h] = widen<C, S>(*e);
      }
    }
    moments3_add<C>(acc, gc->w[p], gc->mono[p], v[0], v[1], true);
  }
  mom3_store<C>(acc, mom, size_t(geo.nslices) * geo.ipad, size_t(jw) * geo.ipad + i);
}

// h = rho S(T, u)/w (1 + amp xi) - 1 (eq. feq0 at N = 4, D = 3) for cells
// [c0, c0 + count); c[Q][3]; fields [count] / [3][count] / [Q][count] or
// null.
template <typename S>
__global__ void __launch_bounds__(BLOCK3)
k_tvd3_init(Geometry geo, S* __restrict__ dst, const double* __restrict__ c, const double* __restrict__ rho,
            const double* __restrict__ u, const double* __restrict__ T, const double* __restrict__ noise,
            double amp, uint32_t c0, uint32_t count) {
  const uint32_t j = blockIdx.x * BLOCK3 + threadIdx.x;
  if (j >= count) return;
  const uint32_t cell = c0 + j;
  const uint32_t s = cell / geo.inner, i = cell - s * geo.inner;
  const size_t elem = size_t(s) * geo.sstride + i;
  const double drho = rho ? rho[j] - 1.0 : 0.0;
  double uv[3];
  for (int d = 0; d < 3; ++d) uv[d] = u ? u[size_t(d) * count + j] : 0.0;
  const double th = T ? T[j] - 1.0 : 0.0;
  const double uu = uv[0] * uv[0] + uv[1] * uv[1] + uv[2] * uv[2];
  constexpr double D = 3.0;
  for (int a = 0; a < D3Q216GH::Q; ++a) {
    const double cx = c[3 * a], cy = c[3 * a + 1], cz = c[3 * a + 2];
    const double cu = cx * uv[0] + cy * uv[1] + cz * uv[2], cc = cx * cx + cy * cy + cz * cz;
    double sm1 = cu + 0.5 * (cu * cu - uu + th * (cc - D)) + cu / 6.0 * (cu * cu - 3.0 * uu + 3.0 * th * (cc - D - 2));
    sm1 += (cu * cu * cu * cu - 6.0 * cu * cu * uu + 3.0 * uu * uu) / 24.0 +
           th / 4.0 * ((cc - D - 2) * (cu * cu - uu) - 2.0 * cu * cu) +
           th * th / 8.0 * (cc * cc - 2.0 * (D + 2) * cc + D * (D + 2));
    double hv = drho * (1.0 + sm1) + sm1;
    if (noise) hv += (1.0 + hv) * amp * noise[size_t(a) * count + j];
    dst[size_t(a) * geo.pstride + elem] = S(hv);
  }
}

// The 14 fields rho, u[3], T, sigma (xx xy xz yy yz zz), q[3] of cells
// [c0, c0 + count) in FP64, written as [14][count].
template <typename S>
__global__ void __launch_bounds__(BLOCK3)
k_tvd3_moments(Geometry geo, const S* __restrict__ src, const GH3Consts<double>* __restrict__ gc,
               const LatConsts<double>* __restrict__ lc, const ProbParams<double>* __restrict__ pp, uint32_t c0,
               uint32_t count, double* __restrict__ out) {
  using L = D3Q216GH;
  const uint32_t j = blockIdx.x * BLOCK3 + threadIdx.x;
  if (j >= count) return;
  const uint32_t cell = c0 + j;
  const uint32_t s = cell / geo.inner, i = cell - s * geo.inner;
  const size_t elem = size_t(s) * geo.sstride + i;
  Moments3<double> acc;
  moments3_zero<double>(acc);
  for (int p = 0; p < L::P; ++p) {
    const double hp = double(src[size_t(p) * geo.pstride + elem]);
    const double hm = double(src[size_t(p + L::P) * geo.pstride + elem]);
    moments3_add<double>(acc, gc->w[p], gc->mono[p], hp, hm, true);
  }
  RawMoments<L, double> m;
  moments3_finish<double>(acc, m);
  double f[14];
  fields_from_moments<L, double>(m, lc, pp, f);
  for (int k = 0; k < 14; ++k) out[size_t(k) * count + j] = f[k];
}

#define ESBGK_TVD3_DISPATCH(storage, CALL)                 \
  do {                                                     \
    if (storage == 0) { using S = double; return CALL; }   \
    if (storage == 1) { using S = float; return CALL; }    \
    if (storage == 2) { using S = _Float16; return CALL; } \
    return hipErrorInvalidValue;                           \
  } while (0)

template <typename S>
static hipError_t tvd3_step_t(const TVDArgs& a) {
  using C = typename StepT<S>::type;
  const uint32_t nchunks = a.geo.ipad >> 6;
  const uint32_t nbands = (a.geo.nslices + Z3 - 1) / Z3;
  const uint32_t nb = nchunks * nbands;
  const uint32_t G = nbands > 8 ? (nchunks + 7) / 8 : nchunks;   // chunks of a group (nchunks >= 1)
  auto* kern = a.geo.nx % 64 == 0 ? k_tvd3<S, true> : k_tvd3<S, false>;
  hipLaunchKernelGGL(kern, dim3(nb), dim3(STEP3), 0, a.stream, a.geo, static_cast<const S*>(a.src),
                     static_cast<S*>(a.dst), static_cast<const C*>(a.msrc), static_cast<C*>(a.mdst),
                     static_cast<const GH3Consts<C>*>(a.gc), static_cast<const LatConsts<C>*>(a.lc),
                     static_cast<const ProbParams<C>*>(a.pp), G);
  return hipGetLastError();
}

template <typename S>
static hipError_t tvd3_walls_t(const TVDArgs& a, const void* walls) {
  using C = typename StepT<S>::type;
  const dim3 grid((a.geo.inner + BLOCK3 - 1) / BLOCK3, 2);
  hipLaunchKernelGGL(k_tvd3_walls<S>, grid, dim3(BLOCK3), 0, a.stream, a.geo, static_cast<S*>(a.dst),
                     static_cast<const TVDWalls3<C>*>(walls), static_cast<C*>(a.mdst),
                     static_cast<const GH3Consts<C>*>(a.gc));
  return hipGetLastError();
}

template <typename S>
static hipError_t tvd3_rawmom_t(const TVDArgs& a, const void* pop, void* mom) {
  using C = typename StepT<S>::type;
  const size_t slots = size_t(a.geo.nslices) * a.geo.ipad;
  const uint32_t nb = uint32_t((slots + BLOCK3 - 1) / BLOCK3);
  hipLaunchKernelGGL(k_tvd3_rawmom<S>, dim3(nb), dim3(BLOCK3), 0, a.stream, a.geo, static_cast<const S*>(pop),
                     static_cast<C*>(mom), static_cast<const GH3Consts<C>*>(a.gc));
  return hipGetLastError();
}

template <typename S>
static hipError_t tvd3_init_t(const TVDArgs& a, const double* c, const double* rho, const double* u,
                              const double* T, const double* noise, double amp, uint32_t c0, uint32_t count) {
  const uint32_t nb = (count + BLOCK3 - 1) / BLOCK3;
  hipLaunchKernelGGL(k_tvd3_init<S>, dim3(nb), dim3(BLOCK3), 0, a.stream, a.geo, static_cast<S*>(a.dst), c, rho, u,
                     T, noise, amp, c0, count);
  return hipGetLastError();
}

template <typename S>
static hipError_t tvd3_moments_t(const TVDArgs& a, uint32_t c0, uint32_t count, double* out) {
  const uint32_t nb = (count + BLOCK3 - 1) / BLOCK3;
  hipLaunchKernelGGL(k_tvd3_moments<S>, dim3(nb), dim3(BLOCK3), 0, a.stream, a.geo, static_cast<const S*>(a.src),
                     static_cast<const GH3Consts<double>*>(a.gc64), static_cast<const LatConsts<double>*>(a.lc64),
                     static_cast<const ProbParams<double>*>(a.pp64), c0, count, out);
  return hipGetLastError();
}

hipError_t launch_tvd3_step(int storage, const TVDArgs& a) { ESBGK_TVD3_DISPATCH(storage, tvd3_step_t<S>(a)); }

hipError_t launch_tvd3_walls(int storage, const TVDArgs& a, const void* walls) {
  ESBGK_TVD3_DISPATCH(storage, (tvd3_walls_t<S>(a, walls)));
}

hipError_t launch_tvd3_rawmom(int storage, const TVDArgs& a, const void* pop, void* mom) {
  ESBGK_TVD3_DISPATCH(storage, (tvd3_rawmom_t<S>(a, pop, mom)));
}

hipError_t launch_tvd3_init(int storage, const TVDArgs& a, const double* c, const double* rho, const double* u,
                            const double* T, const double* noise, double amp, uint32_t c0, uint32_t count) {
  ESBGK_TVD3_DISPATCH(storage, (tvd3_init_t<S>(a, c, rho, u, T, noise, amp, c0, count)));
}

hipError_t launch_tvd3_moments(int storage, const TVDArgs& a, uint32_t c0, uint32_t count, double* out) {
  ESBGK_TVD3_DISPATCH(storage, (tvd3_moments_t<S>(a, c0, count, out)));
}

}  // namespace esbgk
