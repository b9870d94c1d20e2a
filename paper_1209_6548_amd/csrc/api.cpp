// C ABI of the lattice ES-BGK library: handle management, validation,
// workspace layout, parameter upload, state I/O and the step driver.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "../../include/esbgk.h"
#include "kernels.h"
#include "tables.h"

using namespace esbgk;

namespace {

constexpr size_t ALIGN = 256;
constexpr uint32_t STAGE_CELLS = 65536;   // cells per staged host transfer
constexpr double MALL_BYTES = 256.0 * 1024 * 1024;   // MI355X memory-side (Infinity) cache

size_t align_up(size_t n) { return (n + ALIGN - 1) / ALIGN * ALIGN; }

size_t storage_size(int storage) { return storage == ESBGK_F64 ? 8 : (storage == ESBGK_F32 ? 4 : 2); }
size_t compute_size(int storage) { return storage == ESBGK_F64 ? 8 : 4; }

// Workspace layout; every region 256-byte aligned.
struct Layout {
  size_t pop[2], wp[2], lc, pp, lc64, pp64, uprev, red_part, red_out, wprog, level, staging, total;
  size_t staging_bytes;
};

bool valid_shape(const esbgk_shape* s, std::string* why) {
  auto fail = [&](const char* m) { if (why) *why = m; return false; };
  if (!s) return fail("null shape");
  if (s->velset != ESBGK_D2Q37 && s->velset != ESBGK_D3Q39) return fail("velset must be ESBGK_D2Q37 or ESBGK_D3Q39");
  if (s->nx < 1 || s->ny < 1 || s->nz < 1) return fail("extents must be >= 1");
  if (s->velset == ESBGK_D2Q37 && s->nz != 1) return fail("D2Q37 needs nz = 1");
  const uint64_t n = uint64_t(s->nx) * uint64_t(s->ny) * uint64_t(s->nz);
  if (n >= (uint64_t(1) << 31)) return fail("nx*ny*nz must be < 2^31");
  if (s->walls != 0 && s->walls != 1) return fail("walls must be 0 or 1");
  if (s->walls) {
    const int nw = s->velset == ESBGK_D2Q37 ? s->ny : s->nz;
    if (nw < 6) return fail("the wall axis needs at least 6 cells");
  }
  if (s->storage < ESBGK_F64 || s->storage > ESBGK_F16) return fail("storage must be F64, F32 or F16");
  if (!host_lattice(s->velset)) return fail("velocity set tables unavailable");
  Geometry g;
  if (!make_geometry(s->velset == ESBGK_D2Q37 ? 2 : 3, s->velset == ESBGK_D2Q37 ? 37 : 39, uint32_t(s->nx),
                     uint32_t(s->ny), uint32_t(s->nz), s->walls != 0, true, storage_size(s->storage), g))
    return fail("lattice too large for the slice layout (one slice of the populations must be < 4 GiB)");
  if (s->scheme != ESBGK_TRAPEZOID && s->scheme != ESBGK_EULER) return fail("scheme must be TRAPEZOID or EULER");
  if (s->n_ref < 0) return fail("n_ref must be >= 0");
  return true;
}

int ncols_of(const esbgk_shape* s) {
  return s->velset == ESBGK_D2Q37 ? s->nx : s->nx * s->ny;
}

// The single-lattice geometry (slice-blocked layout); the shape is valid.
Geometry geometry_of(const esbgk_shape* s) {
  const HostLattice* lat = host_lattice(s->velset);
  Geometry g;
  make_geometry(lat->D, lat->Q, uint32_t(s->nx), uint32_t(s->ny), uint32_t(s->nz), s->walls != 0, true,
                storage_size(s->storage), g);
  return g;
}


Layout layout_of(const esbgk_shape* s) {
  const HostLattice* lat = host_lattice(s->velset);
  Layout L{};
  const size_t cells = size_t(s->nx) * s->ny * s->nz;
  const size_t ss = storage_size(s->storage), cs = compute_size(s->storage);
  const size_t Q = size_t(lat->Q), D = size_t(lat->D);
  const size_t ncols = size_t(ncols_of(s));
  const Geometry g = geometry_of(s);
  const size_t nblocks = slot_blocks(g);
  size_t off = 0;
  auto take = [&](size_t bytes) { const size_t o = off; off = align_up(off + bytes); return o; };
  const size_t pop_bytes = size_t(g.nslices) * g.sstride * ss;
  L.pop[0] = take(pop_bytes);
  L.pop[1] = take(pop_bytes);
  L.wp[0] = take(6 * ncols * cs);
  L.wp[1] = take(6 * ncols * cs);
  L.lc = take(cs == 8 ? sizeof(LatConsts<double>) : sizeof(LatConsts<float>));
  L.pp = take(cs == 8 ? sizeof(ProbParams<double>) : sizeof(ProbParams<float>));
  // FP64 blocks for the read-out kernels (the same blocks when storage is FP64)
  L.lc64 = cs == 8 ? L.lc : take(sizeof(LatConsts<double>));
  L.pp64 = cs == 8 ? L.pp : take(sizeof(ProbParams<double>));
  L.uprev = take(D * cells * cs);
  L.red_part = take(nblocks * NRED * sizeof(double));
  L.red_out = take(NRED * sizeof(double));
  L.wprog = take(sizeof(WallProgram));
  L.level = take(sizeof(int64_t));
  const size_t stage_cells = std::min<size_t>(cells, STAGE_CELLS);
  const size_t per_cell = std::max<size_t>(nfields(int(D)), 2 + D + Q) * sizeof(double);
  L.staging_bytes = stage_cells * per_cell;
  L.staging = take(L.staging_bytes);
  L.total = off;
  return L;
}

}  // namespace

struct esbgk_ctx {
  esbgk_shape shape{};
  const HostLattice* lat = nullptr;
  Geometry geo{};
  Layout lay{};
  char* ws = nullptr;
  hipStream_t stream = nullptr;
  int device = 0;                 // the GPU current at creation
  int cur = 0;                    // buffer holding the current state
  bool state_set = false;
  int64_t steps = 0;
  int64_t R = 0;                  // fused reduction interval
  int have_prev = 0;
  int64_t last_red_step = -1;
  int sticky = 0;
  std::string err;
  // gas, walls, force
  double Kn = 0.1, Pr = 1.0, varpi = 0.5;
  double Tw[2] = {1.0, 1.0};
  double uw[2][3] = {{0, 0, 0}, {0, 0, 0}};
  double gam[2] = {1.0, 1.0};     // wall accommodation (Maxwell's model)
  double heat_amp[2] = {0, 0}, heat_freq[2] = {0, 0};   // unsteady heating
  bool heating() const { return heat_amp[0] != 0.0 || heat_amp[1] != 0.0; }
  WallProgram wprog{};
  double g[3] = {0, 0, 0};
  int n_ref = 0;
  // host copies of the device parameter blocks
  ProbParams<double> pp64{};
  ProbParams<float> pp32{};
  LatConsts<double> lc64{};
  LatConsts<float> lc32{};

  // HIP graphs of graph_steps consecutive step launches, one per starting
  // buffer, captured on a private stream and replayed on the caller's stream
  int graph_steps = 32;
  hipStream_t cap = nullptr;
  hipGraphExec_t graph[2] = {nullptr, nullptr};
  // in-place pairs of steps (one population buffer per pair), captured per
  // buffer holding the state; inplace: 0 never, 1 always, 2 when it pays
  int inplace = 2;
  hipGraphExec_t graph_pair[2] = {nullptr, nullptr};
  bool pairs() const {
    if (shape.walls && !(gam[0] == 1.0 && gam[1] == 1.0)) return false;
    if (inplace != 2) return inplace == 1;
    // Measured on MI355X (D2Q37 channels, n x n): pairs are faster when the
    // two buffers overflow the 256 MB memory-side cache and one buffer does
    // not exceed it by much (FP32 1024^2: 47.1 against 56.1 us per step,
    // 1448^2: 111.8 against 121.5; FP64 1024^2: 104.1 against 108.9; FP16
    // 1448^2: 55.6 against 63.6); they are slower when both buffers fit
    // (FP32 896^2: 37.3 against 35.1) or one buffer is twice the cache
    // (FP32 2048^2: 236 against 219).
    const double one = double(lay.pop[1] - lay.pop[0]);
    return 2.0 * one > MALL_BYTES && one <= 1.5 * MALL_BYTES;
  }

  char* at(size_t off) const { return ws + off; }
  bool f64() const { return shape.storage == ESBGK_F64; }
};

namespace {

// Message of the last failed esbgk_create on this thread (no handle exists to
// hold it); returned by esbgk_last_error(NULL).
thread_local std::string g_create_error;

int set_err(esbgk_ctx* c, int code, const std::string& msg) {
  if (c) c->err = msg;
  return code;
}

int hip_fail(esbgk_ctx* c, hipError_t e, const char* where) {
  c->sticky = ESBGK_E_HIP;
  c->err = std::string(where) + ": " + hipGetErrorString(e);
  return ESBGK_E_HIP;
}

#define HIP_OR_FAIL(ctx, expr, where)            \
  do {                                           \
    hipError_t _e = (expr);                      \
    if (_e != hipSuccess) return hip_fail(ctx, _e, where); \
  } while (0)

StepArgs args_at(const esbgk_ctx* c, int cur) {
  StepArgs a{};
  a.geo = c->geo;
  a.src = c->at(c->lay.pop[cur]);
  a.dst = c->at(c->lay.pop[1 - cur]);
  a.wp_src = c->at(c->lay.wp[cur]);
  a.wp_dst = c->at(c->lay.wp[1 - cur]);
  a.lc = c->at(c->lay.lc);
  a.pp = c->at(c->lay.pp);
  a.lc64 = c->at(c->lay.lc64);
  a.pp64 = c->at(c->lay.pp64);
  a.uprev = c->at(c->lay.uprev);
  a.have_prev = c->have_prev;
  a.reduce = 0;
  // alternate the tile order between the two buffers for FP32 storage
  // (measured on MI355X at 1024 x 1024: 2-3 % faster for FP32, 5 % slower
  // for FP16 whose lattice fits the memory-side cache, no change for FP64)
  a.rev = c->shape.storage == ESBGK_F32 ? cur : 0;
  a.red_part = reinterpret_cast<double*>(c->at(c->lay.red_part));
  a.stream = c->stream;
  return a;
}

StepArgs base_args(const esbgk_ctx* c) { return args_at(c, c->cur); }

// Unsteady heating: rebuild the wall tables for the step from the level held
// on the device (advance: and move that level on, as a step does).
hipError_t wall_tables(const esbgk_ctx* c, int advance, hipStream_t stream) {
  return launch_wall_tables(c->shape.velset, reinterpret_cast<const WallProgram*>(c->at(c->lay.wprog)),
                            c->at(c->lay.lc64), c->at(c->lay.pp64), c->f64() ? nullptr : c->at(c->lay.pp),
                            reinterpret_cast<int64_t*>(c->at(c->lay.level)), advance, stream);
}

// Copy the host step counter to the device level (after the state was set).
int sync_level(esbgk_ctx* c) {
  HIP_OR_FAIL(c, hipMemcpyAsync(c->at(c->lay.level), &c->steps, sizeof(int64_t), hipMemcpyHostToDevice, c->stream),
              "level");
  HIP_OR_FAIL(c, hipStreamSynchronize(c->stream), "level");
  return ESBGK_OK;
}


// A replay may still be queued or running on the caller's stream (esbgk_step
// returns after hipGraphLaunch): wait for it before the executable graphs go.
void drop_graphs(esbgk_ctx* c) {
  const bool any = c->graph[0] || c->graph[1] || c->graph_pair[0] || c->graph_pair[1];
  if (any && hipStreamSynchronize(c->stream) != hipSuccess) {
    c->sticky = ESBGK_E_HIP;
    c->err = "synchronize before releasing the step graphs failed";
  }
  for (int p = 0; p < 2; ++p) {
    if (c->graph[p]) (void)hipGraphExecDestroy(c->graph[p]);
    if (c->graph_pair[p]) (void)hipGraphExecDestroy(c->graph_pair[p]);
    c->graph[p] = nullptr;
    c->graph_pair[p] = nullptr;
  }
}

// Arguments of step `phase` of an in-place pair on the buffer holding the
// state: the wall partial sums go from the state's to the other buffer's and
// back, so that after the pair they sit with the state as after two steps.
StepArgs pair_args(const esbgk_ctx* c, int phase, int cur) {
  StepArgs a = args_at(c, cur);
  a.dst = c->at(c->lay.pop[cur]);
  a.src = a.dst;
  a.wp_src = c->at(c->lay.wp[phase == 1 ? cur : 1 - cur]);
  a.wp_dst = c->at(c->lay.wp[phase == 1 ? 1 - cur : cur]);
  a.rev = 0;
  return a;
}

// Capture graph_steps plain step launches starting from buffer `parity`.
int build_graph(esbgk_ctx* c, int parity) {
  if (!c->cap) {
    hipError_t e = hipStreamCreateWithFlags(&c->cap, hipStreamNonBlocking);
    if (e != hipSuccess) {
      c->cap = nullptr;
      return hip_fail(c, e, "create capture stream");
    }
  }
  HIP_OR_FAIL(c, hipStreamBeginCapture(c->cap, hipStreamCaptureModeRelaxed), "begin capture");
  int cur = parity;
  hipError_t le = hipSuccess;
  for (int i = 0; i < c->graph_steps && le == hipSuccess; ++i) {
    StepArgs a = args_at(c, cur);
    a.stream = c->cap;
    if (c->heating()) le = wall_tables(c, 1, c->cap);
    if (le == hipSuccess) le = launch_step(c->shape.velset, c->shape.storage, a);
    cur ^= 1;
  }
  hipGraph_t g = nullptr;
  hipError_t ee = hipStreamEndCapture(c->cap, &g);
  if (le != hipSuccess) {
    if (g) (void)hipGraphDestroy(g);
    return hip_fail(c, le, "capture step");
  }
  if (ee != hipSuccess) return hip_fail(c, ee, "end capture");
  hipError_t ie = hipGraphInstantiate(&c->graph[parity], g, nullptr, nullptr, 0);
  (void)hipGraphDestroy(g);
  if (ie != hipSuccess) {
    c->graph[parity] = nullptr;
    return hip_fail(c, ie, "instantiate graph");
  }
  return ESBGK_OK;
}

// Capture graph_steps / 2 in-place pairs on the buffer `parity`.
int build_pair_graph(esbgk_ctx* c, int parity) {
  if (!c->cap) {
    hipError_t e = hipStreamCreateWithFlags(&c->cap, hipStreamNonBlocking);
    if (e != hipSuccess) {
      c->cap = nullptr;
      return hip_fail(c, e, "create capture stream");
    }
  }
  HIP_OR_FAIL(c, hipStreamBeginCapture(c->cap, hipStreamCaptureModeRelaxed), "begin capture");
  hipError_t le = hipSuccess;
  for (int i = 0; i < c->graph_steps && le == hipSuccess; ++i) {
    StepArgs a = pair_args(c, 1 + (i & 1), parity);
    a.stream = c->cap;
    if (c->heating()) le = wall_tables(c, 1, c->cap);
    if (le == hipSuccess) le = launch_pair_step(c->shape.velset, c->shape.storage, 1 + (i & 1), a);
  }
  hipGraph_t g = nullptr;
  hipError_t ee = hipStreamEndCapture(c->cap, &g);
  if (le != hipSuccess) {
    if (g) (void)hipGraphDestroy(g);
    return hip_fail(c, le, "capture step pair");
  }
  if (ee != hipSuccess) return hip_fail(c, ee, "end capture");
  hipError_t ie = hipGraphInstantiate(&c->graph_pair[parity], g, nullptr, nullptr, 0);
  (void)hipGraphDestroy(g);
  if (ie != hipSuccess) {
    c->graph_pair[parity] = nullptr;
    return hip_fail(c, ie, "instantiate graph");
  }
  return ESBGK_OK;
}

int upload_params(esbgk_ctx* c) {
  const HostProblem hp =
      make_problem(*c->lat, c->n_ref, c->shape.scheme, c->Kn, c->Pr, c->varpi, c->g, c->Tw, c->uw, c->gam);
  pack_params<double>(hp, c->lat->Q, c->pp64);
  HIP_OR_FAIL(c, hipMemcpyAsync(c->at(c->lay.pp64), &c->pp64, sizeof(c->pp64), hipMemcpyHostToDevice, c->stream),
              "upload parameters");
  for (int side = 0; side < 2; ++side) {
    c->wprog.T[side] = c->Tw[side];
    c->wprog.amp[side] = c->heat_amp[side];
    c->wprog.freq[side] = c->heat_freq[side];
    for (int i = 0; i < 3; ++i) c->wprog.u[side][i] = c->uw[side][i];
  }
  c->wprog.dt = hp.dt;
  HIP_OR_FAIL(c, hipMemcpyAsync(c->at(c->lay.wprog), &c->wprog, sizeof(c->wprog), hipMemcpyHostToDevice, c->stream),
              "upload parameters");
  if (!c->f64()) {
    pack_params<float>(hp, c->lat->Q, c->pp32);
    HIP_OR_FAIL(c, hipMemcpyAsync(c->at(c->lay.pp), &c->pp32, sizeof(c->pp32), hipMemcpyHostToDevice, c->stream),
                "upload parameters");
  }
  // host-side copies must outlive the asynchronous copy
  HIP_OR_FAIL(c, hipStreamSynchronize(c->stream), "upload parameters");
  return ESBGK_OK;
}

int check_stable(const esbgk_ctx* c, double Kn, double Pr) {
  if (c->shape.scheme != ESBGK_EULER) return ESBGK_OK;
  const double dt = 1.0 / (double(c->n_ref) * c->lat->r);
  const double x = dt * Pr / Kn, y = dt / Kn;   // dt/tau and dt/(Pr tau) at rho = T = 1
  return (x < 2.0 && y < 2.0) ? ESBGK_OK : ESBGK_E_UNSTABLE;
}

int refresh_partials(esbgk_ctx* c) {
  if (!c->shape.walls) return ESBGK_OK;
  StepArgs a = base_args(c);
  a.wp_dst = c->at(c->lay.wp[c->cur]);
  HIP_OR_FAIL(c, launch_wall_partials(c->shape.velset, c->shape.storage, a), "wall partial sums");
  return ESBGK_OK;
}

int fetch_reduction(esbgk_ctx* c, double out[8], int64_t step) {
  double raw[NRED];
  HIP_OR_FAIL(c, hipMemcpyAsync(raw, c->at(c->lay.red_out), sizeof(raw), hipMemcpyDeviceToHost, c->stream),
              "read reduction");
  HIP_OR_FAIL(c, hipStreamSynchronize(c->stream), "read reduction");
  const int D = c->lat->D;
  const double dx = 1.0 / double(c->n_ref);
  out[0] = raw[0];
  out[1] = raw[1];
  out[2] = raw[2];
  out[3] = raw[3];
  out[4] = raw[4];
  out[5] = std::pow(dx, D - 1) / double(c->shape.nx) * raw[2];
  out[6] = raw[6] > 0.0 ? std::sqrt(raw[5] / raw[6]) : 0.0;
  out[7] = double(step);
  if (raw[7] != 0.0 || !std::isfinite(raw[0]) || !std::isfinite(raw[1])) {
    c->sticky = ESBGK_E_NONFINITE;
    c->err = "reduction found a non-finite value, rho <= 0 or T <= 0";
    return ESBGK_E_NONFINITE;
  }
  return ESBGK_OK;
}

#define CHECK_CTX(c)                         \
  do {                                       \
    if (!(c)) return ESBGK_E_INVALID;        \
    if ((c)->sticky) return (c)->sticky;     \
  } while (0)

}  // namespace

extern "C" {

int esbgk_lattice_info(int velset, int* Q, int* D, int* N, double* r, int* e, double* w) {
  const HostLattice* lat = host_lattice(velset);
  if (!lat) return ESBGK_E_INVALID;
  if (Q) *Q = lat->Q;
  if (D) *D = lat->D;
  if (N) *N = lat->N;
  if (r) *r = lat->r;
  if (e)
    for (int a = 0; a < lat->Q; ++a)
      for (int i = 0; i < lat->D; ++i) e[a * lat->D + i] = lat->e[size_t(a) * 3 + i];
  if (w)
    for (int a = 0; a < lat->Q; ++a) w[a] = lat->w[a];
  return ESBGK_OK;
}

size_t esbgk_workspace_bytes(const esbgk_shape* shape) {
  if (!valid_shape(shape, nullptr) || !host_lattice(shape->velset)) return 0;
  return layout_of(shape).total;
}

int esbgk_create(const esbgk_shape* shape, void* d_workspace, size_t ws_bytes, void* hip_stream, esbgk_ctx** out) {
  if (!out) return ESBGK_E_INVALID;
  *out = nullptr;
  std::string why;
  if (!valid_shape(shape, &why)) return ESBGK_E_INVALID;
  const HostLattice* lat = host_lattice(shape->velset);
  if (!lat) return ESBGK_E_INVALID;
  const Layout lay = layout_of(shape);
  if (!d_workspace || ws_bytes < lay.total) return ESBGK_E_NOMEM;
  if (reinterpret_cast<uintptr_t>(d_workspace) % ALIGN) return ESBGK_E_INVALID;
  esbgk_ctx* c = new esbgk_ctx();
  c->shape = *shape;
  c->lat = lat;
  c->lay = lay;
  c->ws = static_cast<char*>(d_workspace);
  c->stream = static_cast<hipStream_t>(hip_stream);
  if (hipGetDevice(&c->device) != hipSuccess) {
    g_create_error = "create: no current device";
    delete c;
    return ESBGK_E_HIP;
  }
  c->n_ref = shape->n_ref > 0 ? shape->n_ref : (shape->walls ? (lat->D == 2 ? shape->ny : shape->nz) : shape->nx);
  c->geo = geometry_of(shape);
  pack_lattice<double>(*lat, c->lc64);
  int rc = ESBGK_OK;
  auto hip = [&](hipError_t e, const char* where) {
    if (rc == ESBGK_OK && e != hipSuccess) {
      rc = ESBGK_E_HIP;
      g_create_error = std::string("create: ") + where + ": " + hipGetErrorString(e);
    }
  };
  hip(hipMemcpyAsync(c->at(lay.lc64), &c->lc64, sizeof(c->lc64), hipMemcpyHostToDevice, c->stream), "upload lattice");
  if (!c->f64()) {
    pack_lattice<float>(*lat, c->lc32);
    hip(hipMemcpyAsync(c->at(lay.lc), &c->lc32, sizeof(c->lc32), hipMemcpyHostToDevice, c->stream), "upload lattice");
  }
  if (rc == ESBGK_OK) {
    rc = upload_params(c);
    if (rc) g_create_error = c->err;
  }
  // wall partial sums start at zero (a state must be set before stepping)
  hip(hipMemsetAsync(c->at(lay.wp[0]), 0, lay.wp[1] - lay.wp[0], c->stream), "clear wall sums");
  hip(hipMemsetAsync(c->at(lay.wp[1]), 0, lay.wp[1] - lay.wp[0], c->stream), "clear wall sums");
  hip(hipStreamSynchronize(c->stream), "synchronize");
  if (rc != ESBGK_OK) {
    delete c;
    return rc;
  }
  *out = c;
  return ESBGK_OK;
}

int esbgk_destroy(esbgk_ctx* ctx) {
  if (!ctx) return ESBGK_E_INVALID;
  drop_graphs(ctx);
  if (ctx->cap) (void)hipStreamDestroy(ctx->cap);
  delete ctx;
  return ESBGK_OK;
}

int esbgk_set_graph_steps(esbgk_ctx* c, int steps) {
  CHECK_CTX(c);
  if (steps < 0 || steps % 2) return set_err(c, ESBGK_E_INVALID, "graph steps must be even and >= 0");
  if (steps != c->graph_steps) drop_graphs(c);
  c->graph_steps = steps;
  return ESBGK_OK;
}

int esbgk_set_inplace(esbgk_ctx* c, int mode) {
  CHECK_CTX(c);
  if (mode < 0 || mode > 2) return set_err(c, ESBGK_E_INVALID, "mode must be 0, 1 or 2");
  c->inplace = mode;
  return ESBGK_OK;
}

int esbgk_inplace_active(const esbgk_ctx* c) { return c ? (c->pairs() ? 1 : 0) : ESBGK_E_INVALID; }

int esbgk_set_gas(esbgk_ctx* c, double Kn, double Pr, double varpi) {
  CHECK_CTX(c);
  if (!(Kn > 0.0) || !std::isfinite(Kn)) return set_err(c, ESBGK_E_INVALID, "Kn must be > 0");
  if (!(Pr >= 2.0 / 3.0 - 1e-12) || !std::isfinite(Pr))
    return set_err(c, ESBGK_E_INVALID, "Pr must be >= 2/3 (b = 1 - 1/Pr >= -1/2)");
  if (!(varpi >= 0.5 && varpi <= 1.0)) return set_err(c, ESBGK_E_INVALID, "varpi must be in [0.5, 1]");
  if (check_stable(c, Kn, Pr) != ESBGK_OK)
    return set_err(c, ESBGK_E_UNSTABLE, "Euler step unstable: dt/tau or dt/(Pr tau) >= 2");
  c->Kn = Kn;
  c->Pr = Pr;
  c->varpi = varpi;
  return upload_params(c);
}

int esbgk_set_wall(esbgk_ctx* c, int side, double T_w, const double u_w[3]) {
  CHECK_CTX(c);
  if (!c->shape.walls) return set_err(c, ESBGK_E_INVALID, "lattice has no walls");
  if (side != 0 && side != 1) return set_err(c, ESBGK_E_INVALID, "side must be 0 or 1");
  if (!(T_w > 0.0) || !std::isfinite(T_w)) return set_err(c, ESBGK_E_INVALID, "T_w must be > 0");
  if (!u_w) return set_err(c, ESBGK_E_INVALID, "u_w is null");
  const int W = c->lat->D - 1;
  if (u_w[W] != 0.0) return set_err(c, ESBGK_E_INVALID, "wall velocity must be tangential");
  for (int i = 0; i < 3; ++i)
    if (!std::isfinite(u_w[i])) return set_err(c, ESBGK_E_INVALID, "u_w must be finite");
  if (!(T_w - std::fabs(c->heat_amp[side]) > 0.0))
    return set_err(c, ESBGK_E_INVALID, "the wall temperature must stay > 0 under the heating amplitude");
  c->Tw[side] = T_w;
  for (int i = 0; i < 3; ++i) c->uw[side][i] = i < c->lat->D ? u_w[i] : 0.0;
  return upload_params(c);
}

int esbgk_set_wall_accommodation(esbgk_ctx* c, int side, double gamma) {
  CHECK_CTX(c);
  if (!c->shape.walls) return set_err(c, ESBGK_E_INVALID, "lattice has no walls");
  if (side != 0 && side != 1) return set_err(c, ESBGK_E_INVALID, "side must be 0 or 1");
  if (!(gamma >= 0.0 && gamma <= 1.0)) return set_err(c, ESBGK_E_INVALID, "gamma must lie in [0, 1]");
  c->gam[side] = gamma;
  return upload_params(c);
}

int esbgk_set_wall_heating(esbgk_ctx* c, int side, double amplitude, double theta) {
  CHECK_CTX(c);
  if (!c->shape.walls) return set_err(c, ESBGK_E_INVALID, "lattice has no walls");
  if (side != 0 && side != 1) return set_err(c, ESBGK_E_INVALID, "side must be 0 or 1");
  if (!std::isfinite(amplitude) || !std::isfinite(theta))
    return set_err(c, ESBGK_E_INVALID, "amplitude and theta must be finite");
  if (!(c->Tw[side] - std::fabs(amplitude) > 0.0))
    return set_err(c, ESBGK_E_INVALID, "the wall temperature must stay > 0 (|amplitude| < T_w)");
  const bool was = c->heating();
  c->heat_amp[side] = amplitude;
  c->heat_freq[side] = theta;
  if (c->heating() != was) drop_graphs(c);   // captured graphs carry the table rebuilds or not
  int rc = upload_params(c);
  if (rc) return rc;
  return sync_level(c);
}

int esbgk_set_body_force(esbgk_ctx* c, const double g[3]) {
  CHECK_CTX(c);
  if (!g) return set_err(c, ESBGK_E_INVALID, "g is null");
  for (int i = 0; i < 3; ++i) {
    if (!std::isfinite(g[i])) return set_err(c, ESBGK_E_INVALID, "g must be finite");
    c->g[i] = i < c->lat->D ? g[i] : 0.0;
  }
  return upload_params(c);
}

int esbgk_init_equilibrium(esbgk_ctx* c, const double* rho, const double* u, const double* T, const double* noise,
                           double amplitude) {
  CHECK_CTX(c);
  if (noise && !std::isfinite(amplitude)) return set_err(c, ESBGK_E_INVALID, "amplitude must be finite");
  const uint32_t cells = c->geo.ncells;
  const int D = c->lat->D, Q = c->lat->Q;
  StepArgs a = base_args(c);
  a.dst = c->at(c->lay.pop[c->cur]);
  const bool staged = rho || u || T || noise;
  if (!staged) {
    HIP_OR_FAIL(c, launch_init(c->shape.velset, c->shape.storage, a, c->lat->r, nullptr, nullptr, nullptr, nullptr,
                               0.0, 0, cells),
                "init");
  } else {
    double* st = reinterpret_cast<double*>(c->at(c->lay.staging));
    for (uint32_t c0 = 0; c0 < cells; c0 += STAGE_CELLS) {
      const uint32_t n = std::min(STAGE_CELLS, cells - c0);
      double* d_rho = st;
      double* d_u = d_rho + n;
      double* d_T = d_u + size_t(D) * n;
      double* d_noise = d_T + n;
      if (rho) HIP_OR_FAIL(c, hipMemcpyAsync(d_rho, rho + c0, n * 8, hipMemcpyHostToDevice, c->stream), "stage");
      if (u)
        for (int d = 0; d < D; ++d)
          HIP_OR_FAIL(c, hipMemcpyAsync(d_u + size_t(d) * n, u + size_t(d) * cells + c0, n * 8,
                                        hipMemcpyHostToDevice, c->stream), "stage");
      if (T) HIP_OR_FAIL(c, hipMemcpyAsync(d_T, T + c0, n * 8, hipMemcpyHostToDevice, c->stream), "stage");
      if (noise)
        for (int q = 0; q < Q; ++q)
          HIP_OR_FAIL(c, hipMemcpyAsync(d_noise + size_t(q) * n, noise + size_t(q) * cells + c0, n * 8,
                                        hipMemcpyHostToDevice, c->stream), "stage");
      HIP_OR_FAIL(c, launch_init(c->shape.velset, c->shape.storage, a, c->lat->r, rho ? d_rho : nullptr,
                                 u ? d_u : nullptr, T ? d_T : nullptr, noise ? d_noise : nullptr, amplitude, c0, n),
                  "init");
      HIP_OR_FAIL(c, hipStreamSynchronize(c->stream), "init");
    }
  }
  int rc = refresh_partials(c);
  if (rc) return rc;
  HIP_OR_FAIL(c, hipStreamSynchronize(c->stream), "init");
  c->state_set = true;
  c->steps = 0;
  c->have_prev = 0;
  c->last_red_step = -1;
  return sync_level(c);
}

}  // extern "C"

namespace {

template <typename S>
void narrow_plane(const double* in, size_t n, std::vector<unsigned char>& out) {
  out.resize(n * sizeof(S));
  S* o = reinterpret_cast<S*>(out.data());
  for (size_t i = 0; i < n; ++i) o[i] = S(in[i]);
}

template <typename S>
void widen_plane(const unsigned char* in, size_t n, double* out) {
  const S* s = reinterpret_cast<const S*>(in);
  for (size_t i = 0; i < n; ++i) out[i] = double(s[i]);
}

// Copy velocity plane q of the current state between a dense host array
// [cells] of the storage type and the slice-blocked device layout.
hipError_t plane_to_device(esbgk_ctx* c, int q, const void* host) {
  const Geometry& g = c->geo;
  const size_t ss = storage_size(c->shape.storage);
  return hipMemcpy2DAsync(c->at(c->lay.pop[c->cur]) + size_t(q) * g.pstride * ss, size_t(g.sstride) * ss, host,
                          size_t(g.inner) * ss, size_t(g.inner) * ss, g.nslices, hipMemcpyHostToDevice, c->stream);
}

hipError_t plane_to_host(esbgk_ctx* c, int q, void* host) {
  const Geometry& g = c->geo;
  const size_t ss = storage_size(c->shape.storage);
  return hipMemcpy2DAsync(host, size_t(g.inner) * ss, c->at(c->lay.pop[c->cur]) + size_t(q) * g.pstride * ss,
                          size_t(g.sstride) * ss, size_t(g.inner) * ss, g.nslices, hipMemcpyDeviceToHost, c->stream);
}

}  // namespace

extern "C" {

int esbgk_set_populations(esbgk_ctx* c, const double* h) {
  CHECK_CTX(c);
  if (!h) return set_err(c, ESBGK_E_INVALID, "h is null");
  const size_t cells = c->geo.ncells;
  std::vector<unsigned char> buf;
  for (int q = 0; q < c->lat->Q; ++q) {
    const double* src = h + size_t(q) * cells;
    if (c->shape.storage == ESBGK_F64) {
      HIP_OR_FAIL(c, plane_to_device(c, q, src), "set populations");
      HIP_OR_FAIL(c, hipStreamSynchronize(c->stream), "set populations");
      continue;
    }
    if (c->shape.storage == ESBGK_F32) narrow_plane<float>(src, cells, buf);
    else narrow_plane<_Float16>(src, cells, buf);
    HIP_OR_FAIL(c, plane_to_device(c, q, buf.data()), "set populations");
    HIP_OR_FAIL(c, hipStreamSynchronize(c->stream), "set populations");
  }
  int rc = refresh_partials(c);
  if (rc) return rc;
  HIP_OR_FAIL(c, hipStreamSynchronize(c->stream), "set populations");
  c->state_set = true;
  c->steps = 0;
  c->have_prev = 0;
  c->last_red_step = -1;
  return sync_level(c);
}

int esbgk_get_populations(esbgk_ctx* c, double* h) {
  CHECK_CTX(c);
  if (!h) return set_err(c, ESBGK_E_INVALID, "h is null");
  if (!c->state_set) return set_err(c, ESBGK_E_STATE, "no state set");
  HIP_OR_FAIL(c, hipStreamSynchronize(c->stream), "get populations");
  const size_t cells = c->geo.ncells, ss = storage_size(c->shape.storage);
  std::vector<unsigned char> buf(cells * ss);
  for (int q = 0; q < c->lat->Q; ++q) {
    HIP_OR_FAIL(c, plane_to_host(c, q, buf.data()), "get populations");
    HIP_OR_FAIL(c, hipStreamSynchronize(c->stream), "get populations");
    double* o = h + size_t(q) * cells;
    if (c->shape.storage == ESBGK_F64) widen_plane<double>(buf.data(), cells, o);
    else if (c->shape.storage == ESBGK_F32) widen_plane<float>(buf.data(), cells, o);
    else widen_plane<_Float16>(buf.data(), cells, o);
  }
  return ESBGK_OK;
}

size_t esbgk_state_bytes(const esbgk_ctx* c) {
  if (!c) return 0;
  return size_t(c->lat->Q) * c->geo.ncells * storage_size(c->shape.storage) + sizeof(int64_t);
}

int esbgk_get_state(esbgk_ctx* c, void* h_raw, size_t nbytes) {
  CHECK_CTX(c);
  if (!h_raw || nbytes != esbgk_state_bytes(c)) return set_err(c, ESBGK_E_INVALID, "state buffer size mismatch");
  if (!c->state_set) return set_err(c, ESBGK_E_STATE, "no state set");
  const size_t pop = nbytes - sizeof(int64_t);
  const size_t plane = pop / size_t(c->lat->Q);
  HIP_OR_FAIL(c, hipStreamSynchronize(c->stream), "get state");
  for (int q = 0; q < c->lat->Q; ++q)
    HIP_OR_FAIL(c, plane_to_host(c, q, static_cast<char*>(h_raw) + size_t(q) * plane), "get state");
  HIP_OR_FAIL(c, hipStreamSynchronize(c->stream), "get state");
  std::memcpy(static_cast<char*>(h_raw) + pop, &c->steps, sizeof(int64_t));
  return ESBGK_OK;
}

int esbgk_set_state(esbgk_ctx* c, const void* h_raw, size_t nbytes) {
  CHECK_CTX(c);
  if (!h_raw || nbytes != esbgk_state_bytes(c)) return set_err(c, ESBGK_E_INVALID, "state buffer size mismatch");
  const size_t pop = nbytes - sizeof(int64_t);
  const size_t plane = pop / size_t(c->lat->Q);
  HIP_OR_FAIL(c, hipStreamSynchronize(c->stream), "set state");
  for (int q = 0; q < c->lat->Q; ++q)
    HIP_OR_FAIL(c, plane_to_device(c, q, static_cast<const char*>(h_raw) + size_t(q) * plane), "set state");
  int rc = refresh_partials(c);
  if (rc) return rc;
  HIP_OR_FAIL(c, hipStreamSynchronize(c->stream), "set state");
  std::memcpy(&c->steps, static_cast<const char*>(h_raw) + pop, sizeof(int64_t));
  c->state_set = true;
  c->have_prev = 0;
  return sync_level(c);
}

int esbgk_step(esbgk_ctx* c, int64_t n) {
  CHECK_CTX(c);
  if (n < 0) return set_err(c, ESBGK_E_INVALID, "n must be >= 0");
  if (!c->state_set) return set_err(c, ESBGK_E_STATE, "no state set");
  const uint32_t nblocks = slot_blocks(c->geo);
  const int64_t G = c->graph_steps;
  if (G > 0 && n > 0) {
    // capture the graphs of both buffers up front, so that no replay waits
    // for a capture (an odd step count moves the state to the other buffer)
    for (int p = 0; p < 2; ++p) {
      hipGraphExec_t have = c->pairs() ? c->graph_pair[p] : c->graph[p];
      if (!have) {
        const int rc = c->pairs() ? build_pair_graph(c, p) : build_graph(c, p);
        if (rc) return rc;
      }
    }
  }
  while (n > 0) {
    // a whole graph when no fused reduction falls inside its G steps
    const bool red_inside = c->R > 0 && ((c->steps / c->R) + 1) * c->R <= c->steps + G;
    // in-place pairs take an even count; an odd count's single two-buffer
    // step comes first, so that the pairs run on the buffer the state ends in
    const bool pairs = c->pairs() && n % 2 == 0;
    if (pairs) {
      if (G > 0 && n >= G && !red_inside) {
        if (!c->graph_pair[c->cur]) {
          const int rc = build_pair_graph(c, c->cur);
          if (rc) return rc;
        }
        HIP_OR_FAIL(c, hipGraphLaunch(c->graph_pair[c->cur], c->stream), "graph launch");
        c->steps += G;
        n -= G;
        continue;
      }
      for (int phase = 1; phase <= 2; ++phase) {
        StepArgs a = pair_args(c, phase, c->cur);
        const bool red = c->R > 0 && ((c->steps + 1) % c->R == 0);
        a.reduce = red ? 1 : 0;
        if (c->heating()) HIP_OR_FAIL(c, wall_tables(c, 1, c->stream), "wall tables");
        HIP_OR_FAIL(c, launch_pair_step(c->shape.velset, c->shape.storage, phase, a), "step");
        if (red) {
          HIP_OR_FAIL(c, launch_reduce_finalize(a.red_part, nblocks,
                                                reinterpret_cast<double*>(c->at(c->lay.red_out)), c->stream),
                      "reduce");
          c->have_prev = 1;
          c->last_red_step = c->steps;
        }
        c->steps += 1;
      }
      n -= 2;
      continue;
    }
    if (!c->pairs() && G > 0 && n >= G && !red_inside) {
      if (!c->graph[c->cur]) {
        const int rc = build_graph(c, c->cur);
        if (rc) return rc;
      }
      HIP_OR_FAIL(c, hipGraphLaunch(c->graph[c->cur], c->stream), "graph launch");
      c->steps += G;   // G is even: the state ends in the same buffer
      n -= G;
      continue;
    }
    StepArgs a = base_args(c);
    const bool red = c->R > 0 && ((c->steps + 1) % c->R == 0);
    a.reduce = red ? 1 : 0;
    if (c->heating()) HIP_OR_FAIL(c, wall_tables(c, 1, c->stream), "wall tables");
    HIP_OR_FAIL(c, launch_step(c->shape.velset, c->shape.storage, a), "step");
    if (red) {
      HIP_OR_FAIL(c, launch_reduce_finalize(a.red_part, nblocks, reinterpret_cast<double*>(c->at(c->lay.red_out)),
                                            c->stream), "reduce");
      c->have_prev = 1;
      c->last_red_step = c->steps;
    }
    c->cur ^= 1;
    c->steps += 1;
    n -= 1;
  }
  return ESBGK_OK;
}

int esbgk_read_moments(esbgk_ctx* c, double* h_out, int* F) {
  CHECK_CTX(c);
  if (!h_out) return set_err(c, ESBGK_E_INVALID, "h_out is null");
  if (!c->state_set) return set_err(c, ESBGK_E_STATE, "no state set");
  const int nf = nfields(c->lat->D);
  if (F) *F = nf;
  const uint32_t cells = c->geo.ncells;
  double* st = reinterpret_cast<double*>(c->at(c->lay.staging));
  std::vector<double> tmp;
  StepArgs a = base_args(c);
  if (c->heating()) HIP_OR_FAIL(c, wall_tables(c, 0, c->stream), "wall tables");
  for (uint32_t c0 = 0; c0 < cells; c0 += STAGE_CELLS) {
    const uint32_t n = std::min(STAGE_CELLS, cells - c0);
    HIP_OR_FAIL(c, launch_moments(c->shape.velset, c->shape.storage, a, c0, n, st), "moments");
    tmp.resize(size_t(nf) * n);
    HIP_OR_FAIL(c, hipMemcpyAsync(tmp.data(), st, tmp.size() * 8, hipMemcpyDeviceToHost, c->stream), "moments");
    HIP_OR_FAIL(c, hipStreamSynchronize(c->stream), "moments");
    for (int f = 0; f < nf; ++f) std::memcpy(h_out + size_t(f) * cells + c0, tmp.data() + size_t(f) * n, n * 8);
  }
  return ESBGK_OK;
}

int esbgk_reduce(esbgk_ctx* c, double out[8]) {
  CHECK_CTX(c);
  if (!out) return set_err(c, ESBGK_E_INVALID, "out is null");
  if (!c->state_set) return set_err(c, ESBGK_E_STATE, "no state set");
  const uint32_t nblocks = slot_blocks(c->geo);
  StepArgs a = base_args(c);
  if (c->heating()) HIP_OR_FAIL(c, wall_tables(c, 0, c->stream), "wall tables");
  HIP_OR_FAIL(c, launch_reduce(c->shape.velset, c->shape.storage, a), "reduce");
  HIP_OR_FAIL(c, launch_reduce_finalize(a.red_part, nblocks, reinterpret_cast<double*>(c->at(c->lay.red_out)),
                                        c->stream), "reduce");
  c->have_prev = 1;
  c->last_red_step = c->steps;
  return fetch_reduction(c, out, c->steps);
}

int esbgk_reduce_noalloc(esbgk_ctx* c, double out[8]) {
  CHECK_CTX(c);
  if (!out) return set_err(c, ESBGK_E_INVALID, "out is null");
  if (!c->state_set) return set_err(c, ESBGK_E_STATE, "no state set");
  double* scr = nullptr;
  HIP_OR_FAIL(c, noalloc_scratch(c->device, &scr), "scratch address");
  StepArgs a = base_args(c);
  if (c->heating()) HIP_OR_FAIL(c, wall_tables(c, 0, c->stream), "wall tables");
  HIP_OR_FAIL(c, launch_reduce_noalloc(c->shape.velset, c->shape.storage, a, scr), "reduce");
  // the sums become the handle's latest reduction, as with esbgk_reduce
  HIP_OR_FAIL(c, hipMemcpyAsync(c->at(c->lay.red_out), scr + size_t(NOALLOC_PARTS) * NRED, NRED * sizeof(double),
                                hipMemcpyDeviceToDevice, c->stream), "reduce");
  c->have_prev = 1;
  c->last_red_step = c->steps;
  return fetch_reduction(c, out, c->steps);
}

int esbgk_set_reduce_interval(esbgk_ctx* c, int64_t R) {
  CHECK_CTX(c);
  if (R < 0) return set_err(c, ESBGK_E_INVALID, "R must be >= 0");
  c->R = R;
  return ESBGK_OK;
}

int esbgk_last_reduction(esbgk_ctx* c, double out[8]) {
  CHECK_CTX(c);
  if (!out) return set_err(c, ESBGK_E_INVALID, "out is null");
  if (c->last_red_step < 0) return set_err(c, ESBGK_E_STATE, "no reduction has run");
  return fetch_reduction(c, out, c->last_red_step);
}

int64_t esbgk_steps_done(const esbgk_ctx* c) { return c ? c->steps : -1; }

const char* esbgk_last_error(const esbgk_ctx* c) { return c ? c->err.c_str() : g_create_error.c_str(); }

}  // extern "C"
