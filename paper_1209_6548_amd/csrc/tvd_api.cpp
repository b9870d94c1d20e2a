// C ABI of the paper's own scheme (Sec. 3.1) on the Gauss-Hermite product
// sets (2-D: 4, 6 or 8 points per axis; 3-D: the paper's 6-point cube):
// handle management, validation, workspace layout, parameter upload, state
// I/O and the step loop.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstring>
#include <string>
#include <vector>

#include "../../include/esbgk.h"
#include "gh3.h"
#include "tables.h"
#include "tvd.h"

using namespace esbgk;

namespace {

constexpr size_t ALIGN = 256;
constexpr uint32_t STAGE_CELLS = 65536;

// The host view of a product set: dimension, sizes, abscissae c[Q][D],
// weights and the largest root (max |c| along an axis).
struct SetTab {
  int velset = 0, D = 0, Q = 0, P = 0, N = 0;
  double cmax = 0.0;
  const double* c = nullptr;
  const double* w = nullptr;
};

bool set_tab(int velset, SetTab& t) {
  t.velset = velset;
  if (velset == ESBGK_D3Q216GH) {
    const HostGH3* g = host_gh3();
    if (!g) return false;
    t.D = 3;
    t.Q = 216;
    t.P = 108;
    t.N = 4;
    t.cmax = g->xi[2];
    t.c = &g->c[0][0];
    t.w = g->w;
    return true;
  }
  const int n = velset == ESBGK_D2Q16GH ? 4 : (velset == ESBGK_D2Q36GH ? 6 : (velset == ESBGK_D2Q64GH ? 8 : 0));
  const HostGH* g = n ? host_gh(n) : nullptr;
  if (!g) return false;
  t.D = 2;
  t.Q = g->Q;
  t.P = g->P;
  t.N = g->N;
  t.cmax = g->xi[n / 2 - 1];
  t.c = &g->c[0][0];
  t.w = g->w;
  return true;
}

int nfields(int D) { return D == 3 ? 14 : 9; }
size_t align_up(size_t n) { return (n + ALIGN - 1) / ALIGN * ALIGN; }
size_t ssize(int storage) { return storage == ESBGK_F64 ? 8 : (storage == ESBGK_F32 ? 4 : 2); }
size_t csize(int storage) { return storage == ESBGK_F64 ? 8 : 4; }

struct TLayout {
  size_t pop[2], mom[2], gc, lc, pp, gc64, lc64, pp64, walls, c, staging, total;
};

bool gh3_groups_ok(const SetTab& t);

bool valid_tvd_shape(const esbgk_shape* s, Geometry* g, std::string* why) {
  auto fail = [&](const char* m) { if (why) *why = m; return false; };
  if (!s) return fail("null shape");
  SetTab t;
  if (!set_tab(s->velset, t))
    return fail("velset must be ESBGK_D2Q16GH, ESBGK_D2Q36GH, ESBGK_D2Q64GH or ESBGK_D3Q216GH");
  if (t.D == 3 && !gh3_groups_ok(t)) return fail("internal: the D3Q216 representatives do not form 18 groups of six");
  if (s->nx < 1 || s->ny < 1 || s->nz < 1) return fail("extents must be >= 1");
  if (t.D == 2 && s->nz != 1) return fail("a 2-D set needs nz = 1");
  if (s->walls != 0 && s->walls != 1) return fail("walls must be 0 (periodic) or 1 (walls across the last axis)");
  const int nwall = t.D == 2 ? s->ny : s->nz;
  if (s->walls && nwall < 3) return fail("a channel needs three nodes across it (two wall nodes and one between)");
  if (s->storage < ESBGK_F64 || s->storage > ESBGK_F16) return fail("storage must be F64, F32 or F16");
  if (s->scheme != ESBGK_EULER) return fail("the paper's scheme is forward Euler (scheme = ESBGK_EULER)");
  if (s->n_ref < 0) return fail("n_ref must be >= 0");
  Geometry tmp;
  if (!make_geometry(t.D, t.Q, uint32_t(s->nx), uint32_t(s->ny), uint32_t(s->nz), s->walls != 0, true,
                     ssize(s->storage), g ? *g : tmp))
    return fail("lattice too large for the slice layout (one slice of populations must be < 4 GiB)");
  return true;
}

template <int D, typename C>
using ConstsOf = typename std::conditional<D == 3, GH3Consts<C>, GHConsts<C>>::type;
template <int D, typename C>
using WallsOf = typename std::conditional<D == 3, TVDWalls3<C>, TVDWalls<C>>::type;

TLayout tlayout(const esbgk_shape* s, const Geometry& g) {
  SetTab t;
  set_tab(s->velset, t);
  TLayout L{};
  const size_t ss = ssize(s->storage), cs = csize(s->storage);
  const size_t cells = size_t(s->nx) * s->ny * s->nz;
  const bool d3 = t.D == 3;
  const size_t gc64 = d3 ? sizeof(ConstsOf<3, double>) : sizeof(ConstsOf<2, double>);
  const size_t gc32 = d3 ? sizeof(ConstsOf<3, float>) : sizeof(ConstsOf<2, float>);
  const size_t w64 = d3 ? sizeof(WallsOf<3, double>) : sizeof(WallsOf<2, double>);
  const size_t w32 = d3 ? sizeof(WallsOf<3, float>) : sizeof(WallsOf<2, float>);
  size_t off = 0;
  auto take = [&](size_t bytes) { const size_t o = off; off = align_up(off + bytes); return o; };
  L.pop[0] = take(size_t(g.nslices) * g.sstride * ss);
  L.pop[1] = take(size_t(g.nslices) * g.sstride * ss);
  // D3Q216: each level's raw moment sums, [MOM3][nslices * ipad] of the compute type
  const size_t mom = d3 ? size_t(MOM3) * g.nslices * g.ipad * cs : 0;
  L.mom[0] = take(mom);
  L.mom[1] = take(mom);
  L.gc = take(cs == 8 ? gc64 : gc32);
  L.lc = take(cs == 8 ? sizeof(LatConsts<double>) : sizeof(LatConsts<float>));
  L.pp = take(cs == 8 ? sizeof(ProbParams<double>) : sizeof(ProbParams<float>));
  L.gc64 = cs == 8 ? L.gc : take(gc64);
  L.lc64 = cs == 8 ? L.lc : take(sizeof(LatConsts<double>));
  L.pp64 = cs == 8 ? L.pp : take(sizeof(ProbParams<double>));
  L.walls = take(cs == 8 ? w64 : w32);
  L.c = take(sizeof(double) * size_t(t.Q) * t.D);
  const size_t stage = std::min<size_t>(cells, STAGE_CELLS);
  // init stages rho, u[D], T and noise[Q]; the read-out stages the fields
  L.staging = take(stage * size_t(std::max(nfields(t.D), 2 + t.D + t.Q)) * sizeof(double));
  L.total = off;
  return L;
}

// Per-set constants of the kernels: weights, monomials, Courant numbers.
template <typename C>
void pack_consts(const SetTab& t, double nu_scale, GHConsts<C>& d) {
  std::memset(&d, 0, sizeof(d));
  for (int p = 0; p < t.P; ++p) {
    const double x = t.c[2 * p], y = t.c[2 * p + 1];
    const double m[GH_MONO] = {x,         y,         x * x,         x * y,         y * y,
                               x * x * x, x * x * y, x * y * y,     y * y * y,     x * x * x * x,
                               x * x * x * y, x * x * y * y, x * y * y * y, y * y * y * y};
    d.w[p] = C(t.w[p]);
    for (int k = 0; k < GH_MONO; ++k) d.mono[p][k] = C(m[k]);
    for (int i = 0; i < 2; ++i) {
      const double nu = t.c[2 * p + i] * nu_scale;
      d.nu[p][i] = C(nu);
      d.nk[p][i] = C(0.5 * std::fabs(nu) * (1.0 - std::fabs(nu)));
    }
  }
}

template <typename C>
void pack_consts(const SetTab& t, double nu_scale, GH3Consts<C>& d) {
  std::memset(&d, 0, sizeof(d));
  for (int p = 0; p < t.P; ++p) {
    const double* cp = t.c + 3 * p;
    d.w[p] = C(t.w[p]);
    for (int k = 0; k < GH3_MONO; ++k) {
      double v = 1.0;
      for (int j = 0; j < MONO3.deg[k]; ++j) v *= cp[MONO3.idx[k][j]];
      d.mono[p][k] = C(v);
    }
    for (int i = 0; i < 3; ++i) {
      const double nu = cp[i] * nu_scale;
      d.nu[p][i] = C(nu);
      d.nk[p][i] = C(0.5 * std::fabs(nu) * (1.0 - std::fabs(nu)));
    }
  }
  // visiting order: the representatives grouped by (c_x, c_y) in order of
  // first appearance, each group's members in velocity order
  int j = 0, g = 0;
  std::vector<bool> taken(size_t(t.P), false);
  for (int p = 0; p < t.P; ++p) {
    if (taken[size_t(p)]) continue;
    const double* cp = t.c + 3 * p;
    for (int k = 0; k < GH3_MONO; ++k) {
      double v = 1.0;
      for (int e = 0; e < MONO3.deg[k]; ++e)
        if (MONO3.idx[k][e] != 2) v *= cp[MONO3.idx[k][e]];
      d.gxy[g][k] = C(v);
    }
    for (int q = p; q < t.P; ++q) {
      const double* cq = t.c + 3 * q;
      if (taken[size_t(q)] || cq[0] != cp[0] || cq[1] != cp[1]) continue;
      taken[size_t(q)] = true;
      d.order[j] = q;
      d.cz[j] = C(cq[2]);
      ++j;
    }
    ++g;
  }
}

// Whether the representatives form GH3_GROUPS groups of GH3_GROUP that share
// (c_x, c_y), which the grouped collision of the 3-D kernel assumes.
bool gh3_groups_ok(const SetTab& t) {
  std::vector<bool> taken(size_t(t.P), false);
  int groups = 0;
  for (int p = 0; p < t.P; ++p) {
    if (taken[size_t(p)]) continue;
    int n = 0;
    for (int q = p; q < t.P; ++q)
      if (!taken[size_t(q)] && t.c[3 * q] == t.c[3 * p] && t.c[3 * q + 1] == t.c[3 * p + 1]) {
        taken[size_t(q)] = true;
        ++n;
      }
    if (n != GH3_GROUP) return false;
    ++groups;
  }
  return groups == GH3_GROUPS;
}

// Wall tables of Sec. 3.2 (see TVDWalls) from the walls' T and u; the walls
// lie across the last axis.
template <class W>
void pack_walls(const SetTab& t, const double Tw[2], const double uw[2][3], W& d) {
  using C = typename std::remove_reference<decltype(d.k0[0])>::type;
  std::memset(&d, 0, sizeof(d));
  std::vector<double> sw(size_t(t.Q));
  for (int side = 0; side < 2; ++side) {
    const double nrm = side == 0 ? 1.0 : -1.0;   // inward normal along the last axis
    double den = 0.0;
    for (int a = 0; a < t.Q; ++a) {
      sw[a] = 1.0 + shat_minus_one_at(t.D, t.N, t.c + size_t(a) * t.D, Tw[side], uw[side]);
      const double cn = nrm * t.c[size_t(a) * t.D + t.D - 1];
      if (cn > 0) den += cn * t.w[a] * sw[a];
    }
    double k0 = 0.0;
    for (int a = 0; a < t.Q; ++a) {
      const double cn = nrm * t.c[size_t(a) * t.D + t.D - 1];
      if (cn < 0) {
        const double k = -cn * t.w[a] / den;
        d.kin[side][a] = C(k);
        k0 += k;
      } else {
        d.sw[side][a] = C(sw[a]);
      }
    }
    d.k0[side] = C(k0);
  }
}

}  // namespace

struct esbgk_tvd {
  esbgk_shape shape{};
  Geometry geo{};
  TLayout lay{};
  char* ws = nullptr;
  hipStream_t stream = nullptr;
  int cur = 0;
  bool state_set = false;
  bool mom_ok = false;          // D3Q216: lay.mom[cur] holds the sums of lay.pop[cur]
  int64_t steps = 0;
  int sticky = 0;
  std::string err;
  double Kn = 0.1, Pr = 1.0, varpi = 0.5, cfl = 0.5, dt = 0.0, dx = 0.0;
  double g[3] = {0, 0, 0};
  SetTab set;                   // the velocity set's host tables
  double Tw[2] = {1.0, 1.0};
  double uw[2][3] = {{0, 0, 0}, {0, 0, 0}};
  char* at(size_t off) const { return ws + off; }
  bool f64() const { return shape.storage == ESBGK_F64; }
};

namespace {

thread_local std::string g_tvd_create_error;

int tset_err(esbgk_tvd* c, int code, const std::string& msg) {
  if (c) c->err = msg;
  return code;
}

int thip_fail(esbgk_tvd* c, hipError_t e, const char* where) {
  c->sticky = ESBGK_E_HIP;
  c->err = std::string(where) + ": " + hipGetErrorString(e);
  return ESBGK_E_HIP;
}

#define TVD_HIP(ctx, expr, where)                                  \
  do {                                                             \
    hipError_t _e = (expr);                                        \
    if (_e != hipSuccess) return thip_fail(ctx, _e, where);        \
  } while (0)

#define TVD_CHECK(c)                         \
  do {                                       \
    if (!(c)) return ESBGK_E_INVALID;        \
    if ((c)->sticky) return (c)->sticky;     \
  } while (0)

TVDArgs targs(const esbgk_tvd* c) {
  TVDArgs a{};
  a.geo = c->geo;
  a.src = c->at(c->lay.pop[c->cur]);
  a.dst = c->at(c->lay.pop[1 - c->cur]);
  a.gc = c->at(c->lay.gc);
  a.lc = c->at(c->lay.lc);
  a.pp = c->at(c->lay.pp);
  a.gc64 = c->at(c->lay.gc64);
  a.lc64 = c->at(c->lay.lc64);
  a.pp64 = c->at(c->lay.pp64);
  a.msrc = c->set.D == 3 ? c->at(c->lay.mom[c->cur]) : nullptr;
  a.mdst = c->set.D == 3 ? c->at(c->lay.mom[1 - c->cur]) : nullptr;
  a.stream = c->stream;
  return a;
}

template <int D>
int upload_consts(esbgk_tvd* c, double nu_scale);

// Gas, force and the Courant-limited time step: dt = CFL dx / max|c|.
// Waits for the stream when it leaves scope, also on an early error return:
// the uploads read thread-local host blocks that the next call refills.
struct StreamIdleOnExit {
  hipStream_t s;
  ~StreamIdleOnExit() { (void)hipStreamSynchronize(s); }
};

int upload_tvd(esbgk_tvd* c) {
  const StreamIdleOnExit idle{c->stream};
  HostProblem hp{};
  hp.dt = c->dt;
  hp.hs = 0.0;
  hp.hsdt = 0.0;
  hp.xcoef = c->dt * c->Pr / c->Kn;
  hp.omv = 1.0 - c->varpi;
  hp.invPr = 1.0 / c->Pr;
  hp.b = 1.0 - 1.0 / c->Pr;
  hp.force = 0;
  for (int i = 0; i < 3; ++i) {
    hp.g[i] = i < c->set.D ? c->g[i] : 0.0;
    if (hp.g[i] != 0.0) hp.force = 1;
  }
  hp.gam[0] = hp.gam[1] = 1.0;
  static thread_local ProbParams<double> pp64;
  static thread_local ProbParams<float> pp32;
  static thread_local LatConsts<double> l64;
  static thread_local LatConsts<float> l32;
  pack_params<double>(hp, 0, pp64);   // the wall tables of ProbParams are not used here
  std::memset(&l64, 0, sizeof(l64));
  l64.r = 1.0;                        // the weights live in the set constants
  TVD_HIP(c, hipMemcpyAsync(c->at(c->lay.pp64), &pp64, sizeof(pp64), hipMemcpyHostToDevice, c->stream), "upload");
  TVD_HIP(c, hipMemcpyAsync(c->at(c->lay.lc64), &l64, sizeof(l64), hipMemcpyHostToDevice, c->stream), "upload");
  if (!c->f64()) {
    pack_params<float>(hp, 0, pp32);
    std::memset(&l32, 0, sizeof(l32));
    l32.r = 1.0f;
    TVD_HIP(c, hipMemcpyAsync(c->at(c->lay.pp), &pp32, sizeof(pp32), hipMemcpyHostToDevice, c->stream), "upload");
    TVD_HIP(c, hipMemcpyAsync(c->at(c->lay.lc), &l32, sizeof(l32), hipMemcpyHostToDevice, c->stream), "upload");
  }
  const int rc = c->set.D == 3 ? upload_consts<3>(c, c->dt / c->dx) : upload_consts<2>(c, c->dt / c->dx);
  if (rc) return rc;
  TVD_HIP(c, hipStreamSynchronize(c->stream), "upload");
  return ESBGK_OK;
}

// The set constants (FP64 always, the compute type too) and the wall
// tables; the host copies stay alive until the synchronisation above.
template <int D>
int upload_consts(esbgk_tvd* c, double nu_scale) {
  static thread_local ConstsOf<D, double> g64;
  static thread_local ConstsOf<D, float> g32;
  static thread_local WallsOf<D, double> w64;
  static thread_local WallsOf<D, float> w32;
  pack_consts<double>(c->set, nu_scale, g64);
  TVD_HIP(c, hipMemcpyAsync(c->at(c->lay.gc64), &g64, sizeof(g64), hipMemcpyHostToDevice, c->stream), "upload");
  if (!c->f64()) {
    pack_consts<float>(c->set, nu_scale, g32);
    TVD_HIP(c, hipMemcpyAsync(c->at(c->lay.gc), &g32, sizeof(g32), hipMemcpyHostToDevice, c->stream), "upload");
  }
  if (c->shape.walls) {
    if (c->f64()) {
      pack_walls(c->set, c->Tw, c->uw, w64);
      TVD_HIP(c, hipMemcpyAsync(c->at(c->lay.walls), &w64, sizeof(w64), hipMemcpyHostToDevice, c->stream), "upload");
    } else {
      pack_walls(c->set, c->Tw, c->uw, w32);
      TVD_HIP(c, hipMemcpyAsync(c->at(c->lay.walls), &w32, sizeof(w32), hipMemcpyHostToDevice, c->stream), "upload");
    }
  }
  return ESBGK_OK;
}

template <typename S>
void narrow_to(const double* in, size_t n, std::vector<unsigned char>& out) {
  out.resize(n * sizeof(S));
  S* o = reinterpret_cast<S*>(out.data());
  for (size_t i = 0; i < n; ++i) o[i] = S(in[i]);
}

template <typename S>
void widen_from(const unsigned char* in, size_t n, double* out) {
  const S* s = reinterpret_cast<const S*>(in);
  for (size_t i = 0; i < n; ++i) out[i] = double(s[i]);
}

hipError_t tplane_to_device(esbgk_tvd* c, int q, const void* host) {
  const Geometry& g = c->geo;
  const size_t ss = ssize(c->shape.storage);
  return hipMemcpy2DAsync(c->at(c->lay.pop[c->cur]) + size_t(q) * g.pstride * ss, size_t(g.sstride) * ss, host,
                          size_t(g.inner) * ss, size_t(g.inner) * ss, g.nslices, hipMemcpyHostToDevice, c->stream);
}

hipError_t tplane_to_host(esbgk_tvd* c, int q, void* host) {
  const Geometry& g = c->geo;
  const size_t ss = ssize(c->shape.storage);
  return hipMemcpy2DAsync(host, size_t(g.inner) * ss, c->at(c->lay.pop[c->cur]) + size_t(q) * g.pstride * ss,
                          size_t(g.sstride) * ss, size_t(g.inner) * ss, g.nslices, hipMemcpyDeviceToHost, c->stream);
}

}  // namespace

extern "C" {

int esbgk_tvd_set_info(int velset, int* Q, int* N, double* c, double* w) {
  SetTab t;
  if (!set_tab(velset, t)) return ESBGK_E_INVALID;
  if (Q) *Q = t.Q;
  if (N) *N = t.N;
  if (c) std::memcpy(c, t.c, sizeof(double) * size_t(t.Q) * t.D);
  if (w) std::memcpy(w, t.w, sizeof(double) * size_t(t.Q));
  return ESBGK_OK;
}

int esbgk_tvd_info(double* c, double* w) { return esbgk_tvd_set_info(ESBGK_D2Q36GH, nullptr, nullptr, c, w); }

size_t esbgk_tvd_workspace_bytes(const esbgk_shape* shape) {
  Geometry g;
  if (!valid_tvd_shape(shape, &g, nullptr)) return 0;
  return tlayout(shape, g).total;
}

int esbgk_tvd_create(const esbgk_shape* shape, double cfl, void* d_workspace, size_t ws_bytes, void* hip_stream,
                     esbgk_tvd** out) {
  if (!out) return ESBGK_E_INVALID;
  *out = nullptr;
  Geometry g;
  if (!valid_tvd_shape(shape, &g, &g_tvd_create_error)) return ESBGK_E_INVALID;
  if (!(cfl > 0.0 && cfl <= 1.0)) {
    g_tvd_create_error = "cfl must lie in (0, 1]";
    return ESBGK_E_INVALID;
  }
  const TLayout lay = tlayout(shape, g);
  if (!d_workspace || ws_bytes < lay.total) {
    g_tvd_create_error = "workspace missing or too small";
    return ESBGK_E_NOMEM;
  }
  if (reinterpret_cast<uintptr_t>(d_workspace) % ALIGN) {
    g_tvd_create_error = "workspace must be 256-byte aligned";
    return ESBGK_E_INVALID;
  }
  esbgk_tvd* c = new esbgk_tvd();
  c->shape = *shape;
  c->geo = g;
  c->lay = lay;
  c->ws = static_cast<char*>(d_workspace);
  c->stream = static_cast<hipStream_t>(hip_stream);
  c->cfl = cfl;
  set_tab(shape->velset, c->set);
  const int nwall = c->set.D == 2 ? shape->ny : shape->nz;
  const int n_ref = shape->n_ref > 0 ? shape->n_ref : (shape->walls ? nwall - 1 : shape->nx);
  c->dx = 1.0 / double(n_ref);
  c->dt = cfl * c->dx / c->set.cmax;
  hipError_t e = hipMemcpyAsync(c->at(lay.c), c->set.c, sizeof(double) * size_t(c->set.Q) * c->set.D,
                                hipMemcpyHostToDevice, c->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
  if (e != hipSuccess) {
    g_tvd_create_error = std::string("create: ") + hipGetErrorString(e);
    delete c;
    return ESBGK_E_HIP;
  }
  const int rc = upload_tvd(c);
  if (rc) {
    g_tvd_create_error = c->err;
    delete c;
    return rc;
  }
  *out = c;
  return ESBGK_OK;
}

int esbgk_tvd_destroy(esbgk_tvd* c) {
  if (!c) return ESBGK_E_INVALID;
  delete c;
  return ESBGK_OK;
}

double esbgk_tvd_time_step(const esbgk_tvd* c) { return c ? c->dt : 0.0; }

int esbgk_tvd_bounded(int velset, int n_ref, double cfl, double Kn, double Pr, int axes) {
  SetTab t;
  if (!set_tab(velset, t)) return ESBGK_E_INVALID;
  if (n_ref < 1 || !(cfl > 0.0 && cfl <= 1.0) || !(Kn > 0.0) || !std::isfinite(Kn) ||
      !(Pr >= 2.0 / 3.0 - 1e-12) || !std::isfinite(Pr) || axes < 1 || axes > t.D)
    return ESBGK_E_INVALID;
  const double dt = cfl / (double(n_ref) * t.cmax);
  const double w = dt * Pr / Kn;   // dt/tau at rho = T = 1
  return double(axes) * cfl <= 1.0 - w ? ESBGK_OK : ESBGK_E_UNSTABLE;
}

int esbgk_tvd_set_gas(esbgk_tvd* c, double Kn, double Pr, double varpi) {
  TVD_CHECK(c);
  if (!(Kn > 0.0) || !std::isfinite(Kn)) return tset_err(c, ESBGK_E_INVALID, "Kn must be > 0");
  if (!(Pr >= 2.0 / 3.0 - 1e-12) || !std::isfinite(Pr)) return tset_err(c, ESBGK_E_INVALID, "Pr must be >= 2/3");
  if (!(varpi >= 0.5 && varpi <= 1.0)) return tset_err(c, ESBGK_E_INVALID, "varpi must lie in [0.5, 1]");
  if (c->dt * Pr / Kn >= 2.0 || c->dt / Kn >= 2.0)
    return tset_err(c, ESBGK_E_UNSTABLE, "forward Euler needs dt/tau < 2 and dt/(Pr tau) < 2 at rho = T = 1");
  c->Kn = Kn;
  c->Pr = Pr;
  c->varpi = varpi;
  return upload_tvd(c);
}

int esbgk_tvd_set_wall(esbgk_tvd* c, int side, double T_w, const double u_w[3]) {
  TVD_CHECK(c);
  if (!c->shape.walls) return tset_err(c, ESBGK_E_INVALID, "the lattice has no walls");
  if (side != 0 && side != 1) return tset_err(c, ESBGK_E_INVALID, "side must be 0 or 1");
  if (!(T_w > 0.0) || !std::isfinite(T_w)) return tset_err(c, ESBGK_E_INVALID, "T_w must be > 0");
  double u[3] = {0, 0, 0};
  const int D = c->set.D;
  if (u_w)
    for (int i = 0; i < 3; ++i) {
      if (!std::isfinite(u_w[i])) return tset_err(c, ESBGK_E_INVALID, "u_w must be finite");
      u[i] = i < D ? u_w[i] : 0.0;
    }
  if (u[D - 1] != 0.0)
    return tset_err(c, ESBGK_E_INVALID, "a wall moves in its own plane (no component across the channel)");
  c->Tw[side] = T_w;
  for (int i = 0; i < 3; ++i) c->uw[side][i] = u[i];
  return upload_tvd(c);
}

int esbgk_tvd_set_body_force(esbgk_tvd* c, const double g[3]) {
  TVD_CHECK(c);
  if (!g) return tset_err(c, ESBGK_E_INVALID, "g is null");
  for (int i = 0; i < 3; ++i) {
    if (!std::isfinite(g[i])) return tset_err(c, ESBGK_E_INVALID, "g must be finite");
    c->g[i] = i < c->set.D ? g[i] : 0.0;
  }
  return upload_tvd(c);
}

int esbgk_tvd_init_equilibrium(esbgk_tvd* c, const double* rho, const double* u, const double* T,
                               const double* noise, double amplitude) {
  TVD_CHECK(c);
  if (noise && !std::isfinite(amplitude)) return tset_err(c, ESBGK_E_INVALID, "amplitude must be finite");
  const uint32_t cells = c->geo.ncells;
  TVDArgs a = targs(c);
  a.dst = c->at(c->lay.pop[c->cur]);
  const double* dc = reinterpret_cast<const double*>(c->at(c->lay.c));
  double* st = reinterpret_cast<double*>(c->at(c->lay.staging));
  for (uint32_t c0 = 0; c0 < cells; c0 += STAGE_CELLS) {
    const uint32_t n = std::min(STAGE_CELLS, cells - c0);
    const int D = c->set.D;
    double* d_rho = st;
    double* d_u = d_rho + n;
    double* d_T = d_u + size_t(D) * n;
    double* d_noise = d_T + n;
    if (rho) TVD_HIP(c, hipMemcpyAsync(d_rho, rho + c0, n * 8, hipMemcpyHostToDevice, c->stream), "stage");
    if (u)
      for (int d = 0; d < D; ++d)
        TVD_HIP(c, hipMemcpyAsync(d_u + size_t(d) * n, u + size_t(d) * cells + c0, n * 8, hipMemcpyHostToDevice,
                                  c->stream), "stage");
    if (T) TVD_HIP(c, hipMemcpyAsync(d_T, T + c0, n * 8, hipMemcpyHostToDevice, c->stream), "stage");
    if (noise)
      for (int q = 0; q < c->set.Q; ++q)
        TVD_HIP(c, hipMemcpyAsync(d_noise + size_t(q) * n, noise + size_t(q) * cells + c0, n * 8,
                                  hipMemcpyHostToDevice, c->stream), "stage");
    if (D == 3)
      TVD_HIP(c, launch_tvd3_init(c->shape.storage, a, dc, rho ? d_rho : nullptr, u ? d_u : nullptr,
                                  T ? d_T : nullptr, noise ? d_noise : nullptr, amplitude, c0, n), "init");
    else
      TVD_HIP(c, launch_tvd_init(c->shape.velset, c->shape.storage, a, dc, rho ? d_rho : nullptr,
                                 u ? d_u : nullptr, T ? d_T : nullptr, noise ? d_noise : nullptr, amplitude, c0, n),
              "init");
    TVD_HIP(c, hipStreamSynchronize(c->stream), "init");
  }
  c->state_set = true;
  c->mom_ok = false;
  c->steps = 0;
  return ESBGK_OK;
}

int esbgk_tvd_set_populations(esbgk_tvd* c, const double* h) {
  TVD_CHECK(c);
  if (!h) return tset_err(c, ESBGK_E_INVALID, "h is null");
  const size_t cells = c->geo.ncells;
  std::vector<unsigned char> buf;
  for (int q = 0; q < c->set.Q; ++q) {
    const double* src = h + size_t(q) * cells;
    const void* p = src;
    if (c->shape.storage == ESBGK_F32) {
      narrow_to<float>(src, cells, buf);
      p = buf.data();
    } else if (c->shape.storage == ESBGK_F16) {
      narrow_to<_Float16>(src, cells, buf);
      p = buf.data();
    }
    TVD_HIP(c, tplane_to_device(c, q, p), "set populations");
    TVD_HIP(c, hipStreamSynchronize(c->stream), "set populations");
  }
  c->state_set = true;
  c->mom_ok = false;
  c->steps = 0;
  return ESBGK_OK;
}

int esbgk_tvd_get_populations(esbgk_tvd* c, double* h) {
  TVD_CHECK(c);
  if (!h) return tset_err(c, ESBGK_E_INVALID, "h is null");
  if (!c->state_set) return tset_err(c, ESBGK_E_STATE, "no state set");
  const size_t cells = c->geo.ncells, ss = ssize(c->shape.storage);
  std::vector<unsigned char> buf(cells * ss);
  TVD_HIP(c, hipStreamSynchronize(c->stream), "get populations");
  for (int q = 0; q < c->set.Q; ++q) {
    TVD_HIP(c, tplane_to_host(c, q, buf.data()), "get populations");
    TVD_HIP(c, hipStreamSynchronize(c->stream), "get populations");
    double* o = h + size_t(q) * cells;
    if (c->shape.storage == ESBGK_F64) widen_from<double>(buf.data(), cells, o);
    else if (c->shape.storage == ESBGK_F32) widen_from<float>(buf.data(), cells, o);
    else widen_from<_Float16>(buf.data(), cells, o);
  }
  return ESBGK_OK;
}

int esbgk_tvd_step(esbgk_tvd* c, int64_t n) {
  TVD_CHECK(c);
  if (n < 0) return tset_err(c, ESBGK_E_INVALID, "n must be >= 0");
  if (!c->state_set) return tset_err(c, ESBGK_E_STATE, "no state set");
  for (int64_t k = 0; k < n; ++k) {
    const TVDArgs a = targs(c);
    if (c->set.D == 3) {
      if (!c->mom_ok) {
        TVD_HIP(c, launch_tvd3_rawmom(c->shape.storage, a, a.src, c->at(c->lay.mom[c->cur])), "moment sums");
        c->mom_ok = true;
      }
      TVD_HIP(c, launch_tvd3_step(c->shape.storage, a), "step");
      if (c->shape.walls) TVD_HIP(c, launch_tvd3_walls(c->shape.storage, a, c->at(c->lay.walls)), "walls");
    } else {
      TVD_HIP(c, launch_tvd_step(c->shape.velset, c->shape.storage, a), "step");
      if (c->shape.walls)
        TVD_HIP(c, launch_tvd_walls(c->shape.velset, c->shape.storage, a, c->at(c->lay.walls)), "walls");
    }
    c->cur ^= 1;
    c->steps += 1;
  }
  return ESBGK_OK;
}

int esbgk_tvd_read_moments(esbgk_tvd* c, double* h_out, int* F) {
  TVD_CHECK(c);
  if (!h_out) return tset_err(c, ESBGK_E_INVALID, "h_out is null");
  if (!c->state_set) return tset_err(c, ESBGK_E_STATE, "no state set");
  const int NF = nfields(c->set.D);
  if (F) *F = NF;
  const uint32_t cells = c->geo.ncells;
  double* st = reinterpret_cast<double*>(c->at(c->lay.staging));
  std::vector<double> tmp;
  const TVDArgs a = targs(c);
  for (uint32_t c0 = 0; c0 < cells; c0 += STAGE_CELLS) {
    const uint32_t n = std::min(STAGE_CELLS, cells - c0);
    if (c->set.D == 3)
      TVD_HIP(c, launch_tvd3_moments(c->shape.storage, a, c0, n, st), "moments");
    else
      TVD_HIP(c, launch_tvd_moments(c->shape.velset, c->shape.storage, a, c0, n, st), "moments");
    tmp.resize(size_t(NF) * n);
    TVD_HIP(c, hipMemcpyAsync(tmp.data(), st, tmp.size() * 8, hipMemcpyDeviceToHost, c->stream), "moments");
    TVD_HIP(c, hipStreamSynchronize(c->stream), "moments");
    for (int f = 0; f < NF; ++f)
      std::memcpy(h_out + size_t(f) * cells + c0, tmp.data() + size_t(f) * n, n * 8);
  }
  return ESBGK_OK;
}

int64_t esbgk_tvd_steps_done(const esbgk_tvd* c) { return c ? c->steps : -1; }

const char* esbgk_tvd_last_error(const esbgk_tvd* c) { return c ? c->err.c_str() : g_tvd_create_error.c_str(); }

}  // extern "C"
