// C ABI of the paper's own scheme (Sec. 3.1) on the 6-point Gauss-Hermite
// product set: handle management, validation, workspace layout, parameter
// upload, state I/O and the step loop.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstring>
#include <string>
#include <vector>

#include "../../include/esbgk.h"
#include "gh.h"
#include "tables.h"
#include "tvd.h"

using namespace esbgk;

namespace {

constexpr size_t ALIGN = 256;
constexpr uint32_t STAGE_CELLS = 65536;
constexpr int QGH_MAX = 64;

// Points of the 1-D rule of a product set (0: not a set of this scheme).
int set_points(int velset) {
  return velset == ESBGK_D2Q16GH ? 4 : (velset == ESBGK_D2Q36GH ? 6 : (velset == ESBGK_D2Q64GH ? 8 : 0));
}
constexpr int NFIELDS = 9;

size_t align_up(size_t n) { return (n + ALIGN - 1) / ALIGN * ALIGN; }
size_t ssize(int storage) { return storage == ESBGK_F64 ? 8 : (storage == ESBGK_F32 ? 4 : 2); }
size_t csize(int storage) { return storage == ESBGK_F64 ? 8 : 4; }

struct TLayout {
  size_t pop[2], gc, lc, pp, gc64, lc64, pp64, walls, c, staging, total;
};

bool valid_tvd_shape(const esbgk_shape* s, Geometry* g, std::string* why) {
  auto fail = [&](const char* m) { if (why) *why = m; return false; };
  if (!s) return fail("null shape");
  if (!set_points(s->velset)) return fail("velset must be ESBGK_D2Q16GH, ESBGK_D2Q36GH or ESBGK_D2Q64GH");
  if (s->nx < 1 || s->ny < 1 || s->nz != 1) return fail("extents: nx, ny >= 1 and nz = 1");
  if (s->walls != 0 && s->walls != 1) return fail("walls must be 0 (periodic) or 1 (walls across y)");
  if (s->walls && s->ny < 3) return fail("a channel needs ny >= 3 (two wall rows and one between)");
  if (s->storage < ESBGK_F64 || s->storage > ESBGK_F16) return fail("storage must be F64, F32 or F16");
  if (s->scheme != ESBGK_EULER) return fail("the paper's scheme is forward Euler (scheme = ESBGK_EULER)");
  if (s->n_ref < 0) return fail("n_ref must be >= 0");
  const HostGH* gh = host_gh(set_points(s->velset));
  if (!gh) return fail("velocity set tables unavailable");
  Geometry tmp;
  if (!make_geometry(2, gh->Q, uint32_t(s->nx), uint32_t(s->ny), 1, s->walls != 0, true, ssize(s->storage),
                     g ? *g : tmp))
    return fail("lattice too large for the slice layout (one row of populations must be < 4 GiB)");
  return true;
}

TLayout tlayout(const esbgk_shape* s, const Geometry& g) {
  TLayout L{};
  const size_t ss = ssize(s->storage), cs = csize(s->storage);
  const size_t cells = size_t(s->nx) * s->ny;
  size_t off = 0;
  auto take = [&](size_t bytes) { const size_t o = off; off = align_up(off + bytes); return o; };
  L.pop[0] = take(size_t(g.nslices) * g.sstride * ss);
  L.pop[1] = take(size_t(g.nslices) * g.sstride * ss);
  L.gc = take(cs == 8 ? sizeof(GHConsts<double>) : sizeof(GHConsts<float>));
  L.lc = take(cs == 8 ? sizeof(LatConsts<double>) : sizeof(LatConsts<float>));
  L.pp = take(cs == 8 ? sizeof(ProbParams<double>) : sizeof(ProbParams<float>));
  L.gc64 = cs == 8 ? L.gc : take(sizeof(GHConsts<double>));
  L.lc64 = cs == 8 ? L.lc : take(sizeof(LatConsts<double>));
  L.pp64 = cs == 8 ? L.pp : take(sizeof(ProbParams<double>));
  L.walls = take(cs == 8 ? sizeof(TVDWalls<double>) : sizeof(TVDWalls<float>));
  L.c = take(sizeof(double) * QGH_MAX * 2);
  const size_t stage = std::min<size_t>(cells, STAGE_CELLS);
  L.staging = take(stage * size_t(std::max(NFIELDS, 4 + QGH_MAX)) * sizeof(double));
  L.total = off;
  return L;
}

template <typename C>
void pack_gh(const HostGH& gh, double nu_scale, GHConsts<C>& d) {
  std::memset(&d, 0, sizeof(d));
  for (int p = 0; p < gh.P; ++p) {
    const double x = gh.c[p][0], y = gh.c[p][1];
    const double m[GH_MONO] = {x,         y,         x * x,         x * y,         y * y,
                               x * x * x, x * x * y, x * y * y,     y * y * y,     x * x * x * x,
                               x * x * x * y, x * x * y * y, x * y * y * y, y * y * y * y};
    d.w[p] = C(gh.w[p]);
    for (int k = 0; k < GH_MONO; ++k) d.mono[p][k] = C(m[k]);
    const double nx = x * nu_scale, ny = y * nu_scale;
    d.nu[p][0] = C(nx);
    d.nu[p][1] = C(ny);
    d.nk[p][0] = C(0.5 * std::fabs(nx) * (1.0 - std::fabs(nx)));
    d.nk[p][1] = C(0.5 * std::fabs(ny) * (1.0 - std::fabs(ny)));
  }
}

// Wall tables of Sec. 3.2 (see TVDWalls) from the walls' T and u.
template <typename C>
void pack_walls(const HostGH& gh, const double Tw[2], const double uw[2][3], TVDWalls<C>& d) {
  std::memset(&d, 0, sizeof(d));
  for (int side = 0; side < 2; ++side) {
    const double nrm = side == 0 ? 1.0 : -1.0;   // inward normal along y
    double den = 0.0, sw[QGH_MAX];
    for (int a = 0; a < gh.Q; ++a) {
      sw[a] = 1.0 + shat_minus_one_at(2, gh.N, gh.c[a], Tw[side], uw[side]);
      const double cn = nrm * gh.c[a][1];
      if (cn > 0) den += cn * gh.w[a] * sw[a];
    }
    double k0 = 0.0;
    for (int a = 0; a < gh.Q; ++a) {
      const double cn = nrm * gh.c[a][1];
      if (cn < 0) {
        const double k = -cn * gh.w[a] / den;
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
  int64_t steps = 0;
  int sticky = 0;
  std::string err;
  double Kn = 0.1, Pr = 1.0, varpi = 0.5, cfl = 0.5, dt = 0.0, dx = 0.0;
  double g[3] = {0, 0, 0};
  const HostGH* gh = nullptr;   // the velocity set's host tables
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
  a.stream = c->stream;
  return a;
}

// Gas, force and the Courant-limited time step: dt = CFL dx / max|c|.
int upload_tvd(esbgk_tvd* c) {
  const HostGH& gh = *c->gh;
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
    hp.g[i] = i < 2 ? c->g[i] : 0.0;
    if (hp.g[i] != 0.0) hp.force = 1;
  }
  hp.gam[0] = hp.gam[1] = 1.0;
  const double nu_scale = c->dt / c->dx;
  static thread_local ProbParams<double> pp64;
  static thread_local ProbParams<float> pp32;
  static thread_local GHConsts<double> g64;
  static thread_local GHConsts<float> g32;
  static thread_local LatConsts<double> l64;
  static thread_local LatConsts<float> l32;
  pack_params<double>(hp, 0, pp64);   // the wall tables of ProbParams are not used here
  pack_gh<double>(gh, nu_scale, g64);
  std::memset(&l64, 0, sizeof(l64));
  l64.r = 1.0;                        // the weights live in GHConsts
  TVD_HIP(c, hipMemcpyAsync(c->at(c->lay.pp64), &pp64, sizeof(pp64), hipMemcpyHostToDevice, c->stream), "upload");
  TVD_HIP(c, hipMemcpyAsync(c->at(c->lay.gc64), &g64, sizeof(g64), hipMemcpyHostToDevice, c->stream), "upload");
  TVD_HIP(c, hipMemcpyAsync(c->at(c->lay.lc64), &l64, sizeof(l64), hipMemcpyHostToDevice, c->stream), "upload");
  if (!c->f64()) {
    pack_params<float>(hp, 0, pp32);
    pack_gh<float>(gh, nu_scale, g32);
    std::memset(&l32, 0, sizeof(l32));
    l32.r = 1.0f;
    TVD_HIP(c, hipMemcpyAsync(c->at(c->lay.pp), &pp32, sizeof(pp32), hipMemcpyHostToDevice, c->stream), "upload");
    TVD_HIP(c, hipMemcpyAsync(c->at(c->lay.gc), &g32, sizeof(g32), hipMemcpyHostToDevice, c->stream), "upload");
    TVD_HIP(c, hipMemcpyAsync(c->at(c->lay.lc), &l32, sizeof(l32), hipMemcpyHostToDevice, c->stream), "upload");
  }
  if (c->shape.walls) {
    static thread_local TVDWalls<double> w64;
    static thread_local TVDWalls<float> w32;
    if (c->f64()) {
      pack_walls<double>(gh, c->Tw, c->uw, w64);
      TVD_HIP(c, hipMemcpyAsync(c->at(c->lay.walls), &w64, sizeof(w64), hipMemcpyHostToDevice, c->stream), "upload");
    } else {
      pack_walls<float>(gh, c->Tw, c->uw, w32);
      TVD_HIP(c, hipMemcpyAsync(c->at(c->lay.walls), &w32, sizeof(w32), hipMemcpyHostToDevice, c->stream), "upload");
    }
  }
  TVD_HIP(c, hipStreamSynchronize(c->stream), "upload");
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
  const int n = set_points(velset);
  const HostGH* gh = n ? host_gh(n) : nullptr;
  if (!gh) return ESBGK_E_INVALID;
  if (Q) *Q = gh->Q;
  if (N) *N = gh->N;
  for (int a = 0; a < gh->Q; ++a) {
    if (c) {
      c[2 * a] = gh->c[a][0];
      c[2 * a + 1] = gh->c[a][1];
    }
    if (w) w[a] = gh->w[a];
  }
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
  const int n_ref = shape->n_ref > 0 ? shape->n_ref : (shape->walls ? shape->ny - 1 : shape->nx);
  c->dx = 1.0 / double(n_ref);
  c->gh = host_gh(set_points(shape->velset));
  const HostGH& gh = *c->gh;
  c->dt = cfl * c->dx / gh.xi[gh.n / 2 - 1];
  double cc[QGH_MAX * 2] = {};
  for (int a = 0; a < gh.Q; ++a) {
    cc[2 * a] = gh.c[a][0];
    cc[2 * a + 1] = gh.c[a][1];
  }
  hipError_t e = hipMemcpyAsync(c->at(lay.c), cc, sizeof(cc), hipMemcpyHostToDevice, c->stream);
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
  if (u_w)
    for (int i = 0; i < 3; ++i) {
      if (!std::isfinite(u_w[i])) return tset_err(c, ESBGK_E_INVALID, "u_w must be finite");
      u[i] = i < 2 ? u_w[i] : 0.0;
    }
  if (u[1] != 0.0) return tset_err(c, ESBGK_E_INVALID, "a wall moves in its own plane (u_w[1] = 0)");
  c->Tw[side] = T_w;
  for (int i = 0; i < 3; ++i) c->uw[side][i] = u[i];
  return upload_tvd(c);
}

int esbgk_tvd_set_body_force(esbgk_tvd* c, const double g[3]) {
  TVD_CHECK(c);
  if (!g) return tset_err(c, ESBGK_E_INVALID, "g is null");
  for (int i = 0; i < 3; ++i) {
    if (!std::isfinite(g[i])) return tset_err(c, ESBGK_E_INVALID, "g must be finite");
    c->g[i] = i < 2 ? g[i] : 0.0;
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
    double* d_rho = st;
    double* d_u = d_rho + n;
    double* d_T = d_u + 2 * size_t(n);
    double* d_noise = d_T + n;
    if (rho) TVD_HIP(c, hipMemcpyAsync(d_rho, rho + c0, n * 8, hipMemcpyHostToDevice, c->stream), "stage");
    if (u)
      for (int d = 0; d < 2; ++d)
        TVD_HIP(c, hipMemcpyAsync(d_u + size_t(d) * n, u + size_t(d) * cells + c0, n * 8, hipMemcpyHostToDevice,
                                  c->stream), "stage");
    if (T) TVD_HIP(c, hipMemcpyAsync(d_T, T + c0, n * 8, hipMemcpyHostToDevice, c->stream), "stage");
    if (noise)
      for (int q = 0; q < c->gh->Q; ++q)
        TVD_HIP(c, hipMemcpyAsync(d_noise + size_t(q) * n, noise + size_t(q) * cells + c0, n * 8,
                                  hipMemcpyHostToDevice, c->stream), "stage");
    TVD_HIP(c, launch_tvd_init(c->shape.velset, c->shape.storage, a, dc, rho ? d_rho : nullptr, u ? d_u : nullptr,
                               T ? d_T : nullptr, noise ? d_noise : nullptr, amplitude, c0, n), "init");
    TVD_HIP(c, hipStreamSynchronize(c->stream), "init");
  }
  c->state_set = true;
  c->steps = 0;
  return ESBGK_OK;
}

int esbgk_tvd_set_populations(esbgk_tvd* c, const double* h) {
  TVD_CHECK(c);
  if (!h) return tset_err(c, ESBGK_E_INVALID, "h is null");
  const size_t cells = c->geo.ncells;
  std::vector<unsigned char> buf;
  for (int q = 0; q < c->gh->Q; ++q) {
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
  for (int q = 0; q < c->gh->Q; ++q) {
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
    TVD_HIP(c, launch_tvd_step(c->shape.velset, c->shape.storage, a), "step");
    if (c->shape.walls)
      TVD_HIP(c, launch_tvd_walls(c->shape.velset, c->shape.storage, a, c->at(c->lay.walls)), "walls");
    c->cur ^= 1;
    c->steps += 1;
  }
  return ESBGK_OK;
}

int esbgk_tvd_read_moments(esbgk_tvd* c, double* h_out, int* F) {
  TVD_CHECK(c);
  if (!h_out) return tset_err(c, ESBGK_E_INVALID, "h_out is null");
  if (!c->state_set) return tset_err(c, ESBGK_E_STATE, "no state set");
  if (F) *F = NFIELDS;
  const uint32_t cells = c->geo.ncells;
  double* st = reinterpret_cast<double*>(c->at(c->lay.staging));
  std::vector<double> tmp;
  const TVDArgs a = targs(c);
  for (uint32_t c0 = 0; c0 < cells; c0 += STAGE_CELLS) {
    const uint32_t n = std::min(STAGE_CELLS, cells - c0);
    TVD_HIP(c, launch_tvd_moments(c->shape.velset, c->shape.storage, a, c0, n, st), "moments");
    tmp.resize(size_t(NFIELDS) * n);
    TVD_HIP(c, hipMemcpyAsync(tmp.data(), st, tmp.size() * 8, hipMemcpyDeviceToHost, c->stream), "moments");
    TVD_HIP(c, hipStreamSynchronize(c->stream), "moments");
    for (int f = 0; f < NFIELDS; ++f)
      std::memcpy(h_out + size_t(f) * cells + c0, tmp.data() + size_t(f) * n, n * 8);
  }
  return ESBGK_OK;
}

int64_t esbgk_tvd_steps_done(const esbgk_tvd* c) { return c ? c->steps : -1; }

const char* esbgk_tvd_last_error(const esbgk_tvd* c) { return c ? c->err.c_str() : g_tvd_create_error.c_str(); }

}  // extern "C"
