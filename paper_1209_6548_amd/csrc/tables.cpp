// Host-side derivation of the velocity-set constants and the per-problem
// parameter block.
//
// Velocity set (Sec. 2.2): the abscissae c = r e and weights w of a
// Gauss-Hermite quadrature for the weight function
// omega(c) = (2 pi)^(-D/2) exp(-c^2/2). The integer vectors are fixed
// (lattice.h); the weights are equal within a shell (vectors related by
// permutations and sign changes) and, with r, follow from requiring every even
// moment up to the set's degree to equal the Gaussian one,
//     sum_s W_s r^(2|a|) sum_{e in s} prod_i e_i^(2 a_i) = prod_i (2 a_i - 1)!!.
// There is one more condition than shell weights. The scale r is the root of
// det[A(r) | G] = 0 (the right-hand side is consistent), found by scanning and
// bisection in long double; the weights then solve the (consistent)
// least-squares system. The admissible root is the one with all weights
// positive.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <functional>
#include <mutex>
#include <vector>

#include "lattice.h"
#include "params.h"
#include "tables.h"
#include "gh3.h"

namespace esbgk {

namespace {

using ld = long double;

template <class L>
void integer_table(HostLattice& out) {
  out.D = L::D;
  out.Q = L::Q;
  out.N = L::N;
  out.P = L::P;
  out.e.assign(size_t(L::Q) * 3, 0);
  for (int a = 0; a < L::Q; ++a)
    for (int i = 0; i < 3; ++i) out.e[size_t(a) * 3 + i] = ecomp<L>(a, i);
}

// determinant of an n x n matrix by Gaussian elimination with partial pivoting
ld det(std::vector<ld> m, int n) {
  ld d = 1;
  for (int c = 0; c < n; ++c) {
    int p = c;
    for (int i = c + 1; i < n; ++i)
      if (std::fabs(m[size_t(i) * n + c]) > std::fabs(m[size_t(p) * n + c])) p = i;
    if (m[size_t(p) * n + c] == 0) return 0;
    if (p != c) {
      for (int j = 0; j < n; ++j) std::swap(m[size_t(p) * n + j], m[size_t(c) * n + j]);
      d = -d;
    }
    d *= m[size_t(c) * n + c];
    for (int i = c + 1; i < n; ++i) {
      const ld f = m[size_t(i) * n + c] / m[size_t(c) * n + c];
      for (int j = c; j < n; ++j) m[size_t(i) * n + j] -= f * m[size_t(c) * n + j];
    }
  }
  return d;
}

// least squares min ||A x - b|| (rows x cols, rows >= cols) by Householder QR
bool lstsq(std::vector<ld> A, std::vector<ld> b, int rows, int cols, std::vector<ld>& x) {
  for (int c = 0; c < cols; ++c) {
    ld nrm = 0;
    for (int i = c; i < rows; ++i) nrm += A[size_t(i) * cols + c] * A[size_t(i) * cols + c];
    nrm = std::sqrt(nrm);
    if (nrm == 0) return false;
    const ld alpha = A[size_t(c) * cols + c] > 0 ? -nrm : nrm;
    std::vector<ld> v(rows, 0);
    for (int i = c; i < rows; ++i) v[i] = A[size_t(i) * cols + c];
    v[c] -= alpha;
    ld vv = 0;
    for (int i = c; i < rows; ++i) vv += v[i] * v[i];
    if (vv == 0) continue;
    for (int j = c; j < cols; ++j) {
      ld s = 0;
      for (int i = c; i < rows; ++i) s += v[i] * A[size_t(i) * cols + j];
      s = 2 * s / vv;
      for (int i = c; i < rows; ++i) A[size_t(i) * cols + j] -= s * v[i];
    }
    ld s = 0;
    for (int i = c; i < rows; ++i) s += v[i] * b[i];
    s = 2 * s / vv;
    for (int i = c; i < rows; ++i) b[i] -= s * v[i];
  }
  x.assign(cols, 0);
  for (int c = cols - 1; c >= 0; --c) {
    ld s = b[c];
    for (int j = c + 1; j < cols; ++j) s -= A[size_t(c) * cols + j] * x[j];
    x[c] = s / A[size_t(c) * cols + c];
  }
  return true;
}

ld dfact_odd(int k) {  // (k-1)!! for even k
  ld out = 1;
  for (int m = k - 1; m > 0; m -= 2) out *= m;
  return out;
}

struct MomentSystem {
  int ns = 0, nc = 0;
  std::vector<int> shell_of;      // per velocity
  std::vector<ld> A0;             // nc x ns integer sums
  std::vector<ld> G;              // nc
  std::vector<int> deg;           // nc: |a|
};

MomentSystem build_system(const HostLattice& lat, int degree) {
  MomentSystem ms;
  const int D = lat.D, Q = lat.Q;
  // shells: sorted absolute components
  std::vector<std::vector<int>> keys;
  ms.shell_of.resize(Q);
  for (int a = 0; a < Q; ++a) {
    std::vector<int> k(D);
    for (int i = 0; i < D; ++i) k[i] = std::abs(lat.e[size_t(a) * 3 + i]);
    std::sort(k.begin(), k.end());
    auto it = std::find(keys.begin(), keys.end(), k);
    if (it == keys.end()) {
      keys.push_back(k);
      ms.shell_of[a] = int(keys.size()) - 1;
    } else {
      ms.shell_of[a] = int(it - keys.begin());
    }
  }
  ms.ns = int(keys.size());
  // even multi-indices a_1 >= a_2 >= ... >= 0 with 2 sum(a) <= degree
  std::vector<std::vector<int>> conds;
  const int half = degree / 2;
  std::vector<int> a(D, 0);
  for (int total = 0; total <= half; ++total) {
    // enumerate non-increasing tuples with the given sum
    std::vector<int> t(D, 0);
    std::function<void(int, int, int)> rec = [&](int pos, int left, int maxv) {
      if (pos == D) {
        if (left == 0) conds.push_back(t);
        return;
      }
      for (int v = std::min(left, maxv); v >= 0; --v) {
        t[pos] = v;
        rec(pos + 1, left - v, v);
      }
    };
    rec(0, total, total);
  }
  ms.nc = int(conds.size());
  ms.A0.assign(size_t(ms.nc) * ms.ns, 0);
  ms.G.assign(ms.nc, 0);
  ms.deg.assign(ms.nc, 0);
  for (int k = 0; k < ms.nc; ++k) {
    ld g = 1;
    int s = 0;
    for (int i = 0; i < D; ++i) {
      g *= dfact_odd(2 * conds[k][i]);
      s += conds[k][i];
    }
    ms.G[k] = g;
    ms.deg[k] = s;
    for (int q = 0; q < Q; ++q) {
      ld p = 1;
      for (int i = 0; i < D; ++i) p *= std::pow(ld(lat.e[size_t(q) * 3 + i]), 2 * conds[k][i]);
      ms.A0[size_t(k) * ms.ns + ms.shell_of[q]] += p;
    }
  }
  return ms;
}

ld consistency(const MomentSystem& ms, ld r) {
  // det [A0 | G r^(-2|a|)], an (ns+1) x (ns+1) matrix
  const int n = ms.nc;
  std::vector<ld> m(size_t(n) * n);
  for (int k = 0; k < n; ++k) {
    for (int s = 0; s < ms.ns; ++s) m[size_t(k) * n + s] = ms.A0[size_t(k) * ms.ns + s];
    m[size_t(k) * n + ms.ns] = ms.G[k] * std::pow(r, ld(-2 * ms.deg[k]));
  }
  return det(m, n);
}

bool derive(HostLattice& lat, int degree) {
  MomentSystem ms = build_system(lat, degree);
  if (ms.nc != ms.ns + 1) return false;
  int found = 0;
  ld r_ok = 0;
  std::vector<ld> W_ok;
  const ld step = 0.001L;
  ld r0 = 0.5L, f0 = consistency(ms, r0);
  for (ld r1 = r0 + step; r1 <= 3.0L; r1 += step) {
    const ld f1 = consistency(ms, r1);
    if ((f0 < 0) != (f1 < 0)) {
      ld lo = r0, hi = r1, flo = f0;
      for (int it = 0; it < 200; ++it) {
        const ld mid = 0.5L * (lo + hi);
        if (mid == lo || mid == hi) break;
        const ld fm = consistency(ms, mid);
        if ((fm < 0) == (flo < 0)) { lo = mid; flo = fm; } else { hi = mid; }
      }
      const ld r = 0.5L * (lo + hi);
      std::vector<ld> A(size_t(ms.nc) * ms.ns), b(ms.nc), W;
      for (int k = 0; k < ms.nc; ++k) {
        const ld sc = std::pow(r, ld(2 * ms.deg[k]));
        for (int s = 0; s < ms.ns; ++s) A[size_t(k) * ms.ns + s] = ms.A0[size_t(k) * ms.ns + s] * sc;
        b[k] = ms.G[k];
      }
      if (lstsq(A, b, ms.nc, ms.ns, W)) {
        bool pos = true;
        for (ld x : W) pos = pos && x > 0;
        if (pos) {
          ++found;
          r_ok = r;
          W_ok = W;
        }
      }
    }
    r0 = r1;
    f0 = f1;
  }
  if (found != 1) return false;
  lat.r = double(r_ok);
  lat.w.assign(lat.Q, 0.0);
  for (int a = 0; a < lat.Q; ++a) lat.w[a] = double(W_ok[ms.shell_of[a]]);
  return true;
}

}  // namespace

const HostLattice* host_lattice(int velset) {
  static HostLattice lat[2];
  static bool ok[2] = {false, false};
  static std::once_flag once[2];
  if (velset != 1 && velset != 2) return nullptr;
  const int i = velset - 1;
  std::call_once(once[i], [&]() {
    HostLattice& L = lat[i];
    L.velset = velset;
    if (velset == 1) {
      integer_table<D2Q37>(L);
      ok[i] = derive(L, 9);
    } else {
      integer_table<D3Q39>(L);
      ok[i] = derive(L, 7);
    }
  });
  return ok[i] ? &lat[i] : nullptr;
}

// 1-D rule of eq. weight: the n roots of the probabilists' Hermite polynomial
// He_n (recurrence He_{k+1} = x He_k - k He_{k-1}), located by a sign scan of
// (-sqrt(4n+2), sqrt(4n+2)) and bisection in long double, and the weights
// n! / [n He_{n-1}(x)]^2.
static bool gauss_hermite_rule(int n, std::vector<ld>& x, std::vector<ld>& w) {
  auto he = [](int k, ld t) {
    ld a = 1, b = t;
    if (k == 0) return a;
    for (int j = 1; j < k; ++j) {
      const ld c = t * b - ld(j) * a;
      a = b;
      b = c;
    }
    return b;
  };
  const ld lim = std::sqrt(ld(4 * n + 2));
  const int scan = 40000;
  x.clear();
  ld prev_t = -lim, prev_v = he(n, -lim);
  for (int k = 1; k <= scan; ++k) {
    const ld t = -lim + 2 * lim * ld(k) / ld(scan);
    const ld v = he(n, t);
    if ((prev_v < 0) != (v < 0)) {
      ld lo = prev_t, hi = t, vlo = prev_v;
      for (int it = 0; it < 200; ++it) {
        const ld mid = 0.5L * (lo + hi), vm = he(n, mid);
        if ((vm < 0) == (vlo < 0)) {
          lo = mid;
          vlo = vm;
        } else {
          hi = mid;
        }
      }
      x.push_back(0.5L * (lo + hi));
    }
    prev_t = t;
    prev_v = v;
  }
  if (int(x.size()) != n) return false;
  ld fact = 1;
  for (int k = 2; k <= n; ++k) fact *= k;
  w.resize(n);
  for (int k = 0; k < n; ++k) {
    const ld h = ld(n) * he(n - 1, x[k]);
    w[k] = fact / (h * h);
  }
  return true;
}

template <class L>
static bool build_gh(HostGH& gh) {
  std::vector<ld> x, w;
  if (!gauss_hermite_rule(L::n, x, w)) return false;
  constexpr int H = L::H;
  // symmetric rule: positive roots x[H..n-1]; rank k in +-1..+-H means
  // sign(k) * xi[|k| - 1]
  ld xi[4], w1[4];
  for (int m = 0; m < H; ++m) {
    xi[m] = 0.5L * (x[H + m] - x[H - 1 - m]);   // average the mirrored pair
    w1[m] = 0.5L * (w[H + m] + w[H - 1 - m]);
    gh.xi[m] = double(xi[m]);
  }
  gh.n = L::n;
  gh.Q = L::Q;
  gh.P = L::P;
  gh.N = L::N;
  for (int a = 0; a < L::Q; ++a) {
    ld wa = 1;
    for (int i = 0; i < 2; ++i) {
      const int k = L::ranks.K[a % L::P][i] * (a < L::P ? 1 : -1);
      const int m = (k < 0 ? -k : k) - 1;
      gh.c[a][i] = double(k < 0 ? -xi[m] : xi[m]);
      wa *= w1[m];
    }
    gh.w[a] = double(wa);
  }
  return true;
}

const HostGH* host_gh(int n) {
  static HostGH tabs[3];
  static bool ok[3] = {false, false, false};
  static std::once_flag once[3];
  const int i = n == 4 ? 0 : (n == 6 ? 1 : (n == 8 ? 2 : -1));
  if (i < 0) return nullptr;
  std::call_once(once[i], [&]() {
    ok[i] = n == 4 ? build_gh<D2Q16GH>(tabs[i]) : (n == 6 ? build_gh<D2Q36GH>(tabs[i]) : build_gh<D2Q64GH>(tabs[i]));
  });
  return ok[i] ? &tabs[i] : nullptr;
}

const HostGH3* host_gh3() {
  static HostGH3 gh;
  static bool ok = false;
  static std::once_flag once;
  std::call_once(once, [&]() {
    using L = D3Q216GH;
    std::vector<ld> x, w;
    if (!gauss_hermite_rule(L::n, x, w)) return;
    constexpr int H = L::H;
    ld xi[H], w1[H];
    for (int m = 0; m < H; ++m) {
      xi[m] = 0.5L * (x[H + m] - x[H - 1 - m]);
      w1[m] = 0.5L * (w[H + m] + w[H - 1 - m]);
      gh.xi[m] = double(xi[m]);
    }
    for (int a = 0; a < L::Q; ++a) {
      ld wa = 1;
      for (int i = 0; i < 3; ++i) {
        const int k = L::ranks.K[a % L::P][i] * (a < L::P ? 1 : -1);
        const int m = (k < 0 ? -k : k) - 1;
        gh.c[a][i] = double(k < 0 ? -xi[m] : xi[m]);
        wa *= w1[m];
      }
      gh.w[a] = double(wa);
    }
    ok = true;
  });
  return ok ? &gh : nullptr;
}

// S(T, u)(c) / w - 1 at the velocity c[D]: eq. feq0 with rho = 1, truncated
// at order N.
double shat_minus_one_at(int D, int N, const double* c, double T, const double u[3]) {
  double cu = 0, uu = 0, cc = 0;
  for (int i = 0; i < D; ++i) {
    cu += c[i] * u[i];
    uu += u[i] * u[i];
    cc += c[i] * c[i];
  }
  const double th = T - 1.0;
  double s = cu + 0.5 * (cu * cu - uu + th * (cc - D)) + cu / 6.0 * (cu * cu - 3.0 * uu + 3.0 * th * (cc - D - 2));
  if (N >= 4) {
    s += (cu * cu * cu * cu - 6.0 * cu * cu * uu + 3.0 * uu * uu) / 24.0 +
         th / 4.0 * ((cc - D - 2) * (cu * cu - uu) - 2.0 * cu * cu) +
         th * th / 8.0 * (cc * cc - 2.0 * (D + 2) * cc + D * (D + 2));
  }
  return s;
}

double shat_minus_one(const HostLattice& lat, int a, double T, const double u[3]) {
  double c[3];
  for (int i = 0; i < lat.D; ++i) c[i] = lat.r * lat.e[size_t(a) * 3 + i];
  return shat_minus_one_at(lat.D, lat.N, c, T, u);
}

HostProblem make_problem(const HostLattice& lat, int n_ref, int scheme, double Kn, double Pr, double varpi,
                         const double g[3], const double Tw[2], const double uw[2][3], const double gam[2]) {
  HostProblem p{};
  const double dx = 1.0 / double(n_ref);
  p.dt = dx / lat.r;
  p.hs = scheme == 0 ? 0.5 * p.dt : 0.0;
  p.hsdt = scheme == 0 ? 0.5 : 0.0;
  p.xcoef = p.dt * Pr / Kn;
  p.omv = 1.0 - varpi;
  p.invPr = 1.0 / Pr;
  p.b = 1.0 - 1.0 / Pr;
  p.force = 0;
  for (int i = 0; i < 3; ++i) {
    p.g[i] = i < lat.D ? g[i] : 0.0;
    if (p.g[i] != 0.0) p.force = 1;
  }
  const int W = lat.D - 1;
  for (int side = 0; side < 2; ++side) {
    double leave = 0, den = 0;
    for (int a = 0; a < lat.Q; ++a) {
      const double em1 = shat_minus_one(lat, a, Tw[side], uw[side]);
      p.Em1[side][a] = em1;
      p.Ehat[side][a] = 1.0 + em1;
      const int en = lat.e[size_t(a) * 3 + W];
      const bool out = side == 0 ? en < 0 : en > 0;
      const bool in = side == 0 ? en > 0 : en < 0;
      if (out) leave += std::abs(en) * lat.w[a];
      if (in) den += std::abs(en) * lat.w[a] * (1.0 + em1);
    }
    p.K0[side] = leave / den - 1.0;
    p.invden[side] = 1.0 / den;
    p.gam[side] = gam[side];
  }
  p.specular = (gam[0] < 1.0 || gam[1] < 1.0) ? 1 : 0;
  return p;
}

template <typename C>
void pack_params(const HostProblem& h, int Q, ProbParams<C>& d) {
  std::memset(&d, 0, sizeof(d));
  d.dt = C(h.dt);
  d.hs = C(h.hs);
  d.hsdt = C(h.hsdt);
  d.xcoef = C(h.xcoef);
  d.omv = C(h.omv);
  d.invPr = C(h.invPr);
  d.b = C(h.b);
  for (int i = 0; i < 3; ++i) d.g[i] = C(h.g[i]);
  d.force = h.force;
  for (int s = 0; s < 2; ++s) {
    for (int a = 0; a < Q; ++a) {
      d.Em1[s][a] = C(h.Em1[s][a]);
      d.Ehat[s][a] = C(h.Ehat[s][a]);
    }
    d.K0[s] = C(h.K0[s]);
    d.invden[s] = C(h.invden[s]);
    d.gam[s] = C(h.gam[s]);
  }
  d.specular = h.specular;
}

template <typename C>
void pack_lattice(const HostLattice& lat, LatConsts<C>& d) {
  std::memset(&d, 0, sizeof(d));
  for (int a = 0; a < lat.Q; ++a) d.w[a] = C(lat.w[a]);
  d.r = C(lat.r);
}

template void pack_params<float>(const HostProblem&, int, ProbParams<float>&);
template void pack_params<double>(const HostProblem&, int, ProbParams<double>&);
template void pack_lattice<float>(const HostLattice&, LatConsts<float>&);
template void pack_lattice<double>(const HostLattice&, LatConsts<double>&);

FastDiv make_fastdiv(uint32_t d) {
  FastDiv f{};
  uint32_t l = 0;
  while ((uint64_t(1) << l) < d) ++l;
  f.l = l;
  f.m = uint32_t(((uint64_t(1) << 32) * ((uint64_t(1) << l) - d)) / d + 1);
  return f;
}

bool make_geometry(int D, int Q, uint32_t nx, uint32_t ny, uint32_t nz, bool walls, bool sliced, size_t ss,
                   Geometry& g) {
  g = Geometry{};
  g.nx = nx;
  g.ny = ny;
  g.nz = nz;
  const uint64_t n = uint64_t(nx) * ny * nz;
  if (n >= (uint64_t(1) << 31)) return false;
  g.ncells = uint32_t(n);
  g.nxy = nx * ny;
  g.walls = walls ? 1u : 0u;
  g.div_nx = make_fastdiv(nx);
  g.div_ny = make_fastdiv(ny);
  g.inner = D == 2 ? nx : nx * ny;
  g.nslices = D == 2 ? ny : nz;
  g.ncols = g.inner;
  const uint64_t ipad = (uint64_t(g.inner) + 63) / 64 * 64;
  if (uint64_t(g.nslices) * ipad >= (uint64_t(1) << 31)) return false;
  g.ipad = uint32_t(ipad);
  g.div_ipad = make_fastdiv(g.ipad);
  if (sliced) {
    const uint64_t ps = ipad;
    const uint64_t sst = uint64_t(Q) * ps + SLICE_PAD;
    if (sst * ss >= (uint64_t(1) << 32)) return false;
    g.pstride = uint32_t(ps);
    g.sstride = uint32_t(sst);
    g.window_ok = 7 * sst * ss < (uint64_t(1) << 32) ? 1u : 0u;
  } else {
    g.pstride = g.ncells;
    g.sstride = g.inner;
  }
  return true;
}

}  // namespace esbgk
