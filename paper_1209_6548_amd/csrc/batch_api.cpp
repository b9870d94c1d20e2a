// C ABI of batched channel problems: validation, workspace layout, binning
// (longest problem first into the lightest bin), the autotuner that picks the
// workgroup size and the number of bins by timing the persistent kernel, and
// the per-problem state I/O.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <numeric>
#include <queue>
#include <string>
#include <vector>

#include "../../include/esbgk.h"
#include "batch.h"
#include "kernels.h"
#include "tables.h"

using namespace esbgk;

namespace {

constexpr size_t ALIGN = 256;
constexpr uint32_t STAGE_CELLS = 65536;

size_t align_up(size_t n) { return (n + ALIGN - 1) / ALIGN * ALIGN; }
size_t ssize(int storage) { return storage == ESBGK_F64 ? 8 : (storage == ESBGK_F32 ? 4 : 2); }
size_t csize(int storage) { return storage == ESBGK_F64 ? 8 : 4; }

struct BLayout {
  size_t bufA, bufB, wpA, wpB, probs, pps, lc, pps64, lc64, bin_first, order, staging, total;
  size_t pop_elems, wp_elems;
};

bool valid_problem(const esbgk_problem& p, const esbgk_problem& first, std::string* why) {
  auto fail = [&](const char* m) { if (why) *why = m; return false; };
  const esbgk_shape& s = p.shape;
  if (s.velset != first.shape.velset || s.storage != first.shape.storage || s.scheme != first.shape.scheme)
    return fail("every problem needs the batch's velset, storage and scheme");
  if (s.velset != ESBGK_D2Q37 && s.velset != ESBGK_D3Q39) return fail("bad velset");
  if (s.nx < 1 || s.ny < 1 || s.nz < 1) return fail("extents must be >= 1");
  if (s.velset == ESBGK_D2Q37 && s.nz != 1) return fail("D2Q37 needs nz = 1");
  if (s.walls != 1) return fail("batched problems are channels (walls = 1)");
  const int nw = s.velset == ESBGK_D2Q37 ? s.ny : s.nz;
  if (nw < 6) return fail("the wall axis needs at least 6 cells");
  if (uint64_t(s.nx) * s.ny * s.nz >= (uint64_t(1) << 31)) return fail("problem too large");
  if (uint64_t(s.nx) * s.ny * s.nz * 39u >= (uint64_t(1) << 32))
    return fail("a problem's populations must number < 2^32 (32-bit offsets)");
  if (s.storage < 0 || s.storage > 2 || (s.scheme != 0 && s.scheme != 1) || s.n_ref < 0) return fail("bad shape");
  if (!(p.Kn > 0.0) || !(p.Pr >= 2.0 / 3.0 - 1e-12) || !(p.varpi >= 0.5 && p.varpi <= 1.0))
    return fail("bad gas parameters");
  const int W = s.velset == ESBGK_D2Q37 ? 1 : 2;   // wall-normal axis
  for (int side = 0; side < 2; ++side) {
    if (!(p.T_w[side] > 0.0)) return fail("T_w must be > 0");
    if (!(p.specular[side] >= 0.0 && p.specular[side] <= 1.0)) return fail("specular must lie in [0, 1]");
    if (p.u_w[side][W] != 0.0) return fail("wall velocity must be tangential");
  }
  return true;
}

uint32_t cells_of(const esbgk_shape& s) { return uint32_t(s.nx) * s.ny * s.nz; }
uint32_t ncols_of(const esbgk_shape& s) { return s.velset == ESBGK_D2Q37 ? s.nx : s.nx * s.ny; }

BLayout blayout(const esbgk_problem* p, int n) {
  const HostLattice* lat = host_lattice(p[0].shape.velset);
  const int storage = p[0].shape.storage;
  BLayout L{};
  size_t pop = 0, wp = 0, maxc = 0;
  for (int i = 0; i < n; ++i) {
    pop += size_t(lat->Q) * cells_of(p[i].shape);
    pop = (pop + 63) / 64 * 64;
    wp += 6 * size_t(ncols_of(p[i].shape));
    maxc = std::max<size_t>(maxc, cells_of(p[i].shape));
  }
  L.pop_elems = pop;
  L.wp_elems = wp;
  size_t off = 0;
  auto take = [&](size_t bytes) { const size_t o = off; off = align_up(off + bytes); return o; };
  L.bufA = take(pop * ssize(storage));
  L.bufB = take(pop * ssize(storage));
  L.wpA = take(wp * csize(storage));
  L.wpB = take(wp * csize(storage));
  L.probs = take(size_t(n) * sizeof(BatchProblem));
  L.pps = take(size_t(n) * (csize(storage) == 8 ? sizeof(ProbParams<double>) : sizeof(ProbParams<float>)));
  L.lc = take(csize(storage) == 8 ? sizeof(LatConsts<double>) : sizeof(LatConsts<float>));
  // FP64 blocks for the read-out kernels (the same blocks when storage is FP64)
  L.pps64 = csize(storage) == 8 ? L.pps : take(size_t(n) * sizeof(ProbParams<double>));
  L.lc64 = csize(storage) == 8 ? L.lc : take(sizeof(LatConsts<double>));
  L.bin_first = take(size_t(n + 1) * 4);
  L.order = take(size_t(n) * 4);
  const size_t sc = std::min<size_t>(maxc, STAGE_CELLS);
  L.staging = take(sc * std::max<size_t>(nfields(lat->D), size_t(lat->Q)) * 8);
  L.total = off;
  return L;
}

}  // namespace

struct esbgk_batch {
  std::vector<esbgk_problem> p;
  std::vector<BatchProblem> bp;
  const HostLattice* lat = nullptr;
  int velset = 0, storage = 0;
  BLayout lay{};
  char* ws = nullptr;
  hipStream_t stream = nullptr;
  int parity = 0;              // 0: current state in A
  bool state_set = false;
  int64_t steps = 0;
  uint32_t threads = 0, nbins = 0;
  int cus = 0;
  int sticky = 0;
  std::string err;
  char* at(size_t o) const { return ws + o; }
};

namespace {

int bfail(esbgk_batch* b, hipError_t e, const char* where) {
  b->sticky = ESBGK_E_HIP;
  b->err = std::string(where) + ": " + hipGetErrorString(e);
  return ESBGK_E_HIP;
}

#define BHIP(b, expr, where)                              \
  do {                                                    \
    hipError_t _e = (expr);                               \
    if (_e != hipSuccess) return bfail(b, _e, where);     \
  } while (0)

// Longest problem first, each into the bin with the fewest cells (counted as
// the kernel's slots: each problem rounded up to a multiple of 64).
int build_bins(esbgk_batch* b, uint32_t nbins) {
  const int n = int(b->p.size());
  nbins = std::max<uint32_t>(1, std::min<uint32_t>(nbins, uint32_t(n)));
  std::vector<int> idx(n);
  std::iota(idx.begin(), idx.end(), 0);
  std::stable_sort(idx.begin(), idx.end(),
                   [&](int x, int y) { return b->bp[x].geo.ncells > b->bp[y].geo.ncells; });
  using Item = std::pair<uint64_t, uint32_t>;   // (cells, bin)
  std::priority_queue<Item, std::vector<Item>, std::greater<Item>> heap;
  for (uint32_t k = 0; k < nbins; ++k) heap.push({0, k});
  std::vector<std::vector<uint32_t>> bins(nbins);
  std::vector<Item> full;
  for (int i : idx) {
    Item it = heap.top();
    heap.pop();
    while (bins[it.second].size() >= size_t(BATCH_MAX_PER_BIN)) {
      full.push_back(it);
      if (heap.empty()) return ESBGK_E_INVALID;
      it = heap.top();
      heap.pop();
    }
    bins[it.second].push_back(uint32_t(i));
    it.first += (b->bp[i].geo.ncells + 63u) & ~63u;
    heap.push(it);
  }
  std::vector<uint32_t> first(nbins + 1), order;
  order.reserve(n);
  for (uint32_t k = 0; k < nbins; ++k) {
    first[k] = uint32_t(order.size());
    for (uint32_t id : bins[k]) order.push_back(id);
  }
  first[nbins] = uint32_t(order.size());
  BHIP(b, hipMemcpyAsync(b->at(b->lay.bin_first), first.data(), first.size() * 4, hipMemcpyHostToDevice, b->stream),
       "bins");
  BHIP(b, hipMemcpyAsync(b->at(b->lay.order), order.data(), order.size() * 4, hipMemcpyHostToDevice, b->stream),
       "bins");
  BHIP(b, hipStreamSynchronize(b->stream), "bins");
  b->nbins = nbins;
  return ESBGK_OK;
}

BatchLaunch launch_args(const esbgk_batch* b, int64_t n) {
  BatchLaunch a{};
  a.probs = reinterpret_cast<const BatchProblem*>(b->at(b->lay.probs));
  a.pps = b->at(b->lay.pps);
  a.bin_first = reinterpret_cast<const uint32_t*>(b->at(b->lay.bin_first));
  a.order = reinterpret_cast<const uint32_t*>(b->at(b->lay.order));
  a.bufA = b->at(b->lay.bufA);
  a.bufB = b->at(b->lay.bufB);
  a.wpA = b->at(b->lay.wpA);
  a.wpB = b->at(b->lay.wpB);
  a.lc = b->at(b->lay.lc);
  a.nsteps = n;
  a.parity = b->parity;
  a.nbins = b->nbins;
  a.threads = b->threads;
  a.stream = b->stream;
  return a;
}

// Single-lattice view of problem i (for init, moments, partial sums).
StepArgs problem_args(const esbgk_batch* b, int i) {
  StepArgs a{};
  const size_t ss = ssize(b->storage), cs = csize(b->storage);
  const BatchProblem& bp = b->bp[i];
  char* cur = b->at(b->parity ? b->lay.bufB : b->lay.bufA) + bp.pop_off * ss;
  char* wcur = b->at(b->parity ? b->lay.wpB : b->lay.wpA) + size_t(bp.wp_off) * cs;
  a.geo = bp.geo;
  a.src = cur;
  a.dst = cur;
  a.wp_src = wcur;
  a.wp_dst = wcur;
  a.lc = b->at(b->lay.lc);
  a.pp = b->at(b->lay.pps) + size_t(i) * (cs == 8 ? sizeof(ProbParams<double>) : sizeof(ProbParams<float>));
  a.lc64 = b->at(b->lay.lc64);
  a.pp64 = b->at(b->lay.pps64) + size_t(i) * sizeof(ProbParams<double>);
  a.stream = b->stream;
  return a;
}

int rest_state(esbgk_batch* b, const double* noise, double amp) {
  size_t noise_off = 0;
  double* st = reinterpret_cast<double*>(b->at(b->lay.staging));
  for (size_t i = 0; i < b->p.size(); ++i) {
    StepArgs a = problem_args(b, int(i));
    const uint32_t cells = a.geo.ncells;
    if (!noise) {
      BHIP(b, launch_init(b->velset, b->storage, a, b->lat->r, nullptr, nullptr, nullptr, nullptr, 0.0, 0, cells),
           "batch init");
    } else {
      for (uint32_t c0 = 0; c0 < cells; c0 += STAGE_CELLS) {
        const uint32_t n = std::min(STAGE_CELLS, cells - c0);
        for (int q = 0; q < b->lat->Q; ++q)
          BHIP(b, hipMemcpyAsync(st + size_t(q) * n, noise + noise_off + size_t(q) * cells + c0, n * 8,
                                 hipMemcpyHostToDevice, b->stream), "batch init");
        BHIP(b, launch_init(b->velset, b->storage, a, b->lat->r, nullptr, nullptr, nullptr, st, amp, c0, n),
             "batch init");
        BHIP(b, hipStreamSynchronize(b->stream), "batch init");
      }
      noise_off += size_t(b->lat->Q) * cells;
    }
    BHIP(b, launch_wall_partials(b->velset, b->storage, a), "batch init");
  }
  BHIP(b, hipStreamSynchronize(b->stream), "batch init");
  return ESBGK_OK;
}

}  // namespace

extern "C" {

size_t esbgk_batch_workspace_bytes(const esbgk_problem* problems, int n) {
  if (!problems || n < 1) return 0;
  for (int i = 0; i < n; ++i)
    if (!valid_problem(problems[i], problems[0], nullptr)) return 0;
  if (!host_lattice(problems[0].shape.velset)) return 0;
  return blayout(problems, n).total;
}

int esbgk_batch_create(const esbgk_problem* problems, int n, void* d_workspace, size_t ws_bytes, void* hip_stream,
                       esbgk_batch** out) {
  if (!out) return ESBGK_E_INVALID;
  *out = nullptr;
  if (!problems || n < 1) return ESBGK_E_INVALID;
  for (int i = 0; i < n; ++i)
    if (!valid_problem(problems[i], problems[0], nullptr)) return ESBGK_E_INVALID;
  const HostLattice* lat = host_lattice(problems[0].shape.velset);
  if (!lat) return ESBGK_E_INVALID;
  const BLayout lay = blayout(problems, n);
  if (!d_workspace || ws_bytes < lay.total) return ESBGK_E_NOMEM;
  if (reinterpret_cast<uintptr_t>(d_workspace) % ALIGN) return ESBGK_E_INVALID;
  esbgk_batch* b = new esbgk_batch();
  b->p.assign(problems, problems + n);
  b->lat = lat;
  b->velset = problems[0].shape.velset;
  b->storage = problems[0].shape.storage;
  b->lay = lay;
  b->ws = static_cast<char*>(d_workspace);
  b->stream = static_cast<hipStream_t>(hip_stream);
  int dev = 0;
  hipDeviceProp_t prop{};
  if (hipGetDevice(&dev) != hipSuccess || hipGetDeviceProperties(&prop, dev) != hipSuccess) {
    delete b;
    return ESBGK_E_HIP;
  }
  b->cus = prop.multiProcessorCount;
  // descriptors and parameter blocks
  size_t pop = 0, wp = 0;
  b->bp.resize(n);
  const size_t ppsz = csize(b->storage) == 8 ? sizeof(ProbParams<double>) : sizeof(ProbParams<float>);
  std::vector<unsigned char> pps(size_t(n) * ppsz);
  std::vector<ProbParams<double>> pps64(n);
  for (int i = 0; i < n; ++i) {
    const esbgk_shape& s = problems[i].shape;
    BatchProblem& q = b->bp[i];
    make_geometry(lat->D, lat->Q, uint32_t(s.nx), uint32_t(s.ny), uint32_t(s.nz), true, false, ssize(b->storage),
                  q.geo);
    q.pop_off = pop;
    q.wp_off = uint32_t(wp);
    pop += size_t(lat->Q) * q.geo.ncells;
    pop = (pop + 63) / 64 * 64;
    wp += 6 * size_t(q.geo.ncols);
    const int nref = s.n_ref > 0 ? s.n_ref : (lat->D == 2 ? s.ny : s.nz);
    const double gam[2] = {1.0 - problems[i].specular[0], 1.0 - problems[i].specular[1]};
    const HostProblem hp = make_problem(*lat, nref, s.scheme, problems[i].Kn, problems[i].Pr, problems[i].varpi,
                                        problems[i].g, problems[i].T_w, problems[i].u_w, gam);
    pack_params<double>(hp, lat->Q, pps64[i]);
    if (csize(b->storage) == 8) pack_params<double>(hp, lat->Q, *reinterpret_cast<ProbParams<double>*>(&pps[i * ppsz]));
    else pack_params<float>(hp, lat->Q, *reinterpret_cast<ProbParams<float>*>(&pps[i * ppsz]));
  }
  int rc = ESBGK_OK;
  auto cp = [&](size_t off, const void* src, size_t bytes) {
    if (rc == ESBGK_OK && hipMemcpyAsync(b->at(off), src, bytes, hipMemcpyHostToDevice, b->stream) != hipSuccess)
      rc = ESBGK_E_HIP;
  };
  cp(lay.probs, b->bp.data(), b->bp.size() * sizeof(BatchProblem));
  cp(lay.pps, pps.data(), pps.size());
  LatConsts<double> l64{};
  LatConsts<float> l32{};
  pack_lattice<double>(*lat, l64);
  if (csize(b->storage) == 8) {
    cp(lay.lc, &l64, sizeof(l64));
  } else {
    pack_lattice<float>(*lat, l32);
    cp(lay.lc, &l32, sizeof(l32));
    cp(lay.lc64, &l64, sizeof(l64));
    cp(lay.pps64, pps64.data(), pps64.size() * sizeof(ProbParams<double>));
  }
  if (rc == ESBGK_OK && hipStreamSynchronize(b->stream) != hipSuccess) rc = ESBGK_E_HIP;
  if (rc != ESBGK_OK) {
    delete b;
    return rc;
  }
  // default layout: the largest workgroup, as many bins as workgroups resident at once
  b->threads = uint32_t(batch_max_threads(ssize(b->storage)));
  const uint32_t per_cu = std::max<uint32_t>(1, 1024u / b->threads);
  if (build_bins(b, uint32_t(b->cus) * per_cu) != ESBGK_OK) {
    const int e = b->sticky ? b->sticky : ESBGK_E_INVALID;
    delete b;
    return e;
  }
  *out = b;
  return ESBGK_OK;
}

int esbgk_batch_destroy(esbgk_batch* b) {
  if (!b) return ESBGK_E_INVALID;
  delete b;
  return ESBGK_OK;
}

int esbgk_batch_set_layout(esbgk_batch* b, int threads, int nbins) {
  if (!b) return ESBGK_E_INVALID;
  if (b->sticky) return b->sticky;
  if (threads < 64 || threads % 64 || threads > batch_max_threads(ssize(b->storage)) || nbins < 1) {
    b->err = "threads must be a multiple of 64 up to the storage type's limit; nbins >= 1";
    return ESBGK_E_INVALID;
  }
  b->threads = uint32_t(threads);
  return build_bins(b, uint32_t(nbins));
}

int esbgk_batch_layout(const esbgk_batch* b, int* threads, int* nbins) {
  if (!b) return ESBGK_E_INVALID;
  if (threads) *threads = int(b->threads);
  if (nbins) *nbins = int(b->nbins);
  return ESBGK_OK;
}

int esbgk_batch_autotune(esbgk_batch* b, int steps_per_trial) {
  if (!b) return ESBGK_E_INVALID;
  if (b->sticky) return b->sticky;
  if (steps_per_trial < 1) {
    b->err = "steps_per_trial must be >= 1";
    return ESBGK_E_INVALID;
  }
  // trials run on the uniform rest state; the state must be set afterwards
  b->parity = 0;
  int rc = rest_state(b, nullptr, 0.0);
  if (rc) return rc;
  b->state_set = false;
  const int maxt = batch_max_threads(ssize(b->storage));
  hipEvent_t e0, e1;
  BHIP(b, hipEventCreate(&e0), "autotune");
  BHIP(b, hipEventCreate(&e1), "autotune");
  float best = 1e30f;
  uint32_t best_t = b->threads, best_n = b->nbins;
  for (int t = 256; t <= maxt; t *= 2) {
    for (int per : {1, 2, 4, 8}) {
      const uint32_t nb = uint32_t(b->cus) * uint32_t(per);
      b->threads = uint32_t(t);
      if (build_bins(b, nb) != ESBGK_OK) continue;
      BatchLaunch a = launch_args(b, 2);
      a.parity = 0;
      BHIP(b, launch_batch(b->velset, b->storage, a), "autotune");
      a.nsteps = steps_per_trial;
      BHIP(b, hipEventRecord(e0, b->stream), "autotune");
      BHIP(b, launch_batch(b->velset, b->storage, a), "autotune");
      BHIP(b, hipEventRecord(e1, b->stream), "autotune");
      BHIP(b, hipEventSynchronize(e1), "autotune");
      float ms = 0;
      BHIP(b, hipEventElapsedTime(&ms, e0, e1), "autotune");
      if (ms < best) {
        best = ms;
        best_t = uint32_t(t);
        best_n = b->nbins;
      }
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  b->threads = best_t;
  return build_bins(b, best_n);
}

int esbgk_batch_init_equilibrium(esbgk_batch* b, const double* noise, double amplitude) {
  if (!b) return ESBGK_E_INVALID;
  if (b->sticky) return b->sticky;
  if (noise && !std::isfinite(amplitude)) return ESBGK_E_INVALID;
  b->parity = 0;
  int rc = rest_state(b, noise, amplitude);
  if (rc) return rc;
  b->state_set = true;
  b->steps = 0;
  return ESBGK_OK;
}

int esbgk_batch_step(esbgk_batch* b, int64_t n) {
  if (!b) return ESBGK_E_INVALID;
  if (b->sticky) return b->sticky;
  if (n < 0) return ESBGK_E_INVALID;
  if (!b->state_set) {
    b->err = "no state set";
    return ESBGK_E_STATE;
  }
  if (n == 0) return ESBGK_OK;
  BatchLaunch a = launch_args(b, n);
  BHIP(b, launch_batch(b->velset, b->storage, a), "batch step");
  b->parity ^= int(n & 1);
  b->steps += n;
  return ESBGK_OK;
}

int esbgk_batch_read_moments(esbgk_batch* b, int i, double* h_out, int* F) {
  if (!b || !h_out || i < 0 || i >= int(b->p.size())) return ESBGK_E_INVALID;
  if (b->sticky) return b->sticky;
  if (!b->state_set) return ESBGK_E_STATE;
  const int nf = nfields(b->lat->D);
  if (F) *F = nf;
  StepArgs a = problem_args(b, i);
  const uint32_t cells = a.geo.ncells;
  double* st = reinterpret_cast<double*>(b->at(b->lay.staging));
  std::vector<double> tmp;
  for (uint32_t c0 = 0; c0 < cells; c0 += STAGE_CELLS) {
    const uint32_t n = std::min(STAGE_CELLS, cells - c0);
    BHIP(b, launch_moments(b->velset, b->storage, a, c0, n, st), "batch moments");
    tmp.resize(size_t(nf) * n);
    BHIP(b, hipMemcpyAsync(tmp.data(), st, tmp.size() * 8, hipMemcpyDeviceToHost, b->stream), "batch moments");
    BHIP(b, hipStreamSynchronize(b->stream), "batch moments");
    for (int f = 0; f < nf; ++f) std::memcpy(h_out + size_t(f) * cells + c0, tmp.data() + size_t(f) * n, n * 8);
  }
  return ESBGK_OK;
}

int esbgk_batch_get_populations(esbgk_batch* b, int i, double* h) {
  if (!b || !h || i < 0 || i >= int(b->p.size())) return ESBGK_E_INVALID;
  if (b->sticky) return b->sticky;
  if (!b->state_set) return ESBGK_E_STATE;
  StepArgs a = problem_args(b, i);
  const size_t cells = a.geo.ncells, ss = ssize(b->storage);
  std::vector<unsigned char> buf(size_t(b->lat->Q) * cells * ss);
  BHIP(b, hipMemcpyAsync(buf.data(), a.src, buf.size(), hipMemcpyDeviceToHost, b->stream), "batch populations");
  BHIP(b, hipStreamSynchronize(b->stream), "batch populations");
  const size_t tot = size_t(b->lat->Q) * cells;
  for (size_t k = 0; k < tot; ++k) {
    if (b->storage == ESBGK_F64) h[k] = reinterpret_cast<const double*>(buf.data())[k];
    else if (b->storage == ESBGK_F32) h[k] = double(reinterpret_cast<const float*>(buf.data())[k]);
    else h[k] = double(reinterpret_cast<const _Float16*>(buf.data())[k]);
  }
  return ESBGK_OK;
}

int64_t esbgk_batch_steps_done(const esbgk_batch* b) { return b ? b->steps : -1; }

const char* esbgk_batch_last_error(const esbgk_batch* b) { return b ? b->err.c_str() : "null handle"; }

}  // extern "C"
