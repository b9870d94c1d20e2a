// C ABI of batched channel problems: validation, workspace layout, binning
// (longest problem, or piece of a cut problem, first into the lightest bin),
// the autotuner that picks the workgroup size, the number of bins and the
// piece size by timing the step launches, and the per-problem state I/O.
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
  size_t bufA, bufB, wpA, wpB, probs, pps, lc, pps64, lc64, bin_first, order, piece_c0, piece_n, staging, total;
  size_t uprev, chunks, red_out, red_level, level;
  size_t pop_elems, wp_elems, max_pieces;
};

constexpr const char* UNSTABLE_MSG = "Euler step unstable: dt/tau or dt/(Pr tau) >= 2";

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
  if (s.scheme == ESBGK_EULER) {
    // forward Euler along the characteristic needs dt/tau < 2 and
    // dt/(Pr tau) < 2 at rho = T = 1 (dt = dx/r, dx = 1/N_L)
    const HostLattice* lat = host_lattice(s.velset);
    const int nref = s.n_ref > 0 ? s.n_ref : nw;
    const double dt = 1.0 / (double(nref) * (lat ? lat->r : 1.0));
    if (!(dt * p.Pr / p.Kn < 2.0 && dt / p.Kn < 2.0)) return fail(UNSTABLE_MSG);
  }
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
  size_t pop = 0, wp = 0, maxc = 0, cells = 0, chunks = 0;
  for (int i = 0; i < n; ++i) {
    pop += size_t(lat->Q) * cells_of(p[i].shape);
    pop = (pop + 63) / 64 * 64;
    wp += 6 * size_t(ncols_of(p[i].shape));
    maxc = std::max<size_t>(maxc, cells_of(p[i].shape));
    cells += cells_of(p[i].shape);
    chunks += (cells_of(p[i].shape) + 63) / 64;
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
  // pieces (whole problems, or problems cut into 64-cell chunks): at most one per chunk
  L.max_pieces = chunks;
  L.bin_first = take(size_t(chunks + 1) * 4);
  L.order = take(chunks * 4);
  L.piece_c0 = take(chunks * 4);
  L.piece_n = take(chunks * 4);
  L.uprev = take(size_t(lat->D) * cells * csize(storage));
  L.chunks = take(chunks * NRED * sizeof(double));
  L.red_out = take(size_t(n) * NRED * sizeof(double));
  L.red_level = take(size_t(n) * sizeof(int64_t));
  L.level = take(sizeof(int64_t));
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
  uint32_t req_bins = 0;       // the bin count last asked for (nbins is that, capped by the piece count)
  uint32_t piece = 0;          // cells per piece of a cut problem (a multiple of 64); 0: whole problems
  bool split = false;          // some problem is cut into several pieces (one step per launch)
  int cus = 0;
  int sticky = 0;
  std::string err;
  int64_t R = 0;               // fused reduction interval (0: none)
  // the persistent launch (kernel + level update) captured once per step
  // count n and replayed; released when the launch changes (layout, R)
  bool use_graphs = true;
  hipStream_t cap = nullptr;
  std::vector<std::pair<int64_t, hipGraphExec_t>> graphs;
  std::vector<uint64_t> bin_slots;   // thread slots (cells rounded up to 64 per problem) of each bin
  std::vector<uint32_t> bin_count;   // problems of each bin
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

// The problems as pieces (b->piece cells each, whole 64-cell chunks, the
// last piece of a problem taking the rest; whole problems when b->piece is 0
// or not smaller), longest piece first, each into the bin with the fewest
// slots (a piece's cells rounded up to a multiple of 64).
int build_bins(esbgk_batch* b, uint32_t nbins) {
  const uint32_t requested = nbins;
  struct Piece {
    uint32_t id, c0, n;
  };
  std::vector<Piece> pcs;
  bool split = false;
  for (size_t i = 0; i < b->p.size(); ++i) {
    const uint32_t nc = b->bp[i].geo.ncells;
    const uint32_t len = b->piece > 0 && b->piece < nc ? b->piece : nc;
    split = split || len < nc;
    for (uint32_t c0 = 0; c0 < nc; c0 += len) pcs.push_back({uint32_t(i), c0, std::min(len, nc - c0)});
  }
  if (pcs.size() > b->lay.max_pieces) return ESBGK_E_INVALID;   // not reached: a piece holds >= 64 cells
  const uint32_t npc = uint32_t(pcs.size());
  nbins = std::max<uint32_t>(1, std::min<uint32_t>(nbins, npc));
  std::vector<uint32_t> idx(npc);
  std::iota(idx.begin(), idx.end(), 0u);
  std::stable_sort(idx.begin(), idx.end(), [&](uint32_t x, uint32_t y) { return pcs[x].n > pcs[y].n; });
  using Item = std::pair<uint64_t, uint32_t>;   // (slots, bin)
  std::priority_queue<Item, std::vector<Item>, std::greater<Item>> heap;
  for (uint32_t k = 0; k < nbins; ++k) heap.push({0, k});
  std::vector<std::vector<uint32_t>> bins(nbins);
  for (uint32_t j : idx) {
    Item it = heap.top();
    heap.pop();
    while (bins[it.second].size() >= size_t(BATCH_MAX_PER_BIN)) {   // a full bin leaves the heap
      if (heap.empty()) return ESBGK_E_INVALID;
      it = heap.top();
      heap.pop();
    }
    bins[it.second].push_back(j);
    it.first += (pcs[j].n + 63u) & ~63u;
    heap.push(it);
  }
  std::vector<uint32_t> first(nbins + 1), order, c0s, ns;
  order.reserve(npc);
  c0s.reserve(npc);
  ns.reserve(npc);
  b->bin_slots.assign(nbins, 0);
  b->bin_count.assign(nbins, 0);
  for (uint32_t k = 0; k < nbins; ++k) {
    first[k] = uint32_t(order.size());
    for (uint32_t j : bins[k]) {
      order.push_back(pcs[j].id);
      c0s.push_back(pcs[j].c0);
      ns.push_back(pcs[j].n);
      b->bin_slots[k] += (pcs[j].n + 63u) & ~63u;
    }
    b->bin_count[k] = uint32_t(bins[k].size());
  }
  first[nbins] = uint32_t(order.size());
  BHIP(b, hipMemcpyAsync(b->at(b->lay.bin_first), first.data(), first.size() * 4, hipMemcpyHostToDevice, b->stream),
       "bins");
  BHIP(b, hipMemcpyAsync(b->at(b->lay.order), order.data(), order.size() * 4, hipMemcpyHostToDevice, b->stream),
       "bins");
  BHIP(b, hipMemcpyAsync(b->at(b->lay.piece_c0), c0s.data(), c0s.size() * 4, hipMemcpyHostToDevice, b->stream),
       "bins");
  BHIP(b, hipMemcpyAsync(b->at(b->lay.piece_n), ns.data(), ns.size() * 4, hipMemcpyHostToDevice, b->stream), "bins");
  BHIP(b, hipStreamSynchronize(b->stream), "bins");
  b->nbins = nbins;
  b->req_bins = requested;
  b->split = split;
  return ESBGK_OK;
}

BatchLaunch launch_args(const esbgk_batch* b, int64_t n) {
  BatchLaunch a{};
  a.probs = reinterpret_cast<const BatchProblem*>(b->at(b->lay.probs));
  a.pps = b->at(b->lay.pps);
  a.bin_first = reinterpret_cast<const uint32_t*>(b->at(b->lay.bin_first));
  a.order = reinterpret_cast<const uint32_t*>(b->at(b->lay.order));
  a.piece_c0 = reinterpret_cast<const uint32_t*>(b->at(b->lay.piece_c0));
  a.piece_n = reinterpret_cast<const uint32_t*>(b->at(b->lay.piece_n));
  a.split = b->split ? 1 : 0;
  a.nprob = uint32_t(b->p.size());
  a.bufA = b->at(b->lay.bufA);
  a.bufB = b->at(b->lay.bufB);
  a.wpA = b->at(b->lay.wpA);
  a.wpB = b->at(b->lay.wpB);
  a.lc = b->at(b->lay.lc);
  a.nsteps = n;
  a.red.level = reinterpret_cast<const int64_t*>(b->at(b->lay.level));
  a.red.R = b->R;
  a.red.uprev = b->at(b->lay.uprev);
  a.red.chunks = reinterpret_cast<double*>(b->at(b->lay.chunks));
  a.red.out = reinterpret_cast<double*>(b->at(b->lay.red_out));
  a.red.red_level = reinterpret_cast<int64_t*>(b->at(b->lay.red_level));
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

// Device step counter = the host's, no reduction recorded yet.
int reset_levels(esbgk_batch* b) {
  BHIP(b, hipMemcpyAsync(b->at(b->lay.level), &b->steps, sizeof(int64_t), hipMemcpyHostToDevice, b->stream),
       "batch level");
  BHIP(b, hipMemsetAsync(b->at(b->lay.red_level), 0xff, b->p.size() * sizeof(int64_t), b->stream), "batch level");
  BHIP(b, hipStreamSynchronize(b->stream), "batch level");
  return ESBGK_OK;
}

// Release the captured launches; a replay may still be queued on the
// caller's stream, so wait for it first.
void drop_batch_graphs(esbgk_batch* b) {
  if (!b->graphs.empty() && hipStreamSynchronize(b->stream) != hipSuccess) {
    b->sticky = ESBGK_E_HIP;
    b->err = "synchronize before releasing the batch graphs failed";
  }
  for (auto& g : b->graphs) (void)hipGraphExecDestroy(g.second);
  b->graphs.clear();
}

// n steps: one persistent launch, or with split problems n launches of one
// step each (the kernel, the per-problem sums, the level update).
hipError_t launch_steps(const esbgk_batch* b, hipStream_t stream, int64_t n) {
  BatchLaunch a = launch_args(b, b->split ? 1 : n);
  a.stream = stream;
  const int64_t launches = b->split ? n : 1;
  for (int64_t k = 0; k < launches; ++k) {
    const hipError_t e = launch_batch(b->velset, b->storage, a);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

// Largest step count captured in one graph with split problems (three
// nodes a step).
constexpr int64_t SPLIT_GRAPH_STEPS = 32;

// The captured launch of n steps (kernel + level update), built on first use.
int batch_graph(esbgk_batch* b, int64_t n, hipGraphExec_t* out) {
  for (auto& g : b->graphs)
    if (g.first == n) {
      *out = g.second;
      return ESBGK_OK;
    }
  if (!b->cap) {
    hipError_t e = hipStreamCreateWithFlags(&b->cap, hipStreamNonBlocking);
    if (e != hipSuccess) {
      b->cap = nullptr;
      return bfail(b, e, "create capture stream");
    }
  }
  if (b->graphs.size() >= 4) drop_batch_graphs(b);   // a few step counts in use at a time
  BHIP(b, hipStreamBeginCapture(b->cap, hipStreamCaptureModeRelaxed), "begin capture");
  const hipError_t le = launch_steps(b, b->cap, n);
  hipGraph_t g = nullptr;
  const hipError_t ee = hipStreamEndCapture(b->cap, &g);
  if (le != hipSuccess) {
    if (g) (void)hipGraphDestroy(g);
    return bfail(b, le, "capture batch step");
  }
  if (ee != hipSuccess) return bfail(b, ee, "end capture");
  hipGraphExec_t ex = nullptr;
  const hipError_t ie = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
  (void)hipGraphDestroy(g);
  if (ie != hipSuccess) return bfail(b, ie, "instantiate batch graph");
  b->graphs.push_back({n, ex});
  *out = ex;
  return ESBGK_OK;
}

// Host form of the raw sums of one problem (as esbgk_reduce): mass, energy,
// momentum, mass flow rate dx^(D-1)/nx sum rho u_x, residual, level.
bool finish_reduction(const esbgk_batch* b, int i, const double* raw, int64_t level, double* out) {
  const esbgk_shape& s = b->p[i].shape;
  const int D = b->lat->D;
  const int nref = s.n_ref > 0 ? s.n_ref : (D == 2 ? s.ny : s.nz);
  const double dx = 1.0 / double(nref);
  for (int k = 0; k < 5; ++k) out[k] = raw[k];
  out[5] = std::pow(dx, D - 1) / double(s.nx) * raw[2];
  out[6] = raw[6] > 0.0 ? std::sqrt(raw[5] / raw[6]) : 0.0;
  out[7] = double(level);
  return raw[7] == 0.0 && std::isfinite(raw[0]) && std::isfinite(raw[1]);
}

int fetch_batch_reduction(esbgk_batch* b, double* out) {
  const size_t n = b->p.size();
  std::vector<double> raw(n * NRED);
  std::vector<int64_t> lev(n);
  BHIP(b, hipMemcpyAsync(raw.data(), b->at(b->lay.red_out), raw.size() * 8, hipMemcpyDeviceToHost, b->stream),
       "batch reduction");
  BHIP(b, hipMemcpyAsync(lev.data(), b->at(b->lay.red_level), n * 8, hipMemcpyDeviceToHost, b->stream),
       "batch reduction");
  BHIP(b, hipStreamSynchronize(b->stream), "batch reduction");
  bool ok = true;
  for (size_t i = 0; i < n; ++i) {
    if (lev[i] < 0) {
      b->err = "no reduction has run since the state was set";
      return ESBGK_E_STATE;
    }
    ok = finish_reduction(b, int(i), raw.data() + i * NRED, lev[i], out + i * 8) && ok;
  }
  if (!ok) {
    b->sticky = ESBGK_E_NONFINITE;
    b->err = "reduction found a non-finite value, rho <= 0 or T <= 0";
    return ESBGK_E_NONFINITE;
  }
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
  for (int i = 0; i < n; ++i) {
    std::string why;
    if (!valid_problem(problems[i], problems[0], &why))
      return why == UNSTABLE_MSG ? ESBGK_E_UNSTABLE : ESBGK_E_INVALID;
  }
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
  size_t pop = 0, wp = 0, cell0 = 0, chunk0 = 0;
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
    q.cell_off = cell0;
    q.chunk_off = uint32_t(chunk0);
    cell0 += q.geo.ncells;
    chunk0 += (q.geo.ncells + 63u) / 64u;
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
  drop_batch_graphs(b);
  if (b->cap) (void)hipStreamDestroy(b->cap);
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
  drop_batch_graphs(b);
  b->threads = uint32_t(threads);
  return build_bins(b, uint32_t(nbins));
}

int esbgk_batch_set_split(esbgk_batch* b, int piece_cells) {
  if (!b) return ESBGK_E_INVALID;
  if (b->sticky) return b->sticky;
  if (piece_cells < 0 || piece_cells % 64) {
    b->err = "piece_cells must be 0 (whole problems) or a positive multiple of 64";
    return ESBGK_E_INVALID;
  }
  drop_batch_graphs(b);
  const uint32_t old = b->piece;
  b->piece = uint32_t(piece_cells);
  const int rc = build_bins(b, b->req_bins);
  if (rc) b->piece = old;
  return rc;
}

int esbgk_batch_split(const esbgk_batch* b, int* piece_cells, int* active) {
  if (!b) return ESBGK_E_INVALID;
  if (piece_cells) *piece_cells = int(b->piece);
  if (active) *active = b->split ? 1 : 0;
  return ESBGK_OK;
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
  drop_batch_graphs(b);
  b->parity = 0;
  b->steps = 0;
  int rc = rest_state(b, nullptr, 0.0);
  if (rc) return rc;
  rc = reset_levels(b);
  if (rc) return rc;
  b->state_set = false;
  const int maxt = batch_max_threads(ssize(b->storage));
  // candidate bin counts: 1, 2, 4, 8 workgroups per compute unit, and one
  // problem per workgroup
  std::vector<uint32_t> bins_c;
  for (int per : {1, 2, 4, 8}) bins_c.push_back(uint32_t(b->cus) * uint32_t(per));
  bins_c.push_back(uint32_t(b->p.size()));
  // candidate pieces: whole problems, and (when the largest problem would
  // fill a compute unit's share of the batch several times over) problems
  // cut so that the pieces outnumber the compute units about 4 to 1
  std::vector<uint32_t> piece_c = {0};
  uint64_t total = 0;
  uint32_t largest = 0;
  for (const auto& q : b->bp) {
    total += q.geo.ncells;
    largest = std::max(largest, q.geo.ncells);
  }
  const uint64_t share = std::max<uint64_t>(64, (total / (4u * uint64_t(b->cus)) + 63) / 64 * 64);
  if (largest > 2 * share) {
    piece_c.push_back(uint32_t(share));
    const uint32_t quarter = uint32_t(std::max<uint64_t>(64, share / 4 / 64 * 64));
    if (quarter != share) piece_c.push_back(quarter);
  }
  hipEvent_t e0, e1;
  BHIP(b, hipEventCreate(&e0), "autotune");
  BHIP(b, hipEventCreate(&e1), "autotune");
  float best = 1e30f;
  uint32_t best_t = b->threads, best_n = b->req_bins, best_p = 0;
  for (uint32_t pc : piece_c) {
    b->piece = pc;
    for (int t = 256; t <= maxt; t *= 2) {
      for (uint32_t nb : bins_c) {
        b->threads = uint32_t(t);
        if (build_bins(b, nb) != ESBGK_OK) continue;
        if (pc > 0 && !b->split) continue;   // no problem was cut: the same as whole problems
        BHIP(b, launch_steps(b, b->stream, 2), "autotune");
        BHIP(b, hipEventRecord(e0, b->stream), "autotune");
        BHIP(b, launch_steps(b, b->stream, steps_per_trial), "autotune");
        BHIP(b, hipEventRecord(e1, b->stream), "autotune");
        BHIP(b, hipEventSynchronize(e1), "autotune");
        float ms = 0;
        BHIP(b, hipEventElapsedTime(&ms, e0, e1), "autotune");
        if (ms < best) {
          best = ms;
          best_t = uint32_t(t);
          best_n = nb;
          best_p = pc;
        }
      }
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  b->threads = best_t;
  b->piece = best_p;
  rc = build_bins(b, best_n);
  if (rc) return rc;
  return reset_levels(b);
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
  return reset_levels(b);
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
  if (b->use_graphs) {
    // split problems: graphs of at most SPLIT_GRAPH_STEPS steps, replayed
    for (int64_t left = n; left > 0;) {
      const int64_t g_n = b->split ? std::min(left, SPLIT_GRAPH_STEPS) : left;
      hipGraphExec_t g = nullptr;
      const int rc = batch_graph(b, g_n, &g);
      if (rc) return rc;
      BHIP(b, hipGraphLaunch(g, b->stream), "batch graph launch");
      left -= g_n;
    }
  } else {
    BHIP(b, launch_steps(b, b->stream, n), "batch step");
  }
  b->parity ^= int(n & 1);
  b->steps += n;
  return ESBGK_OK;
}

int esbgk_batch_use_graphs(esbgk_batch* b, int on) {
  if (!b) return ESBGK_E_INVALID;
  if (b->sticky) return b->sticky;
  if (on != 0 && on != 1) {
    b->err = "on must be 0 or 1";
    return ESBGK_E_INVALID;
  }
  if (!on) drop_batch_graphs(b);
  b->use_graphs = on != 0;
  return ESBGK_OK;
}

int esbgk_batch_set_reduce_interval(esbgk_batch* b, int64_t R) {
  if (!b) return ESBGK_E_INVALID;
  if (b->sticky) return b->sticky;
  if (R < 0) {
    b->err = "R must be >= 0";
    return ESBGK_E_INVALID;
  }
  if (R != b->R) drop_batch_graphs(b);   // R is baked into the captured launches
  b->R = R;
  return ESBGK_OK;
}

int esbgk_batch_reduce(esbgk_batch* b, double* out) {
  if (!b || !out) return ESBGK_E_INVALID;
  if (b->sticky) return b->sticky;
  if (!b->state_set) {
    b->err = "no state set";
    return ESBGK_E_STATE;
  }
  BatchLaunch a = launch_args(b, 0);
  BHIP(b, launch_batch_reduce(b->velset, b->storage, a, b->at(b->lay.pps64), b->at(b->lay.lc64), b->steps),
       "batch reduce");
  return fetch_batch_reduction(b, out);
}

int esbgk_batch_last_reduction(esbgk_batch* b, double* out) {
  if (!b || !out) return ESBGK_E_INVALID;
  if (b->sticky) return b->sticky;
  if (!b->state_set) {
    b->err = "no state set";
    return ESBGK_E_STATE;
  }
  return fetch_batch_reduction(b, out);
}

int esbgk_batch_layout_info(const esbgk_batch* b, int* max_pieces_per_bin, int64_t* max_cells_per_thread) {
  if (!b) return ESBGK_E_INVALID;
  int mp = 0;
  int64_t mc = 0;
  for (size_t k = 0; k < b->bin_slots.size(); ++k) {
    mp = std::max(mp, int(b->bin_count[k]));
    mc = std::max<int64_t>(mc, (int64_t(b->bin_slots[k]) + b->threads - 1) / b->threads);
  }
  if (max_pieces_per_bin) *max_pieces_per_bin = mp;
  if (max_cells_per_thread) *max_cells_per_thread = mc;
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
