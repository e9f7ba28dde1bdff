// Host runtime of libgbs: contexts, resident GBS states, validation, work planning, staging,
// HIP-graph capture and the C ABI declared in include/gbs.h.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <cstdlib>
#include <climits>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <list>
#include <map>
#include <mutex>
#include <string>
#include <tuple>
#include <vector>

#include "gbs.h"
#include "gbs_internal.h"

#include "gbs_chain_table.h"
#include "gbs_tables.h"

using namespace gbs;

namespace {

constexpr size_t kLdsBudget = 160 * 1024;

// ------------------------------------------------------------------ helpers

int64_t subset_count(int n) {
  if (n <= 0 || (n & 1)) return 0;
  return (int64_t(1) << (n / 2)) - 1;
}

// first canonical index of subsets with |Z| = s (s >= 1)
int64_t size_start(int k, int s) {
  int64_t g = 0;
  for (int q = 1; q < s && q <= k; ++q) g += (int64_t)kBinom.v[k][q];
  return g;
}

double flops_subset(const ChainProgram& p, int k, int s) {
  const double d = 2.0 * s;
  return p.nmul * 8.0 * d * d * d + p.npair * 8.0 * d * d + 8.0 * k * (k + 1) / 2.0;
}

struct Plan {
  std::vector<PatternDesc> pats;
  std::vector<WorkItem> items;  // grouped by engine kernel
  struct Group {
    int cls;                     // engine kernel variant (one k per variant)
    int n;                       // photon number of every pattern in the group
    int64_t first, count;
  };
  std::vector<Group> groups;
  std::vector<int64_t> part_off;  // batch + 1 (finalize groups)
  std::vector<int32_t> nvec;
  std::vector<double> sfact;
  std::vector<int64_t> out_idx;  // optional destination index per finalize group
  int64_t n_partials = 0;
  int nmax = 0, kmax = 0;
  int nmin = GBS_N_MAX + 1;  // smallest n that has items
};

// The runs of subset sizes of a size-n pattern that share an engine variant (engine_class), in
// increasing |Z|, each with its range [a, b) of the canonical order clipped to [lo, hi) and its chunk:
// chunk_small subsets per item for |Z| <= 8, chunk_large above.
struct ClassRun {
  int cls;
  int64_t a, b, chunk;
};

constexpr int64_t kDdChunk = 32;

struct ItemLists {
  std::vector<WorkItem> cls[kEngineClasses];  // by engine kernel variant
  std::vector<ClassRun> full_runs[GBS_N_MAX + 1];  // class runs of a whole size-n pattern
  bool have_full[GBS_N_MAX + 1] = {};
};

// Empty a plan and its item lists for the next call, keeping their storage: a batch of the same
// shape then plans without reallocating or touching fresh pages (100,000 twenty-photon patterns are
// 600,000 items).
void plan_reset(Plan& pl, ItemLists& L) {
  pl.pats.clear();
  pl.items.clear();
  pl.groups.clear();
  pl.part_off.clear();
  pl.nvec.clear();
  pl.sfact.clear();
  pl.out_idx.clear();
  pl.n_partials = 0;
  pl.nmax = pl.kmax = 0;
  pl.nmin = GBS_N_MAX + 1;
  for (std::vector<WorkItem>& v : L.cls) v.clear();
  for (bool& h : L.have_full) h = false;  // the launch shape may have changed since
}

}  // namespace

// ------------------------------------------------------------------ objects

struct GraphKey {
  std::vector<int64_t> v;
  bool operator<(const GraphKey& o) const { return v < o.v; }
};

struct gbs_ctx {
  int device = 0;
  int ncu = 0;
  void* ws = nullptr;        // caller-owned workspace
  size_t ws_bytes = 0;
  size_t ws_needed = 0;      // what the last call that found it too small needed
  // ring of pinned staging buffers: a call reuses a buffer once the copy from it (kPinRing calls
  // back) has run. Six let a caller keep three two-call steps in flight without waiting. All of them
  // are (re)allocated together, at the first call and whenever a call needs more: pinned allocation
  // in the middle of a stream of calls stalls the device, so it must not happen in steady state.
  static constexpr int kPinRing = 6;
  void* pinned[kPinRing] = {};
  size_t pinned_bytes = 0;  // every buffer has this size
  hipEvent_t pinned_ev[kPinRing] = {};
  bool pinned_used[kPinRing] = {};
  int pin_idx = 0;
  hipEvent_t done_ev = nullptr;
  bool done_recorded = false;
  hipStream_t cap_stream = nullptr;
  int use_graph = 1;
  int persistent = 1;
  // spread a call's engine kernels over this many streams (forked from and joined back into the
  // caller's stream; in a captured graph the fork and join are edges), so per-variant kernels overlap
  static constexpr int kMaxStreams = 8;
  // default: two (measured no slower than one on every one-size workload and 1.1% faster on the
  // n = 24 batch, whose four kernels then overlap their tails; three were 11% slower there)
  static constexpr int kDefaultStreams = 2;
  int nstreams = 1;
  bool streams_auto = true;  // no gbs_ctx_set_streams yet: one-size calls take the table's count
  hipStream_t aux[kMaxStreams] = {};
  hipEvent_t aux_ev[kMaxStreams] = {};
  hipEvent_t fork_ev = nullptr;
  int precision = kPrecFp64;
  std::map<int, std::pair<int64_t, int64_t>> tuning;
  std::map<int, int> shape;  // engine shape bits per n (kShape*)
  std::string last_error;
  std::list<std::pair<GraphKey, hipGraphExec_t>> graphs;  // most recent first
  // the work plan of the call in progress, kept between calls for its storage (plan_reset)
  Plan plan;
  ItemLists lists;
};

// Views into caller-owned state memory (layout: state_layout).
struct gbs_state {
  int device = 0;
  int m = 0;
  double2* B = nullptr;
  double2* W = nullptr;  // U U^t (marginal probabilities)
  double* r = nullptr;
  double* pref = nullptr;
  double pref_host = 0.0;
  hipEvent_t ready = nullptr;
};

namespace {

int fail(gbs_ctx* ctx, int code, const char* fmt, ...) {
  if (ctx) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    ctx->last_error = buf;
  }
  return code;
}

#define HIPCHK(ctx, expr)                                                                      \
  do {                                                                                         \
    hipError_t e_ = (expr);                                                                    \
    if (e_ != hipSuccess) return fail(ctx, GBS_EHIP, "%s: %s", #expr, hipGetErrorString(e_));  \
  } while (0)

// Debugging hooks. Fault injection: the N-th call (counted from when it was armed) that would
// enqueue compute work returns GBS_EHIP instead and enqueues nothing (GBS_FAULT_INJECT=launch:N in the
// environment, read once, or gbs_debug_fault_inject). Symmetry check of caller-provided matrices
// before the hafnian path runs (GBS_CHECK_SYMMETRY=1, or gbs_debug_check_symmetry).
std::atomic<int64_t> g_launches{0};
std::atomic<int64_t> g_fault_at{-2};  // -2: environment not read yet; <= 0: off
std::atomic<int> g_check_sym{-1};     // -1: environment not read yet

int64_t fault_at() {
  int64_t v = g_fault_at.load(std::memory_order_acquire);
  if (v == -2) {
    int64_t e = 0;
    if (const char* s = std::getenv("GBS_FAULT_INJECT")) {
      long long q = 0;
      if (std::sscanf(s, "launch:%lld", &q) == 1 && q > 0) e = q;
    }
    int64_t expect = -2;
    g_fault_at.compare_exchange_strong(expect, e);
    v = g_fault_at.load(std::memory_order_acquire);
  }
  return v;
}

bool check_symmetry_on() {
  int v = g_check_sym.load(std::memory_order_acquire);
  if (v < 0) {
    const char* s = std::getenv("GBS_CHECK_SYMMETRY");
    int expect = -1;
    g_check_sym.compare_exchange_strong(expect, (s && s[0] && s[0] != '0') ? 1 : 0);
    v = g_check_sym.load(std::memory_order_acquire);
  }
  return v > 0;
}

int launch_gate(gbs_ctx* ctx) {
  const int64_t at = fault_at();
  const int64_t k = g_launches.fetch_add(1, std::memory_order_acq_rel) + 1;
  if (at > 0 && k == at) return fail(ctx, GBS_EHIP, "injected launch failure (launch %lld, GBS_FAULT_INJECT)", (long long)k);
  return GBS_OK;
}

struct DeviceGuard {
  int prev = -1;
  explicit DeviceGuard(int dev) {
    if (hipGetDevice(&prev) != hipSuccess) prev = -1;
    if (prev != dev) (void)hipSetDevice(dev);
  }
  ~DeviceGuard() {
    if (prev >= 0) (void)hipSetDevice(prev);
  }
};

// Built-in launch shape per even n: the autotuner's picks (autotune.tune over chunk sizes and engine
// shapes, then one or two streams, haf_batch on random complex-symmetric matrices, one MI355X;
// python -m paper_1908_10070_amd.autotune --table reproduces it). Rows below n = 16 repeat n = 16's
// (a pattern's subsets fit one item either way). {chunk_small, chunk_large, shape, streams}; the
// streams column applies to calls whose patterns all have that n while the caller has not chosen a
// stream count (one stream at n = 18, 20, where two measured 5% and 1-3% slower).
struct ShapeRow {
  int32_t cs, cl, shape, streams;
};
constexpr ShapeRow kDefaultShape[GBS_N_MAX / 2 + 1] = {
    {2048, 128, 0, 2}, {2048, 128, 0, 2},  {2048, 128, 0, 2},  {2048, 128, 0, 2},  {2048, 128, 0, 2},
    {2048, 128, 0, 2}, {2048, 128, 0, 2},  {2048, 128, 0, 2},  {2048, 128, 0, 2},  {256, 16, 1, 1},
    {256, 64, 0, 1},   {512, 128, 2, 2},   {256, 256, 4, 2},   {512, 32, 4, 2},    {512, 128, 4, 2},
    {256, 256, 4, 2},  {256, 128, 20, 2},  {256, 128, 20, 2},  {256, 128, 20, 2},  {256, 128, 20, 2},
    {256, 128, 20, 2}, {128, 128, 20, 2},  {1024, 128, 20, 2}, {128, 128, 20, 2},
};

void default_chunks(int n, int64_t* cs, int64_t* cl) {
  const ShapeRow& r = kDefaultShape[(n < 0 ? 0 : (n > GBS_N_MAX ? GBS_N_MAX : n)) / 2];
  *cs = r.cs;
  *cl = r.cl;
}

void chunks_for(const gbs_ctx* ctx, int n, int64_t* cs, int64_t* cl) {
  default_chunks(n, cs, cl);
  auto it = ctx->tuning.find(n);
  if (it != ctx->tuning.end()) {
    if (it->second.first > 0) *cs = it->second.first;
    if (it->second.second > 0) *cl = it->second.second;
  }
}

// Engine shape bits for size-n patterns: the caller's (autotuner's) choice, else the built-in table.
int default_shape(int n) { return kDefaultShape[(n < 0 ? 0 : (n > GBS_N_MAX ? GBS_N_MAX : n)) / 2].shape; }
int default_streams(int n) { return kDefaultShape[(n < 0 ? 0 : (n > GBS_N_MAX ? GBS_N_MAX : n)) / 2].streams; }

int shape_for(const gbs_ctx* ctx, int n) {
  auto it = ctx->shape.find(n);
  return it != ctx->shape.end() ? it->second : default_shape(n);
}

// Host-side plan of one call, laid out exactly as it is copied into the device workspace.

std::vector<ClassRun> class_runs(const gbs_ctx* ctx, int n, int64_t lo, int64_t hi) {
  std::vector<ClassRun> out;
  const int k = n / 2;
  int64_t cs, cl;
  chunks_for(ctx, n, &cs, &cl);
  const bool dd = ctx->precision == kPrecDd;
  const int shape = shape_for(ctx, n);
  auto cls_of = [&](int s) { return dd ? engine_class_dd(s) : engine_class(s, k, shape); };
  for (int s_lo = 1; s_lo <= k;) {
    const int cls = cls_of(s_lo);
    int s_hi = s_lo;
    while (s_hi + 1 <= k && cls_of(s_hi + 1) == cls) ++s_hi;
    const int64_t a = std::max(lo, size_start(k, s_lo));
    const int64_t b = std::min(hi, size_start(k, s_hi + 1));
    // double-double items: kDdChunk subsets (a subset there costs ~30 FP64 ones)
    if (a < b) out.push_back(ClassRun{cls, a, b, dd ? kDdChunk : (s_hi <= 8 ? cs : cl)});
    s_lo = s_hi + 1;
  }
  return out;
}

// Split [lo, hi) of pattern p into items: the class runs cut into chunks; partial indices follow
// the runs in increasing |Z|. The runs of a whole pattern depend only on n and are kept per call in
// L.full_runs.
void plan_range(const gbs_ctx* ctx, Plan& pl, ItemLists& L, int p, int n, int64_t lo, int64_t hi) {
  if (hi <= lo) return;
  std::vector<ClassRun> part;
  const std::vector<ClassRun>* runs = &part;
  if (lo == 0 && hi == subset_count(n)) {
    if (!L.have_full[n]) {
      L.full_runs[n] = class_runs(ctx, n, lo, hi);
      L.have_full[n] = true;
    }
    runs = &L.full_runs[n];
  } else {
    part = class_runs(ctx, n, lo, hi);
  }
  for (const ClassRun& r : *runs) {
    std::vector<WorkItem>& out = L.cls[r.cls];
    for (int64_t x = r.a; x < r.b; x += r.chunk) {
      WorkItem w;
      w.lo = x;
      w.hi = std::min(r.b, x + r.chunk);
      w.pattern = p;
      w.partial = (int32_t)pl.n_partials++;
      out.push_back(w);
    }
  }
  pl.nmax = std::max(pl.nmax, n);
  pl.nmin = std::min(pl.nmin, n);
  pl.kmax = std::max(pl.kmax, n / 2);
}

// Item order: launches with the biggest tiles first; within a launch larger n first, so long items
// start early.
void order_items(Plan& pl, ItemLists& L) {
  pl.items.clear();
  pl.groups.clear();
  for (int cls = kEngineClasses - 1; cls >= 0; --cls) {
    const std::vector<WorkItem>& v = L.cls[cls];
    if (v.empty()) continue;
    // stable order by decreasing n: a counting pass over the (at most GBS_N_MAX + 1) sizes; a list of
    // one size is already in that order and is copied as it is
    int64_t count[GBS_N_MAX + 2] = {};
    bool one_size = pl.nmin == pl.nmax;
    if (!one_size) {
      for (const WorkItem& w : v) ++count[GBS_N_MAX - pl.pats[w.pattern].n + 1];
      one_size = count[GBS_N_MAX - pl.pats[v[0].pattern].n + 1] == (int64_t)v.size();
      for (int q = 1; q <= GBS_N_MAX + 1; ++q) count[q] += count[q - 1];
    }
    Plan::Group g;
    g.cls = cls;
    g.first = (int64_t)pl.items.size();
    g.count = (int64_t)v.size();
    pl.items.resize(pl.items.size() + v.size());
    WorkItem* dst = pl.items.data() + g.first;
    if (one_size)
      std::copy(v.begin(), v.end(), dst);
    else
      for (const WorkItem& w : v) dst[count[GBS_N_MAX - pl.pats[w.pattern].n]++] = w;
    g.n = pl.pats[dst[0].pattern].n;
    pl.groups.push_back(g);
  }
}

struct Layout {
  size_t counter, modes, pats, items, part_off, nvec, sfact, out_idx, partials, check, total, staged_bytes;
};

size_t al(size_t x) { return (x + 255) & ~size_t(255); }

Layout layout_for(const Plan& pl, size_t n_modes) {
  Layout L;
  size_t off = 0;
  L.counter = off;
  off += al(sizeof(int32_t) * std::max<size_t>(pl.groups.size(), 1));  // one work counter per engine launch
  const size_t stage_begin = off;
  L.modes = off;
  off += al(sizeof(int32_t) * n_modes);
  L.pats = off;
  off += al(sizeof(PatternDesc) * pl.pats.size());
  L.items = off;
  off += al(sizeof(WorkItem) * pl.items.size());
  L.part_off = off;
  off += al(sizeof(int64_t) * pl.part_off.size());
  L.nvec = off;
  off += al(sizeof(int32_t) * pl.nvec.size());
  L.sfact = off;
  off += al(sizeof(double) * pl.sfact.size());
  L.out_idx = off;
  off += al(sizeof(int64_t) * pl.out_idx.size());
  L.staged_bytes = off - stage_begin;
  L.partials = off;
  off += al(sizeof(gbs_partial) * (size_t)pl.n_partials);
  L.check = off;  // per-pattern flags of the debug symmetry check (only when it is on)
  if (check_symmetry_on()) off += al(sizeof(int32_t) * pl.pats.size());
  L.total = off;
  return L;
}

int ensure_ws(gbs_ctx* ctx, size_t bytes) {
  if (ctx->ws && ctx->ws_bytes >= bytes) return GBS_OK;
  ctx->ws_needed = bytes;
  return fail(ctx, GBS_ENOMEM, "workspace of %zu bytes is smaller than the %zu the call needs", ctx->ws_bytes, bytes);
}

// A pinned staging buffer of at least `bytes` for this call (index in *out): the next one in the
// ring, after its previous copy has run.
int acquire_pin(gbs_ctx* ctx, size_t bytes, int* out) {
  if (ctx->pinned_bytes < bytes) {
    // grow every buffer together (once their copies have run): 2x headroom, at least 1 MiB
    const size_t nb = std::max(std::max(bytes, ctx->pinned_bytes) * 2, size_t(1) << 20);
    for (int i = 0; i < gbs_ctx::kPinRing; ++i) {
      if (ctx->pinned_used[i]) HIPCHK(ctx, hipEventSynchronize(ctx->pinned_ev[i]));
      if (ctx->pinned[i]) (void)hipHostFree(ctx->pinned[i]);
      ctx->pinned[i] = nullptr;
    }
    ctx->pinned_bytes = 0;
    for (int i = 0; i < gbs_ctx::kPinRing; ++i)
      HIPCHK(ctx, hipHostMalloc(&ctx->pinned[i], nb, hipHostMallocDefault));
    ctx->pinned_bytes = nb;
  }
  const int pi = ctx->pin_idx;
  ctx->pin_idx = (pi + 1) % gbs_ctx::kPinRing;
  if (ctx->pinned_used[pi]) HIPCHK(ctx, hipEventSynchronize(ctx->pinned_ev[pi]));
  *out = pi;
  return GBS_OK;
}

// One engine launch: its variant, arguments, grid and LDS bytes.
struct Launch {
  int cls;
  EngineArgs a;
  int grid;
  size_t lds;
};

// Launches for the plan's groups; ea holds the arguments common to all of them.
int build_launches(gbs_ctx* ctx, const std::vector<Plan::Group>& groups, const EngineArgs& ea, const WorkItem* items,
                   int32_t* counters, int persistent, std::vector<Launch>& launches) {
  for (size_t gi = 0; gi < groups.size(); ++gi) {
    const Plan::Group& g = groups[gi];
    Launch ln;
    ln.cls = g.cls;
    ln.a = ea;
    ln.a.persistent = persistent;
    ln.a.n_items = (int32_t)g.count;
    ln.a.items = items + g.first;
    ln.a.counter = counters + gi;
    // every item of a variant has the same n: LDS sized for that n only (staged copy for n <= 32)
    ln.a.nmax = std::max(g.n, 2);
    ln.a.kmax = std::max(g.n / 2, 1);
    ln.a.stage_A = g.n <= 32 ? 1 : 0;
    ln.lds = engine_lds_bytes(g.cls, ln.a.nmax, ln.a.kmax, ln.a.stage_A);
    if (ln.lds > kLdsBudget) return fail(ctx, GBS_EUNSUPPORTED, "plan needs %zu bytes of LDS", ln.lds);
    const int per_cu = engine_blocks_per_cu(g.cls, ln.lds);
    ln.grid = (int)g.count;
    if (persistent) ln.grid = (int)std::min<int64_t>(g.count, (int64_t)ctx->ncu * per_cu);
    launches.push_back(ln);
  }
  return GBS_OK;
}

// Copy the staged part of the plan to the device, launch the engine and the finalize kernel.
int run_plan(gbs_ctx* ctx, const Plan& pl, const int32_t* modes_host, size_t n_modes, const double2* A,
             int32_t m, const double* prefactor_dev, double* prob_out, double2* haf_out, gbs_partial* partial_out,
             hipStream_t stream) {
  DeviceGuard dg(ctx->device);
  if (const int g = launch_gate(ctx)) return g;
  const Layout L = layout_for(pl, n_modes);
  int rc = ensure_ws(ctx, L.total);
  if (rc) return rc;
  // stage into a free pinned buffer
  int pi = 0;
  rc = acquire_pin(ctx, L.staged_bytes, &pi);
  if (rc) return rc;
  unsigned char* h = static_cast<unsigned char*>(ctx->pinned[pi]);
  const size_t base = L.modes;
  if (n_modes) std::memcpy(h + (L.modes - base), modes_host, sizeof(int32_t) * n_modes);
  if (!pl.pats.empty()) std::memcpy(h + (L.pats - base), pl.pats.data(), sizeof(PatternDesc) * pl.pats.size());
  if (!pl.items.empty()) std::memcpy(h + (L.items - base), pl.items.data(), sizeof(WorkItem) * pl.items.size());
  std::memcpy(h + (L.part_off - base), pl.part_off.data(), sizeof(int64_t) * pl.part_off.size());
  if (!pl.nvec.empty()) std::memcpy(h + (L.nvec - base), pl.nvec.data(), sizeof(int32_t) * pl.nvec.size());
  if (!pl.sfact.empty()) std::memcpy(h + (L.sfact - base), pl.sfact.data(), sizeof(double) * pl.sfact.size());
  if (!pl.out_idx.empty())
    std::memcpy(h + (L.out_idx - base), pl.out_idx.data(), sizeof(int64_t) * pl.out_idx.size());

  unsigned char* ws = static_cast<unsigned char*>(ctx->ws);
  if (ctx->done_recorded) HIPCHK(ctx, hipStreamWaitEvent(stream, ctx->done_ev, 0));
  HIPCHK(ctx, hipMemcpyAsync(ws + base, h, L.staged_bytes, hipMemcpyHostToDevice, stream));
  HIPCHK(ctx, hipEventRecord(ctx->pinned_ev[pi], stream));
  ctx->pinned_used[pi] = true;

  // debug: caller-provided matrices must be symmetric (checked before anything else runs on them)
  if (A && !modes_host && check_symmetry_on() && !pl.pats.empty()) {
    int32_t* flags = reinterpret_cast<int32_t*>(ws + L.check);
    launch_sym_check(A, reinterpret_cast<const PatternDesc*>(ws + L.pats), (int64_t)pl.pats.size(), 1e-12, flags,
                     stream);
    std::vector<int32_t> hf(pl.pats.size());
    HIPCHK(ctx, hipMemcpyAsync(hf.data(), flags, sizeof(int32_t) * hf.size(), hipMemcpyDeviceToHost, stream));
    HIPCHK(ctx, hipStreamSynchronize(stream));
    for (size_t b = 0; b < hf.size(); ++b)
      if (hf[b])
        return fail(ctx, GBS_EINVAL, "matrix %zu is not symmetric (|A_ij - A_ji| > 1e-12 max|A|; GBS_CHECK_SYMMETRY)", b);
  }

  // one persistent launch per engine variant, each with its own item list and work counter
  EngineArgs ea{};
  ea.A = A;
  ea.modes = modes_host ? reinterpret_cast<const int32_t*>(ws + L.modes) : nullptr;
  ea.m = m;
  ea.pats = reinterpret_cast<const PatternDesc*>(ws + L.pats);
  ea.partials = reinterpret_cast<gbs_partial*>(ws + L.partials);
  ea.persistent = ctx->persistent;

  std::vector<Launch> launches;
  int32_t* counters = reinterpret_cast<int32_t*>(ws + L.counter);
  rc = build_launches(ctx, pl.groups, ea, reinterpret_cast<const WorkItem*>(ws + L.items), counters, ctx->persistent,
                      launches);
  if (rc) return rc;

  FinalizeArgs fa{};
  fa.partials = ea.partials;
  fa.part_lo = reinterpret_cast<const int64_t*>(ws + L.part_off);
  fa.part_hi = fa.part_lo + 1;
  fa.n = reinterpret_cast<const int32_t*>(ws + L.nvec);
  fa.sfact = reinterpret_cast<const double*>(ws + L.sfact);
  fa.prefactor = prefactor_dev;
  fa.batch = (int64_t)pl.part_off.size() - 1;
  fa.prob_out = prob_out;
  fa.haf_out = haf_out;
  fa.partial_out = partial_out;
  fa.out_idx = pl.out_idx.empty() ? nullptr : reinterpret_cast<const int64_t*>(ws + L.out_idx);

  // With several streams the engine kernels go round-robin to the auxiliary streams, forked from s
  // after the staging copy and the counter reset and joined back before the finalize kernel. Under
  // graph capture the fork and join become graph edges, so a replay runs the kernels side by side.
  // (a call on patterns of one size n, on a context whose stream count the caller has not set, takes
  // the built-in count for n; default_streams never exceeds the kDefaultStreams created with it)
  const int want = ctx->streams_auto && pl.nmin == pl.nmax ? std::min(default_streams(pl.nmin), ctx->nstreams)
                                                           : ctx->nstreams;
  const int ns = want > 1 ? (int)std::min<size_t>((size_t)want, launches.size()) : 1;
  auto enqueue = [&](hipStream_t s) -> hipError_t {
    if (ctx->persistent && !launches.empty()) launch_reset(counters, (int)launches.size(), s);
    if (ns > 1) {
      hipError_t e = hipEventRecord(ctx->fork_ev, s);
      for (int j = 0; j < ns && e == hipSuccess; ++j) e = hipStreamWaitEvent(ctx->aux[j], ctx->fork_ev, 0);
      if (e != hipSuccess) return e;
      for (size_t i = 0; i < launches.size(); ++i) {
        const Launch& ln = launches[i];
        launch_engine(ln.cls, ln.a, ln.grid, ln.lds, ctx->aux[i % ns]);
      }
      for (int j = 0; j < ns && e == hipSuccess; ++j) {
        e = hipEventRecord(ctx->aux_ev[j], ctx->aux[j]);
        if (e == hipSuccess) e = hipStreamWaitEvent(s, ctx->aux_ev[j], 0);
      }
      if (e != hipSuccess) return e;
    } else {
      for (const Launch& ln : launches) launch_engine(ln.cls, ln.a, ln.grid, ln.lds, s);
    }
    if (fa.batch > 0) launch_finalize(fa, s);
    return hipGetLastError();
  };

  if (ctx->use_graph) {
    GraphKey key;
    key.v = {ea.persistent, (int64_t)(intptr_t)A,
             (int64_t)(intptr_t)ea.modes, m, fa.batch, (int64_t)(intptr_t)prefactor_dev, (int64_t)(intptr_t)prob_out,
             (int64_t)(intptr_t)haf_out, (int64_t)(intptr_t)partial_out, (int64_t)(intptr_t)ctx->ws, (int64_t)L.pats,
             (int64_t)L.items, (int64_t)L.partials, (int64_t)L.part_off, (int64_t)L.nvec, (int64_t)L.sfact,
             (int64_t)L.out_idx, (int64_t)pl.out_idx.size(), ns};
    for (const Launch& ln : launches) {
      key.v.push_back(ln.cls);
      key.v.push_back(ln.grid);
      key.v.push_back((int64_t)ln.lds);
      key.v.push_back(ln.a.n_items);
      key.v.push_back(ln.a.nmax);
    }
    hipGraphExec_t exec = nullptr;
    for (auto itg = ctx->graphs.begin(); itg != ctx->graphs.end(); ++itg)
      if (!(itg->first < key) && !(key < itg->first)) {
        exec = itg->second;
        ctx->graphs.splice(ctx->graphs.begin(), ctx->graphs, itg);
        break;
      }
    if (!exec) {
      hipGraph_t g = nullptr;
      HIPCHK(ctx, hipStreamBeginCapture(ctx->cap_stream, hipStreamCaptureModeThreadLocal));
      hipError_t ce = enqueue(ctx->cap_stream);
      hipError_t ee = hipStreamEndCapture(ctx->cap_stream, &g);
      if (ce != hipSuccess || ee != hipSuccess) {
        if (g) (void)hipGraphDestroy(g);
        return fail(ctx, GBS_EHIP, "graph capture: %s", hipGetErrorString(ce != hipSuccess ? ce : ee));
      }
      hipError_t e = hipGraphInstantiate(&exec, g, nullptr, nullptr, 0);
      (void)hipGraphDestroy(g);
      if (e != hipSuccess) return fail(ctx, GBS_EHIP, "hipGraphInstantiate: %s", hipGetErrorString(e));
      ctx->graphs.emplace_front(key, exec);
      while (ctx->graphs.size() > 16) {
        (void)hipGraphExecDestroy(ctx->graphs.back().second);
        ctx->graphs.pop_back();
      }
    }
    HIPCHK(ctx, hipGraphLaunch(exec, stream));
  } else {
    HIPCHK(ctx, enqueue(stream));
  }
  HIPCHK(ctx, hipEventRecord(ctx->done_ev, stream));
  ctx->done_recorded = true;
  return GBS_OK;
}

bool check_gfx950(int device) {
  hipDeviceProp_t p;
  if (hipGetDeviceProperties(&p, device) != hipSuccess) return false;
  return std::strncmp(p.gcnArchName, "gfx950", 6) == 0;
}

// Validate one mode list and compute prod_j s_j! (collision multiplicities, Eq. ProOri).
int pattern_sfact(gbs_ctx* ctx, const int32_t* modes, int64_t len, int32_t m, double* sfact) {
  int32_t tmp[GBS_N_MAX];
  bool sorted = true;
  for (int64_t i = 0; i < len; ++i) {
    if (modes[i] < 0 || modes[i] >= m) return fail(ctx, GBS_ERANGE, "mode %d outside [0, %d)", modes[i], m);
    tmp[i] = modes[i];
    sorted = sorted && (i == 0 || tmp[i - 1] <= tmp[i]);
  }
  if (!sorted) std::sort(tmp, tmp + len);  // mode lists usually come sorted
  double f = 1.0;
  int64_t run = 1;
  for (int64_t i = 1; i <= len; ++i) {
    if (i < len && tmp[i] == tmp[i - 1]) {
      ++run;
      f *= (double)run;
    } else {
      run = 1;
    }
  }
  *sfact = f;
  return GBS_OK;
}

}  // namespace

// =================================================================== C ABI

namespace {

// log of the generalized binomial Gamma(a + 1) / (Gamma(b + 1) Gamma(a - b + 1)) for a + 1 > 0 and
// b + 1 > 0; -inf when a - b is a negative integer (the binomial is zero there).
double log_gbinom_pos(double a, double b) {
  const double d = a - b;
  if (d < 0 && d == std::floor(d)) return -INFINITY;
  return std::lgamma(a + 1) - std::lgamma(b + 1) - std::lgamma(d + 1);
}

// Theorem 1 weight F = (n - k)! / f_n * C((n - k + mu + m)/2 - 1, k - j1 - j2 + m/2 - 1), with
// f_n = n! C((m + n)/2 - 1, n/2); zero outside the theorem's ranges of j1, j2 and mu.
double theorem1_weight(int m, int n, int k, int mu, int j1, int j2) {
  const int jlo = std::max(0, k - n / 2);
  if (j1 < jlo || j2 < jlo || 2 * j1 > k || 2 * j2 > k) return 0.0;
  const int mu_lo = std::max(0, 3 * k - 2 * (j1 + j2) - n), mu_hi = k - 2 * std::max(j1, j2);
  if (mu < mu_lo || mu > mu_hi || ((mu - k) & 1)) return 0.0;
  const double lf = std::lgamma(n + 1.0) + log_gbinom_pos((m + n) / 2.0 - 1.0, n / 2.0);
  const double lc = log_gbinom_pos((n - k + mu + m) / 2.0 - 1.0, k - j1 - j2 + m / 2.0 - 1.0);
  if (std::isinf(lc)) return 0.0;
  return std::exp(std::lgamma(n - k + 1.0) - lf + lc);
}

}  // namespace


extern "C" {

const char* gbs_status_str(int status) {
  switch (status) {
    case GBS_OK: return "ok";
    case GBS_EINVAL: return "invalid argument";
    case GBS_ERANGE: return "value out of range";
    case GBS_ENOMEM: return "out of memory";
    case GBS_EHIP: return "HIP runtime error";
    case GBS_EUNSUPPORTED: return "unsupported";
    default: return "unknown status";
  }
}

const char* gbs_last_error(const gbs_ctx* ctx) { return ctx ? ctx->last_error.c_str() : ""; }

int gbs_ctx_create(int device, void* workspace_dev, size_t workspace_bytes, gbs_ctx** out) {
  if (!out) return GBS_EINVAL;
  *out = nullptr;
  if (workspace_dev == nullptr && workspace_bytes != 0) return GBS_EINVAL;
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || device < 0 || device >= ndev) return GBS_EINVAL;
  if (!check_gfx950(device)) return GBS_EUNSUPPORTED;
  DeviceGuard dg(device);
  gbs_ctx* c = new gbs_ctx();
  c->device = device;
  hipDeviceProp_t p;
  if (hipGetDeviceProperties(&p, device) != hipSuccess) {
    delete c;
    return GBS_EHIP;
  }
  c->ncu = p.multiProcessorCount;
  // device address of the no-allocation entry point's scratch on this device (device current)
  hipError_t se = hipSuccess;
  if (!noalloc_scratch(device, &se)) {
    delete c;
    return GBS_EHIP;
  }
  bool ev_ok = true;
  for (int i = 0; i < gbs_ctx::kPinRing; ++i)
    ev_ok = ev_ok && hipEventCreateWithFlags(&c->pinned_ev[i], hipEventDisableTiming) == hipSuccess;
  if (!ev_ok ||
      hipEventCreateWithFlags(&c->done_ev, hipEventDisableTiming) != hipSuccess ||
      hipStreamCreateWithFlags(&c->cap_stream, hipStreamNonBlocking) != hipSuccess) {
    gbs_ctx_destroy(c);
    return GBS_EHIP;
  }
  if (gbs_ctx_set_streams(c, gbs_ctx::kDefaultStreams) != GBS_OK) {
    gbs_ctx_destroy(c);
    return GBS_EHIP;
  }
  c->streams_auto = true;  // the default, not a caller's choice
  c->ws = workspace_dev;
  c->ws_bytes = workspace_dev ? workspace_bytes : 0;
  *out = c;
  return GBS_OK;
}

int gbs_ctx_destroy(gbs_ctx* c) {
  if (!c) return GBS_EINVAL;
  DeviceGuard dg(c->device);
  (void)hipDeviceSynchronize();
  for (auto& g : c->graphs) (void)hipGraphExecDestroy(g.second);
  for (int i = 0; i < gbs_ctx::kPinRing; ++i) {
    if (c->pinned[i]) (void)hipHostFree(c->pinned[i]);
    if (c->pinned_ev[i]) (void)hipEventDestroy(c->pinned_ev[i]);
  }
  if (c->done_ev) (void)hipEventDestroy(c->done_ev);
  if (c->cap_stream) (void)hipStreamDestroy(c->cap_stream);
  for (int i = 0; i < gbs_ctx::kMaxStreams; ++i) {
    if (c->aux[i]) (void)hipStreamDestroy(c->aux[i]);
    if (c->aux_ev[i]) (void)hipEventDestroy(c->aux_ev[i]);
  }
  if (c->fork_ev) (void)hipEventDestroy(c->fork_ev);
  delete c;
  return GBS_OK;
}

int gbs_ctx_set_workspace(gbs_ctx* ctx, void* workspace_dev, size_t workspace_bytes) {
  if (!ctx) return GBS_EINVAL;
  ctx->last_error.clear();
  if (workspace_dev == nullptr && workspace_bytes != 0) return fail(ctx, GBS_EINVAL, "null workspace");
  DeviceGuard dg(ctx->device);
  if (ctx->done_recorded) HIPCHK(ctx, hipEventSynchronize(ctx->done_ev));
  for (auto& g : ctx->graphs) (void)hipGraphExecDestroy(g.second);
  ctx->graphs.clear();
  ctx->ws = workspace_dev;
  ctx->ws_bytes = workspace_dev ? workspace_bytes : 0;
  return GBS_OK;
}

size_t gbs_ctx_workspace_needed(const gbs_ctx* ctx) { return ctx ? ctx->ws_needed : 0; }

int gbs_ctx_set_exec(gbs_ctx* ctx, int use_graph, int persistent) {
  if (!ctx) return GBS_EINVAL;
  ctx->use_graph = use_graph ? 1 : 0;
  ctx->persistent = persistent ? 1 : 0;
  return GBS_OK;
}

int gbs_debug_fault_inject(int64_t launch_n) {
  g_fault_at.store(launch_n > 0 ? launch_n : 0, std::memory_order_release);
  g_launches.store(0, std::memory_order_release);
  return GBS_OK;
}

int gbs_debug_check_symmetry(int32_t on) {
  g_check_sym.store(on ? 1 : 0, std::memory_order_release);
  return GBS_OK;
}

int gbs_ctx_set_precision(gbs_ctx* ctx, int32_t precision) {
  if (!ctx) return GBS_EINVAL;
  ctx->last_error.clear();
  if (precision != GBS_PREC_FP64 && precision != GBS_PREC_DD)
    return fail(ctx, GBS_EINVAL, "precision %d is neither GBS_PREC_FP64 nor GBS_PREC_DD", precision);
  ctx->precision = precision == GBS_PREC_DD ? kPrecDd : kPrecFp64;
  return GBS_OK;
}

int32_t gbs_ctx_get_precision(const gbs_ctx* ctx) {
  return (ctx && ctx->precision == kPrecDd) ? GBS_PREC_DD : GBS_PREC_FP64;
}

int gbs_ctx_set_streams(gbs_ctx* ctx, int32_t nstreams) {
  if (!ctx) return GBS_EINVAL;
  ctx->last_error.clear();
  if (nstreams < 1 || nstreams > gbs_ctx::kMaxStreams)
    return fail(ctx, GBS_EINVAL, "nstreams = %d outside [1, %d]", nstreams, gbs_ctx::kMaxStreams);
  DeviceGuard dg(ctx->device);
  if (!ctx->fork_ev) HIPCHK(ctx, hipEventCreateWithFlags(&ctx->fork_ev, hipEventDisableTiming));
  for (int i = 0; i < nstreams; ++i) {
    if (!ctx->aux[i]) HIPCHK(ctx, hipStreamCreateWithFlags(&ctx->aux[i], hipStreamNonBlocking));
    if (!ctx->aux_ev[i]) HIPCHK(ctx, hipEventCreateWithFlags(&ctx->aux_ev[i], hipEventDisableTiming));
  }
  ctx->nstreams = nstreams;
  ctx->streams_auto = false;
  return GBS_OK;
}

int gbs_ctx_get_streams(const gbs_ctx* ctx, int32_t* nstreams) {
  if (!ctx || !nstreams) return GBS_EINVAL;
  *nstreams = ctx->nstreams;
  return GBS_OK;
}

int gbs_ctx_set_tuning(gbs_ctx* ctx, int32_t n, int64_t chunk_small, int64_t chunk_large) {
  if (!ctx) return GBS_EINVAL;
  if (n < 0 || n > GBS_N_MAX) return fail(ctx, GBS_ERANGE, "n = %d outside [0, %d]", n, GBS_N_MAX);
  ctx->tuning[n] = {chunk_small, chunk_large};
  return GBS_OK;
}

int gbs_ctx_set_shape(gbs_ctx* ctx, int32_t n, int32_t shape) {
  if (!ctx) return GBS_EINVAL;
  ctx->last_error.clear();
  if (n < 0 || n > GBS_N_MAX) return fail(ctx, GBS_ERANGE, "n = %d outside [0, %d]", n, GBS_N_MAX);
  if (shape == -1) {
    ctx->shape.erase(n);
    return GBS_OK;
  }
  if (shape & ~kShapeMask) return fail(ctx, GBS_EINVAL, "unknown engine shape bits 0x%x", shape);
  ctx->shape[n] = shape;
  return GBS_OK;
}

int gbs_ctx_get_shape(const gbs_ctx* ctx, int32_t n, int32_t* shape) {
  if (!ctx || !shape) return GBS_EINVAL;
  if (n < 0 || n > GBS_N_MAX) return GBS_ERANGE;
  *shape = shape_for(ctx, n);
  return GBS_OK;
}

int gbs_ctx_get_tuning(const gbs_ctx* ctx, int32_t n, int64_t* chunk_small, int64_t* chunk_large) {
  if (!ctx || !chunk_small || !chunk_large) return GBS_EINVAL;
  if (n < 0 || n > GBS_N_MAX) return GBS_ERANGE;
  chunks_for(ctx, n, chunk_small, chunk_large);
  return GBS_OK;
}

int64_t gbs_subset_count(int32_t n) { return (n < 0 || n > GBS_N_MAX) ? 0 : subset_count(n); }

double gbs_haf_flops(int32_t n) {
  if (n <= 0 || (n & 1) || n > GBS_N_MAX) return 0.0;
  const int k = n / 2;
  double f = 0.0;
  // the method as formulated: every subset forms all k traces with the chain program for k
  for (int s = 1; s <= k; ++s) f += (double)kBinom.v[k][s] * flops_subset(kChainTable[k], k, s);
  return f;
}

int haf_batch_varlen(gbs_ctx* ctx, const gbs_c128* A_dev, const int64_t* elem_off_host, const int32_t* n_host,
                     int64_t batch, gbs_c128* haf_out_dev, void* stream) {
  if (!ctx) return GBS_EINVAL;
  ctx->last_error.clear();
  if (batch < 0) return fail(ctx, GBS_EINVAL, "batch < 0");
  if (batch == 0) return GBS_OK;
  if (!elem_off_host || !n_host || !haf_out_dev) return fail(ctx, GBS_EINVAL, "null pointer");
  bool any_data = false;
  for (int64_t b = 0; b < batch && !any_data; ++b) any_data = n_host[b] > 0;
  if (any_data && !A_dev) return fail(ctx, GBS_EINVAL, "null matrix pointer");
  if (batch > (int64_t)1 << 30) return fail(ctx, GBS_ERANGE, "batch too large");
  Plan& pl = ctx->plan;
  ItemLists& lists = ctx->lists;
  plan_reset(pl, lists);
  pl.pats.resize(batch);
  pl.part_off.resize(batch + 1);
  pl.nvec.resize(batch);
  pl.sfact.assign(batch, 1.0);
  pl.part_off[0] = 0;
  for (int64_t b = 0; b < batch; ++b) {
    const int n = n_host[b];
    if (n < 0 || n > GBS_N_MAX) return fail(ctx, GBS_ERANGE, "n = %d outside [0, %d]", n, GBS_N_MAX);
    if (elem_off_host[b] < 0) return fail(ctx, GBS_EINVAL, "negative matrix offset");
    pl.pats[b] = PatternDesc{elem_off_host[b], n, 0};
    pl.nvec[b] = n;
    plan_range(ctx, pl, lists, (int)b, n, 0, subset_count(n));
    pl.part_off[b + 1] = pl.n_partials;
  }
  order_items(pl, lists);
  return run_plan(ctx, pl, nullptr, 0, reinterpret_cast<const double2*>(A_dev), 0, nullptr, nullptr,
                  reinterpret_cast<double2*>(haf_out_dev), nullptr, static_cast<hipStream_t>(stream));
}

int haf_batch(gbs_ctx* ctx, const gbs_c128* A_dev, int32_t n, int64_t batch, int64_t stride_elems,
              gbs_c128* haf_out_dev, void* stream) {
  if (!ctx) return GBS_EINVAL;
  ctx->last_error.clear();
  if (batch < 0) return fail(ctx, GBS_EINVAL, "batch < 0");
  if (n < 0 || n > GBS_N_MAX) return fail(ctx, GBS_ERANGE, "n = %d outside [0, %d]", n, GBS_N_MAX);
  if (batch > 1 && stride_elems < (int64_t)n * n) return fail(ctx, GBS_EINVAL, "stride smaller than n*n");
  if (batch == 0) return GBS_OK;
  std::vector<int64_t> off(batch);
  std::vector<int32_t> nn(batch, n);
  for (int64_t b = 0; b < batch; ++b) off[b] = b * stride_elems;
  return haf_batch_varlen(ctx, A_dev, off.data(), nn.data(), batch, haf_out_dev, stream);
}

namespace {

struct StateLayout {
  size_t B, W, r, pref, total;
};

StateLayout state_layout(int m) {
  StateLayout L;
  const size_t mm = (size_t)m * m;
  size_t off = 0;
  L.B = off;
  off += al(sizeof(double2) * mm);
  L.W = off;
  off += al(sizeof(double2) * mm);
  L.r = off;
  off += al(sizeof(double) * m);
  L.pref = off;
  off += al(sizeof(double));
  L.total = off;
  return L;
}

}  // namespace

size_t gbs_state_bytes(int32_t m) {
  if (m <= 0 || m > 4096) return 0;
  return state_layout(m).total;
}

int haf_batch_noalloc(gbs_ctx* ctx, const gbs_c128* A_dev, int32_t n, int64_t batch, int64_t stride_elems,
                      gbs_c128* haf_out_dev, void* stream) {
  if (!ctx) return GBS_EINVAL;
  ctx->last_error.clear();
  if (batch < 0) return fail(ctx, GBS_EINVAL, "batch < 0");
  if (n < 0 || n > GBS_N_MAX) return fail(ctx, GBS_ERANGE, "n = %d outside [0, %d]", n, GBS_N_MAX);
  if (batch > 1 && stride_elems < (int64_t)n * n) return fail(ctx, GBS_EINVAL, "stride smaller than n*n");
  if (batch == 0) return GBS_OK;
  if (!haf_out_dev || (n > 0 && !A_dev)) return fail(ctx, GBS_EINVAL, "null pointer");
  if (batch > (int64_t)1 << 30) return fail(ctx, GBS_ERANGE, "batch too large");
  DeviceGuard dg(ctx->device);
  if (const int g = launch_gate(ctx)) return g;
  hipError_t se = hipSuccess;
  unsigned char* scr = static_cast<unsigned char*>(noalloc_scratch(ctx->device, &se));
  if (!scr) return fail(ctx, GBS_EHIP, "scratch address: %s", hipGetErrorString(se));
  hipStream_t s = static_cast<hipStream_t>(stream);

  // the per-pattern template: one launch per class run, in the order run_plan uses (largest class
  // first), partial indices in increasing |Z| as plan_range assigns them
  const std::vector<ClassRun> runs = (n > 0 && n % 2 == 0) ? class_runs(ctx, n, 0, subset_count(n))
                                                           : std::vector<ClassRun>();
  NoallocPlanArgs na{};
  std::vector<int32_t> local_base(runs.size());
  int32_t ipp = 0;
  for (size_t r = 0; r < runs.size(); ++r) {
    local_base[r] = ipp;
    ipp += (int32_t)((runs[r].b - runs[r].a + runs[r].chunk - 1) / runs[r].chunk);
  }
  if (runs.size() > (size_t)kNoallocMaxGroups) return fail(ctx, GBS_EUNSUPPORTED, "too many engine launches");
  std::vector<Plan::Group> groups;
  int64_t first = 0;
  for (size_t q = runs.size(); q-- > 0;) {  // classes increase with |Z|: largest first
    const ClassRun& r = runs[q];
    NoallocGroup& G = na.g[groups.size()];
    G.first = first;
    G.a = r.a;
    G.b = r.b;
    G.chunk = r.chunk;
    G.count = (int32_t)((r.b - r.a + r.chunk - 1) / r.chunk);
    G.local_base = local_base[q];
    Plan::Group pg;
    pg.cls = r.cls;
    pg.n = n;
    pg.first = first;
    pg.count = batch * G.count;
    groups.push_back(pg);
    first += pg.count;
  }
  na.n_groups = (int32_t)groups.size();
  na.n = n;
  na.ipp = ipp;
  na.batch = batch;
  na.stride = stride_elems;
  na.total_items = first;
  if (first > INT32_MAX || batch * (int64_t)ipp > INT32_MAX)
    return fail(ctx, GBS_ERANGE, "batch too large for the no-allocation path");

  // scratch layout: counters, patterns, items, partial offsets, n, prod s!, partials
  size_t off = 0;
  const size_t o_cnt = off;
  off += al(sizeof(int32_t) * std::max<size_t>(groups.size(), 1));
  const size_t o_pats = off;
  off += al(sizeof(PatternDesc) * (size_t)batch);
  const size_t o_items = off;
  off += al(sizeof(WorkItem) * (size_t)first);
  const size_t o_poff = off;
  off += al(sizeof(int64_t) * (size_t)(batch + 1));
  const size_t o_n = off;
  off += al(sizeof(int32_t) * (size_t)batch);
  const size_t o_sf = off;
  off += al(sizeof(double) * (size_t)batch);
  const size_t o_part = off;
  off += al(sizeof(gbs_partial) * (size_t)(batch * ipp));
  if (off > noalloc_scratch_bytes())
    return fail(ctx, GBS_ENOMEM, "the call needs %zu bytes of the no-allocation scratch, which holds %zu", off,
                noalloc_scratch_bytes());
  na.pats = reinterpret_cast<PatternDesc*>(scr + o_pats);
  na.items = reinterpret_cast<WorkItem*>(scr + o_items);
  na.part_off = reinterpret_cast<int64_t*>(scr + o_poff);
  na.nvec = reinterpret_cast<int32_t*>(scr + o_n);
  na.sfact = reinterpret_cast<double*>(scr + o_sf);

  EngineArgs ea{};
  ea.A = reinterpret_cast<const double2*>(A_dev);
  ea.modes = nullptr;
  ea.m = 0;
  ea.pats = na.pats;
  ea.partials = reinterpret_cast<gbs_partial*>(scr + o_part);
  std::vector<Launch> launches;
  int32_t* counters = reinterpret_cast<int32_t*>(scr + o_cnt);
  int rc = build_launches(ctx, groups, ea, na.items, counters, 1, launches);
  if (rc) return rc;
  FinalizeArgs fa{};
  fa.partials = ea.partials;
  fa.part_lo = na.part_off;
  fa.part_hi = na.part_off + 1;
  fa.n = na.nvec;
  fa.sfact = na.sfact;
  fa.batch = batch;
  fa.haf_out = reinterpret_cast<double2*>(haf_out_dev);

  if (ctx->done_recorded) HIPCHK(ctx, hipStreamWaitEvent(s, ctx->done_ev, 0));
  launch_noalloc_plan(na, s);
  if (!launches.empty()) launch_reset(counters, (int)launches.size(), s);
  for (const Launch& ln : launches) launch_engine(ln.cls, ln.a, ln.grid, ln.lds, s);
  launch_finalize(fa, s);
  HIPCHK(ctx, hipGetLastError());
  HIPCHK(ctx, hipEventRecord(ctx->done_ev, s));
  ctx->done_recorded = true;
  return GBS_OK;
}

int gbs_state_create(gbs_ctx* ctx, const gbs_c128* U_dev, int32_t m, const double* r_host, void* state_mem_dev,
                     size_t state_mem_bytes, void* stream, gbs_state** out) {
  if (!ctx || !out) return GBS_EINVAL;
  *out = nullptr;
  ctx->last_error.clear();
  if (!U_dev || !r_host || !state_mem_dev) return fail(ctx, GBS_EINVAL, "null pointer");
  if (m <= 0 || m > 4096) return fail(ctx, GBS_ERANGE, "m = %d outside [1, 4096]", m);
  for (int i = 0; i < m; ++i)
    if (!std::isfinite(r_host[i])) return fail(ctx, GBS_EINVAL, "non-finite squeezing parameter");
  const StateLayout L = state_layout(m);
  if (state_mem_bytes < L.total)
    return fail(ctx, GBS_ENOMEM, "state memory of %zu bytes is smaller than the %zu needed", state_mem_bytes, L.total);
  DeviceGuard dg(ctx->device);
  hipStream_t s = static_cast<hipStream_t>(stream);
  // r goes through the context's pinned staging ring
  int pi = 0;
  int rc = acquire_pin(ctx, sizeof(double) * m, &pi);
  if (rc) return rc;
  std::memcpy(ctx->pinned[pi], r_host, sizeof(double) * m);
  gbs_state* st = new gbs_state();
  st->device = ctx->device;
  st->m = m;
  unsigned char* mem = static_cast<unsigned char*>(state_mem_dev);
  st->B = reinterpret_cast<double2*>(mem + L.B);
  st->W = reinterpret_cast<double2*>(mem + L.W);
  st->r = reinterpret_cast<double*>(mem + L.r);
  st->pref = reinterpret_cast<double*>(mem + L.pref);
  hipError_t e = hipEventCreateWithFlags(&st->ready, hipEventDisableTiming);
  if (e == hipSuccess && ctx->done_recorded) e = hipStreamWaitEvent(s, ctx->done_ev, 0);
  if (e == hipSuccess) e = hipMemcpyAsync(st->r, ctx->pinned[pi], sizeof(double) * m, hipMemcpyHostToDevice, s);
  if (e == hipSuccess) e = hipEventRecord(ctx->pinned_ev[pi], s);
  if (e == hipSuccess) {
    ctx->pinned_used[pi] = true;
    launch_state(reinterpret_cast<const double2*>(U_dev), st->r, m, st->B, st->W, st->pref, s);
    e = hipGetLastError();
  }
  if (e == hipSuccess) e = hipMemcpyAsync(&st->pref_host, st->pref, sizeof(double), hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipEventRecord(st->ready, s);
  if (e != hipSuccess) {
    gbs_state_destroy(st);
    return fail(ctx, GBS_EHIP, "state setup: %s", hipGetErrorString(e));
  }
  *out = st;
  return GBS_OK;
}

int gbs_state_destroy(gbs_state* st) {
  if (!st) return GBS_EINVAL;
  DeviceGuard dg(st->device);
  if (st->ready) (void)hipEventSynchronize(st->ready);
  if (st->ready) (void)hipEventDestroy(st->ready);
  delete st;
  return GBS_OK;
}

int gbs_state_info(const gbs_state* st, const gbs_c128** B_dev, int32_t* m, double* prefactor) {
  if (!st) return GBS_EINVAL;
  if (B_dev) *B_dev = reinterpret_cast<const gbs_c128*>(st->B);
  if (m) *m = st->m;
  if (prefactor) {
    DeviceGuard dg(st->device);
    if (hipEventSynchronize(st->ready) != hipSuccess) return GBS_EHIP;
    *prefactor = st->pref_host;
  }
  return GBS_OK;
}

int gbs_state_copy_B(const gbs_state* st, gbs_c128* dst_dev, void* stream) {
  if (!st || !dst_dev) return GBS_EINVAL;
  DeviceGuard dg(st->device);
  hipStream_t s = static_cast<hipStream_t>(stream);
  if (hipStreamWaitEvent(s, st->ready, 0) != hipSuccess) return GBS_EHIP;
  if (hipMemcpyAsync(dst_dev, st->B, sizeof(double2) * (size_t)st->m * st->m, hipMemcpyDeviceToDevice, s) != hipSuccess)
    return GBS_EHIP;
  return GBS_OK;
}

namespace {

int prob_common(gbs_ctx* ctx, const gbs_state* st, const int32_t* modes_host, const int64_t* offsets_host,
                int64_t batch, const int64_t* lo_host, const int64_t* hi_host, double* prob_out, double2* haf_out,
                gbs_partial* partial_out, const int64_t* out_idx_host, hipStream_t stream) {
  ctx->last_error.clear();
  if (batch < 0) return fail(ctx, GBS_EINVAL, "batch < 0");
  if (batch == 0) return GBS_OK;
  if (!st || !offsets_host) return fail(ctx, GBS_EINVAL, "null pointer");
  if (st->device != ctx->device) return fail(ctx, GBS_EINVAL, "state and context are on different devices");
  if (batch > (int64_t)1 << 30) return fail(ctx, GBS_ERANGE, "batch too large");
  if (offsets_host[0] != 0) return fail(ctx, GBS_EINVAL, "offsets[0] must be 0");
  const int64_t total = offsets_host[batch];
  if (total > 0 && !modes_host) return fail(ctx, GBS_EINVAL, "null modes");
  Plan& pl = ctx->plan;
  ItemLists& lists = ctx->lists;
  plan_reset(pl, lists);
  pl.pats.resize(batch);
  pl.part_off.resize(batch + 1);
  pl.nvec.resize(batch);
  pl.sfact.resize(batch);
  pl.part_off[0] = 0;
  for (int64_t b = 0; b < batch; ++b) {
    const int64_t len = offsets_host[b + 1] - offsets_host[b];
    if (len < 0) return fail(ctx, GBS_EINVAL, "offsets must be non-decreasing");
    if (len > GBS_N_MAX) return fail(ctx, GBS_ERANGE, "pattern %lld has n = %lld > %d", (long long)b, (long long)len,
                                     GBS_N_MAX);
    const int n = (int)len;
    int rc = pattern_sfact(ctx, modes_host + offsets_host[b], len, st->m, &pl.sfact[b]);
    if (rc) return rc;
    pl.pats[b] = PatternDesc{offsets_host[b], n, 0};
    pl.nvec[b] = n;
    int64_t lo = 0, hi = subset_count(n);
    if (lo_host) {
      if (lo_host[b] < 0 || hi_host[b] < lo_host[b] || hi_host[b] > hi)
        return fail(ctx, GBS_ERANGE, "slice %lld: [%lld, %lld) outside [0, %lld]", (long long)b, (long long)lo_host[b],
                    (long long)hi_host[b], (long long)hi);
      lo = lo_host[b];
      hi = hi_host[b];
    }
    plan_range(ctx, pl, lists, (int)b, n, lo, hi);
    pl.part_off[b + 1] = pl.n_partials;
  }
  order_items(pl, lists);
  if (out_idx_host) {
    for (int64_t b = 0; b < batch; ++b)
      if (out_idx_host[b] < 0) return fail(ctx, GBS_EINVAL, "negative output index");
    pl.out_idx.assign(out_idx_host, out_idx_host + batch);
  }
  {
    DeviceGuard dg(ctx->device);
    if (hipStreamWaitEvent(stream, st->ready, 0) != hipSuccess) return fail(ctx, GBS_EHIP, "state not ready");
  }
  return run_plan(ctx, pl, modes_host, (size_t)total, st->B, st->m, st->pref, prob_out, haf_out, partial_out, stream);
}

}  // namespace

int gbs_prob_batch(gbs_ctx* ctx, const gbs_state* st, const int32_t* modes_host, const int64_t* offsets_host,
                   int64_t batch, double* prob_out_dev, gbs_c128* haf_out_dev, void* stream) {
  if (!ctx) return GBS_EINVAL;
  if (batch > 0 && !prob_out_dev) return fail(ctx, GBS_EINVAL, "null prob_out");
  return prob_common(ctx, st, modes_host, offsets_host, batch, nullptr, nullptr, prob_out_dev,
                     reinterpret_cast<double2*>(haf_out_dev), nullptr, nullptr, static_cast<hipStream_t>(stream));
}

int gbs_prob_slices(gbs_ctx* ctx, const gbs_state* st, const int32_t* modes_host, const int64_t* offsets_host,
                    const int64_t* lo_host, const int64_t* hi_host, int64_t batch, gbs_partial* partials_dev,
                    const int64_t* out_idx_host, void* stream) {
  if (!ctx) return GBS_EINVAL;
  if (batch > 0 && (!lo_host || !hi_host || !partials_dev)) return fail(ctx, GBS_EINVAL, "null pointer");
  return prob_common(ctx, st, modes_host, offsets_host, batch, lo_host, hi_host, nullptr, nullptr, partials_dev,
                     out_idx_host, static_cast<hipStream_t>(stream));
}

int gbs_finalize(gbs_ctx* ctx, const gbs_state* st, const gbs_partial* partials_dev, const int64_t* part_lo_host,
                 const int64_t* part_hi_host, const int32_t* modes_host, const int64_t* offsets_host, int64_t batch,
                 double* prob_out_dev, gbs_c128* haf_out_dev, void* stream) {
  if (!ctx) return GBS_EINVAL;
  ctx->last_error.clear();
  if (batch < 0) return fail(ctx, GBS_EINVAL, "batch < 0");
  if (batch == 0) return GBS_OK;
  if (!part_lo_host || !part_hi_host || !offsets_host) return fail(ctx, GBS_EINVAL, "null pointer");
  if (prob_out_dev && !st) return fail(ctx, GBS_EINVAL, "prob_out needs a state");
  if (st && st->device != ctx->device) return fail(ctx, GBS_EINVAL, "state and context are on different devices");
  if (offsets_host[0] != 0) return fail(ctx, GBS_EINVAL, "offsets[0] must be 0");
  if (offsets_host[batch] > 0 && !modes_host) return fail(ctx, GBS_EINVAL, "null modes");
  Plan pl;
  pl.part_off.resize(2 * batch);
  pl.nvec.resize(batch);
  pl.sfact.assign(batch, 1.0);
  bool any = false;
  for (int64_t b = 0; b < batch; ++b) {
    if (part_lo_host[b] < 0 || part_hi_host[b] < part_lo_host[b])
      return fail(ctx, GBS_EINVAL, "partial range %lld is malformed", (long long)b);
    const int64_t len = offsets_host[b + 1] - offsets_host[b];
    if (len < 0) return fail(ctx, GBS_EINVAL, "offsets must be non-decreasing");
    if (len > GBS_N_MAX) return fail(ctx, GBS_ERANGE, "pattern %lld has n = %lld > %d", (long long)b, (long long)len,
                                     GBS_N_MAX);
    pl.nvec[b] = (int32_t)len;
    if (prob_out_dev) {
      const int rc = pattern_sfact(ctx, modes_host + offsets_host[b], len, st->m, &pl.sfact[b]);
      if (rc) return rc;
    }
    any |= part_hi_host[b] > part_lo_host[b];
  }
  if (any && !partials_dev) return fail(ctx, GBS_EINVAL, "null partials");
  // stage the ranges (lo then hi, in the part_off region), n and prod_j s_j!
  std::copy(part_lo_host, part_lo_host + batch, pl.part_off.begin());
  std::copy(part_hi_host, part_hi_host + batch, pl.part_off.begin() + batch);
  DeviceGuard dg(ctx->device);
  if (const int g = launch_gate(ctx)) return g;
  const Layout L = layout_for(pl, 0);
  int rc = ensure_ws(ctx, L.total);
  if (rc) return rc;
  int pi = 0;
  rc = acquire_pin(ctx, L.staged_bytes, &pi);
  if (rc) return rc;
  unsigned char* h = static_cast<unsigned char*>(ctx->pinned[pi]);
  const size_t base = L.modes;
  std::memcpy(h + (L.part_off - base), pl.part_off.data(), sizeof(int64_t) * pl.part_off.size());
  std::memcpy(h + (L.nvec - base), pl.nvec.data(), sizeof(int32_t) * pl.nvec.size());
  std::memcpy(h + (L.sfact - base), pl.sfact.data(), sizeof(double) * pl.sfact.size());
  unsigned char* ws = static_cast<unsigned char*>(ctx->ws);
  hipStream_t s = static_cast<hipStream_t>(stream);
  if (ctx->done_recorded) HIPCHK(ctx, hipStreamWaitEvent(s, ctx->done_ev, 0));
  HIPCHK(ctx, hipMemcpyAsync(ws + base, h, L.staged_bytes, hipMemcpyHostToDevice, s));
  HIPCHK(ctx, hipEventRecord(ctx->pinned_ev[pi], s));
  ctx->pinned_used[pi] = true;
  FinalizeArgs fa{};
  fa.partials = partials_dev;
  fa.part_lo = reinterpret_cast<const int64_t*>(ws + L.part_off);
  fa.part_hi = fa.part_lo + batch;
  fa.n = reinterpret_cast<const int32_t*>(ws + L.nvec);
  fa.sfact = reinterpret_cast<const double*>(ws + L.sfact);
  fa.prefactor = st ? st->pref : nullptr;
  fa.batch = batch;
  fa.prob_out = prob_out_dev;
  fa.haf_out = reinterpret_cast<double2*>(haf_out_dev);
  launch_finalize(fa, s);
  HIPCHK(ctx, hipGetLastError());
  HIPCHK(ctx, hipEventRecord(ctx->done_ev, s));
  ctx->done_recorded = true;
  return GBS_OK;
}


namespace {

// Marginals of `batch` prefixes into q_out (device); `extra` bytes of workspace are reserved after
// the marginal's own layout and returned in *extra_dev (for a caller's follow-up kernels).
int marginal_common(gbs_ctx* ctx, const gbs_state* st, int32_t n, const int32_t* modes_host,
                    const int64_t* offsets_host, int64_t batch, double* q_out_dev, size_t extra, void** extra_dev,
                    hipStream_t s);

}  // namespace

int gbs_marginal_batch(gbs_ctx* ctx, const gbs_state* st, int32_t n, const int32_t* modes_host,
                       const int64_t* offsets_host, int64_t batch, double* q_out_dev, void* stream) {
  if (!ctx) return GBS_EINVAL;
  ctx->last_error.clear();
  if (batch < 0) return fail(ctx, GBS_EINVAL, "batch < 0");
  if (batch == 0) return GBS_OK;
  if (!st || !offsets_host || !q_out_dev) return fail(ctx, GBS_EINVAL, "null pointer");
  return marginal_common(ctx, st, n, modes_host, offsets_host, batch, q_out_dev, 0, nullptr,
                         static_cast<hipStream_t>(stream));
}

namespace {

// C(a, b) as an integer, or -1 past 2^62.
int64_t binom_i64(int64_t a, int64_t b) {
  if (b < 0 || a < 0 || b > a) return 0;
  if (b > a - b) b = a - b;
  unsigned __int128 r = 1;
  for (int64_t i = 1; i <= b; ++i) {
    r = r * (unsigned __int128)(a - b + i) / (unsigned __int128)i;
    if (r > ((unsigned __int128)1 << 62)) return -1;
  }
  return (int64_t)r;
}

constexpr int64_t kSweepMaxCount = (int64_t(1) << 31) - 1;

int64_t sweep_count_of(int32_t m, int32_t n, int32_t collisions) {
  if (m <= 0 || n < 0 || n > kSweepMaxN) return -1;
  const int64_t c = collisions ? binom_i64((int64_t)m + n - 1, n) : binom_i64(m, n);
  return (c < 0 || c > kSweepMaxCount) ? -1 : c;
}

}  // namespace

int64_t gbs_sweep_count(int32_t m, int32_t n, int32_t collisions) { return sweep_count_of(m, n, collisions); }

int gbs_prob_sweep(gbs_ctx* ctx, const gbs_state* st, int32_t n, int32_t collisions, double* prob_out_dev,
                   gbs_c128* haf_out_dev, void* stream) {
  if (!ctx) return GBS_EINVAL;
  ctx->last_error.clear();
  if (!st) return fail(ctx, GBS_EINVAL, "null state");
  if (st->device != ctx->device) return fail(ctx, GBS_EINVAL, "state and context are on different devices");
  const int m = st->m;
  const int64_t count = sweep_count_of(m, n, collisions);
  if (count < 0)
    return fail(ctx, GBS_ERANGE, "the sweep of n = %d photons over m = %d modes has too many patterns (or n > %d)", n,
                m, kSweepMaxN);
  if (count == 0) return GBS_OK;  // no pattern (n > m without collisions)
  if (!prob_out_dev && !haf_out_dev) return fail(ctx, GBS_EINVAL, "no output");
  // binomials C(v, i), v below the largest universe m + n - 1, i <= n; per even size its count
  const int U = collisions ? m + n - 1 : m;
  const int bstride = n + 1;
  std::vector<uint64_t> binom((size_t)(U + 1) * bstride, 0);
  for (int v = 0; v <= U; ++v)
    for (int i = 0; i <= n; ++i) {
      const int64_t c = binom_i64(v, i);
      if (c < 0) return fail(ctx, GBS_ERANGE, "binomial C(%d, %d) too large for the sweep's ranks", v, i);
      binom[(size_t)v * bstride + i] = (uint64_t)c;
    }
  std::vector<int64_t> level_count(n + 1, 0);
  int64_t tab_max = 1;
  for (int l = 0; l < n; l += 2) {
    level_count[l] = sweep_count_of(m, l, collisions);
    tab_max = std::max(tab_max, level_count[l]);
  }
  DeviceGuard dg(ctx->device);
  if (const int g = launch_gate(ctx)) return g;
  size_t off = 0;
  const size_t o_binom = off;
  off += al(sizeof(uint64_t) * binom.size());
  const size_t stage = off;
  const size_t o_t0 = off;
  off += al(sizeof(double2) * (size_t)tab_max);
  const size_t o_t1 = off;
  off += al(sizeof(double2) * (size_t)tab_max);
  int rc = ensure_ws(ctx, off);
  if (rc) return rc;
  int pi = 0;
  rc = acquire_pin(ctx, stage, &pi);
  if (rc) return rc;
  std::memcpy(ctx->pinned[pi], binom.data(), sizeof(uint64_t) * binom.size());
  unsigned char* ws = static_cast<unsigned char*>(ctx->ws);
  hipStream_t s = static_cast<hipStream_t>(stream);
  if (ctx->done_recorded) HIPCHK(ctx, hipStreamWaitEvent(s, ctx->done_ev, 0));
  if (hipStreamWaitEvent(s, st->ready, 0) != hipSuccess) return fail(ctx, GBS_EHIP, "state not ready");
  HIPCHK(ctx, hipMemcpyAsync(ws + o_binom, ctx->pinned[pi], stage, hipMemcpyHostToDevice, s));
  HIPCHK(ctx, hipEventRecord(ctx->pinned_ev[pi], s));
  ctx->pinned_used[pi] = true;
  SweepArgs a{};
  a.B = st->B;
  a.m = m;
  a.n = n;
  a.collisions = collisions ? 1 : 0;
  a.bstride = bstride;
  a.binom = reinterpret_cast<const uint64_t*>(ws + o_binom);
  a.count = count;
  a.prefactor = st->pref;
  a.prob_out = prob_out_dev;
  a.haf_out = reinterpret_cast<double2*>(haf_out_dev);
  launch_sweep(a, reinterpret_cast<double2*>(ws + o_t0), reinterpret_cast<double2*>(ws + o_t1), level_count.data(), s);
  HIPCHK(ctx, hipGetLastError());
  HIPCHK(ctx, hipEventRecord(ctx->done_ev, s));
  ctx->done_recorded = true;
  return GBS_OK;
}

int gbs_sweep_sample(gbs_ctx* ctx, const double* prob_dev, int64_t count, const double* uniforms_dev, int64_t nsamples,
                     int64_t* index_out_dev, double* total_out_dev, void* stream) {
  if (!ctx) return GBS_EINVAL;
  ctx->last_error.clear();
  if (count < 0 || nsamples < 0) return fail(ctx, GBS_EINVAL, "negative size");
  if (count == 0 || (nsamples == 0 && !total_out_dev)) return GBS_OK;
  if (!prob_dev || (nsamples > 0 && (!uniforms_dev || !index_out_dev))) return fail(ctx, GBS_EINVAL, "null pointer");
  if (count > kSweepMaxCount) return fail(ctx, GBS_ERANGE, "count too large");
  DeviceGuard dg(ctx->device);
  if (const int g = launch_gate(ctx)) return g;
  const int64_t nb = cdf_blocks(count);
  size_t off = 0;
  const size_t o_cdf = off;
  off += al(sizeof(double) * (size_t)count);
  const size_t o_bsum = off;
  off += al(sizeof(double) * (size_t)nb);
  const size_t o_tot = off;
  off += al(sizeof(double));
  int rc = ensure_ws(ctx, off);
  if (rc) return rc;
  unsigned char* ws = static_cast<unsigned char*>(ctx->ws);
  hipStream_t s = static_cast<hipStream_t>(stream);
  if (ctx->done_recorded) HIPCHK(ctx, hipStreamWaitEvent(s, ctx->done_ev, 0));
  double* cdf = reinterpret_cast<double*>(ws + o_cdf);
  double* total = total_out_dev ? total_out_dev : reinterpret_cast<double*>(ws + o_tot);
  launch_cdf(prob_dev, count, cdf, reinterpret_cast<double*>(ws + o_bsum), total, s);
  if (nsamples > 0) launch_cdf_draw(cdf, count, total, uniforms_dev, nsamples, index_out_dev, s);
  HIPCHK(ctx, hipGetLastError());
  HIPCHK(ctx, hipEventRecord(ctx->done_ev, s));
  ctx->done_recorded = true;
  return GBS_OK;
}

int gbs_photon_number_pmf(int32_t m, double r, int32_t nmax, double* pmf_host) {
  if (m <= 0 || nmax < 0 || !pmf_host || !std::isfinite(r) || r < 0) return GBS_EINVAL;
  for (int n = 0; n <= nmax; ++n) {
    if (n & 1) {
      pmf_host[n] = 0.0;
      continue;
    }
    if (r == 0.0) {
      pmf_host[n] = n == 0 ? 1.0 : 0.0;
      continue;
    }
    // P_n = C((m + n)/2 - 1, n/2) tanh^n r / cosh^m r, the binomial in Gamma form
    const double lb = n == 0 ? 0.0 : log_gbinom_pos((m + n) / 2.0 - 1.0, n / 2.0);
    pmf_host[n] = std::exp(lb + n * std::log(std::tanh(r)) - m * std::log(std::cosh(r)));
  }
  return GBS_OK;
}

int gbs_sample_step(gbs_ctx* ctx, const gbs_state* st, int32_t n, const int32_t* modes_host,
                    const int64_t* offsets_host, int64_t batch, const double* uniforms_dev, double* weights_dev,
                    int32_t* next_dev, void* stream) {
  if (!ctx) return GBS_EINVAL;
  ctx->last_error.clear();
  if (batch < 0) return fail(ctx, GBS_EINVAL, "batch < 0");
  if (batch == 0) return GBS_OK;
  if (!st || !offsets_host || !uniforms_dev || !next_dev) return fail(ctx, GBS_EINVAL, "null pointer");
  if (offsets_host[0] != 0) return fail(ctx, GBS_EINVAL, "offsets[0] must be 0");
  const int m = st->m;
  if ((int64_t)batch * m > (int64_t)1 << 24) return fail(ctx, GBS_ERANGE, "batch x m too large");
  // candidate prefixes: prefix b followed by each mode l
  std::vector<int32_t> cm;
  std::vector<int64_t> co{0};
  for (int64_t b = 0; b < batch; ++b) {
    const int64_t len = offsets_host[b + 1] - offsets_host[b];
    if (len < 0) return fail(ctx, GBS_EINVAL, "offsets must be non-decreasing");
    if (len >= n) return fail(ctx, GBS_ERANGE, "prefix %lld already has n positions", (long long)b);
    if (len > 0 && !modes_host) return fail(ctx, GBS_EINVAL, "null modes");
    for (int l = 0; l < m; ++l) {
      cm.insert(cm.end(), modes_host + offsets_host[b], modes_host + offsets_host[b + 1]);
      cm.push_back(l);
      co.push_back((int64_t)cm.size());
    }
  }
  hipStream_t s = static_cast<hipStream_t>(stream);
  void* scratch = nullptr;
  const size_t wbytes = sizeof(double) * (size_t)batch * m;
  int rc = marginal_common(ctx, st, n, cm.data(), co.data(), batch * m, weights_dev, weights_dev ? 0 : wbytes,
                           &scratch, s);
  if (rc) return rc;
  const double* w = weights_dev ? weights_dev : static_cast<const double*>(scratch);
  DeviceGuard dg(ctx->device);
  launch_draw(w, batch, m, uniforms_dev, next_dev, s);
  HIPCHK(ctx, hipGetLastError());
  HIPCHK(ctx, hipEventRecord(ctx->done_ev, s));
  ctx->done_recorded = true;
  return GBS_OK;
}

namespace {

int marginal_common(gbs_ctx* ctx, const gbs_state* st, int32_t n, const int32_t* modes_host,
                    const int64_t* offsets_host, int64_t batch, double* q_out_dev, size_t extra, void** extra_dev,
                    hipStream_t s) {
  if (!q_out_dev && !extra_dev) return fail(ctx, GBS_EINVAL, "null q_out");
  if (st->device != ctx->device) return fail(ctx, GBS_EINVAL, "state and context are on different devices");
  if (n < 0 || (n & 1) || n > GBS_MARGINAL_NMAX)
    return fail(ctx, GBS_ERANGE, "n = %d must be even and in [0, %d]", n, GBS_MARGINAL_NMAX);
  if (batch > (int64_t)1 << 24) return fail(ctx, GBS_ERANGE, "batch too large");
  if (offsets_host[0] != 0) return fail(ctx, GBS_EINVAL, "offsets[0] must be 0");
  const int m = st->m;
  int kmax = 0;
  for (int64_t b = 0; b < batch; ++b) {
    const int64_t len = offsets_host[b + 1] - offsets_host[b];
    if (len < 0) return fail(ctx, GBS_EINVAL, "offsets must be non-decreasing");
    if (len > n) return fail(ctx, GBS_ERANGE, "prefix %lld has %lld > n positions", (long long)b, (long long)len);
    if (len > GBS_MARGINAL_KMAX)
      return fail(ctx, GBS_ERANGE, "prefix %lld has %lld > %d positions", (long long)b, (long long)len,
                  GBS_MARGINAL_KMAX);
    for (int64_t i = offsets_host[b]; i < offsets_host[b + 1]; ++i)
      if (!modes_host || modes_host[i] < 0 || modes_host[i] >= m)
        return fail(ctx, GBS_ERANGE, "mode out of [0, %d) in prefix %lld", m, (long long)b);
    kmax = std::max(kmax, (int)len);
  }

  // per-prefix tables: hafnian table offsets, weights F, classes (explicit ones only where modes
  // repeat; a collision-free prefix's 2^(k-1) classes are implicit)
  const int jdim = kmax / 2 + 1;
  std::vector<int64_t> h_off(batch + 1, 0), pre_cls(batch + 1, 0), ex_base(batch, -1), F_off(batch);
  std::vector<int32_t> k_vec(batch);
  std::vector<int64_t> cls_mem{0};
  std::vector<double> cls_w, Ftab;
  std::vector<uint32_t> mem;
  std::map<int, int64_t> F_of_k;  // one weight table per distinct prefix length
  // explicit class lists depend only on which positions share a mode: one list per grouping
  std::map<std::vector<int>, std::pair<int64_t, int64_t>> classes_of_grouping;  // -> (first class, count)
  for (int64_t b = 0; b < batch; ++b) {
    const int k = (int)(offsets_host[b + 1] - offsets_host[b]);
    const int32_t* x = modes_host + offsets_host[b];
    k_vec[b] = k;
    h_off[b + 1] = h_off[b] + ((int64_t)1 << k);
    // distinct modes with their multiplicities; code[i] = index of x[i]'s mode
    std::vector<int> code(k);
    std::vector<int32_t> distinct;
    std::vector<int> mult;
    for (int i = 0; i < k; ++i) {
      auto it = std::find(distinct.begin(), distinct.end(), x[i]);
      code[i] = (int)(it - distinct.begin());
      if (it == distinct.end()) {
        distinct.push_back(x[i]);
        mult.push_back(0);
      }
      ++mult[code[i]];
    }
    auto cached = (int)distinct.size() == k ? classes_of_grouping.end() : classes_of_grouping.find(code);
    if ((int)distinct.size() == k) {
      pre_cls[b + 1] = pre_cls[b] + (k == 0 ? 1 : ((int64_t)1 << (k - 1)));
    } else if (cached != classes_of_grouping.end()) {
      ex_base[b] = cached->second.first;
      pre_cls[b + 1] = pre_cls[b] + cached->second.second;
    } else {
      // classes = count vectors (c_t <= multiplicity of mode t, sum = k mod 2); members = every
      // choice of c_t of mode t's positions, for all t; Per(S_{A,B}) = prod c_t!
      const int ng = (int)distinct.size();
      std::vector<std::vector<std::vector<uint32_t>>> combos(ng);  // [t][c] -> position masks
      for (int t = 0; t < ng; ++t) {
        std::vector<int> pos;
        for (int i = 0; i < k; ++i)
          if (code[i] == t) pos.push_back(i);
        combos[t].resize(pos.size() + 1);
        for (uint32_t sm = 0; sm < (1u << pos.size()); ++sm) {
          uint32_t mask = 0;
          for (size_t q = 0; q < pos.size(); ++q)
            if (sm >> q & 1u) mask |= 1u << pos[q];
          combos[t][__builtin_popcount(sm)].push_back(mask);
        }
      }
      ex_base[b] = (int64_t)cls_w.size();
      int64_t nc = 0;
      std::vector<int> cnt(ng, 0), idx(ng);
      for (;;) {
        int tot = 0;
        double w = 1.0;
        for (int t = 0; t < ng; ++t) {
          tot += cnt[t];
          for (int f = 2; f <= cnt[t]; ++f) w *= f;
        }
        if (((tot ^ k) & 1) == 0) {
          // members: the product of the groups' combination lists, first group varying fastest
          std::fill(idx.begin(), idx.end(), 0);
          for (;;) {
            uint32_t A = 0;
            for (int t = 0; t < ng; ++t) A |= combos[t][cnt[t]][idx[t]];
            mem.push_back(A);
            int t = 0;
            while (t < ng && ++idx[t] == (int)combos[t][cnt[t]].size()) idx[t++] = 0;
            if (t == ng) break;
          }
          cls_mem.push_back((int64_t)mem.size());
          cls_w.push_back(w);
          ++nc;
        }
        int t = 0;
        while (t < ng && ++cnt[t] > mult[t]) cnt[t++] = 0;
        if (t == ng) break;
      }
      pre_cls[b + 1] = pre_cls[b] + nc;
      classes_of_grouping.emplace(code, std::make_pair(ex_base[b], nc));
    }
    auto fk = F_of_k.find(k);
    if (fk == F_of_k.end()) {
      fk = F_of_k.emplace(k, (int64_t)Ftab.size()).first;
      for (int mu = 0; mu <= k; ++mu)
        for (int j1 = 0; j1 < jdim; ++j1)
          for (int j2 = 0; j2 < jdim; ++j2) Ftab.push_back(theorem1_weight(m, n, k, mu, j1, j2));
    }
    F_off[b] = fk->second;
  }
  const int64_t ncls = pre_cls[batch];
  const int64_t nx = offsets_host[batch];

  // device layout in the workspace: staged tables, then the hafnian tables, class values, extra
  DeviceGuard dg(ctx->device);
  if (const int g = launch_gate(ctx)) return g;
  size_t off = 0;
  const size_t o_stage = off;
  const size_t o_x = off;
  off += al(sizeof(int32_t) * (size_t)std::max<int64_t>(nx, 1));
  const size_t o_xoff = off;
  off += al(sizeof(int64_t) * (batch + 1));
  const size_t o_hoff = off;
  off += al(sizeof(int64_t) * h_off.size());
  const size_t o_k = off;
  off += al(sizeof(int32_t) * k_vec.size());
  const size_t o_F = off;
  off += al(sizeof(double) * Ftab.size());
  const size_t o_Foff = off;
  off += al(sizeof(int64_t) * F_off.size());
  const size_t o_pre = off;
  off += al(sizeof(int64_t) * pre_cls.size());
  const size_t o_exb = off;
  off += al(sizeof(int64_t) * ex_base.size());
  const size_t o_cm = off;
  off += al(sizeof(int64_t) * cls_mem.size());
  const size_t o_cw = off;
  off += al(sizeof(double) * std::max<size_t>(cls_w.size(), 1));
  const size_t o_mem = off;
  off += al(sizeof(uint32_t) * std::max<size_t>(mem.size(), 1));
  const size_t stage_bytes = off - o_stage;
  const size_t o_h = off;
  off += al(sizeof(double2) * (size_t)h_off[batch]);
  const size_t o_v = off;
  off += al(sizeof(double) * (size_t)std::max<int64_t>(ncls, 1));
  const size_t o_extra = off;
  off += al(extra);
  int rc = ensure_ws(ctx, off);
  if (rc) return rc;
  unsigned char* ws = static_cast<unsigned char*>(ctx->ws);
  if (extra_dev) *extra_dev = ws + o_extra;
  if (!q_out_dev) q_out_dev = reinterpret_cast<double*>(ws + o_extra);

  int pi = 0;
  rc = acquire_pin(ctx, stage_bytes, &pi);
  if (rc) return rc;
  unsigned char* hp = static_cast<unsigned char*>(ctx->pinned[pi]);
  auto put = [&](size_t o, const void* src, size_t bytes) {
    if (bytes) std::memcpy(hp + (o - o_stage), src, bytes);
  };
  put(o_x, modes_host, sizeof(int32_t) * (size_t)nx);
  put(o_xoff, offsets_host, sizeof(int64_t) * (batch + 1));
  put(o_hoff, h_off.data(), sizeof(int64_t) * h_off.size());
  put(o_k, k_vec.data(), sizeof(int32_t) * k_vec.size());
  put(o_F, Ftab.data(), sizeof(double) * Ftab.size());
  put(o_Foff, F_off.data(), sizeof(int64_t) * F_off.size());
  put(o_pre, pre_cls.data(), sizeof(int64_t) * pre_cls.size());
  put(o_exb, ex_base.data(), sizeof(int64_t) * ex_base.size());
  put(o_cm, cls_mem.data(), sizeof(int64_t) * cls_mem.size());
  put(o_cw, cls_w.data(), sizeof(double) * cls_w.size());
  put(o_mem, mem.data(), sizeof(uint32_t) * mem.size());
  if (ctx->done_recorded) HIPCHK(ctx, hipStreamWaitEvent(s, ctx->done_ev, 0));
  if (hipStreamWaitEvent(s, st->ready, 0) != hipSuccess) return fail(ctx, GBS_EHIP, "state not ready");
  HIPCHK(ctx, hipMemcpyAsync(ws + o_stage, hp, stage_bytes, hipMemcpyHostToDevice, s));
  HIPCHK(ctx, hipEventRecord(ctx->pinned_ev[pi], s));
  ctx->pinned_used[pi] = true;

  MargArgs ma{};
  ma.W = st->W;
  ma.m = m;
  ma.x = reinterpret_cast<const int32_t*>(ws + o_x);
  ma.x_off = reinterpret_cast<const int64_t*>(ws + o_xoff);
  ma.h = reinterpret_cast<double2*>(ws + o_h);
  ma.h_off = reinterpret_cast<const int64_t*>(ws + o_hoff);
  ma.k = reinterpret_cast<const int32_t*>(ws + o_k);
  ma.F = reinterpret_cast<const double*>(ws + o_F);
  ma.F_off = reinterpret_cast<const int64_t*>(ws + o_Foff);
  ma.pre_cls = reinterpret_cast<const int64_t*>(ws + o_pre);
  ma.ex_base = reinterpret_cast<const int64_t*>(ws + o_exb);
  ma.cls_mem = reinterpret_cast<const int64_t*>(ws + o_cm);
  ma.cls_w = reinterpret_cast<const double*>(ws + o_cw);
  ma.mem = reinterpret_cast<const uint32_t*>(ws + o_mem);
  ma.n_classes = ncls;
  ma.v = reinterpret_cast<double*>(ws + o_v);
  ma.batch = batch;
  ma.jdim = jdim;
  ma.q_out = q_out_dev;
  launch_marginal(ma, kmax, h_off[batch], s);
  HIPCHK(ctx, hipGetLastError());
  HIPCHK(ctx, hipEventRecord(ctx->done_ev, s));
  ctx->done_recorded = true;
  return GBS_OK;
}

}  // namespace

}  // extern "C"
