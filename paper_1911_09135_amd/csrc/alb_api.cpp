// Host runtime behind include/alb.h: argument validation, the device-resident
// graph, cached per-call workspaces and the round drivers (host loop or one
// persistent launch).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <array>
#include <atomic>
#include <climits>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <tuple>
#include <mutex>
#include <new>
#include <string>
#include <thread>
#include <vector>

#include "../../include/alb.h"
#include "alb_host.h"
#include "alb_internal.h"

using namespace alb;

namespace {

thread_local std::string g_err;

alb_status fail(alb_status s, const char *fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_err = buf;
  return s;
}

#define HIP_TRY(expr)                                                                                   \
  do {                                                                                                  \
    hipError_t e_ = (expr);                                                                             \
    if (e_ != hipSuccess) {                                                                             \
      if (e_ == hipErrorOutOfMemory) return fail(ALB_E_NOMEM, "%s: %s", #expr, hipGetErrorString(e_)); \
      return fail(ALB_E_DEVICE, "%s: %s", #expr, hipGetErrorString(e_));                                \
    }                                                                                                   \
  } while (0)

struct Workspace {
  uint32_t qcap = 0;
  uint32_t hint_cap = 0;
  int32_t n = 0;
  bool busy = false;
  int32_t *q0 = nullptr, *q1 = nullptr, *labels = nullptr;
  int2 *hint = nullptr;
  int4 *huge_rec = nullptr;
  unsigned long long *bar = nullptr, *word = nullptr, *acc = nullptr;
  float *rank = nullptr;
  Ctl *ctl = nullptr;
  Ctl *h_ctl = nullptr;  // pinned host mirror
  hipEvent_t ev[3] = {nullptr, nullptr, nullptr};
  size_t bytes = 0;

  void release() {
    (void)hipFree(q0);
    (void)hipFree(q1);
    (void)hipFree(huge_rec);
    (void)hipFree(hint);
    (void)hipFree(bar);
    (void)hipFree(word);
    (void)hipFree(labels);
    (void)hipFree(rank);
    (void)hipFree(acc);
    (void)hipFree(ctl);
    if (h_ctl) (void)hipHostFree(h_ctl);
    for (auto &e : ev)
      if (e) (void)hipEventDestroy(e);
    *this = Workspace();
  }
};

// Workspace of a batch of queries on a graph set: worklists of
// (query << 32 | vertex) entries, one label per (query, vertex of its graph)
// and the per-query tables.
// Bytes of per-query tables in a batch workspace: three int64 (label offset,
// threshold, label base), an output pointer and four int32 (source, size,
// wavefront and workgroup cutoffs).
constexpr size_t kBatchTableBytes = 3 * sizeof(long long) + sizeof(int32_t *) + 4 * sizeof(int32_t);

struct BatchWs {
  long long lab_cap = 0;
  uint32_t qcap = 0, hint_cap = 0;
  int32_t nq_cap = 0;
  bool busy = false;
  unsigned long long *q0 = nullptr, *q1 = nullptr, *word = nullptr, *bar = nullptr;
  int32_t *out32 = nullptr;
  int2 *hint = nullptr;
  int4 *huge_rec = nullptr;
  // per-query tables (offsets, thresholds, label bases, output pointers,
  // sources, sizes), kBatchTableBytes per query, and their pinned host mirror:
  // one copy uploads a batch's tables
  unsigned char *tab = nullptr, *h_tab = nullptr;
  Ctl *ctl = nullptr;
  Ctl *h_ctl = nullptr;
  hipEvent_t ev[3] = {nullptr, nullptr, nullptr};
  size_t bytes = 0;

  void release() {
    void *p[] = {q0, q1, word, bar, out32, hint, huge_rec, tab, ctl};
    for (void *x : p) (void)hipFree(x);
    if (h_ctl) (void)hipHostFree(h_ctl);
    if (h_tab) (void)hipHostFree(h_tab);
    for (auto &e : ev)
      if (e) (void)hipEventDestroy(e);
    *this = BatchWs();
  }
};

}  // namespace

struct alb_graph_s {
  int32_t n = 0;
  int64_t m = 0;
  int32_t max_deg = 0;
  bool symmetric = false;
  bool weighted = false;
  int device = 0;
  int cus = 0;
  uint64_t clock_khz = 100000;
  int32_t *d_off = nullptr, *d_col = nullptr, *d_w = nullptr;
  int32_t *d_toff = nullptr, *d_tcol = nullptr;  // transposed CSR (ALB_BUILD_TRANSPOSE)
  hipStream_t stream = nullptr;
  size_t graph_bytes = 0;
  std::mutex mu;
  std::vector<Workspace *> pool;
  std::vector<BatchWs *> batch_pool;
  // members of a graph set (a plain graph is a set of one): vertex base in the
  // set's numbering, vertex and edge counts
  std::vector<int32_t> mem_vbase, mem_n;
  std::vector<int64_t> mem_m;
  // per member: the largest out-degree and the degree distribution's
  // signature (the share of edges held by vertices of out-degree in
  // [2^k, 2^(k+1)), in eighths) that the autotuner keys its results by
  std::vector<int32_t> mem_maxdeg;
  std::vector<std::array<uint8_t, 32>> mem_hist;
  std::atomic<int> plans{0};  // live batch plans on this graph
};

namespace {

// --------------------------------------------------------------------------
// CSR validation and host symmetrisation
// --------------------------------------------------------------------------

alb_status validate_csr(int32_t n, int64_t m, const int32_t *off, const int32_t *col, const int32_t *w) {
  if (n < 1) return fail(ALB_E_INVAL, "n must be >= 1 (got %d)", n);
  if (m < 0 || m >= ((int64_t)1 << 31)) return fail(ALB_E_INVAL, "m must be in [0, 2^31) (got %lld)", (long long)m);
  if (!off) return fail(ALB_E_INVAL, "row_offsets is NULL");
  if (m > 0 && !col) return fail(ALB_E_INVAL, "col is NULL");
  if (off[0] != 0) return fail(ALB_E_INVAL, "row_offsets[0] must be 0 (got %d)", off[0]);
  for (int32_t v = 0; v < n; ++v)
    if (off[v + 1] < off[v]) return fail(ALB_E_INVAL, "row_offsets decreases at vertex %d", v);
  if ((int64_t)off[n] != m) return fail(ALB_E_INVAL, "row_offsets[n] = %d differs from m = %lld", off[n], (long long)m);
  for (int64_t p = 0; p < m; ++p)
    if (col[p] < 0 || col[p] >= n) return fail(ALB_E_INVAL, "col[%lld] = %d out of range", (long long)p, col[p]);
  if (w) {
    int64_t wmax = 0;
    for (int64_t p = 0; p < m; ++p) {
      if (w[p] < 0) return fail(ALB_E_INVAL, "weights[%lld] = %d is negative", (long long)p, w[p]);
      wmax = std::max<int64_t>(wmax, w[p]);
    }
    if (wmax * (int64_t)(n - 1) >= (int64_t)INT32_MAX)
      return fail(ALB_E_RANGE, "max weight %lld x (n - 1) = %lld does not fit below INT32_MAX", (long long)wmax,
                  (long long)(wmax * (int64_t)(n - 1)));
  }
  return ALB_OK;
}

template <class F>
void parallel_rows(int32_t n, F f) {
  unsigned t = std::max(1u, std::min(16u, std::thread::hardware_concurrency()));
  if (n < 65536) t = 1;
  std::vector<std::thread> th;
  std::atomic<int32_t> next{0};
  auto body = [&] {
    for (;;) {
      int32_t b = next.fetch_add(4096);
      if (b >= n) break;
      int32_t e = std::min(n, b + 4096);
      for (int32_t v = b; v < e; ++v) f(v);
    }
  };
  for (unsigned i = 1; i < t; ++i) th.emplace_back(body);
  body();
  for (auto &x : th) x.join();
}

// Both directions of every edge, rows sorted, duplicates and self-loops removed.
alb_status symmetrise(int32_t n, const int32_t *off, const int32_t *col, std::vector<int32_t> &soff,
                      std::vector<int32_t> &scol) {
  try {
    int64_t m = off[n];
    std::vector<int64_t> cnt((size_t)n + 1, 0);
    for (int32_t u = 0; u < n; ++u) {
      cnt[u + 1] += off[u + 1] - off[u];
      for (int32_t p = off[u]; p < off[u + 1]; ++p) cnt[(size_t)col[p] + 1]++;
    }
    for (int32_t v = 0; v < n; ++v) cnt[v + 1] += cnt[v];
    std::vector<int32_t> raw((size_t)cnt[n]);
    std::vector<int64_t> cur(cnt.begin(), cnt.end() - 1);
    for (int32_t u = 0; u < n; ++u)
      for (int32_t p = off[u]; p < off[u + 1]; ++p) {
        raw[(size_t)cur[u]++] = col[p];
        raw[(size_t)cur[col[p]]++] = u;
      }
    (void)m;
    std::vector<int64_t> keep((size_t)n, 0);
    parallel_rows(n, [&](int32_t v) {
      int32_t *b = raw.data() + cnt[v], *e = raw.data() + cnt[v + 1];
      std::sort(b, e);
      int64_t k = 0;
      for (int32_t *p = b; p < e; ++p) {
        if (*p == v) continue;
        if (k > 0 && b[k - 1] == *p) continue;
        b[k++] = *p;
      }
      keep[v] = k;
    });
    soff.assign((size_t)n + 1, 0);
    int64_t total = 0;
    for (int32_t v = 0; v < n; ++v) {
      soff[v] = (int32_t)total;
      total += keep[v];
      if (total >= ((int64_t)1 << 31)) return fail(ALB_E_INVAL, "symmetrised graph has 2^31 or more edges");
    }
    soff[n] = (int32_t)total;
    scol.resize((size_t)total);
    parallel_rows(n, [&](int32_t v) {
      std::copy(raw.data() + cnt[v], raw.data() + cnt[v] + keep[v], scol.data() + soff[v]);
    });
  } catch (const std::bad_alloc &) {
    return fail(ALB_E_NOMEM, "host allocation failed while symmetrising");
  }
  return ALB_OK;
}

// --------------------------------------------------------------------------
// Workspaces
// --------------------------------------------------------------------------

// Entries of the huge-edge chunk index: one per 2^kHintMinShift huge edges of
// a round, plus two.  A round's huge edges are at most the worklist capacity
// times the largest degree (a 32-bit total: a larger one is reported as an
// overflow by the reservation); when every vertex enters a round's worklist at
// most once (`unique_edges` >= 0: the edge count of the graph or the batch)
// they are at most those edges.
uint32_t hint_entries(uint64_t qcap, int64_t unique_edges, int64_t max_deg) {
  uint64_t e = std::min<uint64_t>(qcap * (uint64_t)std::max<int64_t>(max_deg, 1), 1ull << 32);
  if (unique_edges >= 0) e = std::min<uint64_t>(e, (uint64_t)unique_edges);
  return (uint32_t)((e >> kHintMinShift) + 2);
}

// The distinct-entry bound of one round's worklist: BFS, k-core and PageRank
// enter each vertex at most once per round, SSSP and CC with dedup too.
int64_t dedup_bound(OpKind op, bool dedup, int64_t m) {
  if (op == OP_SSSP || op == OP_CC) return dedup ? m : -1;
  if (op == OP_RECORD) return -1;
  return m;
}

struct Needs {
  uint32_t qcap;
  uint32_t hint_cap;
};

// Fault injection for tests: while ALB_INJECT_ALLOC_FAILURE=1 is in the
// environment, every device and pinned host allocation of the library fails
// as if memory were exhausted (without calling the allocator).
bool alloc_failure_injected() {
  const char *e = getenv("ALB_INJECT_ALLOC_FAILURE");
  return e && e[0] == '1' && e[1] == 0;
}

template <class T>
hipError_t dalloc(T **p, size_t count, size_t &bytes) {
  if (alloc_failure_injected()) return hipErrorOutOfMemory;
  size_t b = sizeof(T) * std::max<size_t>(count, 1);
  hipError_t e = hipMalloc((void **)p, b);
  if (e == hipSuccess) bytes += b;
  return e;
}

// Pinned host memory (the control-block and table mirrors).
template <class T>
hipError_t palloc(T **p, size_t bytes) {
  if (alloc_failure_injected()) return hipErrorOutOfMemory;
  return hipHostMalloc((void **)p, bytes, hipHostMallocDefault);
}

alb_status ws_fill(Workspace *w, int32_t n, const Needs &nd) {
  w->n = n;
  w->qcap = nd.qcap;
  w->hint_cap = nd.hint_cap;
  HIP_TRY(dalloc(&w->q0, nd.qcap, w->bytes));
  HIP_TRY(dalloc(&w->q1, nd.qcap, w->bytes));
  HIP_TRY(dalloc(&w->huge_rec, nd.qcap, w->bytes));
  HIP_TRY(dalloc(&w->hint, nd.hint_cap, w->bytes));
  HIP_TRY(dalloc(&w->bar, kBarWords, w->bytes));
  HIP_TRY(dalloc(&w->word, (size_t)n, w->bytes));
  HIP_TRY(dalloc(&w->labels, (size_t)n, w->bytes));
  HIP_TRY(dalloc(&w->rank, (size_t)n, w->bytes));
  HIP_TRY(dalloc(&w->acc, (size_t)n, w->bytes));
  HIP_TRY(dalloc(&w->ctl, 1, w->bytes));
  HIP_TRY(palloc(&w->h_ctl, sizeof(Ctl)));
  for (auto &e : w->ev) HIP_TRY(hipEventCreate(&e));
  return ALB_OK;
}

// Take a free cached workspace that `fits`, else grow a free one or make a
// new one with `fill`.
template <class W, class Fits, class Fill>
alb_status pool_acquire(alb_graph g, std::vector<W *> &pool, Fits fits, Fill fill, W **out) {
  std::lock_guard<std::mutex> lk(g->mu);
  for (W *w : pool)
    if (!w->busy && fits(*w)) {
      w->busy = true;
      *out = w;
      return ALB_OK;
    }
  W *w = nullptr;
  for (W *x : pool)
    if (!x->busy) {
      w = x;
      w->release();
      break;
    }
  bool fresh = false;
  if (!w) {
    w = new (std::nothrow) W();
    if (!w) return fail(ALB_E_NOMEM, "host allocation failed");
    fresh = true;
  }
  alb_status s = fill(w);
  if (s != ALB_OK) {
    std::string keep = g_err;
    w->release();
    if (!fresh) pool.erase(std::find(pool.begin(), pool.end(), w));
    delete w;
    g_err = keep;
    return s;
  }
  if (fresh) pool.push_back(w);
  w->busy = true;
  *out = w;
  return ALB_OK;
}

alb_status ws_acquire(alb_graph g, const Needs &nd, Workspace **out) {
  return pool_acquire(
      g, g->pool, [&](const Workspace &w) { return w.qcap >= nd.qcap && w.hint_cap >= nd.hint_cap; },
      [&](Workspace *w) { return ws_fill(w, g->n, nd); }, out);
}

struct BatchNeeds {
  long long labels;
  uint32_t qcap, hint_cap;
  int32_t nq;
};

alb_status bws_fill(BatchWs *w, const BatchNeeds &nd) {
  w->lab_cap = nd.labels;
  w->qcap = nd.qcap;
  w->hint_cap = nd.hint_cap;
  w->nq_cap = nd.nq;
  HIP_TRY(dalloc(&w->q0, nd.qcap, w->bytes));
  HIP_TRY(dalloc(&w->q1, nd.qcap, w->bytes));
  HIP_TRY(dalloc(&w->huge_rec, nd.qcap, w->bytes));
  HIP_TRY(dalloc(&w->hint, nd.hint_cap, w->bytes));
  HIP_TRY(dalloc(&w->bar, kBarWords, w->bytes));
  HIP_TRY(dalloc(&w->word, (size_t)nd.labels, w->bytes));
  HIP_TRY(dalloc(&w->out32, (size_t)nd.labels, w->bytes));
  HIP_TRY(dalloc(&w->tab, kBatchTableBytes * (size_t)nd.nq, w->bytes));
  HIP_TRY(palloc(&w->h_tab, kBatchTableBytes * (size_t)std::max(nd.nq, 1)));
  HIP_TRY(dalloc(&w->ctl, 1, w->bytes));
  HIP_TRY(palloc(&w->h_ctl, sizeof(Ctl)));
  for (auto &e : w->ev) HIP_TRY(hipEventCreate(&e));
  return ALB_OK;
}

alb_status bws_acquire(alb_graph g, const BatchNeeds &nd, BatchWs **out) {
  return pool_acquire(
      g, g->batch_pool,
      [&](const BatchWs &w) {
        return w.lab_cap >= nd.labels && w.qcap >= nd.qcap && w.hint_cap >= nd.hint_cap && w.nq_cap >= nd.nq;
      },
      [&](BatchWs *w) { return bws_fill(w, nd); }, out);
}

template <class W>
void ws_release(alb_graph g, W *w) {
  std::lock_guard<std::mutex> lk(g->mu);
  w->busy = false;
}

template <class W>
struct GuardOf {
  alb_graph g;
  W *w;
  ~GuardOf() {
    if (w) ws_release(g, w);
  }
};
using WsGuard = GuardOf<Workspace>;

// --------------------------------------------------------------------------
// Options
// --------------------------------------------------------------------------

alb_options defaults() {
  alb_options o;
  std::memset(&o, 0, sizeof o);
  o.struct_size = sizeof(alb_options);
  o.mode = ALB_MODE_ALB;
  o.huge_threshold = -1;
  o.wg_size = 256;
  o.wave_cutoff = 64;
  o.wg_cutoff = 0;
  o.distribution = 0;
  o.dedup = -1;
  o.launch = ALB_LAUNCH_AUTO;
  o.grid_wgs = 0;
  o.worklist_capacity = 0;
  o.stream = nullptr;
  o.out_on_device = 0;
  return o;
}

alb_status resolve_options(const alb_options *user, alb_options &o) {
  o = defaults();
  if (user) {
    if (user->struct_size != sizeof(alb_options))
      return fail(ALB_E_INVAL, "alb_options.struct_size = %u, expected %zu (use alb_options_init)", user->struct_size,
                  sizeof(alb_options));
    o = *user;
  }
  if (o.mode < ALB_MODE_ALB || o.mode > ALB_MODE_LB_ALL) return fail(ALB_E_INVAL, "bad mode %d", o.mode);
  if (o.wg_size == 0) o.wg_size = 256;
  if (!supported_wg(o.wg_size)) return fail(ALB_E_UNSUPPORTED, "wg_size %d not built (64, 256, 1024)", o.wg_size);
  if (o.wave_cutoff == 0) o.wave_cutoff = 64;
  if (o.wg_cutoff == 0) o.wg_cutoff = o.wg_size;
  if (o.wave_cutoff < 1 || o.wg_cutoff < 1) return fail(ALB_E_INVAL, "cutoffs must be >= 1");
  if (o.distribution != 0 && o.distribution != 1)
    return fail(ALB_E_UNSUPPORTED, "distribution %d (0 cyclic, 1 blocked)", o.distribution);
  if (o.dedup < -1 || o.dedup > 1) return fail(ALB_E_INVAL, "bad dedup %d", o.dedup);
  if (o.visited_filter < -1 || o.visited_filter > 1) return fail(ALB_E_INVAL, "bad visited_filter %d", o.visited_filter);
  if (o.launch < ALB_LAUNCH_AUTO || o.launch > ALB_LAUNCH_PERSISTENT) return fail(ALB_E_INVAL, "bad launch %d", o.launch);
  if (o.grid_wgs < ALB_GRID_ALL) return fail(ALB_E_INVAL, "grid_wgs must be >= -1");
  if (o.worklist_capacity < 0 || o.worklist_capacity > 0xfffffffeLL) return fail(ALB_E_INVAL, "bad worklist_capacity");
  if (o.huge_threshold < 0 && o.huge_threshold != ALB_THRESHOLD_DEFAULT && o.huge_threshold != ALB_THRESHOLD_LAUNCHED &&
      o.huge_threshold != ALB_THRESHOLD_ADAPTIVE)
    return fail(ALB_E_INVAL, "bad huge_threshold %lld", (long long)o.huge_threshold);
  return ALB_OK;
}

// --------------------------------------------------------------------------
// The round driver shared by every traversal
// --------------------------------------------------------------------------

// The default huge threshold: a vertex is huge when its list is longer than
// a twentieth of one workgroup's share of all edges (m / workgroups), kept
// within [64, 4,096].  A list that long would hold one workgroup well past
// the others in any round that carries a fair part of the graph.  Measured
// against sweeps of t = 32 ... 4,096 on RMAT scales 12 to 22 at the automatic
// grid: within 10 % of the best fixed threshold for SSSP at every scale but
// 16 (scale 22: 4,052, best 2,048-4,096; scale 14: 94, best 64).
int64_t default_threshold(int64_t edges, int grid) {
  const int64_t t = edges / (20 * (int64_t)std::max(grid, 1));
  return std::max<int64_t>(64, std::min<int64_t>(t, 4096));
}

// The default also lowers the threshold in rounds whose worklist is shorter
// than the launched threads, where a few long lists would hold their
// workgroups while the rest of the grid idles: to 64 (kAdaptiveSmall) for
// operators whose pushed value does not depend on the source vertex (BFS
// levels, k-core decrements: their cyclic phase needs no per-edge source
// value), and to a quarter of the default, at least 64, for the others.
// Measured at the automatic grid (device us per query, default without ->
// with the small-round rule): RMAT-14 BFS 170 -> 103, SSSP 262 -> 251;
// RMAT-16 SSSP 428 -> 362; RMAT-20 SSSP 1,150 -> 1,112; RMAT-22 BFS 1,121
// -> 1,017, SSSP 2,318 -> 2,269.
int64_t default_small_threshold(OpKind op, int64_t threshold) {
  if (op == OP_BFS || op == OP_KCORE) return kAdaptiveSmall;
  return std::max<int64_t>(kAdaptiveSmall, threshold / 4);
}

}  // namespace

namespace alb {

// Workgroups for a traversal over `edges` edges: about 2 * cbrt(edges)
// workgroups of 256 threads (the same thread count at other sizes), at least
// 16 of them, at most `resident`.  Measured on RMAT graphs from 228K to 65M
// edges: fewer, cheaper-to-synchronise workgroups win on small graphs and a
// full device only pays off near 10^8 edges (RMAT-14 BFS 0.17 vs 0.26 ms,
// RMAT-20 SSSP 1.27 vs 1.54 ms against every resident workgroup).
alb_status check_options(const alb_options *user, alb_options *out) { return resolve_options(user, *out); }

int auto_grid(int64_t edges, int wg, int resident) {
  const double w256 = std::max(16.0, 2.0 * std::cbrt((double)std::max<int64_t>(edges, 1)));
  const int g = (int)std::lround(w256 * 256.0 / (double)wg);
  return std::max(1, std::min(g, resident));
}

}  // namespace alb

namespace {

// Longest wait at a grid barrier before the persistent launch gives up
// (ALB_BARRIER_TIMEOUT_MS, default 30 s).  Every wave leaves in bounded time.
uint64_t barrier_timeout_ms() {
  const char *e = getenv("ALB_BARRIER_TIMEOUT_MS");
  if (e) {
    long long v = atoll(e);
    if (v > 0) return (uint64_t)v;
  }
  return 30000;
}

// Upper bound on co-resident workgroups of the persistent kernel (op, wg):
// the occupancy calculator's per-CU figure times the CU count.  The
// persistent launch uses this as its grid; membership inside the launch
// decides how many workgroups actually take part.
std::mutex g_res_mu;
std::map<std::tuple<int, int, int>, int> g_res;

alb_status resident_workgroups(alb_graph g, OpKind op, int wg, int *out, bool batch = false, bool open = false) {
  const auto key = std::make_tuple(g->device, (int)op + (batch ? 256 : 0) + (open ? 512 : 0), wg);
  std::lock_guard<std::mutex> lk(g_res_mu);
  auto it = g_res.find(key);
  if (it == g_res.end()) {
    int per_cu = 0;
    HIP_TRY(open    ? open_occupancy(op, wg, &per_cu)
            : batch ? batch_occupancy(op, wg, &per_cu)
                    : op == OP_PR_PULL ? pull_occupancy(wg, &per_cu) : persistent_occupancy(op, wg, &per_cu));
    if (per_cu < 1) return fail(ALB_E_DEVICE, "persistent kernel does not fit on a CU with wg_size %d", wg);
    it = g_res.emplace(key, per_cu * g->cus).first;
  }
  *out = it->second;
  return ALB_OK;
}

struct Job {
  OpKind op;
  int32_t source = -1;        // BFS / SSSP
  uint32_t nfront0 = 0;       // size of the round-0 worklist
  bool identity_first = false;
  bool all_rounds = false;     // PageRank
  int32_t max_rounds = 0;
  float damping = 0.85f;
  int32_t k = 0;               // k-core
  const int32_t *h_frontier = nullptr;  // trace: explicit round-0 worklist (host)
  int32_t *d_hits = nullptr, *d_thread = nullptr;
  int8_t *d_bins = nullptr;
  uint32_t qcap_min = 0;
};

struct RunOut {
  Workspace *ws = nullptr;
  uint32_t qcap = 0;
  int32_t *d_labels = nullptr;  // where labels ended up on the device
  float *d_rank = nullptr;
  hipStream_t stream = nullptr;
};

void zero_stats(alb_stats *st) {
  if (st) std::memset(st, 0, sizeof *st);
}

alb_status abort_error(const Ctl &c) {
  return fail(ALB_E_DEVICE,
              "a grid barrier wait timed out in round %u (%llu of %llu arrivals seen, %u members); the device "
              "run was abandoned",
              c.diag_round, c.diag_seen, c.diag_target, c.n_members);
}

void print_timeline(const Ctl &c, int op, int rounds, long long threshold, uint64_t clock_khz) {
  const double us = 1000.0 / (double)clock_khz;
  fprintf(stderr, "[alb] op %d members %u threshold %lld\n", op, c.n_members, threshold);
  for (int r = 0; r < std::min(rounds, kTimeline); ++r) {
    const unsigned long long *t = &c.tl[4 * r];
    fprintf(stderr, "[alb] round %2d  |F| %9u  huge %7u  twc %8.1f us  lb %8.1f us\n", r,
            (unsigned)(t[3] & 0xffffffffu), (unsigned)(t[3] >> 32), (double)(t[1] - t[0]) * us,
            (double)(t[2] - t[1]) * us);
  }
  static const char *names[kProfParts] = {"inspect", "wg-bin", "wave-bin", "thread-bin", "lb", "barrier"};
  fprintf(stderr, "[alb] workgroup-time per part (us summed over %u members):", c.n_members);
  for (int k = 0; k < kProfParts; ++k) fprintf(stderr, " %s %.0f", names[k], (double)c.prof[k] * us);
  fprintf(stderr, "\n");
}

// Edges per member workgroup in each round: the largest over the mean (1 is
// perfect balance), and over the whole launch.
void print_skew(const uint32_t *d_counts, int rounds, int members) {
  std::vector<uint32_t> h((size_t)kTimeline * kProfMembers);
  if (hipMemcpy(h.data(), d_counts, sizeof(uint32_t) * h.size(), hipMemcpyDeviceToHost) != hipSuccess) return;
  std::vector<unsigned long long> tot((size_t)members, 0);
  for (int r = 0; r < rounds; ++r) {
    unsigned long long sum = 0, mx = 0;
    for (int w = 0; w < members; ++w) {
      const uint32_t x = h[(size_t)r * kProfMembers + w];
      sum += x;
      mx = std::max<unsigned long long>(mx, x);
      tot[w] += x;
    }
    if (sum)
      fprintf(stderr, "[alb] skew round %2d  edges %llu  max/mean per workgroup %.2f\n", r, sum,
              (double)mx * members / (double)sum);
  }
  unsigned long long sum = 0, mx = 0;
  for (unsigned long long x : tot) {
    sum += x;
    mx = std::max(mx, x);
  }
  if (sum) fprintf(stderr, "[alb] skew launch  edges %llu  max/mean per workgroup %.2f\n", sum,
                   (double)mx * members / (double)sum);
}

void fill_stats(alb_stats *st, const Ctl &c, int rounds, int launches, int64_t T, int64_t threshold, hipEvent_t e0,
                hipEvent_t e1, hipEvent_t e2) {
  float ms_all = 0.f, ms_k = 0.f;
  if (e0 && e1 && e2) {  // (untimed without events)
    (void)hipEventElapsedTime(&ms_all, e0, e2);
    (void)hipEventElapsedTime(&ms_k, e1, e2);
  }
  st->rounds = rounds;
  st->kernel_launches = launches;
  st->launched_threads = T;
  st->huge_threshold = threshold;
  st->frontier_vertices = (int64_t)c.st_frontier;
  st->edges_examined = (int64_t)(c.st_edges_twc + c.st_edges_lb);
  st->huge_vertices = (int64_t)c.st_huge_v;
  st->huge_edges = (int64_t)c.st_edges_lb;
  st->pushes = (int64_t)c.st_pushes;
  st->device_ms = ms_all;
  st->kernel_ms = ms_k;
}

// Worklist capacity and chunk-index entries a call needs, and whether it
// suppresses duplicate pushes.
Needs job_needs(alb_graph g, const Job &job, const alb_options &o, bool *dedup_out) {
  bool dedup = false;
  if (job.op == OP_SSSP || job.op == OP_CC) dedup = (o.dedup != 0);
  uint64_t qcap;
  if (o.worklist_capacity > 0)
    qcap = (uint64_t)o.worklist_capacity;
  else if (job.op == OP_BFS || dedup || job.op == OP_PR || job.op == OP_PR_PULL || job.op == OP_KCORE)
    qcap = (uint64_t)g->n;
  else
    qcap = (uint64_t)g->n + (uint64_t)g->m;
  qcap = std::max<uint64_t>(qcap, std::max<uint64_t>(job.qcap_min, job.nfront0));
  qcap = std::max<uint64_t>(qcap, 1);
  if (qcap > 0xfffffffeULL) qcap = 0xfffffffeULL;
  *dedup_out = dedup;
  return Needs{(uint32_t)qcap, hint_entries(qcap, dedup_bound(job.op, dedup, g->m), g->max_deg)};
}

// `fixed`: a workspace laid out by the caller (alb_sssp_noalloc's scratch):
// no workspace is taken from the pool, no event is recorded and nothing is
// allocated; its h_ctl may be pageable host memory.
alb_status run_job(alb_graph g, const Job &job, const alb_options &o, void *dev_out, alb_stats *st, WsGuard &guard,
                   RunOut &ro, Workspace *fixed = nullptr) {
  HIP_TRY(hipSetDevice(g->device));
  const hipStream_t stream = o.stream ? (hipStream_t)o.stream : g->stream;
  ro.stream = stream;
  const int wg = o.wg_size;

  int resident = 0;
  alb_status rs = resident_workgroups(g, job.op, wg, &resident);
  if (rs != ALB_OK) return rs;
  int launch = o.launch;
  if (launch == ALB_LAUNCH_AUTO) launch = ALB_LAUNCH_PERSISTENT;
  const int grid = o.grid_wgs > 0                ? o.grid_wgs
                   : o.grid_wgs == ALB_GRID_ALL ? resident
                                                : auto_grid(g->m, wg, resident);
  if (grid > resident)
    return fail(ALB_E_INVAL, "grid_wgs %d exceeds the %d workgroups the device can hold", grid, resident);
  // T: the host loop launches `grid` workgroups; the persistent launch learns
  // its member count on the device (reported after the run)
  int64_t T = (int64_t)grid * wg;

  int64_t threshold;
  if (o.mode == ALB_MODE_TWC_ONLY)
    threshold = INT64_MAX;
  else if (o.mode == ALB_MODE_LB_ALL)
    threshold = 0;
  else if (o.huge_threshold >= 0)
    threshold = o.huge_threshold;
  else if (o.huge_threshold == ALB_THRESHOLD_LAUNCHED)
    threshold = launch == ALB_LAUNCH_PERSISTENT ? -1 : T;  // the launched thread count (known on the device)
  else
    threshold = default_threshold(g->m, grid);
  // (the recorded single round of alb_trace_round keeps the base value)
  const bool adaptive = o.mode == ALB_MODE_ALB &&
                        (o.huge_threshold == ALB_THRESHOLD_ADAPTIVE ||
                         (o.huge_threshold == ALB_THRESHOLD_DEFAULT && job.op != OP_RECORD));
  const int64_t small_threshold = o.huge_threshold == ALB_THRESHOLD_ADAPTIVE
                                      ? (int64_t)kAdaptiveSmall
                                      : default_small_threshold(job.op, threshold);

  bool dedup = false;
  const Needs nd = job_needs(g, job, o, &dedup);
  const uint64_t qcap = nd.qcap;
  Workspace *ws = fixed;
  if (fixed) {
    if (fixed->qcap < nd.qcap || fixed->hint_cap < nd.hint_cap || fixed->n < g->n)
      return fail(ALB_E_INVAL, "internal: the fixed workspace is smaller than the call needs");
  } else {
    alb_status s = ws_acquire(g, nd, &ws);
    if (s != ALB_OK) return s;
    guard.g = g;
    guard.w = ws;
  }
  ro.ws = ws;
  ro.qcap = (uint32_t)qcap;

  Args a;
  std::memset(&a, 0, sizeof a);
  a.off = g->d_off;
  a.col = g->d_col;
  a.w = g->d_w;
  a.n = g->n;
  a.qcap = (uint32_t)qcap;  // the workspace may be larger; honour the requested capacity
  a.q0 = ws->q0;
  a.q1 = ws->q1;
  a.huge_rec = ws->huge_rec;
  a.hint = ws->hint;
  a.hint_cap = ws->hint_cap;
  a.bar = ws->bar;
  a.ctl = ws->ctl;
  a.threshold = threshold;
  a.c_wave = o.wave_cutoff;
  a.c_wg = o.wg_cutoff;
  a.dedup = dedup ? 1 : 0;
  a.adaptive = adaptive ? 1 : 0;
  a.small_threshold = small_threshold;
  a.blocked = o.distribution == 1;
  a.identity_first = job.identity_first;
  a.all_rounds = job.all_rounds;
  a.max_rounds = job.max_rounds;
  a.round = 0;
  a.timeout_ticks = g->clock_khz * barrier_timeout_ms();
  a.join_window_ticks = std::max<uint64_t>(g->clock_khz / 100, 1);  // 10 us without a new member
  a.profile = (getenv("ALB_TIMELINE") && !fixed) ? 1 : 0;
  if (job.op == OP_BFS) {
    a.level = dev_out ? (int32_t *)dev_out : ws->labels;
    // the reached-vertex bitmap lives in the label words, which BFS does not use
    const bool filter = o.visited_filter == 1 || (o.visited_filter == 0 && g->n >= kVisitedFilterMinVertices);
    if (filter && launch == ALB_LAUNCH_PERSISTENT) a.vbits = (uint32_t *)ws->word;
  }
  if (job.op == OP_SSSP || job.op == OP_CC) {
    a.word = ws->word;
    a.out = dev_out ? (int32_t *)dev_out : ws->labels;
  }
  if ((job.op == OP_CC || job.op == OP_KCORE) && o.visited_filter == 1 && launch == ALB_LAUNCH_PERSISTENT) {
    // only on request (CC gains on graphs whose vertex 0 sits in a giant
    // component, and costs elsewhere); the bitmap lives in the PageRank
    // accumulator, which CC and k-core do not use
    a.vbits = (uint32_t *)ws->acc;
  }
  if (job.op == OP_KCORE) {
    a.level = (int32_t *)ws->word;  // remaining degrees (ws->word has room for n int32)
    a.kcore_k = job.k;
    a.out = dev_out ? (int32_t *)dev_out : ws->labels;
  }
  if (job.op == OP_PR_PULL) {
    a.contrib = (float *)ws->labels;  // ws->labels has room for n fp32
    a.toff = g->d_toff;
    a.tcol = g->d_tcol;
  }
  if (job.op == OP_PR || job.op == OP_PR_PULL) {
    a.rank = dev_out ? (float *)dev_out : ws->rank;
    a.acc = ws->acc;
    a.damping = job.damping;
  }
  a.hits = job.d_hits;
  a.thread_of = job.d_thread;
  a.bins = job.d_bins;
  ro.d_labels = job.op == OP_BFS ? a.level : a.out;
  ro.d_rank = a.rank;

  if (job.h_frontier && job.nfront0)
    HIP_TRY(hipMemcpyAsync(ws->q0, job.h_frontier, sizeof(int32_t) * job.nfront0, hipMemcpyHostToDevice, stream));

  // profiling aid: per-round, per-workgroup edge counts (freed below)
  struct ProfBuf {
    uint32_t *p = nullptr;
    ~ProfBuf() { (void)hipFree(p); }
  } prof;
  if (a.profile && launch == ALB_LAUNCH_PERSISTENT) {
    const size_t nb = sizeof(uint32_t) * (size_t)kTimeline * kProfMembers;
    size_t pb = 0;
    HIP_TRY(dalloc(&prof.p, nb / sizeof(uint32_t), pb));
    HIP_TRY(hipMemsetAsync(prof.p, 0, nb, stream));
    a.prof_wg = prof.p;
  }
  if (ws->ev[0]) HIP_TRY(hipEventRecord(ws->ev[0], stream));
  if (job.op == OP_PR_PULL) {
    HIP_TRY(launch_init(OP_PR, a, -1, job.nfront0, stream));
    HIP_TRY(launch_pull_prepare(a, stream));
  } else {
    HIP_TRY(launch_init(job.op, a, job.source, job.nfront0, stream));
  }
  if (ws->ev[1]) HIP_TRY(hipEventRecord(ws->ev[1], stream));

  int launches = 0;
  int rounds = 0;
  if (launch == ALB_LAUNCH_PERSISTENT) {
    if (job.max_rounds > 0) {
      if (job.op == OP_PR_PULL)
        HIP_TRY(launch_pull_pr(wg, grid, a, stream));
      else
        HIP_TRY(launch_persistent(job.op, wg, grid, a, stream));
      launches = 1;
    }
  } else {
    for (int r = 0; r < job.max_rounds; ++r) {
      a.round = r;
      if (!job.all_rounds) {
        // the worklist for round r is known on the device; stop if empty
        HIP_TRY(hipMemcpyAsync(ws->h_ctl, ws->ctl, sizeof(Ctl), hipMemcpyDeviceToHost, stream));
        HIP_TRY(hipStreamSynchronize(stream));
        if (ws->h_ctl->overflow != 0xffffffffu) break;
        if (ws->h_ctl->qcount[r % 3] == 0) break;
      }
      HIP_TRY(launch_twc(job.op, wg, grid, a, stream));
      ++launches;
      HIP_TRY(hipMemcpyAsync(ws->h_ctl, ws->ctl, sizeof(Ctl), hipMemcpyDeviceToHost, stream));
      HIP_TRY(hipStreamSynchronize(stream));
      if (ws->h_ctl->overflow != 0xffffffffu) break;
      if ((ws->h_ctl->huge[r & 1] >> 32) != 0) {  // launch the LB kernel only when imbalance was found
        HIP_TRY(launch_lb(job.op, wg, grid, a, stream));
        ++launches;
      }
      if (job.op == OP_PR) {
        HIP_TRY(launch_pr_update(wg, grid, a, stream));
        ++launches;
      }
      rounds = r + 1;
    }
  }
  if (job.op == OP_SSSP || job.op == OP_CC || job.op == OP_KCORE) HIP_TRY(launch_finish(job.op, a, stream));
  if (ws->ev[2]) HIP_TRY(hipEventRecord(ws->ev[2], stream));
  HIP_TRY(hipMemcpyAsync(ws->h_ctl, ws->ctl, sizeof(Ctl), hipMemcpyDeviceToHost, stream));
  HIP_TRY(hipStreamSynchronize(stream));
  const Ctl &c = *ws->h_ctl;
  if (c.abort) return abort_error(c);
  if (launch == ALB_LAUNCH_PERSISTENT && launches) {
    T = (int64_t)c.n_members * wg;
    threshold = c.threshold_used;
  }
  if (c.overflow != 0xffffffffu)
    return fail(ALB_E_OVERFLOW, "a worklist exceeded its capacity of %u entries in round %u", a.qcap, c.overflow);
  if (launch == ALB_LAUNCH_PERSISTENT) {
    rounds = (int)c.rounds;
    if (getenv("ALB_TIMELINE")) {  // profiling aid: per-round phase times on stderr
      print_timeline(c, (int)job.op, rounds, (long long)threshold, g->clock_khz);
      if (prof.p) print_skew(prof.p, std::min(rounds, kTimeline), (int)std::min<uint32_t>(c.n_members, kProfMembers));
    }
  }
  if (!job.all_rounds && job.max_rounds > 1 && rounds >= job.max_rounds && c.qcount[rounds % 3] != 0)
    return fail(ALB_E_DEVICE, "no convergence within %d rounds", job.max_rounds);

  if (st) fill_stats(st, c, rounds, launches, T, threshold, ws->ev[0], ws->ev[1], ws->ev[2]);
  return ALB_OK;
}

alb_status check_graph(alb_graph g) {
  if (!g) return fail(ALB_E_INVAL, "graph handle is NULL");
  return ALB_OK;
}

// Traversal entry: run, then copy labels out (host outputs are synchronous).
alb_status traverse(alb_graph g, const Job &job, void *out, size_t elem, const alb_options *user, alb_stats *st) {
  alb_options o;
  alb_status s = resolve_options(user, o);
  if (s != ALB_OK) return s;
  WsGuard guard{nullptr, nullptr};
  RunOut ro;
  s = run_job(g, job, o, o.out_on_device ? out : nullptr, st, guard, ro);
  if (s != ALB_OK) return s;
  if (!o.out_on_device) {
    const void *src = (job.op == OP_PR || job.op == OP_PR_PULL) ? (const void *)ro.d_rank : (const void *)ro.d_labels;
    HIP_TRY(hipMemcpyAsync(out, src, elem * (size_t)g->n, hipMemcpyDeviceToHost, ro.stream));
    HIP_TRY(hipStreamSynchronize(ro.stream));
  }
  return ALB_OK;
}

// A batch of BFS or SSSP queries on a graph set, run in one persistent
// launch.  prepare_batch validates and lays out the per-query tables;
// upload_batch copies them to a workspace; enqueue_batch issues the device
// work (no host synchronisation, no allocation: it is what a captured graph
// replays); finish_batch waits, checks the control block and fills stats.
struct BatchJob {
  OpKind op = OP_BFS;
  alb_options o;
  int32_t count = 0;
  std::vector<long long> qoff, qthr, qlbase;
  std::vector<int32_t> qsrc, qn;
  std::vector<int32_t *> qout;  // filled once the workspace is known
  std::vector<int32_t> qcut;    // per query: wavefront and workgroup bin cutoffs
  bool per_query_thr = false, per_query_cut = false;
  long long labels = 0, edges = 0, thr_min = 0;
  int32_t max_n = 0;
  int32_t max_deg = 0;  // largest out-degree of the queries' members
  uint64_t qcap = 0;
  int grid = 0;
  int64_t threshold = 0;
  hipStream_t stream = nullptr;
  Args a;
};

// `cutoffs`: per query the wavefront and workgroup bin cutoffs ([2q], [2q + 1]), or null.
alb_status prepare_batch(alb_graph g, OpKind op, int32_t count, const int32_t *members, const int32_t *sources,
                         int32_t *const *outs, const int64_t *thresholds, const int32_t *cutoffs,
                         const alb_options *user, BatchJob &j) {
  if (!g) return fail(ALB_E_INVAL, "graph handle is NULL");
  if (count < 1 || count > kMaxBatch) return fail(ALB_E_INVAL, "count %d not in [1, %d]", count, kMaxBatch);
  if (!members || !sources || !outs) return fail(ALB_E_INVAL, "members, sources and outs must not be NULL");
  if (op == OP_SSSP && !g->weighted) return fail(ALB_E_INVAL, "SSSP needs a graph set created with weights");
  alb_options &o = j.o;
  alb_status s = resolve_options(user, o);
  if (s != ALB_OK) return s;
  if (o.launch == ALB_LAUNCH_HOST_LOOP) return fail(ALB_E_UNSUPPORTED, "batches run as one persistent launch only");
  if (thresholds && o.mode != ALB_MODE_ALB) return fail(ALB_E_INVAL, "per-query thresholds need mode ALB");
  if (cutoffs)
    for (int32_t q = 0; q < count; ++q)
      if (cutoffs[2 * q] < 1 || cutoffs[2 * q + 1] < 1)
        return fail(ALB_E_INVAL, "cutoffs of query %d must be >= 1", q);
  j.op = op;
  j.count = count;
  const int32_t nmem = (int32_t)g->mem_n.size();
  j.qoff.resize(count);
  j.qthr.resize(count);
  j.qlbase.resize(count);
  j.qsrc.resize(count);
  j.qn.resize(count);
  j.qout.assign(outs, outs + count);
  j.per_query_thr = thresholds != nullptr;
  j.per_query_cut = cutoffs != nullptr;
  if (cutoffs) j.qcut.assign(cutoffs, cutoffs + 2 * (size_t)count);
  long long labels = 0, edges = 0, thr_min = LLONG_MAX;
  int32_t max_n = 0;
  for (int32_t q = 0; q < count; ++q) {
    const int32_t mb = members[q];
    if (mb < 0 || mb >= nmem) return fail(ALB_E_INVAL, "members[%d] = %d out of range [0, %d)", q, mb, nmem);
    const int32_t n = g->mem_n[mb];
    if (sources[q] < 0 || sources[q] >= n)
      return fail(ALB_E_INVAL, "sources[%d] = %d out of range [0, %d)", q, sources[q], n);
    if (!outs[q]) return fail(ALB_E_INVAL, "outs[%d] is NULL", q);
    if (thresholds && thresholds[q] < 0) return fail(ALB_E_INVAL, "thresholds[%d] must be >= 0", q);
    j.qlbase[q] = labels;
    j.qoff[q] = labels - g->mem_vbase[mb];
    j.qsrc[q] = g->mem_vbase[mb] + sources[q];
    j.qn[q] = n;
    j.qthr[q] = thresholds ? thresholds[q] : 0;
    thr_min = std::min(thr_min, (long long)j.qthr[q]);
    labels += n;
    edges += g->mem_m[mb];
    max_n = std::max(max_n, n);
    j.max_deg = std::max(j.max_deg, g->mem_maxdeg[mb]);
  }
  j.labels = labels;
  j.edges = edges;
  j.thr_min = thresholds ? thr_min : 0;
  j.max_n = max_n;
  // every (query, vertex) enters a round's worklist at most once with the
  // per-round dedup, so one round holds at most `labels` entries and at most
  // `edges` huge edges, which the 32-bit worklist positions must hold
  const bool dedup = op == OP_BFS || o.dedup != 0;
  uint64_t qcap = o.worklist_capacity > 0 ? (uint64_t)o.worklist_capacity
                                          : (uint64_t)labels + (dedup ? 0 : (uint64_t)edges);
  qcap = std::max<uint64_t>(qcap, (uint64_t)count);
  if (qcap > 0xfffffffeULL || edges >= 0xffffffffLL)
    return fail(ALB_E_INVAL, "batch too large for 32-bit worklist positions (%lld labels, %lld edges): split it",
                labels, edges);
  j.qcap = qcap;

  HIP_TRY(hipSetDevice(g->device));
  j.stream = o.stream ? (hipStream_t)o.stream : g->stream;
  const int wg = o.wg_size;
  int resident = 0;
  s = resident_workgroups(g, op, wg, &resident, true);
  if (s != ALB_OK) return s;
  j.grid = o.grid_wgs > 0                ? o.grid_wgs
           : o.grid_wgs == ALB_GRID_ALL ? resident
                                        : auto_grid(edges, wg, resident);
  if (j.grid > resident)
    return fail(ALB_E_INVAL, "grid_wgs %d exceeds the %d workgroups the device can hold", j.grid, resident);
  if (o.mode == ALB_MODE_TWC_ONLY)
    j.threshold = INT64_MAX;
  else if (o.mode == ALB_MODE_LB_ALL)
    j.threshold = 0;
  else if (o.huge_threshold >= 0)
    j.threshold = o.huge_threshold;
  else if (o.huge_threshold == ALB_THRESHOLD_LAUNCHED)
    j.threshold = -1;
  else
    j.threshold = default_threshold(edges, j.grid);

  Args &a = j.a;
  std::memset(&a, 0, sizeof a);
  a.off = g->d_off;
  a.col = g->d_col;
  a.w = g->d_w;
  a.n = g->n;
  a.qcap = (uint32_t)qcap;
  a.threshold = j.threshold;
  a.c_wave = o.wave_cutoff;
  a.c_wg = o.wg_cutoff;
  a.dedup = dedup ? 1 : 0;
  a.adaptive = (!thresholds && o.mode == ALB_MODE_ALB &&
                (o.huge_threshold == ALB_THRESHOLD_ADAPTIVE || o.huge_threshold == ALB_THRESHOLD_DEFAULT))
                   ? 1
                   : 0;
  a.small_threshold = o.huge_threshold == ALB_THRESHOLD_ADAPTIVE ? (int64_t)kAdaptiveSmall
                                                                 : default_small_threshold(op, j.threshold);
  a.blocked = o.distribution == 1;
  a.max_rounds = max_n + 1;
  a.timeout_ticks = g->clock_khz * barrier_timeout_ms();
  a.join_window_ticks = std::max<uint64_t>(g->clock_khz / 100, 1);
  a.profile = getenv("ALB_TIMELINE") ? 1 : 0;
  a.nq = count;
  a.qthr_min = j.thr_min;
  a.nlabels = labels;
  return ALB_OK;
}

BatchNeeds batch_needs(const BatchJob &j) {
  return BatchNeeds{std::max<long long>(j.labels, 1), (uint32_t)j.qcap,
                    hint_entries(j.qcap, j.a.dedup ? j.edges : -1, j.max_deg), j.count};
}

// Point the job at workspace ws and copy its tables there (stream order).
// Host outputs are staged in ws->out32.
alb_status upload_batch(BatchJob &j, BatchWs *ws) {
  Args &a = j.a;
  a.q0 = ws->q0;
  a.q1 = ws->q1;
  a.huge_rec = ws->huge_rec;
  a.hint = ws->hint;
  a.hint_cap = ws->hint_cap;
  a.bar = ws->bar;
  a.ctl = ws->ctl;
  if (j.op == OP_BFS) a.level = (int32_t *)ws->word;
  if (j.op == OP_SSSP) a.word = ws->word;
  // the tables of this batch, packed with stride count: int64 arrays first,
  // then the output pointers, then the int32 arrays (every part stays
  // aligned to its element size)
  const size_t c = (size_t)j.count;
  long long *d_off = (long long *)ws->tab, *h_off = (long long *)ws->h_tab;
  int32_t **d_out = (int32_t **)(d_off + 3 * c), **h_out = (int32_t **)(h_off + 3 * c);
  int32_t *d_i32 = (int32_t *)(d_out + c), *h_i32 = (int32_t *)(h_out + c);
  for (size_t q = 0; q < c; ++q) {
    h_off[q] = j.qoff[q];
    h_off[c + q] = j.qthr[q];
    h_off[2 * c + q] = j.qlbase[q];
    h_out[q] = j.o.out_on_device ? j.qout[q] : ws->out32 + j.qlbase[q];
    h_i32[q] = j.qsrc[q];
    h_i32[c + q] = j.qn[q];
    h_i32[2 * c + 2 * q] = j.per_query_cut ? j.qcut[2 * q] : j.o.wave_cutoff;
    h_i32[2 * c + 2 * q + 1] = j.per_query_cut ? j.qcut[2 * q + 1] : j.o.wg_cutoff;
  }
  a.qoff = d_off;
  a.qthr = j.per_query_thr ? d_off + c : nullptr;
  a.qlbase = d_off + 2 * c;
  a.qout = d_out;
  a.qsrc = d_i32;
  a.qn = d_i32 + c;
  a.qcut = j.per_query_cut ? d_i32 + 2 * c : nullptr;
  const hipStream_t st = j.stream;
  HIP_TRY(hipMemcpyAsync(ws->tab, ws->h_tab, kBatchTableBytes * c, hipMemcpyHostToDevice, st));
  // the pinned mirror is rewritten by the next batch on this workspace: the
  // copy finishes first
  HIP_TRY(hipStreamSynchronize(st));
  return ALB_OK;
}

// The device work of one batch: initialise labels and seed the sources, run
// every round in one persistent launch, write the outputs, and copy the
// control block to the pinned mirror.
alb_status enqueue_batch(const BatchJob &j, BatchWs *ws, hipStream_t st) {
  HIP_TRY(launch_init_batch(j.op, j.a, st));
  HIP_TRY(launch_batch(j.op, j.o.wg_size, j.grid, j.a, st));
  HIP_TRY(launch_finish_batch(j.op, j.a, j.max_n, st));
  HIP_TRY(hipMemcpyAsync(ws->h_ctl, ws->ctl, sizeof(Ctl), hipMemcpyDeviceToHost, st));
  return ALB_OK;
}

// The device window of the last persistent batch launch of this thread (see
// alb::last_launch_window).
struct LaunchWindow {
  bool valid = false;
  double begin_ms = 0, end_ms = 0;
};
thread_local LaunchWindow g_window;

// After the stream reached the end of enqueue_batch: errors, host outputs, stats.
alb_status finish_batch(alb_graph g, const BatchJob &j, BatchWs *ws, int32_t *const *outs, alb_stats *st,
                        hipEvent_t e0, hipEvent_t e1, hipEvent_t e2) {
  const Ctl &c = *ws->h_ctl;
  g_window.valid = c.t_begin != 0 && c.t_end >= c.t_begin;
  g_window.begin_ms = (double)c.t_begin / (double)g->clock_khz;
  g_window.end_ms = (double)c.t_end / (double)g->clock_khz;
  if (c.abort) return abort_error(c);
  if (c.overflow != 0xffffffffu)
    return fail(ALB_E_OVERFLOW, "a worklist exceeded its capacity of %u entries in round %u", j.a.qcap, c.overflow);
  const int rounds = (int)c.rounds;
  if (getenv("ALB_TIMELINE")) print_timeline(c, (int)j.op, rounds, (long long)c.threshold_used, g->clock_khz);
  if (rounds >= j.a.max_rounds && c.qcount[rounds % 3] != 0)
    return fail(ALB_E_DEVICE, "no convergence within %d rounds", j.a.max_rounds);
  if (!j.o.out_on_device) {  // straight from the staging area into each query's host array
    for (int32_t q = 0; q < j.count; ++q)
      HIP_TRY(hipMemcpyAsync(outs[q], ws->out32 + j.qlbase[q], sizeof(int32_t) * (size_t)j.qn[q],
                             hipMemcpyDeviceToHost, j.stream));
    HIP_TRY(hipStreamSynchronize(j.stream));
  }
  if (st)
    fill_stats(st, c, rounds, 1, (int64_t)c.n_members * j.o.wg_size,
               j.per_query_thr ? -1 : (int64_t)c.threshold_used, e0, e1, e2);
  return ALB_OK;
}

// Per-query tuning records as threshold and cutoff arrays.
alb_status split_tuning(int32_t count, const alb_query_tuning *tuning, std::vector<int64_t> &thr,
                        std::vector<int32_t> &cut) {
  if (!tuning) return fail(ALB_E_INVAL, "tuning is NULL");
  if (count < 1 || count > kMaxBatch) return fail(ALB_E_INVAL, "count %d not in [1, %d]", count, kMaxBatch);
  thr.resize((size_t)count);
  cut.resize(2 * (size_t)count);
  for (int32_t q = 0; q < count; ++q) {
    thr[(size_t)q] = tuning[q].huge_threshold;
    cut[2 * (size_t)q] = tuning[q].wave_cutoff;
    cut[2 * (size_t)q + 1] = tuning[q].wg_cutoff;
  }
  return ALB_OK;
}


alb_status run_batch(alb_graph g, OpKind op, int32_t count, const int32_t *members, const int32_t *sources,
                     int32_t *const *outs, const int64_t *thresholds, const int32_t *cutoffs, const alb_options *user,
                     alb_stats *st) {
  g_window.valid = false;
  BatchJob j;
  alb_status s = prepare_batch(g, op, count, members, sources, outs, thresholds, cutoffs, user, j);
  if (s != ALB_OK) return s;
  BatchWs *ws = nullptr;
  s = bws_acquire(g, batch_needs(j), &ws);
  if (s != ALB_OK) return s;
  GuardOf<BatchWs> guard{g, ws};
  s = upload_batch(j, ws);
  if (s != ALB_OK) return s;
  const hipStream_t stream = j.stream;
  HIP_TRY(hipEventRecord(ws->ev[0], stream));
  HIP_TRY(launch_init_batch(op, j.a, stream));
  HIP_TRY(hipEventRecord(ws->ev[1], stream));
  HIP_TRY(launch_batch(op, j.o.wg_size, j.grid, j.a, stream));
  HIP_TRY(launch_finish_batch(op, j.a, j.max_n, stream));
  HIP_TRY(hipEventRecord(ws->ev[2], stream));
  HIP_TRY(hipMemcpyAsync(ws->h_ctl, ws->ctl, sizeof(Ctl), hipMemcpyDeviceToHost, stream));
  HIP_TRY(hipStreamSynchronize(stream));
  return finish_batch(g, j, ws, outs, st, ws->ev[0], ws->ev[1], ws->ev[2]);
}

// --------------------------------------------------------------------------
// Autotuner: per degree distribution, the huge threshold and workgroup size
// (and for one graph the TWC cutoffs) that ran a sample of queries fastest.
// --------------------------------------------------------------------------

struct TuneKey {
  int algo;
  int lg_n, lg_maxdeg;
  int64_t lg_m;
  std::array<uint8_t, 32> hist;
  bool operator<(const TuneKey &o) const {
    return std::tie(algo, lg_n, lg_maxdeg, lg_m, hist) < std::tie(o.algo, o.lg_n, o.lg_maxdeg, o.lg_m, o.hist);
  }
};

struct TuneCand {
  int32_t wg;
  int64_t threshold;
  int32_t c_wave, c_wg;
  double ms;
};

// best candidate per workgroup size, per key
std::mutex g_tune_mu;
std::map<TuneKey, std::vector<TuneCand>> g_tune;
// batch tuning: (algo, the batch's signatures) -> (workgroup size, threshold per signature)
std::map<std::pair<int, std::vector<TuneKey>>, std::pair<int32_t, std::map<TuneKey, int64_t>>> g_tune_batch;

int ilog2(int64_t x) { return x > 0 ? 63 - __builtin_clzll((unsigned long long)x) : -1; }

TuneKey tune_key(alb_graph g, OpKind op, int32_t member) {
  return TuneKey{(int)op, ilog2(g->mem_n[member]), ilog2(g->mem_maxdeg[member]), ilog2(g->mem_m[member]),
                 g->mem_hist[member]};
}

// Median device time of a batch of `k` queries on one member under options o.
// Median device time (3 runs after a warm-up) of a batch under options o and
// optional per-query thresholds; outputs go to the workspace's staging area.
alb_status time_batch(alb_graph g, OpKind op, int32_t count, const int32_t *members, const int32_t *sources,
                      const int64_t *thresholds, const int32_t *cutoffs, const alb_options &o, BatchWs *ws,
                      double *ms) {
  std::vector<int32_t *> outs((size_t)count, (int32_t *)ws);  // placeholders, replaced below
  alb_options oo = o;
  oo.out_on_device = 1;
  BatchJob j;
  alb_status s = prepare_batch(g, op, count, members, sources, outs.data(), thresholds, cutoffs, &oo, j);
  if (s != ALB_OK) return s;
  const BatchNeeds nd = batch_needs(j);
  if (ws->lab_cap < nd.labels || ws->qcap < nd.qcap || ws->hint_cap < nd.hint_cap || ws->nq_cap < nd.nq)
    return fail(ALB_E_INVAL, "tuning workspace too small");
  for (int32_t q = 0; q < count; ++q) j.qout[q] = ws->out32 + j.qlbase[q];
  s = upload_batch(j, ws);
  if (s != ALB_OK) return s;
  double t[4];
  for (int rep = 0; rep < 4; ++rep) {
    HIP_TRY(hipEventRecord(ws->ev[0], j.stream));
    s = enqueue_batch(j, ws, j.stream);
    if (s != ALB_OK) return s;
    HIP_TRY(hipEventRecord(ws->ev[2], j.stream));
    HIP_TRY(hipStreamSynchronize(j.stream));
    s = finish_batch(g, j, ws, nullptr, nullptr, ws->ev[0], ws->ev[0], ws->ev[2]);
    if (s != ALB_OK) return s;
    float f = 0.f;
    HIP_TRY(hipEventElapsedTime(&f, ws->ev[0], ws->ev[2]));
    t[rep] = f;
  }
  std::sort(t + 1, t + 4);  // the first run warms up
  *ms = t[2];
  return ALB_OK;
}

alb_status time_candidate(alb_graph g, OpKind op, int32_t member, int32_t k, const int32_t *sources,
                          const alb_options &o, BatchWs *ws, double *ms) {
  std::vector<int32_t> mb((size_t)k, member);
  return time_batch(g, op, k, mb.data(), sources, nullptr, nullptr, o, ws, ms);
}

// A workspace big enough for `count` queries of this batch.
alb_status batch_scratch(alb_graph g, OpKind op, int32_t count, const int32_t *members, const int32_t *sources,
                         const alb_options &base, BatchWs *ws) {
  alb_options probe = base;
  probe.out_on_device = 1;
  probe.wg_size = 1024;
  BatchJob pj;
  std::vector<int32_t *> dummy((size_t)count, (int32_t *)&pj);
  alb_status s = prepare_batch(g, op, count, members, sources, dummy.data(), nullptr, nullptr, &probe, pj);
  if (s != ALB_OK) return s;
  s = bws_fill(ws, batch_needs(pj));
  if (s != ALB_OK) {
    std::string keep = g_err;
    ws->release();
    g_err = keep;
  }
  return s;
}

// Tune one member (cached by its degree signature): for each workgroup size
// the fastest of the candidate thresholds; with `cutoffs`, then also two TWC
// cutoff pairs at the winner.
alb_status tune_member(alb_graph g, OpKind op, int32_t member, int32_t k, const int32_t *sources,
                       const alb_options &base, bool cutoffs, std::vector<TuneCand> *out) {
  const TuneKey key = tune_key(g, op, member);
  {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    auto it = g_tune.find(key);
    if (it != g_tune.end() && (!cutoffs || it->second.size() > 2)) {
      *out = it->second;
      return ALB_OK;
    }
  }
  std::vector<int32_t> mb((size_t)k, member);
  BatchWs ws;
  alb_status s = batch_scratch(g, op, k, mb.data(), sources, base, &ws);
  if (s != ALB_OK) return s;
  std::vector<TuneCand> best;
  static const int32_t wgs[] = {256, 1024};
  // the paper's threshold plateau (2^8 .. 2^18) sampled every factor of 4,
  // plus one wavefront's worth of edges
  static const int64_t thrs[] = {64, 256, 1024, 4096, 16384};
  for (int32_t wg : wgs) {
    TuneCand b{wg, 0, 64, wg, 1e30};
    for (int64_t t : thrs) {
      alb_options o = base;
      o.mode = ALB_MODE_ALB;
      o.wg_size = wg;
      o.huge_threshold = t;
      o.wave_cutoff = 64;
      o.wg_cutoff = wg;
      o.grid_wgs = 0;
      double ms = 0;
      s = time_candidate(g, op, member, k, sources, o, &ws, &ms);
      if (s != ALB_OK) break;
      if (ms < b.ms) b = TuneCand{wg, t, 64, wg, ms};
    }
    if (s != ALB_OK) break;
    best.push_back(b);
  }
  if (s == ALB_OK && cutoffs) {
    TuneCand w = best[0].ms <= best[1].ms ? best[0] : best[1];
    static const int32_t cw[][2] = {{32, 0}, {128, 0}, {64, -4}};  // -4: wg / 4
    TuneCand c = w;
    for (auto &p : cw) {
      alb_options o = base;
      o.mode = ALB_MODE_ALB;
      o.wg_size = w.wg;
      o.huge_threshold = w.threshold;
      o.wave_cutoff = p[0];
      o.wg_cutoff = p[1] < 0 ? w.wg / -p[1] : w.wg;
      o.grid_wgs = 0;
      double ms = 0;
      s = time_candidate(g, op, member, k, sources, o, &ws, &ms);
      if (s != ALB_OK) break;
      if (ms < c.ms) c = TuneCand{w.wg, w.threshold, o.wave_cutoff, o.wg_cutoff, ms};
    }
    best.push_back(c);
  }
  ws.release();
  if (s != ALB_OK) return s;
  std::lock_guard<std::mutex> lk(g_tune_mu);
  g_tune[key] = best;
  *out = best;
  return ALB_OK;
}

// --------------------------------------------------------------------------
// Batch plans: a batch laid out once and captured into a HIP graph.
// --------------------------------------------------------------------------

}  // namespace

struct alb_plan_s {
  alb_graph g = nullptr;
  BatchJob j;
  BatchWs ws;
  std::vector<int32_t *> outs;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  std::mutex mu;
  void release() {
    if (exec) (void)hipGraphExecDestroy(exec);
    if (graph) (void)hipGraphDestroy(graph);
    exec = nullptr;
    graph = nullptr;
    ws.release();
  }
};

namespace {

}  // namespace

// ==========================================================================
// C ABI
// ==========================================================================

extern "C" {

alb_status alb_options_init(alb_options *opt) {
  if (!opt) return fail(ALB_E_INVAL, "options pointer is NULL");
  *opt = defaults();
  return ALB_OK;
}

const char *alb_status_str(alb_status s) {
  switch (s) {
    case ALB_OK: return "ALB_OK";
    case ALB_E_INVAL: return "ALB_E_INVAL";
    case ALB_E_NOMEM: return "ALB_E_NOMEM";
    case ALB_E_DEVICE: return "ALB_E_DEVICE";
    case ALB_E_RANGE: return "ALB_E_RANGE";
    case ALB_E_OVERFLOW: return "ALB_E_OVERFLOW";
    case ALB_E_UNSUPPORTED: return "ALB_E_UNSUPPORTED";
    case ALB_E_TIMEOUT: return "ALB_E_TIMEOUT";
    case ALB_E_CANCELLED: return "ALB_E_CANCELLED";
  }
  return "ALB_E_UNKNOWN";
}

const char *alb_last_error(void) { return g_err.c_str(); }

}  // extern "C"

namespace {

std::array<uint8_t, 32> degree_signature(int32_t n, const int32_t *off, int32_t *maxdeg) {
  int64_t e[32] = {0}, m = 0;
  int32_t md = 0;
  for (int32_t v = 0; v < n; ++v) {
    const int32_t d = off[v + 1] - off[v];
    md = std::max(md, d);
    if (d > 0) e[31 - __builtin_clz((unsigned)d)] += d;
    m += d;
  }
  std::array<uint8_t, 32> h{};
  for (int k = 0; k < 32; ++k) h[k] = m ? (uint8_t)((8 * e[k] + m / 2) / m) : 0;
  *maxdeg = md;
  return h;
}

// Copy a validated host CSR to the device and make the handle.
alb_status make_graph(int32_t n, int64_t mm, const int32_t *off, const int32_t *cl, const int32_t *w, bool symmetric,
                      alb_graph *out, bool transpose = false) {
  int32_t maxd = 0;
  for (int32_t v = 0; v < n; ++v) maxd = std::max(maxd, off[v + 1] - off[v]);
  int dev = 0;
  HIP_TRY(hipGetDevice(&dev));
  alb_graph g = new (std::nothrow) alb_graph_s();
  if (!g) return fail(ALB_E_NOMEM, "host allocation failed");
  auto cleanup = [&](alb_status st) {
    (void)hipFree(g->d_off);
    (void)hipFree(g->d_col);
    (void)hipFree(g->d_w);
    (void)hipFree(g->d_toff);
    (void)hipFree(g->d_tcol);
    if (g->stream) (void)hipStreamDestroy(g->stream);
    delete g;
    return st;
  };
  g->n = n;
  g->m = mm;
  g->max_deg = maxd;
  g->symmetric = symmetric;
  g->weighted = (w != nullptr);
  g->device = dev;
  g->mem_vbase.assign(1, 0);
  g->mem_n.assign(1, n);
  g->mem_m.assign(1, mm);
  g->mem_maxdeg.assign(1, 0);
  g->mem_hist.assign(1, degree_signature(n, off, &g->mem_maxdeg[0]));
  int attr = 0;
  hipError_t e;
  if ((e = hipDeviceGetAttribute(&g->cus, hipDeviceAttributeMultiprocessorCount, dev)) != hipSuccess)
    return cleanup(fail(ALB_E_DEVICE, "hipDeviceGetAttribute: %s", hipGetErrorString(e)));
  if (hipDeviceGetAttribute(&attr, hipDeviceAttributeWallClockRate, dev) == hipSuccess && attr > 0)
    g->clock_khz = (uint64_t)attr;
  size_t bytes = 0;
  if ((e = dalloc(&g->d_off, (size_t)n + 1, bytes)) != hipSuccess ||
      (e = dalloc(&g->d_col, (size_t)mm, bytes)) != hipSuccess ||
      (w && (e = dalloc(&g->d_w, (size_t)mm, bytes)) != hipSuccess))
    return cleanup(fail(e == hipErrorOutOfMemory ? ALB_E_NOMEM : ALB_E_DEVICE, "hipMalloc: %s", hipGetErrorString(e)));
  if (transpose) {
    // in-edges of every vertex, sources ascending (counting sort)
    std::vector<int32_t> toff, tcol;
    try {
      toff.assign((size_t)n + 1, 0);
      tcol.resize((size_t)mm);
    } catch (const std::bad_alloc &) {
      return cleanup(fail(ALB_E_NOMEM, "host allocation failed"));
    }
    for (int64_t p = 0; p < mm; ++p) ++toff[(size_t)cl[p] + 1];
    for (int32_t v = 0; v < n; ++v) toff[(size_t)v + 1] += toff[(size_t)v];
    std::vector<int32_t> cur(toff.begin(), toff.end() - 1);
    for (int32_t u = 0; u < n; ++u)
      for (int32_t p = off[u]; p < off[u + 1]; ++p) tcol[(size_t)cur[(size_t)cl[p]]++] = u;
    if ((e = dalloc(&g->d_toff, (size_t)n + 1, bytes)) != hipSuccess ||
        (e = dalloc(&g->d_tcol, (size_t)mm, bytes)) != hipSuccess)
      return cleanup(fail(e == hipErrorOutOfMemory ? ALB_E_NOMEM : ALB_E_DEVICE, "hipMalloc: %s", hipGetErrorString(e)));
    if ((e = hipMemcpy(g->d_toff, toff.data(), sizeof(int32_t) * toff.size(), hipMemcpyHostToDevice)) != hipSuccess ||
        (mm && (e = hipMemcpy(g->d_tcol, tcol.data(), sizeof(int32_t) * (size_t)mm, hipMemcpyHostToDevice)) !=
                   hipSuccess))
      return cleanup(fail(ALB_E_DEVICE, "hipMemcpy: %s", hipGetErrorString(e)));
  }
  g->graph_bytes = bytes;
  if ((e = hipStreamCreateWithFlags(&g->stream, hipStreamNonBlocking)) != hipSuccess)
    return cleanup(fail(ALB_E_DEVICE, "hipStreamCreate: %s", hipGetErrorString(e)));
  if ((e = hipMemcpy(g->d_off, off, sizeof(int32_t) * ((size_t)n + 1), hipMemcpyHostToDevice)) != hipSuccess ||
      (mm && (e = hipMemcpy(g->d_col, cl, sizeof(int32_t) * (size_t)mm, hipMemcpyHostToDevice)) != hipSuccess) ||
      (w && mm && (e = hipMemcpy(g->d_w, w, sizeof(int32_t) * (size_t)mm, hipMemcpyHostToDevice)) != hipSuccess))
    return cleanup(fail(ALB_E_DEVICE, "hipMemcpy: %s", hipGetErrorString(e)));
  *out = g;
  return ALB_OK;
}

}  // namespace

extern "C" {

alb_status alb_graph_create(int32_t n, int64_t m, const int32_t *row_offsets, const int32_t *col,
                            const int32_t *weights, uint32_t flags, alb_graph *out) {
  if (!out) return fail(ALB_E_INVAL, "output handle pointer is NULL");
  *out = nullptr;
  if (flags & ~(uint32_t)(ALB_SYMMETRIC | ALB_BUILD_SYMMETRIC | ALB_BUILD_TRANSPOSE))
    return fail(ALB_E_INVAL, "unknown flags 0x%x", flags);
  alb_status s = validate_csr(n, m, row_offsets, col, weights);
  if (s != ALB_OK) return s;
  std::vector<int32_t> soff, scol;
  const int32_t *off = row_offsets, *cl = col, *w = weights;
  int64_t mm = m;
  if (flags & ALB_BUILD_SYMMETRIC) {
    s = symmetrise(n, row_offsets, col, soff, scol);
    if (s != ALB_OK) return s;
    off = soff.data();
    cl = scol.data();
    mm = (int64_t)scol.size();
    w = nullptr;
  }
  return make_graph(n, mm, off, cl, w, (flags & (ALB_SYMMETRIC | ALB_BUILD_SYMMETRIC)) != 0, out,
                    (flags & ALB_BUILD_TRANSPOSE) != 0);
}

alb_status alb_graph_create_set(int32_t count, const int32_t *ns, const int64_t *ms,
                                const int32_t *const *row_offsets, const int32_t *const *cols,
                                const int32_t *const *weights, alb_graph *out) {
  if (!out) return fail(ALB_E_INVAL, "output handle pointer is NULL");
  *out = nullptr;
  if (count < 1 || !ns || !ms || !row_offsets || !cols) return fail(ALB_E_INVAL, "bad graph-set arguments");
  int64_t tn = 0, tm = 0;
  for (int32_t i = 0; i < count; ++i) {
    alb_status s = validate_csr(ns[i], ms[i], row_offsets[i], cols[i], weights ? weights[i] : nullptr);
    if (s != ALB_OK) {
      std::string d = g_err;
      return fail(s, "member %d: %s", i, d.c_str());
    }
    if (weights && !weights[i] && ms[i] > 0) return fail(ALB_E_INVAL, "member %d has no weights", i);
    tn += ns[i];
    tm += ms[i];
  }
  if (tn >= ((int64_t)1 << 31) - 1 || tm >= ((int64_t)1 << 31))
    return fail(ALB_E_INVAL, "graph set too large (%lld vertices, %lld edges)", (long long)tn, (long long)tm);
  std::vector<int32_t> off, col, w;
  std::vector<int32_t> vbase(count), nn(count);
  std::vector<int64_t> mm(count);
  try {
    off.resize((size_t)tn + 1);
    col.resize((size_t)tm);
    if (weights) w.resize((size_t)tm);
  } catch (const std::bad_alloc &) {
    return fail(ALB_E_NOMEM, "host allocation failed");
  }
  int64_t vb = 0, eb = 0;
  for (int32_t i = 0; i < count; ++i) {
    vbase[i] = (int32_t)vb;
    nn[i] = ns[i];
    mm[i] = ms[i];
    for (int32_t v = 0; v < ns[i]; ++v) off[(size_t)(vb + v)] = (int32_t)(eb + row_offsets[i][v]);
    for (int64_t p = 0; p < ms[i]; ++p) col[(size_t)(eb + p)] = (int32_t)(vb + cols[i][p]);
    if (weights && ms[i]) std::memcpy(w.data() + eb, weights[i], sizeof(int32_t) * (size_t)ms[i]);
    vb += ns[i];
    eb += ms[i];
  }
  off[(size_t)tn] = (int32_t)tm;
  alb_status s = make_graph((int32_t)tn, tm, off.data(), col.data(), weights ? w.data() : nullptr, false, out);
  if (s != ALB_OK) return s;
  (*out)->mem_vbase = vbase;
  (*out)->mem_n = nn;
  (*out)->mem_m = mm;
  (*out)->mem_maxdeg.assign(count, 0);
  (*out)->mem_hist.resize(count);
  for (int32_t i = 0; i < count; ++i)
    (*out)->mem_hist[i] = degree_signature(ns[i], row_offsets[i], &(*out)->mem_maxdeg[i]);
  return ALB_OK;
}

alb_status alb_graph_members(alb_graph g, int32_t *count) {
  if (!g || !count) return fail(ALB_E_INVAL, "NULL argument");
  *count = (int32_t)g->mem_n.size();
  return ALB_OK;
}

alb_status alb_graph_member_info(alb_graph g, int32_t member, int32_t *n, int64_t *m, int32_t *vertex_base) {
  if (!g) return fail(ALB_E_INVAL, "graph handle is NULL");
  if (member < 0 || member >= (int32_t)g->mem_n.size()) return fail(ALB_E_INVAL, "member %d out of range", member);
  if (n) *n = g->mem_n[member];
  if (m) *m = g->mem_m[member];
  if (vertex_base) *vertex_base = g->mem_vbase[member];
  return ALB_OK;
}

alb_status alb_graph_destroy(alb_graph g) {
  if (!g) return ALB_OK;
  if (g->plans.load() > 0) return fail(ALB_E_INVAL, "%d batch plans still use this graph", g->plans.load());
  (void)hipSetDevice(g->device);
  if (g->stream) (void)hipStreamSynchronize(g->stream);
  for (Workspace *w : g->pool) {
    w->release();
    delete w;
  }
  for (BatchWs *w : g->batch_pool) {
    w->release();
    delete w;
  }
  (void)hipFree(g->d_off);
  (void)hipFree(g->d_col);
  (void)hipFree(g->d_w);
  (void)hipFree(g->d_toff);
  (void)hipFree(g->d_tcol);
  if (g->stream) (void)hipStreamDestroy(g->stream);
  delete g;
  return ALB_OK;
}

alb_status alb_graph_info(alb_graph g, int32_t *n, int64_t *m, int32_t *max_out_degree, size_t *device_bytes) {
  alb_status s = check_graph(g);
  if (s != ALB_OK) return s;
  if (n) *n = g->n;
  if (m) *m = g->m;
  if (max_out_degree) *max_out_degree = g->max_deg;
  if (device_bytes) {
    std::lock_guard<std::mutex> lk(g->mu);
    size_t b = g->graph_bytes;
    for (Workspace *w : g->pool) b += w->bytes;
    for (BatchWs *w : g->batch_pool) b += w->bytes;
    *device_bytes = b;
  }
  return ALB_OK;
}

alb_status alb_bfs(alb_graph g, int32_t source, int32_t *level, const alb_options *opt, alb_stats *stats) {
  zero_stats(stats);
  alb_status s = check_graph(g);
  if (s != ALB_OK) return s;
  if (!level) return fail(ALB_E_INVAL, "level is NULL");
  if (source < 0 || source >= g->n) return fail(ALB_E_INVAL, "source %d out of range [0, %d)", source, g->n);
  Job job;
  job.op = OP_BFS;
  job.source = source;
  job.nfront0 = 1;
  job.max_rounds = g->n + 1;
  s = traverse(g, job, level, sizeof(int32_t), opt, stats);
  if (s != ALB_OK) zero_stats(stats);
  return s;
}

alb_status alb_sssp(alb_graph g, int32_t source, int32_t *dist, const alb_options *opt, alb_stats *stats) {
  zero_stats(stats);
  alb_status s = check_graph(g);
  if (s != ALB_OK) return s;
  if (!dist) return fail(ALB_E_INVAL, "dist is NULL");
  if (!g->weighted) return fail(ALB_E_INVAL, "alb_sssp needs a graph created with weights");
  if (source < 0 || source >= g->n) return fail(ALB_E_INVAL, "source %d out of range [0, %d)", source, g->n);
  Job job;
  job.op = OP_SSSP;
  job.source = source;
  job.nfront0 = 1;
  job.max_rounds = g->n + 1;
  s = traverse(g, job, dist, sizeof(int32_t), opt, stats);
  if (s != ALB_OK) zero_stats(stats);
  return s;
}

// alb_sssp on the device scratch array: the same job and kernels, with the
// workspace carved from the scratch and the control block read back into a
// host stack copy.  One host mutex per device keeps calls from overlapping.
alb_status alb_sssp_noalloc(alb_graph g, int32_t source, int32_t *dist, const alb_options *opt, alb_stats *stats) {
  zero_stats(stats);
  alb_status s = check_graph(g);
  if (s != ALB_OK) return s;
  if (!dist) return fail(ALB_E_INVAL, "dist is NULL");
  if (!g->weighted) return fail(ALB_E_INVAL, "alb_sssp_noalloc needs a graph created with weights");
  if (source < 0 || source >= g->n) return fail(ALB_E_INVAL, "source %d out of range [0, %d)", source, g->n);
  alb_options o;
  if ((s = resolve_options(opt, o)) != ALB_OK) return s;
  Job job;
  job.op = OP_SSSP;
  job.source = source;
  job.nfront0 = 1;
  job.max_rounds = g->n + 1;
  bool dedup = false;
  const Needs nd = job_needs(g, job, o, &dedup);
  // the workspace, each part on a 256-byte boundary of the scratch
  size_t at = 0;
  auto take = [&](size_t bytes) {
    const size_t p = at;
    at += (bytes + 255) & ~(size_t)255;
    return p;
  };
  const size_t p_q0 = take(sizeof(int32_t) * (size_t)nd.qcap);
  const size_t p_q1 = take(sizeof(int32_t) * (size_t)nd.qcap);
  const size_t p_rec = take(sizeof(int4) * (size_t)nd.qcap);
  const size_t p_hint = take(sizeof(int2) * (size_t)nd.hint_cap);
  const size_t p_bar = take(sizeof(unsigned long long) * kBarWords);
  const size_t p_word = take(sizeof(unsigned long long) * (size_t)g->n);
  const size_t p_ctl = take(sizeof(Ctl));
  if (at > kNoAllocScratchBytes)
    return fail(ALB_E_NOMEM,
                "alb_sssp_noalloc: this graph and worklist capacity need %zu bytes of device scratch, the library "
                "holds %zu (n = %d, worklist capacity %u)",
                at, kNoAllocScratchBytes, g->n, nd.qcap);
  if (g->device < 0 || g->device >= 64) return fail(ALB_E_DEVICE, "device %d out of range", g->device);
  static std::mutex dev_mu[64];
  std::lock_guard<std::mutex> lk(dev_mu[g->device]);
  HIP_TRY(hipSetDevice(g->device));
  void *base = nullptr;
  HIP_TRY(noalloc_scratch(g->device, &base));
  unsigned char *b = (unsigned char *)base;
  Workspace ws;  // views into the scratch (never released)
  ws.n = g->n;
  ws.qcap = nd.qcap;
  ws.hint_cap = nd.hint_cap;
  ws.q0 = (int32_t *)(b + p_q0);
  ws.q1 = (int32_t *)(b + p_q1);
  ws.huge_rec = (int4 *)(b + p_rec);
  ws.hint = (int2 *)(b + p_hint);
  ws.bar = (unsigned long long *)(b + p_bar);
  ws.word = (unsigned long long *)(b + p_word);
  ws.ctl = (Ctl *)(b + p_ctl);
  Ctl host_ctl;
  ws.h_ctl = &host_ctl;
  WsGuard guard{nullptr, nullptr};
  RunOut ro;
  s = run_job(g, job, o, dist, stats, guard, ro, &ws);
  if (s != ALB_OK) zero_stats(stats);
  return s;
}

alb_status alb_cc(alb_graph g, int32_t *label, const alb_options *opt, alb_stats *stats) {
  zero_stats(stats);
  alb_status s = check_graph(g);
  if (s != ALB_OK) return s;
  if (!label) return fail(ALB_E_INVAL, "label is NULL");
  if (!g->symmetric) return fail(ALB_E_INVAL, "alb_cc needs a symmetric graph (ALB_SYMMETRIC or ALB_BUILD_SYMMETRIC)");
  Job job;
  job.op = OP_CC;
  job.identity_first = true;
  job.nfront0 = (uint32_t)g->n;
  job.max_rounds = g->n + 1;
  s = traverse(g, job, label, sizeof(int32_t), opt, stats);
  if (s != ALB_OK) zero_stats(stats);
  return s;
}

alb_status alb_kcore(alb_graph g, int32_t k, int32_t *in_core, const alb_options *opt, alb_stats *stats) {
  zero_stats(stats);
  alb_status s = check_graph(g);
  if (s != ALB_OK) return s;
  if (!in_core) return fail(ALB_E_INVAL, "in_core is NULL");
  if (k < 0) return fail(ALB_E_INVAL, "k must be >= 0");
  if (!g->symmetric)
    return fail(ALB_E_INVAL, "alb_kcore needs a symmetric graph (ALB_SYMMETRIC or ALB_BUILD_SYMMETRIC)");
  Job job;
  job.op = OP_KCORE;
  job.identity_first = true;
  job.nfront0 = (uint32_t)g->n;
  job.max_rounds = g->n + 1;
  job.k = k;
  s = traverse(g, job, in_core, sizeof(int32_t), opt, stats);
  if (s != ALB_OK) zero_stats(stats);
  return s;
}

alb_status alb_pagerank(alb_graph g, float damping, int32_t iterations, float *rank, const alb_options *opt,
                        alb_stats *stats) {
  zero_stats(stats);
  alb_status s = check_graph(g);
  if (s != ALB_OK) return s;
  if (!rank) return fail(ALB_E_INVAL, "rank is NULL");
  if (!(damping > 0.0f && damping < 1.0f)) return fail(ALB_E_INVAL, "damping must be in (0, 1)");
  if (iterations < 0) return fail(ALB_E_INVAL, "iterations must be >= 0");
  Job job;
  job.op = OP_PR;
  job.all_rounds = true;
  job.nfront0 = (uint32_t)g->n;
  job.max_rounds = iterations;
  job.damping = damping;
  s = traverse(g, job, rank, sizeof(float), opt, stats);
  if (s != ALB_OK) zero_stats(stats);
  return s;
}

alb_status alb_pagerank_pull(alb_graph g, float damping, int32_t iterations, float *rank, const alb_options *opt,
                             alb_stats *stats) {
  zero_stats(stats);
  alb_status s = check_graph(g);
  if (s != ALB_OK) return s;
  if (!rank) return fail(ALB_E_INVAL, "rank is NULL");
  if (!(damping > 0.0f && damping < 1.0f)) return fail(ALB_E_INVAL, "damping must be in (0, 1)");
  if (iterations < 0) return fail(ALB_E_INVAL, "iterations must be >= 0");
  if (!g->d_toff) return fail(ALB_E_INVAL, "alb_pagerank_pull needs a graph created with ALB_BUILD_TRANSPOSE");
  if (opt && opt->struct_size == sizeof(alb_options) && opt->launch == ALB_LAUNCH_HOST_LOOP)
    return fail(ALB_E_UNSUPPORTED, "pull PageRank runs as one persistent launch only");
  Job job;
  job.op = OP_PR_PULL;
  job.all_rounds = true;
  job.nfront0 = (uint32_t)g->n;
  job.max_rounds = iterations;
  job.damping = damping;
  s = traverse(g, job, rank, sizeof(float), opt, stats);
  if (s != ALB_OK) zero_stats(stats);
  return s;
}

alb_status alb_trace_round(alb_graph g, const int32_t *frontier, int64_t nf, const alb_options *user, int8_t *bins,
                           int32_t *work, int64_t *nwork, int64_t *prefix, int32_t *edge_hits, int32_t *edge_thread,
                           int32_t *next, int64_t *nnext, alb_stats *stats) {
  zero_stats(stats);
  alb_status s = check_graph(g);
  if (s != ALB_OK) return s;
  if (nf < 1 || nf > g->n) return fail(ALB_E_INVAL, "nf must be in [1, n]");
  if (!frontier || !bins || !work || !nwork || !prefix || !edge_hits || !edge_thread || !nnext)
    return fail(ALB_E_INVAL, "a required pointer is NULL");
  std::vector<int32_t> hoff((size_t)g->n + 1);
  HIP_TRY(hipSetDevice(g->device));
  HIP_TRY(hipMemcpy(hoff.data(), g->d_off, sizeof(int32_t) * hoff.size(), hipMemcpyDeviceToHost));
  int64_t sumdeg = 0;
  for (int64_t i = 0; i < nf; ++i) {
    if (frontier[i] < 0 || frontier[i] >= g->n) return fail(ALB_E_INVAL, "frontier[%lld] out of range", (long long)i);
    sumdeg += hoff[frontier[i] + 1] - hoff[frontier[i]];
  }
  if (sumdeg >= 0xfffffffeLL) return fail(ALB_E_INVAL, "frontier has too many edges for one traced round");
  alb_options o;
  s = resolve_options(user, o);
  if (s != ALB_OK) return s;
  o.out_on_device = 0;
  o.worklist_capacity = 0;
  size_t mm = (size_t)std::max<int64_t>(g->m, 1);
  int32_t *d_hits = nullptr, *d_thread = nullptr;
  int8_t *d_bins = nullptr;
  size_t scratch = 0;
  auto free_all = [&] {
    (void)hipFree(d_hits);
    (void)hipFree(d_thread);
    (void)hipFree(d_bins);
  };
  hipError_t e;
  if ((e = dalloc(&d_hits, mm, scratch)) != hipSuccess || (e = dalloc(&d_thread, mm, scratch)) != hipSuccess ||
      (e = dalloc(&d_bins, (size_t)nf, scratch)) != hipSuccess) {
    free_all();
    return fail(ALB_E_NOMEM, "hipMalloc: %s", hipGetErrorString(e));
  }
  Job job;
  job.op = OP_RECORD;
  job.nfront0 = (uint32_t)nf;
  job.max_rounds = 1;
  job.h_frontier = frontier;
  job.d_hits = d_hits;
  job.d_thread = d_thread;
  job.d_bins = d_bins;
  job.qcap_min = (uint32_t)std::max<int64_t>(sumdeg, nf);
  hipStream_t stream = o.stream ? (hipStream_t)o.stream : g->stream;
  if ((e = hipMemsetAsync(d_hits, 0, sizeof(int32_t) * mm, stream)) != hipSuccess ||
      (e = hipMemsetAsync(d_thread, 0xff, sizeof(int32_t) * mm, stream)) != hipSuccess) {
    free_all();
    return fail(ALB_E_DEVICE, "hipMemsetAsync: %s", hipGetErrorString(e));
  }
  WsGuard guard{nullptr, nullptr};
  RunOut ro;
  s = run_job(g, job, o, nullptr, stats, guard, ro);
  if (s != ALB_OK) {
    free_all();
    zero_stats(stats);
    return s;
  }
  Workspace *ws = ro.ws;
  const Ctl &c = *ws->h_ctl;
  const uint32_t vh = (uint32_t)(c.huge[0] >> 32), ehuge = (uint32_t)c.huge[0];
  const uint32_t nn = std::min(c.qcount[1], ro.qcap);
  std::vector<int4> hr(vh);
  bool ok = true;
  ok = ok && hipMemcpy(bins, d_bins, (size_t)nf, hipMemcpyDeviceToHost) == hipSuccess;
  ok = ok && (vh == 0 || hipMemcpy(hr.data(), ws->huge_rec, sizeof(int4) * vh, hipMemcpyDeviceToHost) == hipSuccess);
  ok = ok && (g->m == 0 || hipMemcpy(edge_hits, d_hits, sizeof(int32_t) * g->m, hipMemcpyDeviceToHost) == hipSuccess);
  ok = ok && (g->m == 0 || hipMemcpy(edge_thread, d_thread, sizeof(int32_t) * g->m, hipMemcpyDeviceToHost) == hipSuccess);
  ok = ok && (!next || nn == 0 || hipMemcpy(next, ws->q1, sizeof(int32_t) * nn, hipMemcpyDeviceToHost) == hipSuccess);
  free_all();
  if (!ok) {
    zero_stats(stats);
    return fail(ALB_E_DEVICE, "copy-out of the traced round failed");
  }
  *nwork = vh;
  for (uint32_t j = 0; j < vh; ++j) {
    work[j] = hr[j].z;
    prefix[j] = (uint32_t)hr[j].x;
  }
  prefix[vh] = ehuge;
  *nnext = nn;
  return ALB_OK;
}

alb_status alb_bfs_batch(alb_graph g, int32_t count, const int32_t *members, const int32_t *sources,
                         int32_t *const *levels, const int64_t *thresholds, const alb_options *opt, alb_stats *stats) {
  zero_stats(stats);
  alb_status s = run_batch(g, OP_BFS, count, members, sources, levels, thresholds, nullptr, opt, stats);
  if (s != ALB_OK) zero_stats(stats);
  return s;
}

alb_status alb_sssp_batch(alb_graph g, int32_t count, const int32_t *members, const int32_t *sources,
                          int32_t *const *dists, const int64_t *thresholds, const alb_options *opt, alb_stats *stats) {
  zero_stats(stats);
  alb_status s = run_batch(g, OP_SSSP, count, members, sources, dists, thresholds, nullptr, opt, stats);
  if (s != ALB_OK) zero_stats(stats);
  return s;
}

alb_status alb_bfs_batch_tuned(alb_graph g, int32_t count, const int32_t *members, const int32_t *sources,
                               int32_t *const *levels, const alb_query_tuning *tuning, const alb_options *opt,
                               alb_stats *stats) {
  zero_stats(stats);
  std::vector<int64_t> thr;
  std::vector<int32_t> cut;
  alb_status s = split_tuning(count, tuning, thr, cut);
  if (s == ALB_OK) s = run_batch(g, OP_BFS, count, members, sources, levels, thr.data(), cut.data(), opt, stats);
  if (s != ALB_OK) zero_stats(stats);
  return s;
}

alb_status alb_sssp_batch_tuned(alb_graph g, int32_t count, const int32_t *members, const int32_t *sources,
                                int32_t *const *dists, const alb_query_tuning *tuning, const alb_options *opt,
                                alb_stats *stats) {
  zero_stats(stats);
  std::vector<int64_t> thr;
  std::vector<int32_t> cut;
  alb_status s = split_tuning(count, tuning, thr, cut);
  if (s == ALB_OK) s = run_batch(g, OP_SSSP, count, members, sources, dists, thr.data(), cut.data(), opt, stats);
  if (s != ALB_OK) zero_stats(stats);
  return s;
}

alb_status alb_autotune(alb_graph g, int32_t algo, int32_t member, int32_t nsources, const int32_t *sources,
                        const alb_options *base, alb_options *tuned, double *best_ms) {
  if (!g || !tuned) return fail(ALB_E_INVAL, "graph handle and tuned must not be NULL");
  if (algo != ALB_ALGO_BFS && algo != ALB_ALGO_SSSP) return fail(ALB_E_UNSUPPORTED, "algo %d cannot be tuned", algo);
  if (member < 0 || member >= (int32_t)g->mem_n.size()) return fail(ALB_E_INVAL, "member %d out of range", member);
  if (nsources < 1 || nsources > 64 || !sources) return fail(ALB_E_INVAL, "nsources must be in [1, 64]");
  alb_options b;
  alb_status s = resolve_options(base, b);
  if (s != ALB_OK) return s;
  std::vector<TuneCand> r;
  s = tune_member(g, algo == ALB_ALGO_BFS ? OP_BFS : OP_SSSP, member, nsources, sources, b, true, &r);
  if (s != ALB_OK) return s;
  const TuneCand &c = r.back();
  b.mode = ALB_MODE_ALB;
  b.wg_size = c.wg;
  b.huge_threshold = c.threshold;
  b.wave_cutoff = c.c_wave;
  b.wg_cutoff = c.c_wg;
  *tuned = b;
  if (best_ms) *best_ms = c.ms;
  return ALB_OK;
}

}  // extern "C"

namespace {

// The batch autotuner's search (see alb_autotune_batch): stage 1 times one
// threshold for every query over the paper's plateau and both workgroup
// sizes; stage 2 moves the threshold of each of the largest degree-signature
// groups 4x down or up.  With `cutoffs`, stage 3 then tries other TWC cutoff
// pairs per group.  A change must gain at least 1 %.
struct BatchTune {
  int32_t wg = 256;
  std::map<TuneKey, int64_t> thr;
  std::map<TuneKey, std::pair<int32_t, int32_t>> cut;  // (wave, workgroup) cutoffs
  double uniform_ms = 0, best_ms = 0;
};

alb_status tune_batch(alb_graph g, OpKind op, int32_t count, const int32_t *members, const int32_t *sources,
                      const alb_options &b, bool cutoffs, BatchTune *out) {
  std::map<TuneKey, std::vector<int32_t>> groups;  // signature -> queries
  std::map<TuneKey, int64_t> group_edges;
  std::vector<TuneKey> key((size_t)count);
  for (int32_t q = 0; q < count; ++q) {
    key[(size_t)q] = tune_key(g, op, members[q]);
    groups[key[(size_t)q]].push_back(q);
    group_edges[key[(size_t)q]] += g->mem_m[members[q]];
  }
  BatchWs ws;
  alb_status s = batch_scratch(g, op, count, members, sources, b, &ws);
  if (s != ALB_OK) return s;
  std::vector<int64_t> thr((size_t)count);
  std::vector<int32_t> cut(2 * (size_t)count);
  auto run = [&](int32_t wg, bool with_cut, double *ms) {
    alb_options o = b;
    o.mode = ALB_MODE_ALB;
    o.wg_size = wg;
    o.wave_cutoff = 64;
    o.wg_cutoff = wg;
    o.grid_wgs = 0;
    return time_batch(g, op, count, members, sources, thr.data(), with_cut ? cut.data() : nullptr, o, &ws, ms);
  };
  static const int32_t wgs[] = {256, 1024};
  static const int64_t thrs[] = {256, 1024, 4096, 16384};
  double best = 1e30;
  int32_t best_wg = 256;
  int64_t best_t = 1024;
  for (int32_t wg : wgs) {
    for (int64_t t : thrs) {
      std::fill(thr.begin(), thr.end(), t);
      double ms = 0;
      s = run(wg, false, &ms);
      if (s != ALB_OK) break;
      if (ms < best) {
        best = ms;
        best_wg = wg;
        best_t = t;
      }
    }
    if (s != ALB_OK) break;
  }
  out->uniform_ms = best;
  std::map<TuneKey, int64_t> gthr;
  std::map<TuneKey, std::pair<int32_t, int32_t>> gcut;
  for (auto &kv : groups) {
    gthr[kv.first] = best_t;
    gcut[kv.first] = {64, best_wg};
  }
  std::vector<std::pair<int64_t, TuneKey>> order;
  for (auto &kv : group_edges) order.push_back({-kv.second, kv.first});
  std::sort(order.begin(), order.end());
  auto fill = [&] {
    for (int32_t q = 0; q < count; ++q) {
      thr[(size_t)q] = gthr[key[(size_t)q]];
      cut[2 * (size_t)q] = gcut[key[(size_t)q]].first;
      cut[2 * (size_t)q + 1] = gcut[key[(size_t)q]].second;
    }
  };
  for (size_t gi = 0; gi < order.size() && gi < 8 && s == ALB_OK; ++gi) {
    const TuneKey &k = order[gi].second;
    const int64_t cur = gthr[k];
    for (int64_t t : {cur / 4, cur * 4}) {
      if (t < 64 || t > ((int64_t)1 << 20)) continue;
      const int64_t keep = gthr[k];
      gthr[k] = t;
      fill();
      double ms = 0;
      s = run(best_wg, false, &ms);
      if (s != ALB_OK) break;
      if (ms < 0.99 * best)
        best = ms;
      else
        gthr[k] = keep;
    }
  }
  if (cutoffs) {
    for (size_t gi = 0; gi < order.size() && gi < 8 && s == ALB_OK; ++gi) {
      const TuneKey &k = order[gi].second;
      const std::pair<int32_t, int32_t> cands[] = {{32, best_wg}, {128, best_wg}, {64, 2 * best_wg}, {64, 4 * best_wg}};
      for (const auto &c : cands) {
        const auto keep = gcut[k];
        gcut[k] = c;
        fill();
        double ms = 0;
        s = run(best_wg, true, &ms);
        if (s != ALB_OK) break;
        if (ms < 0.99 * best)
          best = ms;
        else
          gcut[k] = keep;
      }
    }
  }
  ws.release();
  if (s != ALB_OK) return s;
  out->wg = best_wg;
  out->thr = gthr;
  out->cut = gcut;
  out->best_ms = best;
  return ALB_OK;
}

alb_status check_tune_args(alb_graph g, int32_t algo, int32_t count, const int32_t *members, const int32_t *sources) {
  if (!g || !members || !sources) return fail(ALB_E_INVAL, "NULL argument");
  if (algo != ALB_ALGO_BFS && algo != ALB_ALGO_SSSP) return fail(ALB_E_UNSUPPORTED, "algo %d cannot be tuned", algo);
  if (count < 1 || count > kMaxBatch) return fail(ALB_E_INVAL, "count %d not in [1, %d]", count, kMaxBatch);
  const int32_t nmem = (int32_t)g->mem_n.size();
  for (int32_t q = 0; q < count; ++q)
    if (members[q] < 0 || members[q] >= nmem) return fail(ALB_E_INVAL, "members[%d] out of range", q);
  return ALB_OK;
}

}  // namespace

extern "C" {

alb_status alb_autotune_batch(alb_graph g, int32_t algo, int32_t count, const int32_t *members,
                              const int32_t *sources, const alb_options *base, alb_options *tuned,
                              int64_t *thresholds) {
  if (!tuned || !thresholds) return fail(ALB_E_INVAL, "NULL argument");
  alb_status s = check_tune_args(g, algo, count, members, sources);
  if (s != ALB_OK) return s;
  alb_options b;
  s = resolve_options(base, b);
  if (s != ALB_OK) return s;
  const OpKind op = algo == ALB_ALGO_BFS ? OP_BFS : OP_SSSP;
  // cached by the batch's multiset of member signatures
  std::vector<TuneKey> sig;
  for (int32_t q = 0; q < count; ++q) sig.push_back(tune_key(g, op, members[q]));
  std::sort(sig.begin(), sig.end());
  const auto ckey = std::make_pair((int)op, sig);
  std::pair<int32_t, std::map<TuneKey, int64_t>> res;
  bool cached = false;
  {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    auto it = g_tune_batch.find(ckey);
    if (it != g_tune_batch.end()) {
      res = it->second;
      cached = true;
    }
  }
  if (!cached) {
    BatchTune bt;
    s = tune_batch(g, op, count, members, sources, b, false, &bt);
    if (s != ALB_OK) return s;
    res = std::make_pair(bt.wg, bt.thr);
    std::lock_guard<std::mutex> lk(g_tune_mu);
    g_tune_batch[ckey] = res;
  }
  b.mode = ALB_MODE_ALB;
  b.wg_size = res.first;
  b.wave_cutoff = 64;
  b.wg_cutoff = res.first;
  b.huge_threshold = ALB_THRESHOLD_DEFAULT;
  for (int32_t q = 0; q < count; ++q) thresholds[q] = res.second[tune_key(g, op, members[q])];
  *tuned = b;
  return ALB_OK;
}

alb_status alb_autotune_batch_tuned(alb_graph g, int32_t algo, int32_t count, const int32_t *members,
                                    const int32_t *sources, const alb_options *base, alb_options *tuned,
                                    alb_query_tuning *tuning, double *uniform_ms, double *tuned_ms) {
  if (!tuned || !tuning) return fail(ALB_E_INVAL, "NULL argument");
  alb_status s = check_tune_args(g, algo, count, members, sources);
  if (s != ALB_OK) return s;
  alb_options b;
  s = resolve_options(base, b);
  if (s != ALB_OK) return s;
  const OpKind op = algo == ALB_ALGO_BFS ? OP_BFS : OP_SSSP;
  BatchTune bt;
  s = tune_batch(g, op, count, members, sources, b, true, &bt);
  if (s != ALB_OK) return s;
  b.mode = ALB_MODE_ALB;
  b.wg_size = bt.wg;
  b.wave_cutoff = 64;
  b.wg_cutoff = bt.wg;
  b.huge_threshold = ALB_THRESHOLD_DEFAULT;
  for (int32_t q = 0; q < count; ++q) {
    const TuneKey k = tune_key(g, op, members[q]);
    tuning[q].huge_threshold = bt.thr[k];
    tuning[q].wave_cutoff = bt.cut[k].first;
    tuning[q].wg_cutoff = bt.cut[k].second;
  }
  *tuned = b;
  if (uniform_ms) *uniform_ms = bt.uniform_ms;
  if (tuned_ms) *tuned_ms = bt.best_ms;
  return ALB_OK;
}

alb_status alb_autotune_reset(void) {
  std::lock_guard<std::mutex> lk(g_tune_mu);
  g_tune.clear();
  g_tune_batch.clear();
  return ALB_OK;
}

}  // extern "C"

namespace {

alb_status plan_create(alb_graph g, int32_t algo, int32_t count, const int32_t *members, const int32_t *sources,
                       int32_t *const *outs, const int64_t *thresholds, const int32_t *cutoffs,
                       const alb_options *opt, alb_plan *out) {
  if (!out) return fail(ALB_E_INVAL, "output handle pointer is NULL");
  *out = nullptr;
  if (algo != ALB_ALGO_BFS && algo != ALB_ALGO_SSSP) return fail(ALB_E_UNSUPPORTED, "algo %d cannot be batched", algo);
  alb_plan p = new (std::nothrow) alb_plan_s();
  if (!p) return fail(ALB_E_NOMEM, "host allocation failed");
  auto bail = [&](alb_status st) {
    std::string keep = g_err;
    p->release();
    delete p;
    g_err = keep;
    return st;
  };
  alb_status s = prepare_batch(g, algo == ALB_ALGO_BFS ? OP_BFS : OP_SSSP, count, members, sources, outs, thresholds,
                               cutoffs, opt, p->j);
  if (s != ALB_OK) return bail(s);
  p->g = g;
  p->outs.assign(outs, outs + count);
  s = bws_fill(&p->ws, batch_needs(p->j));
  if (s != ALB_OK) return bail(s);
  s = upload_batch(p->j, &p->ws);
  if (s != ALB_OK) return bail(s);
  // capture on a private stream, so that nothing else issued meanwhile joins the graph
  hipStream_t cs = nullptr;
  hipError_t e = hipStreamCreateWithFlags(&cs, hipStreamNonBlocking);
  if (e != hipSuccess) return bail(fail(ALB_E_DEVICE, "hipStreamCreate: %s", hipGetErrorString(e)));
  e = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
  if (e == hipSuccess) {
    s = enqueue_batch(p->j, &p->ws, cs);
    hipError_t e2 = hipStreamEndCapture(cs, &p->graph);
    if (s == ALB_OK && e2 != hipSuccess) s = fail(ALB_E_DEVICE, "hipStreamEndCapture: %s", hipGetErrorString(e2));
  } else {
    s = fail(ALB_E_DEVICE, "hipStreamBeginCapture: %s", hipGetErrorString(e));
  }
  (void)hipStreamDestroy(cs);
  if (s != ALB_OK) return bail(s);
  e = hipGraphInstantiate(&p->exec, p->graph, nullptr, nullptr, 0);
  if (e != hipSuccess) return bail(fail(ALB_E_DEVICE, "hipGraphInstantiate: %s", hipGetErrorString(e)));
  g->plans.fetch_add(1);
  *out = p;
  return ALB_OK;
}

}  // namespace

extern "C" {

alb_status alb_batch_plan_create(alb_graph g, int32_t algo, int32_t count, const int32_t *members,
                                 const int32_t *sources, int32_t *const *outs, const int64_t *thresholds,
                                 const alb_options *opt, alb_plan *out) {
  return plan_create(g, algo, count, members, sources, outs, thresholds, nullptr, opt, out);
}

alb_status alb_batch_plan_create_tuned(alb_graph g, int32_t algo, int32_t count, const int32_t *members,
                                       const int32_t *sources, int32_t *const *outs, const alb_query_tuning *tuning,
                                       const alb_options *opt, alb_plan *out) {
  if (out) *out = nullptr;
  std::vector<int64_t> thr;
  std::vector<int32_t> cut;
  alb_status s = split_tuning(count, tuning, thr, cut);
  if (s != ALB_OK) return s;
  return plan_create(g, algo, count, members, sources, outs, thr.data(), cut.data(), opt, out);
}

alb_status alb_batch_plan_run(alb_plan p, alb_stats *stats) {
  zero_stats(stats);
  if (!p) return fail(ALB_E_INVAL, "plan handle is NULL");
  std::lock_guard<std::mutex> lk(p->mu);
  HIP_TRY(hipSetDevice(p->g->device));
  const hipStream_t st = p->j.stream;
  HIP_TRY(hipEventRecord(p->ws.ev[0], st));
  HIP_TRY(hipGraphLaunch(p->exec, st));
  HIP_TRY(hipEventRecord(p->ws.ev[2], st));
  HIP_TRY(hipStreamSynchronize(st));
  alb_status s = finish_batch(p->g, p->j, &p->ws, p->outs.data(), stats, p->ws.ev[0], p->ws.ev[0], p->ws.ev[2]);
  if (s != ALB_OK) zero_stats(stats);
  return s;
}

alb_status alb_batch_plan_destroy(alb_plan p) {
  if (!p) return ALB_OK;
  {
    std::lock_guard<std::mutex> lk(p->mu);
    (void)hipSetDevice(p->g->device);
    p->release();
  }
  p->g->plans.fetch_sub(1);
  delete p;
  return ALB_OK;
}

}  // extern "C"

namespace alb {

alb_status set_error(alb_status st, const char *fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_err = buf;
  return st;
}

bool last_launch_window(double *begin_ms, double *end_ms) {
  if (!g_window.valid) return false;
  *begin_ms = g_window.begin_ms;
  *end_ms = g_window.end_ms;
  return true;
}

alb_status batch_resident_workgroups(alb_graph g, int32_t algo, int32_t wg, int *out) {
  if (!g || !out) return fail(ALB_E_INVAL, "NULL argument");
  if (!supported_wg(wg)) return fail(ALB_E_UNSUPPORTED, "wg_size %d not built", wg);
  HIP_TRY(hipSetDevice(g->device));
  return resident_workgroups(g, algo == ALB_ALGO_BFS ? OP_BFS : OP_SSSP, wg, out, true);
}

// --------------------------------------------------------------------------
// Continuous serving: one lane's persistent launch that queries join between
// rounds (k_open), its workspace and the rings shared with it.
// --------------------------------------------------------------------------

struct OpenLane {
  alb_graph g = nullptr;
  alb_options o;
  OpKind op = OP_BFS;  // of the current launch
  int wg = 256, grid = 1, grid_cap = 1, resident = 1;
  int64_t max_m = 0;
  int32_t slots = 0;
  long long label_cap = 0;
  uint64_t qcap = 0;
  uint32_t hint_cap = 0;
  int64_t threshold = 0, small_threshold = 0;
  bool adaptive = false;
  // device
  unsigned long long *q0 = nullptr, *q1 = nullptr, *word = nullptr, *bar = nullptr;
  int4 *huge_rec = nullptr;
  int2 *hint = nullptr;
  long long *qoff = nullptr, *qlbase = nullptr;
  int32_t *qsrc = nullptr, *qn = nullptr, *q_last = nullptr, *q_active = nullptr, *q_admit = nullptr;
  int32_t *q_conv = nullptr;  // finished slots per round
  int32_t *q_unit = nullptr;  // per slot: BFS (unit weights)
  unsigned long long *q_out = nullptr;  // per slot: device address of its pinned output, or 0
  Ctl *ctl = nullptr;
  // pinned host
  OpenShared *sh = nullptr;     // coherent: read and written while the launch runs
  OpenShared *sh_dev = nullptr; // its device address
  Ctl *h_ctl = nullptr;
  // int32 labels of finished queries at their label indices: written by the
  // launch (over the bus) into pinned host memory, read by the host without
  // any copy command, so nothing waits behind the running launch
  int32_t *out = nullptr, *out_dev = nullptr;
  unsigned long long published = 0, completed = 0;
  size_t bytes = 0;
};

void open_lane_destroy(OpenLane *L) {
  if (!L) return;
  void *d[] = {L->q0, L->q1, L->word, L->bar, L->huge_rec, L->hint, L->qoff, L->qlbase, L->qsrc, L->qn,
               L->q_last, L->q_active, L->q_admit, L->q_conv, L->q_unit, L->q_out, L->ctl};
  for (void *x : d) (void)hipFree(x);
  if (L->sh) (void)hipHostFree(L->sh);
  if (L->h_ctl) (void)hipHostFree(L->h_ctl);
  if (L->out) (void)hipHostFree(L->out);
  delete L;
}

alb_status open_lane_create(alb_graph g, const alb_options &o, int32_t slots, long long label_cap, int grid_cap,
                            OpenLane **out) {
  *out = nullptr;
  if (!g) return fail(ALB_E_INVAL, "graph handle is NULL");
  if (slots < 1 || slots > kOpenRing) return fail(ALB_E_INVAL, "slots must be in [1, %d]", kOpenRing);
  if (label_cap < 1 || label_cap > 0xfffffffeLL) return fail(ALB_E_INVAL, "label capacity out of range");
  OpenLane *L = new (std::nothrow) OpenLane();
  if (!L) return fail(ALB_E_NOMEM, "host allocation failed");
  auto bail = [&](alb_status st) {
    open_lane_destroy(L);
    return st;
  };
  L->g = g;
  L->o = o;
  L->wg = o.wg_size ? o.wg_size : 256;
  L->grid_cap = grid_cap;
  L->slots = slots;
  L->label_cap = label_cap;
  L->qcap = (uint64_t)label_cap;  // every (slot, vertex) enters a round's worklist at most once
  if (!supported_wg(L->wg)) return bail(fail(ALB_E_UNSUPPORTED, "wg_size %d not built", L->wg));
  if (hipSetDevice(g->device) != hipSuccess) return bail(fail(ALB_E_DEVICE, "hipSetDevice failed"));
  int32_t max_n = 1;
  int32_t max_deg = 1;
  int64_t max_m = 0;
  for (size_t i = 0; i < g->mem_n.size(); ++i) {
    max_n = std::max(max_n, g->mem_n[i]);
    max_deg = std::max(max_deg, g->mem_maxdeg[i]);
    max_m = std::max(max_m, g->mem_m[i]);
  }
  // one round's huge edges stay below 2^32 (the host admits queries while
  // their members' edges sum below that)
  L->hint_cap = hint_entries(L->qcap, 0xfffffffeLL, max_deg);
  L->max_m = max_m;
  hipError_t e;
  const size_t S = (size_t)slots;
  if ((e = dalloc(&L->q0, L->qcap, L->bytes)) != hipSuccess || (e = dalloc(&L->q1, L->qcap, L->bytes)) != hipSuccess ||
      (e = dalloc(&L->huge_rec, L->qcap, L->bytes)) != hipSuccess ||
      (e = dalloc(&L->hint, L->hint_cap, L->bytes)) != hipSuccess ||
      (e = dalloc(&L->bar, kBarWords, L->bytes)) != hipSuccess ||
      (e = dalloc(&L->word, (size_t)label_cap, L->bytes)) != hipSuccess ||
      (e = dalloc(&L->qoff, S, L->bytes)) != hipSuccess || (e = dalloc(&L->qlbase, S, L->bytes)) != hipSuccess ||
      (e = dalloc(&L->qsrc, S, L->bytes)) != hipSuccess || (e = dalloc(&L->qn, S, L->bytes)) != hipSuccess ||
      (e = dalloc(&L->q_last, S, L->bytes)) != hipSuccess || (e = dalloc(&L->q_active, S, L->bytes)) != hipSuccess ||
      (e = dalloc(&L->q_admit, 2 * (size_t)kOpenRing, L->bytes)) != hipSuccess ||
      (e = dalloc(&L->q_conv, 2 * (size_t)kOpenRing, L->bytes)) != hipSuccess ||
      (e = dalloc(&L->q_unit, S, L->bytes)) != hipSuccess || (e = dalloc(&L->q_out, S, L->bytes)) != hipSuccess ||
      (e = dalloc(&L->ctl, 1, L->bytes)) != hipSuccess)
    return bail(fail(e == hipErrorOutOfMemory ? ALB_E_NOMEM : ALB_E_DEVICE, "hipMalloc: %s", hipGetErrorString(e)));
  if (alloc_failure_injected()) return bail(fail(ALB_E_NOMEM, "hipHostMalloc: out of memory"));
  if ((e = hipHostMalloc((void **)&L->sh, sizeof(OpenShared), hipHostMallocCoherent | hipHostMallocMapped)) !=
          hipSuccess ||
      (e = hipHostMalloc((void **)&L->h_ctl, sizeof(Ctl), hipHostMallocDefault)) != hipSuccess ||
      (e = hipHostMalloc((void **)&L->out, sizeof(int32_t) * (size_t)label_cap,
                         hipHostMallocCoherent | hipHostMallocMapped)) != hipSuccess)
    return bail(fail(e == hipErrorOutOfMemory ? ALB_E_NOMEM : ALB_E_DEVICE, "hipHostMalloc: %s",
                     hipGetErrorString(e)));
  std::memset((void *)L->sh, 0, sizeof(OpenShared));
  if ((e = hipHostGetDevicePointer((void **)&L->sh_dev, L->sh, 0)) != hipSuccess ||
      (e = hipHostGetDevicePointer((void **)&L->out_dev, L->out, 0)) != hipSuccess)
    return bail(fail(ALB_E_DEVICE, "hipHostGetDevicePointer: %s", hipGetErrorString(e)));
  *out = L;
  return ALB_OK;
}

// Start a launch on stream s (the previous one, if any, has ended): clear
// the rings and the device state, then the persistent kernel.
alb_status open_lane_start(OpenLane *L, hipStream_t s, double idle_us, int64_t edges) {
  alb_graph g = L->g;
  HIP_TRY(hipSetDevice(g->device));
  L->op = OP_SSSP;  // BFS queries run as unit-weight shortest paths beside the SSSP ones
  int resident = 0;
  alb_status st = resident_workgroups(g, L->op, L->wg, &resident, false, true);
  if (st != ALB_OK) return st;
  L->resident = resident;
  // the automatic grid of the work queued when the launch starts, at most
  // the lane's share: a grid barrier costs more the more workgroups join
  // it, and a stream of small queries wants few
  L->grid = std::max(1, std::min(auto_grid(std::max<int64_t>(edges, 1), L->wg, resident), L->grid_cap));
  const alb_options &o = L->o;
  if (o.mode == ALB_MODE_TWC_ONLY)
    L->threshold = INT64_MAX;
  else if (o.mode == ALB_MODE_LB_ALL)
    L->threshold = 0;
  else if (o.huge_threshold >= 0)
    L->threshold = o.huge_threshold;
  else if (o.huge_threshold == ALB_THRESHOLD_LAUNCHED)
    L->threshold = -1;
  else
    L->threshold = default_threshold(L->max_m, L->grid);
  L->adaptive = o.mode == ALB_MODE_ALB &&
                (o.huge_threshold == ALB_THRESHOLD_ADAPTIVE || o.huge_threshold == ALB_THRESHOLD_DEFAULT);
  L->small_threshold = o.huge_threshold == ALB_THRESHOLD_ADAPTIVE ? (int64_t)kAdaptiveSmall
                                                                  : default_small_threshold(L->op, L->threshold);
  std::memset((void *)L->sh, 0, sizeof(OpenShared));
  L->published = L->completed = 0;
  Args a;
  std::memset(&a, 0, sizeof a);
  a.off = g->d_off;
  a.col = g->d_col;
  a.w = g->d_w;
  a.n = g->n;
  a.qcap = (uint32_t)L->qcap;
  a.q0 = L->q0;
  a.q1 = L->q1;
  a.huge_rec = L->huge_rec;
  a.hint = L->hint;
  a.hint_cap = L->hint_cap;
  a.bar = L->bar;
  a.ctl = L->ctl;
  a.threshold = L->threshold;
  a.c_wave = o.wave_cutoff;
  a.c_wg = o.wg_cutoff;
  a.blocked = o.distribution == 1;
  a.dedup = o.dedup != 0;  // on unless turned off (the default for shortest paths)
  a.adaptive = L->adaptive ? 1 : 0;
  a.small_threshold = L->small_threshold;
  a.max_rounds = INT32_MAX;
  a.timeout_ticks = g->clock_khz * barrier_timeout_ms();
  a.join_window_ticks = std::max<uint64_t>(g->clock_khz / 100, 1);
  a.word = L->word;
  a.nq = L->slots;
  a.qoff = L->qoff;
  a.qlbase = L->qlbase;
  a.qsrc = L->qsrc;
  a.qn = L->qn;
  a.nlabels = L->label_cap;
  a.open = L->sh_dev;
  a.q_last = L->q_last;
  a.q_active = L->q_active;
  a.q_admit = L->q_admit;
  a.q_conv = L->q_conv;
  a.q_unit = L->q_unit;
  a.q_out = (int32_t **)L->q_out;
  a.open_out = L->out_dev;
  a.nslots = L->slots;
  a.idle_ticks = (uint64_t)std::max(1.0, idle_us * (double)g->clock_khz / 1000.0);
  HIP_TRY(launch_init_open(a, s));
  HIP_TRY(launch_open(L->op, L->wg, L->grid, a, s));
  return ALB_OK;
}

bool open_lane_running(OpenLane *L, hipStream_t s) {
  (void)L;
  return hipStreamQuery(s) == hipErrorNotReady;
}

// Requests the launch has not taken yet.
uint64_t open_lane_backlog(OpenLane *L) {
  const uint64_t head = __atomic_load_n(&L->sh->head, __ATOMIC_ACQUIRE);
  return L->published - head;
}

// Publish one request into `slot`, its labels at [lbase, lbase + n).
// The device address of pinned host memory (hipHostMalloc'd or registered
// with the runtime), or 0 for any other pointer.
static unsigned long long pinned_device_address(const void *p) {
  if (!p) return 0;
  hipPointerAttribute_t at;
  std::memset(&at, 0, sizeof at);
  const hipError_t e = hipPointerGetAttributes(&at, p);
  (void)hipGetLastError();  // an unregistered pointer leaves no error behind for the next caller
  if (e != hipSuccess || at.type != hipMemoryTypeHost || !at.devicePointer) return 0;
  return (unsigned long long)(uintptr_t)at.devicePointer;
}

alb_status open_lane_publish(OpenLane *L, int32_t algo, int32_t slot, int32_t member, int32_t source,
                             long long lbase, int32_t *host_out, bool *direct) {
  alb_graph g = L->g;
  *direct = false;
  if (member < 0 || member >= (int32_t)g->mem_n.size()) return fail(ALB_E_INVAL, "member out of range");
  if (algo == ALB_ALGO_SSSP && !g->weighted) return fail(ALB_E_INVAL, "SSSP needs a graph set created with weights");
  if (L->published - __atomic_load_n(&L->sh->head, __ATOMIC_ACQUIRE) >= (uint64_t)kOpenRing)
    return fail(ALB_E_INVAL, "request ring full");
  const unsigned long long out_dev = pinned_device_address(host_out);
  OpenReq &q = L->sh->req[L->published % kOpenRing];
  q.out = out_dev;
  *direct = out_dev != 0;
  q.slot = slot;
  q.unit = algo == ALB_ALGO_BFS ? 1 : 0;
  q.src = g->mem_vbase[member] + source;
  q.n = g->mem_n[member];
  q.qoff = lbase - g->mem_vbase[member];
  q.lbase = lbase;
  ++L->published;
  __atomic_store_n(&L->sh->tail, L->published, __ATOMIC_RELEASE);
  return ALB_OK;
}

// Slots whose query finished since the last call (at most max of them).
int32_t open_lane_poll(OpenLane *L, int32_t *slots, int32_t max) {
  const uint64_t done = __atomic_load_n(&L->sh->done, __ATOMIC_ACQUIRE);
  int32_t k = 0;
  while (L->completed < done && k < max) {
    slots[k++] = __atomic_load_n(&L->sh->fin[L->completed % kOpenRing], __ATOMIC_RELAXED);
    ++L->completed;
  }
  return k;
}

// Copy a finished query's labels (n of them from lbase) into the caller's
// host array.
// A finished query's int32 labels (n of them from lbase, already in pinned
// host memory) into the caller's host array.
void open_lane_copy_out(OpenLane *L, long long lbase, int32_t n, int32_t *out) {
  std::memcpy(out, L->out + lbase, sizeof(int32_t) * (size_t)n);
}

// After the launch's stream has finished: its status, and its device window.
alb_status open_lane_finish(OpenLane *L, hipStream_t s, double *begin_ms, double *end_ms) {
  HIP_TRY(hipMemcpyAsync(L->h_ctl, L->ctl, sizeof(Ctl), hipMemcpyDeviceToHost, s));
  HIP_TRY(hipStreamSynchronize(s));
  const Ctl &c = *L->h_ctl;
  *begin_ms = (double)c.t_begin / (double)L->g->clock_khz;
  *end_ms = (double)c.t_end / (double)L->g->clock_khz;
  if (getenv("ALB_TIMELINE"))  // profiling aid: the launch's first rounds on stderr
    print_timeline(c, (int)L->op, (int)c.rounds, (long long)c.threshold_used, L->g->clock_khz);
  if (c.abort) return abort_error(c);
  if (c.overflow != 0xffffffffu)
    return fail(ALB_E_OVERFLOW, "a worklist exceeded its capacity of %llu entries in round %u",
                (unsigned long long)L->qcap, c.overflow);
  return ALB_OK;
}

void open_lane_stop(OpenLane *L) { __atomic_store_n(&L->sh->stop, 1u, __ATOMIC_RELEASE); }

int open_lane_grid(const OpenLane *L) { return L->grid; }

int open_lane_grid_for(const OpenLane *L, int64_t edges) {
  return std::max(1, std::min(auto_grid(std::max<int64_t>(edges, 1), L->wg, L->resident), L->grid_cap));
}

int32_t open_lane_untaken(OpenLane *L, int32_t *slots, int32_t max) {
  const uint64_t head = __atomic_load_n(&L->sh->head, __ATOMIC_ACQUIRE);
  int32_t k = 0;
  for (uint64_t i = head; i < L->published && k < max; ++i) slots[k++] = L->sh->req[i % kOpenRing].slot;
  return k;
}

// Allocate `count` batch workspaces for batches of up to `labels` labels and
// `nq` queries and hand them back to g's pool, so that later batches of up
// to that size find one ready.  A workspace that a batch outgrows is freed
// and allocated anew, and freeing device memory waits for the device: done
// while a serving lane's batches run, it stalls the other lanes.
alb_status batch_reserve(alb_graph g, int count, long long labels, int32_t nq) {
  if (!g || count < 1 || labels < 1 || nq < 1) return ALB_OK;
  HIP_TRY(hipSetDevice(g->device));
  const uint32_t qcap = (uint32_t)std::min<long long>(std::max<long long>(labels, nq), 0xfffffffeLL);
  const BatchNeeds nd{labels, qcap, hint_entries(qcap, -1, g->max_deg), nq};
  std::vector<BatchWs *> held;
  alb_status st = ALB_OK;
  for (int i = 0; i < count && st == ALB_OK; ++i) {
    BatchWs *w = nullptr;
    st = bws_acquire(g, nd, &w);
    if (st == ALB_OK) held.push_back(w);
  }
  for (BatchWs *w : held) ws_release(g, w);
  return st;
}

static_assert(kOpenMaxSlots == kOpenRing, "the server's slot bound is the rings' size");

}  // namespace alb
