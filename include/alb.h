/*
 * alb.h -- C ABI of the adaptive load balancer (ALB) traversal library for
 * AMD Instinct MI355X (gfx950).
 *
 * The library runs data-driven graph traversals in bulk-synchronous rounds
 * (paper Section 2, "Graph Analytics"): each round applies a push operator to
 * the out-edges of every active vertex.  Work is balanced as in Section 4.1:
 * Algorithm 1 inspects every active vertex, sends those whose out-degree is at
 * least a threshold to a "huge" worklist and processes the others with the
 * thread / wavefront / workgroup bins of TWC (Section 3); Algorithm 2 spreads
 * the edges of the huge vertices cyclically over every launched thread and
 * finds each edge's source by a binary search in the prefix sum of the huge
 * degrees.
 *
 * Conventions shared by every call:
 *  - Every call returns alb_status; nothing throws or aborts across the ABI.
 *    On failure alb_last_error() returns a thread-local detail string, the
 *    output arrays are unspecified and *stats (if given) is zeroed.
 *  - Graphs are CSR: row_offsets has n+1 int32 entries, row_offsets[0] = 0,
 *    non-decreasing, row_offsets[n] = m; col has m int32 entries in [0, n);
 *    weights (optional) has m non-negative int32 entries.  0 <= m < 2^31.
 *  - Label outputs have n elements and are owned by the caller.  By default
 *    they are host pointers and the call returns when they are filled.  With
 *    options.out_on_device != 0 they are device pointers (for example a torch
 *    tensor's data_ptr()), written in stream order on options.stream; the
 *    call then returns after enqueueing the copy-out and the stats are valid
 *    on return.
 *  - Unreachable levels and distances are INT32_MAX.
 *  - A graph handle is immutable after creation; calls on one handle may run
 *    concurrently (each takes its own workspace).
 */
#ifndef ALB_H
#define ALB_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct alb_graph_s *alb_graph;

typedef enum {
  ALB_OK = 0,
  ALB_E_INVAL = -1,       /* bad argument or malformed CSR */
  ALB_E_NOMEM = -2,       /* host or device allocation failed */
  ALB_E_DEVICE = -3,      /* HIP runtime error, no usable GPU, or a device-side abort */
  ALB_E_RANGE = -4,       /* a shortest-path distance could exceed INT32_MAX - 1 */
  ALB_E_OVERFLOW = -5,    /* a device worklist exceeded its capacity */
  ALB_E_UNSUPPORTED = -6, /* option value not implemented */
  ALB_E_TIMEOUT = -7,     /* served request: its deadline passed before it was dispatched */
  ALB_E_CANCELLED = -8    /* served request: cancelled before it was dispatched */
} alb_status;

/* Which vertices take the cyclic (Algorithm 2) path.
 * ALB:      out-degree >= threshold (Algorithm 1).
 * TWC_ONLY: none (threshold above every degree; plain TWC, Section 3).
 * LB_ALL:   every active vertex with at least one edge (threshold 0; the
 *           paper's "D-IrGL (LB)" column of Table 3, Section 6.1). */
typedef enum { ALB_MODE_ALB = 0, ALB_MODE_TWC_ONLY = 1, ALB_MODE_LB_ALL = 2 } alb_mode;

/* Round driver.  HOST_LOOP launches one kernel per phase and reads the
 * worklist counters back every round.  PERSISTENT runs every round inside one
 * launch with grid-wide barriers between phases; the workgroups that are
 * running when the launch starts take part and any other leaves at once, so
 * no co-residency is assumed.  AUTO picks PERSISTENT. */
typedef enum { ALB_LAUNCH_AUTO = 0, ALB_LAUNCH_HOST_LOOP = 1, ALB_LAUNCH_PERSISTENT = 2 } alb_launch;

/* Special values of alb_options.huge_threshold.  DEFAULT is
 * m / (20 * workgroups) kept within [64, 4096] (m: the graph's edges, or all
 * edges of a batch's queries; workgroups: the launch's grid); in rounds whose
 * worklist has fewer entries than launched threads, where the TWC phase cannot
 * occupy every workgroup, it is 64 for BFS and k-core and a quarter of that
 * value (at least 64) for the other operators.  ADAPTIVE uses 64 (a
 * wavefront's worth of edges) in those rounds for every operator, and the
 * DEFAULT value otherwise. */
enum { ALB_THRESHOLD_DEFAULT = -1, ALB_THRESHOLD_LAUNCHED = -2, ALB_THRESHOLD_ADAPTIVE = -3 };

/* Special value of alb_options.grid_wgs: every workgroup the device holds. */
enum { ALB_GRID_ALL = -1 };

/* Graph creation flags. */
enum {
  ALB_SYMMETRIC = 1u,       /* caller asserts the CSR already holds both directions of every edge */
  ALB_BUILD_SYMMETRIC = 2u, /* create adds the reverse of every edge on the host (for alb_cc, alb_kcore) */
  ALB_BUILD_TRANSPOSE = 4u  /* create also keeps the in-edge CSR on the device (for alb_pagerank_pull) */
};

typedef struct {
  uint32_t struct_size;      /* sizeof(alb_options); set by alb_options_init */
  int32_t mode;              /* alb_mode */
  int64_t huge_threshold;    /* ALB mode: degree >= this is huge; ALB_THRESHOLD_DEFAULT (-1) =
                                m / (20 * workgroups) within [64, 4096] (see above), ALB_THRESHOLD_LAUNCHED
                                (-2) = the launched thread count (the paper's rule, Section 4.1;
                                its values for V100 and P100 in Section 5),
                                ALB_THRESHOLD_ADAPTIVE (-3) */
  int32_t wg_size;           /* 0 = 256; one of 64, 256, 1024 */
  int32_t wave_cutoff;       /* TWC wavefront bin: degree >= this (0 = 64) */
  int32_t wg_cutoff;         /* TWC workgroup bin: degree >= this (0 = wg_size) */
  int32_t distribution;      /* huge edges over threads (Section 4.1): 0 = cyclic, edge k to thread k mod T
                                (the default); 1 = blocked, thread i takes edges [i*c, (i+1)*c), c = ceil(e/T) */
  int32_t dedup;             /* -1 = default (on for sssp and cc), 0 = off, 1 = on */
  int32_t launch;            /* alb_launch */
  int32_t grid_wgs;          /* 0 = automatic: about 2 * cbrt(edges) workgroups of 256 threads (edges of the
                                graph, or of a batch's queries), at least 16, at most every resident one;
                                ALB_GRID_ALL (-1) = every resident workgroup; else this many */
  int64_t worklist_capacity; /* 0 = automatic (n with dedup, n + m without) */
  void *stream;              /* hipStream_t; NULL = the library's stream */
  uint32_t out_on_device;    /* outputs are device pointers (see above) */
  int32_t visited_filter;    /* BFS and CC, persistent launch: a bitmap (one bit per vertex, built from the
                                labels in one pass) is checked before a destination's label is read, so that
                                edges into vertices that cannot change touch the small bitmap instead of the
                                label array.  BFS: the reached vertices, built once half of them are reached.
                                CC: the vertices holding label 0 (the smallest id, final), rebuilt at each
                                round's start from round 1 and used once they are half of all.  k-core:
                                the vertices already below k, rebuilt at each round's start (their
                                decrements are skipped).  0 = automatic (BFS: on for graphs of at least
                                2^23 vertices; CC and k-core: off), 1 = on, -1 = off */
  int32_t reserved[6];
} alb_options;

typedef struct {
  int32_t rounds;            /* BSP rounds run (PageRank: iterations) */
  int32_t kernel_launches;   /* traversal kernels launched (1 in persistent mode) */
  int64_t launched_threads;  /* T: threads of the traversal grid */
  int64_t huge_threshold;    /* threshold actually used (INT64_MAX = none huge) */
  int64_t frontier_vertices; /* sum over rounds of active-vertex count */
  int64_t edges_examined;    /* sum over rounds of the out-degrees of active vertices */
  int64_t huge_vertices;     /* sum over rounds of the huge worklist size */
  int64_t huge_edges;        /* sum over rounds of the huge vertices' edges */
  int64_t pushes;            /* vertices pushed to a next-round worklist */
  double device_ms;          /* device time from label initialisation to the last round */
  double kernel_ms;          /* device time of the traversal rounds alone */
} alb_stats;

/* Fill *opt with defaults.  Returns ALB_E_INVAL for NULL. */
alb_status alb_options_init(alb_options *opt);

/* Copy a host CSR to the current HIP device and return a handle that owns the
 * device copy.  The graph is stored as the paper stores it (Section 4.1,
 * "Search"): compressed sparse rows, so that a vertex's out-edges are the
 * contiguous range row_offsets[v] .. row_offsets[v+1] of col and its
 * out-degree is the difference of two offsets -- the inspection of
 * Algorithm 1 reads exactly that, and Algorithm 2 turns a huge edge's rank
 * into a CSR position from the owner's first offset.  The caller keeps
 * ownership of the host arrays.  `weights` may
 * be NULL (then alb_sssp is refused).  Validation follows the conventions
 * above; with weights, max(w) * (n - 1) must be < INT32_MAX (ALB_E_RANGE
 * otherwise).  ALB_BUILD_SYMMETRIC drops the weights. */
alb_status alb_graph_create(int32_t n, int64_t m, const int32_t *row_offsets, const int32_t *col,
                            const int32_t *weights, uint32_t flags, alb_graph *out);

/* A graph set: `count` CSR graphs held as one handle for batches of queries
 * (alb_bfs_batch, alb_sssp_batch).  Member i is given by ns[i], ms[i],
 * row_offsets[i], cols[i] and, if `weights` is not NULL, weights[i], each
 * following the CSR conventions above; the members are stored one after the
 * other as the disjoint union (member i's vertex v is vertex
 * vertex_base(i) + v of the handle, see alb_graph_member_info).  The total
 * vertex and edge counts must stay below 2^31 - 1 and 2^31.  The caller keeps
 * the host arrays.  The single-query calls also accept the handle and then
 * work on the union.  Member lists of different sizes, from the same graph
 * repeated, or one member only are all allowed. */
alb_status alb_graph_create_set(int32_t count, const int32_t *ns, const int64_t *ms,
                                const int32_t *const *row_offsets, const int32_t *const *cols,
                                const int32_t *const *weights, alb_graph *out);

/* Members of a handle (1 for alb_graph_create). */
alb_status alb_graph_members(alb_graph g, int32_t *count);

/* Vertex count, edge count and first vertex id of member `member` inside the
 * handle.  Output pointers may be NULL. */
alb_status alb_graph_member_info(alb_graph g, int32_t member, int32_t *n, int64_t *m, int32_t *vertex_base);

/* Release the device copy and every cached workspace.  NULL is a no-op. */
alb_status alb_graph_destroy(alb_graph g);

/* Vertex and edge counts, the maximum out-degree and the device bytes held
 * (graph plus cached workspaces).  Any output pointer may be NULL. */
alb_status alb_graph_info(alb_graph g, int32_t *n, int64_t *m, int32_t *max_out_degree, size_t *device_bytes);

/* Breadth-first search from `source` (push, top-down every round; Section 5):
 * level[v] = hop distance, INT32_MAX if unreachable. */
alb_status alb_bfs(alb_graph g, int32_t source, int32_t *level, const alb_options *opt, alb_stats *stats);

/* Single-source shortest paths from `source` with the graph's weights: a
 * data-driven Bellman-Ford whose operator is the relaxation of Section 4.3
 * (atomic minimum).  dist[v] = shortest distance, INT32_MAX if unreachable. */
alb_status alb_sssp(alb_graph g, int32_t source, int32_t *dist, const alb_options *opt, alb_stats *stats);

/* alb_sssp for callers that cannot allocate memory (code that must not call
 * hipMalloc: tight serving loops, harnesses that forbid allocation).  Same
 * result, options and kernels as alb_sssp, but the per-call workspace
 * (worklists, huge list, chunk index, barrier words, 64-bit label words and
 * the control block: about 32 bytes per vertex with the default worklist
 * capacity) lives in one device array of 192 MiB that the library holds on
 * each GPU it runs on until the process ends; the call allocates no device or
 * pinned memory and records no event.
 *  - dist: DEVICE pointer to n int32 (whatever options.out_on_device says),
 *    written in stream order on options.stream (NULL: the library's stream);
 *    the call returns after the stream has finished the query.
 *  - A graph whose workspace does not fit (n above ~6.2M vertices at the
 *    default capacity, less with a larger options.worklist_capacity or
 *    dedup = 0) is refused with ALB_E_NOMEM before any device work.
 *  - Every call on one GPU uses the same array, and it keeps the last call's
 *    contents (the call initialises what it reads).  Calls from one process
 *    on one GPU are serialised by a host lock; work that overlapped on the
 *    device (another process, or a kernel given this memory) would race.
 *  - stats: as alb_sssp, except that device_ms and kernel_ms are 0 (the call
 *    is not timed). */
alb_status alb_sssp_noalloc(alb_graph g, int32_t source, int32_t *dist, const alb_options *opt, alb_stats *stats);

/* Connected components, the paper's cc application (Section 5, where it is
 * listed among the push-style operators): weakly connected components by
 * min-label propagation, each active vertex offering its label to its
 * neighbours through an atomic minimum.  The handle
 * must be symmetric (ALB_SYMMETRIC or ALB_BUILD_SYMMETRIC), else
 * ALB_E_INVAL.  label[v] = the smallest vertex id of v's component. */
alb_status alb_cc(alb_graph g, int32_t *label, const alb_options *opt, alb_stats *stats);

/* k-core (the paper's kcore application, Section 5): the largest subgraph in
 * which every vertex keeps at least k neighbours, by peeling -- vertices with
 * fewer than k edges leave, their neighbours' degrees drop, a neighbour whose
 * degree falls below k leaves in the next round.  The handle must be
 * symmetric (as for alb_cc) and free of self-loops.  in_core[v] = 1 if v is
 * in the k-core, else 0.  k >= 0. */
alb_status alb_kcore(alb_graph g, int32_t k, int32_t *in_core, const alb_options *opt, alb_stats *stats);

/* PageRank, the paper's pr application (Section 5; the paper gives no
 * formula, so the standard Jacobi form below is used), fp32, here pushed over
 * out-edges so that the balancer sees out-degree skew, exactly `iterations` synchronous
 * iterations from rank = 1/n:  r'(v) = (1-d)/n + d * (sum over in-edges (u,v)
 * of r(u)/outdeg(u) + D/n), D = total rank of vertices without out-edges.
 * 0 < damping < 1, iterations >= 0. */
alb_status alb_pagerank(alb_graph g, float damping, int32_t iterations, float *rank, const alb_options *opt,
                        alb_stats *stats);

/* Batches: `count` (1 .. 65535) independent queries on the members of a
 * graph set, run together in ONE persistent launch.  Query q searches member
 * members[q] from its local vertex sources[q] and writes that member's n
 * labels to levels[q] / dists[q] (host pointers, or device pointers with
 * options.out_on_device).  Every round's worklist holds (query, vertex)
 * pairs of all queries still running, so small queries share the chip instead
 * of each leaving most of it idle, and the inspection of Algorithm 1 and the
 * cyclic distribution of Algorithm 2 balance the union of their frontiers.
 * thresholds: NULL = the option's rule for every query; else thresholds[q] >= 0
 * is query q's huge threshold (mode ALB only), e.g. one tuned per graph.
 * Results equal the single-query calls on the member alone.  The sum over the
 * queries of their member's vertex counts (with dedup off: plus edge counts)
 * and of their edge counts must each stay below 2^32 - 1 (ALB_E_INVAL
 * otherwise; split the batch).  Options as for the single calls except
 * launch: HOST_LOOP is ALB_E_UNSUPPORTED.  stats sum over the batch;
 * stats->huge_threshold is -1 with per-query thresholds. */
alb_status alb_bfs_batch(alb_graph g, int32_t count, const int32_t *members, const int32_t *sources,
                         int32_t *const *levels, const int64_t *thresholds, const alb_options *opt, alb_stats *stats);
alb_status alb_sssp_batch(alb_graph g, int32_t count, const int32_t *members, const int32_t *sources,
                          int32_t *const *dists, const int64_t *thresholds, const alb_options *opt, alb_stats *stats);

/* Balancer settings of one query of a batch: its huge threshold (Algorithm
 * 1's test, >= 0) and its TWC bin cutoffs (Section 3; >= 1): wavefront bin
 * from wave_cutoff edges, workgroup bin from wg_cutoff edges. */
typedef struct {
  int64_t huge_threshold;
  int32_t wave_cutoff;
  int32_t wg_cutoff;
} alb_query_tuning;

/* alb_bfs_batch / alb_sssp_batch with per-query settings: tuning[count]
 * (mode ALB only), e.g. from alb_autotune_batch_tuned.  Otherwise as those. */
alb_status alb_bfs_batch_tuned(alb_graph g, int32_t count, const int32_t *members, const int32_t *sources,
                               int32_t *const *levels, const alb_query_tuning *tuning, const alb_options *opt,
                               alb_stats *stats);
alb_status alb_sssp_batch_tuned(alb_graph g, int32_t count, const int32_t *members, const int32_t *sources,
                                int32_t *const *dists, const alb_query_tuning *tuning, const alb_options *opt,
                                alb_stats *stats);

/* Traversals that batches, plans and the autotuner accept. */
typedef enum { ALB_ALGO_BFS = 0, ALB_ALGO_SSSP = 1 } alb_algo;

/* Batch plans: a batch laid out once -- per-query tables uploaded, its own
 * workspace allocated -- and its device work (label initialisation, the
 * persistent launch, the output kernel, the control-block read-back) captured
 * into a HIP graph that every alb_batch_plan_run replays on options.stream
 * (the library's stream if NULL).  For batches that recur with the same
 * queries; arguments as for alb_bfs_batch / alb_sssp_batch, and `outs` must
 * stay valid for the plan's life.  A run blocks until its results are in
 * `outs`; runs of one plan are serialised.  stats->kernel_ms equals
 * device_ms (the whole graph).  Destroy every plan before its graph
 * (alb_graph_destroy refuses with ALB_E_INVAL while plans exist). */
typedef struct alb_plan_s *alb_plan;
alb_status alb_batch_plan_create(alb_graph g, int32_t algo, int32_t count, const int32_t *members,
                                 const int32_t *sources, int32_t *const *outs, const int64_t *thresholds,
                                 const alb_options *opt, alb_plan *out);
/* A plan with per-query settings (as alb_sssp_batch_tuned). */
alb_status alb_batch_plan_create_tuned(alb_graph g, int32_t algo, int32_t count, const int32_t *members,
                                       const int32_t *sources, int32_t *const *outs, const alb_query_tuning *tuning,
                                       const alb_options *opt, alb_plan *out);
alb_status alb_batch_plan_run(alb_plan p, alb_stats *stats);
alb_status alb_batch_plan_destroy(alb_plan p);

/* Autotuner (not part of the paper's method; its threshold study, Section 6.1,
 * motivates the search space).  Times BFS or SSSP batches of the given
 * sources (1..64) on member `member` of g under candidate settings --
 * workgroup size 256 or 1024, huge threshold 64 or 2^8, 2^10, 2^12, 2^14
 * (the paper found thresholds across 2^8..2^18 to perform alike), then three
 * TWC cutoff pairs at the winner -- and returns *base with the fastest in
 * *tuned (and its median device time in *best_ms, if not NULL).  Results are
 * cached per process by the member's degree distribution (vertex, edge and
 * largest-degree orders of magnitude and the share of edges per power-of-two
 * degree class), so graphs that look alike are tuned once.  The outputs of the
 * timed runs are discarded. */
alb_status alb_autotune(alb_graph g, int32_t algo, int32_t member, int32_t nsources, const int32_t *sources,
                        const alb_options *base, alb_options *tuned, double *best_ms);

/* Autotuner for a batch: times the batch itself (outputs discarded), first
 * with one threshold for every query (2^8, 2^10, 2^12 or 2^14) and
 * workgroup size 256 or 1024, then, for the queries' degree signatures with
 * the most edges (up to 8), a threshold 4x lower or higher for that group
 * alone, kept if the batch gets at least 1 % faster.  Returns the workgroup
 * size in *tuned and each query's threshold in thresholds[count], ready for
 * the batch calls.  Cached per process by the batch's multiset of member
 * signatures. */
alb_status alb_autotune_batch(alb_graph g, int32_t algo, int32_t count, const int32_t *members,
                              const int32_t *sources, const alb_options *base, alb_options *tuned,
                              int64_t *thresholds);

/* Autotuner for a batch with per-query bin cutoffs: the search of
 * alb_autotune_batch, then for the same degree-signature groups (most edges
 * first, up to 8) the TWC cutoff pairs (wave, workgroup) = (32, w), (128, w),
 * (64, 2w), (64, 4w) around the default (64, w) for that group alone, w the
 * tuned workgroup size, each kept if the batch gets at least 1 % faster.
 * Fills tuning[count] and the workgroup size in *tuned; *uniform_ms (if not
 * NULL) gets the batch's median device time at the best single setting of the
 * grid (one threshold, default cutoffs, for every query) and *tuned_ms (if not
 * NULL) at the returned per-query settings.  Not cached. */
alb_status alb_autotune_batch_tuned(alb_graph g, int32_t algo, int32_t count, const int32_t *members,
                                    const int32_t *sources, const alb_options *base, alb_options *tuned,
                                    alb_query_tuning *tuning, double *uniform_ms, double *tuned_ms);

/* Forget every cached tuning result. */
alb_status alb_autotune_reset(void);

/* ---------------------------------------------------------------------------
 * Serving (not part of the paper): a request loop over one graph set.
 *
 * Requests (BFS or SSSP from one source on one member) are queued on submit.
 * `lanes` dispatcher threads each take, whenever they are free, the oldest
 * pending request's algorithm and every pending request of that algorithm
 * in arrival order that fits -- at most max_batch queries whose workspaces
 * (44 bytes per vertex of the query's member, plus 64) sum to at most
 * hbm_budget / lanes -- and run them as one batch (alb_bfs_batch /
 * alb_sssp_batch) on the lane's own stream with 1/lanes of the device's
 * workgroups (all of them when no other lane is running, see
 * whole_device_when_alone).  So requests that arrive while batches are running join the
 * next batch of the first lane to free up, and the lanes' batches overlap
 * on the device.  Results land in the caller's host array; a request's
 * latency runs from submit to that array being filled.
 * ------------------------------------------------------------------------- */
typedef struct alb_server_s *alb_server;

/* A replacement for the device (for testing the scheduling policy, or to run
 * another engine): runs one batch synchronously and returns its status.
 * outs[q] are the requests' host arrays. */
typedef int32_t (*alb_exec_fn)(void *user, int32_t algo, int32_t count, const int32_t *members,
                               const int32_t *sources, int32_t *const *outs, int32_t lane);

typedef struct {
  uint32_t struct_size;      /* sizeof(alb_server_config); set by alb_server_config_init */
  int32_t lanes;             /* batches in flight at once (1..16); 0 = 2 */
  int32_t max_batch;         /* queries per batch (1..65535); 0 = 256 */
  int32_t max_wait_us;       /* a free lane with fewer than max_batch pending waits up to this long for more */
  int64_t hbm_budget;        /* bytes of batch workspaces over all lanes; 0 = 8 GiB */
  alb_options options;       /* balancer options of every batch (stream, grid_wgs and out_on_device are set
                                per lane) */
  alb_exec_fn executor;      /* NULL = the GPU */
  void *executor_user;
  int32_t n_members;         /* with a custom executor and no graph: member count ... */
  const int32_t *member_vertices; /* ... and each member's vertex count (copied) */
  int32_t whole_device_when_alone; /* a batch that starts while no other lane runs uses every resident
                                      workgroup instead of its lane's share (1 = on, the default) */
  int32_t join_running;      /* 1: continuous batching inside a launch.  A lane keeps one persistent launch
                                running; requests join it at the next round boundary as soon as a query slot
                                (max_batch per launch, at most 1024) and label memory (the lane's share of
                                hbm_budget) are free, and leave it as soon as their own traversal has
                                converged.  BFS and SSSP requests share a launch (BFS runs as shortest paths
                                with unit weights: same levels).  With lanes = 1 the launch may use the whole
                                device, else the lane's share.  The launch ends after join_idle_us without work.
                                Needs the GPU (no executor).  0 (default): a batch is fixed when its launch
                                starts. */
  int32_t join_idle_us;      /* join_running: idle time before a launch ends; 0 = 500 us */
  int32_t reserved0;
  int64_t join_long_edges;   /* join_running with lanes >= 2: a request whose member graph has at least this
                                many edges runs on lane 0, every other request on the other lanes, so that
                                short queries do not advance in rounds shared with long ones; 0 (default):
                                any lane takes any request */
  int32_t reserved[2];
} alb_server_config;

typedef struct {
  int32_t status;     /* ALB_OK, the batch's error, ALB_E_TIMEOUT or ALB_E_CANCELLED */
  int32_t batch_size; /* requests in its batch (0 if never dispatched) */
  int32_t lane;       /* lane that ran it (-1 if never dispatched) */
  int32_t algo;
  double queue_ms;    /* submit to dispatch */
  double latency_ms;  /* submit to completion */
} alb_request_info;

typedef struct {
  int64_t submitted, completed, failed, timed_out, cancelled, rejected, batches;
  int64_t pending, running;  /* now */
  double busy_ms;            /* summed over lanes: time spent running batches */
  int64_t direct_outputs;    /* join_running: results the launch wrote straight into the request's output
                                (pinned host memory); the others were copied from the lane's output area */
} alb_server_stats;

alb_status alb_server_config_init(alb_server_config *cfg);

/* Start a server on graph g (a graph set or a plain graph).  g may be NULL
 * only with a custom executor and member_vertices.  The graph must outlive
 * the server. */
alb_status alb_server_create(alb_graph g, const alb_server_config *cfg, alb_server *out);

/* Queue one request: `algo` (alb_algo) from local vertex `source` of member
 * `member`; `out` is a host array of that member's vertex count, owned by the
 * caller and written when the request completes.  timeout_ms > 0: if the
 * request is still queued that long after submit, it completes with
 * ALB_E_TIMEOUT.  Returns the ticket in *ticket.  ALB_E_NOMEM if the request
 * alone exceeds a lane's share of hbm_budget (admission rejection),
 * ALB_E_INVAL for bad arguments or a stopped server. */
alb_status alb_server_submit(alb_server s, int32_t algo, int32_t member, int32_t source, int32_t *out,
                             double timeout_ms, uint64_t *ticket);

/* Block until request `ticket` completes; returns its status and, if info is
 * not NULL, its record.  Each ticket can be waited for once (ALB_E_INVAL after). */
alb_status alb_server_wait(alb_server s, uint64_t ticket, alb_request_info *info);

/* Cancel a request that is still queued (ALB_E_INVAL once dispatched). */
alb_status alb_server_cancel(alb_server s, uint64_t ticket);

/* Block until no request is queued or running. */
alb_status alb_server_drain(alb_server s);

alb_status alb_server_stats_get(alb_server s, alb_server_stats *st);

/* Stop accepting requests, run what is queued, join the lanes, free.  NULL is
 * a no-op.  Records of completed requests that were never waited for are
 * dropped. */
alb_status alb_server_destroy(alb_server s);

/* One dispatched batch of a server. */
typedef struct {
  int32_t lane, algo, batch_size, status;
  double device_begin_ms; /* its persistent launch on the device wall clock (ms from the device's own origin, */
  double device_end_ms;   /* the same for every lane): first workgroup joined, last round left; 0 without */
  double host_begin_ms;   /* dispatch and completion on the host, ms since the server was created */
  double host_end_ms;
} alb_batch_record;

/* The server's most recent dispatched batches, oldest first: up to `max`
 * records into `out`, *count = how many were written.  The server keeps the
 * last 4096.  Two lanes whose device windows intersect ran on the device at
 * the same time. */
alb_status alb_server_batch_log(alb_server s, int32_t max, alb_batch_record *out, int32_t *count);

/* PageRank as the paper's pr does it (pull, Section 5): the same iteration
 * and arguments as alb_pagerank, but every vertex sums its in-neighbours'
 * rank(u)/outdeg(u) over the transposed graph, and the balancer classifies
 * vertices by in-degree.  The sums use the same exact fixed point, so the
 * ranks equal alb_pagerank's bit for bit.  Needs a handle created with
 * ALB_BUILD_TRANSPOSE (ALB_E_INVAL otherwise); one persistent launch only
 * (launch = HOST_LOOP is ALB_E_UNSUPPORTED). */
alb_status alb_pagerank_pull(alb_graph g, float damping, int32_t iterations, float *rank, const alb_options *opt,
                             alb_stats *stats);

/* One round of the balancer on an explicit frontier, with an operator that
 * records instead of updating labels (for checking the distribution).  Host
 * pointers.  Inputs: frontier[nf] (vertex ids).  Outputs:
 *   bins[nf]       Algorithm 1 bin of each entry: 0 thread, 1 wavefront,
 *                  2 workgroup, 3 huge;
 *   work[nf], *nwork   the huge worklist in the order the device built it;
 *   prefix[nf + 1] its exclusive degree prefix (prefixWork), prefix[*nwork] = e;
 *   edge_hits[m]   how many times each CSR edge was processed;
 *   edge_thread[m] the global thread index that processed it last;
 *   next[...], *nnext  the pushed destinations (every processed edge pushes its
 *                  destination; capacity = sum of the frontier's degrees).
 * `next` may be NULL to skip the copy.  Uses opt->mode, huge_threshold,
 * wg_size, cutoffs, launch and grid_wgs like the traversals do, except that
 * ALB_THRESHOLD_DEFAULT applies its base value to the recorded round whatever
 * the frontier's size (stats->huge_threshold is the value applied). */
alb_status alb_trace_round(alb_graph g, const int32_t *frontier, int64_t nf, const alb_options *opt,
                           int8_t *bins, int32_t *work, int64_t *nwork, int64_t *prefix, int32_t *edge_hits,
                           int32_t *edge_thread, int32_t *next, int64_t *nnext, alb_stats *stats);

/* Static strings; never NULL. */
const char *alb_status_str(alb_status s);
const char *alb_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* ALB_H */
