// Internal interface between the host runtime (alb_api.cpp) and the device
// kernels (alb_kernels.hip).  Plain structs of device pointers and sizes.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace alb {

constexpr int32_t kInf = 0x7fffffff;
// Edges each lane keeps in flight; one pass of a B-thread workgroup over a
// vertex's edge list covers kEdgesPerLanePass * B edges.
#ifndef ALB_EDGES_PER_LANE
#define ALB_EDGES_PER_LANE 4
#endif
constexpr int kEdgesPerLanePass = ALB_EDGES_PER_LANE;
// PageRank sums: an fp32 contribution c is added as round(c * 2^60) to a
// 64-bit integer.  Integer addition is exact and associative, so the sum of a
// vertex's in-contributions does not depend on the order of the atomics, and
// the rounding is 2^-61 per term.  Every partial sum is at most the total rank
// mass (1), far below 2^64 / 2^60.
constexpr double kFixScale = 1152921504606846976.0;     // 2^60
constexpr double kFixInv = 1.0 / 1152921504606846976.0;  // 2^-60

// Grid barrier: each XCD (one L2) has an arrival counter, an open flag and
// the count of members it holds; the last arrival of an XCD arrives on the
// root counter, and the last root arrival bumps the generation word.  Each
// word sits on its own 256-byte line of the barrier buffer.  XCC_ID has 4
// bits, so up to 16 XCDs are provided for.
constexpr int kBarXcds = 16;
constexpr int kBarStride = 32;  // uint64 words per line
constexpr int kBarRoot = 0, kBarGen = kBarStride, kBarXcdArrive = 2 * kBarStride;
constexpr int kBarXcdFlag = kBarXcdArrive + kBarXcds * kBarStride;
constexpr int kBarXcdMembers = kBarXcdFlag + kBarXcds * kBarStride;
constexpr size_t kBarWords = (size_t)kBarXcdMembers + (size_t)kBarXcds * kBarStride;

// Huge-worklist chunk index: edge index k of the round's huge edges lies in
// chunk k >> hint_shift; hint[c] holds the huge-list slot that owns the first
// edge of chunk c and the end of that slot's edge range.  The shift is at
// least kHintMinShift.
constexpr int kHintMinShift = 10;
// Threshold of the explicit adaptive rule for rounds whose worklist cannot
// give every launched thread an entry: any vertex of at least a wavefront's
// worth of edges goes to the cyclic distribution, which keeps every
// workgroup busy.
constexpr int kAdaptiveSmall = 64;
// BFS turns its filter on by default from this many vertices (CC only on request)
// (a level array of 32 MB, eight times one XCD's L2; its bitmap is 32 times
// smaller).  Measured: -35 % kernel time on the Zipf graph of 2^24
// vertices; on RMAT scales 18 to 22 no gain, the filtering kernel 1-6 %
// slower than the plain one.
constexpr int32_t kVisitedFilterMinVertices = 1 << 23;
constexpr int kHintMaxShift = 20;
// Queries in one batch launch (the output kernel puts one query on each grid row).
constexpr int32_t kMaxBatch = 65535;
// Bytes of the per-GPU device scratch array that alb_sssp_noalloc carves its
// workspace from (worklists, huge list, chunk index, barrier words, label
// words, control block): about 32 bytes per vertex, so graphs of up to ~6.2M
// vertices with the default worklist capacity.
constexpr size_t kNoAllocScratchBytes = (size_t)192 << 20;

// Continuous serving (alb_server with join_running): requests join a running
// persistent batch launch between rounds; BFS and SSSP queries share it (BFS
// as shortest paths with unit weights, whose distances are the levels).  The
// host publishes requests in a ring of pinned, coherent host memory; the
// launch takes them at the end of a round's first phase into free query
// slots (label ranges assigned by the host) and publishes the slots whose
// query has finished in a second ring.
constexpr int kOpenRing = 1024;  // entries of each ring; also the most slots of one launch
struct OpenReq {
  int32_t slot;    // query slot in [0, slots)
  int32_t src;     // source vertex (graph-set id)
  int32_t n;       // vertices of its member
  int32_t unit;    // 1: BFS (every edge weighs 1), 0: SSSP with the graph's weights
  long long qoff;  // label index of (slot, vertex v) = qoff + v
  long long lbase; // first label index of the slot (= qoff + member base)
  unsigned long long out;  // device address of the caller's pinned int32 output, or 0 (open_out)
};
struct OpenShared {
  alignas(256) unsigned long long tail;  // requests published (host)
  alignas(256) unsigned long long head;  // requests taken (device)
  alignas(256) unsigned long long done;  // completions published (device)
  alignas(256) uint32_t stop;            // host: end the launch as soon as no query is active
  alignas(256) uint32_t live;            // device: 1 while the launch runs its rounds
  alignas(256) OpenReq req[kOpenRing];   // request i at req[i % kOpenRing]
  int32_t fin[kOpenRing];                // slot of completion i at fin[i % kOpenRing]
};

// Per-call control block in device memory.  Counters rotate by round so that
// one round can clear the counter two rounds ahead without a separate launch.
struct Ctl {
  uint32_t qcount[3];             // worklist sizes: round r reads [r % 3], pushes into [(r + 1) % 3]
  uint32_t overflow;              // first round in which a worklist overflowed (0xffffffff: none)
  unsigned long long huge[2];     // round r: (count << 32) | edge total of the huge worklist, [r & 1]
  uint32_t rounds;                // rounds completed (written by workgroup 0)
  uint32_t pad0;
  unsigned long long dangling[2]; // PageRank: rank mass without out-edges (fixed point), iteration it in [it & 1]
  alignas(256) unsigned long long chunk[3]; // worklist entries claimed in phase 1 of round r: [r % 3]
  alignas(256) uint32_t abort;    // a barrier wait timed out; every workgroup leaves
  uint32_t diag_round;            // round of the wait that timed out
  unsigned long long diag_seen;   // generation it observed
  unsigned long long diag_target; // generation it waited for
  unsigned long long members;     // persistent launch: tickets taken (top bit: membership closed)
  uint32_t n_members;             // member count, published when membership closes
  uint32_t pad1;
  long long threshold_used;       // huge threshold the persistent launch used
  alignas(256) unsigned long long st_frontier;  // statistics, summed over rounds
  unsigned long long st_edges_twc;
  unsigned long long st_edges_lb;
  unsigned long long st_huge_v;
  unsigned long long st_pushes;
  // per-round timeline of the persistent launch (first kTimeline rounds):
  // wall-clock ticks at round start, after the inspection/TWC phase and after
  // the execution phase, and (worklist size | huge count << 32)
  unsigned long long tl[4 * 64];
  // with Args::profile: wall-clock ticks summed over workgroups, per part of
  // the round (see kProf*)
  unsigned long long prof[8];
  // persistent launch: device wall-clock ticks when its first member joined
  // and when member 0 left the round loop
  unsigned long long t_begin, t_end;
  // reached-vertex filter: vertices whose bit the build of round r set, at [r & 1]
  unsigned long long filt_count[2];
  // continuous serving (member 0's bookkeeping): requests taken, slots
  // admitted in round r, its exit decision and the slots it converts
  // (finished in round r - 1), each at [r & 1] (a slow member may still read
  // round r's entry while member 0 writes round r + 1's), completions
  // published, active slots and the start of the current idle spell
  alignas(256) unsigned long long open_head;
  uint32_t admit_n[2];
  uint32_t open_exit[2];
  uint32_t conv_n[2];
  unsigned long long open_done;
  uint32_t open_active;
  unsigned long long idle_since;
};
constexpr int kTimeline = 64;
// With Args::prof_wg: edges each member workgroup processed in each of the
// first kTimeline rounds, for at most kProfMembers members.
constexpr int kProfMembers = 8192;
enum { kProfInspect = 0, kProfWgBin, kProfWaveBin, kProfThreadBin, kProfLb, kProfBarrier, kProfParts };

enum OpKind : int { OP_BFS = 0, OP_SSSP = 1, OP_CC = 2, OP_PR = 3, OP_RECORD = 4, OP_KCORE = 5, OP_PR_PULL = 6 };

// Everything a traversal kernel reads.  Passed by value.
struct Args {
  const int32_t *off;  // n + 1
  const int32_t *col;  // m
  const int32_t *w;    // m (SSSP)
  int32_t n;
  uint32_t qcap;        // capacity of each worklist and of the huge list
  void *q0;             // worklists (double buffered): int32 vertex ids, or (query << 32 | vertex) for a batch
  void *q1;
  int4 *huge_rec;       // huge list (Algorithm 1 `work`): per slot {prefixWork entry, CSR start, vertex, source value}
  int2 *hint;           // chunk index of the huge edges: {slot owning the chunk's first edge, end of its edges}
  uint32_t hint_cap;
  unsigned long long *bar;  // grid barrier words (kBarWords)
  Ctl *ctl;
  int64_t threshold;    // huge iff degree >= threshold (and degree >= 1); persistent: < 0 = launched threads
  int32_t c_wave;       // TWC cutoffs
  int32_t c_wg;
  int32_t dedup;        // SSSP / CC: push a vertex at most once per round
  int32_t adaptive;     // per-round threshold: small_threshold when the worklist has fewer entries than threads
  int64_t small_threshold;
  int32_t blocked;      // huge edges in contiguous runs per thread instead of cyclically
  int32_t identity_first;  // round 0 works on every vertex (no worklist)
  int32_t all_rounds;      // every round works on every vertex (PageRank)
  int32_t max_rounds;
  int32_t round;           // host-loop mode: the round this launch runs
  uint64_t timeout_ticks;  // barrier wait limit in wall-clock ticks
  uint64_t join_window_ticks;  // persistent launch: close membership after this long without a new member
  int32_t profile;         // accumulate Ctl::prof (profiling aid)
  uint32_t *prof_wg;       // profiling: [kTimeline][kProfMembers] edges per round and member, or null
  // operator state
  int32_t *level;       // BFS levels; k-core: remaining degrees
  uint32_t *vbits;      // BFS, CC: room for the filter bitmap (ceil(n / 32) words), or null: no filter
  int32_t kcore_k;      // k-core: k
  unsigned long long *word;  // SSSP / CC: (label << 32) | tag, tag = 1 + last round that lowered it
  int32_t *out;         // SSSP / CC: int32 labels written by the finishing kernel
  float *rank;          // PageRank: fp32 ranks
  float *contrib;       // pull PageRank: rank(u) / outdeg(u) of the current iteration
  const int32_t *toff;  // pull PageRank: transposed CSR (in-edges), n + 1
  const int32_t *tcol;  //   and m sources
  unsigned long long *acc;  // exact sums of fp32 contributions in 64-bit fixed point (kFix)
  float damping;
  int32_t *hits;        // trace operator
  int32_t *thread_of;
  int8_t *bins;
  // batch of queries sharing one launch (one graph set, see alb_graph_create_set)
  int32_t nq;
  const long long *qoff;   // label index of (query q, vertex v) = qoff[q] + v
  const long long *qthr;   // per-query huge thresholds, or null
  long long qthr_min;      // smallest of them
  const long long *qlbase; // first label index of query q
  const int32_t *qsrc;     // source vertex of query q (graph-set vertex id)
  const int32_t *qn;       // vertex count of query q's graph
  const int32_t *qcut;     // per-query TWC cutoffs: wavefront bin at [2q], workgroup bin at [2q + 1], or null
  int32_t *const *qout;    // output array of query q
  long long nlabels;       // labels of all queries
  // continuous serving: the shared rings (pinned host memory, device
  // address), per-slot round of the last worklist entry, active flags, and
  // how long an idle launch waits for work
  OpenShared *open;
  int32_t *q_last;
  int32_t *q_active;
  int32_t *q_admit;     // [2][kOpenRing]: slots admitted in round r ([r & 1])
  int32_t *q_unit;      // per slot: 1 = a BFS query, run as shortest paths with unit weights
  int32_t *q_conv;      // [2][kOpenRing]: slots whose labels round r writes to open_out ([r & 1])
  int32_t *open_out;    // int32 labels of finished queries, at the slot's label indices
  int32_t **q_out;      // per slot: the caller's pinned output (device address), or null: open_out
  int32_t nslots;
  uint64_t idle_ticks;
};

// Host-callable launchers (alb_kernels.hip).  All return the launch status.
hipError_t launch_init(OpKind op, const Args &a, int32_t source, uint32_t nfront0, hipStream_t s);
hipError_t launch_twc(OpKind op, int wg, int grid, const Args &a, hipStream_t s);
hipError_t launch_lb(OpKind op, int wg, int grid, const Args &a, hipStream_t s);
hipError_t launch_pr_update(int wg, int grid, const Args &a, hipStream_t s);
// Pull PageRank: every iteration in one persistent launch (after launch_init
// with OP_PR and launch_pull_prepare).
hipError_t launch_pull_pr(int wg, int grid, const Args &a, hipStream_t s);
hipError_t launch_pull_prepare(const Args &a, hipStream_t s);
hipError_t pull_occupancy(int wg, int *blocks_per_cu);
hipError_t launch_persistent(OpKind op, int wg, int grid, const Args &a, hipStream_t s);
// SSSP / CC: out[v] = word[v] >> 32; k-core: out[v] = (level[v] >= k).
hipError_t launch_finish(OpKind op, const Args &a, hipStream_t s);
// Workgroups of `wg` threads that fit on one CU for the persistent kernel of
// `op`, by the runtime's occupancy calculator (an upper bound: the launch
// itself finds out how many are co-resident).
hipError_t persistent_occupancy(OpKind op, int wg, int *blocks_per_cu);
bool supported_wg(int wg);
// Batches of BFS / SSSP queries on a graph set (Args::nq queries).
hipError_t batch_occupancy(OpKind op, int wg, int *blocks_per_cu);
hipError_t launch_init_batch(OpKind op, const Args &a, hipStream_t s);
hipError_t launch_batch(OpKind op, int wg, int grid, const Args &a, hipStream_t s);
hipError_t launch_finish_batch(OpKind op, const Args &a, int32_t max_n, hipStream_t s);
// Continuous serving: clear the control block, barrier words and slot flags
// (no query yet), then the persistent launch that admits queries from
// Args::open between rounds until it is idle for Args::idle_ticks or asked to
// stop (BFS and SSSP).
hipError_t launch_init_open(const Args &a, hipStream_t s);
hipError_t launch_open(OpKind op, int wg, int grid, const Args &a, hipStream_t s);
hipError_t open_occupancy(OpKind op, int wg, int *blocks_per_cu);
// Device address of this GPU's scratch array (kNoAllocScratchBytes, 256-byte
// aligned), looked up on the first call for `device` and kept (alb_noalloc.hip).
hipError_t noalloc_scratch(int device, void **ptr);

}  // namespace alb
