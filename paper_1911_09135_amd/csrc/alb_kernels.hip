// Device side of the adaptive load balancer (ALB) for gfx950 (wave64).
//
// One BSP round of a data-driven push traversal (paper Section 2) is two
// phases over the active worklist F:
//
//   phase 1  inspection + TWC (Algorithm 1, Section 3 "TWC").  Each workgroup
//            takes B consecutive entries of F.  A vertex whose out-degree is
//            >= threshold is appended to the huge list; its degree is added
//            to prefixWork in the same wave-aggregated 64-bit atomic, so the
//            exclusive prefix of the huge degrees (Section 4.1 "Search") is
//            known once the phase ends.  Every other vertex is processed at
//            once by the workgroup, wavefront or thread bin of its degree.
//   phase 2  execution (Algorithm 2), only when the huge list is non-empty
//            (Section 4.3).  Huge edge k goes to thread k mod T (the cyclic
//            distribution, Section 4.1), so the 64 lanes of a wavefront take
//            64 consecutive edges and read consecutive col / weight entries.
//            The source of edge k is the last prefixWork entry <= k.  The
//            search starts from a chunk index written when the huge list is
//            reserved (the slot owning the first edge of every 2^s-edge
//            chunk), so it costs one or two probes instead of log2(v) levels.
//
// Each lane keeps kU edges in flight: loads of all of them are issued before
// any operator decision, which hides the random-access latency of the
// destination labels.  The operator (BFS, SSSP, CC, PageRank, or a recorder
// for tests) is a template parameter.  Pushes to the next worklist are
// staged per wavefront in LDS and reserved in batches.
//
// Rounds are driven either from the host (one launch per phase) or inside one
// persistent launch whose phases are separated by a grid-wide barrier.

#include <type_traits>

#include "alb_internal.h"

namespace alb {
namespace {

constexpr int kWave = 64;
constexpr int kU = kEdgesPerLanePass;  // edges in flight per lane
constexpr uint32_t kPushBuf = 512;  // per-wavefront LDS staging of next-worklist pushes

__device__ __forceinline__ uint32_t lane_id() {
  return __builtin_amdgcn_mbcnt_hi(~0u, __builtin_amdgcn_mbcnt_lo(~0u, 0u));
}
// number of set bits of m below this lane
__device__ __forceinline__ uint32_t bits_below(unsigned long long m) {
  return __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
}

template <class T>
__device__ __forceinline__ T ld_relaxed(T *p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
template <class T>
__device__ __forceinline__ void st_relaxed(T *p, T v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
template <class T>
__device__ __forceinline__ T add_relaxed(T *p, T v) {
  return __hip_atomic_fetch_add(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Overflow is recorded as the first round in which it happened; a workgroup
// stops at the start of a later round, so every workgroup decides alike.
__device__ __forceinline__ void flag_overflow(Ctl *c, int round) {
  __hip_atomic_fetch_min(&c->overflow, (uint32_t)round, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// fp32 value -> 64-bit fixed point (round to nearest)
__device__ __forceinline__ unsigned long long to_fix(float x) { return __double2ull_rn((double)x * kFixScale); }

template <class V>
__device__ __forceinline__ int32_t to_bits(V x) {
  return __builtin_bit_cast(int32_t, x);
}
template <class V>
__device__ __forceinline__ V from_bits(int32_t x) {
  return __builtin_bit_cast(V, x);
}

// ---------------------------------------------------------------------------
// Operators.  The work along one edge is split into prepare() (issue the loads
// it needs) and commit() (decide, update the destination, and say whether the
// destination goes to the next worklist), so that a lane can have kU edges'
// loads in flight before the first decision.
// ---------------------------------------------------------------------------

// Label indices (long long) address the label arrays: the vertex id for a
// single query; query offset + vertex id for a batch of queries sharing one
// launch.  Graph indices (CSR positions, vertex ids) are separate.

// BFS: level[dst] = level[src] + 1 on first visit (compare-and-swap from INF).
// Every active vertex of round r has level r, so no source level is read.
struct OpBFS {
  using val_t = int32_t;
  struct pre_t {
    int32_t cur;
  };
  static constexpr bool kPush = true, kNeedSrc = false, kRecord = false, kPR = false, kBatch = true;
  int32_t *level;
  __device__ __forceinline__ val_t load_src(long long, int32_t, uint32_t tag, bool &) const {
    return (int32_t)tag - 1;
  }
  __device__ __forceinline__ pre_t prepare(int32_t, long long dl, val_t, int32_t) const { return {level[dl]}; }
  __device__ __forceinline__ bool commit(const pre_t &p, int32_t, long long dl, val_t sv, int32_t, int32_t,
                                         uint32_t) const {
    if (p.cur != kInf) return false;
    int32_t expected = kInf;
    return __hip_atomic_compare_exchange_strong(&level[dl], &expected, sv + 1, __ATOMIC_RELAXED, __ATOMIC_RELAXED,
                                                __HIP_MEMORY_SCOPE_AGENT);
  }
};

// BFS once the persistent launch has built the reached-vertex bitmap: a
// destination whose bit is set has been reached and its level is not read
// (a clear bit says nothing: the level decides).  A type of its own, so that
// the rounds before the bitmap exists run the plain operator's code.
struct OpBFSFilter : OpBFS {
  const uint32_t *vbits;
  __device__ __forceinline__ pre_t prepare(int32_t, long long dl, val_t, int32_t) const {
    if ((vbits[dl >> 5] >> (dl & 31)) & 1u) return {0};
    return {level[dl]};
  }
};

// SSSP and CC keep one 64-bit word per vertex: (label << 32) | tag, where tag
// is 1 + the round that last lowered the label.  A relaxation in round r
// offers (candidate << 32) | (r + 1) to an atomic minimum: it lowers the word
// exactly when the candidate is smaller (an equal candidate never changes the
// word, its tag being no smaller), and the old word says both whether the
// label dropped and whether it had already dropped this round, in which case
// the vertex is already on the next worklist.  One random atomic per
// relaxation serves as both the update and the push deduplication.
__device__ __forceinline__ bool lower_word(unsigned long long *word, int32_t cand, unsigned long long cur,
                                           uint32_t tag, int32_t dedup) {
  if (cand >= (int32_t)(cur >> 32)) return false;  // a stale (larger) cached word only costs an atomic
  const unsigned long long old = __hip_atomic_fetch_min(word, ((unsigned long long)(uint32_t)cand << 32) | tag,
                                                        __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  return cand < (int32_t)(old >> 32) && (!dedup || (uint32_t)old != tag);
}

// The label of an active vertex.  If its tag shows that it was lowered again
// during the current round, it is already on the next worklist and will be
// processed there with the newer label, so relaxing its edges now (with the
// older, larger label) is skipped.
__device__ __forceinline__ int32_t label_of_active(unsigned long long w, uint32_t tag, bool &skip) {
  skip = (uint32_t)w == tag;
  return (int32_t)(w >> 32);
}

struct OpSSSP {  // relaxation: dist[dst] = min(dist[dst], dist[src] + w)
  using val_t = int32_t;
  struct pre_t {
    int32_t cand;
    unsigned long long cur;
  };
  static constexpr bool kPush = true, kNeedSrc = false, kRecord = false, kPR = false, kBatch = true;
  unsigned long long *word;
  const int32_t *w;
  int32_t dedup;
  __device__ __forceinline__ val_t load_src(long long sl, int32_t, uint32_t tag, bool &skip) const {
    return label_of_active(word[sl], tag, skip);
  }
  // The candidate sv + w saturates at INT32_MAX (the unreached label), which it
  // then cannot lower.  Both terms are in [0, INT32_MAX], so their sum fits in
  // 32 unsigned bits.  A sum beyond INT32_MAX - 1 is never a shortest
  // distance (graph creation bounds those by max(w) * (n - 1)), so dropping
  // it changes no result.
  __device__ __forceinline__ pre_t prepare(int32_t pos, long long dl, val_t sv, int32_t) const {
    const uint32_t c = (uint32_t)sv + (uint32_t)w[pos];
    return {(int32_t)min(c, (uint32_t)kInf), word[dl]};
  }
  __device__ __forceinline__ bool commit(const pre_t &p, int32_t, long long dl, val_t, int32_t, int32_t,
                                         uint32_t tag) const {
    return lower_word(&word[dl], p.cand, p.cur, tag, dedup);
  }
};

// Continuous serving: BFS and SSSP queries in one launch.  A query slot
// flagged unit relaxes every edge with weight 1, so its distances are BFS
// levels; the others use the graph's weights.
struct OpServe : OpSSSP {
  const int32_t *unit;  // per query slot
  __device__ __forceinline__ pre_t prepare(int32_t pos, long long dl, val_t sv, int32_t q) const {
    const uint32_t c = (uint32_t)sv + (unit[q] ? 1u : (uint32_t)w[pos]);
    return {(int32_t)min(c, (uint32_t)kInf), word[dl]};
  }
};

struct OpCC {  // min-label propagation
  using val_t = int32_t;
  struct pre_t {
    unsigned long long cur;
  };
  static constexpr bool kPush = true, kNeedSrc = false, kRecord = false, kPR = false, kBatch = false;
  unsigned long long *word;
  int32_t dedup;
  __device__ __forceinline__ val_t load_src(long long sl, int32_t, uint32_t tag, bool &skip) const {
    return label_of_active(word[sl], tag, skip);
  }
  __device__ __forceinline__ pre_t prepare(int32_t, long long dl, val_t, int32_t) const { return {word[dl]}; }
  __device__ __forceinline__ bool commit(const pre_t &p, int32_t, long long dl, val_t sv, int32_t, int32_t,
                                         uint32_t tag) const {
    return lower_word(&word[dl], sv, p.cur, tag, dedup);
  }
};

// CC with the filter: a set bit says the destination's label is already 0,
// the smallest vertex id, which no relaxation can lower; its word is not
// read (a clear bit says nothing).
struct OpCCFilter : OpCC {
  const uint32_t *vbits;
  __device__ __forceinline__ pre_t prepare(int32_t, long long dl, val_t, int32_t) const {
    if ((vbits[dl >> 5] >> (dl & 31)) & 1u) return {0ull};
    return {word[dl]};
  }
};

// The filtering operator of BFS and CC, and the property its bitmap records.
template <class Op>
struct Filtered;
template <>
struct Filtered<OpBFS> {
  using type = OpBFSFilter;
  __device__ static type make(const OpBFS &op, const Args &a) {
    type f;
    f.level = op.level;
    f.vbits = a.vbits;
    return f;
  }
  __device__ static bool bit(const Args &a, uint32_t v) { return a.level[v] != kInf; }  // reached
};
template <>
struct Filtered<OpCC> {
  using type = OpCCFilter;
  __device__ static type make(const OpCC &op, const Args &a) {
    type f;
    f.word = op.word;
    f.dedup = op.dedup;
    f.vbits = a.vbits;
    return f;
  }
  __device__ static bool bit(const Args &a, uint32_t v) { return (a.word[v] >> 32) == 0ull; }  // label 0
};

// k-core (peeling): an active vertex has left the core; each of its edges
// lowers the neighbour's remaining degree, and the neighbour whose degree
// falls from k to k - 1 leaves in the next round, so every vertex is pushed
// at most once.  Round 0 inspects every vertex (no worklist) and takes those
// with fewer than k edges, judged by the CSR degree rather than the
// remaining degree that other lanes are already lowering.
struct OpKCore {
  using val_t = int32_t;
  struct pre_t {};
  static constexpr bool kPush = true, kNeedSrc = false, kRecord = false, kPR = false, kBatch = false;
  int32_t *rem;
  int32_t k;
  __device__ __forceinline__ val_t load_src(long long, int32_t deg, uint32_t tag, bool &skip) const {
    if (tag == 1u) skip = deg >= k;
    return 0;
  }
  __device__ __forceinline__ pre_t prepare(int32_t, long long, val_t, int32_t) const { return {}; }
  __device__ __forceinline__ bool commit(const pre_t &, int32_t, long long dl, val_t, int32_t, int32_t,
                                         uint32_t) const {
    return __hip_atomic_fetch_add(&rem[dl], -1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == k;
  }
};

// k-core with the filter: a set bit says the destination has already left
// the core (remaining degree below k), so decrementing it changes nothing
// (its degree stays below k and it is never pushed again); the atomic is
// skipped.
struct OpKCoreFilter : OpKCore {
  const uint32_t *vbits;
  struct pre_t {
    bool gone;
  };
  __device__ __forceinline__ pre_t prepare(int32_t, long long dl, val_t, int32_t) const {
    return {((vbits[dl >> 5] >> (dl & 31)) & 1u) != 0u};
  }
  __device__ __forceinline__ bool commit(const pre_t &p, int32_t, long long dl, val_t, int32_t, int32_t,
                                         uint32_t) const {
    if (p.gone) return false;
    return __hip_atomic_fetch_add(&rem[dl], -1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == k;
  }
};
template <>
struct Filtered<OpKCore> {
  using type = OpKCoreFilter;
  __device__ static type make(const OpKCore &op, const Args &a) {
    type f;
    f.rem = op.rem;
    f.k = op.k;
    f.vbits = a.vbits;
    return f;
  }
  __device__ static bool bit(const Args &a, uint32_t v) { return a.level[v] < a.kcore_k; }  // left the core
};

struct OpPR {  // acc[dst] += rank[src] / outdeg(src): fp32 contribution, exact fixed-point sum
  using val_t = float;
  struct pre_t {};
  static constexpr bool kPush = false, kNeedSrc = false, kRecord = false, kPR = true, kBatch = false;
  const float *rank;
  unsigned long long *acc;
  __device__ __forceinline__ val_t load_src(long long sl, int32_t deg, uint32_t, bool &) const {
    return rank[sl] / (float)deg;
  }
  __device__ __forceinline__ pre_t prepare(int32_t, long long, val_t, int32_t) const { return {}; }
  __device__ __forceinline__ bool commit(const pre_t &, int32_t, long long dl, val_t sv, int32_t, int32_t,
                                         uint32_t) const {
    add_relaxed(&acc[dl], to_fix(sv));
    return false;
  }
};

struct OpRecord {  // counts each processed edge and the thread that took it; pushes every destination
  using val_t = int32_t;
  struct pre_t {};
  static constexpr bool kPush = true, kNeedSrc = true, kRecord = true, kPR = false, kBatch = false;
  int32_t *hits;
  int32_t *thread_of;
  __device__ __forceinline__ val_t load_src(long long, int32_t, uint32_t, bool &) const { return 0; }
  __device__ __forceinline__ pre_t prepare(int32_t, long long, val_t, int32_t) const { return {}; }
  __device__ __forceinline__ bool commit(const pre_t &, int32_t pos, long long, val_t, int32_t, int32_t gt,
                                         uint32_t) const {
    add_relaxed(&hits[pos], 1);
    thread_of[pos] = gt;
    return true;
  }
};

template <class Op>
Op make_op(const Args &a);
template <>
OpBFS make_op<OpBFS>(const Args &a) { return OpBFS{a.level}; }
template <>
OpSSSP make_op<OpSSSP>(const Args &a) { return OpSSSP{a.word, a.w, a.dedup}; }
template <>
OpServe make_op<OpServe>(const Args &a) {
  OpServe o;
  o.word = a.word;
  o.w = a.w;
  o.dedup = a.dedup;
  o.unit = a.q_unit;
  return o;
}
template <>
OpCC make_op<OpCC>(const Args &a) { return OpCC{a.word, a.dedup}; }
template <>
OpPR make_op<OpPR>(const Args &a) { return OpPR{a.rank, a.acc}; }
template <>
OpRecord make_op<OpRecord>(const Args &a) { return OpRecord{a.hits, a.thread_of}; }
template <>
OpKCore make_op<OpKCore>(const Args &a) { return OpKCore{a.level, a.kcore_k}; }

// ---------------------------------------------------------------------------
// Per-thread statistics, shared memory, work-distribution grid, push staging.
// ---------------------------------------------------------------------------

struct Acc {
  unsigned long long frontier = 0, edges_twc = 0, edges_lb = 0, huge_v = 0, pushes = 0;
  unsigned long long dangling = 0;  // fixed point
  unsigned long long prof[kProfParts] = {0, 0, 0, 0, 0, 0};
};

// Profiling aid: thread 0 of each workgroup adds the ticks since *t to part k.
__device__ __forceinline__ void prof_mark(const Args &a, Acc &acc, int k, uint64_t &t) {
  if (a.profile && threadIdx.x == 0) {
    const uint64_t now = (uint64_t)wall_clock64();
    acc.prof[k] += now - t;
    t = now;
  }
}

// Profiling aid: the edges this workgroup processed in round r (each wave
// adds its lanes' counts since the last call).
__device__ __forceinline__ void prof_round_edges(const Args &a, const Acc &acc, unsigned long long &last, uint32_t id,
                                                 int r) {
  const unsigned long long now = acc.edges_twc + acc.edges_lb;
  unsigned long long d = now - last;
  last = now;
#pragma unroll
  for (int o = kWave / 2; o > 0; o >>= 1) d += __shfl_xor(d, o);
  if (lane_id() == 0 && d && r < kTimeline && id < (uint32_t)kProfMembers)
    add_relaxed(&a.prof_wg[(size_t)r * kProfMembers + id], (uint32_t)d);
}

// Worklist entries: a vertex id for one query; (query << 32) | vertex for a batch.
template <bool M>
using Entry = typename std::conditional<M, unsigned long long, int32_t>::type;

template <int B, class Op, bool M = false>
struct Smem {
  using V = typename Op::val_t;
  int32_t pos[kU * B];  // thread-bin gather: CSR position, source value and source (batch: query) of each edge
  V sv[kU * B];
  int32_t src[(Op::kNeedSrc || M) ? kU * B : 1];
  int32_t wsum[B / kWave];
  unsigned long long ured[B / kWave][5];
  unsigned long long dred[B / kWave];
  int32_t owner, obeg, odeg, ov;
  V osv;
  int32_t flag;
  uint32_t ticket, members;  // persistent launch: this workgroup's ticket and the member count
  uint32_t xcd, xcd_n, n_xcd;  // its XCD, the members on that XCD, the XCDs holding members
  unsigned long long cbase;  // phase 1: first worklist entry of the current claim
  uint32_t clen;             // and its length
  Entry<M> pbuf[B / kWave][kPushBuf];  // per-wavefront push staging
};

// The workgroup's index and the workgroup count used for work distribution:
// the hardware ones for one-phase launches, the membership ticket and the
// member count inside the persistent launch.
struct Grid {
  uint32_t id;
  uint32_t n;
  uint32_t xcd = 0, xcd_n = 1, n_xcd = 1;  // persistent launch: barrier topology (see grid_barrier)
};

// Next-worklist pushes of one wavefront, staged in LDS and written out in
// batches: one global reservation per batch instead of one per ballot.
template <class E>
struct Pusher {
  E *buf;            // this wavefront's LDS staging area
  uint32_t cnt;      // entries staged (wave-uniform)
  E *qn;             // next worklist
  uint32_t *qn_cnt;  // its size counter
};

template <int B, class Op, bool M>
__device__ void flush_stats(Acc &acc, Smem<B, Op, M> &sm, Ctl *c) {
  const uint32_t lane = lane_id();
  const int w = threadIdx.x / kWave;
  unsigned long long v[5] = {acc.frontier, acc.edges_twc, acc.edges_lb, acc.huge_v, acc.pushes};
#pragma unroll
  for (int k = 0; k < 5; ++k) {
#pragma unroll
    for (int d = kWave / 2; d > 0; d >>= 1) v[k] += __shfl_xor(v[k], d);
    if (lane == 0) sm.ured[w][k] = v[k];
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    unsigned long long t[5] = {0, 0, 0, 0, 0};
    for (int j = 0; j < B / kWave; ++j)
      for (int k = 0; k < 5; ++k) t[k] += sm.ured[j][k];
    if (t[0]) add_relaxed(&c->st_frontier, t[0]);
    if (t[1]) add_relaxed(&c->st_edges_twc, t[1]);
    if (t[2]) add_relaxed(&c->st_edges_lb, t[2]);
    if (t[3]) add_relaxed(&c->st_huge_v, t[3]);
    if (t[4]) add_relaxed(&c->st_pushes, t[4]);
    for (int k = 0; k < kProfParts; ++k)
      if (acc.prof[k]) add_relaxed(&c->prof[k], acc.prof[k]);
  }
  __syncthreads();
  acc = Acc();
}

template <int B, class Op, bool M>
__device__ void flush_dangling(Acc &acc, Smem<B, Op, M> &sm, unsigned long long *dst) {
  unsigned long long x = acc.dangling;
#pragma unroll
  for (int d = kWave / 2; d > 0; d >>= 1) x += __shfl_xor(x, d);
  if (lane_id() == 0) sm.dred[threadIdx.x / kWave] = x;
  __syncthreads();
  if (threadIdx.x == 0) {
    unsigned long long t = 0;
    for (int j = 0; j < B / kWave; ++j) t += sm.dred[j];
    if (t != 0) add_relaxed(dst, t);
  }
  __syncthreads();
  acc.dangling = 0;
}

// Write the staged entries to the next worklist (all lanes call this).
template <class E>
__device__ __forceinline__ void flush_pushes(const Args &a, int round, Pusher<E> &pu) {
  if (pu.cnt == 0) return;
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
  uint32_t base = 0;
  if (lane_id() == 0) base = add_relaxed(pu.qn_cnt, pu.cnt);
  base = __shfl(base, 0);
  for (uint32_t j = lane_id(); j < pu.cnt; j += kWave) {
    const uint32_t idx = base + j;
    if (idx < a.qcap)
      pu.qn[idx] = pu.buf[j];
    else
      flag_overflow(a.ctl, round);
  }
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
  pu.cnt = 0;
}

// Stage v for every lane with pred (all lanes of the wavefront call this).
template <class E>
__device__ __forceinline__ void push_wave(bool pred, E v, const Args &a, int round, Pusher<E> &pu, Acc &acc) {
  const unsigned long long m = __ballot(pred);
  if (m == 0ull) return;
  const uint32_t total = (uint32_t)__popcll(m);
  if (pu.cnt + total > kPushBuf) flush_pushes(a, round, pu);
  if (pred) pu.buf[pu.cnt + bits_below(m)] = v;
  pu.cnt += total;
  if (lane_id() == 0) acc.pushes += total;
}

// log2 of the chunk size of the huge-edge index for a threshold t: the
// largest power of two not above t, clamped, so that a chunk holds at most
// two segment starts when t >= 2^kHintMinShift.
__device__ __forceinline__ uint32_t hint_shift(int64_t t) {
  if (t < (1ll << kHintMinShift)) return kHintMinShift;
  if (t >= (1ll << kHintMaxShift)) return kHintMaxShift;
  return 63u - (uint32_t)__builtin_clzll((unsigned long long)t);
}

// Algorithm 1, "work.push(src)": append every huge lane's vertex to the huge
// list and its degree to the running edge total with ONE 64-bit atomic per
// wavefront on (count << 32 | edges).  Slot j receives the edges of all
// earlier slots as its prefixWork entry, i.e. the exclusive scan of the huge
// degrees in list order, with the vertex's CSR start, the vertex (batch: its
// query) and the source value.  The
// wavefront then writes the chunk index for every chunk whose first edge
// falls in one of its new segments.  All lanes of the wavefront call this.
__device__ __forceinline__ void reserve_huge(bool huge, int32_t v_or_q, int32_t beg, int32_t deg, int32_t sv_bits,
                                             const Args &a, int round, unsigned long long *ctr, uint32_t hs,
                                             Acc &acc) {
  const unsigned long long hm = __ballot(huge);
  if (hm == 0ull) return;
  const uint32_t lane = lane_id();
  const unsigned long long mine = huge ? (unsigned long long)(uint32_t)deg : 0ull;
  unsigned long long incl = mine;
#pragma unroll
  for (int d = 1; d < kWave; d <<= 1) {
    const unsigned long long y = __shfl_up(incl, d);
    if ((int)lane >= d) incl += y;
  }
  const unsigned long long tot_e = __shfl(incl, kWave - 1);
  const uint32_t tot_c = (uint32_t)__popcll(hm);
  unsigned long long base = 0;
  int bad = 0;
  if (lane == kWave - 1) {
    if (tot_e >> 32) {
      bad = 1;
    } else {
      base = add_relaxed(ctr, ((unsigned long long)tot_c << 32) | tot_e);
      if ((unsigned long long)(uint32_t)base + tot_e > 0xffffffffull) bad = 1;
      acc.huge_v += tot_c;
    }
    if (bad) flag_overflow(a.ctl, round);
  }
  base = __shfl(base, kWave - 1);
  bad = __shfl(bad, kWave - 1);
  if (bad) return;  // the round is abandoned; nothing below may be trusted
  uint32_t j = 0, p = 0;
  if (huge) {
    j = (uint32_t)(base >> 32) + bits_below(hm);
    p = (uint32_t)base + (uint32_t)(incl - mine);
    if (j < a.qcap)
      a.huge_rec[j] = make_int4((int32_t)p, beg, v_or_q, sv_bits);
    else
      flag_overflow(a.ctl, round);
  }
  // chunk index: chunk c's first edge c << hs lies in [p, p + deg)
  unsigned long long rem = hm;
  while (rem) {
    const int l = __ffsll(rem) - 1;
    rem &= rem - 1;
    const uint32_t jj = __shfl(j, l), pp = __shfl(p, l);
    const uint32_t dd = (uint32_t)__shfl(deg, l);
    const uint64_t c_lo = ((uint64_t)pp + (1ull << hs) - 1) >> hs;
    const uint64_t c_hi = ((uint64_t)pp + dd - 1) >> hs;
    for (uint64_t c = c_lo + lane; c <= c_hi; c += kWave) {
      if (c < a.hint_cap)
        a.hint[c] = make_int2((int32_t)jj, (int32_t)(pp + dd));
      else
        flag_overflow(a.ctl, round);
    }
  }
}

// Apply the operator along up to kU edges per lane and push; every lane of
// the wavefront calls this (act[u] false for empty slots).  src[u] is the
// source vertex (recorder) or, for a batch, the query of slot u.
template <class Op, bool M>
__device__ __forceinline__ void edges(const bool (&act)[kU], const int32_t (&pos)[kU],
                                      const typename Op::val_t (&sv)[kU], const int32_t (&src)[kU], const Op &op,
                                      const Args &a, uint32_t tag, int round, Pusher<Entry<M>> &pu, Acc &acc,
                                      int32_t gt) {
  int32_t dst[kU];
  long long dl[kU];
  typename Op::pre_t pre[kU];
#pragma unroll
  for (int u = 0; u < kU; ++u) dst[u] = a.col[act[u] ? pos[u] : 0];
  // an empty slot addresses label 0, which always exists (a batch's query
  // offsets can be negative, so no other index is safe for every query)
#pragma unroll
  for (int u = 0; u < kU; ++u) {
    if constexpr (M)
      dl[u] = act[u] ? dst[u] + a.qoff[src[u]] : 0;
    else
      dl[u] = act[u] ? dst[u] : 0;
  }
#pragma unroll
  for (int u = 0; u < kU; ++u) pre[u] = op.prepare(act[u] ? pos[u] : 0, dl[u], sv[u], src[u]);
  bool p[kU];
#pragma unroll
  for (int u = 0; u < kU; ++u) p[u] = act[u] && op.commit(pre[u], pos[u], dl[u], sv[u], src[u], gt, tag);
  if constexpr (Op::kPush) {
#pragma unroll
    for (int u = 0; u < kU; ++u) {
      if constexpr (M)
        push_wave<Entry<M>>(p[u], ((unsigned long long)(uint32_t)src[u] << 32) | (uint32_t)dst[u], a, round, pu,
                            acc);
      else
        push_wave<Entry<M>>(p[u], dst[u], a, round, pu, acc);
    }
  }
}

template <int B>
__device__ __forceinline__ void block_exscan(int32_t x, int32_t &excl, int32_t &total, int32_t *wsum) {
  const uint32_t lane = lane_id();
  const int w = threadIdx.x / kWave;
  int32_t incl = x;
#pragma unroll
  for (int d = 1; d < kWave; d <<= 1) {
    const int32_t y = __shfl_up(incl, d);
    if ((int)lane >= d) incl += y;
  }
  if (lane == kWave - 1) wsum[w] = incl;
  __syncthreads();
  int32_t before = 0, tot = 0;
#pragma unroll
  for (int j = 0; j < B / kWave; ++j) {
    const int32_t s = wsum[j];
    before += (j < w) ? s : 0;
    tot += s;
  }
  excl = before + incl - x;
  total = tot;
  __syncthreads();
}

// Waves per SIMD the persistent kernel's register budget is sized for: the
// traversal is bound by the latency of dependent random loads, so more
// resident waves keep more of them in flight.
#ifndef ALB_WAVES_PER_EU
#define ALB_WAVES_PER_EU 4
#endif

// ---------------------------------------------------------------------------
// Phase 1: inspection (Algorithm 1) fused with the TWC bins.
// ---------------------------------------------------------------------------

// Worklist entries per claim: B, unless the worklist would give a workgroup
// fewer than two claims; then whole wavefronts' worth, just enough for two
// claims per workgroup, so that a short worklist still reaches every
// workgroup instead of leaving most of them idle for the phase.
__device__ __forceinline__ uint32_t twc_chunk(uint32_t nF, uint32_t wgs, int B) {
  const uint64_t per = ((uint64_t)nF + 2ull * wgs - 1) / (2ull * wgs);
  uint64_t c = (per + kWave - 1) / kWave * kWave;
  if (c < (uint64_t)kWave) c = kWave;
  if (c > (uint64_t)B) c = B;
  return (uint32_t)c;
}

// Workgroups take runs of consecutive worklist entries one at a time, so a
// run that takes long does not hold up work queued behind it.  The first run
// of workgroup g is fixed (entries [g * C0, (g + 1) * C0)) and needs no
// atomic; later runs are claimed from a counter over the entries beyond
// those, each sized from the remainder the previous claim's atomic returned
// (guided self-scheduling): B while plenty remain, then fewer whole
// wavefronts, so that the phase ends with short runs and the workgroups
// reach the barrier together.  The counter is only ever touched by the
// atomic (a plain load of a contended counter is slow).  Thread 0 of the
// workgroup holds the state; the caller's workgroup barriers separate one
// claim's reads of the published run from the next claim's writes.
struct Claims {
  uint32_t C0, len;
  unsigned long long S, nxt, seen;
  bool first;
  __device__ Claims(uint32_t nF, Grid gr, int B)
      : C0(twc_chunk(nF, gr.n, B)), len(C0), S((unsigned long long)gr.n * C0),
        nxt((unsigned long long)gr.id * C0), seen(S), first(true) {}
  // Publish the next run as (*base, *n); *base >= nF means no more work.
  __device__ void next(unsigned long long *claim, uint32_t nF, Grid gr, int B, unsigned long long &base,
                       uint32_t &n) {
    if (!first) {
      if (S >= (unsigned long long)nF) {
        nxt = ~0ull;  // the fixed runs covered the worklist
      } else {
        len = twc_chunk(seen < nF ? nF - (uint32_t)seen : 0u, gr.n, B);
        nxt = S + add_relaxed(claim, (unsigned long long)len);
        seen = nxt + len;
      }
    }
    first = false;
    base = nxt;
    n = len;
  }
};


template <int B, class Op, bool M, class S>
__device__ void phase_twc(const Args &a, const Op &op, S &sm, Grid gr, int round,
                          const Entry<M> *F, uint32_t nF, Entry<M> *qn, uint32_t *qn_cnt, unsigned long long *hctr,
                          int64_t threshold, uint32_t hs, Acc &acc) {
  using V = typename Op::val_t;
  const int tid = threadIdx.x;
  const uint32_t lane = lane_id();
  const int32_t gt = (int32_t)(gr.id * B + tid);
  const uint32_t tag = (uint32_t)round + 1u;
  unsigned long long *claim = &a.ctl->chunk[round % 3];
  Pusher<Entry<M>> pu{sm.pbuf[tid / kWave], 0u, qn, qn_cnt};
  uint64_t pt = a.profile ? (uint64_t)wall_clock64() : 0;
  Claims cl(nF, gr, B);
  for (;;) {
    if (tid == 0) cl.next(claim, nF, gr, B, sm.cbase, sm.clen);
    __syncthreads();
    const unsigned long long base = sm.cbase;
    const uint32_t C = sm.clen;
    if (base >= nF) break;
    const uint32_t i = (uint32_t)base + tid;
    const bool mine = tid < (int)C && i < nF;
    int32_t v = -1, beg = 0, deg = 0, q = 0;  // q: the entry's query (batch)
    int64_t thr = threshold;
    int32_t c_wave = a.c_wave, c_wg = a.c_wg;  // TWC cutoffs (a batch's queries may have their own)
    if (mine) {
      if constexpr (M) {
        const unsigned long long e = F[i];
        v = (int32_t)(uint32_t)e;
        q = (int32_t)(e >> 32);
        if (a.qthr) thr = a.qthr[q];
        if (a.qcut) {
          c_wave = a.qcut[2 * q];
          c_wg = a.qcut[2 * q + 1];
        }
      } else {
        v = F ? F[i] : (int32_t)i;
      }
      beg = a.off[v];
      deg = a.off[v + 1] - beg;
    }
    if constexpr (M) {
      // continuous serving: this round had an entry of query slot q.  One
      // plain store per run of equal slots in the wavefront, skipped once
      // the mark already reads this round (the grid barrier publishes it).
      // A store from every wavefront, all to the one address of a lone
      // query's slot, serialised the round: writing through to memory they
      // tripled the inspection phase.
      if (a.q_last) {
        const int32_t qq = mine ? q : -1;
        const int32_t prev = __shfl_up(qq, 1);
        if (mine && (lane == 0 || prev != qq) && a.q_last[qq] != (int32_t)round) a.q_last[qq] = (int32_t)round;
      }
    }
    V sv = V(0);
    if (deg > 0) {
      bool skip = false;
      long long sl = v;
      if constexpr (M) sl += a.qoff[q];
      sv = op.load_src(sl, deg, tag, skip);
      if (skip) deg = 0;
    }
    // inspection: degree >= THRESHOLD goes to the huge list
    const bool huge = v >= 0 && deg > 0 && (int64_t)deg >= thr;
    reserve_huge(huge, M ? q : v, beg, deg, to_bits(sv), a, round, hctr, hs, acc);
    if constexpr (Op::kRecord) {
      if (mine) a.bins[i] = (int8_t)(huge ? 3 : deg >= c_wg ? 2 : deg >= c_wave ? 1 : 0);
    }
    if constexpr (Op::kPR) {
      if (v >= 0 && deg == 0) acc.dangling += to_fix(a.rank[v]);
    }
    if (huge) deg = 0;
    acc.frontier += (v >= 0);
    acc.edges_twc += (unsigned long long)deg;
    prof_mark(a, acc, kProfInspect, pt);

    // workgroup bin: the whole workgroup strides one vertex's edges
    for (;;) {
      if (tid == 0) sm.owner = -1;
      __syncthreads();
      if (deg > 0 && deg >= c_wg) sm.owner = tid;  // any one claimant wins
      __syncthreads();
      const int32_t o = sm.owner;
      if (o < 0) break;
      if (tid == o) {
        sm.obeg = beg;
        sm.odeg = deg;
        sm.osv = sv;
        sm.ov = M ? q : v;
        deg = 0;
      }
      __syncthreads();
      const int32_t ob = sm.obeg, od = sm.odeg, ov = sm.ov;
      const V os = sm.osv;
      for (int32_t j0 = 0; j0 < od; j0 += kU * B) {
        bool act[kU];
        int32_t pos[kU], src[kU];
        V s[kU];
#pragma unroll
        for (int u = 0; u < kU; ++u) {
          const int32_t j = j0 + u * B + tid;
          act[u] = j < od;
          pos[u] = ob + j;
          s[u] = os;
          src[u] = ov;
        }
        edges<Op, M>(act, pos, s, src, op, a, tag, round, pu, acc, gt);
      }
    }

    prof_mark(a, acc, kProfWgBin, pt);
    // wavefront bin: one wavefront strides one vertex's edges
    for (;;) {
      const unsigned long long mm = __ballot(deg > 0 && deg >= c_wave);
      if (mm == 0ull) break;
      const int ld = __ffsll(mm) - 1;
      const int32_t ob = __shfl(beg, ld), od = __shfl(deg, ld), ov = __shfl(M ? q : v, ld);
      const V os = __shfl(sv, ld);
      if ((int)lane == ld) deg = 0;
      for (int32_t j0 = 0; j0 < od; j0 += kU * kWave) {
        bool act[kU];
        int32_t pos[kU], src[kU];
        V s[kU];
#pragma unroll
        for (int u = 0; u < kU; ++u) {
          const int32_t j = j0 + u * kWave + (int32_t)lane;
          act[u] = j < od;
          pos[u] = ob + j;
          s[u] = os;
          src[u] = ov;
        }
        edges<Op, M>(act, pos, s, src, op, a, tag, round, pu, acc, gt);
      }
    }

    prof_mark(a, acc, kProfWaveBin, pt);
    // thread bin: fine-grained gather of the remaining short lists through LDS,
    // kU * B edges at a time, so that the workgroup's lanes stay busy
    int32_t rank, total;
    block_exscan<B>(deg, rank, total, sm.wsum);
    for (int32_t done = 0; done < total; done += kU * B) {
      const int32_t lo = max(rank, done), hi = min(rank + deg, done + kU * B);
      for (int32_t e = lo; e < hi; ++e) {
        sm.pos[e - done] = beg + (e - rank);
        sm.sv[e - done] = sv;
        if constexpr (Op::kNeedSrc || M) sm.src[e - done] = M ? q : v;
      }
      __syncthreads();
      const int32_t cnt = min(kU * B, total - done);
      bool act[kU];
      int32_t pos[kU], src[kU];
      V s[kU];
#pragma unroll
      for (int u = 0; u < kU; ++u) {
        const int32_t idx = u * B + tid;
        act[u] = idx < cnt;
        pos[u] = act[u] ? sm.pos[idx] : 0;
        s[u] = act[u] ? sm.sv[idx] : V(0);
        src[u] = 0;
        if constexpr (Op::kNeedSrc || M) src[u] = act[u] ? sm.src[idx] : 0;
      }
      edges<Op, M>(act, pos, s, src, op, a, tag, round, pu, acc, gt);
      __syncthreads();
    }
    prof_mark(a, acc, kProfThreadBin, pt);
  }
  if constexpr (Op::kPush) flush_pushes(a, round, pu);
  prof_mark(a, acc, kProfThreadBin, pt);
}

// The huge-list slot whose edge range holds huge edge k: the last slot j with
// prefixWork[j] <= k.  The chunk index gives the slot j0 that owns the first
// edge of k's chunk and where j0's edges end; k before that end is j0's,
// otherwise an exponential search forward from j0 + 1, then bisection, finds
// the answer (one probe when every huge degree is at least the chunk size).
__device__ __forceinline__ uint32_t owner_of(const Args &a, uint32_t vh, uint32_t hs, uint32_t k) {
  const int2 h = a.hint[k >> hs];
  if (k < (uint32_t)h.y) return (uint32_t)h.x;  // inside the segment that holds the chunk's first edge
  uint64_t lo = (uint32_t)h.x + 1u, step = 1, hi = lo + 1;
  while (hi < vh && (uint32_t)a.huge_rec[hi].x <= k) {
    lo = hi;
    step <<= 1;
    hi = lo + step;
  }
  if (hi > vh) hi = vh;
  while (hi - lo > 1) {
    const uint64_t mid = lo + ((hi - lo) >> 1);
    if ((uint32_t)a.huge_rec[mid].x <= k)
      lo = mid;
    else
      hi = mid;
  }
  return (uint32_t)lo;
}

// ---------------------------------------------------------------------------
// Phase 2: execution (Algorithm 2) with the cyclic distribution.
// ---------------------------------------------------------------------------
template <int B, class Op, bool M, class S>
__device__ void phase_lb(const Args &a, const Op &op, S &sm, Grid gr, int round, unsigned long long hc,
                         Entry<M> *qn, uint32_t *qn_cnt, uint32_t hs, Acc &acc) {
  using V = typename Op::val_t;
  const uint32_t vh = (uint32_t)(hc >> 32);
  const uint32_t e = (uint32_t)hc;
  if (vh == 0) return;
  // an overflowed reservation leaves the huge list inconsistent: skip
  if (ld_relaxed(&a.ctl->overflow) <= (uint32_t)round) return;
  const uint64_t T = (uint64_t)gr.n * B;
  const uint32_t lane = lane_id();
  const uint64_t g = (uint64_t)gr.id * B + threadIdx.x;
  const uint32_t tag = (uint32_t)round + 1u;
  Pusher<Entry<M>> pu{sm.pbuf[threadIdx.x / kWave], 0u, qn, qn_cnt};
  uint64_t pt = a.profile ? (uint64_t)wall_clock64() : 0;
  // slot u of a pass: huge edge k (if active) -> CSR position, source, source value
  auto take = [&](uint64_t k, bool on, bool &act, int32_t &pos, int32_t &src, V &sv) {
    act = on;
    pos = 0;
    src = 0;
    sv = V(0);
    if (on) {
      const int4 r = a.huge_rec[owner_of(a, vh, hs, (uint32_t)k)];
      pos = r.y + (int32_t)((uint32_t)k - (uint32_t)r.x);
      src = r.z;
      sv = from_bits<V>(r.w);
    }
    acc.edges_lb += on;
  };
  bool act[kU];
  int32_t pos[kU], src[kU];
  V s[kU];
  if (!a.blocked) {
    // cyclic: thread g takes huge edges g, g + T, g + 2T, ...; kU of them per
    // pass, so a wavefront's lanes read consecutive CSR entries
    for (uint64_t k0 = g - lane; k0 < e; k0 += kU * T) {
#pragma unroll
      for (int u = 0; u < kU; ++u) {
        const uint64_t k = k0 + lane + (uint64_t)u * T;
        take(k, k < e, act[u], pos[u], src[u], s[u]);
      }
      edges<Op, M>(act, pos, s, src, op, a, tag, round, pu, acc, (int32_t)g);
    }
  } else {
    // blocked (the alternative of Section 4.1): thread g takes the run
    // [g * c, (g + 1) * c) of c = ceil(e / T) consecutive huge edges
    const uint64_t c = (e + T - 1) / T;
    for (uint64_t j0 = 0; j0 < c; j0 += kU) {
#pragma unroll
      for (int u = 0; u < kU; ++u) {
        const uint64_t j = j0 + (uint64_t)u, k = g * c + j;
        take(k, j < c && k < e, act[u], pos[u], src[u], s[u]);
      }
      edges<Op, M>(act, pos, s, src, op, a, tag, round, pu, acc, (int32_t)g);
    }
  }
  if constexpr (Op::kPush) flush_pushes(a, round, pu);
  prof_mark(a, acc, kProfLb, pt);
}

// PageRank update: r'(v) = (1-d)/n + d * (acc(v) + D/n), rounded to fp32; acc cleared.
template <int B>
__device__ void phase_pr_update(const Args &a, Grid gr, unsigned long long dangling_fix) {
  const double d = (double)a.damping;
  const double N = (double)a.n;
  const double base = (1.0 - d) / N + d * ((double)dangling_fix * kFixInv) / N;
  for (uint32_t v = gr.id * B + threadIdx.x; v < (uint32_t)a.n; v += gr.n * B) {
    const double x = (double)a.acc[v] * kFixInv;
    a.rank[v] = (float)(base + d * x);
    a.acc[v] = 0ull;
  }
}

// The XCD (accelerator complex die, one L2) the calling wave runs on: the
// XCC_ID hardware register, bits [3:0].
__device__ __forceinline__ uint32_t xcd_id() {
  return __builtin_amdgcn_s_getreg((3 << 11) | (0 << 6) | 20) & (uint32_t)(kBarXcds - 1);
}

// Wait until every memory operation this wave issued has completed; also a
// compiler barrier, so no load or store moves across it.
__device__ __forceinline__ void wait_memory() { asm volatile("s_waitcnt vmcnt(0) lgkmcnt(0)" ::: "memory"); }

// Bounded wait of thread 0 until *w reaches target.  Returns false if the
// launch was aborted or this wait outlasted timeout_ticks (which then
// aborts it: every workgroup leaves at its next barrier).
__device__ __forceinline__ bool bar_wait(const Args &a, unsigned long long *w, unsigned long long target, int round) {
  Ctl *c = a.ctl;
  const uint64_t t0 = (uint64_t)wall_clock64();
  unsigned long long seen;
  while ((seen = ld_relaxed(w)) < target) {
    if (ld_relaxed(&c->abort)) return false;
    if ((uint64_t)wall_clock64() - t0 > a.timeout_ticks) {
      st_relaxed(&c->diag_seen, seen);
      st_relaxed(&c->diag_target, target);
      st_relaxed(&c->diag_round, (uint32_t)round);
      st_relaxed(&c->abort, 1u);
      return false;
    }
    __builtin_amdgcn_s_sleep(1);
  }
  return true;
}

// Grid-wide barrier among the members of the persistent launch, with one
// agent-scope release (L2 write-back) per XCD instead of one per workgroup:
// the write-back covers the whole L2 of the XCD it runs on, whichever CU
// wrote the lines, and a hundred of them in a row per L2 made the barrier
// cost grow with the grid.  Every wave first waits until its own memory
// operations have completed, so after the workgroup barrier all of the
// workgroup's stores are in its XCD's L2 (the vector L1 writes through).
// Thread 0 then arrives on its XCD's counter.  The XCD's last arrival does
// the release, arrives on the root counter, waits for the generation and
// opens the XCD's flag; the others wait for the flag.  Every workgroup then
// acquires at agent scope itself (one acquire per XCD followed by an L1-only
// invalidate elsewhere was tried and gave stale reads).  Counters only grow,
// so nothing is reset between barriers.
template <class S>
__device__ bool grid_barrier(const Args &a, S &sm, Grid gr, unsigned long long &epoch, int round,
                             bool sys = false) {
  wait_memory();
  __syncthreads();
  if (threadIdx.x == 0) {
    unsigned long long *b = a.bar;
    const unsigned long long target = epoch + 1;
    const unsigned long long o1 = add_relaxed(&b[kBarXcdArrive + (size_t)kBarStride * gr.xcd], 1ull);
    bool ok;
    if ((o1 + 1) % gr.xcd_n == 0) {
      // the XCD's last arrival releases every store its members made before
      // arriving; `sys`: to the host as well (stores into host memory)
      if (sys)
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "");
      else
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
      const unsigned long long o2 = add_relaxed(&b[kBarRoot], 1ull);
      if ((o2 + 1) % gr.n_xcd == 0) st_relaxed(&b[kBarGen], target);
      ok = bar_wait(a, &b[kBarGen], target, round);
      if (ok) st_relaxed(&b[kBarXcdFlag + (size_t)kBarStride * gr.xcd], target);
    } else {
      ok = bar_wait(a, &b[kBarXcdFlag + (size_t)kBarStride * gr.xcd], target, round);
    }
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    sm.flag = ok ? 1 : 0;
  }
  __syncthreads();
  ++epoch;
  return sm.flag != 0;
}

template <bool M>
__device__ __forceinline__ const Entry<M> *round_frontier(const Args &a, int r) {
  if (a.all_rounds || (r == 0 && a.identity_first)) return nullptr;
  return (const Entry<M> *)((r & 1) ? a.q1 : a.q0);
}
template <bool M>
__device__ __forceinline__ Entry<M> *round_next(const Args &a, int r) {
  return (Entry<M> *)((r & 1) ? a.q0 : a.q1);
}

__device__ __forceinline__ uint32_t round_size(const Args &a, int r) {
  if (a.all_rounds) return (uint32_t)a.n;
  const uint32_t c = ld_relaxed(&a.ctl->qcount[r % 3]);
  return c < a.qcap ? c : a.qcap;
}

// The huge threshold of a round: the configured one, or with the small-round
// rule small_threshold while the worklist has fewer entries than launched
// threads.
__device__ __forceinline__ int64_t round_threshold(const Args &a, uint32_t nF, uint64_t T) {
  if (a.adaptive && (uint64_t)nF < T) return a.small_threshold;
  return a.threshold;
}

// Clear the counters ahead (nobody reads or writes them this round).
__device__ __forceinline__ void clear_ahead(const Args &a, int r) {
  st_relaxed(&a.ctl->chunk[(r + 1) % 3], 0ull);
  st_relaxed(&a.ctl->qcount[(r + 2) % 3], 0u);
  st_relaxed(&a.ctl->huge[(r + 1) & 1], 0ull);
  st_relaxed(&a.ctl->dangling[(r + 1) & 1], 0ull);
}

// Membership of the persistent launch.  The grid may be larger than what the
// device can hold at once, so co-residency is not assumed: every workgroup
// takes a ticket from ctl->members when it starts; the holder of ticket 0
// closes membership (sets the top bit) once all workgroups have joined or
// no new one has joined for join_window_ticks, and publishes the member
// count.  A workgroup whose ticket shows the closed bit is not a member and
// leaves at once.  Members are running when they join and never leave before
// the end, so every barrier among them completes.  Each member also counts
// itself on its XCD, for the barrier.  Returns false for a non-member; *gr
// gets (ticket, member count, XCD, members on that XCD, XCDs in use).
template <class S>
__device__ bool join_members(const Args &a, S &sm, Grid *gr) {
  constexpr unsigned long long kClosed = 1ull << 63;
  if (threadIdx.x == 0) {
    Ctl *c = a.ctl;
    const unsigned long long t = add_relaxed(&c->members, 1ull);
    uint32_t member = (t & kClosed) ? 0u : 1u;
    const uint32_t x = xcd_id();
    if (member) add_relaxed(&a.bar[kBarXcdMembers + (size_t)kBarStride * x], 1ull);
    if (member && t == 0) {
      unsigned long long seen = 1;
      uint64_t t_last = (uint64_t)wall_clock64();
      st_relaxed(&c->t_begin, (unsigned long long)t_last);
      for (;;) {
        const unsigned long long cur = ld_relaxed(&c->members);
        if (cur >= (unsigned long long)gridDim.x) break;
        const uint64_t now = (uint64_t)wall_clock64();
        if (cur != seen) {
          seen = cur;
          t_last = now;
        } else if (now - t_last > a.join_window_ticks) {
          break;
        }
        __builtin_amdgcn_s_sleep(1);
      }
      const unsigned long long prev =
          __hip_atomic_fetch_or(&c->members, kClosed, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      st_relaxed(&c->n_members, (uint32_t)prev);
    }
    uint32_t n = 0, xn = 1, nx = 1;
    if (member) {
      while ((n = ld_relaxed(&c->n_members)) == 0) __builtin_amdgcn_s_sleep(1);
      if ((uint32_t)t >= n) member = 0;  // cannot happen: tickets below the closing count are members
      // every member registers its XCD right after its ticket: wait until all
      // n have, then the per-XCD counts are final (a bounded wait; past the
      // barrier time-out the launch is aborted)
      const uint64_t t0 = (uint64_t)wall_clock64();
      for (;;) {
        unsigned long long tot = 0;
        nx = 0;
        for (int k = 0; k < kBarXcds; ++k) {
          const unsigned long long v = ld_relaxed(&a.bar[kBarXcdMembers + (size_t)kBarStride * k]);
          tot += v;
          nx += v ? 1u : 0u;
        }
        if (tot >= n) break;
        if ((uint64_t)wall_clock64() - t0 > a.timeout_ticks) {
          st_relaxed(&c->abort, 1u);
          break;
        }
        __builtin_amdgcn_s_sleep(1);
      }
      xn = (uint32_t)ld_relaxed(&a.bar[kBarXcdMembers + (size_t)kBarStride * x]);
      if (xn == 0 || nx == 0) {  // only after an abort: keep the barrier arithmetic defined
        xn = 1;
        nx = 1;
      }
    }
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    sm.flag = (int32_t)member;
    sm.ticket = (uint32_t)t;
    sm.members = n;
    sm.xcd = x;
    sm.xcd_n = xn;
    sm.n_xcd = nx;
  }
  __syncthreads();
  const bool member = sm.flag != 0;
  gr->id = sm.ticket;
  gr->n = sm.members;
  gr->xcd = sm.xcd;
  gr->xcd_n = sm.xcd_n;
  gr->n_xcd = sm.n_xcd;
  __syncthreads();
  return member;
}

// ---------------------------------------------------------------------------
// Kernels.
// ---------------------------------------------------------------------------

__global__ void k_init(Args a, int op, int32_t source, uint32_t nfront0) {
  const uint32_t stride = gridDim.x * blockDim.x;
  const uint32_t t = blockIdx.x * blockDim.x + threadIdx.x;
  const float r0 = 1.0f / (float)a.n;
  for (uint32_t v = t; v < (uint32_t)a.n; v += stride) {
    if (op == OP_BFS) a.level[v] = ((int32_t)v == source) ? 0 : kInf;
    if (op == OP_SSSP) a.word[v] = (unsigned long long)(uint32_t)((int32_t)v == source ? 0 : kInf) << 32;
    if (op == OP_CC) a.word[v] = (unsigned long long)v << 32;
    if (op == OP_KCORE) a.level[v] = a.off[v + 1] - a.off[v];
    if (op == OP_PR) {
      a.rank[v] = r0;
      a.acc[v] = 0ull;
    }
  }
  for (size_t i = t; i < kBarWords; i += stride) a.bar[i] = 0ull;
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    Ctl *c = a.ctl;
    c->qcount[0] = nfront0;
    c->qcount[1] = 0;
    c->qcount[2] = 0;
    c->chunk[0] = c->chunk[1] = c->chunk[2] = 0;
    c->overflow = 0xffffffffu;
    c->huge[0] = 0;
    c->huge[1] = 0;
    c->abort = 0;
    c->rounds = 0;
    c->st_frontier = c->st_edges_twc = c->st_edges_lb = c->st_huge_v = c->st_pushes = 0;
    c->dangling[0] = 0;
    c->dangling[1] = 0;
    c->filt_count[0] = c->filt_count[1] = 0;
    c->members = 0;
    c->n_members = 0;
    c->diag_seen = c->diag_target = 0;
    c->diag_round = 0;
    c->threshold_used = a.threshold;
    for (int k = 0; k < kProfParts; ++k) c->prof[k] = 0;
    c->t_begin = c->t_end = 0;
    if (source >= 0 && op != OP_RECORD) ((int32_t *)a.q0)[0] = source;
  }
}

__global__ void k_finish(Args a, int op) {
  const uint32_t stride = gridDim.x * blockDim.x;
  for (uint32_t v = blockIdx.x * blockDim.x + threadIdx.x; v < (uint32_t)a.n; v += stride)
    a.out[v] = op == OP_KCORE ? (int32_t)(a.level[v] >= a.kcore_k) : (int32_t)(a.word[v] >> 32);
}

// Batch set-up, part 1: every label of every query to INF, barrier words and
// the control block cleared (the sources are seeded by k_seed_batch after).
__global__ void k_init_batch(Args a, int op) {
  const size_t stride = (size_t)gridDim.x * blockDim.x;
  const size_t t = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  for (size_t i = t; i < (size_t)a.nlabels; i += stride) {
    if (op == OP_BFS) a.level[i] = kInf;
    if (op == OP_SSSP) a.word[i] = (unsigned long long)(uint32_t)kInf << 32;
  }
  for (size_t i = t; i < kBarWords; i += stride) a.bar[i] = 0ull;
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    Ctl *c = a.ctl;
    c->qcount[0] = (uint32_t)a.nq;
    c->qcount[1] = c->qcount[2] = 0;
    c->chunk[0] = c->chunk[1] = c->chunk[2] = 0;
    c->overflow = 0xffffffffu;
    c->huge[0] = c->huge[1] = 0;
    c->abort = 0;
    c->rounds = 0;
    c->st_frontier = c->st_edges_twc = c->st_edges_lb = c->st_huge_v = c->st_pushes = 0;
    c->dangling[0] = c->dangling[1] = 0;
    c->members = 0;
    c->n_members = 0;
    c->diag_seen = c->diag_target = 0;
    c->diag_round = 0;
    c->threshold_used = a.threshold;
    for (int k = 0; k < kProfParts; ++k) c->prof[k] = 0;
    c->t_begin = c->t_end = 0;
  }
}

// Batch set-up, part 2: query q's source gets label 0 and is entry q of the
// first worklist.
__global__ void k_seed_batch(Args a, int op) {
  for (int32_t q = blockIdx.x * blockDim.x + threadIdx.x; q < a.nq; q += gridDim.x * blockDim.x) {
    const int32_t s = a.qsrc[q];
    const long long l = a.qoff[q] + s;
    if (op == OP_BFS) a.level[l] = 0;
    if (op == OP_SSSP) a.word[l] = 0ull;
    ((unsigned long long *)a.q0)[q] = ((unsigned long long)(uint32_t)q << 32) | (uint32_t)s;
  }
}

// Batch outputs: query blockIdx.y, its vertices strided over blockIdx.x.
__global__ void k_finish_batch(Args a, int op) {
  const int32_t q = blockIdx.y;
  const int32_t n = a.qn[q];
  const long long base = a.qlbase[q];
  int32_t *out = a.qout[q];
  for (int32_t v = blockIdx.x * blockDim.x + threadIdx.x; v < n; v += gridDim.x * blockDim.x)
    out[v] = op == OP_BFS ? a.level[base + v] : (int32_t)(a.word[base + v] >> 32);
}

template <int B, class Op>
__global__ __launch_bounds__(B) void k_twc(Args a, Op op) {
  __shared__ Smem<B, Op> sm;
  Acc acc;
  const int r = a.round;
  const uint32_t nF = round_size(a, r);
  if (blockIdx.x == 0 && threadIdx.x == 0) clear_ahead(a, r);
  const Grid gr{blockIdx.x, gridDim.x};
  const int64_t thr = round_threshold(a, nF, (uint64_t)gr.n * B);
  phase_twc<B, Op, false>(a, op, sm, gr, r, round_frontier<false>(a, r), nF, round_next<false>(a, r),
                          &a.ctl->qcount[(r + 1) % 3],
                   &a.ctl->huge[r & 1], thr, hint_shift(thr), acc);
  if constexpr (Op::kPR) flush_dangling<B, Op>(acc, sm, &a.ctl->dangling[r & 1]);
  flush_stats<B, Op>(acc, sm, a.ctl);
}

template <int B, class Op>
__global__ __launch_bounds__(B) void k_lb(Args a, Op op) {
  __shared__ Smem<B, Op> sm;
  Acc acc;
  const int r = a.round;
  const unsigned long long hc = ld_relaxed(&a.ctl->huge[r & 1]);
  const int64_t thr = round_threshold(a, round_size(a, r), (uint64_t)gridDim.x * B);
  phase_lb<B, Op, false>(a, op, sm, Grid{blockIdx.x, gridDim.x}, r, hc, round_next<false>(a, r),
                         &a.ctl->qcount[(r + 1) % 3],
                  hint_shift(thr), acc);
  flush_stats<B, Op>(acc, sm, a.ctl);
}

template <int B>
__global__ __launch_bounds__(B) void k_pr_update(Args a) {
  phase_pr_update<B>(a, Grid{blockIdx.x, gridDim.x}, ld_relaxed(&a.ctl->dangling[a.round & 1]));
  if (blockIdx.x == 0 && threadIdx.x == 0) st_relaxed(&a.ctl->rounds, (uint32_t)a.round + 1u);
}

// The filter bitmap (BFS: reached; CC: label 0): word x holds vertices
// [32x, 32x + 32).  Each wavefront of the members tests 64 consecutive
// vertices (coalesced loads), two of its lanes store the ballot's halves,
// and lane 0 adds the set bits to *count.
template <int B, class Op>
__device__ __forceinline__ void build_filter(const Args &a, Grid gr, unsigned long long *count) {
  const uint32_t n = (uint32_t)a.n;
  const uint32_t words = (n + 31u) / 32u;
  const uint32_t lane = lane_id();
  const uint32_t nwaves = (uint32_t)gr.n * (B / kWave);
  unsigned long long set = 0;
  for (uint32_t base = ((uint32_t)gr.id * (B / kWave) + threadIdx.x / kWave) * kWave; base < n;
       base += nwaves * kWave) {
    const uint32_t v = base + lane;
    const unsigned long long m = __ballot(v < n && Filtered<Op>::bit(a, v));
    const uint32_t x = base / 32u + lane;
    if (lane < 2 && x < words) a.vbits[x] = (uint32_t)(m >> (32 * lane));
    set += (unsigned long long)__popcll(m);
  }
  if (lane == 0 && set) add_relaxed(count, set);
}

// F: BFS or CC with the filter bitmap (a kernel of its own, so that every
// other launch runs code without it).
template <int B, class Op, bool M, bool F = false>
__global__ __launch_bounds__(B) __attribute__((amdgpu_waves_per_eu(ALB_WAVES_PER_EU))) void k_persistent(Args a,
                                                                                                           Op op) {
  __shared__ Smem<B, Op, M> sm;
  Acc acc;
  Grid gr;
  bool joined;
  if constexpr (F) {  // the filtering kernel has two operator types' phases: everything inlined
    [[clang::always_inline]] joined = join_members(a, sm, &gr);
  } else {
    joined = join_members(a, sm, &gr);
  }
  if (!joined) return;
  if (a.threshold < 0) a.threshold = (int64_t)gr.n * B;  // the launched thread count (the paper's rule)
  unsigned long long epoch = 0, prof_last = 0;
  uint64_t reached = 0;  // BFS: vertices in the worklists so far (each is in exactly one round's)
  bool filtered = false;  // the filter bitmap is in use
  int r = 0;
  for (; r < a.max_rounds; ++r) {
    if (ld_relaxed(&a.ctl->overflow) < (uint32_t)r) break;  // set in an earlier round: seen by all alike
    const uint32_t nF = round_size(a, r);
    if (nF == 0) break;
    if constexpr (F) {
      // BFS: once half of the vertices have been reached (every member
      // decides alike from the worklist sizes), most edges lead to reached
      // vertices: build the bitmap once and filter from this round on.
      // CC: from round 1 on, rebuild the bitmap of label-0 vertices at each
      // round's start and filter once they are at least half of all.
      // k-core: the same from round 0 on, with the vertices below k.
      bool build = false;
      if constexpr (std::is_same<Op, OpBFS>::value) {
        reached += nF;
        build = !filtered && 2 * reached >= (uint64_t)a.n;
      } else if constexpr (std::is_same<Op, OpCC>::value) {
        build = r >= 1;
      } else {
        build = true;
      }
      // the next round's count: nobody reads it before then (this round's
      // members read [r & 1] right after the build's barrier)
      if (gr.id == 0 && threadIdx.x == 0) st_relaxed(&a.ctl->filt_count[(r + 1) & 1], 0ull);
      if (build) {
        build_filter<B, Op>(a, gr, &a.ctl->filt_count[r & 1]);
        bool ok;
        [[clang::always_inline]] ok = grid_barrier(a, sm, gr, epoch, r);
        if (!ok) break;
        if constexpr (std::is_same<Op, OpBFS>::value)
          filtered = true;
        else
          filtered = 2 * ld_relaxed(&a.ctl->filt_count[r & 1]) >= (unsigned long long)a.n;
      }
    }
    const bool tl = gr.id == 0 && threadIdx.x == 0 && r < kTimeline;
    if (gr.id == 0 && threadIdx.x == 0) clear_ahead(a, r);
    if (tl) a.ctl->tl[4 * r] = (unsigned long long)wall_clock64();
    Entry<M> *qn = round_next<M>(a, r);
    uint32_t *qn_cnt = &a.ctl->qcount[(r + 1) % 3];
    const int64_t thr = round_threshold(a, nF, (uint64_t)gr.n * B);
    // batch with per-query thresholds: chunk index sized for the smallest one
    const uint32_t hs = hint_shift(M && a.qthr ? a.qthr_min : thr);
    if constexpr (F) {  // two operator types here: both phases inlined
      if (filtered) {
        using FOp = typename Filtered<Op>::type;
        const FOp fop = Filtered<Op>::make(op, a);
        [[clang::always_inline]] phase_twc<B, FOp, M>(a, fop, sm, gr, r, round_frontier<M>(a, r), nF, qn, qn_cnt,
                                                      &a.ctl->huge[r & 1], thr, hs, acc);
      } else {
        [[clang::always_inline]] phase_twc<B, Op, M>(a, op, sm, gr, r, round_frontier<M>(a, r), nF, qn, qn_cnt,
                                                     &a.ctl->huge[r & 1], thr, hs, acc);
      }
    } else {
      phase_twc<B, Op, M>(a, op, sm, gr, r, round_frontier<M>(a, r), nF, qn, qn_cnt, &a.ctl->huge[r & 1], thr, hs,
                          acc);
    }
    if constexpr (Op::kPR) flush_dangling<B, Op>(acc, sm, &a.ctl->dangling[r & 1]);
    uint64_t pb = a.profile ? (uint64_t)wall_clock64() : 0;
    bool ok1;
    if constexpr (F) {
      [[clang::always_inline]] ok1 = grid_barrier(a, sm, gr, epoch, r);
    } else {
      ok1 = grid_barrier(a, sm, gr, epoch, r);
    }
    if (!ok1) break;
    prof_mark(a, acc, kProfBarrier, pb);
    const unsigned long long hc = ld_relaxed(&a.ctl->huge[r & 1]);
    if (tl) {
      a.ctl->tl[4 * r + 1] = (unsigned long long)wall_clock64();
      a.ctl->tl[4 * r + 3] = (unsigned long long)nF | ((hc >> 32) << 32);
    }
    if ((hc >> 32) != 0) {  // the execution phase runs only when there is imbalance to fix
      if constexpr (F) {
        if (filtered) {
          using FOp = typename Filtered<Op>::type;
          const FOp fop = Filtered<Op>::make(op, a);
          [[clang::always_inline]] phase_lb<B, FOp, M>(a, fop, sm, gr, r, hc, qn, qn_cnt, hs, acc);
        } else {
          [[clang::always_inline]] phase_lb<B, Op, M>(a, op, sm, gr, r, hc, qn, qn_cnt, hs, acc);
        }
      } else {
        phase_lb<B, Op, M>(a, op, sm, gr, r, hc, qn, qn_cnt, hs, acc);
      }
      pb = a.profile ? (uint64_t)wall_clock64() : 0;
      bool ok2;
      if constexpr (F) {
        [[clang::always_inline]] ok2 = grid_barrier(a, sm, gr, epoch, r);
      } else {
        ok2 = grid_barrier(a, sm, gr, epoch, r);
      }
      if (!ok2) break;
      prof_mark(a, acc, kProfBarrier, pb);
    }
    if (tl) a.ctl->tl[4 * r + 2] = (unsigned long long)wall_clock64();
    if (a.prof_wg) prof_round_edges(a, acc, prof_last, gr.id, r);
    if constexpr (Op::kPR) {
      phase_pr_update<B>(a, gr, ld_relaxed(&a.ctl->dangling[r & 1]));
      if (!grid_barrier(a, sm, gr, epoch, r)) break;
    }
  }
  if (gr.id == 0 && threadIdx.x == 0) {
    st_relaxed(&a.ctl->rounds, (uint32_t)r);
    st_relaxed(&a.ctl->threshold_used, (long long)a.threshold);
    st_relaxed(&a.ctl->t_end, (unsigned long long)wall_clock64());
  }
  if constexpr (F) {
    [[clang::always_inline]] flush_stats<B, Op>(acc, sm, a.ctl);
  } else {
    flush_stats<B, Op>(acc, sm, a.ctl);
  }
}

// ---------------------------------------------------------------------------
// Continuous serving: one persistent batch launch that queries join between
// rounds.  Round r is two phases, as a batch's:
//   phase 1  inspection and TWC over round r's worklist (recording, per
//            slot, that it had an entry this round); workgroup 0 then takes
//            the requests the host has published into their slots (tables
//            only) and decides whether the launch ends;
//   -------- grid barrier
//   phase 2  workgroup 0 marks the active slots without an entry this round
//            as finished (their labels have been final since round r - 1);
//            every member initialises the newly admitted slots' labels and
//            writes the labels of the slots finished in round r - 1 to
//            open_out as int32; workgroup 0 appends the new sources to round
//            r + 1's worklist; then the cyclic phase of round r;
//   -------- grid barrier
//   workgroup 0 publishes the slots converted this round to the host.
// A request published while others are on the device thus starts at the
// next round boundary, beside them.  Everything member 0 decides for round r
// (admissions, exit) sits in [r & 1] entries: with only two barriers per
// round a slow member may still read round r's entry while member 0 already
// writes round r + 1's.
// ---------------------------------------------------------------------------
template <class T>
__device__ __forceinline__ T ld_sys(T *p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
}
template <class T>
__device__ __forceinline__ void st_sys(T *p, T v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
}

// Workgroup 0, thread 0, at the end of round r's phase 1: take the published
// requests (at most the ring's size; the host bounds them by its free slots)
// into their slots' tables, list them for phase 2 (admit_n[r & 1]), and
// decide whether the launch ends after this round's first barrier.
__device__ void open_admit(const Args &a, int r, uint32_t nF) {
  Ctl *c = a.ctl;
  OpenShared *sh = a.open;
  const unsigned long long tail = ld_sys(&sh->tail);
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "");  // the entries below were written before the tail
  const unsigned long long head = c->open_head;
  int32_t *admit = a.q_admit + (size_t)(r & 1) * kOpenRing;
  uint32_t k = 0;
  for (unsigned long long i = head; i < tail && k < (uint32_t)kOpenRing; ++i, ++k) {
    OpenReq *q = &sh->req[i % kOpenRing];
    const int32_t slot = ld_sys(&q->slot);
    if (slot < 0 || slot >= a.nslots) {  // cannot happen with a well-formed ring: stop taking requests
      flag_overflow(c, r);
      break;
    }
    admit[k] = slot;
    ((long long *)a.qoff)[slot] = ld_sys(&q->qoff);
    ((long long *)a.qlbase)[slot] = ld_sys(&q->lbase);
    ((int32_t *)a.qsrc)[slot] = ld_sys(&q->src);
    ((int32_t *)a.qn)[slot] = ld_sys(&q->n);
    a.q_unit[slot] = ld_sys(&q->unit);
    a.q_out[slot] = (int32_t *)ld_sys(&q->out);
    a.q_last[slot] = r;  // not finished in this round's phase 2: its source is in round r + 1's worklist
    a.q_active[slot] = 1;
  }
  c->open_head = head + k;
  st_sys(&sh->head, head + k);
  c->admit_n[r & 1] = k;
  c->open_active += k;
  uint32_t ex = 0;
  const bool idle = k == 0 && nF == 0 && c->open_active == 0 && c->conv_n[r & 1] == 0;
  if (!idle) {
    c->idle_since = 0;
  } else {
    const uint64_t now = (uint64_t)wall_clock64();
    if (ld_sys(&sh->stop)) ex = 1;
    if (c->idle_since == 0) c->idle_since = now;
    else if (now - c->idle_since > a.idle_ticks) ex = 1;
    __builtin_amdgcn_s_sleep(8);  // idle: poll the ring less often
  }
  c->open_exit[r & 1] = ex;
}

// Workgroup 0 after round r's first barrier: an active slot without an
// entry in round r's worklist has finished.  It is listed for round r + 1's
// conversion (q_conv[(r + 1) & 1], conv_n[(r + 1) & 1]).
template <int B>
__device__ void open_complete(const Args &a, int r, uint32_t *s_cnt) {
  Ctl *c = a.ctl;
  int32_t *list = a.q_conv + (size_t)((r + 1) & 1) * kOpenRing;
  if (threadIdx.x == 0) *s_cnt = 0;
  __syncthreads();
  for (int32_t q = threadIdx.x; q < a.nslots; q += B) {
    if (a.q_active[q] && ld_relaxed(&a.q_last[q]) != r) {
      a.q_active[q] = 0;
      list[atomicAdd(s_cnt, 1u)] = q;
    }
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    c->conv_n[(r + 1) & 1] = *s_cnt;
    c->open_active -= *s_cnt;
  }
  __syncthreads();
}

// Every member in round r's phase 2: the slots admitted in round r get their
// labels (INF, the source 0); the slots finished in round r - 1 get theirs
// written as int32 (SSSP: the distance half of the label word; BFS: the
// level) into the caller's pinned output, or into open_out.  Workgroup 0 then appends the new sources to round
// r + 1's worklist.
template <class Op>
__device__ void open_prepare(const Args &a, Grid gr, int B, int r, uint32_t k, uint32_t nc) {
  const int32_t *admit = a.q_admit + (size_t)(r & 1) * kOpenRing;
  for (uint32_t i = 0; i < k; ++i) {
    const int32_t slot = admit[i];
    const long long base = a.qlbase[slot];
    const long long sl = a.qoff[slot] + a.qsrc[slot];
    const int32_t n = a.qn[slot];
    for (int32_t v = (int32_t)(gr.id * B + threadIdx.x); v < n; v += (int32_t)(gr.n * B)) {
      const long long l = base + v;
      if constexpr (std::is_same<Op, OpBFS>::value)
        a.level[l] = l == sl ? 0 : kInf;
      else
        a.word[l] = l == sl ? 0ull : (unsigned long long)(uint32_t)kInf << 32;
    }
  }
  const int32_t *conv = a.q_conv + (size_t)(r & 1) * kOpenRing;
  for (uint32_t i = 0; i < nc; ++i) {
    const int32_t slot = conv[i];
    const long long base = a.qlbase[slot];
    const int32_t n = a.qn[slot];
    int32_t *dst = a.q_out[slot];  // the caller's pinned array, else the lane's output area
    if (!dst) dst = a.open_out + base;
    for (int32_t v = (int32_t)(gr.id * B + threadIdx.x); v < n; v += (int32_t)(gr.n * B)) {
      if constexpr (std::is_same<Op, OpBFS>::value)
        dst[v] = a.level[base + v];
      else
        dst[v] = (int32_t)(a.word[base + v] >> 32);
    }
  }
  if (k && gr.id == 0 && threadIdx.x == 0) {
    unsigned long long *F = (unsigned long long *)(((r + 1) & 1) ? a.q1 : a.q0);
    const uint32_t at = add_relaxed(&a.ctl->qcount[(r + 1) % 3], k);  // beside the cyclic phase's pushes
    for (uint32_t i = 0; i < k; ++i) {
      const int32_t slot = admit[i];
      if (at + i < a.qcap)
        F[at + i] = ((unsigned long long)(uint32_t)slot << 32) | (uint32_t)a.qsrc[slot];
      else
        flag_overflow(a.ctl, r);
    }
  }
}

// Workgroup 0, thread 0, after round r's second barrier: the slots converted
// in round r go to the completion ring after a system-scope release, so
// that their int32 labels are in memory when the host copies them.
__device__ void open_publish(const Args &a, int r, uint32_t nc) {
  Ctl *c = a.ctl;
  OpenShared *sh = a.open;
  const int32_t *list = a.q_conv + (size_t)(r & 1) * kOpenRing;
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "");
  for (uint32_t j = 0; j < nc; ++j) st_sys(&sh->fin[(c->open_done + j) % kOpenRing], list[j]);
  c->open_done += nc;
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "");
  st_sys(&sh->done, c->open_done);
}

template <int B, class Op>
__global__ __launch_bounds__(B) __attribute__((amdgpu_waves_per_eu(ALB_WAVES_PER_EU))) void k_open(Args a, Op op) {
  __shared__ Smem<B, Op, true> sm;
  __shared__ uint32_t s_cnt;
  Acc acc;
  Grid gr;
  if (!join_members(a, sm, &gr)) return;
  if (a.threshold < 0) a.threshold = (int64_t)gr.n * B;
  if (gr.id == 0 && threadIdx.x == 0) st_sys(&a.open->live, 1u);
  unsigned long long epoch = 0;
  int r = 0;
  for (;; ++r) {
    if (ld_relaxed(&a.ctl->overflow) < (uint32_t)r) break;
    const uint32_t nF = round_size(a, r);
    const bool tl = gr.id == 0 && threadIdx.x == 0 && r < kTimeline;
    if (gr.id == 0 && threadIdx.x == 0) clear_ahead(a, r);
    if (tl) a.ctl->tl[4 * r] = (unsigned long long)wall_clock64();
    Entry<true> *qn = round_next<true>(a, r);
    uint32_t *qn_cnt = &a.ctl->qcount[(r + 1) % 3];
    const int64_t thr = round_threshold(a, nF, (uint64_t)gr.n * B);
    const uint32_t hs = hint_shift(thr);
    if (nF)
      phase_twc<B, Op, true>(a, op, sm, gr, r, round_frontier<true>(a, r), nF, qn, qn_cnt, &a.ctl->huge[r & 1],
                             thr, hs, acc);
    if (gr.id == 0 && threadIdx.x == 0) open_admit(a, r, nF);
    if (!grid_barrier(a, sm, gr, epoch, r)) break;
    if (ld_relaxed(&a.ctl->open_exit[r & 1])) break;
    if (gr.id == 0) open_complete<B>(a, r, &s_cnt);
    const uint32_t k = ld_relaxed(&a.ctl->admit_n[r & 1]);
    const uint32_t nc = ld_relaxed(&a.ctl->conv_n[r & 1]);
    open_prepare<Op>(a, gr, B, r, k, nc);
    const unsigned long long hc = nF ? ld_relaxed(&a.ctl->huge[r & 1]) : 0ull;
    if (tl) {
      a.ctl->tl[4 * r + 1] = (unsigned long long)wall_clock64();
      a.ctl->tl[4 * r + 3] = (unsigned long long)nF | ((hc >> 32) << 32);
    }
    if ((hc >> 32) != 0) phase_lb<B, Op, true>(a, op, sm, gr, r, hc, qn, qn_cnt, hs, acc);
    // a round that wrote finished labels into host memory releases them at
    // system scope on every XCD before workgroup 0 publishes the slots
    if (!grid_barrier(a, sm, gr, epoch, r, nc != 0)) break;
    if (tl) a.ctl->tl[4 * r + 2] = (unsigned long long)wall_clock64();
    if (nc && gr.id == 0 && threadIdx.x == 0) open_publish(a, r, nc);
  }
  if (gr.id == 0 && threadIdx.x == 0) {
    st_relaxed(&a.ctl->rounds, (uint32_t)r);
    st_relaxed(&a.ctl->threshold_used, (long long)a.threshold);
    st_relaxed(&a.ctl->t_end, (unsigned long long)wall_clock64());
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "");
    st_sys(&a.open->live, 0u);
  }
  flush_stats<B, Op>(acc, sm, a.ctl);
}

// Continuous serving set-up: control block, barrier words, slot flags.
__global__ void k_init_open(Args a) {
  const size_t stride = (size_t)gridDim.x * blockDim.x;
  const size_t t = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  for (size_t i = t; i < kBarWords; i += stride) a.bar[i] = 0ull;
  for (size_t i = t; i < (size_t)a.nslots; i += stride) {
    a.q_active[i] = 0;
    a.q_last[i] = -1;
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    Ctl *c = a.ctl;
    c->qcount[0] = c->qcount[1] = c->qcount[2] = 0;
    c->chunk[0] = c->chunk[1] = c->chunk[2] = 0;
    c->overflow = 0xffffffffu;
    c->huge[0] = c->huge[1] = 0;
    c->abort = 0;
    c->rounds = 0;
    c->st_frontier = c->st_edges_twc = c->st_edges_lb = c->st_huge_v = c->st_pushes = 0;
    c->dangling[0] = c->dangling[1] = 0;
    c->members = 0;
    c->n_members = 0;
    c->diag_seen = c->diag_target = 0;
    c->diag_round = 0;
    c->threshold_used = a.threshold;
    for (int k = 0; k < kProfParts; ++k) c->prof[k] = 0;
    c->t_begin = c->t_end = 0;
    c->open_head = 0;
    c->admit_n[0] = c->admit_n[1] = 0;
    c->open_done = 0;
    c->open_active = 0;
    c->open_exit[0] = c->open_exit[1] = 0;
    c->conv_n[0] = c->conv_n[1] = 0;
    c->idle_since = 0;
  }
}

// ---------------------------------------------------------------------------
// Pull PageRank (the paper's pr, Section 5): each vertex v sums its
// in-neighbours' contributions c(u) = rank(u) / outdeg(u) over the transposed
// graph, so no atomic touches a destination label except for the edges of
// huge in-degree vertices.  Inspection and bins work on in-degrees: the TWC
// bins reduce each vertex's sum inside one workgroup, wavefront or lane and
// store it once; the huge vertices' in-edges take the cyclic distribution of
// Algorithm 2, each wavefront adds its lanes' contributions per vertex
// (segmented by the owning vertex) with one atomic per segment.  The sums use
// the same exact 64-bit fixed point as the push version, so both give
// bitwise the same ranks.
// ---------------------------------------------------------------------------
struct OpPRPull {  // type facts for Smem only; the pull phases do the work
  using val_t = float;
  struct pre_t {};
  static constexpr bool kPush = false, kNeedSrc = false, kRecord = false, kPR = true, kBatch = false;
};

// Fixed-point contributions of up to kU in-edges per lane, loads issued first.
__device__ __forceinline__ unsigned long long pull_edges(const Args &a, const bool (&act)[kU],
                                                         const int32_t (&pos)[kU]) {
  int32_t u[kU];
#pragma unroll
  for (int i = 0; i < kU; ++i) u[i] = a.tcol[act[i] ? pos[i] : 0];
  float c[kU];
#pragma unroll
  for (int i = 0; i < kU; ++i) c[i] = a.contrib[u[i]];
  unsigned long long x = 0;
#pragma unroll
  for (int i = 0; i < kU; ++i) x += act[i] ? to_fix(c[i]) : 0ull;
  return x;
}

template <int B>
__device__ unsigned long long block_sum(unsigned long long x, Smem<B, OpPRPull> &sm) {
#pragma unroll
  for (int d = kWave / 2; d > 0; d >>= 1) x += __shfl_xor(x, d);
  if (lane_id() == 0) sm.dred[threadIdx.x / kWave] = x;
  __syncthreads();
  unsigned long long t = 0;
#pragma unroll
  for (int j = 0; j < B / kWave; ++j) t += sm.dred[j];
  __syncthreads();
  return t;
}

template <int B>
__device__ void pull_gather(const Args &a, Smem<B, OpPRPull> &sm, Grid gr, int it, int64_t thr, uint32_t hs,
                            Acc &acc) {
  const int tid = threadIdx.x;
  const uint32_t lane = lane_id();
  const uint32_t nF = (uint32_t)a.n;
  Claims cl(nF, gr, B);
  for (;;) {
    if (tid == 0) cl.next(&a.ctl->chunk[it % 3], nF, gr, B, sm.cbase, sm.clen);
    __syncthreads();
    const unsigned long long base = sm.cbase;
    const uint32_t C = sm.clen;
    if (base >= nF) break;
    const uint32_t i = (uint32_t)base + tid;
    const bool mine = tid < (int)C && i < nF;
    int32_t v = -1, beg = 0, deg = 0;
    if (mine) {
      v = (int32_t)i;
      beg = a.toff[v];
      deg = a.toff[v + 1] - beg;
    }
    // inspection by in-degree (Algorithm 1); huge vertices wait for phase 2
    const bool huge = deg > 0 && (int64_t)deg >= thr;
    reserve_huge(huge, v, beg, deg, 0, a, it, &a.ctl->huge[it & 1], hs, acc);
    if (huge) deg = 0;
    acc.frontier += mine;
    acc.edges_twc += (unsigned long long)deg;

    // workgroup bin: the workgroup sums one vertex's in-edges, then stores
    for (;;) {
      if (tid == 0) sm.owner = -1;
      __syncthreads();
      if (deg >= a.c_wg) sm.owner = tid;
      __syncthreads();
      const int32_t o = sm.owner;
      if (o < 0) break;
      if (tid == o) {
        sm.obeg = beg;
        sm.odeg = deg;
        sm.ov = v;
        deg = 0;
      }
      __syncthreads();
      const int32_t ob = sm.obeg, od = sm.odeg, ov = sm.ov;
      unsigned long long x = 0;
      for (int32_t j0 = 0; j0 < od; j0 += kU * B) {
        bool act[kU];
        int32_t pos[kU];
#pragma unroll
        for (int u = 0; u < kU; ++u) {
          act[u] = j0 + u * B + tid < od;
          pos[u] = ob + j0 + u * B + tid;
        }
        x += pull_edges(a, act, pos);
      }
      x = block_sum<B>(x, sm);
      if (tid == 0) a.acc[ov] = x;
    }
    // wavefront bin: one wavefront sums one vertex's in-edges
    for (;;) {
      const unsigned long long mm = __ballot(deg >= a.c_wave && deg > 0);
      if (mm == 0ull) break;
      const int ld = __ffsll(mm) - 1;
      const int32_t ob = __shfl(beg, ld), od = __shfl(deg, ld), ov = __shfl(v, ld);
      if ((int)lane == ld) deg = 0;
      unsigned long long x = 0;
      for (int32_t j0 = 0; j0 < od; j0 += kU * kWave) {
        bool act[kU];
        int32_t pos[kU];
#pragma unroll
        for (int u = 0; u < kU; ++u) {
          act[u] = j0 + u * kWave + (int32_t)lane < od;
          pos[u] = ob + j0 + u * kWave + (int32_t)lane;
        }
        x += pull_edges(a, act, pos);
      }
#pragma unroll
      for (int d = kWave / 2; d > 0; d >>= 1) x += __shfl_xor(x, d);
      if ((int)lane == ld) a.acc[ov] = x;
    }
    // thread bin: each lane sums its own short list (fewer than c_wave edges)
    if (deg > 0) {
      unsigned long long x = 0;
      for (int32_t j0 = 0; j0 < deg; j0 += kU) {
        bool act[kU];
        int32_t pos[kU];
#pragma unroll
        for (int u = 0; u < kU; ++u) {
          act[u] = j0 + u < deg;
          pos[u] = beg + j0 + u;
        }
        x += pull_edges(a, act, pos);
      }
      a.acc[v] = x;
    }
    // vertices without in-edges keep the 0 the update phase left
  }
}

template <int B>
__device__ void pull_lb(const Args &a, Grid gr, unsigned long long hc, uint32_t hs, Acc &acc) {
  const uint32_t vh = (uint32_t)(hc >> 32);
  const uint32_t e = (uint32_t)hc;
  if (vh == 0 || ld_relaxed(&a.ctl->overflow) != 0xffffffffu) return;
  const uint64_t T = (uint64_t)gr.n * B;
  const uint32_t lane = lane_id();
  const uint64_t g = (uint64_t)gr.id * B + threadIdx.x;
  for (uint64_t k0 = g - lane; k0 < e; k0 += kU * T) {
#pragma unroll
    for (int u = 0; u < kU; ++u) {
      const uint64_t k = k0 + lane + (uint64_t)u * T;
      const bool act = k < e;
      int32_t v = -1;
      unsigned long long x = 0;
      if (act) {
        const int4 r = a.huge_rec[owner_of(a, vh, hs, (uint32_t)k)];
        v = r.z;
        x = to_fix(a.contrib[a.tcol[r.y + (int32_t)((uint32_t)k - (uint32_t)r.x)]]);
      }
      acc.edges_lb += act;
      // consecutive lanes hold consecutive huge edges, so lanes of one vertex
      // form one run: add each run with one atomic from its last lane
      unsigned long long incl = x;
#pragma unroll
      for (int d = 1; d < kWave; d <<= 1) {
        const unsigned long long y = __shfl_up(incl, d);
        if ((int)lane >= d) incl += y;
      }
      const int32_t vprev = __shfl_up(v, 1), vnext = __shfl_down(v, 1);
      const unsigned long long heads = __ballot(lane == 0 || v != vprev);
      const int start = 63 - __builtin_clzll(heads & ((2ull << lane) - 1ull));
      const unsigned long long before = __shfl(incl, start > 0 ? start - 1 : 0);
      const bool tail = lane == kWave - 1 || v != vnext;
      if (act && tail) add_relaxed(&a.acc[v], incl - (start > 0 ? before : 0ull));
    }
  }
}

// rank(v) from the sums, the next contributions, the next dangling mass.
template <int B>
__device__ void pull_update(const Args &a, Smem<B, OpPRPull> &sm, Grid gr, int it, Acc &acc) {
  const double d = (double)a.damping;
  const double N = (double)a.n;
  const unsigned long long dfix = ld_relaxed(&a.ctl->dangling[it & 1]);
  const double base = (1.0 - d) / N + d * ((double)dfix * kFixInv) / N;
  for (uint32_t v = gr.id * B + threadIdx.x; v < (uint32_t)a.n; v += gr.n * B) {
    const float r = (float)(base + d * ((double)a.acc[v] * kFixInv));
    a.rank[v] = r;
    a.acc[v] = 0ull;  // huge vertices' sums start from 0 in the next phase 2
    const int32_t od = a.off[v + 1] - a.off[v];
    a.contrib[v] = od > 0 ? r / (float)od : 0.0f;
    if (od == 0) acc.dangling += to_fix(r);
  }
  flush_dangling<B, OpPRPull>(acc, sm, &a.ctl->dangling[(it + 1) & 1]);
}

template <int B>
__global__ __launch_bounds__(B) __attribute__((amdgpu_waves_per_eu(ALB_WAVES_PER_EU))) void k_pull_pr(Args a) {
  __shared__ Smem<B, OpPRPull> sm;
  Acc acc;
  Grid gr;
  if (!join_members(a, sm, &gr)) return;
  if (a.threshold < 0) a.threshold = (int64_t)gr.n * B;
  const uint32_t hs = hint_shift(a.threshold);
  unsigned long long epoch = 0;
  int it = 0;
  for (; it < a.max_rounds; ++it) {
    if (gr.id == 0 && threadIdx.x == 0) {
      st_relaxed(&a.ctl->chunk[(it + 1) % 3], 0ull);
      st_relaxed(&a.ctl->huge[(it + 1) & 1], 0ull);
      st_relaxed(&a.ctl->dangling[(it + 1) & 1], 0ull);
    }
    pull_gather<B>(a, sm, gr, it, a.threshold, hs, acc);
    if (!grid_barrier(a, sm, gr, epoch, it)) break;
    const unsigned long long hc = ld_relaxed(&a.ctl->huge[it & 1]);
    if ((hc >> 32) != 0) {
      pull_lb<B>(a, gr, hc, hs, acc);
      if (!grid_barrier(a, sm, gr, epoch, it)) break;
    }
    pull_update<B>(a, sm, gr, it, acc);
    if (!grid_barrier(a, sm, gr, epoch, it)) break;
  }
  if (gr.id == 0 && threadIdx.x == 0) {
    st_relaxed(&a.ctl->rounds, (uint32_t)it);
    st_relaxed(&a.ctl->threshold_used, (long long)a.threshold);
  }
  flush_stats<B, OpPRPull>(acc, sm, a.ctl);
}

// Pull set-up after k_init: contributions of the initial ranks and the
// initial dangling mass (block sums, one atomic per workgroup).
__global__ __launch_bounds__(256) void k_pull_prepare(Args a) {
  __shared__ unsigned long long part[256 / kWave];
  unsigned long long x = 0;
  const float r0 = 1.0f / (float)a.n;
  for (uint32_t v = blockIdx.x * blockDim.x + threadIdx.x; v < (uint32_t)a.n; v += gridDim.x * blockDim.x) {
    const int32_t od = a.off[v + 1] - a.off[v];
    a.contrib[v] = od > 0 ? r0 / (float)od : 0.0f;
    if (od == 0) x += to_fix(r0);
  }
#pragma unroll
  for (int d = kWave / 2; d > 0; d >>= 1) x += __shfl_xor(x, d);
  if (lane_id() == 0) part[threadIdx.x / kWave] = x;
  __syncthreads();
  if (threadIdx.x == 0) {
    unsigned long long t = 0;
    for (int j = 0; j < 256 / kWave; ++j) t += part[j];
    if (t) add_relaxed(&a.ctl->dangling[0], t);
  }
}

// ---------------------------------------------------------------------------
// Dispatch over workgroup size and operator.
// ---------------------------------------------------------------------------

template <int B, class Op>
struct TwcF {
  static hipError_t run(int grid, const Args *a, hipStream_t s) {
    hipLaunchKernelGGL((k_twc<B, Op>), dim3(grid), dim3(B), 0, s, *a, make_op<Op>(*a));
    return hipGetLastError();
  }
};
template <int B, class Op>
struct LbF {
  static hipError_t run(int grid, const Args *a, hipStream_t s) {
    hipLaunchKernelGGL((k_lb<B, Op>), dim3(grid), dim3(B), 0, s, *a, make_op<Op>(*a));
    return hipGetLastError();
  }
};
template <int B, class Op>
struct PersistentF {
  static hipError_t run(int grid, const Args *a, hipStream_t s) {
    if constexpr (std::is_same<Op, OpBFS>::value || std::is_same<Op, OpCC>::value ||
                  std::is_same<Op, OpKCore>::value) {
      if (a->vbits) {  // with the filter bitmap
        hipLaunchKernelGGL((k_persistent<B, Op, false, true>), dim3(grid), dim3(B), 0, s, *a, make_op<Op>(*a));
        return hipGetLastError();
      }
    }
    hipLaunchKernelGGL((k_persistent<B, Op, false>), dim3(grid), dim3(B), 0, s, *a, make_op<Op>(*a));
    return hipGetLastError();
  }
};
template <int B, class Op>
struct OccF {
  static hipError_t run(int *blocks) {
    return hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks, (const void *)k_persistent<B, Op, false>, B, 0);
  }
};
// batches: BFS and SSSP only
template <int B, class Op>
struct BatchF {
  static hipError_t run(int grid, const Args *a, hipStream_t s) {
    if constexpr (Op::kBatch) {
      hipLaunchKernelGGL((k_persistent<B, Op, true>), dim3(grid), dim3(B), 0, s, *a, make_op<Op>(*a));
      return hipGetLastError();
    } else {
      return hipErrorInvalidValue;
    }
  }
};
template <int B, class Op>
struct BatchOccF {
  static hipError_t run(int *blocks) {
    if constexpr (Op::kBatch)
      return hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks, (const void *)k_persistent<B, Op, true>, B, 0);
    else
      return hipErrorInvalidValue;
  }
};

// continuous serving: one operator for BFS and SSSP queries (OP_SSSP)
template <int B, class Op>
struct OpenF {
  static hipError_t run(int grid, const Args *a, hipStream_t s) {
    if constexpr (std::is_same<Op, OpSSSP>::value) {
      hipLaunchKernelGGL((k_open<B, OpServe>), dim3(grid), dim3(B), 0, s, *a, make_op<OpServe>(*a));
      return hipGetLastError();
    } else {
      return hipErrorInvalidValue;
    }
  }
};
template <int B, class Op>
struct OpenOccF {
  static hipError_t run(int *blocks) {
    if constexpr (std::is_same<Op, OpSSSP>::value)
      return hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks, (const void *)k_open<B, OpServe>, B, 0);
    else
      return hipErrorInvalidValue;
  }
};

template <template <int, class> class F, int B, typename... Xs>
hipError_t by_op(OpKind op, Xs... xs) {
  switch (op) {
    case OP_BFS: return F<B, OpBFS>::run(xs...);
    case OP_SSSP: return F<B, OpSSSP>::run(xs...);
    case OP_CC: return F<B, OpCC>::run(xs...);
    case OP_PR: return F<B, OpPR>::run(xs...);
    case OP_RECORD: return F<B, OpRecord>::run(xs...);
    case OP_KCORE: return F<B, OpKCore>::run(xs...);
  }
  return hipErrorInvalidValue;
}

template <template <int, class> class F, typename... Xs>
hipError_t by_wg(OpKind op, int wg, Xs... xs) {
  switch (wg) {
    case 64: return by_op<F, 64>(op, xs...);
    case 256: return by_op<F, 256>(op, xs...);
    case 1024: return by_op<F, 1024>(op, xs...);
  }
  return hipErrorInvalidValue;
}

}  // namespace

bool supported_wg(int wg) { return wg == 64 || wg == 256 || wg == 1024; }

hipError_t launch_init(OpKind op, const Args &a, int32_t source, uint32_t nfront0, hipStream_t s) {
  const int threads = 256;
  int blocks = (int)(((int64_t)a.n + threads - 1) / threads);
  if (blocks > 4096) blocks = 4096;
  if (blocks < 128) blocks = 128;
  hipLaunchKernelGGL(k_init, dim3(blocks), dim3(threads), 0, s, a, (int)op, source, nfront0);
  return hipGetLastError();
}

hipError_t launch_finish(OpKind op, const Args &a, hipStream_t s) {
  const int threads = 256;
  int blocks = (int)(((int64_t)a.n + threads - 1) / threads);
  if (blocks > 4096) blocks = 4096;
  if (blocks < 1) blocks = 1;
  hipLaunchKernelGGL(k_finish, dim3(blocks), dim3(threads), 0, s, a, (int)op);
  return hipGetLastError();
}

hipError_t launch_twc(OpKind op, int wg, int grid, const Args &a, hipStream_t s) {
  return by_wg<TwcF>(op, wg, grid, &a, s);
}
hipError_t launch_lb(OpKind op, int wg, int grid, const Args &a, hipStream_t s) {
  return by_wg<LbF>(op, wg, grid, &a, s);
}
hipError_t launch_persistent(OpKind op, int wg, int grid, const Args &a, hipStream_t s) {
  return by_wg<PersistentF>(op, wg, grid, &a, s);
}
hipError_t persistent_occupancy(OpKind op, int wg, int *blocks_per_cu) {
  return by_wg<OccF>(op, wg, blocks_per_cu);
}
hipError_t batch_occupancy(OpKind op, int wg, int *blocks_per_cu) { return by_wg<BatchOccF>(op, wg, blocks_per_cu); }
hipError_t launch_batch(OpKind op, int wg, int grid, const Args &a, hipStream_t s) {
  return by_wg<BatchF>(op, wg, grid, &a, s);
}

hipError_t launch_init_batch(OpKind op, const Args &a, hipStream_t s) {
  const int threads = 256;
  long long blocks = (a.nlabels + threads - 1) / threads;
  if (blocks > 8192) blocks = 8192;
  if (blocks < 128) blocks = 128;
  hipLaunchKernelGGL(k_init_batch, dim3((unsigned)blocks), dim3(threads), 0, s, a, (int)op);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  const int sblocks = (a.nq + threads - 1) / threads;
  hipLaunchKernelGGL(k_seed_batch, dim3(sblocks < 1 ? 1 : sblocks), dim3(threads), 0, s, a, (int)op);
  return hipGetLastError();
}

hipError_t launch_finish_batch(OpKind op, const Args &a, int32_t max_n, hipStream_t s) {
  const int threads = 256;
  int bx = (max_n + threads - 1) / threads;
  if (bx > 64) bx = 64;
  if (bx < 1) bx = 1;
  hipLaunchKernelGGL(k_finish_batch, dim3(bx, a.nq), dim3(threads), 0, s, a, (int)op);
  return hipGetLastError();
}

hipError_t pull_occupancy(int wg, int *blocks_per_cu) {
  switch (wg) {
    case 64: return hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks_per_cu, (const void *)k_pull_pr<64>, 64, 0);
    case 256: return hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks_per_cu, (const void *)k_pull_pr<256>, 256, 0);
    case 1024:
      return hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks_per_cu, (const void *)k_pull_pr<1024>, 1024, 0);
  }
  return hipErrorInvalidValue;
}

hipError_t launch_init_open(const Args &a, hipStream_t s) {
  hipLaunchKernelGGL(k_init_open, dim3(64), dim3(256), 0, s, a);
  return hipGetLastError();
}
hipError_t launch_open(OpKind op, int wg, int grid, const Args &a, hipStream_t s) {
  return by_wg<OpenF>(op, wg, grid, &a, s);
}
hipError_t open_occupancy(OpKind op, int wg, int *blocks_per_cu) { return by_wg<OpenOccF>(op, wg, blocks_per_cu); }

hipError_t launch_pull_pr(int wg, int grid, const Args &a, hipStream_t s) {
  switch (wg) {
    case 64: hipLaunchKernelGGL(k_pull_pr<64>, dim3(grid), dim3(64), 0, s, a); break;
    case 256: hipLaunchKernelGGL(k_pull_pr<256>, dim3(grid), dim3(256), 0, s, a); break;
    case 1024: hipLaunchKernelGGL(k_pull_pr<1024>, dim3(grid), dim3(1024), 0, s, a); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_pull_prepare(const Args &a, hipStream_t s) {
  int blocks = (int)(((int64_t)a.n + 255) / 256);
  if (blocks > 2048) blocks = 2048;
  if (blocks < 1) blocks = 1;
  hipLaunchKernelGGL(k_pull_prepare, dim3(blocks), dim3(256), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_pr_update(int wg, int grid, const Args &a, hipStream_t s) {
  switch (wg) {
    case 64: hipLaunchKernelGGL(k_pr_update<64>, dim3(grid), dim3(64), 0, s, a); break;
    case 256: hipLaunchKernelGGL(k_pr_update<256>, dim3(grid), dim3(256), 0, s, a); break;
    case 1024: hipLaunchKernelGGL(k_pr_update<1024>, dim3(grid), dim3(1024), 0, s, a); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

}  // namespace alb
