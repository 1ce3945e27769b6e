// Device side of the adaptive load balancer (ALB) for gfx950 (wave64).
//
// One BSP round of a data-driven push traversal (paper Section 2) is two
// phases over the active worklist F:
//
//   phase 1  inspection + TWC (Algorithm 1, Section 3 "TWC").  Each workgroup
//            takes B consecutive entries of F.  A vertex whose out-degree is
//            >= threshold is appended to the huge worklist `work`; its degree is
//            added to `prefixWork` in the same wave-aggregated atomic, so the
//            exclusive prefix of the huge degrees (Section 4.1 "Search") is
//            known once the phase ends.  Every other vertex is processed at
//            once by the workgroup, wavefront or thread bin of its degree.
//   phase 2  execution (Algorithm 2), only when `work` is non-empty
//            (Section 4.3).  Huge edge k goes to global thread k mod T (the
//            cyclic distribution, Section 4.1), so the 64 lanes of a wavefront
//            take 64 consecutive edges and read consecutive col / weight
//            entries.  The source of each edge is the last prefix entry <= k,
//            found once per wavefront-iteration; a second search runs only
//            for lanes past the first source's range.
//
// The operator (BFS, SSSP, CC, PageRank, or a recorder for tests) is a
// template parameter.  Pushes to the next worklist are wave-aggregated: one
// atomic per wavefront, lane offsets from a ballot and mbcnt.
//
// Rounds are driven either from the host (one launch per phase) or inside one
// cooperative persistent launch whose phases are separated by a grid-wide
// barrier with agent-scope release/acquire fences (8 XCDs, separate L2s).

#include "alb_internal.h"

namespace alb {
namespace {

constexpr int kWave = 64;
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

// ---------------------------------------------------------------------------
// Operators.  apply() runs the operator along one edge and returns true when
// the destination must be pushed to the next worklist.
// ---------------------------------------------------------------------------

struct OpBFS {  // level[dst] = level[src] + 1 on first visit
  using val_t = int32_t;
  static constexpr bool kPush = true, kNeedSrc = false, kRecord = false, kPR = false;
  int32_t *level;
  __device__ __forceinline__ val_t load_src(int32_t v, int32_t) const { return level[v]; }
  __device__ __forceinline__ bool apply(val_t sv, int32_t, int32_t dst, int32_t, int32_t) const {
    if (level[dst] != kInf) return false;
    int32_t expected = kInf;
    return __hip_atomic_compare_exchange_strong(&level[dst], &expected, sv + 1, __ATOMIC_RELAXED, __ATOMIC_RELAXED,
                                                __HIP_MEMORY_SCOPE_AGENT);
  }
};

struct OpSSSP {  // relaxation: dist[dst] = min(dist[dst], dist[src] + w)
  using val_t = int32_t;
  static constexpr bool kPush = true, kNeedSrc = false, kRecord = false, kPR = false;
  int32_t *dist;
  const int32_t *w;
  __device__ __forceinline__ val_t load_src(int32_t v, int32_t) const { return dist[v]; }
  __device__ __forceinline__ bool apply(val_t sv, int32_t pos, int32_t dst, int32_t, int32_t) const {
    const int32_t nd = sv + w[pos];
    if (nd >= dist[dst]) return false;  // a stale (larger) cached value only costs an atomic
    const int32_t old = __hip_atomic_fetch_min(&dist[dst], nd, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    return nd < old;
  }
};

struct OpCC {  // min-label propagation
  using val_t = int32_t;
  static constexpr bool kPush = true, kNeedSrc = false, kRecord = false, kPR = false;
  int32_t *lab;
  __device__ __forceinline__ val_t load_src(int32_t v, int32_t) const { return lab[v]; }
  __device__ __forceinline__ bool apply(val_t sv, int32_t, int32_t dst, int32_t, int32_t) const {
    if (sv >= lab[dst]) return false;
    const int32_t old = __hip_atomic_fetch_min(&lab[dst], sv, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    return sv < old;
  }
};

// fp32 value -> 64-bit fixed point (round to nearest)
__device__ __forceinline__ unsigned long long to_fix(float x) { return __double2ull_rn((double)x * kFixScale); }

struct OpPR {  // acc[dst] += rank[src] / outdeg(src): fp32 contribution, exact fixed-point sum
  using val_t = unsigned long long;
  static constexpr bool kPush = false, kNeedSrc = false, kRecord = false, kPR = true;
  const float *rank;
  unsigned long long *acc;
  __device__ __forceinline__ val_t load_src(int32_t v, int32_t deg) const { return to_fix(rank[v] / (float)deg); }
  __device__ __forceinline__ bool apply(val_t sv, int32_t, int32_t dst, int32_t, int32_t) const {
    add_relaxed(&acc[dst], sv);
    return false;
  }
};

struct OpRecord {  // counts each processed edge and the thread that took it; pushes every destination
  using val_t = int32_t;
  static constexpr bool kPush = true, kNeedSrc = true, kRecord = true, kPR = false;
  int32_t *hits;
  int32_t *thread_of;
  __device__ __forceinline__ val_t load_src(int32_t, int32_t) const { return 0; }
  __device__ __forceinline__ bool apply(val_t, int32_t pos, int32_t, int32_t, int32_t gt) const {
    __hip_atomic_fetch_add(&hits[pos], 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    thread_of[pos] = gt;
    return true;
  }
};

template <class Op>
Op make_op(const Args &a);
template <>
OpBFS make_op<OpBFS>(const Args &a) { return OpBFS{a.labels}; }
template <>
OpSSSP make_op<OpSSSP>(const Args &a) { return OpSSSP{a.labels, a.w}; }
template <>
OpCC make_op<OpCC>(const Args &a) { return OpCC{a.labels}; }
template <>
OpPR make_op<OpPR>(const Args &a) { return OpPR{a.rank, a.acc}; }
template <>
OpRecord make_op<OpRecord>(const Args &a) { return OpRecord{a.hits, a.thread_of}; }

// ---------------------------------------------------------------------------
// Per-thread statistics and shared memory.
// ---------------------------------------------------------------------------

struct Acc {
  unsigned long long frontier = 0, edges_twc = 0, edges_lb = 0, huge_v = 0, pushes = 0;
  unsigned long long dangling = 0;  // fixed point
};

template <int B, class Op>
struct Smem {
  using V = typename Op::val_t;
  int32_t pos[B];  // thread-bin gather: CSR position, source value and source of each staged edge
  V sv[B];
  int32_t src[Op::kNeedSrc ? B : 1];
  int32_t wsum[B / kWave];
  unsigned long long ured[B / kWave][5];
  unsigned long long dred[B / kWave];
  int32_t owner, obeg, odeg, ov;  // workgroup-bin broadcast
  V osv;
  int32_t flag;
  int32_t pbuf[B / kWave][kPushBuf];  // per-wavefront push staging
};

// Next-worklist pushes of one wavefront, staged in LDS and written out in
// batches: one global reservation per batch instead of one per ballot.
// The workgroup's index and the workgroup count used for work distribution:
// the hardware ones for one-phase launches, the membership ticket and the
// member count inside the persistent launch.
struct Grid {
  uint32_t id;
  uint32_t n;
};

struct Pusher {
  int32_t *buf;      // this wavefront's LDS staging area
  uint32_t cnt;      // entries staged (wave-uniform)
  int32_t *qn;       // next worklist
  uint32_t *qn_cnt;  // its size counter
};

template <int B, class Op>
__device__ void flush_stats(Acc &acc, Smem<B, Op> &sm, Ctl *c) {
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
  }
  __syncthreads();
  acc = Acc();
}

template <int B, class Op>
__device__ void flush_dangling(Acc &acc, Smem<B, Op> &sm, unsigned long long *dst) {
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

// ---------------------------------------------------------------------------
// Wave-aggregated push and huge-worklist reservation.
// ---------------------------------------------------------------------------

// Write the staged entries to the next worklist (all lanes call this).
__device__ __forceinline__ void flush_pushes(const Args &a, int round, Pusher &pu) {
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
__device__ __forceinline__ void push_wave(bool pred, int32_t v, const Args &a, int round, Pusher &pu, Acc &acc) {
  const unsigned long long m = __ballot(pred);
  if (m == 0ull) return;
  const uint32_t total = (uint32_t)__popcll(m);
  if (pu.cnt + total > kPushBuf) flush_pushes(a, round, pu);
  if (pred) pu.buf[pu.cnt + bits_below(m)] = v;
  pu.cnt += total;
  if (lane_id() == 0) acc.pushes += total;
}

// Algorithm 1, "work.push(src)": append every huge lane's vertex to `work`
// and its degree to the running edge total with ONE 64-bit atomic per
// wavefront on (count << 32 | edges).  Slot j receives prefix[j] = the edges
// of all earlier slots, i.e. the exclusive scan of the huge degrees in
// worklist order.  All lanes of the wavefront must call this.
__device__ __forceinline__ void reserve_huge(bool huge, int32_t v, int32_t deg, const Args &a, int round,
                                             unsigned long long *ctr, Acc &acc) {
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
  if (lane == kWave - 1) {
    if (tot_e >> 32) {
      flag_overflow(a.ctl, round);
    } else {
      base = add_relaxed(ctr, ((unsigned long long)tot_c << 32) | tot_e);
      if ((unsigned long long)(uint32_t)base + tot_e > 0xffffffffull) flag_overflow(a.ctl, round);
      acc.huge_v += tot_c;
    }
  }
  base = __shfl(base, kWave - 1);
  if (huge) {
    const uint32_t j = (uint32_t)(base >> 32) + bits_below(hm);
    const uint32_t p = (uint32_t)base + (uint32_t)(incl - mine);
    if (j < a.qcap) {
      a.work[j] = v;
      a.prefix[j] = p;
    } else {
      flag_overflow(a.ctl, round);
    }
  }
}

// Apply the operator along one edge (if act) and push; every lane calls it.
template <class Op>
__device__ __forceinline__ void edge(bool act, int32_t pos, typename Op::val_t sv, int32_t src, const Op &op,
                                     const Args &a, int round, Pusher &pu, Acc &acc, int32_t gt) {
  bool p = false;
  int32_t dst = 0;
  if (act) {
    dst = a.col[pos];
    p = op.apply(sv, pos, dst, src, gt);
    if constexpr (Op::kPush) {
      // dedup: push once per round; a stamp equal to this round can only have
      // been written this round, so the plain load is a safe filter
      if (p && a.stamp)
        p = a.stamp[dst] != round &&
            __hip_atomic_exchange(&a.stamp[dst], round, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != round;
    }
  }
  if constexpr (Op::kPush) push_wave(p, dst, a, round, pu, acc);
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

// ---------------------------------------------------------------------------
// Phase 1: inspection (Algorithm 1) fused with the TWC bins.
// ---------------------------------------------------------------------------
template <int B, class Op>
__device__ void phase_twc(const Args &a, const Op &op, Smem<B, Op> &sm, Grid gr, int round, const int32_t *F,
                          uint32_t nF, int32_t *qn, uint32_t *qn_cnt, unsigned long long *hctr, Acc &acc) {
  using V = typename Op::val_t;
  const int tid = threadIdx.x;
  const uint32_t lane = lane_id();
  const uint32_t stride = gr.n * B;
  const int32_t gt = (int32_t)(gr.id * B + tid);
  Pusher pu{sm.pbuf[tid / kWave], 0u, qn, qn_cnt};
  for (uint32_t base = gr.id * B; base < nF; base += stride) {
    const uint32_t i = base + tid;
    int32_t v = -1, beg = 0, deg = 0;
    if (i < nF) {
      v = F ? F[i] : (int32_t)i;
      beg = a.off[v];
      deg = a.off[v + 1] - beg;
    }
    // inspection: degree >= THRESHOLD goes to the huge worklist
    const bool huge = v >= 0 && deg > 0 && (int64_t)deg >= a.threshold;
    reserve_huge(huge, v, deg, a, round, hctr, acc);
    if constexpr (Op::kRecord) {
      if (i < nF) a.bins[i] = (int8_t)(huge ? 3 : deg >= a.c_wg ? 2 : deg >= a.c_wave ? 1 : 0);
    }
    if constexpr (Op::kPR) {
      if (v >= 0 && deg == 0) acc.dangling += to_fix(a.rank[v]);
    }
    if (huge) deg = 0;
    acc.frontier += (v >= 0);
    acc.edges_twc += (unsigned long long)deg;
    V sv = V(0);
    if (deg > 0) sv = op.load_src(v, deg);

    // workgroup bin: the whole workgroup strides one vertex's edges
    for (;;) {
      if (tid == 0) sm.owner = -1;
      __syncthreads();
      if (deg > 0 && deg >= a.c_wg) sm.owner = tid;  // any one claimant wins
      __syncthreads();
      const int32_t o = sm.owner;
      if (o < 0) break;
      if (tid == o) {
        sm.obeg = beg;
        sm.odeg = deg;
        sm.osv = sv;
        sm.ov = v;
        deg = 0;
      }
      __syncthreads();
      const int32_t ob = sm.obeg, od = sm.odeg, ov = sm.ov;
      const V os = sm.osv;
      for (int32_t j0 = 0; j0 < od; j0 += B) {
        const int32_t j = j0 + tid;
        edge<Op>(j < od, ob + j, os, ov, op, a, round, pu, acc, gt);
      }
    }

    // wavefront bin: one wavefront strides one vertex's edges
    for (;;) {
      const unsigned long long mm = __ballot(deg > 0 && deg >= a.c_wave);
      if (mm == 0ull) break;
      const int ld = __ffsll((unsigned long long)mm) - 1;
      const int32_t ob = __shfl(beg, ld), od = __shfl(deg, ld), ov = __shfl(v, ld);
      const V os = __shfl(sv, ld);
      if ((int)lane == ld) deg = 0;
      for (int32_t j0 = 0; j0 < od; j0 += kWave) {
        const int32_t j = j0 + (int32_t)lane;
        edge<Op>(j < od, ob + j, os, ov, op, a, round, pu, acc, gt);
      }
    }

    // thread bin: fine-grained gather of the remaining short lists through LDS,
    // B edges at a time, so that the workgroup's lanes stay busy
    int32_t rank, total;
    block_exscan<B>(deg, rank, total, sm.wsum);
    for (int32_t done = 0; done < total; done += B) {
      const int32_t lo = max(rank, done), hi = min(rank + deg, done + B);
      for (int32_t e = lo; e < hi; ++e) {
        sm.pos[e - done] = beg + (e - rank);
        sm.sv[e - done] = sv;
        if constexpr (Op::kNeedSrc) sm.src[e - done] = v;
      }
      __syncthreads();
      const int32_t cnt = min(B, total - done);
      const bool act = tid < cnt;
      int32_t p = 0, s = 0;
      V x = V(0);
      if (act) {
        p = sm.pos[tid];
        x = sm.sv[tid];
        if constexpr (Op::kNeedSrc) s = sm.src[tid];
      }
      edge<Op>(act, p, x, s, op, a, round, pu, acc, gt);
      __syncthreads();
    }
  }
  if constexpr (Op::kPush) flush_pushes(a, round, pu);
}

// Largest j in [lo, vh) with prefix[j] <= k, given prefix[lo] <= k:
// exponential search forward from lo, then bisection.
__device__ __forceinline__ uint32_t owner_from(const uint32_t *prefix, uint32_t vh, uint32_t lo, uint32_t k) {
  uint64_t j = lo, step = 1, hi = (uint64_t)lo + 1;
  while (hi < vh && prefix[hi] <= k) {
    j = hi;
    step <<= 1;
    hi = j + step;
  }
  if (hi > vh) hi = vh;
  while (hi - j > 1) {
    const uint64_t mid = j + ((hi - j) >> 1);
    if (prefix[mid] <= k)
      j = mid;
    else
      hi = mid;
  }
  return (uint32_t)j;
}

// ---------------------------------------------------------------------------
// Phase 2: execution (Algorithm 2) with the cyclic distribution.
// ---------------------------------------------------------------------------
template <int B, class Op>
__device__ void phase_lb(const Args &a, const Op &op, Smem<B, Op> &sm, Grid gr, int round, unsigned long long hc,
                         int32_t *qn, uint32_t *qn_cnt, Acc &acc) {
  using V = typename Op::val_t;
  const uint32_t vh = (uint32_t)(hc >> 32);
  const uint32_t e = (uint32_t)hc;
  if (vh == 0) return;
  // an overflowed reservation leaves prefix inconsistent with the degrees: skip
  if (ld_relaxed(&a.ctl->overflow) <= (uint32_t)round) return;
  const uint64_t T = (uint64_t)gr.n * B;
  const uint32_t lane = lane_id();
  const uint64_t g = (uint64_t)gr.id * B + threadIdx.x;
  uint32_t s = 0;  // owner of the wavefront's first edge; never decreases
  uint32_t c_s = 0xffffffffu;
  int32_t c_src = 0, c_beg = 0;
  uint32_t c_p = 0;
  V c_sv = V(0);
  Pusher pu{sm.pbuf[threadIdx.x / kWave], 0u, qn, qn_cnt};
  for (uint64_t k0 = g - lane; k0 < e; k0 += T) {
    s = owner_from(a.prefix, vh, s, (uint32_t)k0);
    const uint64_t k = k0 + lane;
    const bool act = k < e;
    if (act) {
      uint32_t ss = s;
      const uint32_t nxt = (s + 1 < vh) ? a.prefix[s + 1] : e;
      if ((uint32_t)k >= nxt) ss = owner_from(a.prefix, vh, s + 1, (uint32_t)k);
      if (ss != c_s) {
        c_s = ss;
        c_src = a.work[ss];
        c_beg = a.off[c_src];
        c_p = a.prefix[ss];
        c_sv = op.load_src(c_src, a.off[c_src + 1] - c_beg);
      }
    }
    acc.edges_lb += act;
    edge<Op>(act, c_beg + (int32_t)((uint32_t)k - c_p), c_sv, c_src, op, a, round, pu, acc, (int32_t)g);
  }
  if constexpr (Op::kPush) flush_pushes(a, round, pu);
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

// Grid-wide barrier over a monotone arrival counter.  After the workgroup
// barrier, thread 0 alone releases the workgroup's writes at agent scope
// (L2 write-back across the 8 XCDs), arrives with one RMW and spins with
// relaxed loads and s_sleep until every workgroup has arrived, then acquires
// (L1/L2 invalidate) before the workgroup barrier lets the others on.  A wait
// longer than timeout_ticks sets ctl->abort, which makes every workgroup
// leave at its next barrier.
template <class S>
__device__ bool grid_barrier(const Args &a, S &sm, Grid gr, int round) {
  __syncthreads();
  if (threadIdx.x == 0) {
    Ctl *c = a.ctl;
    const unsigned long long nb = gr.n;
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
    const unsigned long long arrived = add_relaxed(&c->bar_count, 1ull);
    const unsigned long long target = (arrived / nb + 1ull) * nb;
    int ok = 1;
    const uint64_t t0 = (uint64_t)wall_clock64();
    while (ld_relaxed(&c->bar_count) < target) {
      if (ld_relaxed(&c->abort)) {
        ok = 0;
        break;
      }
      if ((uint64_t)wall_clock64() - t0 > a.timeout_ticks) {
        st_relaxed(&c->diag_seen, ld_relaxed(&c->bar_count));
        st_relaxed(&c->diag_target, target);
        st_relaxed(&c->diag_round, (uint32_t)round);
        st_relaxed(&c->abort, 1u);
        ok = 0;
        break;
      }
      __builtin_amdgcn_s_sleep(4);
    }
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    sm.flag = ok;
  }
  __syncthreads();
  return sm.flag != 0;
}

__device__ __forceinline__ const int32_t *round_frontier(const Args &a, int r) {
  if (a.all_rounds || (r == 0 && a.identity_first)) return nullptr;
  return (r & 1) ? a.q1 : a.q0;
}
__device__ __forceinline__ int32_t *round_next(const Args &a, int r) { return (r & 1) ? a.q0 : a.q1; }

__device__ __forceinline__ uint32_t round_size(const Args &a, int r) {
  if (a.all_rounds) return (uint32_t)a.n;
  const uint32_t c = ld_relaxed(&a.ctl->qcount[r % 3]);
  return c < a.qcap ? c : a.qcap;
}

// Clear the counters two rounds ahead (nobody reads or writes them this round).
__device__ __forceinline__ void clear_ahead(const Args &a, int r) {
  st_relaxed(&a.ctl->qcount[(r + 2) % 3], 0u);
  st_relaxed(&a.ctl->huge[(r + 1) & 1], 0ull);
  st_relaxed(&a.ctl->dangling[(r + 1) & 1], 0ull);
}

// ---------------------------------------------------------------------------
// Kernels.
// ---------------------------------------------------------------------------

__global__ void k_init(Args a, int op, int32_t source, uint32_t nfront0) {
  const uint32_t stride = gridDim.x * blockDim.x;
  const float r0 = 1.0f / (float)a.n;
  for (uint32_t v = blockIdx.x * blockDim.x + threadIdx.x; v < (uint32_t)a.n; v += stride) {
    if (a.labels) a.labels[v] = (op == OP_CC) ? (int32_t)v : ((int32_t)v == source ? 0 : kInf);
    if (a.stamp) a.stamp[v] = -1;
    if (op == OP_PR) {
      a.rank[v] = r0;
      a.acc[v] = 0ull;
    }
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    Ctl *c = a.ctl;
    c->qcount[0] = nfront0;
    c->qcount[1] = 0;
    c->qcount[2] = 0;
    c->overflow = 0xffffffffu;
    c->huge[0] = 0;
    c->huge[1] = 0;
    c->bar_count = 0;
    c->abort = 0;
    c->rounds = 0;
    c->st_frontier = c->st_edges_twc = c->st_edges_lb = c->st_huge_v = c->st_pushes = 0;
    c->dangling[0] = 0;
    c->dangling[1] = 0;
    c->members = 0;
    c->n_members = 0;
    c->diag_seen = c->diag_target = 0;
    c->diag_round = 0;
    c->threshold_used = a.threshold;
    if (source >= 0 && op != OP_RECORD) a.q0[0] = source;
  }
}

template <int B, class Op>
__global__ __launch_bounds__(B) void k_twc(Args a, Op op) {
  __shared__ Smem<B, Op> sm;
  Acc acc;
  const int r = a.round;
  const uint32_t nF = round_size(a, r);
  if (blockIdx.x == 0 && threadIdx.x == 0) clear_ahead(a, r);
  const Grid gr{blockIdx.x, gridDim.x};
  phase_twc<B, Op>(a, op, sm, gr, r, round_frontier(a, r), nF, round_next(a, r), &a.ctl->qcount[(r + 1) % 3],
                   &a.ctl->huge[r & 1], acc);
  if constexpr (Op::kPR) flush_dangling<B, Op>(acc, sm, &a.ctl->dangling[r & 1]);
  flush_stats<B, Op>(acc, sm, a.ctl);
}

template <int B, class Op>
__global__ __launch_bounds__(B) void k_lb(Args a, Op op) {
  __shared__ Smem<B, Op> sm;
  Acc acc;
  const int r = a.round;
  const unsigned long long hc = ld_relaxed(&a.ctl->huge[r & 1]);
  phase_lb<B, Op>(a, op, sm, Grid{blockIdx.x, gridDim.x}, r, hc, round_next(a, r), &a.ctl->qcount[(r + 1) % 3],
                  acc);
  flush_stats<B, Op>(acc, sm, a.ctl);
}

template <int B>
__global__ __launch_bounds__(B) void k_pr_update(Args a) {
  phase_pr_update<B>(a, Grid{blockIdx.x, gridDim.x}, ld_relaxed(&a.ctl->dangling[a.round & 1]));
  if (blockIdx.x == 0 && threadIdx.x == 0) st_relaxed(&a.ctl->rounds, (uint32_t)a.round + 1u);
}

// Membership of the persistent launch.  The grid may be larger than what the
// device can hold at once, so co-residency is not assumed: every workgroup
// takes a ticket from ctl->members when it starts; the holder of ticket 0
// closes membership (sets the top bit) once all workgroups have joined or
// no new one has joined for join_window_ticks, and publishes the member
// count.  A workgroup whose ticket shows the closed bit is not a member and
// leaves at once.  Members are running when they join and never leave before
// the end, so every barrier among them completes.  Returns false for a
// non-member; *gr gets (ticket, member count).
template <class S>
__device__ bool join_members(const Args &a, S &sm, Grid *gr) {
  constexpr unsigned long long kClosed = 1ull << 63;
  if (threadIdx.x == 0) {
    Ctl *c = a.ctl;
    const unsigned long long t = add_relaxed(&c->members, 1ull);
    uint32_t member = (t & kClosed) ? 0u : 1u;
    if (member && t == 0) {
      unsigned long long seen = 1;
      uint64_t t_last = (uint64_t)wall_clock64();
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
      const unsigned long long prev = __hip_atomic_fetch_or(&c->members, kClosed, __ATOMIC_RELAXED,
                                                            __HIP_MEMORY_SCOPE_AGENT);
      st_relaxed(&c->n_members, (uint32_t)prev);
    }
    uint32_t n = 0;
    if (member) {
      while ((n = ld_relaxed(&c->n_members)) == 0) __builtin_amdgcn_s_sleep(1);
      if ((uint32_t)t >= n) member = 0;  // cannot happen: tickets below the closing count are members
    }
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    sm.flag = (int32_t)member;
    sm.owner = (int32_t)t;
    sm.obeg = (int32_t)n;
  }
  __syncthreads();
  const bool member = sm.flag != 0;
  gr->id = (uint32_t)sm.owner;
  gr->n = (uint32_t)sm.obeg;
  __syncthreads();
  return member;
}

template <int B, class Op>
__global__ __launch_bounds__(B) void k_persistent(Args a, Op op) {
  __shared__ Smem<B, Op> sm;
  Acc acc;
  Grid gr;
  if (!join_members(a, sm, &gr)) return;
  if (a.threshold < 0) a.threshold = (int64_t)gr.n * B;  // default: the launched thread count
  int r = 0;
  for (; r < a.max_rounds; ++r) {
    if (ld_relaxed(&a.ctl->overflow) < (uint32_t)r) break;  // set in an earlier round: seen by all alike
    const uint32_t nF = round_size(a, r);
    if (nF == 0) break;
    const bool tl = gr.id == 0 && threadIdx.x == 0 && r < kTimeline;
    if (gr.id == 0 && threadIdx.x == 0) clear_ahead(a, r);
    if (tl) a.ctl->tl[4 * r] = (unsigned long long)wall_clock64();
    int32_t *qn = round_next(a, r);
    uint32_t *qn_cnt = &a.ctl->qcount[(r + 1) % 3];
    phase_twc<B, Op>(a, op, sm, gr, r, round_frontier(a, r), nF, qn, qn_cnt, &a.ctl->huge[r & 1], acc);
    if constexpr (Op::kPR) flush_dangling<B, Op>(acc, sm, &a.ctl->dangling[r & 1]);
    if (!grid_barrier(a, sm, gr, r)) break;
    const unsigned long long hc = ld_relaxed(&a.ctl->huge[r & 1]);
    if (tl) {
      a.ctl->tl[4 * r + 1] = (unsigned long long)wall_clock64();
      a.ctl->tl[4 * r + 3] = (unsigned long long)nF | ((hc >> 32) << 32);
    }
    if ((hc >> 32) != 0) {  // the execution phase runs only when there is imbalance to fix
      phase_lb<B, Op>(a, op, sm, gr, r, hc, qn, qn_cnt, acc);
      if (!grid_barrier(a, sm, gr, r)) break;
    }
    if (tl) a.ctl->tl[4 * r + 2] = (unsigned long long)wall_clock64();
    if constexpr (Op::kPR) {
      phase_pr_update<B>(a, gr, ld_relaxed(&a.ctl->dangling[r & 1]));
      if (!grid_barrier(a, sm, gr, r)) break;
    }
  }
  if (gr.id == 0 && threadIdx.x == 0) {
    st_relaxed(&a.ctl->rounds, (uint32_t)r);
    st_relaxed(&a.ctl->threshold_used, (long long)a.threshold);
  }
  flush_stats<B, Op>(acc, sm, a.ctl);
}

// ---------------------------------------------------------------------------
// Dispatch over workgroup size and operator.
// ---------------------------------------------------------------------------

template <int B, class Op>
hipError_t twc_t(int grid, const Args &a, hipStream_t s) {
  hipLaunchKernelGGL((k_twc<B, Op>), dim3(grid), dim3(B), 0, s, a, make_op<Op>(a));
  return hipGetLastError();
}
template <int B, class Op>
hipError_t lb_t(int grid, const Args &a, hipStream_t s) {
  hipLaunchKernelGGL((k_lb<B, Op>), dim3(grid), dim3(B), 0, s, a, make_op<Op>(a));
  return hipGetLastError();
}
template <int B, class Op>
hipError_t persistent_t(int grid, const Args &a, hipStream_t s) {
  hipLaunchKernelGGL((k_persistent<B, Op>), dim3(grid), dim3(B), 0, s, a, make_op<Op>(a));
  return hipGetLastError();
}
template <int B, class Op>
hipError_t occupancy_t(int *blocks) {
  return hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks, (const void *)k_persistent<B, Op>, B, 0);
}

template <template <int, class> class F, int B, typename... Xs>
hipError_t by_op(OpKind op, Xs... xs) {
  switch (op) {
    case OP_BFS: return F<B, OpBFS>::run(xs...);
    case OP_SSSP: return F<B, OpSSSP>::run(xs...);
    case OP_CC: return F<B, OpCC>::run(xs...);
    case OP_PR: return F<B, OpPR>::run(xs...);
    case OP_RECORD: return F<B, OpRecord>::run(xs...);
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

template <int B, class Op>
struct TwcF {
  static hipError_t run(int grid, const Args *a, hipStream_t s) { return twc_t<B, Op>(grid, *a, s); }
};
template <int B, class Op>
struct LbF {
  static hipError_t run(int grid, const Args *a, hipStream_t s) { return lb_t<B, Op>(grid, *a, s); }
};
template <int B, class Op>
struct PersistentF {
  static hipError_t run(int grid, const Args *a, hipStream_t s) { return persistent_t<B, Op>(grid, *a, s); }
};
template <int B, class Op>
struct OccF {
  static hipError_t run(int *blocks) { return occupancy_t<B, Op>(blocks); }
};

}  // namespace

bool supported_wg(int wg) { return wg == 64 || wg == 256 || wg == 1024; }

hipError_t launch_init(OpKind op, const Args &a, int32_t source, uint32_t nfront0, hipStream_t s) {
  const int threads = 256;
  int blocks = (int)(((int64_t)a.n + threads - 1) / threads);
  if (blocks > 4096) blocks = 4096;
  if (blocks < 1) blocks = 1;
  hipLaunchKernelGGL(k_init, dim3(blocks), dim3(threads), 0, s, a, (int)op, source, nfront0);
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
