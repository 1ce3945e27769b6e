// Serving runtime behind the alb_server_* calls of include/alb.h: a queue of
// BFS / SSSP requests on one graph set, admitted by workspace footprint and
// run as batches by a few dispatcher lanes that share the device.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <list>
#include <map>
#include <mutex>
#include <new>
#include <thread>
#include <unordered_map>
#include <vector>

#include "../../include/alb.h"
#include "alb_host.h"

using alb::set_error;
using Clock = std::chrono::steady_clock;

namespace {

// Device bytes one request adds to its batch's workspace: per vertex of its
// member an 8-byte label word, a 4-byte output slot, two 8-byte worklist
// entries and a 16-byte huge-list record; plus its per-query tables.
constexpr size_t kBytesPerVertex = 44;
constexpr size_t kBytesPerQuery = 64;

enum { kPending = 0, kRunning = 1, kDone = 2 };

constexpr int64_t kMaxPositions = 0xffffffffLL;

struct Request {
  int32_t algo = 0, member = 0, source = 0;
  int32_t *out = nullptr;
  int32_t slot = -1;      // continuous batching: its query slot and labels in the lane's launch
  long long lbase = 0;
  size_t footprint = 0;
  int64_t edges = 0;  // edges of its member
  Clock::time_point t_submit, t_dispatch, t_done, deadline;
  int32_t state = kPending;
  int32_t status = ALB_OK;
  int32_t batch_size = 0, lane = -1;
};

double ms_between(Clock::time_point a, Clock::time_point b) {
  return std::chrono::duration<double, std::milli>(b - a).count();
}

// First-fit ranges of a lane's label memory (continuous batching).
struct Arena {
  std::map<long long, long long> free;  // start -> length, disjoint, merged
  explicit Arena(long long cap) {
    if (cap > 0) free[0] = cap;
  }
  long long take(long long n) {
    for (auto it = free.begin(); it != free.end(); ++it) {
      if (it->second >= n) {
        const long long at = it->first, rest = it->second - n;
        free.erase(it);
        if (rest > 0) free[at + n] = rest;
        return at;
      }
    }
    return -1;
  }
  void give(long long at, long long n) {
    auto it = free.emplace(at, n).first;
    auto nx = std::next(it);
    if (nx != free.end() && it->first + it->second == nx->first) {
      it->second += nx->second;
      free.erase(nx);
    }
    if (it != free.begin()) {
      auto pv = std::prev(it);
      if (pv->first + pv->second == it->first) {
        pv->second += it->second;
        free.erase(it);
      }
    }
  }
};

}  // namespace

struct alb_server_s {
  alb_graph g = nullptr;
  alb_server_config cfg;
  std::vector<int32_t> member_n;
  std::vector<int64_t> member_m;
  size_t lane_budget = 0;
  int grid[2] = {0, 0};      // workgroups per lane, by algo
  int grid_all[2] = {0, 0};  // every resident workgroup, by algo
  int busy_lanes = 0;        // lanes running a batch
  std::vector<hipStream_t> streams;
  std::vector<std::thread> lanes;

  std::mutex mu;
  std::condition_variable cv_work;  // a request was queued, or stop
  std::condition_variable cv_done;  // a request completed
  std::list<uint64_t> pending;      // arrival order
  std::unordered_map<uint64_t, Request> reqs;
  uint64_t next_ticket = 1;
  bool stop = false;
  int running = 0;  // requests dispatched and not yet completed
  alb_server_stats st{};
  Clock::time_point t_created = Clock::now();
  std::vector<alb_batch_record> log;  // ring of the last kLogSize batches
  size_t log_next = 0;
  static constexpr size_t kLogSize = 4096;

  void complete(Request &r, int32_t status, Clock::time_point now) {
    r.state = kDone;
    r.status = status;
    r.t_done = now;
    if (status == ALB_OK)
      ++st.completed;
    else if (status == ALB_E_TIMEOUT)
      ++st.timed_out;
    else if (status == ALB_E_CANCELLED)
      ++st.cancelled;
    else
      ++st.failed;
  }

  // Run one batch on lane `lane` (no lock held).
  int32_t execute(int lane, int32_t algo, bool alone, int64_t edges, std::vector<int32_t> &mb,
                  std::vector<int32_t> &src, std::vector<int32_t *> &outs) {
    const int32_t n = (int32_t)mb.size();
    if (cfg.executor) return cfg.executor(cfg.executor_user, algo, n, mb.data(), src.data(), outs.data(), lane);
    alb_options o = cfg.options;
    o.stream = streams[lane];
    o.out_on_device = 0;
    // the batch's automatic grid, capped by the lane's share of the device,
    // or by the whole device when no other lane runs (if the other lane's
    // batch reaches the device first, a batch launched just before it runs
    // on the workgroups still free: correct, only narrower)
    const int cap = alone && cfg.whole_device_when_alone ? grid_all[algo] : grid[algo];
    o.grid_wgs = alb::auto_grid(edges, o.wg_size ? o.wg_size : 256, cap);
    return algo == ALB_ALGO_BFS ? alb_bfs_batch(g, n, mb.data(), src.data(), outs.data(), nullptr, &o, nullptr)
                                : alb_sssp_batch(g, n, mb.data(), src.data(), outs.data(), nullptr, &o, nullptr);
  }

  void log_batch(const alb_batch_record &rec) {
    if (log.size() < kLogSize)
      log.push_back(rec);
    else
      log[log_next] = rec;
    log_next = (log_next + 1) % kLogSize;
  }

  // Continuous batching: keep one persistent launch of one algorithm
  // running; queued requests of that algorithm join it between rounds while
  // a slot and label memory are free, and complete as soon as their own
  // traversal has converged.  The launch ends by itself when idle.
  // join_long_edges: which requests lane `lane` takes
  bool lane_takes(int lane, const Request &r) const {
    if (cfg.join_long_edges <= 0 || cfg.lanes < 2) return true;
    return (r.edges >= cfg.join_long_edges) == (lane == 0);
  }

  bool pending_for(int lane) {
    for (uint64_t t : pending)
      if (lane_takes(lane, reqs[t])) return true;
    return false;
  }

  void lane_main_join(int lane) {
    const long long cap = (long long)(lane_budget / kBytesPerVertex);
    const int32_t nslots = std::min(cfg.max_batch, alb::kOpenMaxSlots);
    alb::OpenLane *L = nullptr;
    // a single lane takes the whole device, several share it
    const int grid_cap = cfg.lanes == 1 ? grid_all[ALB_ALGO_SSSP] : grid[ALB_ALGO_SSSP];
    const alb_status cst = alb::open_lane_create(g, cfg.options, nslots, std::max<long long>(cap, 1), grid_cap, &L);
    Arena arena(cap);
    std::vector<uint64_t> slot_ticket((size_t)nslots, 0);
    std::vector<char> in_use((size_t)nslots, 0);
    std::vector<int32_t> free_slots;
    for (int32_t q = nslots - 1; q >= 0; --q) free_slots.push_back(q);
    std::vector<int32_t> done((size_t)nslots);
    std::vector<char> direct((size_t)nslots, 0);  // the launch writes the slot's labels into its pinned output
    const double idle_us = cfg.join_idle_us > 0 ? (double)cfg.join_idle_us : 500.0;
    int64_t *edges_in_launch = nullptr;
    auto release = [&](Request &r) {
      if (edges_in_launch) *edges_in_launch -= r.edges;
      arena.give(r.lbase, member_n[r.member]);
      free_slots.push_back(r.slot);
      in_use[(size_t)r.slot] = 0;
      r.slot = -1;
    };
    std::unique_lock<std::mutex> lk(mu);
    for (;;) {
      cv_work.wait(lk, [&] { return stop || pending_for(lane); });
      expire(Clock::now());
      if (!pending_for(lane)) {
        if (stop) break;
        continue;
      }
      if (cst != ALB_OK) {  // the lane has no device workspace: fail what it would have run
        fail_pending(-1, cst, Clock::now(), lane);
        continue;
      }
      ++busy_lanes;
      ++st.batches;
      int64_t queued_edges = 0;  // sizes the launch's grid
      {
        int32_t cnt = 0;
        for (uint64_t t : pending)
          if (lane_takes(lane, reqs[t]) && cnt++ < nslots) queued_edges += reqs[t].edges;
      }
      lk.unlock();
      const Clock::time_point t0 = Clock::now();
      const alb_status ls = alb::open_lane_start(L, streams[lane], idle_us, queued_edges);
      lk.lock();
      if (ls != ALB_OK) {
        fail_pending(-1, ls, Clock::now(), lane);
        --busy_lanes;
        continue;
      }
      int32_t admitted = 0;
      int64_t active_edges = 0;  // edges of the members of the queries in the launch (one round's bound)
      edges_in_launch = &active_edges;
      for (;;) {
        // checked first: a launch seen ended has published every completion
        const bool alive = alb::open_lane_running(L, streams[lane]);
        // admit queued requests (BFS and SSSP alike), in order, while a
        // slot, label memory and ring room are free
        std::vector<Request> todo;
        expire(Clock::now());
        bool regrid = false;
        if (alive) {
          uint64_t room = (uint64_t)alb::kOpenMaxSlots - alb::open_lane_backlog(L);
          for (auto it = pending.begin(); it != pending.end() && !free_slots.empty() && room > 0;) {
            Request &r = reqs[*it];
            if (!lane_takes(lane, r)) {  // another lane's class
              ++it;
              continue;
            }
            if (active_edges + r.edges >= kMaxPositions) break;  // one round's huge edges stay 32-bit
            // a query that wants a bigger grid than the launch was started
            // with would run on too few workgroups: the launch ends once it
            // has finished what it holds and the next one is sized for it
            if (alb::open_lane_grid_for(L, r.edges) > alb::open_lane_grid(L)) {
              regrid = true;
              break;
            }
            const long long at = arena.take(member_n[r.member]);
            if (at < 0) break;  // wait for memory: later requests do not overtake
            active_edges += r.edges;
            r.slot = free_slots.back();
            free_slots.pop_back();
            in_use[(size_t)r.slot] = 1;
            r.lbase = at;
            r.state = kRunning;
            r.t_dispatch = Clock::now();
            slot_ticket[(size_t)r.slot] = *it;
            todo.push_back(r);
            ++running;
            ++admitted;
            --room;
            it = pending.erase(it);
          }
        }
        lk.unlock();
        std::vector<std::pair<uint64_t, alb_status>> fin;
        int64_t direct_done = 0;
        for (const Request &r : todo) {
          bool dir = false;
          const alb_status ps = alb::open_lane_publish(L, r.algo, r.slot, r.member, r.source, r.lbase, r.out, &dir);
          direct[(size_t)r.slot] = dir ? 1 : 0;
          if (ps != ALB_OK) fin.emplace_back(slot_ticket[(size_t)r.slot], ps);  // never published
        }
        // completions: each finished query's labels (already in pinned host
        // memory) copied into its request's array, unless the launch wrote
        // them there itself
        const int32_t k = alb::open_lane_poll(L, done.data(), nslots);
        for (int32_t i = 0; i < k; ++i) {
          const int32_t q = done[(size_t)i];
          if (q < 0 || q >= nslots || !in_use[(size_t)q]) continue;
          const uint64_t t = slot_ticket[(size_t)q];
          lk.lock();
          const Request r = reqs[t];
          lk.unlock();
          if (!direct[(size_t)q]) alb::open_lane_copy_out(L, r.lbase, member_n[r.member], r.out);
          fin.emplace_back(t, ALB_OK);
          if (direct[(size_t)q]) ++direct_done;
        }
        lk.lock();
        st.direct_outputs += direct_done;
        const Clock::time_point now = Clock::now();
        for (auto &f : fin) {
          Request &r = reqs[f.first];
          release(r);
          r.batch_size = admitted;
          r.lane = lane;
          --running;
          complete(r, f.second, now);
        }
        if (!fin.empty()) cv_done.notify_all();
        if (!alive) break;
        if (stop || regrid) alb::open_lane_stop(L);
        // nothing taken or finished: wait for a request or the next poll
        if (fin.empty() && todo.empty()) cv_work.wait_for(lk, std::chrono::microseconds(50));
      }
      // the launch has ended: its status; requests it never took go back to
      // the front of the queue, any it still held fail
      lk.unlock();
      double db = 0, de = 0;
      const alb_status fs = alb::open_lane_finish(L, streams[lane], &db, &de);
      std::vector<int32_t> untaken((size_t)nslots);
      const int32_t nu = alb::open_lane_untaken(L, untaken.data(), nslots);
      const Clock::time_point t1 = Clock::now();
      lk.lock();
      std::vector<char> back((size_t)nslots, 0);
      for (int32_t i = 0; i < nu; ++i)
        if (untaken[(size_t)i] >= 0 && untaken[(size_t)i] < nslots) back[(size_t)untaken[(size_t)i]] = 1;
      for (int32_t i = nu - 1; i >= 0; --i) {  // keep their order at the front
        const int32_t q = untaken[(size_t)i];
        if (q < 0 || q >= nslots || !in_use[(size_t)q]) continue;
        const uint64_t t = slot_ticket[(size_t)q];
        Request &r = reqs[t];
        release(r);
        --running;
        --admitted;
        if (fs == ALB_OK) {
          r.state = kPending;
          pending.push_front(t);
        } else {
          complete(r, fs, t1);
        }
      }
      int32_t lost = 0;
      for (int32_t q = 0; q < nslots; ++q) {
        if (!in_use[(size_t)q]) continue;
        Request &r = reqs[slot_ticket[(size_t)q]];
        release(r);
        r.batch_size = admitted;
        r.lane = lane;
        --running;
        complete(r, fs != ALB_OK ? fs : ALB_E_DEVICE, t1);
        ++lost;
      }
      (void)back;
      if (lost || nu) cv_done.notify_all();
      edges_in_launch = nullptr;
      alb_batch_record rec{};
      rec.lane = lane;
      rec.algo = -1;  // BFS and SSSP alike
      rec.batch_size = admitted;
      rec.status = fs;
      rec.device_begin_ms = fs == ALB_OK ? db : 0;
      rec.device_end_ms = fs == ALB_OK ? de : 0;
      rec.host_begin_ms = ms_between(t_created, t0);
      rec.host_end_ms = ms_between(t_created, t1);
      log_batch(rec);
      st.busy_ms += ms_between(t0, t1);
      --busy_lanes;
      cv_work.notify_all();
    }
    lk.unlock();
    alb::open_lane_destroy(L);
  }

  void expire(Clock::time_point now) {
    bool any = false;
    for (auto it = pending.begin(); it != pending.end();) {
      Request &r = reqs[*it];
      if (r.deadline <= now) {
        complete(r, ALB_E_TIMEOUT, now);
        it = pending.erase(it);
        any = true;
      } else {
        ++it;
      }
    }
    if (any) cv_done.notify_all();
  }

  // algo -1: every algorithm; lane >= 0: only the requests that lane takes
  void fail_pending(int32_t algo, alb_status status, Clock::time_point now, int lane = -1) {
    for (auto it = pending.begin(); it != pending.end();) {
      Request &r = reqs[*it];
      if ((algo < 0 || r.algo == algo) && (lane < 0 || lane_takes(lane, r))) {
        complete(r, status, now);
        it = pending.erase(it);
      } else {
        ++it;
      }
    }
    cv_done.notify_all();
  }

  void lane_main(int lane) {
    if (cfg.join_running) {
      lane_main_join(lane);
      return;
    }
    std::vector<uint64_t> batch;
    std::vector<int32_t> mb, src;
    std::vector<int32_t *> outs;
    std::unique_lock<std::mutex> lk(mu);
    for (;;) {
      cv_work.wait(lk, [&] { return stop || !pending.empty(); });
      if (pending.empty()) {
        if (stop) return;
        continue;
      }
      if (cfg.max_wait_us > 0 && !stop && (int)pending.size() < cfg.max_batch) {
        cv_work.wait_for(lk, std::chrono::microseconds(cfg.max_wait_us),
                         [&] { return stop || (int)pending.size() >= cfg.max_batch; });
        if (pending.empty()) continue;  // another lane took them
      }
      // expire overdue requests, then take the oldest request's algorithm and
      // every queued request of it, in order, that still fits the batch
      const Clock::time_point now = Clock::now();
      // a batch also keeps its vertex and edge totals below 2^32 - 1 (the
      // device's worklist positions are 32-bit)
      int32_t algo = -1;
      size_t foot = 0;
      int64_t labels = 0, edges = 0;
      batch.clear();
      bool expired = false;
      for (auto it = pending.begin(); it != pending.end();) {
        Request &r = reqs[*it];
        if (r.deadline <= now) {
          complete(r, ALB_E_TIMEOUT, now);
          it = pending.erase(it);
          expired = true;
          continue;
        }
        if (algo < 0) algo = r.algo;
        if (r.algo == algo && (int)batch.size() < cfg.max_batch && foot + r.footprint <= lane_budget &&
            labels + member_n[r.member] < kMaxPositions && edges + r.edges < kMaxPositions) {
          foot += r.footprint;
          labels += member_n[r.member];
          edges += r.edges;
          batch.push_back(*it);
          r.state = kRunning;
          r.t_dispatch = now;
          it = pending.erase(it);
        } else {
          ++it;
        }
      }
      if (expired) cv_done.notify_all();
      if (batch.empty()) continue;
      mb.clear();
      src.clear();
      outs.clear();
      for (uint64_t t : batch) {
        const Request &r = reqs[t];
        mb.push_back(r.member);
        src.push_back(r.source);
        outs.push_back(r.out);
      }
      running += (int)batch.size();
      ++st.batches;
      const bool alone = busy_lanes == 0;
      ++busy_lanes;
      lk.unlock();
      const Clock::time_point t0 = Clock::now();
      const int32_t status = execute(lane, algo, alone, edges, mb, src, outs);
      const Clock::time_point t1 = Clock::now();
      alb_batch_record rec{};
      rec.lane = lane;
      rec.algo = algo;
      rec.batch_size = (int32_t)batch.size();
      rec.status = status;
      if (cfg.executor || !alb::last_launch_window(&rec.device_begin_ms, &rec.device_end_ms))
        rec.device_begin_ms = rec.device_end_ms = 0;
      rec.host_begin_ms = ms_between(t_created, t0);
      rec.host_end_ms = ms_between(t_created, t1);
      lk.lock();
      log_batch(rec);
      st.busy_ms += ms_between(t0, t1);
      for (uint64_t t : batch) {
        Request &r = reqs[t];
        r.batch_size = (int32_t)batch.size();
        r.lane = lane;
        complete(r, status, t1);
      }
      running -= (int)batch.size();
      --busy_lanes;
      cv_done.notify_all();
    }
  }
};

extern "C" {

alb_status alb_server_config_init(alb_server_config *cfg) {
  if (!cfg) return set_error(ALB_E_INVAL, "cfg is NULL");
  std::memset(cfg, 0, sizeof *cfg);
  cfg->struct_size = sizeof(alb_server_config);
  cfg->lanes = 2;
  cfg->max_batch = 256;
  cfg->max_wait_us = 0;
  cfg->hbm_budget = (int64_t)8 << 30;
  cfg->whole_device_when_alone = 1;
  return alb_options_init(&cfg->options);
}

alb_status alb_server_create(alb_graph g, const alb_server_config *user, alb_server *out) {
  if (!out) return set_error(ALB_E_INVAL, "output handle pointer is NULL");
  *out = nullptr;
  alb_server_config cfg;
  alb_server_config_init(&cfg);
  if (user) {
    if (user->struct_size != sizeof(alb_server_config))
      return set_error(ALB_E_INVAL, "alb_server_config.struct_size = %u, expected %zu", user->struct_size,
                       sizeof(alb_server_config));
    cfg = *user;
  }
  if (cfg.lanes == 0) cfg.lanes = 2;
  if (cfg.max_batch == 0) cfg.max_batch = 256;
  if (cfg.hbm_budget == 0) cfg.hbm_budget = (int64_t)8 << 30;
  if (cfg.lanes < 1 || cfg.lanes > 16) return set_error(ALB_E_INVAL, "lanes must be in [1, 16]");
  if (cfg.max_batch < 1 || cfg.max_batch > 65535) return set_error(ALB_E_INVAL, "max_batch must be in [1, 65535]");
  if (cfg.max_wait_us < 0 || cfg.hbm_budget < 0) return set_error(ALB_E_INVAL, "negative max_wait_us or budget");
  if (cfg.join_running != 0 && cfg.join_running != 1) return set_error(ALB_E_INVAL, "join_running must be 0 or 1");
  if (cfg.join_running && (cfg.executor || !g))
    return set_error(ALB_E_INVAL, "join_running needs the GPU: a graph and no executor");
  if (cfg.join_idle_us < 0) return set_error(ALB_E_INVAL, "join_idle_us must be >= 0");
  if (cfg.join_long_edges < 0) return set_error(ALB_E_INVAL, "join_long_edges must be >= 0");
  if (cfg.join_long_edges > 0 && (!cfg.join_running || cfg.lanes < 2))
    return set_error(ALB_E_INVAL, "join_long_edges needs join_running and at least two lanes");
  {  // the traversal options every batch or launch of the server uses, defaults filled in
    alb_options o;
    const alb_status st = alb::check_options(&cfg.options, &o);
    if (st != ALB_OK) return st;
    cfg.options = o;
  }
  alb_server s = new (std::nothrow) alb_server_s();
  if (!s) return set_error(ALB_E_NOMEM, "host allocation failed");
  s->g = g;
  s->cfg = cfg;
  s->lane_budget = (size_t)cfg.hbm_budget / (size_t)cfg.lanes;
  auto bail = [&](alb_status st) {
    for (hipStream_t x : s->streams) (void)hipStreamDestroy(x);
    delete s;
    return st;
  };
  if (g) {
    int32_t cnt = 0;
    alb_status st = alb_graph_members(g, &cnt);
    if (st != ALB_OK) return bail(st);
    s->member_n.resize(cnt);
    s->member_m.resize(cnt);
    for (int32_t i = 0; i < cnt; ++i) {
      st = alb_graph_member_info(g, i, &s->member_n[i], &s->member_m[i], nullptr);
      if (st != ALB_OK) return bail(st);
    }
  } else {
    if (!cfg.executor || cfg.n_members < 1 || !cfg.member_vertices)
      return bail(set_error(ALB_E_INVAL, "a server without a graph needs an executor and member_vertices"));
    s->member_n.assign(cfg.member_vertices, cfg.member_vertices + cfg.n_members);
    s->member_m.assign(s->member_n.size(), 0);
    for (int32_t n : s->member_n)
      if (n < 1) return bail(set_error(ALB_E_INVAL, "member_vertices must be >= 1"));
  }
  s->cfg.member_vertices = nullptr;  // not kept
  if (!cfg.executor) {
    if (!g) return bail(set_error(ALB_E_INVAL, "graph handle is NULL"));
    const int wg = cfg.options.wg_size;  // filled in above
    for (int32_t algo = 0; algo < 2; ++algo) {
      int res = 0;
      // also makes g's device current for the streams below
      const alb_status st = alb::batch_resident_workgroups(g, algo, wg, &res);
      if (st != ALB_OK) return bail(st);
      s->grid[algo] = std::max(1, res / cfg.lanes);
      s->grid_all[algo] = res;
    }
    for (int i = 0; i < cfg.lanes; ++i) {
      hipStream_t x = nullptr;
      hipError_t e = hipStreamCreateWithFlags(&x, hipStreamNonBlocking);
      if (e != hipSuccess) return bail(set_error(ALB_E_DEVICE, "hipStreamCreate: %s", hipGetErrorString(e)));
      s->streams.push_back(x);
    }
    if (!cfg.join_running) {
      // every lane's largest batch (its share of the budget, at most
      // max_batch queries of the largest member) has a workspace from the
      // start: a batch never frees and reallocates one while others run.
      // Not fatal: without it batches allocate as they grow.
      int32_t max_n = 1;
      for (int32_t n : s->member_n) max_n = std::max(max_n, n);
      const long long labels = std::min<long long>((long long)(s->lane_budget / kBytesPerVertex),
                                                   (long long)cfg.max_batch * max_n);
      if (alb::batch_reserve(g, cfg.lanes, std::min<long long>(labels, kMaxPositions - 1), cfg.max_batch) != ALB_OK)
        alb::set_error(ALB_OK, "%s", "");
    }
  }
  try {
    for (int i = 0; i < cfg.lanes; ++i) s->lanes.emplace_back([s, i] { s->lane_main(i); });
  } catch (...) {
    {
      std::lock_guard<std::mutex> lk(s->mu);
      s->stop = true;
    }
    s->cv_work.notify_all();
    for (auto &t : s->lanes) t.join();
    return bail(set_error(ALB_E_NOMEM, "could not start the lane threads"));
  }
  *out = s;
  return ALB_OK;
}

alb_status alb_server_submit(alb_server s, int32_t algo, int32_t member, int32_t source, int32_t *out,
                             double timeout_ms, uint64_t *ticket) {
  if (!s || !out || !ticket) return set_error(ALB_E_INVAL, "NULL argument");
  if (algo != ALB_ALGO_BFS && algo != ALB_ALGO_SSSP) return set_error(ALB_E_INVAL, "bad algo %d", algo);
  if (member < 0 || member >= (int32_t)s->member_n.size())
    return set_error(ALB_E_INVAL, "member %d out of range [0, %zu)", member, s->member_n.size());
  const int32_t n = s->member_n[member];
  if (source < 0 || source >= n) return set_error(ALB_E_INVAL, "source %d out of range [0, %d)", source, n);
  if (!(timeout_ms >= 0)) return set_error(ALB_E_INVAL, "timeout_ms must be >= 0");
  Request r;
  r.algo = algo;
  r.member = member;
  r.source = source;
  r.out = out;
  r.footprint = kBytesPerVertex * (size_t)n + kBytesPerQuery;
  r.edges = s->member_m[member];
  r.t_submit = Clock::now();
  r.deadline = timeout_ms > 0 ? r.t_submit + std::chrono::duration_cast<Clock::duration>(
                                                  std::chrono::duration<double, std::milli>(timeout_ms))
                              : Clock::time_point::max();
  {
    std::lock_guard<std::mutex> lk(s->mu);
    if (s->stop) return set_error(ALB_E_INVAL, "server is stopping");
    if (r.footprint > s->lane_budget) {
      ++s->st.rejected;
      return set_error(ALB_E_NOMEM, "request needs %zu workspace bytes, a lane's budget is %zu", r.footprint,
                       s->lane_budget);
    }
    const uint64_t t = s->next_ticket++;
    s->reqs.emplace(t, r);
    s->pending.push_back(t);
    ++s->st.submitted;
    *ticket = t;
  }
  // with join_long_edges a lane waits for its own class of requests: wake them all
  if (s->cfg.join_running && s->cfg.join_long_edges > 0)
    s->cv_work.notify_all();
  else
    s->cv_work.notify_one();
  return ALB_OK;
}

alb_status alb_server_wait(alb_server s, uint64_t ticket, alb_request_info *info) {
  if (!s) return set_error(ALB_E_INVAL, "server handle is NULL");
  std::unique_lock<std::mutex> lk(s->mu);
  // look the ticket up again after every wait: submits can rehash the table
  auto it = s->reqs.find(ticket);
  for (;;) {
    if (it == s->reqs.end()) return set_error(ALB_E_INVAL, "unknown ticket %llu", (unsigned long long)ticket);
    if (it->second.state == kDone) break;
    if (it->second.state == kPending && it->second.deadline != Clock::time_point::max()) {
      const Clock::time_point dl = it->second.deadline;
      const bool timed_out = s->cv_done.wait_until(lk, dl) == std::cv_status::timeout;
      it = s->reqs.find(ticket);
      if (timed_out && it != s->reqs.end() && it->second.state == kPending) {
        s->pending.remove(ticket);
        s->complete(it->second, ALB_E_TIMEOUT, Clock::now());
      }
    } else {
      s->cv_done.wait(lk);
      it = s->reqs.find(ticket);
    }
  }
  const Request r = it->second;
  s->reqs.erase(it);
  if (info) {
    info->status = r.status;
    info->batch_size = r.batch_size;
    info->lane = r.lane;
    info->algo = r.algo;
    info->queue_ms = r.lane >= 0 ? ms_between(r.t_submit, r.t_dispatch) : ms_between(r.t_submit, r.t_done);
    info->latency_ms = ms_between(r.t_submit, r.t_done);
  }
  if (r.status == ALB_E_TIMEOUT) return set_error(ALB_E_TIMEOUT, "request %llu timed out in the queue",
                                                  (unsigned long long)ticket);
  if (r.status == ALB_E_CANCELLED) return set_error(ALB_E_CANCELLED, "request %llu was cancelled",
                                                    (unsigned long long)ticket);
  return (alb_status)r.status;
}

alb_status alb_server_cancel(alb_server s, uint64_t ticket) {
  if (!s) return set_error(ALB_E_INVAL, "server handle is NULL");
  std::lock_guard<std::mutex> lk(s->mu);
  auto it = s->reqs.find(ticket);
  if (it == s->reqs.end()) return set_error(ALB_E_INVAL, "unknown ticket %llu", (unsigned long long)ticket);
  if (it->second.state != kPending) return set_error(ALB_E_INVAL, "request already dispatched");
  s->pending.remove(ticket);
  s->complete(it->second, ALB_E_CANCELLED, Clock::now());
  s->cv_done.notify_all();
  return ALB_OK;
}

alb_status alb_server_drain(alb_server s) {
  if (!s) return set_error(ALB_E_INVAL, "server handle is NULL");
  std::unique_lock<std::mutex> lk(s->mu);
  s->cv_done.wait(lk, [&] { return s->pending.empty() && s->running == 0; });
  return ALB_OK;
}

alb_status alb_server_stats_get(alb_server s, alb_server_stats *st) {
  if (!s || !st) return set_error(ALB_E_INVAL, "NULL argument");
  std::lock_guard<std::mutex> lk(s->mu);
  *st = s->st;
  st->pending = (int64_t)s->pending.size();
  st->running = s->running;
  return ALB_OK;
}

alb_status alb_server_batch_log(alb_server s, int32_t max, alb_batch_record *out, int32_t *count) {
  if (!s || !count || (max > 0 && !out)) return set_error(ALB_E_INVAL, "NULL argument");
  if (max < 0) return set_error(ALB_E_INVAL, "max must be >= 0");
  std::lock_guard<std::mutex> lk(s->mu);
  const size_t have = s->log.size();
  const size_t k = std::min(have, (size_t)max);
  // oldest of the most recent k: the ring's write position minus k
  const size_t start = (s->log_next + have - k) % std::max<size_t>(have, 1);
  for (size_t i = 0; i < k; ++i) out[i] = s->log[(start + i) % have];
  *count = (int32_t)k;
  return ALB_OK;
}

alb_status alb_server_destroy(alb_server s) {
  if (!s) return ALB_OK;
  {
    std::lock_guard<std::mutex> lk(s->mu);
    s->stop = true;
  }
  s->cv_work.notify_all();
  for (auto &t : s->lanes) t.join();
  for (hipStream_t x : s->streams) (void)hipStreamDestroy(x);
  delete s;
  return ALB_OK;
}

}  // extern "C"
