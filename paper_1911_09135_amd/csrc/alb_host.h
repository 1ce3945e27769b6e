// Host-side internal interface between the runtime's C++ files (not ABI).
#pragma once

#include <hip/hip_runtime.h>

#include "../../include/alb.h"

namespace alb {

// Set the calling thread's alb_last_error() text; returns s.
alb_status set_error(alb_status s, const char *fmt, ...);

// Validate `user` (NULL: the defaults) and fill its defaults into *out.
alb_status check_options(const alb_options *user, alb_options *out);

// The automatic grid of a traversal over `edges` edges (alb_options.grid_wgs = 0).
int auto_grid(int64_t edges, int wg, int resident);

// Workgroups of `wg` threads the device holds at once for a batch launch of
// `algo` on g's device.
alb_status batch_resident_workgroups(alb_graph g, int32_t algo, int32_t wg, int *out);

// Keep `count` batch workspaces for batches of up to `labels` labels and
// `nq` queries in g's pool (allocated now, free for the next batches).
alb_status batch_reserve(alb_graph g, int count, long long labels, int32_t nq);

// The device wall-clock window (ms, the device's own origin) of the last
// persistent launch this thread completed through a batch call: when its
// first workgroup joined and when it left its last round.  False if that
// call failed or ran no persistent launch.
bool last_launch_window(double *begin_ms, double *end_ms);

// Continuous serving: one lane's launch that queries join between rounds.
// create sizes it for `slots` queries whose labels fit in label_cap; start
// clears it and launches on stream s with the automatic grid of `edges` (the
// queued queries' edges) within grid_cap (it ends itself after idle_us
// without work, or once stopped and idle); publish hands one BFS or SSSP
// query to the running launch; poll returns finished slots; copy_out
// fetches a finished query's int32 labels (the launch wrote them to pinned
// host memory) unless the launch wrote them into the request's own pinned
// output; finish reads the ended launch's status and device window.
struct OpenLane;
constexpr int32_t kOpenMaxSlots = 1024;  // query slots of one launch (the rings' size)
// Slots published but never taken by a launch that has ended.
int32_t open_lane_untaken(OpenLane *L, int32_t *slots, int32_t max);
alb_status open_lane_create(alb_graph g, const alb_options &o, int32_t slots, long long label_cap, int grid_cap,
                            OpenLane **out);
void open_lane_destroy(OpenLane *L);
alb_status open_lane_start(OpenLane *L, hipStream_t s, double idle_us, int64_t edges);
bool open_lane_running(OpenLane *L, hipStream_t s);
uint64_t open_lane_backlog(OpenLane *L);
// host_out: the request's int32 output; when it is pinned host memory the
// launch writes the labels there itself (*direct), else copy_out fetches them.
alb_status open_lane_publish(OpenLane *L, int32_t algo, int32_t slot, int32_t member, int32_t source,
                             long long lbase, int32_t *host_out, bool *direct);
int32_t open_lane_poll(OpenLane *L, int32_t *slots, int32_t max);
void open_lane_copy_out(OpenLane *L, long long lbase, int32_t n, int32_t *out);
alb_status open_lane_finish(OpenLane *L, hipStream_t s, double *begin_ms, double *end_ms);
void open_lane_stop(OpenLane *L);
// The running launch's workgroups, and those the automatic grid gives a
// query of `edges` edges within the lane's share: a query that wants more
// than the launch has waits for a launch of its own size.
int open_lane_grid(const OpenLane *L);
int open_lane_grid_for(const OpenLane *L, int64_t edges);

}  // namespace alb
