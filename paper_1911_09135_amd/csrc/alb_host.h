// Host-side internal interface between the runtime's C++ files (not ABI).
#pragma once

#include "../../include/alb.h"

namespace alb {

// Set the calling thread's alb_last_error() text; returns s.
alb_status set_error(alb_status s, const char *fmt, ...);

// The automatic grid of a traversal over `edges` edges (alb_options.grid_wgs = 0).
int auto_grid(int64_t edges, int wg, int resident);

// Workgroups of `wg` threads the device holds at once for a batch launch of
// `algo` on g's device.
alb_status batch_resident_workgroups(alb_graph g, int32_t algo, int32_t wg, int *out);

// The device wall-clock window (ms, the device's own origin) of the last
// persistent launch this thread completed through a batch call: when its
// first workgroup joined and when it left its last round.  False if that
// call failed or ran no persistent launch.
bool last_launch_window(double *begin_ms, double *end_ms);

}  // namespace alb
