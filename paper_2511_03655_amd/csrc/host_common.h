// Host-side helpers shared by the context runtime, the serving loop and the
// allocation-free entry point.
#pragma once

#include <atomic>

#include "../../include/irkgl16.h"
#include "device_common.h"

namespace irk {

// IRKGL16_OK if a problem of a built-in kind is well formed (kind, n, d,
// masses, couplings, constants), else IRKGL16_EINVAL.  Allocates nothing.
int validate_problem(const irkgl16_problem& p);

// Totals of per-instance statistics into `stats` (nullable; its per-instance
// arrays are filled when non-NULL, device_ms and step_iters are left alone).
// Returns the worst status: the most negative error, else ENOCONV if a step
// stopped at the iteration cap, else OK.  Allocates nothing.
int summarize_stats(const InstStat* st, int32_t n, irkgl16_stats* stats);

// Streams that the library's contexts and servers have created and not yet
// destroyed, in this process.  HIP gives a process GPU_MAX_HW_QUEUES hardware
// queues (4 unless set) and maps further streams onto them, and the kernels
// of streams that share a queue run one after another.
std::atomic<int>& live_streams();

}  // namespace irk
