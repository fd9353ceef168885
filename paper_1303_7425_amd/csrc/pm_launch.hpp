// Launchers of the gfx950 kernels (defined in pm_kernels.hip).
#pragma once

#include <algorithm>

#include "pm_plan.hpp"

namespace pm {

hipError_t launch_stats(const DevSeg *segs, int nseg, int nvars, int bits, int ring, u64 *out, u32 *flags,
                        hipStream_t st);
// Everything after validation: zero the per-call state, compress keys, tile /
// expand, radix passes, reduction and dense compaction.  Enqueued on `st`.
hipError_t launch_pipeline(const Plan &P, const Ctx &C, hipStream_t st, int cus);
// The dense path's inner-loop ceiling kernel: grid x 64 tiles of 64 x 64 pairs.
hipError_t launch_dense_ceiling(int ring, int grid, int tiles, hipStream_t st);
int profile_enable(int on);
int profile_read(int i, char *name, int cap, double *total_ms, int64_t *launches);
// Device pointers of every workspace region of plan P placed at `ws`.
Ctx make_ctx(const Plan &P, void *ws);

}  // namespace pm
