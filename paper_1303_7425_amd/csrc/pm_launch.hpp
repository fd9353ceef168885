// Launchers of the gfx950 kernels (defined in pm_kernels.hip).
#pragma once

#include <algorithm>

#include "pm_plan.hpp"

namespace pm {

hipError_t launch_stats(const DevSeg *segs, int nseg, int nvars, int bits, int ring, u64 *out, u32 *flags,
                        hipStream_t st);
// Everything after validation: zero the per-call state, compress keys, tile /
// expand, radix passes, reduction and dense compaction.  Enqueued on `st`.
// `part` (optional) enqueues one part only, so that a caller can space the
// tile launches of a large product out: PART_HEAD (zeroing, key compression,
// tile launch 0), PART_CHUNK (tile launch `chunk`), PART_TAIL (everything
// after the tile launches).  Parts must be enqueued in that order.
enum PipelinePart { PART_ALL = 0, PART_HEAD = 1, PART_CHUNK = 2, PART_TAIL = 3 };
hipError_t launch_pipeline(const Plan &P, const Ctx &C, hipStream_t st, int cus, int part = PART_ALL,
                           int64_t chunk = 0);
// Number of tile launches of plan P (0 without tiles).
int64_t tile_launches(const Plan &P);
// The dense path's inner-loop ceiling kernel: grid x 64 tiles of 64 x 64 pairs.
hipError_t launch_dense_ceiling(int ring, int grid, int tiles, hipStream_t st);
int profile_enable(int on);
int profile_read(int i, char *name, int cap, double *total_ms, int64_t *launches);
// Device pointers of every workspace region of plan P placed at `ws`.
Ctx make_ctx(const Plan &P, void *ws);

}  // namespace pm
