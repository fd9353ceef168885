// Host-side helpers shared by the product API and the server.
#pragma once

#include <hip/hip_runtime.h>

#include <vector>

#include "../../include/polymul.h"
#include "pm_plan.hpp"

namespace pm {

// Pinned host staging for the statistics read-back and descriptor uploads,
// plus a small device buffer for bound-only calls.  Not thread-safe: each
// user (the global API under its mutex, each server) owns one.
struct HostStage {
    void *pin = nullptr;
    size_t cap = 0;
    bool fixed = false;  // pin is caller-provided pageable memory of cap bytes: never grown or freed, no event
    hipEvent_t ev = nullptr;
    bool used = false;
    void *dtmp = nullptr;
    size_t dtmp_cap = 0;
    ~HostStage();
    int reserve(size_t bytes);
    int device_tmp(size_t bytes, void **out);
};

void set_error(const char *what, hipError_t e);
int device_cus();
int check_args(const pm_layout *L, int64_t count, const pm_cpoly *f, const pm_cpoly *g, const pm_poly *h);
int stats_roundtrip(HostStage &hs, const pm_layout *L, int64_t count, const pm_cpoly *f, const pm_cpoly *g,
                    void *dev, hipStream_t st, std::vector<SegInput> &in, const uint64_t **stats,
                    const uint32_t **flags, bool sync = true);
int stats_and_plan(HostStage &hs, const pm_layout *L, int64_t count, const pm_cpoly *f, const pm_cpoly *g,
                   void *dev, hipStream_t st, const Tuning &tune, Plan &P);
// ust: stream of the descriptor copy (null: st); st waits for it.
int upload_descriptors(HostStage &hs, Plan &P, void *ws, hipStream_t st, hipStream_t ust = nullptr);
// part: PipelinePart of pm_launch.hpp (default: the whole pipeline).
int upload_and_launch(HostStage &hs, Plan &P, const pm_poly *h, void *ws, hipStream_t st, hipStream_t ust = nullptr,
                      int part = 0);
int bound_impl(HostStage &hs, const pm_layout *L, int64_t count, const pm_cpoly *f, const pm_cpoly *g,
               int64_t *max_terms, int64_t *ws_bytes, hipStream_t st, const Tuning &tune);
int mul_impl(HostStage &hs, const pm_layout *L, int64_t count, const pm_cpoly *f, const pm_cpoly *g,
             const pm_poly *h, void *ws, int64_t ws_bytes, hipStream_t st, const Tuning &tune, Plan *plan_out);
Tuning &default_tuning();
// Exact integer coefficients (PM_Z192) through three modular products.
int z192_bound(HostStage &hs, const pm_layout *L, const pm_cpoly *f, const pm_cpoly *g, int64_t *max_terms,
               int64_t *ws_bytes, hipStream_t st, const Tuning &tune);
int z192_mul(HostStage &hs, const pm_layout *L, const pm_cpoly *f, const pm_cpoly *g, const pm_poly *h, void *ws,
             int64_t ws_bytes, hipStream_t st, const Tuning &tune);

}  // namespace pm
