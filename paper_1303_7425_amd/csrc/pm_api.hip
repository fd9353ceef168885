// C ABI of the sparse polynomial product (include/polymul.h): argument checks,
// the validation / statistics round trip, planning and launch.
#include <hip/hip_runtime.h>
#include <stdint.h>
#include <string.h>

#include <algorithm>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/polymul.h"
#include "pm_api_internal.hpp"
#include "pm_launch.hpp"

namespace pm {

static thread_local std::string g_last_error;
static thread_local void *g_last_counters = nullptr;
struct LastCall {
    void *dyn = nullptr;
    int nseg = 0, passes = 0, ksize = 0, vsize = 0;
    int64_t box = 0;
};
static thread_local LastCall g_last;

void set_error(const char *what, hipError_t e) {
    g_last_error = std::string(what) + ": " + hipGetErrorString(e);
}

int device_cus() {
    static int cus = 0;
    static std::once_flag once;
    std::call_once(once, [] {
        int dev = 0;
        hipDeviceProp_t prop;
        if (hipGetDevice(&dev) == hipSuccess && hipGetDeviceProperties(&prop, dev) == hipSuccess)
            cus = prop.multiProcessorCount;
        if (cus <= 0) cus = 256;
    });
    return cus;
}

HostStage::~HostStage() {
    if (pin && !fixed) (void)hipHostFree(pin);
    if (ev) (void)hipEventDestroy(ev);
    if (dtmp) (void)hipFree(dtmp);
}

// Pinned host staging of at least `bytes`; waits until the last upload that
// read from it has completed.
int HostStage::reserve(size_t bytes) {
    if (fixed) {
        // pageable memory: an upload from it has been staged by the time
        // hipMemcpyAsync returns, so it is free again at once
        if (bytes > cap) {
            set_error("host staging of the no-allocation entry point", hipErrorOutOfMemory);
            return PM_ENOMEM;
        }
        return PM_OK;
    }
    if (!ev) {
        hipError_t e = hipEventCreateWithFlags(&ev, hipEventDisableTiming);
        if (e != hipSuccess) {
            set_error("hipEventCreate", e);
            return PM_EDEVICE;
        }
    }
    if (used) {
        hipError_t e = hipEventSynchronize(ev);
        if (e != hipSuccess) {
            set_error("hipEventSynchronize", e);
            return PM_EDEVICE;
        }
        used = false;
    }
    if (bytes > cap) {
        if (pin) (void)hipHostFree(pin);
        pin = nullptr;
        cap = 0;
        size_t want = std::max<size_t>(bytes, 1 << 20);
        hipError_t e = hipHostMalloc(&pin, want, hipHostMallocDefault);
        if (e != hipSuccess) {
            set_error("hipHostMalloc", e);
            return PM_EDEVICE;
        }
        cap = want;
    }
    return PM_OK;
}

int HostStage::device_tmp(size_t bytes, void **out) {
    if (bytes > dtmp_cap) {
        if (dtmp) (void)hipFree(dtmp);
        dtmp = nullptr;
        dtmp_cap = 0;
        hipError_t e = hipMalloc(&dtmp, bytes);
        if (e != hipSuccess) {
            set_error("hipMalloc", e);
            return PM_EDEVICE;
        }
        dtmp_cap = bytes;
    }
    *out = dtmp;
    return PM_OK;
}

static int check_layout(const pm_layout *L) {
    if (!L) return PM_EINVAL;
    if (L->nvars < 1 || L->bits < 1 || (uint64_t)L->nvars * L->bits > 64) return PM_EINVAL;
    if (L->ring != PM_MODP61 && L->ring != PM_F64 && L->ring != PM_I64 && L->ring != PM_MODQ64 && L->ring != PM_Z192)
        return PM_EINVAL;
    if (L->reserved != 0) return PM_EINVAL;
    return PM_OK;
}

static int check_operand(const pm_cpoly *p) {
    if (!p || p->n < 0) return PM_EINVAL;
    if (p->n > 0 && (!p->keys || !p->coefs)) return PM_EINVAL;
    return PM_OK;
}

int check_args(const pm_layout *L, int64_t count, const pm_cpoly *f, const pm_cpoly *g, const pm_poly *h) {
    int rc = check_layout(L);
    if (rc) return rc;
    if (count < 0 || count > (int64_t)1 << 24) return PM_EINVAL;
    if (count > 0 && (!f || !g)) return PM_EINVAL;
    for (int64_t q = 0; q < count; q++) {
        if ((rc = check_operand(f + q)) || (rc = check_operand(g + q))) return rc;
        if (h) {
            const pm_poly &o = h[q];
            if (!o.n_out || o.capacity < 0) return PM_EINVAL;
            if (o.capacity > 0 && (!o.keys || !o.coefs)) return PM_EINVAL;
        }
    }
    return PM_OK;
}

// Validation + statistics round trip for `count` products: fills `in` and
// returns the statistics and flags (inside the pinned staging, valid until the
// next use of `hs`).  `dev` is device memory of at least stats_region_bytes +
// sizeof(DevSeg)*count.
int stats_roundtrip(HostStage &hs, const pm_layout *L, int64_t count, const pm_cpoly *f, const pm_cpoly *g,
                    void *dev, hipStream_t st, std::vector<SegInput> &in, const uint64_t **stats,
                    const uint32_t **flags, bool sync) {
    const int S = (int)count, nv = (int)L->nvars;
    const size_t sreg = stats_region_bytes(S, nv);
    const size_t segb = sizeof(DevSeg) * S;
    const size_t sb = stats_bytes(S, nv);
    const size_t up_off = 0, dn_off = (segb + 255) & ~(size_t)255;
    int rc = hs.reserve(dn_off + sreg);
    if (rc) return rc;
    DevSeg *hseg = (DevSeg *)((char *)hs.pin + up_off);
    in.resize(S);
    for (int q = 0; q < S; q++) {
        DevSeg d = DevSeg();
        d.fk = f[q].keys;
        d.fc = (const u64 *)f[q].coefs;
        d.gk = g[q].keys;
        d.gc = (const u64 *)g[q].coefs;
        d.na = f[q].n;
        d.nb = g[q].n;
        hseg[q] = d;
        in[q] = SegInput{d.fk, d.fc, d.gk, d.gc, d.na, d.nb};
    }
    char *dbase = (char *)dev;
    hipError_t e = hipMemcpyAsync(dbase + sreg, hseg, segb, hipMemcpyHostToDevice, st);
    if (e == hipSuccess) e = launch_stats((const DevSeg *)(dbase + sreg), S, nv, (int)L->bits, L->ring, (u64 *)dbase,
                                          (u32 *)(dbase + ((sb + 255) & ~(size_t)255)), st);
    char *hstats = (char *)hs.pin + dn_off;
    if (e == hipSuccess) e = hipMemcpyAsync(hstats, dbase, sreg, hipMemcpyDeviceToHost, st);
    if (e == hipSuccess && sync) e = hipStreamSynchronize(st);
    if (e != hipSuccess) {
        set_error("validation", e);
        return PM_EDEVICE;
    }
    *stats = (const uint64_t *)hstats;
    *flags = (const uint32_t *)(hstats + ((sb + 255) & ~(size_t)255));
    return PM_OK;
}

// Validation + statistics round trip and planning for `count` products.
int stats_and_plan(HostStage &hs, const pm_layout *L, int64_t count, const pm_cpoly *f, const pm_cpoly *g,
                   void *dev, hipStream_t st, const Tuning &tune, Plan &P) {
    std::vector<SegInput> in;
    const uint64_t *stats = nullptr;
    const uint32_t *flags = nullptr;
    int rc = stats_roundtrip(hs, L, count, f, g, dev, st, in, &stats, &flags);
    if (rc) return rc;
    return plan_build((int)L->nvars, (int)L->bits, L->ring, in, stats, flags, tune, P, device_cus());
}

// Upload the descriptor block of plan P (output pointers filled) and enqueue
// the pipeline.
int upload_descriptors(HostStage &hs, Plan &P, void *ws, hipStream_t st, hipStream_t ust) {
    int rc = hs.reserve(P.r_desc.bytes);
    if (rc) return rc;
    char *pin = (char *)hs.pin;
    const size_t d0 = P.r_desc.off;
    memcpy(pin + (P.o_segs - d0), P.segs.data(), sizeof(DevSeg) * P.nseg);
    if (!P.vars.empty()) memcpy(pin + (P.o_vars - d0), P.vars.data(), sizeof(VarParam) * P.vars.size());
    memcpy(pin + (P.o_tile_pre - d0), P.tile_pre.data(), 8 * P.tile_pre.size());
    if (!P.tile_seg.empty()) memcpy(pin + (P.o_tile_seg - d0), P.tile_seg.data(), 4 * P.tile_seg.size());
    memcpy(pin + (P.o_dpart_pre - d0), P.dpart_pre.data(), 8 * P.dpart_pre.size());
    if (!P.dseg.empty()) memcpy(pin + (P.o_dseg - d0), P.dseg.data(), 4 * P.dseg.size());
    memcpy(pin + (P.o_cpre - d0), P.cpre.data(), 8 * P.cpre.size());
    memcpy(pin + (P.o_iv_pre - d0), P.iv_pre.data(), 8 * P.iv_pre.size());
    if (!P.iv_seg.empty()) memcpy(pin + (P.o_iv_seg - d0), P.iv_seg.data(), 4 * P.iv_seg.size());
    if (!P.bk_tile_pre.empty()) memcpy(pin + (P.o_bk_tile_pre - d0), P.bk_tile_pre.data(), 8 * P.bk_tile_pre.size());
    if (!P.bk_seg.empty()) memcpy(pin + (P.o_bk_seg - d0), P.bk_seg.data(), 4 * P.bk_seg.size());
    if (!P.bk_sb_pre.empty()) memcpy(pin + (P.o_bk_sb_pre - d0), P.bk_sb_pre.data(), 8 * P.bk_sb_pre.size());
    // the copy runs on `ust` (default: the launch stream); the launch stream
    // then waits for it, so the staging is free once `ust` has run the copy
    if (!ust) ust = st;
    hipError_t e = hipMemcpyAsync((char *)ws + d0, pin, P.r_desc.bytes, hipMemcpyHostToDevice, ust);
    if (e == hipSuccess) e = hs.fixed ? hipStreamSynchronize(ust) : hipEventRecord(hs.ev, ust);
    if (e == hipSuccess && !hs.fixed && ust != st) e = hipStreamWaitEvent(st, hs.ev, 0);
    if (e != hipSuccess) {
        set_error("descriptor upload", e);
        return PM_EDEVICE;
    }
    hs.used = !hs.fixed;
    return PM_OK;
}

int upload_and_launch(HostStage &hs, Plan &P, const pm_poly *h, void *ws, hipStream_t st, hipStream_t ust, int part) {
    for (int q = 0; q < P.nseg; q++) {
        P.segs[q].hk = h[q].keys;
        P.segs[q].hc = (u64 *)h[q].coefs;
        P.segs[q].n_out = h[q].n_out;
        P.segs[q].cap = h[q].capacity;
    }
    int rc = upload_descriptors(hs, P, ws, st, ust);
    if (rc) return rc;
    hipError_t e;
    g_last_counters = (char *)ws + P.o_counters;
    g_last.dyn = (char *)ws + P.o_dyn;
    g_last.nseg = P.nseg;
    g_last.passes = P.passes;
    g_last.ksize = P.ksize;
    g_last.vsize = P.vsize;
    g_last.box = P.nbox;
    Ctx C = make_ctx(P, ws);
    e = launch_pipeline(P, C, st, device_cus(), part);
    if (e != hipSuccess) {
        set_error("kernel launch", e);
        return PM_EDEVICE;
    }
    return PM_OK;
}

static std::mutex g_mu;
static HostStage g_stage;
static Tuning g_tune;

Tuning &default_tuning() { return g_tune; }

int bound_impl(HostStage &hs, const pm_layout *L, int64_t count, const pm_cpoly *f, const pm_cpoly *g,
               int64_t *max_terms, int64_t *ws_bytes, hipStream_t st, const Tuning &tune) {
    if (count == 0) {
        if (ws_bytes) *ws_bytes = 0;
        return PM_OK;
    }
    const size_t need = stats_region_bytes((int)count, (int)L->nvars) + sizeof(DevSeg) * count;
    void *dev = nullptr;
    int rc = hs.device_tmp(need, &dev);
    if (rc) return rc;
    Plan P;
    rc = stats_and_plan(hs, L, count, f, g, dev, st, tune, P);
    if (rc) return rc;
    if (max_terms)
        for (int64_t q = 0; q < count; q++) max_terms[q] = P.bound[q];
    if (ws_bytes) *ws_bytes = (int64_t)P.total;
    return PM_OK;
}

int mul_impl(HostStage &hs, const pm_layout *L, int64_t count, const pm_cpoly *f, const pm_cpoly *g,
             const pm_poly *h, void *ws, int64_t ws_bytes, hipStream_t st, const Tuning &tune, Plan *plan_out) {
    if (count == 0) return PM_OK;
    const size_t need0 = stats_region_bytes((int)count, (int)L->nvars) + sizeof(DevSeg) * count;
    if (!ws || ws_bytes < (int64_t)need0) return PM_ENOMEM;
    if ((uintptr_t)ws & 255) return PM_EINVAL;  // kernels use 16-byte loads from workspace regions
    Plan P;
    int rc = stats_and_plan(hs, L, count, f, g, ws, st, tune, P);
    if (rc) return rc;
    if ((int64_t)P.total > ws_bytes) return PM_ENOMEM;
    rc = upload_and_launch(hs, P, h, ws, st);
    if (plan_out) *plan_out = P;
    return rc;
}

}  // namespace pm

using namespace pm;

extern "C" {

int pm_mul_bound(const pm_layout *layout, const pm_cpoly *f, const pm_cpoly *g, int64_t *max_terms,
                 int64_t *workspace_bytes, void *stream) {
    int rc = check_args(layout, 1, f, g, nullptr);
    if (rc) return rc;
    std::lock_guard<std::mutex> lk(g_mu);
    if (layout->ring == PM_Z192)
        return z192_bound(g_stage, layout, f, g, max_terms, workspace_bytes, (hipStream_t)stream, g_tune);
    return bound_impl(g_stage, layout, 1, f, g, max_terms, workspace_bytes, (hipStream_t)stream, g_tune);
}

int pm_mul(const pm_layout *layout, const pm_cpoly *f, const pm_cpoly *g, const pm_poly *h, void *workspace,
           int64_t workspace_bytes, void *stream) {
    int rc = check_args(layout, 1, f, g, h);
    if (rc) return rc;
    if (!h) return PM_EINVAL;
    std::lock_guard<std::mutex> lk(g_mu);
    if (layout->ring == PM_Z192)
        return z192_mul(g_stage, layout, f, g, h, workspace, workspace_bytes, (hipStream_t)stream, g_tune);
    return mul_impl(g_stage, layout, 1, f, g, h, workspace, workspace_bytes, (hipStream_t)stream, g_tune, nullptr);
}

int pm_mul_batch_bound(const pm_layout *layout, int64_t count, const pm_cpoly *f, const pm_cpoly *g,
                       int64_t *max_terms, int64_t *workspace_bytes, void *stream) {
    int rc = check_args(layout, count, f, g, nullptr);
    if (rc) return rc;
    if (layout->ring == PM_Z192) return PM_EINVAL;
    std::lock_guard<std::mutex> lk(g_mu);
    return bound_impl(g_stage, layout, count, f, g, max_terms, workspace_bytes, (hipStream_t)stream, g_tune);
}

int pm_mul_batch(const pm_layout *layout, int64_t count, const pm_cpoly *f, const pm_cpoly *g, const pm_poly *h,
                 void *workspace, int64_t workspace_bytes, void *stream) {
    int rc = check_args(layout, count, f, g, h);
    if (rc) return rc;
    if (count > 0 && !h) return PM_EINVAL;
    if (layout->ring == PM_Z192) return PM_EINVAL;
    std::lock_guard<std::mutex> lk(g_mu);
    return mul_impl(g_stage, layout, count, f, g, h, workspace, workspace_bytes, (hipStream_t)stream, g_tune,
                    nullptr);
}


// Batched products in waves, each wave's results drained to host memory and
// handed to the caller while the next wave runs on the device.
int pm_mul_batch_drain(const pm_layout *layout, int64_t count, const pm_cpoly *f, const pm_cpoly *g,
                       void *device_buffer, int64_t device_bytes, void *host_buffer, int64_t host_bytes,
                       pm_drain_fn fn, void *user, void *stream, int64_t *waves_out) {
    int rc = check_args(layout, count, f, g, nullptr);
    if (rc) return rc;
    if (layout->ring == PM_Z192 || !fn || !device_buffer || !host_buffer || device_bytes <= 0 || host_bytes <= 0)
        return PM_EINVAL;
    if ((uintptr_t)device_buffer & 255) return PM_EINVAL;
    if (waves_out) *waves_out = 0;
    if (count == 0) return PM_OK;
    std::lock_guard<std::mutex> lk(g_mu);
    hipStream_t st = (hipStream_t)stream;
    const int nv = (int)layout->nvars;
    const size_t need0 = stats_region_bytes((int)count, nv) + sizeof(DevSeg) * count;
    if ((size_t)device_bytes < need0) return PM_ENOMEM;
    // one statistics round trip for all products: bounds and planning inputs
    std::vector<SegInput> in;
    const uint64_t *st_p = nullptr;
    const uint32_t *fl_p = nullptr;
    rc = stats_roundtrip(g_stage, layout, count, f, g, device_buffer, st, in, &st_p, &fl_p);
    if (rc) return rc;
    const size_t sw = (size_t)4 * nv;
    std::vector<uint64_t> stats(st_p, st_p + (size_t)count * sw);
    std::vector<uint32_t> flags(fl_p, fl_p + (size_t)count * 2);
    auto al = [](size_t x) { return (x + 255) & ~(size_t)255; };
    const size_t half = ((size_t)device_bytes / 2) & ~(size_t)255;
    // products [a, e) as one wave: their planned workspace, bound-sized device
    // outputs and counts must fit half of the device buffer, their bound-sized
    // results the host buffer
    std::vector<int64_t> bound(count);
    auto wave_fits = [&](int64_t a, int64_t e, size_t *ws_out) -> int {
        std::vector<SegInput> sub(in.begin() + a, in.begin() + e);
        Plan P;
        const int r = plan_build(nv, (int)layout->bits, layout->ring, sub, stats.data() + (size_t)a * sw,
                                 flags.data() + (size_t)a * 2, g_tune, P, device_cus());
        if (r) return r;
        size_t dev = al(8 * (size_t)(e - a)), host = 0;
        for (int64_t q = a; q < e; q++) {
            bound[q] = P.bound[q - a];
            dev += 2 * al(8 * (size_t)std::max<int64_t>(bound[q], 1));
            host += 16 * (size_t)bound[q];
        }
        if (ws_out) *ws_out = P.total;
        return (dev + P.total <= half && host <= (size_t)host_bytes) ? PM_OK : PM_ENOMEM;
    };
    std::vector<int64_t> starts;
    for (int64_t a = 0; a < count;) {
        int r = wave_fits(a, a + 1, nullptr);
        if (r) return r;  // a single product that does not fit (or a validation error)
        int64_t good = a + 1, step = 1;
        while (good < count) {  // doubling, then bisection
            const int64_t e = std::min<int64_t>(count, good + step);
            if (wave_fits(a, e, nullptr) != PM_OK) break;
            good = e;
            step *= 2;
        }
        int64_t lo = good, hi = std::min<int64_t>(count, good + step);
        while (hi - lo > 1) {
            const int64_t mid = (lo + hi) / 2;
            if (wave_fits(a, mid, nullptr) == PM_OK) lo = mid;
            else hi = mid;
        }
        starts.push_back(a);
        a = lo;
    }
    starts.push_back(count);
    const int64_t nw = (int64_t)starts.size() - 1;
    hipStream_t cst = nullptr;
    hipError_t e = hipStreamCreateWithFlags(&cst, hipStreamNonBlocking);
    if (e != hipSuccess) {
        set_error("hipStreamCreate", e);
        return PM_EDEVICE;
    }
    // device layout of a wave in its half: counts, then per product keys and
    // coefficients (bound-sized), then the workspace
    struct Wave {
        int64_t a = 0, e = 0;
        char *base = nullptr;
        std::vector<size_t> ok, oc;
        size_t ws_off = 0;
    };
    auto place = [&](int64_t w) {
        Wave W;
        W.a = starts[w];
        W.e = starts[w + 1];
        W.base = (char *)device_buffer + (size_t)(w & 1) * half;
        size_t o = al(8 * (size_t)(W.e - W.a));
        for (int64_t q = W.a; q < W.e; q++) {
            W.ok.push_back(o);
            o += al(8 * (size_t)std::max<int64_t>(bound[q], 1));
            W.oc.push_back(o);
            o += al(8 * (size_t)std::max<int64_t>(bound[q], 1));
        }
        W.ws_off = o;
        return W;
    };
    std::vector<int64_t> counts;
    // copy wave W's results to the host buffer on the copy stream (after its
    // kernels, which the next wave's validation round trip has waited for),
    // then hand them to the caller
    auto drain = [&](const Wave &W) -> int {
        const int64_t n = W.e - W.a;
        counts.resize(n);
        hipError_t x = hipMemcpyAsync(counts.data(), W.base, 8 * (size_t)n, hipMemcpyDeviceToHost, cst);
        if (x == hipSuccess) x = hipStreamSynchronize(cst);
        char *hp = (char *)host_buffer;
        std::vector<std::pair<char *, char *>> at(n);
        for (int64_t i = 0; i < n && x == hipSuccess; i++) {
            const int64_t q = W.a + i, m = std::min(counts[i], bound[q]);
            at[i] = {hp, hp + 8 * (size_t)m};
            if (m > 0) {
                x = hipMemcpyAsync(at[i].first, W.base + W.ok[i], 8 * (size_t)m, hipMemcpyDeviceToHost, cst);
                if (x == hipSuccess)
                    x = hipMemcpyAsync(at[i].second, W.base + W.oc[i], 8 * (size_t)m, hipMemcpyDeviceToHost, cst);
            }
            hp += 16 * (size_t)m;
        }
        if (x == hipSuccess) x = hipStreamSynchronize(cst);
        if (x != hipSuccess) {
            set_error("result drain", x);
            return PM_EDEVICE;
        }
        for (int64_t i = 0; i < n; i++)
            fn(user, W.a + i, (const uint64_t *)at[i].first, at[i].second, std::min(counts[i], bound[W.a + i]));
        return PM_OK;
    };
    Wave prev;
    bool have_prev = false;
    for (int64_t w = 0; w < nw && rc == PM_OK; w++) {
        Wave W = place(w);
        const int64_t n = W.e - W.a;
        std::vector<pm_poly> h(n);
        for (int64_t i = 0; i < n; i++)
            h[i] = pm_poly{std::max<int64_t>(bound[W.a + i], 0), (int64_t *)(W.base + 8 * i), (uint64_t *)(W.base + W.ok[i]),
                           W.base + W.oc[i]};
        rc = mul_impl(g_stage, layout, n, f + W.a, g + W.a, h.data(), W.base + W.ws_off,
                      (int64_t)(half - W.ws_off), st, g_tune, nullptr);
        if (rc == PM_OK && have_prev) rc = drain(prev);  // overlaps wave w on the device
        prev = W;
        have_prev = true;
    }
    if (rc == PM_OK && have_prev) {
        e = hipStreamSynchronize(st);
        rc = e == hipSuccess ? drain(prev) : PM_EDEVICE;
        if (e != hipSuccess) set_error("drain", e);
    }
    (void)hipStreamSynchronize(cst);
    (void)hipStreamDestroy(cst);
    if (waves_out) *waves_out = nw;
    return rc;
}

}  // extern "C"

// ---------------------------------------------------------------------------
// pm_mul_noalloc: pm_mul with the workspace in a static device array.
// ---------------------------------------------------------------------------
// Each device that loads the library holds its own copy of `scratch` until the
// process ends.  In host code the array's name is only a stand-in: its device
// address comes from hipGetSymbolAddress, once per device, with that device
// current, and only that address is passed on.  The host side stages
// descriptors and statistics through a static pageable buffer.
static constexpr size_t NOALLOC_SCRATCH = (size_t)PM_NOALLOC_SCRATCH_BYTES;
static_assert(NOALLOC_SCRATCH % 256 == 0, "scratch size");
static __device__ __align__(256) unsigned char scratch[NOALLOC_SCRATCH];

namespace {
constexpr size_t NOALLOC_HOST = (size_t)4 << 20;
constexpr int NOALLOC_MAX_DEVICES = 64;
alignas(256) unsigned char g_noalloc_host[NOALLOC_HOST];
void *g_scratch_addr[NOALLOC_MAX_DEVICES];
HostStage g_noalloc_stage;

// Device address of `scratch` on the current device (caller holds g_mu).
int scratch_address(void **out) {
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) {
        set_error("hipGetDevice", e);
        return PM_EDEVICE;
    }
    if (dev < 0 || dev >= NOALLOC_MAX_DEVICES) {
        set_error("device index beyond the no-allocation table", hipErrorInvalidDevice);
        return PM_EDEVICE;
    }
    if (!g_scratch_addr[dev]) {
        void *p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p) {
            set_error("hipGetSymbolAddress(scratch)", e);
            return PM_EDEVICE;
        }
        g_scratch_addr[dev] = p;
    }
    *out = g_scratch_addr[dev];
    return PM_OK;
}
}  // namespace

extern "C" int pm_mul_noalloc(const pm_layout *layout, const pm_cpoly *f, const pm_cpoly *g, const pm_poly *h,
                              void *stream) {
    int rc = check_args(layout, 1, f, g, h);
    if (rc) return rc;
    if (!h || layout->ring == PM_Z192) return PM_EINVAL;
    std::lock_guard<std::mutex> lk(g_mu);
    void *ws = nullptr;
    rc = scratch_address(&ws);
    if (rc) return rc;
    if (!g_noalloc_stage.fixed) {
        g_noalloc_stage.fixed = true;
        g_noalloc_stage.pin = g_noalloc_host;
        g_noalloc_stage.cap = NOALLOC_HOST;
    }
    const size_t need0 = stats_region_bytes(1, (int)layout->nvars) + sizeof(DevSeg);
    if (need0 > NOALLOC_SCRATCH) return PM_ENOMEM;
    Plan P;
    rc = stats_and_plan(g_noalloc_stage, layout, 1, f, g, ws, (hipStream_t)stream, g_tune, P);
    if (rc) return rc;
    if (P.total > NOALLOC_SCRATCH) {
        set_error("workspace beyond the static scratch of pm_mul_noalloc", hipErrorOutOfMemory);
        return PM_ENOMEM;
    }
    return upload_and_launch(g_noalloc_stage, P, h, ws, (hipStream_t)stream);
}

struct pm_batch {
    pm::Plan plan;
    void *ws = nullptr;
    hipStream_t cap = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
};

extern "C" {

int pm_batch_prepare(const pm_layout *layout, int64_t count, const pm_cpoly *f, const pm_cpoly *g, const pm_poly *h,
                     void *workspace, int64_t workspace_bytes, void *stream, pm_batch **out) {
    if (!out) return PM_EINVAL;
    *out = nullptr;
    int rc = check_args(layout, count, f, g, h);
    if (rc) return rc;
    if (count < 1 || !h || layout->ring == PM_Z192) return PM_EINVAL;
    std::lock_guard<std::mutex> lk(g_mu);
    hipStream_t st = (hipStream_t)stream;
    const size_t need0 = stats_region_bytes((int)count, (int)layout->nvars) + sizeof(DevSeg) * count;
    if (!workspace || workspace_bytes < (int64_t)need0) return PM_ENOMEM;
    if ((uintptr_t)workspace & 255) return PM_EINVAL;
    pm_batch *b = new pm_batch();
    rc = stats_and_plan(g_stage, layout, count, f, g, workspace, st, g_tune, b->plan);
    if (!rc && (int64_t)b->plan.total > workspace_bytes) rc = PM_ENOMEM;
    if (rc) {
        delete b;
        return rc;
    }
    Plan &P = b->plan;
    b->ws = workspace;
    for (int q = 0; q < P.nseg; q++) {
        P.segs[q].hk = h[q].keys;
        P.segs[q].hc = (u64 *)h[q].coefs;
        P.segs[q].n_out = h[q].n_out;
        P.segs[q].cap = h[q].capacity;
    }
    // descriptors: upload once and wait, the graph only reads them
    rc = upload_descriptors(g_stage, P, workspace, st);
    hipError_t e = hipSuccess;
    if (!rc) e = hipStreamSynchronize(st);
    if (!rc && e == hipSuccess) e = hipStreamCreateWithFlags(&b->cap, hipStreamNonBlocking);
    if (!rc && e == hipSuccess) e = hipStreamBeginCapture(b->cap, hipStreamCaptureModeThreadLocal);
    if (!rc && e == hipSuccess) {
        Ctx C = make_ctx(P, workspace);
        hipError_t le = launch_pipeline(P, C, b->cap, device_cus());
        e = hipStreamEndCapture(b->cap, &b->graph);
        if (e == hipSuccess) e = le;
    }
    if (!rc && e == hipSuccess) e = hipGraphInstantiate(&b->exec, b->graph, nullptr, nullptr, 0);
    if (!rc && e != hipSuccess) {
        set_error("graph capture", e);
        rc = PM_EDEVICE;
    }
    if (rc) {
        pm_batch_destroy(b);
        return rc;
    }
    *out = b;
    return PM_OK;
}

int pm_batch_launch(pm_batch *b, void *stream) {
    if (!b || !b->exec) return PM_EINVAL;
    hipError_t e = hipGraphLaunch(b->exec, (hipStream_t)stream);
    if (e != hipSuccess) {
        set_error("hipGraphLaunch", e);
        return PM_EDEVICE;
    }
    g_last_counters = (char *)b->ws + b->plan.o_counters;
    g_last.dyn = (char *)b->ws + b->plan.o_dyn;
    g_last.nseg = b->plan.nseg;
    g_last.passes = b->plan.passes;
    g_last.ksize = b->plan.ksize;
    g_last.vsize = b->plan.vsize;
    g_last.box = b->plan.nbox;
    return PM_OK;
}

void pm_batch_destroy(pm_batch *b) {
    if (!b) return;
    if (b->exec) (void)hipGraphExecDestroy(b->exec);
    if (b->graph) (void)hipGraphDestroy(b->graph);
    if (b->cap) (void)hipStreamDestroy(b->cap);
    delete b;
}

int pm_autotune(const pm_layout *layout, const pm_cpoly *f, const pm_cpoly *g, const pm_poly *h, void *workspace,
                int64_t workspace_bytes, void *stream, int32_t *tile_cfg, int32_t *combine, int32_t *digits) {
    int rc = check_args(layout, 1, f, g, h);
    if (rc) return rc;
    if (!h || layout->ring == PM_Z192) return PM_EINVAL;
    std::lock_guard<std::mutex> lk(g_mu);
    hipStream_t st = (hipStream_t)stream;
    // which path does this product take?
    Plan P0;
    Tuning base = g_tune;
    base.tile_cfg = -1;
    base.combine = -1;
    base.digits = -1;
    rc = mul_impl(g_stage, layout, 1, f, g, h, workspace, workspace_bytes, st, base, &P0);
    if (rc) return rc;
    if (P0.nseg < 1 || P0.segs[0].mode == SEG_EMPTY) return PM_OK;
    const bool dense = P0.segs[0].mode == SEG_DENSE;
    struct Cand {
        int tile_cfg, combine, digits;
    };
    std::vector<Cand> cands;  // radix-sorted settings are tried with both digit schedules
    const int G = RADIX_DIGITS_GREEDY, B = RADIX_DIGITS_BALANCED;
    if (dense) {
        for (int t = 0; t < N_TILE_CFGS; t++) cands.push_back({t, 0, -1});
    } else if (layout->ring != PM_F64) {
        cands.push_back({-1, 3, -1});
        cands.push_back({-1, 2, -1});
        cands.push_back({-1, 0, B});
        cands.push_back({-1, 0, G});
        cands.push_back({0, 1, B});
        cands.push_back({0, 1, G});
    } else {
        cands.push_back({-1, 3, -1});
        cands.push_back({-1, 2, -1});
        cands.push_back({-1, 0, B});
        cands.push_back({-1, 0, G});
    }
    hipEvent_t e0, e1;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) return PM_EDEVICE;
    float best = 1e30f;
    Cand choice = cands[0];
    for (auto &cd : cands) {
        Tuning t = base;
        t.tile_cfg = cd.tile_cfg;
        t.combine = cd.combine;
        t.digits = cd.digits;
        rc = mul_impl(g_stage, layout, 1, f, g, h, workspace, workspace_bytes, st, t, nullptr);  // warm-up
        if (rc == PM_ENOMEM) {  // this setting needs more workspace than given: not a candidate
            rc = PM_OK;
            continue;
        }
        if (rc) break;
        float total = 0;
        for (int rep = 0; rep < 2 && !rc; rep++) {
            (void)hipEventRecord(e0, st);
            rc = mul_impl(g_stage, layout, 1, f, g, h, workspace, workspace_bytes, st, t, nullptr);
            (void)hipEventRecord(e1, st);
            (void)hipEventSynchronize(e1);
            float ms = 0;
            (void)hipEventElapsedTime(&ms, e0, e1);
            total += ms;
        }
        if (rc) break;
        if (total < best) {
            best = total;
            choice = cd;
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (rc) return rc;
    const uint64_t pairs = (uint64_t)f->n * (uint64_t)g->n;
    tune_store(TuneClass{layout->ring, dense ? 1 : 0, log2_floor(pairs)}, choice.tile_cfg, choice.combine,
               choice.digits);
    if (tile_cfg) *tile_cfg = choice.tile_cfg;
    if (combine) *combine = choice.combine;
    if (digits) *digits = choice.digits;
    return PM_OK;
}

void pm_autotune_reset(void) { tune_reset(); }

int pm_autotune_save(const char *path) { return path ? tune_save(path) : PM_EINVAL; }

int pm_autotune_load(const char *path) { return path ? tune_load(path) : PM_EINVAL; }

int pm_plan_from_stats(const pm_layout *layout, int64_t count, const int64_t *na, const int64_t *nb,
                       const uint64_t *stats, int64_t *max_terms, int64_t *workspace_bytes) {
    int rc = check_layout(layout);
    if (rc) return rc;
    if (count < 0 || (count > 0 && (!na || !nb || !stats)) || layout->ring == PM_Z192) return PM_EINVAL;
    std::vector<SegInput> in(count);
    for (int64_t q = 0; q < count; q++) {
        if (na[q] < 0 || nb[q] < 0) return PM_EINVAL;
        in[q] = SegInput{nullptr, nullptr, nullptr, nullptr, na[q], nb[q]};
    }
    std::vector<uint32_t> flags(2 * count, 0);
    Plan P;
    rc = plan_build((int)layout->nvars, (int)layout->bits, layout->ring, in, stats, flags.data(), g_tune, P);
    if (rc) return rc;
    if (max_terms)
        for (int64_t q = 0; q < count; q++) max_terms[q] = P.bound[q];
    if (workspace_bytes) *workspace_bytes = (int64_t)P.total;
    return PM_OK;
}

int pm_dense_ceiling(int32_t ring, double *pairs_per_second, void *stream) {
    if (!pairs_per_second || (ring != PM_MODP61 && ring != PM_I64 && ring != PM_MODQ64)) return PM_EINVAL;
    hipStream_t st = (hipStream_t)stream;
    const int grid = device_cus() * 8, tiles = 64;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    hipError_t e = hipEventCreate(&e0);
    if (e == hipSuccess) e = hipEventCreate(&e1);
    if (e == hipSuccess) e = launch_dense_ceiling(ring, grid, tiles, st);  // warm-up
    if (e == hipSuccess) e = hipEventRecord(e0, st);
    for (int r = 0; r < 3 && e == hipSuccess; r++) e = launch_dense_ceiling(ring, grid, tiles, st);
    if (e == hipSuccess) e = hipEventRecord(e1, st);
    if (e == hipSuccess) e = hipEventSynchronize(e1);
    float ms = 0;
    if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    if (e != hipSuccess) {
        set_error("dense ceiling", e);
        return PM_EDEVICE;
    }
    *pairs_per_second = 3.0 * grid * tiles * 4096.0 / (ms * 1e-3);
    return PM_OK;
}

int pm_ival_grid(int64_t na, int64_t nb, int32_t l, int64_t *rows, int64_t *cols) {
    if (na < 1 || nb < 1 || l < 0 || l > 63 || !rows || !cols) return PM_EINVAL;
    const int64_t ns = (int64_t)(l + 1) * (l + 1);
    for (int64_t t = 0; t < ns; t++) ival_grid_point(na, nb, l, t, rows[t], cols[t]);
    return PM_OK;
}

int pm_ival_splitters(const uint64_t *fkeys, int64_t na, const uint64_t *gkeys, int64_t nb, int32_t l,
                      uint64_t *spl, int64_t *nspl) {
    if (na < 1 || nb < 1 || l < 0 || l > 63 || !fkeys || !gkeys || !spl || !nspl) return PM_EINVAL;
    const int64_t ns = (int64_t)(l + 1) * (l + 1);
    std::vector<uint64_t> v(ns);
    for (int64_t t = 0; t < ns; t++) {
        int64_t i, j;
        ival_grid_point(na, nb, l, t, i, j);
        v[t] = fkeys[i] + gkeys[j];
    }
    std::sort(v.begin(), v.end());
    const uint64_t kmin = fkeys[0] + gkeys[0], kend = fkeys[na - 1] + gkeys[nb - 1] + 1;
    int64_t n = 0;
    spl[n++] = kmin;
    for (int64_t t = 0; t < ns; t++)
        if (v[t] > kmin && v[t] < kend && (t == 0 || v[t - 1] != v[t])) spl[n++] = v[t];
    spl[n++] = kend;
    *nspl = n;
    return PM_OK;
}

int pm_set_tuning(int32_t tile_cfg, int32_t combine, int32_t allow_dense) {
    std::lock_guard<std::mutex> lk(g_mu);
    if (tile_cfg < -1 || tile_cfg >= N_TILE_CFGS || combine < -1 || combine > 3) return PM_EINVAL;
    g_tune.tile_cfg = tile_cfg;
    g_tune.combine = combine;
    g_tune.allow_dense = allow_dense ? 1 : 0;
    return PM_OK;
}

int pm_set_radix(int32_t digits) {
    std::lock_guard<std::mutex> lk(g_mu);
    if (digits < -1 || digits > 1) return PM_EINVAL;
    g_tune.digits = digits;
    return PM_OK;
}

int pm_last_call_info(void *stream, int64_t *staged_pairs, int32_t *passes, int32_t *key_bytes,
                      int32_t *payload_bytes, int64_t *box_cells) {
    hipError_t e = hipStreamSynchronize((hipStream_t)stream);
    if (e != hipSuccess) {
        set_error("hipStreamSynchronize", e);
        return PM_EDEVICE;
    }
    int64_t staged = 0;
    if (g_last.dyn && g_last.nseg > 0) {
        std::vector<DevSegDyn> d(g_last.nseg);
        e = hipMemcpy(d.data(), g_last.dyn, sizeof(DevSegDyn) * g_last.nseg, hipMemcpyDeviceToHost);
        if (e != hipSuccess) {
            set_error("hipMemcpy", e);
            return PM_EDEVICE;
        }
        for (auto &x : d) staged += x.n;
    }
    if (staged_pairs) *staged_pairs = staged;
    if (passes) *passes = g_last.passes;
    if (key_bytes) *key_bytes = g_last.ksize;
    if (payload_bytes) *payload_bytes = g_last.vsize;
    if (box_cells) *box_cells = g_last.box;
    return PM_OK;
}

int pm_profile_enable(int32_t enable) { return profile_enable(enable); }

int pm_profile_read(int32_t i, char *name, int32_t name_cap, double *total_ms, int64_t *launches) {
    return profile_read(i, name, name_cap, total_ms, launches);
}

const char *pm_strerror(int code) {
    switch (code) {
        case PM_OK: return "ok";
        case PM_EINVAL: return "invalid argument (null pointer, bad layout, negative size or key bits outside the fields)";
        case PM_EUNSORTED: return "operand keys are not strictly ascending";
        case PM_EOVERFLOW: return "exponent sum does not fit its field (PM_Z192: or the coefficient bound exceeds 2^187)";
        case PM_ERANGE: return "coefficient out of range (residue >= 2^61-1 or non-finite double)";
        case PM_ECAPACITY: return "output capacity below the result bound";
        case PM_ENOMEM: return "workspace or arena too small";
        case PM_EDEVICE: return "HIP runtime error";
        case PM_EBUSY: return "server queue full";
        default: return "unknown error";
    }
}

const char *pm_last_error(void) { return g_last_error.c_str(); }

int pm_last_call_status(void *stream) {
    hipError_t e = hipStreamSynchronize((hipStream_t)stream);
    if (e != hipSuccess) {
        set_error("hipStreamSynchronize", e);
        return PM_EDEVICE;
    }
    if (!g_last_counters) return PM_OK;
    uint32_t flag = 0;
    e = hipMemcpy(&flag, (char *)g_last_counters + 4 * CNT_ERR_SPIN, 4, hipMemcpyDeviceToHost);
    if (e != hipSuccess) {
        set_error("hipMemcpy", e);
        return PM_EDEVICE;
    }
    if (flag) {
        g_last_error = std::string("device consistency check failed, flags ") + std::to_string(flag);
        return PM_EDEVICE;
    }
    return PM_OK;
}

const char *pm_version(void) { return "polymul-gfx950 1.0"; }

}  // extern "C"
