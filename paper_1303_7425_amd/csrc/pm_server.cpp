// Serving loop (continuous batching) of the sparse polynomial product; see
// pm_server_* in include/polymul.h.
//
// One scheduler thread per server.  Submitted requests wait in a FIFO queue.
// The scheduler takes the oldest requests that share a layout and starts
// their validation (statistics kernel and read-back on the planning stream)
// without waiting for it; the read-back is polled like the completions.  Once
// it has arrived, the batch is planned on the host; the longest prefix whose
// workspace fits the free part of the server's HBM arena is admitted (the
// rest waits for a later round; a single request that can never fit fails
// with PM_ENOMEM).  Descriptors are uploaded on the planning stream and the
// batch is launched round-robin on the server's streams, which wait for the
// upload, so new work starts while earlier batches still run.  Completion is
// detected with events; the batch's device error flag (read back behind its
// kernels) decides between PM_OK and PM_EDEVICE, the arena range is returned
// and the tickets finish.  A batch whose tile work spans several launches
// (large dense products) is enqueued one tile launch at a time: after each,
// the next waits while other batches are in flight or queued (at most
// DENSE_YIELD_US), so small requests run beside one tile launch at most
// instead of beside the whole product.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <deque>
#include <map>
#include <mutex>
#include <thread>
#include <unordered_map>
#include <vector>

#include "../../include/polymul.h"
#include "pm_api_internal.hpp"
#include "pm_launch.hpp"

namespace pm {

static double now_us() {
    using namespace std::chrono;
    return duration<double, std::micro>(steady_clock::now().time_since_epoch()).count();
}

// First-fit allocator over [0, size) in 256-byte units.
struct Arena {
    int64_t size = 0;
    std::map<int64_t, int64_t> free_;  // offset -> length
    void init(int64_t s) {
        size = s;
        free_.clear();
        free_[0] = s;
    }
    int64_t largest() const {
        int64_t m = 0;
        for (auto &f : free_) m = std::max(m, f.second);
        return m;
    }
    int64_t alloc(int64_t n) {
        n = (n + 255) & ~(int64_t)255;
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second >= n) {
                const int64_t off = it->first, len = it->second;
                free_.erase(it);
                if (len > n) free_[off + n] = len - n;
                return off;
            }
        }
        return -1;
    }
    void release(int64_t off, int64_t n) {
        n = (n + 255) & ~(int64_t)255;
        auto it = free_.emplace(off, n).first;
        auto nx = std::next(it);
        if (nx != free_.end() && it->first + it->second == nx->first) {
            it->second += nx->second;
            free_.erase(nx);
        }
        if (it != free_.begin()) {
            auto pv = std::prev(it);
            if (pv->first + pv->second == it->first) {
                pv->second += it->second;
                free_.erase(it);
            }
        }
    }
};

struct Request {
    uint64_t ticket;
    pm_layout L;
    pm_cpoly f, g;
    pm_poly h;
    double t_submit;
    double latency = 0;  // completion seen by the scheduler minus submission, microseconds
    int status = PM_OK;
    bool done = false;
};

constexpr double DENSE_YIELD_US = 2000.0;

struct InFlight {
    std::vector<Request *> reqs;
    hipEvent_t ev = nullptr;
    int64_t off = 0, bytes = 0;
    int slot = 0;  // pinned word receiving the batch's device error flag
    // staged tile launches: the plan, its stream, the next launch to enqueue
    // (== nchunks: the tail), and when the previous part was seen done
    bool staged = false;
    Plan P;
    hipStream_t st = nullptr;
    int64_t next_chunk = 0, nchunks = 0;
    double t_ready = -1;
};

// A batch whose statistics read-back is in flight.
struct Validation {
    bool active = false;
    std::vector<Request *> group;
    int64_t off0 = -1, need0 = 0;
    hipEvent_t ev = nullptr;
    std::vector<SegInput> in;
    const uint64_t *stats = nullptr;
    const uint32_t *flags = nullptr;
};

}  // namespace pm

using namespace pm;

struct pm_server {
    void *arena_ptr = nullptr;
    Arena arena;
    std::vector<hipStream_t> streams;
    hipStream_t plan_stream = nullptr;
    int next_stream = 0;
    std::mutex mu;
    std::condition_variable cv_submit, cv_done;
    std::deque<Request *> pending;
    std::unordered_map<uint64_t, Request *> reqs;
    std::vector<InFlight> inflight;
    std::vector<double> latencies;
    std::thread th;
    bool stop = false;
    uint64_t next_ticket = 1;
    HostStage stage;  // used by the scheduler thread only
    Validation val;
    uint32_t *err_host = nullptr;  // pinned, one word per in-flight batch
    std::vector<int> free_slots;
    size_t max_pending = 1 << 16;
    int max_batch = 64;
    int max_inflight = 8;
    int device = 0;
};

static void finish(pm_server *s, Request *r, int status, double t) {
    r->status = status;
    r->latency = t - r->t_submit;
    r->done = true;
    if (status == PM_OK) s->latencies.push_back(r->latency);
}

// Remove r from the pending queue (caller holds s->mu).
static void unqueue(pm_server *s, Request *r) {
    auto it = std::find(s->pending.begin(), s->pending.end(), r);
    if (it != s->pending.end()) s->pending.erase(it);
}

// The validation of s->val has arrived: plan, admit a prefix that fits the
// arena and launch it.  Returns after launching or deferring the batch.
static void plan_and_launch(pm_server *s, std::vector<hipEvent_t> &free_events) {
    Validation &v = s->val;
    const pm_layout L = v.group[0]->L;
    const int nv = (int)L.nvars;
    const size_t sw = (size_t)4 * nv;
    int k = (int)v.group.size();
    // the statistics live in the pinned staging, which the upload reuses
    std::vector<uint64_t> stats(v.stats, v.stats + (size_t)k * sw);
    std::vector<uint32_t> flags(v.flags, v.flags + (size_t)k * 2);
    std::vector<SegInput> in = v.in;
    std::vector<Request *> group = v.group;
    {
        std::lock_guard<std::mutex> lk(s->mu);
        s->arena.release(v.off0, v.need0);
    }
    v.active = false;
    const int cus = device_cus();
    const Tuning &tune = default_tuning();
    auto plan_prefix = [&](int n, Plan &P) {
        std::vector<SegInput> sub(in.begin(), in.begin() + n);
        return plan_build(nv, (int)L.bits, L.ring, sub, stats.data(), flags.data(), tune, P, cus);
    };
    // requests that fail validation or have too small result arrays fail alone
    {
        std::vector<Request *> g2;
        std::vector<SegInput> in2;
        std::vector<uint64_t> st2;
        std::vector<uint32_t> fl2;
        for (int i = 0; i < k; i++) {
            Plan P1;
            std::vector<SegInput> one{in[i]};
            int rc = plan_build(nv, (int)L.bits, L.ring, one, stats.data() + i * sw, flags.data() + 2 * i, tune, P1,
                                cus);
            if (rc == PM_OK && group[i]->h.capacity < P1.bound[0]) rc = PM_ECAPACITY;
            if (rc == PM_OK && (int64_t)P1.total > s->arena.size) rc = PM_ENOMEM;
            if (rc != PM_OK) {
                std::lock_guard<std::mutex> lk(s->mu);
                unqueue(s, group[i]);
                finish(s, group[i], rc, now_us());
                s->cv_done.notify_all();
                continue;
            }
            g2.push_back(group[i]);
            in2.push_back(in[i]);
            st2.insert(st2.end(), stats.begin() + i * sw, stats.begin() + (i + 1) * sw);
            fl2.insert(fl2.end(), flags.begin() + 2 * i, flags.begin() + 2 * i + 2);
        }
        group.swap(g2);
        in.swap(in2);
        stats.swap(st2);
        flags.swap(fl2);
        k = (int)group.size();
    }
    // the longest admissible prefix (halving); the rest stays queued
    while (k >= 1) {
        Plan P;
        int rc = plan_prefix(k, P);
        if (rc != PM_OK) return;  // not reached: every request planned alone
        int64_t off = -1;
        {
            std::lock_guard<std::mutex> lk(s->mu);
            off = s->arena.alloc((int64_t)P.total);
        }
        if (off < 0) {
            if (k == 1) return;  // wait for memory; it is validated again later
            k /= 2;
            continue;
        }
        std::vector<pm_poly> h(k);
        for (int i = 0; i < k; i++) h[i] = group[i]->h;
        void *ws = (char *)s->arena_ptr + off;
        hipStream_t st = s->streams[s->next_stream];
        s->next_stream = (s->next_stream + 1) % (int)s->streams.size();
        const int slot = s->free_slots.back();
        s->free_slots.pop_back();
        s->err_host[slot] = 0;
        const int64_t nchunks = tile_launches(P);
        const bool staged = nchunks > 1;
        rc = upload_and_launch(s->stage, P, h.data(), ws, st, s->plan_stream, staged ? PART_HEAD : PART_ALL);
        if (rc == PM_OK && !staged &&
            hipMemcpyAsync(&s->err_host[slot], (char *)ws + P.o_counters + sizeof(u32) * CNT_ERR_SPIN, sizeof(u32),
                           hipMemcpyDeviceToHost, st) != hipSuccess)
            rc = PM_EDEVICE;
        hipEvent_t ev = nullptr;
        if (!free_events.empty()) {
            ev = free_events.back();
            free_events.pop_back();
        } else {
            (void)hipEventCreateWithFlags(&ev, hipEventDisableTiming);
        }
        if (rc == PM_OK && hipEventRecord(ev, st) != hipSuccess) rc = PM_EDEVICE;
        std::lock_guard<std::mutex> lk(s->mu);
        for (int i = 0; i < k; i++) unqueue(s, group[i]);
        if (rc != PM_OK) {
            const double t = now_us();
            for (int i = 0; i < k; i++) finish(s, group[i], rc, t);
            s->arena.release(off, (int64_t)P.total);
            free_events.push_back(ev);
            s->free_slots.push_back(slot);
            s->cv_done.notify_all();
        } else {
            InFlight b;
            b.reqs.assign(group.begin(), group.begin() + k);
            b.ev = ev;
            b.off = off;
            b.bytes = (int64_t)P.total;
            b.slot = slot;
            if (nchunks > 1) {
                b.staged = true;
                b.P = P;
                b.st = st;
                b.next_chunk = 1;
                b.nchunks = nchunks;
            }
            s->inflight.push_back(b);
        }
        return;
    }
}

static void scheduler(pm_server *s) {
    (void)hipSetDevice(s->device);
    std::vector<hipEvent_t> free_events;
    Validation &v = s->val;
    (void)hipEventCreateWithFlags(&v.ev, hipEventDisableTiming);
    while (true) {
        bool progress = false;
        // 1. completions: the batch's error flag arrived before its event;
        // a staged batch whose last part is done enqueues its next part, after
        // yielding to other work for at most DENSE_YIELD_US
        {
            bool others = false;
            {
                std::lock_guard<std::mutex> lk(s->mu);
                others = !s->pending.empty() || v.active;
            }
            for (auto &b : s->inflight) others = others || !b.staged;
            std::vector<InFlight> still;
            for (auto &b : s->inflight) {
                if (b.staged && hipEventQuery(b.ev) == hipSuccess) {
                    const double t = now_us();
                    if (b.t_ready < 0) b.t_ready = t;
                    if (others && t - b.t_ready < DENSE_YIELD_US) {
                        still.push_back(b);
                        continue;
                    }
                    void *ws = (char *)s->arena_ptr + b.off;
                    const Ctx C = make_ctx(b.P, ws);
                    hipError_t e = hipSuccess;
                    if (b.next_chunk < b.nchunks) {
                        e = launch_pipeline(b.P, C, b.st, device_cus(), PART_CHUNK, b.next_chunk);
                        b.next_chunk++;
                    } else {
                        e = launch_pipeline(b.P, C, b.st, device_cus(), PART_TAIL);
                        if (e == hipSuccess)
                            e = hipMemcpyAsync(&s->err_host[b.slot], (char *)ws + b.P.o_counters + sizeof(u32) * CNT_ERR_SPIN,
                                               sizeof(u32), hipMemcpyDeviceToHost, b.st);
                        b.staged = false;
                    }
                    if (e == hipSuccess) e = hipEventRecord(b.ev, b.st);
                    if (e != hipSuccess) {
                        s->err_host[b.slot] = 1;  // reported as PM_EDEVICE once the stream drains
                        b.staged = false;
                        (void)hipEventRecord(b.ev, b.st);
                    }
                    b.t_ready = -1;
                    progress = true;
                    still.push_back(b);
                    continue;
                }
                if (!b.staged && hipEventQuery(b.ev) == hipSuccess) {
                    const double t = now_us();
                    const int status = s->err_host[b.slot] ? PM_EDEVICE : PM_OK;
                    std::lock_guard<std::mutex> lk(s->mu);
                    for (Request *r : b.reqs) finish(s, r, status, t);
                    s->arena.release(b.off, b.bytes);
                    free_events.push_back(b.ev);
                    s->free_slots.push_back(b.slot);
                    s->cv_done.notify_all();
                    progress = true;
                } else {
                    still.push_back(b);
                }
            }
            s->inflight.swap(still);
        }
        // 2. a validation whose read-back has arrived
        if (v.active) {
            const hipError_t q = hipEventQuery(v.ev);
            if (q == hipSuccess) {
                plan_and_launch(s, free_events);
                progress = true;
            } else if (q != hipErrorNotReady) {
                std::lock_guard<std::mutex> lk(s->mu);
                for (Request *r : v.group) {
                    unqueue(s, r);
                    finish(s, r, PM_EDEVICE, now_us());
                }
                s->arena.release(v.off0, v.need0);
                v.active = false;
                s->cv_done.notify_all();
            }
        }
        // 3. start the validation of the oldest requests sharing a layout
        if (!v.active && (int)s->inflight.size() < s->max_inflight) {
            std::vector<Request *> group;
            {
                std::lock_guard<std::mutex> lk(s->mu);
                if (!s->pending.empty()) {
                    const pm_layout L0 = s->pending.front()->L;
                    for (Request *r : s->pending) {
                        if (r->L.nvars == L0.nvars && r->L.bits == L0.bits && r->L.ring == L0.ring) group.push_back(r);
                        if ((int)group.size() >= s->max_batch) break;
                    }
                }
            }
            if (!group.empty()) {
                const int k = (int)group.size();
                const int64_t need0 = (int64_t)(stats_region_bytes(k, (int)group[0]->L.nvars) + sizeof(DevSeg) * k);
                int64_t off0 = -1;
                {
                    std::lock_guard<std::mutex> lk(s->mu);
                    off0 = s->arena.alloc(need0);
                }
                if (off0 >= 0) {
                    std::vector<pm_cpoly> f(k), g(k);
                    for (int i = 0; i < k; i++) {
                        f[i] = group[i]->f;
                        g[i] = group[i]->g;
                    }
                    int rc = stats_roundtrip(s->stage, &group[0]->L, k, f.data(), g.data(),
                                             (char *)s->arena_ptr + off0, s->plan_stream, v.in, &v.stats, &v.flags,
                                             false);
                    if (rc == PM_OK && hipEventRecord(v.ev, s->plan_stream) != hipSuccess) rc = PM_EDEVICE;
                    if (rc != PM_OK) {
                        std::lock_guard<std::mutex> lk(s->mu);
                        for (Request *r : group) {
                            unqueue(s, r);
                            finish(s, r, rc, now_us());
                        }
                        s->arena.release(off0, need0);
                        s->cv_done.notify_all();
                    } else {
                        v.group = group;
                        v.off0 = off0;
                        v.need0 = need0;
                        v.active = true;
                    }
                    progress = true;
                }
            }
        }
        if (!progress) {
            std::unique_lock<std::mutex> lk(s->mu);
            if (s->stop && s->pending.empty() && s->inflight.empty() && !v.active) break;
            if (s->inflight.empty() && !v.active) {
                s->cv_submit.wait_for(lk, std::chrono::milliseconds(1));
            } else {
                lk.unlock();
                std::this_thread::sleep_for(std::chrono::microseconds(20));
            }
        }
    }
    for (hipEvent_t e : free_events) (void)hipEventDestroy(e);
    (void)hipEventDestroy(v.ev);
}

extern "C" {

pm_server *pm_server_create(int64_t hbm_budget_bytes, int32_t nstreams) {
    if (hbm_budget_bytes < (1 << 20) || nstreams < 1 || nstreams > 8) return nullptr;
    pm_server *s = new pm_server();
    (void)hipGetDevice(&s->device);
    hipError_t e = hipMalloc(&s->arena_ptr, (size_t)hbm_budget_bytes);
    if (e != hipSuccess) {
        set_error("server arena", e);
        delete s;
        return nullptr;
    }
    s->arena.init(hbm_budget_bytes);
    e = hipHostMalloc((void **)&s->err_host, sizeof(uint32_t) * s->max_inflight, hipHostMallocDefault);
    if (e != hipSuccess) {
        set_error("server error flags", e);
        (void)hipFree(s->arena_ptr);
        delete s;
        return nullptr;
    }
    for (int i = 0; i < s->max_inflight; i++) s->free_slots.push_back(i);
    for (int i = 0; i < nstreams && e == hipSuccess; i++) {
        hipStream_t st;
        e = hipStreamCreateWithFlags(&st, hipStreamNonBlocking);
        if (e == hipSuccess) s->streams.push_back(st);
    }
    if (e == hipSuccess) e = hipStreamCreateWithFlags(&s->plan_stream, hipStreamNonBlocking);
    if (e != hipSuccess) {
        set_error("server streams", e);
        for (auto st : s->streams) (void)hipStreamDestroy(st);
        (void)hipFree(s->arena_ptr);
        (void)hipHostFree(s->err_host);
        delete s;
        return nullptr;
    }
    s->th = std::thread(scheduler, s);
    return s;
}

int pm_server_submit(pm_server *s, const pm_layout *layout, const pm_cpoly *f, const pm_cpoly *g, const pm_poly *h,
                     uint64_t *ticket) {
    if (!s || !ticket || !h) return PM_EINVAL;
    int rc = check_args(layout, 1, f, g, h);
    if (rc) return rc;
    if (layout->ring == PM_Z192) return PM_EINVAL;
    // the capacity check against the bound needs the device statistics: the
    // scheduler fails a request whose result arrays are too small
    Request *r = new Request();
    r->L = *layout;
    r->f = *f;
    r->g = *g;
    r->h = *h;
    r->t_submit = now_us();
    std::lock_guard<std::mutex> lk(s->mu);
    if (s->pending.size() >= s->max_pending) {
        delete r;
        return PM_EBUSY;
    }
    r->ticket = s->next_ticket++;
    s->reqs[r->ticket] = r;
    s->pending.push_back(r);
    *ticket = r->ticket;
    s->cv_submit.notify_one();
    return PM_OK;
}

int pm_server_poll(pm_server *s, uint64_t ticket, int32_t *done, int32_t *status) {
    if (!s || !done) return PM_EINVAL;
    std::lock_guard<std::mutex> lk(s->mu);
    auto it = s->reqs.find(ticket);
    if (it == s->reqs.end()) return PM_EINVAL;
    *done = it->second->done ? 1 : 0;
    if (status) *status = it->second->status;
    return PM_OK;
}

int pm_server_wait(pm_server *s, uint64_t ticket, int32_t *status) {
    if (!s) return PM_EINVAL;
    std::unique_lock<std::mutex> lk(s->mu);
    auto it = s->reqs.find(ticket);
    if (it == s->reqs.end()) return PM_EINVAL;
    Request *r = it->second;
    s->cv_done.wait(lk, [&] { return r->done; });
    if (status) *status = r->status;
    return PM_OK;
}

int pm_server_latency(pm_server *s, uint64_t ticket, double *latency_us) {
    if (!s || !latency_us) return PM_EINVAL;
    std::lock_guard<std::mutex> lk(s->mu);
    auto it = s->reqs.find(ticket);
    if (it == s->reqs.end()) return PM_EINVAL;
    if (!it->second->done) return PM_EBUSY;
    *latency_us = it->second->latency;
    return PM_OK;
}

int64_t pm_server_latencies(pm_server *s, double *latency_us, int64_t cap) {
    if (!s) return 0;
    std::lock_guard<std::mutex> lk(s->mu);
    const int64_t n = (int64_t)s->latencies.size();
    if (latency_us)
        for (int64_t i = 0; i < std::min(n, cap); i++) latency_us[i] = s->latencies[i];
    return n;
}

void pm_server_destroy(pm_server *s) {
    if (!s) return;
    {
        std::lock_guard<std::mutex> lk(s->mu);
        s->stop = true;
        s->cv_submit.notify_all();
    }
    if (s->th.joinable()) s->th.join();
    for (auto st : s->streams) {
        (void)hipStreamSynchronize(st);
        (void)hipStreamDestroy(st);
    }
    if (s->plan_stream) (void)hipStreamDestroy(s->plan_stream);
    if (s->arena_ptr) (void)hipFree(s->arena_ptr);
    if (s->err_host) (void)hipHostFree(s->err_host);
    for (auto &kv : s->reqs) delete kv.second;
    delete s;
}

}  // extern "C"
