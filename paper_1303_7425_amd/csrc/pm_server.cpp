// Serving loop (continuous batching) of the sparse polynomial product; see
// pm_server_* in include/polymul.h.
//
// One scheduler thread per server.  Submitted requests wait in a FIFO queue.
// Each scheduling round takes the oldest requests that share a layout, plans
// them as one batch (one validation round trip), and admits the batch when
// its workspace fits the free part of the server's HBM arena; otherwise it
// halves the batch, and a single request that does not fit yet waits for
// earlier batches to complete (one that can never fit fails with PM_ENOMEM).
// Admitted batches are launched round-robin on the server's streams, so new
// work starts while earlier batches still run.  Completion is detected with
// events; the arena range is then returned and the tickets finish.
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

struct InFlight {
    std::vector<Request *> reqs;
    hipEvent_t ev = nullptr;
    int64_t off = 0, bytes = 0;
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

static void scheduler(pm_server *s) {
    (void)hipSetDevice(s->device);
    std::vector<hipEvent_t> free_events;
    while (true) {
        // 1. completions
        {
            std::vector<InFlight> still;
            for (auto &b : s->inflight) {
                if (hipEventQuery(b.ev) == hipSuccess) {
                    const double t = now_us();
                    std::lock_guard<std::mutex> lk(s->mu);
                    for (Request *r : b.reqs) finish(s, r, PM_OK, t);
                    s->arena.release(b.off, b.bytes);
                    free_events.push_back(b.ev);
                    s->cv_done.notify_all();
                } else {
                    still.push_back(b);
                }
            }
            s->inflight.swap(still);
        }
        // 2. take the oldest requests sharing the head's layout
        std::vector<Request *> group;
        {
            std::unique_lock<std::mutex> lk(s->mu);
            if (s->stop && s->pending.empty() && s->inflight.empty()) break;
            if (s->pending.empty() || (int)s->inflight.size() >= s->max_inflight) {
                if (s->inflight.empty()) {
                    s->cv_submit.wait_for(lk, std::chrono::milliseconds(1));
                } else {
                    lk.unlock();
                    std::this_thread::sleep_for(std::chrono::microseconds(20));
                }
                continue;
            }
            const pm_layout L0 = s->pending.front()->L;
            for (Request *r : s->pending) {
                if (r->L.nvars == L0.nvars && r->L.bits == L0.bits && r->L.ring == L0.ring) group.push_back(r);
                if ((int)group.size() >= s->max_batch) break;
            }
        }
        // 3. plan; halve the batch until its workspace fits the free arena
        int k = (int)group.size();
        bool launched = false;
        while (k >= 1 && !launched) {
            std::vector<pm_cpoly> f(k), g(k);
            std::vector<pm_poly> h(k);
            for (int i = 0; i < k; i++) {
                f[i] = group[i]->f;
                g[i] = group[i]->g;
                h[i] = group[i]->h;
            }
            int64_t need0 = (int64_t)(stats_region_bytes(k, (int)group[0]->L.nvars) + sizeof(DevSeg) * k);
            int64_t off0 = -1;
            {
                std::lock_guard<std::mutex> lk(s->mu);
                off0 = s->arena.alloc(need0);
            }
            if (off0 < 0) break;  // not even room to validate: wait for completions
            Plan P;
            void *dev0 = (char *)s->arena_ptr + off0;
            int rc = stats_and_plan(s->stage, &group[0]->L, k, f.data(), g.data(), dev0, s->plan_stream,
                                    default_tuning(), P);
            {
                std::lock_guard<std::mutex> lk(s->mu);
                s->arena.release(off0, need0);
            }
            if (rc != PM_OK) {
                if (k == 1) {
                    // this request is invalid (or can never be planned): fail it alone
                    std::lock_guard<std::mutex> lk(s->mu);
                    s->pending.erase(std::find(s->pending.begin(), s->pending.end(), group[0]));
                    finish(s, group[0], rc, now_us());
                    s->cv_done.notify_all();
                    launched = true;
                    break;
                }
                k /= 2;  // isolate the failing request
                continue;
            }
            // result arrays must hold each product's bound
            bool short_cap = false;
            {
                std::lock_guard<std::mutex> lk(s->mu);
                for (int i = 0; i < k; i++) {
                    if (group[i]->h.capacity < P.bound[i]) {
                        s->pending.erase(std::find(s->pending.begin(), s->pending.end(), group[i]));
                        finish(s, group[i], PM_ECAPACITY, now_us());
                        short_cap = true;
                    }
                }
                if (short_cap) s->cv_done.notify_all();
            }
            if (short_cap) {
                launched = true;  // regroup in the next round
                break;
            }
            int64_t off = -1;
            {
                std::lock_guard<std::mutex> lk(s->mu);
                if ((int64_t)P.total > s->arena.size) {
                    if (k == 1) {
                        s->pending.erase(std::find(s->pending.begin(), s->pending.end(), group[0]));
                        finish(s, group[0], PM_ENOMEM, now_us());
                        s->cv_done.notify_all();
                        launched = true;
                        break;
                    }
                } else {
                    off = s->arena.alloc((int64_t)P.total);
                }
            }
            if (off < 0) {
                if (k == 1) break;  // wait for memory
                k /= 2;
                continue;
            }
            // the statistics went to a scratch range; the plan's own workspace is `off`
            void *ws = (char *)s->arena_ptr + off;
            hipStream_t st = s->streams[s->next_stream];
            s->next_stream = (s->next_stream + 1) % (int)s->streams.size();
            rc = upload_and_launch(s->stage, P, h.data(), ws, st);
            hipEvent_t ev = nullptr;
            if (!free_events.empty()) {
                ev = free_events.back();
                free_events.pop_back();
            } else {
                (void)hipEventCreateWithFlags(&ev, hipEventDisableTiming);
            }
            if (rc == PM_OK && hipEventRecord(ev, st) != hipSuccess) rc = PM_EDEVICE;
            std::lock_guard<std::mutex> lk(s->mu);
            for (int i = 0; i < k; i++) s->pending.erase(std::find(s->pending.begin(), s->pending.end(), group[i]));
            if (rc != PM_OK) {
                const double t = now_us();
                for (int i = 0; i < k; i++) finish(s, group[i], rc, t);
                s->arena.release(off, (int64_t)P.total);
                free_events.push_back(ev);
                s->cv_done.notify_all();
            } else {
                InFlight b;
                b.reqs.assign(group.begin(), group.begin() + k);
                b.ev = ev;
                b.off = off;
                b.bytes = (int64_t)P.total;
                s->inflight.push_back(b);
            }
            launched = true;
        }
        if (!launched) std::this_thread::sleep_for(std::chrono::microseconds(20));
    }
    for (hipEvent_t e : free_events) (void)hipEventDestroy(e);
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
    for (auto &kv : s->reqs) delete kv.second;
    delete s;
}

}  // extern "C"
