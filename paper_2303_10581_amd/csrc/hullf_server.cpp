// Request loop of include/hullf_server.h: admission by device memory, copy
// stream, continuous batching over hull_filter_segments, host finishing.
//
// Threads and what each one owns:
//  - scheduler: admission (arena regions, slots), residency checks, batch
//    launches on the compute stream, batch completion;
//  - copiers (2 by default): host-to-device copies of admitted requests, each on
//    its own copy stream (direct from page-locked memory, else through its
//    pinned staging slots), so that several copies are in flight;
//  - finishers: survivor copies back (one stream each), arena release, and
//    the host monotone chain.
// Every request moves queue -> copy -> loading -> ready -> batch -> finish
// -> done; the lists live under one mutex.

#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <cstdlib>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <thread>
#include <unordered_map>
#include <vector>

#include "hull_host.h"
#include "hullf.h"
#include "hullf_server.h"

namespace {

using Clock = std::chrono::steady_clock;

constexpr uint64_t kGranule = 64;               // arena allocation unit (points): 512-byte aligned regions
constexpr uint64_t kStagePoints = 1ull << 20;   // pinned staging slot (8 MiB)
constexpr int kStageSlots = 4;                  // per copier
constexpr int kMaxCopiers = 4;                  // copier threads, each with its own copy stream
constexpr uint64_t kCountNonFinite = UINT64_MAX;

double us_between(Clock::time_point a, Clock::time_point b) {
    return std::chrono::duration<double, std::micro>(b - a).count();
}

// First-fit allocator of [0, cap) in granules, coalescing on release.
class Arena {
   public:
    explicit Arena(uint64_t cap) : cap_(cap) {
        if (cap) free_[0] = cap;
    }
    uint64_t alloc(uint64_t len) {
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second < len) continue;
            const uint64_t b = it->first, l = it->second;
            free_.erase(it);
            if (l > len) free_[b + len] = l - len;
            used_ += len;
            peak_ = std::max(peak_, used_);
            return b;
        }
        return UINT64_MAX;
    }
    void release(uint64_t b, uint64_t len) {
        used_ -= len;
        auto next = free_.lower_bound(b);
        if (next != free_.end() && b + len == next->first) {
            len += next->second;
            next = free_.erase(next);
        }
        if (next != free_.begin()) {
            auto prev = std::prev(next);
            if (prev->first + prev->second == b) {
                prev->second += len;
                return;
            }
        }
        free_[b] = len;
    }
    uint64_t peak() const { return peak_; }

   private:
    uint64_t cap_;
    uint64_t used_ = 0, peak_ = 0;
    std::map<uint64_t, uint64_t> free_;
};

struct Req {
    uint64_t id = 0;
    const hullf_pt* h = nullptr;
    uint64_t n = 0;
    bool pinned = false;
    Clock::time_point t0, t_adm, t_res, t_launch, t_filt, t_done;
    uint64_t begin = 0, span = 0;   // arena region (points)
    hipEvent_t loaded = nullptr;
    uint64_t count = 0;
    uint64_t batch = 0;
    uint32_t batch_n = 0;
    hullf_status status = HULLF_OK;
    bool done = false;
    std::vector<uint32_t> hull;
};

hullf_status map_err(hipError_t e) {
    if (e == hipSuccess) return HULLF_OK;
    if (e == hipErrorOutOfMemory) return HULLF_ENOMEM;
    return HULLF_EDEVICE;
}

}  // namespace

struct hullf_server {
    int device = 0;
    hullf_server_config cfg{};
    hullf_ctx_t ctx = nullptr;
    // device memory
    hullf_pt* d_pts = nullptr;
    uint32_t* d_surv = nullptr;
    uint64_t* d_seg = nullptr;
    uint64_t* d_counts = nullptr;
    // pinned host memory
    uint64_t* h_seg = nullptr;
    uint64_t* h_counts = nullptr;
    int copiers = 2;
    hullf_pt* stage[kMaxCopiers][kStageSlots] = {};
    hipEvent_t stage_ev[kMaxCopiers][kStageSlots] = {};
    // streams and events
    hipStream_t compute = nullptr, copy[kMaxCopiers] = {};
    hipEvent_t batch_ev = nullptr;
    std::vector<hipEvent_t> ev_pool;

    std::mutex mu;
    std::condition_variable cv_sched, cv_copy, cv_finish, cv_done;
    std::unique_ptr<Arena> arena;
    std::unordered_map<uint64_t, std::unique_ptr<Req>> reqs;
    std::deque<Req*> queue, copy_q, finish_q;
    std::vector<Req*> loading, ready, running;
    uint64_t next_id = 1;
    uint32_t inflight = 0;
    bool stop = false, stop_workers = false;
    Clock::time_point batch_t0;
    hullf_server_counters st{};

    std::thread sched_th, copy_th[kMaxCopiers];
    std::vector<std::thread> finish_th;
    std::vector<hullf_ctx_t> fctx;   // one context per finisher thread

    // -- scheduler ----------------------------------------------------------
    void admit_locked() {
        const auto now = Clock::now();
        while (!queue.empty() && inflight < cfg.max_inflight) {
            Req* r = queue.front();
            const uint64_t span = (r->n + kGranule - 1) / kGranule * kGranule;
            const uint64_t b = arena->alloc(span);
            if (b == UINT64_MAX) break;   // arrival order: wait for memory
            queue.pop_front();
            r->begin = b;
            r->span = span;
            r->t_adm = now;
            ++inflight;
            copy_q.push_back(r);
        }
        if (!copy_q.empty()) cv_copy.notify_all();
    }

    void fail_locked(Req* r, hullf_status s) {
        if (r->status == HULLF_OK) r->status = s;
        finish_q.push_back(r);
        cv_finish.notify_one();
    }

    void launch(std::vector<Req*>& batch) {
        std::sort(batch.begin(), batch.end(), [](const Req* a, const Req* b) { return a->begin < b->begin; });
        const uint32_t S = (uint32_t)batch.size();
        for (uint32_t k = 0; k < S; ++k) {
            h_seg[2 * k] = batch[k]->begin;
            h_seg[2 * k + 1] = batch[k]->n;
        }
        hipError_t e = hipMemcpyAsync(d_seg, h_seg, 16ull * S, hipMemcpyHostToDevice, compute);
        hullf_status s = map_err(e);
        if (s == HULLF_OK)
            s = hull_filter_segments(ctx, d_pts, d_seg, S, cfg.arena_points, d_surv, d_counts, compute);
        if (s == HULLF_OK)
            s = map_err(hipMemcpyAsync(h_counts, d_counts, 8ull * S, hipMemcpyDeviceToHost, compute));
        if (s == HULLF_OK) s = map_err(hipEventRecord(batch_ev, compute));
        std::lock_guard<std::mutex> lk(mu);
        const auto now = Clock::now();
        st.batches += 1;
        st.batched_requests += S;
        for (Req* r : batch) {
            r->t_launch = now;
            r->batch = st.batches;
            r->batch_n = S;
        }
        if (s != HULLF_OK) {
            for (Req* r : batch) fail_locked(r, s);
            batch.clear();
            return;
        }
        batch_t0 = now;
        running = std::move(batch);
        batch.clear();
    }

    void sched_loop() {
        (void)hipSetDevice(device);
        std::unique_lock<std::mutex> lk(mu);
        for (;;) {
            admit_locked();
            // residency
            for (size_t k = 0; k < loading.size();) {
                Req* r = loading[k];
                const hipError_t e = hipEventQuery(r->loaded);
                if (e == hipErrorNotReady) {
                    ++k;
                    continue;
                }
                loading[k] = loading.back();
                loading.pop_back();
                ev_pool.push_back(r->loaded);
                r->loaded = nullptr;
                r->t_res = Clock::now();
                if (e == hipSuccess) ready.push_back(r);
                else fail_locked(r, map_err(e));
            }
            // completion of the running batch
            if (!running.empty()) {
                const hipError_t e = hipEventQuery(batch_ev);
                if (e != hipErrorNotReady) {
                    const auto now = Clock::now();
                    st.batch_ms += us_between(batch_t0, now) * 1e-3;
                    for (size_t k = 0; k < running.size(); ++k) {
                        Req* r = running[k];
                        r->t_filt = now;
                        if (e != hipSuccess) r->status = map_err(e);
                        else r->count = h_counts[k];
                        finish_q.push_back(r);
                    }
                    running.clear();
                    cv_finish.notify_all();
                }
            }
            // next batch: every resident request
            if (running.empty() && !ready.empty()) {
                std::vector<Req*> batch;
                batch.swap(ready);
                lk.unlock();
                launch(batch);
                lk.lock();
                continue;
            }
            const bool busy = !running.empty() || !loading.empty();
            if (stop && queue.empty() && copy_q.empty() && !busy && ready.empty() && inflight == 0) break;
            if (busy) cv_sched.wait_for(lk, std::chrono::microseconds(50));
            else cv_sched.wait(lk);
        }
    }

    // -- copier -------------------------------------------------------------
    hipError_t upload(Req* r, uint64_t& slot, int id) {
        hullf_pt* dst = d_pts + r->begin;
        if (r->pinned)
            return hipMemcpyAsync(dst, r->h, r->n * sizeof(hullf_pt), hipMemcpyHostToDevice, copy[id]);
        for (uint64_t o = 0; o < r->n; o += kStagePoints) {
            const uint64_t m = std::min<uint64_t>(kStagePoints, r->n - o);
            const int k = (int)(slot++ % kStageSlots);
            hipError_t e = hipEventSynchronize(stage_ev[id][k]);
            if (e != hipSuccess) return e;
            std::memcpy(stage[id][k], r->h + o, m * sizeof(hullf_pt));
            e = hipMemcpyAsync(dst + o, stage[id][k], m * sizeof(hullf_pt), hipMemcpyHostToDevice, copy[id]);
            if (e != hipSuccess) return e;
            e = hipEventRecord(stage_ev[id][k], copy[id]);
            if (e != hipSuccess) return e;
        }
        return hipSuccess;
    }

    // Copier `id`: takes admitted requests in turn with the other copiers,
    // on its own stream, so that two host-to-device copies are in flight.
    void copy_loop(int id) {
        (void)hipSetDevice(device);
        uint64_t slot = 0;
        std::unique_lock<std::mutex> lk(mu);
        for (;;) {
            cv_copy.wait(lk, [&] { return stop_workers || !copy_q.empty(); });
            if (copy_q.empty()) break;
            Req* r = copy_q.front();
            copy_q.pop_front();
            hipEvent_t ev = nullptr;
            if (!ev_pool.empty()) {
                ev = ev_pool.back();
                ev_pool.pop_back();
            }
            lk.unlock();
            hipError_t e = hipSuccess;
            if (!ev) e = hipEventCreateWithFlags(&ev, hipEventDisableTiming);
            if (e == hipSuccess) e = upload(r, slot, id);
            if (e == hipSuccess) e = hipEventRecord(ev, copy[id]);
            lk.lock();
            if (e != hipSuccess) {
                if (ev) ev_pool.push_back(ev);
                r->t_res = Clock::now();
                fail_locked(r, map_err(e));
            } else {
                r->loaded = ev;
                loading.push_back(r);
            }
            cv_sched.notify_one();
        }
    }

    // -- finishers ----------------------------------------------------------
    void finish_loop(hullf_ctx_t fctx) {
        (void)hipSetDevice(device);
        hipStream_t fs = nullptr;
        hipError_t se = hipStreamCreateWithFlags(&fs, hipStreamNonBlocking);
        std::vector<uint32_t> hbuf(1u << 16);
        std::unique_lock<std::mutex> lk(mu);
        for (;;) {
            cv_finish.wait(lk, [&] { return stop_workers || !finish_q.empty(); });
            if (finish_q.empty()) break;
            Req* r = finish_q.front();
            finish_q.pop_front();
            lk.unlock();
            hullf_status s = r->status;
            uint64_t c = 0;
            if (s == HULLF_OK) {
                c = r->count;
                if (c == kCountNonFinite) s = HULLF_ENONFINITE;
                else if (c > r->n) s = HULLF_EDEVICE;
                else if (se != hipSuccess) s = map_err(se);
            }
            if (s == HULLF_OK && c > 0) {
                // hull of the resident survivors (device sort and chains for
                // large sets); the arena region is read until this returns
                uint64_t h = 0;
                s = hull_from_survivors(fctx, d_pts + r->begin, r->n, d_surv + r->begin, c, hbuf.data(),
                                        hbuf.size(), &h, fs);
                if (s == HULLF_ECAPACITY) {
                    hbuf.resize(h);
                    s = hull_from_survivors(fctx, d_pts + r->begin, r->n, d_surv + r->begin, c, hbuf.data(),
                                            hbuf.size(), &h, fs);
                }
                if (s == HULLF_OK) r->hull.assign(hbuf.begin(), hbuf.begin() + h);
            }
            lk.lock();
            if (r->span) {
                arena->release(r->begin, r->span);
                r->span = 0;
                --inflight;
                cv_sched.notify_one();
            }
            r->status = s;
            r->count = c;
            r->t_done = Clock::now();
            r->done = true;
            st.completed += 1;
            cv_done.notify_all();
        }
        lk.unlock();
        if (fs) (void)hipStreamDestroy(fs);
    }

    void release_all() {
        (void)hipSetDevice(device);
        if (compute) (void)hipStreamSynchronize(compute);
        for (hipStream_t q : copy)
            if (q) (void)hipStreamSynchronize(q);
        void* dev[] = {d_pts, d_surv, d_seg, d_counts};
        for (void* q : dev)
            if (q) (void)hipFree(q);
        if (h_seg) (void)hipHostFree(h_seg);
        if (h_counts) (void)hipHostFree(h_counts);
        for (int i = 0; i < kMaxCopiers; ++i)
            for (int k = 0; k < kStageSlots; ++k) {
                if (stage[i][k]) (void)hipHostFree(stage[i][k]);
                if (stage_ev[i][k]) (void)hipEventDestroy(stage_ev[i][k]);
            }
        for (hipEvent_t e : ev_pool) (void)hipEventDestroy(e);
        for (auto& kv : reqs)
            if (kv.second->loaded) (void)hipEventDestroy(kv.second->loaded);
        if (batch_ev) (void)hipEventDestroy(batch_ev);
        for (hullf_ctx_t f : fctx) hullf_destroy(f);
        if (compute) (void)hipStreamDestroy(compute);
        for (hipStream_t q : copy)
            if (q) (void)hipStreamDestroy(q);
        if (ctx) hullf_destroy(ctx);
    }
};

extern "C" {

hullf_status hullf_server_create(int device, const hullf_server_config* cfg, hullf_server_t* out) {
    if (!out) return HULLF_EINVAL;
    hullf_server_config c{};
    if (cfg) c = *cfg;
    if (c.arena_points == 0) c.arena_points = 1ull << 28;
    if (c.max_inflight == 0) c.max_inflight = 1024;
    if (c.finish_threads == 0) c.finish_threads = 4;
    c.arena_points = (c.arena_points + kGranule - 1) / kGranule * kGranule;
    if (c.arena_points >= (1ull << 32) || c.max_inflight > (1u << 20) || c.finish_threads > 256)
        return HULLF_EINVAL;
    hullf_server* s = new (std::nothrow) hullf_server();
    if (!s) return HULLF_ENOMEM;
    s->device = device;
    s->cfg = c;
    hullf_status r = hullf_create(device, 0, &s->ctx);
    if (r != HULLF_OK) {
        s->ctx = nullptr;
        delete s;
        return r;
    }
    (void)hipSetDevice(device);
    hipError_t e = hipSuccess;
    const uint64_t A = c.arena_points, M = c.max_inflight;
    if (e == hipSuccess) e = hipMalloc((void**)&s->d_pts, A * sizeof(hullf_pt));
    if (e == hipSuccess) e = hipMalloc((void**)&s->d_surv, A * sizeof(uint32_t));
    if (e == hipSuccess) e = hipMalloc((void**)&s->d_seg, 16ull * M);
    if (e == hipSuccess) e = hipMalloc((void**)&s->d_counts, 8ull * M);
    if (e == hipSuccess) e = hipHostMalloc((void**)&s->h_seg, 16ull * M, hipHostMallocDefault);
    if (e == hipSuccess) e = hipHostMalloc((void**)&s->h_counts, 8ull * M, hipHostMallocDefault);
    if (const char* v = std::getenv("HULLF_SERVER_COPIERS"))
        s->copiers = std::min(kMaxCopiers, std::max(1, std::atoi(v)));
    for (int i = 0; i < s->copiers; ++i)
        for (int k = 0; k < kStageSlots && e == hipSuccess; ++k) {
            e = hipHostMalloc((void**)&s->stage[i][k], kStagePoints * sizeof(hullf_pt), hipHostMallocDefault);
            if (e == hipSuccess) e = hipEventCreateWithFlags(&s->stage_ev[i][k], hipEventDisableTiming);
        }
    if (e == hipSuccess) e = hipStreamCreateWithFlags(&s->compute, hipStreamNonBlocking);
    for (int i = 0; i < s->copiers && e == hipSuccess; ++i)
        e = hipStreamCreateWithFlags(&s->copy[i], hipStreamNonBlocking);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&s->batch_ev, hipEventDisableTiming);
    // one launch over max_inflight empty segments sizes the batched scratch
    // for the largest batch, so serving allocates nothing later
    r = map_err(e);
    if (r == HULLF_OK) {
        std::memset(s->h_seg, 0, 16ull * M);
        r = map_err(hipMemcpyAsync(s->d_seg, s->h_seg, 16ull * M, hipMemcpyHostToDevice, s->compute));
    }
    if (r == HULLF_OK) r = hull_filter_segments(s->ctx, s->d_pts, s->d_seg, (uint32_t)M, A, s->d_surv,
                                                s->d_counts, s->compute);
    if (r == HULLF_OK) r = map_err(hipStreamSynchronize(s->compute));
    for (uint32_t k = 0; k < c.finish_threads && r == HULLF_OK; ++k) {
        hullf_ctx_t f = nullptr;
        r = hullf_create(device, 0, &f);
        if (r == HULLF_OK) s->fctx.push_back(f);
    }
    if (r != HULLF_OK) {
        s->release_all();
        delete s;
        return r;
    }
    s->arena.reset(new Arena(A));
    s->st.arena_points = A;
    s->sched_th = std::thread([s] { s->sched_loop(); });
    for (int i = 0; i < s->copiers; ++i) s->copy_th[i] = std::thread([s, i] { s->copy_loop(i); });
    for (uint32_t k = 0; k < c.finish_threads; ++k) {
        hullf_ctx_t f = s->fctx[k];
        s->finish_th.emplace_back([s, f] { s->finish_loop(f); });
    }
    *out = s;
    return HULLF_OK;
}

void hullf_server_destroy(hullf_server_t s) {
    if (!s) return;
    {
        std::lock_guard<std::mutex> lk(s->mu);
        s->stop = true;
    }
    s->cv_sched.notify_all();
    s->sched_th.join();
    {
        std::lock_guard<std::mutex> lk(s->mu);
        s->stop_workers = true;
    }
    s->cv_copy.notify_all();
    s->cv_finish.notify_all();
    for (std::thread& t : s->copy_th)
        if (t.joinable()) t.join();
    for (auto& t : s->finish_th) t.join();
    s->release_all();
    delete s;
}

hullf_status hullf_server_submit(hullf_server_t s, const hullf_pt* h_pts, uint64_t n, uint64_t* id) {
    if (!s || !id || n >= (1ull << 32) || (n > 0 && !h_pts)) return HULLF_EINVAL;
    if (n > s->cfg.arena_points) return HULLF_ENOMEM;
    std::unique_ptr<Req> r(new (std::nothrow) Req());
    if (!r) return HULLF_ENOMEM;
    r->h = h_pts;
    r->n = n;
    r->t0 = Clock::now();
    if (n > 0) {
        hipPointerAttribute_t a;
        if (hipPointerGetAttributes(&a, h_pts) == hipSuccess && a.type == hipMemoryTypeHost) r->pinned = true;
        else (void)hipGetLastError();
    }
    std::lock_guard<std::mutex> lk(s->mu);
    if (s->stop) return HULLF_EINVAL;
    r->id = s->next_id++;
    *id = r->id;
    s->st.submitted += 1;
    Req* q = r.get();
    s->reqs.emplace(q->id, std::move(r));
    if (n == 0) {
        q->t_adm = q->t_res = q->t_launch = q->t_filt = q->t_done = q->t0;
        q->done = true;
        s->st.completed += 1;
        s->cv_done.notify_all();
        return HULLF_OK;
    }
    s->queue.push_back(q);
    s->cv_sched.notify_one();
    return HULLF_OK;
}

hullf_status hullf_server_wait(hullf_server_t s, uint64_t id, int timeout_ms, uint32_t* h_hull, uint64_t cap,
                               uint64_t* h_count, hullf_request_info* info) {
    if (!s || !h_count || (cap > 0 && !h_hull)) return HULLF_EINVAL;
    std::unique_lock<std::mutex> lk(s->mu);
    auto it = s->reqs.find(id);
    if (it == s->reqs.end()) return HULLF_EINVAL;
    Req* r = it->second.get();
    if (timeout_ms < 0) s->cv_done.wait(lk, [&] { return r->done; });
    else if (timeout_ms > 0)
        s->cv_done.wait_for(lk, std::chrono::milliseconds(timeout_ms), [&] { return r->done; });
    if (!r->done) return HULLF_EAGAIN;
    if (info) {
        info->admitted_us = us_between(r->t0, r->t_adm);
        info->resident_us = us_between(r->t0, r->t_res);
        info->launched_us = us_between(r->t0, r->t_launch);
        info->filtered_us = us_between(r->t0, r->t_filt);
        info->done_us = us_between(r->t0, r->t_done);
        info->n = r->n;
        info->survivors = r->count;
        info->hull = r->hull.size();
        info->batch = r->batch;
        info->batch_requests = r->batch_n;
        info->status = (uint32_t)r->status;
    }
    const hullf_status st = r->status;
    *h_count = st == HULLF_OK ? r->hull.size() : 0;
    if (st == HULLF_OK && r->hull.size() > cap) return HULLF_ECAPACITY;
    if (st == HULLF_OK && !r->hull.empty()) std::memcpy(h_hull, r->hull.data(), r->hull.size() * sizeof(uint32_t));
    s->reqs.erase(it);
    return st;
}

hullf_status hullf_server_stats(hullf_server_t s, hullf_server_counters* out) {
    if (!s || !out) return HULLF_EINVAL;
    std::lock_guard<std::mutex> lk(s->mu);
    *out = s->st;
    out->arena_peak_points = s->arena->peak();
    out->inflight = s->inflight;
    out->queued = (uint32_t)s->queue.size();
    return HULLF_OK;
}

}  // extern "C"
