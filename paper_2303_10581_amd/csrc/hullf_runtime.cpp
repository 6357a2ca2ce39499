// Host runtime and C ABI (include/hullf.h): contexts, scratch memory,
// launch shapes, HIP-graph cache of the batched launch, the autotuner, event
// timing, and the synchronous convex_hull() driver.

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <vector>

#include "hull_host.h"
#include "hullf.h"
#include "hullf_internal.h"

using namespace hullf;

namespace {

constexpr int kKinds = 4;   // 0 reduce, 1 filter, 2 batched, 3 octagon set-up

struct GraphEntry {
    const void* pts;
    const void* off;
    uint32_t S;
    uint64_t n_total;
    void* surv;
    void* counts;
    Shape shape;
    hipGraph_t graph;
    hipGraphExec_t exec;
};

struct Timed {
    int kind;
    hipEvent_t a, b;
};

}  // namespace

struct hullf_ctx {
    int device = 0;
    int cus = 256;
    // one point set
    ReduceSlots* slots = nullptr;
    Octagon* oct = nullptr;
    unsigned long long* part = nullptr;   // 9 * kReduceMaxGrid
    uint64_t* status = nullptr;
    uint64_t status_cap = 0;
    uint64_t* count = nullptr;
    uint32_t* surv = nullptr;
    uint64_t surv_cap = 0;
    float2* gather = nullptr;
    uint64_t gather_cap = 0;
    uint32_t* h_surv = nullptr;
    float2* h_xy = nullptr;
    uint64_t h_cap = 0;
    uint64_t h_xy_cap = 0;
    uint64_t* h_count = nullptr;
    Octagon* h_oct = nullptr;
    Shape filter_shape{512, 16};
    // batched
    uint32_t b_sets_cap = 0;
    SetInfo* b_sets = nullptr;
    Octagon* b_octs = nullptr;
    BatchTotals* b_tot = nullptr;
    unsigned long long* b_part = nullptr;
    uint64_t b_part_cap = 0;   // records (9 words each)
    uint64_t* b_status = nullptr;
    uint64_t b_status_cap = 0;
    Shape batch_shape{256, 16};
    hipStream_t capture = nullptr;
    std::vector<GraphEntry> graphs;
    // timing
    bool timing = false;
    std::vector<Timed> pending;
    std::vector<hipEvent_t> pool;
    uint64_t launches[kKinds] = {0, 0, 0, 0};
    double total_ms[kKinds] = {0, 0, 0, 0};
};

namespace {

class DeviceGuard {
   public:
    explicit DeviceGuard(int dev) {
        if (hipGetDevice(&prev_) != hipSuccess) prev_ = -1;
        if (prev_ != dev) (void)hipSetDevice(dev);
    }
    ~DeviceGuard() {
        int cur = -1;
        if (prev_ >= 0 && hipGetDevice(&cur) == hipSuccess && cur != prev_) (void)hipSetDevice(prev_);
    }

   private:
    int prev_ = -1;
};

hullf_status map_err(hipError_t e) {
    if (e == hipSuccess) return HULLF_OK;
    if (e == hipErrorOutOfMemory) return HULLF_ENOMEM;
    return HULLF_EDEVICE;
}

#define CHECK_HIP(expr)                         \
    do {                                        \
        hipError_t e_ = (expr);                 \
        if (e_ != hipSuccess) return map_err(e_); \
    } while (0)

template <class T>
hipError_t grow_device(T** p, uint64_t* cap, uint64_t need, hipStream_t stream) {
    if (need <= *cap && *p) return hipSuccess;
    uint64_t want = std::max<uint64_t>(need + need / 4, 64);
    if (*p) {
        hipError_t e = hipStreamSynchronize(stream);
        if (e != hipSuccess) return e;
        (void)hipFree(*p);
        *p = nullptr;
        *cap = 0;
    }
    hipError_t e = hipMalloc((void**)p, want * sizeof(T));
    if (e != hipSuccess) {
        *p = nullptr;
        return e;
    }
    *cap = want;
    return hipSuccess;
}

template <class T>
hipError_t grow_host(T** p, uint64_t* cap, uint64_t need) {
    if (need <= *cap && *p) return hipSuccess;
    uint64_t want = std::max<uint64_t>(need + need / 4, 64);
    if (*p) (void)hipHostFree(*p);
    *p = nullptr;
    *cap = 0;
    hipError_t e = hipHostMalloc((void**)p, want * sizeof(T), hipHostMallocDefault);
    if (e != hipSuccess) {
        *p = nullptr;
        return e;
    }
    *cap = want;
    return hipSuccess;
}

hipEvent_t take_event(hullf_ctx* c) {
    if (!c->pool.empty()) {
        hipEvent_t e = c->pool.back();
        c->pool.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
}

template <class F>
hipError_t timed(hullf_ctx* c, int kind, hipStream_t s, F launch) {
    if (!c->timing) return launch();
    hipEvent_t a = take_event(c), b = take_event(c);
    if (!a || !b) return hipErrorOutOfMemory;
    hipError_t e = hipEventRecord(a, s);
    if (e != hipSuccess) return e;
    e = launch();
    if (e != hipSuccess) return e;
    e = hipEventRecord(b, s);
    if (e != hipSuccess) return e;
    c->pending.push_back({kind, a, b});
    return hipSuccess;
}

int reduce_grid(const hullf_ctx* c, uint64_t n) {
    const uint64_t ch = reduce_chunk_points();
    const uint64_t nch = (n + ch - 1) / ch;
    const uint64_t g = std::min<uint64_t>((uint64_t)c->cus * 8, (uint64_t)kReduceMaxGrid);
    return (int)std::max<uint64_t>(1, std::min<uint64_t>(nch, g));
}

bool aligned8(const void* p) { return ((uintptr_t)p & 7u) == 0u; }

void drop_graphs(hullf_ctx* c) {
    for (auto& g : c->graphs) {
        (void)hipGraphExecDestroy(g.exec);
        (void)hipGraphDestroy(g.graph);
    }
    c->graphs.clear();
}

// Enqueue reduce + filter for one set (n >= 1).
hullf_status enqueue_filter(hullf_ctx* c, const hullf_pt* d_pts, uint64_t n, uint32_t* d_surv,
                            uint64_t cap, uint64_t* d_count, hipStream_t s) {
    const float2* pts = reinterpret_cast<const float2*>(d_pts);
    const uint64_t T = filter_tile_points(c->filter_shape);
    const uint64_t tiles = (n + T - 1) / T;
    CHECK_HIP(grow_device(&c->status, &c->status_cap, tiles, s));
    const int rg = reduce_grid(c, n);
    CHECK_HIP(timed(c, 0, s, [&] {
        return launch_reduce(pts, n, c->slots, c->part, c->status, (uint32_t)tiles, rg, s);
    }));
    CHECK_HIP(timed(c, 3, s, [&] { return launch_setup(pts, n, c->oct, c->part, (uint32_t)rg, s); }));
    const int per_cu = c->filter_shape.block >= 512 ? 4 : 8;
    const int fg = (int)std::max<uint64_t>(1, std::min<uint64_t>(tiles, (uint64_t)c->cus * per_cu));
    CHECK_HIP(timed(c, 1, s, [&] {
        return launch_filter(pts, n, c->oct, c->slots, c->status, (uint32_t)tiles, d_surv, cap,
                             d_count, c->filter_shape, fg, s);
    }));
    return HULLF_OK;
}

hullf_status ensure_batch(hullf_ctx* c, uint32_t S, uint64_t n_total, Shape shape, hipStream_t s) {
    bool realloc = false;
    if (S > c->b_sets_cap) {
        CHECK_HIP(hipStreamSynchronize(s));
        (void)hipFree(c->b_sets);
        (void)hipFree(c->b_octs);
        c->b_sets = nullptr;
        c->b_octs = nullptr;
        c->b_sets_cap = 0;
        const uint32_t cap = std::max<uint32_t>(S, 64);
        CHECK_HIP(hipMalloc((void**)&c->b_sets, cap * sizeof(SetInfo)));
        CHECK_HIP(hipMalloc((void**)&c->b_octs, cap * sizeof(Octagon)));
        c->b_sets_cap = cap;
        realloc = true;
    }
    const uint64_t ftiles = batch_max_tiles(n_total, S, shape);
    const uint64_t rtiles = batch_max_rtiles(n_total, S);
    if (ftiles > 0xFFFFFFFFull || rtiles > 0xFFFFFFFFull) return HULLF_EINVAL;
    if (ftiles > c->b_status_cap || !c->b_status) {
        CHECK_HIP(grow_device(&c->b_status, &c->b_status_cap, ftiles, s));
        realloc = true;
    }
    if (rtiles > c->b_part_cap || !c->b_part) {
        uint64_t words = c->b_part_cap * 9;
        CHECK_HIP(grow_device(&c->b_part, &words, rtiles * 9, s));
        c->b_part_cap = words / 9;
        realloc = true;
    }
    if (realloc) drop_graphs(c);
    return HULLF_OK;
}

hullf_status enqueue_batched(hullf_ctx* c, const hullf_pt* d_pts, const uint64_t* d_off, uint32_t S,
                             uint64_t n_total, uint32_t* d_surv, uint64_t* d_counts, Shape shape,
                             hipStream_t s, bool seg = false) {
    const float2* pts = reinterpret_cast<const float2*>(d_pts);
    CHECK_HIP(launch_batch(pts, d_off, seg, S, n_total, c->b_sets, c->b_tot, c->b_part,
                           (uint32_t)std::min<uint64_t>(c->b_part_cap, 0xFFFFFFFFull), c->b_octs, c->b_status,
                           (uint32_t)std::min<uint64_t>(c->b_status_cap, 0xFFFFFFFFull), d_surv, d_counts,
                           shape, c->cus, s));
    return HULLF_OK;
}

hullf_status check_batch_args(hullf_ctx* c, const hullf_pt* d_pts, const uint64_t* d_off, uint32_t S,
                              uint64_t n_total, uint32_t* d_surv, uint64_t* d_counts) {
    if (!c) return HULLF_EINVAL;
    if (S == 0) return HULLF_OK;
    if (!d_off || !d_counts) return HULLF_EINVAL;
    if (n_total >= (1ull << 32)) return HULLF_EINVAL;
    if (n_total > 0 && (!d_pts || !d_surv || !aligned8(d_pts))) return HULLF_EINVAL;
    if (S > (1u << 30)) return HULLF_EINVAL;
    return HULLF_OK;
}

}  // namespace

extern "C" {

const char* hullf_status_str(hullf_status s) {
    switch (s) {
        case HULLF_OK: return "ok";
        case HULLF_EINVAL: return "invalid argument";
        case HULLF_ENONFINITE: return "non-finite input coordinate";
        case HULLF_ECAPACITY: return "output capacity too small";
        case HULLF_ENOMEM: return "out of memory";
        case HULLF_EDEVICE: return "HIP device error";
        case HULLF_EAGAIN: return "request not finished";
    }
    return "unknown status";
}

hullf_status hullf_create(int device, hullf_ctx_t* out) {
    if (!out) return HULLF_EINVAL;
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || device < 0 || device >= ndev) return HULLF_EINVAL;
    DeviceGuard g(device);
    hullf_ctx* c = new (std::nothrow) hullf_ctx();
    if (!c) return HULLF_ENOMEM;
    c->device = device;
    int cus = 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, device) == hipSuccess && cus > 0)
        c->cus = cus;
    if (const char* e = std::getenv("HULLF_FILTER_SHAPE")) {   // "block,ppt"
        Shape sh{0, 0};
        if (std::sscanf(e, "%d,%d", &sh.block, &sh.ppt) == 2 && shape_supported(sh)) c->filter_shape = sh;
    }
    hipError_t e = hipSuccess;
    if (e == hipSuccess) e = hipMalloc((void**)&c->slots, sizeof(ReduceSlots));
    if (e == hipSuccess) e = hipMalloc((void**)&c->oct, sizeof(Octagon));
    if (e == hipSuccess) e = hipMalloc((void**)&c->part, 9ull * kReduceMaxGrid * sizeof(unsigned long long));
    if (e == hipSuccess) e = hipMalloc((void**)&c->count, sizeof(uint64_t));
    if (e == hipSuccess) e = hipMalloc((void**)&c->b_tot, sizeof(BatchTotals));
    if (e == hipSuccess) e = hipHostMalloc((void**)&c->h_count, sizeof(uint64_t), hipHostMallocDefault);
    if (e == hipSuccess) e = hipHostMalloc((void**)&c->h_oct, sizeof(Octagon), hipHostMallocDefault);
    if (e == hipSuccess) e = hipStreamCreateWithFlags(&c->capture, hipStreamNonBlocking);
    if (e == hipSuccess) e = launch_init_slots(c->slots, 1, nullptr);
    if (e == hipSuccess) e = hipDeviceSynchronize();
    if (e != hipSuccess) {
        hullf_destroy(c);
        return map_err(e);
    }
    *out = c;
    return HULLF_OK;
}

void hullf_destroy(hullf_ctx_t c) {
    if (!c) return;
    DeviceGuard g(c->device);
    (void)hipDeviceSynchronize();
    drop_graphs(c);
    for (auto& t : c->pending) {
        (void)hipEventDestroy(t.a);
        (void)hipEventDestroy(t.b);
    }
    for (auto e : c->pool) (void)hipEventDestroy(e);
    void* dev[] = {c->slots, c->oct, c->part, c->status, c->count, c->surv, c->gather,
                   c->b_sets, c->b_octs, c->b_tot, c->b_part, c->b_status};
    for (void* p : dev)
        if (p) (void)hipFree(p);
    void* host[] = {c->h_surv, c->h_xy, c->h_count, c->h_oct};
    for (void* p : host)
        if (p) (void)hipHostFree(p);
    if (c->capture) (void)hipStreamDestroy(c->capture);
    delete c;
}

hullf_status hullf_octagon(hullf_ctx_t c, const hullf_pt* d_pts, uint64_t n, uint32_t idx_out[8],
                           void* stream) {
    if (!c || !d_pts || !idx_out || n == 0 || n >= (1ull << 32) || !aligned8(d_pts)) return HULLF_EINVAL;
    DeviceGuard g(c->device);
    hipStream_t s = (hipStream_t)stream;
    const float2* pts = reinterpret_cast<const float2*>(d_pts);
    const int rg = reduce_grid(c, n);
    CHECK_HIP(timed(c, 0, s, [&] { return launch_reduce(pts, n, c->slots, c->part, nullptr, 0, rg, s); }));
    CHECK_HIP(timed(c, 3, s, [&] { return launch_setup(pts, n, c->oct, c->part, (uint32_t)rg, s); }));
    CHECK_HIP(hipMemcpyAsync(c->h_oct, c->oct, sizeof(Octagon), hipMemcpyDeviceToHost, s));
    CHECK_HIP(hipStreamSynchronize(s));
    if (c->h_oct->status == 1) return HULLF_ENONFINITE;
    if (c->h_oct->status != 0) return HULLF_EDEVICE;
    std::memcpy(idx_out, c->h_oct->idx, 8 * sizeof(uint32_t));
    return HULLF_OK;
}

hullf_status hull_filter(hullf_ctx_t c, const hullf_pt* d_pts, uint64_t n, uint32_t* d_surv,
                         uint64_t cap, uint64_t* d_count, void* stream) {
    if (!c || !d_count || n >= (1ull << 32)) return HULLF_EINVAL;
    if (n > 0 && (!d_pts || !aligned8(d_pts) || (cap > 0 && !d_surv))) return HULLF_EINVAL;
    DeviceGuard g(c->device);
    hipStream_t s = (hipStream_t)stream;
    if (n == 0) {
        CHECK_HIP(launch_write_count(d_count, 0, s));
        return HULLF_OK;
    }
    return enqueue_filter(c, d_pts, n, d_surv, cap, d_count, s);
}

hullf_status hullf_flags(hullf_ctx_t c, const hullf_pt* d_pts, uint64_t n, uint8_t* d_flags, void* stream) {
    if (!c || n >= (1ull << 32)) return HULLF_EINVAL;
    if (n == 0) return HULLF_OK;
    if (!d_pts || !d_flags || !aligned8(d_pts)) return HULLF_EINVAL;
    DeviceGuard g(c->device);
    hipStream_t s = (hipStream_t)stream;
    const float2* pts = reinterpret_cast<const float2*>(d_pts);
    const int rg = reduce_grid(c, n);
    CHECK_HIP(launch_reduce(pts, n, c->slots, c->part, nullptr, 0, rg, s));
    CHECK_HIP(launch_setup(pts, n, c->oct, c->part, (uint32_t)rg, s));
    const int grid = (int)std::max<uint64_t>(1, std::min<uint64_t>((n + 255) / 256, (uint64_t)c->cus * 16));
    CHECK_HIP(launch_flags(pts, n, c->oct, d_flags, grid, s));
    return HULLF_OK;
}

hullf_status convex_hull(hullf_ctx_t c, const hullf_pt* d_pts, uint64_t n, uint32_t* h_hull,
                         uint64_t cap, uint64_t* h_count, void* stream) {
    if (!c || !h_count || n >= (1ull << 32)) return HULLF_EINVAL;
    if (n > 0 && (!d_pts || !aligned8(d_pts) || (cap > 0 && !h_hull))) return HULLF_EINVAL;
    *h_count = 0;
    if (n == 0) return HULLF_OK;
    DeviceGuard g(c->device);
    hipStream_t s = (hipStream_t)stream;
    CHECK_HIP(grow_device(&c->surv, &c->surv_cap, n, s));
    hullf_status st = enqueue_filter(c, d_pts, n, c->surv, n, c->count, s);
    if (st != HULLF_OK) return st;
    CHECK_HIP(hipMemcpyAsync(c->h_count, c->count, sizeof(uint64_t), hipMemcpyDeviceToHost, s));
    CHECK_HIP(hipStreamSynchronize(s));
    const uint64_t m = *c->h_count;
    if (m == kCountNonFinite) return HULLF_ENONFINITE;
    if (m > n) return HULLF_EDEVICE;
    CHECK_HIP(grow_device(&c->gather, &c->gather_cap, m, s));
    CHECK_HIP(grow_host(&c->h_surv, &c->h_cap, m));
    CHECK_HIP(grow_host(&c->h_xy, &c->h_xy_cap, m));
    const float2* pts = reinterpret_cast<const float2*>(d_pts);
    const int grid = (int)std::max<uint64_t>(1, std::min<uint64_t>((m + 255) / 256, (uint64_t)c->cus * 8));
    CHECK_HIP(launch_gather(pts, c->surv, c->count, m, n, c->gather, grid, s));
    CHECK_HIP(hipMemcpyAsync(c->h_surv, c->surv, m * sizeof(uint32_t), hipMemcpyDeviceToHost, s));
    CHECK_HIP(hipMemcpyAsync(c->h_xy, c->gather, m * sizeof(float2), hipMemcpyDeviceToHost, s));
    CHECK_HIP(hipStreamSynchronize(s));
    std::vector<HostPt> p(m);
    for (uint64_t k = 0; k < m; ++k) p[k] = HostPt{c->h_xy[k].x, c->h_xy[k].y, c->h_surv[k]};
    std::vector<uint32_t> out;
    monotone_chain(p, out);
    *h_count = out.size();
    if (out.size() > cap) return HULLF_ECAPACITY;
    std::copy(out.begin(), out.end(), h_hull);
    return HULLF_OK;
}

hullf_status hull_filter_batched_shape(hullf_ctx_t c, const hullf_pt* d_pts, const uint64_t* d_off,
                                       uint32_t S, uint64_t n_total, uint32_t* d_surv,
                                       uint64_t* d_counts, int block, int ppt, void* stream) {
    hullf_status st = check_batch_args(c, d_pts, d_off, S, n_total, d_surv, d_counts);
    if (st != HULLF_OK || S == 0) return st;
    Shape shape = c->batch_shape;
    if (block) shape.block = block;
    if (ppt) shape.ppt = ppt;
    if (!shape_supported(shape)) return HULLF_EINVAL;
    DeviceGuard g(c->device);
    hipStream_t s = (hipStream_t)stream;
    st = ensure_batch(c, S, n_total, shape, s);
    if (st != HULLF_OK) return st;
    hullf_status r = HULLF_OK;
    CHECK_HIP(timed(c, 2, s, [&] {
        r = enqueue_batched(c, d_pts, d_off, S, n_total, d_surv, d_counts, shape, s);
        return r == HULLF_OK ? hipSuccess : hipErrorLaunchFailure;
    }));
    return r;
}

hullf_status hull_filter_segments(hullf_ctx_t c, const hullf_pt* d_pts, const uint64_t* d_seg, uint32_t S,
                                  uint64_t n_total, uint32_t* d_surv, uint64_t* d_counts, void* stream) {
    hullf_status st = check_batch_args(c, d_pts, d_seg, S, n_total, d_surv, d_counts);
    if (st != HULLF_OK || S == 0) return st;
    DeviceGuard g(c->device);
    hipStream_t s = (hipStream_t)stream;
    const Shape shape = c->batch_shape;
    st = ensure_batch(c, S, n_total, shape, s);
    if (st != HULLF_OK) return st;
    hullf_status r = HULLF_OK;
    CHECK_HIP(timed(c, 2, s, [&] {
        r = enqueue_batched(c, d_pts, d_seg, S, n_total, d_surv, d_counts, shape, s, true);
        return r == HULLF_OK ? hipSuccess : hipErrorLaunchFailure;
    }));
    return r;
}

hullf_status hull_filter_batched(hullf_ctx_t c, const hullf_pt* d_pts, const uint64_t* d_off, uint32_t S,
                                 uint64_t n_total, uint32_t* d_surv, uint64_t* d_counts, void* stream) {
    hullf_status st = check_batch_args(c, d_pts, d_off, S, n_total, d_surv, d_counts);
    if (st != HULLF_OK || S == 0) return st;
    DeviceGuard g(c->device);
    hipStream_t s = (hipStream_t)stream;
    const Shape shape = c->batch_shape;
    st = ensure_batch(c, S, n_total, shape, s);
    if (st != HULLF_OK) return st;
    GraphEntry* hit = nullptr;
    for (auto& ge : c->graphs)
        if (ge.pts == d_pts && ge.off == d_off && ge.S == S && ge.n_total == n_total && ge.surv == d_surv &&
            ge.counts == d_counts && ge.shape.block == shape.block && ge.shape.ppt == shape.ppt)
            hit = &ge;
    if (!hit) {
        if (c->graphs.size() >= 16) drop_graphs(c);
        GraphEntry ge{d_pts, d_off, S, n_total, d_surv, d_counts, shape, nullptr, nullptr};
        CHECK_HIP(hipStreamBeginCapture(c->capture, hipStreamCaptureModeThreadLocal));
        hullf_status r = enqueue_batched(c, d_pts, d_off, S, n_total, d_surv, d_counts, shape, c->capture);
        hipError_t e = hipStreamEndCapture(c->capture, &ge.graph);
        if (r != HULLF_OK) {
            if (ge.graph) (void)hipGraphDestroy(ge.graph);
            return r;
        }
        CHECK_HIP(e);
        e = hipGraphInstantiate(&ge.exec, ge.graph, nullptr, nullptr, 0);
        if (e != hipSuccess) {
            (void)hipGraphDestroy(ge.graph);
            return map_err(e);
        }
        c->graphs.push_back(ge);
        hit = &c->graphs.back();
    }
    hipGraphExec_t exec = hit->exec;
    CHECK_HIP(timed(c, 2, s, [&] { return hipGraphLaunch(exec, s); }));
    return HULLF_OK;
}

hullf_status hullf_autotune_batched(hullf_ctx_t c, const hullf_pt* d_pts, const uint64_t* d_off,
                                    uint32_t S, uint64_t n_total, uint32_t* d_surv, uint64_t* d_counts,
                                    int reps, int* best_block, int* best_ppt, float* best_ms,
                                    void* stream) {
    hullf_status st = check_batch_args(c, d_pts, d_off, S, n_total, d_surv, d_counts);
    if (st != HULLF_OK) return st;
    if (S == 0 || reps < 1) return HULLF_EINVAL;
    DeviceGuard g(c->device);
    hipStream_t s = (hipStream_t)stream;
    const Shape shapes[] = {{256, 8}, {256, 16}, {256, 32}, {512, 8}, {512, 16}, {512, 32}};
    hipEvent_t a = nullptr, b = nullptr;
    CHECK_HIP(hipEventCreate(&a));
    if (hipEventCreate(&b) != hipSuccess) {
        (void)hipEventDestroy(a);
        return HULLF_EDEVICE;
    }
    Shape best{0, 0};
    float bms = 0.0f;
    hullf_status r = HULLF_OK;
    for (const Shape& sh : shapes) {
        r = ensure_batch(c, S, n_total, sh, s);
        if (r != HULLF_OK) break;
        r = enqueue_batched(c, d_pts, d_off, S, n_total, d_surv, d_counts, sh, s);   // warm-up
        if (r != HULLF_OK) break;
        if (hipEventRecord(a, s) != hipSuccess) { r = HULLF_EDEVICE; break; }
        for (int k = 0; k < reps && r == HULLF_OK; ++k)
            r = enqueue_batched(c, d_pts, d_off, S, n_total, d_surv, d_counts, sh, s);
        if (r != HULLF_OK) break;
        if (hipEventRecord(b, s) != hipSuccess || hipEventSynchronize(b) != hipSuccess) { r = HULLF_EDEVICE; break; }
        float ms = 0.0f;
        (void)hipEventElapsedTime(&ms, a, b);
        ms /= (float)reps;
        if (best.block == 0 || ms < bms) {
            best = sh;
            bms = ms;
        }
    }
    (void)hipEventDestroy(a);
    (void)hipEventDestroy(b);
    if (r != HULLF_OK) return r;
    c->batch_shape = best;
    drop_graphs(c);
    if (best_block) *best_block = best.block;
    if (best_ppt) *best_ppt = best.ppt;
    if (best_ms) *best_ms = bms;
    return HULLF_OK;
}

hullf_status hullf_timing_enable(hullf_ctx_t c, int enable) {
    if (!c) return HULLF_EINVAL;
    c->timing = enable != 0;
    return HULLF_OK;
}

hullf_status hullf_timing_read(hullf_ctx_t c, uint64_t* launches, double* total_ms) {
    if (!c || !launches || !total_ms) return HULLF_EINVAL;
    DeviceGuard g(c->device);
    for (auto& t : c->pending) {
        CHECK_HIP(hipEventSynchronize(t.b));
        float ms = 0.0f;
        CHECK_HIP(hipEventElapsedTime(&ms, t.a, t.b));
        c->launches[t.kind] += 1;
        c->total_ms[t.kind] += ms;
        c->pool.push_back(t.a);
        c->pool.push_back(t.b);
    }
    c->pending.clear();
    for (int k = 0; k < kKinds; ++k) {
        launches[k] = c->launches[k];
        total_ms[k] = c->total_ms[k];
        c->launches[k] = 0;
        c->total_ms[k] = 0.0;
    }
    return HULLF_OK;
}

}  // extern "C"
