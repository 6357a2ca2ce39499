// Host runtime and C ABI (include/hullf.h): contexts, scratch memory,
// launch shapes, HIP-graph cache of the batched launch, the autotuner, event
// timing, and the synchronous convex_hull() driver.

#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <string>
#include <sys/stat.h>
#include <unistd.h>
#include <thread>
#include <unordered_map>
#include <vector>

#include "hull_host.h"
#include "hullf.h"
#include "hullf_internal.h"

using namespace hullf;

namespace {

constexpr int kKinds = 5;   // 0 reduce, 1 inside test, 2 batched, 3 octagon set-up, 4 compaction
constexpr uint32_t kMaxBlocks = kFilterMaxBlocks;   // blocks of the two compaction passes

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
    // device workspace: every scratch buffer is counted against ws_cap
    // (0 = no cap); a request beyond it fails with HULLF_ENOMEM
    uint64_t ws_cap = 0;
    uint64_t ws_used = 0;
    std::unordered_map<void*, uint64_t> ws_sizes;
    // one point set
    Octagon* oct = nullptr;
    unsigned long long* part = nullptr;   // 9 * kReduceMaxGrid
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
    // the 16-direction filter (allocated on first use)
    Poly16* poly16 = nullptr;
    unsigned long long* part16 = nullptr;   // kPart16Words * kReduceMaxGrid
    Poly16* h_poly16 = nullptr;
    // hull finishing on the device (large survivor sets)
    // finishing keys and point indices: 0 sorted, 1 and 3 the two sides' run
    // representatives, then level outputs (side 0: 1 <-> 2, side 1: 3 <-> 0)
    uint64_t* fk[4] = {nullptr, nullptr, nullptr, nullptr};
    uint32_t* fv[4] = {nullptr, nullptr, nullptr, nullptr};
    uint32_t* fchain = nullptr;
    uint32_t* fcnt = nullptr;
    uint32_t* fblk = nullptr;
    uint32_t* bws = nullptr;               // batched finishing: split arrays and set digit prefixes
    uint64_t bws_cap = 0;
    uint32_t* fhist = nullptr;
    uint32_t* frow = nullptr;     // 256 row sums + 1 total
    uint64_t f_cap = 0;           // entries of fk/fv/fchain
    uint64_t fhist_cap = 0;
    uint64_t* h_fk = nullptr;
    uint32_t* h_fv = nullptr;
    uint64_t h_f_cap = 0;
    uint64_t h_fv_cap = 0;
    unsigned char* h_stage = nullptr;      // convex_hull: count + few survivors, written by the device
    uint64_t h_stage_cap = 0;
    uint64_t* h_bk[2] = {nullptr, nullptr};   // batched finishing: each side's chains
    uint32_t* h_bv[2] = {nullptr, nullptr};
    uint64_t h_bk_cap[2] = {0, 0};
    uint64_t h_bv_cap[2] = {0, 0};
    uint32_t* h_total = nullptr;
    Shape filter_shape{512, 16};
    bool host_finish = false;              // hull finishing always on the host
    uint32_t chain_chunk = 32;             // sorted points per chain thread (16..64)
    int classify_per_cu = 0;               // classify blocks per CU (0: what occupancy allows)
    int compact_block = 512;               // threads per compaction block
    int reduce_grid_max = 0;               // reduction blocks (0: 4 per CU)
    int batch_reduce_per_cu = 0;           // batched reduction blocks per CU (0: default)
    uint64_t* bits = nullptr;              // keep bits, 2 words per 128 points
    uint64_t bits_cap = 0;
    uint32_t* blkcnt = nullptr;            // kMaxBlocks survivor counts
    float4* boxes = nullptr;               // reduction boxes (region skip), 4 per 2048 points
    uint64_t boxes_cap = 0;
    unsigned long long* groups_read = nullptr;   // device counter of groups the inside test read
    unsigned long long* lb = nullptr;            // single-pass filter: ticket + tile status words
    uint64_t lb_cap = 0;
    bool single_pass = false;                    // hull_filter in one pass (decoupled look-back)
    uint64_t groups_total = 0;                   // groups it would read without the skip
    bool region_skip = true;
    // batched
    uint32_t b_sets_cap = 0;
    SetInfo* b_sets = nullptr;
    Octagon* b_octs = nullptr;
    BatchTotals* b_tot = nullptr;
    unsigned long long* b_part = nullptr;
    uint64_t b_part_cap = 0;   // records (9 words each)
    float4* b_boxes = nullptr;   // region-skip boxes, batch_tile_boxes() per record
    uint64_t b_boxes_cap = 0;
    uint64_t* b_bits = nullptr;            // two-pass: keep bits per work item
    uint32_t* b_blkcnt = nullptr;          // two-pass: survivors per work item
    uint64_t b_items_cap = 0;
    Shape batch_shape{256, 16};
    // Tune cache of the batched launch: the autotuner's choice per
    // (architecture, CU count, set-count class, mean-set-size class), kept
    // in a text file across processes (empty path: not persisted).
    std::string arch;
    std::string tune_path;
    std::map<std::string, Shape> tune;
    hipStream_t capture = nullptr;
    std::vector<GraphEntry> graphs;
    // timing
    uint32_t timing = 0;   // bit k: kernels of kind k are timed
    std::vector<Timed> pending;
    std::vector<hipEvent_t> pool;
    uint64_t launches[kKinds] = {0, 0, 0, 0, 0};
    double total_ms[kKinds] = {0, 0, 0, 0, 0};
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

// Device scratch of a context, counted against its workspace cap.  Over the
// cap the allocation is refused with hipErrorOutOfMemory (HULLF_ENOMEM).
hipError_t ws_alloc(hullf_ctx* c, void** p, uint64_t bytes) {
    *p = nullptr;
    if (c->ws_cap != 0 && c->ws_used + bytes > c->ws_cap) return hipErrorOutOfMemory;
    hipError_t e = hipMalloc(p, bytes);
    if (e != hipSuccess) {
        *p = nullptr;
        return e;
    }
    c->ws_sizes[*p] = bytes;
    c->ws_used += bytes;
    return hipSuccess;
}

template <class T>
hipError_t ws_alloc(hullf_ctx* c, T** p, uint64_t count) {
    return ws_alloc(c, reinterpret_cast<void**>(p), count * sizeof(T));
}

void ws_free(hullf_ctx* c, void* p) {
    if (!p) return;
    auto it = c->ws_sizes.find(p);
    if (it != c->ws_sizes.end()) {
        c->ws_used -= it->second;
        c->ws_sizes.erase(it);
    }
    (void)hipFree(p);
}

// Grow a device buffer to at least `need` elements (with a quarter of slack
// when the workspace cap leaves room for it).
template <class T>
hipError_t grow_device(hullf_ctx* c, T** p, uint64_t* cap, uint64_t need, hipStream_t stream) {
    if (need <= *cap && *p) return hipSuccess;
    uint64_t want = std::max<uint64_t>(need + need / 4, 64);
    if (*p) {
        hipError_t e = hipStreamSynchronize(stream);
        if (e != hipSuccess) return e;
        ws_free(c, *p);
        *p = nullptr;
        *cap = 0;
    }
    if (c->ws_cap != 0) {
        const uint64_t room = c->ws_cap > c->ws_used ? (c->ws_cap - c->ws_used) / sizeof(T) : 0;
        want = std::max<uint64_t>(need, std::min<uint64_t>(want, room));
    }
    hipError_t e = ws_alloc(c, p, want);
    if (e != hipSuccess) return e;
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
    // Timestamps only: without the system-scope fence an event record does
    // not write back and invalidate the caches between the kernels it
    // brackets (with it, each record adds a cache flush to the timed work).
    hipEvent_t e = nullptr;
    if (hipEventCreateWithFlags(&e, hipEventDisableSystemFence) != hipSuccess) return nullptr;
    return e;
}

template <class F>
hipError_t timed(hullf_ctx* c, int kind, hipStream_t s, F launch) {
    if (!((c->timing >> kind) & 1u)) return launch();
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
    return plan_filter(n, c->cus, c->filter_shape, c->classify_per_cu, c->reduce_grid_max).reduce_grid;
}

bool aligned8(const void* p) { return ((uintptr_t)p & 7u) == 0u; }

void drop_graphs(hullf_ctx* c) {
    for (auto& g : c->graphs) {
        (void)hipGraphExecDestroy(g.exec);
        (void)hipGraphDestroy(g.graph);
    }
    c->graphs.clear();
}

// Enqueue reduce + set-up + inside test and compaction for one set (n >= 1).
hullf_status enqueue_filter(hullf_ctx* c, const hullf_pt* d_pts, uint64_t n, uint32_t* d_surv,
                            uint64_t cap, uint64_t* d_count, hipStream_t s) {
    const float2* pts = reinterpret_cast<const float2*>(d_pts);
    const FilterPlan p = plan_filter(n, c->cus, c->filter_shape, c->classify_per_cu, c->reduce_grid_max);
    CHECK_HIP(grow_device(c, &c->bits, &c->bits_cap, p.bits_words, s));
    float4* box = nullptr;
    uint64_t nbox = 0;
    if (c->region_skip) {
        nbox = p.boxes;
        CHECK_HIP(grow_device(c, &c->boxes, &c->boxes_cap, nbox, s));
        box = c->boxes;
    }
    const int rg = p.reduce_grid;
    if (c->single_pass) {
        // inside test and compaction in one launch; the reduction clears
        // its ticket and status words
        const uint32_t tiles = filter1p_tiles(n);
        CHECK_HIP(grow_device(c, &c->lb, &c->lb_cap, (uint64_t)tiles + 1, s));
        CHECK_HIP(timed(c, 0, s, [&] { return launch_reduce(pts, n, c->part, box, rg, s, c->lb, tiles + 1); }));
        CHECK_HIP(timed(c, 3, s, [&] { return launch_setup(pts, n, c->oct, c->part, (uint32_t)rg, s); }));
        CHECK_HIP(timed(c, 1, s, [&] {
            return launch_filter1p(pts, n, c->oct, box, nbox, c->lb, d_surv, cap, d_count, c->groups_read, s);
        }));
        c->groups_total += (n + 127) / 128;
        return HULLF_OK;
    }
    CHECK_HIP(timed(c, 0, s, [&] { return launch_reduce(pts, n, c->part, box, rg, s); }));
    CHECK_HIP(timed(c, 3, s, [&] { return launch_setup(pts, n, c->oct, c->part, (uint32_t)rg, s); }));
    CHECK_HIP(timed(c, 1, s, [&] {
        return launch_classify(pts, n, c->oct, p.spans, c->bits, c->blkcnt, box, nbox, c->groups_read, p.shape,
                               p.grid, s);
    }));
    c->groups_total += (n + 127) / 128;
    CHECK_HIP(timed(c, 4, s, [&] {
        return launch_compact(c->bits, c->blkcnt, n, p.spans, c->oct, d_surv, cap, d_count, c->compact_block,
                              p.grid, s);
    }));
    return HULLF_OK;
}

hipError_t ensure_poly16(hullf_ctx* c) {
    hipError_t e = hipSuccess;
    if (!c->poly16 && (e = ws_alloc(c, &c->poly16, 1)) != hipSuccess) return e;
    if (!c->part16 && (e = ws_alloc(c, &c->part16, (uint64_t)kPart16Words * kReduceMaxGrid)) != hipSuccess) return e;
    if (!c->h_poly16 && (e = hipHostMalloc((void**)&c->h_poly16, sizeof(Poly16), hipHostMallocDefault)) != hipSuccess)
        return e;
    return hipSuccess;
}

// Enqueue the 16-direction filter for one set (n >= 1): reduction of the 16
// keys, the polygon set-up, then the octagon filter's inside-test and
// compaction launches over the polygon's edges.
hullf_status enqueue_filter16(hullf_ctx* c, const hullf_pt* d_pts, uint64_t n, uint32_t* d_surv, uint64_t cap,
                              uint64_t* d_count, hipStream_t s) {
    const float2* pts = reinterpret_cast<const float2*>(d_pts);
    CHECK_HIP(ensure_poly16(c));
    const FilterPlan p = plan_filter(n, c->cus, c->filter_shape, c->classify_per_cu, c->reduce_grid_max);
    CHECK_HIP(grow_device(c, &c->bits, &c->bits_cap, p.bits_words, s));
    float4* box = nullptr;
    uint64_t nbox = 0;
    if (c->region_skip) {
        nbox = p.boxes;
        CHECK_HIP(grow_device(c, &c->boxes, &c->boxes_cap, nbox, s));
        box = c->boxes;
    }
    const int rg = reduce16_grid(n, c->cus);
    CHECK_HIP(timed(c, 0, s, [&] { return launch_reduce16(pts, n, c->part16, box, rg, s); }));
    CHECK_HIP(timed(c, 3, s, [&] { return launch_setup16(pts, n, c->poly16, c->part16, (uint32_t)rg, s); }));
    CHECK_HIP(timed(c, 1, s, [&] {
        return launch_classify(pts, n, c->poly16, p.spans, c->bits, c->blkcnt, box, nbox, c->groups_read, p.shape,
                               p.grid, s);
    }));
    c->groups_total += (n + 127) / 128;
    CHECK_HIP(timed(c, 4, s, [&] {
        return launch_compact(c->bits, c->blkcnt, n, p.spans, c->poly16, d_surv, cap, d_count, c->compact_block,
                              p.grid, s);
    }));
    return HULLF_OK;
}

constexpr uint32_t kChainChunkMin = 16;        // least sorted points per chain thread
constexpr uint32_t kChainMaxChunk = 64;        // most sorted points per chain thread
constexpr uint32_t kRsTileItems = 4096;        // items per radix-sort tile
constexpr uint64_t kDeviceFinishMin = 1u << 14;   // survivors from which the device sorts and chains
constexpr uint64_t kEagerHull = 4096;             // survivors convex_hull stages before it knows the count
constexpr uint32_t kLevelStop = 1u << 16;         // chunk levels stop at this many candidates

hipError_t ensure_finish(hullf_ctx* c, uint64_t m, hipStream_t s) {
    if (m > c->f_cap) {
        hipError_t e = hipStreamSynchronize(s);
        if (e != hipSuccess) return e;
        for (int k = 0; k < 4; ++k) {
            ws_free(c, c->fk[k]);
            ws_free(c, c->fv[k]);
            c->fk[k] = nullptr;
            c->fv[k] = nullptr;
        }
        ws_free(c, c->fchain);
        ws_free(c, c->fcnt);
        ws_free(c, c->fblk);
        c->fchain = nullptr;
        c->fcnt = nullptr;
        c->fblk = nullptr;
        c->f_cap = 0;
        const uint64_t cap = m + m / 8 + 1024;
        for (int k = 0; k < 4; ++k) {
            if ((e = ws_alloc(c, &c->fk[k], cap)) != hipSuccess) return e;
            if ((e = ws_alloc(c, &c->fv[k], cap)) != hipSuccess) return e;
        }
        if ((e = ws_alloc(c, &c->fchain, cap)) != hipSuccess) return e;
        // chunk counts / merge offsets, then the run pass's tile counts
        if ((e = ws_alloc(c, &c->fcnt, cap / kChainChunkMin + 2 + cap / kRunTile + 2)) != hipSuccess) return e;
        if ((e = ws_alloc(c, &c->fblk, (cap / kChainChunkMin + 2) / 4096 + 2)) != hipSuccess) return e;
        c->f_cap = cap;
    }
    const uint64_t hw = 256ull * finish_sort_tiles((uint32_t)m);
    hipError_t e = grow_device(c, &c->fhist, &c->fhist_cap, hw, s);
    if (e != hipSuccess) return e;
    // frow: 256 row sums, [256] a total, [258..259] the bad-index flag (uint64)
    if (!c->frow && (e = ws_alloc(c, &c->frow, 260)) != hipSuccess) return e;
    if (!c->h_total && (e = hipHostMalloc((void**)&c->h_total, sizeof(uint32_t), hipHostMallocDefault)) != hipSuccess)
        return e;
    return hipSuccess;
}

inline float unord_host(uint32_t k) {
    const uint32_t u = (k & 0x80000000u) ? (k & 0x7FFFFFFFu) : ~k;
    float f;
    std::memcpy(&f, &u, sizeof f);
    return f;
}

// Sort the m survivors on the device, reduce them by chunked monotone
// chains, merge the chunk chains on the device (merge tree) into the lower
// and the upper hull chain, and copy back only those two chains; the host
// joins them.
hullf_status finish_on_device(hullf_ctx* c, const float2* pts, uint64_t n, const uint32_t* d_surv, uint64_t m,
                              std::vector<uint32_t>& out, hipStream_t s) {
    CHECK_HIP(ensure_finish(c, m, s));
    const uint32_t mm = (uint32_t)m;
    const int grid = (int)std::max<uint64_t>(1, std::min<uint64_t>((m + 255) / 256, (uint64_t)c->cus * 8));
    uint64_t* bad = reinterpret_cast<uint64_t*>(c->frow + 258);
    CHECK_HIP(launch_write_count(bad, 0, s));
    CHECK_HIP(launch_finish_keys(pts, n, d_surv, mm, c->fk[0], c->fv[0], bad, grid, s));
    CHECK_HIP(hipMemcpyAsync(c->h_count, bad, sizeof(uint64_t), hipMemcpyDeviceToHost, s));
    CHECK_HIP(hipStreamSynchronize(s));
    if (*c->h_count != 0) return HULLF_EINVAL;
    // sort by x alone (four passes over the key's high half, stable)
    CHECK_HIP(launch_finish_sort(c->fk[0], c->fv[0], c->fk[1], c->fv[1], mm, c->fhist, c->frow, 32, s));
    std::vector<HostPt> lists[2];
    uint32_t* const off_b = c->fchain + c->f_cap / 2;   // second offset array of the merge rounds
    uint2* const br = reinterpret_cast<uint2*>(c->fchain);
    // each side's representative of every run of equal x, in order
    // (distinct points, sorted by (x, y)), per tile of the run pass: lower
    // side into buffer 1, upper into 3; the first chunk level reads them
    // through the scanned tile counts
    uint32_t* const tcnt = c->fcnt + c->f_cap / kChainChunkMin + 2;
    const uint32_t ntiles = (mm + kRunTile - 1) / kRunTile;
    CHECK_HIP(launch_runs(c->fk[0], c->fv[0], mm, c->fk[1], c->fv[1], c->fk[3], c->fv[3], tcnt, s));
    CHECK_HIP(launch_scan_counts(tcnt, ntiles, c->frow + 256, c->fblk, s));
    CHECK_HIP(hipMemcpyAsync(c->h_total, c->frow + 256, sizeof(uint32_t), hipMemcpyDeviceToHost, s));
    CHECK_HIP(hipStreamSynchronize(s));
    const uint32_t reps = *c->h_total;
    if (reps == 0 || reps > mm) return HULLF_EDEVICE;
    for (int side = 0; side < 2; ++side) {
        const int sign = side == 0 ? 1 : -1;
        const int ba = side == 0 ? 1 : 3, bb = side == 0 ? 2 : 0;   // the side's two buffers
        const uint32_t* toff = tcnt;
        int cur = ba;
        uint32_t cm = reps, nc = 0;
        // chunk levels while they shrink the set well
        for (;;) {
            const int nxt = (cur == ba) ? bb : ba;
            const uint32_t C = c->chain_chunk;
            const uint32_t nch = (cm + C - 1) / C;
            CHECK_HIP(launch_chain(c->fk[cur], cm, C, sign, toff, toff ? ntiles : 0u, c->fchain, c->fcnt, s));
            CHECK_HIP(launch_scan_counts(c->fcnt, nch, c->frow + 256, c->fblk, s));
            CHECK_HIP(hipMemcpyAsync(c->h_total, c->frow + 256, sizeof(uint32_t), hipMemcpyDeviceToHost, s));
            CHECK_HIP(hipStreamSynchronize(s));
            const uint32_t tot = *c->h_total;
            if (tot > cm) return HULLF_EDEVICE;
            const int gg = (int)std::max<uint64_t>(
                1, std::min<uint64_t>(((uint64_t)nch * C + 255) / 256, (uint64_t)c->cus * 16));
            CHECK_HIP(launch_chain_gather(c->fk[cur], c->fv[cur], nch, C, c->fchain, c->fcnt, tot,
                                          c->fk[nxt], c->fv[nxt], gg, s));
            const bool slow = (uint64_t)tot * 4 > (uint64_t)cm * 3;   // little left to gain
            cur = nxt;
            cm = tot;
            nc = nch;
            toff = nullptr;
            if (slow || cm <= kLevelStop) break;
        }
        // merge tree: the chunk chains of the last level, pairwise, until
        // one chain (the side's hull) is left; no host round trip between
        // rounds
        CHECK_HIP(launch_copy_u32(c->fcnt + nc, c->frow + 256, s));   // off[nc] = total
        uint32_t* off_in = c->fcnt;
        uint32_t* off_out = off_b;
        while (nc > 1) {
            const uint32_t np = (nc + 1) / 2;
            const int nxt = (cur == ba) ? bb : ba;
            const int gg = (int)std::max<uint32_t>(1, std::min<uint32_t>((np + 3) / 4, (uint32_t)c->cus * 8));
            CHECK_HIP(launch_bridge(c->fk[cur], off_in, nc, sign, br, off_out, gg, s));
            CHECK_HIP(launch_scan_counts(off_out, np, off_out + np, c->fblk, s));
            CHECK_HIP(launch_merge_gather(c->fk[cur], c->fv[cur], off_in, nc, br, off_out, c->fk[nxt], c->fv[nxt],
                                          c->cus * 4, s));
            std::swap(off_in, off_out);
            cur = nxt;
            nc = np;
        }
        CHECK_HIP(hipMemcpyAsync(c->h_total, off_in + 1, sizeof(uint32_t), hipMemcpyDeviceToHost, s));
        CHECK_HIP(hipStreamSynchronize(s));
        cm = *c->h_total;
        if (cm > mm) return HULLF_EDEVICE;
        CHECK_HIP(grow_host(&c->h_fk, &c->h_f_cap, cm));
        CHECK_HIP(grow_host(&c->h_fv, &c->h_fv_cap, cm));
        CHECK_HIP(hipMemcpyAsync(c->h_fk, c->fk[cur], (uint64_t)cm * sizeof(uint64_t), hipMemcpyDeviceToHost, s));
        CHECK_HIP(hipMemcpyAsync(c->h_fv, c->fv[cur], (uint64_t)cm * sizeof(uint32_t), hipMemcpyDeviceToHost, s));
        CHECK_HIP(hipStreamSynchronize(s));
        std::vector<HostPt>& L = lists[side];
        L.resize(cm);
        for (uint32_t k = 0; k < cm; ++k)
            L[k] = HostPt{unord_host((uint32_t)(c->h_fk[k] >> 32)), unord_host((uint32_t)c->h_fk[k]), c->h_fv[k]};
    }
    // the two chain ends the run representatives leave out: the greatest
    // point (the upper chain's last) ends the lower chain, the smallest (the
    // lower chain's first) starts the upper one
    if (lists[0].empty() || lists[1].empty()) return HULLF_EDEVICE;
    lists[0].push_back(lists[1].back());
    lists[1].insert(lists[1].begin(), lists[0].front());
    chain_sorted(lists[0], lists[1], out);
    return HULLF_OK;
}

// Hulls of every set of a batch from its survivors (hull_filter_batched's
// layout: set s = pts[off[s] .. off[s+1]), its counts[s] survivors as
// set-local indices at surv + off[s]), all sets at once: one sort in which
// every set is sorted on its own (tiles never cross a set), then the run
// pass, chunk levels and merge rounds of finish_on_device over splits of
// every set (pieces never cross a set; each kernel finds a piece's set by
// binary search in S + 1 words).  hull: the sets' hulls one after another
// (set-local indices), hoff: S + 1 offsets into it.
hullf_status finish_batch(hullf_ctx* c, const float2* pts, const uint64_t* d_off, uint32_t S, uint64_t n_total,
                          const uint32_t* d_surv, const uint64_t* d_counts, uint32_t* h_hull, uint64_t cap,
                          uint64_t* hoff, hipStream_t s) {
    std::fill(hoff, hoff + (size_t)S + 1, 0ull);
    std::vector<uint64_t> off((size_t)S + 1), cnt(S);
    CHECK_HIP(hipMemcpyAsync(off.data(), d_off, off.size() * sizeof(uint64_t), hipMemcpyDeviceToHost, s));
    CHECK_HIP(hipMemcpyAsync(cnt.data(), d_counts, cnt.size() * sizeof(uint64_t), hipMemcpyDeviceToHost, s));
    CHECK_HIP(hipStreamSynchronize(s));
    if (off[0] != 0 || off[S] > n_total) return HULLF_EINVAL;
    const uint32_t S1 = S + 1;
    std::vector<uint32_t> ipos(S1), sft(S1), rft(S1);
    uint64_t M = 0, T1 = 0, NRT = 0;
    for (uint32_t k = 0; k < S; ++k) {
        if (off[k + 1] < off[k]) return HULLF_EINVAL;
        if (cnt[k] == kCountNonFinite) return HULLF_ENONFINITE;
        if (cnt[k] > off[k + 1] - off[k]) return HULLF_EINVAL;   // also the other error codes
        ipos[k] = (uint32_t)M;
        sft[k] = (uint32_t)T1;
        rft[k] = (uint32_t)NRT;
        M += cnt[k];
        T1 += (cnt[k] + kRsTileItems - 1) / kRsTileItems;
        NRT += (cnt[k] + kRunTile - 1) / kRunTile;
    }
    ipos[S] = (uint32_t)M;
    sft[S] = (uint32_t)T1;
    rft[S] = (uint32_t)NRT;
    if (M == 0) return HULLF_OK;
    const uint64_t need = std::max<uint64_t>(M + (uint64_t)S * kChainMaxChunk, NRT * kRunTile);
    if (need + need / 8 + 4096 >= (1ull << 32)) return HULLF_EINVAL;
    CHECK_HIP(ensure_finish(c, need, s));
    CHECK_HIP(grow_device(c, &c->fhist, &c->fhist_cap, 256ull * std::max<uint64_t>(T1, 1), s));
    // split arrays: ipos, sft, rft, level ranges, level first chunks, take
    // indices, take results, set digit prefixes, then the merge rounds'
    // (first, start) pairs
    constexpr uint32_t kMaxRounds = 34;
    const uint64_t words = 7ull * S1 + 256ull * S + 2ull * kMaxRounds * S1;
    CHECK_HIP(grow_device(c, &c->bws, &c->bws_cap, words, s));
    uint32_t* const d_ipos = c->bws;
    uint32_t* const d_sft = d_ipos + S1;
    uint32_t* const d_rft = d_sft + S1;
    uint32_t* const d_rng = d_rft + S1;
    uint32_t* const d_fcs = d_rng + S1;
    uint32_t* const d_tix = d_fcs + S1;
    uint32_t* const d_tout = d_tix + S1;
    uint32_t* const d_sdp = d_tout + S1;
    uint32_t* const d_rounds = d_sdp + 256ull * S;
    CHECK_HIP(hipMemcpyAsync(d_ipos, ipos.data(), S1 * sizeof(uint32_t), hipMemcpyHostToDevice, s));
    CHECK_HIP(hipMemcpyAsync(d_sft, sft.data(), S1 * sizeof(uint32_t), hipMemcpyHostToDevice, s));
    CHECK_HIP(hipMemcpyAsync(d_rft, rft.data(), S1 * sizeof(uint32_t), hipMemcpyHostToDevice, s));
    const uint32_t mm = (uint32_t)M;
    uint64_t* bad = reinterpret_cast<uint64_t*>(c->frow + 258);
    CHECK_HIP(launch_write_count(bad, 0, s));
    const SetSplit sp_sort{d_sft, d_ipos, S, kRsTileItems};
    CHECK_HIP(launch_bfin_keys(pts, d_off, d_surv, sp_sort, (uint32_t)T1, c->fk[0], c->fv[0], bad, s));
    CHECK_HIP(hipMemcpyAsync(c->h_count, bad, sizeof(uint64_t), hipMemcpyDeviceToHost, s));
    CHECK_HIP(hipStreamSynchronize(s));
    if (*c->h_count != 0) return HULLF_EINVAL;
    CHECK_HIP(launch_finish_sort_sets(c->fk[0], c->fv[0], c->fk[1], c->fv[1], mm, sp_sort, (uint32_t)T1, c->fhist,
                                      c->frow, d_sdp, s));
    // S + 1 words of src at the host indices idx (through d_tix / d_tout)
    std::vector<uint32_t> took(S1);
    auto take = [&](const uint32_t* src, const uint32_t* d_idx) -> hipError_t {
        hipError_t e = launch_take_u32(src, d_idx, S1, d_tout, s);
        if (e == hipSuccess) e = hipMemcpyAsync(took.data(), d_tout, S1 * sizeof(uint32_t), hipMemcpyDeviceToHost, s);
        if (e == hipSuccess) e = hipStreamSynchronize(s);
        return e;
    };
    std::vector<uint32_t> soff[2];   // per side: each set's chain in the side's host arrays
    uint32_t* const off_b = c->fchain + c->f_cap / 2;   // second offset array of the merge rounds
    uint2* const br = reinterpret_cast<uint2*>(c->fchain);
    uint32_t* const tcnt = c->fcnt + c->f_cap / kChainChunkMin + 2;
    const uint32_t C = c->chain_chunk;
    std::vector<uint32_t> rng(S1), fcs(S1), rounds;
    // run representatives of both sides per run tile (lower into buffer 1,
    // upper into 3), then each set's range of them
    const SetSplit sp_run{d_rft, d_ipos, S, kRunTile};
    CHECK_HIP(launch_runs(c->fk[0], c->fv[0], mm, c->fk[1], c->fv[1], c->fk[3], c->fv[3], tcnt, s, sp_run,
                          (uint32_t)NRT));
    CHECK_HIP(launch_scan_counts(tcnt, (uint32_t)NRT, c->frow + 256, c->fblk, s));
    CHECK_HIP(launch_copy_u32(tcnt + NRT, c->frow + 256, s));   // toff[NRT] = the total
    CHECK_HIP(take(tcnt, d_rft));
    const std::vector<uint32_t> reps = took;
    if (reps[S] == 0 || reps[S] > mm) return HULLF_EDEVICE;
    for (int side = 0; side < 2; ++side) {
        const int sign = side == 0 ? 1 : -1;
        const int ba = side == 0 ? 1 : 3, bb = side == 0 ? 2 : 0;   // the side's two buffers
        rng = reps;
        // chunk levels
        const uint32_t* toff = tcnt;
        int cur = ba;
        uint32_t cm = rng[S], nc = 0;
        for (;;) {
            const int nxt = (cur == ba) ? bb : ba;
            uint64_t nct = 0;
            for (uint32_t k = 0; k < S; ++k) {
                fcs[k] = (uint32_t)nct;
                nct += (rng[k + 1] - rng[k] + C - 1) / C;
            }
            fcs[S] = (uint32_t)nct;
            CHECK_HIP(hipMemcpyAsync(d_rng, rng.data(), S1 * sizeof(uint32_t), hipMemcpyHostToDevice, s));
            CHECK_HIP(hipMemcpyAsync(d_fcs, fcs.data(), S1 * sizeof(uint32_t), hipMemcpyHostToDevice, s));
            const SetSplit sp_chunk{d_fcs, d_rng, S, C};
            CHECK_HIP(launch_chain(c->fk[cur], cm, C, sign, toff, toff ? (uint32_t)NRT : 0u, c->fchain, c->fcnt, s,
                                   sp_chunk, (uint32_t)nct));
            CHECK_HIP(launch_scan_counts(c->fcnt, (uint32_t)nct, c->frow + 256, c->fblk, s));
            CHECK_HIP(launch_copy_u32(c->fcnt + nct, c->frow + 256, s));
            CHECK_HIP(take(c->fcnt, d_fcs));   // each set's first chain vertex
            const uint32_t tot = took[S];
            if (tot > cm) return HULLF_EDEVICE;
            const int gg = (int)std::max<uint64_t>(1, std::min<uint64_t>((nct * C + 255) / 256, (uint64_t)c->cus * 16));
            CHECK_HIP(launch_chain_gather(c->fk[cur], c->fv[cur], (uint32_t)nct, C, c->fchain, c->fcnt, tot,
                                          c->fk[nxt], c->fv[nxt], gg, s));
            const bool slow = (uint64_t)tot * 4 > (uint64_t)cm * 3;
            cur = nxt;
            cm = tot;
            nc = (uint32_t)nct;
            toff = nullptr;
            rng = took;
            if (slow || cm <= kLevelStop) break;
        }
        // merge rounds inside each set: its chains [fcs[k], fcs[k+1]) of
        // the last level, pairwise, until one per set; every round's split
        // (pairs per set, each set's first chain) is known on the host
        std::vector<uint32_t> kch(S), cs(fcs.begin(), fcs.end());
        uint32_t maxk = 0;
        for (uint32_t k = 0; k < S; ++k) {
            kch[k] = fcs[k + 1] - fcs[k];
            maxk = std::max(maxk, kch[k]);
        }
        rounds.clear();
        uint32_t nr = 0;
        std::vector<uint32_t> nps;
        while (maxk > 1) {
            if (nr == kMaxRounds) return HULLF_EDEVICE;
            std::vector<uint32_t> pps(S1);
            uint64_t np = 0;
            maxk = 0;
            for (uint32_t k = 0; k < S; ++k) {
                pps[k] = (uint32_t)np;
                np += (kch[k] + 1) / 2;
                kch[k] = (kch[k] + 1) / 2;
                maxk = std::max(maxk, kch[k]);
            }
            pps[S] = (uint32_t)np;
            rounds.insert(rounds.end(), pps.begin(), pps.end());   // the round's first pairs
            rounds.insert(rounds.end(), cs.begin(), cs.end());     // and its first chains
            nps.push_back((uint32_t)np);
            cs = pps;
            ++nr;
        }
        if (nr) CHECK_HIP(hipMemcpyAsync(d_rounds, rounds.data(), rounds.size() * sizeof(uint32_t),
                                         hipMemcpyHostToDevice, s));
        CHECK_HIP(launch_copy_u32(c->fcnt + nc, c->frow + 256, s));   // off[nc] = total
        uint32_t* off_in = c->fcnt;
        uint32_t* off_out = off_b;
        uint32_t ncur = nc;
        for (uint32_t r = 0; r < nr; ++r) {
            const uint32_t np = nps[r];
            const int nxt = (cur == ba) ? bb : ba;
            const SetSplit sp_pair{d_rounds + 2ull * r * S1, d_rounds + 2ull * r * S1 + S1, S, 2u};
            const int gg = (int)std::max<uint32_t>(1, std::min<uint32_t>((np + 3) / 4, (uint32_t)c->cus * 8));
            CHECK_HIP(launch_bridge(c->fk[cur], off_in, ncur, sign, br, off_out, gg, s, sp_pair, np));
            CHECK_HIP(launch_scan_counts(off_out, np, off_out + np, c->fblk, s));
            CHECK_HIP(launch_merge_gather(c->fk[cur], c->fv[cur], off_in, ncur, br, off_out, c->fk[nxt], c->fv[nxt],
                                          c->cus * 4, s, sp_pair, np));
            std::swap(off_in, off_out);
            cur = nxt;
            ncur = np;
        }
        // each set's chain (none for a set without survivors)
        CHECK_HIP(hipMemcpyAsync(d_tix, cs.data(), S1 * sizeof(uint32_t), hipMemcpyHostToDevice, s));
        CHECK_HIP(take(off_in, d_tix));
        const uint32_t total = took[S];
        if (total > mm) return HULLF_EDEVICE;
        CHECK_HIP(grow_host(&c->h_bk[side], &c->h_bk_cap[side], total));
        CHECK_HIP(grow_host(&c->h_bv[side], &c->h_bv_cap[side], total));
        CHECK_HIP(hipMemcpyAsync(c->h_bk[side], c->fk[cur], (uint64_t)total * sizeof(uint64_t),
                                 hipMemcpyDeviceToHost, s));
        CHECK_HIP(hipMemcpyAsync(c->h_bv[side], c->fv[cur], (uint64_t)total * sizeof(uint32_t),
                                 hipMemcpyDeviceToHost, s));
        soff[side] = took;
    }
    CHECK_HIP(hipStreamSynchronize(s));
    // per set, on a pool of host threads: the two chain ends the run
    // representatives leave out, then the join; sets in blocks of 16
    std::vector<std::vector<uint32_t>> outs(S);
    std::atomic<uint32_t> next{0};
    std::atomic<bool> bad_chain{false};
    auto work = [&] {
        std::vector<HostPt> lo, up;
        for (;;) {
            const uint32_t k0 = next.fetch_add(16);
            if (k0 >= S) break;
            for (uint32_t k = k0; k < std::min(S, k0 + 16); ++k) {
                if (cnt[k] == 0) continue;
                lo.clear();
                up.clear();
                for (int side = 0; side < 2; ++side) {
                    std::vector<HostPt>& L = side == 0 ? lo : up;
                    const uint64_t* hk = c->h_bk[side];
                    const uint32_t* hv = c->h_bv[side];
                    for (uint32_t q = soff[side][k]; q < soff[side][k + 1]; ++q)
                        L.push_back(HostPt{unord_host((uint32_t)(hk[q] >> 32)), unord_host((uint32_t)hk[q]), hv[q]});
                }
                if (lo.empty() || up.empty()) {
                    bad_chain = true;
                    continue;
                }
                lo.push_back(up.back());
                up.insert(up.begin(), lo.front());
                chain_sorted(lo, up, outs[k]);
            }
        }
    };
    const unsigned nt = std::max(1u, std::min(16u, std::thread::hardware_concurrency()));
    std::vector<std::thread> pool;
    for (unsigned t = 1; t < nt; ++t) pool.emplace_back(work);
    work();
    for (std::thread& t : pool) t.join();
    if (bad_chain) return HULLF_EDEVICE;
    uint64_t total = 0;
    for (uint32_t k = 0; k < S; ++k) {
        hoff[k] = total;
        total += outs[k].size();
    }
    hoff[S] = total;
    if (total > cap) return HULLF_ECAPACITY;
    for (uint32_t k = 0; k < S; ++k) std::copy(outs[k].begin(), outs[k].end(), h_hull + hoff[k]);
    return HULLF_OK;
}

// Hull of pts[d_surv[0..m)] (m indices below n, ascending): the host chain
// for few survivors, the device sort and chains for many.
// Host monotone chain of the m survivors staged in h_surv / h_xy.
hullf_status host_hull(hullf_ctx* c, uint64_t n, uint64_t m, std::vector<uint32_t>& out) {
    std::vector<HostPt> p(m);
    for (uint64_t k = 0; k < m; ++k) {
        if (c->h_surv[k] >= n) return HULLF_EINVAL;
        p[k] = HostPt{c->h_xy[k].x, c->h_xy[k].y, c->h_surv[k]};
    }
    monotone_chain(p, out);
    return HULLF_OK;
}

hullf_status hull_of(hullf_ctx* c, const float2* pts, uint64_t n, const uint32_t* d_surv, uint64_t m,
                     std::vector<uint32_t>& out, hipStream_t s) {
    out.clear();
    if (m == 0) return HULLF_OK;
    if (m >= kDeviceFinishMin && !c->host_finish) return finish_on_device(c, pts, n, d_surv, m, out, s);
    CHECK_HIP(grow_device(c, &c->gather, &c->gather_cap, m, s));
    CHECK_HIP(grow_host(&c->h_surv, &c->h_cap, m));
    CHECK_HIP(grow_host(&c->h_xy, &c->h_xy_cap, m));
    const int grid = (int)std::max<uint64_t>(1, std::min<uint64_t>((m + 255) / 256, (uint64_t)c->cus * 8));
    CHECK_HIP(launch_write_count(c->count, m, s));
    CHECK_HIP(launch_gather(pts, d_surv, c->count, m, n, c->gather, grid, s));
    CHECK_HIP(hipMemcpyAsync(c->h_surv, d_surv, m * sizeof(uint32_t), hipMemcpyDeviceToHost, s));
    CHECK_HIP(hipMemcpyAsync(c->h_xy, c->gather, m * sizeof(float2), hipMemcpyDeviceToHost, s));
    CHECK_HIP(hipStreamSynchronize(s));
    return host_hull(c, n, m, out);
}

// Tune-cache key of a batch: floor(log2 S) and floor(log2(mean set size)).
std::string tune_key(const hullf_ctx* c, uint32_t S, uint64_t n_total) {
    const uint64_t mean = std::max<uint64_t>(1, n_total / std::max<uint32_t>(S, 1));
    int sc = 0, mc = 0;
    while ((2ull << sc) <= S) ++sc;
    while ((2ull << mc) <= mean) ++mc;
    char buf[160];
    std::snprintf(buf, sizeof buf, "%s:%d:s%d:m%d", c->arch.c_str(), c->cus, sc, mc);
    return buf;
}

// The shape the batched launch uses: the tune cache's entry for the batch's
// class, else the context's (default or last tuned) shape.
Shape batch_shape_for(const hullf_ctx* c, uint32_t S, uint64_t n_total) {
    auto it = c->tune.find(tune_key(c, S, n_total));
    return it != c->tune.end() ? it->second : c->batch_shape;
}

// Cache file: one "key block ppt" line per entry; unknown or malformed
// lines and unsupported shapes are ignored.
void tune_load(hullf_ctx* c) {
    if (c->tune_path.empty()) return;
    FILE* f = std::fopen(c->tune_path.c_str(), "r");
    if (!f) return;
    char key[160];
    int b = 0, p = 0;
    while (std::fscanf(f, "%159s %d %d", key, &b, &p) == 3) {
        const Shape sh{b, p};
        if (shape_supported(sh)) c->tune[key] = sh;
    }
    std::fclose(f);
}

// Rewrite the cache file with the context's entries merged into the ones
// already stored (written to a temporary file, then renamed).
void tune_save(hullf_ctx* c) {
    if (c->tune_path.empty()) return;
    std::map<std::string, Shape> merged;
    {
        hullf_ctx tmp;
        tmp.tune_path = c->tune_path;
        tune_load(&tmp);
        merged = tmp.tune;
    }
    for (auto& kv : c->tune) merged[kv.first] = kv.second;
    const std::string dir = c->tune_path.substr(0, c->tune_path.find_last_of('/'));
    if (!dir.empty() && dir != c->tune_path) {
        std::string part;
        for (size_t i = 0; i <= dir.size(); ++i)
            if (i == dir.size() || dir[i] == '/') {
                part = dir.substr(0, i);
                if (!part.empty()) (void)mkdir(part.c_str(), 0755);
            }
    }
    const std::string tmpf = c->tune_path + ".tmp" + std::to_string((unsigned long)getpid());
    FILE* f = std::fopen(tmpf.c_str(), "w");
    if (!f) return;
    for (auto& kv : merged) std::fprintf(f, "%s %d %d\n", kv.first.c_str(), kv.second.block, kv.second.ppt);
    const bool ok = std::fclose(f) == 0;
    if (ok) (void)std::rename(tmpf.c_str(), c->tune_path.c_str());
    else (void)std::remove(tmpf.c_str());
}

hullf_status ensure_batch(hullf_ctx* c, uint32_t S, uint64_t n_total, hipStream_t s) {
    bool realloc = false;
    if (S > c->b_sets_cap) {
        CHECK_HIP(hipStreamSynchronize(s));
        ws_free(c, c->b_sets);
        ws_free(c, c->b_octs);
        c->b_sets = nullptr;
        c->b_octs = nullptr;
        c->b_sets_cap = 0;
        const uint32_t cap = std::max<uint32_t>(S, 64);
        CHECK_HIP(ws_alloc(c, &c->b_sets, cap));
        CHECK_HIP(ws_alloc(c, &c->b_octs, cap));
        c->b_sets_cap = cap;
        realloc = true;
    }
    const uint64_t items = batch_max_items(n_total, S);
    const uint64_t rtiles = batch_max_rtiles(n_total, S);
    if (items > 0xFFFFFFFFull || rtiles > 0xFFFFFFFFull) return HULLF_EINVAL;
    if (items > c->b_items_cap || !c->b_bits || !c->b_blkcnt) {
        CHECK_HIP(hipStreamSynchronize(s));
        ws_free(c, c->b_bits);
        ws_free(c, c->b_blkcnt);
        c->b_bits = nullptr;
        c->b_blkcnt = nullptr;
        c->b_items_cap = 0;
        const uint64_t cap = items + items / 4 + 64;
        CHECK_HIP(ws_alloc(c, &c->b_bits, cap * batch_item_words()));
        CHECK_HIP(ws_alloc(c, &c->b_blkcnt, cap));
        c->b_items_cap = cap;
        realloc = true;
    }
    if (rtiles > c->b_part_cap || !c->b_part) {
        uint64_t words = c->b_part_cap * 9;
        CHECK_HIP(grow_device(c, &c->b_part, &words, rtiles * 9, s));
        c->b_part_cap = words / 9;
        realloc = true;
    }
    if (c->region_skip && (c->b_boxes_cap < c->b_part_cap * batch_tile_boxes() || !c->b_boxes)) {
        CHECK_HIP(grow_device(c, &c->b_boxes, &c->b_boxes_cap, c->b_part_cap * batch_tile_boxes(), s));
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
                           (uint32_t)std::min<uint64_t>(c->b_part_cap, 0xFFFFFFFFull), c->b_octs, c->b_bits,
                           c->b_blkcnt, (uint32_t)std::min<uint64_t>(c->b_items_cap, 0xFFFFFFFFull), d_surv,
                           d_counts, c->region_skip ? c->b_boxes : nullptr, shape, c->cus, c->batch_reduce_per_cu,
                           s));
    return HULLF_OK;
}

hullf_status check_batch_args(hullf_ctx* c, const hullf_pt* d_pts, const uint64_t* d_off, uint32_t S,
                              uint64_t n_total, const uint32_t* d_surv, const uint64_t* d_counts) {
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

hullf_status hullf_create(int device, size_t workspace_bytes, hullf_ctx_t* out) {
    if (!out) return HULLF_EINVAL;
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || device < 0 || device >= ndev) return HULLF_EINVAL;
    DeviceGuard g(device);
    hullf_ctx* c = new (std::nothrow) hullf_ctx();
    if (!c) return HULLF_ENOMEM;
    c->device = device;
    c->ws_cap = workspace_bytes;
    int cus = 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, device) == hipSuccess && cus > 0)
        c->cus = cus;
    if (const char* e = std::getenv("HULLF_FILTER_SHAPE")) {   // "block,ppt"
        Shape sh{0, 0};
        if (std::sscanf(e, "%d,%d", &sh.block, &sh.ppt) == 2 && shape_supported(sh)) c->filter_shape = sh;
    }
    if (const char* e = std::getenv("HULLF_FINISH")) c->host_finish = std::strcmp(e, "host") == 0;
    if (const char* e = std::getenv("HULLF_SINGLE_PASS")) c->single_pass = std::atoi(e) != 0;
    if (const char* e = std::getenv("HULLF_CHAIN_CHUNK")) {
        const int v = std::atoi(e);
        if (v >= (int)kChainChunkMin && v <= 64) c->chain_chunk = (uint32_t)v;
    }
    if (const char* e = std::getenv("HULLF_REGION_SKIP")) c->region_skip = std::atoi(e) != 0;
    if (const char* e = std::getenv("HULLF_CLASSIFY_PER_CU")) c->classify_per_cu = std::max(0, std::atoi(e));
    if (const char* e = std::getenv("HULLF_REDUCE_GRID")) c->reduce_grid_max = std::max(0, std::atoi(e));
    if (const char* e = std::getenv("HULLF_BATCH_REDUCE_PER_CU"))
        c->batch_reduce_per_cu = std::min(16, std::max(0, std::atoi(e)));
    if (const char* e = std::getenv("HULLF_COMPACT_BLOCK")) {
        const int b = std::atoi(e);
        if (b == 256 || b == 512 || b == 1024) c->compact_block = b;
    }
    {
        hipDeviceProp_t prop;
        if (hipGetDeviceProperties(&prop, device) == hipSuccess) {
            std::string a = prop.gcnArchName;
            c->arch = a.substr(0, a.find(':'));
        }
        if (c->arch.empty()) c->arch = "unknown";
        if (const char* e = std::getenv("HULLF_TUNE_CACHE")) {
            c->tune_path = e;
        } else if (const char* x = std::getenv("XDG_CACHE_HOME")) {
            c->tune_path = std::string(x) + "/hullf/tune.txt";
        } else if (const char* h = std::getenv("HOME")) {
            c->tune_path = std::string(h) + "/.cache/hullf/tune.txt";
        }
        tune_load(c);
    }
    hipError_t e = hipSuccess;
    if (e == hipSuccess) e = ws_alloc(c, &c->oct, 1);
    if (e == hipSuccess) e = ws_alloc(c, &c->part, 9ull * kReduceMaxGrid);
    if (e == hipSuccess) e = ws_alloc(c, &c->count, 1);
    if (e == hipSuccess) e = ws_alloc(c, &c->blkcnt, kMaxBlocks);
    if (e == hipSuccess) e = ws_alloc(c, &c->groups_read, 1);
    if (e == hipSuccess) e = hipMemset(c->groups_read, 0, sizeof(unsigned long long));
    if (e == hipSuccess) e = ws_alloc(c, &c->b_tot, 1);
    if (e == hipSuccess) e = hipHostMalloc((void**)&c->h_count, sizeof(uint64_t), hipHostMallocDefault);
    if (e == hipSuccess) e = hipHostMalloc((void**)&c->h_oct, sizeof(Octagon), hipHostMallocDefault);
    if (e == hipSuccess) e = hipStreamCreateWithFlags(&c->capture, hipStreamNonBlocking);
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
    void* dev[] = {c->oct, c->part, c->count, c->surv, c->gather, c->bits, c->blkcnt, c->boxes,
                   c->groups_read, c->poly16, c->part16, c->lb, c->bws,
                   c->b_sets, c->b_octs, c->b_tot, c->b_part, c->b_boxes, c->b_bits, c->b_blkcnt};
    for (void* p : dev)
        if (p) (void)hipFree(p);
    void* fin[] = {c->fk[0], c->fk[1], c->fk[2],  c->fk[3], c->fv[0], c->fv[1],  c->fv[2],
                   c->fv[3], c->fchain, c->fcnt, c->fblk,  c->fhist, c->frow};
    for (void* p : fin)
        if (p) (void)hipFree(p);
    void* host[] = {c->h_surv,   c->h_xy,     c->h_count,  c->h_oct,   c->h_fk,    c->h_fv,   c->h_total,
                    c->h_poly16, c->h_bk[0], c->h_bk[1], c->h_bv[0], c->h_bv[1], c->h_stage};
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
    CHECK_HIP(timed(c, 0, s, [&] { return launch_reduce(pts, n, c->part, nullptr, rg, s); }));
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

hullf_status hullf_polygon16(hullf_ctx_t c, const hullf_pt* d_pts, uint64_t n, uint32_t idx_out[16],
                             void* stream) {
    if (!c || !d_pts || !idx_out || n == 0 || n >= (1ull << 32) || !aligned8(d_pts)) return HULLF_EINVAL;
    DeviceGuard g(c->device);
    hipStream_t s = (hipStream_t)stream;
    CHECK_HIP(ensure_poly16(c));
    const float2* pts = reinterpret_cast<const float2*>(d_pts);
    const int rg = reduce16_grid(n, c->cus);
    CHECK_HIP(timed(c, 0, s, [&] { return launch_reduce16(pts, n, c->part16, nullptr, rg, s); }));
    CHECK_HIP(timed(c, 3, s, [&] { return launch_setup16(pts, n, c->poly16, c->part16, (uint32_t)rg, s); }));
    CHECK_HIP(hipMemcpyAsync(c->h_poly16, c->poly16, sizeof(Poly16), hipMemcpyDeviceToHost, s));
    CHECK_HIP(hipStreamSynchronize(s));
    if (c->h_poly16->status == 1) return HULLF_ENONFINITE;
    if (c->h_poly16->status != 0) return HULLF_EDEVICE;
    std::memcpy(idx_out, c->h_poly16->idx, 16 * sizeof(uint32_t));
    return HULLF_OK;
}

hullf_status hull_filter16(hullf_ctx_t c, const hullf_pt* d_pts, uint64_t n, uint32_t* d_surv, uint64_t cap,
                           uint64_t* d_count, void* stream) {
    if (!c || !d_count || n >= (1ull << 32)) return HULLF_EINVAL;
    if (n > 0 && (!d_pts || !aligned8(d_pts) || (cap > 0 && !d_surv))) return HULLF_EINVAL;
    DeviceGuard g(c->device);
    hipStream_t s = (hipStream_t)stream;
    if (n == 0) {
        CHECK_HIP(launch_write_count(d_count, 0, s));
        return HULLF_OK;
    }
    return enqueue_filter16(c, d_pts, n, d_surv, cap, d_count, s);
}

hullf_status hullf_flags(hullf_ctx_t c, const hullf_pt* d_pts, uint64_t n, uint8_t* d_flags, void* stream) {
    if (!c || n >= (1ull << 32)) return HULLF_EINVAL;
    if (n == 0) return HULLF_OK;
    if (!d_pts || !d_flags || !aligned8(d_pts)) return HULLF_EINVAL;
    DeviceGuard g(c->device);
    hipStream_t s = (hipStream_t)stream;
    const float2* pts = reinterpret_cast<const float2*>(d_pts);
    const int rg = reduce_grid(c, n);
    CHECK_HIP(launch_reduce(pts, n, c->part, nullptr, rg, s));
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
    CHECK_HIP(grow_device(c, &c->surv, &c->surv_cap, n, s));
    hullf_status st = enqueue_filter(c, d_pts, n, c->surv, n, c->count, s);
    if (st != HULLF_OK) return st;
    // Few survivors (the usual case) are staged for the host chain right
    // behind the filter, before the count is known (the gather reads it on
    // the device and stages nothing above kEagerHull): one host round trip
    // instead of two.
    const float2* pts = reinterpret_cast<const float2*>(d_pts);
    const uint32_t eager = (uint32_t)std::min<uint64_t>(n, kEagerHull);
    // the stage is page-locked host memory the kernel writes through its
    // device address: no copy back, only the synchronisation
    CHECK_HIP(grow_host(&c->h_stage, &c->h_stage_cap, stage_small_bytes(eager)));
    unsigned char* d_stage = nullptr;
    CHECK_HIP(hipHostGetDevicePointer((void**)&d_stage, c->h_stage, 0));
    CHECK_HIP(launch_stage_small(pts, n, c->surv, c->count, eager, d_stage, s));
    CHECK_HIP(hipStreamSynchronize(s));
    uint64_t m = 0;
    std::memcpy(&m, c->h_stage, sizeof m);
    if (m == kCountNonFinite) return HULLF_ENONFINITE;
    if (m > n) return HULLF_EDEVICE;
    std::vector<uint32_t> out;
    if (m <= eager && (m < kDeviceFinishMin || c->host_finish)) {
        const float2* xy = reinterpret_cast<const float2*>(c->h_stage + 16);
        const uint32_t* idx = reinterpret_cast<const uint32_t*>(c->h_stage + 16 + 8ull * eager);
        std::vector<HostPt> p(m);
        for (uint64_t k = 0; k < m; ++k) {
            if (idx[k] >= n) return HULLF_EINVAL;
            p[k] = HostPt{xy[k].x, xy[k].y, idx[k]};
        }
        monotone_chain(p, out);
    } else {
        st = hull_of(c, pts, n, c->surv, m, out, s);
    }
    if (st != HULLF_OK) return st;
    *h_count = out.size();
    if (out.size() > cap) return HULLF_ECAPACITY;
    std::copy(out.begin(), out.end(), h_hull);
    return HULLF_OK;
}

hullf_status hull_from_survivors(hullf_ctx_t c, const hullf_pt* d_pts, uint64_t n, const uint32_t* d_surv,
                                 uint64_t m, uint32_t* h_hull, uint64_t cap, uint64_t* h_count, void* stream) {
    if (!c || !h_count || n >= (1ull << 32) || m > n) return HULLF_EINVAL;
    if (m > 0 && (!d_pts || !d_surv || !aligned8(d_pts) || (cap > 0 && !h_hull))) return HULLF_EINVAL;
    *h_count = 0;
    if (m == 0) return HULLF_OK;
    DeviceGuard g(c->device);
    std::vector<uint32_t> out;
    const hullf_status st = hull_of(c, reinterpret_cast<const float2*>(d_pts), n, d_surv, m, out,
                                    (hipStream_t)stream);
    if (st != HULLF_OK) return st;
    *h_count = out.size();
    if (out.size() > cap) return HULLF_ECAPACITY;
    std::copy(out.begin(), out.end(), h_hull);
    return HULLF_OK;
}

hullf_status hull_from_survivors_batched(hullf_ctx_t c, const hullf_pt* d_pts, const uint64_t* d_off, uint32_t S,
                                         uint64_t n_total, const uint32_t* d_surv, const uint64_t* d_counts,
                                         uint32_t* h_hull, uint64_t cap, uint64_t* h_hull_off, void* stream) {
    if (!h_hull_off || (cap > 0 && !h_hull)) return HULLF_EINVAL;
    hullf_status st = check_batch_args(c, d_pts, d_off, S, n_total, d_surv, d_counts);
    if (st != HULLF_OK) return st;
    if (S == 0) {
        h_hull_off[0] = 0;
        return HULLF_OK;
    }
    DeviceGuard g(c->device);
    return finish_batch(c, reinterpret_cast<const float2*>(d_pts), d_off, S, n_total, d_surv, d_counts, h_hull, cap,
                        h_hull_off, (hipStream_t)stream);
}

hullf_status hull_filter_batched_shape(hullf_ctx_t c, const hullf_pt* d_pts, const uint64_t* d_off,
                                       uint32_t S, uint64_t n_total, uint32_t* d_surv,
                                       uint64_t* d_counts, int block, int ppt, void* stream) {
    hullf_status st = check_batch_args(c, d_pts, d_off, S, n_total, d_surv, d_counts);
    if (st != HULLF_OK || S == 0) return st;
    Shape shape = batch_shape_for(c, S, n_total);
    if (block) shape.block = block;
    if (ppt) shape.ppt = ppt;
    if (!shape_supported(shape)) return HULLF_EINVAL;
    DeviceGuard g(c->device);
    hipStream_t s = (hipStream_t)stream;
    st = ensure_batch(c, S, n_total, s);
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
    const Shape shape = batch_shape_for(c, S, n_total);
    st = ensure_batch(c, S, n_total, s);
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
    const Shape shape = batch_shape_for(c, S, n_total);
    st = ensure_batch(c, S, n_total, s);
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
    const Shape shapes[] = {{256, 8}, {256, 16}, {512, 8}, {512, 16}};
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
        r = ensure_batch(c, S, n_total, s);
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
    c->tune[tune_key(c, S, n_total)] = best;
    tune_save(c);
    drop_graphs(c);
    if (best_block) *best_block = best.block;
    if (best_ppt) *best_ppt = best.ppt;
    if (best_ms) *best_ms = bms;
    return HULLF_OK;
}

hullf_status hullf_skip_stats(hullf_ctx_t c, uint64_t* groups_read, uint64_t* groups_total) {
    if (!c || !groups_read || !groups_total) return HULLF_EINVAL;
    DeviceGuard g(c->device);
    CHECK_HIP(hipDeviceSynchronize());
    unsigned long long v = 0;
    CHECK_HIP(hipMemcpy(&v, c->groups_read, sizeof v, hipMemcpyDeviceToHost));
    CHECK_HIP(hipMemset(c->groups_read, 0, sizeof v));
    *groups_read = v;
    *groups_total = c->groups_total;
    c->groups_total = 0;
    return HULLF_OK;
}

hullf_status hullf_workspace(hullf_ctx_t c, uint64_t* used_bytes, uint64_t* cap_bytes) {
    if (!c || !used_bytes || !cap_bytes) return HULLF_EINVAL;
    *used_bytes = c->ws_used;
    *cap_bytes = c->ws_cap;
    return HULLF_OK;
}

hullf_status hullf_timing_enable(hullf_ctx_t c, int enable) {
    if (!c) return HULLF_EINVAL;
    c->timing = (uint32_t)enable & ((1u << kKinds) - 1u);
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
