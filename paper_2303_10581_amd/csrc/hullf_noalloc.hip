// hull_filter_noalloc: the single-set filter (Sec. 3.1, 3.2, 4.1.1) with its
// scratch in a fixed device array instead of a context's allocations, for
// callers that cannot allocate device memory (code under HIP graph capture,
// serving loops that forbid allocation).
//
// The array `hullf_noalloc_scratch` below is a host-side stand-in in host
// code: kernels get the device address that hipGetSymbolAddress returns for
// the current device, looked up once per device on the first call and kept
// in `g_scratch`.  Every call on one device shares that device's array, so calls
// that overlap on one device race (the caller orders them).  Nothing in the
// scratch has to start at zero: the reduction writes every partial record the
// set-up reads, the inside test writes every keep word and block count the
// compaction reads.

#include <hip/hip_runtime.h>

#include <mutex>

#include "hullf.h"
#include "hullf_internal.h"

using namespace hullf;

namespace {

constexpr uint64_t kScratchBytes = HULLF_NOALLOC_SCRATCH_BYTES;
constexpr int kMaxDevices = 64;

}  // namespace

// External linkage on purpose: a device variable with internal linkage
// (`static`) is a LOCAL symbol of the code object, which the runtime does
// not resolve by name when the module is loaded for the lookup below (the
// process aborted); the library-unique name avoids clashes instead.
__device__ __align__(256) __attribute__((used)) unsigned char hullf_noalloc_scratch[kScratchBytes];

namespace {

std::mutex g_mu;
void* g_scratch[kMaxDevices] = {};
int g_cus[kMaxDevices] = {};

uint64_t up256(uint64_t b) { return (b + 255) & ~uint64_t(255); }

// Device address of this device's array (and its CU count), looked up once.
hipError_t scratch_of(int dev, unsigned char** p, int* cus) {
    if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lk(g_mu);
    if (!g_scratch[dev]) {
        void* ptr = nullptr;
        hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(hullf_noalloc_scratch));
        if (e != hipSuccess) return e;
        if (!ptr) return hipErrorInvalidSymbol;
        int c = 0;
        e = hipDeviceGetAttribute(&c, hipDeviceAttributeMultiprocessorCount, dev);
        if (e != hipSuccess) return e;
        g_cus[dev] = c > 0 ? c : 256;
        g_scratch[dev] = ptr;
    }
    *p = static_cast<unsigned char*>(g_scratch[dev]);
    *cus = g_cus[dev];
    return hipSuccess;
}

// Layout of the array for n points: partial records, octagon, block counts,
// keep bits, region-skip boxes, each 256-byte aligned.
struct Layout {
    uint64_t part, oct, blkcnt, bits, box, end;
};

Layout layout_of(const FilterPlan& p) {
    Layout l;
    l.part = 0;
    l.oct = up256(l.part + 9ull * kReduceMaxGrid * sizeof(unsigned long long));
    l.blkcnt = up256(l.oct + sizeof(Octagon));
    l.bits = up256(l.blkcnt + kFilterMaxBlocks * sizeof(uint32_t));
    l.box = up256(l.bits + p.bits_words * sizeof(uint64_t));
    l.end = up256(l.box + p.boxes * sizeof(float4));
    return l;
}

hullf_status to_status(hipError_t e) {
    if (e == hipSuccess) return HULLF_OK;
    return e == hipErrorOutOfMemory ? HULLF_ENOMEM : HULLF_EDEVICE;
}

}  // namespace

extern "C" hullf_status hull_filter_noalloc(const hullf_pt* d_pts, uint64_t n, uint32_t* d_surv, uint64_t cap,
                                            uint64_t* d_count, void* stream) {
    if (!d_count) return HULLF_EINVAL;
    if (n > 0 && (!d_pts || ((uintptr_t)d_pts & 7u) || (cap > 0 && !d_surv))) return HULLF_EINVAL;
    if (n > HULLF_NOALLOC_MAX_POINTS) return HULLF_ENOMEM;
    hipStream_t s = (hipStream_t)stream;
    if (n == 0) return to_status(launch_write_count(d_count, 0, s));
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return HULLF_EDEVICE;
    unsigned char* base = nullptr;
    int cus = 0;
    if ((e = scratch_of(dev, &base, &cus)) != hipSuccess) return HULLF_EDEVICE;
    const FilterPlan p = plan_filter(n, cus, Shape{512, 16}, 0, 0);
    const Layout l = layout_of(p);
    if (l.end > kScratchBytes) return HULLF_ENOMEM;
    auto* part = reinterpret_cast<unsigned long long*>(base + l.part);
    auto* oct = reinterpret_cast<Octagon*>(base + l.oct);
    auto* blkcnt = reinterpret_cast<uint32_t*>(base + l.blkcnt);
    auto* bits = reinterpret_cast<uint64_t*>(base + l.bits);
    auto* box = reinterpret_cast<float4*>(base + l.box);
    const float2* pts = reinterpret_cast<const float2*>(d_pts);
    if ((e = launch_reduce(pts, n, part, box, p.reduce_grid, s)) != hipSuccess) return to_status(e);
    if ((e = launch_setup(pts, n, oct, part, (uint32_t)p.reduce_grid, s)) != hipSuccess) return to_status(e);
    if ((e = launch_classify(pts, n, oct, p.spans, bits, blkcnt, box, p.boxes, nullptr, p.shape, p.grid, s)) !=
        hipSuccess)
        return to_status(e);
    e = launch_compact(bits, blkcnt, n, p.spans, oct, d_surv, cap, d_count, 512, p.grid, s);
    return to_status(e);
}
