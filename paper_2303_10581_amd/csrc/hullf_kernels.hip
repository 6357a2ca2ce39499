// HIP kernels (gfx950, wave64) for the octagon filter of Carrasco et al.,
// "An Evaluation of GPU Filters for Accelerating the 2D Convex Hull":
//   k_reduce    Sec. 3.1, the eight extremes by a min/max reduction
//   k_setup     the octagon record (edges, FP32 prefilter, quick-accept box)
//   k_classify  Sec. 3.2, the inside test, keep bits in point order
//   k_compact   Sec. 4.1.1, stream compaction of the keep bits (ballot,
//               popcount and wave scans; block offsets from block counts)
//   k_batch_*   the same steps for many sets in one graph of launches
//
// Data layout: points are float2 (x, y), 8 bytes, AoS.  A block reads a
// chunk/tile of consecutive points as float4 pairs: pair slot j of thread t
// covers points base + 2*(j*BLOCK + t) + {0, 1}, so every load instruction
// of a wave reads 1 KiB of consecutive memory.  Output indices are uint32.
//
// Built with -ffp-contract=off: the binary64 inside test below must be
// evaluated operation by operation.

#include <math.h>

#include <algorithm>
#include <type_traits>

#include "hullf_internal.h"

namespace hullf {
namespace {

// (3 + 16e) e with e = 2^-53: the orientation error bound "A" of
// Shewchuk (1997) for a 2x2 determinant of differences.
constexpr double kBoundC = 0x1.8000000000004p-52;
constexpr float kInfF = __builtin_huge_valf();

// ---------------------------------------------------------------------------
// small helpers
// ---------------------------------------------------------------------------

// Order-preserving map of a float to uint32 (numeric order, -0 == +0).
__device__ __forceinline__ uint32_t ordered_bits(float f) {
    f = (f == 0.0f) ? 0.0f : f;
    uint32_t u = __float_as_uint(f);
    return (u & 0x80000000u) ? ~u : (u | 0x80000000u);
}

// Packed (key, index) for a 64-bit atomic maximum: larger key wins, and on
// equal keys the lower index wins.
__device__ __forceinline__ unsigned long long pack_key(float key, uint32_t idx) {
    return ((unsigned long long)ordered_bits(key) << 32) | (unsigned long long)(0xFFFFFFFFu - idx);
}

__device__ __forceinline__ uint32_t unpack_idx(unsigned long long p) {
    return 0xFFFFFFFFu - (uint32_t)p;
}

__device__ __forceinline__ uint32_t lane_id() { return threadIdx.x & 63u; }

// Number of set bits of `mask` below this lane.
__device__ __forceinline__ uint32_t rank_below(unsigned long long mask) {
    return __builtin_amdgcn_mbcnt_hi((uint32_t)(mask >> 32),
                                     __builtin_amdgcn_mbcnt_lo((uint32_t)mask, 0u));
}

// The 16 low bits of x moved to the even bit positions (bit i -> bit 2i).
__device__ __forceinline__ uint32_t spread16(uint32_t x) {
    x = (x | (x << 8)) & 0x00FF00FFu;
    x = (x | (x << 4)) & 0x0F0F0F0Fu;
    x = (x | (x << 2)) & 0x33333333u;
    x = (x | (x << 1)) & 0x55555555u;
    return x;
}

__device__ __forceinline__ float wave_max(float v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = fmaxf(v, __shfl_xor(v, o, 64));
    return v;
}
__device__ __forceinline__ float wave_min(float v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = fminf(v, __shfl_xor(v, o, 64));
    return v;
}
__device__ __forceinline__ uint32_t wave_min_u32(uint32_t v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = min(v, (uint32_t)__shfl_xor((int)v, o, 64));
    return v;
}
__device__ __forceinline__ uint64_t wave_sum_u64(uint64_t v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        uint32_t lo = (uint32_t)v, hi = (uint32_t)(v >> 32);
        lo = (uint32_t)__shfl_xor((int)lo, o, 64);
        hi = (uint32_t)__shfl_xor((int)hi, o, 64);
        v += ((uint64_t)hi << 32) | lo;
    }
    return v;
}

// Minimum / maximum over the wave with DPP (fused into the ALU op, no LDS):
// quad swaps, half-row and row mirrors, then the two row broadcasts; the
// result is exact in lane 63 and returned as a wave-uniform value.
template <bool MAX>
__device__ __forceinline__ float wave_minmax_dpp(float x) {
#define HULLF_DPP_STEP(CTRL, ROWS)                                                                          \
    {                                                                                                      \
        const float y = __int_as_float(__builtin_amdgcn_update_dpp(__float_as_int(x), __float_as_int(x),   \
                                                                   CTRL, ROWS, 0xF, false));              \
        x = MAX ? fmaxf(x, y) : fminf(x, y);                                                               \
    }
    HULLF_DPP_STEP(0xB1, 0xF)    // quad_perm [1,0,3,2]
    HULLF_DPP_STEP(0x4E, 0xF)    // quad_perm [2,3,0,1]
    HULLF_DPP_STEP(0x141, 0xF)   // row_half_mirror
    HULLF_DPP_STEP(0x140, 0xF)   // row_mirror
    HULLF_DPP_STEP(0x142, 0xA)   // row_bcast:15 into rows 1 and 3
    HULLF_DPP_STEP(0x143, 0xC)   // row_bcast:31 into rows 2 and 3
#undef HULLF_DPP_STEP
    return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(x), 63));
}

__device__ __forceinline__ uint64_t readlane_u64(uint64_t v, uint32_t l) {
    const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)v, (int)l);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(v >> 32), (int)l);
    return ((uint64_t)hi << 32) | lo;
}

typedef float f32x4 __attribute__((ext_vector_type(4)));

// Buffer resource (V#) over `bytes` bytes at a wave-uniform base: raw
// buffer, stride 0, gfx9-family format word.
__device__ __forceinline__ __amdgpu_buffer_rsrc_t make_rsrc(const void* base, uint32_t bytes) {
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(base), (short)0, (int)bytes, 0x00020000);
}
constexpr int kAuxNT = 2;      // non-temporal (streaming) cache policy, for point loads
constexpr int kAuxStore = 0;   // survivor stores: default policy (non-temporal stores of
                               // partial lines measured 1.5x slower)

// Streaming load of the point pair at byte offset voff + soff of a buffer:
// the per-lane part (voff) is one 32-bit VGPR, the per-slot part (soff) a
// scalar, so a tile needs no 64-bit per-lane addresses.
// VEC4: one 16-byte load (base and offsets 16-byte aligned); otherwise two
// 8-byte loads (base only 8-byte aligned).
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));
typedef unsigned int u32x2 __attribute__((ext_vector_type(2)));
template <bool VEC4>
__device__ __forceinline__ float4 load_pair_buf(__amdgpu_buffer_rsrc_t r, uint32_t voff, uint32_t soff) {
    if constexpr (VEC4) {
        const u32x4 v = __builtin_amdgcn_raw_buffer_load_b128(r, (int)voff, (int)soff, kAuxNT);
        return make_float4(__uint_as_float(v.x), __uint_as_float(v.y), __uint_as_float(v.z), __uint_as_float(v.w));
    } else {
        const u32x2 a = __builtin_amdgcn_raw_buffer_load_b64(r, (int)voff, (int)soff, kAuxNT);
        const u32x2 b = __builtin_amdgcn_raw_buffer_load_b64(r, (int)(voff + 8u), (int)soff, kAuxNT);
        return make_float4(__uint_as_float(a.x), __uint_as_float(a.y), __uint_as_float(b.x), __uint_as_float(b.y));
    }
}

// ---------------------------------------------------------------------------
// Sec. 3.1: the eight extremes
// ---------------------------------------------------------------------------
// Tracked keys per thread: 0 max x, 1 max s, 2 max y, 3 min d, 4 min x,
// 5 min s, 6 min y, 7 max d, with s = fl32(x+y), d = fl32(x-y).  Slot j of
// the packed result is E_j: for the "min" trackers the packed key is the
// negated value (E3 maximises fl32(y-x) = -fl32(x-y)).
//
// The hot loop keeps only the running value of each key and the chunk in
// which it last strictly improved (so the first chunk that reached it).
// After the loop, the lowest such chunk over the threads whose value equals
// the block's best holds the block's lowest index attaining it.  One point
// set: the block records that chunk, and k_setup scans only the chunk that
// wins over all blocks (8 chunks per set instead of up to 8 per block, whose
// scattered reloads at the end of the grid were costly on sets with many
// ties).  Batches: the block reloads the winning threads' points itself.
// Either way the streaming loop stays at about 8 VALU operations per point
// instead of 24 for per-point index selects.

// The value tracked for key j (x, fl32(x+y), y or fl32(x-y); the sign is
// applied by the caller), without branches for a j known only at run time:
// x + 0, 0 + y, x + y and x + (-y) are exactly x, y, fl32(x+y) and
// fl32(x-y) (up to the sign of a zero, which equality ignores).
__device__ __forceinline__ float key_select(int j, float x, float y) {
    const int m = j & 3;
    const float a = (m == 2) ? 0.0f : x;
    const float b = (m == 0) ? 0.0f : ((m == 3) ? -y : y);
    return a + b;
}

// The 16-direction filter of the related work (Sec. 2) rotates the points
// at three angles; its 16 directions are k * 22.5 degrees counter-clockwise
// from +x.  A rotation scaled by 1 / cos keeps every argmax, so the key of
// direction (1, t) is x + t*y, and with t = T = fl32(tan 22.5 deg) it is one
// fused multiply-add (one rounding, like fl32(x+y)).  Eight lines carry the
// 16 keys: key k (k < 8) is line k and key k + 8 its negation, which is
// exact, so the maximiser of key k + 8 is the minimiser of line k.  The even
// keys are the octagon's: x, fl32(x+y), y, fl32(y-x) and their negations.
constexpr float kTan22_5 = 0x1.a8279ap-2f;
__device__ __forceinline__ float line16(int k, float x, float y) {
    switch (k & 7) {
        case 0: return x;
        case 1: return fmaf(kTan22_5, y, x);
        case 2: return x + y;
        case 3: return fmaf(kTan22_5, x, y);
        case 4: return y;
        case 5: return fmaf(-kTan22_5, x, y);
        case 6: return y - x;
        default: return fmaf(kTan22_5, y, -x);
    }
}
__device__ __forceinline__ float key16(int k, float x, float y) {
    const float v = line16(k, x, y);
    return k < 8 ? v : -v;
}

// IEEE-754 2019 maximum/minimum (NaN-propagating) lower to gfx950's
// v_maximum3_f32 / v_minimum3_f32 without operand canonicalisation.  NaN
// inputs are detected separately, so their propagation is harmless.
__device__ __forceinline__ float max3f(float a, float b, float c) {
    return __builtin_elementwise_maximum(__builtin_elementwise_maximum(a, b), c);
}
__device__ __forceinline__ float min3f(float a, float b, float c) {
    return __builtin_elementwise_minimum(__builtin_elementwise_minimum(a, b), c);
}
__device__ __forceinline__ float max8(const float* v) {
    return max3f(max3f(v[0], v[1], v[2]), max3f(v[3], v[4], v[5]), __builtin_elementwise_maximum(v[6], v[7]));
}
__device__ __forceinline__ float min8(const float* v) {
    return min3f(min3f(v[0], v[1], v[2]), min3f(v[3], v[4], v[5]), __builtin_elementwise_minimum(v[6], v[7]));
}

// Point of a sub-range at local index p (0 <= p < span) with the validity
// test lo_rel <= p < hi_rel; one 8-byte buffer load, executed only for valid
// lanes (the descriptor's record limit hi_rel also stops any access beyond it).
__device__ __forceinline__ float2 load_point_checked(__amdgpu_buffer_rsrc_t r, uint32_t p, uint32_t lo_rel,
                                                     uint32_t hi_rel, bool& ok) {
    ok = (p >= lo_rel) && (p < hi_rel);
    float2 v = make_float2(0.0f, 0.0f);
    if (ok) {
        const u32x2 a = __builtin_amdgcn_raw_buffer_load_b64(r, (int)(8u * p), 0, 0);
        v = make_float2(__uint_as_float(a.x), __uint_as_float(a.y));
    }
    return v;
}

// Wave-uniform copies in scalar registers.  readfirstlane yields a signed
// int: the low word goes through uint32_t so that it is not sign-extended
// into the high word.
__device__ __forceinline__ uint32_t uniform_u32(uint32_t x) {
    return (uint32_t)__builtin_amdgcn_readfirstlane((int)x);
}
__device__ __forceinline__ uint64_t uniform_u64(uint64_t x) {
    return ((uint64_t)uniform_u32((uint32_t)(x >> 32)) << 32) | (uint64_t)uniform_u32((uint32_t)x);
}

// Descriptor and relative bounds of points [lo, hi) seen from base b
// covering `span` points.
struct RangeView {
    __amdgpu_buffer_rsrc_t r;
    uint32_t lo_rel, hi_rel;
};
__device__ __forceinline__ RangeView range_view(const float2* __restrict__ pts, uint64_t b, uint32_t span,
                                                uint64_t lo, uint64_t hi) {
    // every field is wave-uniform; readfirstlane keeps the descriptor in
    // scalar registers (a vector-register descriptor forces a loop per access)
    RangeView v;
    v.lo_rel = uniform_u32(lo > b ? (uint32_t)min<uint64_t>(lo - b, span) : 0u);
    v.hi_rel = uniform_u32(hi > b ? (uint32_t)min<uint64_t>(hi - b, span) : 0u);
    const uint64_t a = uniform_u64(reinterpret_cast<uint64_t>(pts + b));
    v.r = make_rsrc(reinterpret_cast<const void*>(a), 8u * v.hi_rel);
    return v;
}

// The lane index as an opaque value: offsets derived from it inside a rarely
// taken branch are then computed there instead of being hoisted (and kept
// live, or spilled) across the whole kernel.
__device__ __forceinline__ uint32_t opaque_tid() {
    uint32_t t = threadIdx.x;
    asm volatile("" : "+v"(t));
    return t;
}

// Reduction of points [lo, hi) over chunks c = c0, c0+cstep, ... < nch of
// CH = BLOCK*G*2 points starting at the even base al <= lo (with DEFER,
// lo - 1 <= al: the recorded position must not be negative).  On return (all threads), rec[j] (j < 8) holds the block's packed
// (key, position) for direction j, or 0 if the block saw no point, and
// rec[8] is 1 if a NaN was seen.  The position is the lowest index relative
// to lo attaining the key (DEFER false), or, with DEFER, the chunk holding
// that index, as its first point + 1 - lo: the block then skips the reload
// and the consumer scans the one chunk that wins across blocks.
// box (optional): box[c*NW + w] = (min x, max x, min y, max y) of the
// points wave w read in chunk c -- groups 4k+w (k < G) of 128 points of the
// chunk; NaN for a partial chunk.
// PF: full chunks are loaded one chunk ahead (two register sets), so a wave
// keeps two chunks of loads in flight; for callers that run at low
// occupancy and have the registers to spare.
template <int BLOCK, int G, bool VEC4, bool DEFER, bool PF = false>
__device__ __forceinline__ void reduce_points(const float2* __restrict__ pts, uint64_t lo, uint64_t hi, uint64_t al,
                                              uint32_t c0, uint32_t cstep, uint32_t nch,
                                              unsigned long long* rec, float4* __restrict__ box) {
    constexpr uint32_t CH = BLOCK * G * 2;
    constexpr int NW = BLOCK / 64;
    __shared__ float sh_v[8][NW];

    const uint32_t t = threadIdx.x;
    float v[8] = {-kInfF, -kInfF, -kInfF, kInfF, kInfF, kInfF, kInfF, -kInfF};
    uint32_t grp[8];
#pragma unroll
    for (int j = 0; j < 8; ++j) grp[j] = c0;
    bool bad = false;
    // Boxes of this wave's chunks, lane k holding the k-th chunk it read,
    // stored 64 at a time: a store per chunk would make the next chunk's
    // loads wait for its write acknowledgement (vector loads and stores
    // share one completion counter).
    const uint32_t wv = t >> 6;
    float4 bacc = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
    uint32_t nb = 0, cfirst = c0;
    auto put_box = [&](uint32_t c, float4 b) {
        if (lane_id() == nb) bacc = b;
        if (++nb == 64u) {
            box[(uint64_t)(cfirst + lane_id() * cstep) * NW + wv] = bacc;
            nb = 0;
            cfirst = c + cstep;
        }
    };

    auto full_at = [&](uint32_t c) {
        const uint64_t cb = al + (uint64_t)c * CH;
        return c < nch && cb >= lo && cb + CH <= hi;
    };
    auto fold_full = [&](uint32_t c, const float4* q) {
        static_assert(G == 4, "the hot loop folds 8 points per group");
        float xs[8], ys[8], ss[8], ds[8];
#pragma unroll
        for (int k = 0; k < G; ++k) {
            xs[2 * k] = q[k].x;
            ys[2 * k] = q[k].y;
            xs[2 * k + 1] = q[k].z;
            ys[2 * k + 1] = q[k].w;
        }
#pragma unroll
        for (int i = 0; i < 8; ++i) {
            ss[i] = xs[i] + ys[i];
            ds[i] = xs[i] - ys[i];
        }
        const float m0 = max8(xs), m1 = max8(ss), m2 = max8(ys), m3 = min8(ds);
        const float m4 = min8(xs), m5 = min8(ss), m6 = min8(ys), m7 = max8(ds);
        // maximum() propagates NaN: one test on the x+y maximum covers
        // every NaN coordinate of the group
        bad |= __builtin_isnan(m1);
        if (m0 > v[0]) { v[0] = m0; grp[0] = c; }
        if (m1 > v[1]) { v[1] = m1; grp[1] = c; }
        if (m2 > v[2]) { v[2] = m2; grp[2] = c; }
        if (m3 < v[3]) { v[3] = m3; grp[3] = c; }
        if (m4 < v[4]) { v[4] = m4; grp[4] = c; }
        if (m5 < v[5]) { v[5] = m5; grp[5] = c; }
        if (m6 < v[6]) { v[6] = m6; grp[6] = c; }
        if (m7 > v[7]) { v[7] = m7; grp[7] = c; }
        if (box) {
            const float b0 = wave_minmax_dpp<false>(m4), b1 = wave_minmax_dpp<true>(m0);
            const float b2 = wave_minmax_dpp<false>(m6), b3 = wave_minmax_dpp<true>(m2);
            put_box(c, make_float4(b0, b1, b2, b3));
        }
    };
    auto fold_partial = [&](uint32_t c) {
        const uint64_t cb = al + (uint64_t)c * CH;
        if (box) {
            const float qn = __builtin_nanf("");
            put_box(c, make_float4(qn, qn, qn, qn));
        }
        // a partial chunk: all 2G loads issued before any is used (one
        // memory round trip); the descriptor ends at the range's end, so
        // loads past it read nothing, and points before lo are masked
        const RangeView rv = range_view(pts, cb, CH, lo, hi);
        const uint32_t tt = opaque_tid();
        float2 pq[2 * G];
#pragma unroll
        for (uint32_t k = 0; k < 2 * G; ++k) {
            const uint32_t p = 2u * ((k >> 1) * BLOCK + tt) + (k & 1u);
            const u32x2 a = __builtin_amdgcn_raw_buffer_load_b64(rv.r, (int)(8u * p), 0, 0);
            pq[k] = make_float2(__uint_as_float(a.x), __uint_as_float(a.y));
        }
#pragma unroll
        for (uint32_t k = 0; k < 2 * G; ++k) {
            const uint32_t p = 2u * ((k >> 1) * BLOCK + tt) + (k & 1u);
            if (p < rv.lo_rel || p >= rv.hi_rel) continue;
            const float x = pq[k].x, y = pq[k].y;
            const float s = x + y, d = x - y;
            bad |= __builtin_isnan(s);
            if (x > v[0]) { v[0] = x; grp[0] = c; }
            if (s > v[1]) { v[1] = s; grp[1] = c; }
            if (y > v[2]) { v[2] = y; grp[2] = c; }
            if (d < v[3]) { v[3] = d; grp[3] = c; }
            if (x < v[4]) { v[4] = x; grp[4] = c; }
            if (s < v[5]) { v[5] = s; grp[5] = c; }
            if (y < v[6]) { v[6] = y; grp[6] = c; }
            if (d > v[7]) { v[7] = d; grp[7] = c; }
        }
    };

    if constexpr (!PF) {
        // (the single-set pass keeps the folds written out here: with them as
        // the shared lambdas above its 64-register build spills)
        for (uint32_t c = c0; c < nch; c += cstep) {
            const uint64_t cb = al + (uint64_t)c * CH;
            if (cb >= lo && cb + CH <= hi) {
                static_assert(G == 4, "the hot loop folds 8 points per group");
                const __amdgpu_buffer_rsrc_t rs = make_rsrc(pts + cb, CH * 8u);
                float4 q[G];
#pragma unroll
                for (int k = 0; k < G; ++k) q[k] = load_pair_buf<VEC4>(rs, 16u * t, 16u * k * BLOCK);
                float xs[8], ys[8], ss[8], ds[8];
#pragma unroll
                for (int k = 0; k < G; ++k) {
                    xs[2 * k] = q[k].x;
                    ys[2 * k] = q[k].y;
                    xs[2 * k + 1] = q[k].z;
                    ys[2 * k + 1] = q[k].w;
                }
#pragma unroll
                for (int i = 0; i < 8; ++i) {
                    ss[i] = xs[i] + ys[i];
                    ds[i] = xs[i] - ys[i];
                }
                const float m0 = max8(xs), m1 = max8(ss), m2 = max8(ys), m3 = min8(ds);
                const float m4 = min8(xs), m5 = min8(ss), m6 = min8(ys), m7 = max8(ds);
                // maximum() propagates NaN: one test on the x+y maximum covers
                // every NaN coordinate of the group
                bad |= __builtin_isnan(m1);
                if (m0 > v[0]) { v[0] = m0; grp[0] = c; }
                if (m1 > v[1]) { v[1] = m1; grp[1] = c; }
                if (m2 > v[2]) { v[2] = m2; grp[2] = c; }
                if (m3 < v[3]) { v[3] = m3; grp[3] = c; }
                if (m4 < v[4]) { v[4] = m4; grp[4] = c; }
                if (m5 < v[5]) { v[5] = m5; grp[5] = c; }
                if (m6 < v[6]) { v[6] = m6; grp[6] = c; }
                if (m7 > v[7]) { v[7] = m7; grp[7] = c; }
                if (box) {
                    const float b0 = wave_minmax_dpp<false>(m4), b1 = wave_minmax_dpp<true>(m0);
                    const float b2 = wave_minmax_dpp<false>(m6), b3 = wave_minmax_dpp<true>(m2);
                    put_box(c, make_float4(b0, b1, b2, b3));
                }
            } else {
                if (box) {
                    const float qn = __builtin_nanf("");
                    put_box(c, make_float4(qn, qn, qn, qn));
                }
                // a partial chunk: all 2G loads issued before any is used (one
                // memory round trip); the descriptor ends at the range's end, so
                // loads past it read nothing, and points before lo are masked
                const RangeView rv = range_view(pts, cb, CH, lo, hi);
                const uint32_t tt = opaque_tid();
                float2 pq[2 * G];
#pragma unroll
                for (uint32_t k = 0; k < 2 * G; ++k) {
                    const uint32_t p = 2u * ((k >> 1) * BLOCK + tt) + (k & 1u);
                    const u32x2 a = __builtin_amdgcn_raw_buffer_load_b64(rv.r, (int)(8u * p), 0, 0);
                    pq[k] = make_float2(__uint_as_float(a.x), __uint_as_float(a.y));
                }
#pragma unroll
                for (uint32_t k = 0; k < 2 * G; ++k) {
                    const uint32_t p = 2u * ((k >> 1) * BLOCK + tt) + (k & 1u);
                    if (p < rv.lo_rel || p >= rv.hi_rel) continue;
                    const float x = pq[k].x, y = pq[k].y;
                    const float s = x + y, d = x - y;
                    bad |= __builtin_isnan(s);
                    if (x > v[0]) { v[0] = x; grp[0] = c; }
                    if (s > v[1]) { v[1] = s; grp[1] = c; }
                    if (y > v[2]) { v[2] = y; grp[2] = c; }
                    if (d < v[3]) { v[3] = d; grp[3] = c; }
                    if (x < v[4]) { v[4] = x; grp[4] = c; }
                    if (s < v[5]) { v[5] = s; grp[5] = c; }
                    if (y < v[6]) { v[6] = y; grp[6] = c; }
                    if (d > v[7]) { v[7] = d; grp[7] = c; }
                }
            }
        }
    } else {
        // Loads of chunk c are issued unconditionally, through a descriptor
        // of zero records unless c is a full chunk (such loads read nothing
        // and return zero): the loop stays straight-line, so each fold waits
        // only for its own chunk's loads.
        auto issue = [&](uint32_t c, float4* q) {
            const bool f = full_at(c);
            const __amdgpu_buffer_rsrc_t rs = make_rsrc(f ? (const void*)(pts + al + (uint64_t)c * CH) : (const void*)pts,
                                                        f ? CH * 8u : 0u);
#pragma unroll
            for (int k = 0; k < G; ++k) q[k] = load_pair_buf<VEC4>(rs, 16u * t, 16u * k * BLOCK);
        };
        float4 qa[G], qb[G];
        issue(c0, qa);
        for (uint32_t c = c0; c < nch; c += 2u * cstep) {
            const uint32_t c1 = c + cstep;
            issue(c1, qb);
            if (full_at(c)) fold_full(c, qa);
            else fold_partial(c);
            if (c1 >= nch) break;
            issue(c1 + cstep, qa);
            if (full_at(c1)) fold_full(c1, qb);
            else fold_partial(c1);
        }
    }

    if (box && nb != 0u && lane_id() < nb) box[(uint64_t)(cfirst + lane_id() * cstep) * NW + wv] = bacc;

    // Block best per key.
    const uint32_t lane = lane_id(), wave = t >> 6;
#pragma unroll
    for (int j = 0; j < 8; ++j) {
        const bool is_max = (j == 0 || j == 1 || j == 2 || j == 7);
        const float w = is_max ? wave_max(v[j]) : wave_min(v[j]);
        if (lane == 0) sh_v[j][wave] = w;
    }
    auto block_best = [&](int j) {
        const bool is_max = (j == 0 || j == 1 || j == 2 || j == 7);
        float best = sh_v[j][0];
        for (int w = 1; w < NW; ++w) best = is_max ? fmaxf(best, sh_v[j][w]) : fminf(best, sh_v[j][w]);
        return best;
    };
    // A thread "holds" key j if its own best equals the block's; grp[j] is
    // the first chunk where it reached that value, and the lowest such chunk
    // over the holders contains the block's lowest index attaining it (the
    // chunks are disjoint and ascending).
    __shared__ uint32_t sh_cm[8];
    if (t < 8) sh_cm[t] = 0xFFFFFFFFu;
    __syncthreads();
    uint32_t holdm = 0;
#pragma unroll
    for (int j = 0; j < 8; ++j)
        if (v[j] == block_best(j) && grp[j] < nch) holdm |= 1u << j;
#pragma unroll
    for (int j = 0; j < 8; ++j) {
        const uint32_t cw = wave_min_u32((holdm >> j) & 1u ? grp[j] : 0xFFFFFFFFu);
        if (lane == 0 && cw != 0xFFFFFFFFu) atomicMin(&sh_cm[j], cw);
    }
    if constexpr (DEFER) {
        // Record the chunk itself: rec[j] packs (key, al + c*CH + 1 - lo),
        // a value >= 0 because al >= lo - 1.  The consumer scans that chunk.
        const int any_bad = __syncthreads_or(bad ? 1 : 0);
        if (t < 8) {
            const int j = (int)t;
            const bool is_max = (j == 0 || j == 1 || j == 2 || j == 7);
            const float best = block_best(j);
            const uint32_t c = sh_cm[j];
            rec[j] = (c != 0xFFFFFFFFu) ? pack_key(is_max ? best : -best, (uint32_t)(al + (uint64_t)c * CH + 1u - lo))
                                        : 0ull;
        } else if (t == 8) {
            rec[8] = any_bad ? 1ull : 0ull;
        }
        __syncthreads();
    } else {
        // The holders in that chunk queue (chunk, key, thread) requests and
        // the whole block serves them: each request reloads the 2G points
        // the thread read in the chunk, so most blocks pay one memory round
        // trip here however the holders are spread over waves and keys.
        static_assert(BLOCK == 256, "a request packs the thread index into 8 bits");
        __shared__ uint32_t sh_q[8 * BLOCK];
        __shared__ uint32_t sh_n;
        __shared__ uint32_t sh_lo[8];
        if (t == 0) sh_n = 0;
        if (t < 8) sh_lo[t] = 0xFFFFFFFFu;
        __syncthreads();
#pragma unroll
        for (int j = 0; j < 8; ++j)
            if (grp[j] != sh_cm[j]) holdm &= ~(1u << j);
        if (holdm) {
            uint32_t slot = atomicAdd(&sh_n, (uint32_t)__builtin_popcount(holdm));
#pragma unroll
            for (int j = 0; j < 8; ++j)
                if (holdm & (1u << j)) sh_q[slot++] = (grp[j] << 11) | ((uint32_t)j << 8) | t;
        }
        __syncthreads();
        const uint32_t nreq = sh_n;
        for (uint32_t r = t; r < nreq; r += BLOCK) {
            const uint32_t e = sh_q[r];
            const uint32_t tt = e & 0xFFu;
            const int j = (int)((e >> 8) & 7u);
            const uint64_t cb = al + (uint64_t)(e >> 11) * CH;
            const float best = block_best(j);
            float2 q[2 * G];
#pragma unroll
            for (uint32_t k = 0; k < 2 * G; ++k) {
                const uint64_t g = cb + 2u * ((k >> 1) * BLOCK + tt) + (k & 1u);
                q[k] = (g >= lo && g < hi) ? pts[g] : make_float2(__builtin_nanf(""), __builtin_nanf(""));
            }
            // descending point order: the last match kept is the lowest index
            uint32_t cand = 0xFFFFFFFFu;
#pragma unroll
            for (int k = 2 * G - 1; k >= 0; --k) {
                const uint64_t g = cb + 2u * (((uint32_t)k >> 1) * BLOCK + tt) + ((uint32_t)k & 1u);
                if (key_select(j, q[k].x, q[k].y) == best) cand = (uint32_t)(g - lo);
            }
            if (cand != 0xFFFFFFFFu) atomicMin(&sh_lo[j], cand);
        }
        const int any_bad = __syncthreads_or(bad ? 1 : 0);
        if (t < 8) {
            const int j = (int)t;
            const bool is_max = (j == 0 || j == 1 || j == 2 || j == 7);
            const float best = block_best(j);
            const uint32_t idx = sh_lo[j];
            rec[j] = (idx != 0xFFFFFFFFu) ? pack_key(is_max ? best : -best, idx) : 0ull;
        } else if (t == 8) {
            rec[8] = any_bad ? 1ull : 0ull;
        }
        __syncthreads();
    }
}

// ---------------------------------------------------------------------------
// Octagon set-up (Sec. 3.1 -> Sec. 3.2), one thread, after all blocks of a
// set have published.
// ---------------------------------------------------------------------------
//
// FP32 prefilter bound.  Let W, H be the bounding-box extents, (cx, cy) an
// FP32 point inside the box, and for an edge with exact differences EX, EY
// let M = |EX| H + |EY| W and s = 2^k with 1/(32 u M) < s <= 1/(16 u M),
// u = 2^-24.  With A = fl32(s ex), NB = fl32(-s ey), C0 = fl32(s k),
// k = ex (cy - ay) - ey (cx - ax) in binary64, qx = fl32(x - cx),
// qy = fl32(y - cy), the value d = fma(A, qy, fma(NB, qx, C0)) differs from
// s D (D = exact edge value of the point) by at most about 7 u s M <= 0.45,
// plus absolute underflow terms below 2^-20 because |A|, |NB|, |C0| <= 2^100.
// Hence d < -1 implies D < 0: the binary64 rule keeps the point (it is
// sound, so it never reports "strictly inside" when D <= 0).  And d > 2
// implies D > 1.5/s >= 24 u M, far above the binary64 rule's own error plus
// bound (< 7.01 e M): the rule reports "strictly inside" for that edge.
// Points with every d > 2 are discarded, points with some d < -1 kept, and
// the rest take the binary64 rule itself, so decisions are identical.
//
// Quick-accept box.  A box [XL, XH] x [YL, YH] inside the bounding box is
// accepted only if every corner q has a binary64 edge value above
// 2^-48 M = 32 e M on every edge.  Edge values are affine, so every point of
// the box then has D > 27 e M > 7.01 e M and the rule discards it.

// Executed by all 64 lanes of one wave; lane l works on vertex/edge
// l mod NV, and lanes below 4*NV check one (edge, box corner) pair each.
// The NV vertices are counter-clockwise from the maximum of x, at equal
// angular steps of their directions, so vertex 0 is max x, NV/4 max y, NV/2
// min x, 3NV/4 min y, and the odd multiples of NV/8 are the four diagonal
// (octagon corner) directions.
// `p` is the merged packed key of direction lane mod NV (0 if none), `nf`
// the merged NaN flag; `known`, if not null, holds the NV vertices'
// coordinates (else they are read from pts).
// Returns the status it wrote (0 ok, 1 non-finite, 3 internal), uniform.
template <int NV>
__device__ __forceinline__ int setup_octagon(const float2* __restrict__ pts, uint64_t lo, uint64_t n,
                                             unsigned long long p, uint32_t nf, Poly<NV>* o,
                                             const float2* known = nullptr) {
#pragma clang fp contract(off)
    static_assert(NV == 8 || NV == 16, "octagon or 16-gon");
    constexpr uint32_t VM = NV - 1;
    constexpr unsigned long long VMASK = (1ull << NV) - 1ull;
    const uint32_t lane = lane_id();
    const int j = (int)(lane & VM);
    const uint32_t id = unpack_idx(p);
    const bool miss = (p == 0ull) || ((uint64_t)id >= n);
    if (lane < NV) o->idx[j] = id;
    if (lane == 0) {
        o->mode = 0;
        o->fast = 0;
        o->m = 0;
        o->skip = 0;
        o->bxl = kInfF;
        o->bxh = -kInfF;
        o->byl = kInfF;
        o->byh = -kInfF;
    }
    if (__ballot(miss) != 0ull) {   // no candidate for some direction: only if NaN hid every point
        const int st = nf ? 1 : 3;
        if (lane == 0) o->status = st;
        return st;
    }
    const float2 q = known ? known[j] : pts[lo + id];
    const float vx = q.x, vy = q.y;
    // bounding box: vertex 0 max x, NV/2 min x, NV/4 max y, 3NV/4 min y
    const float xmax = __shfl(vx, 0, 64), xmin = __shfl(vx, NV / 2, 64);
    const float ymax = __shfl(vy, NV / 4, 64), ymin = __shfl(vy, 3 * NV / 4, 64);
    const bool bad = nf || !isfinite(xmax) || !isfinite(xmin) || !isfinite(ymax) || !isfinite(ymin);
    if (lane == 0) o->status = bad ? 1 : 0;
    if (bad) return 1;

    const float nx = __shfl(vx, (j + 1) & VM, 64), ny = __shfl(vy, (j + 1) & VM, 64);
    const bool deg = (vx == nx) && (vy == ny);
    bool first = true;   // first vertex with these coordinates
#pragma unroll
    for (int k = 0; k < NV; ++k) {
        const float kx = __shfl(vx, k, 64), ky = __shfl(vy, k, 64);
        if (k < j && kx == vx && ky == vy) first = false;
    }
    const int distinct = __popcll(__ballot(lane < NV && first));
    const unsigned long long ndm = __ballot(lane < NV && !deg) & VMASK;
    const int m = __popcll(ndm);
    if (lane == 0) o->m = m;
    // Fewer than three distinct vertices: no point can be strictly inside
    // every edge (the rule is sound and the polygon has no interior).
    if (distinct < 3 || m == 0) return 0;

    // edge slot j: the j-th non-degenerate edge, or the first one as padding
    int src = __ffsll((long long)ndm) - 1;
    {
        int cnt = 0;
#pragma unroll
        for (int k = 0; k < NV; ++k)
            if ((ndm >> k) & 1ull) {
                if (cnt == j) src = k;
                ++cnt;
            }
    }
    const float sax = __shfl(vx, src, 64), say = __shfl(vy, src, 64);
    const float sbx = __shfl(nx, src, 64), sby = __shfl(ny, src, 64);
    const double ax = sax, ay = say;
    const double ex = (double)sbx - ax, ey = (double)sby - ay;
    if (lane < NV) {
        o->ax[j] = ax;
        o->ay[j] = ay;
        o->ex[j] = ex;
        o->ey[j] = ey;
    }

    const double up = 1.0 + 0x1p-40;
    const double W = ((double)xmax - (double)xmin) * (1.0 + 0x1p-50);
    const double H = ((double)ymax - (double)ymin) * (1.0 + 0x1p-50);
    const float cx = (float)(0.5 * (double)xmin + 0.5 * (double)xmax);
    const float cy = (float)(0.5 * (double)ymin + 0.5 * (double)ymax);
    const double M = (fabs(ex) * H + fabs(ey) * W) * up;
    const bool mok = isfinite(W) && isfinite(H) && (M > 0.0) && isfinite(M);
    if (lane < NV) o->sm[j] = 0x1p-48 * M;
    const bool skipok = __ballot(lane < NV && !mok) == 0ull;
    bool ok = mok;
    int E = 0;
    (void)frexp(ok ? M * 0x1p-20 : 1.0, &E);   // 16 u M = f 2^E, f in [0.5, 1)
    const double sc = ldexp(1.0, -E);
    const double a = sc * ex;
    const double nb = -sc * ey;
    const double kk = ex * ((double)cy - ay) - ey * ((double)cx - ax);
    const double c0 = sc * kk;
    ok = ok && fabs(a) <= 0x1p100 && fabs(nb) <= 0x1p100 && fabs(c0) <= 0x1p100;
    if (lane < NV) {
        o->A[j] = (float)a;
        o->NB[j] = (float)nb;
        o->C0[j] = (float)c0;
    }
    const bool fast = __ballot(lane < NV && !ok) == 0ull;

    // quick-accept box: candidate from the corner vertices, shrunk towards
    // the centre until all four corners pass every edge
    constexpr int D1 = NV / 8, D3 = 3 * NV / 8, D5 = 5 * NV / 8, D7 = 7 * NV / 8;
    float XL = fmaxf(__shfl(vx, D3, 64), __shfl(vx, D5, 64)), XH = fminf(__shfl(vx, D1, 64), __shfl(vx, D7, 64));
    float YL = fmaxf(__shfl(vy, D5, 64), __shfl(vy, D7, 64)), YH = fminf(__shfl(vy, D1, 64), __shfl(vy, D3, 64));
    bool boxok = fast && XL < XH && YL < YH;
    const int corner = (int)((lane / NV) & 3u);
    for (int it = 0; boxok && it < 8; ++it) {
        const double qx = (corner & 1) ? (double)XH : (double)XL;
        const double qy = (corner & 2) ? (double)YH : (double)YL;
        const double D = ex * (qy - ay) - ey * (qx - ax);
        const bool pass = (lane >= 4 * NV) || (D > 0x1p-48 * M);
        if (__ballot(!pass) == 0ull) break;
        if (it == 7) {
            boxok = false;
            break;
        }
        XL = (float)((double)cx + 0.75 * ((double)XL - (double)cx));
        XH = (float)((double)cx + 0.75 * ((double)XH - (double)cx));
        YL = (float)((double)cy + 0.75 * ((double)YL - (double)cy));
        YH = (float)((double)cy + 0.75 * ((double)YH - (double)cy));
        boxok = XL < XH && YL < YH;
    }
    if (lane == 0) {
        o->cx = cx;
        o->cy = cy;
        o->fast = fast ? 1 : 0;
        if (boxok) {
            o->bxl = XL;
            o->bxh = XH;
            o->byl = YL;
            o->byh = YH;
        }
        o->skip = skipok ? 1 : 0;
        o->mode = 1;
    }
    return 0;
}

// ---------------------------------------------------------------------------
// Sec. 3.2: inside test
// ---------------------------------------------------------------------------

// The binary64 rule: strictly inside every edge (mode == 1 implies m >= 3).
// P points to the polygon record in any address space; in the constant one
// the edge data come in by scalar loads, whose wait does not also wait for
// the vector loads in flight.
template <int NV, typename P>
__device__ __forceinline__ bool contract_inside(P o, float px, float py) {
#pragma clang fp contract(off)
    const double x = px, y = py;
    bool in = true;
    // one edge at a time: this is the rare path, keep its registers few
#pragma unroll 1
    for (int e = 0; e < NV; ++e) {
        const double qx = x - o->ax[e];
        const double qy = y - o->ay[e];
        const double l = o->ex[e] * qy;
        const double r = o->ey[e] * qx;
        const double det = l - r;
        const double bnd = kBoundC * (fabs(l) + fabs(r));
        in = in & (det > bnd);
    }
    return in;
}

// Minimum over the edges of the scaled FP32 edge values (fast == 1).
// The octagon record is written by an earlier launch and only read by the
// kernels that test points: read through the constant address space, its
// uniform fields become scalar loads (scalar cache, their own wait counter)
// instead of vector loads whose waits would also drain the point stream.
template <int NV>
using PolyK = const __attribute__((address_space(4))) Poly<NV>;
typedef PolyK<8> OctagonK;
template <int NV>
__device__ __forceinline__ PolyK<NV>* as_const(const Poly<NV>* o) { return (PolyK<NV>*)o; }

// Minimum of NV values (NV = 8 or 16).
template <int NV>
__device__ __forceinline__ float min_n(const float* d) {
    if constexpr (NV == 8) return min8(d);
    else return __builtin_elementwise_minimum(min8(d), min8(d + 8));
}

// The octagon fields of the FP32 fast paths, read once per kernel (or per
// set) into registers: read inside the sub-tile loop they were reloaded by
// every pair slot's branch, each reload a scalar-memory wait, and C0 copied
// into vector registers again each time (an FMA reads one scalar operand).
template <int NV>
struct EdgeRegsN {
    float A[NV], NB[NV], C0[NV];
    float cx, cy, bxl, bxh, byl, byh;
    int mode, fast;
};
typedef EdgeRegsN<8> EdgeRegs;
template <int NV>
__device__ __forceinline__ EdgeRegsN<NV> load_edges(const Poly<NV>* __restrict__ o) {
    PolyK<NV>* ok = as_const(o);
    EdgeRegsN<NV> r;
#pragma unroll
    for (int e = 0; e < NV; ++e) {
        r.A[e] = ok->A[e];
        r.NB[e] = ok->NB[e];
        // held in a vector register: the inner FMA's other scalar operand
        // is the coefficient A or NB
        float c = ok->C0[e];
        asm volatile("" : "+v"(c));
        r.C0[e] = c;
    }
    r.cx = ok->cx;
    r.cy = ok->cy;
    r.bxl = ok->bxl;
    r.bxh = ok->bxh;
    r.byl = ok->byl;
    r.byh = ok->byh;
    r.mode = ok->mode;
    r.fast = ok->fast;
    return r;
}
template <int NV>
__device__ __forceinline__ float edge_min(const EdgeRegsN<NV>& k, float x, float y) {
    const float qx = x - k.cx, qy = y - k.cy;
    float d[NV];
#pragma unroll
    for (int e = 0; e < NV; ++e) d[e] = fmaf(k.A[e], qy, fmaf(k.NB[e], qx, k.C0[e]));
    return min_n<NV>(d);
}

// 1 = the point survives.  Decision-equivalent to the binary64 rule.
template <int NV>
__device__ __forceinline__ bool keep_point(const Poly<NV>* __restrict__ o, const EdgeRegsN<NV>& ek, float x,
                                           float y) {
    if (ek.mode == 0) return true;
    const bool inbox = (ek.bxl < x) & (x < ek.bxh) & (ek.byl < y) & (y < ek.byh);
    if (inbox) return false;
    if (ek.fast) {
        const float mn = edge_min(ek, x, y);
        if (mn < -1.0f) return true;
        if (mn > 2.0f) return false;
    }
    return !contract_inside<NV>(o, x, y);
}

// ---------------------------------------------------------------------------
// Sub-tiles: loading and testing
// ---------------------------------------------------------------------------
// A sub-tile is ST = BLOCK*PPT points; pair slot j of thread t in a sub-tile
// with base sb covers points sb + 2*(j*BLOCK + t) + {0, 1}.  Masks hold bit
// 2j+h for point h of pair slot j.

// Load one sub-tile; returns the validity mask (bit 2j+h).  Pair slots with
// bit j of skipm set (full sub-tiles only) are not read; their points are
// marked invalid.
template <int BLOCK, int PPT, bool VEC4>
__device__ __forceinline__ uint32_t load_sub(const float2* __restrict__ pts, uint64_t lo, uint64_t hi,
                                             uint64_t sb, float4 (&q)[PPT / 2], uint32_t skipm = 0u) {
    constexpr int NP = PPT / 2;
    constexpr uint32_t ST = BLOCK * PPT;
    const uint32_t t = threadIdx.x;
    if (sb >= lo && sb + ST <= hi) {
        const __amdgpu_buffer_rsrc_t rs = make_rsrc(pts + sb, ST * 8u);
        uint32_t validm = 0;
#pragma unroll
        for (int j = 0; j < NP; ++j) {
            if ((skipm >> j) & 1u) {   // wave-uniform
                q[j] = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
            } else {
                q[j] = load_pair_buf<VEC4>(rs, 16u * t, 16u * j * BLOCK);
                validm |= 3u << (2 * j);
            }
        }
        return validm;
    }
    const RangeView rv = range_view(pts, sb, ST, lo, hi);
    const uint32_t tt = opaque_tid();
    uint32_t validm = 0;
#pragma unroll
    for (int j = 0; j < NP; ++j) {
        bool v0, v1;
        const uint32_t p = 2u * (j * BLOCK + tt);
        const float2 a = load_point_checked(rv.r, p, rv.lo_rel, rv.hi_rel, v0);
        const float2 b = load_point_checked(rv.r, p + 1u, rv.lo_rel, rv.hi_rel, v1);
        q[j] = make_float4(a.x, a.y, b.x, b.y);
        validm |= (v0 ? 1u : 0u) << (2 * j);
        validm |= (v1 ? 1u : 0u) << (2 * j + 1);
    }
    return validm;
}

// Inside test of NP loaded pair slots (lane l of slot j holds two
// consecutive points of a 128-point group: q[j].xy the even one, q[j].zw the
// odd one; bit 2j+h of validm marks point h valid, the same in every lane
// when UNI; TEST = false: mode 0, every valid point is kept).  The
// decisions are taken on wave masks: every comparison is balloted on its own
// (a ballot of a comparison is the comparison's own lane mask) and the masks
// are combined with scalar operations; the two masks left per slot are the
// group's keep words (even points, odd points).  Lane j receives slot j's
// words in (m0, m1) and `total` (uniform) gains the number of kept points.
//
// The scaled FP32 edge values come first; the quick-accept box and the
// binary64 rule only for the points they leave undecided (rare).  The order
// does not change a decision: a point inside the box has every scaled edge
// value above -0.45, so the FP32 test never keeps it, and whatever it
// discards the rule discards.  Testing the box first would only spare the
// edge values of pair slots whose points all lie in the box, which the
// region skip already spares on clouds, and costs a test per point on data
// that mostly survives.
template <int NP, int NV, bool UNI, bool TEST = true>
__device__ __forceinline__ void keep_masks(const Poly<NV>* __restrict__ o, const EdgeRegsN<NV>& ek,
                                           const float4 (&q)[NP], uint32_t validm, unsigned long long& m0,
                                           unsigned long long& m1, uint32_t& total) {
    const uint32_t lane = lane_id();
    if (UNI) validm = uniform_u32(validm);
    const unsigned long long live = __ballot(1);
    uint32_t e0lo = 0, e0hi = 0, e1lo = 0, e1hi = 0;
    if (__ballot(validm != 0u) != 0ull) {   // else every group of the wave was skipped
        const bool fast = ek.fast != 0;
#pragma unroll
        for (int j = 0; j < NP; ++j) {
            unsigned long long v0, v1;   // valid points
            if (UNI) {
                v0 = ((validm >> (2 * j)) & 1u) ? live : 0ull;
                v1 = ((validm >> (2 * j + 1)) & 1u) ? live : 0ull;
            } else {
                v0 = __ballot(((validm >> (2 * j)) & 1u) != 0u);
                v1 = __ballot(((validm >> (2 * j + 1)) & 1u) != 0u);
            }
            unsigned long long b0 = v0, b1 = v1;   // mode 0 keeps every point
            if (TEST && (v0 | v1) != 0ull) {
                unsigned long long u0 = v0, u1 = v1;   // undecided
                b0 = 0ull;
                b1 = 0ull;
                if (fast) {
                    const float mn0 = edge_min(ek, q[j].x, q[j].y);
                    const float mn1 = edge_min(ek, q[j].z, q[j].w);
                    const unsigned long long o0 = __ballot(mn0 < -1.0f), o1 = __ballot(mn1 < -1.0f);
                    b0 = v0 & o0;
                    b1 = v1 & o1;
                    u0 = v0 & ~o0 & ~__ballot(mn0 > 2.0f);
                    u1 = v1 & ~o1 & ~__ballot(mn1 > 2.0f);
                }
                if (__builtin_expect((u0 | u1) != 0ull, 0)) {   // the quick-accept box, then the binary64 rule
                    const float bxl = ek.bxl, bxh = ek.bxh, byl = ek.byl, byh = ek.byh;
                    const bool in0 = (bxl < q[j].x) & (q[j].x < bxh) & (byl < q[j].y) & (q[j].y < byh);
                    const bool in1 = (bxl < q[j].z) & (q[j].z < bxh) & (byl < q[j].w) & (q[j].w < byh);
                    // an opaque copy of the pointer keeps the compiler from
                    // hoisting the binary64 edge data into registers
                    PolyK<NV>* oo = as_const(o);
                    asm volatile("" : "+s"(oo));
                    const bool p0 = ((u0 >> lane) & 1ull) && !in0, p1 = ((u1 >> lane) & 1ull) && !in1;
                    b0 |= __ballot(p0 && !contract_inside<NV>(oo, q[j].x, q[j].y));
                    b1 |= __ballot(p1 && !contract_inside<NV>(oo, q[j].z, q[j].w));
                }
            }
            total += (uint32_t)(__popcll(b0) + __popcll(b1));
            if (lane == (uint32_t)j) {
                e0lo = (uint32_t)b0;
                e0hi = (uint32_t)(b0 >> 32);
                e1lo = (uint32_t)b1;
                e1hi = (uint32_t)(b1 >> 32);
            }
        }
    }
    m0 = ((unsigned long long)e0hi << 32) | e0lo;
    m1 = ((unsigned long long)e1hi << 32) | e1lo;
}

// Keep words of one sub-tile, as keep_masks gives them: (m0, m1) per lane,
// total (uniform) the number of kept points.
struct TileOut {
    unsigned long long m0, m1;
    uint32_t total;
};

// The sub-tiles that are not a full run of unskipped groups of a polygon in
// mode 1 (a partial last sub-tile, skipped groups, mode 0): out of line, so
// the kernel's hot loop stays a short run of code (a copy of the unrolled
// test per sub-tile kind had made the kernel ~10 000 instructions, beyond
// the instruction cache).
template <int BLOCK, int PPT, bool VEC4, int NV>
__device__ __attribute__((noinline)) TileOut classify_tile_cold(const Poly<NV>* __restrict__ o,
                                                               const float2* __restrict__ pts, uint64_t lo,
                                                               uint64_t hi, uint64_t sb, uint32_t skipm) {
    constexpr int NP = PPT / 2;
    constexpr uint32_t ST = BLOCK * PPT;
    // the arguments of a call arrive in vector registers: the uniform ones
    // go back to scalar registers (buffer descriptors and scalar loads)
    o = reinterpret_cast<const Poly<NV>*>(uniform_u64(reinterpret_cast<uint64_t>(o)));
    pts = reinterpret_cast<const float2*>(uniform_u64(reinterpret_cast<uint64_t>(pts)));
    lo = uniform_u64(lo);
    hi = uniform_u64(hi);
    sb = uniform_u64(sb);
    skipm = uniform_u32(skipm);
    const EdgeRegsN<NV> ek = load_edges(o);
    float4 q[NP];
    TileOut r{0ull, 0ull, 0u};
    const bool full = sb >= lo && sb + ST <= hi;
    const uint32_t validm = load_sub<BLOCK, PPT, VEC4>(pts, lo, hi, sb, q, full ? skipm : 0u);
    if (ek.mode == 0) keep_masks<NP, NV, false, false>(o, ek, q, validm, r.m0, r.m1, r.total);
    else keep_masks<NP, NV, false>(o, ek, q, validm, r.m0, r.m1, r.total);
    return r;
}

// Load and test one sub-tile of the range [lo, hi) (skipm: pair slots whose
// groups the region skip discards, full sub-tiles only): the wave's keep
// words in (m0, m1) as keep_masks gives them.  A full sub-tile with nothing
// skipped (every sub-tile of circle-like data) is one straight run of loads
// followed by the tests, so the test of slot j waits only for slot j's load
// and not for the whole sub-tile.
template <int BLOCK, int PPT, bool VEC4, int NV>
__device__ __forceinline__ void classify_tile(const Poly<NV>* __restrict__ o, const EdgeRegsN<NV>& ek,
                                              const float2* __restrict__ pts, uint64_t lo, uint64_t hi,
                                              uint64_t sb, uint32_t skipm, unsigned long long& m0,
                                              unsigned long long& m1, uint32_t& total) {
    constexpr int NP = PPT / 2;
    constexpr uint32_t ST = BLOCK * PPT;
    if (ek.mode != 0 && skipm == 0u && sb >= lo && sb + ST <= hi) {
        float4 q[NP];
        const __amdgpu_buffer_rsrc_t rs = make_rsrc(pts + sb, ST * 8u);
#pragma unroll
        for (int j = 0; j < NP; ++j) q[j] = load_pair_buf<VEC4>(rs, 16u * threadIdx.x, 16u * j * BLOCK);
        keep_masks<NP, NV, true>(o, ek, q, (NP == 16) ? 0xFFFFFFFFu : ((1u << (2 * NP)) - 1u), m0, m1, total);
    } else {
        const TileOut r = classify_tile_cold<BLOCK, PPT, VEC4, NV>(o, pts, lo, hi, sb, skipm);
        m0 = r.m0;
        m1 = r.m1;
        total += uniform_u32(r.total);
    }
}

// ---------------------------------------------------------------------------
// kernels: one point set
// ---------------------------------------------------------------------------

constexpr int kRBlock = 256;
constexpr int kRG = 4;   // pairs per thread per chunk: 8 points
constexpr uint32_t kRChunk = kRBlock * kRG * 2;

// One point set, pass 1.  Every block writes its packed candidates to its
// own partial record with plain stores.  There is deliberately no
// cross-block fence or completion counter here: on this multi-XCD device an
// agent-scope release writes back the XCD's L2, and one per block costs more
// than the whole streaming pass.  k_setup (next launch on the stream) merges
// the records; the kernel boundary makes them visible.
//
// zero[0 .. nzero) is cleared on the way (the single-pass filter's ticket
// and status words; nothing reads them before the filter launch).
template <bool VEC4>
__global__ __launch_bounds__(kRBlock) __attribute__((amdgpu_waves_per_eu(8, 8))) void k_reduce(
    const float2* __restrict__ pts, uint64_t n, unsigned long long* __restrict__ part, float4* __restrict__ box,
    unsigned long long* __restrict__ zero, uint32_t nzero) {
    constexpr uint32_t CH = kRBlock * kRG * 2;
    const uint32_t nch = (uint32_t)((n + CH - 1) / CH);
    for (uint32_t i = blockIdx.x * kRBlock + threadIdx.x; i < nzero; i += gridDim.x * kRBlock) zero[i] = 0ull;
    __shared__ unsigned long long rec[9];
    reduce_points<kRBlock, kRG, VEC4, true>(pts, 0, n, 0, blockIdx.x, gridDim.x, nch, rec, box);
    if (threadIdx.x < 9) part[(uint64_t)threadIdx.x * kReduceMaxGrid + blockIdx.x] = rec[threadIdx.x];
}

// Inverse of ordered_bits (for a value it produced).
__device__ __forceinline__ float from_ordered(uint32_t o) {
    return __uint_as_float((o & 0x80000000u) ? (o & 0x7FFFFFFFu) : ~o);
}

// The lowest index (relative to lo) in [lo, hi) of a point of chunk
// position p (first point lo + p - 1, kRChunk points) whose key j equals
// `best`, or 0xFFFFFFFF; one wave, every lane gets the result, and the
// lane that found it stores the point to *pt.  The window scanned starts at
// the chunk's first point in range and may run one point past the chunk:
// the lowest index attaining `best` lies in the chunk, so the first match in
// the window is still that index.
// NV = 8: key j is the octagon reduction's tracked value (key_select);
// NV = 16: key j is key16(j).
template <int NV = 8>
__device__ __forceinline__ uint32_t scan_chunk(const float2* __restrict__ pts, uint64_t lo, uint64_t hi,
                                               uint32_t p, int j, float best, float2* pt) {
    constexpr uint32_t K = kRChunk / 64;
    const uint32_t lane = lane_id();
    // wave-uniform window [st, st + w) as a buffer: loads past w return 0
    // without a branch or an access, and are masked to NaN, which equals no key
    const uint64_t st = uniform_u64(lo + (uint64_t)max(p, 1u) - 1u);
    const uint32_t w = uniform_u32(st < hi ? (uint32_t)min<uint64_t>(hi - st, kRChunk) : 0u);
    const __amdgpu_buffer_rsrc_t r = make_rsrc(pts + st, 8u * w);
    float2 q[K];
#pragma unroll
    for (uint32_t i = 0; i < K; ++i) {
        const uint32_t e = lane + 64u * i;
        const u32x2 a = __builtin_amdgcn_raw_buffer_load_b64(r, (int)(8u * e), 0, 0);
        q[i] = (e < w) ? make_float2(__uint_as_float(a.x), __uint_as_float(a.y))
                       : make_float2(__builtin_nanf(""), __builtin_nanf(""));
    }
    uint32_t cand = 0xFFFFFFFFu;
    float2 qc = make_float2(0.0f, 0.0f);
#pragma unroll
    for (int i = (int)K - 1; i >= 0; --i)
        if ((NV == 8 ? key_select(j, q[i].x, q[i].y) : key16(j, q[i].x, q[i].y)) == best) {
            cand = (uint32_t)(st + lane + 64u * (uint32_t)i - lo);
            qc = q[i];
        }
    const uint32_t lowest = wave_min_u32(cand);
    if (lowest != 0xFFFFFFFFu && cand == lowest) *pt = qc;
    return lowest;
}

// One point set, pass 2 (one block of NV waves): wave j merges direction j
// of the `nblocks` partial records (direction-major rows: a wave reads its
// row with lane-strided loads, all issued before any is used, then a wave
// maximum; wave 0 also ORs the NaN-flag row), finds the lowest index
// attaining key j in the chunk that won it, and wave 0 builds the polygon
// record.  No barrier separates a direction's merge from its scan: two
// dependent memory round trips in all.  NV = 8: the octagon (keys as the
// reduction tracks them, the "min" directions negated); NV = 16: the
// 16-direction polygon (every key a maximum).
template <int NV>
__global__ __launch_bounds__(64 * NV) void k_setup(const float2* __restrict__ pts, uint64_t n, Poly<NV>* poly,
                                                   const unsigned long long* __restrict__ part, uint32_t nblocks) {
    constexpr uint32_t R = kReduceMaxGrid / 64;   // words per lane of a full row
    __shared__ unsigned long long sh_k[NV];
    __shared__ unsigned long long sh_nf;
    __shared__ float2 sh_pt[NV];
    const uint32_t lane = lane_id(), j = threadIdx.x >> 6;
    const unsigned long long* row = part + (uint64_t)j * kReduceMaxGrid;
    const unsigned long long* nfrow = part + (uint64_t)NV * kReduceMaxGrid;
    unsigned long long m = 0ull, nf = 0ull;
    // lanes read words lane, lane + 64, ...: 16 at a time, all loads of a
    // batch issued before the maxima (one round trip for up to 1024 blocks)
#pragma unroll 1
    for (uint32_t k0 = 0; k0 < R && 64u * k0 < nblocks; k0 += 16u) {
        unsigned long long w[16], f[16];
#pragma unroll
        for (uint32_t k = 0; k < 16; ++k) {
            const uint32_t b = lane + 64u * (k0 + k);
            w[k] = (b < nblocks) ? row[b] : 0ull;
            f[k] = (j == 0 && b < nblocks) ? nfrow[b] : 0ull;
        }
#pragma unroll
        for (uint32_t k = 0; k < 16; ++k) {
            m = max(m, w[k]);
            nf |= f[k];
        }
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        const uint32_t lo = (uint32_t)__shfl_xor((int)(uint32_t)m, o, 64);
        const uint32_t hi = (uint32_t)__shfl_xor((int)(uint32_t)(m >> 32), o, 64);
        m = max(m, ((unsigned long long)hi << 32) | lo);
        const uint32_t flo = (uint32_t)__shfl_xor((int)(uint32_t)nf, o, 64);
        const uint32_t fhi = (uint32_t)__shfl_xor((int)(uint32_t)(nf >> 32), o, 64);
        nf |= ((unsigned long long)fhi << 32) | flo;
    }
    m = uniform_u64(m);
    unsigned long long res = 0ull;
    if (m != 0ull) {
        const float kv = from_ordered((uint32_t)(m >> 32));
        const bool neg = (NV == 8) && !(j == 0 || j == 1 || j == 2 || j == 7);
        const uint32_t idx = scan_chunk<NV>(pts, 0, n, unpack_idx(m), (int)j, neg ? -kv : kv, &sh_pt[j]);
        if (idx != 0xFFFFFFFFu) res = (m & 0xFFFFFFFF00000000ull) | (unsigned long long)(0xFFFFFFFFu - idx);
    }
    if (lane == 0) {
        sh_k[j] = res;
        if (j == 0) sh_nf = nf;
    }
    __syncthreads();
    if (j == 0) (void)setup_octagon<NV>(pts, 0, n, sh_k[lane & (NV - 1)], (uint32_t)sh_nf, poly, sh_pt);
}

// ---------------------------------------------------------------------------
// Sec. 2 (related work): the 16 extremes of the rotated point set
// ---------------------------------------------------------------------------
// Same chunk geometry as k_reduce (256 threads, 8 points per thread per
// 2048-point chunk, the same four region-skip boxes per chunk), 16 keys.
// Every key is tracked as a maximum (keys k + 8 as the negated minimum of
// line k), with the chunk in which it last strictly improved; the block
// records (key, first point of the lowest such chunk over its holders + 1),
// and k_setup<16> scans that chunk for the lowest index.  Up to 128 registers
// per lane (32 running values and chunks, 16 coordinates).
constexpr int kR16PerCU = 4;   // blocks per CU at the occupancy the registers allow

template <bool VEC4>
__global__ __launch_bounds__(kRBlock) __attribute__((amdgpu_waves_per_eu(4, 8))) void k_reduce16(
    const float2* __restrict__ pts, uint64_t n, unsigned long long* __restrict__ part, float4* __restrict__ box) {
    constexpr uint32_t CH = kRChunk;
    constexpr int NW = kRBlock / 64;
    __shared__ float sh_v[16][NW];
    __shared__ uint32_t sh_cm[16];
    const uint32_t t = threadIdx.x, lane = lane_id(), wv = t >> 6;
    const uint32_t nch = (uint32_t)((n + CH - 1) / CH);
    const uint32_t c0 = blockIdx.x, cstep = gridDim.x;
    float v[16];
    uint32_t grp[16];
#pragma unroll
    for (int j = 0; j < 16; ++j) {
        v[j] = -kInfF;
        grp[j] = c0;
    }
    bool bad = false;
    float4 bacc = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
    uint32_t nb = 0, cfirst = c0;
    auto put_box = [&](uint32_t c, float4 b) {
        if (lane == nb) bacc = b;
        if (++nb == 64u) {
            box[(uint64_t)(cfirst + lane * cstep) * NW + wv] = bacc;
            nb = 0;
            cfirst = c + cstep;
        }
    };
    for (uint32_t c = c0; c < nch; c += cstep) {
        const uint64_t cb = (uint64_t)c * CH;
        if (cb + CH <= n) {
            const __amdgpu_buffer_rsrc_t rs = make_rsrc(pts + cb, CH * 8u);
            float4 q[kRG];
#pragma unroll
            for (int k = 0; k < kRG; ++k) q[k] = load_pair_buf<VEC4>(rs, 16u * t, 16u * k * kRBlock);
            float xs[8], ys[8];
#pragma unroll
            for (int k = 0; k < kRG; ++k) {
                xs[2 * k] = q[k].x;
                ys[2 * k] = q[k].y;
                xs[2 * k + 1] = q[k].z;
                ys[2 * k + 1] = q[k].w;
            }
            float bx0 = 0.0f, bx1 = 0.0f, by0 = 0.0f, by1 = 0.0f;
#pragma unroll
            for (int i = 0; i < 8; ++i) {
                float L[8];
#pragma unroll
                for (int k = 0; k < 8; ++k) L[k] = line16(i, xs[k], ys[k]);
                const float mx = max8(L), mn = min8(L);
                if (i == 2) bad |= __builtin_isnan(mx);   // maximum() propagates NaN: x+y covers every coordinate
                if (i == 0) { bx0 = mn; bx1 = mx; }
                if (i == 4) { by0 = mn; by1 = mx; }
                if (mx > v[i]) { v[i] = mx; grp[i] = c; }
                if (-mn > v[i + 8]) { v[i + 8] = -mn; grp[i + 8] = c; }
            }
            if (box) {
                const float b0 = wave_minmax_dpp<false>(bx0), b1 = wave_minmax_dpp<true>(bx1);
                const float b2 = wave_minmax_dpp<false>(by0), b3 = wave_minmax_dpp<true>(by1);
                put_box(c, make_float4(b0, b1, b2, b3));
            }
        } else {
            if (box) {
                const float qn = __builtin_nanf("");
                put_box(c, make_float4(qn, qn, qn, qn));
            }
            const RangeView rv = range_view(pts, cb, CH, 0, n);
            const uint32_t tt = opaque_tid();
#pragma unroll 1
            for (uint32_t k = 0; k < 2 * kRG; ++k) {
                bool ok;
                const uint32_t p = 2u * ((k >> 1) * kRBlock + tt) + (k & 1u);
                const float2 pq = load_point_checked(rv.r, p, rv.lo_rel, rv.hi_rel, ok);
                if (!ok) continue;
                bad |= __builtin_isnan(pq.x + pq.y);
#pragma unroll
                for (int i = 0; i < 8; ++i) {
                    const float L = line16(i, pq.x, pq.y);
                    if (L > v[i]) { v[i] = L; grp[i] = c; }
                    if (-L > v[i + 8]) { v[i + 8] = -L; grp[i + 8] = c; }
                }
            }
        }
    }
    if (box && nb != 0u && lane < nb) box[(uint64_t)(cfirst + lane * cstep) * NW + wv] = bacc;

    // block best per key; the holders' lowest first-improvement chunk
#pragma unroll
    for (int j = 0; j < 16; ++j) {
        const float w = wave_max(v[j]);
        if (lane == 0) sh_v[j][wv] = w;
    }
    if (t < 16) sh_cm[t] = 0xFFFFFFFFu;
    __syncthreads();
#pragma unroll
    for (int j = 0; j < 16; ++j) {
        float best = sh_v[j][0];
#pragma unroll
        for (int w = 1; w < NW; ++w) best = fmaxf(best, sh_v[j][w]);
        const bool hold = (v[j] == best) && (grp[j] < nch);
        const uint32_t cw = wave_min_u32(hold ? grp[j] : 0xFFFFFFFFu);
        if (lane == 0 && cw != 0xFFFFFFFFu) atomicMin(&sh_cm[j], cw);
    }
    const int any_bad = __syncthreads_or(bad ? 1 : 0);
    if (t < 16) {
        const int j = (int)t;
        float best = sh_v[j][0];
#pragma unroll
        for (int w = 1; w < NW; ++w) best = fmaxf(best, sh_v[j][w]);
        const uint32_t c = sh_cm[j];
        part[(uint64_t)j * kReduceMaxGrid + blockIdx.x] =
            (c != 0xFFFFFFFFu) ? pack_key(best, (uint32_t)((uint64_t)c * CH + 1u)) : 0ull;
    } else if (t == 16) {
        part[16ull * kReduceMaxGrid + blockIdx.x] = any_bad ? 1ull : 0ull;
    }
}

// ---------------------------------------------------------------------------
// Two-pass compaction: classify (inside test, keep bits) then compact
// ---------------------------------------------------------------------------
// Pass 1 streams the points once and stores the keep bits in point order:
// group g is points [128g, 128g+128); word 2g holds the even points and
// word 2g+1 the odd ones, bit l of word 2g+h being point 128g + 2l + h
// (the layout of one wave's two ballots over a pair slot).  Block b owns the
// points [b*R, (b+1)*R), R = spans * kSpan, and writes its survivor count;
// no block waits for another.  Pass 2 runs the same blocks over the same
// ranges: the sum of the earlier blocks' counts is block b's output offset,
// and each span of kSpan points (64 groups, one per lane) is ordered by a
// wave-wide scan of the group counts.  Both passes read or write every byte
// once: 8 bytes per point and 1/4 byte of keep bits per point in pass 1,
// the keep bits and 4 bytes per survivor in pass 2.

constexpr uint32_t kSpan = 8192;
constexpr uint32_t kSpanGroups = kSpan / 128;
// Per-wave LDS of the compaction: a stage of up to 1024 survivor indices,
// then the span's keep bits in point order (64 groups x 4 words).
constexpr uint32_t kStageIdx = 1024;
constexpr uint32_t kStageWords = kStageIdx + 4 * 64;
static_assert(kSpanGroups == 64, "one group per lane");

// Region skip.  Each k_classify block tests the reduction boxes of its range
// against the octagon: a box passes iff all four corners have a binary64
// edge value above sm[e] on every edge e -- the test the quick-accept box
// passes in the octagon set-up, so every point in the box is discarded by
// the rule.  The block then does not read groups whose box passed.
// Group g of a set was read in the reduction by wave g % 4 of chunk g / 16:
// its box is 4 * (g / 16) + g % 4.
static_assert(kRBlock * kRG * 2 == 16 * 128 && kRBlock / 64 == 4, "box of group g: chunk g/16, wave g%4");

// True iff all four corners of box b have a binary64 edge value above sm[e]
// on every edge e (false for a NaN box).
template <int NV>
__device__ __forceinline__ bool box_inside(float4 b, PolyK<NV>* __restrict__ ok) {
    bool pass = true;
#pragma unroll 1
    for (int e = 0; e < NV; ++e) {   // one edge's data live at a time
        const double ax = ok->ax[e], ay = ok->ay[e], ex = ok->ex[e], ey = ok->ey[e], sm = ok->sm[e];
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            const double qx = (double)((k & 1) ? b.y : b.x);
            const double qy = (double)((k & 2) ? b.w : b.z);
            const double D = ex * (qy - ay) - ey * (qx - ax);
            pass = pass && (D > sm);
        }
    }
    return pass;
}

// Skip words held per inside-test block: one bit per reduction box of the
// block's range (64 boxes, 32768 points, per word).  A range longer than
// kSkipWords words is not skipped past them.
constexpr uint32_t kSkipWords = 1024;
// Sparse inside test: a block whose unread groups (inside passing boxes) are
// at least 3/4 of its groups, and whose other groups fit in kSparseList
// entries, lists the groups to read and tests only those, NP per wave at a
// time with all their loads issued together; the skipped groups get zero
// keep words.  Walking the range sub-tile by sub-tile instead costs one
// memory round trip per sub-tile even when almost nothing is read.
constexpr uint32_t kSparseList = 2048;

// Skip bit of group g (0 if its box is not covered by the block's words).
__device__ __forceinline__ bool group_skipped(const unsigned long long* sh_skip, uint64_t g, uint64_t w0,
                                              uint32_t nw) {
    const uint64_t rel = (g >> 8) - w0;
    if (rel >= nw) return false;
    const uint32_t bit = (uint32_t)(4u * ((g >> 4) & 15u) + (g & 3u));
    return (sh_skip[rel] >> bit) & 1ull;
}

// Load the points of NP listed groups (slot k: group list[k], valid for
// k < cnt): lane l holds points 128 g + 2l and 128 g + 2l + 1 of slot k, the
// layout of a pair slot; returns the validity mask (bit 2k+h).
template <int NP, bool VEC4>
__device__ __forceinline__ uint32_t load_groups(const float2* __restrict__ pts, uint64_t n,
                                                const uint32_t* list, uint32_t cnt, float4 (&q)[NP]) {
    const uint32_t lane = lane_id();
    uint32_t validm = 0;
#pragma unroll
    for (int k = 0; k < NP; ++k) {
        q[k] = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
        if ((uint32_t)k < cnt) {   // wave-uniform
            const uint64_t g = uniform_u32(list[k]);
            const uint64_t i0 = 128ull * g + 2u * lane;
            const float2* gp = pts + 128ull * g;   // uniform base
            if (128ull * g + 128ull <= n) {
                if constexpr (VEC4) {
                    q[k] = reinterpret_cast<const float4*>(gp)[lane];
                } else {
                    const float2 a = gp[2u * lane], b = gp[2u * lane + 1u];
                    q[k] = make_float4(a.x, a.y, b.x, b.y);
                }
                validm |= 3u << (2 * k);
            } else {
                const bool v0 = i0 < n, v1 = i0 + 1u < n;
                const float2 a = v0 ? gp[2u * lane] : make_float2(0.0f, 0.0f);
                const float2 b = v1 ? gp[2u * lane + 1u] : make_float2(0.0f, 0.0f);
                q[k] = make_float4(a.x, a.y, b.x, b.y);
                validm |= ((v0 ? 1u : 0u) | (v1 ? 2u : 0u)) << (2 * k);
            }
        }
    }
    return validm;
}


template <int BLOCK, int PPT, bool VEC4, int NV>
__global__ __launch_bounds__(BLOCK) __attribute__((amdgpu_waves_per_eu(6, 8))) void k_classify(
    const float2* __restrict__ pts, uint64_t n, const Poly<NV>* __restrict__ oct, uint32_t spans,
    uint64_t* __restrict__ bits, uint32_t* __restrict__ blkcnt, const float4* __restrict__ box, uint64_t nbox,
    unsigned long long* loaded) {
    constexpr int NP = PPT / 2;
    constexpr int NW = BLOCK / 64;
    constexpr uint32_t ST = BLOCK * PPT;
    static_assert(kSpan % ST == 0, "sub-tiles tile a span");
    static_assert(NP <= 64, "one lane per pair slot stores the bits");
    __shared__ uint32_t sh_w[NW], sh_g[NW];
    __shared__ unsigned long long sh_skip[kSkipWords];
    __shared__ uint32_t sh_list[kSparseList];
    __shared__ uint32_t sh_nlist;
    if (oct->status != 0) return;
    const uint32_t lane = lane_id();
    const uint32_t wave = uniform_u32(threadIdx.x >> 6);   // keeps wave-derived addresses scalar
    const uint64_t r0 = (uint64_t)blockIdx.x * spans * kSpan;
    const uint64_t r1 = min<uint64_t>(n, r0 + (uint64_t)spans * kSpan);
    const uint64_t ngroups = (n + 127) / 128;
    // Region skip: the block tests the reduction boxes of its own range
    // against the octagon and keeps one bit per box in LDS (word i - w0 covers
    // points [i*32768, (i+1)*32768)).  Each wave's 64 consecutive boxes make
    // one ballot, so every lane of a wave takes the same loop trips.
    PolyK<NV>* ok = as_const(oct);
    const bool skipon = box != nullptr && ok->mode == 1 && ok->skip != 0;
    const uint64_t w0 = r0 >> 15;
    const uint32_t nw = (uint32_t)min<uint64_t>(((r1 + 32767u) >> 15) - w0, kSkipWords);
    const EdgeRegsN<NV> ek = load_edges(oct);
    // any skip bit set in the block's words (else no group is skipped)
    bool anyskip = false;
    if (skipon) {
        for (uint32_t i = threadIdx.x; i < nw * 64u; i += BLOCK) {
            const uint64_t bi = (w0 << 6) + i;
            bool pass = false;
            if (bi < nbox) {
                const float4 b = box[bi];
                // FP32 screen of the corners: a scaled edge value below -1 at a
                // corner means D < 0 there (the box fails); above 2 at all four
                // corners on every edge means D > 24 u M_e > sm[e] there (the box
                // passes, NaN never does); only the others take the binary64
                // corner test
                bool decided = false;
                if (ek.fast != 0) {
                    const float mn = min(min(edge_min(ek, b.x, b.z), edge_min(ek, b.y, b.z)),
                                         min(edge_min(ek, b.x, b.w), edge_min(ek, b.y, b.w)));
                    decided = (mn < -1.0f) || (mn > 2.0f);
                    pass = mn > 2.0f;
                }
                if (!decided) pass = box_inside<NV>(b, ok);
            }
            const unsigned long long m = __ballot(pass);
            if (lane == 0) sh_skip[i >> 6] = m;
        }
        __syncthreads();
        unsigned long long any = 0ull;
        for (uint32_t i = 0; i < nw; ++i) any |= sh_skip[i];
        anyskip = any != 0ull;
    }
    uint32_t total = 0, groups = 0;
    // Sparse inside test: list the groups to read (lane per group) and
    // decide whether the block takes the listed path.
    bool sparse = false;
    const uint64_t g0 = r0 >> 7, g1 = (r1 + 127) >> 7;
    if (anyskip) {
        if (threadIdx.x == 0) sh_nlist = 0u;
        __syncthreads();
        for (uint64_t gb = g0 + (uint64_t)wave * 64u; gb < g1; gb += (uint64_t)NW * 64u) {
            const uint64_t g = gb + lane;
            const bool need = g < g1 && !group_skipped(sh_skip, g, w0, nw);
            const unsigned long long m = __ballot(need);
            uint32_t base = 0;
            if (lane == 0 && m != 0ull) base = atomicAdd(&sh_nlist, (uint32_t)__popcll(m));
            base = uniform_u32((uint32_t)__shfl((int)base, 0, 64));
            const uint32_t pos = base + rank_below(m);
            if (need && pos < kSparseList) sh_list[pos] = (uint32_t)g;
        }
        __syncthreads();
        const uint32_t nl = sh_nlist;
        sparse = nl <= kSparseList && 4ull * nl <= g1 - g0;
    }
    if (sparse) {
        const uint32_t nl = sh_nlist;
        // the listed groups, NPL per wave at a time (8 whatever the sub-tile
        // shape: the list is short, and a round of loads is a memory round trip)
        constexpr int NPL = 8;
        for (uint32_t b = wave * (uint32_t)NPL; b < nl; b += (uint32_t)(NW * NPL)) {
            const uint32_t cnt = min((uint32_t)NPL, nl - b);
            float4 q[NPL];
            const uint32_t validm = load_groups<NPL, VEC4>(pts, n, sh_list + b, cnt, q);
            unsigned long long m0, m1;
            keep_masks<NPL, NV, false>(oct, ek, q, validm, m0, m1, total);
            if (lane < cnt) {
                const uint64_t g = sh_list[b + lane];
                *reinterpret_cast<ulonglong2*>(bits + 2 * g) = make_ulonglong2(m0, m1);
            }
            groups += cnt;
        }
        // zero keep words for the groups that were not read, needed only if
        // the block kept a point: the compaction skips blocks whose count is 0
        if (lane == 0) sh_g[wave] = total;
        __syncthreads();
        uint32_t any = 0;
#pragma unroll
        for (int w = 0; w < NW; ++w) any |= sh_g[w];
        __syncthreads();   // sh_g is rewritten below
        if (any != 0u) {
            for (uint64_t gb = g0 + (uint64_t)wave * 64u; gb < g1; gb += (uint64_t)NW * 64u) {
                const uint64_t g = gb + lane;
                if (g < g1 && group_skipped(sh_skip, g, w0, nw))
                    *reinterpret_cast<ulonglong2*>(bits + 2 * g) = make_ulonglong2(0ull, 0ull);
            }
        }
    }
    // Dense blocks (no group of the range skipped: every block of circle-like
    // data): the loads of sub-tile i+1 are issued before sub-tile i is
    // tested, so a wave keeps a sub-tile of loads in flight while it
    // computes (two register buffers, used in turn).
    // (two buffers of 8 slots would not fit the register budget; mode 0 keeps
    // every point and takes the out-of-line path)
    const bool dense = !anyskip && NP <= 4 && ek.mode != 0;
    uint64_t rs0 = r0;   // where the sub-tile loop below starts
    if (dense) {
        constexpr uint32_t allv = (NP == 16) ? 0xFFFFFFFFu : ((1u << (2 * NP)) - 1u);
        const uint64_t rf = r0 + ((r1 - r0) / ST) * ST;   // end of the full sub-tiles
        // past rf the descriptor is empty: the loads return zeros and read nothing
        auto load = [&](uint64_t sb, float4(&q)[NP]) {
            const bool in = sb < rf;
            const __amdgpu_buffer_rsrc_t rs = make_rsrc(pts + (in ? sb : 0), in ? ST * 8u : 0u);
#pragma unroll
            for (int j = 0; j < NP; ++j) q[j] = load_pair_buf<VEC4>(rs, 16u * threadIdx.x, 16u * j * BLOCK);
        };
        auto test_store = [&](uint64_t sb, const float4(&q)[NP]) {
            unsigned long long m0, m1;
            keep_masks<NP, NV, true>(oct, ek, q, allv, m0, m1, total);
            const uint64_t g = (sb >> 7) + (uint64_t)(lane * NW + wave);
            if (lane < (uint32_t)NP) *reinterpret_cast<ulonglong2*>(bits + 2 * g) = make_ulonglong2(m0, m1);
            groups += (uint32_t)NP;
        };
        if (NP <= 4 && rf > r0) {
            float4 qa[NP], qb[NP];
            load(r0, qa);
            for (uint64_t sb = r0; sb < rf; sb += 2ull * ST) {
                load(sb + ST, qb);
                test_store(sb, qa);
                if (sb + ST >= rf) break;
                load(sb + 2ull * ST, qa);
                test_store(sb + ST, qb);
            }
        }
        rs0 = rf;   // the partial sub-tile, if any
    }
    for (uint64_t sb = rs0; !sparse && sb < r1; sb += ST) {
        uint32_t skipm = 0;
        const uint64_t rel = (sb >> 15) - w0;
        if (anyskip && sb + ST <= n && rel < nw) {
            // this sub-tile's boxes are 4*ST/2048 consecutive bits of one word
            const uint64_t word = sh_skip[rel];
#pragma unroll
            for (int j = 0; j < NP; ++j) {
                const uint64_t gg = (sb >> 7) + (uint64_t)(j * NW) + wave;
                const uint64_t bi = (gg >> 4) * 4 + (gg & 3);
                skipm |= (uint32_t)((word >> (bi & 63)) & 1ull) << j;
            }
        }
        groups += (uint32_t)(NP - __popc(skipm));
        // lane j holds the two keep words of pair slot j, then all NP groups
        // of this wave are stored by one instruction
        unsigned long long m0, m1;
        classify_tile<BLOCK, PPT, VEC4, NV>(oct, ek, pts, 0, n, sb, skipm, m0, m1, total);
        const uint64_t g = (sb >> 7) + (uint64_t)(lane * NW + wave);
        if (lane < (uint32_t)NP && g < ngroups) {
            ulonglong2 v;
            v.x = m0;
            v.y = m1;
            *reinterpret_cast<ulonglong2*>(bits + 2 * g) = v;
        }
    }
    if (lane == 0) {
        sh_w[wave] = total;
        sh_g[wave] = groups;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        uint32_t sum = 0, g = 0;
#pragma unroll
        for (int w = 0; w < NW; ++w) {
            sum += sh_w[w];
            g += sh_g[w];
        }
        blkcnt[blockIdx.x] = sum;
        if (loaded) atomicAdd(loaded, (unsigned long long)g);   // groups of 128 points read
    }
}


// Survivors of one span: (w0, w1) are this lane's group words (lane = group),
// written in ascending order to out[base ...] through the wave's LDS stage;
// a span whose 64 groups are all full is stored directly.
__device__ __forceinline__ void compact_span(unsigned long long w0, unsigned long long w1, uint64_t sb,
                                             uint64_t base, uint64_t cap, uint32_t idx_shift,
                                             uint32_t* __restrict__ out, uint32_t* stage) {
    const uint32_t lane = lane_id();
    const uint32_t c = (uint32_t)(__popcll(w0) + __popcll(w1));
    const uint64_t room = cap > base ? cap - base : 0ull;
    const uint32_t lim = room < (uint64_t)kSpan ? (uint32_t)room : kSpan;
    const __amdgpu_buffer_rsrc_t ro = make_rsrc(out + base, 4u * lim);
    if (__ballot(c == 128u) == ~0ull && lim == kSpan) {
        // every group full: the survivors are the kSpan consecutive indices
        // from sb, stored as h single words up to a 16-byte boundary, then
        // aligned 16-byte quads, then the remaining words
        const uint32_t i0 = (uint32_t)sb - idx_shift;
        const uint32_t h = (uint32_t)((16u - ((uint32_t)reinterpret_cast<uintptr_t>(out + base) & 15u)) & 15u) >> 2;
        if (lane < h) __builtin_amdgcn_raw_buffer_store_b32(i0 + lane, ro, (int)(4u * lane), 0, kAuxStore);
        const uint32_t nq = (kSpan - h) >> 2;
        for (uint32_t u = lane; u < nq; u += 64u) {
            const uint32_t q = i0 + h + 4u * u;
            __builtin_amdgcn_raw_buffer_store_b128((u32x4){q, q + 1u, q + 2u, q + 3u}, ro, (int)(4u * (h + 4u * u)),
                                                   0, kAuxStore);
        }
        const uint32_t t0 = h + 4u * nq;
        if (t0 + lane < kSpan)
            __builtin_amdgcn_raw_buffer_store_b32(i0 + t0 + lane, ro, (int)(4u * (t0 + lane)), 0, kAuxStore);
        return;
    }
    // Partly full span: eight rounds of 1024 points (8 groups).  Each lane
    // first interleaves its group's two words into the group's 128 keep bits
    // in point order (four words in the wave's LDS table).  In round e lane l
    // takes the 16 points [16l, 16l+16) of the round, i.e. half-word l & 7 of
    // group 8e + (l >> 3); it writes the indices of its kept points to the
    // stage at their rank, and the wave stores the stage's run with
    // consecutive lanes.  Nothing is done group by group: a wave-wide step
    // per group costs ~30 vector instructions and an LDS round trip.
    uint32_t* mt = stage + kStageIdx;
    {
        const uint32_t a0 = (uint32_t)w0, a1 = (uint32_t)(w0 >> 32);
        const uint32_t b0 = (uint32_t)w1, b1 = (uint32_t)(w1 >> 32);
        uint4 m;
        m.x = spread16(a0 & 0xFFFFu) | (spread16(b0 & 0xFFFFu) << 1);
        m.y = spread16(a0 >> 16) | (spread16(b0 >> 16) << 1);
        m.z = spread16(a1 & 0xFFFFu) | (spread16(b1 & 0xFFFFu) << 1);
        m.w = spread16(a1 >> 16) | (spread16(b1 >> 16) << 1);
        *reinterpret_cast<uint4*>(mt + 4u * lane) = m;
    }
    __builtin_amdgcn_wave_barrier();
    const unsigned long long roundm = __ballot(c != 0u);   // bit g: group g kept a point
    uint32_t P = 0;
    const uint32_t ib = (uint32_t)sb - idx_shift;
#pragma unroll 1
    for (uint32_t e = 0; e < 8u; ++e) {
        if (((roundm >> (8u * e)) & 0xFFull) == 0ull) continue;   // uniform: round empty
        uint32_t m = reinterpret_cast<const uint16_t*>(mt)[64u * e + lane];
        const uint32_t cnt = (uint32_t)__popc(m);
        // exclusive prefix of cnt (<= 16) over the lanes, one bit plane at a time
        uint32_t r = 0, tot = 0;
#pragma unroll
        for (uint32_t b = 0; b < 5u; ++b) {
            const unsigned long long bal = __ballot((cnt >> b) & 1u);
            r += rank_below(bal) << b;
            tot += (uint32_t)__popcll(bal) << b;
        }
        const uint32_t i0 = ib + 1024u * e + 16u * lane;
        while (m) {
            stage[r++] = i0 + (uint32_t)__builtin_ctz(m);
            m &= m - 1u;
        }
        __builtin_amdgcn_wave_barrier();
        for (uint32_t w = 0; w < tot; w += 256u) {
            uint32_t v[4];
#pragma unroll
            for (uint32_t h = 0; h < 4u; ++h) {
                const uint32_t k = w + 64u * h + lane;
                v[h] = k < tot ? stage[k] : 0u;
            }
#pragma unroll
            for (uint32_t h = 0; h < 4u; ++h) {
                const uint32_t k = w + 64u * h + lane;
                const uint32_t pos = P + k;
                if (k < tot && pos < lim) __builtin_amdgcn_raw_buffer_store_b32(v[h], ro, (int)(4u * pos), 0, kAuxStore);
            }
        }
        __builtin_amdgcn_wave_barrier();
        P += tot;
    }
}

// Pass 2 of one set.  Each round the block's waves take consecutive spans
// (one each); the next round's keep bits are loaded before this round's
// survivors are stored, so the loads do not wait behind the stores.
template <int BLOCK, int NV>
__global__ __launch_bounds__(BLOCK) void k_compact(const uint64_t* __restrict__ bits,
                                                   const uint32_t* __restrict__ blkcnt, uint64_t n,
                                                   uint32_t spans, const Poly<NV>* __restrict__ oct,
                                                   uint32_t* __restrict__ out, uint64_t cap, uint64_t* count) {
    constexpr int NW = BLOCK / 64;
    __shared__ __attribute__((aligned(16))) uint32_t sh_stage[NW][kStageWords];
    __shared__ uint64_t sh_part[NW];
    __shared__ uint32_t sh_tot[2][NW];
    const uint32_t lane = lane_id(), wave = threadIdx.x >> 6;
    if (oct->status != 0) {
        if (blockIdx.x == 0 && threadIdx.x == 0) *count = (oct->status == 1) ? kCountNonFinite : kCountInternal;
        return;
    }
    // output offset of this block: the survivors of all earlier blocks
    uint64_t pre = 0;
    for (uint32_t b = threadIdx.x; b < blockIdx.x; b += BLOCK) pre += blkcnt[b];
    pre = wave_sum_u64(pre);
    if (lane == 0) sh_part[wave] = pre;
    __syncthreads();
    uint64_t base = 0;
#pragma unroll
    for (int w = 0; w < NW; ++w) base += sh_part[w];
    base = uniform_u64(base);
    if (blkcnt[blockIdx.x] == 0u) {   // nothing to write; its keep words are not read
        if (blockIdx.x == gridDim.x - 1 && threadIdx.x == 0) *count = base;
        return;
    }

    const uint64_t r0 = (uint64_t)blockIdx.x * spans * kSpan;
    const uint64_t r1 = min<uint64_t>(n, r0 + (uint64_t)spans * kSpan);
    const uint64_t ngroups = (n + 127) / 128;
    auto load_words = [&](uint64_t sb, unsigned long long& w0, unsigned long long& w1) {
        w0 = 0ull;
        w1 = 0ull;
        const uint64_t g = (sb >> 7) + lane;
        if (sb < r1 && g < ngroups) {
            const ulonglong2 v = *reinterpret_cast<const ulonglong2*>(bits + 2 * g);
            w0 = v.x;
            w1 = v.y;
        }
    };
    unsigned long long w0, w1;
    load_words(r0 + (uint64_t)wave * kSpan, w0, w1);
    uint32_t par = 0;
    for (uint64_t rb = r0; rb < r1; rb += (uint64_t)NW * kSpan, par ^= 1u) {
        const uint64_t sb = rb + (uint64_t)wave * kSpan;
        unsigned long long n0, n1;
        load_words(sb + (uint64_t)NW * kSpan, n0, n1);
        const uint32_t c = (uint32_t)(__popcll(w0) + __popcll(w1));
        uint32_t tot = c;
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) tot += (uint32_t)__shfl_xor((int)tot, o, 64);
        if (lane == 0) sh_tot[par][wave] = tot;
        __syncthreads();
        uint64_t mine = base, all = 0;
#pragma unroll
        for (int w = 0; w < NW; ++w) {
            const uint32_t t = sh_tot[par][w];
            if (w < (int)wave) mine += t;
            all += t;
        }
        if (sb < r1) compact_span(w0, w1, sb, uniform_u64(mine), cap, 0u, out, sh_stage[wave]);
        base += all;
        w0 = n0;
        w1 = n1;
    }
    if (blockIdx.x == gridDim.x - 1 && threadIdx.x == 0) *count = base;
}

// ---------------------------------------------------------------------------
// One set, inside test and compaction in one pass (decoupled look-back)
// ---------------------------------------------------------------------------
// Each block takes tiles of one span (kSpan points, 64 groups) in ticket
// order: a block draws the next tile number from an atomic counter, so a
// tile only ever waits for tiles whose blocks have already started, and the
// waits end.  The tile is tested like a k_classify sub-tile (region skip
// from the tile's 16 reduction boxes), its keep words stay in LDS, and its
// survivor offset comes from a decoupled look-back over the tiles before it:
// the tile publishes its count (flag A), wave 0 sums the counts of its
// predecessors back to the nearest one that has published its inclusive
// prefix (flag P), then publishes its own prefix.  Survivors are written by
// compact_span straight from the keep words: no keep bits go through memory
// and the writes of some tiles overlap the reads of others.
//
// st[0] is the ticket counter and st[1 + t] tile t's status word (zeroed
// before the launch): 0 = nothing yet, A | count, P | inclusive prefix.
constexpr uint64_t kLbA = 1ull << 62;
constexpr uint64_t kLbP = 2ull << 62;
constexpr uint64_t kLbValue = kLbA - 1ull;
// Polls of one look-back window before the pass gives up (a tile's
// predecessors have all started, so the waits end; this only turns a defect
// into an error instead of a hang).
constexpr uint32_t kLbSpinLimit = 1u << 18;

__device__ __forceinline__ uint64_t lb_load(const unsigned long long* p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void lb_store(unsigned long long* p, uint64_t v) {
    __hip_atomic_store(p, (unsigned long long)v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Exclusive prefix of tile t's count (wave 0, every lane gets it); `ok`
// turns false if a window's predecessors did not publish within the limit.
__device__ __forceinline__ uint64_t lookback(unsigned long long* __restrict__ st, uint32_t t, uint64_t total,
                                             bool& ok) {
    const uint32_t lane = lane_id();
    if (t == 0u) {
        if (lane == 0) lb_store(st + 1, kLbP | total);
        return 0ull;
    }
    if (lane == 0) lb_store(st + 1 + t, kLbA | total);
    uint64_t excl = 0;
    int64_t j = (int64_t)t - 1;   // window: tiles j, j - 1, ..., j - 63 (lane order)
    for (;;) {
        const int64_t i = j - (int64_t)lane;
        uint64_t v = (i >= 0) ? lb_load(st + 1 + i) : kLbP;   // before tile 0: prefix 0
        uint32_t spins = 0;
        for (;;) {
            // lanes up to the nearest inclusive prefix must have published
            const unsigned long long pm = __ballot((v >> 62) == 2ull);
            const unsigned long long zm = __ballot((v >> 62) == 0ull);
            const unsigned long long need = pm ? ((2ull << (__ffsll((long long)pm) - 1)) - 1ull) : ~0ull;
            if ((zm & need) == 0ull) break;
            if (++spins > kLbSpinLimit) {
                ok = false;
                break;
            }
            if ((v >> 62) == 0ull) v = lb_load(st + 1 + i);
        }
        const unsigned long long pm = __ballot((v >> 62) == 2ull);
        if (pm != 0ull) {
            const uint32_t p = (uint32_t)(__ffsll((long long)pm) - 1);
            excl += wave_sum_u64(lane <= p ? (v & kLbValue) : 0ull);
            break;
        }
        excl += wave_sum_u64(v & kLbValue);
        j -= 64;
    }
    excl = uniform_u64(excl);
    if (lane == 0) lb_store(st + 1 + t, kLbP | (excl + total));
    return excl;
}

template <int BLOCK, int PPT, bool VEC4, int NV>
__global__ __launch_bounds__(BLOCK) __attribute__((amdgpu_waves_per_eu(4, 8))) void k_filter1p(
    const float2* __restrict__ pts, uint64_t n, const Poly<NV>* __restrict__ oct, const float4* __restrict__ box,
    uint64_t nbox, unsigned long long* __restrict__ st, uint32_t* __restrict__ out, uint64_t cap,
    uint64_t* count, unsigned long long* loaded) {
    constexpr int NP = PPT / 2;
    constexpr int NW = BLOCK / 64;
    constexpr uint32_t ST = BLOCK * PPT;
    static_assert(ST == kSpan, "a tile is one span");
    static_assert(NW * NP == 64, "the tile's 64 groups: pair slot j of wave w is group j * NW + w");
    __shared__ __attribute__((aligned(16))) uint32_t sh_stage[kStageWords];
    __shared__ unsigned long long sh_kw[2 * 64];
    __shared__ uint32_t sh_w[NW], sh_g[NW];
    __shared__ uint32_t sh_t, sh_skip;
    const uint32_t lane = lane_id();
    const uint32_t wave = uniform_u32(threadIdx.x >> 6);
    const uint32_t ntiles = (uint32_t)((n + ST - 1) / ST);
    if (oct->status != 0) {
        if (blockIdx.x == 0 && threadIdx.x == 0) *count = (oct->status == 1) ? kCountNonFinite : kCountInternal;
        return;
    }
    PolyK<NV>* ok = as_const(oct);
    const bool skipon = box != nullptr && ok->mode == 1 && ok->skip != 0;
    if (threadIdx.x == 0) sh_t = atomicAdd(reinterpret_cast<unsigned int*>(st), 1u);
    __syncthreads();
    const uint32_t t = sh_t;
    if (t >= ntiles) return;   // more blocks than tiles: nothing drawn
    const uint64_t sb = (uint64_t)t * ST;
    const bool full = sb + ST <= n;
    // region skip: the tile's 16 boxes (4 per 2048-point reduction chunk)
    if (wave == 0) {
        bool pass = false;
        if (skipon && full && lane < 16u) {
            const uint64_t bi = (uint64_t)t * 16u + lane;
            pass = bi < nbox && box_inside<NV>(box[bi], ok);
        }
        const unsigned long long m = __ballot(pass);
        if (lane == 0) sh_skip = (uint32_t)m;
    }
    __syncthreads();
    const uint32_t tskip = sh_skip;
    uint32_t skipm = 0;
#pragma unroll
    for (int j = 0; j < NP; ++j) {
        const uint32_t g = (uint32_t)(j * NW) + wave;   // group of the tile
        skipm |= ((tskip >> ((g >> 4) * 4u + (g & 3u))) & 1u) << j;
    }
    uint32_t total = 0;
    unsigned long long m0 = 0ull, m1 = 0ull;
    if (tskip != 0xFFFFu) {
        const EdgeRegsN<NV> ek = load_edges(oct);
        classify_tile<BLOCK, PPT, VEC4, NV>(oct, ek, pts, 0, n, sb, full ? skipm : 0u, m0, m1, total);
    }
    if (lane < (uint32_t)NP) {
        const uint32_t g = lane * NW + wave;
        sh_kw[2 * g] = m0;
        sh_kw[2 * g + 1] = m1;
    }
    if (lane == 0) {
        sh_w[wave] = total;
        sh_g[wave] = (tskip != 0xFFFFu) ? (uint32_t)(NP - __popc(full ? skipm : 0u)) : 0u;
    }
    __syncthreads();
    if (wave != 0) return;
    uint64_t sum = 0;
    uint32_t groups = 0;
#pragma unroll
    for (int w = 0; w < NW; ++w) {
        sum += sh_w[w];
        groups += sh_g[w];
    }
    bool good = true;
    const uint64_t excl = lookback(st, t, sum, good);
    if (lane == 0) {
        if (loaded && groups) atomicAdd(loaded, (unsigned long long)groups);
        if (!good) *count = kCountInternal;
        else if (t == ntiles - 1u) *count = excl + sum;
    }
    if (sum != 0ull && good)
        compact_span(sh_kw[2 * lane], sh_kw[2 * lane + 1], sb, excl, cap, 0u, out, sh_stage);
}

template <bool VEC4>
__global__ __launch_bounds__(256) void k_flags(const float2* __restrict__ pts, uint64_t n,
                                               const Octagon* __restrict__ oct, uint8_t* flags) {
    const bool bad = oct->status != 0;
    const EdgeRegs ek = load_edges(oct);
    for (uint64_t i = (uint64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (uint64_t)gridDim.x * 256) {
        if (bad) {
            flags[i] = 2;
            continue;
        }
        const float2 p = pts[i];
        flags[i] = keep_point(oct, ek, p.x, p.y) ? 1 : 0;
    }
}

__global__ void k_write_count(uint64_t* count, uint64_t value) { *count = value; }

__global__ __launch_bounds__(256) void k_gather(const float2* __restrict__ pts,
                                                const uint32_t* __restrict__ surv,
                                                const uint64_t* __restrict__ count, uint64_t cap,
                                                uint64_t n, float2* __restrict__ out) {
    const uint64_t c = *count;
    if (c > cap) return;   // error sentinels, or more survivors than staged
    for (uint64_t i = (uint64_t)blockIdx.x * 256 + threadIdx.x; i < c; i += (uint64_t)gridDim.x * 256) {
        const uint32_t k = surv[i];
        out[i] = (k < n) ? pts[k] : make_float2(__builtin_nanf(""), __builtin_nanf(""));
    }
}

// ---------------------------------------------------------------------------
// kernels: many sets in one graph of five launches
// ---------------------------------------------------------------------------
// Sets are CSR ranges of one point array (or a list of (begin, count)
// segments).  Launch 1 (plan, one block) cuts every set into reduction tiles
// of kBatchRT points and work items of kBatchItem points (both counted from
// the set's start rounded down to 16 points) and computes their prefix counts.  Launch 2
// streams all reduction tiles and writes one partial record per tile (and
// the tiles' region-skip boxes); launch 3 merges each set's records and
// builds its octagon (one wave per set); launch 4 runs the inside test on
// every work item (keep bits + one count per item) and launch 5 compacts
// every item at its offset inside its set.  Cross-block results only flow
// across launch boundaries, so no kernel needs a device-wide fence.

// A set's tiles and work items are counted from its first point rounded
// down to a multiple of 16 points (128 bytes), so that every full chunk a
// wave loads is line-aligned (measured on one 1e8 set: 16-byte-aligned
// chunks that straddle lines cost up to 8 % in the reduction); the points
// before the set's start are masked like any point outside the set.
constexpr uint64_t kBatchAlign = 15;
constexpr uint32_t kBatchRChunks = 16;
constexpr uint32_t kBatchRT = kRBlock * kRG * 2 * kBatchRChunks;   // reduction tile (points)
constexpr uint32_t kBatchTileBoxes = 4 * kBatchRChunks;             // region-skip boxes per tile

// Last set s with start[s] <= k (start non-decreasing, start[0] == 0).
__device__ __forceinline__ uint32_t set_of(const SetInfo* __restrict__ sets, uint32_t S, uint32_t k, bool f) {
    uint32_t lo = 0, hi = S - 1;
    while (lo < hi) {
        const uint32_t mid = (lo + hi + 1) >> 1;
        const uint32_t st = f ? sets[mid].f_tile0 : sets[mid].r_tile0;
        if (st <= k) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

// The sets of a block's next kAhead tiles (or work items) r0, r0 + step, ...
// (those below lim), looked up by kAhead lanes at once: one round of binary
// searches, all in flight together, instead of one dependent search per
// tile.  sh[k] holds the set of tile r0 + k * step.
constexpr uint32_t kAhead = 64;
constexpr uint32_t kTicketTiles = 2;   // reduction tiles per ticket
__device__ __forceinline__ void sets_ahead(const SetInfo* __restrict__ sets, uint32_t S, uint32_t r0, uint32_t step,
                                           uint32_t lim, bool f, uint32_t* sh) {
    __syncthreads();   // the previous round's readers of sh are done
    if (threadIdx.x < kAhead) {
        const uint64_t r = (uint64_t)r0 + (uint64_t)threadIdx.x * step;
        sh[threadIdx.x] = (r < lim) ? set_of(sets, S, (uint32_t)r, f) : 0u;
    }
    __syncthreads();
}

// Last set s with start[s] <= k, found by one wave: each round cuts the
// remaining range into 64 parts, one lane reads the first start of each, and
// the last part that starts at or before k holds the answer (two rounds of
// loads for up to 4096 sets, three up to 2^18).  Every lane returns it.
__device__ __forceinline__ uint32_t set_of_wave(const SetInfo* __restrict__ sets, uint32_t S, uint32_t k, bool f) {
    uint32_t lo = 0, span = S;
    while (span > 1u) {
        const uint32_t step = (span + 63u) >> 6;
        const uint32_t idx = lo + lane_id() * step;
        const bool ok = (idx < lo + span) && (f ? sets[idx].f_tile0 : sets[idx].r_tile0) <= k;
        const uint64_t m = __ballot(ok);   // lane 0 always holds: start[lo] <= k
        const uint32_t j = 63u - (uint32_t)__builtin_clzll(m);
        lo += j * step;
        span = min(step, span - j * step);
    }
    return lo;
}

// Exclusive scan of one value per thread over a block of 1024 threads;
// returns the exclusive prefix and adds the block total to *carry.
__device__ __forceinline__ uint32_t block_exclusive_scan(uint32_t v, uint32_t* sh, uint32_t* carry) {
    const uint32_t t = threadIdx.x;
    sh[t] = v;
    __syncthreads();
    for (uint32_t o = 1; o < 1024; o <<= 1) {
        const uint32_t u = (t >= o) ? sh[t - o] : 0u;
        __syncthreads();
        sh[t] += u;
        __syncthreads();
    }
    const uint32_t r = *carry + sh[t] - v;
    const uint32_t tot = sh[1023];
    __syncthreads();
    if (t == 0) *carry += tot;
    __syncthreads();
    return r;
}

// Set s spans [b, e): CSR offsets (b, e) = (off[s], off[s+1]), or a segment
// list of (begin, count) pairs, (b, e) = (seg[2s], seg[2s] + seg[2s+1]).
template <bool SEG>
__device__ __forceinline__ void set_span(const uint64_t* __restrict__ a, uint32_t s, uint64_t& b, uint64_t& e) {
    if (SEG) {
        b = a[2ull * s];
        e = b + a[2ull * s + 1];
    } else {
        b = a[s];
        e = a[s + 1];
    }
}

template <bool SEG>
__global__ __launch_bounds__(1024) void k_batch_plan(const uint64_t* __restrict__ off, uint32_t S,
                                                     SetInfo* sets, BatchTotals* tot, uint64_t* counts,
                                                     uint32_t max_ftiles, uint32_t max_rtiles, uint64_t n_total,
                                                     uint32_t ft) {
    __shared__ uint32_t sh_scan[1024];
    __shared__ uint32_t sh_carry[2];
    const uint32_t t = threadIdx.x;
    if (t == 0) sh_carry[0] = sh_carry[1] = 0u;
    // CSR: offsets start at 0, end at n_total and never decrease.  Segments:
    // each ends within n_total, after its begin, and before the next begins
    // (ascending, disjoint).
    int bad = 0;
    for (uint32_t s = t; s < S; s += 1024) {
        uint64_t b, e;
        set_span<SEG>(off, s, b, e);
        bad |= (e < b || e > n_total) ? 1 : 0;
        if (SEG && s + 1 < S) bad |= (e > off[2ull * (s + 1)]) ? 1 : 0;
    }
    if (!SEG && t == 0) bad |= (off[0] != 0ull || off[S] != n_total) ? 1 : 0;
    bad = __syncthreads_or(bad);
    if (bad) {
        // every set empty for the later launches, every count flagged
        for (uint32_t s = t; s < S; s += 1024) {
            counts[s] = kCountBadOffsets;
            sets[s].begin = 0ull;
            sets[s].n = 0ull;
            sets[s].r_tiles = 0u;
            sets[s].f_tiles = 0u;
            sets[s].r_tile0 = 0u;
            sets[s].f_tile0 = 0u;
        }
        if (t == 0) {
            tot->r_tiles = 0u;
            tot->f_tiles = 0u;
            tot->r_next = 0u;
        }
        return;
    }
    for (uint32_t base = 0; base < S; base += 1024) {
        const uint32_t s = base + t;
        uint32_t rt = 0, fc = 0;
        uint64_t b = 0, n = 0;
        if (s < S) {
            uint64_t e;
            set_span<SEG>(off, s, b, e);
            n = e - b;
            const uint64_t al = b & ~kBatchAlign;
            rt = n ? (uint32_t)((b + n - al + kBatchRT - 1) / kBatchRT) : 0u;
            fc = n ? (uint32_t)((b + n - al + ft - 1) / ft) : 0u;
        }
        const uint32_t r0 = block_exclusive_scan(rt, sh_scan, &sh_carry[0]);
        const uint32_t f0 = block_exclusive_scan(fc, sh_scan, &sh_carry[1]);
        if (s < S) {
            sets[s].begin = b;
            sets[s].n = n;
            sets[s].r_tiles = rt;
            sets[s].f_tiles = fc;
            sets[s].r_tile0 = r0;
            sets[s].f_tile0 = f0;
            if (n == 0) counts[s] = 0ull;
        }
    }
    const uint32_t rtiles = sh_carry[0], ftiles = sh_carry[1];
    const bool fits = ftiles <= max_ftiles && rtiles <= max_rtiles;
    if (t == 0) {
        tot->r_tiles = fits ? rtiles : 0u;
        tot->f_tiles = fits ? ftiles : 0u;
        tot->r_next = 0u;
    }
}

template <bool VEC4>
// Four waves per SIMD, 128 registers: the streaming loop keeps two chunks of
// loads in flight per wave (two register sets) to make up for the low
// occupancy.  At 5 or 6 waves per SIMD the kernel spills (54-124 registers),
// and at 8 it spilled inside the streaming loop even with one chunk in flight.
__global__ __launch_bounds__(kRBlock) __attribute__((amdgpu_waves_per_eu(4, 8))) void k_batch_reduce(
    const float2* __restrict__ pts, uint32_t S, const SetInfo* __restrict__ sets,
    BatchTotals* __restrict__ tot, unsigned long long* __restrict__ part, float4* __restrict__ box) {
    // Tiles are handed out by ticket, kTicketTiles consecutive ones at a
    // time, so blocks that drew small tiles (the last tile of a set) draw
    // again instead of the grid waiting on a fixed share per block.  The
    // next ticket is drawn before the current tiles are streamed.
    const uint32_t rtiles = tot->r_tiles;
    __shared__ uint32_t sh_set[kTicketTiles];
    __shared__ uint32_t sh_tk[2];
    __shared__ unsigned long long rec[9];
    if (threadIdx.x == 0) sh_tk[0] = atomicAdd(&tot->r_next, kTicketTiles);
    for (uint32_t round = 0;; ++round) {
        __syncthreads();   // this round's ticket is visible
        const uint32_t r0 = sh_tk[round & 1u];
        if (r0 >= rtiles) break;
        if (threadIdx.x == 0) sh_tk[(round + 1) & 1u] = atomicAdd(&tot->r_next, kTicketTiles);
        // the sets of this ticket's tiles, one wave per tile
        static_assert(kTicketTiles <= kRBlock / 64, "one wave per tile of a ticket");
        __syncthreads();   // the previous round's readers of sh_set are done
        {
            const uint32_t w = threadIdx.x >> 6;
            if (w < kTicketTiles && r0 + w < rtiles) {
                const uint32_t s = set_of_wave(sets, S, r0 + w, false);
                if (lane_id() == 0) sh_set[w] = s;
            }
        }
        __syncthreads();
        for (uint32_t k = 0; k < kTicketTiles && r0 + k < rtiles; ++k) {
            const uint32_t r = r0 + k;
            const uint32_t s = uniform_u32(sh_set[k]);
            const uint64_t b = sets[s].begin, n = sets[s].n;
            const uint64_t tb = (b & ~kBatchAlign) + (uint64_t)(r - sets[s].r_tile0) * kBatchRT;
            reduce_points<kRBlock, kRG, VEC4, false, true>(pts, b, b + n, tb, 0u, 1u, kBatchRChunks, rec,
                                                     box ? box + (uint64_t)r * kBatchTileBoxes : nullptr);
            if (threadIdx.x < 9) part[(uint64_t)r * 9 + threadIdx.x] = rec[threadIdx.x];
        }
    }
}

// One wave per set: merge the set's partial records, build its octagon.
__global__ __launch_bounds__(256) void k_batch_setup(const float2* __restrict__ pts, uint32_t S,
                                                     const SetInfo* __restrict__ sets,
                                                     const unsigned long long* __restrict__ part,
                                                     Octagon* octs, uint64_t* counts) {
    const uint32_t lane = lane_id();
    const uint32_t nwaves = gridDim.x * 4;
    for (uint32_t s = blockIdx.x * 4 + (threadIdx.x >> 6); s < S; s += nwaves) {
        const uint64_t n = sets[s].n;
        if (n == 0) continue;
        const uint32_t r0 = sets[s].r_tile0, rt = sets[s].r_tiles;
        unsigned long long m[9];
#pragma unroll
        for (int j = 0; j < 9; ++j) m[j] = 0ull;
        for (uint32_t r = lane; r < rt; r += 64) {
#pragma unroll
            for (int j = 0; j < 9; ++j) {
                const unsigned long long v = part[(uint64_t)(r0 + r) * 9 + j];
                m[j] = (j == 8) ? (m[j] | v) : max(m[j], v);
            }
        }
        unsigned long long mine = 0ull, nf = 0ull;
#pragma unroll
        for (int j = 0; j < 9; ++j) {
            unsigned long long v = m[j];
#pragma unroll
            for (int o = 32; o > 0; o >>= 1) {
                const uint32_t lo = (uint32_t)__shfl_xor((int)(uint32_t)v, o, 64);
                const uint32_t hi = (uint32_t)__shfl_xor((int)(uint32_t)(v >> 32), o, 64);
                const unsigned long long u = ((unsigned long long)hi << 32) | lo;
                v = (j == 8) ? (v | u) : max(v, u);
            }
            if (j == (int)(lane & 7u)) mine = v;
            if (j == 8) nf = v;
        }
        const int st = setup_octagon(pts, sets[s].begin, n, mine, (uint32_t)nf, &octs[s]);
        if (lane == 0 && st != 0) counts[s] = (st == 1) ? kCountNonFinite : kCountInternal;
    }
}

// Two-pass compaction of a batch.  Every set is cut into work items of
// kBatchItem points counted from its start rounded down to 16 points
// (SetInfo f_tiles / f_tile0 count items).  Item i owns kBatchItem/64 words
// of keep bits (same layout as the single-set pass, groups counted from the
// item's first point) and one survivor count.
constexpr uint32_t kBatchItem = 4 * kSpan;

template <int BLOCK, int PPT, bool VEC4>
__global__ __launch_bounds__(BLOCK) __attribute__((amdgpu_waves_per_eu(6, 8))) void k_batch_classify(
    const float2* __restrict__ pts, uint32_t S, const SetInfo* __restrict__ sets,
    const Octagon* __restrict__ octs, const BatchTotals* __restrict__ tot, uint64_t* __restrict__ bits,
    uint32_t* __restrict__ blkcnt, const float4* __restrict__ box) {
    constexpr int NP = PPT / 2;
    constexpr int NW = BLOCK / 64;
    constexpr uint32_t ST = BLOCK * PPT;
    static_assert(kBatchItem % ST == 0, "sub-tiles tile an item");
    static_assert(kBatchItem / kBatchRT * kBatchTileBoxes == 64, "one skip word per item");
    __shared__ uint32_t sh_w[NW];
    const uint32_t lane = lane_id(), wave = threadIdx.x >> 6;
    const uint32_t items = tot->f_tiles;
    __shared__ uint32_t sh_set[kAhead];
    for (uint64_t i0 = blockIdx.x; i0 < items; i0 += (uint64_t)gridDim.x * kAhead)
    for (uint32_t k = 0; k < kAhead; ++k) {
        if (k == 0) sets_ahead(sets, S, (uint32_t)i0, gridDim.x, items, true, sh_set);
        const uint64_t ii = i0 + (uint64_t)k * gridDim.x;
        if (ii >= items) break;
        const uint32_t it = (uint32_t)ii;
        const uint32_t s = uniform_u32(sh_set[k]);
        const Octagon* o = &octs[s];
        const EdgeRegs ek = load_edges(o);
        uint32_t total = 0;
        if (o->status == 0) {
            const uint64_t b = sets[s].begin, hi = b + sets[s].n;
            const uint32_t li = it - sets[s].f_tile0;
            const uint64_t r0 = (b & ~kBatchAlign) + (uint64_t)li * kBatchItem;
            const uint64_t r1 = min<uint64_t>(hi, r0 + kBatchItem);
            uint64_t* ib = bits + (uint64_t)it * (kBatchItem / 64);
            // Region skip: the item's 64 groups of 512 points have the 64
            // consecutive boxes of its four reduction tiles; lane l tests
            // box l.  The corner test uses the FP32 edge coefficients: d > 2
            // at a point of the bounding box means an exact edge value above
            // 24 u M there, and edge values are affine, so every point of a
            // box whose corners all pass is discarded by the binary64 rule.
            unsigned long long word = 0ull;
            if (box != nullptr && ek.mode == 1 && ek.fast) {
                const uint32_t bl = li * 64u + lane;
                bool pass = false;
                if (bl < sets[s].r_tiles * kBatchTileBoxes) {
                    const float4 bx = box[(uint64_t)sets[s].r_tile0 * kBatchTileBoxes + bl];
                    pass = (edge_min(ek, bx.x, bx.z) > 2.0f) & (edge_min(ek, bx.y, bx.z) > 2.0f) &
                           (edge_min(ek, bx.x, bx.w) > 2.0f) & (edge_min(ek, bx.y, bx.w) > 2.0f);
                }
                word = __ballot(pass);
            }
            for (uint64_t sb = r0; sb < r1; sb += ST) {
                uint32_t skipm = 0;
                if (word != 0ull) {
#pragma unroll
                    for (int j = 0; j < NP; ++j) {
                        const uint32_t gg = (uint32_t)((sb - r0) >> 7) + (uint32_t)(j * NW) + wave;
                        skipm |= (uint32_t)((word >> ((gg >> 4) * 4u + (gg & 3u))) & 1ull) << j;
                    }
                }
                unsigned long long m0, m1;
                classify_tile<BLOCK, PPT, VEC4, 8>(o, ek, pts, b, hi, sb, skipm, m0, m1, total);
                const uint32_t g = (uint32_t)((sb - r0) >> 7) + lane * NW + wave;
                if (lane < (uint32_t)NP) {
                    ulonglong2 v;
                    v.x = m0;
                    v.y = m1;
                    *reinterpret_cast<ulonglong2*>(ib + 2 * g) = v;
                }
            }
        }
        if (lane == 0) sh_w[wave] = total;
        __syncthreads();
        if (threadIdx.x == 0) {
            uint32_t sum = 0;
#pragma unroll
            for (int w = 0; w < NW; ++w) sum += sh_w[w];
            blkcnt[it] = sum;
        }
        __syncthreads();
    }
}

// Pass 2 of a batch: one work item (kBatchItem = 4 spans) per block and
// round, one span per wave.
template <int BLOCK>
__global__ __launch_bounds__(BLOCK) void k_batch_compact(uint32_t S, const SetInfo* __restrict__ sets,
                                                         const Octagon* __restrict__ octs,
                                                         const BatchTotals* __restrict__ tot,
                                                         const uint64_t* __restrict__ bits,
                                                         const uint32_t* __restrict__ blkcnt,
                                                         uint32_t* __restrict__ surv, uint64_t* counts) {
    constexpr int NW = BLOCK / 64;
    static_assert(NW * kSpan == kBatchItem, "one span per wave");
    __shared__ __attribute__((aligned(16))) uint32_t sh_stage[NW][kStageWords];
    __shared__ uint64_t sh_part[NW];
    __shared__ uint32_t sh_tot[NW];
    const uint32_t lane = lane_id(), wave = threadIdx.x >> 6;
    const uint32_t items = tot->f_tiles;
    __shared__ uint32_t sh_set[kAhead];
    for (uint64_t i0 = blockIdx.x; i0 < items; i0 += (uint64_t)gridDim.x * kAhead)
    for (uint32_t k = 0; k < kAhead; ++k) {
        if (k == 0) sets_ahead(sets, S, (uint32_t)i0, gridDim.x, items, true, sh_set);
        const uint64_t ii = i0 + (uint64_t)k * gridDim.x;
        if (ii >= items) break;
        const uint32_t it = (uint32_t)ii;
        const uint32_t s = uniform_u32(sh_set[k]);
        const uint32_t first = sets[s].f_tile0, li = it - first;
        const int ost = octs[s].status;
        if (ost != 0) {
            if (li == 0 && threadIdx.x == 0) counts[s] = (ost == 1) ? kCountNonFinite : kCountInternal;
            continue;
        }
        const uint64_t b = sets[s].begin, n = sets[s].n;
        const uint64_t r0 = (b & ~kBatchAlign) + (uint64_t)li * kBatchItem;
        const uint64_t r1 = min<uint64_t>(b + n, r0 + kBatchItem);
        const uint64_t sb = r0 + (uint64_t)wave * kSpan;
        // this wave's span words (issued before the offset sums below)
        unsigned long long w0 = 0ull, w1 = 0ull;
        if (sb + 128ull * lane < r1) {
            const ulonglong2 v = *reinterpret_cast<const ulonglong2*>(
                bits + (uint64_t)it * (kBatchItem / 64) + 2 * ((uint64_t)wave * kSpanGroups + lane));
            w0 = v.x;
            w1 = v.y;
        }
        // offset inside the set: survivors of the set's earlier items
        uint64_t pre = 0;
        for (uint32_t k = threadIdx.x; k < li; k += BLOCK) pre += blkcnt[first + k];
        pre = wave_sum_u64(pre);
        uint32_t t = (uint32_t)(__popcll(w0) + __popcll(w1));
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) t += (uint32_t)__shfl_xor((int)t, o, 64);
        __syncthreads();   // the previous item's reads of sh_part / sh_tot are done
        if (lane == 0) {
            sh_part[wave] = pre;
            sh_tot[wave] = t;
        }
        __syncthreads();
        uint64_t base = 0, mine = 0;
#pragma unroll
        for (int w = 0; w < NW; ++w) {
            base += sh_part[w];
            if (w < (int)wave) mine += sh_tot[w];
        }
        uint64_t all = base;
#pragma unroll
        for (int w = 0; w < NW; ++w) all += sh_tot[w];
        if (sb < r1)
            compact_span(w0, w1, sb, uniform_u64(base + mine), n, (uint32_t)b, surv + b, sh_stage[wave]);
        if (li == sets[s].f_tiles - 1 && threadIdx.x == 0) counts[s] = all;
    }
}

bool is_vec4(const float2* p) { return ((uintptr_t)p & 15u) == 0u; }

}  // namespace

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------

uint32_t reduce_chunk_points() { return kRChunk; }

bool shape_supported(Shape s) {
    return (s.block == 256 || s.block == 512) && (s.ppt == 8 || s.ppt == 16);
}

hipError_t launch_reduce(const float2* pts, uint64_t n, unsigned long long* part, float4* box, int grid,
                         hipStream_t stream, unsigned long long* zero, uint32_t nzero) {
    if (grid < 1 || grid > kReduceMaxGrid || (nzero > 0u && zero == nullptr)) return hipErrorInvalidValue;
    if (is_vec4(pts))
        hipLaunchKernelGGL(k_reduce<true>, dim3(grid), dim3(kRBlock), 0, stream, pts, n, part, box, zero, nzero);
    else
        hipLaunchKernelGGL(k_reduce<false>, dim3(grid), dim3(kRBlock), 0, stream, pts, n, part, box, zero, nzero);
    return hipGetLastError();
}

hipError_t launch_setup(const float2* pts, uint64_t n, Octagon* oct, const unsigned long long* part,
                        uint32_t nblocks, hipStream_t stream) {
    if (nblocks < 1 || nblocks > (uint32_t)kReduceMaxGrid) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_setup<8>, dim3(1), dim3(512), 0, stream, pts, n, oct, part, nblocks);
    return hipGetLastError();
}

int reduce16_grid(uint64_t n, int cus) {
    const uint64_t nch = (n + kRChunk - 1) / kRChunk;
    const uint64_t g = std::min<uint64_t>((uint64_t)cus * kR16PerCU, (uint64_t)kReduceMaxGrid);
    return (int)std::max<uint64_t>(1, std::min<uint64_t>(nch, g));
}

hipError_t launch_reduce16(const float2* pts, uint64_t n, unsigned long long* part, float4* box, int grid,
                           hipStream_t stream) {
    if (grid < 1 || grid > kReduceMaxGrid) return hipErrorInvalidValue;
    if (is_vec4(pts))
        hipLaunchKernelGGL(k_reduce16<true>, dim3(grid), dim3(kRBlock), 0, stream, pts, n, part, box);
    else
        hipLaunchKernelGGL(k_reduce16<false>, dim3(grid), dim3(kRBlock), 0, stream, pts, n, part, box);
    return hipGetLastError();
}

hipError_t launch_setup16(const float2* pts, uint64_t n, Poly16* poly, const unsigned long long* part,
                          uint32_t nblocks, hipStream_t stream) {
    if (nblocks < 1 || nblocks > (uint32_t)kReduceMaxGrid) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_setup<16>, dim3(1), dim3(1024), 0, stream, pts, n, poly, part, nblocks);
    return hipGetLastError();
}

uint32_t compact_span_points() { return kSpan; }

FilterPlan plan_filter(uint64_t n, int cus, Shape shape, int per_cu, int reduce_grid_max) {
    FilterPlan p;
    const uint64_t nch = (n + kRChunk - 1) / kRChunk;
    // 4 blocks per CU: measured faster than 2, 6, 8, 12 or 16 (1e8 points:
    // 122 us against 130-136 us with 8)
    const uint64_t want = reduce_grid_max > 0 ? (uint64_t)reduce_grid_max : (uint64_t)cus * 4;
    const uint64_t g = std::min<uint64_t>(want, (uint64_t)kReduceMaxGrid);
    p.reduce_grid = (int)std::max<uint64_t>(1, std::min<uint64_t>(nch, g));
    p.shape = classify_shape_supported(shape) ? shape : Shape{512, 16};
    const uint64_t nspans = (n + kSpan - 1) / kSpan;
    const int pc = per_cu > 0 ? per_cu : (p.shape.block >= 512 ? 3 : 6);
    const uint64_t target = std::min<uint64_t>((uint64_t)cus * pc, kFilterMaxBlocks);
    p.spans = (uint32_t)((nspans + target - 1) / target);
    p.grid = (int)((nspans + p.spans - 1) / p.spans);
    p.bits_words = 2 * ((n + 127) / 128);
    p.boxes = 4 * nch;
    return p;
}

bool classify_shape_supported(Shape s) {
    return shape_supported(s) && kSpan % (uint32_t)(s.block * s.ppt) == 0u;
}

#define HULLF_CLASSIFY_SHAPES(X) X(256, 8) X(256, 16) X(512, 8) X(512, 16)

template <int NV>
hipError_t classify_launch(const float2* pts, uint64_t n, const Poly<NV>* oct, uint32_t spans, uint64_t* bits,
                           uint32_t* blkcnt, const float4* box, uint64_t nbox, unsigned long long* loaded,
                           Shape shape, int grid, hipStream_t stream) {
    const bool v = is_vec4(pts);
#define X(B, P)                                                                                           \
    if (shape.block == B && shape.ppt == P) {                                                             \
        if (v)                                                                                            \
            hipLaunchKernelGGL((k_classify<B, P, true, NV>), dim3(grid), dim3(B), 0, stream, pts, n, oct, spans, \
                               bits, blkcnt, box, nbox, loaded);                                          \
        else                                                                                              \
            hipLaunchKernelGGL((k_classify<B, P, false, NV>), dim3(grid), dim3(B), 0, stream, pts, n, oct,   \
                               spans, bits, blkcnt, box, nbox, loaded);                                   \
        return hipGetLastError();                                                                         \
    }
    HULLF_CLASSIFY_SHAPES(X)
#undef X
    return hipErrorInvalidValue;
}

hipError_t launch_classify(const float2* pts, uint64_t n, const Octagon* oct, uint32_t spans, uint64_t* bits,
                           uint32_t* blkcnt, const float4* box, uint64_t nbox, unsigned long long* loaded,
                           Shape shape, int grid, hipStream_t stream) {
    return classify_launch<8>(pts, n, oct, spans, bits, blkcnt, box, nbox, loaded, shape, grid, stream);
}

hipError_t launch_classify(const float2* pts, uint64_t n, const Poly16* poly, uint32_t spans, uint64_t* bits,
                           uint32_t* blkcnt, const float4* box, uint64_t nbox, unsigned long long* loaded,
                           Shape shape, int grid, hipStream_t stream) {
    return classify_launch<16>(pts, n, poly, spans, bits, blkcnt, box, nbox, loaded, shape, grid, stream);
}

template <int NV>
hipError_t compact_launch(const uint64_t* bits, const uint32_t* blkcnt, uint64_t n, uint32_t spans,
                          const Poly<NV>* oct, uint32_t* out, uint64_t cap, uint64_t* count, int block, int grid,
                          hipStream_t stream) {
    if (block == 1024)
        hipLaunchKernelGGL((k_compact<1024, NV>), dim3(grid), dim3(1024), 0, stream, bits, blkcnt, n, spans, oct,
                           out, cap, count);
    else if (block == 512)
        hipLaunchKernelGGL((k_compact<512, NV>), dim3(grid), dim3(512), 0, stream, bits, blkcnt, n, spans, oct, out,
                           cap, count);
    else
        hipLaunchKernelGGL((k_compact<256, NV>), dim3(grid), dim3(256), 0, stream, bits, blkcnt, n, spans, oct, out,
                           cap, count);
    return hipGetLastError();
}

hipError_t launch_compact(const uint64_t* bits, const uint32_t* blkcnt, uint64_t n, uint32_t spans,
                          const Octagon* oct, uint32_t* out, uint64_t cap, uint64_t* count, int block, int grid,
                          hipStream_t stream) {
    return compact_launch<8>(bits, blkcnt, n, spans, oct, out, cap, count, block, grid, stream);
}

hipError_t launch_compact(const uint64_t* bits, const uint32_t* blkcnt, uint64_t n, uint32_t spans,
                          const Poly16* poly, uint32_t* out, uint64_t cap, uint64_t* count, int block, int grid,
                          hipStream_t stream) {
    return compact_launch<16>(bits, blkcnt, n, spans, poly, out, cap, count, block, grid, stream);
}

uint32_t filter1p_tiles(uint64_t n) { return (uint32_t)((n + kSpan - 1) / kSpan); }

hipError_t launch_filter1p(const float2* pts, uint64_t n, const Octagon* oct, const float4* box, uint64_t nbox,
                           unsigned long long* st, uint32_t* out, uint64_t cap, uint64_t* count,
                           unsigned long long* loaded, hipStream_t stream) {
    const uint32_t tiles = filter1p_tiles(n);
    if (tiles == 0u) return hipSuccess;
    if (is_vec4(pts))
        hipLaunchKernelGGL((k_filter1p<512, 16, true, 8>), dim3(tiles), dim3(512), 0, stream, pts, n, oct, box, nbox,
                           st, out, cap, count, loaded);
    else
        hipLaunchKernelGGL((k_filter1p<512, 16, false, 8>), dim3(tiles), dim3(512), 0, stream, pts, n, oct, box,
                           nbox, st, out, cap, count, loaded);
    return hipGetLastError();
}

hipError_t launch_flags(const float2* pts, uint64_t n, const Octagon* oct, uint8_t* flags, int grid,
                        hipStream_t stream) {
    hipLaunchKernelGGL(k_flags<true>, dim3(grid), dim3(256), 0, stream, pts, n, oct, flags);
    return hipGetLastError();
}

hipError_t launch_write_count(uint64_t* count, uint64_t value, hipStream_t stream) {
    hipLaunchKernelGGL(k_write_count, dim3(1), dim3(1), 0, stream, count, value);
    return hipGetLastError();
}

hipError_t launch_gather(const float2* pts, const uint32_t* surv, const uint64_t* count, uint64_t cap,
                         uint64_t n, float2* out, int grid, hipStream_t stream) {
    hipLaunchKernelGGL(k_gather, dim3(grid), dim3(256), 0, stream, pts, surv, count, cap, n, out);
    return hipGetLastError();
}

uint64_t batch_max_items(uint64_t n_total, uint32_t S) { return n_total / kBatchItem + 2ull * S + 1ull; }

uint32_t batch_item_words() { return kBatchItem / 64; }

uint64_t batch_max_rtiles(uint64_t n_total, uint32_t S) { return n_total / kBatchRT + 2ull * S + 1ull; }

uint32_t batch_tile_boxes() { return kBatchTileBoxes; }

#define HULLF_BATCH_CLASSIFY(B, P)                                                                         \
    if (shape.block == B && shape.ppt == P) {                                                              \
        if (v)                                                                                             \
            hipLaunchKernelGGL((k_batch_classify<B, P, true>), dim3(fgrid), dim3(B), 0, stream, pts, S, sets, \
                               octs, tot, bits, blkcnt, box);                                             \
        else                                                                                               \
            hipLaunchKernelGGL((k_batch_classify<B, P, false>), dim3(fgrid), dim3(B), 0, stream, pts, S,     \
                               sets, octs, tot, bits, blkcnt, box);                                       \
        e = hipGetLastError();                                                                             \
        done = true;                                                                                       \
    }

hipError_t launch_batch(const float2* pts, const uint64_t* off, bool seg, uint32_t S, uint64_t n_total,
                        SetInfo* sets, BatchTotals* tot, unsigned long long* part, uint32_t max_rtiles,
                        Octagon* octs, uint64_t* bits, uint32_t* blkcnt, uint32_t max_items, uint32_t* surv,
                        uint64_t* counts, float4* box, Shape shape, int cus, int reduce_per_cu,
                        hipStream_t stream) {
    if (!shape_supported(shape)) return hipErrorInvalidValue;
    if (seg)
        hipLaunchKernelGGL(k_batch_plan<true>, dim3(1), dim3(1024), 0, stream, off, S, sets, tot, counts, max_items,
                           max_rtiles, n_total, kBatchItem);
    else
        hipLaunchKernelGGL(k_batch_plan<false>, dim3(1), dim3(1024), 0, stream, off, S, sets, tot, counts,
                           max_items, max_rtiles, n_total, kBatchItem);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    const bool v = is_vec4(pts);
    const int rgrid = cus * (reduce_per_cu > 0 ? reduce_per_cu : 4);   // the occupancy k_batch_reduce allows
    if (v)
        hipLaunchKernelGGL(k_batch_reduce<true>, dim3(rgrid), dim3(kRBlock), 0, stream, pts, S, sets, tot, part,
                           box);
    else
        hipLaunchKernelGGL(k_batch_reduce<false>, dim3(rgrid), dim3(kRBlock), 0, stream, pts, S, sets, tot, part,
                           box);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    const uint32_t sblocks = (uint32_t)std::min<uint64_t>((S + 3) / 4, (uint64_t)cus * 8);
    hipLaunchKernelGGL(k_batch_setup, dim3(sblocks), dim3(256), 0, stream, pts, S, sets, part, octs, counts);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    const int fgrid = cus * (shape.block >= 512 ? 3 : 6);
    bool done = false;
    HULLF_BATCH_CLASSIFY(256, 8)
    HULLF_BATCH_CLASSIFY(256, 16)
    HULLF_BATCH_CLASSIFY(512, 8)
    HULLF_BATCH_CLASSIFY(512, 16)
    if (!done) return hipErrorInvalidValue;
    if (e != hipSuccess) return e;
    // 6 blocks per CU: each holds 4 x 5 KB of LDS (stage and keep-bit table)
    hipLaunchKernelGGL(k_batch_compact<256>, dim3(cus * 6), dim3(256), 0, stream, S, sets, octs, tot, bits, blkcnt,
                       surv, counts);
    return hipGetLastError();
}

}  // namespace hullf
