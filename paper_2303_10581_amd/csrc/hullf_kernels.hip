// HIP kernels (gfx950, wave64) for the octagon filter of Carrasco et al.,
// "An Evaluation of GPU Filters for Accelerating the 2D Convex Hull":
//   k_reduce   Sec. 3.1, the eight extremes by a min/max reduction
//   k_filter   Sec. 3.2 + Sec. 4.1.1, inside test fused with a single-pass
//              stream compaction (ballot/popcount inside a wave, LDS scan
//              across waves, decoupled look-back across tiles)
//   k_batch    both steps for many sets in one persistent launch
//
// Data layout: points are float2 (x, y), 8 bytes, AoS.  A block reads a
// chunk/tile of consecutive points as float4 pairs: pair slot j of thread t
// covers points base + 2*(j*BLOCK + t) + {0, 1}, so every load instruction
// of a wave reads 1 KiB of consecutive memory.  Output indices are uint32.
//
// Built with -ffp-contract=off: the binary64 inside test below must be
// evaluated operation by operation.

#include <math.h>

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

__device__ __forceinline__ uint64_t status_load(const uint64_t* p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void status_store(uint64_t* p, uint64_t v) {
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

template <bool VEC4>
__device__ __forceinline__ float4 load_pair(const float2* __restrict__ pts, uint64_t g) {
    if constexpr (VEC4) {
        return *reinterpret_cast<const float4*>(pts + g);
    } else {
        float2 a = pts[g], b = pts[g + 1];
        return make_float4(a.x, a.y, b.x, b.y);
    }
}

// Pair load with per-point range checks against [lo, hi).
__device__ __forceinline__ float4 load_pair_checked(const float2* __restrict__ pts, uint64_t g,
                                                    uint64_t lo, uint64_t hi, bool& v0, bool& v1) {
    v0 = (g >= lo) && (g < hi);
    v1 = (g + 1 >= lo) && (g + 1 < hi);
    float2 a = v0 ? pts[g] : make_float2(0.0f, 0.0f);
    float2 b = v1 ? pts[g + 1] : make_float2(0.0f, 0.0f);
    return make_float4(a.x, a.y, b.x, b.y);
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
// After the loop, the threads whose value equals the block's best reload
// that one chunk and pick the first point attaining it; their minimum index
// is the block's candidate.  This keeps the streaming loop at about 8 VALU
// operations per point instead of 24 for per-point index selects.

__device__ __forceinline__ float key_of(int j, float x, float y) {
    switch (j) {
        case 0: case 4: return x;
        case 1: case 5: return x + y;
        case 2: case 6: return y;
        default: return x - y;
    }
}

template <int N>
__device__ __forceinline__ float tree_max(const float (&v)[N]) {
    float r[N];
#pragma unroll
    for (int i = 0; i < N; ++i) r[i] = v[i];
#pragma unroll
    for (int w = 1; w < N; w *= 2)
#pragma unroll
        for (int i = 0; i + w < N; i += 2 * w) r[i] = fmaxf(r[i], r[i + w]);
    return r[0];
}
template <int N>
__device__ __forceinline__ float tree_min(const float (&v)[N]) {
    float r[N];
#pragma unroll
    for (int i = 0; i < N; ++i) r[i] = v[i];
#pragma unroll
    for (int w = 1; w < N; w *= 2)
#pragma unroll
        for (int i = 0; i + w < N; i += 2 * w) r[i] = fminf(r[i], r[i + w]);
    return r[0];
}

struct BlockExtremes {
    float key[8];       // block best per slot (packed orientation: maxima)
    uint32_t idx[8];    // lowest index attaining it (relative to lo), or ~0
    int bad;            // NaN seen
};

// Reduction of points [lo, hi) over chunks c = c0, c0+cstep, ... < nch of
// CH = BLOCK*G*2 points starting at the pair-aligned base al <= lo.  The
// block result is left in `res` (valid in every thread after return).
template <int BLOCK, int G, bool VEC4>
__device__ void reduce_points(const float2* __restrict__ pts, uint64_t lo, uint64_t hi, uint64_t al,
                              uint32_t c0, uint32_t cstep, uint32_t nch, BlockExtremes& res) {
    constexpr uint32_t CH = BLOCK * G * 2;
    constexpr int NW = BLOCK / 64;
    __shared__ float sh_v[8][NW];
    __shared__ uint32_t sh_i[8][NW];

    const uint32_t t = threadIdx.x;
    float v[8] = {-kInfF, -kInfF, -kInfF, kInfF, kInfF, kInfF, kInfF, -kInfF};
    uint32_t grp[8];
#pragma unroll
    for (int j = 0; j < 8; ++j) grp[j] = c0;
    bool bad = false;

    for (uint32_t c = c0; c < nch; c += cstep) {
        const uint64_t cb = al + (uint64_t)c * CH;
        if (cb >= lo && cb + CH <= hi) {
            float4 q[G];
#pragma unroll
            for (int k = 0; k < G; ++k) q[k] = load_pair<VEC4>(pts, cb + 2ull * (k * BLOCK + t));
            float xs[2 * G], ys[2 * G], ss[2 * G], ds[2 * G];
#pragma unroll
            for (int k = 0; k < G; ++k) {
                xs[2 * k] = q[k].x;
                ys[2 * k] = q[k].y;
                xs[2 * k + 1] = q[k].z;
                ys[2 * k + 1] = q[k].w;
            }
#pragma unroll
            for (int i = 0; i < 2 * G; ++i) {
                ss[i] = xs[i] + ys[i];
                ds[i] = xs[i] - ys[i];
            }
#pragma unroll
            for (int i = 0; i < 2 * G; i += 2) bad |= __builtin_isunordered(ss[i], ss[i + 1]);
            const float m0 = tree_max(xs), m1 = tree_max(ss), m2 = tree_max(ys), m3 = tree_min(ds);
            const float m4 = tree_min(xs), m5 = tree_min(ss), m6 = tree_min(ys), m7 = tree_max(ds);
            if (m0 > v[0]) { v[0] = m0; grp[0] = c; }
            if (m1 > v[1]) { v[1] = m1; grp[1] = c; }
            if (m2 > v[2]) { v[2] = m2; grp[2] = c; }
            if (m3 < v[3]) { v[3] = m3; grp[3] = c; }
            if (m4 < v[4]) { v[4] = m4; grp[4] = c; }
            if (m5 < v[5]) { v[5] = m5; grp[5] = c; }
            if (m6 < v[6]) { v[6] = m6; grp[6] = c; }
            if (m7 > v[7]) { v[7] = m7; grp[7] = c; }
        } else {
#pragma unroll 1
            for (int k = 0; k < G; ++k) {
                bool ok0, ok1;
                const float4 q = load_pair_checked(pts, cb + 2ull * (k * BLOCK + t), lo, hi, ok0, ok1);
#pragma unroll
                for (int h = 0; h < 2; ++h) {
                    const bool ok = h ? ok1 : ok0;
                    if (!ok) continue;
                    const float x = h ? q.z : q.x, y = h ? q.w : q.y;
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
    }

    // block best per key
    const uint32_t lane = lane_id(), wave = t >> 6;
#pragma unroll
    for (int j = 0; j < 8; ++j) {
        const bool is_max = (j == 0 || j == 1 || j == 2 || j == 7);
        const float w = is_max ? wave_max(v[j]) : wave_min(v[j]);
        if (lane == 0) sh_v[j][wave] = w;
    }
    __syncthreads();
    float best[8];
#pragma unroll
    for (int j = 0; j < 8; ++j) {
        const bool is_max = (j == 0 || j == 1 || j == 2 || j == 7);
        float b = sh_v[j][0];
        for (int w = 1; w < NW; ++w) b = is_max ? fmaxf(b, sh_v[j][w]) : fminf(b, sh_v[j][w]);
        best[j] = b;
    }
    // lowest index attaining the best: reload the chunk where this thread
    // first reached it
    uint32_t cand[8];
#pragma unroll
    for (int j = 0; j < 8; ++j) {
        cand[j] = 0xFFFFFFFFu;
        if (v[j] == best[j] && grp[j] < nch) {
            const uint64_t cb = al + (uint64_t)grp[j] * CH;
            for (int k = 0; k < G && cand[j] == 0xFFFFFFFFu; ++k) {
                const uint64_t g = cb + 2ull * (k * BLOCK + t);
                bool ok0, ok1;
                const float4 q = load_pair_checked(pts, g, lo, hi, ok0, ok1);
                if (ok0 && key_of(j, q.x, q.y) == best[j]) cand[j] = (uint32_t)(g - lo);
                else if (ok1 && key_of(j, q.z, q.w) == best[j]) cand[j] = (uint32_t)(g + 1 - lo);
            }
        }
    }
    __syncthreads();   // sh_v reads done before reuse of shared state
#pragma unroll
    for (int j = 0; j < 8; ++j) {
        const uint32_t w = wave_min_u32(cand[j]);
        if (lane == 0) sh_i[j][wave] = w;
    }
    const int any_bad = __syncthreads_or(bad ? 1 : 0);
#pragma unroll
    for (int j = 0; j < 8; ++j) {
        uint32_t b = sh_i[j][0];
        for (int w = 1; w < NW; ++w) b = min(b, sh_i[j][w]);
        res.idx[j] = b;
        const bool is_max = (j == 0 || j == 1 || j == 2 || j == 7);
        res.key[j] = is_max ? best[j] : -best[j];
    }
    res.bad = any_bad;
    __syncthreads();
}

// Merge a block result into the set's slots (thread 0 only).
__device__ __forceinline__ void publish_extremes(const BlockExtremes& r, ReduceSlots* slots) {
#pragma unroll
    for (int j = 0; j < 8; ++j)
        if (r.idx[j] != 0xFFFFFFFFu) atomicMax(&slots->key[j], pack_key(r.key[j], r.idx[j]));
    if (r.bad) atomicOr(&slots->nonfinite, 1u);
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

__device__ void setup_octagon(const float2* __restrict__ pts, uint64_t lo, uint64_t n,
                              ReduceSlots* slots, Octagon* o) {
#pragma clang fp contract(off)
    float vx[8], vy[8];
    uint32_t id[8];
    bool missing = false;
    for (int j = 0; j < 8; ++j) {
        const unsigned long long p =
            __hip_atomic_load(&slots->key[j], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        id[j] = unpack_idx(p);
        missing |= (p == 0ull) || ((uint64_t)id[j] >= n);
        o->idx[j] = id[j];
    }
    o->mode = 0;
    o->fast = 0;
    o->m = 0;
    o->bxl = kInfF;
    o->bxh = -kInfF;
    o->byl = kInfF;
    o->byh = -kInfF;
    if (missing) {   // no candidate for some direction: never expected
        o->status = 3;
        return;
    }
    for (int j = 0; j < 8; ++j) {
        const float2 q = pts[lo + id[j]];
        vx[j] = q.x;
        vy[j] = q.y;
    }
    const uint32_t nf = __hip_atomic_load(&slots->nonfinite, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    const bool bad = nf || !isfinite(vx[0]) || !isfinite(vx[4]) || !isfinite(vy[2]) || !isfinite(vy[6]);
    o->status = bad ? 1 : 0;
    if (bad) return;

    // distinct vertices
    int distinct = 0;
    for (int j = 0; j < 8; ++j) {
        bool seen = false;
        for (int k = 0; k < j; ++k) seen |= (vx[k] == vx[j] && vy[k] == vy[j]);
        distinct += seen ? 0 : 1;
    }
    // non-degenerate edges, binary64
    double ax[8], ay[8], ex[8], ey[8];
    int m = 0;
    for (int j = 0; j < 8; ++j) {
        const int k = (j + 1) & 7;
        if (vx[j] == vx[k] && vy[j] == vy[k]) continue;
        ax[m] = vx[j];
        ay[m] = vy[j];
        ex[m] = (double)vx[k] - (double)vx[j];
        ey[m] = (double)vy[k] - (double)vy[j];
        ++m;
    }
    o->m = m;
    // Fewer than three distinct vertices: no point can be strictly inside
    // every edge (the rule is sound and the polygon has no interior).
    if (distinct < 3 || m == 0) return;
    for (int e = m; e < 8; ++e) {
        ax[e] = ax[0];
        ay[e] = ay[0];
        ex[e] = ex[0];
        ey[e] = ey[0];
    }
    for (int e = 0; e < 8; ++e) {
        o->ax[e] = ax[e];
        o->ay[e] = ay[e];
        o->ex[e] = ex[e];
        o->ey[e] = ey[e];
    }
    o->mode = 1;

    // bounding box (E4, E0 give x; E6, E2 give y)
    const float xmin = vx[4], xmax = vx[0], ymin = vy[6], ymax = vy[2];
    const double up = 1.0 + 0x1p-40;
    const double W = ((double)xmax - (double)xmin) * (1.0 + 0x1p-50);
    const double H = ((double)ymax - (double)ymin) * (1.0 + 0x1p-50);
    const float cx = (float)(0.5 * (double)xmin + 0.5 * (double)xmax);
    const float cy = (float)(0.5 * (double)ymin + 0.5 * (double)ymax);
    o->cx = cx;
    o->cy = cy;
    double M[8];
    bool fast = isfinite(W) && isfinite(H);
    for (int e = 0; e < 8; ++e) {
        M[e] = (fabs(ex[e]) * H + fabs(ey[e]) * W) * up;
        if (!(M[e] > 0.0) || !isfinite(M[e])) {
            fast = false;
            M[e] = 0.0;
            continue;
        }
        int E;
        (void)frexp(M[e] * 0x1p-20, &E);   // 16 u M = m 2^E, m in [0.5, 1)
        const double s = ldexp(1.0, -E);
        const double a = s * ex[e];
        const double nb = -s * ey[e];
        const double k = ex[e] * ((double)cy - ay[e]) - ey[e] * ((double)cx - ax[e]);
        const double c0 = s * k;
        if (!(fabs(a) <= 0x1p100 && fabs(nb) <= 0x1p100 && fabs(c0) <= 0x1p100)) fast = false;
        o->A[e] = (float)a;
        o->NB[e] = (float)nb;
        o->C0[e] = (float)c0;
    }
    o->fast = fast ? 1 : 0;

    // quick-accept box
    float XL = fmaxf(vx[3], vx[5]), XH = fminf(vx[1], vx[7]);
    float YL = fmaxf(vy[5], vy[7]), YH = fminf(vy[1], vy[3]);
    bool ok = fast && XL < XH && YL < YH;
    for (int it = 0; ok && it < 8; ++it) {
        bool pass = true;
        for (int c = 0; c < 4 && pass; ++c) {
            const double qx = (c & 1) ? (double)XH : (double)XL;
            const double qy = (c & 2) ? (double)YH : (double)YL;
            for (int e = 0; e < 8; ++e) {
                const double D = ex[e] * (qy - ay[e]) - ey[e] * (qx - ax[e]);
                if (!(D > 0x1p-48 * M[e])) {
                    pass = false;
                    break;
                }
            }
        }
        if (pass) break;
        if (it == 7) {
            ok = false;
            break;
        }
        XL = (float)((double)cx + 0.75 * ((double)XL - (double)cx));
        XH = (float)((double)cx + 0.75 * ((double)XH - (double)cx));
        YL = (float)((double)cy + 0.75 * ((double)YL - (double)cy));
        YH = (float)((double)cy + 0.75 * ((double)YH - (double)cy));
        ok = XL < XH && YL < YH;
    }
    if (ok) {
        o->bxl = XL;
        o->bxh = XH;
        o->byl = YL;
        o->byh = YH;
    }
}

__device__ __forceinline__ void reset_slots(ReduceSlots* s) {
    for (int j = 0; j < 8; ++j) s->key[j] = 0ull;
    s->nonfinite = 0u;
    s->done = 0u;
}

// ---------------------------------------------------------------------------
// Sec. 3.2: inside test
// ---------------------------------------------------------------------------

// The binary64 rule: strictly inside every edge (mode == 1 implies m >= 3).
__device__ __forceinline__ bool contract_inside(const Octagon* __restrict__ o, float px, float py) {
#pragma clang fp contract(off)
    const double x = px, y = py;
    bool in = true;
#pragma unroll
    for (int e = 0; e < 8; ++e) {
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

// 1 = the point survives.  Decision-equivalent to the binary64 rule.
__device__ __forceinline__ bool keep_point(const Octagon* __restrict__ o, float x, float y) {
    if (o->mode == 0) return true;
    const bool inbox = (o->bxl < x) & (x < o->bxh) & (o->byl < y) & (y < o->byh);
    if (inbox) return false;
    if (o->fast) {
        const float qx = x - o->cx, qy = y - o->cy;
        float mn = kInfF;
#pragma unroll
        for (int e = 0; e < 8; ++e) mn = fminf(mn, fmaf(o->A[e], qy, fmaf(o->NB[e], qx, o->C0[e])));
        if (mn < -1.0f) return true;
        if (mn > 2.0f) return false;
    }
    return !contract_inside(o, x, y);
}

// ---------------------------------------------------------------------------
// Sec. 4.1.1: compaction of one tile with decoupled look-back
// ---------------------------------------------------------------------------
// Tile `tile` of a set covers points [al + tile*T, al + (tile+1)*T) clipped
// to [lo, hi).  Survivors are written as indices relative to lo, ascending,
// at out + (prefix), entries >= cap dropped.  status: the set's tile status
// words (flag in bits 62-63: 0 not ready, 1 aggregate, 2 inclusive prefix).
// `count` (if non-null, for the set's last tile) receives the total.

template <int BLOCK, int PPT, bool VEC4>
__device__ void filter_tile(const float2* __restrict__ pts, uint64_t lo, uint64_t hi, uint64_t al,
                            uint32_t tile, const Octagon* __restrict__ o, uint64_t* status,
                            uint32_t* __restrict__ out, uint64_t cap, uint64_t* count) {
    constexpr int NP = PPT / 2;
    constexpr int NW = BLOCK / 64;
    constexpr int NS = NP * NW;   // wave segments per tile, in index order (j, wave)
    constexpr uint32_t T = BLOCK * PPT;
    static_assert(NS <= 128, "tile shape");
    __shared__ uint32_t sh_off[NS];
    __shared__ uint64_t sh_excl;

    const uint32_t t = threadIdx.x, lane = lane_id(), wave = t >> 6;
    const uint64_t tb = al + (uint64_t)tile * T;
    const bool full = (tb >= lo) && (tb + T <= hi);

    uint32_t k0m = 0, k1m = 0;
    uint32_t rank[NP];
#pragma unroll
    for (int j = 0; j < NP; ++j) {
        const uint64_t g = tb + 2ull * (j * BLOCK + t);
        float4 q;
        bool v0 = true, v1 = true;
        if (full) q = load_pair<VEC4>(pts, g);
        else q = load_pair_checked(pts, g, lo, hi, v0, v1);
        const bool k0 = v0 && keep_point(o, q.x, q.y);
        const bool k1 = v1 && keep_point(o, q.z, q.w);
        const unsigned long long b0 = __ballot(k0), b1 = __ballot(k1);
        rank[j] = rank_below(b0) + rank_below(b1);
        if (lane == 0) sh_off[j * NW + wave] = (uint32_t)(__popcll(b0) + __popcll(b1));
        k0m |= (k0 ? 1u : 0u) << j;
        k1m |= (k1 ? 1u : 0u) << j;
    }
    __syncthreads();

    if (wave == 0) {
        // exclusive scan of the NS segment counts (two per lane at most)
        uint32_t a = (lane < NS) ? sh_off[lane] : 0u;
        uint32_t b = (lane + 64 < NS) ? sh_off[lane + 64] : 0u;
        uint32_t ia = a;
#pragma unroll
        for (int o2 = 1; o2 < 64; o2 <<= 1) {
            const uint32_t u = (uint32_t)__shfl_up((int)ia, o2, 64);
            if ((int)lane >= o2) ia += u;
        }
        const uint32_t tot_a = (uint32_t)__shfl((int)ia, 63, 64);
        uint32_t ib = b;
#pragma unroll
        for (int o2 = 1; o2 < 64; o2 <<= 1) {
            const uint32_t u = (uint32_t)__shfl_up((int)ib, o2, 64);
            if ((int)lane >= o2) ib += u;
        }
        const uint32_t tot_b = (uint32_t)__shfl((int)ib, 63, 64);
        if (lane < NS) sh_off[lane] = ia - a;
        if (lane + 64 < NS) sh_off[lane + 64] = tot_a + ib - b;
        const uint64_t agg = (uint64_t)tot_a + tot_b;

        // decoupled look-back
        uint64_t excl = 0;
        if (tile == 0) {
            if (lane == 0) status_store(&status[0], kFlagP | agg);
        } else {
            if (lane == 0) status_store(&status[tile], kFlagA | agg);
            int64_t look = (int64_t)tile - 1;
            for (;;) {
                const int64_t idx = look - (int64_t)lane;
                const uint64_t s = (idx >= 0) ? status_load(&status[idx]) : kFlagP;
                const uint32_t flag = (uint32_t)(s >> 62);
                const unsigned long long pm = __ballot(flag == 2u);
                const unsigned long long xm = __ballot(flag == 0u);
                const int first_p = pm ? (__ffsll((long long)pm) - 1) : 64;
                const unsigned long long need = (first_p >= 63) ? ~0ull : ((2ull << first_p) - 1ull);
                if (xm & need) {
                    __builtin_amdgcn_s_sleep(1);
                    continue;
                }
                const uint64_t part = ((int)lane <= first_p) ? (s & kValMask) : 0ull;
                excl += wave_sum_u64(part);
                if (first_p < 64) break;
                look -= 64;
            }
            if (lane == 0) status_store(&status[tile], kFlagP | (excl + agg));
        }
        if (lane == 0) {
            sh_excl = excl;
            if (count) *count = excl + agg;
        }
    }
    __syncthreads();

    const uint64_t excl = sh_excl;
#pragma unroll
    for (int j = 0; j < NP; ++j) {
        const bool k0 = (k0m >> j) & 1u, k1 = (k1m >> j) & 1u;
        if (!(k0 | k1)) continue;
        const uint64_t g = tb + 2ull * (j * BLOCK + t);
        const uint64_t pos = excl + sh_off[j * NW + wave] + rank[j];
        if (k0 && pos < cap) __builtin_nontemporal_store((uint32_t)(g - lo), out + pos);
        const uint64_t pos1 = pos + (k0 ? 1u : 0u);
        if (k1 && pos1 < cap) __builtin_nontemporal_store((uint32_t)(g + 1 - lo), out + pos1);
    }
    __syncthreads();
}

// ---------------------------------------------------------------------------
// kernels: one point set
// ---------------------------------------------------------------------------

constexpr int kRBlock = 256;
constexpr int kRG = 8;   // pairs per thread per chunk: 16 points

__global__ void k_init_slots(ReduceSlots* s, uint32_t count) {
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < count) {
        reset_slots(&s[i]);
        s[i].ticket = 0u;
        s[i].ready = 0u;
    }
}

template <bool VEC4>
__global__ __launch_bounds__(kRBlock) void k_reduce(const float2* __restrict__ pts, uint64_t n,
                                                    ReduceSlots* slots, Octagon* oct,
                                                    uint64_t* tile_status, uint32_t num_tiles) {
    // clear the look-back state of the compaction kernel that follows
    for (uint64_t i = (uint64_t)blockIdx.x * kRBlock + threadIdx.x; i < num_tiles;
         i += (uint64_t)gridDim.x * kRBlock)
        tile_status[i] = 0ull;
    if (blockIdx.x == 0 && threadIdx.x == 0) slots->ticket = 0u;

    constexpr uint32_t CH = kRBlock * kRG * 2;
    const uint32_t nch = (uint32_t)((n + CH - 1) / CH);
    __shared__ int sh_last;
    BlockExtremes r;
    reduce_points<kRBlock, kRG, VEC4>(pts, 0, n, 0, blockIdx.x, gridDim.x, nch, r);
    if (threadIdx.x == 0) {
        publish_extremes(r, slots);
        __threadfence();
        const uint32_t prev = atomicAdd(&slots->done, 1u);
        sh_last = (prev == gridDim.x - 1);
    }
    __syncthreads();
    if (sh_last && threadIdx.x == 0) {
        __threadfence();
        setup_octagon(pts, 0, n, slots, oct);
        reset_slots(slots);
        __threadfence();
    }
}

template <int BLOCK, int PPT, bool VEC4>
__global__ __launch_bounds__(BLOCK) void k_filter(const float2* __restrict__ pts, uint64_t n,
                                                  const Octagon* __restrict__ oct, ReduceSlots* slots,
                                                  uint64_t* tile_status, uint32_t num_tiles,
                                                  uint32_t* __restrict__ surv, uint64_t cap,
                                                  uint64_t* count) {
    if (oct->status != 0) {
        if (blockIdx.x == 0 && threadIdx.x == 0)
            *count = (oct->status == 1) ? kCountNonFinite : kCountInternal;
        return;
    }
    __shared__ uint32_t sh_tile;
    for (;;) {
        if (threadIdx.x == 0) sh_tile = atomicAdd(&slots->ticket, 1u);
        __syncthreads();
        const uint32_t tile = sh_tile;
        if (tile >= num_tiles) break;
        filter_tile<BLOCK, PPT, VEC4>(pts, 0, n, 0, tile, oct, tile_status, surv, cap,
                                      tile == num_tiles - 1 ? count : nullptr);
    }
}

template <bool VEC4>
__global__ __launch_bounds__(256) void k_flags(const float2* __restrict__ pts, uint64_t n,
                                               const Octagon* __restrict__ oct, uint8_t* flags) {
    const bool bad = oct->status != 0;
    for (uint64_t i = (uint64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (uint64_t)gridDim.x * 256) {
        if (bad) {
            flags[i] = 2;
            continue;
        }
        const float2 p = pts[i];
        flags[i] = keep_point(oct, p.x, p.y) ? 1 : 0;
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
// kernels: many sets, one persistent launch
// ---------------------------------------------------------------------------
// Work list.  Set s has r_tiles reduction tiles (kRBlock*kRG*2 points each)
// and f_tiles compaction tiles.  The list interleaves them so that the
// compaction of set s comes after the reduction tiles of the sets that end
// within `lag` points after it: its reduction has long finished when its
// compaction tiles are handed out (few waits), and its points are still in
// the last-level cache when they are read the second time.
//   segment order: R(0), F(s : j(s) = 0), R(1), F(s : j(s) = 1), ...
//   j(s) = max(s, first set j with off[j+1] >= off[s+1] + lag), at most S-1
// Tickets are taken from one atomic counter; a ticket's segment is found by
// binary search.  A compaction tile spins until its set's octagon is
// published; this cannot deadlock because every reduction tile of that set
// holds an earlier ticket and never waits.

__device__ __forceinline__ uint32_t first_set_reaching(const uint64_t* off, uint32_t S, uint64_t target) {
    // smallest j in [0, S) with off[j+1] >= target, or S-1
    uint32_t lo = 0, hi = S - 1;
    while (lo < hi) {
        const uint32_t mid = (lo + hi) >> 1;
        if (off[mid + 1] >= target) hi = mid;
        else lo = mid + 1;
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

template <int BLOCK, int PPT>
__global__ __launch_bounds__(1024) void k_batch_plan(const uint64_t* __restrict__ off, uint32_t S,
                                                     SetInfo* sets, ReduceSlots* slots,
                                                     uint32_t* seg_start, uint32_t* seg_code,
                                                     uint32_t* ticket, uint32_t* total,
                                                     uint64_t* tile_status, uint32_t max_tiles,
                                                     uint64_t lag, uint64_t n_total, uint64_t* counts) {
    // one block of 1024 threads
    constexpr uint32_t RT = BLOCK * kRG * 2;   // reduction tile = one chunk
    constexpr uint32_t FT = BLOCK * PPT;       // compaction tile
    __shared__ uint32_t sh_scan[1024];
    __shared__ uint32_t sh_carry[2];
    const uint32_t t = threadIdx.x;
    if (t == 0) {
        *ticket = 0u;
        sh_carry[0] = sh_carry[1] = 0u;
    }
    // offsets must start at 0, end at n_total and never decrease
    int bad = 0;
    for (uint32_t s = t; s < S; s += 1024) bad |= (off[s + 1] < off[s]) ? 1 : 0;
    if (t == 0) bad |= (off[0] != 0ull || off[S] != n_total) ? 1 : 0;
    bad = __syncthreads_or(bad);
    if (bad) {
        for (uint32_t s = t; s < S; s += 1024) counts[s] = kCountBadOffsets;
        if (t == 0) *total = 0u;
        return;
    }
    // tile counts and their prefixes
    for (uint32_t base = 0; base < S; base += 1024) {
        const uint32_t s = base + t;
        uint32_t rt = 0, ft = 0;
        uint64_t b = 0, n = 0;
        if (s < S) {
            b = off[s];
            n = off[s + 1] - b;
            const uint64_t al = b & ~1ull;
            rt = n ? (uint32_t)((b + n - al + RT - 1) / RT) : 0u;
            ft = n ? (uint32_t)((b + n - al + FT - 1) / FT) : 0u;
        }
        const uint32_t r0 = block_exclusive_scan(rt, sh_scan, &sh_carry[0]);
        const uint32_t f0 = block_exclusive_scan(ft, sh_scan, &sh_carry[1]);
        if (s < S) {
            sets[s].begin = b;
            sets[s].n = n;
            sets[s].r_tiles = rt;
            sets[s].f_tiles = ft;
            sets[s].r_tile0 = r0;
            sets[s].f_tile0 = f0;
            sets[s].r_done = 0u;
            reset_slots(&slots[s]);
            slots[s].ready = 0u;
            if (n == 0) counts[s] = 0ull;
        }
    }
    const uint32_t rtiles = sh_carry[0], ftiles = sh_carry[1];
    for (uint32_t i = t; i < ftiles && i < max_tiles; i += 1024) tile_status[i] = 0ull;
    __syncthreads();
    // segments (see the work-list comment above)
    for (uint32_t s = t; s < S; s += 1024) {
        const uint32_t js = max(s, first_set_reaching(off, S, off[s + 1] + lag));
        uint32_t lo_i = 0, hi_i = S;   // m(s): first s' with j(s') >= s
        while (lo_i < hi_i) {
            const uint32_t mid = (lo_i + hi_i) >> 1;
            if (max(mid, first_set_reaching(off, S, off[mid + 1] + lag)) >= s) hi_i = mid;
            else lo_i = mid + 1;
        }
        const uint32_t ms = lo_i;
        const uint32_t sumF_lt_ms = (ms < S) ? sets[ms].f_tile0 : ftiles;
        const uint32_t iR = s + ms, iF = js + 1 + s;
        seg_start[iR] = sets[s].r_tile0 + sumF_lt_ms;
        seg_code[iR] = s << 1;
        seg_start[iF] = sets[js].r_tile0 + sets[js].r_tiles + sets[s].f_tile0;
        seg_code[iF] = (s << 1) | 1u;
    }
    if (t == 0) {
        seg_start[2 * S] = rtiles + ftiles;
        *total = (ftiles <= max_tiles) ? rtiles + ftiles : 0u;
    }
}

template <int BLOCK, int PPT, bool VEC4>
__global__ __launch_bounds__(BLOCK) void k_batch(const float2* __restrict__ pts, uint32_t S,
                                                 SetInfo* sets, ReduceSlots* slots, Octagon* octs,
                                                 const uint32_t* __restrict__ seg_start,
                                                 const uint32_t* __restrict__ seg_code,
                                                 uint32_t* ticket, const uint32_t* total_p,
                                                 uint64_t* tile_status, uint32_t* __restrict__ surv,
                                                 uint64_t* counts) {
    constexpr uint32_t RT = BLOCK * kRG * 2;   // reduction tile = one chunk
    __shared__ uint32_t sh_ticket;
    __shared__ int sh_last;
    const uint32_t total = *total_p;
    for (;;) {
        if (threadIdx.x == 0) sh_ticket = atomicAdd(ticket, 1u);
        __syncthreads();
        const uint32_t tk = sh_ticket;
        if (tk >= total) break;
        // segment of this ticket: last k with seg_start[k] <= tk
        uint32_t lo = 0, hi = 2 * S - 1;
        while (lo < hi) {
            const uint32_t mid = (lo + hi + 1) >> 1;
            if (seg_start[mid] <= tk) lo = mid;
            else hi = mid - 1;
        }
        const uint32_t code = seg_code[lo];
        const uint32_t s = code >> 1;
        const uint32_t local = tk - seg_start[lo];
        const uint64_t b = sets[s].begin, n = sets[s].n;
        const uint64_t al = b & ~1ull;
        if ((code & 1u) == 0u) {
            // reduction tile `local`: points [al + local*RT, +RT) of the set
            const uint64_t tb = al + (uint64_t)local * RT;
            BlockExtremes r;
            reduce_points<BLOCK, kRG, VEC4>(pts, b, b + n, tb, 0u, 1u, 1u, r);
            if (threadIdx.x == 0) {
                publish_extremes(r, &slots[s]);
                __threadfence();
                const uint32_t prev = atomicAdd(&sets[s].r_done, 1u);
                sh_last = (prev == sets[s].r_tiles - 1);
            }
            __syncthreads();
            if (sh_last && threadIdx.x == 0) {
                __threadfence();
                setup_octagon(pts, b, n, &slots[s], &octs[s]);
                reset_slots(&slots[s]);
                __threadfence();
                __hip_atomic_store(&slots[s].ready, 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
                if (octs[s].status != 0)
                    counts[s] = (octs[s].status == 1) ? kCountNonFinite : kCountInternal;
            }
            __syncthreads();
        } else {
            // compaction tile `local` of set s: wait for its octagon
            if (threadIdx.x == 0) {
                while (__hip_atomic_load(&slots[s].ready, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT) == 0u)
                    __builtin_amdgcn_s_sleep(2);
            }
            __syncthreads();
            const Octagon* o = &octs[s];
            if (o->status == 0) {
                filter_tile<BLOCK, PPT, VEC4>(pts, b, b + n, al, local, o,
                                              tile_status + sets[s].f_tile0,
                                              surv + b, n, local == sets[s].f_tiles - 1 ? &counts[s] : nullptr);
            }
            __syncthreads();
        }
    }
}

template <int BLOCK, int PPT>
hipError_t launch_filter_t(const float2* pts, uint64_t n, const Octagon* oct, ReduceSlots* slots,
                           uint64_t* tile_status, uint32_t num_tiles, uint32_t* surv, uint64_t cap,
                           uint64_t* count, bool vec4, int grid, hipStream_t stream) {
    if (vec4)
        hipLaunchKernelGGL((k_filter<BLOCK, PPT, true>), dim3(grid), dim3(BLOCK), 0, stream, pts, n,
                           oct, slots, tile_status, num_tiles, surv, cap, count);
    else
        hipLaunchKernelGGL((k_filter<BLOCK, PPT, false>), dim3(grid), dim3(BLOCK), 0, stream, pts, n,
                           oct, slots, tile_status, num_tiles, surv, cap, count);
    return hipGetLastError();
}

template <int BLOCK, int PPT>
hipError_t launch_batch_t(const float2* pts, uint32_t S, const SetInfo* sets, ReduceSlots* slots,
                          Octagon* octs, const uint32_t* seg_start, const uint32_t* seg_code,
                          uint32_t* ticket, const uint32_t* total, uint64_t* tile_status,
                          uint32_t* surv, uint64_t* counts, bool vec4, int grid, hipStream_t stream) {
    SetInfo* ms = const_cast<SetInfo*>(sets);
    if (vec4)
        hipLaunchKernelGGL((k_batch<BLOCK, PPT, true>), dim3(grid), dim3(BLOCK), 0, stream, pts, S, ms,
                           slots, octs, seg_start, seg_code, ticket, total, tile_status, surv, counts);
    else
        hipLaunchKernelGGL((k_batch<BLOCK, PPT, false>), dim3(grid), dim3(BLOCK), 0, stream, pts, S, ms,
                           slots, octs, seg_start, seg_code, ticket, total, tile_status, surv, counts);
    return hipGetLastError();
}

template <int BLOCK, int PPT>
hipError_t launch_plan_t(const uint64_t* off, uint32_t S, SetInfo* sets, ReduceSlots* slots,
                         uint32_t* seg_start, uint32_t* seg_code, uint32_t* ticket, uint32_t* total,
                         uint64_t* tile_status, uint32_t max_tiles, uint64_t lag, uint64_t n_total,
                         uint64_t* counts, hipStream_t stream) {
    hipLaunchKernelGGL((k_batch_plan<BLOCK, PPT>), dim3(1), dim3(1024), 0, stream, off, S, sets, slots,
                       seg_start, seg_code, ticket, total, tile_status, max_tiles, lag, n_total,
                       counts);
    return hipGetLastError();
}

bool is_vec4(const float2* p) { return ((uintptr_t)p & 15u) == 0u; }

}  // namespace

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------

uint32_t reduce_chunk_points() { return kRBlock * kRG * 2; }

uint32_t filter_tile_points(Shape s) { return (uint32_t)(s.block * s.ppt); }

bool shape_supported(Shape s) {
    return (s.block == 256 || s.block == 512) && (s.ppt == 8 || s.ppt == 16 || s.ppt == 32);
}

hipError_t launch_init_slots(ReduceSlots* slots, uint32_t count, hipStream_t stream) {
    if (count == 0) return hipSuccess;
    hipLaunchKernelGGL(k_init_slots, dim3((count + 255) / 256), dim3(256), 0, stream, slots, count);
    return hipGetLastError();
}

hipError_t launch_reduce(const float2* pts, uint64_t n, ReduceSlots* slots, Octagon* oct,
                         uint64_t* tile_status, uint32_t num_tiles, int grid, hipStream_t stream) {
    if (is_vec4(pts))
        hipLaunchKernelGGL(k_reduce<true>, dim3(grid), dim3(kRBlock), 0, stream, pts, n, slots, oct,
                           tile_status, num_tiles);
    else
        hipLaunchKernelGGL(k_reduce<false>, dim3(grid), dim3(kRBlock), 0, stream, pts, n, slots, oct,
                           tile_status, num_tiles);
    return hipGetLastError();
}

#define HULLF_SHAPES(X) X(256, 8) X(256, 16) X(256, 32) X(512, 8) X(512, 16) X(512, 32)

hipError_t launch_filter(const float2* pts, uint64_t n, const Octagon* oct, ReduceSlots* slots,
                         uint64_t* tile_status, uint32_t num_tiles, uint32_t* surv, uint64_t cap,
                         uint64_t* count, Shape shape, int grid, hipStream_t stream) {
    const bool v = is_vec4(pts);
#define X(B, P)                                                                                   \
    if (shape.block == B && shape.ppt == P)                                                       \
        return launch_filter_t<B, P>(pts, n, oct, slots, tile_status, num_tiles, surv, cap, count, \
                                     v, grid, stream);
    HULLF_SHAPES(X)
#undef X
    return hipErrorInvalidValue;
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

uint64_t batch_max_tiles(uint64_t n_total, uint32_t S, Shape shape) {
    // each non-empty set needs at most n/T + 2 tiles (one for the pair
    // alignment of its first point)
    return n_total / (uint64_t)(shape.block * shape.ppt) + 2ull * S + 1ull;
}

hipError_t launch_batch_plan(const uint64_t* off, uint32_t S, SetInfo* sets, ReduceSlots* slots,
                             uint32_t* seg_start, uint32_t* seg_code, uint32_t* ticket,
                             uint32_t* total_tickets, uint64_t* tile_status, uint32_t max_tiles,
                             uint64_t lag_points, uint64_t n_total, uint64_t* counts, Shape shape,
                             hipStream_t stream) {
#define X(B, P)                                                                                  \
    if (shape.block == B && shape.ppt == P)                                                      \
        return launch_plan_t<B, P>(off, S, sets, slots, seg_start, seg_code, ticket, total_tickets, \
                                   tile_status, max_tiles, lag_points, n_total, counts, stream);
    HULLF_SHAPES(X)
#undef X
    return hipErrorInvalidValue;
}

hipError_t launch_batch_persistent(const float2* pts, uint32_t S, const SetInfo* sets,
                                   ReduceSlots* slots, Octagon* octs, const uint32_t* seg_start,
                                   const uint32_t* seg_code, uint32_t* ticket,
                                   const uint32_t* total_tickets, uint64_t* tile_status,
                                   uint32_t* surv, uint64_t* counts, Shape shape, int grid,
                                   hipStream_t stream) {
    const bool v = is_vec4(pts);
#define X(B, P)                                                                                     \
    if (shape.block == B && shape.ppt == P)                                                         \
        return launch_batch_t<B, P>(pts, S, sets, slots, octs, seg_start, seg_code, ticket,          \
                                    total_tickets, tile_status, surv, counts, v, grid, stream);
    HULLF_SHAPES(X)
#undef X
    return hipErrorInvalidValue;
}

}  // namespace hullf
