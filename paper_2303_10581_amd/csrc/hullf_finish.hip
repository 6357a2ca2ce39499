// Hull finishing on the device (the monotone chain of Sec. 3.3 for large
// survivor sets): sort of the survivors by x, one representative point per
// run of equal x and side, monotone chains over fixed chunks of the
// representatives, repeated on the chain vertices while that pays, then a
// merge tree of the chunk chains; only the lower and the upper hull chains
// go back to the host.
//
//   k_fin_keys     64-bit key (x, then y, order-preserving bits, -0 = +0)
//                  and the point index of every survivor
//   k_rs_*         stable LSD radix sort of (key, index), passes of 8 bits
//                  (the hull path sorts by the key's x half only)
//   k_runs         per run of equal x, the first point of least (lower
//                  side) or greatest (upper side) y
//   k_chain        one thread per chunk: strict lower or upper chain of the
//                  chunk (positions into the sorted sequence)
//   k_scan_counts  exclusive scan of the chunk chain lengths (one block)
//   k_chain_gather the chain vertices of all chunks, in order
//   k_bridge       merge tree over the chunk chains: the bridge of each pair
//                  of adjacent chains (one wave per pair)
//   k_merge_gather the merged chains (prefix of the left chain up to the
//                  bridge, suffix of the right one from it), in order
//
// Why chunks are enough: a point that is not a vertex of its chunk's lower
// chain lies on or above a segment between two points of the chunk, so it
// is not a strict vertex of the lower hull of all points (likewise upper).
// The sort is stable and the survivors come in ascending index order, so a
// run of equal x holds its points in index order and its representative is
// the lowest index among equal coordinates; representatives are distinct
// and strictly increasing in x.
//
// Orientation is exact: binary64 determinant with Shewchuk's error bound
// first; then, if the coordinate differences and the two products are exact
// in binary64 (checked), the sign of the determinant's one rounding;
// otherwise the determinant of FP32 coordinates is the sum of six products
// that binary64 represents exactly, summed as a floating-point expansion
// (Two-Sum, Grow-Expansion), whose largest component gives the sign.  Built
// with -ffp-contract=off.

#include <hip/hip_runtime.h>

#include <algorithm>

#include "hullf_internal.h"

namespace hullf {
namespace {

constexpr int kRsBlock = 256;
constexpr int kRsItems = 16;
constexpr uint32_t kRsTile = kRsBlock * kRsItems;   // 4096 items per tile
constexpr int kRsBins = 256;

__device__ __forceinline__ uint32_t ord32(float f) {
    f = (f == 0.0f) ? 0.0f : f;
    const uint32_t u = __float_as_uint(f);
    return (u & 0x80000000u) ? ~u : (u | 0x80000000u);
}
__device__ __forceinline__ float unord32(uint32_t k) {
    return __uint_as_float((k & 0x80000000u) ? (k & 0x7FFFFFFFu) : ~k);
}
__device__ __forceinline__ float key_x(uint64_t k) { return unord32((uint32_t)(k >> 32)); }
__device__ __forceinline__ float key_y(uint64_t k) { return unord32((uint32_t)k); }

// Piece k of a batch split: its set s and its items [b, e) (binary search
// for the set: the largest s with first[s] <= k, which skips empty sets).
__device__ __forceinline__ void piece_of(const SetSplit& sp, uint32_t k, uint32_t& s, uint32_t& b, uint32_t& e) {
    uint32_t lo = 0, hi = sp.S - 1u;
    while (lo < hi) {
        const uint32_t mid = (lo + hi + 1u) / 2u;
        if (sp.first[mid] <= k) lo = mid;
        else hi = mid - 1u;
    }
    s = lo;
    b = sp.start[s] + (k - sp.first[s]) * sp.size;
    e = min(sp.start[s + 1u], b + sp.size);
}

// ---------------------------------------------------------------------------
// keys
// ---------------------------------------------------------------------------
// An index >= n is not read: it sets *bad and takes the point (0, 0).
__global__ __launch_bounds__(256) void k_fin_keys(const float2* __restrict__ pts, uint64_t n,
                                                  const uint32_t* __restrict__ surv, uint32_t m,
                                                  uint64_t* __restrict__ keys, uint32_t* __restrict__ vals,
                                                  uint64_t* bad) {
    for (uint32_t i = blockIdx.x * 256u + threadIdx.x; i < m; i += gridDim.x * 256u) {
        const uint32_t j = surv[i];
        float2 p = make_float2(0.0f, 0.0f);
        if (j < n) p = pts[j];
        else *bad = 1ull;
        keys[i] = ((uint64_t)ord32(p.x) << 32) | ord32(p.y);
        vals[i] = j;
    }
}

// Batched keys.  Block k takes sort tile k of the split (items [b, e) of set
// s, sp.start = the exclusive prefix of the survivor counts): item i is set
// s's survivor j = i - sp.start[s], whose set-local index is
// surv[off[s] + j] and whose point is pts[off[s] + that index].  A local
// index >= the set's size sets *bad and takes the point (0, 0).
__global__ __launch_bounds__(256) void k_bfin_keys(const float2* __restrict__ pts, const uint64_t* __restrict__ off,
                                                   const uint32_t* __restrict__ surv, SetSplit sp,
                                                   uint64_t* __restrict__ keys, uint32_t* __restrict__ vals,
                                                   uint64_t* bad) {
    uint32_t set, b, e;
    piece_of(sp, blockIdx.x, set, b, e);
    const uint64_t o = off[set];
    const uint64_t ns = off[set + 1] - o;
    const uint32_t j0 = b - sp.start[set];
    for (uint32_t i = threadIdx.x; b + i < e; i += 256u) {
        const uint32_t loc = surv[o + j0 + i];
        float2 q = make_float2(0.0f, 0.0f);
        if (loc < ns) q = pts[o + loc];
        else *bad = 1ull;
        keys[b + i] = ((uint64_t)ord32(q.x) << 32) | ord32(q.y);
        vals[b + i] = loc;
    }
}

// ---------------------------------------------------------------------------
// radix sort
// ---------------------------------------------------------------------------
// Tiles are kRsTile consecutive items, or, for a batch of sets sorted each
// on its own, the pieces of a split of size kRsTile (never crossing a set).
// hist[d * tiles + t] = items of tile t with digit d (then, after the two
// scans, the output position of the first of them).

// Tile of block b of a grid of n blocks, one per tile.  Blocks go to the 8
// XCDs in turn (block b to XCD b mod 8), each with its own L2; this gives
// every XCD a contiguous range of tiles, taken in order, so that the runs
// that neighbouring tiles write next to each other (a digit's run of tile t
// ends where tile t+1's begins; hist entries of consecutive tiles share
// lines) meet in one L2 and leave it as whole lines.
__device__ __forceinline__ uint32_t xcd_tile(uint32_t b, uint32_t n) {
    const uint32_t x = b & 7u, j = b >> 3, q = n >> 3, r = n & 7u;
    return x * q + min(x, r) + j;
}

// A pass whose digits take few values (the top byte of clustered
// coordinates) would serialise up to 64 LDS atomics on one address: each
// round first peels off up to four large groups of lanes with equal digits
// (one lane adds the group's size); the lanes left add one each.
__global__ __launch_bounds__(kRsBlock) void k_rs_hist(const uint64_t* __restrict__ keys, uint32_t m, uint32_t shift,
                                                      uint32_t tiles, SetSplit sp, uint32_t* __restrict__ hist) {
    __shared__ uint32_t h[kRsBins];
    const uint32_t t = threadIdx.x, lane = t & 63u, tile = xcd_tile(blockIdx.x, tiles);
    h[t] = 0u;
    __syncthreads();
    uint64_t base = (uint64_t)tile * kRsTile;
    uint32_t nt = (uint32_t)min<uint64_t>(kRsTile, (uint64_t)m - base);
    if (sp.first) {
        uint32_t set, b, e;
        piece_of(sp, tile, set, b, e);
        base = b;
        nt = e - b;
    }
    uint64_t k[kRsItems];
#pragma unroll
    for (int r = 0; r < kRsItems; ++r) {
        const uint32_t i = (uint32_t)r * kRsBlock + t;
        k[r] = (i < nt) ? keys[base + i] : 0ull;
    }
#pragma unroll
    for (int r = 0; r < kRsItems; ++r) {
        const bool valid = (uint32_t)r * kRsBlock + t < nt;
        const uint32_t d = (uint32_t)(k[r] >> shift) & 255u;
        unsigned long long rem = __ballot(valid);
        for (int it = 0; it < 4 && rem != 0ull; ++it) {
            const int leader = __ffsll((long long)rem) - 1;
            const uint32_t dl = (uint32_t)__builtin_amdgcn_readlane((int)d, leader);
            const unsigned long long grp = __ballot(valid && d == dl);
            if (__popcll(grp) < 8) break;   // small groups: plain atomics
            if (lane == (uint32_t)leader) atomicAdd(&h[dl], (uint32_t)__popcll(grp));
            rem &= ~grp;
        }
        if ((rem >> lane) & 1ull) atomicAdd(&h[d], 1u);
    }
    __syncthreads();
    hist[(uint64_t)t * tiles + tile] = h[t];
}

// Block d: total of digit d over all tiles.
__global__ __launch_bounds__(256) void k_rs_rowsum(const uint32_t* __restrict__ hist, uint32_t tiles,
                                                   uint32_t* __restrict__ rowsum) {
    __shared__ uint32_t s[256];
    const uint32_t d = blockIdx.x, t = threadIdx.x;
    uint32_t acc = 0;
    for (uint32_t i = t; i < tiles; i += 256) acc += hist[(uint64_t)d * tiles + i];
    s[t] = acc;
    __syncthreads();
    for (uint32_t o = 128; o > 0; o >>= 1) {
        if (t < o) s[t] += s[t + o];
        __syncthreads();
    }
    if (t == 0) rowsum[d] = s[0];
}

// Block d: output positions of digit d per tile = (items of smaller digits)
// + (items of digit d in earlier tiles).  Each round scans 1024 tiles: four
// consecutive per thread, a shuffle scan inside each wave, one LDS exchange
// of the four wave totals.
//
// With rowend (tile tables: every set sorted on its own) the row is scanned
// from 0 instead, and its total goes to rowend[d]; k_rs_setpre then turns
// the prefixes into positions inside each set.
__global__ __launch_bounds__(256) void k_rs_rowscan(uint32_t* __restrict__ hist, uint32_t tiles,
                                                    const uint32_t* __restrict__ rowsum, uint32_t* rowend) {
    constexpr int NW = 256 / 64;
    __shared__ uint32_t s[256];
    __shared__ uint32_t wsum[NW];
    __shared__ uint32_t carry;
    const uint32_t d = blockIdx.x, t = threadIdx.x, lane = t & 63u, wave = t >> 6;
    s[t] = (!rowend && t < d) ? rowsum[t] : 0u;
    __syncthreads();
    for (uint32_t o = 128; o > 0; o >>= 1) {
        if (t < o) s[t] += s[t + o];
        __syncthreads();
    }
    if (t == 0) carry = s[0];
    __syncthreads();
    uint32_t* row = hist + (uint64_t)d * tiles;
    for (uint32_t b = 0; b < tiles; b += 1024u) {
        uint32_t v[4], sum = 0;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const uint32_t i = b + 4u * t + (uint32_t)q;
            v[q] = (i < tiles) ? row[i] : 0u;
            sum += v[q];
        }
        uint32_t incl = sum;
#pragma unroll
        for (int o = 1; o < 64; o <<= 1) {
            const uint32_t u = (uint32_t)__shfl_up((int)incl, o, 64);
            if ((int)lane >= o) incl += u;
        }
        if (lane == 63u) wsum[wave] = incl;
        __syncthreads();
        uint32_t before = carry, all = 0;
#pragma unroll
        for (int w = 0; w < NW; ++w) {
            const uint32_t x = wsum[w];
            if (w < (int)wave) before += x;
            all += x;
        }
        uint32_t e = before + incl - sum;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const uint32_t i = b + 4u * t + (uint32_t)q;
            if (i < tiles) row[i] = e;
            e += v[q];
        }
        __syncthreads();   // every thread has read carry and wsum
        if (t == 0) carry += all;
        __syncthreads();
    }
    if (rowend && t == 0) rowend[d] = carry;
}

// Batched sort, block per set s (thread per digit): digit d of set s starts
// at ipos[s] + (items of s with smaller digits); tile t of s, with row
// prefix P[d][t] (k_rs_rowscan from 0), puts its first digit-d item at
// that start + P[d][t] - P[d][first tile of s].  sdp[s][d] receives the
// start minus P[d][first tile of s], so the scatter adds P[d][t].  ipos
// and sft: the split's item starts and first tiles.
__global__ __launch_bounds__(256) void k_rs_setpre(const uint32_t* __restrict__ hist, uint32_t tiles,
                                                   const uint32_t* __restrict__ rowend, SetSplit sp,
                                                   uint32_t* __restrict__ sdp) {
    const uint32_t* __restrict__ sft = sp.first;
    const uint32_t* __restrict__ ipos = sp.start;
    __shared__ uint32_t wsum[4];
    const uint32_t s = blockIdx.x, d = threadIdx.x, lane = d & 63u, wave = d >> 6;
    const uint32_t t0 = sft[s], t1 = sft[s + 1];
    auto P = [&](uint32_t t) { return t < tiles ? hist[(uint64_t)d * tiles + t] : rowend[d]; };
    const uint32_t p0 = (t0 < t1) ? P(t0) : 0u;
    const uint32_t c = (t0 < t1) ? P(t1) - p0 : 0u;   // items of set s with digit d
    uint32_t incl = c;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const uint32_t u = (uint32_t)__shfl_up((int)incl, o, 64);
        if ((int)lane >= o) incl += u;
    }
    if (lane == 63u) wsum[wave] = incl;
    __syncthreads();
    uint32_t before = 0;
    for (uint32_t w = 0; w < wave; ++w) before += wsum[w];
    sdp[(uint64_t)s * kRsBins + d] = ipos[s] + before + incl - c - p0;
}

// Stable scatter of one tile.  Items are ranked in tile order (round r,
// then thread) per digit: lanes of a wave with equal digits are found with
// eight ballots, earlier waves and rounds through LDS counters.  Items are
// first placed in LDS in digit order, then written out so that each
// digit's run of the tile is a contiguous store.
__global__ __launch_bounds__(kRsBlock) void k_rs_scatter(const uint64_t* __restrict__ kin,
                                                         const uint32_t* __restrict__ vin, uint32_t m,
                                                         uint32_t shift, uint32_t tiles,
                                                         const uint32_t* __restrict__ hist, SetSplit sp,
                                                         const uint32_t* __restrict__ sdp,
                                                         uint64_t* __restrict__ kout,
                                                         uint32_t* __restrict__ vout) {
    // Wave w ranks the tile's items [w*IW, (w+1)*IW) by itself: in each round
    // of 64, lanes with equal digits find each other with 8 ballots, and a
    // running count per digit in the wave's own LDS row gives every item its
    // rank among the wave's earlier items of that digit (LDS operations of
    // one wave take effect in program order, so no barrier is needed).  The
    // block then turns the per-wave counts into offsets once.  Within a
    // digit, items keep their input order: the sort is stable.
    constexpr int NW = kRsBlock / 64;
    constexpr uint32_t IW = kRsTile / NW;   // items per wave
    constexpr int RW = (int)(IW / 64);      // rounds per wave
    static_assert(kRsBins == kRsBlock, "one digit per thread");
    __shared__ uint64_t sk[kRsTile];
    __shared__ uint32_t sv[kRsTile];
    __shared__ uint32_t wcnt[NW][kRsBins];   // per-wave digit counts, then their offsets in the tile
    __shared__ uint32_t tofs[kRsBins];       // tile-level exclusive digit offsets
    __shared__ uint32_t gpos[kRsBins];       // output position of the tile's first item per digit
    __shared__ uint32_t wsum[NW];
    const uint32_t t = threadIdx.x, lane = t & 63u, wave = t >> 6, tile = xcd_tile(blockIdx.x, tiles);
    uint64_t base = (uint64_t)tile * kRsTile;
    uint32_t nt = (uint32_t)min<uint64_t>(kRsTile, (uint64_t)m - base);
    uint32_t set = 0;
    if (sp.first) {
        uint32_t b, e;
        piece_of(sp, tile, set, b, e);
        base = b;
        nt = e - b;
    }
#pragma unroll
    for (int w = 0; w < NW; ++w) wcnt[w][t] = 0u;
    gpos[t] = hist[(uint64_t)t * tiles + tile] + (sp.first ? sdp[(uint64_t)set * kRsBins + t] : 0u);
    __syncthreads();
    uint64_t k[RW];
    uint32_t v[RW], rk[RW];
    uint32_t* wc = wcnt[wave];
    const unsigned long long below = (1ull << lane) - 1ull;
#pragma unroll
    for (int r = 0; r < RW; ++r) {
        const uint32_t i = wave * IW + (uint32_t)r * 64u + lane;
        const bool valid = i < nt;
        k[r] = valid ? kin[base + i] : 0ull;
        v[r] = valid ? vin[base + i] : 0u;
    }
#pragma unroll
    for (int r = 0; r < RW; ++r) {
        const uint32_t i = wave * IW + (uint32_t)r * 64u + lane;
        const bool valid = i < nt;
        const uint32_t d = (uint32_t)(k[r] >> shift) & 255u;
        unsigned long long peers = __ballot(valid);
#pragma unroll
        for (int bb = 0; bb < 8; ++bb) {
            const unsigned long long m1 = __ballot((d >> bb) & 1u);
            peers &= ((d >> bb) & 1u) ? m1 : ~m1;
        }
        const uint32_t rank = (uint32_t)__popcll(peers & below);
        const uint32_t prev = valid ? wc[d] : 0u;
        rk[r] = prev + rank;
        if (valid && rank == 0u) wc[d] = prev + (uint32_t)__popcll(peers);
    }
    __syncthreads();
    // digit t: total over the waves, exclusive scan over the digits
    uint32_t c[NW], tot = 0;
#pragma unroll
    for (int w = 0; w < NW; ++w) {
        c[w] = wcnt[w][t];
        tot += c[w];
    }
    uint32_t incl = tot;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const uint32_t u = (uint32_t)__shfl_up((int)incl, o, 64);
        if ((int)lane >= o) incl += u;
    }
    if (lane == 63u) wsum[wave] = incl;
    __syncthreads();
    uint32_t ex = incl - tot;
    for (uint32_t w = 0; w < wave; ++w) ex += wsum[w];
    tofs[t] = ex;
#pragma unroll
    for (int w = 0; w < NW; ++w) {
        wcnt[w][t] = ex;
        ex += c[w];
    }
    __syncthreads();
    // the tile in digit order in LDS
#pragma unroll
    for (int r = 0; r < RW; ++r) {
        const uint32_t i = wave * IW + (uint32_t)r * 64u + lane;
        if (i < nt) {
            const uint32_t d = (uint32_t)(k[r] >> shift) & 255u;
            const uint32_t q = wc[d] + rk[r];
            if (q < kRsTile) {
                sk[q] = k[r];
                sv[q] = v[r];
            }
        }
    }
    __syncthreads();
    // item q of digit d goes to gpos[d] + (q - tofs[d])
#pragma unroll 1
    for (uint32_t q = t; q < nt; q += kRsBlock) {
        const uint64_t key = sk[q];
        const uint32_t d = (uint32_t)(key >> shift) & 255u;
        const uint32_t o = gpos[d] + (q - tofs[d]);
        if (o < m) {
            kout[o] = key;
            vout[o] = sv[q];
        }
    }
}

// ---------------------------------------------------------------------------
// exact orientation
// ---------------------------------------------------------------------------
__device__ __forceinline__ void two_sum(double a, double b, double& s, double& e) {
    s = a + b;
    const double bv = s - a;
    const double av = s - bv;
    e = (a - av) + (b - bv);
}

// Exact sign of (a-o) x (b-o) for FP32 coordinates: the six products are
// exact in binary64 (24-bit significands, no underflow for FP32 inputs).
__device__ __noinline__ int orient_exact_dev(float ox, float oy, float ax, float ay, float bx, float by) {
    double t[6];
    t[0] = (double)ax * (double)by;
    t[1] = -((double)ay * (double)bx);
    t[2] = -((double)ax * (double)oy);
    t[3] = (double)ay * (double)ox;
    t[4] = -((double)ox * (double)by);
    t[5] = (double)oy * (double)bx;
    double h[6];
    int len = 0;
    for (int i = 0; i < 6; ++i) {
        double q = t[i];
        for (int j = 0; j < len; ++j) {
            double s, e;
            two_sum(q, h[j], s, e);
            h[j] = e;
            q = s;
        }
        h[len++] = q;
    }
    for (int j = len - 1; j >= 0; --j)
        if (h[j] != 0.0) return h[j] > 0.0 ? 1 : -1;
    return 0;
}

// True if a - b of two binary32 values is exact in binary64: with
// a = Ma 2^(Ea-23), b = Mb 2^(Eb-23) (|M| < 2^24, E from the exponent field,
// at least -126), the difference is K 2^(min(Ea,Eb)-23) with
// |K| < 2^(25 + |Ea - Eb|), so |Ea - Eb| <= 28 keeps K within 53 bits.
__device__ __forceinline__ bool diff_exact(float a, float b) {
    const int ea = max((int)((__float_as_uint(a) >> 23) & 0xFFu), 1);
    const int eb = max((int)((__float_as_uint(b) >> 23) & 0xFFu), 1);
    return abs(ea - eb) <= 28;
}

__device__ __forceinline__ int orient_dev(float ox, float oy, float ax, float ay, float bx, float by) {
    const double dx1 = (double)ax - (double)ox, dy2 = (double)by - (double)oy;
    const double dy1 = (double)ay - (double)oy, dx2 = (double)bx - (double)ox;
    const double l = dx1 * dy2;
    const double r = dy1 * dx2;
    const double det = l - r;
    const double bound = 0x1.8000000000004p-52 * (fabs(l) + fabs(r));
    if (det > bound) return 1;
    if (-det > bound) return -1;
    // Near-degenerate (nearly collinear points, as on a densely sampled
    // circle): when the four differences and the two products are exact
    // (an FMA returns each product's rounding error, zero iff it is exact;
    // no underflow is possible for binary32 inputs), det is the one rounding
    // of the exact determinant and has its sign.
    if (diff_exact(ax, ox) && diff_exact(by, oy) && diff_exact(ay, oy) && diff_exact(bx, ox) &&
        fma(dx1, dy2, -l) == 0.0 && fma(dy1, dx2, -r) == 0.0)
        return (det > 0.0) ? 1 : ((det < 0.0) ? -1 : 0);
    return orient_exact_dev(ox, oy, ax, ay, bx, by);
}

// ---------------------------------------------------------------------------
// chunk chains
// ---------------------------------------------------------------------------
// Thread c takes positions [c*C, min(m, (c+1)*C)) of the sorted keys and
// writes the positions of its strict lower chain (sign = 1: pop while the
// turn is not counter-clockwise) or upper chain (sign = -1) to
// out[c*C ...], their number to cnt[c].  With toff, the positions are those
// of the run pass's output packed together: tile t (of kRunTile slots)
// holds toff[t+1] - toff[t] keys from slot t*kRunTile on (toff is the
// exclusive scan of the tile counts, ntiles entries, m their total), so
// position p lies in the tile t with toff[t] <= p < toff[t+1], at slot
// t*kRunTile + p - toff[t]; the chain's entries are then slots.
//
// The stack lives in LDS: per entry its coordinates and its offset in the
// chunk (CMAX * 64 * 9 bytes per block of 64 threads), so a pop reads LDS
// only, and the chain is copied out at the end.
constexpr uint32_t kChainMaxC = 64;
constexpr uint32_t kChainPrefetch = 16;   // keys loaded together

// Slot of packed position p, walking forward from tile t (tile t spans
// packed positions [tb, te)).
struct TileWalk {
    uint32_t t, tb, te;
};
__device__ __forceinline__ TileWalk tile_of(const uint32_t* __restrict__ toff, uint32_t ntiles, uint32_t m,
                                            uint32_t p) {
    uint32_t lo = 0, hi = ntiles - 1;   // the largest t with toff[t] <= p
    while (lo < hi) {
        const uint32_t mid = (lo + hi + 1u) / 2u;
        if (toff[mid] <= p) lo = mid;
        else hi = mid - 1u;
    }
    return TileWalk{lo, toff[lo], (lo + 1u < ntiles) ? toff[lo + 1u] : m};
}
__device__ __forceinline__ uint32_t slot_of(const uint32_t* __restrict__ toff, uint32_t ntiles, uint32_t m,
                                            TileWalk& w, uint32_t p) {
    while (p >= w.te) {
        ++w.t;
        w.tb = w.te;
        w.te = (w.t + 1u < ntiles) ? toff[w.t + 1u] : m;
    }
    return w.t * kRunTile + (p - w.tb);
}

//
// With a split sp (pieces of C: a batch, chunks never cross a set) chunk c
// is piece c instead; its chain still goes to out[c*C ...].
template <uint32_t CMAX>
__global__ __launch_bounds__(64) void k_chain(const uint64_t* __restrict__ keys, uint32_t m, uint32_t C, int sign,
                                              const uint32_t* __restrict__ toff, uint32_t ntiles, SetSplit sp,
                                              uint32_t nct, uint32_t* __restrict__ out, uint32_t* __restrict__ cnt) {
    static_assert(CMAX <= kChainMaxC && CMAX <= 256u, "stack offsets are one byte");
    __shared__ uint8_t sh_st[CMAX][64];
    __shared__ float2 sh_xy[CMAX][64];
    const uint32_t c = blockIdx.x * 64u + threadIdx.x;
    const uint32_t nch = sp.first ? nct : (m + C - 1) / C;
    if (c >= nch) return;
    uint32_t b, e;
    if (sp.first) {
        uint32_t set;
        piece_of(sp, c, set, b, e);
    } else {
        b = c * C;
        e = min(m, b + C);
    }
    uint8_t* st = &sh_st[0][threadIdx.x];   // entry j at st[64 * j]: lanes hit distinct banks
    float2* sxy = &sh_xy[0][threadIdx.x];
    TileWalk w0{0u, 0u, 0xFFFFFFFFu};
    if (toff) w0 = tile_of(toff, ntiles, m, b);
    TileWalk w = w0;
    uint32_t len = 0;
    float x1 = 0.f, y1 = 0.f, x2 = 0.f, y2 = 0.f;   // top (2) and below-top (1) of the stack
    // The chunk's keys are read kChainPrefetch at a time, the next batch's
    // loads issued before the current batch is walked.
    uint64_t kb[kChainPrefetch];
#pragma unroll
    for (uint32_t u = 0; u < kChainPrefetch; ++u) {
        const uint32_t p = b + u;
        kb[u] = (p < e) ? keys[toff ? slot_of(toff, ntiles, m, w, p) : p] : 0ull;
    }
    for (uint32_t i0 = b; i0 < e; i0 += kChainPrefetch) {
        uint64_t kn[kChainPrefetch];
#pragma unroll
        for (uint32_t u = 0; u < kChainPrefetch; ++u) {
            const uint32_t p = i0 + kChainPrefetch + u;
            kn[u] = (p < e) ? keys[toff ? slot_of(toff, ntiles, m, w, p) : p] : 0ull;
        }
#pragma unroll
        for (uint32_t u = 0; u < kChainPrefetch; ++u) {
            const uint32_t i = i0 + u;
            if (i >= e) break;
            const uint64_t k = kb[u];
            const float x = key_x(k), y = key_y(k);
            while (len >= 2 && orient_dev(x1, y1, x2, y2, x, y) * sign <= 0) {
                --len;
                x2 = x1;
                y2 = y1;
                if (len >= 2) {
                    const float2 q = sxy[64u * (len - 2)];
                    x1 = q.x;
                    y1 = q.y;
                }
            }
            st[64u * len] = (uint8_t)(i - b);
            sxy[64u * len] = make_float2(x, y);
            ++len;
            x1 = x2;
            y1 = y2;
            x2 = x;
            y2 = y;
        }
#pragma unroll
        for (uint32_t u = 0; u < kChainPrefetch; ++u) kb[u] = kn[u];
    }
    uint32_t* o = out + (uint64_t)c * C;
    for (uint32_t j = 0; j < len; ++j) {
        const uint32_t p = b + st[64u * j];
        o[j] = toff ? slot_of(toff, ntiles, m, w0, p) : p;
    }
    cnt[c] = len;
}

// Run representatives of keys sorted by x alone (stable, so every run of
// equal x holds its points in ascending index order), both sides in one
// pass: for the lower side (rk0 / rv0) the first point of least y of each
// run, for the upper side (rk1 / rv1) the first point of greatest y.  A
// point above (below) another of the same x is no strict vertex of the
// lower (upper) hull, except the two ends of the hull's chains: the
// lexicographically greatest point ends the lower chain and the smallest
// starts the upper one; the host adds those two back when it joins the
// chains.
//
// Wave w owns the runs whose first point lies in its tile, positions
// [w*T, (w+1)*T) with T = kRunTile, and writes their representatives, in
// order, to rk0/rv0 and rk1/rv1 [w*T ...] (key and value; at most T) and
// their number to cnt[w].  It walks the tile 64 positions a step (lane l reads position
// i0 + l; the tile's loads are all issued before the first step), and past
// the tile's end while a run it owns is still open.  In a step every lane
// needs the least (y', position) of its run so far, y' the order-preserving
// bits of y for the lower side and their complement for the upper, so the
// least is the first point of least (greatest) y: a prefix minimum over the
// lanes of (64 - g, y', lane), g the number of run heads at or below the
// lane, in which lanes of earlier runs (smaller g) never win.  The run open
// at the end of a step is carried into the next.
constexpr uint32_t kRunSteps = kRunTile / 64u;

// v from the lane CTRL names (row_shr within rows of 16, or a row
// broadcast into the rows of ROWS); all ones where there is none.
template <int CTRL, int ROWS>
__device__ __forceinline__ uint64_t dpp_u64(uint64_t v) {
    const uint32_t lo = (uint32_t)__builtin_amdgcn_update_dpp(-1, (int)(uint32_t)v, CTRL, ROWS, 0xF, false);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_update_dpp(-1, (int)(uint32_t)(v >> 32), CTRL, ROWS, 0xF, false);
    return ((uint64_t)hi << 32) | lo;
}

// Inclusive prefix minimum over the lanes of the wave: within rows of 16
// (row_shr 1, 2, 4, 8), then row 0's last lane into row 1 and row 2's into
// row 3 (row_bcast:15), then lane 31 into rows 2 and 3 (row_bcast:31).
__device__ __forceinline__ uint64_t wave_prefix_min(uint64_t v) {
    v = min(v, dpp_u64<0x111, 0xF>(v));
    v = min(v, dpp_u64<0x112, 0xF>(v));
    v = min(v, dpp_u64<0x114, 0xF>(v));
    v = min(v, dpp_u64<0x118, 0xF>(v));
    v = min(v, dpp_u64<0x142, 0xA>(v));
    v = min(v, dpp_u64<0x143, 0xC>(v));
    return v;
}

struct RunCarry {
    bool open;       // a run is open before this step
    bool own;        // the wave owns it
    uint32_t x;      // its x (ordered bits)
    uint64_t best[2];   // per side: least (y', position) of it so far
    uint32_t val[2];    // the value at that position
};

// One step at positions [i0, i0 + 64) (key k and value kv per lane), both
// sides at once (the runs, and so the output slots, are the same; side 0
// takes y' = the ordered bits of y, side 1 their complement); false once
// the wave is done.
__device__ __forceinline__ bool run_step(uint64_t k, uint32_t kv, uint32_t i0, uint32_t m, uint32_t e, uint32_t lane,
                                         uint64_t upto, RunCarry& c, uint64_t* __restrict__ rk0,
                                         uint32_t* __restrict__ rv0, uint64_t* __restrict__ rk1,
                                         uint32_t* __restrict__ rv1, uint32_t& len) {
    const uint32_t i = i0 + lane;
    const bool valid = i < m;
    const uint32_t kx = (uint32_t)(k >> 32);
    const uint32_t px = (uint32_t)__shfl_up((int)kx, 1, 64);
    const bool head = !valid || (lane == 0u ? (!c.open || kx != c.x) : kx != px);
    const uint64_t H = __ballot(head);
    const uint32_t g = (uint32_t)__popcll(H & upto);   // runs starting at or below this lane
    const uint64_t runs = (uint64_t)(64u - g) << 40;
    const bool carried = g == 0u;   // this lane is in the run carried in
    uint64_t sb[2];
    uint32_t svb[2];
#pragma unroll
    for (int side = 0; side < 2; ++side) {
        const uint32_t ky = side == 0 ? (uint32_t)k : ~(uint32_t)k;
        const uint64_t v = wave_prefix_min(runs | ((uint64_t)ky << 6) | lane);
        sb[side] = ((uint64_t)(uint32_t)(v >> 6) << 32) | (i0 + (uint32_t)(v & 63u));
        svb[side] = (uint32_t)__shfl((int)kv, (int)(v & 63u), 64);
        if (carried && c.best[side] < sb[side]) {
            sb[side] = c.best[side];
            svb[side] = c.val[side];
        }
    }
    const bool own = carried ? c.own : (i0 < e);
    const bool end = valid && (lane < 63u ? ((H >> lane) & 2ull) != 0ull : i + 1u == m);
    const bool emit = end && own;
    const bool cemit = c.open && c.own && (H & 1ull) != 0ull;   // the carried run ended at i0 - 1
    const uint64_t E = __ballot(emit);
    const uint32_t base = len + (cemit ? 1u : 0u);
    if (cemit && lane == 0u) {
        rk0[len] = ((uint64_t)c.x << 32) | (uint32_t)(c.best[0] >> 32);
        rv0[len] = c.val[0];
        rk1[len] = ((uint64_t)c.x << 32) | ~(uint32_t)(c.best[1] >> 32);
        rv1[len] = c.val[1];
    }
    if (emit) {
        const uint32_t o = base + (uint32_t)__popcll(E & (upto >> 1));
        rk0[o] = ((uint64_t)kx << 32) | (uint32_t)(sb[0] >> 32);
        rv0[o] = svb[0];
        rk1[o] = ((uint64_t)kx << 32) | ~(uint32_t)(sb[1] >> 32);
        rv1[o] = svb[1];
    }
    len = base + (uint32_t)__popcll(E);
    if (i0 + 64u >= m) return false;
    c.x = (uint32_t)__shfl((int)kx, 63, 64);
#pragma unroll
    for (int side = 0; side < 2; ++side) {
        c.best[side] = __shfl(sb[side], 63, 64);
        c.val[side] = (uint32_t)__shfl((int)svb[side], 63, 64);
    }
    c.own = __shfl((int)own, 63, 64) != 0;
    c.open = true;
    return !(i0 + 64u >= e && !c.own);   // past the tile with no owned run open: done
}

// With a split sp (pieces of kRunTile) the keys are a batch of sets sorted
// each on its own: wave w takes the runs that start in its piece, walks at
// most to its set's end (runs never cross sets), and a piece that starts a
// set has no run open before it.
__global__ __launch_bounds__(256) void k_runs(const uint64_t* __restrict__ keys, const uint32_t* __restrict__ vals,
                                              uint32_t m, SetSplit sp, uint64_t* __restrict__ rk0,
                                              uint32_t* __restrict__ rv0, uint64_t* __restrict__ rk1,
                                              uint32_t* __restrict__ rv1, uint32_t* __restrict__ cnt) {
    const uint32_t lane = threadIdx.x & 63u;
    const uint32_t w = blockIdx.x * 4u + (threadIdx.x >> 6);
    const uint32_t nt = sp.first ? sp.first[sp.S] : (m + kRunTile - 1u) / kRunTile;
    if (w >= nt) return;   // whole waves only
    uint32_t b, e, se;
    bool first;
    if (sp.first) {
        uint32_t set;
        piece_of(sp, w, set, b, e);
        se = sp.start[set + 1u];
        first = w == sp.first[set];
    } else {
        b = w * kRunTile;
        e = min(m, b + kRunTile);
        se = m;
        first = b == 0u;
    }
    const uint64_t upto = (2ull << lane) - 1ull;   // this lane and those below (lane 63: all)
    uint64_t kr[kRunSteps];
    uint32_t vr[kRunSteps];
#pragma unroll
    for (uint32_t u = 0; u < kRunSteps; ++u) {
        const uint32_t i = b + 64u * u + lane;
        kr[u] = (i < se) ? keys[i] : 0ull;
        vr[u] = (i < se) ? vals[i] : 0u;
    }
    // a run open at b started in the previous tile: not this wave's
    RunCarry c{!first, false, first ? 0u : (uint32_t)(keys[b - 1u] >> 32), {~0ull, ~0ull}, {0u, 0u}};
    const uint64_t o0 = (uint64_t)w * kRunTile;   // tile w's slots
    uint64_t* ok0 = rk0 + o0;
    uint32_t* ov0 = rv0 + o0;
    uint64_t* ok1 = rk1 + o0;
    uint32_t* ov1 = rv1 + o0;
    uint32_t len = 0;
    bool more = true;
#pragma unroll
    for (uint32_t u = 0; u < kRunSteps; ++u) {
        more = run_step(kr[u], vr[u], b + 64u * u, se, e, lane, upto, c, ok0, ov0, ok1, ov1, len);
        if (!more) break;
    }
    // past the tile: the owned run still open
    for (uint32_t i0 = b + kRunTile; more; i0 += 64u) {
        const uint32_t i = i0 + lane;
        more = run_step((i < se) ? keys[i] : 0ull, (i < se) ? vals[i] : 0u, i0, se, e, lane, upto, c, ok0, ov0, ok1,
                        ov1, len);
    }
    if (lane == 0u) cnt[w] = len;
}

// Exclusive scan in place of a[b, b + 4096) (clipped to n) by a block of
// 1024, starting from `carry`; returns the segment's total (every thread).
// Four consecutive counts per thread, a shuffle scan inside each wave, and
// one LDS exchange of the 16 wave totals.
__device__ __forceinline__ uint32_t scan_4096(uint32_t* __restrict__ a, uint32_t b, uint32_t n, uint32_t carry,
                                              uint32_t* wsum) {
    constexpr int NW = 1024 / 64;
    const uint32_t t = threadIdx.x, lane = t & 63u, wave = t >> 6;
    uint32_t v[4], s = 0;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const uint32_t i = b + 4u * t + (uint32_t)q;
        v[q] = (i < n) ? a[i] : 0u;
        s += v[q];
    }
    uint32_t incl = s;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const uint32_t u = (uint32_t)__shfl_up((int)incl, o, 64);
        if ((int)lane >= o) incl += u;
    }
    if (lane == 63u) wsum[wave] = incl;
    __syncthreads();
    uint32_t before = carry, all = 0;
#pragma unroll
    for (int w = 0; w < NW; ++w) {
        const uint32_t x = wsum[w];
        if (w < (int)wave) before += x;
        all += x;
    }
    uint32_t e = before + incl - s;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const uint32_t i = b + 4u * t + (uint32_t)q;
        if (i < n) a[i] = e;
        e += v[q];
    }
    __syncthreads();   // every thread has read wsum
    return all;
}

// Exclusive scan of n counts in place (one block of 1024, 4096 counts a
// round); the total goes to *total.
__global__ __launch_bounds__(1024) void k_scan_counts(uint32_t* __restrict__ a, uint32_t n, uint32_t* total) {
    __shared__ uint32_t wsum[16];
    uint32_t carry = 0;
    for (uint32_t b = 0; b < n; b += 4096u) carry += scan_4096(a, b, n, carry, wsum);
    if (threadIdx.x == 0) *total = carry;
}

// Many counts: block k sums a[4096k, 4096(k+1)) into bs[k]; bs is then
// scanned by k_scan_counts, and k_scan_apply scans each segment from its
// offset.
__global__ __launch_bounds__(1024) void k_scan_blocksum(const uint32_t* __restrict__ a, uint32_t n,
                                                        uint32_t* __restrict__ bs) {
    __shared__ uint32_t wsum[16];
    const uint32_t t = threadIdx.x, lane = t & 63u, wave = t >> 6;
    const uint32_t b = blockIdx.x * 4096u;
    uint32_t s = 0;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const uint32_t i = b + 4u * t + (uint32_t)q;
        s += (i < n) ? a[i] : 0u;
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) s += (uint32_t)__shfl_xor((int)s, o, 64);
    if (lane == 0u) wsum[wave] = s;
    __syncthreads();
    if (t == 0) {
        uint32_t all = 0;
        for (int w = 0; w < 16; ++w) all += wsum[w];
        bs[blockIdx.x] = all;
    }
}

__global__ __launch_bounds__(1024) void k_scan_apply(uint32_t* __restrict__ a, uint32_t n,
                                                     const uint32_t* __restrict__ bs) {
    __shared__ uint32_t wsum[16];
    (void)scan_4096(a, blockIdx.x * 4096u, n, bs[blockIdx.x], wsum);
}

// Chain vertices of every chunk, in order: chunk c's entries chain[c*C + j]
// (j < its length, i.e. next offset - offset) go to position off[c] + j.
// One thread per slot of the chain array (chunk chains are short: a wave
// per chunk left most lanes idle).
__global__ __launch_bounds__(256) void k_chain_gather(const uint64_t* __restrict__ keys,
                                                      const uint32_t* __restrict__ vals, uint32_t nch, uint32_t C,
                                                      const uint32_t* __restrict__ chain,
                                                      const uint32_t* __restrict__ off, uint32_t total,
                                                      uint64_t* __restrict__ kout, uint32_t* __restrict__ vout) {
    const uint32_t slots = nch * C;   // slots + the grid stride < 2^32 (checked at launch)
    for (uint32_t i = blockIdx.x * 256u + threadIdx.x; i < slots; i += gridDim.x * 256u) {
        const uint32_t c = i / C, j = i - c * C;
        const uint32_t o = off[c];
        const uint32_t end = (c + 1 < nch) ? off[c + 1] : total;
        if (o + j < end) {
            const uint32_t src = chain[i];
            kout[o + j] = keys[src];
            vout[o + j] = vals[src];
        }
    }
}

// ---------------------------------------------------------------------------
// merge tree of chains
// ---------------------------------------------------------------------------
// Chains c = 0..nc-1 occupy [off[c], off[c+1]) of the key array, each a
// strict lower (sign 1) or upper (sign -1) chain of consecutive points of
// the sorted sequence, so every point of chain 2p precedes every point of
// chain 2p+1.  The hull of their union is a prefix A[0..i*] of the left
// chain A followed by a suffix B[j*..] of the right chain B (the bridge).
// With s(a, b, c) = sign * orient(a, b, c):
//   tangent from a point q before B: t(q) = the first j with
//     s(q, B[j], B[j+1]) > 0 (else the last index) -- the slopes from q to
//     the vertices of the convex chain B fall and then rise, and t(q) is the
//     last vertex of least slope, so B points collinear with q and B[t(q)]
//     lie between them and are not strict vertices;
//   i* = the first i with s(A[i], B[t(A[i])], A[i+1]) >= 0 (else the last
//     index): left of i* the next vertex of A lies strictly below the
//     tangent line (A[i+1] is a hull vertex), from i* on it does not, and
//     the first such i is the left end of the bridge when several A points
//     lie on it;
//   j* = t(A[i*]).
// Both searches are over monotone predicates.  The tangent search is
// wave-parallel (64 samples per step); the search over A is a binary search
// whose steps each run one tangent search.
__device__ __forceinline__ int orient_keys(uint64_t a, uint64_t b, uint64_t c) {
    return orient_dev(key_x(a), key_y(a), key_x(b), key_y(b), key_x(c), key_y(c));
}

// First j in [0, lb) with j == lb - 1 or s(q, B[j], B[j+1]) > 0 (lb >= 1);
// every lane returns it.
__device__ __forceinline__ uint32_t tangent_from(const uint64_t* __restrict__ B, uint32_t lb, uint64_t q, int sign) {
    const uint32_t lane = threadIdx.x & 63u;
    uint32_t lo = 0, hi = lb - 1;   // the answer is in [lo, hi]; the predicate holds at hi
    while (hi > lo) {
        const uint32_t n = hi - lo;
        const uint32_t step = (n + 63u) / 64u;
        const uint32_t at = lo + (lane + 1u) * step - 1u;   // lane samples: the last one reaches hi - 1
        bool v = true;
        if (at < hi) v = orient_keys(q, B[at], B[at + 1u]) * sign > 0;
        const unsigned long long m = __ballot(v);
        if (m == 0ull) {   // every sample (up to hi - 1) fails: the answer is hi
            lo = hi;
            break;
        }
        const uint32_t f = (uint32_t)(__ffsll((long long)m) - 1);
        const uint32_t af = lo + (f + 1u) * step - 1u;
        const uint32_t nlo = (f == 0u) ? lo : lo + f * step;   // one past the previous sample
        hi = min(af, hi);
        lo = nlo;
    }
    return lo;
}

// Pair p merges chains 2p and 2p+1 (if there is one), or, in a batch, the
// one or two chains of piece p of a split of size 2 over each set's chains:
// the pairs never cross a set.
__device__ __forceinline__ void pair_of(const SetSplit& sp, uint32_t nc, uint32_t p, uint32_t& left, bool& right) {
    if (sp.first) {
        uint32_t set, e;
        piece_of(sp, p, set, left, e);
        right = e - left == 2u;
    } else {
        left = 2u * p;
        right = 2u * p + 1u < nc;
    }
}

__global__ __launch_bounds__(256) void k_bridge(const uint64_t* __restrict__ keys, const uint32_t* __restrict__ off,
                                                uint32_t nc, int sign, SetSplit sp, uint32_t np_tab,
                                                uint2* __restrict__ br, uint32_t* __restrict__ len) {
    const uint32_t lane = threadIdx.x & 63u;
    const uint32_t np = sp.first ? np_tab : (nc + 1u) / 2u;
    for (uint32_t p = blockIdx.x * 4u + (threadIdx.x >> 6); p < np; p += gridDim.x * 4u) {
        uint32_t left;
        bool right;
        pair_of(sp, nc, p, left, right);
        const uint32_t a0 = off[left], a1 = off[left + 1u];
        const uint32_t b1 = right ? off[left + 2u] : a1;
        const uint32_t la = a1 - a0, lb = b1 - a1;
        uint32_t keep = la, j = 0;   // A[0..keep) ++ B[j..lb)
        if (la > 0u && lb > 0u) {
            const uint64_t* A = keys + a0;
            const uint64_t* B = keys + a1;
            uint32_t lo = 0, hi = la - 1u;
            while (lo < hi) {
                const uint32_t mid = (lo + hi) / 2u;
                const uint64_t am = A[mid];
                const uint32_t t = tangent_from(B, lb, am, sign);
                if (orient_keys(am, B[t], A[mid + 1u]) * sign >= 0) hi = mid;
                else lo = mid + 1u;
            }
            keep = lo + 1u;
            j = tangent_from(B, lb, A[lo], sign);
        }
        if (lane == 0u) {
            br[p] = make_uint2(keep, j);
            len[p] = keep + (lb - j);
        }
    }
}

// The merged chains in order: pair p's chain goes to noff[p].  Task
// (p, c) copies part c of pair p's merged chain (bpp parts per pair), so
// that the last rounds, with few and long chains, still spread the copy
// over many waves.
__global__ __launch_bounds__(256) void k_merge_gather(const uint64_t* __restrict__ keys,
                                                      const uint32_t* __restrict__ vals,
                                                      const uint32_t* __restrict__ off, uint32_t nc,
                                                      SetSplit sp, uint32_t np_tab, const uint2* __restrict__ br,
                                                      const uint32_t* __restrict__ noff, uint32_t bpp,
                                                      uint64_t* __restrict__ kout, uint32_t* __restrict__ vout) {
    const uint32_t np = sp.first ? np_tab : (nc + 1u) / 2u;
    const uint64_t tasks = (uint64_t)np * bpp;
    for (uint64_t task = blockIdx.x; task < tasks; task += gridDim.x) {
        const uint32_t p = (uint32_t)(task / bpp), c = (uint32_t)(task % bpp);
        uint32_t left;
        bool right;
        pair_of(sp, nc, p, left, right);
        const uint32_t a0 = off[left], a1 = off[left + 1u];
        const uint32_t b1 = right ? off[left + 2u] : a1;
        const uint2 r = br[p];
        const uint32_t o = noff[p];
        const uint32_t len = r.x + ((b1 - a1) - r.y);
        const uint32_t k0 = (uint32_t)((uint64_t)len * c / bpp), k1 = (uint32_t)((uint64_t)len * (c + 1u) / bpp);
        for (uint32_t k = k0 + threadIdx.x; k < k1; k += 256u) {
            const uint32_t src = (k < r.x) ? a0 + k : a1 + r.y + (k - r.x);
            kout[o + k] = keys[src];
            vout[o + k] = vals[src];
        }
    }
}

// Few survivors for the host chain, in one block of (page-locked host)
// memory: stage = [count (u64), pad, points (float2 x cap), indices (u32 x
// cap)]; the points and indices only when count <= cap (the count read on
// the device: the filter's, or an error code).
__global__ __launch_bounds__(256) void k_stage_small(const float2* __restrict__ pts, uint64_t n,
                                                     const uint32_t* __restrict__ surv,
                                                     const uint64_t* __restrict__ count, uint32_t cap,
                                                     unsigned char* __restrict__ stage) {
    const uint64_t c = *count;
    if (blockIdx.x == 0 && threadIdx.x == 0) *reinterpret_cast<uint64_t*>(stage) = c;
    if (c > cap) return;
    float2* xy = reinterpret_cast<float2*>(stage + 16);
    uint32_t* idx = reinterpret_cast<uint32_t*>(stage + 16 + 8ull * cap);
    for (uint32_t i = blockIdx.x * 256u + threadIdx.x; i < (uint32_t)c; i += gridDim.x * 256u) {
        const uint32_t k = surv[i];
        xy[i] = (k < n) ? pts[k] : make_float2(__builtin_nanf(""), __builtin_nanf(""));
        idx[i] = k;
    }
}

__global__ void k_copy_u32(uint32_t* dst, const uint32_t* src) { *dst = *src; }

// dst[i] = src[idx[i]] for i < n.
__global__ __launch_bounds__(256) void k_take_u32(const uint32_t* __restrict__ src, const uint32_t* __restrict__ idx,
                                                  uint32_t n, uint32_t* __restrict__ dst) {
    for (uint32_t i = blockIdx.x * 256u + threadIdx.x; i < n; i += gridDim.x * 256u) dst[i] = src[idx[i]];
}

}  // namespace

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------

uint32_t finish_sort_tiles(uint32_t m) { return (m + kRsTile - 1) / kRsTile; }

hipError_t launch_finish_keys(const float2* pts, uint64_t n, const uint32_t* surv, uint32_t m, uint64_t* keys,
                              uint32_t* vals, uint64_t* bad, int grid, hipStream_t stream) {
    hipLaunchKernelGGL(k_fin_keys, dim3(grid), dim3(256), 0, stream, pts, n, surv, m, keys, vals, bad);
    return hipGetLastError();
}

hipError_t launch_finish_sort(uint64_t* keys, uint32_t* vals, uint64_t* keys2, uint32_t* vals2, uint32_t m,
                              uint32_t* hist, uint32_t* rowsum, uint32_t first_shift, hipStream_t stream) {
    const uint32_t tiles = finish_sort_tiles(m);
    uint64_t* ka = keys;
    uint32_t* va = vals;
    uint64_t* kb = keys2;
    uint32_t* vb = vals2;
    for (uint32_t shift = first_shift; shift < 64; shift += 8) {
        hipLaunchKernelGGL(k_rs_hist, dim3(tiles), dim3(kRsBlock), 0, stream, ka, m, shift, tiles, SetSplit{}, hist);
        hipLaunchKernelGGL(k_rs_rowsum, dim3(kRsBins), dim3(256), 0, stream, hist, tiles, rowsum);
        hipLaunchKernelGGL(k_rs_rowscan, dim3(kRsBins), dim3(256), 0, stream, hist, tiles, rowsum, nullptr);
        hipLaunchKernelGGL(k_rs_scatter, dim3(tiles), dim3(kRsBlock), 0, stream, ka, va, m, shift, tiles, hist,
                           SetSplit{}, nullptr, kb, vb);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
        std::swap(ka, kb);
        std::swap(va, vb);
    }
    return hipSuccess;   // an even number of passes: the result is back in keys / vals
}

hipError_t launch_finish_sort_sets(uint64_t* keys, uint32_t* vals, uint64_t* keys2, uint32_t* vals2, uint32_t m,
                                   const SetSplit& sp, uint32_t tiles, uint32_t* hist, uint32_t* rowend, uint32_t* sdp,
                                   hipStream_t stream) {
    if (tiles == 0u) return hipSuccess;
    if (sp.first == nullptr || sp.size != kRsTile) return hipErrorInvalidValue;
    uint64_t* ka = keys;
    uint32_t* va = vals;
    uint64_t* kb = keys2;
    uint32_t* vb = vals2;
    for (uint32_t shift = 32; shift < 64; shift += 8) {
        hipLaunchKernelGGL(k_rs_hist, dim3(tiles), dim3(kRsBlock), 0, stream, ka, m, shift, tiles, sp, hist);
        hipLaunchKernelGGL(k_rs_rowscan, dim3(kRsBins), dim3(256), 0, stream, hist, tiles, nullptr, rowend);
        hipLaunchKernelGGL(k_rs_setpre, dim3(sp.S), dim3(kRsBins), 0, stream, hist, tiles, rowend, sp, sdp);
        hipLaunchKernelGGL(k_rs_scatter, dim3(tiles), dim3(kRsBlock), 0, stream, ka, va, m, shift, tiles, hist, sp,
                           sdp, kb, vb);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
        std::swap(ka, kb);
        std::swap(va, vb);
    }
    return hipSuccess;   // four passes: the result is back in keys / vals
}

hipError_t launch_bfin_keys(const float2* pts, const uint64_t* off, const uint32_t* surv, const SetSplit& sp,
                            uint32_t tiles, uint64_t* keys, uint32_t* vals, uint64_t* bad, hipStream_t stream) {
    if (tiles == 0u) return hipSuccess;
    hipLaunchKernelGGL(k_bfin_keys, dim3(tiles), dim3(256), 0, stream, pts, off, surv, sp, keys, vals, bad);
    return hipGetLastError();
}

hipError_t launch_chain(const uint64_t* keys, uint32_t m, uint32_t C, int sign, const uint32_t* toff,
                        uint32_t ntiles, uint32_t* chain, uint32_t* cnt, hipStream_t stream, const SetSplit& sp,
                        uint32_t nsp) {
    if (C == 0 || C > kChainMaxC || (toff && ntiles == 0) || (sp.first && sp.size != C))
        return hipErrorInvalidValue;
    const uint32_t nch = sp.first ? nsp : (m + C - 1) / C;
    if (nch == 0) return hipSuccess;
    const dim3 grid((nch + 63) / 64);
    if (C <= 32u)
        hipLaunchKernelGGL(k_chain<32>, grid, dim3(64), 0, stream, keys, m, C, sign, toff, ntiles, sp, nsp, chain,
                           cnt);
    else
        hipLaunchKernelGGL(k_chain<64>, grid, dim3(64), 0, stream, keys, m, C, sign, toff, ntiles, sp, nsp, chain,
                           cnt);
    return hipGetLastError();
}

hipError_t launch_runs(const uint64_t* keys, const uint32_t* vals, uint32_t m, uint64_t* rk0, uint32_t* rv0,
                       uint64_t* rk1, uint32_t* rv1, uint32_t* cnt, hipStream_t stream, const SetSplit& sp,
                       uint32_t nsp) {
    const uint32_t nt = sp.first ? nsp : (m + kRunTile - 1u) / kRunTile;
    if (nt == 0u) return hipSuccess;
    hipLaunchKernelGGL(k_runs, dim3((nt + 3u) / 4u), dim3(256), 0, stream, keys, vals, m, sp, rk0, rv0, rk1, rv1,
                       cnt);
    return hipGetLastError();
}

hipError_t launch_scan_counts(uint32_t* cnt, uint32_t n, uint32_t* total, uint32_t* blk, hipStream_t stream) {
    const uint32_t nb = (n + 4095u) / 4096u;
    if (nb <= 4u || blk == nullptr) {
        hipLaunchKernelGGL(k_scan_counts, dim3(1), dim3(1024), 0, stream, cnt, n, total);
        return hipGetLastError();
    }
    hipLaunchKernelGGL(k_scan_blocksum, dim3(nb), dim3(1024), 0, stream, cnt, n, blk);
    hipLaunchKernelGGL(k_scan_counts, dim3(1), dim3(1024), 0, stream, blk, nb, total);
    hipLaunchKernelGGL(k_scan_apply, dim3(nb), dim3(1024), 0, stream, cnt, n, blk);
    return hipGetLastError();
}

hipError_t launch_chain_gather(const uint64_t* keys, const uint32_t* vals, uint32_t nch, uint32_t C,
                               const uint32_t* chain, const uint32_t* off, uint32_t total, uint64_t* kout,
                               uint32_t* vout, int grid, hipStream_t stream) {
    // slot indices and the grid stride stay below 2^32
    if (C == 0 || grid <= 0 || (uint64_t)nch * C + (uint64_t)grid * 256u >= (1ull << 32))
        return hipErrorInvalidValue;
    if (nch == 0) return hipSuccess;
    hipLaunchKernelGGL(k_chain_gather, dim3(grid), dim3(256), 0, stream, keys, vals, nch, C, chain, off, total, kout,
                       vout);
    return hipGetLastError();
}

hipError_t launch_copy_u32(uint32_t* dst, const uint32_t* src, hipStream_t stream) {
    hipLaunchKernelGGL(k_copy_u32, dim3(1), dim3(1), 0, stream, dst, src);
    return hipGetLastError();
}

uint64_t stage_small_bytes(uint32_t cap) { return 16ull + 12ull * cap; }

hipError_t launch_stage_small(const float2* pts, uint64_t n, const uint32_t* surv, const uint64_t* count,
                              uint32_t cap, unsigned char* stage, hipStream_t stream) {
    hipLaunchKernelGGL(k_stage_small, dim3(std::max<uint32_t>(1u, std::min<uint32_t>((cap + 255u) / 256u, 16u))),
                       dim3(256), 0, stream, pts, n, surv, count, cap, stage);
    return hipGetLastError();
}

hipError_t launch_take_u32(const uint32_t* src, const uint32_t* idx, uint32_t n, uint32_t* dst, hipStream_t stream) {
    if (n == 0u) return hipSuccess;
    const uint32_t grid = std::min<uint32_t>((n + 255u) / 256u, 1024u);
    hipLaunchKernelGGL(k_take_u32, dim3(grid), dim3(256), 0, stream, src, idx, n, dst);
    return hipGetLastError();
}

hipError_t launch_bridge(const uint64_t* keys, const uint32_t* off, uint32_t nc, int sign, uint2* br, uint32_t* len,
                         int grid, hipStream_t stream, const SetSplit& sp, uint32_t nsp) {
    if (sp.first && sp.size != 2u) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_bridge, dim3(grid), dim3(256), 0, stream, keys, off, nc, sign, sp, nsp, br, len);
    return hipGetLastError();
}

hipError_t launch_merge_gather(const uint64_t* keys, const uint32_t* vals, const uint32_t* off, uint32_t nc,
                               const uint2* br, const uint32_t* noff, uint64_t* kout, uint32_t* vout, int grid,
                               hipStream_t stream, const SetSplit& sp, uint32_t nsp) {
    if (sp.first && sp.size != 2u) return hipErrorInvalidValue;
    const uint32_t np = sp.first ? nsp : (nc + 1u) / 2u;
    if (np == 0u) return hipSuccess;
    const uint32_t bpp = std::max<uint32_t>(1u, (uint32_t)grid / std::max<uint32_t>(np, 1u));
    const uint64_t tasks = (uint64_t)np * bpp;
    const int g = (int)std::min<uint64_t>(tasks, (uint64_t)std::max(grid, 1));
    hipLaunchKernelGGL(k_merge_gather, dim3(g), dim3(256), 0, stream, keys, vals, off, nc, sp, nsp, br, noff, bpp,
                       kout, vout);
    return hipGetLastError();
}

}  // namespace hullf
