// Internal interface between the HIP kernels (hullf_kernels.hip) and the
// host runtime (hullf_runtime.cpp).  Not part of the public C ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace hullf {

// Polygon record computed on the device from the NV extremes and read by
// every inside-test kernel (Sec. 3.2).  NV = 8: the octagon of Sec. 3.1;
// NV = 16: the 16-direction polygon of the related-work filter (Sec. 2).
//
// Edges: the non-degenerate directed edges (V_j, V_j+1) in binary64
// (vertex a, difference b-a); unused slots repeat edge 0 so that loops can
// always run over NV entries.
// Prefilter (fast == 1): for each edge, FP32 coefficients of the edge line
// scaled by a power of two s_e so that the FP32 evaluation
//   d_e = fma(A, y - cy, fma(NB, x - cx, C0))
// is within 0.5 of s_e times the exact edge value (see setup_octagon).
// Quick-accept box (bxl < x < bxh, byl < y < byh): every point inside it is
// discarded by the binary64 rule; empty when bxl > bxh.
// The four status words come first, at the same offsets for every NV.
template <int NV>
struct alignas(16) Poly {
    int32_t status;   // 0 ok, 1 non-finite input, 3 internal error (no candidate)
    int32_t mode;     // 0 keep every point (fewer than 3 distinct vertices), 1 test
    int32_t fast;     // FP32 prefilter usable
    int32_t m;        // number of non-degenerate edges
    uint32_t idx[NV];
    float bxl, bxh, byl, byh;
    float cx, cy, pad0, pad1;
    float A[NV], NB[NV], C0[NV];
    double ax[NV], ay[NV], ex[NV], ey[NV];
    // Region skip (skip == 1): a box whose four corners all have binary64
    // edge values above sm[e] on every edge lies strictly inside the rule's
    // discard region, with the margin of the quick-accept box proof.
    double sm[NV];
    int32_t skip;
    int32_t pad2[3];
};
using Octagon = Poly<8>;
using Poly16 = Poly<16>;

// Per-set bookkeeping of the batched launch (written by the plan kernel).
struct alignas(16) SetInfo {
    uint64_t begin;        // first point of the set
    uint64_t n;            // points in the set
    uint32_t r_tiles;      // reduction tiles
    uint32_t f_tiles;      // classify/compact work items
    uint32_t r_tile0;      // reduction tiles of all earlier sets (partial record offset)
    uint32_t f_tile0;      // work items of all earlier sets
};

// Batch-wide totals (device).
struct alignas(16) BatchTotals {
    uint32_t r_tiles;
    uint32_t f_tiles;
    uint32_t r_next;   // reduction-tile tickets handed out (reset by the plan)
    uint32_t pad;
};

constexpr uint64_t kCountNonFinite = ~0ull;
constexpr uint64_t kCountBadOffsets = ~0ull - 1;
constexpr uint64_t kCountInternal = ~0ull - 2;

struct Shape {
    int block;
    int ppt;
};


// Launchers (all asynchronous on `stream`; return the launch error).
// Extremes of one set in two launches: launch_reduce (grid <=
// kReduceMaxGrid) writes 9 uint64 partial records per block to `part`
// (9 * kReduceMaxGrid words, direction-major: part[j * kReduceMaxGrid + b])
// and, if box is not null, 4 boxes per reduce_chunk_points() points
// (box_count(n) float4); launch_setup merges the records and writes the
// octagon.  zero[0 .. nzero) is cleared by the same launch (the
// single-pass filter's status words).
hipError_t launch_reduce(const float2* pts, uint64_t n, unsigned long long* part, float4* box, int grid,
                         hipStream_t stream, unsigned long long* zero = nullptr, uint32_t nzero = 0);
hipError_t launch_setup(const float2* pts, uint64_t n, Octagon* oct, const unsigned long long* part,
                        uint32_t nblocks, hipStream_t stream);
constexpr int kReduceMaxGrid = 4096;
hipError_t launch_flags(const float2* pts, uint64_t n, const Octagon* oct, uint8_t* flags,
                        int grid, hipStream_t stream);
hipError_t launch_write_count(uint64_t* count, uint64_t value, hipStream_t stream);
hipError_t launch_gather(const float2* pts, const uint32_t* surv, const uint64_t* count,
                         uint64_t cap, uint64_t n, float2* out, int grid, hipStream_t stream);

uint32_t reduce_chunk_points();
bool shape_supported(Shape shape);

// Launch plan of the single-set filter (reduction, set-up, inside test,
// compaction) for n >= 1 points on a device with `cus` compute units.
// reduce_grid_max / per_cu: 0 = defaults.  Scratch sizes in elements.
struct FilterPlan {
    int reduce_grid;      // reduction blocks (partial records to merge)
    Shape shape;          // inside-test shape
    uint32_t spans;       // compaction spans per block
    int grid;             // inside-test and compaction blocks
    uint64_t bits_words;  // keep-bit words (uint64)
    uint64_t boxes;       // region-skip boxes (float4)
};
FilterPlan plan_filter(uint64_t n, int cus, Shape shape, int per_cu, int reduce_grid_max);
constexpr uint32_t kFilterMaxBlocks = 4096;   // blocks of the two compaction passes

// Two-pass compaction of one set: classify (inside test -> keep bits in
// point order, one survivor count per block), then compact (ascending
// indices).  Block b of both launches owns points [b*R, (b+1)*R) with
// R = spans * compact_span_points(); grid = ceil(n / R) blocks.
// bits: 2 * ceil(n / 128) words; blkcnt: grid words.
uint32_t compact_span_points();
bool classify_shape_supported(Shape shape);
// Region skip: box (nbox = box_count(n) boxes from launch_reduce, or null:
// no skipping); launch_classify does not read groups whose reduction box
// lies inside the discard region of the octagon.
// loaded (may be null): incremented by the number of 128-point groups read.
hipError_t launch_classify(const float2* pts, uint64_t n, const Octagon* oct, uint32_t spans, uint64_t* bits,
                           uint32_t* blkcnt, const float4* box, uint64_t nbox, unsigned long long* loaded,
                           Shape shape, int grid, hipStream_t stream);
// block: 256, 512 or 1024 threads (one span per wave and round).
hipError_t launch_compact(const uint64_t* bits, const uint32_t* blkcnt, uint64_t n, uint32_t spans,
                          const Octagon* oct, uint32_t* out, uint64_t cap, uint64_t* count, int block, int grid,
                          hipStream_t stream);

// The 16-direction filter (Sec. 2, related work): reduction of the 16
// directional keys (17 partial words per block, direction-major:
// part[j * kReduceMaxGrid + b], plus boxes as launch_reduce), the polygon
// set-up, and the inside test / compaction over its edges (same spans,
// keep bits and block counts as the octagon's launches).
constexpr int kPart16Words = 17;
hipError_t launch_reduce16(const float2* pts, uint64_t n, unsigned long long* part, float4* box, int grid,
                           hipStream_t stream);
int reduce16_grid(uint64_t n, int cus);
hipError_t launch_setup16(const float2* pts, uint64_t n, Poly16* poly, const unsigned long long* part,
                          uint32_t nblocks, hipStream_t stream);
hipError_t launch_classify(const float2* pts, uint64_t n, const Poly16* poly, uint32_t spans, uint64_t* bits,
                           uint32_t* blkcnt, const float4* box, uint64_t nbox, unsigned long long* loaded,
                           Shape shape, int grid, hipStream_t stream);
hipError_t launch_compact(const uint64_t* bits, const uint32_t* blkcnt, uint64_t n, uint32_t spans,
                          const Poly16* poly, uint32_t* out, uint64_t cap, uint64_t* count, int block, int grid,
                          hipStream_t stream);
// Single-pass filter of one set (inside test and compaction, decoupled
// look-back; after launch_reduce / launch_setup): st holds
// filter1p_tiles(n) + 1 words, zero at launch (launch_reduce clears them).
// Same outputs as launch_classify + launch_compact.
uint32_t filter1p_tiles(uint64_t n);
hipError_t launch_filter1p(const float2* pts, uint64_t n, const Octagon* oct, const float4* box, uint64_t nbox,
                           unsigned long long* st, uint32_t* out, uint64_t cap, uint64_t* count,
                           unsigned long long* loaded, hipStream_t stream);

// Batched: plan, reduction, octagon set-up, classify and compact (five
// launches).  part: 9 * max_rtiles uint64 scratch.  off: S+1 CSR offsets,
// or (seg) S (begin, count) pairs, ascending and disjoint.  bits holds
// max_items * batch_item_words() words and blkcnt max_items counts
// (max_items >= batch_max_items).
hipError_t launch_batch(const float2* pts, const uint64_t* off, bool seg, uint32_t S, uint64_t n_total,
                        SetInfo* sets, BatchTotals* tot, unsigned long long* part, uint32_t max_rtiles,
                        Octagon* octs, uint64_t* bits, uint32_t* blkcnt, uint32_t max_items, uint32_t* surv,
                        uint64_t* counts, float4* box, Shape shape, int cus, int reduce_per_cu,
                        hipStream_t stream);
uint64_t batch_max_items(uint64_t n_total, uint32_t S);
uint32_t batch_item_words();
uint64_t batch_max_rtiles(uint64_t n_total, uint32_t S);
// Region-skip boxes per reduction tile (box: max_rtiles * batch_tile_boxes()
// float4, or null for no region skip).
uint32_t batch_tile_boxes();

// Hull finishing on the device (hullf_finish.hip).
// keys: (ordered x << 32 | ordered y), vals: point indices.  The sort needs
// a second key/val buffer pair of m entries, hist of 256 * tiles words and
// rowsum of 256 words; the result is back in keys / vals.
uint32_t finish_sort_tiles(uint32_t m);
// An index >= n sets *bad (a word the caller zeroed) instead of being read.
hipError_t launch_finish_keys(const float2* pts, uint64_t n, const uint32_t* surv, uint32_t m, uint64_t* keys,
                              uint32_t* vals, uint64_t* bad, int grid, hipStream_t stream);
// Stable LSD passes of 8 bits from bit first_shift up to bit 63 (0: the
// whole key; 32: x alone); first_shift must leave an even number of passes.
hipError_t launch_finish_sort(uint64_t* keys, uint32_t* vals, uint64_t* keys2, uint32_t* vals2, uint32_t m,
                              uint32_t* hist, uint32_t* rowsum, uint32_t first_shift, hipStream_t stream);
// A batch of sets cut into pieces (sort tiles, run tiles, chain chunks,
// merge pairs): set s's items [start[s], start[s+1]) in pieces of `size`;
// piece k belongs to the set s with first[s] <= k < first[s+1] (first and
// start: S + 1 words, first[S] the number of pieces).  first == nullptr:
// not a batch.
struct SetSplit {
    const uint32_t* first = nullptr;
    const uint32_t* start = nullptr;
    uint32_t S = 0;
    uint32_t size = 0;
};
// A batch of sets, items of set s at [sp.start[s], sp.start[s+1]) (m in
// all), sort tiles = pieces of kRsTile.  launch_bfin_keys writes the keys
// and set-local indices of every set's survivors (off: S + 1 point offsets;
// surv: set s's survivors at surv + off[s]; `tiles` pieces);
// launch_finish_sort_sets sorts each set's items by x alone (stable, 4
// passes), in place.  Scratch: hist 256 * tiles words, rowend 256, sdp
// 256 * S.
hipError_t launch_bfin_keys(const float2* pts, const uint64_t* off, const uint32_t* surv, const SetSplit& sp,
                            uint32_t tiles, uint64_t* keys, uint32_t* vals, uint64_t* bad, hipStream_t stream);
hipError_t launch_finish_sort_sets(uint64_t* keys, uint32_t* vals, uint64_t* keys2, uint32_t* vals2, uint32_t m,
                                   const SetSplit& sp, uint32_t tiles, uint32_t* hist, uint32_t* rowend, uint32_t* sdp,
                                   hipStream_t stream);
// Run representatives of keys sorted by x alone (see k_runs), both sides:
// their keys and values into rk0 / rv0 (lower side) and rk1 / rv1 (upper
// side) (tile t's at t*kRunTile, cnt[t] of them on each side), counts per
// tile into cnt: ceil(m / kRunTile) tiles, or with a split sp (pieces of
// kRunTile, a batch) its nsp pieces.
constexpr uint32_t kRunTile = 1024;
hipError_t launch_runs(const uint64_t* keys, const uint32_t* vals, uint32_t m, uint64_t* rk0, uint32_t* rv0,
                       uint64_t* rk1, uint32_t* rv1, uint32_t* cnt, hipStream_t stream,
                       const SetSplit& sp = SetSplit{}, uint32_t nsp = 0);
// Chains of chunks of C sorted points (C at most 64): chain holds a slot
// per point (chunk c's chain at c*C), cnt one word per chunk: ceil(m/C)
// chunks, or with a split sp (pieces of C, never crossing a set) its nsp
// pieces.  With toff (the exclusive scan of the run pass's ntiles tile
// counts, m their total) the points are the run pass's output packed
// together and the chain entries are its slots.  sign 1 = lower, -1 =
// upper.
hipError_t launch_chain(const uint64_t* keys, uint32_t m, uint32_t C, int sign, const uint32_t* toff,
                        uint32_t ntiles, uint32_t* chain, uint32_t* cnt, hipStream_t stream,
                        const SetSplit& sp = SetSplit{}, uint32_t nsp = 0);
// Exclusive scan of n counts in place, the total to *total; blk (at least
// ceil(n / 4096) words, or null for one block) holds partial sums.
hipError_t launch_scan_counts(uint32_t* cnt, uint32_t n, uint32_t* total, uint32_t* blk, hipStream_t stream);
// Merge tree over chains c < nc at [off[c], off[c+1]) (off holds nc + 1
// words): pair p = chains 2p, 2p+1 (the last one alone when nc is odd), or
// with a split sp of size 2 over each set's chains (a batch) its nsp
// pieces.  launch_bridge writes br[p] = (points kept of the left chain,
// first point kept of the right one) and len[p] = the merged length; after
// an exclusive scan of len into noff (np + 1 words, the total last),
// launch_merge_gather writes the merged chains.
hipError_t launch_bridge(const uint64_t* keys, const uint32_t* off, uint32_t nc, int sign, uint2* br, uint32_t* len,
                         int grid, hipStream_t stream, const SetSplit& sp = SetSplit{}, uint32_t nsp = 0);
hipError_t launch_merge_gather(const uint64_t* keys, const uint32_t* vals, const uint32_t* off, uint32_t nc,
                               const uint2* br, const uint32_t* noff, uint64_t* kout, uint32_t* vout, int grid,
                               hipStream_t stream, const SetSplit& sp = SetSplit{}, uint32_t nsp = 0);
hipError_t launch_copy_u32(uint32_t* dst, const uint32_t* src, hipStream_t stream);
// The filter's count and, when it is at most cap, the survivors' points and
// indices, staged in one block of stage_small_bytes(cap) bytes: [u64 count,
// 8 bytes pad, float2 points[cap], u32 indices[cap]].
uint64_t stage_small_bytes(uint32_t cap);
hipError_t launch_stage_small(const float2* pts, uint64_t n, const uint32_t* surv, const uint64_t* count,
                              uint32_t cap, unsigned char* stage, hipStream_t stream);
// dst[i] = src[idx[i]], i < n.
hipError_t launch_take_u32(const uint32_t* src, const uint32_t* idx, uint32_t n, uint32_t* dst, hipStream_t stream);
// The chain vertices of nch chunks (chunk c's at chain[c*C ...], off: the
// exclusive scan of their lengths, total last) packed in order.
hipError_t launch_chain_gather(const uint64_t* keys, const uint32_t* vals, uint32_t nch, uint32_t C,
                               const uint32_t* chain, const uint32_t* off, uint32_t total, uint64_t* kout,
                               uint32_t* vout, int grid, hipStream_t stream);

}  // namespace hullf
