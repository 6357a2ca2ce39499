/*
 * hullf.h -- C ABI of the MI355X (gfx950) octagon filter and convex hull.
 *
 * Method: Carrasco, Ferrada, Navarro, Hitschfeld, "An Evaluation of GPU
 * Filters for Accelerating the 2D Convex Hull" (arXiv 2303.10581),
 * Algorithm 1: findingPolygon (Sec. 3.1), buildingFilter (Sec. 3.2),
 * compactingFilteredPoints (Sec. 3.2, Sec. 4.1.1), convexHull_algorithm
 * (Sec. 3.3).
 *
 * Conventions shared by every entry point
 *  - Points are FP32 (x, y) pairs stored as an array of hullf_pt (8 bytes
 *    each, x first).  Device arrays must be at least 8-byte aligned; 16-byte
 *    alignment enables the vectorised loads.
 *  - "d_" arguments are device pointers, "h_" arguments host pointers.  The
 *    caller owns every input and output buffer; the library never frees or
 *    keeps caller memory beyond the call (the batched graph cache keeps the
 *    pointer values, see hull_filter_batched).
 *  - "stream" is a hipStream_t (NULL = the default stream).  Asynchronous
 *    calls only enqueue work; synchronous ones return after the stream has
 *    drained up to their last operation.
 *  - A context serialises its own scratch memory: calls that share one
 *    context must be issued from one host thread and on one stream (or be
 *    ordered by the caller).  Different contexts are independent.
 *  - Errors come back as hullf_status; nothing aborts or throws.  After
 *    HULLF_EDEVICE the context stays usable if the device still is.
 *  - n counts points.  n must be below 2^32 (indices are uint32).
 *
 * Extremes (Sec. 3.1).  E0..E7 are, counter-clockwise from the right-most
 * point: max x, max fl32(x+y), max y, max fl32(y-x), min x, min fl32(x+y),
 * min y, max fl32(x-y).  The corner keys are the Manhattan distance to the
 * bounding-box corner up to a constant.  Ties go to the lowest index, and
 * -0 equals +0.
 *
 * Inside test (Sec. 3.2).  For each edge (a, b) = (E_j, E_j+1) whose end
 * points differ, with binary64 operations and no fused multiply-add:
 *   ex=bx-ax ey=by-ay qx=px-ax qy=py-ay l=ex*qy r=ey*qx det=l-r
 *   bnd=(3+16e)e*(|l|+|r|), e=2^-53;  strictly inside iff det > bnd.
 * A point is discarded iff it is strictly inside every such edge (and one
 * exists).  Every other point survives, so points on or within rounding
 * distance of the boundary are kept: the filter never drops a hull vertex.
 *
 * Hull (Sec. 3.3).  Strict vertices (no collinear or repeated points), the
 * lowest index per repeated coordinate, counter-clockwise, starting at the
 * lexicographically smallest (x, y), no closing repeat.  One distinct point
 * gives one vertex; collinear points give the two end points.
 */
#ifndef HULLF_H
#define HULLF_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct {
    float x, y;
} hullf_pt;

typedef struct hullf_ctx *hullf_ctx_t;

typedef enum {
    HULLF_OK = 0,
    HULLF_EINVAL = 1,      /* bad argument: null pointer, n >= 2^32, misaligned */
    HULLF_ENONFINITE = 2,  /* an input coordinate is NaN or infinite */
    HULLF_ECAPACITY = 3,   /* output capacity too small; the count is still written */
    HULLF_ENOMEM = 4,      /* allocation failed, or the context's workspace cap is reached */
    HULLF_EDEVICE = 5,     /* a HIP runtime call failed */
    HULLF_EAGAIN = 6       /* a served request is not finished yet */
} hullf_status;

/* Written to *d_count by the asynchronous calls when an input coordinate is
 * not finite (they cannot return HULLF_ENONFINITE without a host sync). */
#define HULLF_COUNT_NONFINITE UINT64_MAX
/* Written to a batched count when d_off is not a valid offset array
 * (d_off[0] != 0, decreasing, or d_off[S] != n_total), or a segment list is
 * not ascending and disjoint within n_total. */
#define HULLF_COUNT_BAD_OFFSETS (UINT64_MAX - 1)
/* Written when the device reduction produced no vertex for a direction
 * (an internal error; never expected). */
#define HULLF_COUNT_INTERNAL (UINT64_MAX - 2)

/* Create a context on HIP device `device`; it owns the scratch memory
 * (partial extreme records, octagon record, region-skip boxes, keep bits,
 * survivor staging, hull-finishing buffers) and the tuned launch shapes.
 * workspace_bytes caps the device memory the context may hold at once
 * (0 = no cap: buffers grow on demand).  Creation itself needs about 320 KB;
 * a call whose scratch would exceed the cap returns HULLF_ENOMEM without
 * enqueuing work, and the context stays usable for smaller calls.  Caller
 * buffers (points, survivors, counts) never count against it.
 * *out is set only on HULLF_OK.  Launch settings read from the environment
 * at creation (all optional; results do not depend on them):
 *   HULLF_FILTER_SHAPE=block,ppt  inside-test shape (256|512, 8|16)
 *   HULLF_REGION_SKIP=0           no region skip (every group is read)
 *   HULLF_CLASSIFY_PER_CU=k       inside-test blocks per compute unit
 *   HULLF_COMPACT_BLOCK=b         compaction block size (256|512|1024)
 *   HULLF_REDUCE_GRID=g           reduction blocks, 1..4096 (default 4 per CU)
 *   HULLF_BATCH_REDUCE_PER_CU=k   batched reduction blocks per CU (1..16)
 *   HULLF_CHAIN_CHUNK=c           sorted points per hull-chain thread (16..64,
 *                                 default 32)
 *   HULLF_SINGLE_PASS=1           hull_filter's inside test and compaction in one
 *                                 launch (decoupled look-back; slower, kept for
 *                                 comparison)
 *   HULLF_FINISH=host             hull finishing always on the host
 *   HULLF_TUNE_CACHE=path         tune cache file of the batched launch
 *                                 (default $XDG_CACHE_HOME/hullf/tune.txt or
 *                                 ~/.cache/hullf/tune.txt; empty: none) */
hullf_status hullf_create(int device, size_t workspace_bytes, hullf_ctx_t *out);

/* Release the context and its device memory.  NULL is ignored. */
void hullf_destroy(hullf_ctx_t ctx);

/* Device workspace the context holds now (*used_bytes) and its cap
 * (*cap_bytes, 0 = none). */
hullf_status hullf_workspace(hullf_ctx_t ctx, uint64_t *used_bytes, uint64_t *cap_bytes);

/* Static string for a status code. */
const char *hullf_status_str(hullf_status s);

/* Step findingPolygon of Algorithm 1 (Sec. 3.1), synchronous.
 * d_pts: n >= 1 device points.  idx_out: host array of 8 indices E0..E7.
 * Returns HULLF_ENONFINITE if a coordinate is not finite, HULLF_EINVAL for
 * n == 0. */
hullf_status hullf_octagon(hullf_ctx_t ctx, const hullf_pt *d_pts, uint64_t n,
                           uint32_t idx_out[8], void *stream);

/* Steps findingPolygon, buildingFilter and compactingFilteredPoints of
 * Algorithm 1 (Sec. 3.1, 3.2, 4.1.1), asynchronous on `stream`.
 * d_surv: device array receiving the ascending indices of the surviving
 * points; at most `cap` entries are written (cap >= n always suffices).
 * d_count: one device uint64 receiving the number of survivors (also when it
 * exceeds cap), or HULLF_COUNT_NONFINITE.  n == 0 writes 0. */
hullf_status hull_filter(hullf_ctx_t ctx, const hullf_pt *d_pts, uint64_t n,
                         uint32_t *d_surv, uint64_t cap, uint64_t *d_count,
                         void *stream);

/* Algorithm 1 end to end, synchronous: hull_filter, then the monotone-chain
 * hull (Sec. 3.3) of the survivors (hull_from_survivors).
 * h_hull: host array receiving the counter-clockwise vertex indices (into
 * d_pts) with capacity `cap`; *h_count receives the vertex count.  Returns
 * HULLF_ECAPACITY (with *h_count set) if cap is too small. */
hullf_status convex_hull(hullf_ctx_t ctx, const hullf_pt *d_pts, uint64_t n,
                         uint32_t *h_hull, uint64_t cap, uint64_t *h_count,
                         void *stream);

/* Hull finishing (Sec. 3.3) of a survivor list, synchronous.
 * d_surv: m device uint32 indices into d_pts (n points), ascending, as
 * hull_filter and the batched calls write them; every index must be below n
 * (otherwise HULLF_EINVAL).  h_hull / cap / h_count as for convex_hull: the
 * hull of the listed points, by indices into d_pts; of repeated
 * coordinates the first listed index is kept.  From 2^14 survivors on the
 * points are sorted, reduced by chunked monotone chains and the chunk
 * chains merged on the device; only the lower and upper hull chains are
 * copied back. */
hullf_status hull_from_survivors(hullf_ctx_t ctx, const hullf_pt *d_pts, uint64_t n,
                                 const uint32_t *d_surv, uint64_t m, uint32_t *h_hull,
                                 uint64_t cap, uint64_t *h_count, void *stream);

/* The 16-direction filter of the related work (Sec. 2): 16 extreme points
 * of the point set rotated at three angles, then the points strictly inside
 * their polygon discarded.  Directions k * 22.5 degrees, k = 0..15,
 * counter-clockwise from +x; vertex k maximises key k, the first index on
 * ties:  key k = line k and key k+8 = -(line k) for k < 8, with
 *   line 0 = x, 1 = fma(T, y, x), 2 = fl32(x+y), 3 = fma(T, x, y), 4 = y,
 *   5 = fma(-T, x, y), 6 = fl32(y-x), 7 = fma(T, y, -x),
 * T = fl32(tan 22.5 deg) = 0x1.a8279ap-2, each fma rounded once.  The even
 * vertices are the octagon's E0..E7.  The inside test is the rule above
 * over the 16 edges (V_k, V_k+1) whose end points differ.
 * hullf_polygon16: vertices V0..V15 (host array), synchronous; errors as
 * hullf_octagon.  hull_filter16: survivors and count as hull_filter,
 * asynchronous. */
hullf_status hullf_polygon16(hullf_ctx_t ctx, const hullf_pt *d_pts, uint64_t n,
                             uint32_t idx_out[16], void *stream);
hullf_status hull_filter16(hullf_ctx_t ctx, const hullf_pt *d_pts, uint64_t n,
                           uint32_t *d_surv, uint64_t cap, uint64_t *d_count,
                           void *stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, serving loops or harnesses that forbid hipMalloc): the same work
 * and results as hull_filter, with no context.  Its scratch (partial extreme
 * records, octagon record, block counts, keep bits, region-skip boxes) lives
 * in a fixed device array of HULLF_NOALLOC_SCRATCH_BYTES that every device
 * the library runs on holds until the process ends; the call allocates
 * nothing.  Runs on the current device; the first call on a device looks
 * up that device's array (make it outside any graph capture).  n above
 * HULLF_NOALLOC_MAX_POINTS returns HULLF_ENOMEM with nothing enqueued and
 * the outputs untouched; other arguments and results as for hull_filter.
 * Every call on one device shares that device's array and the array keeps
 * the last call's contents, so calls that overlap on one device (other
 * streams, other host threads) race: the caller must order them. */
#define HULLF_NOALLOC_MAX_POINTS (1ull << 25)
#define HULLF_NOALLOC_SCRATCH_BYTES (6ull << 20)
hullf_status hull_filter_noalloc(const hullf_pt *d_pts, uint64_t n, uint32_t *d_surv,
                                 uint64_t cap, uint64_t *d_count, void *stream);

/* Debug export of the bit vector of Sec. 3.2 (one byte per point, 1 =
 * survives), asynchronous.  d_flags: n device bytes.  If a coordinate is not
 * finite every flag is set to 2. */
hullf_status hullf_flags(hullf_ctx_t ctx, const hullf_pt *d_pts, uint64_t n,
                         uint8_t *d_flags, void *stream);

/* Many independent point sets in one persistent launch (Algorithm 1 per
 * set), asynchronous, replayed from a cached HIP graph.
 * d_pts: all sets back to back; d_off: S+1 device uint64 CSR offsets
 * (set s is d_pts[d_off[s] .. d_off[s+1])), d_off[0] == 0 and
 * d_off[S] == n_total (host value, the caller sized d_pts with it).
 * d_surv: n_total device uint32; the survivors of set s are written as
 * set-local ascending indices at d_surv + d_off[s].
 * d_counts: S device uint64, survivors per set (HULLF_COUNT_NONFINITE for a
 * set with a non-finite coordinate).  Sets may be empty.
 * The graph cache is keyed by the argument values; a new key captures a new
 * graph. */
hullf_status hull_filter_batched(hullf_ctx_t ctx, const hullf_pt *d_pts,
                                 const uint64_t *d_off, uint32_t S,
                                 uint64_t n_total, uint32_t *d_surv,
                                 uint64_t *d_counts, void *stream);

/* Hull finishing (Sec. 3.3) of every set of a batch at once, synchronous:
 * the survivors of hull_filter_batched (same d_pts, d_off, S, n_total,
 * d_surv, d_counts) go through one device sort in which every set is
 * sorted on its own, then run representatives, chunked monotone chains and
 * merge rounds that never cross a set; only the sets' hull chains come back
 * to the host.  Set s's hull (counter-clockwise, set-local indices, the
 * conventions of convex_hull) goes to h_hull[h_hull_off[s] ..
 * h_hull_off[s+1]); h_hull_off: S + 1 host words, written also when cap is
 * too small (then HULLF_ECAPACITY and h_hull untouched).  A set counted
 * HULLF_COUNT_NONFINITE gives HULLF_ENONFINITE; a count above its set's
 * size, a survivor index outside its set, or more than 3.5e9 survivors in
 * all (sorted positions are 32-bit) gives HULLF_EINVAL. */
hullf_status hull_from_survivors_batched(hullf_ctx_t ctx, const hullf_pt *d_pts,
                                         const uint64_t *d_off, uint32_t S,
                                         uint64_t n_total, const uint32_t *d_surv,
                                         const uint64_t *d_counts, uint32_t *h_hull,
                                         uint64_t cap, uint64_t *h_hull_off,
                                         void *stream);

/* Same work as hull_filter_batched for sets placed anywhere in d_pts,
 * launched directly (no graph).  d_seg: S (begin, count) pairs of device
 * uint64; set s is d_pts[begin .. begin+count).  Sets must be in ascending
 * order and disjoint, and end within n_total (gaps are allowed and not
 * read).  d_surv: n_total device uint32; the survivors of set s are written
 * as set-local ascending indices at d_surv + begin.  d_counts as for
 * hull_filter_batched; an invalid list sets every count to
 * HULLF_COUNT_BAD_OFFSETS.  This is the form a resident arena of requests
 * uses (see hullf_server.h). */
hullf_status hull_filter_segments(hullf_ctx_t ctx, const hullf_pt *d_pts,
                                  const uint64_t *d_seg, uint32_t S,
                                  uint64_t n_total, uint32_t *d_surv,
                                  uint64_t *d_counts, void *stream);

/* Same work as hull_filter_batched, launched directly (no graph), with an
 * explicit launch shape.  block in {256, 512}, ppt (points per thread per
 * tile) in {8, 16}; 0 picks the tuned or default value. */
hullf_status hull_filter_batched_shape(hullf_ctx_t ctx, const hullf_pt *d_pts,
                                       const uint64_t *d_off, uint32_t S,
                                       uint64_t n_total, uint32_t *d_surv,
                                       uint64_t *d_counts, int block, int ppt,
                                       void *stream);

/* Autotuner: time every supported (block, ppt) shape of the batched kernel
 * on the given batch (`reps` launches each, after one warm-up), keep the
 * fastest in the context for later batched calls, and report it.
 * The choice is also stored in the tune cache under the batch's class
 * (architecture, CU count, floor(log2 S), floor(log2 of the mean set size))
 * and persisted to the cache file, which contexts read at creation: a later
 * batched call of the same class uses that shape (in this and later
 * processes).  The kind of point distribution is not part of the key: the
 * library cannot know it before the batch is filtered.
 * best_block / best_ppt / best_ms may be NULL.  Synchronous. */
hullf_status hullf_autotune_batched(hullf_ctx_t ctx, const hullf_pt *d_pts,
                                    const uint64_t *d_off, uint32_t S,
                                    uint64_t n_total, uint32_t *d_surv,
                                    uint64_t *d_counts, int reps,
                                    int *best_block, int *best_ppt,
                                    float *best_ms, void *stream);

/* Per-kernel device timing.  When enabled, every kernel the library
 * launches is bracketed by HIP events on its stream (timestamp events
 * without a system-scope fence, so recording them flushes no cache between
 * the kernels they bracket).  hullf_timing_read
 * waits for those events and returns, per kernel kind, the number of
 * launches and their summed duration in milliseconds, then clears them.
 * kinds: 0 = extremes reduction, 1 = inside test (the classify pass, with
 * its region-skip box test), 2 = batched launch (plan + persistent
 * kernels), 3 = octagon set-up (merge of the reduction's per-block records,
 * scan of the winning chunks), 4 = compaction pass.  Arrays hold at least
 * 5 entries.  `enable` is a mask of the kinds to time (bit k = kind k;
 * HULLF_TIMING_ALL = every kind, 0 = off); kernels of other kinds are
 * launched without events. */
#define HULLF_TIMING_ALL 0x1F
hullf_status hullf_timing_enable(hullf_ctx_t ctx, int enable);
hullf_status hullf_timing_read(hullf_ctx_t ctx, uint64_t *launches,
                               double *total_ms);

/* Region-skip statistics (the inside test does not read 128-point groups
 * whose bounding box, recorded by the extremes reduction, lies inside the
 * discard region).  Returns, summed over this context's hull_filter and
 * convex_hull calls since the previous call, the groups the inside test read
 * and the groups it would have read without the skip, then resets both.
 * Synchronises the device. */
hullf_status hullf_skip_stats(hullf_ctx_t ctx, uint64_t *groups_read,
                              uint64_t *groups_total);

#ifdef __cplusplus
}
#endif

#endif /* HULLF_H */
