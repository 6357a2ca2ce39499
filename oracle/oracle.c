/*
 * oracle.c -- plain, slow, obviously correct CPU reference for the octagon
 * filter and the convex hull of Carrasco, Ferrada, Navarro and Hitschfeld,
 * "An Evaluation of GPU Filters for Accelerating the 2D Convex Hull"
 * (arXiv 2303.10581).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product (the HIP library and its
 * Python binding) may include, link, load or call this file.  Only the test
 * suite, the smoke check and the CPU-baseline leg of the benchmark use it.
 * It shares no code, header, constant table or helper with the GPU path.
 *
 * Build: gcc -O2 -ffp-contract=off -fno-fast-math -shared -fPIC
 *        (FMA contraction must stay off: the predicate is defined operation by
 *        operation in binary64.)
 *
 * Steps follow Algorithm 1 (findingPolygon, buildingFilter,
 * compactingFilteredPoints, convexHull_algorithm):
 *   oracle_validate   -- every coordinate finite (inputs are FP32, Sec. 6)
 *   oracle_extremes   -- Sec. 3.1: the four axis extremes, then the four
 *                        points of least Manhattan distance to the corners of
 *                        the bounding box, counter-clockwise from the
 *                        right-most point
 *   oracle_keep       -- Sec. 3.2: one test per point against the octagon
 *   oracle_survivors  -- Sec. 4.1.1: compaction of the flags (ascending)
 *   oracle_hull       -- Sec. 3.3: hull of a point set (Andrew's monotone
 *                        chain with exact orientation)
 *
 * Readings of the paper taken here (the paper is silent on them):
 *  - Corner keys.  For the top-right corner (X, Y) = (max x, max y) the
 *    Manhattan distance of p is (X - x) + (Y - y) = (X + Y) - (x + y), so the
 *    nearest point maximises x + y; likewise top-left maximises y - x,
 *    bottom-left minimises x + y, bottom-right maximises x - y.  Keys are
 *    evaluated in FP32 (the paper's precision): fl32(x+y), fl32(x-y).
 *    Ties go to the lowest index.  Comparisons are numeric (-0 == +0).
 *  - Vertex order: E0..E7 = right, top-right, top, top-left, left,
 *    bottom-left, bottom, bottom-right (counter-clockwise).
 *  - Inside test, conservative in binary64: for a directed edge (a,b) and a
 *    point p, with no fused multiply-add,
 *       ex=bx-ax  ey=by-ay  qx=px-ax  qy=py-ay  l=ex*qy  r=ey*qx
 *       det=l-r   bnd=C*(|l|+|r|),  C=(3+16*eps)*eps, eps=2^-53
 *    (C is the orientation error bound "A" of Shewchuk, 1997).  The point is
 *    strictly inside the edge iff det > bnd.  Edges whose end points have
 *    equal coordinates are skipped.  A point is discarded iff at least one
 *    edge remains and the point is strictly inside every remaining edge;
 *    points on or near the boundary survive.
 *  - Hull: strict vertices (collinear and duplicate points dropped, the
 *    lowest index kept per duplicate coordinate), counter-clockwise, starting
 *    at the lexicographically smallest (x, y), no closing repeat.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

/* ------------------------------------------------------------------------ */
/* Validation                                                               */
/* ------------------------------------------------------------------------ */

/* Returns 0 if every coordinate is finite, 2 otherwise. */
int oracle_validate(const float *xy, uint64_t n)
{
    for (uint64_t i = 0; i < 2 * n; ++i)
        if (!isfinite(xy[i]))
            return 2;
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Sec. 3.1: extreme points and corner points                               */
/* ------------------------------------------------------------------------ */

/* idx[0..7] = right, top-right, top, top-left, left, bottom-left, bottom,
 * bottom-right.  n must be >= 1 and every coordinate finite. */
void oracle_extremes(const float *xy, uint64_t n, uint32_t idx[8])
{
    /* Axis extremes: right-most (max x), upper-most (max y), left-most
     * (min x), lowest (min y).  First occurrence wins. */
    uint64_t right = 0, top = 0, left = 0, low = 0;
    for (uint64_t i = 1; i < n; ++i) {
        float x = xy[2 * i], y = xy[2 * i + 1];
        if (x > xy[2 * right]) right = i;
        if (y > xy[2 * top + 1]) top = i;
        if (x < xy[2 * left]) left = i;
        if (y < xy[2 * low + 1]) low = i;
    }
    /* Corner points: least Manhattan distance to each corner of the bounding
     * box; as derived in the header, that is the extreme of x+y or x-y,
     * evaluated in FP32. */
    uint64_t tr = 0, tl = 0, bl = 0, br = 0;
    float best_tr = 0, best_tl = 0, best_bl = 0, best_br = 0;
    for (uint64_t i = 0; i < n; ++i) {
        float x = xy[2 * i], y = xy[2 * i + 1];
        float s = x + y;     /* fl32(x+y) */
        float d = x - y;     /* fl32(x-y); fl32(y-x) is its negation */
        if (i == 0 || s > best_tr) { best_tr = s; tr = i; }
        if (i == 0 || -d > best_tl) { best_tl = -d; tl = i; }
        if (i == 0 || s < best_bl) { best_bl = s; bl = i; }
        if (i == 0 || d > best_br) { best_br = d; br = i; }
    }
    idx[0] = (uint32_t)right;
    idx[1] = (uint32_t)tr;
    idx[2] = (uint32_t)top;
    idx[3] = (uint32_t)tl;
    idx[4] = (uint32_t)left;
    idx[5] = (uint32_t)bl;
    idx[6] = (uint32_t)low;
    idx[7] = (uint32_t)br;
}

/* ------------------------------------------------------------------------ */
/* Sec. 3.2: the inside test                                                */
/* ------------------------------------------------------------------------ */

/* (3 + 16 eps) eps with eps = 2^-53; exactly representable in binary64. */
static double bound_constant(void)
{
    const double eps = ldexp(1.0, -53);
    return (3.0 + 16.0 * eps) * eps;
}

/* 1 iff p is strictly inside the directed edge a->b under the binary64
 * rule stated in the header. */
static int strictly_inside(double ax, double ay, double bx, double by,
                           double px, double py)
{
    const double C = bound_constant();
    volatile double ex = bx - ax;
    volatile double ey = by - ay;
    volatile double qx = px - ax;
    volatile double qy = py - ay;
    volatile double l = ex * qy;
    volatile double r = ey * qx;
    volatile double det = l - r;
    volatile double sum = fabs(l) + fabs(r);
    volatile double bnd = C * sum;
    return det > bnd;
}

/* keep[i] = 1 if point i survives the octagon of vertex indices idx[8]. */
void oracle_keep(const float *xy, uint64_t n, const uint32_t idx[8],
                 uint8_t *keep)
{
    /* Non-degenerate edges (a, b) = (E_j, E_{j+1 mod 8}) with a != b. */
    double ax[8], ay[8], bx[8], by[8];
    int m = 0;
    for (int j = 0; j < 8; ++j) {
        float x0 = xy[2 * (uint64_t)idx[j]], y0 = xy[2 * (uint64_t)idx[j] + 1];
        int k = (j + 1) % 8;
        float x1 = xy[2 * (uint64_t)idx[k]], y1 = xy[2 * (uint64_t)idx[k] + 1];
        if (x0 == x1 && y0 == y1)
            continue;
        ax[m] = x0; ay[m] = y0; bx[m] = x1; by[m] = y1;
        ++m;
    }
    for (uint64_t i = 0; i < n; ++i) {
        double px = xy[2 * i], py = xy[2 * i + 1];
        int inside_all = (m >= 1);
        for (int e = 0; e < m; ++e)
            if (!strictly_inside(ax[e], ay[e], bx[e], by[e], px, py))
                inside_all = 0;
        keep[i] = inside_all ? 0 : 1;
    }
}

/* Sec. 4.1.1: survivors = ascending indices of kept points.  Returns the
 * count (or -2 if a coordinate is not finite).  surv must hold n entries. */
int64_t oracle_survivors(const float *xy, uint64_t n, uint32_t *surv,
                         uint32_t idx_out[8])
{
    if (oracle_validate(xy, n) != 0)
        return -2;
    if (n == 0)
        return 0;
    uint32_t idx[8];
    oracle_extremes(xy, n, idx);
    if (idx_out)
        memcpy(idx_out, idx, sizeof idx);
    uint8_t *keep = (uint8_t *)malloc(n ? n : 1);
    if (!keep)
        return -4;
    oracle_keep(xy, n, idx, keep);
    int64_t c = 0;
    for (uint64_t i = 0; i < n; ++i)
        if (keep[i])
            surv[c++] = (uint32_t)i;
    free(keep);
    return c;
}

/* ------------------------------------------------------------------------ */
/* Exact orientation: small signed big integers                             */
/* ------------------------------------------------------------------------ */

/* Every FP32 value v equals V * 2^-149 with V an integer, |V| < 2^277.
 * Differences stay below 2^278 and products below 2^556; 20 limbs of 32
 * bits (640 bits) hold all of them. */
#define LIMBS 20
typedef struct {
    int neg;                 /* 1 if negative */
    uint32_t w[LIMBS];       /* magnitude, least significant limb first */
} big;

static void big_zero(big *a) { memset(a, 0, sizeof *a); }

/* V = v * 2^149 for an FP32 value v. */
static void big_from_float(big *a, float v)
{
    uint32_t bits;
    memcpy(&bits, &v, 4);
    big_zero(a);
    uint32_t e = (bits >> 23) & 0xff, f = bits & 0x7fffff;
    uint64_t mant;
    unsigned shift;
    if (e == 0) { mant = f; shift = 0; }
    else { mant = (uint64_t)f | (1u << 23); shift = e - 1; }
    /* place mant << shift */
    unsigned limb = shift / 32, off = shift % 32;
    uint64_t wide = mant << off;                /* at most 24 + 31 bits */
    a->w[limb] = (uint32_t)wide;
    if (limb + 1 < LIMBS) a->w[limb + 1] = (uint32_t)(wide >> 32);
    a->neg = (bits >> 31) && mant != 0;
}

static int mag_cmp(const big *a, const big *b)
{
    for (int i = LIMBS - 1; i >= 0; --i) {
        if (a->w[i] != b->w[i])
            return a->w[i] < b->w[i] ? -1 : 1;
    }
    return 0;
}

static int big_is_zero(const big *a)
{
    for (int i = 0; i < LIMBS; ++i)
        if (a->w[i]) return 0;
    return 1;
}

/* r = |a| + |b| (magnitudes only) */
static void mag_add(big *r, const big *a, const big *b)
{
    uint64_t c = 0;
    for (int i = 0; i < LIMBS; ++i) {
        uint64_t s = (uint64_t)a->w[i] + b->w[i] + c;
        r->w[i] = (uint32_t)s;
        c = s >> 32;
    }
}

/* r = |a| - |b| assuming |a| >= |b| */
static void mag_sub(big *r, const big *a, const big *b)
{
    int64_t br = 0;
    for (int i = 0; i < LIMBS; ++i) {
        int64_t s = (int64_t)a->w[i] - b->w[i] - br;
        br = s < 0;
        r->w[i] = (uint32_t)(s + (br ? ((int64_t)1 << 32) : 0));
    }
}

/* r = a - b (signed) */
static void big_sub(big *r, const big *a, const big *b)
{
    big nb = *b;
    nb.neg = !b->neg;
    big out;
    big_zero(&out);
    if (a->neg == nb.neg) {
        mag_add(&out, a, &nb);
        out.neg = a->neg;
    } else if (mag_cmp(a, &nb) >= 0) {
        mag_sub(&out, a, &nb);
        out.neg = a->neg;
    } else {
        mag_sub(&out, &nb, a);
        out.neg = nb.neg;
    }
    if (big_is_zero(&out)) out.neg = 0;
    *r = out;
}

/* r = a * b (signed); inputs below 2^320 in magnitude */
static void big_mul(big *r, const big *a, const big *b)
{
    big out;
    big_zero(&out);
    for (int i = 0; i < LIMBS / 2; ++i) {
        uint64_t carry = 0;
        for (int j = 0; j < LIMBS / 2; ++j) {
            uint64_t t = (uint64_t)a->w[i] * b->w[j] + out.w[i + j] + carry;
            out.w[i + j] = (uint32_t)t;
            carry = t >> 32;
        }
        out.w[i + LIMBS / 2] = (uint32_t)carry;
    }
    out.neg = (a->neg != b->neg) && !big_is_zero(&out);
    *r = out;
}

/* Sign of (a-o) x (b-o) computed exactly from the FP32 coordinates. */
int oracle_orient_exact(float ox, float oy, float ax, float ay,
                        float bx, float by)
{
    big Ox, Oy, Ax, Ay, Bx, By, dax, day, dbx, dby, l, r, det;
    big_from_float(&Ox, ox); big_from_float(&Oy, oy);
    big_from_float(&Ax, ax); big_from_float(&Ay, ay);
    big_from_float(&Bx, bx); big_from_float(&By, by);
    big_sub(&dax, &Ax, &Ox); big_sub(&day, &Ay, &Oy);
    big_sub(&dbx, &Bx, &Ox); big_sub(&dby, &By, &Oy);
    big_mul(&l, &dax, &dby);
    big_mul(&r, &day, &dbx);
    big_sub(&det, &l, &r);
    if (big_is_zero(&det)) return 0;
    return det.neg ? -1 : 1;
}

/* Orientation with a binary64 filter first (same bound as the inside test),
 * falling back to the exact computation when the filter is not certain. */
static int orient(float ox, float oy, float ax, float ay, float bx, float by)
{
    const double C = bound_constant();
    volatile double ex = (double)ax - (double)ox;
    volatile double ey = (double)ay - (double)oy;
    volatile double qx = (double)bx - (double)ox;
    volatile double qy = (double)by - (double)oy;
    volatile double l = ex * qy;
    volatile double r = ey * qx;
    volatile double det = l - r;
    volatile double bnd = C * (fabs(l) + fabs(r));
    if (det > bnd) return 1;
    if (-det > bnd) return -1;
    return oracle_orient_exact(ox, oy, ax, ay, bx, by);
}

/* ------------------------------------------------------------------------ */
/* Sec. 3.3: convex hull (Andrew's monotone chain)                          */
/* ------------------------------------------------------------------------ */

typedef struct {
    float x, y;
    uint32_t i;
} rec;

static int rec_cmp(const void *pa, const void *pb)
{
    const rec *a = (const rec *)pa, *b = (const rec *)pb;
    if (a->x < b->x) return -1;
    if (a->x > b->x) return 1;
    if (a->y < b->y) return -1;
    if (a->y > b->y) return 1;
    return (a->i > b->i) - (a->i < b->i);
}

/* Hull of the points listed in subset[0..m) (all n points if subset is
 * NULL).  Writes counter-clockwise vertex indices to out (capacity >= the
 * number of distinct points) and returns their count. */
uint64_t oracle_hull(const float *xy, uint64_t n, const uint32_t *subset,
                     uint64_t m, uint32_t *out)
{
    uint64_t cnt = subset ? m : n;
    if (cnt == 0) return 0;
    rec *p = (rec *)malloc(cnt * sizeof(rec));
    for (uint64_t k = 0; k < cnt; ++k) {
        uint32_t i = subset ? subset[k] : (uint32_t)k;
        p[k].x = xy[2 * (uint64_t)i];
        p[k].y = xy[2 * (uint64_t)i + 1];
        p[k].i = i;
    }
    qsort(p, cnt, sizeof(rec), rec_cmp);
    /* drop duplicate coordinates; the lowest index sorts first */
    uint64_t d = 0;
    for (uint64_t k = 0; k < cnt; ++k) {
        if (d > 0 && p[k].x == p[d - 1].x && p[k].y == p[d - 1].y)
            continue;
        p[d++] = p[k];
    }
    if (d == 1) {
        out[0] = p[0].i;
        free(p);
        return 1;
    }
    rec *h = (rec *)malloc(2 * d * sizeof(rec));
    uint64_t t = 0;
    for (uint64_t k = 0; k < d; ++k) {            /* lower chain */
        while (t >= 2 && orient(h[t - 2].x, h[t - 2].y, h[t - 1].x, h[t - 1].y,
                                p[k].x, p[k].y) <= 0)
            --t;
        h[t++] = p[k];
    }
    uint64_t lower = t + 1;
    for (uint64_t k = d - 1; k-- > 0;) {           /* upper chain */
        while (t >= lower && orient(h[t - 2].x, h[t - 2].y, h[t - 1].x,
                                    h[t - 1].y, p[k].x, p[k].y) <= 0)
            --t;
        h[t++] = p[k];
    }
    --t;                       /* the last point repeats the first */
    for (uint64_t k = 0; k < t; ++k)
        out[k] = h[k].i;
    free(h);
    free(p);
    return t;
}

/* ------------------------------------------------------------------------ */
/* All-core build of the filter (CPU baseline timing only)                  */
/* ------------------------------------------------------------------------ */

/* oracle_survivors over `threads` OpenMP threads (<= 0: the runtime's
 * default), for timing the filter on every host core.  Same arithmetic:
 * each thread takes a contiguous slice of the points, finds the slice's
 * extremes with the comparisons of oracle_extremes, and the slices are
 * merged in ascending order keeping the earlier slice on equal keys, so the
 * first index attaining each key wins as in the one-thread scan.  The inside
 * test is strictly_inside per point and edge; the survivors of each slice
 * are written at the slice's offset (an exclusive sum of the slice counts).
 * Returns what oracle_survivors returns. */
#include <omp.h>

#define OMP_MAX_SLICES 1024

int64_t oracle_survivors_omp(const float *xy, uint64_t n, uint32_t *surv,
                             uint32_t idx_out[8], int threads)
{
    int T = threads > 0 ? threads : omp_get_max_threads();
    if (T > OMP_MAX_SLICES) T = OMP_MAX_SLICES;
    if ((uint64_t)T > n) T = n > 0 ? (int)n : 1;
    int bad = 0;
#pragma omp parallel for num_threads(T) reduction(| : bad) schedule(static)
    for (int64_t i = 0; i < (int64_t)(2 * n); ++i)
        bad |= !isfinite(xy[i]);
    if (bad)
        return -2;
    if (n == 0)
        return 0;

    /* per slice: the first index attaining each key, and its key value;
     * key order: x, y (max), x, y (min), x+y, y-x (max), x+y (min), x-y (max) */
    uint64_t (*sidx)[8] = malloc(sizeof(uint64_t[8]) * (size_t)T);
    float (*sval)[8] = malloc(sizeof(float[8]) * (size_t)T);
    uint64_t *cnt = malloc(sizeof(uint64_t) * ((size_t)T + 1));
    uint8_t *keep = (uint8_t *)malloc(n);
    if (!sidx || !sval || !cnt || !keep) {
        free(sidx); free(sval); free(cnt); free(keep);
        return -4;
    }
#pragma omp parallel num_threads(T)
    {
        int t = omp_get_thread_num();
        uint64_t lo = n * (uint64_t)t / (uint64_t)T, hi = n * (uint64_t)(t + 1) / (uint64_t)T;
        uint64_t right = lo, top = lo, left = lo, low = lo, tr = lo, tl = lo, bl = lo, br = lo;
        float best_tr = 0, best_tl = 0, best_bl = 0, best_br = 0;
        for (uint64_t i = lo; i < hi; ++i) {
            float x = xy[2 * i], y = xy[2 * i + 1];
            if (x > xy[2 * right]) right = i;
            if (y > xy[2 * top + 1]) top = i;
            if (x < xy[2 * left]) left = i;
            if (y < xy[2 * low + 1]) low = i;
            float s = x + y;
            float d = x - y;
            if (i == lo || s > best_tr) { best_tr = s; tr = i; }
            if (i == lo || -d > best_tl) { best_tl = -d; tl = i; }
            if (i == lo || s < best_bl) { best_bl = s; bl = i; }
            if (i == lo || d > best_br) { best_br = d; br = i; }
        }
        if (lo < hi) {
            sidx[t][0] = right; sval[t][0] = xy[2 * right];
            sidx[t][1] = top;   sval[t][1] = xy[2 * top + 1];
            sidx[t][2] = left;  sval[t][2] = xy[2 * left];
            sidx[t][3] = low;   sval[t][3] = xy[2 * low + 1];
            sidx[t][4] = tr;    sval[t][4] = best_tr;
            sidx[t][5] = tl;    sval[t][5] = best_tl;
            sidx[t][6] = bl;    sval[t][6] = best_bl;
            sidx[t][7] = br;    sval[t][7] = best_br;
        }
    }
    /* merge: keys 0, 1, 4, 5, 7 are maxima, 2, 3, 6 minima; a later slice
     * replaces the current choice only if strictly better */
    uint64_t m_idx[8];
    float m_val[8];
    for (int k = 0; k < 8; ++k) { m_idx[k] = sidx[0][k]; m_val[k] = sval[0][k]; }
    for (int t = 1; t < T; ++t) {
        for (int k = 0; k < 8; ++k) {
            int is_min = (k == 2 || k == 3 || k == 6);
            int better = is_min ? (sval[t][k] < m_val[k]) : (sval[t][k] > m_val[k]);
            if (better) { m_idx[k] = sidx[t][k]; m_val[k] = sval[t][k]; }
        }
    }
    uint32_t idx[8] = {(uint32_t)m_idx[0], (uint32_t)m_idx[4], (uint32_t)m_idx[1], (uint32_t)m_idx[5],
                       (uint32_t)m_idx[2], (uint32_t)m_idx[6], (uint32_t)m_idx[3], (uint32_t)m_idx[7]};
    if (idx_out)
        memcpy(idx_out, idx, sizeof idx);

    /* edges exactly as in oracle_keep */
    double ax[8], ay[8], bx[8], by[8];
    int m = 0;
    for (int j = 0; j < 8; ++j) {
        float x0 = xy[2 * (uint64_t)idx[j]], y0 = xy[2 * (uint64_t)idx[j] + 1];
        int k = (j + 1) % 8;
        float x1 = xy[2 * (uint64_t)idx[k]], y1 = xy[2 * (uint64_t)idx[k] + 1];
        if (x0 == x1 && y0 == y1)
            continue;
        ax[m] = x0; ay[m] = y0; bx[m] = x1; by[m] = y1;
        ++m;
    }
#pragma omp parallel num_threads(T)
    {
        int t = omp_get_thread_num();
        uint64_t lo = n * (uint64_t)t / (uint64_t)T, hi = n * (uint64_t)(t + 1) / (uint64_t)T;
        uint64_t c = 0;
        for (uint64_t i = lo; i < hi; ++i) {
            double px = xy[2 * i], py = xy[2 * i + 1];
            int inside_all = (m >= 1);
            for (int e = 0; e < m; ++e)
                if (!strictly_inside(ax[e], ay[e], bx[e], by[e], px, py))
                    inside_all = 0;
            keep[i] = inside_all ? 0 : 1;
            c += keep[i];
        }
        cnt[t + 1] = c;
#pragma omp barrier
#pragma omp single
        {
            cnt[0] = 0;
            for (int u = 1; u <= T; ++u) cnt[u] += cnt[u - 1];
        }
        uint64_t o = cnt[t];
        for (uint64_t i = lo; i < hi; ++i)
            if (keep[i])
                surv[o++] = (uint32_t)i;
    }
    int64_t total = (int64_t)cnt[T];
    free(sidx); free(sval); free(cnt); free(keep);
    return total;
}

/* ------------------------------------------------------------------------ */
/* Related-work variant (Sec. 2): the 16-direction filter                   */
/* ------------------------------------------------------------------------ */

/* Sec. 2 describes a filter that finds 16 hull points by rotating the
 * point set at three angles and discards the points inside their polygon.
 * Reading taken here: the 16 directions are k * 22.5 degrees, k = 0..15
 * (rotations by 22.5, 45 and 67.5 degrees, plus the unrotated axes; each
 * rotation contributes min and max of both coordinates).  A rotation by
 * angle a scaled by 1 / cos a keeps every argmax, so the key of direction
 * (1, t) is x + t*y; with t = T = fl32(tan 22.5 deg) it is evaluated in FP32
 * as one fused multiply-add (one rounding, like fl32(x+y)).  The even
 * directions are the octagon's eight keys, so vertex 2j is octagon vertex
 * E_j.  Vertex k maximises key_k below, first index on ties. */
#define TAN_22_5_F32 0x1.a8279ap-2f

static float key16(int k, float x, float y)
{
    const float T = TAN_22_5_F32;
    switch (k) {
    case 0: return x;                      /* 0 deg: max x            */
    case 1: return fmaf(T, y, x);          /* 22.5: (1, T)            */
    case 2: return x + y;                  /* 45                      */
    case 3: return fmaf(T, x, y);          /* 67.5: (T, 1)            */
    case 4: return y;                      /* 90                      */
    case 5: return fmaf(-T, x, y);         /* 112.5: (-T, 1)          */
    case 6: return -(x - y);               /* 135: fl32(y-x)          */
    case 7: return fmaf(T, y, -x);         /* 157.5: (-1, T)          */
    case 8: return -x;                     /* 180: min x              */
    case 9: return -fmaf(T, y, x);         /* 202.5: min of key 1     */
    case 10: return -(x + y);              /* 225: min fl32(x+y)      */
    case 11: return -fmaf(T, x, y);        /* 247.5: min of key 3     */
    case 12: return -y;                    /* 270: min y              */
    case 13: return -fmaf(-T, x, y);       /* 292.5: min of key 5     */
    case 14: return x - y;                 /* 315                     */
    default: return -fmaf(T, y, -x);       /* 337.5: min of key 7     */
    }
}

/* idx[0..15]: vertex k is the first point maximising key16(k, .). */
void oracle_extremes16(const float *xy, uint64_t n, uint32_t idx[16])
{
    for (int k = 0; k < 16; ++k) {
        uint64_t best_i = 0;
        float best = key16(k, xy[0], xy[1]);
        for (uint64_t i = 1; i < n; ++i) {
            float v = key16(k, xy[2 * i], xy[2 * i + 1]);
            if (v > best) { best = v; best_i = i; }
        }
        idx[k] = (uint32_t)best_i;
    }
}

/* keep[i] = 1 if point i survives the polygon whose vertices are the points
 * idx[0..k) in order: the rule of oracle_keep over the edges
 * (idx[j], idx[(j+1) mod k]) whose end points differ. */
void oracle_keep_poly(const float *xy, uint64_t n, const uint32_t *idx, int k,
                      uint8_t *keep)
{
    double *ax = malloc(4 * sizeof(double) * (size_t)k);
    double *ay = ax + k, *bx = ax + 2 * k, *by = ax + 3 * k;
    int m = 0;
    for (int j = 0; j < k; ++j) {
        float x0 = xy[2 * (uint64_t)idx[j]], y0 = xy[2 * (uint64_t)idx[j] + 1];
        int j1 = (j + 1) % k;
        float x1 = xy[2 * (uint64_t)idx[j1]], y1 = xy[2 * (uint64_t)idx[j1] + 1];
        if (x0 == x1 && y0 == y1)
            continue;
        ax[m] = x0; ay[m] = y0; bx[m] = x1; by[m] = y1;
        ++m;
    }
    for (uint64_t i = 0; i < n; ++i) {
        double px = xy[2 * i], py = xy[2 * i + 1];
        int inside_all = (m >= 1);
        for (int e = 0; e < m; ++e)
            if (!strictly_inside(ax[e], ay[e], bx[e], by[e], px, py))
                inside_all = 0;
        keep[i] = inside_all ? 0 : 1;
    }
    free(ax);
}

/* Survivors of the 16-direction filter (ascending); returns the count, -2
 * for a non-finite coordinate. */
int64_t oracle_survivors16(const float *xy, uint64_t n, uint32_t *surv,
                           uint32_t idx_out[16])
{
    if (oracle_validate(xy, n) != 0)
        return -2;
    if (n == 0)
        return 0;
    uint32_t idx[16];
    oracle_extremes16(xy, n, idx);
    if (idx_out)
        memcpy(idx_out, idx, sizeof idx);
    uint8_t *keep = (uint8_t *)malloc(n);
    if (!keep)
        return -4;
    oracle_keep_poly(xy, n, idx, 16, keep);
    int64_t c = 0;
    for (uint64_t i = 0; i < n; ++i)
        if (keep[i])
            surv[c++] = (uint32_t)i;
    free(keep);
    return c;
}

/* out[i] = key of direction k of point i (exported for the key-level pins). */
void oracle_key16_values(const float *xy, uint64_t n, int k, float *out)
{
    for (uint64_t i = 0; i < n; ++i)
        out[i] = key16(k, xy[2 * i], xy[2 * i + 1]);
}
