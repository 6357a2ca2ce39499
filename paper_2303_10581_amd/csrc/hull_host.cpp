// Host finishing step of Algorithm 1 (convexHull_algorithm, Sec. 3.3):
// Andrew's monotone chain over the filter's survivors, with an exact
// orientation predicate.
//
// Orientation: binary64 determinant with the Shewchuk (1997) error bound
// first; when that is inconclusive, the determinant is evaluated exactly as
// a floating-point expansion (TwoSum / TwoProduct, Shewchuk's
// Grow-Expansion) and its sign read from the largest component.  FP32
// inputs keep every intermediate inside the binary64 normal range (products
// between 2^-351 and 2^258), so the expansion is exact.
//
// Compiled with -ffp-contract=off: TwoSum must not be contracted.

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <thread>
#include <vector>

#include "hull_host.h"

namespace hullf {
namespace {

inline void two_sum(double a, double b, double& s, double& e) {
    s = a + b;
    const double bv = s - a;
    const double av = s - bv;
    e = (a - av) + (b - bv);
}

inline void two_prod(double a, double b, double& p, double& e) {
    p = a * b;
    e = std::fma(a, b, -p);
}

// Exact sign of (a-o) x (b-o).
int orient_exact(double ox, double oy, double ax, double ay, double bx, double by) {
    double u[2], v[2], w[2], z[2];   // a.x-o.x, b.y-o.y, a.y-o.y, b.x-o.x as 2-term expansions
    two_sum(ax, -ox, u[1], u[0]);
    two_sum(by, -oy, v[1], v[0]);
    two_sum(ay, -oy, w[1], w[0]);
    two_sum(bx, -ox, z[1], z[0]);
    double terms[16];
    int k = 0;
    for (int i = 0; i < 2; ++i)
        for (int j = 0; j < 2; ++j) {
            double p, e;
            two_prod(u[i], v[j], p, e);
            terms[k++] = p;
            terms[k++] = e;
            two_prod(w[i], z[j], p, e);
            terms[k++] = -p;
            terms[k++] = -e;
        }
    double h[17];
    int len = 0;
    for (int t = 0; t < 16; ++t) {
        double q = terms[t];
        for (int i = 0; i < len; ++i) {
            double s, e;
            two_sum(q, h[i], s, e);
            h[i] = e;
            q = s;
        }
        h[len++] = q;
    }
    for (int i = len - 1; i >= 0; --i)
        if (h[i] != 0.0) return h[i] > 0.0 ? 1 : -1;
    return 0;
}

inline int orient(const HostPt& o, const HostPt& a, const HostPt& b) {
    const double ox = o.x, oy = o.y;
    const double l = ((double)a.x - ox) * ((double)b.y - oy);
    const double r = ((double)a.y - oy) * ((double)b.x - ox);
    const double det = l - r;
    const double bound = 0x1.8000000000004p-52 * (std::fabs(l) + std::fabs(r));
    if (det > bound) return 1;
    if (-det > bound) return -1;
    return orient_exact(ox, oy, a.x, a.y, b.x, b.y);
}

inline bool less_xyi(const HostPt& a, const HostPt& b) {
    if (a.x != b.x) return a.x < b.x;
    if (a.y != b.y) return a.y < b.y;
    return a.i < b.i;
}

// Parallel sort: sort P slices in threads, then merge pairwise in rounds.
void sort_points(std::vector<HostPt>& p, unsigned max_threads) {
    const size_t n = p.size();
    unsigned hw = std::thread::hardware_concurrency();
    size_t P = std::min<size_t>(hw ? hw : 1, std::max(1u, max_threads));
    if (n < (1u << 20) || P < 2) {
        std::sort(p.begin(), p.end(), less_xyi);
        return;
    }
    std::vector<size_t> cut(P + 1);
    for (size_t k = 0; k <= P; ++k) cut[k] = n * k / P;
    {
        std::vector<std::thread> th;
        for (size_t k = 0; k < P; ++k)
            th.emplace_back([&, k] { std::sort(p.begin() + cut[k], p.begin() + cut[k + 1], less_xyi); });
        for (auto& t : th) t.join();
    }
    std::vector<HostPt> buf(n);
    std::vector<HostPt>* src = &p;
    std::vector<HostPt>* dst = &buf;
    while (cut.size() > 2) {
        std::vector<size_t> nc;
        std::vector<std::thread> th;
        for (size_t k = 0; k + 1 < cut.size(); k += 2) {
            if (k + 2 < cut.size()) {
                const size_t a = cut[k], m = cut[k + 1], b = cut[k + 2];
                th.emplace_back([=] {
                    std::merge(src->begin() + a, src->begin() + m, src->begin() + m, src->begin() + b,
                               dst->begin() + a, less_xyi);
                });
                nc.push_back(a);
            } else {
                const size_t a = cut[k], b = cut[k + 1];
                th.emplace_back([=] { std::copy(src->begin() + a, src->begin() + b, dst->begin() + a); });
                nc.push_back(a);
            }
        }
        for (auto& t : th) t.join();
        nc.push_back(n);
        cut.swap(nc);
        std::swap(src, dst);
    }
    if (src != &p) p.swap(buf);
}

}  // namespace

void monotone_chain(std::vector<HostPt>& p, std::vector<uint32_t>& out, unsigned max_threads) {
    out.clear();
    if (p.empty()) return;
    sort_points(p, max_threads);
    // one entry per coordinate pair: the lowest index sorts first
    size_t d = 0;
    for (size_t k = 0; k < p.size(); ++k) {
        if (d > 0 && p[k].x == p[d - 1].x && p[k].y == p[d - 1].y) continue;
        p[d++] = p[k];
    }
    p.resize(d);
    if (d == 1) {
        out.push_back(p[0].i);
        return;
    }
    std::vector<HostPt> h;
    h.reserve(2 * d);
    for (size_t k = 0; k < d; ++k) {   // lower chain, left to right
        while (h.size() >= 2 && orient(h[h.size() - 2], h[h.size() - 1], p[k]) <= 0) h.pop_back();
        h.push_back(p[k]);
    }
    const size_t lower = h.size() + 1;
    for (size_t k = d - 1; k-- > 0;) {   // upper chain, right to left
        while (h.size() >= lower && orient(h[h.size() - 2], h[h.size() - 1], p[k]) <= 0) h.pop_back();
        h.push_back(p[k]);
    }
    h.pop_back();   // repeats the first vertex
    out.reserve(h.size());
    for (const HostPt& q : h) out.push_back(q.i);
}

namespace {

// Drop repeated coordinates of a sorted list, keeping the first of a run.
std::vector<HostPt> unique_sorted(const std::vector<HostPt>& p) {
    std::vector<HostPt> u;
    u.reserve(p.size());
    for (const HostPt& q : p)
        if (u.empty() || q.x != u.back().x || q.y != u.back().y) u.push_back(q);
    return u;
}

}  // namespace

void chain_sorted(const std::vector<HostPt>& lower, const std::vector<HostPt>& upper, std::vector<uint32_t>& out) {
    out.clear();
    const std::vector<HostPt> lo = unique_sorted(lower), up = unique_sorted(upper);
    if (lo.empty()) return;
    std::vector<HostPt> h;
    h.reserve(lo.size() + up.size());
    for (const HostPt& q : lo) {   // lower chain, left to right
        while (h.size() >= 2 && orient(h[h.size() - 2], h[h.size() - 1], q) <= 0) h.pop_back();
        h.push_back(q);
    }
    std::vector<HostPt> g;
    g.reserve(up.size());
    for (size_t k = up.size(); k-- > 0;) {   // upper chain, right to left
        while (g.size() >= 2 && orient(g[g.size() - 2], g[g.size() - 1], up[k]) <= 0) g.pop_back();
        g.push_back(up[k]);
    }
    out.reserve(h.size() + g.size());
    for (const HostPt& q : h) out.push_back(q.i);
    for (size_t k = 1; k + 1 < g.size(); ++k) out.push_back(g[k].i);
}

int orient_sign(float ox, float oy, float ax, float ay, float bx, float by) {
    HostPt o{ox, oy, 0}, a{ax, ay, 0}, b{bx, by, 0};
    return orient(o, a, b);
}

}  // namespace hullf
