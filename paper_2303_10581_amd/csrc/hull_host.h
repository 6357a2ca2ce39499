// Host monotone-chain hull (Sec. 3.3) used by convex_hull().
#pragma once

#include <cstdint>
#include <vector>

namespace hullf {

struct HostPt {
    float x, y;
    uint32_t i;
};

// Strict counter-clockwise hull of p (reordered in place) starting at the
// lexicographically smallest point; the lowest index is kept per repeated
// coordinate pair.  The sort uses at most max_threads threads.
void monotone_chain(std::vector<HostPt>& p, std::vector<uint32_t>& out, unsigned max_threads = 16);

// Hull from candidate lists sorted by (x, y): `lower` holds every vertex of
// the lower hull, `upper` every vertex of the upper hull (both may hold
// more points, and repeats, of which the first counts).  Same output
// convention as monotone_chain.
void chain_sorted(const std::vector<HostPt>& lower, const std::vector<HostPt>& upper, std::vector<uint32_t>& out);

// Exact sign of (a-o) x (b-o) for FP32 points.
int orient_sign(float ox, float oy, float ax, float ay, float bx, float by);

}  // namespace hullf
