"""Exact brute-force references in pure Python integers (tiny inputs only).

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).  These functions pin the
C oracle to definitions that do not depend on its code:

  exact_int(v)          FP32 value v as the integer v * 2^149 (exact)
  orient(o, a, b)       exact sign of (a-o) x (b-o)
  det_exact(a, b, p)    exact (b-a) x (p-a), scaled by 2^298
  hull_brute(xy)        hull by testing every ordered pair as an edge
                        (Sec. 3.3 asks only for "the convex hull"; this is its
                        plain definition)
  extremes_manhattan(xy) the eight octagon vertices by the definition of
                        Sec. 3.1: axis extremes, then least Manhattan distance
                        to the bounding-box corners, in exact arithmetic
"""
from __future__ import annotations

from fractions import Fraction

import numpy as np

SCALE_BITS = 149


def exact_int(v) -> int:
    """Exact integer V with V * 2^-149 == v for an FP32 value v."""
    f = float(np.float32(v))
    num, den = f.as_integer_ratio()
    # den is a power of two <= 2^149 for every FP32 value
    return num * ((1 << SCALE_BITS) // den)


def _pt(xy, i):
    return exact_int(xy[i][0]), exact_int(xy[i][1])


def orient_int(o, a, b) -> int:
    d = (a[0] - o[0]) * (b[1] - o[1]) - (a[1] - o[1]) * (b[0] - o[0])
    return (d > 0) - (d < 0)


def det_exact(a, b, p) -> int:
    """(b - a) x (p - a) on integer-scaled points (scale 2^298)."""
    return (b[0] - a[0]) * (p[1] - a[1]) - (b[1] - a[1]) * (p[0] - a[0])


def orient(o, a, b) -> int:
    """Exact orientation of three FP32 points given as (x, y) pairs."""
    return orient_int((exact_int(o[0]), exact_int(o[1])),
                      (exact_int(a[0]), exact_int(a[1])),
                      (exact_int(b[0]), exact_int(b[1])))


def _on_closed_segment(a, b, p) -> bool:
    return (min(a[0], b[0]) <= p[0] <= max(a[0], b[0])
            and min(a[1], b[1]) <= p[1] <= max(a[1], b[1]))


def distinct_points(xy):
    """[(index, (X, Y))] keeping the lowest index per coordinate pair."""
    seen = {}
    for i in range(len(xy)):
        p = _pt(xy, i)
        if p not in seen:
            seen[p] = i
    return sorted(((i, p) for p, i in seen.items()), key=lambda t: t[0])


def hull_brute(xy) -> list:
    """Counter-clockwise strict hull vertex indices, starting at the
    lexicographically smallest point; O(n^3), for n up to a few hundred.

    (i, j) is a hull edge iff every other distinct point is strictly left of
    i->j or lies on the closed segment [i, j]."""
    pts = distinct_points(xy)
    if not pts:
        return []
    if len(pts) == 1:
        return [pts[0][0]]
    nxt = {}
    for ia, a in pts:
        for ib, b in pts:
            if ia == ib:
                continue
            ok = True
            for ic, c in pts:
                if ic == ia or ic == ib:
                    continue
                o = orient_int(a, b, c)
                if o < 0 or (o == 0 and not _on_closed_segment(a, b, c)):
                    ok = False
                    break
            if ok:
                nxt[ia] = ib
    start = min(pts, key=lambda t: (t[1][0], t[1][1]))[0]
    out = [start]
    cur = nxt[start]
    while cur != start:
        out.append(cur)
        cur = nxt[cur]
        if len(out) > len(pts):
            raise RuntimeError("hull edges do not form a cycle")
    return out


def extremes_manhattan(xy) -> list:
    """E0..E7 by the paper's definition, in exact arithmetic:
    right-most, nearest (Manhattan) to the top-right corner of the bounding
    box, upper-most, nearest to top-left, left-most, nearest to bottom-left,
    lowest, nearest to bottom-right.  Lowest index on ties."""
    P = [_pt(xy, i) for i in range(len(xy))]
    n = len(P)
    X = max(p[0] for p in P)
    Y = max(p[1] for p in P)
    x0 = min(p[0] for p in P)
    y0 = min(p[1] for p in P)

    def first(key):
        best = None
        bi = -1
        for i in range(n):
            k = key(P[i])
            if best is None or k < best:
                best, bi = k, i
        return bi

    right = first(lambda p: -p[0])
    top = first(lambda p: -p[1])
    left = first(lambda p: p[0])
    low = first(lambda p: p[1])
    tr = first(lambda p: (X - p[0]) + (Y - p[1]))
    tl = first(lambda p: (p[0] - x0) + (Y - p[1]))
    bl = first(lambda p: (p[0] - x0) + (p[1] - y0))
    br = first(lambda p: (X - p[0]) + (p[1] - y0))
    return [right, tr, top, tl, left, bl, low, br]


def octagon_edges(xy, idx):
    """Non-degenerate directed edges (a, b) of the octagon with vertex
    indices idx, as exact integer points."""
    V = [_pt(xy, int(i)) for i in idx]
    return [(V[j], V[(j + 1) % 8]) for j in range(8) if V[j] != V[(j + 1) % 8]]


def strictly_inside_exact(xy, idx, i) -> bool:
    """Exact rule: point i is strictly left of every non-degenerate edge."""
    E = octagon_edges(xy, idx)
    p = _pt(xy, i)
    return bool(E) and all(det_exact(a, b, p) > 0 for a, b in E)


def rounding_margin(a, b, p) -> Fraction:
    """8 * 2^-53 * (|ex*qy| + |ey*qx|), exact, on integer-scaled points: a
    generous multiple of the binary64 rounding error of the edge test."""
    ex, ey = b[0] - a[0], b[1] - a[1]
    qx, qy = p[0] - a[0], p[1] - a[1]
    return Fraction(8 * (abs(ex * qy) + abs(ey * qx)), 1 << 53)


# --- Sec. 2: the 16-direction filter ---------------------------------------

# binary32 nearest to tan(22.5 deg) = sqrt(2) - 1
TAN_22_5 = Fraction(float.fromhex("0x1.a8279ap-2"))


def rnd32(q: Fraction) -> np.float32:
    """q rounded to binary32, to nearest with ties to even (overflow gives
    +-inf)."""
    if q == 0:
        return np.float32(0.0)
    c = np.float32(float(q))
    if np.isinf(c):
        return c
    best = None
    for v in (np.nextafter(c, np.float32(-np.inf)), c, np.nextafter(c, np.float32(np.inf))):
        if np.isinf(v):
            continue
        d = abs(Fraction(float(v)) - q)
        even = (int(np.array(v, dtype=np.float32).view(np.uint32)) & 1) == 0
        key = (d, not even)
        if best is None or key < best[0]:
            best = (key, v)
    return best[1]


def key16_exact(k: int, x, y) -> np.float32:
    """The key of direction k (k * 22.5 degrees) of the FP32 point (x, y):
    one rounding of the exact x + T y (or its rotations) to binary32, the
    axis keys exact, the diagonal keys fl32(x +- y), negated for the
    directions taken as minima."""
    X, Y, T = Fraction(float(x)), Fraction(float(y)), TAN_22_5
    base = {
        0: lambda: np.float32(x),
        1: lambda: rnd32(X + T * Y),
        2: lambda: rnd32(X + Y),
        3: lambda: rnd32(T * X + Y),
        4: lambda: np.float32(y),
        5: lambda: rnd32(-T * X + Y),
        6: lambda: -rnd32(X - Y),
        7: lambda: rnd32(T * Y - X),
    }
    # directions 8..15 are the opposite of 0..7: the negated key of k - 8
    return base[k]() if k < 8 else -base[k - 8]()


def extremes16_exact(xy) -> list:
    """V0..V15: for each direction the first index of the maximal key."""
    out = []
    for k in range(16):
        best_i, best = 0, None
        for i in range(len(xy)):
            v = key16_exact(k, xy[i][0], xy[i][1])
            if best is None or v > best:
                best, best_i = v, i
        out.append(best_i)
    return out


def poly_edges(xy, idx):
    """Exact (a, b) of the non-degenerate edges (idx[j], idx[j+1]) of a
    polygon of input points, in order."""
    V = [_pt(xy, int(i)) for i in idx]
    k = len(V)
    return [(V[j], V[(j + 1) % k]) for j in range(k) if V[j] != V[(j + 1) % k]]


def strictly_inside_poly_exact(xy, idx, i) -> bool:
    """Exact rule: point i strictly left of every non-degenerate edge."""
    E = poly_edges(xy, idx)
    p = _pt(xy, i)
    return len(E) >= 1 and all(det_exact(a, b, p) > 0 for a, b in E)
