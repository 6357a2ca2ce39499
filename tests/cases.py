"""Edge-case and adversarial inputs shared by the oracle tests and the GPU
parity tests.  Construction only: nothing here evaluates the filter."""
from __future__ import annotations

import json
import os

import numpy as np

from paper_2303_10581_amd import workloads

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def golden_cases():
    with open(os.path.join(GOLDEN, "regular_octagon.json")) as f:
        d = json.load(f)
    out = []
    for c in d["cases"]:
        xy = np.array([[float.fromhex(x), float.fromhex(y)] for x, y, _ in c["points"]],
                      dtype=np.float32)
        out.append((c["name"], xy, c))
    return out


def ulp_nudge(v: np.ndarray, k: np.ndarray) -> np.ndarray:
    """Move each float32 v by k[i] units in the last place."""
    v = np.asarray(v, dtype=np.float32).copy()
    for step in range(int(np.abs(k).max()) if len(k) else 0):
        mask = np.abs(k) > step
        up = mask & (k > 0)
        dn = mask & (k < 0)
        v[up] = np.nextafter(v[up], np.float32(np.inf))
        v[dn] = np.nextafter(v[dn], np.float32(-np.inf))
    return v


def near_edges(base: np.ndarray, vertices: np.ndarray, per_edge: int, seed: int,
               max_ulps: int = 3) -> np.ndarray:
    """Points on the segments between consecutive vertices (rounded to
    float32), nudged by up to max_ulps units in x and/or y."""
    rng = np.random.default_rng(seed)
    V = base[vertices].astype(np.float64)
    k = len(vertices)
    pts = []
    for j in range(k):
        a, b = V[j], V[(j + 1) % k]
        t = rng.uniform(0.05, 0.95, per_edge)
        p = (a[None, :] * (1 - t)[:, None] + b[None, :] * t[:, None]).astype(np.float32)
        kx = rng.integers(-max_ulps, max_ulps + 1, per_edge)
        ky = rng.integers(-max_ulps, max_ulps + 1, per_edge)
        p[:, 0] = ulp_nudge(p[:, 0], kx)
        p[:, 1] = ulp_nudge(p[:, 1], ky)
        pts.append(p)
    return np.concatenate(pts, axis=0)


def _keys(xy: np.ndarray) -> np.ndarray:
    x = xy[:, 0]
    y = xy[:, 1]
    s = (x + y).astype(np.float32)
    d = (x - y).astype(np.float32)
    return np.stack([x, s, y, -d, -x, -s, -y, d], axis=1)


def with_near_edge_points(base: np.ndarray, extremes_fn, per_edge: int = 200,
                          seed: int = 0, max_ulps: int = 3) -> np.ndarray:
    """base plus adversarial near-edge points that leave the octagon's
    vertices unchanged: a candidate is kept only if it is strictly below
    every vertex's own direction key."""
    v = extremes_fn(base)
    extra = near_edges(base, v, per_edge, seed, max_ulps)
    top = _keys(base)[v, np.arange(8)]
    ok = (_keys(extra) < top[None, :]).all(axis=1)
    xy = np.concatenate([base, extra[ok]], axis=0)
    assert np.array_equal(extremes_fn(xy), v)
    return xy


# binary32 nearest to tan(22.5 deg), as a float64 (the 16-direction keys)
_T16 = float.fromhex("0x1.a8279ap-2")


def _keys16_f64(xy: np.ndarray) -> np.ndarray:
    """The 16 direction keys in float64 (construction only: used to keep
    added points clear of every direction's maximum)."""
    x = xy[:, 0].astype(np.float64)
    y = xy[:, 1].astype(np.float64)
    T = _T16
    half = [x, x + T * y, x + y, T * x + y, y, -T * x + y, y - x, T * y - x]
    return np.stack(half + [-h for h in half], axis=1)


def with_near_edge_points16(base: np.ndarray, extremes16_fn, per_edge: int = 100,
                            seed: int = 0, max_ulps: int = 3) -> np.ndarray:
    """base plus points a few ulps either side of the 16 edges of the
    16-direction polygon, leaving its vertices unchanged: a candidate is kept
    only if its key is clearly below each direction's maximum."""
    v = extremes16_fn(base)
    extra = near_edges(base, v, per_edge, seed, max_ulps)
    top = _keys16_f64(base)[v, np.arange(16)]
    margin = 8.0 * np.spacing(np.abs(top).astype(np.float32)).astype(np.float64)
    ok = (_keys16_f64(extra) < (top - margin)[None, :]).all(axis=1)
    xy = np.concatenate([base, extra[ok]], axis=0)
    assert np.array_equal(extremes16_fn(xy), v)
    return xy


def transformed(xy: np.ndarray, scale: float, shift: tuple) -> np.ndarray:
    return (xy.astype(np.float64) * scale + np.array(shift)).astype(np.float32)


def small_integer_grid(n: int, span: int, seed: int) -> np.ndarray:
    """Points on a small integer grid: many duplicates and collinear runs."""
    rng = np.random.default_rng(seed)
    return rng.integers(-span, span + 1, (n, 2)).astype(np.float32)


def named_sets(n: int, seed: int):
    """The study-case distributions at a small size, plus scaled/shifted and
    degenerate variants."""
    out = {
        "normal": workloads.normal(n, seed),
        "circle": workloads.circle(n, seed + 1),
        "displaced": workloads.displaced(n, seed + 2, 0.05),
        "circle_jitter": workloads.circle_jitter(n, seed + 3, 0.01),
    }
    out["normal_far"] = transformed(out["normal"], 0.1, (100.0, -100.0))
    out["displaced_huge"] = transformed(out["displaced"], 1e30, (0.0, 0.0))
    out["displaced_tiny"] = transformed(out["displaced"], 1e-30, (0.0, 0.0))
    out["subnormal"] = transformed(out["normal"], 1e-40, (0.0, 0.0))
    out["grid"] = small_integer_grid(n, 50, seed + 4)
    rng = np.random.default_rng(seed + 5)
    line = rng.uniform(-1, 1, n).astype(np.float32)
    out["collinear_h"] = np.stack([line, np.full(n, 0.5, np.float32)], axis=1)
    out["collinear_diag"] = np.stack([line, line], axis=1)
    out["all_equal"] = np.full((n, 2), 3.25, dtype=np.float32)
    return out


def keep_pattern_set(seed: int, lead: int = 0) -> np.ndarray:
    """Points whose survivors form structured patterns span by span (8192
    points per span): ring points (radius 1, kept) and points near the centre
    (discarded) laid out as all kept, none kept, runs of 16, one kept per 1024
    points, alternating full and empty 128-point groups, one full 1024-point
    round, all but the last, only the first, then spans of random density,
    and a ragged tail.  `lead` centre points in front shift every output
    offset (16-byte alignment of the stored runs)."""
    rng = np.random.default_rng(seed)
    span = 8192
    pats = [np.ones(span, bool), np.zeros(span, bool),
            (np.arange(span) // 16) % 2 == 0,
            (np.arange(span) % 1024) == 1023,
            (np.arange(span) // 128) % 2 == 1,
            (np.arange(span) // 1024) == 3,
            np.arange(span) < span - 1,
            np.arange(span) == 0]
    for p in (0.01, 0.3, 0.5, 0.9, 0.99, 0.5, 0.999, 0.001):
        pats.append(rng.random(span) < p)
    pats.append(rng.random(1000) < 0.5)
    keep = np.concatenate([np.zeros(lead, bool)] + pats)
    n = keep.size
    th = rng.uniform(0.0, 2.0 * np.pi, n)
    ring = np.stack([np.cos(th), np.sin(th)], axis=1)
    centre = rng.uniform(-0.01, 0.01, (n, 2))
    return np.where(keep[:, None], ring, centre).astype(np.float32)
