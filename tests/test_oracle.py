"""Pins of the CPU oracle to things other than itself (CPU only).

Each test ties a step of the oracle to the paper's definitions, to exact
arithmetic, to a library routine or to a closed form:
  - hand-built golden cases (tests/golden/regular_octagon.json)
  - extremes == first argmax of the FP32 keys (numpy), and == the paper's
    Manhattan-distance definition (Sec. 3.1) in exact integer arithmetic
  - inside test == exact strict rule wherever binary64 is exact; elsewhere
    sound (every discarded point is exactly inside) and tight (every extra
    survivor is within the rounding margin of an edge)
  - compaction == flatnonzero of the flags
  - hull == brute force over every ordered pair (exact), == Qhull's vertex
    set in general position, and satisfies the hull invariants
  - exact orientation == Python integer arithmetic
  - displaced circumference discard fraction == its closed form
"""
from __future__ import annotations

import math

import numpy as np
import pytest
from hypothesis import HealthCheck, given, settings
from hypothesis import strategies as st

from oracle import brute
from tests import cases
from paper_2303_10581_amd import workloads


# --------------------------------------------------------------------------
# golden fixture
# --------------------------------------------------------------------------

@pytest.mark.parametrize("name,xy,case", cases.golden_cases(), ids=lambda v: v if isinstance(v, str) else "")
def test_golden_cases(oracle_mod, name, xy, case):
    assert oracle_mod.extremes(xy).tolist() == case["extremes"]
    assert oracle_mod.survivors(xy).tolist() == case["survivors"]
    if "hull" in case:
        assert oracle_mod.hull(xy).tolist() == case["hull"]
        assert oracle_mod.convex_hull(xy).tolist() == case["hull"]


# --------------------------------------------------------------------------
# Sec. 3.1 extremes
# --------------------------------------------------------------------------

def _argmax_keys(xy):
    x = xy[:, 0]
    y = xy[:, 1]
    s = (x + y).astype(np.float32)
    d = (x - y).astype(np.float32)
    keys = [x, s, y, -d, -x, -s, -y, d]
    return [int(np.argmax(k)) for k in keys]


@pytest.mark.parametrize("kind", ["normal", "circle", "displaced", "circle_jitter", "normal_far",
                                  "displaced_huge", "displaced_tiny", "subnormal", "grid",
                                  "collinear_h", "collinear_diag", "all_equal"])
def test_extremes_are_first_argmax(oracle_mod, kind):
    xy = cases.named_sets(20000, 11)[kind]
    assert oracle_mod.extremes(xy).tolist() == _argmax_keys(xy)


@settings(max_examples=60, deadline=None, suppress_health_check=[HealthCheck.too_slow])
@given(st.integers(1, 60), st.integers(1, 1000), st.integers(0, 2**31 - 1))
def test_extremes_match_manhattan_definition_exact(oracle_mod, n, span, seed):
    # Integer coordinates: the FP32 keys are exact, so the oracle must pick
    # exactly the paper's points (lowest index on ties).
    xy = cases.small_integer_grid(n, span, seed)
    assert oracle_mod.extremes(xy).tolist() == brute.extremes_manhattan(xy)


# --------------------------------------------------------------------------
# Sec. 3.2 inside test
# --------------------------------------------------------------------------

def _exact_keep(xy, idx):
    return np.array([0 if brute.strictly_inside_exact(xy, idx, i) else 1 for i in range(len(xy))],
                    dtype=np.uint8)


@settings(max_examples=60, deadline=None, suppress_health_check=[HealthCheck.too_slow])
@given(st.integers(1, 120), st.sampled_from([1, 2, 3, 10, 1000, 2**20]), st.integers(0, 2**31 - 1))
def test_keep_equals_exact_rule_on_integer_points(oracle_mod, n, span, seed):
    # |coords| <= 2^20: every binary64 step is exact and the bound is < 1, so
    # the conservative rule and the exact strict rule must agree.
    xy = cases.small_integer_grid(n, span, seed)
    idx = oracle_mod.extremes(xy)
    assert np.array_equal(oracle_mod.keep(xy, idx), _exact_keep(xy, idx))


def _check_sound_and_tight(oracle_mod, xy):
    idx = oracle_mod.extremes(xy)
    k = oracle_mod.keep(xy, idx)
    E = brute.octagon_edges(xy, idx)
    extra = 0
    for i in range(len(xy)):
        p = (brute.exact_int(xy[i, 0]), brute.exact_int(xy[i, 1]))
        D = [brute.det_exact(a, b, p) for a, b in E]
        inside = bool(E) and all(v > 0 for v in D)
        if k[i] == 0:
            assert inside, f"point {i} discarded but not strictly inside"
        elif inside:
            # kept although exactly inside: only allowed within the rounding
            # margin of some edge
            extra += 1
            assert any(v <= brute.rounding_margin(a, b, p) for v, (a, b) in zip(D, E)), \
                f"point {i} kept far from every edge"
    return extra


@pytest.mark.parametrize("kind", ["normal", "displaced", "circle_jitter", "normal_far",
                                  "displaced_huge", "displaced_tiny", "subnormal"])
def test_keep_sound_and_tight_near_edges(oracle_mod, kind):
    base = cases.named_sets(300, 5)[kind]
    xy = cases.with_near_edge_points(base, oracle_mod.extremes, per_edge=40, seed=3)
    assert xy.shape[0] > base.shape[0]
    _check_sound_and_tight(oracle_mod, xy)


def test_keep_sound_on_circle(oracle_mod):
    xy = workloads.circle(3000, 9)
    extra = _check_sound_and_tight(oracle_mod, xy)
    assert extra == 0


def test_keep_with_one_or_two_distinct_points(oracle_mod):
    one = np.full((5, 2), -1.5, np.float32)
    assert oracle_mod.keep(one).tolist() == [1] * 5
    two = np.array([[0, 0], [1, 2], [0.5, 1.0], [0, 0]], np.float32)
    assert oracle_mod.keep(two).tolist() == [1] * 4


def test_compaction_is_flatnonzero(oracle_mod):
    for kind, xy in cases.named_sets(50000, 21).items():
        k = oracle_mod.keep(xy)
        s = oracle_mod.survivors(xy)
        assert np.array_equal(s, np.flatnonzero(k).astype(np.uint32)), kind
        assert s.dtype == np.uint32


def test_empty_and_nonfinite(oracle_mod):
    e = np.zeros((0, 2), np.float32)
    assert oracle_mod.survivors(e).size == 0
    assert oracle_mod.hull(e).size == 0
    for bad in (np.nan, np.inf, -np.inf):
        xy = workloads.normal(100, 1)
        xy[37, 1] = bad
        with pytest.raises(oracle_mod.NonFiniteInput):
            oracle_mod.survivors(xy)


def test_displaced_discard_fraction_closed_form(oracle_mod):
    # For large n the octagon of a band r ~ 1 + U[-p, p] tends to the regular
    # octagon of circumradius 1+p; a point at angle phi from the nearest edge
    # normal is inside iff r < (1+p) cos(pi/8) / cos(phi).  Averaging the
    # uniform-r probability over phi gives the expected discard fraction.
    p = 0.05
    phi = (np.arange(200000) + 0.5) / 200000 * (math.pi / 8)
    lim = (1 + p) * math.cos(math.pi / 8) / np.cos(phi)
    frac = float(np.clip((lim - (1 - p)) / (2 * p), 0, 1).mean())
    n = 1_000_000
    xy = workloads.displaced(n, 4, p)
    discarded = 1.0 - oracle_mod.survivors(xy).size / n
    assert abs(discarded - frac) < 3e-3, (discarded, frac)
    assert 0.45 < frac < 0.47


def test_circle_keeps_almost_everything(oracle_mod):
    n = 1_000_000
    xy = workloads.circle(n, 3)
    assert oracle_mod.survivors(xy).size >= n - n // 10000


def test_hull_vertices_never_discarded(oracle_mod):
    for kind, xy in cases.named_sets(20000, 31).items():
        s = set(oracle_mod.survivors(xy).tolist())
        h = oracle_mod.hull(xy)
        assert set(h.tolist()) <= s, kind


# --------------------------------------------------------------------------
# Sec. 3.3 hull
# --------------------------------------------------------------------------

def _float32s(lo=-1048576.0, hi=1048576.0):
    return st.floats(lo, hi, width=32, allow_nan=False, allow_infinity=False)


point_sets = st.one_of(
    st.lists(st.tuples(_float32s(), _float32s()), min_size=1, max_size=40),
    st.lists(st.tuples(st.integers(-4, 4).map(float), st.integers(-4, 4).map(float)),
             min_size=1, max_size=40),
    st.lists(st.tuples(st.sampled_from([-0.0, 0.0, 1e-45, -1e-45, 1.0, 3e38, -3e38]).map(lambda v: float(np.float32(v))),
                       st.sampled_from([-0.0, 0.0, 1e-45, 2.5, -3e38]).map(lambda v: float(np.float32(v)))), min_size=1, max_size=12),
)


@settings(max_examples=150, deadline=None, suppress_health_check=[HealthCheck.too_slow])
@given(point_sets)
def test_hull_equals_brute_force(oracle_mod, pts):
    xy = np.array(pts, dtype=np.float32)
    want = brute.hull_brute(xy)
    assert oracle_mod.hull(xy).tolist() == want
    # Algorithm 1: filtering first must not change the hull
    assert oracle_mod.convex_hull(xy).tolist() == want


@pytest.mark.parametrize("seed", range(5))
def test_hull_brute_random_near_collinear(oracle_mod, seed):
    rng = np.random.default_rng(seed)
    t = rng.uniform(-1, 1, 60)
    xy = np.stack([t, 0.3 * t + 0.1], axis=1).astype(np.float32)
    xy = np.concatenate([xy, rng.uniform(-1, 1, (5, 2)).astype(np.float32)])
    assert oracle_mod.hull(xy).tolist() == brute.hull_brute(xy)


def test_hull_matches_qhull_vertex_set(oracle_mod):
    from scipy.spatial import ConvexHull
    for seed, kind in enumerate(["normal", "displaced", "circle_jitter"]):
        xy = workloads.by_kind(kind, 100000, 40 + seed)
        h = oracle_mod.hull(xy)
        q = ConvexHull(xy.astype(np.float64)).vertices
        assert set(h.tolist()) == set(q.tolist()), kind


def _check_hull_invariants(xy, h):
    """ccw, strictly convex, every input point left of or on every edge."""
    P = xy.astype(np.float64)
    H = P[h]
    m = len(h)
    assert m >= 3
    lex = min(range(len(xy)), key=lambda i: (xy[i, 0], xy[i, 1]))
    assert tuple(xy[h[0]]) == tuple(xy[lex])
    for j in range(m):
        a, b, c = h[j], h[(j + 1) % m], h[(j + 2) % m]
        assert brute.orient(xy[a], xy[b], xy[c]) > 0
    for j in range(m):
        a, b = H[j], H[(j + 1) % m]
        ex, ey = b - a
        cross = ex * (P[:, 1] - a[1]) - ey * (P[:, 0] - a[0])
        mag = np.abs(ex * (P[:, 1] - a[1])) + np.abs(ey * (P[:, 0] - a[0]))
        unsure = np.flatnonzero(cross <= 8e-16 * mag)
        for i in unsure:
            assert brute.orient(xy[h[j]], xy[h[(j + 1) % m]], xy[i]) >= 0


@pytest.mark.parametrize("kind,n", [("normal", 200000), ("displaced", 200000), ("circle", 4000)])
def test_hull_invariants_large(oracle_mod, kind, n):
    for seed in range(1):
        xy = workloads.by_kind(kind, n, 50 + seed)
        h = oracle_mod.convex_hull(xy)
        assert np.array_equal(h, oracle_mod.hull(xy))
        _check_hull_invariants(xy, h)


# --------------------------------------------------------------------------
# exact orientation
# --------------------------------------------------------------------------

@settings(max_examples=300, deadline=None)
@given(st.lists(_float32s(float(np.float32(-3e38)), float(np.float32(3e38))), min_size=6, max_size=6))
def test_orient_exact_matches_python_ints(oracle_mod, v):
    o, a, b = (v[0], v[1]), (v[2], v[3]), (v[4], v[5])
    assert oracle_mod.orient_exact(o, a, b) == brute.orient(o, a, b)


def test_orient_exact_near_collinear(oracle_mod):
    rng = np.random.default_rng(7)
    for _ in range(2000):
        o = rng.uniform(-1, 1, 2).astype(np.float32)
        d = rng.uniform(-1, 1, 2)
        a = (o + d * rng.uniform(0.1, 2)).astype(np.float32)
        b = (o + d * rng.uniform(0.1, 2)).astype(np.float32)
        b = cases.ulp_nudge(b, rng.integers(-1, 2, 2))
        assert oracle_mod.orient_exact(o, a, b) == brute.orient(o, a, b)


def _tie_heavy(n: int, seed: int) -> np.ndarray:
    """Every key attained many times across the array (so across slices)."""
    rng = np.random.default_rng(seed)
    xy = rng.integers(-5, 6, (n, 2)).astype(np.float32)
    xy[rng.choice(n, n // 10, replace=False)] = (0.0, -0.0)
    return xy


@pytest.mark.parametrize("threads", [1, 2, 3, 8, 13])
def test_all_core_filter_equals_one_thread(oracle_mod, threads):
    """The OpenMP build of the filter (all-core CPU baseline) returns the
    one-thread oracle's survivors and octagon, also when every extreme is
    tied across slices (the slice merge keeps the first index)."""
    sets = cases.named_sets(30_011, 29)
    sets["ties"] = _tie_heavy(20_003, 3)
    sets["tiny"] = workloads.normal(5, 2)
    for name, xy in sets.items():
        want = oracle_mod.survivors(xy)
        got = oracle_mod.survivors_omp(xy, threads)
        assert np.array_equal(got, want), (name, threads)


def test_all_core_filter_nonfinite_and_empty(oracle_mod):
    xy = workloads.normal(1000, 4)
    xy[17, 0] = np.inf
    with pytest.raises(oracle_mod.NonFiniteInput):
        oracle_mod.survivors_omp(xy, 4)
    assert oracle_mod.survivors_omp(np.zeros((0, 2), np.float32), 4).size == 0
