"""GPU parity of the 16-direction filter (the related-work filter of Sec. 2:
16 extreme points of the point set rotated at three angles, the points
strictly inside their polygon discarded) against the oracle, through the
C ABI: the 16 vertex indices and the ascending survivor list, bit for bit.
Sizes span many tiles and ragged tails; near-edge sets put points a few
ulps either side of all 16 edges."""
from __future__ import annotations

import numpy as np
import pytest

import oracle
from paper_2303_10581_amd import hullf, workloads
from tests import cases
from tests.gpu_common import ctx, say, torch_dev, upload  # noqa: F401

pytestmark = pytest.mark.gpu


def _surv16(ctx, t):
    return ctx.survivors16(t).cpu().numpy().astype(np.uint32)


def _check16(ctx, dev, xy, name, offset=0):
    say(f"[gpu] filter16 {name}: n={xy.shape[0]} offset={offset}")
    t = upload(xy, dev, offset)
    v = oracle.extremes16(xy)
    assert ctx.polygon16(t).tolist() == v.tolist(), name
    want = oracle.survivors16(xy)
    got = _surv16(ctx, t)
    assert got.shape == want.shape, (name, got.shape, want.shape)
    assert np.array_equal(got, want), name
    return want


@pytest.mark.parametrize("kind", ["normal", "circle", "displaced", "circle_jitter", "normal_far",
                                  "displaced_huge", "displaced_tiny", "subnormal", "grid",
                                  "collinear_h", "collinear_diag", "all_equal"])
def test_named_sets16(ctx, torch_dev, kind):
    xy = cases.named_sets(200003, 17)[kind]
    _check16(ctx, torch_dev, xy, kind)


@pytest.mark.parametrize("kind", ["normal", "displaced", "circle_jitter", "normal_far", "displaced_tiny"])
def test_near_edge_adversarial16(ctx, torch_dev, kind):
    base = cases.named_sets(50000, 23)[kind]
    xy = cases.with_near_edge_points16(base, oracle.extremes16, per_edge=2000, seed=9)
    _check16(ctx, torch_dev, xy, "near-edge " + kind)


@pytest.mark.parametrize("n", [1, 2, 3, 5, 17, 64, 2047, 2048, 2049, 8191, 12289])
def test_small_and_ragged_sizes16(ctx, torch_dev, n):
    for kind in ("normal", "circle", "displaced"):
        xy = workloads.by_kind(kind, n, 200 + n)
        _check16(ctx, torch_dev, xy, f"{kind} n={n}")


def test_even_vertices_are_the_octagon(ctx, torch_dev):
    for kind in ("normal", "circle", "grid"):
        xy = cases.named_sets(100_003, 29)[kind]
        t = upload(xy, torch_dev)
        assert np.array_equal(ctx.polygon16(t)[::2], ctx.octagon(t)), kind


def test_ties_take_lowest_index16(ctx, torch_dev):
    # integer points on a small grid: every direction's maximum is attained
    # many times across the whole array and across reduction blocks
    xy = cases.small_integer_grid(3_000_017, 6, 71)
    _check16(ctx, torch_dev, xy, "integer grid ties")


def test_misaligned_and_repeated16(ctx, torch_dev):
    xy = workloads.displaced(100001, 5)
    _check16(ctx, torch_dev, xy, "displaced misaligned", offset=1)
    for seed, n in enumerate((300_007, 30_011, 120_001)):
        for kind in ("normal", "circle", "displaced"):
            _check16(ctx, torch_dev, workloads.by_kind(kind, n, seed), f"repeat {kind} {n}")


def test_region_skip_scattered16(ctx, torch_dev):
    base = cases.named_sets(1_000_003, 37)["normal"]
    xy = cases.with_near_edge_points16(base, oracle.extremes16, per_edge=200, seed=11)
    xy = xy[np.random.default_rng(5).permutation(xy.shape[0])]
    ctx.skip_stats()   # reset the counters
    _check16(ctx, torch_dev, xy, "scattered near-edge normal")
    read, total = ctx.skip_stats()
    assert 0 < read < total, (read, total)


def test_hull_of_16_survivors_is_the_hull(ctx, torch_dev):
    # the filter keeps every hull vertex: the hull of its survivors is the
    # hull of all points
    for kind in ("normal", "displaced", "circle_jitter"):
        xy = cases.named_sets(300_007, 47)[kind]
        t = upload(xy, torch_dev)
        s = ctx.survivors16(t)
        h = ctx.hull_from_survivors(t, s, s.numel())
        assert np.array_equal(h, oracle.hull(xy)), kind


@pytest.mark.parametrize("bad", [np.nan, np.inf, -np.inf])
def test_nonfinite16(ctx, torch_dev, bad):
    xy = workloads.normal(100000, 3)
    xy[4321, 1] = bad
    t = upload(xy, torch_dev)
    surv, count = ctx.hull_filter16(t)
    assert (int(count.item()) & ((1 << 64) - 1)) == hullf.COUNT_NONFINITE
    with pytest.raises(hullf.HullfError) as e:
        ctx.polygon16(t)
    assert e.value.status == hullf.ENONFINITE
    ok = workloads.normal(1000, 4)
    assert np.array_equal(_surv16(ctx, upload(ok, torch_dev)), oracle.survivors16(ok))


def test_empty16(ctx, torch_dev):
    import torch
    t = torch.zeros((0, 2), dtype=torch.float32, device=torch_dev)
    surv, count = ctx.hull_filter16(t)
    assert int(count.item()) == 0
    with pytest.raises(hullf.HullfError) as e:
        ctx.polygon16(t)
    assert e.value.status == hullf.EINVAL


def test_16_discards_at_least_what_the_octagon_discards_on_circles(ctx, torch_dev):
    # not a rule of the method in general (rounded vertices), but on these
    # sets the 16-gon contains the octagon with room to spare
    for kind, seed in (("displaced", 3), ("circle_jitter", 4)):
        xy = workloads.by_kind(kind, 2_000_003, seed)
        t = upload(xy, torch_dev)
        s8 = set(ctx.survivors(t).cpu().numpy().tolist())
        s16 = _check16(ctx, torch_dev, xy, f"{kind} 2e6")
        assert set(s16.tolist()) <= s8, kind
        assert s16.size < len(s8), kind
