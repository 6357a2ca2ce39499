"""GPU parity of the single-set inside test in every sub-tile shape
(HULLF_FILTER_SHAPE = block,ppt; the default is 512,16): each shape has its
own code -- the 4-slot shapes (256 x 8, 512 x 8) load the next sub-tile
while they test the current one when no group of the block is skipped, the
8-slot shapes do not -- and all of them share the out-of-line path for
partial, skipped and degenerate sub-tiles.  Survivors and their count bit
for bit against the oracle on data that skips nothing (circle, displaced),
data that skips most groups (normal, the listed path), near-edge points,
ragged sizes, misaligned input and a degenerate octagon."""
from __future__ import annotations

import os

import numpy as np
import pytest

import oracle
from paper_2303_10581_amd import hullf, workloads
from tests import cases
from tests.gpu_common import say, survivors_np, torch_dev, upload  # noqa: F401

pytestmark = pytest.mark.gpu

SHAPES = [(256, 8), (256, 16), (512, 8), (512, 16)]


@pytest.fixture(scope="module", params=SHAPES, ids=lambda s: f"{s[0]}x{s[1]}")
def shape_ctx(request, torch_dev):
    old = os.environ.get("HULLF_FILTER_SHAPE")
    os.environ["HULLF_FILTER_SHAPE"] = f"{request.param[0]},{request.param[1]}"
    try:
        c = hullf.Context(0)
    finally:
        if old is None:
            del os.environ["HULLF_FILTER_SHAPE"]
        else:
            os.environ["HULLF_FILTER_SHAPE"] = old
    yield request.param, c
    c.close()


def _check(shape_ctx, dev, xy, name, offset=0):
    shape, c = shape_ctx
    say(f"[gpu] shape {shape[0]}x{shape[1]} {name}: n={xy.shape[0]} offset={offset}")
    want = oracle.survivors(xy)
    got = survivors_np(c, upload(xy, dev, offset))
    assert got.shape == want.shape, (shape, name, got.shape, want.shape)
    assert np.array_equal(got, want), (shape, name)


def test_every_kind(shape_ctx, torch_dev):
    sets = cases.named_sets(400_003, 31)
    for kind in ("normal", "circle", "displaced", "circle_jitter", "grid", "all_equal", "collinear_h"):
        _check(shape_ctx, torch_dev, sets[kind], kind)


@pytest.mark.parametrize("n", [1, 65, 8191, 8193, 16385, 98_305, 1_000_003])
def test_ragged_sizes(shape_ctx, torch_dev, n):
    """Partial last sub-tiles and blocks whose range is shorter than one
    sub-tile; circle points make every block take the dense path."""
    for kind in ("circle", "normal"):
        _check(shape_ctx, torch_dev, workloads.by_kind(kind, n, 300 + n), f"{kind} n={n}")


def test_near_edge_points_misaligned(shape_ctx, torch_dev):
    """Points within a few ulps of the octagon's edges (the undecided band:
    the quick-accept box and the binary64 rule) at an 8-byte aligned base."""
    base = cases.named_sets(600_011, 37)["displaced"]
    xy = cases.with_near_edge_points(base, oracle.extremes, per_edge=300, seed=23)
    xy = xy[np.random.default_rng(5).permutation(xy.shape[0])]
    _check(shape_ctx, torch_dev, xy, "near-edge displaced", offset=0)
    _check(shape_ctx, torch_dev, xy, "near-edge displaced", offset=1)


def test_cloud_with_rings(shape_ctx, torch_dev):
    """Blocks that skip most groups next to blocks that skip none."""
    cloud = workloads.normal(2_000_003, 41)
    ring = (workloads.circle(600_001, 42).astype(np.float64) * 6.0).astype(np.float32)
    xy = np.concatenate([cloud, ring, cloud[:300_000]], axis=0)
    _check(shape_ctx, torch_dev, xy, "cloud, ring, cloud")
