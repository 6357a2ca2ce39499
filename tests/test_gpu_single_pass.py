"""GPU parity of the single-pass filter (HULLF_SINGLE_PASS=1: inside test and
compaction in one launch, survivor offsets by a decoupled look-back over
tiles drawn in ticket order) against the oracle: the ascending survivor
list and its count bit for bit, the hull through convex_hull, at ragged
sizes, every output alignment, with region skip, limited capacity,
non-finite input, and at the full sizes of the study cases (stored oracle
results, compared through SHA-256)."""
from __future__ import annotations

import hashlib
import json
import os

import numpy as np
import pytest

import oracle
from paper_2303_10581_amd import hullf, workloads
from tests import cases
from tests.gpu_common import say, survivors_np, torch_dev, upload  # noqa: F401

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


@pytest.fixture(scope="module")
def ctx1(torch_dev):
    old = os.environ.get("HULLF_SINGLE_PASS")
    os.environ["HULLF_SINGLE_PASS"] = "1"
    try:
        c = hullf.Context(0)
    finally:
        if old is None:
            del os.environ["HULLF_SINGLE_PASS"]
        else:
            os.environ["HULLF_SINGLE_PASS"] = old
    yield c
    c.close()


def _check(c, dev, xy, name, hull=True, offset=0):
    say(f"[gpu] single pass {name}: n={xy.shape[0]} offset={offset}")
    t = upload(xy, dev, offset)
    want = oracle.survivors(xy)
    got = survivors_np(c, t)
    assert got.shape == want.shape, (name, got.shape, want.shape)
    assert np.array_equal(got, want), name
    if hull:
        assert np.array_equal(c.convex_hull(t), oracle.hull(xy, want)), name


@pytest.mark.parametrize("kind", ["normal", "circle", "displaced", "circle_jitter", "normal_far", "displaced_huge",
                                  "displaced_tiny", "subnormal", "grid", "collinear_h", "all_equal"])
def test_named_sets_single_pass(ctx1, torch_dev, kind):
    _check(ctx1, torch_dev, cases.named_sets(300_007, 23)[kind], kind)


@pytest.mark.parametrize("n", [1, 2, 3, 63, 64, 65, 8191, 8192, 8193, 16383, 16385, 24577, 531_441])
def test_ragged_sizes_single_pass(ctx1, torch_dev, n):
    """Tile counts of 1, 2, 3 and many, with a partial last tile."""
    for kind in ("normal", "circle", "displaced"):
        _check(ctx1, torch_dev, workloads.by_kind(kind, n, 200 + n), f"{kind} n={n}", hull=n < 100_000)


@pytest.mark.parametrize("k", [0, 1, 2, 3, 5])
def test_dense_tiles_at_every_output_alignment(ctx1, torch_dev, k):
    ring = workloads.circle(100_003, 53)
    xy = np.concatenate([np.zeros((k, 2), np.float32), ring], axis=0)
    _check(ctx1, torch_dev, xy, f"dense tiles, {k} centre points", hull=False)


@pytest.mark.parametrize("lead", [0, 1, 3])
def test_structured_keep_patterns_single_pass(ctx1, torch_dev, lead):
    _check(ctx1, torch_dev, cases.keep_pattern_set(61, lead), f"keep patterns, lead {lead}", hull=False)


def test_skipping_and_dense_tiles_in_one_set(ctx1, torch_dev):
    """Long runs of tiles whose boxes all pass (count 0, no points read)
    between tiles that keep every point: look-backs across many tiles that
    only published their counts."""
    cloud = workloads.normal(3_000_017, 61)
    ring = (workloads.circle(2_000_003, 62).astype(np.float64) * 6.0).astype(np.float32)
    xy = np.concatenate([cloud, ring, cloud[:500_000], ring[:70_001]], axis=0)
    ctx1.skip_stats()
    _check(ctx1, torch_dev, xy, "cloud, ring, cloud, ring", hull=False)
    read, total = ctx1.skip_stats()
    assert 0 < read < total, (read, total)


def test_region_skip_misaligned_single_pass(ctx1, torch_dev):
    base = cases.named_sets(1_000_003, 59)["normal"]
    xy = cases.with_near_edge_points(base, oracle.extremes, per_edge=300, seed=19)
    xy = xy[np.random.default_rng(11).permutation(xy.shape[0])]
    _check(ctx1, torch_dev, xy, "scattered near-edge normal, misaligned", hull=False, offset=1)


def test_repeated_calls_single_pass(ctx1, torch_dev):
    """Larger and smaller sets in turn: status words and tickets of an
    earlier call must not leak into a later one."""
    for seed, n in enumerate((300_007, 30_011, 1_200_001, 5_003, 8_192)):
        for kind in ("normal", "circle", "displaced"):
            xy = workloads.by_kind(kind, n, seed)
            assert np.array_equal(survivors_np(ctx1, upload(xy, torch_dev)), oracle.survivors(xy)), (kind, n)


def test_capacity_smaller_than_count_single_pass(ctx1, torch_dev):
    import torch
    xy = workloads.circle(50_000, 6)
    want = oracle.survivors(xy)
    t = upload(xy, torch_dev)
    cap = 1000
    surv = torch.full((cap + 16,), -1, dtype=torch.int32, device=torch_dev)
    _, count = ctx1.hull_filter(t, surv=surv, cap=cap)
    assert int(count.item()) == want.size
    got = surv.cpu().numpy()
    assert np.array_equal(got[:cap].astype(np.uint32), want[:cap])
    assert (got[cap:] == -1).all()


@pytest.mark.parametrize("bad", [np.nan, np.inf])
def test_nonfinite_single_pass(ctx1, torch_dev, bad):
    xy = workloads.normal(100_000, 3)
    xy[12345, 1] = bad
    _, count = ctx1.hull_filter(upload(xy, torch_dev))
    assert (int(count.item()) & ((1 << 64) - 1)) == hullf.COUNT_NONFINITE
    ok = workloads.normal(1000, 4)
    assert np.array_equal(survivors_np(ctx1, upload(ok, torch_dev)), oracle.survivors(ok))


def test_empty_single_pass(ctx1, torch_dev):
    import torch
    _, count = ctx1.hull_filter(torch.zeros((0, 2), dtype=torch.float32, device=torch_dev))
    assert int(count.item()) == 0


def _sha(a: np.ndarray) -> str:
    return hashlib.sha256(np.ascontiguousarray(a).tobytes()).hexdigest()


@pytest.mark.parametrize("name", ["normal_1e8", "circle_1e8", "displaced_1e8", "circle_jitter_5e8"])
def test_full_size_single_pass(ctx1, torch_dev, name):
    import torch
    with open(os.path.join(GOLDEN, "full_size.json")) as f:
        rec = json.load(f)[name]
    say(f"[gpu] single pass full size {name}: n={rec['n']}")
    xy = workloads.by_kind(rec["kind"], rec["n"], rec["seed"])
    assert _sha(xy) == rec["points_sha256"], "the input generator changed; rerun make_full_size.py"
    t = torch.from_numpy(xy).to(torch_dev)
    del xy
    surv, count = ctx1.hull_filter(t)
    c = int(count.item())
    assert c == rec["survivors"], (name, c, rec["survivors"])
    assert _sha(surv[:c].cpu().numpy().astype("<u4")) == rec["survivors_sha256"], name
    del surv, t
    torch.cuda.empty_cache()
