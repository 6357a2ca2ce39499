"""GPU parity: the HIP path (through the C ABI) against the CPU oracle.

Integer/index results are compared bit for bit: the eight octagon vertex
indices, the ascending survivor index list and its count, and the
counter-clockwise hull index list.  Sizes span many tiles and ragged tails;
the full-size cases use the shapes the benchmark times."""
from __future__ import annotations

import numpy as np
import pytest

import oracle
from paper_2303_10581_amd import hullf, workloads
from tests import cases
from tests.gpu_common import ctx, say, survivors_np, torch_dev, upload  # noqa: F401

pytestmark = pytest.mark.gpu


def _check_all(ctx, dev, xy, name, hull=True, offset=0):
    say(f"[gpu] {name}: n={xy.shape[0]} offset={offset}")
    t = upload(xy, dev, offset)
    want_idx = oracle.extremes(xy)
    assert ctx.octagon(t).tolist() == want_idx.tolist(), name
    want = oracle.survivors(xy)
    got = survivors_np(ctx, t)
    assert got.shape == want.shape, (name, got.shape, want.shape)
    assert np.array_equal(got, want), name
    flags = ctx.flags(t).cpu().numpy()
    assert np.array_equal(np.flatnonzero(flags == 1).astype(np.uint32), want), name
    if hull:
        h = ctx.convex_hull(t)
        assert np.array_equal(h, oracle.hull(xy, want)), name


@pytest.mark.parametrize("name,xy,case", cases.golden_cases(), ids=lambda v: v if isinstance(v, str) else "")
def test_golden(ctx, torch_dev, name, xy, case):
    t = upload(xy, torch_dev)
    assert ctx.octagon(t).tolist() == case["extremes"]
    assert survivors_np(ctx, t).tolist() == case["survivors"]
    if "hull" in case:
        assert ctx.convex_hull(t).tolist() == case["hull"]


@pytest.mark.parametrize("kind", ["normal", "circle", "displaced", "circle_jitter", "normal_far",
                                  "displaced_huge", "displaced_tiny", "subnormal", "grid",
                                  "collinear_h", "collinear_diag", "all_equal"])
def test_named_sets(ctx, torch_dev, kind):
    # 200003 points: ~49 compaction tiles of 4096 and a ragged tail
    xy = cases.named_sets(200003, 17)[kind]
    _check_all(ctx, torch_dev, xy, kind)


@pytest.mark.parametrize("kind", ["normal", "displaced", "circle_jitter", "normal_far",
                                  "displaced_huge", "displaced_tiny", "subnormal"])
def test_near_edge_adversarial(ctx, torch_dev, kind):
    base = cases.named_sets(50000, 23)[kind]
    xy = cases.with_near_edge_points(base, oracle.extremes, per_edge=4000, seed=9)
    _check_all(ctx, torch_dev, xy, "near-edge " + kind)


@pytest.mark.parametrize("n", [1, 2, 3, 4, 5, 63, 64, 65, 4095, 4096, 4097, 8191, 12289])
def test_small_and_ragged_sizes(ctx, torch_dev, n):
    for kind in ("normal", "circle"):
        xy = workloads.by_kind(kind, n, 100 + n)
        _check_all(ctx, torch_dev, xy, f"{kind} n={n}")


def _tie_set(n: int, seed: int) -> np.ndarray:
    """A normal cloud folded to x <= 0 in which every extreme is attained at
    300 positions spread over the whole array: max x = 0 by planted +0 and
    -0, the other seven by planted copies of four far points."""
    rng = np.random.default_rng(seed)
    xy = workloads.normal(n, seed)
    xy[:, 0] = -np.abs(xy[:, 0])
    k = 300
    pos = rng.choice(n, 5 * k, replace=False).reshape(5, k)
    xy[pos[0], 0] = np.where(np.arange(k) % 2 == 0, np.float32(0.0), np.float32(-0.0))
    xy[pos[1]] = (-3.0, 12.0)
    xy[pos[2]] = (-12.0, -12.0)
    xy[pos[3]] = (-14.0, 1.0)
    xy[pos[4]] = (-1.0, -13.0)
    return xy


@pytest.mark.parametrize("n", [300_007, 9_000_011])
def test_extreme_ties_take_lowest_index(ctx, torch_dev, n):
    # 9e6 points: more chunks than reduction blocks, so a block meets the
    # tied values in several chunks and many blocks tie with each other
    _check_all(ctx, torch_dev, _tie_set(n, 31), f"ties n={n}")


def test_all_nan_is_nonfinite(ctx, torch_dev):
    t = upload(np.full((50_001, 2), np.nan, np.float32), torch_dev)
    surv, count = ctx.hull_filter(t)
    assert (int(count.item()) & ((1 << 64) - 1)) == hullf.COUNT_NONFINITE
    with pytest.raises(hullf.HullfError) as e:
        ctx.octagon(t)
    assert e.value.status == hullf.ENONFINITE


def test_misaligned_pointer(ctx, torch_dev):
    xy = workloads.displaced(100001, 5)
    _check_all(ctx, torch_dev, xy, "displaced misaligned", offset=1)


def test_empty_input(ctx, torch_dev):
    import torch
    t = torch.zeros((0, 2), dtype=torch.float32, device=torch_dev)
    surv, count = ctx.hull_filter(t)
    assert int(count.item()) == 0
    assert ctx.convex_hull(t).size == 0
    with pytest.raises(hullf.HullfError) as e:
        ctx.octagon(t)
    assert e.value.status == hullf.EINVAL


@pytest.mark.parametrize("bad", [np.nan, np.inf, -np.inf])
@pytest.mark.parametrize("where", [0, 12345, 99999])
def test_nonfinite(ctx, torch_dev, bad, where):
    xy = workloads.normal(100000, 3)
    xy[where, where % 2] = bad
    t = upload(xy, torch_dev)
    say(f"[gpu] nonfinite {bad} at {where}")
    surv, count = ctx.hull_filter(t)
    assert (int(count.item()) & ((1 << 64) - 1)) == hullf.COUNT_NONFINITE
    with pytest.raises(hullf.HullfError) as e:
        ctx.convex_hull(t)
    assert e.value.status == hullf.ENONFINITE
    with pytest.raises(hullf.HullfError) as e:
        ctx.octagon(t)
    assert e.value.status == hullf.ENONFINITE
    assert (ctx.flags(t).cpu().numpy() == 2).all()
    # the context stays usable
    ok = workloads.normal(1000, 4)
    assert np.array_equal(survivors_np(ctx, upload(ok, torch_dev)), oracle.survivors(ok))


def test_overflowing_keys_are_legal(ctx, torch_dev):
    # x + y overflows to +-inf for finite inputs: a legal key, not an error
    xy = workloads.normal(5000, 8) * np.float32(3e38 / 6)
    xy[10] = [3.0e38, 3.0e38]
    xy[11] = [-3.0e38, -3.0e38]
    _check_all(ctx, torch_dev, xy.astype(np.float32), "overflowing keys")


def test_capacity_smaller_than_count(ctx, torch_dev):
    import torch
    xy = workloads.circle(50000, 6)
    want = oracle.survivors(xy)
    t = upload(xy, torch_dev)
    cap = 1000
    surv = torch.full((cap + 16,), -1, dtype=torch.int32, device=torch_dev)
    _, count = ctx.hull_filter(t, surv=surv, cap=cap)
    assert int(count.item()) == want.size
    got = surv.cpu().numpy()
    assert np.array_equal(got[:cap].astype(np.uint32), want[:cap])
    assert (got[cap:] == -1).all()
    out_cap = 3
    with pytest.raises(hullf.HullfError) as e:
        import ctypes
        buf = np.zeros(out_cap, np.uint32)
        h = ctypes.c_uint64(0)
        st = hullf._load().convex_hull(ctx.handle, t.data_ptr(), t.shape[0], buf.ctypes.data, out_cap,
                                        ctypes.byref(h), hullf._stream(None))
        assert h.value == oracle.hull(xy, want).size
        hullf._check(st, "convex_hull")
    assert e.value.status == hullf.ECAPACITY


def test_repeated_calls_same_context(ctx, torch_dev):
    # larger and smaller sets in turn: an earlier call's per-block records,
    # boxes, keep bits and counts must not leak into a later one
    for seed, n in enumerate((300_007, 30_011, 120_001, 5_003)):
        for kind in ("normal", "circle", "displaced"):
            xy = workloads.by_kind(kind, n, seed)
            t = upload(xy, torch_dev)
            assert np.array_equal(survivors_np(ctx, t), oracle.survivors(xy)), (kind, seed)


@pytest.mark.parametrize("kind", ["normal", "normal_far", "displaced_tiny"])
def test_region_skip_with_scattered_near_edge_points(ctx, torch_dev, kind):
    """Groups whose reduction box lies inside the discard region are not
    read by the inside test; near-edge points scattered through the set put
    some of them in boxes that must not be skipped."""
    base = cases.named_sets(1_000_003, 37)[kind]
    xy = cases.with_near_edge_points(base, oracle.extremes, per_edge=300, seed=11)
    xy = xy[np.random.default_rng(5).permutation(xy.shape[0])]
    _check_all(ctx, torch_dev, xy, "scattered near-edge " + kind, hull=False)


@pytest.mark.parametrize("grid", [1, 7, 64, 2048, 4096])
def test_small_reduce_grid(torch_dev, monkeypatch, grid):
    """Few reduction blocks: every wave reads many chunks (its region-skip
    boxes are written 64 at a time), and the set-up merges few records;
    many blocks: the set-up merges its rows in several batches of loads."""
    monkeypatch.setenv("HULLF_REDUCE_GRID", str(grid))
    c = hullf.Context(0)
    try:
        # enough 2048-point chunks for every block of the largest grids
        base = cases.named_sets(2_000_003 if grid < 2048 else 9_000_011, 41)["normal"]
        xy = cases.with_near_edge_points(base, oracle.extremes, per_edge=200, seed=13)
        xy = xy[np.random.default_rng(7).permutation(xy.shape[0])]
        _check_all(c, torch_dev, xy, f"reduce grid {grid}", hull=False)
        read, total = c.skip_stats()
        assert 0 < read < total, (read, total)
    finally:
        c.close()


@pytest.mark.parametrize("k", [0, 1, 2, 3, 5])
def test_dense_spans_at_every_output_alignment(ctx, torch_dev, k):
    """Points on a circle survive, so spans of 8192 of them are stored as
    runs of consecutive indices; k centre points at the front (discarded)
    shift every run's output offset, covering each 16-byte alignment."""
    ring = workloads.circle(100_003, 53)
    xy = np.concatenate([np.zeros((k, 2), np.float32), ring], axis=0)
    _check_all(ctx, torch_dev, xy, f"dense spans, {k} centre points", hull=False)


@pytest.mark.parametrize("lead", [0, 1, 3])
def test_structured_keep_patterns(ctx, torch_dev, lead):
    """Compaction rounds see every shape of span: full, empty, runs of 16,
    single survivors per round, alternating groups, one full round, random
    densities, a ragged tail, at several output alignments."""
    xy = cases.keep_pattern_set(61, lead)
    _check_all(ctx, torch_dev, xy, f"structured keep patterns, lead {lead}", hull=False)


@pytest.mark.parametrize("shape,compact,skip,per_cu", [
    ("256,8", "256", "1", "0"), ("256,16", "1024", "1", "5"),
    ("512,8", "512", "0", "2"), ("512,16", "256", "0", "1"), ("512,16", "1024", "1", "0")])
def test_launch_settings(torch_dev, monkeypatch, shape, compact, skip, per_cu):
    """Every inside-test shape, compaction block size, region skip on and
    off, and several blocks per compute unit give the oracle's results."""
    for k, v in (("HULLF_FILTER_SHAPE", shape), ("HULLF_COMPACT_BLOCK", compact),
                 ("HULLF_REGION_SKIP", skip), ("HULLF_CLASSIFY_PER_CU", per_cu)):
        monkeypatch.setenv(k, v)
    c = hullf.Context(0)
    try:
        sets = cases.named_sets(300_007, 43)
        for kind in ("normal", "circle", "displaced", "grid"):
            _check_all(c, torch_dev, sets[kind], f"{kind} shape {shape} compact {compact} skip {skip}", hull=False)
        xy = cases.with_near_edge_points(sets["normal"], oracle.extremes, per_edge=500, seed=17)
        xy = xy[np.random.default_rng(9).permutation(xy.shape[0])]
        _check_all(c, torch_dev, xy, f"near-edge normal shape {shape}", hull=False)
    finally:
        c.close()


def test_config_small_normal_1e6(ctx, torch_dev):
    xy = workloads.normal(1_000_000, 1)
    _check_all(ctx, torch_dev, xy, "normal 1e6 seed 1")


def test_region_skip_misaligned(ctx, torch_dev):
    """Region skip with 8-byte (not 16-byte) aligned points: blocks that read
    only the few groups outside their passing boxes load them with 8-byte
    loads."""
    base = cases.named_sets(1_000_003, 59)["normal"]
    xy = cases.with_near_edge_points(base, oracle.extremes, per_edge=300, seed=19)
    xy = xy[np.random.default_rng(11).permutation(xy.shape[0])]
    _check_all(ctx, torch_dev, xy, "scattered near-edge normal, misaligned", hull=False, offset=1)


def test_skipping_and_dense_blocks_in_one_set(ctx, torch_dev):
    """A normal cloud (most groups inside the discard region) followed by a
    ring around it (every group read): blocks that list the few groups to
    read and blocks that stream every group run in the same launch."""
    cloud = workloads.normal(3_000_017, 61)
    ring = (workloads.circle(2_000_003, 62).astype(np.float64) * 6.0).astype(np.float32)
    xy = np.concatenate([cloud, ring, cloud[:500_000]], axis=0)
    ctx.skip_stats()
    _check_all(ctx, torch_dev, xy, "cloud then ring", hull=False)
    read, total = ctx.skip_stats()
    assert 0 < read < total, (read, total)
