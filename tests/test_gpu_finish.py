"""GPU parity of hull finishing on the device (sort + chunked monotone
chains, used by convex_hull from 2^14 survivors on): the counter-clockwise
hull index list must equal the oracle's bit for bit, also with repeated
coordinates (lowest index kept), collinear and single-point sets, and must
equal the host finishing path."""
from __future__ import annotations

import numpy as np
import pytest

import oracle
from paper_2303_10581_amd import hullf, workloads
from tests import cases
from tests.gpu_common import ctx, say, torch_dev, upload  # noqa: F401

pytestmark = pytest.mark.gpu

DEVICE_MIN = 1 << 14


def _hull_check(ctx, dev, xy, name, need_device=True):
    t = upload(xy, dev)
    want_s = oracle.survivors(xy)
    if need_device:
        assert want_s.size >= DEVICE_MIN, (name, want_s.size)
    say(f"[gpu] finish {name}: n={xy.shape[0]} survivors={want_s.size}")
    got = ctx.convex_hull(t)
    want = oracle.hull(xy, want_s)
    assert np.array_equal(got, want), (name, got.size, want.size)
    return got


@pytest.mark.parametrize("kind", ["circle", "collinear_h", "collinear_diag", "all_equal"])
def test_named_sets_device_finish(ctx, torch_dev, kind):
    xy = cases.named_sets(600_011, 29)[kind]
    _hull_check(ctx, torch_dev, xy, kind)


@pytest.mark.parametrize("kind", ["displaced", "circle_jitter", "displaced_huge", "displaced_tiny", "subnormal",
                                  "grid", "normal_far"])
def test_named_sets_any_finish(ctx, torch_dev, kind):
    xy = cases.named_sets(600_011, 29)[kind]
    _hull_check(ctx, torch_dev, xy, kind, need_device=False)


def test_repeated_points_keep_lowest_index(ctx, torch_dev):
    base = workloads.circle(200_003, 41)
    rng = np.random.default_rng(5)
    xy = np.concatenate([base, base[rng.permutation(base.shape[0])], base[:50_000]], axis=0)
    _hull_check(ctx, torch_dev, xy, "circle with repeats")


def test_signed_zero_and_far_values(ctx, torch_dev):
    c = workloads.circle(560_017, 43)
    xy = c.copy()
    xy[::7, 0] = 0.0
    xy[1::7, 0] = -0.0
    xy[2::11, 1] = -0.0
    _hull_check(ctx, torch_dev, xy * np.float32(3.0e30), "circle scaled 3e30 with zeros")


@pytest.mark.parametrize("kind,n,seed", [("circle", 10_000_000, 3), ("displaced", 20_000_000, 4)])
def test_large_device_finish(ctx, torch_dev, kind, n, seed):
    xy = workloads.by_kind(kind, n, seed)
    _hull_check(ctx, torch_dev, xy, f"{kind} {n}")


def test_device_finish_equals_host_finish(ctx, torch_dev, monkeypatch):
    xy = workloads.displaced(3_000_017, 47)
    t = upload(xy, torch_dev)
    dev_h = ctx.convex_hull(t)
    monkeypatch.setenv("HULLF_FINISH", "host")
    c2 = hullf.Context(0)
    try:
        host_h = c2.convex_hull(t)
    finally:
        c2.close()
    assert np.array_equal(dev_h, host_h)


def test_hulls_of_batched_survivors(ctx, torch_dev):
    """The batched filter, then hull_from_survivors per set (set-local
    indices into that set's points)."""
    import torch
    sizes = [5, 1, 0, 3000, 70_001, 300_007, 2]
    parts = [workloads.request(workloads.KINDS[k % 3], n, 600 + k) if n else np.zeros((0, 2), np.float32)
             for k, n in enumerate(sizes)]
    parts[5] = workloads.circle(300_007, 61)   # device finishing
    off = np.zeros(len(parts) + 1, np.uint64)
    off[1:] = np.cumsum([p.shape[0] for p in parts])
    pts = np.concatenate(parts, axis=0)
    t = upload(pts, torch_dev)
    o = torch.from_numpy(off.astype(np.int64)).to(torch_dev)
    say("[gpu] finish: hulls of batched survivors")
    surv, counts = ctx.hull_filter_batched(t, o)
    torch.cuda.synchronize()
    cn = counts.cpu().numpy()
    for k, xy in enumerate(parts):
        a, b = int(off[k]), int(off[k + 1])
        h = ctx.hull_from_survivors(t[a:b], surv[a:], m=int(cn[k]))
        want = oracle.convex_hull(xy) if b > a else np.zeros(0, np.uint32)
        assert np.array_equal(h, want), k


@pytest.mark.parametrize("m", [1000, 300_000])
def test_out_of_range_survivor_index(ctx, torch_dev, m):
    import torch
    xy = workloads.circle(m, 67)
    t = upload(xy, torch_dev)
    s = torch.arange(m, dtype=torch.int32, device=torch_dev)
    s[m // 2] = m + 5
    say(f"[gpu] finish: out-of-range index, m={m}")
    with pytest.raises(hullf.HullfError) as e:
        ctx.hull_from_survivors(t, s)
    assert e.value.status == hullf.EINVAL
    s[m // 2] = m // 2
    assert np.array_equal(ctx.hull_from_survivors(t, s), oracle.hull(xy))


@pytest.mark.parametrize("radius", [100.0, 1000.0, 30000.0])
def test_grid_snapped_circle_device_finish(ctx, torch_dev, radius):
    """Circle points rounded to an integer grid: long runs of repeated
    points, runs of equal x across chunk boundaries (vertical runs at both
    ends), and collinear points on the hull, through the chunk chains and
    the device merge of the chunk chains."""
    c = workloads.circle(1_000_003, 71)
    xy = np.round(c.astype(np.float64) * radius).astype(np.float32)
    _hull_check(ctx, torch_dev, xy, f"grid-snapped circle r={radius}")


def test_merge_tree_many_chunks(ctx, torch_dev):
    """A displaced circumference large enough that the chunk levels stop
    with many chunk chains, so the merge tree runs many rounds, with an odd
    number of chains in some of them."""
    xy = workloads.displaced(6_000_037, 73)
    _hull_check(ctx, torch_dev, xy, "displaced 6e6")


@pytest.mark.parametrize("n", [(1 << 14) - 1, 1 << 14, (1 << 14) + 1, 40_009])
def test_finish_at_the_device_threshold(ctx, torch_dev, n):
    """Circle points all survive: just below the threshold the host chains
    them, from it on the device sorts, chains and merges them."""
    xy = workloads.circle(n, 79)
    _hull_check(ctx, torch_dev, xy, f"circle n={n}", need_device=n >= DEVICE_MIN)


@pytest.mark.parametrize("lines", [1, 3, 40])
def test_vertical_runs_device_finish(ctx, torch_dev, lines):
    """Points on a few vertical lines (every point survives a degenerate or
    thin octagon): runs of equal x hundreds of thousands long, each walked by
    the one wave whose tile it starts in, and the chain ends that only the
    longest runs hold."""
    rng = np.random.default_rng(83 + lines)
    n = 300_007
    xs = rng.integers(0, lines, n).astype(np.float32) * np.float32(0.5)
    ys = rng.standard_normal(n).astype(np.float32)
    xy = np.stack([xs, ys], axis=1)
    xy[rng.choice(n, 50, replace=False)] = xy[rng.choice(n, 50, replace=False)]   # repeats
    _hull_check(ctx, torch_dev, xy, f"{lines} vertical lines", need_device=False)


def _runs_set(seed, n):
    """Runs of equal x whose lengths sit at and around the run pass's step
    (64) and tile (1024) sizes, x increasing between runs, y random (with
    repeated points), so run heads, run ends and carried runs fall on every
    lane and tile position."""
    rng = np.random.default_rng(seed)
    lens = np.array([1, 1, 2, 3, 63, 64, 65, 127, 1023, 1024, 1025, 2047, 2049, 5000])
    parts, x, total = [], 0.0, 0
    while total < n:
        k = int(min(rng.choice(lens), n - total))
        x += float(rng.integers(1, 4))
        ys = rng.standard_normal(k).astype(np.float32) * np.float32(1 + x / 50.0)
        if k > 4:
            ys[rng.integers(0, k, 2)] = ys[rng.integers(0, k)]   # repeated points in the run
        parts.append(np.stack([np.full(k, x, np.float32), ys], axis=1))
        total += k
    return np.concatenate(parts, axis=0)


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_run_lengths_around_step_and_tile(ctx, torch_dev, seed):
    """hull_from_survivors over every point of _runs_set: the representative
    of each run (first lowest / highest y) and the chains built on them."""
    xy = _runs_set(90 + seed, 400_003)
    t = upload(xy, torch_dev)
    import torch
    s = torch.arange(xy.shape[0], dtype=torch.int32, device=torch_dev)
    say(f"[gpu] finish runs around 64/1024: seed {seed}, n={xy.shape[0]}")
    assert np.array_equal(ctx.hull_from_survivors(t, s), oracle.hull(xy))


@pytest.mark.parametrize("chunk", [16, 48, 64])
def test_chain_chunk_sizes(torch_dev, monkeypatch, chunk):
    """The chain pass with other chunk sizes (HULLF_CHAIN_CHUNK; 48 is no
    divisor of the run pass's tile, so chunks straddle its tiles unevenly):
    other chunk levels and merge trees, the same hull."""
    monkeypatch.setenv("HULLF_CHAIN_CHUNK", str(chunk))
    c = hullf.Context(0)
    try:
        for kind in ("circle", "grid", "collinear_diag"):
            xy = cases.named_sets(300_007, 31)[kind]
            say(f"[gpu] finish chunk {chunk}: {kind}")
            t = upload(xy, torch_dev)
            assert np.array_equal(c.convex_hull(t), oracle.hull(xy, oracle.survivors(xy))), (chunk, kind)
        xy = _runs_set(97, 200_003)
        import torch
        s = torch.arange(xy.shape[0], dtype=torch.int32, device=torch_dev)
        assert np.array_equal(c.hull_from_survivors(upload(xy, torch_dev), s), oracle.hull(xy))
    finally:
        c.close()
