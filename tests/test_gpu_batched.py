"""GPU parity of the batched persistent launch: every set's count and
set-local survivor list must equal the oracle run on that set alone (and so
the plain single-set launch)."""
from __future__ import annotations

import numpy as np
import pytest

import oracle
from paper_2303_10581_amd import hullf, workloads
from tests.gpu_common import ctx, say, torch_dev, upload  # noqa: F401

pytestmark = pytest.mark.gpu

SHAPES = [(256, 8), (256, 16), (512, 8), (512, 16)]


def _mixed_batch(seed: int, S: int):
    """Sets of mixed kinds and sizes, including empty, single-point and
    odd-offset sets."""
    rng = np.random.default_rng(seed)
    parts = []
    for s in range(S):
        r = rng.random()
        if r < 0.08:
            n = 0
        elif r < 0.16:
            n = int(rng.integers(1, 4))
        else:
            n = int(np.exp(rng.uniform(np.log(5), np.log(60000))))
        kind = workloads.KINDS[s % 3]
        xy = workloads.request(kind, n, seed * 100000 + s) if n else np.zeros((0, 2), np.float32)
        parts.append(xy)
    off = np.zeros(S + 1, dtype=np.uint64)
    off[1:] = np.cumsum([p.shape[0] for p in parts])
    pts = np.concatenate(parts, axis=0) if off[-1] else np.zeros((0, 2), np.float32)
    return pts.astype(np.float32), off


def _run(ctx, dev, pts, off, block=None, ppt=None, offset=0):
    import torch
    t = upload(pts if pts.shape[0] else np.zeros((1, 2), np.float32), dev, offset)
    if pts.shape[0] == 0:
        t = t[:0]
    o = torch.from_numpy(off.astype(np.int64)).to(dev)
    surv, counts = ctx.hull_filter_batched(t, o, n_total=pts.shape[0], block=block, ppt=ppt)
    torch.cuda.synchronize()
    return surv.cpu().numpy().astype(np.uint32), counts.cpu().numpy().astype(np.uint64)


def _check(pts, off, sv, cn, name):
    S = off.size - 1
    for s in range(S):
        a, b = int(off[s]), int(off[s + 1])
        want = oracle.survivors(pts[a:b]) if b > a else np.zeros(0, np.uint32)
        assert int(cn[s]) == want.size, (name, s, int(cn[s]), want.size)
        assert np.array_equal(sv[a:a + want.size], want), (name, s)


@pytest.mark.parametrize("block,ppt", SHAPES)
def test_mixed_batch_every_shape(ctx, torch_dev, block, ppt):
    pts, off = _mixed_batch(1, 120)
    say(f"[gpu] batched mixed S=120 n={pts.shape[0]} shape=({block},{ppt})")
    sv, cn = _run(ctx, torch_dev, pts, off, block, ppt)
    _check(pts, off, sv, cn, f"shape {block}x{ppt}")


def test_graph_replay_sees_new_data(ctx, torch_dev):
    import torch
    pts, off = _mixed_batch(2, 200)
    t = upload(pts, torch_dev)
    o = torch.from_numpy(off.astype(np.int64)).to(torch_dev)
    surv = torch.empty(pts.shape[0], dtype=torch.int32, device=torch_dev)
    counts = torch.empty(200, dtype=torch.int64, device=torch_dev)
    for rep in range(3):
        say(f"[gpu] batched graph replay {rep}")
        data = pts if rep % 2 == 0 else (pts[::-1] * np.float32(0.5)).copy()
        t.copy_(torch.from_numpy(data).to(torch_dev))
        ctx.hull_filter_batched(t, o, surv=surv, counts=counts)
        torch.cuda.synchronize()
        _check(data, off, surv.cpu().numpy().astype(np.uint32), counts.cpu().numpy(), f"replay {rep}")


def test_misaligned_batch(ctx, torch_dev):
    pts, off = _mixed_batch(3, 50)
    say(f"[gpu] batched misaligned n={pts.shape[0]}")
    sv, cn = _run(ctx, torch_dev, pts, off, offset=1)
    _check(pts, off, sv, cn, "misaligned")


def test_single_set_and_empty_sets(ctx, torch_dev):
    xy = workloads.displaced(300001, 8)
    off = np.array([0, xy.shape[0]], np.uint64)
    sv, cn = _run(ctx, torch_dev, xy, off)
    _check(xy, off, sv, cn, "single set")
    off2 = np.array([0, 0, 0, xy.shape[0], xy.shape[0]], np.uint64)
    sv, cn = _run(ctx, torch_dev, xy, off2)
    _check(xy, off2, sv, cn, "empty sets around one")


def test_nonfinite_set_is_isolated(ctx, torch_dev):
    pts, off = _mixed_batch(4, 40)
    s_bad = next(s for s in range(40) if off[s + 1] - off[s] > 100)
    pts = pts.copy()
    pts[int(off[s_bad]) + 7, 0] = np.nan
    sv, cn = _run(ctx, torch_dev, pts, off)
    assert int(cn[s_bad]) == hullf.COUNT_NONFINITE
    for s in range(40):
        if s == s_bad:
            continue
        a, b = int(off[s]), int(off[s + 1])
        want = oracle.survivors(pts[a:b]) if b > a else np.zeros(0, np.uint32)
        assert int(cn[s]) == want.size and np.array_equal(sv[a:a + want.size], want)


def test_all_nan_and_tied_sets(ctx, torch_dev):
    """A set of NaN only is reported non-finite; sets whose extremes tie at
    many positions (equal points, a grid) keep exact survivors."""
    pts, off = _mixed_batch(6, 30)
    big = [s for s in range(30) if off[s + 1] - off[s] > 3000][:3]
    pts = pts.copy()
    a, b = int(off[big[0]]), int(off[big[0] + 1])
    pts[a:b] = np.nan
    a, b = int(off[big[1]]), int(off[big[1] + 1])
    pts[a:b] = (2.5, -1.0)
    a, b = int(off[big[2]]), int(off[big[2] + 1])
    g = np.arange(b - a)
    pts[a:b, 0], pts[a:b, 1] = g % 37, g // 37
    sv, cn = _run(ctx, torch_dev, pts, off)
    assert int(cn[big[0]]) == hullf.COUNT_NONFINITE
    for s in range(30):
        if s == big[0]:
            continue
        a, b = int(off[s]), int(off[s + 1])
        want = oracle.survivors(pts[a:b]) if b > a else np.zeros(0, np.uint32)
        assert int(cn[s]) == want.size and np.array_equal(sv[a:a + want.size], want), s


def test_dense_sets_at_odd_offsets(ctx, torch_dev):
    """Circle sets (nearly every point survives) starting at odd offsets:
    their dense spans are stored at every output alignment."""
    parts = [workloads.circle(n, 70 + n % 7) for n in (1, 3, 40_001, 2, 70_003, 5, 33_333)]
    off = np.zeros(len(parts) + 1, np.uint64)
    off[1:] = np.cumsum([p.shape[0] for p in parts])
    pts = np.concatenate(parts, axis=0)
    sv, cn = _run(ctx, torch_dev, pts, off)
    _check(pts, off, sv, cn, "dense sets at odd offsets")


@pytest.mark.parametrize("skip", ["1", "0"])
def test_region_skip_in_batches(torch_dev, monkeypatch, skip):
    """Large normal sets (most groups skipped by the region skip) mixed with
    sets whose near-edge points are scattered through them (their boxes must
    not be skipped), with the region skip on and off."""
    from tests import cases
    monkeypatch.setenv("HULLF_REGION_SKIP", skip)
    c = hullf.Context(0)
    try:
        parts = []
        for k, n in enumerate((300_007, 5, 120_001, 70_000, 250_003)):
            xy = workloads.normal(n, 90 + k)
            if k % 2 == 0 and n > 1000:
                xy = cases.with_near_edge_points(xy, oracle.extremes, per_edge=150, seed=k)
                xy = xy[np.random.default_rng(k).permutation(xy.shape[0])]
            parts.append(xy)
        off = np.zeros(len(parts) + 1, np.uint64)
        off[1:] = np.cumsum([p.shape[0] for p in parts])
        pts = np.concatenate(parts, axis=0)
        say(f"[gpu] batched region skip {skip}: {len(parts)} sets, {pts.shape[0]} points")
        sv, cn = _run(c, torch_dev, pts, off)
        _check(pts, off, sv, cn, f"region skip {skip}")
        sv, cn = _run(c, torch_dev, pts, off, offset=1)
        _check(pts, off, sv, cn, f"region skip {skip}, misaligned")
    finally:
        c.close()


def test_bad_offsets_are_reported(ctx, torch_dev):
    pts, off = _mixed_batch(5, 10)
    off = off.copy()
    off[3], off[4] = off[4], off[3]   # decreasing
    if off[3] == off[4]:
        off[4] += 1
    sv, cn = _run(ctx, torch_dev, pts, off)
    assert (cn == np.uint64(hullf.COUNT_BAD_OFFSETS)).all()


def test_autotune_then_parity(ctx, torch_dev):
    import torch
    pts, off = _mixed_batch(6, 300)
    t = upload(pts, torch_dev)
    o = torch.from_numpy(off.astype(np.int64)).to(torch_dev)
    surv = torch.empty(pts.shape[0], dtype=torch.int32, device=torch_dev)
    counts = torch.empty(300, dtype=torch.int64, device=torch_dev)
    say("[gpu] batched autotune")
    b, p, ms = ctx.autotune_batched(t, o, surv, counts, reps=2)
    assert (b, p) in SHAPES and ms > 0
    ctx.hull_filter_batched(t, o, surv=surv, counts=counts)
    torch.cuda.synchronize()
    _check(pts, off, surv.cpu().numpy().astype(np.uint32), counts.cpu().numpy(), "after autotune")


@pytest.mark.parametrize("block,ppt", SHAPES)
def test_batched_structured_keep_patterns(ctx, torch_dev, block, ppt):
    """Sets whose survivors form structured patterns, at odd set offsets."""
    from tests import cases
    parts = [cases.keep_pattern_set(70 + k, lead) for k, lead in enumerate((0, 1, 3, 5))]
    parts.insert(2, workloads.request("normal", 77, 5))
    off = np.zeros(len(parts) + 1, dtype=np.uint64)
    off[1:] = np.cumsum([p.shape[0] for p in parts])
    pts = np.concatenate(parts, axis=0).astype(np.float32)
    say(f"[gpu] batched structured keep patterns block={block} ppt={ppt}")
    sv, cn = _run(ctx, torch_dev, pts, off, block=block, ppt=ppt)
    _check(pts, off, sv, cn, f"structured {block}x{ppt}")
