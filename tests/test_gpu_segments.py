"""GPU parity of the segment-list batched launch (sets at arbitrary places in
one device array, gaps not read): every segment's count and set-local
survivor list must equal the oracle run on that segment alone."""
from __future__ import annotations

import numpy as np
import pytest

import oracle
from paper_2303_10581_amd import hullf, workloads
from tests.gpu_common import ctx, say, torch_dev  # noqa: F401

pytestmark = pytest.mark.gpu


def _layout(seed: int, S: int, max_n: int = 40000):
    """Sets of mixed kinds placed in ascending order with random gaps; the
    gaps hold NaN, so a read outside a segment would flag it non-finite."""
    rng = np.random.default_rng(seed)
    sets, seg = [], []
    pos = int(rng.integers(0, 5))
    for s in range(S):
        r = rng.random()
        n = 0 if r < 0.08 else (int(rng.integers(1, 4)) if r < 0.16 else
                                int(np.exp(rng.uniform(np.log(5), np.log(max_n)))))
        xy = workloads.request(workloads.KINDS[s % 3], n, seed * 7919 + s) if n else np.zeros((0, 2), np.float32)
        seg.append((pos, n))
        sets.append(xy)
        pos += n + (0 if rng.random() < 0.3 else int(rng.integers(1, 200)))
    n_total = pos + int(rng.integers(0, 100))
    arena = np.full((n_total, 2), np.nan, dtype=np.float32)
    for (b, n), xy in zip(seg, sets):
        arena[b:b + n] = xy
    return arena, np.array(seg, dtype=np.uint64).reshape(-1, 2), sets


def _run(ctx, dev, arena, seg):
    import torch
    t = torch.from_numpy(arena).to(dev)
    s = torch.from_numpy(seg.astype(np.int64)).to(dev)
    surv, counts = ctx.hull_filter_segments(t, s, n_total=arena.shape[0])
    torch.cuda.synchronize()
    return surv.cpu().numpy().astype(np.uint32), counts.cpu().numpy().astype(np.uint64)


def _check(sets, seg, sv, cn, name):
    for k, ((b, n), xy) in enumerate(zip(seg.tolist(), sets)):
        want = oracle.survivors(xy) if n else np.zeros(0, np.uint32)
        assert int(cn[k]) == want.size, (name, k, int(cn[k]), want.size)
        assert np.array_equal(sv[b:b + want.size], want), (name, k)


@pytest.mark.parametrize("seed,S", [(11, 1), (12, 37), (13, 400)])
def test_segments_with_gaps(ctx, torch_dev, seed, S):
    arena, seg, sets = _layout(seed, S)
    say(f"[gpu] segments seed={seed} S={S} n_total={arena.shape[0]}")
    sv, cn = _run(ctx, torch_dev, arena, seg)
    _check(sets, seg, sv, cn, f"segments {seed}")


def test_segments_match_csr(ctx, torch_dev):
    """Back-to-back segments give exactly the CSR batched result."""
    import torch
    arena, seg, sets = _layout(14, 60)
    pts = np.concatenate([s for s in sets if s.shape[0]], axis=0)
    counts = np.array([s.shape[0] for s in sets], np.uint64)
    off = np.zeros(len(sets) + 1, np.uint64)
    off[1:] = np.cumsum(counts)
    seg2 = np.stack([off[:-1], counts], axis=1)
    say("[gpu] segments vs csr")
    sv_s, cn_s = _run(ctx, torch_dev, pts, seg2)
    t = torch.from_numpy(pts).to(torch_dev)
    o = torch.from_numpy(off.astype(np.int64)).to(torch_dev)
    sv_c, cn_c = ctx.hull_filter_batched(t, o, block=256, ppt=16)
    torch.cuda.synchronize()
    cn_c = cn_c.cpu().numpy().astype(np.uint64)
    sv_c = sv_c.cpu().numpy().astype(np.uint32)
    assert np.array_equal(cn_s, cn_c)
    for k in range(len(sets)):
        a, c = int(off[k]), int(cn_s[k])
        assert np.array_equal(sv_s[a:a + c], sv_c[a:a + c]), k


@pytest.mark.parametrize("what", ["overlap", "descending", "past_end"])
def test_invalid_segment_lists(ctx, torch_dev, what):
    arena, seg, sets = _layout(15, 12)
    seg = seg.copy()
    if what == "overlap":
        k = next(k for k in range(11) if seg[k, 1] > 1)
        seg[k + 1, 0] = seg[k, 0] + 1
    elif what == "descending":
        k = next(k for k in range(11) if seg[k, 1] > 0 and seg[k + 1, 1] > 0)
        seg[[k, k + 1]] = seg[[k + 1, k]]
    else:
        seg[-1, 1] = arena.shape[0] - int(seg[-1, 0]) + 1
    say(f"[gpu] segments invalid ({what})")
    sv, cn = _run(ctx, torch_dev, arena, seg)
    assert (cn == np.uint64(hullf.COUNT_BAD_OFFSETS)).all(), what
