"""GPU parity of hull finishing for a whole batch at once
(hull_from_survivors_batched: one device sort in which every set is sorted
on its own, run representatives, chunk chains and merge rounds that never
cross a set): every set's counter-clockwise hull index list bit for bit
against the oracle, for batches with empty, one-point, collinear, repeated,
vertical-line and large sets, and for the 4096-set batched configuration
(stored oracle hashes)."""
from __future__ import annotations

import hashlib
import os

import numpy as np
import pytest

import oracle
from paper_2303_10581_amd import hullf, workloads
from tests import cases
from tests.gpu_common import ctx, say, torch_dev  # noqa: F401

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def _set(kind: str, n: int, seed: int) -> np.ndarray:
    rng = np.random.default_rng(seed)
    if n == 0:
        return np.zeros((0, 2), np.float32)
    if kind == "equal":
        return np.full((n, 2), 1.5, np.float32)
    if kind == "collinear":
        t = rng.uniform(-1.0, 1.0, n)
        return np.stack([t, 0.5 * t + 0.25], axis=1).astype(np.float32)
    if kind == "vertical":
        xs = rng.integers(0, 3, n).astype(np.float32)
        return np.stack([xs, rng.standard_normal(n).astype(np.float32)], axis=1)
    if kind == "grid":
        return cases.named_sets(max(n, 8), seed)["grid"][:n]
    xy = workloads.by_kind(kind, n, seed)
    if kind != "normal" and n > 10:
        xy[rng.integers(0, n, 5)] = xy[rng.integers(0, n)]   # repeated points
    return xy


def _batch(spec, seed0):
    sets = [_set(k, n, seed0 + i) for i, (k, n) in enumerate(spec)]
    off = np.zeros(len(sets) + 1, np.int64)
    off[1:] = np.cumsum([s.shape[0] for s in sets])
    pts = np.concatenate(sets, axis=0) if off[-1] else np.zeros((0, 2), np.float32)
    return sets, off, pts


def _check_batch(ctx, dev, spec, seed0, name):
    import torch
    sets, off, pts = _batch(spec, seed0)
    say(f"[gpu] batch finish {name}: S={len(sets)} n={pts.shape[0]}")
    tp = torch.from_numpy(np.ascontiguousarray(pts)).to(dev)
    to = torch.from_numpy(off).to(dev)
    surv, counts = ctx.hull_filter_batched(tp, to)
    hulls, hoff = ctx.hulls_batched(tp, to, surv, counts)
    for s, xy in enumerate(sets):
        want = oracle.hull(xy, oracle.survivors(xy)) if xy.shape[0] else np.zeros(0, np.uint32)
        got = hulls[hoff[s]:hoff[s + 1]]
        assert np.array_equal(got, want), (name, s, spec[s], got[:8], want[:8])


def test_small_and_degenerate_sets(ctx, torch_dev):
    spec = [("normal", 0), ("normal", 1), ("circle", 2), ("normal", 3), ("equal", 5), ("collinear", 7),
            ("vertical", 64), ("circle", 65), ("normal", 0), ("displaced", 1000), ("grid", 100),
            ("circle", 4097), ("equal", 3000), ("collinear", 2500), ("normal", 1)]
    _check_batch(ctx, torch_dev, spec, 300, "small and degenerate")


@pytest.mark.parametrize("seed", [0, 1])
def test_mixed_sizes(ctx, torch_dev, seed):
    """Sets across every tile border of the sort (4096), the run pass (1024)
    and the chunk size, some large enough for several chunk levels and merge
    rounds."""
    rng = np.random.default_rng(400 + seed)
    kinds = ["normal", "circle", "displaced", "circle_jitter", "vertical", "collinear"]
    sizes = [1023, 1024, 1025, 4095, 4096, 4097, 20_000, 150_001, 700_003, 31, 0, 9]
    spec = [(kinds[rng.integers(0, len(kinds))], int(n)) for n in rng.permutation(sizes)]
    _check_batch(ctx, torch_dev, spec, 500 + 50 * seed, f"mixed sizes {seed}")


def test_many_small_sets(ctx, torch_dev):
    """Thousands of sets, most of them below one sort tile: binary searches
    over many sets, pieces of every size."""
    rng = np.random.default_rng(77)
    sizes = np.exp(rng.uniform(np.log(1), np.log(3000), 3000)).astype(int)
    kinds = ["normal", "circle", "displaced"]
    spec = [(kinds[int(rng.integers(0, 3))], int(n)) for n in sizes]
    _check_batch(ctx, torch_dev, spec, 900, "3000 small sets")


def test_one_large_set_equals_convex_hull(ctx, torch_dev):
    """A batch of one set gives convex_hull's result."""
    import torch
    xy = workloads.circle(1_000_003, 17)
    tp = torch.from_numpy(xy).to(torch_dev)
    to = torch.tensor([0, xy.shape[0]], dtype=torch.int64, device=torch_dev)
    surv, counts = ctx.hull_filter_batched(tp, to)
    hulls, hoff = ctx.hulls_batched(tp, to, surv, counts)
    assert np.array_equal(hulls, ctx.convex_hull(tp))


def test_nonfinite_set_is_reported(ctx, torch_dev):
    import torch
    a = workloads.normal(1000, 1)
    b = workloads.normal(1000, 2)
    b[17, 0] = np.nan
    pts = np.concatenate([a, b], axis=0)
    tp = torch.from_numpy(pts).to(torch_dev)
    to = torch.tensor([0, 1000, 2000], dtype=torch.int64, device=torch_dev)
    surv, counts = ctx.hull_filter_batched(tp, to)
    with pytest.raises(hullf.HullfError) as e:
        ctx.hulls_batched(tp, to, surv, counts)
    assert e.value.status == hullf.ENONFINITE


def test_capacity_and_bad_counts(ctx, torch_dev):
    """Too small a host array: HULLF_ECAPACITY with every set's offset
    written; a count above its set's size: HULLF_EINVAL."""
    import torch
    sets, off, pts = _batch([("circle", 3000), ("normal", 500), ("displaced", 2000)], 700)
    tp = torch.from_numpy(pts).to(torch_dev)
    to = torch.from_numpy(off).to(torch_dev)
    surv, counts = ctx.hull_filter_batched(tp, to)
    hulls, hoff = ctx.hulls_batched(tp, to, surv, counts)
    lib = hullf._load()
    S = len(sets)
    out = np.zeros(4, np.uint32)
    ho = np.zeros(S + 1, np.uint64)
    st = lib.hull_from_survivors_batched(ctx.handle, tp.data_ptr(), to.data_ptr(), S, pts.shape[0],
                                         surv.data_ptr(), counts.data_ptr(), out.ctypes.data, 4, ho.ctypes.data,
                                         hullf._stream(None))
    assert st == hullf.ECAPACITY
    assert ho.astype(np.int64).tolist() == hoff.tolist()
    assert (out == 0).all()
    bad = counts.clone()
    bad[1] = 501
    with pytest.raises(hullf.HullfError) as e:
        ctx.hulls_batched(tp, to, surv, bad)
    assert e.value.status == hullf.EINVAL


def _sha(a: np.ndarray) -> str:
    return hashlib.sha256(np.ascontiguousarray(a).tobytes()).hexdigest()


def test_full_batched_config_hulls_at_once(ctx, torch_dev):
    """The 4096-set configuration: every set's hull from one batched
    finishing call, against the oracle's stored hashes."""
    import torch
    rows = {}
    head = None
    with open(os.path.join(GOLDEN, "batch_4096.txt")) as f:
        for line in f:
            if line.startswith("# sha256(points)="):
                head = line.split()[1].split("=")[1]
            elif line.strip() and not line.startswith("#"):
                s, nsurv, nhull, hs, hh = line.split()
                rows[int(s)] = (int(nsurv), int(nhull), hs, hh)
    pts, off, _ = workloads.batch(S=4096, seed=6)
    assert _sha(pts) == head, "the input generator changed; rerun make_full_size.py"
    say(f"[gpu] batched config, hulls at once: n={pts.shape[0]}")
    tp = torch.from_numpy(pts).to(torch_dev)
    to = torch.from_numpy(off.astype(np.int64)).to(torch_dev)
    surv, counts = ctx.hull_filter_batched(tp, to)
    hulls, hoff = ctx.hulls_batched(tp, to, surv, counts)
    bad = []
    for s in range(off.size - 1):
        nsurv, nhull, hs, hh = rows[s]
        h = hulls[hoff[s]:hoff[s + 1]].astype("<u4")
        if h.size != nhull or _sha(h)[:16] != hh:
            bad.append((s, h.size, nhull))
    assert not bad, bad[:10]
