"""GPU tests of the request loop (continuous batching): every request's hull
is bit-identical to the oracle hull of its points, alone and in a mix of
concurrent requests, under memory pressure, with page-locked and pageable
inputs; failures stay with their own request."""
from __future__ import annotations

import numpy as np
import pytest

import oracle
from paper_2303_10581_amd import hullf, workloads
from tests.gpu_common import say, torch_dev  # noqa: F401

pytestmark = pytest.mark.gpu


def _requests(seed: int, m: int, lo: float, hi: float):
    rng = np.random.default_rng(seed)
    sizes = np.rint(np.exp(rng.uniform(np.log(lo), np.log(hi), m))).astype(np.int64)
    return [workloads.request(workloads.KINDS[k % 3], int(n), seed * 1000 + k) for k, n in enumerate(sizes)]


def _oracle_hulls(reqs):
    return [oracle.hull(xy) for xy in reqs]


@pytest.fixture(scope="module")
def mix():
    reqs = _requests(21, 36, 1e3, 3e5)
    return reqs, _oracle_hulls(reqs)


def test_alone_equals_mix_equals_oracle(torch_dev, mix):
    reqs, want = mix
    with hullf.Server(0, arena_points=1 << 24) as srv:
        say(f"[gpu] server alone: {len(reqs)} requests one at a time")
        alone = []
        for xy in reqs:
            rid = srv.submit(xy)
            h, info = srv.wait(rid)
            assert info["batch_requests"] == 1
            alone.append(h)
        say(f"[gpu] server mix: {len(reqs)} requests at once")
        ids = [srv.submit(xy) for xy in reqs]
        got = [srv.wait(i) for i in ids]
        st = srv.stats()
    for k, (xy, w) in enumerate(zip(reqs, want)):
        assert np.array_equal(alone[k], w), ("alone", k, xy.shape[0])
        assert np.array_equal(got[k][0], w), ("mix", k, xy.shape[0])
        assert got[k][1]["survivors"] >= w.size
    assert st["completed"] == st["submitted"] == 2 * len(reqs)
    # the mix really was batched: fewer launches than requests
    assert st["batches"] < 2 * len(reqs)


def test_admission_waits_for_memory(torch_dev, mix):
    """An arena that holds only a few requests at once: later requests wait
    for memory and still get their exact hulls."""
    reqs, want = mix
    big = max(x.shape[0] for x in reqs)
    with hullf.Server(0, arena_points=big + 4096, max_inflight=8, finish_threads=2) as srv:
        say(f"[gpu] server small arena ({big + 4096} points)")
        ids = [srv.submit(xy) for xy in reqs]
        got = [srv.wait(i) for i in ids]
        st = srv.stats()
    for k, w in enumerate(want):
        assert np.array_equal(got[k][0], w), k
    assert st["arena_peak_points"] <= big + 4096 + 64


def test_pinned_inputs(torch_dev, mix):
    import torch
    reqs, want = mix
    pinned = []
    for xy in reqs[:12]:
        t = torch.empty(xy.shape, dtype=torch.float32, pin_memory=True)
        t.copy_(torch.from_numpy(xy))
        pinned.append(t)
    with hullf.Server(0, arena_points=1 << 23) as srv:
        say("[gpu] server pinned inputs")
        ids = [srv.submit(t) for t in pinned]
        got = [srv.wait(i) for i in ids]
    for k in range(12):
        assert np.array_equal(got[k][0], want[k]), k


def test_large_pageable_request_through_staging(torch_dev):
    # more than the staging slots hold at once (4 x 2^20 points)
    xy = workloads.displaced(5_000_003, 31)
    want = oracle.convex_hull(xy)
    with hullf.Server(0, arena_points=1 << 23) as srv:
        say("[gpu] server 5e6-point pageable request")
        h, info = srv.wait(srv.submit(xy))
    assert np.array_equal(h, want)
    assert info["survivors"] == oracle.survivors(xy).size


def test_failures_stay_with_their_request(torch_dev, mix):
    reqs, want = mix
    bad = reqs[5].copy()
    bad[17, 1] = np.inf
    with hullf.Server(0, arena_points=1 << 22) as srv:
        say("[gpu] server non-finite request in a mix")
        ids = [srv.submit(xy) for xy in reqs[:5]] + [srv.submit(bad)] + [srv.submit(xy) for xy in reqs[6:12]]
        empty = srv.submit(np.zeros((0, 2), np.float32))
        with pytest.raises(hullf.HullfError) as e:
            srv.wait(ids[5])
        assert e.value.status == hullf.ENONFINITE
        for k in list(range(5)) + list(range(6, 12)):
            assert np.array_equal(srv.wait(ids[k])[0], want[k]), k
        h, info = srv.wait(empty)
        assert h.size == 0
        with pytest.raises(hullf.HullfError) as e:
            srv.submit(np.zeros(((1 << 22) + 1, 2), np.float32))
        assert e.value.status == hullf.ENOMEM


def test_degenerate_requests(torch_dev):
    one = np.array([[1.5, -2.0]], np.float32)
    same = np.repeat(one, 1000, axis=0)
    line = np.stack([np.arange(5000, dtype=np.float32), np.arange(5000, dtype=np.float32) * 2], axis=1)
    with hullf.Server(0, arena_points=1 << 20) as srv:
        say("[gpu] server degenerate requests")
        ids = [srv.submit(x) for x in (one, same, line)]
        got = [srv.wait(i)[0] for i in ids]
    for x, g in zip((one, same, line), got):
        assert np.array_equal(g, oracle.hull(x))
