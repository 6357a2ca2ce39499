"""A context created with a workspace cap refuses calls whose scratch would
exceed it (HULLF_ENOMEM), leaves the caller's outputs untouched, and stays
usable for calls that fit.  The condition is forced from the host by the cap
itself; no kernel runs out of memory."""
from __future__ import annotations

import numpy as np
import pytest

import oracle
from paper_2303_10581_amd import hullf, workloads
from tests.gpu_common import say, torch_dev, upload  # noqa: F401

pytestmark = pytest.mark.gpu


def test_workspace_cap_gives_enomem_and_context_stays_usable(torch_dev):
    import torch
    cap = 1 << 20
    c = hullf.Context(0, workspace_bytes=cap)
    try:
        used, got_cap = c.workspace()
        assert got_cap == cap and 0 < used <= cap
        small = workloads.normal(1_000_000, 3)   # keep bits 125 KB + boxes 31 KB: fits
        ts = upload(small, torch_dev)
        say("[gpu] workspace cap 1 MiB: 1e6 points")
        s, n = c.hull_filter(ts)
        torch.cuda.synchronize()
        assert np.array_equal(s[:int(n.item())].cpu().numpy().astype(np.uint32), oracle.survivors(small))
        assert c.workspace()[0] <= cap

        big = workloads.normal(10_000_000, 4)    # keep bits alone: 1.25 MB
        tb = upload(big, torch_dev)
        surv = torch.full((16,), -7, dtype=torch.int32, device=torch_dev)
        count = torch.full((1,), -5, dtype=torch.int64, device=torch_dev)
        say("[gpu] workspace cap 1 MiB: 1e7 points (refused)")
        with pytest.raises(hullf.HullfError) as e:
            c.hull_filter(tb, surv=surv, count=count, cap=16)
        assert e.value.status == hullf.ENOMEM
        torch.cuda.synchronize()
        assert int(count.item()) == -5 and (surv.cpu().numpy() == -7).all()
        with pytest.raises(hullf.HullfError) as e:
            c.convex_hull(tb)
        assert e.value.status == hullf.ENOMEM
        assert c.workspace()[0] <= cap

        say("[gpu] workspace cap 1 MiB: 1e6 points again")
        s, n = c.hull_filter(ts)
        torch.cuda.synchronize()
        assert np.array_equal(s[:int(n.item())].cpu().numpy().astype(np.uint32), oracle.survivors(small))
    finally:
        c.close()


def test_workspace_cap_below_creation_needs(torch_dev):
    with pytest.raises(hullf.HullfError) as e:
        hullf.Context(0, workspace_bytes=4096)
    assert e.value.status == hullf.ENOMEM


def test_uncapped_context_reports_its_workspace(torch_dev):
    c = hullf.Context(0)
    try:
        xy = workloads.circle(300_007, 12)
        s, n = c.hull_filter(upload(xy, torch_dev))
        used, cap = c.workspace()
        assert cap == 0 and used > 300_007 // 8
    finally:
        c.close()
