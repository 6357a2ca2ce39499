"""GPU parity at the full sizes of the study cases, hull included.

The oracle's results for these sets take minutes on one host thread (the
hull of 1e8 circle points alone about 90 s), so they are stored in
tests/golden/ by make_full_size.py, which calls only the oracle.  Lists are
compared through SHA-256 of their little-endian uint32 bytes, which is a bit
for bit comparison; the generated points are hashed first so that a changed
generator is reported as such, not as a wrong result.

Compared per set: the eight octagon vertices (Sec. 3.1), the survivor count
and list (Sec. 3.2, 4.1.1), the counter-clockwise hull (Sec. 3.3), through
the C ABI's hullf_octagon, hull_filter and convex_hull.  For the 4096-set
batch: every set's survivors from hull_filter_batched and its hull from
hull_from_survivors."""
from __future__ import annotations

import hashlib
import json
import os

import numpy as np
import pytest

from paper_2303_10581_amd import workloads
from tests.gpu_common import ctx, say, torch_dev, upload  # noqa: F401

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def _sha(a: np.ndarray) -> str:
    return hashlib.sha256(np.ascontiguousarray(a).tobytes()).hexdigest()


def _full():
    with open(os.path.join(GOLDEN, "full_size.json")) as f:
        return json.load(f)


@pytest.mark.parametrize("name", ["normal_1e8", "circle_1e8", "displaced_1e8", "circle_jitter_5e8"])
def test_full_size_octagon_survivors_hull(ctx, torch_dev, name):
    import torch
    rec = _full()[name]
    say(f"[gpu] full size {name}: n={rec['n']} seed={rec['seed']}")
    xy = workloads.by_kind(rec["kind"], rec["n"], rec["seed"])
    assert _sha(xy) == rec["points_sha256"], "the input generator changed; rerun make_full_size.py"
    t = torch.from_numpy(xy).to(torch_dev)
    del xy
    assert ctx.octagon(t).tolist() == rec["extremes"], name
    surv, count = ctx.hull_filter(t)
    c = int(count.item())
    assert c == rec["survivors"], (name, c, rec["survivors"])
    got = surv[:c].cpu().numpy().astype("<u4")
    assert _sha(got) == rec["survivors_sha256"], name
    del surv, got
    say(f"[gpu] full size {name}: hull")
    h = ctx.convex_hull(t).astype("<u4")
    assert h.size == rec["hull"], (name, h.size, rec["hull"])
    assert h[:8].tolist() == rec["hull_head"], name
    assert _sha(h) == rec["hull_sha256"], name
    del t
    torch.cuda.empty_cache()


def _batch_golden():
    rows = {}
    head = None
    with open(os.path.join(GOLDEN, "batch_4096.txt")) as f:
        for line in f:
            if line.startswith("# sha256(points)="):
                head = line.split()[1].split("=")[1]
            elif line.strip() and not line.startswith("#"):
                s, nsurv, nhull, hs, hh = line.split()
                rows[int(s)] = (int(nsurv), int(nhull), hs, hh)
    return head, rows


def test_full_batched_config_survivors_and_hulls(ctx, torch_dev):
    import torch
    head, rows = _batch_golden()
    pts, off, _ = workloads.batch(S=4096, seed=6)
    assert _sha(pts) == head, "the input generator changed; rerun make_full_size.py"
    S = off.size - 1
    say(f"[gpu] batched config: S={S} n={pts.shape[0]}")
    tp = torch.from_numpy(pts).to(torch_dev)
    to = torch.from_numpy(off.astype(np.int64)).to(torch_dev)
    surv, counts = ctx.hull_filter_batched(tp, to)
    torch.cuda.synchronize()
    cn = counts.cpu().numpy()
    sv = surv.cpu().numpy().astype("<u4")
    bad = []
    for s in range(S):
        a = int(off[s])
        nsurv, nhull, hs, hh = rows[s]
        if int(cn[s]) != nsurv or _sha(sv[a:a + nsurv])[:16] != hs:
            bad.append(("survivors", s))
    assert not bad, bad[:10]
    say("[gpu] batched config: hull of every set from its survivors")
    for s in range(S):
        a, b = int(off[s]), int(off[s + 1])
        nsurv, nhull, hs, hh = rows[s]
        h = ctx.hull_from_survivors(tp[a:b], surv[a:a + nsurv], nsurv).astype("<u4")
        if h.size != nhull or _sha(h)[:16] != hh:
            bad.append(("hull", s, h.size, nhull))
    assert not bad, bad[:10]


def _full16():
    with open(os.path.join(GOLDEN, "full_size16.json")) as f:
        return json.load(f)


@pytest.mark.parametrize("name", ["normal_1e8", "circle_1e8", "displaced_1e8", "circle_jitter_5e8"])
def test_full_size_filter16(ctx, torch_dev, name):
    """The 16-direction filter (Sec. 2) at the full sizes: its 16 vertices
    and its survivor list, bit for bit."""
    import torch
    rec = _full16()[name]
    say(f"[gpu] full size filter16 {name}: n={rec['n']} seed={rec['seed']}")
    xy = workloads.by_kind(rec["kind"], rec["n"], rec["seed"])
    assert _sha(xy) == rec["points_sha256"], "the input generator changed; rerun make_full_size.py"
    t = torch.from_numpy(xy).to(torch_dev)
    del xy
    assert ctx.polygon16(t).tolist() == rec["vertices"], name
    surv, count = ctx.hull_filter16(t)
    c = int(count.item())
    assert c == rec["survivors"], (name, c, rec["survivors"])
    got = surv[:c].cpu().numpy().astype("<u4")
    assert _sha(got) == rec["survivors_sha256"], name
    del surv, got, t
    torch.cuda.empty_cache()
