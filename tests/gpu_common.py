"""Helpers for the GPU tests: device context, uploads, oracle comparison."""
from __future__ import annotations

import sys

import numpy as np
import pytest


def say(msg: str):
    """Flushed progress line naming the case before each GPU step."""
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="session")
def torch_dev():
    import torch
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a ROCm GPU")
    return torch.device("cuda:0")


@pytest.fixture(scope="session")
def ctx(torch_dev):
    from paper_2303_10581_amd import hullf
    c = hullf.Context(0)
    yield c
    c.close()


def upload(xy: np.ndarray, dev, offset_points: int = 0):
    """Copy points to the device; offset_points > 0 places them at an
    8-byte (not 16-byte) aligned address inside a larger buffer."""
    import torch
    a = np.ascontiguousarray(xy, dtype=np.float32)
    if offset_points == 0:
        return torch.from_numpy(a).to(dev)
    buf = torch.zeros((a.shape[0] + offset_points, 2), dtype=torch.float32, device=dev)
    buf[offset_points:] = torch.from_numpy(a).to(dev)
    return buf[offset_points:]


def survivors_np(ctx, t) -> np.ndarray:
    s = ctx.survivors(t)
    return s.cpu().numpy().astype(np.uint32)
