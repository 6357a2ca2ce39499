"""Seeded synthetic point sets (the three study cases of Sec. 5).

This module holds no arithmetic of the method: it only draws inputs.  Both
the HIP path's tests and the oracle's tests take their inputs from here.

Recipes (numpy PCG64; values drawn in float64, rounded once to float32, AoS
rows [x, y]; generated in chunks of 2^22 points, chunk k seeded by
SeedSequence(seed).spawn(...)[k], so that large sets are reproducible without
large temporaries):

  normal(n, seed)             x, y ~ N(0, 1) i.i.d.
  circle(n, seed)             theta ~ U[0, 2 pi), (cos theta, sin theta)
  displaced(n, seed, p)       theta ~ U[0, 2 pi), radius 1 + U[-p, p]
  circle_jitter(n, seed, s)   theta ~ U[0, 2 pi), radius 1 + N(0, s)
  batch(S, seed, ...)         S sets, sizes log-uniform, kind uniform over
                              {normal, circle, displaced p=0.05}, each set
                              moved to a centre ~ U[-100, 100]^2 and scaled by
                              U[0.1, 10]; returns points, CSR offsets, kinds
  arrivals(m, seed, qps, ...) Poisson arrival times and request sizes
"""
from __future__ import annotations

import math
import os
from concurrent.futures import ThreadPoolExecutor

import numpy as np

CHUNK = 1 << 22
KINDS = ("normal", "circle", "displaced")


def _threads() -> int:
    return max(1, min(16, os.cpu_count() or 1))


def _chunked(n: int, seed: int, fill) -> np.ndarray:
    out = np.empty((n, 2), dtype=np.float32)
    if n == 0:
        return out
    nch = (n + CHUNK - 1) // CHUNK
    seqs = np.random.SeedSequence(seed).spawn(nch)

    def work(k):
        lo = k * CHUNK
        hi = min(n, lo + CHUNK)
        rng = np.random.Generator(np.random.PCG64(seqs[k]))
        out[lo:hi] = fill(rng, hi - lo)

    if nch == 1:
        work(0)
    else:
        with ThreadPoolExecutor(_threads()) as ex:
            list(ex.map(work, range(nch)))
    return out


def _normal(rng, m):
    return rng.standard_normal((m, 2))


def _ring(rng, m, radius):
    th = rng.uniform(0.0, 2.0 * math.pi, m)
    r = radius(rng, m)
    return np.stack([r * np.cos(th), r * np.sin(th)], axis=1)


def normal(n: int, seed: int = 1) -> np.ndarray:
    return _chunked(n, seed, _normal)


def circle(n: int, seed: int = 3) -> np.ndarray:
    return _chunked(n, seed, lambda rng, m: _ring(rng, m, lambda r, k: 1.0))


def displaced(n: int, seed: int = 4, p: float = 0.05) -> np.ndarray:
    return _chunked(n, seed, lambda rng, m: _ring(
        rng, m, lambda r, k: 1.0 + r.uniform(-p, p, k)))


def circle_jitter(n: int, seed: int = 5, sigma: float = 0.01) -> np.ndarray:
    return _chunked(n, seed, lambda rng, m: _ring(
        rng, m, lambda r, k: 1.0 + sigma * r.standard_normal(k)))


def by_kind(kind: str, n: int, seed: int) -> np.ndarray:
    if kind == "normal":
        return normal(n, seed)
    if kind == "circle":
        return circle(n, seed)
    if kind == "displaced":
        return displaced(n, seed, 0.05)
    if kind == "circle_jitter":
        return circle_jitter(n, seed, 0.01)
    raise ValueError(kind)


def log_uniform_sizes(rng, count: int, lo: float, hi: float) -> np.ndarray:
    return np.rint(np.exp(rng.uniform(math.log(lo), math.log(hi), count))).astype(np.int64)


def batch(S: int = 4096, seed: int = 6, lo: float = 1e2, hi: float = 1e6):
    """Returns (points float32 (N, 2), off uint64 (S+1,), kinds list)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    sizes = log_uniform_sizes(rng, S, lo, hi)
    kinds = [KINDS[k] for k in rng.integers(0, 3, S)]
    centre = rng.uniform(-100.0, 100.0, (S, 2))
    scale = rng.uniform(0.1, 10.0, S)
    off = np.zeros(S + 1, dtype=np.uint64)
    off[1:] = np.cumsum(sizes)
    pts = np.empty((int(off[-1]), 2), dtype=np.float32)
    seqs = np.random.SeedSequence(seed).spawn(S)

    def work(s):
        r = np.random.Generator(np.random.PCG64(seqs[s]))
        m = int(sizes[s])
        if kinds[s] == "normal":
            base = _normal(r, m)
        elif kinds[s] == "circle":
            base = _ring(r, m, lambda g, k: 1.0)
        else:
            base = _ring(r, m, lambda g, k: 1.0 + g.uniform(-0.05, 0.05, k))
        pts[int(off[s]):int(off[s + 1])] = centre[s] + scale[s] * base

    with ThreadPoolExecutor(_threads()) as ex:
        list(ex.map(work, range(S)))
    return pts, off, kinds


def request(kind: str, n: int, seed: int) -> np.ndarray:
    """One serving request: a set of the given kind, moved and scaled as in
    batch()."""
    rng = np.random.Generator(np.random.PCG64(seed))
    centre = rng.uniform(-100.0, 100.0, 2)
    scale = rng.uniform(0.1, 10.0)
    if kind == "normal":
        base = _normal(rng, n)
    elif kind == "circle":
        base = _ring(rng, n, lambda g, k: 1.0)
    else:
        base = _ring(rng, n, lambda g, k: 1.0 + g.uniform(-0.05, 0.05, k))
    return (centre + scale * base).astype(np.float32)


def arrivals(m: int, seed: int = 7, qps: float = 100.0, lo: float = 1e3, hi: float = 1e7):
    """Poisson arrivals: (times in s, sizes, kinds, per-request seeds)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    gaps = rng.exponential(1.0 / qps, m)
    times = np.cumsum(gaps)
    sizes = log_uniform_sizes(rng, m, lo, hi)
    kinds = [KINDS[k] for k in rng.integers(0, 3, m)]
    seeds = rng.integers(0, 2**31 - 1, m)
    return times, sizes, kinds, seeds
