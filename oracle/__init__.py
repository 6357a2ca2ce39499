"""CPU oracle for the octagon filter and the convex hull (arXiv 2303.10581).

TEST INFRASTRUCTURE ONLY: imported by ``tests/``, by ``__graft_entry__.smoke``
and by the ``cpu_baseline`` leg of ``bench.py``; never by the product path.
It shares no code with the HIP library.  ``oracle.c`` holds the arithmetic;
this module only builds it and marshals numpy arrays.

Functions follow Algorithm 1 of the paper:
  extremes(xy)   -- Sec. 3.1, the eight octagon vertices (indices)
  keep(xy, idx)  -- Sec. 3.2, the inside test (1 = survives)
  survivors(xy)  -- Sec. 4.1.1, ascending indices of the survivors
  survivors_omp  -- the same on every host core (CPU baseline timing)
  extremes16, keep_poly, survivors16
                 -- Sec. 2, the 16-direction filter of the related work
  hull(xy, sub)  -- Sec. 3.3, counter-clockwise hull vertex indices
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lib = None


def build(force: bool = False) -> str:
    """Compile oracle.c with gcc (FMA contraction off) into liboracle.so."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call([
            "gcc", "-O2", "-std=c99", "-ffp-contract=off", "-fno-fast-math",
            "-fexcess-precision=standard", "-fopenmp", "-shared", "-fPIC", "-o", tmp, _SRC, "-lm",
        ])
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        build()
        lib = ctypes.CDLL(_LIB)
        P = ctypes.c_void_p
        U64 = ctypes.c_uint64
        lib.oracle_validate.argtypes = [P, U64]
        lib.oracle_validate.restype = ctypes.c_int
        lib.oracle_extremes.argtypes = [P, U64, P]
        lib.oracle_extremes.restype = None
        lib.oracle_keep.argtypes = [P, U64, P, P]
        lib.oracle_keep.restype = None
        lib.oracle_survivors.argtypes = [P, U64, P, P]
        lib.oracle_survivors.restype = ctypes.c_int64
        lib.oracle_survivors_omp.argtypes = [P, U64, P, P, ctypes.c_int]
        lib.oracle_survivors_omp.restype = ctypes.c_int64
        lib.oracle_extremes16.argtypes = [P, U64, P]
        lib.oracle_extremes16.restype = None
        lib.oracle_keep_poly.argtypes = [P, U64, P, ctypes.c_int, P]
        lib.oracle_keep_poly.restype = None
        lib.oracle_survivors16.argtypes = [P, U64, P, P]
        lib.oracle_survivors16.restype = ctypes.c_int64
        lib.oracle_key16_values.argtypes = [P, U64, ctypes.c_int, P]
        lib.oracle_key16_values.restype = None
        lib.oracle_hull.argtypes = [P, U64, P, U64, P]
        lib.oracle_hull.restype = U64
        F = ctypes.c_float
        lib.oracle_orient_exact.argtypes = [F, F, F, F, F, F]
        lib.oracle_orient_exact.restype = ctypes.c_int
        _lib = lib
    return _lib


class NonFiniteInput(ValueError):
    """A coordinate is NaN or infinite."""


def _pts(xy) -> np.ndarray:
    a = np.ascontiguousarray(xy, dtype=np.float32)
    if a.ndim != 2 or a.shape[1] != 2:
        raise ValueError("points must have shape (n, 2)")
    return a


def validate(xy) -> bool:
    a = _pts(xy)
    return _load().oracle_validate(a.ctypes.data, a.shape[0]) == 0


def extremes(xy) -> np.ndarray:
    """Indices E0..E7 (right, top-right, top, top-left, left, bottom-left,
    bottom, bottom-right), lowest index on ties."""
    a = _pts(xy)
    if a.shape[0] == 0:
        raise ValueError("empty point set has no extremes")
    if not validate(a):
        raise NonFiniteInput("non-finite coordinate")
    out = np.zeros(8, dtype=np.uint32)
    _load().oracle_extremes(a.ctypes.data, a.shape[0], out.ctypes.data)
    return out


def keep(xy, idx=None) -> np.ndarray:
    """uint8 flags, 1 = point survives the octagon with vertex indices idx
    (the octagon of extremes(xy) if idx is None)."""
    a = _pts(xy)
    n = a.shape[0]
    if n == 0:
        return np.zeros(0, dtype=np.uint8)
    if idx is None:
        idx = extremes(a)
    idx = np.ascontiguousarray(idx, dtype=np.uint32)
    out = np.zeros(n, dtype=np.uint8)
    _load().oracle_keep(a.ctypes.data, n, idx.ctypes.data, out.ctypes.data)
    return out


def survivors(xy) -> np.ndarray:
    """Ascending uint32 indices of the points that survive the filter."""
    a = _pts(xy)
    n = a.shape[0]
    out = np.zeros(max(n, 1), dtype=np.uint32)
    c = _load().oracle_survivors(a.ctypes.data, n, out.ctypes.data, None)
    if c == -2:
        raise NonFiniteInput("non-finite coordinate")
    if c < 0:
        raise MemoryError("oracle allocation failed")
    return out[:c].copy()


def survivors_omp(xy, threads: int = 0) -> np.ndarray:
    """survivors(xy) computed on `threads` OpenMP threads (0: all), for the
    all-core CPU baseline; same arithmetic and result as survivors()."""
    a = _pts(xy)
    n = a.shape[0]
    out = np.zeros(max(n, 1), dtype=np.uint32)
    c = _load().oracle_survivors_omp(a.ctypes.data, n, out.ctypes.data, None, int(threads))
    if c == -2:
        raise NonFiniteInput("non-finite coordinate")
    if c < 0:
        raise MemoryError("oracle allocation failed")
    return out[:c].copy()


def extremes16(xy) -> np.ndarray:
    """Indices V0..V15 of the 16-direction filter (Sec. 2; directions at
    22.5-degree steps counter-clockwise from +x, first index on ties);
    V[2j] is octagon vertex E_j."""
    a = _pts(xy)
    if a.shape[0] == 0:
        raise ValueError("empty point set has no extremes")
    if not validate(a):
        raise NonFiniteInput("non-finite coordinate")
    out = np.zeros(16, dtype=np.uint32)
    _load().oracle_extremes16(a.ctypes.data, a.shape[0], out.ctypes.data)
    return out


def key16_values(xy, k: int) -> np.ndarray:
    """float32 key of direction k (k * 22.5 degrees) of every point."""
    a = _pts(xy)
    out = np.zeros(a.shape[0], dtype=np.float32)
    if a.shape[0]:
        _load().oracle_key16_values(a.ctypes.data, a.shape[0], int(k), out.ctypes.data)
    return out


def keep_poly(xy, idx) -> np.ndarray:
    """uint8 flags, 1 = survives the polygon with vertex indices idx (in
    order, any length >= 1) under the binary64 rule of keep()."""
    a = _pts(xy)
    n = a.shape[0]
    idx = np.ascontiguousarray(idx, dtype=np.uint32)
    out = np.zeros(n, dtype=np.uint8)
    if n:
        _load().oracle_keep_poly(a.ctypes.data, n, idx.ctypes.data, int(idx.size), out.ctypes.data)
    return out


def survivors16(xy) -> np.ndarray:
    """Ascending indices of the points that survive the 16-direction filter."""
    a = _pts(xy)
    n = a.shape[0]
    out = np.zeros(max(n, 1), dtype=np.uint32)
    c = _load().oracle_survivors16(a.ctypes.data, n, out.ctypes.data, None)
    if c == -2:
        raise NonFiniteInput("non-finite coordinate")
    if c < 0:
        raise MemoryError("oracle allocation failed")
    return out[:c].copy()


def hull(xy, subset=None) -> np.ndarray:
    """Counter-clockwise hull vertex indices of xy (or of xy[subset])."""
    a = _pts(xy)
    n = a.shape[0]
    if not validate(a):
        raise NonFiniteInput("non-finite coordinate")
    if subset is None:
        m, sp = n, None
    else:
        sub = np.ascontiguousarray(subset, dtype=np.uint32)
        m, sp = sub.shape[0], sub.ctypes.data
    out = np.zeros(max(m, 1), dtype=np.uint32)
    h = _load().oracle_hull(a.ctypes.data, n, sp, m, out.ctypes.data)
    return out[:h].copy()


def convex_hull(xy) -> np.ndarray:
    """Algorithm 1 end to end: filter, compact, then the hull of the
    survivors."""
    a = _pts(xy)
    if a.shape[0] == 0:
        return np.zeros(0, dtype=np.uint32)
    return hull(a, survivors(a))


def orient_exact(o, a, b) -> int:
    """Exact sign of (a-o) x (b-o) for FP32 points."""
    f = np.float32
    return _load().oracle_orient_exact(f(o[0]), f(o[1]), f(a[0]), f(a[1]), f(b[0]), f(b[1]))
