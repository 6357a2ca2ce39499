"""Python binding of libhullf.so (C ABI in include/hullf.h).

Argument marshalling only: every step of the path runs in the library's HIP
kernels (and, for convex_hull, its host monotone chain).  PyTorch provides
device memory and streams.  There is no fallback: if the library is missing,
every call raises.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libhullf.so")

OK, EINVAL, ENONFINITE, ECAPACITY, ENOMEM, EDEVICE, EAGAIN = range(7)
COUNT_NONFINITE = (1 << 64) - 1
COUNT_BAD_OFFSETS = (1 << 64) - 2

_lib = None


class HullfError(RuntimeError):
    def __init__(self, status: int, what: str):
        self.status = status
        super().__init__(f"{what}: {_load().hullf_status_str(status).decode()} (status {status})")


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with `python -m paper_2303_10581_amd.build`")
    lib = ctypes.CDLL(LIB_PATH)
    P, U64, U32, I = ctypes.c_void_p, ctypes.c_uint64, ctypes.c_uint32, ctypes.c_int
    st = ctypes.c_int
    sig = {
        "hullf_create": ([I, ctypes.c_size_t, ctypes.POINTER(P)], st),
        "hullf_workspace": ([P, ctypes.POINTER(U64), ctypes.POINTER(U64)], st),
        "hullf_destroy": ([P], None),
        "hullf_status_str": ([st], ctypes.c_char_p),
        "hullf_octagon": ([P, P, U64, P, P], st),
        "hull_filter": ([P, P, U64, P, U64, P, P], st),
        "hull_filter_noalloc": ([P, U64, P, U64, P, P], st),
        "hullf_polygon16": ([P, P, U64, P, P], st),
        "hull_filter16": ([P, P, U64, P, U64, P, P], st),
        "convex_hull": ([P, P, U64, P, U64, P, P], st),
        "hullf_flags": ([P, P, U64, P, P], st),
        "hull_from_survivors": ([P, P, U64, P, U64, P, U64, P, P], st),
        "hull_from_survivors_batched": ([P, P, P, U32, U64, P, P, P, U64, P, P], st),
        "hull_filter_batched": ([P, P, P, U32, U64, P, P, P], st),
        "hull_filter_segments": ([P, P, P, U32, U64, P, P, P], st),
        "hull_filter_batched_shape": ([P, P, P, U32, U64, P, P, I, I, P], st),
        "hullf_autotune_batched": ([P, P, P, U32, U64, P, P, I, P, P, P, P], st),
        "hullf_timing_enable": ([P, I], st),
        "hullf_skip_stats": ([P, ctypes.POINTER(U64), ctypes.POINTER(U64)], st),
        "hullf_timing_read": ([P, P, P], st),
        "hullf_server_create": ([I, P, ctypes.POINTER(P)], st),
        "hullf_server_destroy": ([P], None),
        "hullf_server_submit": ([P, P, U64, ctypes.POINTER(U64)], st),
        "hullf_server_wait": ([P, U64, I, P, U64, ctypes.POINTER(U64), P], st),
        "hullf_server_stats": ([P, P], st),
    }
    for name, (args, res) in sig.items():
        fn = getattr(lib, name)
        fn.argtypes = args
        fn.restype = res
    _lib = lib
    return lib


def _check(status: int, what: str):
    if status != OK:
        raise HullfError(status, what)


def _torch():
    import torch
    return torch


def _stream(stream):
    torch = _torch()
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


def _points(pts):
    torch = _torch()
    if not isinstance(pts, torch.Tensor) or not pts.is_cuda:
        raise TypeError("points must be a CUDA tensor")
    if pts.dtype != torch.float32 or pts.dim() != 2 or pts.shape[1] != 2 or not pts.is_contiguous():
        raise TypeError("points must be a contiguous float32 tensor of shape (n, 2)")
    return pts


class Context:
    """Owns a hullf context (scratch memory, tuned shapes, graph cache)."""

    def __init__(self, device: int = 0, workspace_bytes: int = 0):
        lib = _load()
        h = ctypes.c_void_p()
        _check(lib.hullf_create(int(device), int(workspace_bytes), ctypes.byref(h)), "hullf_create")
        self.handle = h
        self.device = int(device)

    def workspace(self):
        """(device bytes held now, cap in bytes or 0)."""
        u, c = ctypes.c_uint64(0), ctypes.c_uint64(0)
        _check(_load().hullf_workspace(self.handle, ctypes.byref(u), ctypes.byref(c)), "hullf_workspace")
        return u.value, c.value

    def close(self):
        if self.handle:
            _load().hullf_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -- steps ---------------------------------------------------------------
    def octagon(self, pts, stream=None) -> np.ndarray:
        """Indices E0..E7 of the octagon vertices (synchronous)."""
        pts = _points(pts)
        out = np.zeros(8, dtype=np.uint32)
        _check(_load().hullf_octagon(self.handle, pts.data_ptr(), pts.shape[0], out.ctypes.data,
                                     _stream(stream)), "hullf_octagon")
        return out

    def hull_filter(self, pts, surv=None, count=None, cap=None, stream=None):
        """Enqueue the filter; returns (surv uint32[cap], count uint64[1]) device tensors."""
        torch = _torch()
        pts = _points(pts)
        n = pts.shape[0]
        if surv is None:
            surv = torch.empty(max(n, 1), dtype=torch.int32, device=pts.device)
        if count is None:
            count = torch.empty(1, dtype=torch.int64, device=pts.device)
        if cap is None:
            cap = surv.numel()
        _check(_load().hull_filter(self.handle, pts.data_ptr(), n, surv.data_ptr(), int(cap),
                                   count.data_ptr(), _stream(stream)), "hull_filter")
        return surv, count

    def polygon16(self, pts, stream=None) -> np.ndarray:
        """Indices V0..V15 of the 16-direction filter's polygon (synchronous)."""
        pts = _points(pts)
        out = np.zeros(16, dtype=np.uint32)
        _check(_load().hullf_polygon16(self.handle, pts.data_ptr(), pts.shape[0], out.ctypes.data,
                                       _stream(stream)), "hullf_polygon16")
        return out

    def hull_filter16(self, pts, surv=None, count=None, cap=None, stream=None):
        """Enqueue the 16-direction filter; returns (surv, count) like hull_filter."""
        torch = _torch()
        pts = _points(pts)
        n = pts.shape[0]
        if surv is None:
            surv = torch.empty(max(n, 1), dtype=torch.int32, device=pts.device)
        if count is None:
            count = torch.empty(1, dtype=torch.int64, device=pts.device)
        if cap is None:
            cap = surv.numel()
        _check(_load().hull_filter16(self.handle, pts.data_ptr(), n, surv.data_ptr(), int(cap),
                                     count.data_ptr(), _stream(stream)), "hull_filter16")
        return surv, count

    def survivors16(self, pts, stream=None):
        """Ascending survivors of the 16-direction filter (synchronises)."""
        surv, count = self.hull_filter16(pts, stream=stream)
        c = int(count.item()) & ((1 << 64) - 1)
        if c == COUNT_NONFINITE:
            raise HullfError(ENONFINITE, "hull_filter16")
        return surv[:c]

    def survivors(self, pts, stream=None):
        """Ascending survivor indices as an int32 device tensor (synchronises)."""
        surv, count = self.hull_filter(pts, stream=stream)
        c = int(count.item()) & ((1 << 64) - 1)
        if c == COUNT_NONFINITE:
            raise HullfError(ENONFINITE, "hull_filter")
        return surv[:c]

    def flags(self, pts, stream=None):
        """One byte per point: 1 survives, 0 discarded, 2 non-finite input."""
        torch = _torch()
        pts = _points(pts)
        out = torch.empty(pts.shape[0], dtype=torch.uint8, device=pts.device)
        _check(_load().hullf_flags(self.handle, pts.data_ptr(), pts.shape[0], out.data_ptr(),
                                   _stream(stream)), "hullf_flags")
        return out

    def convex_hull(self, pts, stream=None) -> np.ndarray:
        """Counter-clockwise hull vertex indices (synchronous)."""
        pts = _points(pts)
        n = pts.shape[0]
        cap = max(n, 1)
        out = np.zeros(cap, dtype=np.uint32)
        h = ctypes.c_uint64(0)
        _check(_load().convex_hull(self.handle, pts.data_ptr(), n, out.ctypes.data, cap,
                                   ctypes.byref(h), _stream(stream)), "convex_hull")
        return out[:h.value].copy()

    def hull_from_survivors(self, pts, surv, m=None, stream=None) -> np.ndarray:
        """Counter-clockwise hull (indices into pts) of the points listed by
        the ascending int32 device tensor surv (first m entries)."""
        pts = _points(pts)
        if m is None:
            m = surv.numel()
        cap = max(int(m), 1)
        out = np.zeros(cap, dtype=np.uint32)
        h = ctypes.c_uint64(0)
        _check(_load().hull_from_survivors(self.handle, pts.data_ptr(), pts.shape[0], surv.data_ptr(), int(m),
                                           out.ctypes.data, cap, ctypes.byref(h), _stream(stream)),
               "hull_from_survivors")
        return out[:h.value].copy()

    def hulls_batched(self, pts, off, surv, counts, n_total=None, stream=None):
        """Hulls of every set of a batch from hull_filter_batched's survivors
        (device tensors: pts (n_total, 2) float32, off S+1 int64, surv
        n_total int32, counts S int64), all sets finished together.  Returns
        (hulls, offsets): set s's counter-clockwise hull, set-local indices,
        is hulls[offsets[s]:offsets[s+1]]."""
        pts = _points(pts)
        S = off.numel() - 1
        if n_total is None:
            n_total = pts.shape[0]
        hoff = np.zeros(S + 1, dtype=np.uint64)
        cap = max(int(n_total), 1)
        out = np.zeros(cap, dtype=np.uint32)
        _check(_load().hull_from_survivors_batched(self.handle, pts.data_ptr(), off.data_ptr(), S, int(n_total),
                                                   surv.data_ptr(), counts.data_ptr(), out.ctypes.data, cap,
                                                   hoff.ctypes.data, _stream(stream)),
               "hull_from_survivors_batched")
        return out[:int(hoff[S])].copy(), hoff.astype(np.int64)

    # -- batched -------------------------------------------------------------
    def hull_filter_batched(self, pts, off, n_total=None, surv=None, counts=None, stream=None,
                            block=None, ppt=None):
        """Enqueue the batched filter.  off: uint64/int64 device tensor (S+1).
        Returns (surv int32[n_total], counts int64[S]); survivors of set s are
        set-local indices at surv[off[s]:off[s]+counts[s]].  With block/ppt
        given, launches that shape directly instead of the cached graph."""
        torch = _torch()
        pts = _points(pts)
        S = off.numel() - 1
        if n_total is None:
            n_total = pts.shape[0]
        if surv is None:
            surv = torch.empty(max(n_total, 1), dtype=torch.int32, device=pts.device)
        if counts is None:
            counts = torch.empty(max(S, 1), dtype=torch.int64, device=pts.device)
        lib = _load()
        if block is None and ppt is None:
            st = lib.hull_filter_batched(self.handle, pts.data_ptr(), off.data_ptr(), S, int(n_total),
                                         surv.data_ptr(), counts.data_ptr(), _stream(stream))
        else:
            st = lib.hull_filter_batched_shape(self.handle, pts.data_ptr(), off.data_ptr(), S,
                                               int(n_total), surv.data_ptr(), counts.data_ptr(),
                                               int(block or 0), int(ppt or 0), _stream(stream))
        _check(st, "hull_filter_batched")
        return surv, counts

    def hull_filter_segments(self, pts, seg, n_total=None, surv=None, counts=None, stream=None):
        """Enqueue the batched filter over sets at arbitrary places.
        seg: uint64/int64 device tensor (S, 2) of (begin, count), ascending
        and disjoint.  Returns (surv int32[n_total], counts int64[S]);
        survivors of set s are set-local indices at surv[begin:begin+counts[s]]."""
        torch = _torch()
        pts = _points(pts)
        if seg.dim() != 2 or seg.shape[1] != 2 or not seg.is_contiguous():
            raise TypeError("seg must be a contiguous (S, 2) tensor")
        S = seg.shape[0]
        if n_total is None:
            n_total = pts.shape[0]
        if surv is None:
            surv = torch.empty(max(n_total, 1), dtype=torch.int32, device=pts.device)
        if counts is None:
            counts = torch.empty(max(S, 1), dtype=torch.int64, device=pts.device)
        _check(_load().hull_filter_segments(self.handle, pts.data_ptr(), seg.data_ptr(), S, int(n_total),
                                            surv.data_ptr(), counts.data_ptr(), _stream(stream)),
               "hull_filter_segments")
        return surv, counts

    def autotune_batched(self, pts, off, surv, counts, reps: int = 3, stream=None):
        """Pick the fastest (block, ppt) for the batched kernel; returns
        (block, ppt, ms)."""
        pts = _points(pts)
        S = off.numel() - 1
        b, p, ms = ctypes.c_int(0), ctypes.c_int(0), ctypes.c_float(0)
        _check(_load().hullf_autotune_batched(self.handle, pts.data_ptr(), off.data_ptr(), S,
                                              pts.shape[0], surv.data_ptr(), counts.data_ptr(), reps,
                                              ctypes.byref(b), ctypes.byref(p), ctypes.byref(ms),
                                              _stream(stream)), "hullf_autotune_batched")
        return b.value, p.value, ms.value

    # -- timing --------------------------------------------------------------
    _TIMING_KINDS = ("reduce", "filter", "batched", "setup", "compact")

    def timing(self, enable: bool, kinds=None):
        """Per-kernel HIP-event timing on or off; `kinds` (names as in
        timing_read) limits it to those kernels, the others run without
        events."""
        mask = 0
        if enable:
            sel = self._TIMING_KINDS if kinds is None else kinds
            for k in sel:
                mask |= 1 << self._TIMING_KINDS.index(k)
        _check(_load().hullf_timing_enable(self.handle, mask), "hullf_timing_enable")

    def skip_stats(self):
        """(groups read, groups without the region skip) of 128 points by the
        inside test since the previous call (synchronous; resets)."""
        r, t = ctypes.c_uint64(0), ctypes.c_uint64(0)
        _check(_load().hullf_skip_stats(self.handle, ctypes.byref(r), ctypes.byref(t)), "hullf_skip_stats")
        return r.value, t.value

    def timing_read(self):
        """{kind: (launches, total_ms)} for kinds reduce, filter (inside
        test), batched, setup, compact."""
        kinds = ("reduce", "filter", "batched", "setup", "compact")
        launches = (ctypes.c_uint64 * len(kinds))()
        ms = (ctypes.c_double * len(kinds))()
        _check(_load().hullf_timing_read(self.handle, launches, ms), "hullf_timing_read")
        return {k: (launches[i], ms[i]) for i, k in enumerate(kinds)}


class _ServerConfig(ctypes.Structure):
    _fields_ = [("arena_points", ctypes.c_uint64), ("max_inflight", ctypes.c_uint32),
                ("finish_threads", ctypes.c_uint32), ("reserved", ctypes.c_uint32 * 2)]


class _RequestInfo(ctypes.Structure):
    _fields_ = [("admitted_us", ctypes.c_double), ("resident_us", ctypes.c_double),
                ("launched_us", ctypes.c_double), ("filtered_us", ctypes.c_double),
                ("done_us", ctypes.c_double), ("n", ctypes.c_uint64), ("survivors", ctypes.c_uint64),
                ("hull", ctypes.c_uint64), ("batch", ctypes.c_uint64), ("batch_requests", ctypes.c_uint32),
                ("status", ctypes.c_uint32)]


class _ServerStats(ctypes.Structure):
    _fields_ = [("submitted", ctypes.c_uint64), ("completed", ctypes.c_uint64),
                ("batches", ctypes.c_uint64), ("batched_requests", ctypes.c_uint64),
                ("arena_points", ctypes.c_uint64), ("arena_peak_points", ctypes.c_uint64),
                ("inflight", ctypes.c_uint32), ("queued", ctypes.c_uint32), ("batch_ms", ctypes.c_double)]


def _fields(obj):
    return {name: getattr(obj, name) for name, _ in obj._fields_ if name != "reserved"}


def _host_points(pts):
    """(pointer, n, keep-alive object) of a host (n, 2) float32 array."""
    try:
        import torch
        if isinstance(pts, torch.Tensor):
            if pts.is_cuda or pts.dtype != torch.float32 or pts.dim() != 2 or pts.shape[1] != 2 \
                    or not pts.is_contiguous():
                raise TypeError("points must be a contiguous host float32 tensor of shape (n, 2)")
            return pts.data_ptr(), pts.shape[0], pts
    except ImportError:
        pass
    a = np.ascontiguousarray(pts, dtype=np.float32)
    if a.ndim != 2 or a.shape[1] != 2:
        raise TypeError("points must have shape (n, 2)")
    return a.ctypes.data, a.shape[0], a


class Server:
    """Request loop with continuous batching (include/hullf_server.h).

    submit() returns an id at once; the server keeps a reference to the
    points until wait() has returned that request's result."""

    def __init__(self, device: int = 0, arena_points: int = 0, max_inflight: int = 0,
                 finish_threads: int = 0):
        lib = _load()
        cfg = _ServerConfig(arena_points, max_inflight, finish_threads)
        h = ctypes.c_void_p()
        _check(lib.hullf_server_create(int(device), ctypes.byref(cfg), ctypes.byref(h)),
               "hullf_server_create")
        self.handle = h
        self._keep = {}

    def close(self):
        if self.handle:
            _load().hullf_server_destroy(self.handle)
            self.handle = None
            self._keep.clear()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def submit(self, pts) -> int:
        ptr, n, keep = _host_points(pts)
        rid = ctypes.c_uint64(0)
        _check(_load().hullf_server_submit(self.handle, ptr, n, ctypes.byref(rid)), "hullf_server_submit")
        self._keep[rid.value] = keep
        return rid.value

    def wait(self, rid: int, timeout_ms: int = -1):
        """(hull uint32 array, info dict) of a finished request; None if it
        has not finished within timeout_ms.  Raises HullfError for a failed
        request."""
        lib = _load()
        keep = self._keep.get(rid)
        cap = 64 if keep is None else max(len(keep), 1)
        info = _RequestInfo()
        for _ in range(2):
            out = np.zeros(cap, dtype=np.uint32)
            h = ctypes.c_uint64(0)
            st = lib.hullf_server_wait(self.handle, int(rid), int(timeout_ms), out.ctypes.data, cap,
                                       ctypes.byref(h), ctypes.byref(info))
            if st == EAGAIN:
                return None
            if st == ECAPACITY:
                cap = int(h.value)
                continue
            self._keep.pop(rid, None)
            _check(st, "hullf_server_wait")
            return out[:h.value].copy(), _fields(info)
        raise HullfError(ECAPACITY, "hullf_server_wait")

    def stats(self) -> dict:
        s = _ServerStats()
        _check(_load().hullf_server_stats(self.handle, ctypes.byref(s)), "hullf_server_stats")
        return _fields(s)


NOALLOC_MAX_POINTS = 1 << 25


def hull_filter_noalloc(pts, surv=None, count=None, cap=None, stream=None):
    """hull_filter without a context and without device allocation inside the
    library (scratch in a fixed device array).  Enqueues on the current
    device; returns (surv int32[cap], count int64[1]) device tensors."""
    torch = _torch()
    pts = _points(pts)
    n = pts.shape[0]
    if surv is None:
        surv = torch.empty(max(n, 1), dtype=torch.int32, device=pts.device)
    if count is None:
        count = torch.empty(1, dtype=torch.int64, device=pts.device)
    if cap is None:
        cap = surv.numel()
    _check(_load().hull_filter_noalloc(pts.data_ptr(), n, surv.data_ptr(), int(cap), count.data_ptr(),
                                       _stream(stream)), "hull_filter_noalloc")
    return surv, count


def exported_symbols():
    """Names of the C-ABI functions the binding expects."""
    return ["hullf_create", "hullf_destroy", "hullf_workspace", "hullf_status_str", "hullf_octagon", "hull_filter",
            "hull_filter_noalloc", "hullf_polygon16", "hull_filter16", "convex_hull", "hullf_flags",
            "hull_from_survivors", "hull_from_survivors_batched", "hull_filter_batched", "hull_filter_segments",
            "hull_filter_batched_shape", "hullf_autotune_batched", "hullf_timing_enable",
            "hullf_timing_read", "hullf_skip_stats", "hullf_server_create", "hullf_server_destroy", "hullf_server_submit",
            "hullf_server_wait", "hullf_server_stats"]
