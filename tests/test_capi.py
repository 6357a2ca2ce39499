"""CPU checks of the C-ABI library: it loads without a GPU and exports every
function include/hullf.h declares; no compute call is made here."""
from __future__ import annotations

import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADERS = [os.path.join(ROOT, "include", h) for h in sorted(os.listdir(os.path.join(ROOT, "include")))
           if h.endswith(".h")]


def declared_functions():
    names = set()
    for h in HEADERS:
        src = re.sub(r"/\*.*?\*/", "", open(h).read(), flags=re.S)
        names |= set(re.findall(r"^(?:hullf_status|void|const char \*)\s*\**\s*(\w+)\s*\(", src, flags=re.M))
    return sorted(names)


@pytest.fixture(scope="module")
def lib():
    from paper_2303_10581_amd import hullf
    if not os.path.exists(hullf.LIB_PATH):
        from paper_2303_10581_amd import build
        build.build()
    return hullf._load()


def test_header_declares_the_boundary():
    names = declared_functions()
    for required in ("hull_filter", "convex_hull", "hullf_octagon", "hull_filter_batched",
                     "hull_filter_segments", "hullf_create", "hullf_destroy", "hullf_status_str",
                     "hullf_server_create", "hullf_server_submit", "hullf_server_wait"):
        assert required in names


def test_library_exports_every_declared_function(lib):
    for name in declared_functions():
        assert hasattr(lib, name), name


def test_binding_covers_the_header():
    from paper_2303_10581_amd import hullf
    assert sorted(hullf.exported_symbols()) == declared_functions()


def test_status_strings(lib):
    for s in range(7):
        assert lib.hullf_status_str(s)
    assert b"ok" == lib.hullf_status_str(0)


def test_create_without_gpu_fails_cleanly(lib):
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    h = ctypes.c_void_p()
    assert lib.hullf_create(0, 0, ctypes.byref(h)) != 0
    assert not h.value


def test_server_create_without_gpu_fails_cleanly(lib):
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    h = ctypes.c_void_p()
    assert lib.hullf_server_create(0, None, ctypes.byref(h)) != 0
    assert not h.value


def test_binding_refuses_without_library(monkeypatch, tmp_path):
    from paper_2303_10581_amd import hullf
    monkeypatch.setattr(hullf, "_lib", None)
    monkeypatch.setattr(hullf, "LIB_PATH", str(tmp_path / "missing.so"))
    with pytest.raises(RuntimeError):
        hullf._load()
