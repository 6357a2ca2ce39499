"""CPU checks of the gfx950 code the kernels compile to.

- No scalar-memory writes (stores, atomics, write-back or discard through
  the scalar data cache): every kernel writes through vector memory.
- No packed FP32 arithmetic (the build turns the feature off).
- No fused multiply-add in binary64: the inside test is defined operation
  by operation (a fused a*b+c would round once instead of twice).
"""
from __future__ import annotations

import os
import re
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2303_10581_amd", "csrc")
HIP_SOURCES = sorted(f for f in os.listdir(CSRC) if f.endswith(".hip"))


@pytest.fixture(scope="module")
def asm(tmp_path_factory):
    from paper_2303_10581_amd import build
    hipcc = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(hipcc):
        pytest.skip("hipcc not available")
    out = {}
    d = tmp_path_factory.mktemp("isa")
    for src in HIP_SOURCES:
        s = str(d / (src + ".s"))
        cmd = [hipcc, *build.COMMON, *build.HIP_FLAGS, "--cuda-device-only", "-S",
               os.path.join(CSRC, src), "-o", s]
        r = subprocess.run(cmd, capture_output=True, text=True)
        assert r.returncode == 0, r.stderr[-2000:]
        out[src] = open(s).read()
    return out


def _instructions(text):
    for line in text.splitlines():
        t = line.strip()
        if not t or t.startswith((";", ".", "//")) or t.endswith(":"):
            continue
        yield t.split()[0]


def test_no_scalar_memory_writes(asm):
    bad = re.compile(r"^s_(store|buffer_store|scratch_store|atomic|buffer_atomic|dcache_wb|dcache_discard)")
    for src, text in asm.items():
        found = sorted({op for op in _instructions(text) if bad.match(op)})
        assert not found, (src, found)


def test_no_packed_fp32(asm):
    for src, text in asm.items():
        found = sorted({op for op in _instructions(text) if re.match(r"^v_pk_(add|mul|fma|mov)_f32", op)})
        assert not found, (src, found)


def test_no_fp64_fma_in_the_filter(asm):
    text = asm["hullf_kernels.hip"]
    found = sorted({op for op in _instructions(text) if re.match(r"^v_fmac?_f64", op)})
    assert not found, found
