"""Plant plausible mistakes in a copy of the oracle (on the CPU) and check
that the pins catch every one of them.

Each mutant is oracle.c with one textual change (a dropped term, a flipped
sign or comparison, a transposed operand, a wrong index, a wrong tie rule),
compiled to a temporary library and swapped into the oracle module.  The
pins are a fast subset of tests/test_oracle.py."""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np
import pytest

import oracle
from oracle import brute
from tests import cases
from paper_2303_10581_amd import workloads

MUTANTS = {
    "tie_last_occurrence": ("if (x > xy[2 * right]) right = i;", "if (x >= xy[2 * right]) right = i;"),
    "corner_key_sign": ("if (i == 0 || d > best_br) { best_br = d; br = i; }",
                        "if (i == 0 || -d > best_br) { best_br = -d; br = i; }"),
    "vertex_order_swapped": ("idx[1] = (uint32_t)tr;\n    idx[2] = (uint32_t)top;",
                             "idx[1] = (uint32_t)top;\n    idx[2] = (uint32_t)tr;"),
    "dropped_term": ("volatile double det = l - r;", "volatile double det = l;"),
    "transposed_operand": ("volatile double qx = px - ax;", "volatile double qx = ax - px;"),
    "not_conservative": ("return det > bnd;", "return det > -bnd;"),
    "boundary_discarded": ("return det > bnd;", "return det >= 0.0;"),
    "wrong_edge_index": ("int k = (j + 1) % 8;", "int k = (j + 2) % 8;"),
    "degenerate_edges_kept": ("if (x0 == x1 && y0 == y1)\n            continue;", ""),
    "flags_inverted": ("keep[i] = inside_all ? 0 : 1;", "keep[i] = inside_all ? 1 : 0;"),
    "hull_keeps_collinear": ("p[k].x, p[k].y) <= 0)\n            --t;", "p[k].x, p[k].y) < 0)\n            --t;"),
    "dedupe_highest_index": ("return (a->i > b->i) - (a->i < b->i);", "return (a->i < b->i) - (a->i > b->i);"),
    "bigint_borrow": ("br = s < 0;", "br = 0;"),
    "bigint_product_sign": ("out.neg = (a->neg != b->neg) && !big_is_zero(&out);", "out.neg = a->neg && !big_is_zero(&out);"),
}


# the 16-direction filter (Sec. 2)
MUTANTS16 = {
    "tan_off_by_one_ulp": ("#define TAN_22_5_F32 0x1.a8279ap-2f", "#define TAN_22_5_F32 0x1.a8279cp-2f"),
    "fma_split_in_two_roundings": ("case 1: return fmaf(T, y, x);", "case 1: return x + T * y;"),
    "odd_vertices_swapped": ("case 3: return fmaf(T, x, y);          /* 67.5: (T, 1)            */\n"
                             "    case 4: return y;",
                             "case 3: return y;\n    case 4: return fmaf(T, x, y);"),
    "min_taken_as_max": ("case 11: return -fmaf(T, x, y);", "case 11: return fmaf(T, x, y);"),
    "rotation_sign": ("case 5: return fmaf(-T, x, y);", "case 5: return fmaf(T, x, -y);"),
    "poly_edge_skips_a_vertex": ("int j1 = (j + 1) % k;", "int j1 = (j + 2) % k;"),
    "poly_last_edge_dropped": ("    for (int j = 0; j < k; ++j) {\n        float x0",
                               "    for (int j = 0; j < k - 1; ++j) {\n        float x0"),
    "tie_last_occurrence16": ("if (v > best) { best = v; best_i = i; }", "if (v >= best) { best = v; best_i = i; }"),
}


def _build_mutant(tmp_path, name, old, new):
    src = open(os.path.join(os.path.dirname(oracle.__file__), "oracle.c")).read()
    assert old in src, f"mutation anchor for {name} not found"
    mut = src.replace(old, new, 1)
    c = tmp_path / f"{name}.c"
    so = tmp_path / f"{name}.so"
    c.write_text(mut)
    subprocess.check_call(["gcc", "-O2", "-std=c99", "-ffp-contract=off", "-fopenmp", "-shared", "-fPIC",
                           "-o", str(so), str(c), "-lm"])
    return str(so)


def _pins_pass() -> bool:
    """Fast subset of the oracle pins; False as soon as one fails."""
    try:
        for _, xy, case in cases.golden_cases():
            if oracle.extremes(xy).tolist() != case["extremes"]:
                return False
            if oracle.survivors(xy).tolist() != case["survivors"]:
                return False
            if "hull" in case and oracle.hull(xy).tolist() != case["hull"]:
                return False
        for seed in range(25):
            xy = cases.small_integer_grid(40, [2, 10, 1000][seed % 3], seed)
            idx = oracle.extremes(xy)
            if idx.tolist() != brute.extremes_manhattan(xy):
                return False
            exact = [0 if brute.strictly_inside_exact(xy, idx, i) else 1 for i in range(len(xy))]
            if oracle.keep(xy, idx).tolist() != exact:
                return False
            if oracle.hull(xy).tolist() != brute.hull_brute(xy):
                return False
        base = workloads.displaced(200, 3)
        xy = cases.with_near_edge_points(base, oracle.extremes, per_edge=30, seed=1)
        idx = oracle.extremes(xy)
        k = oracle.keep(xy, idx)
        E = brute.octagon_edges(xy, idx)
        for i in np.flatnonzero(k == 0):
            p = (brute.exact_int(xy[i, 0]), brute.exact_int(xy[i, 1]))
            if not all(brute.det_exact(a, b, p) > 0 for a, b in E):
                return False
        rng = np.random.default_rng(0)
        for _ in range(300):
            v = rng.uniform(-1, 1, 6).astype(np.float32) * np.float32(rng.choice([1e-30, 1.0, 1e30]))
            o, a, b = v[0:2], v[2:4], v[4:6]
            if oracle.orient_exact(o, a, b) != brute.orient(o, a, b):
                return False
        for _ in range(300):
            # nearly collinear: the exact fallback must resolve the sign
            o = rng.uniform(-1, 1, 2).astype(np.float32)
            d = rng.uniform(-1, 1, 2)
            a = (o + d * rng.uniform(0.1, 2)).astype(np.float32)
            b = cases.ulp_nudge((o + d * rng.uniform(0.1, 2)).astype(np.float32),
                                rng.integers(-1, 2, 2))
            if oracle.orient_exact(o, a, b) != brute.orient(o, a, b):
                return False
        return True
    except (AssertionError, RuntimeError, KeyError, IndexError):
        return False


def _pins16_pass() -> bool:
    """Fast subset of the 16-direction pins (tests/test_oracle16.py)."""
    try:
        rng = np.random.default_rng(1)
        xy = np.concatenate([workloads.normal(120, 3),
                             rng.integers(-2**20, 2**20, (60, 2)).astype(np.float32)]).astype(np.float32)
        for k in range(16):
            want = np.array([brute.key16_exact(k, a, b) for a, b in xy], dtype=np.float32)
            if not np.array_equal(oracle.key16_values(xy, k), want):
                return False
        for seed in range(8):
            xy = cases.named_sets(150, seed)["normal"] if seed % 2 else cases.small_integer_grid(80, 3, seed)
            idx = oracle.extremes16(xy)
            if idx.tolist() != brute.extremes16_exact(xy):
                return False
        for seed in range(12):
            xy = cases.small_integer_grid(60, [2, 10, 1000][seed % 3], seed)
            idx = oracle.extremes16(xy)
            exact = [0 if brute.strictly_inside_poly_exact(xy, idx, i) else 1 for i in range(len(xy))]
            if oracle.keep_poly(xy, idx).tolist() != exact:
                return False
        base = workloads.displaced(300, 3)
        xy = cases.with_near_edge_points16(base, oracle.extremes16, per_edge=15, seed=1)
        idx = oracle.extremes16(xy)
        k = oracle.keep_poly(xy, idx)
        E = brute.poly_edges(xy, idx)
        for i in np.flatnonzero(k == 0):
            p = (brute.exact_int(xy[i, 0]), brute.exact_int(xy[i, 1]))
            if not all(brute.det_exact(a, b, p) > 0 for a, b in E):
                return False
        n = 200_000
        h = set(oracle.hull(workloads.displaced(n, 4)).tolist())
        if not h <= set(oracle.survivors16(workloads.displaced(n, 4)).tolist()):
            return False
        return True
    except (AssertionError, RuntimeError, KeyError, IndexError):
        return False


def test_unmutated_oracle_passes_the_pins():
    oracle.build()
    assert _pins_pass()
    assert _pins16_pass()


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_pins_catch_mutant(tmp_path, monkeypatch, name):
    old, new = MUTANTS[name]
    so = _build_mutant(tmp_path, name, old, new)
    oracle.build()
    real = oracle._load()
    lib = ctypes.CDLL(so)
    _wire(lib, real)
    monkeypatch.setattr(oracle, "_lib", lib)
    assert not _pins_pass(), f"mutant {name} survived the pins"


_FUNCS = ("oracle_validate", "oracle_extremes", "oracle_keep", "oracle_survivors", "oracle_hull",
          "oracle_orient_exact", "oracle_extremes16", "oracle_keep_poly", "oracle_survivors16",
          "oracle_key16_values")


def _wire(lib, real):
    for fn in _FUNCS:
        getattr(lib, fn).argtypes = getattr(real, fn).argtypes
        getattr(lib, fn).restype = getattr(real, fn).restype


@pytest.mark.parametrize("name", sorted(MUTANTS16))
def test_pins16_catch_mutant(tmp_path, monkeypatch, name):
    old, new = MUTANTS16[name]
    so = _build_mutant(tmp_path, name, old, new)
    oracle.build()
    real = oracle._load()
    lib = ctypes.CDLL(so)
    _wire(lib, real)
    monkeypatch.setattr(oracle, "_lib", lib)
    assert not _pins16_pass(), f"mutant {name} survived the pins"
