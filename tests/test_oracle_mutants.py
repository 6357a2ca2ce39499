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


def _build_mutant(tmp_path, name, old, new):
    src = open(os.path.join(os.path.dirname(oracle.__file__), "oracle.c")).read()
    assert old in src, f"mutation anchor for {name} not found"
    mut = src.replace(old, new, 1)
    c = tmp_path / f"{name}.c"
    so = tmp_path / f"{name}.so"
    c.write_text(mut)
    subprocess.check_call(["gcc", "-O2", "-std=c99", "-ffp-contract=off", "-shared", "-fPIC",
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


def test_unmutated_oracle_passes_the_pins():
    oracle.build()
    assert _pins_pass()


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_pins_catch_mutant(tmp_path, monkeypatch, name):
    old, new = MUTANTS[name]
    so = _build_mutant(tmp_path, name, old, new)
    oracle.build()
    real = oracle._load()
    lib = ctypes.CDLL(so)
    for fn in ("oracle_validate", "oracle_extremes", "oracle_keep", "oracle_survivors",
               "oracle_hull", "oracle_orient_exact"):
        getattr(lib, fn).argtypes = getattr(real, fn).argtypes
        getattr(lib, fn).restype = getattr(real, fn).restype
    monkeypatch.setattr(oracle, "_lib", lib)
    assert not _pins_pass(), f"mutant {name} survived the pins"
