"""Writes the stored oracle results for the full-size workloads.

    python tests/golden/make_full_size.py [--only NAME ...]

Computing the oracle's hull of 1e8 circle points takes about a minute on one
host thread, and of the 5e8-point set several minutes, so the GPU parity
tests compare against values stored here instead of recomputing them.  This
script calls only the oracle (and the seeded input generators, which hold no
arithmetic of the method).  Every list is stored as the SHA-256 of its
little-endian uint32 bytes, with its length; the input points are hashed as
well, so a test can tell a changed generator from a wrong result.

Outputs:
  full_size.json  one record per single-set workload: the eight extreme
                  indices (Sec. 3.1), the survivor count and hash
                  (Sec. 3.2, 4.1.1), the hull length and hash (Sec. 3.3)
  batch_4096.txt  the 4096-set batch (seed 6): one line per set with the
                  set's survivor count, hull length, and 16-hex-digit
                  prefixes of the survivor and hull hashes
  full_size16.json  the 16-direction filter of the related work (Sec. 2)
                  on the same single-set workloads: its 16 vertex indices and
                  the survivor count and hash
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from paper_2303_10581_amd import workloads  # noqa: E402

FULL = os.path.join(HERE, "full_size.json")
FULL16 = os.path.join(HERE, "full_size16.json")
BATCH = os.path.join(HERE, "batch_4096.txt")

# (name, kind, n, seed): the single-set workloads of the study cases
SINGLE = [
    ("normal_1e8", "normal", 100_000_000, 2),
    ("circle_1e8", "circle", 100_000_000, 3),
    ("displaced_1e8", "displaced", 100_000_000, 4),
    ("circle_jitter_5e8", "circle_jitter", 500_000_000, 5),
]


def sha(a: np.ndarray) -> str:
    return hashlib.sha256(np.ascontiguousarray(a).tobytes()).hexdigest()


def single(name, kind, n, seed):
    t0 = time.time()
    xy = workloads.by_kind(kind, n, seed)
    rec = {"kind": kind, "n": n, "seed": seed, "points_sha256": sha(xy)}
    rec["extremes"] = [int(v) for v in oracle.extremes(xy)]
    surv = oracle.survivors(xy)
    rec["survivors"] = int(surv.size)
    rec["survivors_sha256"] = sha(surv.astype("<u4"))
    h = oracle.hull(xy, surv)
    rec["hull"] = int(h.size)
    rec["hull_sha256"] = sha(h.astype("<u4"))
    rec["hull_head"] = [int(v) for v in h[:8]]
    print(f"{name}: {rec['survivors']} survivors, {rec['hull']} hull vertices "
          f"({time.time() - t0:.0f} s)", flush=True)
    return rec


def single16(name, kind, n, seed):
    t0 = time.time()
    xy = workloads.by_kind(kind, n, seed)
    rec = {"kind": kind, "n": n, "seed": seed, "points_sha256": sha(xy)}
    rec["vertices"] = [int(v) for v in oracle.extremes16(xy)]
    surv = oracle.survivors16(xy)
    rec["survivors"] = int(surv.size)
    rec["survivors_sha256"] = sha(surv.astype("<u4"))
    print(f"{name} (16 directions): {rec['survivors']} survivors ({time.time() - t0:.0f} s)", flush=True)
    return rec


def batch_lines():
    pts, off, _ = workloads.batch(S=4096, seed=6)
    lines = [f"# sha256(points)={sha(pts)} S=4096 seed=6 n_total={pts.shape[0]}",
             "# set survivors hull survivors_sha16 hull_sha16"]
    for s in range(off.size - 1):
        a, b = int(off[s]), int(off[s + 1])
        xy = pts[a:b]
        surv = oracle.survivors(xy)
        h = oracle.hull(xy, surv)
        lines.append(f"{s} {surv.size} {h.size} {sha(surv.astype('<u4'))[:16]} {sha(h.astype('<u4'))[:16]}")
    return lines


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--only", nargs="*", default=None)
    ap.add_argument("--filter16", action="store_true", help="only the 16-direction records")
    args = ap.parse_args()
    want = set(args.only) if args.only else None
    data = {}
    if os.path.exists(FULL):
        with open(FULL) as f:
            data = json.load(f)
    data16 = {}
    if os.path.exists(FULL16):
        with open(FULL16) as f:
            data16 = json.load(f)
    for name, kind, n, seed in SINGLE:
        if want is None or name in want:
            if not args.filter16:
                data[name] = single(name, kind, n, seed)
                with open(FULL, "w") as f:
                    json.dump(data, f, indent=1, sort_keys=True)
            data16[name] = single16(name, kind, n, seed)
            with open(FULL16, "w") as f:
                json.dump(data16, f, indent=1, sort_keys=True)
    if args.filter16:
        return
    if want is None or "batch_4096" in want:
        t0 = time.time()
        lines = batch_lines()
        with open(BATCH, "w") as f:
            f.write("\n".join(lines) + "\n")
        print(f"batch_4096: {len(lines) - 2} sets ({time.time() - t0:.0f} s)", flush=True)


if __name__ == "__main__":
    main()
