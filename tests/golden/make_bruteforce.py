"""Writes the oracle's brute-force pair counts of the parameter-study inputs.

CPU only: oracle.bruteforce (every pair within r, FP64 in the definition's
order) on the seeded uniform points of the paper's parameter study
(Sec. IV-A: the unit d-cube, radius of Eq. r_FMT* with eta = 0).  The count
is the ground truth of the success rate (reported pairs over true pairs):
RTG reports a subset of these pairs, so its success rate is its pair count
over this one.

Writes bruteforce_fmt_uniform.json next to this script.
Usage: python tests/golden/make_bruteforce.py   (about a minute per case)
"""
from __future__ import annotations

import hashlib
import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

# (n, d, point seed): the study's n = 102400, d = 9 set, and a smaller one
# the GPU tests run the chosen parameters on.
CASES = [(102400, 9, 9), (20000, 9, 10), (20000, 6, 11)]


def main() -> int:
    import oracle
    from paper_1409_8112_amd import workloads
    out = []
    for n, d, seed in CASES:
        r = workloads.fmt_radius(n, d)
        t0 = time.perf_counter()
        res = oracle.bruteforce(workloads.uniform_points(n, d, seed), r)
        up = res.upper_pairs()
        out.append({"n": n, "d": d, "point_seed": seed, "r": r, "pairs": int(len(up)),
                    "upper_pairs_sha256": hashlib.sha256(
                        np.ascontiguousarray(up, dtype="<i8").tobytes()).hexdigest()})
        print(n, d, len(up), f"{time.perf_counter() - t0:.1f} s", flush=True)
    path = os.path.join(HERE, "bruteforce_fmt_uniform.json")
    with open(path, "w") as fh:
        json.dump({"note": "oracle.bruteforce on workloads.uniform_points(n, d, point_seed) "
                           "with r = workloads.fmt_radius(n, d) (tests/golden/make_bruteforce.py)",
                   "cases": out}, fh, indent=1)
        fh.write("\n")
    print("wrote", path)
    return 0


if __name__ == "__main__":
    sys.exit(main())
