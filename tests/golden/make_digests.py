"""Writes the oracle's digests of the benchmark-size workloads.

CPU only: every expected value here comes from the oracle (``oracle/``) run
on the seeded inputs of ``paper_1409_8112_amd/workloads.py``; nothing is
read from the GPU library.  Each result is reduced to its sizes and the
SHA-256 of its two arrays (row_ptr as little-endian int64, col as
little-endian int32), so the GPU tests can compare whole outputs of
multi-million-point instances without running the oracle on the GPU host.

Files written next to this script:
  digest_clustered_d12.json  the clustered n = 4e6, d = 12, k = 8 instance
  digest_batched_4096.json   each of the 4096 batched instances
  digest_serving_replay.json the seeded 1% sample of the 1000-request mix

Usage: python tests/golden/make_digests.py [--jobs J] [--only NAME ...]
The clustered instance and the largest served requests take minutes each.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time
from concurrent.futures import ProcessPoolExecutor, as_completed

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402


def digest(row_ptr: np.ndarray, col: np.ndarray) -> dict:
    rp = np.ascontiguousarray(row_ptr, dtype="<i8")
    c = np.ascontiguousarray(col, dtype="<i4")
    return {"n": int(len(rp) - 1), "nnz": int(len(c)),
            "row_ptr_sha256": hashlib.sha256(rp.tobytes()).hexdigest(),
            "col_sha256": hashlib.sha256(c.tobytes()).hexdigest()}


def _oracle_digest(task: tuple) -> tuple:
    """(key, digest, seconds) of the oracle's lists for one workload."""
    import oracle
    spec, wl = task
    t0 = time.perf_counter()
    res = oracle.rtg(wl.points(), wl.r, wl.k, wl.alpha, wl.seed)
    out = digest(res.row_ptr, res.col)
    out.update({"d": wl.d, "r": wl.r, "k": wl.k, "alpha": wl.alpha, "seed": wl.seed,
                "point_seed": wl.point_seed})
    return spec, out, time.perf_counter() - t0


def main(argv=None) -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--jobs", type=int, default=max(1, (os.cpu_count() or 2) - 1))
    ap.add_argument("--only", nargs="*", default=["clustered_d12", "batched", "serving"])
    args = ap.parse_args(argv)
    from paper_1409_8112_amd import workloads

    def write(name, payload, indent=1):
        path = os.path.join(HERE, name)
        with open(path, "w") as fh:
            json.dump(payload, fh, indent=indent, sort_keys=True)
            fh.write("\n")
        print("wrote", path, flush=True)

    note = ("oracle digests (tests/golden/make_digests.py): SHA-256 of row_ptr (<i8) and "
            "col (<i4) of oracle.rtg on the seeded workload")
    tasks = []
    groups: dict = {}
    if "clustered_d12" in args.only:
        tasks.append((("clustered_d12", 0), workloads.skewed_clustered_d12()))
        groups["clustered_d12"] = 1
    if "serving" in args.only:
        mix = workloads.serving_mix()
        sample = [int(i) for i in mix.replay_sample()]
        # largest first, so the long ones start early
        tasks += sorted(((("serving", i), mix.requests[i]) for i in sample),
                        key=lambda t: -t[1].n * t[1].d)
        groups["serving"] = len(sample)
    if "batched" in args.only:
        wls = workloads.batched_instances(4096)
        tasks += [(("batched", q), wls[q]) for q in range(4096)]
        groups["batched"] = 4096

    def finish(group):
        if group == "clustered_d12":
            write("digest_clustered_d12.json",
                  {"note": note, "workload": workloads.skewed_clustered_d12().name,
                   "result": got[("clustered_d12", 0)]})
        elif group == "batched":
            # one compact row per instance: n, nnz, row_ptr digest, col digest
            rows = [[got[("batched", q)][f] for f in ("n", "nnz", "row_ptr_sha256", "col_sha256")]
                    for q in range(4096)]
            write("digest_batched_4096.json",
                  {"note": note, "workload": "workloads.batched_instances(4096)",
                   "fields": ["n", "nnz", "row_ptr_sha256", "col_sha256"], "instances": rows},
                  indent=None)
        else:
            write("digest_serving_replay.json",
                  {"note": note, "workload": "workloads.serving_mix(), replay_sample()",
                   "sample": sample,
                   "requests": {str(i): got[("serving", i)] for i in sample}})

    got: dict = {}
    left = dict(groups)
    t0 = time.perf_counter()
    with ProcessPoolExecutor(max_workers=args.jobs) as ex:
        futs = [ex.submit(_oracle_digest, t) for t in tasks]
        for i, f in enumerate(as_completed(futs)):
            spec, dg, dt = f.result()
            got[spec] = dg
            if dt > 5 or (i + 1) % 256 == 0:
                print(f"{i + 1}/{len(tasks)} {spec} {dt:.1f} s "
                      f"(elapsed {time.perf_counter() - t0:.0f} s)", flush=True)
            left[spec[0]] -= 1
            if left[spec[0]] == 0:
                finish(spec[0])
    return 0


if __name__ == "__main__":
    sys.exit(main())
