"""The stored whole-output digests come from the oracle: a few of the
cheapest entries are recomputed here from the oracle on the same seeded
inputs (CPU only), and every file lists the workloads it claims to cover."""
import hashlib
import json
import os

import numpy as np
import pytest

import oracle
from paper_1409_8112_amd import workloads

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def _load(name):
    with open(os.path.join(GOLDEN, name)) as fh:
        return json.load(fh)


def _matches(wl, e):
    res = oracle.rtg(wl.points(), wl.r, wl.k, wl.alpha, wl.seed)
    rp = hashlib.sha256(np.ascontiguousarray(res.row_ptr, dtype="<i8").tobytes()).hexdigest()
    col = hashlib.sha256(np.ascontiguousarray(res.col, dtype="<i4").tobytes()).hexdigest()
    return (wl.n, len(res.col), rp, col) == (e["n"], e["nnz"], e["row_ptr_sha256"],
                                            e["col_sha256"])


def test_batched_digests_are_the_oracles():
    wls = workloads.batched_instances(4096)
    want = [dict(zip(("n", "nnz", "row_ptr_sha256", "col_sha256"), row))
            for row in _load("digest_batched_4096.json")["instances"]]
    assert len(want) == 4096
    assert [e["n"] for e in want] == [w.n for w in wls]
    smallest = sorted(range(4096), key=lambda q: wls[q].n)[:6]
    for q in smallest:
        assert _matches(wls[q], want[q]), f"instance {q}"


def test_serving_digests_are_the_oracles():
    mix = workloads.serving_mix()
    want = _load("digest_serving_replay.json")
    assert want["sample"] == [int(i) for i in mix.replay_sample()]
    smallest = sorted(want["sample"], key=lambda q: mix.requests[q].n)[:3]
    for q in smallest:
        assert _matches(mix.requests[q], want["requests"][str(q)]), f"request {q}"


def test_clustered_digest_names_its_workload():
    wl = workloads.skewed_clustered_d12()
    e = _load("digest_clustered_d12.json")["result"]
    assert (e["n"], e["d"], e["k"], e["seed"], e["point_seed"]) == (wl.n, wl.d, wl.k, wl.seed,
                                                                   wl.point_seed)
    assert e["r"] == pytest.approx(wl.r, rel=0, abs=0)
