"""The brute-force neighbour search that bench.py's recall measurement
compares the GPU's lists with: for sampled rows it equals the oracle's
brute force (every pair within r, by the definition) exactly, across
dimensions, chunk boundaries and rows with no neighbour."""
import numpy as np
import pytest

import oracle
from paper_1409_8112_amd import workloads


@pytest.mark.parametrize("n,d,r,chunk", [(3000, 3, 0.08, 700), (5000, 6, 0.3, 1024),
                                         (2000, 12, 0.6, 333), (1500, 2, 0.001, 512)])
def test_brute_force_rows_equal_the_oracle(n, d, r, chunk):
    import bench
    p = workloads.uniform_points(n, d, seed=d + n)
    ref = oracle.bruteforce(p, r)
    rows = np.sort(np.random.default_rng(n).choice(n, 300, replace=False))
    got = bench.brute_force_rows(p, r, rows, chunk=chunk)
    for g, i in zip(got, rows):
        assert sorted(g) == ref.col[ref.row_ptr[i]:ref.row_ptr[i + 1]].tolist(), f"row {i}"


def test_coincident_points_are_neighbours():
    import bench
    p = np.repeat(workloads.uniform_points(50, 4, seed=3), 3, axis=0)
    got = bench.brute_force_rows(p, 1e-6, np.arange(len(p)), chunk=64)
    for i, g in enumerate(got):
        base = (i // 3) * 3
        assert sorted(g) == [j for j in range(base, base + 3) if j != i]
