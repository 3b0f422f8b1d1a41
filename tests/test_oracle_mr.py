"""Pins of the oracle's MR-metric (Sec. IV-C: the distance between two
configurations of several robots is the sum of the robots' own distances):
a hand-worked example, exact arithmetic on random inputs, the special cases
that reduce to textbook metrics, the norm bounds between the MR and the
Euclidean distance, and that the grids stay the Euclidean ones (only the
pair test changes)."""
import json
import os

import numpy as np
import pytest
from scipy.spatial.distance import cdist

import oracle
from paper_1409_8112_amd import workloads
from tests.exact import mr_margin

# A pair this close to the radius could fall either way in FP64; random
# inputs essentially never produce one, and the tests say so when they do.
TIE = 1e-12


def _pairs(csr):
    return set(map(tuple, csr.upper_pairs().tolist()))


def _flags(robots):
    return oracle.robots(robots)


def test_hand_example(golden_dir):
    with open(os.path.join(golden_dir, "mr_hand_example.json")) as f:
        g = json.load(f)
    p = np.array(g["points"], np.float32)
    fl = _flags(g["robots"])
    assert _pairs(oracle.bruteforce(p, g["r"], fl)) == set(map(tuple, g["mr_pairs"]))
    assert _pairs(oracle.bruteforce(p, g["r"])) == set(map(tuple, g["euclidean_pairs"]))
    R, u = np.array(g["R"]), np.array(g["u"])
    got = oracle.rtg_with_transforms(p, g["r"], g["alpha"], R, u, fl)
    assert _pairs(got) == set(map(tuple, g["mr_pairs"]))


@pytest.mark.parametrize("d,robots", [(6, 2), (6, 3), (4, 2), (9, 3), (5, 5)])
def test_bruteforce_matches_exact_arithmetic(d, robots):
    rng = np.random.default_rng(d * 10 + robots)
    p = rng.random((70, d)).astype(np.float32)
    r = 0.45 * np.sqrt(d / 3.0)
    got = _pairs(oracle.bruteforce(p, r, _flags(robots)))
    want, ties = set(), 0
    for i in range(len(p)):
        for j in range(i + 1, len(p)):
            m = mr_margin(p[i], p[j], r, robots)
            ties += abs(m) < TIE * r
            if m <= 0:
                want.add((i, j))
    assert ties == 0
    assert 0 < len(want) < len(p) * (len(p) - 1) // 2
    assert got == want


def test_one_axis_per_robot_is_the_manhattan_metric():
    p = workloads.uniform_points(400, 6, seed=3)
    r = 0.9
    got = _pairs(oracle.bruteforce(p, r, _flags(6)))
    D = cdist(p.astype(np.float64), p.astype(np.float64), "cityblock")
    iu = np.triu_indices(len(p), 1)
    near = np.abs(D[iu] - r) < TIE
    assert not near.any()
    want = {(int(i), int(j)) for i, j in zip(*iu) if D[i, j] <= r}
    assert len(want) > 100
    assert got == want


def test_robots_that_stand_still_leave_the_euclidean_metric():
    """When every configuration shares robot 2's position, the MR distance
    is robot 1's Euclidean distance, i.e. the Euclidean one."""
    rng = np.random.default_rng(8)
    p = np.zeros((300, 6), np.float32)
    p[:, :3] = rng.random((300, 3))
    p[:, 3:] = np.float32(0.25)
    r = 0.2
    D = cdist(p.astype(np.float64), p.astype(np.float64))
    iu = np.triu_indices(len(p), 1)
    assert not (np.abs(D[iu] - r) < TIE).any()
    want = {(int(i), int(j)) for i, j in zip(*iu) if D[i, j] <= r}
    assert _pairs(oracle.bruteforce(p, r, _flags(2))) == want
    assert _pairs(oracle.bruteforce(p, r)) == want


@pytest.mark.parametrize("robots", [2, 3, 6])
def test_norm_bounds(robots):
    """||x||_2 <= sum_b ||x_b||_2 <= sqrt(robots) ||x||_2 (triangle and
    Cauchy-Schwarz inequalities): the MR ball of radius r lies inside the
    Euclidean ball of radius r and contains the one of radius r/sqrt(robots)."""
    p = workloads.uniform_points(600, 6, seed=robots)
    r = 0.5
    mr = _pairs(oracle.bruteforce(p, r, _flags(robots)))
    outer = _pairs(oracle.bruteforce(p, r * (1 + TIE)))
    inner = _pairs(oracle.bruteforce(p, r / np.sqrt(robots) * (1 - TIE)))
    assert inner <= mr <= outer
    assert len(inner) < len(mr) < len(outer)


@pytest.mark.parametrize("flags", [0, oracle.NO_ROTATE])
def test_grids_are_the_euclidean_ones(flags):
    """RTG under the MR-metric reports exactly the pairs of Euclidean RTG
    (same r, alpha and transforms, hence the same cells) whose MR distance
    is at most r -- every MR neighbour is a Euclidean neighbour."""
    p = workloads.uniform_points(3000, 6, seed=11)
    r = workloads.prm_radius(3000, 6, 1.5)
    R, u = oracle.make_transforms(5, 6, 6, flags)
    mr = _pairs(oracle.rtg_with_transforms(p, r, 2.0, R, u, _flags(2)))
    eu = _pairs(oracle.rtg_with_transforms(p, r, 2.0, R, u))
    ij = np.array(sorted(eu))
    x = p[ij[:, 0]].astype(np.float64) - p[ij[:, 1]].astype(np.float64)
    dist = np.linalg.norm(x[:, :3], axis=1) + np.linalg.norm(x[:, 3:], axis=1)
    assert not (np.abs(dist - r) < 1e-9 * r).any()
    want = {(int(i), int(j)) for (i, j), t in zip(ij, dist) if t <= r}
    assert mr == want
    assert 0 < len(mr) < len(eu)
    assert mr <= _pairs(oracle.bruteforce(p, r, _flags(2)))


def test_rows_and_queries_follow_the_metric():
    p = workloads.uniform_points(1500, 6, seed=12)
    r = workloads.prm_radius(1500, 6, 1.5)
    fl = _flags(3)
    R, u = oracle.make_transforms(9, 5, 6)
    full = oracle.rtg_with_transforms(p, r, 2.0, R, u, fl)
    rows = np.array([0, 7, 500, 1499])
    got = oracle.rtg_rows(p, r, 2.0, R, u, rows, fl)
    for s, row in zip(rows, got):
        assert row.tolist() == full.col[full.row_ptr[s]:full.row_ptr[s + 1]].tolist()
    # a query equal to point s meets s itself and s's neighbours
    q = oracle.rtg_query(p, p[rows], r, 2.0, R, u, fl)
    for t, s in enumerate(rows):
        want = sorted(full.col[full.row_ptr[s]:full.row_ptr[s + 1]].tolist() + [int(s)])
        assert q.col[q.row_ptr[t]:q.row_ptr[t + 1]].tolist() == want


def test_robot_counts():
    p = workloads.uniform_points(200, 4, seed=2)
    for bad in (3, 5, 255):
        with pytest.raises(oracle.OracleError) as e:
            oracle.bruteforce(p, 0.3, _flags(bad))
        assert e.value.code == oracle.EINVAL
        with pytest.raises(oracle.OracleError):
            oracle.rtg(p, 0.3, 2, 2.0, 0, _flags(bad))
    # zero or one robot: the Euclidean metric
    eu = _pairs(oracle.bruteforce(p, 0.3))
    assert _pairs(oracle.bruteforce(p, 0.3, _flags(1))) == eu
    assert _pairs(oracle.bruteforce(p, 0.3, _flags(0))) == eu
