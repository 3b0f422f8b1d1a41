"""Pins of the query-mode oracle: a hand-worked example, the special cases
that reduce to brute force or to the all-pairs rows, and the invariants of
a union over grids."""
import json
import os

import numpy as np
import pytest

import oracle
from paper_1409_8112_amd import workloads
from tests.exact import exact_within


def _rows(csr):
    return [csr.col[csr.row_ptr[s]:csr.row_ptr[s + 1]].tolist() for s in range(len(csr.row_ptr) - 1)]


def test_hand_example(golden_dir):
    with open(os.path.join(golden_dir, "query_hand_example.json")) as f:
        g = json.load(f)
    res = oracle.rtg_query(np.array(g["points"], np.float32), np.array(g["queries"], np.float32),
                           g["r"], g["alpha"], np.array(g["R"]), np.array(g["u"]))
    assert _rows(res) == g["rows"]


def test_one_huge_cell_is_an_exact_ball_query():
    """With every point and query in one cell (huge alpha, shift away from
    the cell faces) query mode reports exactly the points within r,
    checked in exact rational arithmetic."""
    rng = np.random.default_rng(5)
    p = rng.random((300, 3)).astype(np.float32)
    q = rng.random((40, 3)).astype(np.float32)
    R, u = oracle.make_transforms(0, 64, 3)
    t = next(t for t in range(64) if np.all((u[t] > 0.01) & (u[t] < 0.99)))
    r = 0.2
    res = oracle.rtg_query(p, q, r, 1e4, R[t:t + 1], u[t:t + 1])
    for s in range(len(q)):
        want = [i for i in range(len(p)) if exact_within(q[s], p[i], r)]
        assert _rows(res)[s] == want


def test_queries_equal_to_the_points_give_the_all_pairs_rows_plus_self():
    p = workloads.uniform_points(600, 3, seed=2)
    r, k, alpha = 0.12, 4, 2.0
    R, u = oracle.make_transforms(9, k, 3)
    allp = oracle.rtg_with_transforms(p, r, alpha, R, u)
    res = oracle.rtg_query(p, p, r, alpha, R, u)
    for i, row in enumerate(_rows(res)):
        base = allp.col[allp.row_ptr[i]:allp.row_ptr[i + 1]].tolist()
        assert row == sorted(base + [i])


def test_union_over_grids_and_prefix():
    rng = np.random.default_rng(8)
    p = rng.random((500, 4)).astype(np.float32)
    q = rng.random((120, 4)).astype(np.float32)
    r, alpha = 0.25, 1.5
    R, u = oracle.make_transforms(3, 5, 4)
    full = _rows(oracle.rtg_query(p, q, r, alpha, R, u))
    single = [_rows(oracle.rtg_query(p, q, r, alpha, R[t:t + 1], u[t:t + 1])) for t in range(5)]
    for s in range(len(q)):
        assert full[s] == sorted(set().union(*[set(single[t][s]) for t in range(5)]))
    fewer = _rows(oracle.rtg_query(p, q, r, alpha, R[:3], u[:3]))
    for s in range(len(q)):
        assert set(fewer[s]) <= set(full[s])
        # every reported point is within r, exactly
        assert all(exact_within(q[s], p[i], r) for i in full[s])


def test_query_order_permutes_rows():
    rng = np.random.default_rng(11)
    p = rng.random((400, 2)).astype(np.float32)
    q = rng.random((90, 2)).astype(np.float32)
    R, u = oracle.make_transforms(1, 3, 2)
    a = _rows(oracle.rtg_query(p, q, 0.1, 2.0, R, u))
    perm = rng.permutation(len(q))
    b = _rows(oracle.rtg_query(p, q[perm], 0.1, 2.0, R, u))
    assert [a[i] for i in perm] == b


def test_empty_inputs_and_errors():
    p = workloads.uniform_points(50, 3, seed=1)
    R, u = oracle.make_transforms(0, 2, 3)
    res = oracle.rtg_query(p, np.zeros((0, 3), np.float32), 0.1, 2.0, R, u)
    assert len(res.row_ptr) == 1
    res = oracle.rtg_query(np.zeros((0, 3), np.float32), p[:5], 0.1, 2.0, R, u)
    assert res.row_ptr.tolist() == [0] * 6
    bad = p[:5].copy()
    bad[2, 1] = np.nan
    with pytest.raises(oracle.OracleError):
        oracle.rtg_query(p, bad, 0.1, 2.0, R, u)
