"""Parameter choice for a target recall: the oracle's recall model pinned to
closed forms and to measured RTG recall, the library's model against it, and
the chosen parameters against the target."""
import math

import numpy as np
import pytest

import oracle
from oracle import recall_model as M
from paper_1409_8112_amd import rtg, workloads


def test_one_axis_closed_form():
    """d = 1, shift only: p = 1 - x/alpha, so recall = 1 - 1/(alpha^k (k+1))."""
    for k, alpha in [(1, 1.5), (3, 1.2), (5, 2.0)]:
        exact = 1.0 - 1.0 / (alpha ** k * (k + 1))
        assert abs(M.model_recall(1, k, alpha, rotate=False, samples=200_000) - exact) < 3e-3
        assert abs(M.model_recall(1, k, alpha, rotate=True) - exact) < 3e-3


def test_two_axis_rotated_closed_form():
    """d = 2, random orientation: 1 - 4 rho/(pi c) + rho^2/(pi c^2), rho <= c."""
    c = 1.0
    for rho in (0.1, 0.4, 0.8):
        exact = 1.0 - 4.0 * rho / (math.pi * c) + rho * rho / (math.pi * c * c)
        assert abs(M.rotated_cocell_probability(rho, c, 2) - exact) < 3e-3


@pytest.mark.parametrize("d,k,alpha", [(3, 4, 2.0), (6, 8, 1.5), (4, 3, 1.2)])
def test_model_matches_measured_recall(d, k, alpha):
    """The model against RTG itself (the oracle) on uniform points, five
    seeds; boundary and sampling effects stay within 0.02."""
    n = 3000 if d <= 4 else 2000
    r = workloads.calibrate_radius_uniform(n, d, 12.0)
    got = []
    for s in range(5):
        p = workloads.uniform_points(n, d, seed=900 + s)
        truth = len(oracle.bruteforce(p, r).col)
        got.append(len(oracle.rtg(p, r, k, alpha, s).col) / truth)
    assert abs(np.mean(got) - M.model_recall(d, k, alpha)) < 0.02, (np.mean(got),)


@pytest.mark.parametrize("d", [2, 3, 6, 9, 12])
@pytest.mark.parametrize("rotate", [True, False])
def test_library_model_matches_oracle_model(d, rotate):
    flags = 0 if rotate else rtg.NO_ROTATE
    for k, alpha in [(4, 2.0), (12, 1.5), (30, 1.25)]:
        lib = rtg.model_recall(d, k, alpha, flags)
        ref = M.model_recall(d, k, alpha, rotate=rotate)
        assert abs(lib - ref) < 6e-3, (k, alpha, lib, ref)


@pytest.mark.parametrize("d,target", [(3, 0.95), (6, 0.98), (9, 0.98), (12, 0.95)])
def test_chosen_parameters_reach_the_target(d, target):
    k, alpha, rec = rtg.choose_params(d, target, 20.0)
    assert rec >= target
    assert M.model_recall(d, k, alpha) >= target - 6e-3
    # one grid fewer misses the target (k is the least for that alpha)
    if k > 1:
        assert rtg.model_recall(d, k - 1, alpha) < target


def test_choice_trades_grids_for_cell_size():
    """Denser neighbourhoods make tests dearer: the choice moves to smaller
    cells and more grids; a higher target never costs fewer grids at the
    same cell size."""
    k_sparse, a_sparse, _ = rtg.choose_params(6, 0.98, 2.0)
    k_dense, a_dense, _ = rtg.choose_params(6, 0.98, 2000.0)
    assert a_dense <= a_sparse and k_dense >= k_sparse
    assert rtg.model_recall(6, 10, 1.5) < rtg.model_recall(6, 20, 1.5)


def test_errors():
    for args in [(0, 0.9, 10.0), (65, 0.9, 10.0), (6, 1.0, 10.0), (6, 0.9, 0.0)]:
        with pytest.raises(rtg.RTGError) as e:
            rtg.choose_params(*args)
        assert e.value.code == rtg.EINVAL
    for args in [(6, 0, 1.5), (6, 4, 0.0), (0, 4, 1.5)]:
        with pytest.raises(rtg.RTGError) as e:
            rtg.model_recall(*args)
        assert e.value.code == rtg.EINVAL
