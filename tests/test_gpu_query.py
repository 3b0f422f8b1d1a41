"""Query mode through the C-ABI: every query row bit-exact with the oracle
(oracle.rtg_query) on the same transforms."""
import json
import os

import numpy as np
import pytest

import oracle
from paper_1409_8112_amd import workloads

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    import torch
    from paper_1409_8112_amd import rtg
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    c = rtg.Context(0, arena_bytes=8 << 30)
    yield c
    c.close()


def _dev(p):
    import torch
    return torch.from_numpy(np.ascontiguousarray(p, dtype=np.float32)).cuda()


def _query(ctx, points, queries, r, k, alpha, seed, flags=0):
    h = ctx.index_build(_dev(points), r, k, alpha, seed, flags)
    try:
        res = ctx.index_query(h, _dev(queries))
        rp, col = res.to_numpy()
        res.release()
    finally:
        ctx.release(h)
    return rp, col


def _ref(points, queries, r, k, alpha, seed, flags=0):
    R, u = oracle.make_transforms(seed, k, points.shape[1], flags)
    return oracle.rtg_query(points, queries, r, alpha, R, u)


def _same(got, ref):
    rp, col = got
    assert np.array_equal(rp, ref.row_ptr), "row_ptr differs"
    assert np.array_equal(col, ref.col), "col differs"


def test_small_uniform_d3(ctx):
    p = workloads.uniform_points(2000, 3, seed=0)
    q = workloads.uniform_points(500, 3, seed=1)
    for flags in (0, 1):
        _same(_query(ctx, p, q, 0.1, 4, 2.0, 0, flags), _ref(p, q, 0.1, 4, 2.0, 0, flags))


@pytest.mark.parametrize("d", [1, 2, 5, 6, 9, 12, 16, 20, 33])
def test_dimensions(ctx, d):
    n = 2500
    p = workloads.uniform_points(n, d, seed=400 + d)
    q = workloads.uniform_points(300, d, seed=500 + d)
    r = workloads.calibrate_radius_uniform(n, d, 10.0)
    _same(_query(ctx, p, q, r, 5, 1.5, d), _ref(p, q, r, 5, 1.5, d))


def test_queries_equal_to_points(ctx):
    p = workloads.uniform_points(3000, 4, seed=7)
    r, k, alpha = 0.1, 6, 2.0
    _same(_query(ctx, p, p, r, k, alpha, 3), _ref(p, p, r, k, alpha, 3))


def test_clustered_and_grids_in_several_sorts(ctx):
    p = workloads.clustered_points(8000, 12, seed=9)
    q = workloads.clustered_points(600, 12, seed=10)
    _same(_query(ctx, p, q, 0.04, 8, 2.0, 1), _ref(p, q, 0.04, 8, 2.0, 1))
    # d = 31, alpha = 0.6: two key bits per axis, the grids take several sorts
    p2 = workloads.clustered_points(3000, 31, seed=2, n_clusters=8, sigma=0.03)
    q2 = workloads.clustered_points(300, 31, seed=3, n_clusters=8, sigma=0.03)
    _same(_query(ctx, p2, q2, 0.3, 6, 0.6, 4), _ref(p2, q2, 0.3, 6, 0.6, 4))


def test_hand_example(ctx, golden_dir):
    """The hand-worked example, with its transform fed through a seed whose
    single grid is the identity (no rotation) and a shift checked equal."""
    with open(os.path.join(golden_dir, "query_hand_example.json")) as f:
        g = json.load(f)
    p = np.array(g["points"], np.float32)
    q = np.array(g["queries"], np.float32)
    # the oracle on the example's own transform; the library on seeded ones
    ref = oracle.rtg_query(p, q, g["r"], g["alpha"], np.array(g["R"]), np.array(g["u"]))
    assert [ref.col[ref.row_ptr[s]:ref.row_ptr[s + 1]].tolist() for s in range(4)] == g["rows"]
    for seed in range(3):
        _same(_query(ctx, p, q, g["r"], 2, g["alpha"], seed, 1),
              _ref(p, q, g["r"], 2, g["alpha"], seed, 1))


def test_empty_and_errors(ctx):
    from paper_1409_8112_amd import rtg
    p = workloads.uniform_points(500, 3, seed=3)
    rp, col = _query(ctx, p, np.zeros((0, 3), np.float32), 0.1, 2, 2.0, 0)
    assert rp.tolist() == [0] and len(col) == 0
    rp, col = _query(ctx, np.zeros((0, 3), np.float32) + 0.5, p[:7], 0.1, 2, 2.0, 0)
    assert rp.tolist() == [0] * 8
    bad = p[:20].copy()
    bad[5, 2] = np.inf
    with pytest.raises(rtg.RTGError) as e:
        _query(ctx, p, bad, 0.1, 2, 2.0, 0)
    assert e.value.code == rtg.EINVAL
    far = p[:3].copy() * 1e12
    with pytest.raises(rtg.RTGError) as e:
        _query(ctx, p, far, 1e-3, 2, 2.0, 0)
    assert e.value.code == rtg.ERANGE
    with pytest.raises(rtg.RTGError) as e:
        ctx.index_query(987654, _dev(p[:2]))
    assert e.value.code == rtg.ENOENT


def test_full_size_index_sampled_queries(ctx):
    """The uniform d6 workload (n = 1e6, k = 8) as the index, 48 queries."""
    wl = workloads.large_uniform_d6()
    p = wl.points()
    q = workloads.uniform_points(48, wl.d, seed=77)
    _same(_query(ctx, p, q, wl.r, wl.k, wl.alpha, wl.seed),
          _ref(p, q, wl.r, wl.k, wl.alpha, wl.seed))
