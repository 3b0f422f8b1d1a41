"""The MR-metric (Sec. IV-C: the distance of two multi-robot configurations
is the sum of the robots' own distances) through the C-ABI: every list
bit-exact with the oracle on the same transforms, under both pair screens,
in batches mixed with Euclidean instances, in the request loop and in
query mode; pairs at r exactly; full benchmark size by sampled rows."""
import os

import numpy as np
import pytest

import oracle
from paper_1409_8112_amd import workloads

pytestmark = pytest.mark.gpu


def _context(**env):
    import torch
    from paper_1409_8112_amd import rtg
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    old = {k: os.environ.get(k) for k in env}
    os.environ.update({k: str(v) for k, v in env.items()})
    try:
        return rtg.Context(0, arena_bytes=8 << 30)
    finally:
        for k, v in old.items():
            if v is None:
                del os.environ[k]
            else:
                os.environ[k] = v


@pytest.fixture(scope="module", params=["vector", "matrix"])
def screen(request):
    c = _context(RTG_PAIRS=request.param)
    yield request.param, c
    c.close()


@pytest.fixture(scope="module")
def ctx():
    c = _context()
    yield c
    c.close()


def _say(msg):
    print(msg, flush=True)


def _dev(p):
    import torch
    return torch.from_numpy(np.ascontiguousarray(p, dtype=np.float32)).cuda()


def _lists(res):
    rp, col = res.to_numpy()
    res.release()
    return rp, col


def _same(got, ref):
    rp, col = got
    assert np.array_equal(rp, ref.row_ptr), "row_ptr differs"
    assert np.array_equal(col, ref.col), "col differs"


def _fl(robots, extra=0):
    from paper_1409_8112_amd import rtg
    return rtg.robots(robots) | extra


@pytest.mark.parametrize("d,robots", [(6, 2), (6, 3), (6, 6), (4, 2), (9, 3), (12, 4), (2, 2)])
def test_parity_both_screens(screen, d, robots):
    mode, c = screen
    n = 3001  # several tiles and a ragged tail
    p = workloads.uniform_points(n, d, seed=d * 7 + robots)
    r = workloads.prm_radius(n, d, 1.6)
    for flags in (0, 1, 2, 4):
        fl = _fl(robots, flags)
        _say(f"MR {mode}: n={n} d={d} robots={robots} flags={flags}")
        got = _lists(c.all_pairs(_dev(p), r, 5, 2.0, 3, fl))
        _same(got, oracle.rtg(p, r, 5, 2.0, 3, oracle.robots(robots) | (flags & 3)))


def test_wide_d_and_clusters(ctx):
    for d, robots in ((20, 2), (33, 3), (64, 8)):
        p = workloads.clustered_points(1500, d, seed=d)
        r = 0.05 * np.sqrt(d)
        _say(f"MR wide: d={d} robots={robots}")
        got = _lists(ctx.all_pairs(_dev(p), r, 3, 1.5, 1, _fl(robots)))
        _same(got, oracle.rtg(p, r, 3, 1.5, 1, oracle.robots(robots)))


def test_fewer_pairs_than_euclidean(ctx):
    p = workloads.uniform_points(20000, 6, seed=4)
    r = workloads.prm_radius(20000, 6, 1.5)
    eu = _lists(ctx.all_pairs(_dev(p), r, 8, 2.0, 0))
    st_eu = ctx.stats()
    mr = _lists(ctx.all_pairs(_dev(p), r, 8, 2.0, 0, _fl(2)))
    st_mr = ctx.stats()
    assert 0 < len(mr[1]) < len(eu[1])
    assert st_mr["unique_pairs"] == len(mr[1]) // 2
    assert st_mr["band_rechecks"] >= st_eu["unique_pairs"]  # every Euclidean candidate tested
    # every MR pair is a Euclidean pair of the same grids
    rows = lambda rp, col: set(zip(np.repeat(np.arange(len(rp) - 1), np.diff(rp)).tolist(),
                                   col.tolist()))
    assert rows(*mr) <= rows(*eu)


def test_pairs_at_r_exactly(ctx):
    """r set to the FP64 MR distance of chosen pairs (square roots correctly
    rounded, robots in order): those pairs are reported, as the definition
    (<= r) says; one ulp less and they are not."""
    p = workloads.uniform_points(600, 6, seed=21)
    # one cell holds every point (y = p / (50 r) + 0.5 < 1): the test alone decides
    R, u = np.eye(6)[None], np.full((1, 6), 0.5)
    for a, b in ((0, 1), (5, 9), (100, 300)):
        x = p[a].astype(np.float64) - p[b].astype(np.float64)
        t1 = (x[0] * x[0] + x[1] * x[1]) + x[2] * x[2]
        t2 = (x[3] * x[3] + x[4] * x[4]) + x[5] * x[5]
        r = float(np.sqrt(t1) + np.sqrt(t2))
        for rr in (r, np.nextafter(r, 0.0)):
            alpha = 50.0
            got = _lists(ctx.all_pairs_with_transforms(_dev(p), rr, alpha, R, u, _fl(2)))
            ref = oracle.rtg_with_transforms(p, rr, alpha, R, u, oracle.robots(2))
            _same(got, ref)
            rp, col = got
            listed = b in col[rp[a]:rp[a + 1]].tolist()
            assert listed == (rr == r)


def test_batched_mixed_with_euclidean(ctx):
    reqs = []
    for q in range(24):
        n = 500 + 331 * q
        p = workloads.uniform_points(n, 6, seed=100 + q)
        rob = (0, 2, 3, 6)[q % 4]
        reqs.append(dict(points=p, r=workloads.prm_radius(n, 6, 1.4), k=3 + q % 5, alpha=2.0,
                         seed=q, flags=_fl(rob, (0, 1)[q % 2]) if rob else (0, 1)[q % 2],
                         robots=rob))
    keep = [_dev(q["points"]) for q in reqs]
    outs = ctx.all_pairs_batched([dict(q, points=t) for t, q in zip(keep, reqs)])
    for q, res in zip(reqs, outs):
        ref = oracle.rtg(q["points"], q["r"], q["k"], q["alpha"], q["seed"],
                         oracle.robots(q["robots"]) | (q["flags"] & 1))
        _same(_lists(res), ref)


def test_served_requests(ctx):
    reqs = []
    for q in range(12):
        n = 800 + 900 * q
        p = workloads.uniform_points(n, 6, seed=300 + q)
        reqs.append((p, workloads.prm_radius(n, 6, 1.4), 4, 2.0, q, (0, 2)[q % 2]))
    tickets = [ctx.submit(_dev(p), r, k, a, s, _fl(rb) if rb else 0) for p, r, k, a, s, rb in reqs]
    for (p, r, k, a, s, rb), t in zip(reqs, tickets):
        got = _lists(ctx.wait(t, timeout_s=60))
        _same(got, oracle.rtg(p, r, k, a, s, oracle.robots(rb)))


@pytest.mark.parametrize("d,robots", [(6, 2), (6, 3), (12, 3), (20, 4)])
def test_query_mode(ctx, d, robots):
    p = workloads.uniform_points(5000, d, seed=d)
    q = workloads.uniform_points(700, d, seed=d + 1)
    q[:50] = p[:50]  # queries equal to indexed points
    r = workloads.prm_radius(5000, d, 1.6)
    h = ctx.index_build(_dev(p), r, 6, 2.0, 7, _fl(robots))
    try:
        got = _lists(ctx.index_query(h, _dev(q)))
    finally:
        ctx.release(h)
    R, u = oracle.make_transforms(7, 6, d)
    _same(got, oracle.rtg_query(p, q, r, 2.0, R, u, oracle.robots(robots)))


def test_invalid_robot_counts(ctx):
    from paper_1409_8112_amd import rtg
    p = _dev(workloads.uniform_points(100, 6, seed=0))
    for bad in (_fl(4), _fl(5), _fl(7), _fl(255), 1 << 16, 1 << 30):
        with pytest.raises(rtg.RTGError) as e:
            ctx.all_pairs(p, 0.2, 2, 2.0, 0, bad)
        assert e.value.code == rtg.EINVAL
        with pytest.raises(rtg.RTGError) as e:
            ctx.index_build(p, 0.2, 2, 2.0, 0, bad)
        assert e.value.code == rtg.EINVAL
    # zero or one robot: the Euclidean metric
    a = _lists(ctx.all_pairs(p, 0.3, 2, 2.0, 0, _fl(1)))
    b = _lists(ctx.all_pairs(p, 0.3, 2, 2.0, 0))
    assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])


def test_full_size_two_robots_sampled(ctx):
    """The uniform d = 6 benchmark instance read as two robots in 3-D space
    (the multi-robot setting of Sec. IV-C): every listed pair is within r
    under the MR-metric, and sampled rows equal the oracle's."""
    wl = workloads.large_uniform_d6()
    p = wl.points()
    _say(f"MR full size {wl.name}: GPU")
    rp, col = _lists(ctx.all_pairs(_dev(p), wl.r, wl.k, wl.alpha, wl.seed, _fl(2)))
    n = wl.n
    rows = np.repeat(np.arange(n, dtype=np.int64), np.diff(rp))
    c64 = col.astype(np.int64)
    assert rp[0] == 0 and rp[-1] == len(col) and np.all(c64 != rows)
    x = p[rows].astype(np.float64) - p[c64].astype(np.float64)
    dist = np.sqrt((x[:, 0] * x[:, 0] + x[:, 1] * x[:, 1]) + x[:, 2] * x[:, 2]) + \
        np.sqrt((x[:, 3] * x[:, 3] + x[:, 4] * x[:, 4]) + x[:, 5] * x[:, 5])
    assert np.all(dist <= wl.r)
    _say("  oracle rows x128")
    R, u = oracle.make_transforms(wl.seed, wl.k, wl.d)
    sample = np.random.default_rng(77).choice(n, size=128, replace=False)
    ref = oracle.rtg_rows(p, wl.r, wl.alpha, R, u, sample, oracle.robots(2))
    for s_i, row in enumerate(sample):
        assert np.array_equal(col[rp[row]:rp[row + 1]], ref[s_i]), f"row {row}"
