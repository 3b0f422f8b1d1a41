"""The three rules that remove pairs found by several grids -- first owner
(default), sort-unique (RTG_DEDUP_SORT) and the pair bitmap
(RTG_DEDUP_BITMAP, the paper's upper-triangle bitset, Sec. III-B) -- each
bit-exact with the oracle, alone, in batches, with the MR-metric, and
falling back to the first-owner rule when the bitmap would be too large."""
import numpy as np
import pytest

import oracle
from paper_1409_8112_amd import workloads

pytestmark = pytest.mark.gpu

K_PAIR_HIST, K_UNIQUE = 6, 8


@pytest.fixture(scope="module")
def ctx():
    """Small instances through the general pipeline too (the de-duplication
    kernels are its steps; the two-launch small path has its own tests)."""
    import os
    import torch
    from paper_1409_8112_amd import rtg
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    old = os.environ.get("RTG_SMALL")
    os.environ["RTG_SMALL"] = "0"
    try:
        c = rtg.Context(0, arena_bytes=24 << 30)
    finally:
        if old is None:
            del os.environ["RTG_SMALL"]
        else:
            os.environ["RTG_SMALL"] = old
    yield c
    c.close()


def _dev(p):
    import torch
    return torch.from_numpy(np.ascontiguousarray(p, dtype=np.float32)).cuda()


def _lists(res):
    rp, col = res.to_numpy()
    res.release()
    return rp, col


def _same(got, ref):
    assert np.array_equal(got[0], ref.row_ptr), "row_ptr differs"
    assert np.array_equal(got[1], ref.col), "col differs"


@pytest.mark.parametrize("n,d", [(2, 3), (65, 2), (2000, 3), (7777, 6), (3001, 9), (1500, 20)])
def test_every_rule_matches_the_oracle(ctx, n, d):
    from paper_1409_8112_amd import rtg
    p = workloads.uniform_points(n, d, seed=n + d)
    r = workloads.prm_radius(max(n, 3), d, 1.5)
    for extra in (0, rtg.UPPER_ONLY, rtg.NO_ROTATE):
        ref = oracle.rtg(p, r, 6, 2.0, 5, extra)
        for rule in (0, rtg.DEDUP_SORT, rtg.DEDUP_BITMAP):
            print(f"dedup rule={rule} n={n} d={d} flags={extra}", flush=True)
            _same(_lists(ctx.all_pairs(_dev(p), r, 6, 2.0, 5, rule | extra)), ref)
            st = ctx.stats()
            if rule == rtg.DEDUP_BITMAP and st["candidates"] > 0:
                assert st["kernel_launches"][K_UNIQUE] >= 1  # the bitmap pass ran
                assert st["candidates"] >= st["unique_pairs"]


def test_bitmap_needs_no_pair_sort(ctx):
    from paper_1409_8112_amd import rtg
    p = workloads.uniform_points(20000, 6, seed=3)
    r = workloads.prm_radius(20000, 6, 1.5)
    _lists(ctx.all_pairs(_dev(p), r, 8, 2.0, 0, rtg.DEDUP_BITMAP))
    st = ctx.stats()
    assert st["kernel_launches"][K_PAIR_HIST] == 0
    assert st["candidates"] > st["unique_pairs"]  # repeats were found and dropped
    _lists(ctx.all_pairs(_dev(p), r, 8, 2.0, 0, rtg.DEDUP_SORT))
    st_sort = ctx.stats()
    assert st_sort["kernel_launches"][K_PAIR_HIST] > 0
    assert st_sort["candidates"] == st["candidates"]
    assert st_sort["unique_pairs"] == st["unique_pairs"]


def test_coincident_points(ctx):
    from paper_1409_8112_amd import rtg
    p = np.repeat(workloads.uniform_points(40, 3, seed=1), 25, axis=0)  # 1000 points, 25 copies
    ref = oracle.rtg(p, 0.05, 5, 2.0, 2)
    _same(_lists(ctx.all_pairs(_dev(p), 0.05, 5, 2.0, 2, rtg.DEDUP_BITMAP)), ref)


def test_bitmap_with_the_mr_metric(ctx):
    from paper_1409_8112_amd import rtg
    p = workloads.uniform_points(6000, 6, seed=8)
    r = workloads.prm_radius(6000, 6, 1.7)
    ref = oracle.rtg(p, r, 6, 2.0, 1, oracle.robots(2))
    _same(_lists(ctx.all_pairs(_dev(p), r, 6, 2.0, 1, rtg.DEDUP_BITMAP | rtg.robots(2))), ref)


def test_batched_bitmaps(ctx):
    """Every instance of a batch owns its own range of bits."""
    from paper_1409_8112_amd import rtg
    reqs = []
    for q in range(16):
        n = 300 + 577 * q
        p = workloads.uniform_points(n, 3, seed=50 + q)
        reqs.append(dict(points=p, r=workloads.prm_radius(n, 3, 1.3), k=4 + q % 3, alpha=2.0,
                         seed=q, flags=rtg.DEDUP_BITMAP | (q % 2)))
    keep = [_dev(q["points"]) for q in reqs]
    outs = ctx.all_pairs_batched([dict(q, points=t) for t, q in zip(keep, reqs)])
    for q, res in zip(reqs, outs):
        ref = oracle.rtg(q["points"], q["r"], q["k"], q["alpha"], q["seed"], q["flags"] & 1)
        _same(_lists(res), ref)


def test_too_large_bitmap_falls_back(ctx):
    """n = 10^6 would need 62.5 GB of bits: the first-owner rule runs, and
    the result is the default one."""
    from paper_1409_8112_amd import rtg
    wl = workloads.large_uniform_d6()
    p = _dev(wl.points())
    a = _lists(ctx.all_pairs(p, wl.r, wl.k, wl.alpha, wl.seed, rtg.DEDUP_BITMAP))
    st = ctx.stats()
    assert st["kernel_launches"][K_UNIQUE] == 0
    b = _lists(ctx.all_pairs(p, wl.r, wl.k, wl.alpha, wl.seed))
    assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])


def test_sort_and_bitmap_together_are_invalid(ctx):
    from paper_1409_8112_amd import rtg
    p = _dev(workloads.uniform_points(100, 3, seed=0))
    with pytest.raises(rtg.RTGError) as e:
        ctx.all_pairs(p, 0.1, 2, 2.0, 0, rtg.DEDUP_SORT | rtg.DEDUP_BITMAP)
    assert e.value.code == rtg.EINVAL
