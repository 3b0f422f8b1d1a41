"""The batched entry point: every query's lists equal the oracle's (and so
the plain call's) whatever batch it shares, across dimensions, sizes, radii,
grid counts and list flags."""
import os

import numpy as np
import pytest

import oracle
from paper_1409_8112_amd import workloads

pytestmark = pytest.mark.gpu


def _ctx(**env):
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


@pytest.fixture(scope="module")
def ctx():
    c = _ctx()
    yield c
    c.close()


def _dev(p):
    import torch
    return torch.from_numpy(np.ascontiguousarray(p, dtype=np.float32)).cuda()


def _queries(seed, count, dims=(2, 3, 6, 9), n_lo=2, n_hi=3000):
    rng = np.random.default_rng(seed)
    qs = []
    for q in range(count):
        d = int(rng.choice(dims))
        n = int(np.exp(rng.uniform(np.log(n_lo), np.log(n_hi))))
        p = workloads.uniform_points(n, d, seed=seed * 1000 + q)
        r = workloads.prm_radius(max(n, 3), d, 0.9) if n > 2 else 0.3
        qs.append(dict(points=p, r=r, k=int(rng.integers(1, 7)), alpha=float(rng.uniform(1.2, 2.5)),
                       seed=q, flags=int(rng.choice([0, 0, 1, 2]))))
    return qs


def _run(ctx, qs):
    dev = [dict(q, points=_dev(q["points"])) for q in qs]
    res = ctx.all_pairs_batched(dev)
    out = [r.to_numpy() for r in res]
    for r in res:
        r.release()
    return out


def _check(qs, got):
    for q, (rp, col) in zip(qs, got):
        ref = oracle.rtg(q["points"], q["r"], q["k"], q["alpha"], q["seed"], q["flags"] & 3)
        assert np.array_equal(rp, ref.row_ptr) and np.array_equal(col, ref.col), \
            (len(q["points"]), q["points"].shape[1], q["k"], q["flags"])


def test_mixed_batch_equals_oracle(ctx):
    qs = _queries(1, 40)
    _check(qs, _run(ctx, qs))


def test_batch_with_empty_and_single_point_queries(ctx):
    qs = _queries(2, 6)
    qs.insert(2, dict(points=np.zeros((0, 3), np.float32), r=0.1, k=2, alpha=2.0, seed=0, flags=0))
    qs.insert(4, dict(points=np.full((1, 6), 0.5, np.float32), r=0.1, k=2, alpha=2.0, seed=0,
                      flags=0))
    got = _run(ctx, qs)
    _check(qs, got)


def test_batch_equals_plain_calls(ctx):
    qs = _queries(3, 12, dims=(3,), n_lo=500, n_hi=5000)
    got = _run(ctx, qs)
    for q, (rp, col) in zip(qs, got):
        res = ctx.all_pairs(_dev(q["points"]), q["r"], q["k"], q["alpha"], q["seed"], q["flags"])
        rp1, col1 = res.to_numpy()
        res.release()
        assert np.array_equal(rp, rp1) and np.array_equal(col, col1)


def test_batches_split_by_point_budget():
    """With a small point budget the queries of one dimension run as several
    batches; results do not depend on the split."""
    c = _ctx(RTG_BATCH_POINTS=4000)
    try:
        qs = _queries(4, 25, dims=(2, 6))
        _check(qs, _run(c, qs))
    finally:
        c.close()


def test_sort_unique_mode_in_batches(ctx):
    from paper_1409_8112_amd import rtg
    qs = _queries(5, 10)
    for q in qs:
        q["flags"] |= rtg.DEDUP_SORT
    _check(qs, _run(ctx, qs))


def test_invalid_query_fails_the_batch_and_keeps_nothing(ctx):
    from paper_1409_8112_amd import rtg
    qs = _queries(6, 5)
    bad = qs[3]["points"].copy()
    if len(bad) > 1:
        bad[0, 0] = np.nan
    else:
        bad = np.array([[np.nan] * bad.shape[1], [0.0] * bad.shape[1]], np.float32)
    qs[3] = dict(qs[3], points=bad)
    with pytest.raises(rtg.RTGError) as e:
        _run(ctx, qs)
    assert e.value.code == rtg.EINVAL
    # the context still works
    ok = _queries(7, 3)
    _check(ok, _run(ctx, ok))


def test_instances_without_pairs_between_others(ctx):
    """Copying a batch's lists into per-instance results: instances with no
    pairs (a radius too small for any) at the start, the end and in runs in
    the middle, many small instances sharing one run of the copy and large
    ones spanning several -- every result equals the oracle's."""
    qs = []
    for q in range(30):
        none = q in (0, 1, 7, 8, 9, 15, 28, 29)
        n = 3 if q % 5 == 4 else (40 + 13 * q if q % 3 else 2500 + 400 * q)
        p = workloads.uniform_points(n, 3, seed=900 + q)
        r = 1e-7 if none else workloads.prm_radius(max(n, 3), 3, 1.2)
        qs.append(dict(points=p, r=r, k=3, alpha=2.0, seed=q, flags=(0, 1)[q % 2]))
    got = _run(ctx, qs)
    _check(qs, got)
    assert sum(len(col) for _, col in got) > 200_000  # several runs of the copy
    assert all(len(got[q][1]) == 0 for q in (0, 1, 7, 8, 9, 15, 28, 29))


def test_result_views_made_on_first_use(ctx):
    """row_ptr and col are device views into the arena, made on first access
    and equal to the copied-out lists."""
    import torch
    qs = _queries(8, 5, dims=(3,), n_lo=200, n_hi=2000)
    res = ctx.all_pairs_batched([dict(q, points=_dev(q["points"])) for q in qs])
    try:
        for q, r in zip(qs, res):
            ref = oracle.rtg(q["points"], q["r"], q["k"], q["alpha"], q["seed"], q["flags"] & 3)
            assert r.row_ptr.is_cuda and r.row_ptr.dtype == torch.int64
            assert r.col.dtype == torch.int32 and r.row_ptr.shape[0] == r.n + 1
            assert r.col.shape[0] == r.nnz == len(ref.col)
            assert np.array_equal(r.row_ptr.cpu().numpy(), ref.row_ptr)
            assert np.array_equal(r.col.cpu().numpy(), ref.col)
    finally:
        for r in res:
            r.release()


def test_two_lanes_in_a_small_budget():
    """Batches run several at a time; in a budget that holds about two passes
    a pass may run out of memory beside the others and runs again alone.
    Every result equals the oracle's, and equals one lane's."""
    qs = []
    for q in range(6):
        n = 40000 - 1500 * q
        p = workloads.uniform_points(n, 3, seed=700 + q)
        qs.append(dict(points=p, r=workloads.prm_radius(n, 3, 0.6), k=4, alpha=2.0, seed=q,
                       flags=0))
    small = _small_ctx(48 << 20, RTG_BATCH_POINTS=40000)
    try:
        got = _run(small, qs)
    finally:
        small.close()
    one = _small_ctx(48 << 20, RTG_BATCH_POINTS=40000, RTG_BATCH_LANES=1)
    try:
        alone = _run(one, qs)
    finally:
        one.close()
    _check(qs, got)
    for (a, b), (x, y) in zip(got, alone):
        assert np.array_equal(a, x) and np.array_equal(b, y)


def _small_ctx(arena_bytes, **env):
    import torch
    from paper_1409_8112_amd import rtg
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    old = {k: os.environ.get(k) for k in env}
    os.environ.update({k: str(v) for k, v in env.items()})
    try:
        return rtg.Context(0, arena_bytes=arena_bytes)
    finally:
        for k, v in old.items():
            if v is None:
                del os.environ[k]
            else:
                os.environ[k] = v


def test_release_many(ctx):
    """One call releases a batch's results; releasing them again is
    RTG_ENOENT, and a negative count or a missing array is RTG_EINVAL."""
    import ctypes
    from paper_1409_8112_amd import rtg
    qs = _queries(9, 12, dims=(3, 6), n_lo=100, n_hi=3000)
    res = ctx.all_pairs_batched([dict(q, points=_dev(q["points"])) for q in qs])
    handles = np.array([r.handle for r in res], dtype=np.uint64)
    ctx.release_many(res)
    assert all(r.released for r in res)
    ctx.release_many(res)  # nothing left to release: no call
    ptr = handles.ctypes.data_as(ctypes.POINTER(ctypes.c_uint64))
    assert rtg.lib().rtg_release_many(ctx.h, ptr, len(handles)) == rtg.ENOENT
    assert rtg.lib().rtg_release_many(ctx.h, ptr, -1) == rtg.EINVAL
    assert rtg.lib().rtg_release_many(ctx.h, None, 3) == rtg.EINVAL
    assert rtg.lib().rtg_release_many(ctx.h, None, 0) == rtg.OK
    # the context still works and the memory came back
    _check(qs[:4], _run(ctx, qs[:4]))
