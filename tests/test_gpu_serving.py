"""The request loop (rtg_submit / rtg_poll): every served result equals the
oracle's and the lone call's, whatever it was batched with; requests are
batched; the loop admits work by device memory; errors stay with their
request; a small request that finds the device idle runs alone on the
two-launch small path."""
import os

import numpy as np
import pytest

import oracle
from paper_1409_8112_amd import workloads

pytestmark = pytest.mark.gpu


def _context(arena_bytes, **env):
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


@pytest.fixture(scope="module")
def ctx():
    """Small requests batched too (RTG_SMALL=0): the batching tests below
    take sizes the small path would otherwise run alone."""
    c = _context(8 << 30, RTG_SMALL=0)
    yield c
    c.close()


def _dev(p):
    import torch
    return torch.from_numpy(np.ascontiguousarray(p, dtype=np.float32)).cuda()


def _requests(seed, count, dims=(3, 6, 12), n_lo=2, n_hi=4000):
    rng = np.random.default_rng(seed)
    out = []
    for q in range(count):
        d = int(rng.choice(dims))
        n = int(np.exp(rng.uniform(np.log(n_lo), np.log(n_hi))))
        p = workloads.uniform_points(n, d, seed=seed * 1000 + q)
        r = workloads.prm_radius(max(n, 3), d, 0.9 if d < 12 else 1.0)
        out.append(dict(points=p, r=r, k=int(rng.integers(2, 9)), alpha=2.0, seed=q,
                        flags=int(rng.choice([0, 0, 1, 2]))))
    return out


def _oracle(q):
    return oracle.rtg(q["points"], q["r"], q["k"], q["alpha"], q["seed"], q["flags"] & 3)


def _serve(ctx, reqs):
    """Submit every request, then collect every result (host arrays)."""
    tickets = []
    keep = []
    for q in reqs:
        p = _dev(q["points"])
        keep.append(p)
        t = ctx.submit(p, q["r"], q["k"], q["alpha"], q["seed"], q["flags"])
        assert t is not None
        tickets.append(t)
    out = []
    for t in tickets:
        res = ctx.wait(t, timeout_s=60)
        out.append(res.to_numpy())
        res.release()
    return out


def test_served_results_equal_oracle_and_lone_calls(ctx):
    reqs = _requests(1, 48)
    before = ctx.stats()
    got = _serve(ctx, reqs)
    after = ctx.stats()
    for q, (rp, col) in zip(reqs, got):
        ref = _oracle(q)
        assert np.array_equal(rp, ref.row_ptr) and np.array_equal(col, ref.col)
        res = ctx.all_pairs(_dev(q["points"]), q["r"], q["k"], q["alpha"], q["seed"], q["flags"])
        rp1, col1 = res.to_numpy()
        res.release()
        assert np.array_equal(rp, rp1) and np.array_equal(col, col1)
    served = after["served_requests"] - before["served_requests"]
    passes = after["served_batches"] - before["served_batches"]
    tiny = sum(len(q["points"]) <= 1 for q in reqs)
    assert served == len(reqs) - tiny
    assert passes < served, "requests submitted together were never batched"


def test_small_requests_on_an_idle_device_take_the_small_path():
    c = _context(8 << 30)
    try:
        # one at a time: each finds the device idle and runs on the small path
        small = _requests(11, 10, dims=(3, 6), n_lo=50, n_hi=1500)
        before = c.stats()
        for q in small:
            (rp, col), = _serve(c, [q])
            ref = _oracle(q)
            assert np.array_equal(rp, ref.row_ptr) and np.array_equal(col, ref.col)
        after = c.stats()
        assert after["served_small"] - before["served_small"] == len(small)
        # submitted together with larger ones: whichever path each takes,
        # the lists are the oracle's
        large = _requests(12, 12, dims=(12,), n_lo=500, n_hi=4000)
        more = _requests(13, 24, dims=(3, 6), n_lo=50, n_hi=1500)
        reqs = []
        for i, q in enumerate(more):
            reqs.append(q)
            if i % 2:
                reqs.append(large[i // 2])
        got = _serve(c, reqs)
        for q, (rp, col) in zip(reqs, got):
            ref = _oracle(q)
            assert np.array_equal(rp, ref.row_ptr) and np.array_equal(col, ref.col)
    finally:
        c.close()


def test_submit_copies_the_points(ctx):
    q = _requests(2, 1, dims=(6,), n_lo=3000, n_hi=3001)[0]
    p = _dev(q["points"])
    t = ctx.submit(p, q["r"], q["k"], q["alpha"], q["seed"], q["flags"])
    p.fill_(0.5)  # the caller reuses its buffer at once
    res = ctx.wait(t)
    rp, col = res.to_numpy()
    res.release()
    ref = _oracle(q)
    assert np.array_equal(rp, ref.row_ptr) and np.array_equal(col, ref.col)


def test_tiny_requests_and_ticket_lifetime(ctx):
    from paper_1409_8112_amd import rtg
    t0 = ctx.submit(_dev(np.zeros((0, 3), np.float32)), 0.1, 2, 2.0, 0)
    t1 = ctx.submit(_dev(np.full((1, 5), 0.25, np.float32)), 0.1, 2, 2.0, 0)
    for t, n in ((t0, 0), (t1, 1)):
        res = ctx.wait(t)
        assert res.n == n and res.nnz == 0
        again = ctx.poll(t)  # a collected ticket still names its result
        assert again.handle == res.handle and again.n == n
        res.release()
        with pytest.raises(rtg.RTGError) as e:
            ctx.poll(t)
        assert e.value.code == rtg.ENOENT
    with pytest.raises(rtg.RTGError) as e:
        ctx.poll(987654321)
    assert e.value.code == rtg.ENOENT


def test_bad_request_fails_alone(ctx):
    from paper_1409_8112_amd import rtg
    reqs = _requests(3, 10, dims=(6,), n_lo=200, n_hi=3000)
    bad = reqs[4]["points"].copy()
    bad[len(bad) // 2, 1] = np.inf
    reqs[4] = dict(reqs[4], points=bad)
    tickets = [ctx.submit(_dev(q["points"]), q["r"], q["k"], q["alpha"], q["seed"], q["flags"])
               for q in reqs]
    for i, (q, t) in enumerate(zip(reqs, tickets)):
        if i == 4:
            with pytest.raises(rtg.RTGError) as e:
                ctx.wait(t)
            assert e.value.code == rtg.EINVAL
            continue
        res = ctx.wait(t)
        rp, col = res.to_numpy()
        res.release()
        ref = _oracle(q)
        assert np.array_equal(rp, ref.row_ptr) and np.array_equal(col, ref.col)


def test_admission_by_memory_budget():
    """With a budget that holds about one request's working set at a time,
    requests run one after another and every result is still right; a
    request larger than the whole budget is refused at submit.  Finished
    results count against the budget until they are released, and a request
    that does not fit beside them waits for the release rather than fail."""
    from paper_1409_8112_amd import rtg
    c = _context(96 << 20)
    try:
        reqs = _requests(4, 6, dims=(3,), n_lo=60000, n_hi=80000)
        for q in reqs:
            q["k"] = 4
        got = _serve(c, reqs)
        for q, (rp, col) in zip(reqs, got):
            ref = _oracle(q)
            assert np.array_equal(rp, ref.row_ptr) and np.array_equal(col, ref.col)
        big = workloads.uniform_points(2_000_000, 3, seed=5)
        with pytest.raises(rtg.RTGError) as e:
            c.submit(_dev(big), 0.01, 8, 2.0, 0)
        assert e.value.code == rtg.ENOMEM
    finally:
        c.close()


def test_one_lane_and_small_batches():
    c = _context(4 << 30, RTG_LANES=1, RTG_BATCH_POINTS=5000)
    try:
        reqs = _requests(5, 20, dims=(2, 9))
        got = _serve(c, reqs)
        for q, (rp, col) in zip(reqs, got):
            ref = _oracle(q)
            assert np.array_equal(rp, ref.row_ptr) and np.array_equal(col, ref.col)
    finally:
        c.close()


def test_close_with_requests_in_flight():
    c = _context(2 << 30)
    reqs = _requests(6, 12, dims=(6,), n_lo=2000, n_hi=8000)
    keep = [_dev(q["points"]) for q in reqs]
    for q, p in zip(reqs, keep):
        assert c.submit(p, q["r"], q["k"], q["alpha"], q["seed"], q["flags"]) is not None
    c.close()  # must not hang; queued requests are dropped
