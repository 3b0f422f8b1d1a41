"""Plans (rtg_plan_*): batched calls of one shape replayed from captured HIP
graphs.  Every run of a plan -- the sizing run, the capturing run and each
replay -- returns the oracle's lists for its own queries (new points, radii
and seeds on each run), with eager work of the program and synchronisations
between the replays; a shape other than the plan's is refused; timing the
captured kernels runs them as ordinary launches, still exact."""
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


def _shape(seed, count, dims=(3, 6), n_lo=2, n_hi=4000):
    """(n, d, k, flags) per query: the shape a plan is made for."""
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(count):
        d = int(rng.choice(dims))
        n = int(np.exp(rng.uniform(np.log(n_lo), np.log(n_hi))))
        out.append((n, d, int(rng.integers(1, 6)), int(rng.choice([0, 0, 1, 2]))))
    return out


def _queries(shape, run):
    """Queries of the given shape with this run's own points, radii, cell
    factors and seeds."""
    rng = np.random.default_rng(1000 + run)
    qs = []
    for i, (n, d, k, flags) in enumerate(shape):
        p = workloads.uniform_points(n, d, seed=run * 7919 + i)
        r = workloads.prm_radius(max(n, 3), d, float(rng.uniform(0.8, 1.0))) if n > 2 else 0.3
        qs.append(dict(host=p, points=_dev(p), r=r, k=k, alpha=float(rng.uniform(1.5, 2.2)),
                       seed=run * 31 + i, flags=flags))
    return qs


def _check(qs, res):
    for q, r in zip(qs, res):
        rp, col = r.to_numpy()
        ref = oracle.rtg(q["host"], q["r"], q["k"], q["alpha"], q["seed"], q["flags"] & 3)
        assert np.array_equal(rp, ref.row_ptr) and np.array_equal(col, ref.col), \
            (len(q["host"]), q["host"].shape[1], q["k"], q["flags"])


def _eager_work(ctx, run):
    """The program's own work between replays: a torch reduction and an
    unplanned batched call on the same context, each synchronised."""
    import torch
    x = torch.rand(1 << 20, device="cuda")
    assert float(x.sum()) > 0
    torch.cuda.synchronize()
    qs = _queries(_shape(50 + run, 3, dims=(2,), n_lo=100, n_hi=2000), 90 + run)
    res = ctx.all_pairs_batched(qs)
    _check(qs, res)
    ctx.release_many(res)


def test_every_run_of_a_plan_equals_the_oracle(ctx):
    shape = _shape(1, 16)
    plan = ctx.plan_create(_queries(shape, 0))
    try:
        for run in range(5):
            qs = _queries(shape, run)
            res = plan.run(qs)
            _check(qs, res)
            ctx.release_many(res)
            info = plan.info()
            print("run", run, info, flush=True)
            _eager_work(ctx, run)
        # run 0 sizes the workspaces, run 1 captures, later runs replay
        # (a run whose cell-key layout differs recaptures)
        assert info["workspace_bytes"] > 0
        assert info["captures"] >= 2          # two dimensions: two batches
        assert info["replays"] >= 2
    finally:
        plan.destroy()


def test_plan_of_several_batches_on_two_lanes():
    """A small point budget splits the queries into several batches, which
    two lanes take in turn: each batch keeps its own workspace and graph."""
    c = _ctx(RTG_BATCH_POINTS=6000)
    try:
        shape = _shape(2, 20, dims=(6,), n_lo=500, n_hi=3000)
        plan = c.plan_create(_queries(shape, 0))
        for run in range(4):
            qs = _queries(shape, 10 + run)
            res = plan.run(qs)
            _check(qs, res)
            c.release_many(res)
        info = plan.info()
        print(info, flush=True)
        assert info["captures"] >= 3 and info["replays"] >= 3
        plan.destroy()
    finally:
        c.close()


def test_plan_refuses_another_shape(ctx):
    from paper_1409_8112_amd import rtg
    shape = _shape(3, 4, dims=(3,), n_lo=50, n_hi=500)
    plan = ctx.plan_create(_queries(shape, 0))
    try:
        other = list(shape)
        n, d, k, f = other[1]
        other[1] = (n + 1, d, k, f)
        with pytest.raises(rtg.RTGError) as e:
            plan.run(_queries(other, 1))
        assert e.value.code == rtg.EINVAL
        with pytest.raises(rtg.RTGError):
            plan.run(_queries(shape[:3], 1))
        qs = _queries(shape, 2)               # the plan still works
        res = plan.run(qs)
        _check(qs, res)
        ctx.release_many(res)
    finally:
        plan.destroy()


def test_timed_plan_runs_without_the_graph(ctx):
    from paper_1409_8112_amd import rtg
    shape = _shape(4, 6, dims=(6,), n_lo=1000, n_hi=4000)
    plan = ctx.plan_create(_queries(shape, 0))
    try:
        for run in range(2):
            res = plan.run(_queries(shape, run))
            ctx.release_many(res)
        before = plan.info()
        ctx.set_timing(1 << rtg.KERNELS.index("keys"))
        try:
            qs = _queries(shape, 5)
            res = plan.run(qs)
            st = ctx.stats()
        finally:
            ctx.set_timing(0)
        _check(qs, res)
        ctx.release_many(res)
        assert plan.info()["replays"] == before["replays"]
        assert st["kernel_ms"][rtg.KERNELS.index("keys")] > 0
        qs = _queries(shape, 6)               # untimed again: replayed
        res = plan.run(qs)
        _check(qs, res)
        ctx.release_many(res)
        assert plan.info()["replays"] + plan.info()["captures"] > \
            before["replays"] + before["captures"]
    finally:
        plan.destroy()
