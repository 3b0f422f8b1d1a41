"""The two-launch path for small instances (n <= 4096, n d <= 12288,
k n <= 12288, d <= 8, Euclidean): its lists equal the oracle's bit for bit
across dimensions, sizes, flags, both in-LDS sorts (counting over few
cells, bitonic over many), one to eight workgroups per grid (slices cut at
cell boundaries, with cells larger than a slice), coincident points and
pairs at r exactly and one ulp either side; it is the path that ran (no key kernel); and whatever it
cannot take -- keys wider than 31 bits, more pairs than its list holds
(131072), rows longer than 128 -- falls back to the general pipeline with
the same result, while bad points and out-of-range cells give the general
path's errors.  Lists of over 32768 entries are ordered in memory rather
than LDS."""
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


def _run(ctx, p, r, k, alpha, seed, flags=0):
    from paper_1409_8112_amd import rtg
    print(f"small: n={len(p)} d={p.shape[1]} r={r} k={k} alpha={alpha} flags={flags}", flush=True)
    res = ctx.all_pairs(_dev(p), r, k, alpha, seed, flags)
    rp, col = res.to_numpy()
    res.release()
    ref = oracle.rtg(p, r, k, alpha, seed, flags & 3)
    assert np.array_equal(rp, ref.row_ptr) and np.array_equal(col, ref.col)
    st = ctx.stats()
    small = st["kernel_launches"][rtg.KERNELS.index("keys")] == 0
    return small, st


@pytest.mark.parametrize("d", [1, 2, 3, 4, 5, 6, 7, 8])
def test_dimensions(ctx, d):
    n = 1500
    p = workloads.uniform_points(n, d, seed=40 + d)
    small, _ = _run(ctx, p, workloads.prm_radius(n, d, 1.0), 4, 2.0, d)
    assert small


@pytest.mark.parametrize("n", [2, 3, 63, 64, 65, 1000, 4095, 4096])
def test_sizes(ctx, n):
    p = workloads.uniform_points(n, 3, seed=n)
    small, _ = _run(ctx, p, 0.12, 3, 1.7, 2)
    assert small


def test_many_cells_bitonic_sort(ctx):
    # cells 0.03 wide: about 34 a side, 6 bits a field, 18 bits a cell --
    # past the counting sort's 12 -- with an 11-bit index: 29-bit keys
    p = workloads.uniform_points(2000, 3, seed=21)
    small, st = _run(ctx, p, 0.02, 4, 1.5, 5)
    assert small and st["cells"] > 0


def test_pairs_split_at_cell_boundaries(ctx):
    # With few grids each grid's pair tests are split over several
    # workgroups at cell boundaries.  One cell holding every point (all
    # slices but the last are empty), clusters larger than a slice, cells of
    # every size in between, and enough grids that each has one workgroup.
    rng = np.random.default_rng(44)
    one = (0.5 + rng.random((120, 3)) * 1e-4).astype(np.float32)
    small, st = _run(ctx, one, 0.01, 2, 2.0, 3)
    assert small and st["unique_pairs"] == 120 * 119 // 2
    centres = rng.random((10, 3))
    clusters = np.concatenate([c + rng.normal(size=(100, 3)) * 4e-3 for c in centres])
    small, _ = _run(ctx, clusters.astype(np.float32), 0.05, 4, 2.0, 8)
    assert small
    # k n <= 12288: fewer points as k grows (k > 32: fewer parts per grid;
    # k = 200: one workgroup per grid)
    for n, ks in ((1200, (1, 3, 8)), (180, (40, 64)), (90, (128,))):
        mixed = np.concatenate([workloads.uniform_points(n, 2, seed=45),
                                (0.3 + rng.random((n // 20, 2)) * 2e-3)]).astype(np.float32)
        for k in ks:
            small, _ = _run(ctx, mixed, 0.02 * (1200 / n) ** 0.5, k, 2.5, k)
            assert small
    small, _ = _run(ctx, workloads.uniform_points(50, 1, seed=46), 0.03, 200, 2.0, 5)
    assert small


def test_rows_under_the_limit(ctx):
    # a cluster of 100 points: rows of 99 entries, under the 128 the path takes
    rng = np.random.default_rng(6)
    p = np.concatenate([workloads.uniform_points(1000, 3, seed=6),
                        (0.5 + rng.normal(size=(100, 3)) * 1e-3)]).astype(np.float32)
    small, _ = _run(ctx, p, 0.05, 3, 2.0, 2)
    assert small


def test_lists_past_the_lds(ctx):
    from paper_1409_8112_amd import rtg
    # 13777 pairs: 27554 entries (in LDS) in both orientations; 3000 points
    # with 4 times the pairs: 110000 entries (in memory)
    p = workloads.uniform_points(1500, 2, seed=30)
    for flags in (0, rtg.UPPER_ONLY):
        small, st = _run(ctx, p, 0.07, 2, 2.0, 4, flags)
        assert small and 12288 < st["unique_pairs"] <= 16384
    p = workloads.uniform_points(3000, 2, seed=31)
    small, st = _run(ctx, p, 0.07, 2, 2.0, 4)
    assert small and st["unique_pairs"] > 40000


def test_workload_small_d3_all_flags(ctx):
    from paper_1409_8112_amd import rtg
    wl = workloads.small_uniform_d3()
    p = wl.points()
    for flags in (0, rtg.NO_ROTATE, rtg.UPPER_ONLY, rtg.NO_ROTATE | rtg.UPPER_ONLY,
                  rtg.DEDUP_SORT, rtg.DEDUP_BITMAP):
        small, st = _run(ctx, p, wl.r, wl.k, wl.alpha, wl.seed, flags)
        assert small and st["tests"] > 0 and st["cells"] > 0


def test_coincident_points_and_pairs_at_r(ctx):
    p = np.repeat(workloads.uniform_points(50, 4, seed=9), 7, axis=0)
    small, _ = _run(ctx, p, 0.07, 3, 2.0, 1)
    assert small
    # a lattice and its points moved by an ulp: pairs at exactly r and one ulp
    # either side (r = 0.3125 is exact in binary)
    rng = np.random.default_rng(17)
    gx, gy = np.meshgrid(np.arange(16), np.arange(16))
    base = np.stack([gx.ravel(), gy.ravel()], axis=1).astype(np.float32)
    q = base + np.array([3 * 0.0625, 4 * 0.0625], dtype=np.float32)
    steps = rng.integers(-1, 2, size=q.shape)
    q = np.where(steps > 0, np.nextafter(q, np.float32(np.inf)),
                 np.where(steps < 0, np.nextafter(q, np.float32(-np.inf)), q)).astype(np.float32)
    small, _ = _run(ctx, np.concatenate([base, q]), 0.3125, 4, 3.0, 11)
    assert small


def test_larger_instances_take_the_general_path(ctx):
    p = workloads.uniform_points(4097, 3, seed=3)
    small, _ = _run(ctx, p, 0.05, 3, 2.0, 0)
    assert not small
    p = workloads.uniform_points(500, 9, seed=3)
    small, _ = _run(ctx, p, 0.3, 3, 2.0, 0)
    assert not small
    p = workloads.uniform_points(1537, 8, seed=3)  # n d over 12288
    small, _ = _run(ctx, p, 0.4, 2, 2.0, 0)
    assert not small
    p = workloads.uniform_points(3000, 3, seed=3)  # k n over 12288
    small, _ = _run(ctx, p, 0.1, 5, 2.0, 0)
    assert not small


def test_wide_keys_fall_back(ctx):
    # d = 8 over a wide box with small cells: 8 fields of 8 bits and more
    p = (workloads.uniform_points(2000, 8, seed=5) * 200.0).astype(np.float32)
    small, _ = _run(ctx, p, 0.6, 2, 1.5, 3)
    assert not small


def test_many_pairs_fall_back(ctx):
    # about n^2 / 2 = 4.5e6 pairs within r: more than the small list holds
    p = workloads.uniform_points(3000, 2, seed=8)
    small, st = _run(ctx, p, 2.0, 2, 2.0, 1)
    assert not small and st["unique_pairs"] > 131072


def test_long_rows_fall_back(ctx):
    # a tight cluster of 300 points: rows of 299 entries
    rng = np.random.default_rng(4)
    p = np.concatenate([workloads.uniform_points(1000, 3, seed=4),
                        (0.5 + rng.normal(size=(300, 3)) * 1e-3)]).astype(np.float32)
    small, _ = _run(ctx, p, 0.05, 3, 2.0, 2)
    assert not small


def test_errors_match_the_general_path(ctx):
    from paper_1409_8112_amd import rtg
    p = workloads.uniform_points(100, 3, seed=1)
    p[17, 1] = np.nan
    with pytest.raises(rtg.RTGError) as e:
        ctx.all_pairs(_dev(p), 0.1, 3, 2.0, 0)
    assert e.value.code == rtg.EINVAL
    p = workloads.uniform_points(100, 3, seed=1)
    p[3, 0] = 3e38
    with pytest.raises(rtg.RTGError) as e:
        ctx.all_pairs(_dev(p), 1e-3, 3, 2.0, 0)
    assert e.value.code == rtg.ERANGE


def test_results_released_and_repeated(ctx):
    p = workloads.uniform_points(2000, 3, seed=12)
    outs = []
    for _ in range(3):
        res = ctx.all_pairs(_dev(p), 0.1, 4, 2.0, 7)
        outs.append(res.to_numpy())
        res.release()
    for rp, col in outs[1:]:
        assert np.array_equal(rp, outs[0][0]) and np.array_equal(col, outs[0][1])


def test_one_query_batches_and_plans(ctx):
    """A batch of one small query and a plan of one small instance take the
    two-launch path too (a plan then captures nothing) with the same lists."""
    from paper_1409_8112_amd import rtg
    p = workloads.uniform_points(1800, 4, seed=44)
    r = workloads.prm_radius(1800, 4, 1.0)
    q = dict(points=_dev(p), r=r, k=3, alpha=2.0, seed=9)
    ref = oracle.rtg(p, r, 3, 2.0, 9, 0)
    res = ctx.all_pairs_batched([q])
    rp, col = res[0].to_numpy()
    ctx.release_many(res)
    assert np.array_equal(rp, ref.row_ptr) and np.array_equal(col, ref.col)
    assert ctx.stats()["kernel_launches"][rtg.KERNELS.index("keys")] == 0
    plan = ctx.plan_create([q])
    try:
        for _ in range(3):
            res = plan.run([q])
            rp, col = res[0].to_numpy()
            ctx.release_many(res)
            assert np.array_equal(rp, ref.row_ptr) and np.array_equal(col, ref.col)
        assert plan.info()["captures"] == 0 and plan.info()["replays"] == 0
    finally:
        plan.destroy()
