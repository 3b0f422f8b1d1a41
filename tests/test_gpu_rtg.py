"""Parity of the HIP path with the CPU oracle, through the C-ABI.

Bit-exact comparisons: integer cell coordinates, and the whole CSR neighbour
list (row_ptr and col) -- the pair set is integer output, so the bar is
equality, and the FP32 screen with its FP64 band must not change a single
decision.  At the full benchmark sizes the oracle is too slow for the whole
list; there every row of a seeded sample is compared exactly with the
oracle's row, and the rest is checked by properties that hold at any size."""
import json
import os

import numpy as np
import pytest

import oracle
from paper_1409_8112_amd import workloads
from tests.exact import check_csr

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    """A context whose small instances also take the general pipeline (the
    two-launch small path has its own tests, test_gpu_small.py)."""
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


def _dev(points):
    import torch
    return torch.from_numpy(np.ascontiguousarray(points, dtype=np.float32)).cuda()


def _gpu(ctx, points, r, k, alpha, seed, flags=0):
    res = ctx.all_pairs(_dev(points), r, k, alpha, seed, flags)
    rp, col = res.to_numpy()
    res.release()
    return rp, col


def _assert_same(rp, col, ref):
    assert np.array_equal(rp, ref.row_ptr), "row_ptr differs"
    assert np.array_equal(col, ref.col), "col differs"


def _say(msg):
    print(msg, flush=True)


# --- stage parity: cell coordinates ------------------------------------------

def _near_face_points(n, d, c, u, rng):
    """Points whose shift-only cell coordinate y = p/c + u lies within a few
    float32 ulps of an integer, on both sides."""
    m = rng.integers(-20, 20, size=(n, d))
    base = ((m - u[None, :]) * c).astype(np.float32)
    jitter = rng.integers(-3, 4, size=(n, d))
    return _ulp_shift(base, jitter)


def _ulp_shift(x, steps):
    out = x.copy()
    for s in range(1, 4):
        up = steps >= s
        dn = steps <= -s
        out[up] = np.nextafter(out[up], np.float32(np.inf))
        out[dn] = np.nextafter(out[dn], np.float32(-np.inf))
    return out


@pytest.mark.parametrize("d", [1, 2, 3, 5, 6, 9, 12, 16, 17, 33, 64])
def test_cell_coords_bit_exact(ctx, d):
    _say(f"cell coords d={d}")
    rng = np.random.default_rng(d)
    r, alpha = 0.05, 1.7
    p = workloads.uniform_points(5000, d, seed=d)
    R, u = oracle.make_transforms(3, 2, d)
    for t in range(2):
        got = ctx.debug_cell_coords(_dev(p), r, alpha, R[t], u[t])
        ref = oracle.cell_coords(p, R[t], u[t], 1.0 / (alpha * r))
        assert np.array_equal(got, ref)
    # shift-only grid, points a few ulps either side of a cell face
    Ri, ui = oracle.make_transforms(4, 1, d, oracle.NO_ROTATE)
    q = _near_face_points(3000, d, alpha * r, ui[0], rng)
    got = ctx.debug_cell_coords(_dev(q), r, alpha, Ri[0], ui[0])
    ref = oracle.cell_coords(q, Ri[0], ui[0], 1.0 / (alpha * r))
    assert np.array_equal(got, ref)


# --- whole-output parity --------------------------------------------------------

def test_small_uniform_d3_bit_exact(ctx):
    wl = workloads.small_uniform_d3()
    _say(f"workload {wl.name}")
    p = wl.points()
    from paper_1409_8112_amd import rtg
    for flags in (0, oracle.NO_ROTATE, oracle.UPPER_ONLY):
        ref = oracle.rtg(p, wl.r, wl.k, wl.alpha, wl.seed, flags)
        for dedup in (0, rtg.DEDUP_SORT):
            rp, col = _gpu(ctx, p, wl.r, wl.k, wl.alpha, wl.seed, flags | dedup)
            _assert_same(rp, col, ref)
    bf = oracle.bruteforce(p, wl.r)
    recall = len(ref.col) / max(1, len(bf.col) // 2)
    _say(f"recall vs brute force {recall:.4f}")


@pytest.mark.parametrize("n", [2, 3, 63, 64, 65, 127, 4095, 4096, 4097, 8193])
def test_ragged_sizes(ctx, n):
    _say(f"ragged n={n}")
    p = workloads.uniform_points(n, 3, seed=n)
    r = 0.6 * (8.0 / max(n, 8)) ** (1 / 3)
    rp, col = _gpu(ctx, p, r, 3, 2.0, n)
    ref = oracle.rtg(p, r, 3, 2.0, n)
    _assert_same(rp, col, ref)


@pytest.mark.parametrize("d", list(range(1, 17)) + [20, 33, 64])
def test_dimensions(ctx, d):
    _say(f"dimension d={d}")
    n = 3000
    p = workloads.uniform_points(n, d, seed=100 + d)
    r = workloads.calibrate_radius_uniform(n, d, 10.0)
    rp, col = _gpu(ctx, p, r, 4, 1.5, d)
    ref = oracle.rtg(p, r, 4, 1.5, d)
    _assert_same(rp, col, ref)
    if d <= 16:
        assert len(ref.col) > 0


def test_clustered_d12_small(ctx):
    _say("clustered d=12 n=20000")
    p = workloads.clustered_points(20000, 12, seed=5)
    r = 0.04
    ref = oracle.rtg(p, r, 8, 2.0, 0)
    from paper_1409_8112_amd import rtg
    for dedup in (0, rtg.DEDUP_SORT):
        rp, col = _gpu(ctx, p, r, 8, 2.0, 0, dedup)
        _assert_same(rp, col, ref)


def test_grids_in_several_sorts(ctx):
    """d = 31 with alpha = 0.6 needs two key bits per axis (62 bits), so the
    six grids are split over several sorts; the first-owner rule must look
    back across sorts."""
    from paper_1409_8112_amd import rtg
    d, n = 31, 4000
    p = workloads.clustered_points(n, d, seed=2, n_clusters=8, sigma=0.03)
    r = 0.3
    ref = oracle.rtg(p, r, 6, 0.6, 4)
    for dedup in (0, rtg.DEDUP_SORT):
        rp, col = _gpu(ctx, p, r, 6, 0.6, 4, dedup)
        _assert_same(rp, col, ref)
        assert ctx.stats()["transforms_per_sort"] < 6
    assert len(ref.col) > 0


def test_one_huge_cell_many_tiles(ctx):
    """All 3000 points in one cell: 47 tiles of 64, 1128 tile pairs."""
    _say("one huge cell")
    n, d, r = 3000, 3, 0.08
    p = workloads.uniform_points(n, d, seed=9)
    R, u = oracle.make_transforms(0, 64, d)
    t = next(t for t in range(64) if np.all((u[t] > 0.01) & (u[t] < 0.99)))
    res = ctx.all_pairs_with_transforms(_dev(p), r, 1e4, R[t:t + 1], u[t:t + 1])
    rp, col = res.to_numpy()
    res.release()
    _assert_same(rp, col, oracle.bruteforce(p, r))


def test_coincident_points(ctx):
    p = np.repeat(workloads.uniform_points(50, 2, seed=1), 7, axis=0)
    rp, col = _gpu(ctx, p, 0.02, 2, 2.0, 3)
    _assert_same(rp, col, oracle.rtg(p, 0.02, 2, 2.0, 3))


def test_hand_examples(ctx, golden_dir):
    with open(os.path.join(golden_dir, "hand_examples.json")) as f:
        cases = json.load(f)["cases"]
    for case in cases:
        p = np.array(case["points"], dtype=np.float32)
        R = np.array(case["R"], dtype=np.float64)[None]
        u = np.array(case["u"], dtype=np.float64)[None]
        res = ctx.all_pairs_with_transforms(_dev(p), case["r"], case["alpha"], R, u,
                                            oracle.UPPER_ONLY)
        rp, col = res.to_numpy()
        res.release()
        rows = np.repeat(np.arange(len(p)), np.diff(rp))
        assert [[int(a), int(b)] for a, b in zip(rows, col)] == case["pairs"], case["name"]


def test_distance_band_decisions(ctx):
    """Pairs at squared distance exactly r^2 in FP64 and one float32 ulp
    either side: the FP32 screen puts them in the band and the FP64 re-test
    must decide each as the definition does."""
    _say("distance band")
    rng = np.random.default_rng(7)
    r = 0.3125  # 5 * 2^-4: offsets (3s, 4s) with s = 2^-4 are exactly r long
    gx, gy = np.meshgrid(np.arange(20), np.arange(20))
    base = np.stack([gx.ravel(), gy.ravel()], axis=1).astype(np.float32)  # 1 apart
    q = base + np.array([3 * 0.0625, 4 * 0.0625], dtype=np.float32)
    q = _ulp_shift(q.astype(np.float32), rng.integers(-1, 2, size=q.shape))
    p = np.concatenate([base, q]).astype(np.float32)
    R, u = oracle.make_transforms(11, 4, 2, oracle.NO_ROTATE)
    res = ctx.all_pairs_with_transforms(_dev(p), r, 50.0, R, u)
    rp, col = res.to_numpy()
    res.release()
    ref = oracle.rtg_with_transforms(p, r, 50.0, R, u)
    _assert_same(rp, col, ref)
    assert len(ref.col) > 0
    st = ctx.stats()
    assert st["band_rechecks"] > 0


def test_aliased_cells_are_never_reported(ctx):
    """d = 12 over a wide box needs more key bits than a 64-bit key holds, so
    cells that agree in the low bits of every axis share a key; such points
    are at least (2^b - 1) alpha r apart and must not be reported."""
    _say("aliasing")
    d, n, r, alpha = 12, 6000, 0.5, 2.0
    rng = np.random.default_rng(3)
    p = (rng.random((n, d)) * 400.0).astype(np.float32)
    # twins 2^5 and 2^6 cells apart on axis 0 under the identity grid
    twins = p[:200].copy()
    twins[:, 0] += np.float32(32 * alpha * r)
    near = p[:300].copy()
    near[:, 3] += np.float32(0.3 * r)
    p = np.concatenate([p, twins, near]).astype(np.float32)
    R, u = oracle.make_transforms(8, 4, d, oracle.NO_ROTATE)
    res = ctx.all_pairs_with_transforms(_dev(p), r, alpha, R, u)
    rp, col = res.to_numpy()
    res.release()
    ref = oracle.rtg_with_transforms(p, r, alpha, R, u)
    _assert_same(rp, col, ref)
    assert len(ref.col) > 0
    st = ctx.stats()
    assert st["key_bits"] <= 64
    # each twin shares a key with its original under every grid, so at least
    # those 4 x 200 aliased pairs were tested and rejected
    assert st["tests"] >= 4 * 200


def test_empty_and_single_point(ctx):
    for n in (0, 1):
        rp, col = _gpu(ctx, np.zeros((n, 4), np.float32) + 0.5, 0.1, 2, 2.0, 0)
        assert rp.tolist() == [0] * (n + 1) and len(col) == 0


def test_invalid_arguments(ctx):
    import torch
    from paper_1409_8112_amd import rtg
    p = workloads.uniform_points(100, 3, seed=0)
    bad = p.copy()
    bad[17, 1] = np.nan
    cases = [
        (lambda: ctx.all_pairs(_dev(bad), 0.1, 2, 2.0, 0), rtg.EINVAL),
        (lambda: ctx.all_pairs(_dev(p), 0.0, 2, 2.0, 0), rtg.EINVAL),
        (lambda: ctx.all_pairs(_dev(p), 0.1, 0, 2.0, 0), rtg.EINVAL),
        (lambda: ctx.all_pairs(_dev(p), 0.1, 2, -1.0, 0), rtg.EINVAL),
        (lambda: ctx.all_pairs(_dev(p), 1e-40, 2, 2.0, 0), rtg.ERANGE),
        (lambda: ctx.all_pairs(_dev(p * np.float32(1e9)), 1e-3, 2, 2.0, 0), rtg.ERANGE),
    ]
    for fn, code in cases:
        with pytest.raises(rtg.RTGError) as e:
            fn()
        assert e.value.code == code
    # a host pointer is refused before any kernel runs
    host = torch.from_numpy(p)
    out = rtg.rtg_csr()
    rc = rtg.lib().rtg_all_pairs(ctx.h, host.data_ptr(), 100, 3, 0.1, 2, 2.0, 0, 0, out)
    assert rc == rtg.EINVAL
    # the context still works afterwards
    rp, col = _gpu(ctx, p, 0.2, 2, 2.0, 0)
    _assert_same(rp, col, oracle.rtg(p, 0.2, 2, 2.0, 0))


def test_onesweep_sort_matches(ctx):
    """The onesweep radix sort (RTG_SORT=onesweep) gives the same lists as the
    default reduce-then-scan sort."""
    from paper_1409_8112_amd import rtg
    os.environ["RTG_SORT"] = "onesweep"
    try:
        other = rtg.Context(0, arena_bytes=4 << 30)
    finally:
        del os.environ["RTG_SORT"]
    try:
        for n, d, r in [(5000, 3, 0.06), (20000, 6, 0.3)]:
            p = workloads.uniform_points(n, d, seed=n + d)
            res = other.all_pairs(_dev(p), r, 4, 2.0, 1)
            rp, col = res.to_numpy()
            res.release()
            _assert_same(rp, col, oracle.rtg(p, r, 4, 2.0, 1))
    finally:
        other.close()


def test_oversized_buckets_take_the_global_sort(ctx):
    """Neighbour-list buckets too large for LDS are sorted by the global radix
    sort; a context with a tiny bucket capacity sends most buckets there."""
    from paper_1409_8112_amd import rtg
    os.environ["RTG_BUCKET_CAP"] = "40"
    try:
        other = rtg.Context(0, arena_bytes=4 << 30)
    finally:
        del os.environ["RTG_BUCKET_CAP"]
    try:
        p = workloads.uniform_points(6000, 3, seed=77)
        for flags in (0, oracle.UPPER_ONLY, rtg.DEDUP_SORT):
            res = other.all_pairs(_dev(p), 0.08, 4, 2.0, 5, flags)
            rp, col = res.to_numpy()
            res.release()
            _assert_same(rp, col, oracle.rtg(p, 0.08, 4, 2.0, 5, flags & ~rtg.DEDUP_SORT))
    finally:
        other.close()


def test_dense_rows_contiguous_in_index_order(ctx):
    """Clustered points ordered along one axis put the heavy rows side by
    side, so several neighbour-list buckets overflow LDS at once; they share
    one global sort.  Also with a bucket capacity that only some exceed."""
    from paper_1409_8112_amd import rtg
    p = workloads.clustered_points(12000, 3, seed=9, n_clusters=8, sigma=0.03)
    p = p[np.argsort(p[:, 0], kind="stable")]
    ref = oracle.rtg(p, 0.06, 4, 2.0, 1)
    res = ctx.all_pairs(_dev(p), 0.06, 4, 2.0, 1)
    rp, col = res.to_numpy()
    res.release()
    _assert_same(rp, col, ref)
    os.environ["RTG_BUCKET_CAP"] = "3000"
    try:
        other = rtg.Context(0, arena_bytes=4 << 30)
    finally:
        del os.environ["RTG_BUCKET_CAP"]
    try:
        for flags in (0, oracle.UPPER_ONLY):
            res = other.all_pairs(_dev(p), 0.06, 4, 2.0, 1, flags)
            rp, col = res.to_numpy()
            res.release()
            _assert_same(rp, col, oracle.rtg(p, 0.06, 4, 2.0, 1, flags))
    finally:
        other.close()


@pytest.mark.parametrize("env", [{"RTG_UNITS": "roundrobin"}, {"RTG_PAIR_BLOCKS": "7"},
                                 {"RTG_PAIR_BLOCKS": "60000"},
                                 {"RTG_PAIR_BLOCKS": "3", "RTG_PAIRS": "vector"}])
def test_wave_work_assignment(env):
    """Pair-kernel waves dealt units round-robin, a tiny grid (long runs of
    units per wave) and a grid far larger than the work (many empty runs):
    the same lists as the oracle."""
    from paper_1409_8112_amd import rtg
    old = {k: os.environ.get(k) for k in env}
    os.environ.update(env)
    try:
        other = rtg.Context(0, arena_bytes=4 << 30)
    finally:
        for k, v in old.items():
            if v is None:
                del os.environ[k]
            else:
                os.environ[k] = v
    try:
        cases = [(workloads.uniform_points(3000, 6, seed=41), 6, 0.3),
                 (workloads.clustered_points(5000, 3, seed=42), 3, 0.05),
                 (workloads.uniform_points(700, 2, seed=43), 2, 0.08)]
        for p, d, r in cases:
            print(f"work assignment {env}: n={len(p)} d={d}", flush=True)
            res = other.all_pairs(_dev(p), r, 5, 2.0, 3)
            rp, col = res.to_numpy()
            res.release()
            _assert_same(rp, col, oracle.rtg(p, r, 5, 2.0, 3))
    finally:
        other.close()


def test_sparse_acceptance_fits_a_small_budget():
    """At d = 12 with cells as wide as the cube, about 1e10 pairs are tested
    for about 1e7 within r: the room first taken for the pairs must follow
    the points, not the tests, or a 4 GB context cannot run it."""
    from paper_1409_8112_amd import rtg
    c = rtg.Context(0, arena_bytes=4 << 30)
    try:
        n, r = 1_000_000, 0.45
        p = workloads.uniform_points(n, 12, seed=12)
        print("sparse acceptance: n=1e6 d=12", flush=True)
        res = c.all_pairs(_dev(p), r, 8, 2.0, 4)
        st = c.stats()
        rp, col = res.to_numpy()
        res.release()
        assert st["tests"] > 1000 * st["unique_pairs"] > 0
        R, u = oracle.make_transforms(4, 8, 12)
        rows = np.random.default_rng(5).choice(n, size=24, replace=False)
        for s_i, row in zip(range(len(rows)), oracle.rtg_rows(p, r, 2.0, R, u, rows)):
            assert np.array_equal(col[rp[rows[s_i]]:rp[rows[s_i] + 1]], row)
    finally:
        c.close()


def test_release_and_determinism(ctx):
    from paper_1409_8112_amd import rtg
    p = workloads.uniform_points(20000, 4, seed=2)
    a = ctx.all_pairs(_dev(p), 0.05, 4, 2.0, 1)
    b = ctx.all_pairs(_dev(p), 0.05, 4, 2.0, 1)
    ra, ca = a.to_numpy()
    rb, cb = b.to_numpy()
    assert np.array_equal(ra, rb) and np.array_equal(ca, cb)
    a.release()
    with pytest.raises(rtg.RTGError) as e:
        ctx.release(a.handle)
    assert e.value.code == rtg.ENOENT
    b.release()


# --- full benchmark sizes: sampled rows + properties ----------------------------

def _check_full(ctx, wl, nsample):
    import torch
    p = wl.points()
    _say(f"full size {wl.name}: GPU")
    res = ctx.all_pairs(_dev(p), wl.r, wl.k, wl.alpha, wl.seed)
    rp, col = res.to_numpy()
    res.release()
    n = wl.n
    _say(f"  pairs {len(col) // 2}; layout checks")
    assert rp.shape == (n + 1,) and rp[0] == 0 and rp[-1] == len(col)
    rows = np.repeat(np.arange(n, dtype=np.int64), np.diff(rp))
    c64 = col.astype(np.int64)
    assert np.all(c64 != rows)
    same = rows[1:] == rows[:-1]
    assert np.all(c64[1:][same] > c64[:-1][same])
    # symmetry: the (row, col) and (col, row) multisets agree
    fwd = rows * n + c64
    bwd = c64 * n + rows
    assert np.array_equal(np.sort(fwd), np.sort(bwd))
    # every reported pair is within r (FP64 sum in axis order)
    s = np.zeros(len(col))
    for l in range(wl.d):
        dl = p[rows, l].astype(np.float64) - p[c64, l].astype(np.float64)
        s = s + dl * dl
    assert np.all(s <= wl.r * wl.r)
    # sampled rows, each computed by the oracle on its own
    _say(f"  oracle rows x{nsample}")
    R, u = oracle.make_transforms(wl.seed, wl.k, wl.d)
    sample = np.random.default_rng(1234).choice(n, size=nsample, replace=False)
    ref = oracle.rtg_rows(p, wl.r, wl.alpha, R, u, sample)
    for s_i, row in enumerate(sample):
        assert np.array_equal(col[rp[row]:rp[row + 1]], ref[s_i]), f"row {row}"


def test_full_size_uniform_d6_sampled(ctx):
    _check_full(ctx, workloads.large_uniform_d6(), 256)


def test_full_size_clustered_d12_sampled(ctx):
    _check_full(ctx, workloads.skewed_clustered_d12(), 48)


def test_too_few_key_bits_is_out_of_range(ctx):
    """d = 40 with alpha = 0.6 needs 2 bits per axis to keep aliased cells
    apart (80 > 64 bits): the library refuses with RTG_ERANGE, as declared,
    rather than report pairs from keys that could not separate cells."""
    from paper_1409_8112_amd import rtg
    _say("too few key bits d=40 alpha=0.6")
    p = workloads.clustered_points(3000, 40, seed=12, n_clusters=6, sigma=0.04)
    with pytest.raises(rtg.RTGError) as e:
        _gpu(ctx, p, 0.35, 5, 0.6, 2)
    assert e.value.code == rtg.ERANGE


@pytest.mark.parametrize("alpha", [0.8, 1.0, 1.02, 3.0])
def test_signature_widths(ctx, alpha):
    """alpha below ~1 needs 2 signature bits per axis, above 1.01 one bit."""
    _say(f"signature widths alpha={alpha}")
    d, n = 5, 4000
    p = workloads.uniform_points(n, d, seed=int(alpha * 100))
    r = workloads.calibrate_radius_uniform(n, d, 12.0)
    ref = oracle.rtg(p, r, 7, alpha, 9)
    rp, col = _gpu(ctx, p, r, 7, alpha, 9)
    _assert_same(rp, col, ref)


def test_long_rows_in_lists(ctx):
    """Tight clusters of 40, 150, 700 and 1500 points (every pair within r)
    in a sparse background give neighbour rows of every length the list
    build distinguishes: counted in place, sorted by one wave, and rows too
    long for LDS (their bucket takes the global sort)."""
    _say("long rows")
    rng = np.random.default_rng(21)
    d, r = 4, 0.05
    parts = [rng.random((6000, d))]
    for size in (40, 150, 700, 1500):
        centre = rng.random(d) * 0.8 + 0.1
        parts.append(centre + (rng.random((size, d)) - 0.5) * (0.6 * r / np.sqrt(d)))
    p = np.concatenate(parts).astype(np.float32)
    p = p[rng.permutation(len(p))]
    ref = oracle.rtg(p, r, 3, 2.0, 5)
    rp, col = _gpu(ctx, p, r, 3, 2.0, 5)
    _assert_same(rp, col, ref)
    assert np.diff(ref.row_ptr).max() >= 1499
