"""rtg_all_pairs_noalloc -- the entry point for callers that cannot
allocate -- against rtg_all_pairs on the same inputs, through the C-ABI:
calls in a row, each smaller than the one before, every output compared
element by element; a too-small col buffer and the size limit fail cleanly
and leave the next call correct."""
import numpy as np
import pytest

from paper_1409_8112_amd import workloads

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    import torch
    from paper_1409_8112_amd import rtg
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    c = rtg.Context(0, arena_bytes=4 << 30)
    yield c
    c.close()


def _dev(p):
    import torch
    return torch.from_numpy(np.ascontiguousarray(p, dtype=np.float32)).cuda()


def _reference(ctx, pts, r, k, alpha, seed, flags):
    res = ctx.all_pairs(pts, r, k, alpha, seed, flags)
    rp, col = res.to_numpy()
    res.release()
    return rp, col


def _noalloc(ctx, pts, r, k, alpha, seed, flags, capacity):
    import torch
    n = pts.shape[0]
    rp = torch.full((n + 1,), -7, dtype=torch.int64, device="cuda:0")
    col = torch.full((capacity,), -7, dtype=torch.int32, device="cuda:0")
    nnz = ctx.all_pairs_noalloc(pts, r, k, alpha, seed, rp, col, flags)
    return nnz, rp.cpu().numpy(), col.cpu().numpy()


def test_noalloc_equals_all_pairs_on_calls_in_a_row(ctx):
    from paper_1409_8112_amd import rtg
    cases = [
        (workloads.uniform_points(120_000, 6, seed=31),
         workloads.calibrate_radius_uniform(120_000, 6, 20.0), 8, 2.0, 3, 0),
        (workloads.uniform_points(20_000, 9, seed=32),
         workloads.calibrate_radius_uniform(20_000, 9, 15.0), 6, 2.0, 4, rtg.UPPER_ONLY),
        (workloads.small_uniform_d3().points(), 0.1, 4, 2.0, 0, 0),
    ]
    for p, r, k, alpha, seed, flags in cases:
        print(f"noalloc n={len(p)} d={p.shape[1]} k={k} flags={flags}", flush=True)
        pts = _dev(p)
        rp_ref, col_ref = _reference(ctx, pts, r, k, alpha, seed, flags)
        spare = 17
        nnz, rp, col = _noalloc(ctx, pts, r, k, alpha, seed, flags, len(col_ref) + spare)
        assert nnz == len(col_ref)
        assert np.array_equal(rp, rp_ref)
        assert np.array_equal(col[:nnz], col_ref)
        assert np.all(col[nnz:] == -7), "wrote past the entries"


def test_small_col_buffer_and_size_limit(ctx):
    from paper_1409_8112_amd import rtg
    wl = workloads.small_uniform_d3()
    pts = _dev(wl.points())
    rp_ref, col_ref = _reference(ctx, pts, wl.r, wl.k, wl.alpha, wl.seed, 0)
    with pytest.raises(rtg.RTGError) as e:
        _noalloc(ctx, pts, wl.r, wl.k, wl.alpha, wl.seed, 0, len(col_ref) - 1)
    assert e.value.code == rtg.ENOMEM and e.value.needed == len(col_ref)
    big = _dev(workloads.uniform_points(4_000_000, 3, seed=33))
    with pytest.raises(rtg.RTGError) as e:
        _noalloc(ctx, big, 0.01, 8, 2.0, 0, 0, 16)
    assert e.value.code == rtg.ENOMEM
    # the call after the refusals is right
    nnz, rp, col = _noalloc(ctx, pts, wl.r, wl.k, wl.alpha, wl.seed, 0, len(col_ref))
    assert nnz == len(col_ref) and np.array_equal(rp, rp_ref) and np.array_equal(col, col_ref)


def test_empty_and_single_point(ctx):
    import torch
    for n in (0, 1):
        pts = torch.zeros((n, 3), dtype=torch.float32, device="cuda:0")
        nnz, rp, col = _noalloc(ctx, pts, 0.1, 4, 2.0, 0, 0, 0)
        assert nnz == 0 and np.array_equal(rp, np.zeros(n + 1, dtype=np.int64))
