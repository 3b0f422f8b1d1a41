"""The autotuner: whatever launch settings it installs, or a caller sets,
the lists stay bit-exact with the oracle (settings change how the work is
launched, never what is computed); entries survive a JSON round trip; bad
entries and files are refused; rtg_tune_params returns parameters whose
modelled recall reaches the target, measured on the caller's points."""
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


def _batch(d, count, seed):
    rng = np.random.default_rng(seed)
    out = []
    for q in range(count):
        n = int(rng.integers(500, 20000))
        p = workloads.uniform_points(n, d, seed=seed * 100 + q)
        out.append(dict(host=p, points=_dev(p), r=workloads.prm_radius(n, d, 0.9), k=5,
                        alpha=2.0, seed=q, flags=0))
    return out


def _check(ctx, qs):
    res = ctx.all_pairs_batched(qs)
    for q, r in zip(qs, res):
        rp, col = r.to_numpy()
        ref = oracle.rtg(q["host"], q["r"], q["k"], q["alpha"], q["seed"])
        assert np.array_equal(rp, ref.row_ptr) and np.array_equal(col, ref.col)
    ctx.release_many(res)


def test_autotuned_batch_is_exact(ctx):
    qs = _batch(6, 12, 1)
    entry = ctx.autotune(qs, reps=1)
    print("tuned", entry, flush=True)
    assert entry["d"] == 6 and entry["ms"] > 0
    npts = sum(len(q["host"]) for q in qs)
    got = ctx.get_tuning(6, npts)
    for key in ("tests_per_wave", "unit_tiles", "part_threads", "bucket_blocks",
                "bucket_entries", "sort"):
        assert got[key] == entry[key]
    _check(ctx, qs)


@pytest.mark.parametrize("setting", [
    dict(tests_per_wave=1000, unit_tiles=4, part_threads=1024, bucket_blocks=1,
         bucket_entries=256, sort=0),
    dict(tests_per_wave=10_000_000, unit_tiles=64, part_threads=256, bucket_blocks=4096,
         bucket_entries=16384, sort=1),
])
def test_extreme_settings_are_exact(ctx, setting):
    qs = _batch(3, 6, 2)
    npts = sum(len(q["host"]) for q in qs)
    log2 = int(np.ceil(np.log2(npts)))
    ctx.set_tuning(dict(d=3, log2_points=log2, **setting))
    assert ctx.get_tuning(3, npts)["unit_tiles"] == setting["unit_tiles"]
    _check(ctx, qs)
    wl = workloads.small_uniform_d3()
    ctx.set_tuning(dict(d=3, log2_points=int(np.ceil(np.log2(wl.n))), **setting))
    res = ctx.all_pairs(_dev(wl.points()), wl.r, wl.k, wl.alpha, wl.seed)
    rp, col = res.to_numpy()
    res.release()
    ref = oracle.rtg(wl.points(), wl.r, wl.k, wl.alpha, wl.seed)
    assert np.array_equal(rp, ref.row_ptr) and np.array_equal(col, ref.col)


def test_tuning_file_round_trip_and_refusals(ctx, tmp_path):
    from paper_1409_8112_amd import rtg
    ctx.set_tuning(dict(d=9, log2_points=17, tests_per_wave=45000, unit_tiles=2,
                        part_threads=1024, bucket_blocks=128, bucket_entries=10240, sort=1))
    path = str(tmp_path / "tuning.json")
    ctx.save_tuning(path)
    c2 = rtg.Context(0, arena_bytes=1 << 30)
    try:
        c2.load_tuning(path)
        got = c2.get_tuning(9, 100_000)
        assert (got["tests_per_wave"], got["unit_tiles"], got["part_threads"],
                got["bucket_blocks"], got["bucket_entries"], got["sort"]) == (
                    45000, 2, 1024, 128, 10240, 1)
        with pytest.raises(rtg.RTGError) as e:
            c2.set_tuning(dict(d=9, log2_points=17, tests_per_wave=45000, unit_tiles=2,
                               part_threads=512, bucket_blocks=128, bucket_entries=10240, sort=1))
        assert e.value.code == rtg.EINVAL
        bad = tmp_path / "bad.json"
        bad.write_text(open(path).read().replace('"part_threads": 1024', '"part_threads": 3'))
        with pytest.raises(rtg.RTGError) as e:
            c2.load_tuning(str(bad))
        assert e.value.code == rtg.EINVAL
        with pytest.raises(rtg.RTGError) as e:
            c2.load_tuning(str(tmp_path / "missing.json"))
        assert e.value.code == rtg.ENOENT
    finally:
        c2.close()


def test_tuned_parameters_reach_the_modelled_target(ctx):
    from paper_1409_8112_amd import rtg
    n, d = 20000, 9
    p = workloads.uniform_points(n, d, seed=10)
    r = workloads.fmt_radius(n, d)
    k, alpha, rec, ms = ctx.tune_params(_dev(p), r, 0.98, reps=1)
    print(f"tuned parameters k={k} alpha={alpha} recall(model)={rec:.4f} {ms:.2f} ms", flush=True)
    assert rec >= 0.98 and rtg.model_recall(d, k, alpha) == pytest.approx(rec)
    assert 1 <= k <= 128 and 1.0 <= alpha <= 2.5
