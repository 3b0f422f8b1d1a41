#!/usr/bin/env python
"""Throughput of all-pairs r-NN by randomly transformed grids on one MI355X.

One step = one rtg_all_pairs call through the C-ABI over the whole pipeline
(stage, FP64 cell keys, key sort, cells, pair tests, pair sort + unique,
symmetric CSR) on points already resident in HBM; the result stays on the
device.  Value = unique neighbour pairs reported per second.

Default workload: n = 1e6 points uniform in [0,1]^6 (FP32), k = 8 grids,
alpha = 2, r for ~20 mean neighbours, seed 0.

Prints one JSON line.  Besides throughput it carries:
  roofline      the dominant kernel's algorithmic bytes (or flops) per launch
                over its average launch time, timed live with HIP events on
                the library's stream during the timed steps; the pair kernel
                counts 2d FP32 flops per tested pair (a difference, a square
                and a sum per coordinate, the square and sum fused);
  phases        per pipeline phase (key, key sort, cells, pairs, lists):
                algorithmic bytes, device time and the fraction of HBM peak;
  configs       the small d3 and the clustered d12 workloads, each timed the
                same way (ms, pairs/s, pair-kernel roofline, phases);
  cpu_baseline  the CPU oracle on the same workload, single-threaded, and on
                a sample of the batched instances over every host core.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0      # MI355X HBM3E, GB/s
FP32_VEC_PEAK_TFLOPS = 157.3  # MI355X FP32 vector and FP32 matrix (dense) peak
FP64_VEC_PEAK_TFLOPS = 78.6   # MI355X FP64 vector peak

# kernel ids whose launches are single kernels (candidates for the roofline)
SINGLE_KERNELS = {"keys": "k_keys", "key_hist": "k_radix_hist", "key_scatter": "k_radix_scatter<true>",
                  "pairs": "k_cell_pairs", "pair_hist": "k_radix_hist",
                  "pair_scatter": "k_radix_scatter<false>", "stage": "k_stage",
                  "gather": "k_gather_units", "compact": "k_seg_compact"}


def measured_traffic(kernel_name: str, summary: str = "k_cell_pairs_uniform_n1e6_d6_traffic.txt"):
    """HBM bytes per launch of the dominant kernel from the committed counter
    summary, or None when it is missing, names another kernel, or the kernel
    source changed since the counters were taken."""
    import hashlib
    path = os.path.join(ROOT, "profiles", summary)
    src = os.path.join(ROOT, "paper_1409_8112_amd", "csrc", "rtg_kernels.hip")
    try:
        kv = {}
        for line in open(path):
            if "=" in line and not line.lstrip().startswith("#"):
                k, v = line.split("=", 1)
                kv[k.strip()] = v.strip()
        sha = hashlib.sha256(open(src, "rb").read()).hexdigest()
    except OSError:
        return None
    if kv.get("source_sha256") != sha or not kernel_name.startswith(kv.get("kernel", "?")[:12]):
        return None
    return float(kv["traffic_bytes_per_launch"])


def workload_by_name(name):
    from paper_1409_8112_amd import workloads
    return {"uniform_d6": workloads.large_uniform_d6,
            "small_d3": workloads.small_uniform_d3,
            "clustered_d12": workloads.skewed_clustered_d12}[name]()


def cpu_baseline(points, wl, budget_s: float):
    """The oracle (test infrastructure) timed on this host, one thread."""
    import oracle
    t0 = time.perf_counter()
    res = oracle.rtg(points, wl.r, wl.k, wl.alpha, wl.seed)
    dt = time.perf_counter() - t0
    pairs = len(res.col) // 2
    return {"value": pairs / dt, "unit": "pairs/s", "cores": 1, "kind": "oracle",
            "sample": f"the whole workload ({wl.name}), single-threaded C oracle, {dt:.1f} s",
            "seconds": dt, "pairs": pairs}


def _oracle_pairs(wl):
    """Pairs the oracle reports for one batched instance (a pool worker)."""
    import oracle
    pts = wl.points()
    t0 = time.perf_counter()
    res = oracle.rtg(pts, wl.r, wl.k, wl.alpha, wl.seed)
    return len(res.col) // 2, time.perf_counter() - t0


def cpu_baseline_all_cores(count: int = 4096, sample: int = 512) -> dict:
    """The oracle on every host core: the first `sample` of the batched
    instances, one instance per task over a process pool (instances are
    independent, so nothing is merged)."""
    from concurrent.futures import ProcessPoolExecutor
    from paper_1409_8112_amd import workloads
    cores = max(1, min(16, os.cpu_count() or 1))
    specs = workloads.batched_instances(count)[:sample]
    import multiprocessing
    with ProcessPoolExecutor(max_workers=cores, mp_context=multiprocessing.get_context("fork")) as ex:
        list(ex.map(_oracle_pairs, specs[:cores]))  # workers up, oracle loaded
        t0 = time.perf_counter()
        got = list(ex.map(_oracle_pairs, specs))
        dt = time.perf_counter() - t0
    pairs = sum(p for p, _ in got)
    return {"value": pairs / dt, "unit": "pairs/s", "cores": cores, "kind": "oracle",
            "sample": f"first {sample} of the {count} batched instances, one process per core, "
                      f"{dt:.1f} s wall ({sum(t for _, t in got):.1f} s of oracle time)",
            "seconds": dt, "pairs": pairs}


def bench_batched(ctx, count: int, reps: int = 3) -> dict:
    """Many instances in one rtg_all_pairs_batched call against the same
    instances run one rtg_all_pairs call at a time (points resident)."""
    import torch
    from paper_1409_8112_amd import workloads
    wls = workloads.batched_instances(count)
    pts = [torch.from_numpy(w.points()).to("cuda:0") for w in wls]
    queries = [dict(points=p, r=w.r, k=w.k, alpha=w.alpha, seed=w.seed) for p, w in zip(pts, wls)]
    torch.cuda.synchronize()

    def batched_once():
        res = ctx.all_pairs_batched(queries)
        pairs = sum(r.pairs for r in res)
        ctx.release_many(res)
        return pairs

    def timed():
        times, got = [], 0
        for _ in range(reps):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            got = batched_once()
            torch.cuda.synchronize()
            times.append(time.perf_counter() - t0)
        return float(np.median(times)), got

    batched_once()  # warm-up
    t_default, _ = timed()
    # the autotuner, one dimension at a time (its entries cover the passes of
    # that dimension), then the batch again with the tuned settings.  Each
    # dimension is tuned alone while the whole batch runs its dimensions'
    # passes on several lanes at once, so the tuned entries are kept only if
    # the whole batch is faster with them (else the entries in use before
    # are put back and the batch timed again).
    dims = sorted({w.d for w in wls})
    before = {d: ctx.get_tuning(d, 1 << 22) for d in dims}
    tuned = []
    t0 = time.perf_counter()
    for d in dims:
        tuned.append(ctx.autotune([q for q, w in zip(queries, wls) if w.d == d], reps=2))
    tune_s = time.perf_counter() - t0
    t_b, pairs = timed()
    t_tuned, kept = t_b, t_b <= t_default
    if not kept:
        for e in tuned:
            ctx.set_tuning({**before[e["d"]], "d": e["d"], "log2_points": e["log2_points"]})
        t_b, pairs = timed()
    plan = bench_plan(ctx, queries, reps)

    torch.cuda.synchronize()
    t0 = time.perf_counter()
    pairs_plain = 0
    for q in queries:
        r = ctx.all_pairs(q["points"], q["r"], q["k"], q["alpha"], q["seed"])
        pairs_plain += r.pairs
        r.release()
    torch.cuda.synchronize()
    t_p = time.perf_counter() - t0
    total_n = sum(w.n for w in wls)
    return {"workload": f"{count} instances, n log-uniform [1e3, 6.4e4] (sum {total_n}), "
                        "d in {2,3,6,9}, uniform, ~15 nb, k=6, alpha=2",
            "value": pairs / t_b, "unit": "pairs/s", "ms": t_b * 1e3, "pairs": pairs,
            "plain_value": pairs_plain / t_p, "plain_ms": t_p * 1e3,
            "plain_pairs": pairs_plain, "speedup_vs_plain": t_p / t_b,
            "same_pairs_as_plain": pairs == pairs_plain,
            "default_settings_ms": t_default * 1e3, "tuning_s": tune_s, "tuned": tuned,
            "tuned_ms": t_tuned * 1e3, "tuned_kept": kept,
            "plan": plan}


def brute_force_rows(points: np.ndarray, r: float, rows: np.ndarray, chunk: int = 16384) -> list:
    """Every point within r of each sampled row by direct search, the row
    itself excluded: a Gram-expansion screen with a wide margin, then the
    exact FP64 decision (squared differences summed axis by axis)."""
    p = points.astype(np.float64)
    q = p[rows]
    r2 = r * r
    qn = (q * q).sum(1)
    found = [[] for _ in range(len(rows))]
    t_last = time.perf_counter()
    for s0 in range(0, len(p), chunk):
        if time.perf_counter() - t_last > 20.0:
            print(f"#   brute force: {s0} of {len(p)} points", file=sys.stderr, flush=True)
            t_last = time.perf_counter()
        b = p[s0:s0 + chunk]
        approx = qn[:, None] + (b * b).sum(1)[None, :] - 2.0 * (q @ b.T)
        qi, bj = np.nonzero(approx <= r2 * (1.0 + 1e-6) + 1e-9)
        if len(qi) == 0:
            continue
        diff = q[qi] - b[bj]
        acc = np.zeros(len(qi))
        for l in range(p.shape[1]):
            acc = acc + diff[:, l] * diff[:, l]
        j = bj + s0
        keep = (acc <= r2) & (j != rows[qi])
        for a, c in zip(qi[keep].tolist(), j[keep].tolist()):
            found[a].append(c)
    return found


def measure_recall(ctx, pts, pts_host, wl, nrows: int) -> dict:
    """Recall of the GPU's neighbour lists against brute force on sampled
    rows (all rows when nrows >= n), and the count of listed neighbours
    farther than r (zero by construction)."""
    rows = np.arange(wl.n) if nrows >= wl.n else np.sort(
        np.random.default_rng(12345).choice(wl.n, size=nrows, replace=False))
    res = ctx.all_pairs(pts, wl.r, wl.k, wl.alpha, wl.seed)
    rp, col = res.to_numpy()
    res.release()
    t0 = time.perf_counter()
    bf = brute_force_rows(pts_host, wl.r, rows)
    hit = want = outside = 0
    for a, row in enumerate(rows.tolist()):
        got = set(col[rp[row]:rp[row + 1]].tolist())
        truth = set(bf[a])
        hit += len(got & truth)
        want += len(truth)
        outside += len(got - truth)
    return {"rows": int(len(rows)), "neighbours_brute_force": want, "found": hit,
            "recall": hit / max(want, 1), "listed_beyond_r": outside,
            "brute_force_s": time.perf_counter() - t0}


def bench_auto(ctx, pts, wl, target: float, mean_neighbours: float, reps: int = 10) -> dict:
    """The workload with (k, alpha) chosen by the library for a target recall
    (modelled), against its fixed parameters' modelled recall."""
    import torch
    from paper_1409_8112_amd import rtg
    k, alpha, rec = rtg.choose_params(wl.d, target, mean_neighbours)
    times, pairs = [], 0
    for i in range(reps + 2):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        res = ctx.all_pairs(pts, wl.r, k, alpha, wl.seed)
        pairs = res.pairs
        res.release()
        torch.cuda.synchronize()
        if i >= 2:
            times.append(time.perf_counter() - t0)
    t = float(np.median(times))
    return {"target_recall": target, "k": k, "alpha": alpha, "model_recall": rec,
            "fixed_model_recall": rtg.model_recall(wl.d, wl.k, wl.alpha),
            "ms": t * 1e3, "pairs": pairs, "pairs_per_s": pairs / t}


def _median_call_ms(ctx, pts, r, k, alpha, seed, flags, reps):
    import torch
    times, pairs = [], 0
    for i in range(reps + 2):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        res = ctx.all_pairs(pts, r, k, alpha, seed, flags)
        pairs = res.pairs
        res.release()
        torch.cuda.synchronize()
        if i >= 2:
            times.append(time.perf_counter() - t0)
    return float(np.median(times)) * 1e3, pairs


def bench_variants(ctx, pts, wl, reps: int = 10) -> dict:
    """The rules that remove repeated pairs -- first owner (default),
    sort-unique and the pair bitmap -- on a small, a mid-size and the
    workload's instance (the bitmap does not fit the last one and falls back
    to the first owner), and the Euclidean metric against the MR-metric of
    two robots (d = 6 as two robots in 3-D) on the workload."""
    import torch
    from paper_1409_8112_amd import rtg, workloads
    rules = {"first_owner": 0, "sort_unique": rtg.DEDUP_SORT, "bitmap": rtg.DEDUP_BITMAP}
    cases = [(workloads.small_uniform_d3(), None),
             (workloads.Workload("uniform n=64000 d=6 k=8 alpha=2 (~20 nb)", 64000, 6,
                                 workloads.calibrate_radius_uniform(64000, 6, 20.0), 8, 2.0, 0, 0),
              None),
             (wl, pts)]
    dedup = {}
    for w, dev in cases:
        if dev is None:
            dev = torch.from_numpy(w.points()).to("cuda:0")
        row = {}
        for name, fl in rules.items():
            if name == "bitmap" and w.n * (w.n - 1) // 2 > 8 * (4 << 30):
                continue  # larger than the bitmap limit: it would run the first-owner rule
            ms, pairs = _median_call_ms(ctx, dev, w.r, w.k, w.alpha, w.seed, fl, reps)
            row[name + "_ms"] = ms
            row["pairs"] = pairs
        dedup[w.name] = row
    eu_ms, eu_pairs = _median_call_ms(ctx, pts, wl.r, wl.k, wl.alpha, wl.seed, 0, reps)
    mr_ms, mr_pairs = _median_call_ms(ctx, pts, wl.r, wl.k, wl.alpha, wl.seed, rtg.robots(2), reps)
    return {"dedup": dedup,
            "metric": {"workload": wl.name, "euclidean_ms": eu_ms, "euclidean_pairs": eu_pairs,
                       "mr_2_robots_ms": mr_ms, "mr_2_robots_pairs": mr_pairs}}


def bench_param_study(ctx, reps: int = 3) -> dict:
    """The paper's parameter study (Sec. IV-A) on the GPU path: n = 102400
    points uniform in [0,1]^9, radius of Eq. r_FMT* (eta = 0).  Success rate
    = reported pairs over the oracle's brute-force pairs (RTG reports a
    subset of them), and the time of one all-pairs call (points resident,
    median of reps):
      vs_m      m = 5..60 grids at c~ = 1.1,
      vs_c      c~ = 1.0..2.0 at m = 20,
      table_ii  Table II's rule over a (m, c~) grid: the fastest pair with
                success >= 0.98,
      model     the library's modelled choice for 0.98 (rtg_choose_params),
                measured the same way,
      tuned     the library's measured choice (rtg_tune_params: modelled
                recall >= 0.98, fastest measured time), measured the same
                way."""
    import torch
    from paper_1409_8112_amd import rtg, workloads
    with open(os.path.join(ROOT, "tests", "golden", "bruteforce_fmt_uniform.json")) as fh:
        case = [c for c in json.load(fh)["cases"] if (c["n"], c["d"]) == (102400, 9)][0]
    n, d, r, truth = case["n"], case["d"], case["r"], case["pairs"]
    pts = torch.from_numpy(workloads.uniform_points(n, d, case["point_seed"])).to("cuda:0")
    torch.cuda.synchronize()

    def run(k, alpha):
        times, pairs = [], 0
        for i in range(reps + 1):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            res = ctx.all_pairs(pts, r, k, alpha, 0)
            pairs = res.pairs
            res.release()
            torch.cuda.synchronize()
            if i:
                times.append(time.perf_counter() - t0)
        return {"k": k, "alpha": alpha, "ms": float(np.median(times)) * 1e3, "pairs": pairs,
                "success": pairs / truth}

    vs_m = [run(k, 1.1) for k in (5, 10, 15, 20, 25, 30, 35, 40, 45, 50, 60)]
    vs_c = [run(20, round(c, 3)) for c in np.arange(1.0, 2.0001, 0.1)]
    grid = [run(k, round(c, 3)) for k in range(10, 61, 5) for c in np.arange(1.0, 1.6001, 0.05)]
    ok = [g for g in grid if g["success"] >= 0.98]
    best = min(ok, key=lambda g: g["ms"]) if ok else None
    nu = 2.0 * truth / n
    k_m, a_m, rec_m = rtg.choose_params(d, 0.98, nu)
    model = run(k_m, a_m)
    model["model_recall"] = rec_m
    # modelled recall, measured time: the library's own Table II rule
    k_t, a_t, rec_t, _ms = ctx.tune_params(pts, r, 0.98, reps=2)
    tuned = run(k_t, a_t)
    tuned["model_recall"] = rec_t
    del pts
    return {"workload": f"n={n} uniform in [0,1]^{d}, r={r:.4f} (Eq. r_FMT*, eta=0), "
                        f"{truth} brute-force pairs (oracle), {nu:.1f} mean neighbours",
            "vs_m_at_c1.1": vs_m, "vs_c_at_m20": vs_c, "grid_points": len(grid),
            "table_ii_choice": best, "model_choice": model, "tuned_choice": tuned}


def bench_query(ctx, pts, wl, m: int = 1_000_000, reps: int = 5) -> dict:
    """Query mode: an index of the workload's points (its k sorted grids),
    then m uniform query points per call."""
    import torch
    from paper_1409_8112_amd import workloads
    q = torch.from_numpy(workloads.uniform_points(m, wl.d, seed=4242)).to("cuda:0")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    h = ctx.index_build(pts, wl.r, wl.k, wl.alpha, wl.seed)
    torch.cuda.synchronize()
    build_ms = (time.perf_counter() - t0) * 1e3
    res = ctx.index_query(h, q)  # warm-up
    res.release()
    times, found = [], 0
    for _ in range(reps):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        res = ctx.index_query(h, q)
        torch.cuda.synchronize()
        times.append(time.perf_counter() - t0)
        found = res.nnz
        res.release()
    ctx.release(h)
    t = float(np.median(times))
    return {"workload": f"index of {wl.name}; {m} uniform query points per call",
            "queries_per_s": m / t, "ms": t * 1e3, "neighbours": found,
            "neighbours_per_s": found / t, "index_build_ms": build_ms}


def serving_points(count: int):
    """The request mix's points, on the device (workloads.serving_mix)."""
    import torch
    from paper_1409_8112_amd import workloads
    mix = workloads.serving_mix(count)
    pts = [torch.from_numpy(w.points()).to("cuda:0") for w in mix.requests]
    torch.cuda.synchronize()
    return mix, pts


def bench_serving(ctx, mix, pts, rate: float) -> dict:
    """Poisson arrivals through rtg_submit / rtg_poll: the mix's requests at
    its arrival times rescaled to `rate`.  Latency runs from a request's
    scheduled arrival to the poll that sees it done."""
    count = len(mix.requests)
    arrivals = mix.arrivals * (1000.0 / rate)  # the mix is drawn at 1000 requests/s
    reqs = [(p, w.r, w.seed) for p, w in zip(pts, mix.requests)]
    ns = np.array([w.n for w in mix.requests])
    before = ctx.stats()

    lat, pairs = [], 0
    pending = {}
    i = 0
    t0 = time.perf_counter()
    last_done = t0
    while i < count or pending:
        now = time.perf_counter() - t0
        while i < count and arrivals[i] <= now:
            p, r, s = reqs[i]
            t = ctx.submit(p, r, mix.requests[i].k, mix.requests[i].alpha, s)
            if t is None:
                break  # no room to stage it yet
            pending[t] = arrivals[i]
            i += 1
        done = []
        for t, arr in pending.items():
            res = ctx.poll(t)
            if res is not None:
                fin = time.perf_counter()
                lat.append((fin - t0 - arr) * 1e3)
                pairs += res.pairs
                res.release()
                done.append(t)
                last_done = fin
        for t in done:
            del pending[t]
        if not done:
            time.sleep(5e-5)
    after = ctx.stats()
    span = last_done - t0 - arrivals[0]
    served = after["served_requests"] - before["served_requests"]
    passes = after["served_batches"] - before["served_batches"]
    return {"workload": f"{count} requests, Poisson {rate:g}/s, n log-uniform [500, 2e6] "
                        f"(sum {int(ns.sum())}), d in {{3,6,12}}, uniform, ~15 nb, k=8, alpha=2",
            "rate_per_s": rate,
            "value": pairs / span, "unit": "pairs/s", "pairs": pairs,
            "latency_ms": {"p50": float(np.percentile(lat, 50)),
                           "p99": float(np.percentile(lat, 99)),
                           "max": float(np.max(lat))},
            "offered_s": float(arrivals[-1]), "span_s": span,
            "requests_per_pass": served / max(passes, 1)}


# Phases of one query: kernel ids whose launches they group (rtg.KERNELS).
PHASES = {"stage": ["stage"], "key": ["keys"], "key_sort": ["key_hist", "key_scatter"],
          "cells": ["cells"], "pairs": ["pairs"], "compact": ["compact"],
          "lists": ["csr"], "scans": ["scan"]}


def phase_block(stats_sum: dict, steps: int) -> dict:
    """Per phase: the library's algorithmic bytes (what its kernels must read
    and write), device time (HIP events around each launch) and the rate as a
    fraction of HBM peak, per query."""
    from paper_1409_8112_amd import rtg
    out = {}
    for name, kids in PHASES.items():
        ix = [rtg.KERNELS.index(k) for k in kids]
        by = sum(stats_sum["kernel_bytes"][i] for i in ix) / steps
        ms = sum(stats_sum["kernel_ms"][i] for i in ix) / steps
        la = sum(stats_sum["kernel_launches"][i] for i in ix) / steps
        gbs = by / (ms / 1e3) / 1e9 if ms > 0 else 0.0
        out[name] = {"bytes": by, "us": ms * 1e3, "launch_groups": la, "GB/s": gbs,
                     "frac_hbm": gbs / HBM_PEAK_GBS}
    return out


def _sum_stats(acc, st):
    if acc is None:
        return {k: (list(v) if isinstance(v, list) else v) for k, v in st.items()}
    for k in ("kernel_bytes", "kernel_ms", "kernel_launches"):
        acc[k] = [a + b for a, b in zip(acc[k], st[k])]
    return acc


def probe_steps(ctx, step, steps: int):
    """steps queries with every kernel id timed: summed stats."""
    from paper_1409_8112_amd import rtg
    ctx.set_timing((1 << rtg.NKERNELS) - 1)
    acc = None
    for _ in range(steps):
        step()
        acc = _sum_stats(acc, ctx.stats())
    ctx.set_timing(0)
    return acc


def pair_roofline(d: int, tests: float, pair_ms: float, matrix: bool, small: bool = False) -> dict:
    """The pair kernel against FP32 peak: 2d flops per tested pair (the
    small path tests every pair in FP64: against the FP64 peak)."""
    peak = FP64_VEC_PEAK_TFLOPS if small else FP32_VEC_PEAK_TFLOPS
    achieved = 2.0 * d * tests / (pair_ms / 1e3) / 1e12
    return {"bound": "mfma" if matrix else "alu", "achieved": achieved,
            "peak": peak, "unit": "TFLOP/s",
            "frac": achieved / peak, "avg_launch_ms": pair_ms,
            "flops_per_test": 2 * d, "tests": tests,
            "kernel": ("k_tiny_grids+k_tiny_lists" if small
                       else "k_cell_pairs_gram" if matrix else "k_cell_pairs")}


def bench_plan(ctx, queries, steps: int) -> dict:
    """The same queries run as a plan (rtg_plan_*): two runs size the
    workspaces and capture the graphs, then steps timed runs replay them."""
    import torch
    plan = ctx.plan_create(queries)
    try:
        for _ in range(2):
            ctx.release_many(plan.run(queries))
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        pairs = 0
        for _ in range(steps):
            res = plan.run(queries)
            pairs = sum(r.pairs for r in res)
            ctx.release_many(res)
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t0) * 1e3 / steps
        return {"ms": ms, "pairs": pairs, "pairs_per_s": pairs / (ms / 1e3), **plan.info()}
    finally:
        plan.destroy()


def bench_config(ctx, wl, steps: int, warmup: int, probes: int = 3) -> dict:
    """One workload: ms per query (wall clock, points resident), pairs/s,
    the pair kernel's roofline and the phases."""
    import torch
    from paper_1409_8112_amd import rtg
    pts = torch.from_numpy(wl.points()).to("cuda:0")
    torch.cuda.synchronize()

    def step():
        res = ctx.all_pairs(pts, wl.r, wl.k, wl.alpha, wl.seed)
        pairs = res.pairs
        res.release()
        return pairs

    for _ in range(warmup):
        step()
    acc = probe_steps(ctx, step, probes)
    st = ctx.stats()
    pk = rtg.KERNELS.index("pairs")
    pair_ms = acc["kernel_ms"][pk] / max(acc["kernel_launches"][pk], 1)
    lat = []
    pairs = 0
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        s0 = time.perf_counter()
        pairs = step()
        lat.append((time.perf_counter() - s0) * 1e3)
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3 / steps
    plan = bench_plan(ctx, [dict(points=pts, r=wl.r, k=wl.k, alpha=wl.alpha, seed=wl.seed)], steps)
    del pts
    # no key-kernel launch: the two-launch small path ran, both launches
    # timed together under the pair kernel id
    small = acc["kernel_launches"][rtg.KERNELS.index("keys")] == 0
    return {"workload": wl.name, "n": wl.n, "d": wl.d, "k": wl.k, "alpha": wl.alpha, "r": wl.r,
            "steps": steps, "ms": ms, "pairs": pairs, "pairs_per_s": pairs / (ms / 1e3),
            "path": "small" if small else "general",
            "plan": plan,
            "latency_ms": {"p50": float(np.percentile(lat, 50)),
                           "p99": float(np.percentile(lat, 99))},
            "pair_kernel": pair_roofline(wl.d, st["tests"], pair_ms,
                                         st["matrix_screen_launches"] > 0, small),
            "phases": phase_block(acc, probes)}


def main(argv=None) -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="uniform_d6",
                    choices=["uniform_d6", "small_d3", "clustered_d12"])
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-budget", type=float, default=60.0)
    ap.add_argument("--arena-gb", type=float, default=48.0)
    ap.add_argument("--no-configs", action="store_true",
                    help="skip the small d3 and clustered d12 workloads")
    ap.add_argument("--no-batched", action="store_true",
                    help="skip the batched-instances measurement")
    ap.add_argument("--no-serving", action="store_true",
                    help="skip the request-loop measurement")
    ap.add_argument("--no-query", action="store_true", help="skip the query-mode measurement")
    ap.add_argument("--no-variants", action="store_true",
                    help="skip the dedup-rule and metric-variant measurements")
    ap.add_argument("--no-auto", action="store_true",
                    help="skip the run with parameters chosen for a target recall")
    ap.add_argument("--no-param-study", action="store_true",
                    help="skip the parameter study (success rate and time vs m and c~)")
    ap.add_argument("--copy-calibration-mib", type=int, default=0,
                    help="run one device copy of this many MiB first (a known-size "
                         "kernel for scaling hardware byte counters)")
    ap.add_argument("--recall-rows", type=int, default=0,
                    help="recall against brute force on this many sampled rows (0: skip)")
    ap.add_argument("--batched-count", type=int, default=4096)
    ap.add_argument("--serving-requests", type=int, default=1000)
    ap.add_argument("--serving-rates", default="1000,500",
                    help="arrival rates (requests/s) of the request-loop runs")
    args = ap.parse_args(argv)

    if args.gpus != 1:
        print(f"bench.py: measures one GPU; --gpus {args.gpus} is not supported "
              "(instances and requests would shard across GPUs without communication)",
              file=sys.stderr)
        return 2

    all_cores = None
    if not args.no_cpu_baseline:
        # before anything touches the GPU: the pool forks plain CPU workers
        print("# cpu baseline, all cores (oracle)", file=sys.stderr, flush=True)
        all_cores = cpu_baseline_all_cores(args.batched_count)

    import torch
    from paper_1409_8112_amd import rtg

    wl = workload_by_name(args.workload)
    pts_host = wl.points()
    ctx = rtg.Context(0, arena_bytes=int(args.arena_gb * (1 << 30)))
    pts = torch.from_numpy(pts_host).to("cuda:0")
    torch.cuda.synchronize()
    if args.copy_calibration_mib > 0:
        # reads and writes exactly copy_calibration_mib MiB each
        src = torch.ones(args.copy_calibration_mib << 18, dtype=torch.float32, device="cuda:0")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst

    def step():
        res = ctx.all_pairs(pts, wl.r, wl.k, wl.alpha, wl.seed)
        pairs = res.pairs
        res.release()
        return pairs

    print(f"# workload {wl.name}: warmup {args.warmup}", file=sys.stderr, flush=True)
    for _ in range(args.warmup):
        step()

    # Untimed steps with every kernel timed: the phases, and the dominant
    # single kernel for the roofline.
    probe = probe_steps(ctx, step, 3)
    ms_by = {name: probe["kernel_ms"][rtg.KERNELS.index(name)] for name in SINGLE_KERNELS}
    dominant = max(ms_by, key=ms_by.get)
    kid = rtg.KERNELS.index(dominant)
    ctx.set_timing(1 << kid)

    print(f"# timed: {args.steps} steps; dominant kernel {dominant}", file=sys.stderr, flush=True)
    lat = []
    k_ms = k_bytes = 0.0
    k_launch = 0
    tests = 0
    pairs = 0
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        s0 = time.perf_counter()
        pairs = step()
        lat.append((time.perf_counter() - s0) * 1e3)
        st = ctx.stats()
        k_ms += st["kernel_ms"][kid]
        k_bytes += st["kernel_bytes"][kid]
        k_launch += st["kernel_launches"][kid]
        tests += st["tests"]
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ctx.set_timing(0)

    ms_per_step = (t1 - t0) * 1e3 / args.steps
    value = pairs / (ms_per_step / 1e3)
    st = ctx.stats()

    avg_ms = k_ms / max(k_launch, 1)
    if dominant == "pairs":
        roof = pair_roofline(wl.d, tests / max(k_launch, 1), avg_ms,
                             st["matrix_screen_launches"] > 0,
                             probe["kernel_launches"][rtg.KERNELS.index("keys")] == 0)
        roof["traffic"] = (measured_traffic("k_cell_pairs")
                           if args.workload == "uniform_d6" and st["matrix_screen_launches"]
                           else None)
    else:
        per_launch = k_bytes / max(k_launch, 1)
        achieved = per_launch / (avg_ms / 1e3) / 1e9
        roof = {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": achieved / HBM_PEAK_GBS, "traffic": None,
                "kernel": SINGLE_KERNELS[dominant]}
    roof.update({"kernel_id": dominant, "avg_launch_ms": avg_ms,
                 "launches_per_step": k_launch / args.steps,
                 "algorithmic_bytes_per_launch": k_bytes / max(k_launch, 1)})

    out = {
        "metric": "r-neighbor pairs/sec at 1 MI355X (plain single-instance path)",
        "value": value,
        "unit": "pairs/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32+f64",
        "data": "synthetic",
        "config": {"workload": wl.name, "n": wl.n, "d": wl.d, "k": wl.k, "alpha": wl.alpha,
                   "r": wl.r, "seed": wl.seed, "point_seed": wl.point_seed,
                   "parallelism": "single GPU"},
        "pairs": pairs,
        "latency_ms": {"p50": float(np.percentile(lat, 50)), "p99": float(np.percentile(lat, 99))},
        "stats": {k: st[k] for k in ("cells", "tests", "candidates", "band_rechecks",
                                     "unique_pairs", "key_bits", "key_passes", "pair_bits",
                                     "transforms_per_sort")},
        "roofline": roof,
        "phases": phase_block(probe, 3),
        "probe_kernel_ms": {name: probe["kernel_ms"][i] / 3 for i, name in enumerate(rtg.KERNELS)},
        # the same step through a plan (graph replay of the device-sized stretch)
        "plan": bench_plan(ctx, [dict(points=pts, r=wl.r, k=wl.k, alpha=wl.alpha, seed=wl.seed)],
                           args.steps),
    }
    del pts
    if not args.no_configs and args.workload == "uniform_d6":
        from paper_1409_8112_amd import workloads
        out["configs"] = {}
        for name, w, steps in (("small_d3", workloads.small_uniform_d3(), 50),
                               ("clustered_d12", workloads.skewed_clustered_d12(), 10)):
            print(f"# config {w.name}", file=sys.stderr, flush=True)
            out["configs"][name] = bench_config(ctx, w, steps, 3)
    pts = torch.from_numpy(pts_host).to("cuda:0")
    if args.recall_rows > 0:
        print(f"# recall on {args.recall_rows} sampled rows", file=sys.stderr, flush=True)
        out["recall"] = measure_recall(ctx, pts, pts_host, wl, args.recall_rows)
    if not args.no_auto and args.workload == "uniform_d6":
        print("# parameters chosen for recall 0.98", file=sys.stderr, flush=True)
        out["auto_params"] = bench_auto(ctx, pts, wl, 0.98, 20.0)
    if not args.no_param_study and args.workload == "uniform_d6":
        print("# parameter study (n=102400, d=9)", file=sys.stderr, flush=True)
        out["param_study"] = bench_param_study(ctx)
    if not args.no_query and args.workload == "uniform_d6":
        print("# query mode", file=sys.stderr, flush=True)
        out["query"] = bench_query(ctx, pts, wl)
    if not args.no_variants and args.workload == "uniform_d6":
        print("# dedup rules and metric variants", file=sys.stderr, flush=True)
        out["variants"] = bench_variants(ctx, pts, wl)
    del pts
    if not args.no_batched:
        print(f"# batched: {args.batched_count} instances", file=sys.stderr, flush=True)
        out["batched"] = bench_batched(ctx, args.batched_count)
    if not args.no_serving:
        mix, spts = serving_points(args.serving_requests)
        out["serving"] = []
        for rate in (float(x) for x in args.serving_rates.split(",")):
            print(f"# serving: {args.serving_requests} requests at {rate}/s",
                  file=sys.stderr, flush=True)
            out["serving"].append(bench_serving(ctx, mix, spts, rate))
        del spts
    ctx.close()
    if not args.no_cpu_baseline:
        print("# cpu baseline (oracle)", file=sys.stderr, flush=True)
        out["cpu_baseline"] = cpu_baseline(pts_host, wl, args.cpu_budget)
        out["cpu_baseline_all_cores"] = all_cores
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
