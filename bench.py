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
                the library's stream during the timed steps;
  cpu_baseline  the CPU oracle on the same workload, single-threaded.
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
FP32_VEC_PEAK_TFLOPS = 157.3

# kernel ids whose launches are single kernels (candidates for the roofline)
SINGLE_KERNELS = {"keys": "k_keys", "key_hist": "k_radix_hist", "key_scatter": "k_radix_scatter<true>",
                  "pairs": "k_cell_pairs", "pair_hist": "k_radix_hist",
                  "pair_scatter": "k_radix_scatter<false>", "stage": "k_stage"}


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
    args = ap.parse_args(argv)

    if args.gpus != 1:
        print(f"bench.py: this build runs on one GPU; --gpus {args.gpus} is not supported "
              "(instances and requests shard across GPUs without communication; see the design "
              "notes)", file=sys.stderr)
        return 2

    import torch
    from paper_1409_8112_amd import rtg

    wl = workload_by_name(args.workload)
    pts_host = wl.points()
    ctx = rtg.Context(0, arena_bytes=int(args.arena_gb * (1 << 30)))
    pts = torch.from_numpy(pts_host).to("cuda:0")
    torch.cuda.synchronize()

    def step():
        res = ctx.all_pairs(pts, wl.r, wl.k, wl.alpha, wl.seed)
        pairs = res.pairs
        res.release()
        return pairs

    print(f"# workload {wl.name}: warmup {args.warmup}", file=sys.stderr, flush=True)
    for _ in range(args.warmup):
        step()

    # One untimed step with every kernel timed picks the dominant single kernel.
    ctx.set_timing((1 << rtg.NKERNELS) - 1)
    step()
    probe = ctx.stats()
    ms_by = {name: probe["kernel_ms"][rtg.KERNELS.index(name)] for name in SINGLE_KERNELS}
    dominant = max(ms_by, key=ms_by.get)
    kid = rtg.KERNELS.index(dominant)
    ctx.set_timing(1 << kid)

    print(f"# timed: {args.steps} steps; dominant kernel {dominant}", file=sys.stderr, flush=True)
    lat = []
    k_ms = k_bytes = 0.0
    k_launch = 0
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
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ctx.set_timing(0)

    ms_per_step = (t1 - t0) * 1e3 / args.steps
    value = pairs / (ms_per_step / 1e3)
    st = ctx.stats()

    avg_ms = k_ms / max(k_launch, 1)
    if dominant == "pairs":
        # ALU bound: FP32 flops of the screen, 3 per coordinate (sub, mul, add)
        flops = 3.0 * wl.d * st["tests"] * args.steps / max(k_launch, 1)
        achieved = flops / (avg_ms / 1e3) / 1e12
        roof = {"bound": "alu", "achieved": achieved, "peak": FP32_VEC_PEAK_TFLOPS,
                "unit": "TFLOP/s", "frac": achieved / FP32_VEC_PEAK_TFLOPS, "traffic": None}
    else:
        per_launch = k_bytes / max(k_launch, 1)
        achieved = per_launch / (avg_ms / 1e3) / 1e9
        roof = {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": achieved / HBM_PEAK_GBS, "traffic": None}
    roof.update({"kernel": SINGLE_KERNELS[dominant], "kernel_id": dominant,
                 "avg_launch_ms": avg_ms, "launches_per_step": k_launch / args.steps,
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
        "probe_kernel_ms": {name: probe["kernel_ms"][i] for i, name in enumerate(rtg.KERNELS)},
        "roofline": roof,
    }
    ctx.close()
    if not args.no_cpu_baseline:
        print("# cpu baseline (oracle)", file=sys.stderr, flush=True)
        out["cpu_baseline"] = cpu_baseline(pts_host, wl, args.cpu_budget)
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
