"""Seeded synthetic inputs shaped like the paper's workloads.

This module holds input generation only and none of the RTG arithmetic: the
tests, the smoke check and the benchmark draw points and radii from here and
hand them both to the GPU library and to the CPU oracle.

Shapes follow the paper's experiments: points uniform in the unit d-cube
(Sec. IV-A and IV-B), dimensions 2..12, and a radius of the form
gamma * (ln n / n)^(1/d) as in the PRM* and FMT* radii (Eq. r_PRM*, Eq. r_FMT*).
The obstacle-cluttered sample sets of the paper's motion-planning scenes are
not available; a Gaussian-cluster mixture stands in for uneven occupancy.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np


def uniform_points(n: int, d: int, seed: int) -> np.ndarray:
    """n points i.i.d. uniform in [0,1)^d, float32, row-major [n, d]."""
    rng = np.random.default_rng(seed)
    return rng.random((n, d), dtype=np.float32)


def clustered_points(n: int, d: int, seed: int, n_clusters: int = 64, sigma: float = 0.02,
                     cluster_frac: float = 0.8) -> np.ndarray:
    """Gaussian-cluster mixture in [0,1]^d (centres uniform, clipped to the box),
    with a uniform background; rows shuffled.  float32 [n, d]."""
    rng = np.random.default_rng(seed)
    n_cl = int(round(cluster_frac * n))
    centres = rng.random((n_clusters, d))
    which = rng.integers(0, n_clusters, size=n_cl)
    pts_cl = centres[which] + sigma * rng.standard_normal((n_cl, d))
    pts_cl = np.clip(pts_cl, 0.0, 1.0)
    pts_un = rng.random((n - n_cl, d))
    pts = np.concatenate([pts_cl, pts_un]).astype(np.float32)
    rng.shuffle(pts, axis=0)
    return np.ascontiguousarray(pts)


def unit_ball_volume(d: int) -> float:
    """zeta_d, the volume of the d-dimensional unit ball."""
    return math.pi ** (d / 2.0) / math.gamma(d / 2.0 + 1.0)


def fmt_radius(n: int, d: int, eta: float = 0.0, free_volume: float = 1.0) -> float:
    """The FMT* radius 2(1+eta)[(1/d)(mu/zeta_d)(ln n / n)]^(1/d) (Eq. r_FMT*),
    with mu = 1 for the unit cube; the paper's parameter study uses it."""
    return 2.0 * (1.0 + eta) * ((1.0 / d) * (free_volume / unit_ball_volume(d))
                                * (math.log(n) / n)) ** (1.0 / d)


def prm_radius(n: int, d: int, gamma: float) -> float:
    """gamma * (ln n / n)^(1/d): the shape shared by the PRM* and FMT* radii."""
    return gamma * (math.log(n) / n) ** (1.0 / d)


def expected_neighbours_uniform(n: int, d: int, r: float, samples: int = 200_000,
                                seed: int = 12345) -> float:
    """Mean number of neighbours within r of a point, for n uniform points in
    the unit cube: (n-1) * zeta_d r^d * E_B[prod_j (1 - r|B_j|)_+], B uniform in
    the unit ball (the cube-boundary correction), by seeded Monte Carlo."""
    rng = np.random.default_rng(seed)
    g = rng.standard_normal((samples, d))
    g /= np.linalg.norm(g, axis=1, keepdims=True)
    rad = rng.random(samples) ** (1.0 / d)
    b = g * rad[:, None]
    inside = np.prod(np.clip(1.0 - r * np.abs(b), 0.0, None), axis=1).mean()
    return (n - 1) * unit_ball_volume(d) * r ** d * inside


def calibrate_radius_uniform(n: int, d: int, target_neighbours: float) -> float:
    """Radius r with expected_neighbours_uniform(n, d, r) == target (bisection)."""
    lo, hi = 0.0, math.sqrt(d)
    for _ in range(60):
        mid = 0.5 * (lo + hi)
        if expected_neighbours_uniform(n, d, mid) < target_neighbours:
            lo = mid
        else:
            hi = mid
    return 0.5 * (lo + hi)


@dataclass
class Workload:
    """One all-pairs r-NN instance: points and the RTG parameters."""
    name: str
    n: int
    d: int
    r: float
    k: int
    alpha: float
    seed: int          # RTG transform seed
    point_seed: int    # input generator seed
    kind: str = "uniform"
    extra: dict = field(default_factory=dict)

    def points(self) -> np.ndarray:
        if self.kind == "uniform":
            return uniform_points(self.n, self.d, self.point_seed)
        if self.kind == "clustered":
            return clustered_points(self.n, self.d, self.point_seed, **self.extra)
        raise ValueError(self.kind)


# Radii frozen from calibrate_radius_uniform (uniform sets) and from a
# brute-force neighbour count on a subsample (the clustered set).
R_UNIFORM_1E6_D6 = 0.13027  # ~20 mean neighbours at n = 1e6, d = 6
R_CLUSTERED_4E6_D12 = 0.040  # ~30 mean neighbours at n = 4e6, d = 12 (clustered)


def small_uniform_d3() -> Workload:
    """n = 2000 uniform in [0,1]^3, r = 0.1 (~8 mean neighbours), k = 4, alpha = 2."""
    return Workload("uniform n=2000 d=3 r=0.1 k=4 alpha=2", 2000, 3, 0.1, 4, 2.0, 0, 0)


def large_uniform_d6() -> Workload:
    """n = 1e6 uniform in [0,1]^6, r for ~20 mean neighbours, k = 8, alpha = 2."""
    return Workload("uniform n=1e6 d=6 k=8 alpha=2 (~20 nb)", 1_000_000, 6, R_UNIFORM_1E6_D6, 8, 2.0,
                    0, 0)


def skewed_clustered_d12() -> Workload:
    """n = 4e6 in [0,1]^12: 80% from 64 Gaussian clusters (sigma 0.02), 20% uniform;
    r for ~30 mean neighbours, k = 8, alpha = 2."""
    return Workload("clustered n=4e6 d=12 k=8 alpha=2 (~30 nb)", 4_000_000, 12, R_CLUSTERED_4E6_D12,
                    8, 2.0, 0, 0, kind="clustered")


def batched_instances(count: int = 4096, seed: int = 0, n_lo: int = 1000, n_hi: int = 64000,
                      dims=(2, 3, 6, 9), target_neighbours: float = 15.0, k: int = 6,
                      alpha: float = 2.0) -> list[Workload]:
    """Many instances: n log-uniform in [n_lo, n_hi], d drawn from dims, uniform
    points, per-instance radius gamma_d (ln n / n)^(1/d) with gamma_d set for
    ~target_neighbours mean neighbours at the geometric-mean n."""
    rng = np.random.default_rng(seed)
    n_mid = int(round(math.sqrt(n_lo * n_hi)))
    gammas = {d: calibrate_radius_uniform(n_mid, d, target_neighbours)
              / (math.log(n_mid) / n_mid) ** (1.0 / d) for d in dims}
    out = []
    for q in range(count):
        n = int(round(math.exp(rng.uniform(math.log(n_lo), math.log(n_hi)))))
        d = int(rng.choice(dims))
        r = prm_radius(n, d, gammas[d])
        out.append(Workload(f"batched[{q}]", n, d, r, k, alpha, seed=q, point_seed=1_000_000 + q))
    return out


@dataclass
class ServingMix:
    """A request stream: Poisson arrival times (seconds from the start) and
    one uniform all-pairs instance per request."""
    arrivals: np.ndarray
    requests: list

    def replay_sample(self, frac: float = 0.01, seed: int = 2024) -> np.ndarray:
        """Indices of a seeded sample of the requests (frac of them, at least
        one), ascending: the requests whose results are checked in full."""
        m = max(1, int(round(frac * len(self.requests))))
        rng = np.random.default_rng(seed)
        return np.sort(rng.choice(len(self.requests), size=m, replace=False))


def serving_mix(count: int = 1000, rate: float = 1000.0, seed: int = 0, n_lo: int = 500,
                n_hi: int = 2_000_000, dims=(3, 6, 12), target_neighbours: float = 15.0,
                k: int = 8, alpha: float = 2.0) -> ServingMix:
    """Poisson arrivals at `rate` per second; request i has n log-uniform in
    [n_lo, n_hi], d drawn from dims, points uniform in [0,1)^d (point seed
    2_000_000 + i), radius gamma_d (ln n / n)^(1/d) with gamma_d set for
    ~target_neighbours mean neighbours at the geometric-mean n; RTG seed i."""
    rng = np.random.default_rng(seed)
    arrivals = np.cumsum(rng.exponential(1.0 / rate, size=count))
    ns = np.exp(rng.uniform(np.log(n_lo), np.log(n_hi), size=count)).round().astype(np.int64)
    ds = rng.choice(list(dims), size=count)
    n_mid = int(round(math.sqrt(n_lo * n_hi)))
    gammas = {int(d): calibrate_radius_uniform(n_mid, int(d), target_neighbours)
              / (math.log(n_mid) / n_mid) ** (1.0 / d) for d in dims}
    reqs = []
    for i in range(count):
        n, d = int(ns[i]), int(ds[i])
        reqs.append(Workload(f"served[{i}]", n, d, prm_radius(n, d, gammas[d]), k, alpha,
                             seed=i, point_seed=2_000_000 + i))
    return ServingMix(arrivals, reqs)
