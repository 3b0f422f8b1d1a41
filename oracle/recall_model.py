"""Recall model of randomly transformed grids -- TEST INFRASTRUCTURE ONLY.

Plain Monte Carlo of the probability that k grids report a pair within r,
used to check the library's parameter choice.  It follows the grids'
definition (Alg. "Randomly Shifted Grids" and its random-orientation
variant, Sec. III): one grid of cell side c = alpha r with a uniform random
shift puts two points displaced by Delta in one cell with probability
prod_j (1 - |Delta_j| / c)_+ (the shift is uniform per axis); with a random
orientation each grid sees Delta rotated uniformly; the k grids are
independent.  Neighbour pairs are taken locally uniform: the distance
rho <= r has density d rho^(d-1) / r^d and the direction is uniform on the
sphere.  Recall = E[1 - (1 - p)^k].  Shares nothing with the library.
"""
from __future__ import annotations

import numpy as np


def _directions(rng, count: int, d: int) -> np.ndarray:
    g = rng.standard_normal((count, d))
    return g / np.linalg.norm(g, axis=1, keepdims=True)


def cocell_probability(delta: np.ndarray, c: float) -> np.ndarray:
    """P(one shifted grid of side c holds both points), per row of delta."""
    return np.prod(np.clip(1.0 - np.abs(delta) / c, 0.0, None), axis=-1)


def rotated_cocell_probability(rho: float, c: float, d: int, samples: int = 200_000,
                               seed: int = 1) -> float:
    """P(one randomly oriented, shifted grid holds two points rho apart)."""
    u = _directions(np.random.default_rng(seed), samples, d)
    return float(cocell_probability(rho * u, c).mean())


def model_recall(d: int, k: int, alpha: float, rotate: bool = True, radii: int = 200,
                 samples: int = 20_000, seed: int = 7) -> float:
    """Expected share of pairs within r that k grids report."""
    rng = np.random.default_rng(seed)
    if rotate:
        # p depends on rho only; 1 - (1 - p)^k is averaged over rho
        v = (np.arange(radii) + 0.5) / radii
        rho = v ** (1.0 / d)  # rho / r with density d x^(d-1)
        u = _directions(rng, samples, d)
        p = np.array([cocell_probability(x * u, alpha).mean() for x in rho])
        return float(np.mean(1.0 - (1.0 - p) ** k))
    # one orientation for all grids: p depends on the pair's direction too
    n = radii * samples // 20
    x = rng.random(n) ** (1.0 / d)
    u = _directions(rng, n, d)
    p = cocell_probability(x[:, None] * u, alpha)
    return float(np.mean(1.0 - (1.0 - p) ** k))
