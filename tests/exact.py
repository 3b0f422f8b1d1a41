"""Exact rational arithmetic for checking reported pairs independently of any
floating-point summation order.  Every float32/float64 value is a dyadic
rational, so squared distances can be compared with r^2 exactly."""
from __future__ import annotations

from fractions import Fraction

import numpy as np


def to_fractions(points: np.ndarray) -> list[list[Fraction]]:
    return [[Fraction(float(x)) for x in row] for row in np.asarray(points, dtype=np.float32)]


def exact_sqdist(fp: list[list[Fraction]], i: int, j: int) -> Fraction:
    return sum(((a - b) * (a - b) for a, b in zip(fp[i], fp[j])), Fraction(0))


def exact_pairs_within(points: np.ndarray, r: float) -> set[tuple[int, int]]:
    """All i<j with ||p_i - p_j||^2 <= r^2, in exact arithmetic (brute force)."""
    fp = to_fractions(points)
    r2 = Fraction(float(r)) ** 2
    n = len(fp)
    return {(i, j) for i in range(n) for j in range(i + 1, n) if exact_sqdist(fp, i, j) <= r2}


def pair_set(pairs) -> set[tuple[int, int]]:
    return {(int(a), int(b)) for a, b in np.asarray(pairs).reshape(-1, 2)}


def check_csr(row_ptr: np.ndarray, col: np.ndarray, n: int, symmetric: bool = True) -> None:
    """Layout invariants of a neighbour list: monotone row_ptr, rows strictly
    ascending (no duplicates), no self-pairs, columns in range, symmetry."""
    row_ptr = np.asarray(row_ptr)
    col = np.asarray(col)
    assert row_ptr.shape == (n + 1,)
    assert row_ptr[0] == 0 and row_ptr[-1] == len(col)
    assert np.all(np.diff(row_ptr) >= 0)
    rows = np.repeat(np.arange(n), np.diff(row_ptr))
    assert np.all((col >= 0) & (col < n))
    assert not np.any(col == rows), "self-pair"
    same_row = rows[1:] == rows[:-1]
    assert np.all(col[1:][same_row] > col[:-1][same_row]), "row not strictly ascending"
    if symmetric:
        fwd = set(zip(rows.tolist(), col.tolist()))
        assert all((c, r) in fwd for r, c in fwd), "not symmetric"
    else:
        assert np.all(col > rows)


def exact_within(a, b, r: float) -> bool:
    """||a - b|| <= r in exact rational arithmetic on the float32 inputs
    and the double r (no rounding anywhere)."""
    s = sum((Fraction(float(x)) - Fraction(float(y))) ** 2 for x, y in zip(a, b))
    return s <= Fraction(float(r)) ** 2


def mr_margin(a, b, r: float, robots: int) -> float:
    """sum over robots of ||a_b - b_b|| minus r for the MR-metric (robots of
    d / robots consecutive axes each), from the exact squared displacements
    of the float32 inputs with 60-digit decimal square roots: its sign
    decides the MR test unless it is within about 1e-55 of zero."""
    from decimal import Decimal, localcontext
    a = [Fraction(float(x)) for x in a]
    b = [Fraction(float(x)) for x in b]
    sub = len(a) // robots
    with localcontext() as ctx:
        ctx.prec = 60
        total = Decimal(0)
        for q in range(robots):
            s = sum((x - y) ** 2 for x, y in zip(a[q * sub:(q + 1) * sub], b[q * sub:(q + 1) * sub]))
            total += (Decimal(s.numerator) / Decimal(s.denominator)).sqrt()
        return float(total - Decimal(float(r)))
