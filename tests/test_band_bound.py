"""The matrix-core screen's band E against exact arithmetic (CPU only).

The GPU's matrix-core pair screen decides most pairs from an FP32 Gram
expansion and sends a pair to the FP64 definition only when its FP32 value
x = |a'|^2 + (|b'|^2 - lo) - 2 a'.b' lies within E of the threshold.  That
is exact only if E bounds the rounding of x.  This test restates the
kernel's tile-pair arithmetic in exact rational arithmetic with explicit
FP32 rounding, under every accumulation model the matrix cores could follow
(products rounded or exact; the K terms summed one at a time in either
order, two at a time, or with one rounding at the end), on adversarial
tiles: coordinates far from zero so that centring a - o rounds, the origin
at one corner of the cell and the pairs around the opposite corner (the
largest |a'|^2, |b'|^2 with distances near r, where the expansion cancels
the most), and pairs whose FP64 squared distance is exactly r^2 or one ulp
either side.  It checks |x - (s - lo)| <= E for the exact squared distance s
of the FP32 inputs, and that every decision outside the band agrees with
the FP64 definition; and that E, evaluated in FP32 as the kernel does,
covers the error model's worst case for every d the screen runs at.

The error model (derived by recursive-summation bounds, u = 2^-24):
  centring   |a'_l - (a_l - o_l)| <= u |a_l - o_l|
  norms      n_a = sum a'_l^2 by an FMA chain: within gamma_D |a'|^2
  B row      n_b - lo rounded once: within u |n_b - lo|
  Gram sum   K = KA augmented terms, each product possibly rounded, summed
             in any order: within gamma_(K+1) sum |terms|
  total      |x - (s - lo)| <= u S (2K + D + 7) + u r^2 (K + 2) + O(u^2),
             S = max |a'|^2 + max |b'|^2 over the tile pair,
which E = 1.5 (2K + D + 8) u (S + r^2) + 4 u r^2 covers with room for the
second-order terms and for E's own FP32 evaluation; flushed subnormal
products are covered by E's absolute 1e-36.
"""
from fractions import Fraction
import math

import numpy as np
import pytest

U = Fraction(1, 2 ** 24)


def f32(x: Fraction) -> Fraction:
    """x rounded to the nearest FP32 value (ties to even), exactly."""
    if x == 0:
        return Fraction(0)
    sign = -1 if x < 0 else 1
    a = abs(x)
    e = math.floor(math.log2(a.numerator) - math.log2(a.denominator))
    # fix e so that 2^e <= a < 2^(e+1)
    while Fraction(2) ** e > a:
        e -= 1
    while Fraction(2) ** (e + 1) <= a:
        e += 1
    e = max(e, -126)                      # subnormals share the least exponent
    q = a / Fraction(2) ** (e - 23)       # 24-bit significand scale
    n = q.numerator // q.denominator
    rem = q - n
    if rem > Fraction(1, 2) or (rem == Fraction(1, 2) and n % 2 == 1):
        n += 1
    return sign * Fraction(n) * Fraction(2) ** (e - 23)


def F(v) -> Fraction:
    return Fraction(float(np.float32(v)))


def fma32(x, y, z):
    return f32(x * y + z)


def kernel_constants(D):
    KA = (D + 3) & ~1
    gain = f32(Fraction(3, 2) * (2 * KA + D + 8) * U)
    return KA, gain


def band(amax, bmax, r2f, gain):
    """E, lo, hi, W as the kernel forms them (FP32 operations in its order)."""
    E = f32(f32(f32(f32(amax + bmax) + r2f) * gain) + f32(r2f * 4 * U))
    E = f32(E + F(1e-36))
    all_fp64 = not (E < r2f)
    lo = Fraction(0) if all_fp64 else f32(f32(r2f - E) * f32(1 - Fraction(1, 2 ** 20)))
    hi = f32(f32(r2f + E) * f32(1 + Fraction(1, 2 ** 20)))
    W = f32(hi - lo)
    return E, lo, hi, W, all_fp64


def gram_models(arow, brow):
    """x under each accumulation model of the K-term dot product."""
    exact = [a * b for a, b in zip(arow, brow)]
    rounded = [f32(p) for p in exact]
    out = {}
    for pname, prods in (("exact products", exact), ("rounded products", rounded)):
        acc = Fraction(0)
        for p in prods:
            acc = f32(acc + p)
        out[pname + ", forward"] = acc
        acc = Fraction(0)
        for p in reversed(prods):
            acc = f32(acc + p)
        out[pname + ", backward"] = acc
        acc = Fraction(0)
        for k in range(0, len(prods), 2):   # two terms per matrix-core step
            acc = f32(acc + prods[k] + prods[k + 1])
        out[pname + ", pairs"] = acc
    out["one rounding"] = f32(sum(exact))
    return out


def tile_pair(A, B, D, r2):
    """Checks the bound for every (a, b) of the tiles; returns the number of
    pairs decided outside the band."""
    KA, gain = kernel_constants(D)
    o = [F(v) for v in A[0]]
    ap = [[f32(F(v) - o[l]) for l, v in enumerate(a)] for a in A]
    bp = [[f32(F(v) - o[l]) for l, v in enumerate(b)] for b in B]

    def norm(v):
        n = Fraction(0)
        for x in v:
            n = fma32(x, x, n)
        return n

    na = [norm(v) for v in ap]
    nb = [norm(v) for v in bp]
    r2f = F(r2)
    E, lo, hi, W, all_fp64 = band(max(na), max(nb), r2f, gain)
    decided = 0
    for i, a in enumerate(A):
        arow = ap[i] + [na[i], Fraction(1)] + [Fraction(0)] * (KA - D - 2)
        for j, b in enumerate(B):
            brow = [f32(-2 * x) for x in bp[j]] + [Fraction(1), f32(nb[j] - lo)]
            brow += [Fraction(0)] * (KA - D - 2)
            s = sum((F(x) - F(y)) ** 2 for x, y in zip(a, b))      # exact
            s64 = 0.0
            for x, y in zip(a, b):
                dl = float(np.float32(x)) - float(np.float32(y))
                s64 = s64 + dl * dl                                 # the definition
            for name, x in gram_models(arow, brow).items():
                assert abs(x - (s - lo)) <= E, (name, float(x), float(s - lo), float(E))
                if all_fp64:
                    continue
                if x < 0:
                    assert s64 <= r2, name
                    decided += 1
                elif x > W:
                    assert s64 > r2, name
                    decided += 1
    return decided


def _far_cell(rng, n, D, side, offset):
    """n FP32 points spread over a cube of the given side whose corner sits at
    offset: coordinates large enough that a - o is rounded."""
    corner = np.full(D, offset, dtype=np.float64)
    return (corner + rng.random((n, D)) * side).astype(np.float32)


@pytest.mark.parametrize("D,alpha,offset", [(3, 2.0, 0.0), (6, 2.0, 1e4), (6, 2.0, 3.3e6),
                                            (9, 1.5, 7.7e3), (12, 1.2, 1e5)])
def test_band_bounds_gram_rounding(D, alpha, offset):
    rng = np.random.default_rng(D * 1000 + int(offset) % 997)
    r = 0.37
    side = alpha * r
    A = _far_cell(rng, 6, D, side, offset)
    B = _far_cell(rng, 6, D, side, offset)
    # the origin o = A[0] at one corner of the cell and the other points
    # around the opposite corner, within r of each other: every |a'|^2,
    # |b'|^2 is near its largest, D side^2, while the pairs' distances are
    # near r, so the Gram expansion cancels the most
    A[0] = np.float32(offset)
    far = np.float64(offset) + side - 0.5 * r / math.sqrt(D)
    A[1:] = (far + (rng.random((5, D)) - 0.5) * r / math.sqrt(D)).astype(np.float32)
    B[:] = (far + (rng.random((6, D)) - 0.5) * r / math.sqrt(D)).astype(np.float32)
    # pairs at r: r^2 is the FP64 squared distance of one (a, b) pair, and
    # the neighbouring doubles make pairs one ulp inside and outside
    s64 = 0.0
    for x, y in zip(A[4], B[5]):
        dl = float(x) - float(y)
        s64 = s64 + dl * dl
    for r2 in (s64, np.nextafter(s64, 0.0), np.nextafter(s64, np.inf)):
        tile_pair(A, B, D, float(r2))


def test_band_bound_decides_most_pairs():
    """With small coordinates the band is narrow: nearly every pair of a
    tile pair is decided in FP32 (the screen is useful, not only sound)."""
    rng = np.random.default_rng(5)
    D, r = 6, 0.2
    A = _far_cell(rng, 8, D, 2 * r, 0.25)
    B = _far_cell(rng, 8, D, 2 * r, 0.25)
    assert tile_pair(A, B, D, r * r) >= 60 * 7  # 64 pairs x 7 models, most decided


def test_f32_rounding_helper():
    for v in (1.0, 0.1, 3.3e6 + 0.37, -2.5e-3, 1e30, 1.401298464324817e-45 * 3):
        assert f32(Fraction(v)) == Fraction(float(np.float32(v)))
    # a tie rounds to even
    t = Fraction(1) + Fraction(1, 2 ** 24)
    assert f32(t) == 1


def test_band_covers_the_model_bound():
    """E >= the model's worst case, u S (2K + D + 7) + u r^2 (K + 2), with the
    second-order terms bounded by (K + D + 3)^2 u^2 (S + r^2), for every
    D <= 16 and norms from zero to far beyond the cell."""
    for D in range(1, 17):
        KA, gain = kernel_constants(D)
        for r2 in (Fraction(2) ** -100, Fraction(1, 7), Fraction(1), Fraction(2) ** 100):
            r2f = f32(r2)
            for mult in (0, 1, 3, 24, 48, 200, 1000):
                amax = f32(r2f * mult)
                bmax = f32(r2f * mult / 2)
                S = amax + bmax
                E = band(amax, bmax, r2f, gain)[0]
                model = U * S * (2 * KA + D + 7) + U * r2f * (KA + 2)
                model += (KA + D + 3) ** 2 * U * U * (S + r2f)
                assert E >= model, (D, float(r2), mult)


def _haar(rng, d):
    q, r = np.linalg.qr(rng.normal(size=(d, d)))
    return q * np.sign(np.diag(r))


def _norms32(P, o):
    """|fl(p - o)|^2 for each row p, in FP32 as the screen forms it (centred
    coordinates rounded to FP32, squares summed by an FMA chain)."""
    c = (P.astype(np.float32) - o.astype(np.float32)).astype(np.float32)
    acc = np.zeros(len(P), dtype=np.float32)
    for l in range(P.shape[1]):
        x = c[:, l].astype(np.float64)
        acc = (x * x + acc.astype(np.float64)).astype(np.float32)
    return acc


@pytest.mark.parametrize("d,side,offset", [(2, 0.3, 0.0), (3, 1.7, 5e3), (6, 0.26, 0.0),
                                           (6, 0.26, 3e4), (9, 0.9, 1e2), (12, 2.0, 7e5),
                                           (16, 0.05, 1e1)])
def test_cell_diagonal_bounds_the_band_norms(d, side, offset):
    """The unit-wide band takes S <= s_bound = 2 d c^2 (1 + 2^-10) (rounded
    to FP32) for any three points a, b, o of one grid cell.  Points of one
    cell -- its corners and random interior points, mapped back through the
    grid's rotation and shift, rounded to FP32, kept only if their FP64 cell
    is still that cell -- all have |fl(p - o)|^2 <= s_bound / 2 for every
    origin o among them."""
    rng = np.random.default_rng(d * 7 + int(offset) % 13)
    R = _haar(rng, d)
    u = rng.random(d)
    kappa = np.floor(rng.normal(size=d) * 3 + offset / side)
    # corners pulled in by more than the FP32 spacing of the coordinates, so
    # that rounding keeps them in the cell
    m = max(1e-3, 4.0 * (abs(offset) + 10.0) * 2.0 ** -23 / side)
    bits = rng.random((32, d)) < 0.5
    corners = np.concatenate([np.where(bits, 1 - m, m), np.where(bits, m, 1 - m)])
    y = np.concatenate([kappa + corners, kappa + rng.random((200, d))])
    P = ((y - u) * side) @ R                       # R^T applied row-wise
    P32 = P.astype(np.float32)
    cell = np.floor((P32.astype(np.float64) @ R.T) / side + u)
    P32 = P32[(cell == kappa).all(axis=1)]
    assert len(P32) > 150
    s_bound = np.float32(2.0 * d * side * side * (1.0 + 2.0 ** -10))
    worst = max(float(_norms32(P32, o).max()) for o in P32[:40])
    assert 2 * worst <= float(s_bound), (worst, float(s_bound))
    # and the bound is not loose: opposite corners (both kept) come near it
    assert 2 * worst >= 0.9 * (1 - 2 * m) ** 2 * float(s_bound)
