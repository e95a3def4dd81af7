"""Exact rational brute force for tiny inputs -- TEST INFRASTRUCTURE ONLY.

Evaluates the lens equation (eq. 1), the many-Schwarzschild deflection
(eq. 2) and the macro model (eq. 6) of Thompson et al. (2009) in exact
rational arithmetic (``fractions.Fraction``) from the exact values of the
float32 lens records and the float32 ray coordinates, then bins the exact
source position into the half-open pixel floor((y - lo) * n / (hi - lo)).

It is an independent evaluation of the same definition: no rounding at all,
so it pins the FP64 oracle's evaluation order, indexing and binning on
inputs small enough for pure-Python loops.
"""
from __future__ import annotations

import math
from fractions import Fraction

import numpy as np


def exact_coord(lo: float, hi: float, n: int, i: int) -> Fraction:
    """Exact cell centre lo + (i + 1/2) (hi - lo) / n (no rounding)."""
    return Fraction(lo) + (Fraction(2 * i + 1, 2)) * (Fraction(hi) - Fraction(lo)) / n


def round_to_float32(q: Fraction) -> float:
    """Round an exact rational to the nearest float32 (ties to even)."""
    if q == 0:
        return 0.0
    sign = -1 if q < 0 else 1
    a = abs(q)
    e = math.floor(math.log2(a.numerator) - math.log2(a.denominator))
    # fix e so that 2**e <= a < 2**(e+1)
    while Fraction(2) ** e > a:
        e -= 1
    while Fraction(2) ** (e + 1) <= a:
        e += 1
    e = max(e, -126)
    scale = Fraction(2) ** (23 - e)
    m = a * scale
    fl = math.floor(m)
    rem = m - fl
    if rem > Fraction(1, 2) or (rem == Fraction(1, 2) and fl % 2 == 1):
        fl += 1
    return sign * float(Fraction(fl) / scale)


def alpha(lenses: np.ndarray, x1: Fraction, x2: Fraction):
    """Exact deflection sum_i m_i (x - x_i) / |x - x_i|^2; None if a ray sits on a lens."""
    s1, s2 = Fraction(0), Fraction(0)
    for rec in lenses:
        f1 = x1 - Fraction(float(rec[0]))
        f2 = x2 - Fraction(float(rec[1]))
        r2 = f1 * f1 + f2 * f2
        if r2 == 0:
            return None
        d = Fraction(float(rec[2])) / r2
        s1 += d * f1
        s2 += d * f2
    return s1, s2


def trace(lenses, kappa_c, gamma, grid_lo, grid_hi, grid_n, map_lo, map_hi, map_n, x1, x2):
    """Exact (y1, y2, pixel) of a ray at the float32 position (x1, x2); pixel -1 = lost."""
    X1, X2 = Fraction(float(x1)), Fraction(float(x2))
    a = alpha(lenses, X1, X2)
    if a is None:
        return None, None, -1
    lam1 = Fraction(float((1.0 - gamma) - kappa_c))
    lam2 = Fraction(float((1.0 + gamma) - kappa_c))
    y1 = lam1 * X1 - a[0]
    y2 = lam2 * X2 - a[1]
    p1 = math.floor((y1 - Fraction(map_lo[0])) * map_n[0] / (Fraction(map_hi[0]) - Fraction(map_lo[0])))
    p2 = math.floor((y2 - Fraction(map_lo[1])) * map_n[1] / (Fraction(map_hi[1]) - Fraction(map_lo[1])))
    if not (0 <= p1 < map_n[0] and 0 <= p2 < map_n[1]):
        return y1, y2, -1
    return y1, y2, p2 * map_n[0] + p1
