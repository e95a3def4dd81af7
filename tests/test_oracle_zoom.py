"""Pin of the zoom's cell bound (oracle/zoom.py): over many image-plane rectangles (far from
every lens, close to one, straddling the field's caustic-rich centre) every ray of a dense
sub-grid of the rectangle maps inside the bound box around y(c).  Dropping the remainder, the
near-lens term or the shear of the Jacobian makes some rectangle fail (checked below), and a
rectangle holding a lens is unbounded.
"""
import numpy as np

import oracle
import synth
from oracle import zoom


def _rects(seed, n, half, size):
    u = synth.uniform(seed, 99, 0, 4 * n).reshape(n, 4)
    c = (u[:, :2] * 2 - 1) * half
    h = np.stack([size * (0.2 + u[:, 2]), size * (0.2 + u[:, 3])], 1)
    return c, h


def _max_excursion(L, lam, c, h, k=17):
    g1 = c[0] + np.linspace(-h[0], h[0], k)
    g2 = c[1] + np.linspace(-h[1], h[1], k)
    X = np.stack(np.meshgrid(g1, g2), -1).reshape(-1, 2)
    a = oracle.deflect(L, X)
    y = np.stack([lam[0] * X[:, 0], lam[1] * X[:, 1]], 1) - a
    return y


def test_bound_holds_over_many_rectangles():
    L, _ = synth.lens_field(3, 400, kappa_star=0.45)
    lam = (0.55, 1.45)
    c, h = _rects(4, 300, 8.0, 0.15)
    worst = 0.0
    for ci, hi in zip(c, h):
        y0, E = zoom.cell_bound(L, lam, ci, hi)
        if not np.all(np.isfinite(E)):
            continue
        y = _max_excursion(L, lam, ci, hi)
        ex = np.abs(y - y0[None, :]).max(0)
        assert np.all(ex <= E), (ci, hi, ex, E)
        worst = max(worst, float(np.max(ex / E)))
    assert worst > 0.05         # the bound is not vacuous


def test_lens_inside_is_unbounded_and_slips_fail():
    L = np.array([[0.0, 0.0, 1.0, 0.0], [2.0, 0.3, 0.5, 0.0]], np.float32)
    y0, E = zoom.cell_bound(L, (1.0, 1.0), (0.01, 0.02), (0.1, 0.1))
    assert np.all(np.isinf(E))
    # a rectangle next to a lens: the near-lens term carries the bound
    c, h = np.array([0.5, 0.0]), np.array([0.1, 0.1])
    y0, E = zoom.cell_bound(L, (1.0, 1.0), c, h)
    ex = np.abs(_max_excursion(L, (1.0, 1.0), c, h) - y0[None, :]).max(0)
    assert np.all(ex <= E)
    # a rectangle at 3-5 half-diagonals from a lens: without the remainder the linear term
    # alone under-covers the excursion
    c, h = np.array([0.9, 0.1]), np.array([0.12, 0.12])
    L1 = L[:1]
    y0, E = zoom.cell_bound(L1, (1.0, 1.0), c, h)
    ex = np.abs(_max_excursion(L1, (1.0, 1.0), c, h) - y0[None, :]).max(0)
    assert np.all(ex <= E)
    f = c - L1[0, :2].astype(np.float64)
    r2 = f @ f
    a = (f[1] ** 2 - f[0] ** 2) / r2 ** 2
    b = -2 * f[0] * f[1] / r2 ** 2
    lin = np.abs(np.array([[1 - a, -b], [-b, 1 + a]])) @ h
    assert np.any(ex > lin)
