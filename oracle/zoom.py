"""FP64 oracle of the zoom's cell bound -- TEST INFRASTRUCTURE ONLY.

A zoom (section 4: a selected source-plane area recomputed at higher ray density) may skip an
image-plane cell only if no ray in it can land in the area.  For the rectangle c +- h of the
image plane and the lens equation y = diag(l1, l2) x - alpha(x) (eqs. 1, 2, 6) this module
bounds y over the rectangle, written from the mathematics:

  lenses at r = |c - x_i| >= 3 rho (rho = |h|): the deflection is m / conj(z - z_i) in complex
  form, so its Jacobian at c is m / r^4 [[f2^2 - f1^2, -2 f1 f2], [-2 f1 f2, f1^2 - f2^2]] and its
  second derivative has norm 2 m / r^3; Taylor's theorem bounds the remainder over the segment
  by rho^2 sum m / (r - rho)^3 <= rho^2 (3/2)^3 sum m / r^3;
  lenses closer than 3 rho: |alpha_i(x) - alpha_i(c)| <= |alpha_i(x)| + |alpha_i(c)| <= 2 m / delta_i
  (delta_i = distance from the lens to the rectangle); a lens inside the rectangle leaves y
  unbounded.

Returns y(c) and the per-axis half-widths E of a box that holds y over the whole rectangle.
"""
from __future__ import annotations

import numpy as np


def cell_bound(lenses, lam, c, h):
    L = np.asarray(lenses, dtype=np.float64).reshape(-1, 4)
    c = np.asarray(c, dtype=np.float64)
    h = np.asarray(h, dtype=np.float64)
    f = c[None, :] - L[:, :2]
    m = L[:, 2]
    r2 = f[:, 0] ** 2 + f[:, 1] ** 2
    alpha = np.array([np.sum(m * f[:, 0] / r2), np.sum(m * f[:, 1] / r2)])
    y = np.array([lam[0] * c[0], lam[1] * c[1]]) - alpha
    rho = float(np.hypot(h[0], h[1]))
    near = r2 < 9.0 * rho * rho
    ex = np.maximum(np.abs(f[near, 0]) - h[0], 0.0)
    ey = np.maximum(np.abs(f[near, 1]) - h[1], 0.0)
    delta = np.hypot(ex, ey)
    if np.any(delta == 0.0):
        return y, np.array([np.inf, np.inf])
    far = ~near
    mf, ff, rf2 = m[far], f[far], r2[far]
    a = np.sum(mf * (ff[:, 1] ** 2 - ff[:, 0] ** 2) / rf2 ** 2)
    b = np.sum(-2.0 * mf * ff[:, 0] * ff[:, 1] / rf2 ** 2)
    J = np.array([[lam[0] - a, -b], [-b, lam[1] + a]])        # d y / d x from the far lenses
    lin = np.abs(J) @ h
    rem = rho * rho * 3.375 * np.sum(mf / rf2 ** 1.5)
    nearv = 2.0 * np.sum(m[near] / delta)
    return y, lin + rem + nearv
