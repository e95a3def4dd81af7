"""FP64 oracle of the far-field split of the deflection sum -- TEST INFRASTRUCTURE ONLY.

For a tile of the ray grid (its rectangle is the union of its rays' grid cells), the lenses
closer than r_near to the rectangle (FP64 Euclidean distance from the lens to the rectangle)
form the near set; all others form the far set.  The deflection (section 1, eq. 2) splits
into the two subset sums (section 2, eq. 5): alpha = alpha_near + alpha_far.  The far part's
affine base at the tile centre c is alpha_far(c) + J(c) (x - c) with
J = d alpha_far / d x; for a point lens m at x_i with d = x - x_i, r^2 = |d|^2:
    d alpha_1/d x_1 = m (d_2^2 - d_1^2) / r^4,  d alpha_1/d x_2 = -2 m d_1 d_2 / r^4,
    d alpha_2/d x_2 = m (d_1^2 - d_2^2) / r^4.
The fit target at a sample point p = c + u h (rounded to float32) is the residual
alpha_far(p) - [alpha_far(c) + J (p - c)], normalised by its RMS over the tile's samples.
"""
from __future__ import annotations

import numpy as np

from . import deflect


def tile_rect(w, window, tile_rays, tx, ty):
    """(lo, hi, c, h, (i0, n)) of tile (tx, ty) of the window ((wlo1, wlo2), (wn1, wn2))."""
    (wl1, wl2), (wn1, wn2) = window
    t = [(w.grid_hi[k] - w.grid_lo[k]) / w.grid_n[k] for k in range(2)]
    i0 = (wl1 + tx * tile_rays[0], wl2 + ty * tile_rays[1])
    n = (min(tile_rays[0], wl1 + wn1 - i0[0]), min(tile_rays[1], wl2 + wn2 - i0[1]))
    lo = np.array([w.grid_lo[k] + i0[k] * t[k] for k in range(2)])
    hi = np.array([w.grid_lo[k] + (i0[k] + n[k]) * t[k] for k in range(2)])
    return lo, hi, 0.5 * (lo + hi), 0.5 * (hi - lo), (i0, n)


def near_mask(lenses, lo, hi, r_near):
    """True for lenses closer than r_near to the rectangle [lo, hi]."""
    x = lenses[:, 0].astype(np.float64)
    y = lenses[:, 1].astype(np.float64)
    ex = np.maximum(np.maximum(lo[0] - x, x - hi[0]), 0.0)
    ey = np.maximum(np.maximum(lo[1] - y, y - hi[1]), 0.0)
    return ex * ex + ey * ey < r_near * r_near


def affine_base(lenses, c):
    """alpha(c) (2) and the 2x2 Jacobian J(c) of the deflection of `lenses`, FP64."""
    d = np.asarray(c, dtype=np.float64)[None, :] - lenses[:, :2].astype(np.float64)
    m = lenses[:, 2].astype(np.float64)
    r2 = d[:, 0] ** 2 + d[:, 1] ** 2
    a = np.array([np.sum(m * d[:, 0] / r2), np.sum(m * d[:, 1] / r2)])
    j11 = np.sum(m * (d[:, 1] ** 2 - d[:, 0] ** 2) / r2 ** 2)
    j12 = np.sum(-2.0 * m * d[:, 0] * d[:, 1] / r2 ** 2)
    j22 = np.sum(m * (d[:, 0] ** 2 - d[:, 1] ** 2) / r2 ** 2)
    return a, np.array([[j11, j12], [j12, j22]])


def tile_targets(w, window, tile_rays, tx, ty, r_near, samples, threads=8):
    """Residual samples (n x 2, unnormalised), their RMS s_t, alpha_far(c), J, and the far set."""
    from concurrent.futures import ThreadPoolExecutor
    lo, hi, c, h, _ = tile_rect(w, window, tile_rays, tx, ty)
    far = ~near_mask(w.lenses, lo, hi, r_near)
    Lf = np.ascontiguousarray(w.lenses[far])
    a0, J = affine_base(Lf, c)
    p = (c[None, :] + samples.astype(np.float64) * h[None, :]).astype(np.float32).astype(np.float64)
    parts = np.array_split(p, threads)
    with ThreadPoolExecutor(threads) as ex:
        af = np.concatenate(list(ex.map(lambda q: deflect(Lf, q), parts)))
    res = af - (a0[None, :] + (p - c[None, :]) @ J.T)
    st = float(np.sqrt(np.mean(res ** 2)))
    return res, (st if st > 0 else 1.0), a0, J, far
