"""FP64 oracle of light curves read off a magnification map -- TEST INFRASTRUCTURE ONLY.

Only the tests, the smoke check and the benchmark's CPU baseline use this module; it shares
no code with the HIP library.

Thompson et al. 2009 (section 1) turn each map pixel's ray count into a magnification,
mu = N / N_av (eq. 4), and use the maps to produce light curves: a source of finite size
moving across the map.  Written out plainly here, for every track point and over EVERY map
pixel (no bounding box):

  pixel centre  c_k = lo_k + (p_k + 1/2) w_k,   w_k = (hi_k - lo_k) / n_k
  track point   y = s + f (e - s),  f = k / (n_points - 1)   (f = 0 when n_points = 1)
  weight        w_p = exp(-|c - y|^2 / (2 sigma^2))  (Gaussian)  or 1 (uniform disc),
                only for pixels with |c - y|^2 <= R^2  (R = cutoff sigma, cutoff 0 -> 4;
                R = radius for the disc)
  mu(y)         = sum w_p N_p / (N_av sum w_p)    (NaN when no pixel centre is inside)
  delta m       = -2.5 log10 mu

Readings (the paper describes the use, not the estimator): the source brightness profile is a
circular Gaussian or a uniform disc sampled at pixel centres and renormalised over the pixels
that fall inside the map, so a source near the edge sees only the map's part of itself.
"""
from __future__ import annotations

import numpy as np


def _support(kind: str, size: float, cutoff: float) -> float:
    if kind == "gaussian":
        return (cutoff if cutoff > 0 else 4.0) * size
    if kind == "disc":
        return size
    raise ValueError(kind)


def light_curve(counts, map_lo, map_hi, map_n, n_av, tracks, n_points, kind="gaussian", size=0.1,
                cutoff=0.0, sums=False):
    """mu and delta-m, each (n_tracks, n_points); with sums=True also the weighted count sum and
    the weight sum of every point.

    counts is one map read by every point, or a stack of n_points maps of which point k reads
    map k (a field whose lenses move between the frames, section 4)."""
    pix = int(map_n[0]) * int(map_n[1])
    counts = np.asarray(counts)
    if counts.size == pix:
        frames = [counts.reshape(int(map_n[1]), int(map_n[0])).astype(np.float64)] * n_points
    elif counts.size == pix * n_points:
        frames = [f.astype(np.float64) for f in counts.reshape(n_points, int(map_n[1]), int(map_n[0]))]
    else:
        raise ValueError("counts must hold one map or n_points maps")
    tracks = np.asarray(tracks, dtype=np.float64).reshape(-1, 4)
    w0 = (map_hi[0] - map_lo[0]) / map_n[0]
    w1 = (map_hi[1] - map_lo[1]) / map_n[1]
    c1 = map_lo[0] + (np.arange(map_n[0], dtype=np.float64) + 0.5) * w0      # column centres
    c2 = map_lo[1] + (np.arange(map_n[1], dtype=np.float64) + 0.5) * w1      # row centres
    R = _support(kind, size, cutoff)
    nt = len(tracks)
    mu = np.empty((nt, n_points))
    num = np.empty((nt, n_points))
    den = np.empty((nt, n_points))
    for t in range(nt):
        s1, s2, e1, e2 = tracks[t]
        for k in range(n_points):
            f = k / (n_points - 1) if n_points > 1 else 0.0
            y1 = s1 + f * (e1 - s1)
            y2 = s2 + f * (e2 - s2)
            d1 = c1[None, :] - y1
            d2 = c2[:, None] - y2
            r2 = d1 * d1 + d2 * d2
            inside = r2 <= R * R
            wgt = np.exp(-r2 / (2.0 * size * size)) if kind == "gaussian" else np.ones_like(r2)
            wgt = np.where(inside, wgt, 0.0)
            num[t, k] = np.sum(wgt * frames[k])
            den[t, k] = np.sum(wgt)
            mu[t, k] = num[t, k] / (den[t, k] * n_av) if den[t, k] > 0 else np.nan
    with np.errstate(divide="ignore", invalid="ignore"):
        mag = -2.5 * np.log10(mu)
    return (mu, mag, num, den) if sums else (mu, mag)
