"""Pins of the far-field split oracle (oracle/farfield.py)."""
import numpy as np

import oracle
import synth
from oracle import farfield as ff


def _field():
    lenses, r = synth.lens_field(41, 3000, kappa_star=0.5)
    return lenses


def test_near_rule_cases():
    L = np.array([[0.5, 0.5, 1, 0], [9.0, 0.5, 1, 0], [-7.9, 0.2, 1, 0], [6.0, 6.0, 1, 0],
                  [6.5, 6.5, 1, 0]], dtype=np.float32)
    lo, hi = np.array([0.0, 0.0]), np.array([1.0, 1.0])
    # inside; 8.0 to the right (not < 8); 7.9 to the left; corner at distance 5 sqrt(2); 5.5 sqrt(2)
    assert list(ff.near_mask(L, lo, hi, 8.0)) == [True, False, True, True, True]
    assert list(ff.near_mask(L, lo, hi, 7.5)) == [True, False, False, True, False]


def test_jacobian_matches_finite_differences_and_is_harmonic():
    L = _field()
    c = np.array([3.3, -1.7])
    far = ~ff.near_mask(L, c - 0.5, c + 0.5, 8.0)
    Lf = L[far]
    a, J = ff.affine_base(Lf, c)
    assert np.allclose(a, oracle.deflect(Lf, c[None])[0], rtol=1e-12)
    h = 1e-4
    fd = np.zeros((2, 2))
    for k in range(2):
        e = np.zeros(2)
        e[k] = h
        fd[:, k] = (oracle.deflect(Lf, (c + e)[None])[0] - oracle.deflect(Lf, (c - e)[None])[0]) / (2 * h)
    assert np.allclose(J, fd, rtol=1e-6, atol=1e-9)
    # a sum of point-lens fields is curl- and divergence-free away from the lenses
    assert abs(fd[0, 1] - fd[1, 0]) < 1e-8 and abs(fd[0, 0] + fd[1, 1]) < 1e-8


def test_affine_remainder_is_second_order():
    L = _field()
    c = np.array([-2.0, 4.0])
    Lf = L[~ff.near_mask(L, c - 1, c + 1, 8.0)]
    a, J = ff.affine_base(Lf, c)
    d = np.array([0.6, -0.35])
    r1 = np.linalg.norm(oracle.deflect(Lf, (c + d)[None])[0] - a - J @ d)
    r2 = np.linalg.norm(oracle.deflect(Lf, (c + d / 2)[None])[0] - a - J @ (d / 2))
    assert 3.0 < r1 / r2 < 5.0


def test_near_plus_far_is_all():
    L = _field()
    lo, hi = np.array([0.0, 0.0]), np.array([2.0, 0.5])
    m = ff.near_mask(L, lo, hi, 8.0)
    pts = np.array([[0.3, 0.1], [1.7, 0.45]])
    assert np.allclose(oracle.deflect(L[m], pts) + oracle.deflect(L[~m], pts), oracle.deflect(L, pts), rtol=1e-12)


def test_tile_targets_small_and_normalised():
    w = synth.workload_farfield(n_lens=20000, grid=8192)   # 64-ray tiles are 1.9 x 0.27 Einstein radii
    win = ((4032, 4064), (128, 64))
    res, st, a0, J, far = ff.tile_targets(w, win, (64, 64), 1, 0, 8.0, synth.fit_samples(3, 1024))
    assert res.shape == (1024, 2) and st > 0
    assert abs(np.sqrt(np.mean((res / st) ** 2)) - 1) < 1e-12
    # the residual after the affine base is far smaller than the far field itself
    assert st < 1e-2 * np.linalg.norm(a0)


def test_quad_samples_layout():
    g = synth.fit_samples_quads(7, 4096)
    assert g.shape == (4096, 2) and g.dtype == np.float32 and np.all(np.abs(g) <= 1.0)
    q = g.reshape(16, 4, 64, 2)
    assert np.array_equal(q[:, 1:, :, 0], np.broadcast_to(q[:, :1, :, 0], (16, 3, 64)))
    assert len(np.unique(g[:, 0])) == 1024 and len(np.unique(g[:, 1])) == 4096
    assert abs(g[:, 0].mean()) < 0.1 and abs(g[:, 1].mean()) < 0.1
