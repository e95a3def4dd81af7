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


def test_tile_rect_hand_computed_ragged_window():
    # grid [-3, 5) x [-2, 2) cut into 16 x 8 cells of 0.5; window of 10 x 5 rays at (3, 1); tiles of
    # 4 x 3 rays.  Tile (2, 1) starts at ray (11, 4) and is ragged: 2 x 2 rays, the cells
    # [2.5, 3.5) x [0, 1)
    w = synth.Workload("rect", np.zeros((0, 4), np.float32), 0.0, 0.0, (-3.0, -2.0), (5.0, 2.0), (16, 8),
                       (-1.0, -1.0), (1.0, 1.0), (4, 4))
    win = ((3, 1), (10, 5))
    lo, hi, c, h, (i0, n) = ff.tile_rect(w, win, (4, 3), 2, 1)
    assert tuple(i0) == (11, 4) and tuple(n) == (2, 2)
    assert list(lo) == [2.5, 0.0] and list(hi) == [3.5, 1.0]
    assert list(c) == [3.0, 0.5] and list(h) == [0.5, 0.5]
    # an interior tile: rays (3..6) x (1..3), cells [-1.5, 0.5) x [-1.5, 0)
    lo, hi, c, h, (i0, n) = ff.tile_rect(w, win, (4, 3), 0, 0)
    assert tuple(i0) == (3, 1) and tuple(n) == (4, 3)
    assert list(lo) == [-1.5, -1.5] and list(hi) == [0.5, 0.0] and list(h) == [1.0, 0.75]


def _complex_residual(m, zl, c, p):
    """Residual of one point lens after its affine base at c, in complex form: the deflection of
    a point lens is a(z) = m / conj(z - z_l), whose derivative along conj(z) is -m / conj(z - z_l)^2,
    so a(p) - a(c) - (-m / conj(c - z_l)^2) conj(p - c)."""
    a = lambda z: m / np.conj(z - zl)
    return a(p) - a(c) + m / np.conj(c - zl) ** 2 * np.conj(p - c)


def test_tile_targets_one_far_lens_closed_form():
    # Near lenses leave the target; the one far lens gives a residual known in closed form at the
    # tile's corners and centre, which pins the far set, the sample placement p = c + u h, the
    # Jacobian's signs and orientation and the affine subtraction
    grid_lo, grid_hi, gn = (-4.0, -2.0), (4.0, 2.0), (64, 32)        # cells of 1/8
    L = np.array([[0.3, 0.1, 1.0, 0], [-2.0, 1.5, 0.4, 0],            # near the tile
                  [11.0, -6.5, 0.7, 0]], dtype=np.float32)           # 12.6 from the tile: far
    w = synth.Workload("one-far", L, 0.0, 0.0, grid_lo, grid_hi, gn, (-1.0, -1.0), (1.0, 1.0), (4, 4))
    win = ((8, 4), (48, 24))
    u = np.array([[-1, -1], [1, 1], [1, -1], [-1, 1], [0, 0], [0.5, -0.25]], dtype=np.float32)
    res, st, a0, J, far = ff.tile_targets(w, win, (16, 8), 1, 1, 8.0, u, threads=1)
    assert list(far) == [False, False, True]
    # tile (1, 1): rays (24..39) x (12..19), cells [-1, 1) x [-0.5, 0.5)
    c = 0.0 + 0.0j
    corners = np.array([-1 - 0.5j, 1 + 0.5j, 1 - 0.5j, -1 + 0.5j, 0j, 0.5 - 0.125j])
    zl = complex(11.0, -6.5)
    m = float(np.float32(0.7))                          # the lens record's float32 mass
    want = _complex_residual(m, zl, c, corners)
    got = res[:, 0] + 1j * res[:, 1]
    assert np.allclose(got, want, rtol=1e-9, atol=1e-15), np.abs(got - want).max()
    assert abs(got[4]) < 1e-15                         # u = 0 is the centre: no residual
    a = m / np.conj(c - zl)
    assert np.allclose(a0, [a.real, a.imag], rtol=1e-14)
    # the residual grows as the square of the offset: u = 1/2 against u = 1 along the diagonal
    half = _complex_residual(m, zl, c, np.array([0.5 + 0.25j]))[0]
    assert 3.5 < abs(want[1]) / abs(half) < 4.5


def test_tile_targets_residual_is_second_order_in_tile_size():
    # the same field and samples on tiles of 64 x 64 and 32 x 32 rays around one centre: the RMS
    # residual after the exact affine base falls by about 4 when the tile halves
    w = synth.workload_farfield(n_lens=20000, grid=8192)
    u = synth.fit_samples(5, 1024)
    big = ff.tile_targets(w, ((4032, 4064), (64, 64)), (64, 64), 0, 0, 8.0, u)
    small = ff.tile_targets(w, ((4048, 4080), (32, 32)), (32, 32), 0, 0, 8.0, u)
    lo_b, hi_b, c_b, *_ = ff.tile_rect(w, ((4032, 4064), (64, 64)), (64, 64), 0, 0)
    lo_s, hi_s, c_s, *_ = ff.tile_rect(w, ((4048, 4080), (32, 32)), (32, 32), 0, 0)
    assert np.array_equal(c_b, c_s)
    # compare on the lenses far from both tiles (the smaller tile's far set is larger)
    both = big[4] & small[4]
    Lf = np.ascontiguousarray(w.lenses[both])
    rms = []
    for lo, hi, c in ((lo_b, hi_b, c_b), (lo_s, hi_s, c_s)):
        h = 0.5 * (hi - lo)
        p = (c[None, :] + u.astype(np.float64) * h[None, :]).astype(np.float32).astype(np.float64)
        a0, J = ff.affine_base(Lf, c)
        r = oracle.deflect(Lf, p) - (a0[None, :] + (p - c[None, :]) @ J.T)
        rms.append(np.sqrt(np.mean(r ** 2)))
    assert 3.5 < rms[0] / rms[1] < 4.5, rms
    # and tile_targets' own residual of the big tile agrees with that construction on its far set
    assert abs(big[1] / rms[0] - 1) < 0.2
