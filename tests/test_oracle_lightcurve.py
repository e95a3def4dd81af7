"""Pins of the light-curve oracle (oracle/lightcurve.py) against closed forms and special cases.

Each pin is chosen so that a plausible slip fails it: a transposed map index or axis (the
rectangular and tilted maps), a missing half-pixel centre offset (the symmetric linear map), a
wrong Gaussian exponent or normalisation (the exponential map's exact moment), a wrong
inclusion or edge handling (the half-map edge case and off-map NaN), the magnitude convention,
and the whole chain on the analytic point-lens map (the uniform-disc closed form at the lens and
the point-source magnification along a track).
"""
import numpy as np

import synth
from oracle import lightcurve as lc


def test_uniform_map_is_unit_magnification():
    n_av = 7.0
    counts = np.full((30, 40), 7, np.uint32)
    tr = np.array([[3.0, 4.0, 35.0, 20.0]])
    for kind, size in (("gaussian", 2.5), ("disc", 4.0)):
        mu, mag = lc.light_curve(counts, (0, 0), (40, 30), (40, 30), n_av, tr, 9, kind, size)
        assert np.allclose(mu, 1.0, rtol=1e-15, atol=0) and np.allclose(mag, 0.0, atol=1e-15)


def test_magnitude_convention():
    counts = np.full((16, 16), 500, np.uint32)
    mu, mag = lc.light_curve(counts, (0, 0), (1, 1), (16, 16), 5.0, np.array([[0.5, 0.5, 0.5, 0.5]]), 1,
                             "disc", 0.2)
    assert mu[0, 0] == 100.0 and abs(mag[0, 0] + 5.0) < 1e-14   # 100x brighter = 5 magnitudes


def test_tiny_source_reads_single_pixels_of_a_rectangular_map():
    # support 0.4 pixel around a pixel centre holds exactly that pixel: mu = N_p / N_av
    n0, n1 = 37, 23
    counts = synth.count_map(9, (n0, n1), 50.0)
    lo, hi = (-3.0, 2.0), (-3.0 + 0.25 * n0, 2.0 + 0.5 * n1)
    # track along row 5 from column 2 to column 32 (n_points = 31 lands on every centre)
    y2 = lo[1] + 5.5 * 0.5
    tr = np.array([[lo[0] + 2.5 * 0.25, y2, lo[0] + 32.5 * 0.25, y2]])
    mu, _ = lc.light_curve(counts, lo, hi, (n0, n1), 2.0, tr, 31, "gaussian", 0.025)
    assert np.array_equal(mu[0], counts[5, 2:33] / 2.0)
    # the same along a column (axis 2)
    x1 = lo[0] + 11.5 * 0.25
    tr = np.array([[x1, lo[1] + 0.5 * 0.5, x1, lo[1] + 22.5 * 0.5]])
    mu, _ = lc.light_curve(counts, lo, hi, (n0, n1), 2.0, tr, 23, "disc", 0.1)
    assert np.array_equal(mu[0], counts[:, 11] / 2.0)


def test_linear_map_averages_to_centre_value():
    # N = a + b p1 + c p2 is odd about a pixel centre: any radially symmetric profile centred on
    # a pixel centre (support inside the map) returns the centre's value exactly
    n0, n1 = 64, 48
    p1, p2 = np.meshgrid(np.arange(n0), np.arange(n1))
    a, b, c = 1000, 7, 3
    counts = (a + b * p1 + c * p2).astype(np.uint32)
    pts = [(20, 30), (40, 10), (31, 24)]
    tr = np.array([[q1 + 0.5, q2 + 0.5, q1 + 0.5, q2 + 0.5] for q1, q2 in pts])
    for kind, size in (("gaussian", 2.0), ("disc", 6.3)):
        mu, _ = lc.light_curve(counts, (0, 0), (n0, n1), (n0, n1), 10.0, tr, 1, kind, size)
        want = np.array([(a + b * q1 + c * q2) / 10.0 for q1, q2 in pts])
        assert np.allclose(mu[:, 0], want, rtol=1e-13, atol=0), (kind, mu[:, 0], want)


def test_gaussian_moment_on_exponential_map():
    # for N = A exp(b1 x1 + b2 x2) a Gaussian of width sigma averages to
    # A exp(b . y) exp(|b|^2 sigma^2 / 2); with sigma = 8 pixels the pixel sum equals the integral
    # to far below the test tolerance, and a cutoff of 8 sigma (inside the map) drops a
    # negligible tail
    n, half = 192, 1.5
    sig = 8.0 * (2 * half / n)
    b1, b2 = 0.5 / sig, -0.25 / sig
    x = -half + (np.arange(n) + 0.5) * (2 * half / n)
    X1, X2 = np.meshgrid(x, x)
    A = 1.0e5
    N = np.rint(A * np.exp(b1 * X1 + b2 * X2))
    assert N.max() < 2.0 ** 32
    counts = N.astype(np.uint32)
    tr = np.array([[-0.3, 0.2, 0.4, -0.1]])
    mu, _ = lc.light_curve(counts, (-half, -half), (half, half), (n, n), A, tr, 5, "gaussian", sig, cutoff=8.0)
    f = np.linspace(0, 1, 5)
    y1, y2 = -0.3 + f * 0.7, 0.2 - f * 0.3
    want = np.exp(b1 * y1 + b2 * y2) * np.exp((b1 ** 2 + b2 ** 2) * sig ** 2 / 2)
    assert np.allclose(mu[0], want, rtol=2e-5), (mu[0] / want - 1)


def _point_lens_map(n, half, scale):
    # counts proportional to the point-lens magnification (u^2 + 2) / (u sqrt(u^2 + 4)) at pixel
    # centres (no pixel centre falls on the lens: n even)
    x = -half + (np.arange(n) + 0.5) * (2 * half / n)
    X1, X2 = np.meshgrid(x, x)
    u = np.hypot(X1, X2)
    mu = (u * u + 2) / (u * np.sqrt(u * u + 4))
    return np.rint(scale * mu).astype(np.uint32)


def test_uniform_disc_on_point_lens_closed_form():
    # a uniform disc of radius rho centred on a point lens: mu = sqrt(1 + 4 / rho^2)
    n, half, scale = 2000, 1.0, 1000.0
    counts = _point_lens_map(n, half, scale)
    tr = np.array([[0.0, 0.0, 0.0, 0.0]])
    for rho in (0.5, 0.9):
        mu, _ = lc.light_curve(counts, (-half, -half), (half, half), (n, n), scale, tr, 1, "disc", rho)
        want = np.sqrt(1 + 4 / rho ** 2)
        assert abs(mu[0, 0] / want - 1) < 2e-3, (rho, mu[0, 0], want)


def test_small_source_follows_point_lens_curve():
    # a source much smaller than its impact parameter sees the point-source magnification
    n, half, scale = 1000, 2.5, 1.0e4
    counts = _point_lens_map(n, half, scale)
    tr = np.array([[0.5, 0.1, 2.0, 0.1]])
    mu, mag = lc.light_curve(counts, (-half, -half), (half, half), (n, n), scale, tr, 7, "gaussian", 0.01)
    u = np.hypot(np.linspace(0.5, 2.0, 7), 0.1)
    want = (u * u + 2) / (u * np.sqrt(u * u + 4))
    assert np.allclose(mu[0], want, rtol=2e-3)
    assert np.allclose(mag[0], -2.5 * np.log10(want), atol=2.5e-3)


def test_edges_and_empty_support():
    # left half of the map holds a, right half b; a disc centred on the left edge sees only
    # the in-map half of itself, i.e. a; a source wholly off the map has no magnification
    counts = np.zeros((40, 40), np.uint32)
    counts[:, :20] = 30
    counts[:, 20:] = 90
    tr = np.array([[0.0, 20.0, 0.0, 20.0], [-10.0, 20.0, -10.0, 20.0]])
    mu, mag = lc.light_curve(counts, (0, 0), (40, 40), (40, 40), 3.0, tr, 1, "disc", 5.0)
    assert mu[0, 0] == 10.0
    assert np.isnan(mu[1, 0]) and np.isnan(mag[1, 0])


def test_single_point_track_uses_start():
    counts = synth.count_map(4, (20, 20), 10.0)
    a, _ = lc.light_curve(counts, (0, 0), (20, 20), (20, 20), 1.0, np.array([[5.5, 6.5, 15.0, 1.0]]), 1,
                          "disc", 0.3)
    assert a[0, 0] == counts[6, 5]


def test_synth_generators():
    m = synth.count_map(1, (300, 200), 25.0)
    assert m.shape == (200, 300) and m.dtype == np.uint32 and abs(m.mean() / 25.0 - 1) < 0.02
    t = synth.light_tracks(2, 50, (-1, -2), (3, 4), 1.5)
    assert t.shape == (50, 4)
    assert np.allclose(np.hypot(t[:, 2] - t[:, 0], t[:, 3] - t[:, 1]), 1.5)
    assert (t[:, 0] >= -1).all() and (t[:, 0] < 3).all() and (t[:, 1] >= -2).all() and (t[:, 1] < 4).all()


def test_frame_stack_reads_one_frame_per_point():
    # uniform frames of value c_k: point k sees c_k / N_av whatever the source; identical frames
    # reproduce the single-map curve
    n = (24, 16)
    vals = np.array([3, 9, 27, 81, 5], np.uint32)
    stack = np.stack([np.full((n[1], n[0]), v, np.uint32) for v in vals])
    tr = np.array([[2.0, 3.0, 20.0, 12.0], [5.5, 5.5, 5.5, 5.5]])
    mu, _ = lc.light_curve(stack, (0, 0), n, n, 3.0, tr, 5, "gaussian", 1.3)
    assert np.allclose(mu, np.broadcast_to(vals / 3.0, (2, 5)), rtol=1e-15, atol=0)
    one = synth.count_map(8, n, 12.0)
    mu1, _ = lc.light_curve(one, (0, 0), n, n, 3.0, tr, 5, "disc", 2.2)
    mus, _ = lc.light_curve(np.stack([one] * 5), (0, 0), n, n, 3.0, tr, 5, "disc", 2.2)
    assert np.array_equal(mu1, mus)
