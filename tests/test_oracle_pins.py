"""Pins of the FP64 CPU oracle against facts fixed by the paper and by the mathematics.

None of these checks retypes the oracle's formula: each compares it with a
closed form, an exact integer count, an exact rational evaluation, a
symmetry, or a published fixture, chosen so that a dropped term, a wrong
sign, a swapped axis or a wrong index in the oracle fails at least one.
"""
import math
import os
from fractions import Fraction

import numpy as np
import pytest

import oracle
import synth
from oracle import exact

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _wl(lenses, kappa_c, gamma, glo, ghi, gn, mlo, mhi, mn, name="t"):
    return synth.Workload(name, np.ascontiguousarray(lenses, dtype=np.float32).reshape(-1, 4),
                          kappa_c, gamma, tuple(glo), tuple(ghi), tuple(gn), tuple(mlo), tuple(mhi),
                          tuple(mn))


# ---------------------------------------------------------------- generators

def test_splitmix64_published_outputs():
    vals = [int(l, 16) for l in open(os.path.join(GOLDEN, "splitmix64_seed0.txt"))
            if l.strip() and not l.startswith("#")]
    got = synth.mix64(synth.GOLDEN * np.arange(1, 4, dtype=np.uint64))
    assert [int(v) for v in got] == vals


def test_lens_field_statistics():
    lenses, r = synth.lens_field(11, 20000, kappa_star=0.45)
    m = lenses[:, 2].astype(np.float64)
    # sum(m) / R^2 equals the requested convergence
    assert abs(m.sum() / r ** 2 - 0.45) < 1e-6
    # Salpeter slope 2.35 on [0.1, 1]: <m> = (p/(p+1)) (b^(p+1)-a^(p+1))/(b^p-a^p), p = -1.35
    p = -1.35
    mean = (p / (p + 1)) * (1 - 0.1 ** (p + 1)) / (1 - 0.1 ** p)
    assert abs(m.mean() - mean) < 4 * m.std() / math.sqrt(len(m))
    assert m.min() >= 0.1 and m.max() <= 1.0
    rad = np.hypot(lenses[:, 0].astype(np.float64), lenses[:, 1].astype(np.float64))
    assert rad.max() < r
    # uniform in the disc: fraction inside R/2 is 1/4
    frac = np.mean(rad < r / 2)
    assert abs(frac - 0.25) < 4 * math.sqrt(0.25 * 0.75 / len(rad))
    # deterministic in the seed
    again, _ = synth.lens_field(11, 20000, kappa_star=0.45)
    assert np.array_equal(again, lenses)


def test_shooting_region_is_dyadic_lattice():
    w = synth.workload_paper(n_lens=1000, grid=4096)  # region does not depend on N_* here
    lo, hi, n = synth.shooting_region((10.0, 10.0), 0.45, 0.45, (4096, 4096), 222.9)
    assert lo == (-120.0, -12.0) and hi == (120.0, 12.0)
    step = [(hi[k] - lo[k]) / n[k] for k in range(2)]
    q = 2 * synth.ulp32(120 + 222.9)
    for s in step:
        assert (Fraction(s) / Fraction(q)).denominator == 1
    assert w.grid_n == (4096, 4096)


# ---------------------------------------------------------------- ray grid

@pytest.mark.parametrize("lo,hi,n", [(-120.0, 120.0, 4096), (-12.0, 12.0, 4096), (-2.0, 6.0, 64)])
def test_axis_dyadic_is_exact_cell_centre(lo, hi, n):
    got = oracle.axis(lo, hi, n)
    for i in list(range(0, n, max(1, n // 97))) + [n - 1]:
        assert float(got[i]) == exact.round_to_float32(exact.exact_coord(lo, hi, n, i))


def test_axis_non_dyadic_within_one_ulp():
    got = oracle.axis(-10.0, 10.0, 1000)
    for i in range(0, 1000, 7):
        ex = exact.exact_coord(-10.0, 10.0, 1000, i)
        assert abs(Fraction(float(got[i])) - ex) <= Fraction(float(np.spacing(np.float32(abs(float(ex))))))
    # symmetric grid: coordinate i and n-1-i are negatives
    assert np.array_equal(got, -got[::-1])


# ---------------------------------------------------------------- deflection

def test_square_of_lenses_closed_form():
    # Four equal masses at the fourth roots of unity (exact in float32).  With
    # z = x1 + i x2, conj(alpha) = sum m / (z - z_k) = 4 m z^3 / (z^4 - 1).
    m = 0.75
    L = np.array([[1, 0, m, 0], [0, 1, m, 0], [-1, 0, m, 0], [0, -1, m, 0]], dtype=np.float32)
    rng = np.random.default_rng(3)
    pts = rng.uniform(-3, 3, size=(200, 2))
    a = oracle.deflect(L, pts)
    z = pts[:, 0] + 1j * pts[:, 1]
    ref = np.conj(4 * m * z ** 3 / (z ** 4 - 1))
    assert np.allclose(a[:, 0], ref.real, rtol=1e-11, atol=1e-11)
    assert np.allclose(a[:, 1], ref.imag, rtol=1e-11, atol=1e-11)


def test_regular_polygon_closed_form():
    # N masses on a circle of radius a (float32-rounded vertices): conj(alpha) ~ N m z^(N-1)/(z^N - a^N)
    N, a, m = 7, 2.5, 0.3
    ang = 2 * np.pi * np.arange(N) / N
    L = np.zeros((N, 4), dtype=np.float32)
    L[:, 0], L[:, 1], L[:, 2] = a * np.cos(ang), a * np.sin(ang), m
    rng = np.random.default_rng(5)
    pts = np.concatenate([rng.uniform(-1.5, 1.5, size=(100, 2)), rng.uniform(4, 8, size=(100, 2))])
    got = oracle.deflect(L, pts)
    z = pts[:, 0] + 1j * pts[:, 1]
    ref = np.conj(N * m * z ** (N - 1) / (z ** N - a ** N))
    # float32 rounding of the vertices perturbs alpha by ~1e-7 relative
    assert np.allclose(got[:, 0] + 1j * got[:, 1], ref, rtol=2e-6, atol=2e-7)


def test_deflection_additive_over_lens_sets():
    lenses, _ = synth.lens_field(7, 300, kappa_star=0.4)
    rng = np.random.default_rng(8)
    pts = rng.uniform(-10, 10, size=(64, 2))
    a_all = oracle.deflect(lenses, pts)
    a_sum = oracle.deflect(lenses[:120], pts) + oracle.deflect(lenses[120:], pts)
    assert np.allclose(a_all, a_sum, rtol=1e-12, atol=1e-12)


def test_single_lens_far_field_is_point_mass():
    L = np.array([[0.5, -0.25, 0.6, 0]], dtype=np.float32)
    pts = np.array([[100.0, 0.0], [0.0, -300.0]])
    a = oracle.deflect(L, pts)
    d = pts - np.array([0.5, -0.25])
    ref = 0.6 * d / (d ** 2).sum(1, keepdims=True)
    assert np.allclose(a, ref, rtol=1e-14)


# ---------------------------------------------------------------- brute force

@pytest.mark.parametrize("seed", [1, 2, 3])
def test_oracle_matches_exact_rational(seed):
    rng = np.random.default_rng(seed)
    n_l = int(rng.integers(1, 4))
    L = np.zeros((n_l, 4), dtype=np.float32)
    L[:, :2] = rng.uniform(-1.5, 1.5, size=(n_l, 2))
    L[:, 2] = rng.uniform(0.1, 1.0, size=n_l)
    kc, g = [(0.0, 0.0), (0.25, 0.125), (0.3, -0.2)][seed - 1]
    w = _wl(L, kc, g, (-2.0, -2.0), (2.0, 2.0), (16, 16), (-1.5, -1.5), (1.5, 1.5), (12, 12))
    idx = np.arange(256)
    y, pix = oracle.trace(w, idx)
    xs1 = oracle.axis(-2.0, 2.0, 16)
    for r in idx:
        i1, i2 = r % 16, r // 16
        ey1, ey2, ep = exact.trace(L, kc, g, w.grid_lo, w.grid_hi, w.grid_n, w.map_lo, w.map_hi,
                                   w.map_n, xs1[i1], xs1[i2])
        assert pix[r] == ep
        if ey1 is not None:
            assert abs(y[r, 0] - float(ey1)) <= 1e-12 * max(1.0, abs(float(ey1)))
            assert abs(y[r, 1] - float(ey2)) <= 1e-12 * max(1.0, abs(float(ey2)))


def test_ray_on_a_lens_is_lost():
    # lens exactly at a ray position: the deflection is undefined, the ray is lost
    xs = oracle.axis(-1.0, 1.0, 8)
    L = np.array([[xs[3], xs[5], 1.0, 0]], dtype=np.float32)
    w = _wl(L, 0.0, 0.0, (-1.0, -1.0), (1.0, 1.0), (8, 8), (-4.0, -4.0), (4.0, 4.0), (4, 4))
    y, pix = oracle.trace(w, [5 * 8 + 3, 0])
    assert pix[0] == -1 and not np.isfinite(y[0]).all()
    assert pix[1] >= 0
    counts, lost = oracle.shoot(w)
    assert lost >= 1 and counts.sum() + lost == 64


# ---------------------------------------------------------------- single lens

def _single_lens_setup(n=1200, half=4.0):
    L = np.array([[0.0, 0.0, 1.0, 0.0]], dtype=np.float32)
    return _wl(L, 0.0, 0.0, (-half, -half), (half, half), (n, n), (-4.0, -4.0), (4.0, 4.0), (8, 8))


def test_single_lens_disc_count_identity():
    # For m=1 at the origin |y| = | |x| - 1/|x| |, so |y| < u  <=>  r- < |x| < r+ with
    # r+- = (sqrt(u^2+4) +- u)/2: an exact integer identity between ray counts.
    w = _single_lens_setup(n=600)
    xs = oracle.axis(w.grid_lo[0], w.grid_hi[0], w.grid_n[0]).astype(np.float64)
    X1, X2 = np.meshgrid(xs, xs)
    rx = np.hypot(X1, X2).ravel()
    y, _ = oracle.trace_parallel(w, np.arange(w.n_rays))
    ry = np.hypot(y[:, 0], y[:, 1])
    for u in (0.1, 0.5, 1.0, 2.0, 3.0):
        rp = (math.sqrt(u * u + 4) + u) / 2
        rm = (math.sqrt(u * u + 4) - u) / 2
        amb = (np.abs(rx - rp) < 1e-9) | (np.abs(rx - rm) < 1e-9) | (np.abs(ry - u) < 1e-9)
        lhs = np.sum((ry < u) & ~amb)
        rhs = np.sum((rx > rm) & (rx < rp) & ~amb)
        assert lhs == rhs and lhs > 0


def test_single_lens_annulus_mean_magnification():
    # Image area mapped into |y| < u is pi u sqrt(u^2+4), so the mean magnification over the
    # source annulus [ua, ub) is (ub sqrt(ub^2+4) - ua sqrt(ua^2+4)) / (ub^2 - ua^2).
    w = _single_lens_setup(n=1600)
    y, _ = oracle.trace_parallel(w, np.arange(w.n_rays))
    ry = np.hypot(y[:, 0], y[:, 1])
    cell = ((w.grid_hi[0] - w.grid_lo[0]) / w.grid_n[0]) ** 2
    for ua, ub in [(0.05, 0.1), (0.2, 0.3), (0.5, 0.7), (1.0, 1.5), (2.0, 3.0)]:
        n_in = np.sum((ry >= ua) & (ry < ub))
        mu_meas = n_in * cell / (math.pi * (ub * ub - ua * ua))
        mu_ref = (ub * math.sqrt(ub * ub + 4) - ua * math.sqrt(ua * ua + 4)) / (ub * ub - ua * ua)
        assert abs(mu_meas / mu_ref - 1) < 5e-3, (ua, ub, mu_meas, mu_ref)


def test_single_lens_mu_of_u_profile():
    # point-source magnification mu(u) = (u^2 + 2) / (u sqrt(u^2 + 4)) from thin annuli
    w = _single_lens_setup(n=1600)
    y, _ = oracle.trace_parallel(w, np.arange(w.n_rays))
    ry = np.hypot(y[:, 0], y[:, 1])
    cell = ((w.grid_hi[0] - w.grid_lo[0]) / w.grid_n[0]) ** 2
    for u in (0.3, 0.6, 1.0, 2.0):
        du = 0.02
        n_in = np.sum((ry >= u - du) & (ry < u + du))
        mu_meas = n_in * cell / (math.pi * ((u + du) ** 2 - (u - du) ** 2))
        mu_ref = (u * u + 2) / (u * math.sqrt(u * u + 4))
        assert abs(mu_meas / mu_ref - 1) < 1e-2, (u, mu_meas, mu_ref)


# ---------------------------------------------------------------- smooth sheet + shear

def _exact_axis_counts(lo, hi, n, lam, mlo, mhi, mn):
    """Per source pixel, how many float32 grid coordinates X satisfy mlo + p d <= lam X < mlo + (p+1) d."""
    lamq = Fraction(lam)
    out = np.zeros(mn, dtype=np.int64)
    for i in range(n):
        X = Fraction(exact.round_to_float32(exact.exact_coord(lo, hi, n, i)))
        p = math.floor((lamq * X - Fraction(mlo)) * mn / (Fraction(mhi) - Fraction(mlo)))
        if 0 <= p < mn:
            out[p] += 1
    return out


@pytest.mark.parametrize("kappa_c,gamma", [(0.25, 0.125), (0.5, -0.25), (1.25, 0.0), (0.0, 0.0)])
def test_smooth_sheet_exact_pixel_counts(kappa_c, gamma):
    # N_* = 0: y_k = lambda_k x_k with lambda_1 = 1 - kappa_c - gamma, lambda_2 = 1 - kappa_c + gamma.
    # Each pixel count is the product of two exact 1-D lattice counts.
    w = _wl(np.zeros((0, 4)), kappa_c, gamma, (-8.0, -6.0), (8.0, 6.0), (256, 192), (-3.0, -2.5),
            (3.0, 2.5), (24, 20))
    counts, lost = oracle.shoot(w)
    c1 = _exact_axis_counts(-8.0, 8.0, 256, 1 - kappa_c - gamma, -3.0, 3.0, 24)
    c2 = _exact_axis_counts(-6.0, 6.0, 192, 1 - kappa_c + gamma, -2.5, 2.5, 20)
    assert np.array_equal(counts.astype(np.int64), np.outer(c2, c1))
    assert counts.sum() + lost == w.n_rays


def test_n_av_is_unlensed_rays_per_pixel():
    # eq. 4: N_av is the number of rays a pixel receives without lensing, so with no lenses and no
    # macro term every pixel whose edges fall on ray-cell edges holds exactly N_av rays (mu = 1);
    # under a smooth sheet y = x / 2 (kappa_c = 1/2) a pixel's preimage is twice as wide per axis,
    # so it receives 4 N_av rays and mu = 1 / lambda^2 = 4 exactly
    w = _wl(np.zeros((0, 4)), 0.0, 0.0, (-1.0, -1.5), (1.0, 1.5), (64, 48), (-1.0, -1.5), (1.0, 1.5), (16, 12))
    counts, lost = oracle.shoot(w)
    assert oracle.n_av(w) == 16.0 and lost == 0
    assert np.array_equal(counts, np.full((12, 16), 16, np.uint32))
    assert np.array_equal(counts / oracle.n_av(w), np.ones((12, 16)))
    w = _wl(np.zeros((0, 4)), 0.5, 0.0, (-2.0, -2.0), (2.0, 2.0), (128, 128), (-1.0, -1.0), (1.0, 1.0), (16, 16))
    counts, lost = oracle.shoot(w)
    assert oracle.n_av(w) == 16.0
    assert np.array_equal(counts / oracle.n_av(w), np.full((16, 16), 4.0))


# ---------------------------------------------------------------- random fields

def test_mean_magnification_identity():
    # Over a large source area the mean magnification is 1/|(1-kappa)^2 - gamma^2|.  One
    # realisation scatters by ~3.5% (finite star count); four seeds average to ~1.8%.
    ks, g = 0.3, 0.2
    ref = 1.0 / abs((1 - ks) ** 2 - g ** 2)
    vals = []
    for seed in (21, 22, 23, 24):
        lenses, r = synth.lens_field(seed, 8000, kappa_star=ks)
        lo, hi, n = synth.shooting_region((10.0, 10.0), ks, g, (600, 600), r, margin=1.6)
        w = _wl(lenses, 0.0, g, lo, hi, n, (-10.0, -10.0), (10.0, 10.0), (40, 40))
        counts, lost = oracle.shoot_parallel(w)
        assert counts.sum() + lost == w.n_rays
        vals.append(counts.sum() / (oracle.n_av(w) * 40 * 40))
    assert abs(np.mean(vals) / ref - 1) < 0.05, (vals, ref)


def test_windows_add_up_to_whole_grid():
    w = synth.workload_small()
    full, lost = oracle.shoot(w)
    assert full.sum() + lost == w.n_rays
    acc = np.zeros_like(full)
    acc_lost = 0
    for (a, b) in [((0, 0), (1000, 300)), ((0, 300), (400, 700)), ((400, 300), (600, 700))]:
        c, l = oracle.shoot(w, (a, b))
        acc += c
        acc_lost += l
    assert np.array_equal(acc, full) and acc_lost == lost


def test_mirror_symmetry_is_exact():
    w = synth.workload_small()
    mir = np.array(w.lenses)
    mir[:, 0] = -mir[:, 0]
    wm = _wl(mir, 0.0, 0.0, w.grid_lo, w.grid_hi, w.grid_n, w.map_lo, w.map_hi, w.map_n)
    a, la = oracle.shoot(w)
    b, lb = oracle.shoot(wm)
    assert la == lb
    assert np.array_equal(a, b[:, ::-1])


# ---------------------------------------------------------------- paper fixtures

def test_flop_convention_reproduces_paper_rates():
    # Gflop/s = 10 flop x N_av x N_pix x N_* / T (appendix A; section 3.1)
    rows = [list(map(float, l.split())) for l in open(os.path.join(GOLDEN, "paper_table2.txt"))
            if l.strip() and not l.startswith("#")]
    quoted = {1: 182.0, 2: 364.0, 3: 1287.0}
    for side, *hours in rows:
        if side < 1024:
            continue  # small grids are overhead-dominated in the paper's own data
        for col, h in enumerate(hours, start=1):
            if h <= 0:
                continue
            gflops = 10 * 100 * side * side * 1e6 / (h * 3600) / 1e9
            assert abs(gflops / quoted[col] - 1) < 0.06, (side, col, gflops)


# ---------------------------------------------------------------- jittered (Monte Carlo) rays

def test_oracle_splitmix_matches_published_outputs():
    vals = [int(l, 16) for l in open(os.path.join(GOLDEN, "splitmix64_seed0.txt"))
            if l.strip() and not l.startswith("#")]
    G = 0x9E3779B97F4A7C15
    assert [oracle.lib().orc_mix64((G * (i + 1)) & 0xFFFFFFFFFFFFFFFF) for i in range(3)] == vals


def test_oracle_jitter_equals_generator_module_draws():
    # two independent implementations of the same counter hash (C oracle, numpy generators)
    for seed in (0, 7, 2 ** 63 + 5):
        r = np.array([0, 1, 5, 999, 123456789], dtype=np.int64)
        for k in range(2):
            c = [oracle.lib().orc_jitter_u(seed, k, int(i)) for i in r]
            py = [synth.uniform(seed, 8 + k, int(i), 1)[0] for i in r]
            assert c == py


def _jw(seed, n=(300, 200)):
    return _wl(np.zeros((0, 4)), 0.0, 0.0, (-3.0, -2.0), (3.0, 2.0), n, (-1.0, -1.0), (1.0, 1.0), (8, 8))


def test_jittered_rays_lie_in_their_cells_and_are_uniform():
    w = _jw(3)
    w.jitter_seed = 3
    idx = np.arange(w.n_rays)
    xy = oracle.ray_positions(w, idx).astype(np.float64)
    i1, i2 = idx % w.grid_n[0], idx // w.grid_n[0]
    t1, t2 = 6.0 / 300, 4.0 / 200
    u1 = (xy[:, 0] + 3.0) / t1 - i1
    u2 = (xy[:, 1] + 2.0) / t2 - i2
    eps = 1e-5
    assert np.all((u1 > -eps) & (u1 < 1 + eps) & (u2 > -eps) & (u2 < 1 + eps))
    for u in (u1, u2):
        assert abs(u.mean() - 0.5) < 4 * math.sqrt(1 / 12 / len(u))
        assert abs(u.var() - 1 / 12) < 0.01
    assert abs(np.corrcoef(u1, u2)[0, 1]) < 4 / math.sqrt(len(u1))
    # centres when jitter is off; a different seed moves every ray
    w.jitter_seed = None
    c = oracle.ray_positions(w, idx[:50]).astype(np.float64)
    assert np.allclose(c[:, 0], -3.0 + (i1[:50] + 0.5) * t1, atol=1e-6)
    w.jitter_seed = 4
    assert np.all(oracle.ray_positions(w, idx[:50]) != xy[:50].astype(np.float32))


def test_jittered_windows_add_up_and_single_lens_magnification():
    L = np.array([[0.0, 0.0, 1.0, 0.0]], dtype=np.float32)
    w = _wl(L, 0.0, 0.0, (-4.0, -4.0), (4.0, 4.0), (800, 800), (-2.0, -2.0), (2.0, 2.0), (4, 4))
    w.jitter_seed = 11
    full, lost = oracle.shoot_parallel(w)
    part = np.zeros_like(full)
    pl = 0
    for win in (((0, 0), (800, 333)), ((0, 333), (800, 467))):
        c, l = oracle.shoot(w, win)
        part += c
        pl += l
    assert np.array_equal(part, full) and pl == lost
    # annulus mean magnification of a point lens from stratified random rays
    y, _ = oracle.trace_parallel(w, np.arange(w.n_rays))
    ry = np.hypot(y[:, 0], y[:, 1])
    cell = (8.0 / 800) ** 2
    for ua, ub in [(0.2, 0.3), (1.0, 1.5)]:
        mu = np.sum((ry >= ua) & (ry < ub)) * cell / (math.pi * (ub * ub - ua * ua))
        ref = (ub * math.sqrt(ub * ub + 4) - ua * math.sqrt(ua * ua + 4)) / (ub * ub - ua * ua)
        assert abs(mu / ref - 1) < 5e-3
