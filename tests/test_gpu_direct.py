"""GPU parity of the direct inverse ray-shooting path (rs_shoot) against the FP64 oracle.

Tolerances (the plain path): at most 1e-5 of the rays may land in a different
pixel than the FP64 oracle puts them in (pixel or lost outcome compared ray by
ray).  Results that do not depend on float32 rounding are compared exactly:
integer counts against the kernel's own per-ray pixels, conservation,
determinism, tiling invariance, window streaming, and N_* = 0 exact lattice
counts.
"""
import math

import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu

SWITCH_TOL = 1e-5
U32 = 2.0 ** -24


def _torch():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def _P():
    import paper_0905_2453_amd as P
    P.lib()  # raises if the HIP library is missing: no fallback
    return P


def run(w, opts=None, window=None, dump=False, lenses=None):
    """Shoot a workload on cuda:0; returns (counts np.uint32, lost int, ray_y, ray_pix)."""
    torch = _torch()
    P = _P()
    o = P.Opts() if opts is None else opts
    dev = torch.device("cuda:0")
    if lenses is None:
        lenses = torch.from_numpy(np.ascontiguousarray(w.lenses)).to(dev)
    if window is None:
        window = ((0, 0), (w.grid_n[0], w.grid_n[1]))
    nr = int(window[1][0]) * int(window[1][1])
    ry = rp = None
    if dump:
        ry = torch.full((max(nr, 1), 2), float("nan"), dtype=torch.float64, device=dev)
        rp = torch.full((max(nr, 1),), -7, dtype=torch.int32, device=dev)
        o.ray_y = ry.data_ptr()
        o.ray_pix = rp.data_ptr()
    counts, lost = P.shoot(lenses, w.kappa_c, w.gamma, w.grid_lo, w.grid_hi, w.grid_n, w.map_lo, w.map_hi,
                           w.map_n, window=window, opts=o, jitter_seed=w.jitter_seed)
    torch.cuda.synchronize()
    out = (counts.cpu().numpy().view(np.uint32), int(lost.item()))
    if dump:
        return out + (ry.cpu().numpy()[:nr], rp.cpu().numpy()[:nr])
    return out + (None, None)


def switch_fraction(pix_a, pix_b):
    """Rays whose (pixel or lost) outcome differs / rays in the map in either run."""
    diff = np.sum(pix_a != pix_b)
    inmap = np.sum((pix_a >= 0) | (pix_b >= 0))
    return diff / max(1, inmap), int(diff)


def test_small_workload_full_parity():
    w = synth.workload_small()
    counts, lost, ry, rp = run(w, dump=True)
    n = w.n_rays
    # conservation and binning are exact
    assert int(counts.sum()) + lost == n
    assert np.array_equal(counts.ravel().astype(np.int64),
                          np.bincount(rp[rp >= 0], minlength=counts.size))
    assert lost == int(np.sum(rp == -1))
    # every ray against the oracle
    y_o, p_o = oracle.trace_parallel(w, np.arange(n))
    frac, nd = switch_fraction(rp.astype(np.int64), p_o)
    print(f"small workload: {nd} of {n} rays switch pixel (fraction {frac:.2e})")
    assert frac <= SWITCH_TOL
    # map agreement follows: per-pixel |diff| summed is at most 2 x switched rays
    co, lo_ = oracle.shoot_parallel(w)
    assert np.abs(counts.astype(np.int64) - co.astype(np.int64)).sum() <= 2 * nd
    # per-ray source positions within the float32 forward-error bound
    ok = np.isfinite(y_o).all(1) & np.isfinite(ry).all(1)
    L = w.lenses.astype(np.float64)
    xs1 = oracle.axis(w.grid_lo[0], w.grid_hi[0], w.grid_n[0]).astype(np.float64)
    idx = np.nonzero(ok)[0][::97]
    x = np.stack([xs1[idx % w.grid_n[0]], xs1[idx // w.grid_n[0]]], 1)
    s = np.zeros(len(idx))
    for rec in L:
        s += rec[2] / np.hypot(x[:, 0] - rec[0], x[:, 1] - rec[1])
    bound = (8 + 16) * U32 * s + 1e-12
    err = np.abs(ry[idx] - y_o[idx]).max(1)
    assert np.all(err <= bound), (err / bound).max()


def test_deterministic_and_tiling_invariant():
    w = synth.workload_small(seed=9)
    P = _P()
    ref = run(w, dump=True)
    again = run(w, dump=True)
    assert np.array_equal(ref[0], again[0]) and ref[1] == again[1]
    assert np.array_equal(ref[2], again[2])
    # lens tile and map window change speed only, never values; so do the rows and columns of a
    # several-column block (pairs of rows share a reciprocal there, four rows in the one-column
    # block, so the two families are compared within themselves)
    o = P.Opts()
    o.block_cols, o.block_rows = 2, 2
    ref_m = run(w, opts=o, dump=True)
    assert np.abs(ref_m[0].astype(np.int64) - ref[0].astype(np.int64)).sum() <= 8
    for (K1, K2), LT, W in [((1, 4), 256, 16), ((1, 4), 512, -1), ((4, 4), 512, 64), ((2, 4), 512, -1),
                            ((2, 2), 512, 32), ((4, 2), 256, 64), ((2, 8), 256, 32)]:
        o = P.Opts()
        o.block_cols, o.block_rows, o.lens_tile, o.map_window = K1, K2, LT, W
        got = run(w, opts=o, dump=True)
        want = ref if K1 == 1 else ref_m
        assert np.array_equal(got[0], want[0]), (K1, K2, LT, W)
        assert got[1] == want[1]
        assert np.array_equal(got[2], want[2]) and np.array_equal(got[3], want[3])


@pytest.mark.parametrize("T", [8, 16, 32])
def test_fp32_run_length_variants_within_tolerance(T):
    P = _P()
    w = synth.workload_small(seed=3)
    o = P.Opts()
    o.fp32_run = T
    counts, lost, ry, rp = run(w, opts=o, dump=True)
    _, p_o = oracle.trace_parallel(w, np.arange(w.n_rays))
    frac, nd = switch_fraction(rp.astype(np.int64), p_o)
    assert frac <= SWITCH_TOL, (T, nd)
    assert int(counts.sum()) + lost == w.n_rays


def test_dump_does_not_change_map():
    w = synth.workload_small(seed=4)
    a = run(w)
    b = run(w, dump=True)
    assert np.array_equal(a[0], b[0]) and a[1] == b[1]


def test_window_streaming_adds_up():
    torch = _torch()
    P = _P()
    w = synth.workload_small(seed=5)
    full = run(w)
    dev = torch.device("cuda:0")
    lenses = torch.from_numpy(w.lenses).to(dev)
    counts = torch.zeros((w.map_n[1], w.map_n[0]), dtype=torch.int32, device=dev)
    lost = torch.zeros(1, dtype=torch.int64, device=dev)
    # ragged, uneven windows in both axes, starting on every grid row modulo 4
    for (a, b) in [((0, 0), (1000, 137)), ((0, 137), (301, 863)), ((301, 137), (699, 250)),
                   ((301, 387), (699, 251)), ((301, 638), (699, 362))]:
        P.shoot(lenses, w.kappa_c, w.gamma, w.grid_lo, w.grid_hi, w.grid_n, w.map_lo, w.map_hi, w.map_n,
                counts=counts, lost=lost, window=(a, b))
    torch.cuda.synchronize()
    assert np.array_equal(counts.cpu().numpy().view(np.uint32), full[0])
    assert int(lost.item()) == full[1]


@pytest.mark.parametrize("n_lens", [1, 255, 257, 1000])
def test_ragged_lens_counts_and_grid(n_lens):
    lenses, r = synth.lens_field(30 + n_lens, n_lens, kappa_star=0.3)
    lo, hi, n = synth.shooting_region((4.0, 3.0), 0.3, 0.1, (203, 77), r)
    w = synth.Workload("ragged", lenses, 0.05, 0.1, lo, hi, n, (-4.0, -3.0), (4.0, 3.0), (37, 23))
    counts, lost, ry, rp = run(w, dump=True)
    assert int(counts.sum()) + lost == w.n_rays
    assert np.array_equal(counts.ravel().astype(np.int64), np.bincount(rp[rp >= 0], minlength=counts.size))
    _, p_o = oracle.trace(w, np.arange(w.n_rays))
    frac, nd = switch_fraction(rp.astype(np.int64), p_o)
    assert nd <= max(1, int(SWITCH_TOL * w.n_rays)), nd


def test_empty_window_and_no_lenses():
    torch = _torch()
    w = synth.Workload("sheet", np.zeros((0, 4), np.float32), 0.25, 0.125, (-8.0, -6.0), (8.0, 6.0),
                       (256, 192), (-3.0, -2.5), (3.0, 2.5), (24, 20))
    counts, lost, _, _ = run(w, window=((10, 10), (0, 50)))
    assert counts.sum() == 0 and lost == 0
    counts, lost, _, _ = run(w)
    assert int(counts.sum()) + lost == w.n_rays


def _exact_axis_counts(lo, hi, n, lam, mlo, mhi, mn):
    from fractions import Fraction
    from oracle import exact
    out = np.zeros(mn, dtype=np.int64)
    for i in range(n):
        X = Fraction(exact.round_to_float32(exact.exact_coord(lo, hi, n, i)))
        p = math.floor((Fraction(lam) * X - Fraction(mlo)) * mn / (Fraction(mhi) - Fraction(mlo)))
        if 0 <= p < mn:
            out[p] += 1
    return out


@pytest.mark.parametrize("kappa_c,gamma", [(0.25, 0.125), (1.25, 0.0), (0.5, -0.25)])
def test_smooth_sheet_exact_counts_on_gpu(kappa_c, gamma):
    w = synth.Workload("sheet", np.zeros((0, 4), np.float32), kappa_c, gamma, (-8.0, -6.0), (8.0, 6.0),
                       (256, 192), (-3.0, -2.5), (3.0, 2.5), (24, 20))
    counts, lost, _, _ = run(w)
    c1 = _exact_axis_counts(-8.0, 8.0, 256, 1 - kappa_c - gamma, -3.0, 3.0, 24)
    c2 = _exact_axis_counts(-6.0, 6.0, 192, 1 - kappa_c + gamma, -2.5, 2.5, 20)
    assert np.array_equal(counts.astype(np.int64), np.outer(c2, c1))


def test_single_lens_disc_count_identity_on_gpu():
    L = np.array([[0.0, 0.0, 1.0, 0.0]], dtype=np.float32)
    w = synth.Workload("one", L, 0.0, 0.0, (-4.0, -4.0), (4.0, 4.0), (600, 600), (-4.0, -4.0), (4.0, 4.0),
                       (8, 8))
    _, _, ry, _ = run(w, dump=True)
    xs = oracle.axis(-4.0, 4.0, 600).astype(np.float64)
    X1, X2 = np.meshgrid(xs, xs)
    rx = np.hypot(X1, X2).ravel()
    r_y = np.hypot(ry[:, 0], ry[:, 1])
    for u in (0.1, 0.5, 1.0, 2.0, 3.0):
        rp_ = (math.sqrt(u * u + 4) + u) / 2
        rm_ = (math.sqrt(u * u + 4) - u) / 2
        amb = (np.abs(rx - rp_) < 1e-5) | (np.abs(rx - rm_) < 1e-5) | (np.abs(r_y - u) < 1e-5)
        assert np.sum((r_y < u) & ~amb) == np.sum((rx > rm_) & (rx < rp_) & ~amb)


@pytest.mark.parametrize("row", [4, 5, 6])
@pytest.mark.parametrize("block", [(1, 4), (2, 4)])
def test_ray_on_lens_is_lost_on_gpu(row, block):
    # rows share reciprocals (grid rows 4k..4k+3 in one-column blocks, (even, odd) pairs in
    # several-column ones): the ray on the lens is lost, the rows that share its reciprocal (which
    # land inside the map here) are not
    P = _P()
    xs = oracle.axis(-1.0, 1.0, 8)
    L = np.array([[xs[3], xs[row], 1.0, 0], [0.37, -0.61, 0.5, 0]], dtype=np.float32)
    w = synth.Workload("hit", L, 0.0, 0.0, (-1.0, -1.0), (1.0, 1.0), (8, 8), (-8.0, -8.0), (8.0, 8.0), (16, 16))
    o = P.Opts()
    o.block_cols, o.block_rows = block
    counts, lost, ry, rp = run(w, opts=o, dump=True)
    _, p_o = oracle.trace(w, np.arange(64))
    share = [r for r in (range(row & ~3, (row & ~3) + 4) if block[0] == 1 else (row & ~1, row | 1)) if r != row]
    assert rp[row * 8 + 3] == -1 and all(p_o[r * 8 + 3] >= 0 for r in share)
    assert np.array_equal(rp.astype(np.int64), p_o)


@pytest.mark.parametrize("block", [(1, 4), (2, 4)])
def test_ray_on_lens_among_many_lenses(block):
    # 1000 lenses (31 full groups of 32 and a partial one), one of them exactly on a grid ray: the
    # lane holding that ray is redone with one reciprocal per ray in the same runs and groups; the
    # ray is lost, every other ray lands where the oracle puts it, within the float32 bound
    P = _P()
    rng = np.random.default_rng(21)
    n = 32
    xs = oracle.axis(-1.0, 1.0, n)
    L = np.zeros((1000, 4), dtype=np.float32)
    r = 30.0 * np.sqrt(rng.random(1000))
    t = 2 * np.pi * rng.random(1000)
    L[:, 0], L[:, 1], L[:, 2] = r * np.cos(t), r * np.sin(t), 0.1 + 0.9 * rng.random(1000)
    L[517, 0], L[517, 1] = xs[5], xs[13]
    w = synth.Workload("hit-many", L, 0.0, 0.1, (-1.0, -1.0), (1.0, 1.0), (n, n), (-20.0, -20.0), (20.0, 20.0),
                       (64, 64))
    o = P.Opts()
    o.block_cols, o.block_rows = block
    counts, lost, ry, rp = run(w, opts=o, dump=True)
    y_o, p_o = oracle.trace(w, np.arange(n * n))
    hit = 13 * n + 5
    share = (12, 14, 15) if block[0] == 1 else (12,)
    assert rp[hit] == -1 and p_o[hit] == -1 and all(p_o[k * n + 5] >= 0 for k in share)
    assert np.array_equal(rp.astype(np.int64), p_o)
    ok = np.isfinite(y_o).all(1)
    assert ok.sum() == n * n - 1
    x = np.stack(np.meshgrid(xs, xs), -1).reshape(-1, 2).astype(np.float64)
    Ld = L.astype(np.float64)
    s = np.zeros(n * n)
    for rec in Ld:
        with np.errstate(divide="ignore"):
            s += rec[2] / np.hypot(x[:, 0] - rec[0], x[:, 1] - rec[1])
    err = np.abs(ry[ok] - y_o[ok]).max(1)
    assert np.all(err <= (8 + 16) * U32 * s[ok] + 1e-12), float((err / s[ok]).max() / U32)


def test_odd_window_dump_matches_oracle():
    # a window starting on an odd row and column, ragged in both axes: per-ray dumps keep the
    # caller's window indexing and every ray matches the oracle
    w = synth.workload_small(seed=6)
    win = ((3, 5), (301, 77))
    counts, lost, ry, rp = run(w, window=win, dump=True)
    c, r = np.meshgrid(np.arange(win[0][0], win[0][0] + win[1][0]), np.arange(win[0][1], win[0][1] + win[1][1]))
    idx = (r * w.grid_n[0] + c).ravel()
    y_o, p_o = oracle.trace_parallel(w, idx)
    assert int(counts.sum()) + lost == idx.size
    frac, nd = switch_fraction(rp.astype(np.int64), p_o)
    assert nd <= max(1, int(SWITCH_TOL * idx.size)), nd
    # per-ray source positions within the float32 forward-error bound
    ok = np.nonzero(np.isfinite(y_o).all(1) & np.isfinite(ry).all(1))[0]
    xs1 = oracle.axis(w.grid_lo[0], w.grid_hi[0], w.grid_n[0]).astype(np.float64)
    xs2 = oracle.axis(w.grid_lo[1], w.grid_hi[1], w.grid_n[1]).astype(np.float64)
    x = np.stack([xs1[idx[ok] % w.grid_n[0]], xs2[idx[ok] // w.grid_n[0]]], 1)
    s = np.zeros(len(ok))
    for rec in w.lenses.astype(np.float64):
        s += rec[2] / np.hypot(x[:, 0] - rec[0], x[:, 1] - rec[1])
    err = np.abs(ry[ok] - y_o[ok]).max(1)
    assert np.all(err <= (8 + 16) * U32 * s + 1e-12)


def allowed_switches(n_inmap):
    """Largest switch count consistent with a true fraction of at most 1e-5: the count of a
    sample of n rays is Poisson with mean <= 1e-5 n, so 3 standard deviations are allowed."""
    mean = SWITCH_TOL * n_inmap
    return mean + 3.0 * math.sqrt(mean)


def test_paper_scale_sampled_parity():
    # 1e5 power-law lenses, kappa_*=0.45, gamma=0.45, 4096^2 rays, 1024^2 map: the full
    # workload in the launch configuration the benchmark times; 2^22 sampled rays (a quarter of
    # the grid) checked one by one against the FP64 oracle and the switches counted.
    w = synth.workload_paper()
    counts, lost, ry, rp = run(w, dump=True)
    assert int(counts.sum()) + lost == w.n_rays
    assert np.array_equal(counts.ravel().astype(np.int64), np.bincount(rp[rp >= 0], minlength=counts.size))
    idx = synth.sample_indices(12, w.n_rays, 1 << 22)
    print(f"paper-scale parity: oracle on {len(idx)} rays x {w.n_lens} lenses", flush=True)
    y_o, p_o = oracle.trace_parallel(w, idx, threads=16)
    frac, nd = switch_fraction(rp[idx].astype(np.int64), p_o)
    inmap = int(np.sum((rp[idx] >= 0) | (p_o >= 0)))
    ok = np.isfinite(y_o).all(1) & (p_o >= 0)
    dpix = (w.map_hi[0] - w.map_lo[0]) / w.map_n[0]
    dy = ry[idx][ok] - y_o[ok]
    # Second, sharper check: for source positions spread uniformly over a pixel, a ray with error
    # (d1, d2) changes pixel with probability (|d1| + |d2|) / pixel, so the mean is the expected
    # switch fraction without the counting noise.
    est = np.mean(np.abs(dy).sum(1)) / dpix
    # No systematic error proportional to the deflection (a biased reciprocal would show here).
    lam1 = (1 - w.gamma) - w.kappa_c
    xs1 = oracle.axis(w.grid_lo[0], w.grid_hi[0], w.grid_n[0]).astype(np.float64)
    a1 = lam1 * xs1[idx[ok] % w.grid_n[0]] - y_o[ok, 0]
    slope = float(np.dot(dy[:, 0], a1) / np.dot(a1, a1))
    print(f"paper-scale sample: {nd} of {inmap} rays in the map switch (counted fraction {frac:.2e}); "
          f"estimated switch fraction {est:.2e}; error/deflection slope {slope:.2e}")
    assert nd <= allowed_switches(inmap), (nd, inmap)
    assert est <= SWITCH_TOL
    assert abs(slope) < 1.5e-9
    # the whole map: mean N / N_av over the 20 x 20 source region is the field's mean
    # magnification 1 / |(1 - kappa)^2 - gamma^2| = 10 (eq. 4 with the macro model of eq. 6)
    mu_mean = counts.astype(np.float64).mean() / oracle.n_av(w)
    want = 1.0 / abs((1 - w.kappa_star - w.kappa_c) ** 2 - w.gamma ** 2)
    print(f"paper-scale mean magnification {mu_mean:.3f} (theory {want:.3f})")
    assert abs(mu_mean / want - 1) < 0.03


_FOLD_REF = {}


@pytest.mark.parametrize("block", [(2, 4), (4, 4), (2, 8), (2, 2), (4, 2)])
def test_folded_block_shapes_power_law_masses(block):
    # Blocks of several columns fold the mass into the shared differences, q (m dx), which rounds
    # differently from the one-column m / r^2 when masses differ from 1.  On a power-law field
    # (2e4 lenses on the paper grid) each such shape must meet the 1e-5 switch bar against the
    # FP64 oracle on its own, and every sampled ray must stay within the float32 forward-error bound.
    P = _P()
    w = synth.workload_paper(n_lens=20000)
    idx = synth.sample_indices(31, w.n_rays, 1 << 20)
    if "p" not in _FOLD_REF:
        print(f"folded shapes: oracle on {len(idx)} rays x {w.n_lens} lenses", flush=True)
        _FOLD_REF["y"], _FOLD_REF["p"] = oracle.trace_parallel(w, idx, threads=16)
    y_o, p_o = _FOLD_REF["y"], _FOLD_REF["p"]
    o = P.Opts()
    o.block_cols, o.block_rows = block
    print(f"folded shapes: block {block}", flush=True)
    counts, lost, ry, rp = run(w, opts=o, dump=True)
    assert int(counts.sum()) + lost == w.n_rays
    assert np.array_equal(counts.ravel().astype(np.int64), np.bincount(rp[rp >= 0], minlength=counts.size))
    frac, nd = switch_fraction(rp[idx].astype(np.int64), p_o)
    inmap = int(np.sum((rp[idx] >= 0) | (p_o >= 0)))
    print(f"block {block}: {nd} of {inmap} sampled rays switch (fraction {frac:.2e})")
    assert nd <= allowed_switches(inmap), (block, nd, inmap)
    # per-ray bound on 2048 of the sampled rays: (8 + 16) ulp32 x sum m / r
    sub = np.nonzero(np.isfinite(y_o).all(1))[0][:2048]
    xs1 = oracle.axis(w.grid_lo[0], w.grid_hi[0], w.grid_n[0]).astype(np.float64)
    xs2 = oracle.axis(w.grid_lo[1], w.grid_hi[1], w.grid_n[1]).astype(np.float64)
    g = idx[sub]
    x = np.stack([xs1[g % w.grid_n[0]], xs2[g // w.grid_n[0]]], 1)
    L = w.lenses.astype(np.float64)
    s = np.zeros(len(sub))
    for c0 in range(0, len(L), 4096):
        Lc = L[c0:c0 + 4096]
        s += np.sum(Lc[None, :, 2] / np.hypot(x[:, None, 0] - Lc[None, :, 0], x[:, None, 1] - Lc[None, :, 1]), 1)
    err = np.abs(ry[g] - y_o[sub]).max(1)
    assert np.all(err <= (8 + 16) * U32 * s + 1e-12), (block, float((err / s).max() / U32))


@pytest.mark.parametrize("which", ["small", "paper"])
def test_cell_centred_ray_positions_bit_identical_to_oracle(which):
    # no lenses, no macro term: y = x, so the kernel's FP64 y is its float32 ray position; the
    # 1000^2 grid on [-10, 10]^2 (cell 0.02, not a binary fraction) and the paper's 4096^2 grid
    base = synth.workload_small() if which == "small" else synth.workload_paper(n_lens=1)
    w = synth.Workload("pos", np.zeros((0, 4), np.float32), 0.0, 0.0, base.grid_lo, base.grid_hi, base.grid_n,
                       base.grid_lo, base.grid_hi, (64, 64))
    counts, lost, ry, rp = run(w, dump=True)
    xs1 = oracle.axis(w.grid_lo[0], w.grid_hi[0], w.grid_n[0]).astype(np.float64)
    xs2 = oracle.axis(w.grid_lo[1], w.grid_hi[1], w.grid_n[1]).astype(np.float64)
    assert np.array_equal(ry[:, 0].reshape(w.grid_n[1], w.grid_n[0]), np.broadcast_to(xs1, (w.grid_n[1], w.grid_n[0])))
    assert np.array_equal(ry[:, 1].reshape(w.grid_n[1], w.grid_n[0]),
                          np.broadcast_to(xs2[:, None], (w.grid_n[1], w.grid_n[0])))
    assert int(counts.sum()) + lost == w.n_rays


# ---------------------------------------------------------------- jittered (Monte Carlo) rays

def test_jittered_positions_bit_identical_to_oracle():
    # no lenses, no macro term: y = x, so the kernel's FP64 y is its float32 ray position
    w = synth.Workload("pos", np.zeros((0, 4), np.float32), 0.0, 0.0, (-120.0, -12.0), (120.0, 12.0), (777, 301),
                       (-130.0, -13.0), (130.0, 13.0), (10, 10), jitter_seed=2 ** 40 + 17)
    counts, lost, ry, rp = run(w, dump=True)
    xy = oracle.ray_positions(w, np.arange(w.n_rays)).astype(np.float64)
    assert np.array_equal(ry, xy)
    assert lost == 0 and int(counts.sum()) == w.n_rays


def test_jittered_small_workload_parity():
    w = synth.workload_small(seed=6)
    w.jitter_seed = 99
    counts, lost, ry, rp = run(w, dump=True)
    assert int(counts.sum()) + lost == w.n_rays
    assert np.array_equal(counts.ravel().astype(np.int64), np.bincount(rp[rp >= 0], minlength=counts.size))
    _, p_o = oracle.trace_parallel(w, np.arange(w.n_rays))
    frac, nd = switch_fraction(rp.astype(np.int64), p_o)
    print(f"jittered small workload: {nd} switches (fraction {frac:.1e})")
    assert frac <= SWITCH_TOL
    # jitter moves the rays: the map differs from the cell-centred one
    w.jitter_seed = None
    c0, _, _, _ = run(w)
    assert not np.array_equal(c0, counts)


def test_jittered_windows_and_block_shapes_agree():
    torch = _torch()
    P = _P()
    w = synth.workload_small(seed=8)
    w.jitter_seed = 5
    ref = run(w, dump=True)
    ref_m = None
    for K1, K2 in [(2, 2), (2, 4), (4, 4)]:
        o = P.Opts()
        o.block_cols, o.block_rows = K1, K2
        got = run(w, opts=o, dump=True)
        ref_m = got if ref_m is None else ref_m
        assert np.array_equal(got[0], ref_m[0]) and np.array_equal(got[2], ref_m[2]), (K1, K2)
    dev = torch.device("cuda:0")
    lenses = torch.from_numpy(w.lenses).to(dev)
    counts = torch.zeros((w.map_n[1], w.map_n[0]), dtype=torch.int32, device=dev)
    lost = torch.zeros(1, dtype=torch.int64, device=dev)
    for (a, b) in [((0, 0), (1000, 411)), ((0, 411), (1000, 589))]:
        P.shoot(lenses, w.kappa_c, w.gamma, w.grid_lo, w.grid_hi, w.grid_n, w.map_lo, w.map_hi, w.map_n,
                counts=counts, lost=lost, window=(a, b), jitter_seed=5)
    torch.cuda.synchronize()
    assert np.array_equal(counts.cpu().numpy().view(np.uint32), ref[0]) and int(lost.item()) == ref[1]
