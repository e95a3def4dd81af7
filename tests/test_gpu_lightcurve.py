"""GPU parity of light curves (rs_light_curve) against the FP64 oracle (oracle/lightcurve.py).

Bar: a uniform-disc source sums integer counts with unit weights, so its magnification is
bit-identical to the oracle's (both take the same inclusion decisions from the same FP64
expressions); a Gaussian source differs only by the rounding of exp and of the summation order,
|d mu| / mu <= 1e-12.  Magnitudes then agree to 1e-11.  Maps and tracks come from the seeded
generators or from the oracle's own ray shooting, never from the HIP path.
"""
import numpy as np
import pytest

import oracle
import synth
from oracle import lightcurve as lc

pytestmark = pytest.mark.gpu

MU_RTOL = 1e-12
MAG_ATOL = 1e-11
LAYOUT = {"v": 0}


@pytest.fixture(params=["lanes", "waves"], autouse=True)
def layout(request):
    # every test runs on both evaluation layouts of the kernel
    LAYOUT["v"] = request.param
    yield request.param
    LAYOUT["v"] = 0


def _env():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_0905_2453_amd as P
    P.lib()  # raises if the HIP library is missing: no fallback
    return torch, P


def _gpu(counts, lo, hi, n, n_av, tracks, n_points, kind, size, cutoff=0.0):
    torch, P = _env()
    dev = torch.device("cuda:0")
    c = torch.from_numpy(np.ascontiguousarray(counts).view(np.int32)).to(dev)
    t = torch.from_numpy(np.ascontiguousarray(tracks, dtype=np.float64)).to(dev)
    mu, mag = P.light_curve(c, lo, hi, n, n_av, t, n_points, kind, size, cutoff, layout=LAYOUT["v"])
    torch.cuda.synchronize()
    return mu.cpu().numpy(), mag.cpu().numpy()


def _compare(mu_g, mag_g, mu_o, mag_o, exact):
    assert np.array_equal(np.isnan(mu_g), np.isnan(mu_o))
    ok = ~np.isnan(mu_o)
    if exact:
        assert np.array_equal(mu_g[ok], mu_o[ok])
    else:
        zero = ok & (mu_o == 0)
        assert np.all(mu_g[zero] == 0)             # every pixel in the support is empty
        nz = ok & (mu_o != 0)
        rel = np.abs(mu_g[nz] - mu_o[nz]) / np.abs(mu_o[nz])
        assert np.all(rel <= MU_RTOL), rel.max()
    fin = ok & (mu_o > 0)
    assert np.all(np.abs(mag_g[fin] - mag_o[fin]) <= MAG_ATOL)
    return int(ok.sum())


# rectangular map with non-unit, unequal pixels and an offset corner; tracks leave the map
LO, N = (-3.0, 1.0), (300, 200)
HI = (LO[0] + 0.05 * N[0], LO[1] + 0.08 * N[1])


@pytest.mark.parametrize("radius", [0.27, 4.0])   # 4.0: box wider than the LDS staging
def test_disc_bit_exact_on_seeded_map(radius):
    counts = synth.count_map(21, N, 40.0)
    tr = synth.light_tracks(22, 12, LO, HI, 9.0)
    mu_g, mag_g = _gpu(counts, LO, HI, N, 40.0, tr, 37, "disc", radius)
    mu_o, mag_o = lc.light_curve(counts, LO, HI, N, 40.0, tr, 37, "disc", radius)
    if radius < 1:
        assert np.isnan(mu_o).any() and (~np.isnan(mu_o)).sum() > 300   # some points leave the map
    _compare(mu_g, mag_g, mu_o, mag_o, exact=True)


# (2.0, 4.0): support box wider than the wave layout's LDS staging (per-pixel path);
# (0.002, 30.0): a source far narrower than a pixel (the lane layout's direct-exp path)
@pytest.mark.parametrize("sigma,cutoff", [(0.11, 0.0), (0.04, 6.0), (0.9, 3.0), (2.0, 4.0), (0.002, 30.0)])
def test_gaussian_parity_on_seeded_map(sigma, cutoff):
    counts = synth.count_map(23, N, 40.0)
    tr = synth.light_tracks(24, 10, LO, HI, 7.0)
    mu_g, mag_g = _gpu(counts, LO, HI, N, 40.0, tr, 29, "gaussian", sigma, cutoff)
    mu_o, mag_o = lc.light_curve(counts, LO, HI, N, 40.0, tr, 29, "gaussian", sigma, cutoff)
    _compare(mu_g, mag_g, mu_o, mag_o, exact=False)


def test_parity_on_oracle_shot_map():
    # the 100-lens workload's map shot by the oracle: a real caustic network
    w = synth.workload_small()
    co, _ = oracle.shoot_parallel(w)
    nav = oracle.n_av(w)
    tr = synth.light_tracks(25, 8, w.map_lo, w.map_hi, 12.0)
    for kind, size in (("gaussian", 0.3), ("disc", 0.5)):
        mu_g, mag_g = _gpu(co, w.map_lo, w.map_hi, w.map_n, nav, tr, 61, kind, size)
        mu_o, mag_o = lc.light_curve(co, w.map_lo, w.map_hi, w.map_n, nav, tr, 61, kind, size)
        _compare(mu_g, mag_g, mu_o, mag_o, exact=(kind == "disc"))


def test_full_size_sampled_points():
    # the light-curve workload timed by the benchmark: 1024^2 map over 20 x 20 Einstein radii,
    # 1024 tracks of 10 Einstein radii, 1024 points each, Gaussian sigma 0.05; the oracle checks
    # a seeded sample of points
    lo, hi, n = (-10.0, -10.0), (10.0, 10.0), (1024, 1024)
    counts = synth.count_map(26, n, 16.0)
    tr = synth.light_tracks(27, 1024, lo, hi, 10.0)
    mu_g, mag_g = _gpu(counts, lo, hi, n, 16.0, tr, 1024, "gaussian", 0.05)
    pick = synth.sample_indices(28, 1024 * 1024, 64)
    ti, ki = pick // 1024, pick % 1024
    checked = 0
    for t, k in zip(ti, ki):
        f = k / 1023.0
        s1, s2, e1, e2 = tr[t]
        # a one-point track at the sampled position; f is reproduced exactly by the oracle
        one = np.array([[s1 + f * (e1 - s1), s2 + f * (e2 - s2)] * 2])
        mu_o, mag_o = lc.light_curve(counts, lo, hi, n, 16.0, one, 1, "gaussian", 0.05)
        checked += _compare(mu_g[t:t + 1, k:k + 1], mag_g[t:t + 1, k:k + 1], mu_o, mag_o, exact=False)
    assert checked >= 40          # most sampled points lie on the map


def test_edge_cases():
    counts = synth.count_map(29, (64, 48), 10.0)
    lo, hi, n = (0.0, 0.0), (64.0, 48.0), (64, 48)
    # a disc covering the whole map returns the map mean exactly; off-map and between-centre
    # sources have no pixel in their support
    tr = np.array([[32.0, 24.0, 32.0, 24.0], [-50.0, 5.0, -40.0, 5.0], [10.0, 10.0, 10.0, 10.0]])
    mu_g, mag_g = _gpu(counts, lo, hi, n, 10.0, tr, 3, "disc", 100.0)
    assert np.all(mu_g[0] == counts.astype(np.float64).sum() / (counts.size * 10.0))
    mu_g, _ = _gpu(counts, lo, hi, n, 10.0, tr[1:2], 3, "disc", 5.0)       # wholly off the map
    assert np.isnan(mu_g).all()
    mu_g, _ = _gpu(counts, lo, hi, n, 10.0, tr[2:], 2, "disc", 0.3)        # (10, 10) is a pixel corner
    assert np.isnan(mu_g).all()
    # one-point tracks and empty calls
    mu_g, _ = _gpu(counts, lo, hi, n, 10.0, np.array([[5.5, 6.5, 60.0, 1.0]]), 1, "gaussian", 0.1)
    assert mu_g[0, 0] == counts[6, 5] / 10.0
    mu_g, mag_g = _gpu(counts, lo, hi, n, 10.0, np.zeros((0, 4)), 5, "disc", 1.0)
    assert mu_g.shape == (0, 5)
    # a zero-count pixel gives mu = 0 and an infinite magnitude change
    z = np.zeros((4, 4), np.uint32)
    mu_g, mag_g = _gpu(z, (0, 0), (4, 4), (4, 4), 1.0, np.array([[2.0, 2.0, 2.0, 2.0]]), 1, "disc", 1.0)
    assert mu_g[0, 0] == 0.0 and mag_g[0, 0] == np.inf


def test_shoot_then_light_curve_chain():
    # the GPU map of the 100-lens workload feeds the GPU light curve; against the oracle's map and
    # light curve the difference is bounded by the rays that switched pixel:
    # |d mu| <= sum_p w_p |dN_p| / (N_av sum_p w_p) <= L1(dN) / (N_av sum_p w_p)
    torch, P = _env()
    w = synth.workload_small()
    dev = torch.device("cuda:0")
    lenses = torch.from_numpy(np.ascontiguousarray(w.lenses)).to(dev)
    counts, lost = P.shoot(lenses, w.kappa_c, w.gamma, w.grid_lo, w.grid_hi, w.grid_n, w.map_lo, w.map_hi,
                           w.map_n)
    nav = oracle.n_av(w)
    tr = synth.light_tracks(30, 6, w.map_lo, w.map_hi, 15.0)
    t = torch.from_numpy(tr).to(dev)
    mu, _ = P.light_curve(counts, w.map_lo, w.map_hi, w.map_n, nav, t, 101, "gaussian", 0.25, layout=LAYOUT["v"])
    torch.cuda.synchronize()
    mu_g = mu.cpu().numpy()
    cg = counts.cpu().numpy().view(np.uint32).astype(np.int64)
    co, _ = oracle.shoot_parallel(w)
    l1 = np.abs(cg - co.astype(np.int64)).sum()
    mu_o, _, _, den = lc.light_curve(co, w.map_lo, w.map_hi, w.map_n, nav, tr, 101, "gaussian", 0.25, sums=True)
    ok = ~np.isnan(mu_o)
    assert np.array_equal(ok, ~np.isnan(mu_g))
    bound = l1 / (nav * den[ok]) + 1e-12 * mu_o[ok]
    assert np.all(np.abs(mu_g[ok] - mu_o[ok]) <= bound)


def test_frame_stack_parity():
    # one map per point (a time-evolving field): 7 seeded frames of the rectangular map
    frames = np.stack([synth.count_map(40 + k, N, 30.0) for k in range(7)])
    tr = synth.light_tracks(41, 5, LO, HI, 6.0)
    for kind, size, exact in (("disc", 0.3, True), ("gaussian", 0.12, False)):
        mu_g, mag_g = _gpu(frames, LO, HI, N, 30.0, tr, 7, kind, size)
        mu_o, mag_o = lc.light_curve(frames, LO, HI, N, 30.0, tr, 7, kind, size)
        _compare(mu_g, mag_g, mu_o, mag_o, exact=exact)


def test_moving_field_light_curve_chain():
    # the 100-lens field with moving lenses: 6 frames shot as one GPU batch, the source moving
    # one track point per frame; against the oracle's frames and light curve, bounded by the
    # rays that switched pixel (as for a static map)
    torch, P = _env()
    w = synth.workload_small()
    v = synth.lens_velocities(42, w.n_lens, 0.2)
    dev = torch.device("cuda:0")
    L, V = torch.from_numpy(np.ascontiguousarray(w.lenses)).to(dev), torch.from_numpy(v).to(dev)
    F = 6
    stack = torch.zeros((F, w.map_n[1], w.map_n[0]), dtype=torch.int32, device=dev)
    losts = torch.zeros((F,), dtype=torch.int64, device=dev)
    jobs = [P.make_job(L, w.kappa_c, w.gamma, w.grid_lo, w.grid_hi, w.grid_n, w.map_lo, w.map_hi, w.map_n,
                       stack[k], losts[k:k + 1], velocities=V, time=0.5 * k) for k in range(F)]
    ws = torch.empty(P.batched_workspace_bytes(jobs), dtype=torch.uint8, device=dev)
    P.shoot_batched(jobs, ws)
    nav = oracle.n_av(w)
    tr = synth.light_tracks(43, 4, w.map_lo, w.map_hi, 6.0)
    mu, _ = P.light_curve(stack, w.map_lo, w.map_hi, w.map_n, nav, torch.from_numpy(tr).to(dev), F, "gaussian",
                          0.4, layout=LAYOUT["v"])
    torch.cuda.synchronize()
    mu_g = mu.cpu().numpy()
    frames_o, l1 = [], []
    cg = stack.cpu().numpy().view(np.uint32).astype(np.int64)
    for k in range(F):
        wt = synth.Workload(w.name, oracle.lenses_at(w.lenses, v, 0.5 * k), w.kappa_c, w.gamma, w.grid_lo,
                            w.grid_hi, w.grid_n, w.map_lo, w.map_hi, w.map_n)
        co, _ = oracle.shoot_parallel(wt, threads=16)
        frames_o.append(co)
        l1.append(np.abs(cg[k] - co.astype(np.int64)).sum())
    mu_o, _, _, den = lc.light_curve(np.stack(frames_o), w.map_lo, w.map_hi, w.map_n, nav, tr, F, "gaussian", 0.4,
                                     sums=True)
    ok = ~np.isnan(mu_o)
    assert np.array_equal(ok, ~np.isnan(mu_g)) and ok.sum() > 10
    bound = np.array(l1)[None, :] / (nav * np.where(ok, den, 1.0)) + 1e-12 * np.abs(np.nan_to_num(mu_o))
    assert np.all(np.abs(mu_g[ok] - mu_o[ok]) <= bound[ok])
    assert not np.allclose(mu_g[:, 0], mu_g[:, -1])          # the frames differ
