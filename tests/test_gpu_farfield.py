"""GPU tests of the learned far-field closure (rs_farfield_fit / rs_farfield_eval).

Checked against the FP64 oracles (oracle/farfield.py for the affine base and the exact
far-field samples, oracle/mlp.py with bfloat16 operand emulation for the gradient and
training), and against the plain direct sum (rs_shoot) as the reference for the map error.
Surrogate tolerance: map L1 relative error sum|N_s - N_p| / sum N_p <= 1% at the stated ray
density; the affine base alone (network off) must fail that bound.
"""
import numpy as np
import pytest

import oracle
import synth
from oracle import farfield as off
from oracle import mlp

pytestmark = pytest.mark.gpu

R_NEAR = 8.0
TILE = (64, 64)


def _env():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_0905_2453_amd as P
    P.lib()
    return torch, P


def _fit(torch, P, w, window, steps, n_samples=4096, batch=512, seed=1, debug=False):
    dev = torch.device("cuda:0")
    lenses = torch.from_numpy(w.lenses).to(dev)
    counts = torch.zeros((w.map_n[1], w.map_n[0]), dtype=torch.int32, device=dev)
    lost = torch.zeros(1, dtype=torch.int64, device=dev)
    job = P.make_job(lenses, w.kappa_c, w.gamma, w.grid_lo, w.grid_hi, w.grid_n, w.map_lo, w.map_hi, w.map_n,
                     counts, lost, window=window)
    u = synth.fit_samples(seed, n_samples)
    p0 = synth.init_params(seed)
    ut = torch.from_numpy(u).to(dev)
    pt = torch.from_numpy(p0).to(dev)
    ntx = (window[1][0] + TILE[0] - 1) // TILE[0]
    nty = (window[1][1] + TILE[1] - 1) // TILE[1]
    dg = torch.zeros((ntx * nty, mlp.N_PARAMS), dtype=torch.float32, device=dev) if debug else None
    dt = torch.zeros((ntx * nty, n_samples, 2), dtype=torch.float32, device=dev) if debug else None
    cfg = P.ff_config(ut, pt, tile_rays=TILE, r_near=R_NEAR, steps=steps, batch=batch, lr=1e-2,
                      debug_grad=dg, debug_targets=dt)
    model = torch.zeros(P.farfield_model_bytes(job, cfg), dtype=torch.uint8, device=dev)
    ws = torch.empty(P.farfield_fit_workspace_bytes(job, cfg), dtype=torch.uint8, device=dev)
    P.farfield_fit(job, cfg, model, ws)
    torch.cuda.synchronize()
    keep = (lenses, counts, lost, ut, pt, ws)
    return job, cfg, model, dg, dt, u, p0, keep


def _records(model, n_tiles):
    m = model.cpu().numpy()
    rec = (len(m) - 256) // n_tiles
    hdr = np.stack([m[256 + t * rec: 256 + t * rec + 80].view(np.float64) for t in range(n_tiles)])
    w16 = np.stack([m[256 + t * rec + 128: 256 + t * rec + 128 + 2 * mlp.N_PARAMS].view(np.uint16)
                    for t in range(n_tiles)])
    boff = 256 + 128 + ((2 * mlp.N_PARAMS + 15) // 16) * 16
    bias = np.stack([m[t * rec + boff: t * rec + boff + 520].view(np.float32) for t in range(n_tiles)])
    weights = (w16.astype(np.uint32) << 16).view(np.float32).astype(np.float64)
    return hdr, weights, bias


def _small_field():
    return synth.workload_farfield(n_lens=20000, grid=8192)   # 64-ray tiles: 1.9 x 0.27 Einstein radii


WIN = ((4032, 4064), (256, 128))   # 4 x 2 tiles around the grid centre


def test_affine_base_and_far_samples_match_oracle():
    torch, P = _env()
    w = _small_field()
    job, cfg, model, dg, dt, u, p0, keep = _fit(torch, P, w, WIN, steps=0, debug=True)
    hdr, _, _ = _records(model, 8)
    tg = dt.cpu().numpy()
    for t in (0, 5):
        tx, ty = t % 4, t // 4
        res, st, a0, J, far = off.tile_targets(w, WIN, TILE, tx, ty, R_NEAR, u, threads=16)
        lo, hi, c, h, _ = off.tile_rect(w, WIN, TILE, tx, ty)
        assert np.allclose(hdr[t, 0:2], c, rtol=0, atol=1e-12) and np.allclose(hdr[t, 2:4], h, rtol=1e-14)
        assert np.allclose(hdr[t, 4:6], a0, rtol=1e-10, atol=1e-12)
        assert np.allclose(hdr[t, 6:9], [J[0, 0], J[0, 1], J[1, 1]], rtol=1e-9, atol=1e-12)
        # float32 far-field sums with FP64 combination vs FP64: 0.2% of the residual's RMS
        err = np.sqrt(np.mean((tg[t] - res) ** 2))
        assert err <= 2e-3 * st, (t, err, st)
        assert abs(hdr[t, 9] / st - 1) < 2e-3


def test_first_step_gradient_matches_bf16_oracle():
    torch, P = _env()
    w = _small_field()
    job, cfg, model, dg, dt, u, p0, keep = _fit(torch, P, w, WIN, steps=1, debug=True)
    g_gpu = dg.cpu().numpy()
    for t in (0, 6):
        res, st, *_ = off.tile_targets(w, WIN, TILE, t % 4, t // 4, R_NEAR, u, threads=16)
        g = mlp.gradient(p0.astype(np.float64), u[:512].astype(np.float64), res[:512] / st, bf=True)
        rel = np.linalg.norm(g_gpu[t] - g) / np.linalg.norm(g)
        assert rel < 2e-3, (t, rel)
        for lo_, hi_ in [(mlp.OFF_W1, mlp.OFF_B1), (mlp.OFF_W2, mlp.OFF_B2), (mlp.OFF_W3, mlp.N_PARAMS)]:
            assert np.allclose(g_gpu[t][lo_:hi_], g[lo_:hi_], rtol=0, atol=5e-3 * np.abs(g[lo_:hi_]).max())


def test_training_steps_match_bf16_oracle():
    torch, P = _env()
    w = _small_field()
    steps = 12
    job, cfg, model, dg, dt, u, p0, keep = _fit(torch, P, w, WIN, steps=steps)
    _, wts, bias = _records(model, 8)
    t = 3
    res, st, *_ = off.tile_targets(w, WIN, TILE, t % 4, t // 4, R_NEAR, u, threads=16)
    tgt = res / st
    p_o = mlp.train(p0.astype(np.float64), u.astype(np.float64), tgt, steps=steps, batch=512, lr=1e-2, bf=True)
    p_g = wts[t].copy()
    p_g[mlp.OFF_B1:mlp.OFF_W2] = bias[t][:64]
    p_g[mlp.OFF_B2:mlp.OFF_W3] = bias[t][64:128]
    p_g[mlp.OFF_B3:] = bias[t][128:130]
    moved = np.linalg.norm(p_o - p0)
    assert np.linalg.norm(p_g - p_o) / moved < 0.05
    l0 = mlp.loss(p0.astype(np.float64), u, tgt, bf=True)
    lg = mlp.loss(p_g, u, tgt, bf=True)
    lo_ = mlp.loss(p_o, u, tgt, bf=True)
    assert lg < 0.9 * l0 and abs(lg / lo_ - 1) < 0.05, (l0, lg, lo_)


def _map(torch, P, job, counts, lost):
    torch.cuda.synchronize()
    return counts.cpu().numpy().view(np.uint32).astype(np.int64), int(lost.item())


def test_surrogate_map_error_vs_plain_judge():
    # 1e6 lenses, kappa_* = 0.6, gamma = 0.3: the learned-closure workload's field and tiles,
    # on a 1024 x 512-ray window of its 8192^2 grid (128 tiles)
    torch, P = _env()
    w = synth.workload_farfield()
    win = ((3584, 3840), (1024, 512))
    job, cfg, model, dg, dt, u, p0, keep = _fit(torch, P, w, win, steps=2000)
    lenses, counts, lost = keep[0], keep[1], keep[2]
    dev = torch.device("cuda:0")
    nr = win[1][0] * win[1][1]
    ews = torch.empty(P.farfield_eval_workspace_bytes(job, cfg), dtype=torch.uint8, device=dev)

    def run_eval(flags):
        counts.zero_()
        lost.zero_()
        ry = torch.empty((nr, 2), dtype=torch.float64, device=dev)
        rp = torch.full((nr,), -7, dtype=torch.int32, device=dev)
        o = P.Opts()
        o.ray_y, o.ray_pix, o.flags = ry.data_ptr(), rp.data_ptr(), flags
        P.farfield_eval(job, cfg, model, ews, o)
        c, l = _map(torch, P, job, counts, lost)
        return c, l, ry.cpu().numpy(), rp.cpu().numpy()

    cs, ls, ys, ps = run_eval(0)
    ca, la, ya, pa = run_eval(P._abi.RS_FLAG_AFFINE_ONLY)
    # the judge: the plain direct sum on the same rays
    counts.zero_()
    lost.zero_()
    ry = torch.empty((nr, 2), dtype=torch.float64, device=dev)
    rp = torch.empty((nr,), dtype=torch.int32, device=dev)
    o = P.Opts()
    o.ray_y, o.ray_pix = ry.data_ptr(), rp.data_ptr()
    ws = torch.empty(P.workspace_bytes(job, o), dtype=torch.uint8, device=dev)
    P.shoot_job(job, ws, o)
    cp, lp = _map(torch, P, job, counts, lost)
    yp, pp = ry.cpu().numpy(), rp.cpu().numpy()
    assert int(cs.sum()) + ls == nr and int(cp.sum()) + lp == nr
    assert np.array_equal(cs.ravel(), np.bincount(ps[ps >= 0], minlength=cs.size))
    l1 = np.abs(cs - cp).sum() / cp.sum()
    l1_aff = np.abs(ca - cp).sum() / cp.sum()
    sw = np.mean(ps != pp)
    dyn = np.abs(ys - yp)[np.isfinite(yp).all(1)]
    print(f"surrogate: map L1 {l1:.2e}, affine-only {l1_aff:.2e}; ray switch {sw:.2e}; "
          f"median |dy| {np.median(dyn):.2e}, p99 {np.percentile(dyn, 99):.2e}")
    assert l1 <= 1e-2
    assert l1_aff > 1e-2 and l1_aff > 3 * l1


def test_sample_layouts_give_identical_targets():
    # a fit with many tiles takes four samples per thread, one with few tiles two: the exact
    # far-field targets of the tiles they share must agree bit for bit
    torch, P = _env()
    w = _small_field()
    dev = torch.device("cuda:0")
    lenses = torch.from_numpy(w.lenses).to(dev)
    counts = torch.zeros((w.map_n[1], w.map_n[0]), dtype=torch.int32, device=dev)
    lost = torch.zeros(1, dtype=torch.int64, device=dev)
    ut = torch.from_numpy(synth.fit_samples_quads(5, 1024)).to(dev)
    pt = torch.from_numpy(synth.init_params(5)).to(dev)
    got = []
    for tiles in ((64, 64), (4, 2)):          # 4096 tiles (four per thread), 8 tiles (two per thread)
        win = ((0, 0), (TILE[0] * tiles[0], TILE[1] * tiles[1]))
        job = P.make_job(lenses, w.kappa_c, w.gamma, w.grid_lo, w.grid_hi, w.grid_n, w.map_lo, w.map_hi,
                         w.map_n, counts, lost, window=win)
        dt = torch.zeros((tiles[0] * tiles[1], 1024, 2), dtype=torch.float32, device=dev)
        cfg = P.ff_config(ut, pt, tile_rays=TILE, r_near=R_NEAR, steps=1, batch=512, debug_targets=dt,
                          shared_x=True)
        model = torch.zeros(P.farfield_model_bytes(job, cfg), dtype=torch.uint8, device=dev)
        ws = torch.empty(P.farfield_fit_workspace_bytes(job, cfg), dtype=torch.uint8, device=dev)
        P.farfield_fit(job, cfg, model, ws)
        torch.cuda.synchronize()
        got.append(dt.cpu().numpy().reshape(tiles[1], tiles[0], 1024, 2))
        del model, ws
    assert np.isfinite(got[1]).all() and np.abs(got[1]).max() > 0
    assert np.array_equal(got[0][:2, :4], got[1])


def test_fit_is_deterministic():
    # fixed-order reductions everywhere: two fits of the same input give the same bytes
    torch, P = _env()
    w = _small_field()
    a = _fit(torch, P, w, WIN, steps=50)
    b = _fit(torch, P, w, WIN, steps=50)
    assert np.array_equal(a[2].cpu().numpy(), b[2].cpu().numpy())


def test_mismatched_model_is_rejected():
    torch, P = _env()
    w = _small_field()
    job, cfg, model, dg, dt, u, p0, keep = _fit(torch, P, w, WIN, steps=1)
    ews = torch.empty(P.farfield_eval_workspace_bytes(job, cfg), dtype=torch.uint8, device="cuda:0")
    cfg.steps = 2
    with pytest.raises(P.RayShootError) as ei:
        P.farfield_eval(job, cfg, model, ews)
    assert ei.value.status == -5


def test_binding_keeps_tensors_alive_and_checks_debug_sizes():
    """The binding's structs hold raw device addresses: they keep their tensors alive, and a debug
    buffer too small for the job's tiles is refused before any library call."""
    import gc
    torch, P = _env()
    w = _small_field()
    dev = torch.device("cuda:0")
    job = P.make_job(torch.from_numpy(w.lenses).to(dev), w.kappa_c, w.gamma, w.grid_lo, w.grid_hi, w.grid_n,
                     w.map_lo, w.map_hi, w.map_n,
                     torch.zeros((w.map_n[1], w.map_n[0]), dtype=torch.int32, device=dev),
                     torch.zeros(1, dtype=torch.int64, device=dev), window=WIN)
    gc.collect()
    assert job._tensors[0].data_ptr() == job.lenses and job._tensors[1].data_ptr() == job.counts
    ntx = (WIN[1][0] + TILE[0] - 1) // TILE[0]
    nty = (WIN[1][1] + TILE[1] - 1) // TILE[1]
    ut = torch.from_numpy(synth.fit_samples(1, 1024)).to(dev)
    pt = torch.from_numpy(synth.init_params(1)).to(dev)
    small = torch.zeros((ntx * nty - 1, mlp.N_PARAMS), dtype=torch.float32, device=dev)
    cfg = P.ff_config(ut, pt, tile_rays=TILE, r_near=R_NEAR, steps=1, batch=512, debug_grad=small)
    model = torch.zeros(P.farfield_model_bytes(job, cfg), dtype=torch.uint8, device=dev)
    ws = torch.empty(P.farfield_fit_workspace_bytes(job, cfg), dtype=torch.uint8, device=dev)
    with pytest.raises(ValueError, match="debug_grad"):
        P.farfield_fit(job, cfg, model, ws)
    short = torch.zeros((ntx * nty, 1023, 2), dtype=torch.float32, device=dev)
    cfg = P.ff_config(ut, pt, tile_rays=TILE, r_near=R_NEAR, steps=1, batch=512, debug_targets=short)
    with pytest.raises(ValueError, match="debug_targets"):
        P.farfield_fit(job, cfg, model, ws)
    with pytest.raises(ValueError, match="dtype"):
        P.ff_config(ut, pt, debug_grad=small.double())


# ---------------------------------------------------------------- moving field, one closure

def _eval(torch, P, job, cfg, model, counts, lost, flags=0, dump=False):
    dev = torch.device("cuda:0")
    counts.zero_()
    lost.zero_()
    ews = torch.empty(P.farfield_eval_workspace_bytes(job, cfg), dtype=torch.uint8, device=dev)
    o = P.Opts()
    o.flags = flags
    nr = job.grid.win_n[0] * job.grid.win_n[1]
    ry = rp = None
    if dump:
        ry = torch.full((nr, 2), float("nan"), dtype=torch.float64, device=dev)
        rp = torch.full((nr,), -7, dtype=torch.int32, device=dev)
        o.ray_y, o.ray_pix = ry.data_ptr(), rp.data_ptr()
    P.farfield_eval(job, cfg, model, ews, o)
    torch.cuda.synchronize()
    c = counts.cpu().numpy().view(np.uint32).astype(np.int64)
    return (c, ry.cpu().numpy(), rp.cpu().numpy()) if dump else c


def _moving_job(P, job, w, lenses, counts, lost, vel, t):
    return P.make_job(lenses, w.kappa_c, w.gamma, w.grid_lo, w.grid_hi, w.grid_n, w.map_lo, w.map_hi, w.map_n,
                      counts, lost, window=((job.grid.win_lo[0], job.grid.win_lo[1]),
                                            (job.grid.win_n[0], job.grid.win_n[1])), velocities=vel, time=t)


def test_moving_eval_at_time_zero_equals_static():
    torch, P = _env()
    w = _small_field()
    job, cfg, model, dg, dt, u, p0, keep = _fit(torch, P, w, WIN, steps=20)
    lenses, counts, lost = keep[0], keep[1], keep[2]
    vel = torch.from_numpy(synth.lens_velocities(21, w.n_lens, 0.3)).to("cuda:0")
    c_static = _eval(torch, P, job, cfg, model, counts, lost)
    c_t0 = _eval(torch, P, _moving_job(P, job, w, lenses, counts, lost, vel, 0.0), cfg, model, counts, lost)
    assert c_static.sum() > 0 and np.array_equal(c_static, c_t0)


def test_moving_eval_affine_and_near_field_match_oracle():
    # network off: y = lambda x - (affine base of the far set at time t + near set at time t),
    # near and far sets chosen by the fit-time positions
    torch, P = _env()
    w = _small_field()
    job, cfg, model, dg, dt, u, p0, keep = _fit(torch, P, w, WIN, steps=1)
    lenses, counts, lost = keep[0], keep[1], keep[2]
    v = synth.lens_velocities(22, w.n_lens, 0.3)
    t = 1.5
    vel = torch.from_numpy(v).to("cuda:0")          # the job holds only its address: keep it alive
    mj = _moving_job(P, job, w, lenses, counts, lost, vel, t)
    _, ry, _ = _eval(torch, P, mj, cfg, model, counts, lost, flags=P._abi.RS_FLAG_AFFINE_ONLY, dump=True)
    Lt = oracle.lenses_at(w.lenses, v, t)
    lam = (1.0 - w.gamma - w.kappa_c, 1.0 + w.gamma - w.kappa_c)
    (wl1, wl2), (wn1, wn2) = WIN
    for tile in (0, 5):
        tx, ty = tile % 4, tile // 4
        lo, hi, c, h, (i0, n) = off.tile_rect(w, WIN, TILE, tx, ty)
        near = off.near_mask(w.lenses, lo, hi, R_NEAR)
        a0, J = off.affine_base(np.ascontiguousarray(Lt[~near]), c)
        idx = synth.sample_indices(23 + tile, n[0] * n[1], 400)
        ix, iy = idx % n[0], idx // n[0]
        g1, g2 = i0[0] + ix, i0[1] + iy
        x = np.stack([oracle.axis(w.grid_lo[0], w.grid_hi[0], w.grid_n[0])[g1],
                      oracle.axis(w.grid_lo[1], w.grid_hi[1], w.grid_n[1])[g2]], 1).astype(np.float64)
        Ln = np.ascontiguousarray(Lt[near])
        an = oracle.deflect(Ln, x)
        y_o = np.stack([lam[0] * x[:, 0], lam[1] * x[:, 1]], 1) - (a0[None, :] + (x - c[None, :]) @ J.T + an)
        rw = (g2 - wl2) * wn1 + (g1 - wl1)
        s = np.sum(Ln[None, :, 2] / np.hypot(x[:, None, 0] - Ln[None, :, 0], x[:, None, 1] - Ln[None, :, 1]), 1)
        bound = 48 * 2.0 ** -24 * s[:, None] + 1e-9 * (1 + np.abs(y_o))
        assert np.all(np.abs(ry[rw] - y_o) <= bound), np.max(np.abs(ry[rw] - y_o) / bound)


def test_moving_surrogate_error_vs_plain_moving_field():
    # the 1e6-lens closure workload's field and tiles on a 1024 x 512-ray window (128 tiles),
    # fitted once at time 0 and evaluated at time 2 with a velocity dispersion of 0.05 per axis
    # (0.1 Einstein radii RMS displacement); the plain direct sum of the moved field judges it
    torch, P = _env()
    w = synth.workload_farfield()
    win = ((3584, 3840), (1024, 512))
    job, cfg, model, dg, dt, u, p0, keep = _fit(torch, P, w, win, steps=2000)
    lenses, counts, lost = keep[0], keep[1], keep[2]
    dev = torch.device("cuda:0")
    vel = torch.from_numpy(synth.lens_velocities(24, w.n_lens, 0.05)).to(dev)
    t = 2.0
    mj = _moving_job(P, job, w, lenses, counts, lost, vel, t)
    c_mov = _eval(torch, P, mj, cfg, model, counts, lost)
    c_frozen = _eval(torch, P, job, cfg, model, counts, lost)        # the closure ignoring the motion
    counts.zero_()
    lost.zero_()
    ws = torch.empty(P.workspace_bytes(mj), dtype=torch.uint8, device=dev)
    P.shoot_job(mj, ws)
    torch.cuda.synchronize()
    c_pl = counts.cpu().numpy().view(np.uint32).astype(np.int64)
    l1 = np.abs(c_mov - c_pl).sum() / c_pl.sum()
    l1_frozen = np.abs(c_frozen - c_pl).sum() / c_pl.sum()
    print(f"moving field at t={t}: closure map L1 {l1:.2e}, frozen closure {l1_frozen:.2e}")
    assert l1 <= 1e-2 and l1_frozen > 3 * l1


def test_shared_x_samples_fit_is_bit_identical():
    # samples in quads sharing their first coordinate let the fit share x-differences; every
    # sample still sees the same operations, so the model must not change by a single bit
    torch, P = _env()
    w = _small_field()
    dev = torch.device("cuda:0")
    lenses = torch.from_numpy(w.lenses).to(dev)
    counts = torch.zeros((w.map_n[1], w.map_n[0]), dtype=torch.int32, device=dev)
    lost = torch.zeros(1, dtype=torch.int64, device=dev)
    job = P.make_job(lenses, w.kappa_c, w.gamma, w.grid_lo, w.grid_hi, w.grid_n, w.map_lo, w.map_hi, w.map_n,
                     counts, lost, window=WIN)
    ut = torch.from_numpy(synth.fit_samples_quads(3)).to(dev)
    pt = torch.from_numpy(synth.init_params(3)).to(dev)
    models = []
    for shared in (False, True):
        cfg = P.ff_config(ut, pt, tile_rays=TILE, r_near=R_NEAR, steps=30, batch=512, lr=1e-2, shared_x=shared)
        model = torch.zeros(P.farfield_model_bytes(job, cfg), dtype=torch.uint8, device=dev)
        ws = torch.empty(P.farfield_fit_workspace_bytes(job, cfg), dtype=torch.uint8, device=dev)
        P.farfield_fit(job, cfg, model, ws)
        torch.cuda.synchronize()
        models.append(model.cpu().numpy())
    assert np.array_equal(models[0], models[1])
    # samples that do not share their first coordinates as declared are refused before any launch
    bad = torch.from_numpy(synth.fit_samples(3, 4096)).to(dev)
    cfg = P.ff_config(bad, pt, tile_rays=TILE, r_near=R_NEAR, steps=1, shared_x=True)
    model = torch.zeros(P.farfield_model_bytes(job, cfg), dtype=torch.uint8, device=dev)
    ws = torch.empty(P.farfield_fit_workspace_bytes(job, cfg), dtype=torch.uint8, device=dev)
    with pytest.raises(P.RayShootError) as ei:
        P.farfield_fit(job, cfg, model, ws)
    assert ei.value.status == -1
