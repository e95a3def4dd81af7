"""GPU tests of moving lenses (section 4: stars move between frames).

Bars: advanced lens records bit-identical to the oracle's (FP64 motion, float32 rounding on
both sides); a job with velocities and a time gives exactly the counts of the same job shot on
the oracle's advanced records (the positions are identical, so is every later operation); a
batch of frames equals its frames shot one by one; a moving-field zoom equals its full
fine-grid map; against the FP64 oracle the usual 1e-5 pixel-switch bar holds.
"""
import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu


def _env():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_0905_2453_amd as P
    P.lib()  # raises if the HIP library is missing: no fallback
    return torch, P


def _dev(a):
    torch, _ = _env()
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda:0")


def test_advance_lenses_bit_exact():
    torch, P = _env()
    L, _ = synth.lens_field(8, 100_003, kappa_star=0.5)
    v = synth.lens_velocities(9, 100_003, 0.05)
    for t in (0.0, 1.0, -7.25, 123.456):
        out = P.advance_lenses(_dev(L), _dev(v), t)
        torch.cuda.synchronize()
        assert np.array_equal(out.cpu().numpy().view(np.uint32), oracle.lenses_at(L, v, t).view(np.uint32)), t
    # in place
    Ld = _dev(L)
    P.advance_lenses(Ld, _dev(v), 2.5, out=Ld)
    torch.cuda.synchronize()
    assert np.array_equal(Ld.cpu().numpy(), oracle.lenses_at(L, v, 2.5))


def _shoot(P, torch, w, lenses_np, vel=None, t=0.0):
    dev = torch.device("cuda:0")
    counts = torch.zeros((w.map_n[1], w.map_n[0]), dtype=torch.int32, device=dev)
    lost = torch.zeros(1, dtype=torch.int64, device=dev)
    L = _dev(lenses_np)
    V = _dev(vel) if vel is not None else None
    job = P.make_job(L, w.kappa_c, w.gamma, w.grid_lo, w.grid_hi, w.grid_n, w.map_lo, w.map_hi, w.map_n, counts,
                     lost, velocities=V, time=t)
    ws = torch.empty(P.workspace_bytes(job), dtype=torch.uint8, device=dev)
    P.shoot_job(job, ws)
    torch.cuda.synchronize()
    return counts.cpu().numpy().view(np.uint32).copy(), int(lost.item())


def test_moving_job_equals_materialised_field_and_oracle():
    torch, P = _env()
    w = synth.workload_small()
    v = synth.lens_velocities(10, w.n_lens, 0.3)
    for t in (0.0, 1.5, 4.0):
        cm, lm = _shoot(P, torch, w, w.lenses, v, t)
        Lt = oracle.lenses_at(w.lenses, v, t)
        cs, ls = _shoot(P, torch, w, Lt)
        assert np.array_equal(cm, cs) and lm == ls, t
        wt = synth.Workload(w.name, Lt, w.kappa_c, w.gamma, w.grid_lo, w.grid_hi, w.grid_n, w.map_lo, w.map_hi,
                            w.map_n)
        co, lo_ = oracle.shoot_parallel(wt, threads=16)
        l1 = int(np.abs(cm.astype(np.int64) - co.astype(np.int64)).sum())
        assert l1 <= 2 * 1e-5 * w.n_rays + 2, (t, l1)
    # the field really moved
    assert not np.array_equal(_shoot(P, torch, w, w.lenses, v, 0.0)[0], _shoot(P, torch, w, w.lenses, v, 4.0)[0])


def test_frames_in_one_batch_equal_single_frames():
    # 12 frames of a 20000-lens field (kappa_* = gamma = 0.45), 1024^2 rays, 256^2 map, one
    # persistent launch; each frame against the same job shot alone
    torch, P = _env()
    w = synth.workload_paper(n_lens=20000, grid=1024, mapn=256)
    v = synth.lens_velocities(11, w.n_lens, 0.02)
    dev = torch.device("cuda:0")
    L, V = _dev(w.lenses), _dev(v)
    times = [0.5 * k for k in range(12)]
    maps, losts, jobs = [], [], []
    for t in times:
        c = torch.zeros((w.map_n[1], w.map_n[0]), dtype=torch.int32, device=dev)
        lo = torch.zeros(1, dtype=torch.int64, device=dev)
        maps.append(c)
        losts.append(lo)
        jobs.append(P.make_job(L, w.kappa_c, w.gamma, w.grid_lo, w.grid_hi, w.grid_n, w.map_lo, w.map_hi, w.map_n,
                               c, lo, velocities=V, time=t))
    ws = torch.empty(P.batched_workspace_bytes(jobs), dtype=torch.uint8, device=dev)
    P.shoot_batched(jobs, ws)
    torch.cuda.synchronize()
    prev = None
    for k, t in enumerate(times):
        cs, ls = _shoot(P, torch, w, w.lenses, v, t)
        got = maps[k].cpu().numpy().view(np.uint32)
        assert np.array_equal(got, cs) and int(losts[k].item()) == ls, t
        if prev is not None:
            assert not np.array_equal(got, prev)
        prev = got.copy()


def test_zoom_on_moving_field_equals_fine_grid():
    torch, P = _env()
    w = synth.workload_paper(n_lens=20000, grid=2048)
    v = synth.lens_velocities(12, w.n_lens, 0.05)
    dev = torch.device("cuda:0")
    L, V = _dev(w.lenses), _dev(v)
    mlo, mhi, mn = (-1.0, -1.5), (1.5, 1.0), (128, 128)
    out = []
    for zoom in (False, True):
        c = torch.zeros((mn[1], mn[0]), dtype=torch.int32, device=dev)
        lo = torch.zeros(1, dtype=torch.int64, device=dev)
        job = P.make_job(L, w.kappa_c, w.gamma, w.grid_lo, w.grid_hi, w.grid_n, mlo, mhi, mn, c, lo,
                         velocities=V, time=3.0)
        if zoom:
            z = P.zoom_params()
            ws = torch.empty(P.zoom_workspace_bytes(job, z), dtype=torch.uint8, device=dev)
            P.shoot_zoom(job, z, ws)
            st = P.zoom_stats(ws)
            assert st["slots_shot"] < st["slots"]
        else:
            ws = torch.empty(P.workspace_bytes(job), dtype=torch.uint8, device=dev)
            P.shoot_job(job, ws)
        torch.cuda.synchronize()
        out.append(c.cpu().numpy().view(np.uint32).copy())
    assert out[0].sum() > 0 and np.array_equal(out[0], out[1])


def test_frame_batch_full_size_sampled_parity():
    # The benchmark's frame leg at full size: the paper workload (1e5 lenses, 4096^2 rays, 1024^2
    # map) at times 0..7 with a velocity dispersion of 0.05 per axis, one persistent launch; every
    # frame bit-identical to its moving job shot alone, and 2048 seeded rays of each frame's dump
    # against the FP64 oracle on the advanced field (switches counted over all frames against the
    # 1e-5 bar with its Poisson allowance).
    import math
    torch, P = _env()
    w = synth.workload_paper()
    v = synth.lens_velocities(13, w.n_lens, 0.05)
    dev = torch.device("cuda:0")
    L, V = _dev(w.lenses), _dev(v)
    times = [float(k) for k in range(8)]
    maps = [torch.zeros((w.map_n[1], w.map_n[0]), dtype=torch.int32, device=dev) for _ in times]
    losts = [torch.zeros(1, dtype=torch.int64, device=dev) for _ in times]
    jobs = [P.make_job(L, w.kappa_c, w.gamma, w.grid_lo, w.grid_hi, w.grid_n, w.map_lo, w.map_hi, w.map_n,
                       maps[k], losts[k], velocities=V, time=t) for k, t in enumerate(times)]
    ws = torch.empty(P.batched_workspace_bytes(jobs), dtype=torch.uint8, device=dev)
    P.shoot_batched(jobs, ws)
    torch.cuda.synchronize()
    del ws
    nr = w.n_rays
    n_sw = n_in = 0
    for k, t in enumerate(times):
        c = torch.zeros_like(maps[k])
        lo = torch.zeros(1, dtype=torch.int64, device=dev)
        j = P.make_job(L, w.kappa_c, w.gamma, w.grid_lo, w.grid_hi, w.grid_n, w.map_lo, w.map_hi, w.map_n, c, lo,
                       velocities=V, time=t)
        ry = torch.empty((nr, 2), dtype=torch.float64, device=dev)
        rp = torch.empty((nr,), dtype=torch.int32, device=dev)
        o = P.Opts()
        o.ray_y, o.ray_pix = ry.data_ptr(), rp.data_ptr()
        wsj = torch.empty(P.workspace_bytes(j, o), dtype=torch.uint8, device=dev)
        P.shoot_job(j, wsj, o)
        torch.cuda.synchronize()
        assert torch.equal(c, maps[k]) and int(lo.item()) == int(losts[k].item()), t
        assert int(c.sum().item()) + int(lo.item()) == nr
        idx = synth.sample_indices(200 + k, nr, 2048)
        p_g = rp[torch.from_numpy(idx).to(dev)].cpu().numpy().astype(np.int64)
        del ry, rp, wsj
        wt = synth.Workload(w.name, oracle.lenses_at(w.lenses, v, t), w.kappa_c, w.gamma, w.grid_lo, w.grid_hi,
                            w.grid_n, w.map_lo, w.map_hi, w.map_n)
        _, p_o = oracle.trace_parallel(wt, idx, threads=16)
        n_sw += int(np.sum(p_g != p_o))
        n_in += int(np.sum((p_g >= 0) | (p_o >= 0)))
    mean = 1e-5 * n_in
    print(f"8 moving frames at full size: {n_sw} of {n_in} sampled rays in a map switch pixel")
    assert n_sw <= mean + 3.0 * math.sqrt(mean)
