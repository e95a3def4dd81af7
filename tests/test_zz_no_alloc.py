"""GPU test of rs_shoot_noalloc (the entry point for callers that cannot allocate) against rs_shoot.

Both run the same kernels, so the bar is bit equality: counts, lost rays and the per-ray dumps
(FP64 source position and pixel) of rs_shoot_noalloc must equal rs_shoot's on the same job.
Two calls in a row, the second on a smaller map and window, check that the fixed scratch array
is cleared for each call (nothing left from the larger first call leaks into the second).
"""
import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu


def _env():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_0905_2453_amd as P
    P.lib()
    return torch, P


def _run(torch, P, w, window, noalloc, jitter_seed=None):
    dev = torch.device("cuda:0")
    lenses = torch.from_numpy(w.lenses).to(dev)
    counts = torch.zeros((w.map_n[1], w.map_n[0]), dtype=torch.int32, device=dev)
    lost = torch.zeros(1, dtype=torch.int64, device=dev)
    job = P.make_job(lenses, w.kappa_c, w.gamma, w.grid_lo, w.grid_hi, w.grid_n, w.map_lo, w.map_hi, w.map_n,
                     counts, lost, window=window, jitter_seed=jitter_seed)
    nr = window[1][0] * window[1][1]
    ry = torch.full((nr, 2), float("nan"), dtype=torch.float64, device=dev)
    rp = torch.full((nr,), -7, dtype=torch.int32, device=dev)
    o = P.Opts()
    o.ray_y, o.ray_pix = ry.data_ptr(), rp.data_ptr()
    print(f"no-alloc test: {w.name} window {window} noalloc={noalloc}", flush=True)
    if noalloc:
        P.shoot_job_noalloc(job, o)
    else:
        ws = torch.empty(P.workspace_bytes(job, o), dtype=torch.uint8, device=dev)
        P.shoot_job(job, ws, o)
    torch.cuda.synchronize()
    return (counts.cpu().numpy().view(np.uint32).copy(), int(lost.item()), ry.cpu().numpy(), rp.cpu().numpy())


def test_noalloc_equals_shoot_two_calls_second_smaller():
    torch, P = _env()
    # call 1: the largest map the fixed scratch takes (1024 x 1024 bins), 2e4 power-law lenses,
    # a ragged window that starts on an odd row; call 2: a 100 x 100 map and a smaller window
    big = synth.workload_paper(n_lens=20000)
    small = synth.workload_small(seed=3)
    cases = [(big, ((1500, 1801), (1000, 333)), None), (small, ((7, 3), (411, 129)), None),
             (small, ((0, 0), (1000, 1000)), 77)]
    got = [_run(torch, P, w, win, True, js) for w, win, js in cases]
    want = [_run(torch, P, w, win, False, js) for w, win, js in cases]
    for (w, win, _), g, r in zip(cases, got, want):
        nr = win[1][0] * win[1][1]
        assert int(g[0].sum()) + g[1] == nr
        assert np.array_equal(g[0], r[0]) and g[1] == r[1], w.name
        assert np.array_equal(g[2], r[2]) and np.array_equal(g[3], r[3]), w.name


def test_noalloc_rejects_maps_beyond_its_scratch():
    torch, P = _env()
    w = synth.workload_small()
    dev = torch.device("cuda:0")
    lenses = torch.from_numpy(w.lenses).to(dev)
    counts = torch.zeros((1024, 1025), dtype=torch.int32, device=dev)
    lost = torch.zeros(1, dtype=torch.int64, device=dev)
    job = P.make_job(lenses, w.kappa_c, w.gamma, w.grid_lo, w.grid_hi, w.grid_n, w.map_lo, w.map_hi, (1025, 1024),
                     counts, lost)
    with pytest.raises(P.RayShootError) as ei:
        P.shoot_job_noalloc(job)
    assert ei.value.status == -2 and "at most" in ei.value.detail
    torch.cuda.synchronize()
    assert int(counts.sum().item()) == 0 and int(lost.item()) == 0
