"""GPU tests of the magnification estimator rs_magnification (section 1, eq. 4: mu = N / N_av).

The bar is bit equality: the library's FP64 quotient must equal the oracle's counts / N_av for
the same counts, with N_av = pixel area / ray-cell area computed by the oracle.
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
    P.lib()
    return torch, P


def _mu(torch, P, counts_np, w, offset=0):
    dev = torch.device("cuda:0")
    c = torch.from_numpy(counts_np.astype(np.uint32).view(np.int32).copy()).to(dev)
    out = None
    if offset:
        # an output that is only 8-byte aligned (the kernel then stores one double at a time)
        buf = torch.full((counts_np.size + offset,), float("nan"), dtype=torch.float64, device=dev)
        out = buf[offset:].view(counts_np.shape)
    print(f"magnification: {w.name} map {w.map_n} offset {offset}", flush=True)
    mu, nav = P.magnification(c, w.grid_lo, w.grid_hi, w.grid_n, w.map_lo, w.map_hi, w.map_n, mu=out)
    torch.cuda.synchronize()
    return mu.cpu().numpy(), nav


def test_oracle_map_bit_exact():
    torch, P = _env()
    w = synth.workload_small()
    counts, lost = oracle.shoot_parallel(w)
    for off in (0, 1):
        mu, nav = _mu(torch, P, counts, w, off)
        assert nav == oracle.n_av(w)
        assert np.array_equal(mu, counts.astype(np.float64) / oracle.n_av(w))


def test_ragged_maps_and_gpu_counts():
    # map sizes that are not multiples of four bins (tail path), and a map the GPU shot
    torch, P = _env()
    w = synth.workload_small(seed=4)
    w.map_n = (37, 13)
    counts, _ = oracle.shoot_parallel(w)
    mu, _ = _mu(torch, P, counts, w)
    assert np.array_equal(mu, counts.astype(np.float64) / oracle.n_av(w))
    w1 = synth.workload_small(seed=4)
    w1.map_n = (1, 1)
    mu, _ = _mu(torch, P, np.array([[12345]], np.uint32), w1)
    assert mu[0, 0] == 12345 / oracle.n_av(w1)
    # the paper workload's map: mean mu over the source region is 1 / |(1 - kappa)^2 - gamma^2| = 10
    wp = synth.workload_paper()
    dev = torch.device("cuda:0")
    counts_t, lost = P.shoot(torch.from_numpy(wp.lenses).to(dev), wp.kappa_c, wp.gamma, wp.grid_lo, wp.grid_hi,
                             wp.grid_n, wp.map_lo, wp.map_hi, wp.map_n)
    mu_t, nav = P.magnification(counts_t, wp.grid_lo, wp.grid_hi, wp.grid_n, wp.map_lo, wp.map_hi, wp.map_n)
    torch.cuda.synchronize()
    cnp = counts_t.cpu().numpy().view(np.uint32)
    assert np.array_equal(mu_t.cpu().numpy(), cnp.astype(np.float64) / oracle.n_av(wp))
    want = 1.0 / abs((1 - wp.kappa_star - wp.kappa_c) ** 2 - wp.gamma ** 2)
    assert abs(float(mu_t.mean().item()) / want - 1) < 0.03
