"""GPU check of the ray budget planner: a planned grid shot through a field of known mean
convergence gives a map whose mean N / N_av is the mean magnification 1 / |(1-k)^2 - g^2| of
that field (section 1 eq. 4; the macro model of section 3.2), averaged over seeded fields."""
import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu


def test_planned_grid_gives_mean_magnification():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_0905_2453_amd as P
    P.lib()
    ks, g = 0.3, 0.2
    mlo, mhi, mn = (-8.0, -8.0), (8.0, 8.0), (128, 128)
    ratios = []
    for seed in range(4):
        lenses, r = synth.lens_field(40 + seed, 6000, kappa_star=ks)
        lo, hi, n, nav = P.plan_grid(mlo, mhi, mn, 60.0, kappa_star=ks, gamma=g, lens_extent=r)
        assert r > 1.3 * max(abs(lo[0]), abs(hi[0]), abs(lo[1]), abs(hi[1]))   # field covers the region
        counts, lost = P.shoot(torch.from_numpy(lenses).to("cuda:0"), 0.0, g, lo, hi, n, mlo, mhi, mn)
        torch.cuda.synchronize()
        c = counts.cpu().numpy().view(np.uint32)
        assert int(c.sum()) + int(lost.item()) == n[0] * n[1]
        ratios.append(c.mean() / nav)
    want = 1.0 / abs((1 - ks) ** 2 - g ** 2)
    print("mean N / N_av per field:", ratios, "theory", want)
    assert abs(np.mean(ratios) / want - 1) < 0.05
