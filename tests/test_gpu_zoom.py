"""GPU tests of the interactive zoom (rs_shoot_zoom).

The zoom map is defined as the map that the whole fine ray grid gives on the selected window,
so the bar is exact: its counts must equal rs_shoot's on the same fine job bit for bit, while
fewer ray tiles are shot.  Against the FP64 oracle's fine-grid map the usual pixel-switch bar
applies (|d N| summed <= 2 x 1e-5 x rays in the window, plus rounding slack of one ray).
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


def _fine(w, refine):
    return (w.grid_n[0] * refine, w.grid_n[1] * refine)


def _run(w, grid_n, map_lo, map_hi, map_n, window=None, zoom=None, opts=None, jitter_seed=None):
    """Plain fine shoot and zoom of the same job; returns (plain counts, zoom counts, stats)."""
    torch, P = _env()
    dev = torch.device("cuda:0")
    lenses = torch.from_numpy(np.ascontiguousarray(w.lenses)).to(dev)
    cp = torch.zeros((map_n[1], map_n[0]), dtype=torch.int32, device=dev)
    cz = torch.zeros_like(cp)
    lp = torch.zeros(1, dtype=torch.int64, device=dev)
    lz = torch.zeros_like(lp)
    o = opts if opts is not None else P.Opts()
    jp = P.make_job(lenses, w.kappa_c, w.gamma, w.grid_lo, w.grid_hi, grid_n, map_lo, map_hi, map_n, cp, lp,
                    window=window, jitter_seed=jitter_seed)
    jz = P.make_job(lenses, w.kappa_c, w.gamma, w.grid_lo, w.grid_hi, grid_n, map_lo, map_hi, map_n, cz, lz,
                    window=window, jitter_seed=jitter_seed)
    z = zoom if zoom is not None else P.zoom_params()
    ws = torch.empty(P.workspace_bytes(jp, o), dtype=torch.uint8, device=dev)
    P.shoot_job(jp, ws, o)
    wz = torch.empty(P.zoom_workspace_bytes(jz, z, o), dtype=torch.uint8, device=dev)
    P.shoot_zoom(jz, z, wz, o)
    st = P.zoom_stats(wz)
    torch.cuda.synchronize()
    return (cp.cpu().numpy().view(np.uint32), cz.cpu().numpy().view(np.uint32), st)


def test_zoom_equals_fine_grid_small_field():
    # 100 unit lenses; the 1000^2 grid refined 3x; a 3 x 3 window near the centre at 150^2
    w = synth.workload_small()
    cp, cz, st = _run(w, _fine(w, 3), (-2.0, 0.5), (1.0, 3.5), (150, 150))
    print("small field zoom:", st, "counts", int(cp.sum()))
    assert cp.sum() > 0 and np.array_equal(cp, cz)
    assert st["slots_shot"] < 0.5 * st["slots"] and st["cells_kept"] < st["cells"]


def test_zoom_against_oracle_fine_map():
    w = synth.workload_small()
    fine = _fine(w, 3)
    mlo, mhi, mn = (-2.0, 0.5), (1.0, 3.5), (150, 150)
    _, cz, _ = _run(w, fine, mlo, mhi, mn)
    wf = synth.Workload(w.name + "-fine", w.lenses, w.kappa_c, w.gamma, w.grid_lo, w.grid_hi, fine, mlo, mhi, mn,
                        kappa_star=w.kappa_star, lens_radius=w.lens_radius)
    co, _ = oracle.shoot_parallel(wf, threads=16)
    l1 = int(np.abs(cz.astype(np.int64) - co.astype(np.int64)).sum())
    print(f"zoom vs oracle fine map: L1 {l1} over {int(co.sum())} rays in the window")
    assert l1 <= 2 * 1e-5 * fine[0] * fine[1] + 2


@pytest.mark.parametrize("block,jitter", [((1, 4), None), ((2, 4), None), ((1, 4), 17)])
def test_zoom_equals_fine_grid_paper_field(block, jitter):
    # 1e5 power-law lenses, kappa_* = gamma = 0.45: the paper workload's field and shooting
    # region, rays 2x denser (8192^2), zoomed into a 2.5 x 2.5 window at 256^2
    torch, P = _env()
    w = synth.workload_paper(grid=8192)
    o = P.Opts()
    o.block_cols, o.block_rows = block
    cp, cz, st = _run(w, w.grid_n, (-1.25, -1.25), (1.25, 1.25), (256, 256), opts=o, jitter_seed=jitter)
    print("paper field zoom:", block, jitter, st, "counts", int(cp.sum()))
    assert cp.sum() > 0 and np.array_equal(cp, cz)
    assert st["cells_kept"] < 0.06 * st["cells"] and st["slots_shot"] < 0.06 * st["slots"]


def test_zoom_equals_fine_grid_bench_configuration():
    # the configuration the benchmark times: the paper workload's field and shooting region at 4x
    # the ray density per axis (16384^2 fine rays), a 2.5 x 2.5 window at 256^2, automatic cells
    w = synth.workload_paper()
    fine = (4 * w.grid_n[0], 4 * w.grid_n[1])
    cp, cz, st = _run(w, fine, (-1.25, -1.25), (1.25, 1.25), (256, 256))
    print("bench zoom configuration:", st, "counts", int(cp.sum()))
    assert cp.sum() > 0 and np.array_equal(cp, cz)
    assert st["slots_shot"] < 0.05 * st["slots"]


@pytest.mark.parametrize("block,jitter,cell", [((2, 4), None, (5, 7)), ((1, 4), 29, (0, 0)), ((4, 2), 3, (3, 9))])
def test_zoom_odd_window_blocks_and_jitter(block, jitter, cell):
    # a window starting on an odd row and column, several lane shapes, jittered rays and odd cell
    # sizes: the zoom still adds exactly the plain shoot's counts (rows sharing a reciprocal stay aligned)
    torch, P = _env()
    w = synth.workload_paper(n_lens=20000, grid=4096)
    o = P.Opts()
    o.block_cols, o.block_rows = block
    win = ((1001, 777), (1999, 2501))
    cp, cz, st = _run(w, w.grid_n, (0.5, -3.0), (3.0, -0.5), (200, 200), window=win, opts=o,
                      jitter_seed=jitter, zoom=P.zoom_params(cell))
    assert cp.sum() > 0 and np.array_equal(cp, cz), (block, jitter, cell)
    assert st["slots_shot"] < st["slots"]


def test_zoom_window_cells_and_margin():
    # a ray window that is not a multiple of the tile or cell sizes, explicit cells and a margin
    torch, P = _env()
    w = synth.workload_paper(n_lens=20000, grid=4096)
    win = ((1000, 333), (2500, 3001))
    for cell, margin in (((7, 13), 0.0), ((1, 1), 0.05), ((64, 64), 0.0)):
        cp, cz, st = _run(w, w.grid_n, (0.5, -3.0), (3.0, -0.5), (200, 200), window=win,
                          zoom=P.zoom_params(cell, margin))
        assert np.array_equal(cp, cz), (cell, margin)
        assert st["cells"] == -(-2500 // cell[0]) * -(-3001 // cell[1]) and st["slots_shot"] < st["slots"]


def test_zoom_far_from_every_ray_and_empty_window():
    torch, P = _env()
    w = synth.workload_small()
    cp, cz, st = _run(w, w.grid_n, (500.0, 500.0), (501.0, 501.0), (10, 10))
    assert cp.sum() == 0 and cz.sum() == 0
    assert st["slots_shot"] <= st["slots"] // 4
    cp, cz, st = _run(w, w.grid_n, (-1.0, -1.0), (1.0, 1.0), (10, 10), window=((5, 5), (0, 7)))
    assert cz.sum() == 0 and st["slots_shot"] == 0
