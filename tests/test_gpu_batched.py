"""GPU tests of the persistent batched launch (rs_shoot_batched) and its autotuner.

Each job of a batch is computed exactly as rs_shoot computes it (same block shape and float32
run length), so maps must be bit-identical to per-job rs_shoot calls; one job is also checked
against the FP64 oracle.  Graph replays are checked one by one against the eager result, with
eager work and synchronisation between replays.
"""
import os

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


def _batch(seed=3, scale=8):
    jobs = synth.batched_jobs(seed=seed, n_jobs=12, scale=scale)
    # edge cases: no lenses, an empty window, a ragged window
    jobs[0] = synth.Workload("nolens", np.zeros((0, 4), np.float32), 0.2, 0.1, (-9.0, -7.0), (9.0, 7.0),
                             (200, 150), (-5.0, -5.0), (5.0, 5.0), (64, 48))
    jobs[1].extra["window"] = ((5, 5), (0, 10))
    jobs[2].extra["window"] = ((3, 11), (jobs[2].grid_n[0] - 7, jobs[2].grid_n[1] - 19))
    jobs[3].jitter_seed = 1234          # one Monte Carlo (jittered) job in the batch
    jobs[2].jitter_seed = 77
    return jobs


def _jobs_on_device(torch, P, ws_list):
    dev = torch.device("cuda:0")
    out = []
    for w in ws_list:
        lenses = torch.from_numpy(np.ascontiguousarray(w.lenses)).to(dev)
        counts = torch.zeros((w.map_n[1], w.map_n[0]), dtype=torch.int32, device=dev)
        lost = torch.zeros(1, dtype=torch.int64, device=dev)
        j = P.make_job(lenses, w.kappa_c, w.gamma, w.grid_lo, w.grid_hi, w.grid_n, w.map_lo, w.map_hi,
                       w.map_n, counts, lost, window=w.extra.get("window"), jitter_seed=w.jitter_seed)
        out.append((j, lenses, counts, lost))
    return out


def _reference(torch, P, ws_list, opts):
    refs = []
    for j, lenses, counts, lost in _jobs_on_device(torch, P, ws_list):
        ws = torch.empty(P.workspace_bytes(j, opts), dtype=torch.uint8, device="cuda:0")
        P.shoot_job(j, ws, opts)
        torch.cuda.synchronize()
        refs.append((counts.cpu().numpy().copy(), int(lost.item())))
    return refs


@pytest.mark.parametrize("shape", [(1, 4), (2, 4), (4, 4)])
@pytest.mark.parametrize("graph", [False, True])
def test_batched_bit_identical_to_single_launches(shape, graph):
    torch, P = _env()
    wl = _batch()
    opts = P.Opts()
    opts.block_cols, opts.block_rows = shape
    if not graph:
        opts.flags = P._abi.RS_FLAG_NO_GRAPH
    refs = _reference(torch, P, wl, opts)
    dj = _jobs_on_device(torch, P, wl)
    jobs = [d[0] for d in dj]
    ws = torch.empty(P.batched_workspace_bytes(jobs), dtype=torch.uint8, device="cuda:0")
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        P.shoot_batched(jobs, ws, opts, stream=stream)
    stream.synchronize()
    for k, ((c_ref, l_ref), d) in enumerate(zip(refs, dj)):
        assert np.array_equal(d[2].cpu().numpy(), c_ref), k
        assert int(d[3].item()) == l_ref, k
    # conservation per job
    for w, d in zip(wl, dj):
        win = w.extra.get("window", ((0, 0), w.grid_n))
        assert int(d[2].sum().item()) + int(d[3].item()) == win[1][0] * win[1][1]


def test_graph_replays_match_eager_every_time():
    torch, P = _env()
    wl = _batch(seed=5)
    opts = P.Opts()
    eager = P.Opts()
    eager.flags = P._abi.RS_FLAG_NO_GRAPH
    dj = _jobs_on_device(torch, P, wl)
    jobs = [d[0] for d in dj]
    ws = torch.empty(P.batched_workspace_bytes(jobs), dtype=torch.uint8, device="cuda:0")
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        P.shoot_batched(jobs, ws, eager, stream=stream)
    stream.synchronize()
    ref = [(d[2].cpu().numpy().copy(), int(d[3].item())) for d in dj]
    for rep in range(4):
        with torch.cuda.stream(stream):
            for d in dj:            # the program's own eager work between replays
                d[2].zero_()
                d[3].zero_()
            P.shoot_batched(jobs, ws, opts, stream=stream)
        stream.synchronize()
        for k, (d, (c, l)) in enumerate(zip(dj, ref)):
            assert np.array_equal(d[2].cpu().numpy(), c), (rep, k)
            assert int(d[3].item()) == l, (rep, k)
        _ = torch.randn(1 << 20, device="cuda:0").sum().item()  # unrelated eager work + sync


def test_batched_job_against_oracle():
    torch, P = _env()
    wl = _batch(seed=7)
    dj = _jobs_on_device(torch, P, wl)
    jobs = [d[0] for d in dj]
    ws = torch.empty(P.batched_workspace_bytes(jobs), dtype=torch.uint8, device="cuda:0")
    P.shoot_batched(jobs, ws)
    torch.cuda.synchronize()
    k = max(range(3, len(wl)), key=lambda i: wl[i].n_lens * 0 + (wl[i].n_rays < 300000) * wl[i].n_lens)
    w = wl[k]
    co, lo_ = oracle.shoot_parallel(w, threads=16)
    got = dj[k][2].cpu().numpy().view(np.uint32)
    # each switched ray changes at most two bins by one
    diff = np.abs(got.astype(np.int64) - co.astype(np.int64)).sum()
    assert diff <= 2 * max(1, int(1e-5 * w.n_rays)), diff


def test_autotune_and_cache(tmp_path):
    torch, P = _env()
    wl = _batch(seed=9)
    dj = _jobs_on_device(torch, P, wl)
    jobs = [d[0] for d in dj]
    ws = torch.empty(P.batched_workspace_bytes(jobs), dtype=torch.uint8, device="cuda:0")
    cache = str(tmp_path / "tune.txt")
    best = P.autotune_batched(jobs, ws, cache_path=cache)
    assert (best.block_cols, best.block_rows) in [(1, 4), (2, 4), (4, 4), (2, 8)]
    assert best.map_window in (32, 64)
    # the autotuner never touches the jobs' maps
    for d in dj:
        assert int(d[2].sum().item()) == 0 and int(d[3].item()) == 0
    line = open(cache).read().split()
    assert line[1:3] == [str(best.block_cols), str(best.block_rows)]
    # a cached entry is used as is
    with open(cache, "w") as f:
        f.write(f"{line[0]} 2 8 256 32\n")
    again = P.autotune_batched(jobs, ws, cache_path=cache)
    assert (again.block_cols, again.block_rows, again.map_window) == (2, 8, 32)
    P.shoot_batched(jobs, ws, again)
    torch.cuda.synchronize()
    assert all(int(d[2].sum().item()) + int(d[3].item()) > 0 for d in dj[2:])
