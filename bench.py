#!/usr/bin/env python3
"""Benchmark of direct inverse ray-shooting on one MI355X.

A step is one pass of the whole hot path over one synthetic map: the ray grid
is generated on the device, every ray is deflected by direct summation over all
lenses, mapped through the lens equation and binned (rs_shoot).  Inputs are
resident in HBM before the timed region starts.

Prints one JSON line.  The flop convention is the paper's: 10 flop per
ray-lens interaction (Thompson et al. 2009, appendix A).
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "ray·lens interactions/s & Gflop/s; rays/s surrogate vs direct at ≤1% map err"
FLOP_PER_INTERACTION = 10
PEAK_FP32_TFLOPS = 157.3          # MI355X published FP32 vector peak (packed FMA)
PEAK_HBM_GBS = 8000.0


def parse():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="paper", choices=["paper", "small", "batched", "farfield", "large"])
    ap.add_argument("--ff-steps", type=int, default=2000, help="surrogate workloads: Adam steps per tile")
    ap.add_argument("--ff-tile", type=int, default=0,
                    help="surrogate workloads: rays per tile side (default 64, large 1024)")
    ap.add_argument("--ff-samples", type=int, default=0,
                    help="surrogate workloads: fit samples per tile (multiple of 1024; default 4096, large 1024)")
    ap.add_argument("--autotune-cache", default="", help="batched workload: autotuner cache file")
    ap.add_argument("--block", default="", help="rays per lane as COLSxROWS, e.g. 2x4 (default: library's)")
    ap.add_argument("--lens-tile", type=int, default=0)
    ap.add_argument("--fp32-run", type=int, default=0)
    ap.add_argument("--map-window", type=int, default=0)
    ap.add_argument("--jitter-seed", type=int, default=None,
                    help="one seeded random ray per cell (Monte Carlo placement) instead of cell centres")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--plain-only", action="store_true",
                    help="default workload: skip the light-curve, batched and learned far-field measurements")
    ap.add_argument("--legs", default="light_curves,zoom,frames,batched,farfield,large",
                    help="default workload: comma-separated extra measurements to run after the plain one")
    ap.add_argument("--cpu-rays", type=int, default=1 << 22,
                    help="rays of the CPU oracle sample (timed baseline and counted parity)")
    ap.add_argument("--microbench", action="store_true",
                    help="only run the issue-rate probes and print the direct sum's instruction-mix ceiling")
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="MIB",
                    help="only run 3 plain device-to-device copies of MIB MiB (HBM counter calibration)")
    return ap.parse_args()


def calibrate_copy(mib: int):
    """Plain copies of a known size, so HBM byte counters can be scaled against them."""
    import torch
    n = mib * (1 << 20) // 4
    src = torch.ones(n, dtype=torch.float32, device="cuda:0")
    dst = torch.empty_like(src)
    for _ in range(3):
        dst.copy_(src)
    torch.cuda.synchronize()
    print(json.dumps({"calibrate_copy_mib": mib, "bytes_read_per_copy": n * 4, "bytes_written_per_copy": n * 4}))


def measured_traffic(workload_name: str, opts) -> float | None:
    """HBM bytes per k_direct launch from the committed rocprofv3 counter passes, or None when the
    kernel source or the launch shape differs from the one the counters were taken on."""
    import hashlib
    path = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(path):
        return None
    rec = json.load(open(path)).get("k_direct")
    if not rec:
        return None
    src = open(os.path.join(ROOT, rec["source"]), "rb").read()
    if hashlib.sha256(src).hexdigest() != rec["source_sha256"] or rec["workload"] != workload_name:
        return None
    cols, rows = (opts.block_cols or 1), (opts.block_rows or 4)
    if f"{cols}x{rows}" != rec["block"] or (opts.fp32_run or (8 if cols == 1 else 16)) != rec["fp32_run"] \
            or (opts.lens_tile or 256) != rec["lens_tile"]:
        return None
    return float(rec["hbm_bytes_per_launch"])


PROBES = {"fmac_f32": 0, "fma_f32": 1, "mul_f32": 2, "rcp_f32": 3, "mix_13fmac_1rcp": 4, "add_f64": 5}


def issue_rates(P):
    """Lane instructions per second of each issue-rate probe (rs_probe_issue_rate)."""
    import ctypes
    import torch
    L = P.lib()
    out = {}
    stream = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    for name, op in PROBES.items():
        r, sec = ctypes.c_double(), ctypes.c_double()
        P._check(L.rs_probe_issue_rate(op, ctypes.byref(r), ctypes.byref(sec), stream))
        out[name] = r.value
    return out


def mix_ceiling(rates: dict, opts) -> dict | None:
    """Instruction-mix ceiling of the direct sum's lens loop: the loop's instructions per interaction
    (counted in this build's gfx950 assembly, profiles/k_direct_isa_mix.json, valid while direct.hip
    is unchanged) priced at the probe rates.  A reciprocal costs what it adds to a 13 : 1 mix of
    v_fmac_f32 and v_rcp_f32 (the lens loop's own proportion), 14 / R_mix - 13 / R_fmac."""
    import hashlib
    path = os.path.join(ROOT, "profiles", "k_direct_isa_mix.json")
    if not os.path.exists(path):
        return None
    rec = json.load(open(path))
    src = open(os.path.join(ROOT, rec["source"]), "rb").read()
    cols, rows = (opts.block_cols or 1), (opts.block_rows or 4)
    if hashlib.sha256(src).hexdigest() != rec["source_sha256"] or f"{cols}x{rows}" != rec["block"] \
            or (opts.fp32_run or (8 if cols == 1 else 16)) != rec["fp32_run"] \
            or (opts.lens_tile or 256) != rec["lens_tile"]:
        return None
    k = rec["per_interaction"]
    rcp_cost = 14.0 / rates["mix_13fmac_1rcp"] - 13.0 / rates["fmac_f32"]
    t = (k["vop2_f32"] / rates["fmac_f32"] + k["vop3_f32"] / rates["fma_f32"] + k["rcp_f32"] * rcp_cost
         + (k["cvt_f64"] + k["add_f64"]) / rates["add_f64"])
    return {"interactions_per_s": 1.0 / t, "tflops_10flop": FLOP_PER_INTERACTION / t / 1e12,
            "per_interaction": {n: k[n] for n in ("vop2_f32", "vop3_f32", "rcp_f32", "cvt_f64", "add_f64")},
            "rcp_cost_in_fmac_slots": rcp_cost * rates["fmac_f32"],
            "isa_source": "profiles/k_direct_isa_mix.json"}


def workload(name):
    import synth
    if name == "small":
        return synth.workload_small()
    return synth.workload_paper()


def cpu_baseline(w, n_rays: int, gpu_pix=None, gpu_y=None):
    """The FP64 oracle on a bounded sample of the same workload (n_rays rays drawn with the counter
    hash: by default the 2^22 of the paper-scale parity test, about 30 s on 16 host threads), timed
    on the host threads; with the GPU's per-ray pixels of the whole grid (gpu_pix) the same sample
    gives the counted pixel-switch fraction of the benchmark's own launch, and with its per-ray
    source positions (gpu_y) the expected fraction: a ray whose position is off by (d1, d2) changes
    pixel with probability d1 / pixel1 + d2 / pixel2 when sources are spread evenly over a pixel, so
    the mean of that over the sample estimates the fraction without the counting noise."""
    import math
    import oracle
    import synth
    threads = max(1, min(16, os.cpu_count() or 1))
    idx = synth.sample_indices(12, w.n_rays, max(1, min(w.n_rays, n_rays)))
    t0 = time.perf_counter()
    y_o, p_o = oracle.trace_parallel(w, idx, threads=threads)
    dt = time.perf_counter() - t0
    inter = len(idx) * w.n_lens
    base = {"value": inter / dt, "unit": "interactions/s", "cores": threads, "kind": "oracle",
            "sample": f"{len(idx)} rays drawn by counter hash from the {w.name} grid x all {w.n_lens} lenses, "
                      f"FP64 single-threaded oracle on {threads} threads, {dt:.1f} s wall"}
    parity = None
    if gpu_pix is not None:
        g = gpu_pix[idx].astype(np.int64)
        diff = int(np.sum(g != p_o))
        inmap = int(np.sum((g >= 0) | (p_o >= 0)))
        # a true fraction of at most 1e-5 gives a Poisson count of mean <= 1e-5 n: 3 sigma allowed
        parity = {"rays_checked": int(len(idx)), "rays_in_map": inmap, "rays_switched": diff,
                  "switch_fraction": diff / max(1, inmap), "bar": 1e-5,
                  "switches_allowed": 1e-5 * inmap + 3.0 * math.sqrt(1e-5 * inmap),
                  "reference": "FP64 oracle, same rays, pixel or lost outcome per ray"}
        if gpu_y is not None:
            ok = np.isfinite(y_o).all(1) & (p_o >= 0)
            d = np.abs(gpu_y[idx][ok] - y_o[ok])
            px = [(w.map_hi[k] - w.map_lo[k]) / w.map_n[k] for k in (0, 1)]
            parity["switch_fraction_expected"] = float(np.mean(d[:, 0] / px[0] + d[:, 1] / px[1]))
    return base, parity


def _time_batch(P, torch, wl, steps, warmup, cache=None):
    """Autotune, then time one batched launch of the workloads `wl` and the same maps as separate
    rs_shoot launches; returns (batched_ms, separate_ms, wall_s, opts, tune_s, interactions, rays)."""
    dev = torch.device("cuda:0")
    dj = []
    for w in wl:
        lenses = torch.from_numpy(w.lenses).to(dev)
        counts = torch.zeros((w.map_n[1], w.map_n[0]), dtype=torch.int32, device=dev)
        lost = torch.zeros(1, dtype=torch.int64, device=dev)
        dj.append((P.make_job(lenses, w.kappa_c, w.gamma, w.grid_lo, w.grid_hi, w.grid_n, w.map_lo, w.map_hi,
                              w.map_n, counts, lost), lenses, counts, lost))
    jobs = [d[0] for d in dj]
    ws = torch.empty(P.batched_workspace_bytes(jobs), dtype=torch.uint8, device=dev)
    stream = torch.cuda.Stream()
    t0 = time.perf_counter()
    with torch.cuda.stream(stream):
        opts = P.autotune_batched(jobs, ws, cache_path=cache, stream=stream)
    tune_s = time.perf_counter() - t0
    inter = float(sum(w.n_rays * w.n_lens for w in wl))
    rays = float(sum(w.n_rays for w in wl))

    def zero():
        for d in dj:
            d[2].zero_()
            d[3].zero_()

    with torch.cuda.stream(stream):
        for _ in range(max(1, warmup)):
            P.shoot_batched(jobs, ws, opts, stream=stream)
        stream.synchronize()
        zero()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        stream.synchronize()
        t0 = time.perf_counter()
        e0.record(stream)
        for _ in range(steps):
            P.shoot_batched(jobs, ws, opts, stream=stream)
        e1.record(stream)
        stream.synchronize()
        wall = time.perf_counter() - t0
        batched_ms = e0.elapsed_time(e1) / steps
        total = sum(int(d[2].sum().item()) + int(d[3].item()) for d in dj)
        if total != int(rays) * steps:
            print("bench.py: ray conservation failed in the batch", file=sys.stderr)
            sys.exit(3)
        # the same maps as separate plain launches (default rs_shoot tuning)
        wss = [torch.empty(P.workspace_bytes(d[0]), dtype=torch.uint8, device=dev) for d in dj]
        for d, w in zip(dj, wss):
            P.shoot_job(d[0], w, None, stream)
        stream.synchronize()
        e0.record(stream)
        for _ in range(steps):
            for d, w in zip(dj, wss):
                P.shoot_job(d[0], w, None, stream)
        e1.record(stream)
        stream.synchronize()
        separate_ms = e0.elapsed_time(e1) / steps
    return batched_ms, separate_ms, wall, opts, tune_s, inter, rays


def bench_batched(args, emit=True):
    """64 maps in one persistent, graph-replayed launch vs 64 separate rs_shoot launches; also 256
    small maps (grids 128^2-512^2), where separate launches are dominated by launch overhead."""
    import torch
    import paper_0905_2453_amd as P
    import synth
    wl = synth.batched_jobs()
    batched_ms, separate_ms, wall, opts, tune_s, inter, rays = _time_batch(
        P, torch, wl, args.steps, args.warmup, args.autotune_cache or None)
    small = synth.batched_jobs(seed=5, n_jobs=256, scale=8)
    s_b, s_s, _, s_opts, _, s_inter, s_rays = _time_batch(P, torch, small, args.steps, args.warmup)
    value = inter * args.steps / wall
    out = {
        "metric": METRIC, "value": value, "unit": "interactions/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": 1e3 * wall / args.steps, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": "batched-64maps", "n_maps": len(wl), "interactions": inter, "rays": rays,
                   "parallelism": "1 GPU"},
        "gflops": value * FLOP_PER_INTERACTION / 1e9,
        "batched_ms": batched_ms, "separate_launches_ms": separate_ms, "speedup_vs_separate": separate_ms / batched_ms,
        "autotuned": {"block": f"{opts.block_cols}x{opts.block_rows}", "map_window": opts.map_window,
                      "lens_tile": opts.lens_tile, "tune_seconds": tune_s},
        "small_maps": {"n_maps": len(small), "interactions": s_inter, "rays": s_rays,
                       "grids": "128^2-512^2", "lenses": "125-12500", "batched_ms": s_b, "separate_launches_ms": s_s,
                       "speedup_vs_separate": s_s / s_b, "interactions_per_s": s_inter / (s_b * 1e-3),
                       "autotuned_block": f"{s_opts.block_cols}x{s_opts.block_rows}"},
        "roofline": {"bound": "alu", "achieved": FLOP_PER_INTERACTION * inter / (batched_ms * 1e-3) / 1e12,
                     "peak": PEAK_FP32_TFLOPS, "unit": "TFLOP/s",
                     "frac": FLOP_PER_INTERACTION * inter / (batched_ms * 1e-3) / 1e12 / PEAK_FP32_TFLOPS,
                     "traffic": None, "kernel": "k_batched"},
    }
    if emit:
        print(json.dumps(out), flush=True)
    return out


def rebinned_p99(cs, cp, k=4):
    """99th percentile of |N_s - N_p| / N_p over the pixels of k x k-rebinned maps with N_p > 0."""
    h, w_ = (cs.shape[0] // k) * k, (cs.shape[1] // k) * k
    rs = cs[:h, :w_].reshape(h // k, k, w_ // k, k).sum((1, 3))
    rp = cp[:h, :w_].reshape(h // k, k, w_ // k, k).sum((1, 3))
    m = rp > 0
    return float(np.percentile(np.abs(rs[m] - rp[m]) / rp[m], 99)) if m.any() else 0.0


def bench_surrogate(args, which=None, emit=True):
    """Learned far-field closure vs the plain direct sum on the same rays.

    farfield: 1e6 lenses, 8192^2 rays in 64x64-ray tiles; the plain sum judges the whole map.
    large:    1e7 lenses, 32768^2 rays in 1024x1024-ray tiles; the closure shoots the whole grid,
              the plain sum judges a seeded 1% of the tiles (both paths shoot those tiles).
    """
    import torch
    import paper_0905_2453_amd as P
    import synth
    dev = torch.device("cuda:0")
    large = (which or args.workload) == "large"
    w = synth.workload_large() if large else synth.workload_farfield()
    # 64^2-ray tiles on the 1e6-lens field (its configuration); 1024^2 on the 1e7-lens one, where
    # the fit (samples x tiles x lenses) dominates: map error 0.37% at 1024^2 (0.14% at 512^2, 0.75%
    # at 2048^2) for an end-to-end gain of about 700x (210x, 1250x)
    tile = (args.ff_tile, args.ff_tile) if args.ff_tile else ((1024, 1024) if large else (64, 64))
    lenses = torch.from_numpy(w.lenses).to(dev)
    counts = torch.zeros((w.map_n[1], w.map_n[0]), dtype=torch.int32, device=dev)
    lost = torch.zeros(1, dtype=torch.int64, device=dev)
    job = P.make_job(lenses, w.kappa_c, w.gamma, w.grid_lo, w.grid_hi, w.grid_n, w.map_lo, w.map_hi, w.map_n,
                     counts, lost)
    # seeded uniform fit samples per tile, in quads that share their first coordinate (the fit shares
    # x-differences within a quad; the targets are those of the same points listed freely): 4096 on the
    # 1e6-lens field, whose configuration fixes that number; 1024 on the 1e7-lens field, where the exact
    # samples are most of the cost (4096 there: map error 0.11%, end-to-end 63x; 1024: 0.14%, 210x)
    n_samples = args.ff_samples or (1024 if large else 4096)
    samples = torch.from_numpy(synth.fit_samples_quads(7, n_samples)).to(dev)
    init = torch.from_numpy(synth.init_params(7)).to(dev)
    cfg = P.ff_config(samples, init, tile_rays=tile, r_near=8.0, steps=args.ff_steps, batch=512, lr=1e-2,
                      shared_x=True)
    model = torch.empty(P.farfield_model_bytes(job, cfg), dtype=torch.uint8, device=dev)
    fws = torch.empty(P.farfield_fit_workspace_bytes(job, cfg), dtype=torch.uint8, device=dev)
    ews = torch.empty(P.farfield_eval_workspace_bytes(job, cfg), dtype=torch.uint8, device=dev)
    stream = torch.cuda.current_stream()
    ev = lambda: torch.cuda.Event(enable_timing=True)

    def timed(fn):
        a, b = ev(), ev()
        torch.cuda.synchronize()
        a.record(stream)
        fn()
        b.record(stream)
        torch.cuda.synchronize()
        return a.elapsed_time(b) * 1e-3

    fit_s = timed(lambda: P.farfield_fit(job, cfg, model, fws))
    ntx = (w.grid_n[0] + tile[0] - 1) // tile[0]
    nty = (w.grid_n[1] + tile[1] - 1) // tile[1]
    n_tiles = ntx * nty
    if large:
        judge = np.sort(synth.sample_indices(11, n_tiles, max(1, n_tiles // 100))).astype(np.int32)
    else:
        judge = np.arange(n_tiles, dtype=np.int32)
    judge_t = torch.from_numpy(judge).to(dev)
    # surrogate over the whole grid (warm once, then timed)
    P.farfield_eval(job, cfg, model, ews)
    counts.zero_()
    lost.zero_()
    eval_s = timed(lambda: P.farfield_eval(job, cfg, model, ews))
    if int(counts.sum().item()) + int(lost.item()) != w.n_rays:
        print("bench.py: surrogate ray conservation failed", file=sys.stderr)
        sys.exit(3)
    # the judged tiles: surrogate, affine-only ablation, plain direct sum
    sub_cfg = P.ff_config(samples, init, tile_rays=tile, r_near=8.0, steps=args.ff_steps, batch=512, lr=1e-2,
                          eval_tiles=judge_t, shared_x=True)

    def surrogate_map(flags):
        counts.zero_()
        lost.zero_()
        o = P.Opts()
        o.flags = flags
        P.farfield_eval(job, sub_cfg if large else cfg, model, ews, o)
        torch.cuda.synchronize()
        return counts.cpu().numpy().view(np.uint32).astype(np.int64)

    m_sur = surrogate_map(0)
    m_aff = surrogate_map(P._abi.RS_FLAG_AFFINE_ONLY)
    counts.zero_()
    lost.zero_()
    pws = torch.empty(P.workspace_bytes(job), dtype=torch.uint8, device=dev)
    judge_rays = 0
    plain_jobs = []
    for t in judge:
        tx, ty = int(t) % ntx, int(t) // ntx
        a = (tx * tile[0], ty * tile[1])
        n = (min(tile[0], w.grid_n[0] - a[0]), min(tile[1], w.grid_n[1] - a[1]))
        judge_rays += n[0] * n[1]
        plain_jobs.append(P.make_job(lenses, w.kappa_c, w.gamma, w.grid_lo, w.grid_hi, w.grid_n, w.map_lo,
                                     w.map_hi, w.map_n, counts, lost, window=(a, n)))

    bws = torch.empty(P.batched_workspace_bytes(plain_jobs), dtype=torch.uint8, device=dev) if large else None

    def plain():
        if large:   # the judged tiles as one persistent batched launch (full occupancy)
            P.shoot_batched(plain_jobs, bws, None, stream)
        else:
            P.shoot_job(job, pws, None, stream)

    plain_s = timed(plain)
    m_pl = counts.cpu().numpy().view(np.uint32).astype(np.int64)
    moving = None
    if not large:
        # the same closure reused across frames of a moving field (velocity dispersion 0.05 per
        # axis): each frame refreshes the far set's affine base and moves the near lenses; the
        # last frame is judged by the plain direct sum of the moved field
        vel = torch.from_numpy(synth.lens_velocities(24, w.n_lens, 0.05)).to(dev)
        frame_s, times = [], [1.0, 2.0, 4.0]
        for t_f in times:
            mj = P.make_job(lenses, w.kappa_c, w.gamma, w.grid_lo, w.grid_hi, w.grid_n, w.map_lo, w.map_hi,
                            w.map_n, counts, lost, velocities=vel, time=t_f)
            counts.zero_()
            lost.zero_()
            frame_s.append(timed(lambda: P.farfield_eval(mj, cfg, model, ews)))
        m_mov = counts.cpu().numpy().view(np.uint32).astype(np.int64)
        counts.zero_()
        lost.zero_()
        mov_plain_s = timed(lambda: P.shoot_job(mj, pws, None, stream))
        m_mpl = counts.cpu().numpy().view(np.uint32).astype(np.int64)
        moving = {"sigma_v": 0.05, "times": times, "frame_s": frame_s,
                  "plain_frame_s": mov_plain_s, "speedup_vs_plain_per_frame": mov_plain_s / float(np.mean(frame_s)),
                  "map_l1_rel_err_last_frame": float(np.abs(m_mov - m_mpl).sum() / max(1, m_mpl.sum())),
                  "frozen_closure_l1_last_frame": float(np.abs(m_sur - m_mpl).sum() / max(1, m_mpl.sum()))}
    l1 = float(np.abs(m_sur - m_pl).sum() / max(1, m_pl.sum()))
    l1_aff = float(np.abs(m_aff - m_pl).sum() / max(1, m_pl.sum()))
    shape = (w.map_n[1], w.map_n[0])
    p99 = rebinned_p99(m_sur.reshape(shape), m_pl.reshape(shape))
    p99_aff = rebinned_p99(m_aff.reshape(shape), m_pl.reshape(shape))
    plain_rays_s = judge_rays / plain_s
    sur_rays_s = w.n_rays / eval_s
    e2e_rays_s = w.n_rays / (fit_s + eval_s)
    out = {
        "metric": METRIC, "value": sur_rays_s, "unit": "rays/s", "n_gpus": 1, "steps": 1, "warmup": 1,
        "ms_per_step": 1e3 * (fit_s + eval_s), "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32+bf16", "data": "synthetic",
        "config": {"workload": w.name, "n_lens": w.n_lens, "ray_grid": list(w.grid_n), "map": list(w.map_n),
                   "tile_rays": list(tile), "r_near": 8.0, "fit_samples": f"{n_samples} seeded uniform, quads sharing x", "adam_steps": args.ff_steps,
                   "judged_tiles": int(len(judge)), "n_tiles": int(n_tiles), "parallelism": "1 GPU"},
        "fit_s": fit_s, "eval_s": eval_s, "plain_s_on_judged_tiles": plain_s,
        "rays_per_s": {"surrogate_eval": sur_rays_s, "surrogate_end_to_end": e2e_rays_s, "plain": plain_rays_s},
        "speedup_vs_plain": {"eval_only": sur_rays_s / plain_rays_s, "end_to_end": e2e_rays_s / plain_rays_s},
        # rays per tile at which shooting a tile plainly costs as much as fitting its closure
        "break_even_rays_per_tile": fit_s * plain_rays_s / n_tiles,
        "map_l1_rel_err": {"surrogate": l1, "affine_only": l1_aff, "tolerance": 0.01},
        # per-pixel side of the tolerance: 99th percentile of |N_s - N_p| / N_p over the pixels of
        # 4 x 4-rebinned maps that the plain sum reaches
        "p99_pixel_rel_err_4x4": {"surrogate": p99, "affine_only": p99_aff},
    }
    if moving is not None:
        out["moving_frames"] = moving
    if l1 > 0.01:
        print(f"bench.py: surrogate map error {l1:.3e} above the 1% tolerance", file=sys.stderr)
        sys.exit(3)
    if emit:
        print(json.dumps(out), flush=True)
    return out


LC_TRACKS, LC_POINTS, LC_SIGMA, LC_LENGTH = 1024, 1024, 0.05, 10.0


def bench_light_curves(P, torch, counts, w, n_av, stream, reps=5):
    """Light curves off the map just shot: LC_TRACKS seeded straight tracks of LC_LENGTH Einstein
    radii, LC_POINTS points each, Gaussian source of width LC_SIGMA (support 4 sigma)."""
    import synth
    dev = counts.device
    tr = torch.from_numpy(synth.light_tracks(27, LC_TRACKS, w.map_lo, w.map_hi, LC_LENGTH)).to(dev)
    mu, _ = P.light_curve(counts, w.map_lo, w.map_hi, w.map_n, n_av, tr, LC_POINTS, "gaussian", LC_SIGMA,
                          stream=stream)
    torch.cuda.synchronize()
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(reps)]
    for a, b in ev:
        a.record(stream)
        P.light_curve(counts, w.map_lo, w.map_hi, w.map_n, n_av, tr, LC_POINTS, "gaussian", LC_SIGMA,
                      stream=stream)
        b.record(stream)
    torch.cuda.synchronize()
    ms = float(np.mean([a.elapsed_time(b) for a, b in ev]))
    pts = LC_TRACKS * LC_POINTS
    pix = (w.map_hi[0] - w.map_lo[0]) / w.map_n[0]
    box = (2 * int(np.ceil(4 * LC_SIGMA / pix)) + 1) ** 2          # support bounding box, pixels
    m = mu.cpu().numpy()
    return {"kernel": "k_light_curve", "tracks": LC_TRACKS, "points_per_track": LC_POINTS,
            "source": f"gaussian sigma {LC_SIGMA} (support 4 sigma)", "track_length": LC_LENGTH,
            "kernel_ms": ms, "points_per_s": pts / (ms * 1e-3), "box_pixels_per_s": pts * box / (ms * 1e-3),
            "mean_mu": float(np.nanmean(m))}


ZOOM_REFINE, ZOOM_LO, ZOOM_HI, ZOOM_N = 4, (-1.25, -1.25), (1.25, 1.25), (256, 256)


def bench_zoom(P, torch, w, lenses, stream):
    """Interactive zoom: the workload's field and shooting region at ZOOM_REFINE x the ray density
    per axis, a 2.5 x 2.5 Einstein-radius window at 256^2; zoom vs the full fine-grid shoot, whose
    counts it must equal exactly."""
    dev = lenses.device
    fine = (w.grid_n[0] * ZOOM_REFINE, w.grid_n[1] * ZOOM_REFINE)
    cp = torch.zeros((ZOOM_N[1], ZOOM_N[0]), dtype=torch.int32, device=dev)
    cz = torch.zeros_like(cp)
    lp = torch.zeros(1, dtype=torch.int64, device=dev)
    lz = torch.zeros_like(lp)
    jp = P.make_job(lenses, w.kappa_c, w.gamma, w.grid_lo, w.grid_hi, fine, ZOOM_LO, ZOOM_HI, ZOOM_N, cp, lp)
    jz = P.make_job(lenses, w.kappa_c, w.gamma, w.grid_lo, w.grid_hi, fine, ZOOM_LO, ZOOM_HI, ZOOM_N, cz, lz)
    zp = P.zoom_params()
    ws = torch.empty(max(P.workspace_bytes(jp), P.zoom_workspace_bytes(jz, zp)), dtype=torch.uint8, device=dev)

    def timed(fn):
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record(stream)
        fn()
        b.record(stream)
        torch.cuda.synchronize()
        return a.elapsed_time(b) * 1e-3

    P.shoot_zoom(jz, zp, ws, stream=stream)            # warm-up (also checks the arguments)
    torch.cuda.synchronize()
    cz.zero_()
    lz.zero_()
    t_zoom = timed(lambda: P.shoot_zoom(jz, zp, ws, stream=stream))
    st = P.zoom_stats(ws, stream)
    t_full = timed(lambda: P.shoot_job(jp, ws, None, stream))
    exact = bool(torch.equal(cp, cz))
    rays = fine[0] * fine[1]
    return {"config": {"field": w.name, "fine_ray_grid": list(fine), "window": [list(ZOOM_LO), list(ZOOM_HI)],
                       "map": list(ZOOM_N), "cell": "auto (~64 rays, square), 5 culling levels halving the cell side"},
            "zoom_s": t_zoom, "full_fine_s": t_full, "speedup_vs_full": t_full / t_zoom,
            "ray_slots_shot_frac": st["slots_shot"] / max(1, st["slots"]),
            "cells_kept_frac": st["cells_kept"] / max(1, st["cells"]),
            "equal_to_full": exact, "effective_rays_per_s": rays / t_zoom}


N_FRAMES, FRAME_SIGMA_V = 8, 0.05


def bench_frames(P, torch, w, lenses, stream):
    """Time-evolving field: N_FRAMES maps of the workload at times 0, 1, ..., stars moving with
    a velocity dispersion of FRAME_SIGMA_V Einstein radii per unit time per axis, shot as one
    batch (lens motion applied while staging; nothing is materialised per frame)."""
    import synth
    dev = lenses.device
    vel = torch.from_numpy(synth.lens_velocities(13, w.n_lens, FRAME_SIGMA_V)).to(dev)
    maps = [torch.zeros((w.map_n[1], w.map_n[0]), dtype=torch.int32, device=dev) for _ in range(N_FRAMES)]
    losts = [torch.zeros(1, dtype=torch.int64, device=dev) for _ in range(N_FRAMES)]
    jobs = [P.make_job(lenses, w.kappa_c, w.gamma, w.grid_lo, w.grid_hi, w.grid_n, w.map_lo, w.map_hi, w.map_n,
                       maps[k], losts[k], velocities=vel, time=float(k)) for k in range(N_FRAMES)]
    ws = torch.empty(P.batched_workspace_bytes(jobs), dtype=torch.uint8, device=dev)
    P.shoot_batched(jobs, ws, stream=stream)       # warm-up: builds the graph
    torch.cuda.synchronize()
    for m in maps:
        m.zero_()
    for lo in losts:
        lo.zero_()
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record(stream)
    P.shoot_batched(jobs, ws, stream=stream)
    b.record(stream)
    torch.cuda.synchronize()
    sec = a.elapsed_time(b) * 1e-3
    total = sum(int(m.sum().item()) + int(lo.item()) for m, lo in zip(maps, losts))
    if total != N_FRAMES * w.n_rays:
        print("bench.py: frame batch lost rays", file=sys.stderr)
        sys.exit(3)
    return {"frames": N_FRAMES, "sigma_v": FRAME_SIGMA_V, "frame_times": [0, N_FRAMES - 1], "batch_s": sec,
            "frames_per_s": N_FRAMES / sec, "interactions_per_s": N_FRAMES * float(w.n_rays) * w.n_lens / sec}


def main():
    args = parse()
    if args.calibrate_copy:
        calibrate_copy(args.calibrate_copy)
        return
    if args.microbench:
        import torch
        import paper_0905_2453_amd as P
        torch.cuda.set_device(0)
        rates = issue_rates(P)
        print(json.dumps({"issue_rates_lane_ops_per_s": rates,
                          "mix_ceiling_1x4": mix_ceiling(rates, P.Opts())}), flush=True)
        return
    if args.gpus != 1:
        print(f"bench.py: runs on one GPU only (asked for --gpus {args.gpus}); "
              "multi-GPU sharding is described in the design notes but not implemented", file=sys.stderr)
        sys.exit(2)
    import torch
    import paper_0905_2453_amd as P

    if not torch.cuda.is_available():
        print("bench.py: no GPU visible", file=sys.stderr)
        sys.exit(1)
    if args.workload == "batched":
        bench_batched(args)
        return
    if args.workload in ("farfield", "large"):
        bench_surrogate(args)
        return
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    w = workload(args.workload)
    w.jitter_seed = args.jitter_seed
    lenses = torch.from_numpy(w.lenses).to(dev)
    counts = torch.zeros((w.map_n[1], w.map_n[0]), dtype=torch.int32, device=dev)
    lost = torch.zeros(1, dtype=torch.int64, device=dev)
    opts = P.Opts()
    if args.block:
        opts.block_cols, opts.block_rows = (int(v) for v in args.block.lower().split("x"))
    opts.lens_tile = args.lens_tile
    opts.fp32_run, opts.map_window = args.fp32_run, args.map_window
    job = P.make_job(lenses, w.kappa_c, w.gamma, w.grid_lo, w.grid_hi, w.grid_n, w.map_lo, w.map_hi, w.map_n,
                     counts, lost, jitter_seed=args.jitter_seed)
    ws = torch.empty(P.workspace_bytes(job, opts), dtype=torch.uint8, device=dev)
    stream = torch.cuda.current_stream()

    for _ in range(args.warmup):
        counts.zero_()
        lost.zero_()
        P.shoot_job(job, ws, opts, stream)
    torch.cuda.synchronize()
    counts.zero_()
    lost.zero_()

    starts = [torch.cuda.Event(enable_timing=True) for _ in range(args.steps)]
    ends = [torch.cuda.Event(enable_timing=True) for _ in range(args.steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(args.steps):
        starts[i].record(stream)
        P.shoot_job(job, ws, opts, stream)
        ends[i].record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    launch_ms = [s.elapsed_time(e) for s, e in zip(starts, ends)]
    ms_step = 1e3 * wall / args.steps
    inter = float(w.n_rays) * float(w.n_lens)
    value = inter * args.steps / wall
    kernel_s = float(np.mean(launch_ms)) * 1e-3
    achieved_tf = FLOP_PER_INTERACTION * inter / kernel_s / 1e12
    total = int(counts.sum().item()) + int(lost.item())
    if total != w.n_rays * args.steps:
        print(f"bench.py: ray conservation failed ({total} != {w.n_rays * args.steps})", file=sys.stderr)
        sys.exit(3)

    out = {
        "metric": METRIC,
        "value": value,
        "unit": "interactions/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": w.name, "n_lens": w.n_lens, "ray_grid": list(w.grid_n),
                   "map": list(w.map_n), "kappa_star": w.kappa_star, "kappa_c": w.kappa_c, "gamma": w.gamma,
                   "masses": "unit" if args.workload == "small" else "power law 2.35 on [0.1,1]",
                   "fp64_combine": True, "parallelism": "1 GPU",
                   "rays": "cell centres" if args.jitter_seed is None else f"jittered, seed {args.jitter_seed}"},
        "gflops": value * FLOP_PER_INTERACTION / 1e9,
        "rays_per_s": w.n_rays * args.steps / wall,
        "roofline": {"bound": "alu", "achieved": achieved_tf, "peak": PEAK_FP32_TFLOPS, "unit": "TFLOP/s",
                     "frac": achieved_tf / PEAK_FP32_TFLOPS, "traffic": measured_traffic(w.name, opts),
                     "kernel": "k_direct", "flop_per_interaction": FLOP_PER_INTERACTION,
                     "kernel_ms": kernel_s * 1e3},
    }
    # the measured instruction-mix ceiling of the lens loop (issue-rate probes x counted mix)
    rates = issue_rates(P)
    ceil = mix_ceiling(rates, opts)
    out["roofline"]["issue_rates_lane_ops_per_s"] = rates
    if ceil is not None:
        ceil["frac_achieved"] = (inter / kernel_s) / ceil["interactions_per_s"]
        out["roofline"]["mix_ceiling"] = ceil
    legs = [] if args.workload != "paper" or args.plain_only else args.legs.split(",")
    if "light_curves" in legs:
        print("bench.py: plain direct sum done; light curves next", file=sys.stderr, flush=True)
        # the map now holds `steps` passes of the ray grid, so N_av scales by the same factor
        nav = ((w.map_hi[0] - w.map_lo[0]) / w.map_n[0]) * ((w.map_hi[1] - w.map_lo[1]) / w.map_n[1]) / (
            ((w.grid_hi[0] - w.grid_lo[0]) / w.grid_n[0]) * ((w.grid_hi[1] - w.grid_lo[1]) / w.grid_n[1]))
        out["light_curves"] = bench_light_curves(P, torch, counts, w, nav * args.steps, stream)
    if "zoom" in legs:
        print("bench.py: interactive zoom next", file=sys.stderr, flush=True)
        out["zoom"] = bench_zoom(P, torch, w, lenses, stream)
        if not out["zoom"]["equal_to_full"]:
            print("bench.py: zoom map differs from the full fine-grid map", file=sys.stderr)
            sys.exit(3)
    if "frames" in legs:
        print("bench.py: time-evolving frames next", file=sys.stderr, flush=True)
        out["frames"] = bench_frames(P, torch, w, lenses, stream)
    if "batched" in legs:
        print("bench.py: batched maps next", file=sys.stderr, flush=True)
        b = bench_batched(argparse.Namespace(**{**vars(args), "steps": 2, "warmup": 1}), emit=False)
        out["batched"] = {k: b[k] for k in ("value", "batched_ms", "separate_launches_ms", "speedup_vs_separate",
                                            "autotuned", "config", "small_maps")}
    for which in ("farfield", "large"):
        if which in legs:
            print(f"bench.py: learned far field ({which}) next", file=sys.stderr, flush=True)
            r = bench_surrogate(args, which=which, emit=False)
            out[f"surrogate_{which}"] = {k: r[k] for k in ("config", "fit_s", "eval_s", "plain_s_on_judged_tiles",
                                                            "rays_per_s", "speedup_vs_plain",
                                                            "break_even_rays_per_tile", "map_l1_rel_err",
                                                            "p99_pixel_rel_err_4x4")}
            if "moving_frames" in r:
                out[f"surrogate_{which}"]["moving_frames"] = r["moving_frames"]
    if not args.no_cpu_baseline:
        print("bench.py: CPU oracle baseline and counted parity next", file=sys.stderr, flush=True)
        # one more launch of the timed configuration with per-ray dumps (the map is unchanged by them)
        rp = torch.empty(w.n_rays, dtype=torch.int32, device=dev)
        ry = torch.empty((w.n_rays, 2), dtype=torch.float64, device=dev)
        dopts = P.Opts.from_buffer_copy(opts)
        dopts.ray_y, dopts.ray_pix = ry.data_ptr(), rp.data_ptr()
        counts.zero_()
        lost.zero_()
        P.shoot_job(job, ws, dopts, stream)
        torch.cuda.synchronize()
        pix = rp.cpu().numpy()
        ray_y = ry.cpu().numpy()
        del ry, rp
        out["cpu_baseline"], out["parity"] = cpu_baseline(w, args.cpu_rays, pix, ray_y)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
