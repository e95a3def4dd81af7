"""Python binding of librs: MI355X inverse ray-shooting (Thompson et al. 2009).

Argument marshalling only.  Every step of the computation runs in the HIP
kernels of ``librs.so`` behind the C ABI declared in ``include/rs.h``; torch
supplies device memory and streams.  If the library is missing the binding
raises -- there is no CPU fallback.
"""
from __future__ import annotations

import ctypes
import os

from . import _abi
from ._abi import RayShootError, Opts  # noqa: F401

PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(PKG, "librs.so")

_lib = None


def lib():
    """The loaded librs.so (raises RuntimeError when it has not been built).

    torch is imported first so that librs binds to the HIP runtime torch has loaded: the streams
    and device pointers it hands over belong to that runtime, and a second runtime loaded ahead
    of it would not see the device."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with paper_0905_2453_amd.build.build()")
        import torch  # noqa: F401
        _lib = _abi.bind(ctypes.CDLL(LIB_PATH))
    return _lib


def _torch():
    import torch
    return torch


def _check(st: int):
    if st != 0:
        L = lib()
        raise RayShootError(st, L.rs_status_str(st).decode(), L.rs_last_error().decode())


def _stream_handle(stream):
    torch = _torch()
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


def _require_cuda(t, name, dtype=None):
    torch = _torch()
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise ValueError(f"{name} must be a CUDA (HIP) tensor")
    if dtype is not None and t.dtype != dtype:
        raise ValueError(f"{name} must have dtype {dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")


def make_job(lenses, kappa_c, gamma, grid_lo, grid_hi, grid_n, map_lo, map_hi, map_n, counts, lost,
             window=None, jitter_seed=None, velocities=None, time=0.0) -> _abi.Job:
    """Fill an rs_job from device tensors and plain numbers (no copies).

    velocities: optional device float32 (n_lens, 2) tensor; the job then shoots the field at
    `time` (lens i at x_i + v_i time)."""
    torch = _torch()
    _require_cuda(lenses, "lenses", torch.float32)
    if lenses.dim() != 2 or lenses.shape[1] != 4:
        raise ValueError("lenses must be an n x 4 float32 tensor (x1, x2, m, 0)")
    _require_cuda(counts, "counts", torch.int32)
    _require_cuda(lost, "lost", torch.int64)
    if counts.numel() != int(map_n[0]) * int(map_n[1]):
        raise ValueError("counts must hold map_n[1] * map_n[0] bins")
    if window is None:
        window = ((0, 0), (int(grid_n[0]), int(grid_n[1])))
    j = _abi.Job()
    j.lenses = ctypes.c_void_p(lenses.data_ptr() if lenses.shape[0] else 0)
    j.n_lens = int(lenses.shape[0])
    j.macro.kappa_c = float(kappa_c)
    j.macro.gamma = float(gamma)
    for k in range(2):
        j.grid.lo[k] = float(grid_lo[k])
        j.grid.hi[k] = float(grid_hi[k])
        j.grid.n[k] = int(grid_n[k])
        j.grid.win_lo[k] = int(window[0][k])
        j.grid.win_n[k] = int(window[1][k])
        j.map.lo[k] = float(map_lo[k])
        j.map.hi[k] = float(map_hi[k])
        j.map.n[k] = int(map_n[k])
    if jitter_seed is not None:
        j.grid.jitter, j.grid.jitter_seed = 1, int(jitter_seed) & 0xFFFFFFFFFFFFFFFF
    j.counts = ctypes.c_void_p(counts.data_ptr())
    j.n_lost = ctypes.c_void_p(lost.data_ptr())
    if velocities is not None:
        _require_cuda(velocities, "velocities", torch.float32)
        if velocities.shape != (lenses.shape[0], 2):
            raise ValueError("velocities must be an n_lens x 2 float32 tensor")
        j.velocities = ctypes.c_void_p(velocities.data_ptr() if lenses.shape[0] else 0)
        j.time = float(time)
    j._tensors = (lenses, counts, lost, velocities)     # the struct holds their raw addresses
    return j


def plan_grid(map_lo, map_hi, map_n, n_av, kappa_star=0.0, kappa_c=0.0, gamma=0.0, lens_extent=0.0,
              margin=0.0):
    """rs_plan_grid: a ray grid with at least n_av rays per map pixel.

    Returns (grid_lo, grid_hi, grid_n, planned_n_av)."""
    m = _abi.Map()
    for k in range(2):
        m.lo[k], m.hi[k], m.n[k] = float(map_lo[k]), float(map_hi[k]), int(map_n[k])
    mac = _abi.Macro()
    mac.kappa_c, mac.gamma = float(kappa_c), float(gamma)
    g = _abi.RayGrid()
    nav = ctypes.c_double()
    _check(lib().rs_plan_grid(ctypes.byref(m), ctypes.byref(mac), float(kappa_star), float(lens_extent),
                              float(n_av), float(margin), ctypes.byref(g), ctypes.byref(nav)))
    return (g.lo[0], g.lo[1]), (g.hi[0], g.hi[1]), (int(g.n[0]), int(g.n[1])), nav.value


def advance_lenses(lenses, velocities, time, out=None, stream=None):
    """rs_advance_lenses: the lens records of a moving field at `time` (device tensors)."""
    torch = _torch()
    _require_cuda(lenses, "lenses", torch.float32)
    _require_cuda(velocities, "velocities", torch.float32)
    if lenses.dim() != 2 or lenses.shape[1] != 4 or velocities.shape != (lenses.shape[0], 2):
        raise ValueError("lenses must be n x 4 and velocities n x 2 float32")
    if out is None:
        out = torch.empty_like(lenses)
    _check(lib().rs_advance_lenses(ctypes.c_void_p(lenses.data_ptr()), ctypes.c_void_p(velocities.data_ptr()),
                                   int(lenses.shape[0]), float(time), ctypes.c_void_p(out.data_ptr()),
                                   _stream_handle(stream)))
    return out


def workspace_bytes(job: _abi.Job, opts: Opts | None = None) -> int:
    n = lib().rs_workspace_bytes(ctypes.byref(job), ctypes.byref(opts) if opts else None)
    if n == 0:
        _check(-1)
    return int(n)


def shoot_job(job: _abi.Job, workspace, opts: Opts | None = None, stream=None) -> None:
    """rs_shoot on a filled job with a caller-owned workspace tensor (uint8/any dtype)."""
    _require_cuda(workspace, "workspace")
    nbytes = workspace.numel() * workspace.element_size()
    _check(lib().rs_shoot(ctypes.byref(job), ctypes.c_void_p(workspace.data_ptr()), nbytes,
                          _stream_handle(stream), ctypes.byref(opts) if opts else None))


def shoot_job_noalloc(job: _abi.Job, opts: Opts | None = None, stream=None) -> None:
    """rs_shoot_noalloc: rs_shoot with the library's fixed scratch instead of a workspace (maps of at
    most 1024 x 1024 bins; calls on one GPU must not overlap)."""
    _check(lib().rs_shoot_noalloc(ctypes.byref(job), _stream_handle(stream), ctypes.byref(opts) if opts else None))


def magnification(counts, grid_lo, grid_hi, grid_n, map_lo, map_hi, map_n, mu=None, stream=None):
    """rs_magnification: mu = counts / N_av (FP64, eq. 4) on the device; returns (mu, N_av).

    counts: the int32 view of a map (map_n[1] x map_n[0]); mu: optional float64 tensor of the same
    shape (allocated when None)."""
    torch = _torch()
    _require_cuda(counts, "counts", torch.int32)
    if counts.numel() != int(map_n[0]) * int(map_n[1]):
        raise ValueError("counts must hold map_n[1] * map_n[0] bins")
    if mu is None:
        mu = torch.empty(counts.shape, dtype=torch.float64, device=counts.device)
    _require_cuda(mu, "mu", torch.float64)
    if mu.numel() != counts.numel():
        raise ValueError("mu must have as many elements as counts")
    g = _abi.RayGrid()
    m = _abi.Map()
    for k in range(2):
        g.lo[k], g.hi[k], g.n[k] = float(grid_lo[k]), float(grid_hi[k]), int(grid_n[k])
        g.win_n[k] = int(grid_n[k])
        m.lo[k], m.hi[k], m.n[k] = float(map_lo[k]), float(map_hi[k]), int(map_n[k])
    nav = ctypes.c_double()
    _check(lib().rs_magnification(ctypes.c_void_p(counts.data_ptr()), ctypes.byref(g), ctypes.byref(m),
                                  ctypes.c_void_p(mu.data_ptr()), ctypes.byref(nav), _stream_handle(stream)))
    return mu, nav.value


def zoom_params(cell=(0, 0), margin=0.0) -> _abi.Zoom:
    z = _abi.Zoom()
    z.cell[0], z.cell[1] = int(cell[0]), int(cell[1])
    z.margin = float(margin)
    return z


def zoom_workspace_bytes(job: _abi.Job, zoom: _abi.Zoom, opts: Opts | None = None) -> int:
    n = lib().rs_zoom_workspace_bytes(ctypes.byref(job), ctypes.byref(zoom), ctypes.byref(opts) if opts else None)
    if n == 0:
        raise ValueError(f"invalid zoom job: {lib().rs_last_error().decode()}")
    return n


def shoot_zoom(job: _abi.Job, zoom: _abi.Zoom, workspace, opts: Opts | None = None, stream=None) -> None:
    """rs_shoot_zoom: the fine-grid map of job->map, shooting only the ray tiles that can reach it."""
    _require_cuda(workspace, "workspace")
    nbytes = workspace.numel() * workspace.element_size()
    _check(lib().rs_shoot_zoom(ctypes.byref(job), ctypes.byref(zoom), ctypes.c_void_p(workspace.data_ptr()), nbytes,
                               _stream_handle(stream), ctypes.byref(opts) if opts else None))


def zoom_stats(workspace, stream=None) -> dict:
    """Statistics of the last zoom on `workspace` (synchronises the stream)."""
    out = (ctypes.c_uint64 * 4)()
    _check(lib().rs_zoom_stats(ctypes.c_void_p(workspace.data_ptr()), ctypes.byref(out), _stream_handle(stream)))
    return {"cells_kept": out[0], "cells": out[1], "slots_shot": out[2], "slots": out[3]}


def shoot(lenses, kappa_c, gamma, grid_lo, grid_hi, grid_n, map_lo, map_hi, map_n, counts=None,
          lost=None, window=None, opts: Opts | None = None, workspace=None, stream=None, jitter_seed=None):
    """Shoot a ray-grid window and add its counts into ``counts`` (int32 view of uint32 bins).

    Returns (counts, lost): counts is map_n[1] x map_n[0], lost a 1-element int64 tensor.
    Both accumulate when passed in.
    """
    torch = _torch()
    dev = lenses.device
    if counts is None:
        counts = torch.zeros((int(map_n[1]), int(map_n[0])), dtype=torch.int32, device=dev)
    if lost is None:
        lost = torch.zeros(1, dtype=torch.int64, device=dev)
    job = make_job(lenses, kappa_c, gamma, grid_lo, grid_hi, grid_n, map_lo, map_hi, map_n, counts, lost,
                   window, jitter_seed)
    if workspace is None:
        workspace = torch.empty(workspace_bytes(job, opts), dtype=torch.uint8, device=dev)
    shoot_job(job, workspace, opts, stream)
    return counts, lost


def shoot_workload(w, device="cuda", opts: Opts | None = None, window=None, lenses=None, stream=None):
    """Convenience: shoot a ``synth.Workload``-like object (lenses uploaded unless given)."""
    torch = _torch()
    if lenses is None:
        lenses = torch.from_numpy(w.lenses).to(device)
    return shoot(lenses, w.kappa_c, w.gamma, w.grid_lo, w.grid_hi, w.grid_n, w.map_lo, w.map_hi, w.map_n,
                 window=window, opts=opts, stream=stream)


# ---------------------------------------------------------------- batches

def job_array(jobs):
    """A contiguous host array of rs_job structs (keeps no reference to the tensors)."""
    return (_abi.Job * len(jobs))(*jobs)


def batched_workspace_bytes(jobs) -> int:
    arr = job_array(jobs)
    n = lib().rs_batched_workspace_bytes(arr, len(jobs))
    if n == 0:
        _check(-1)
    return int(n)


def shoot_batched(jobs, workspace, opts: Opts | None = None, stream=None) -> None:
    """rs_shoot_batched: every job's counts are added to its own map (one persistent launch)."""
    _require_cuda(workspace, "workspace")
    arr = job_array(jobs)
    nbytes = workspace.numel() * workspace.element_size()
    _check(lib().rs_shoot_batched(arr, len(jobs), ctypes.c_void_p(workspace.data_ptr()), nbytes,
                                  _stream_handle(stream), ctypes.byref(opts) if opts else None))


def autotune_batched(jobs, workspace, cache_path: str | None = None, opts: Opts | None = None,
                     stream=None) -> Opts:
    """rs_autotune_batched: the fastest block shape / window for this batch (synchronises)."""
    _require_cuda(workspace, "workspace")
    best = Opts()
    if opts is not None:
        ctypes.memmove(ctypes.byref(best), ctypes.byref(opts), ctypes.sizeof(Opts))
    arr = job_array(jobs)
    nbytes = workspace.numel() * workspace.element_size()
    _check(lib().rs_autotune_batched(arr, len(jobs), ctypes.c_void_p(workspace.data_ptr()), nbytes,
                                     _stream_handle(stream), cache_path.encode() if cache_path else None,
                                     ctypes.byref(best)))
    return best


def release_graphs() -> None:
    lib().rs_release_graphs()


# ---------------------------------------------------------------- learned far field

FFConfig = _abi.FFConfig


def ff_config(samples, init_params, tile_rays=(64, 64), r_near=8.0, steps=2000, batch=512, lr=1e-2,
              cell_size=0.0, debug_grad=None, debug_targets=None, eval_tiles=None, shared_x=False) -> FFConfig:
    """rs_ff_config from device tensors: samples (n x 2 float32 in [-1,1]^2), init_params (5378 float32).

    shared_x=True declares that samples 64 (4 g + k) + i, k = 0..3, share their first coordinate
    (faster fit, same model)."""
    torch = _torch()
    _require_cuda(samples, "samples", torch.float32)
    _require_cuda(init_params, "init_params", torch.float32)
    if samples.dim() != 2 or samples.shape[1] != 2:
        raise ValueError("samples must be n x 2")
    if init_params.numel() != _abi.N_PARAMS:
        raise ValueError(f"init_params must hold {_abi.N_PARAMS} values")
    c = FFConfig()
    c.tile_rays[0], c.tile_rays[1] = int(tile_rays[0]), int(tile_rays[1])
    c.r_near = float(r_near)
    c.n_samples = int(samples.shape[0])
    c.steps, c.batch, c.lr, c.cell_size = int(steps), int(batch), float(lr), float(cell_size)
    c.samples = samples.data_ptr()
    c.init_params = init_params.data_ptr()
    if debug_grad is not None:
        _require_cuda(debug_grad, "debug_grad", torch.float32)
        c.debug_grad = debug_grad.data_ptr()
    if debug_targets is not None:
        _require_cuda(debug_targets, "debug_targets", torch.float32)
        c.debug_targets = debug_targets.data_ptr()
    if eval_tiles is not None:
        _require_cuda(eval_tiles, "eval_tiles", torch.int32)
        c.eval_tiles, c.n_eval_tiles = eval_tiles.data_ptr(), int(eval_tiles.numel())
    c.shared_x = 1 if shared_x else 0
    # the struct holds raw addresses: keep the tensors alive with it, and remember the debug
    # buffers' sizes for the check against the job's tile count
    c._tensors = (samples, init_params, debug_grad, debug_targets, eval_tiles)
    c._debug_numel = (debug_grad.numel() if debug_grad is not None else None,
                      debug_targets.numel() if debug_targets is not None else None)
    return c


def _check_debug(job, cfg) -> None:
    """The optional debug buffers must hold n_tiles x 5378 and n_tiles x n_samples x 2 floats."""
    grad_n, targ_n = getattr(cfg, "_debug_numel", (None, None))
    if grad_n is None and targ_n is None:
        return
    tx, ty = int(cfg.tile_rays[0]), int(cfg.tile_rays[1])
    if tx <= 0 or ty <= 0:
        return                                  # the library rejects the configuration itself
    n_tiles = -(-int(job.grid.win_n[0]) // tx) * -(-int(job.grid.win_n[1]) // ty)
    if grad_n is not None and grad_n < n_tiles * _abi.N_PARAMS:
        raise ValueError(f"debug_grad holds {grad_n} floats < {n_tiles} tiles x {_abi.N_PARAMS}")
    if targ_n is not None and targ_n < n_tiles * int(cfg.n_samples) * 2:
        raise ValueError(f"debug_targets holds {targ_n} floats < {n_tiles} tiles x {int(cfg.n_samples)} x 2")


def _size(fn, job, cfg):
    n = fn(ctypes.byref(job), ctypes.byref(cfg))
    if n == 0:
        _check(-1)
    return int(n)


def farfield_model_bytes(job, cfg) -> int:
    return _size(lib().rs_farfield_model_bytes, job, cfg)


def farfield_fit_workspace_bytes(job, cfg) -> int:
    return _size(lib().rs_farfield_fit_workspace_bytes, job, cfg)


def farfield_eval_workspace_bytes(job, cfg) -> int:
    return _size(lib().rs_farfield_eval_workspace_bytes, job, cfg)


def farfield_fit(job, cfg, model, workspace, stream=None) -> None:
    """rs_farfield_fit: fill `model` (uint8 device tensor) with every tile's fitted closure."""
    _require_cuda(model, "model")
    _require_cuda(workspace, "workspace")
    _check_debug(job, cfg)
    _check(lib().rs_farfield_fit(ctypes.byref(job), ctypes.byref(cfg), ctypes.c_void_p(model.data_ptr()),
                                 model.numel() * model.element_size(), ctypes.c_void_p(workspace.data_ptr()),
                                 workspace.numel() * workspace.element_size(), _stream_handle(stream)))


def farfield_eval(job, cfg, model, workspace, opts: Opts | None = None, stream=None) -> None:
    """rs_farfield_eval: shoot the job's rays with the fitted closure, adding into the job's map."""
    _require_cuda(model, "model")
    _require_cuda(workspace, "workspace")
    _check(lib().rs_farfield_eval(ctypes.byref(job), ctypes.byref(cfg), ctypes.c_void_p(model.data_ptr()),
                                  model.numel() * model.element_size(), ctypes.c_void_p(workspace.data_ptr()),
                                  workspace.numel() * workspace.element_size(), _stream_handle(stream),
                                  ctypes.byref(opts) if opts else None))


# ---------------------------------------------------------------- light curves

def light_curve(counts, map_lo, map_hi, map_n, n_av, tracks, n_points, kind="gaussian", size=0.1,
                cutoff=0.0, stream=None, layout=0):
    """rs_light_curve: light curves of a source profile along straight tracks over a device map.

    counts: one map (map_n[1] x map_n[0]) read by every point, or a stack of n_points maps
    (n_points x map_n[1] x map_n[0]) of which point k reads map k (a time-evolving field).
    tracks: device float64 tensor (n_tracks, 4) of (start1, start2, end1, end2).
    Returns (mu, dmag), device float64 tensors of shape (n_tracks, n_points)."""
    torch = _torch()
    _require_cuda(counts, "counts")
    _require_cuda(tracks, "tracks")
    pix = int(map_n[0]) * int(map_n[1])
    if counts.element_size() != 4 or not counts.is_contiguous():
        raise ValueError("counts must be a contiguous 32-bit map or stack of maps")
    if counts.numel() == pix:
        stride = 0
    elif counts.numel() == pix * int(n_points):
        stride = pix
    else:
        raise ValueError("counts must hold one map or n_points maps of map_n[1] x map_n[0] pixels")
    if tracks.dtype != torch.float64 or tracks.dim() != 2 or tracks.shape[1] != 4 or not tracks.is_contiguous():
        raise ValueError("tracks must be a contiguous (n_tracks, 4) float64 tensor")
    m = _abi.Map()
    for k in range(2):
        m.lo[k], m.hi[k], m.n[k] = float(map_lo[k]), float(map_hi[k]), int(map_n[k])
    s = _abi.Source()
    s.kind = {"gaussian": 0, "disc": 1}[kind]
    s.size, s.cutoff = float(size), float(cutoff)
    s.layout = {0: 0, 1: 1, 2: 2, "auto": 0, "lanes": 1, "waves": 2}[layout]
    nt = int(tracks.shape[0])
    mu = torch.empty((nt, int(n_points)), dtype=torch.float64, device=counts.device)
    mag = torch.empty_like(mu)
    _check(lib().rs_light_curve(ctypes.c_void_p(counts.data_ptr()), ctypes.byref(m), float(n_av), ctypes.byref(s),
                                ctypes.c_void_p(tracks.data_ptr()), nt, int(n_points), stride,
                                ctypes.c_void_p(mu.data_ptr()), ctypes.c_void_p(mag.data_ptr()),
                                _stream_handle(stream)))
    return mu, mag
