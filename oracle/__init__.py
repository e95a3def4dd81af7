"""FP64 CPU oracle for inverse ray-shooting -- TEST INFRASTRUCTURE ONLY.

Only the tests, the smoke check and the benchmark's CPU-baseline leg may
import this package.  It shares no code with the HIP library; the two meet
only in the seeded input generators of ``synth``.

The arithmetic lives in ``rs_oracle.c`` (lens equation, eq. 1; deflection,
eq. 2; macro model, eq. 6; estimator, eq. 4 of Thompson et al. 2009), the
exact rational brute force in ``exact.py`` and the network oracle for the
learned far field in ``mlp.py``.
"""
from __future__ import annotations

import ctypes
import os
from concurrent.futures import ThreadPoolExecutor

import numpy as np

from . import build as _build

_lib = None
_P = ctypes.c_void_p


def lib():
    """Load liboracle.so, compiling it first when it is absent."""
    global _lib
    if _lib is None:
        if not os.path.exists(_build.LIB):
            _build.build()
        L = ctypes.CDLL(_build.LIB)
        L.orc_axis.argtypes = [ctypes.c_double, ctypes.c_double, ctypes.c_int64, ctypes.c_int64,
                               ctypes.c_int64, _P]
        L.orc_axis.restype = None
        L.orc_deflect_points.argtypes = [_P, ctypes.c_int64, _P, ctypes.c_int64, _P]
        L.orc_deflect_points.restype = None
        L.orc_trace.argtypes = [_P, ctypes.c_int64, ctypes.c_double, ctypes.c_double, _P, _P, _P,
                                ctypes.c_uint64, ctypes.c_int, _P, _P, _P, _P, ctypes.c_int64, _P, _P]
        L.orc_trace.restype = None
        L.orc_shoot.argtypes = [_P, ctypes.c_int64, ctypes.c_double, ctypes.c_double, _P, _P, _P,
                                ctypes.c_uint64, ctypes.c_int, _P, _P, _P, _P, _P, _P, _P]
        L.orc_shoot.restype = ctypes.c_int64
        L.orc_mix64.argtypes = [ctypes.c_uint64]
        L.orc_mix64.restype = ctypes.c_uint64
        L.orc_jitter_u.argtypes = [ctypes.c_uint64, ctypes.c_int, ctypes.c_int64]
        L.orc_jitter_u.restype = ctypes.c_double
        L.orc_ray_positions.argtypes = [_P, _P, _P, ctypes.c_uint64, ctypes.c_int, _P, ctypes.c_int64, _P]
        L.orc_ray_positions.restype = None
        _lib = L
    return _lib


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


def _lens(lenses) -> np.ndarray:
    a = np.ascontiguousarray(lenses, dtype=np.float32)
    if a.ndim != 2 or a.shape[1] != 4:
        raise ValueError("lenses must be n x 4 float32 (x1, x2, m, 0)")
    return a


def axis(lo: float, hi: float, n: int, i0: int = 0, count: int | None = None) -> np.ndarray:
    """float32 ray coordinates of cells i0 .. i0+count-1 of the axis [lo, hi) cut into n."""
    count = n - i0 if count is None else count
    out = np.empty(count, dtype=np.float32)
    lib().orc_axis(float(lo), float(hi), int(n), int(i0), int(count), _ptr(out))
    return out


def deflect(lenses, pts) -> np.ndarray:
    """FP64 deflection alpha (eq. 2) at the points pts (n x 2, float64)."""
    L = _lens(lenses)
    p = np.ascontiguousarray(pts, dtype=np.float64).reshape(-1, 2)
    out = np.empty_like(p)
    lib().orc_deflect_points(_ptr(L), L.shape[0], _ptr(p), p.shape[0], _ptr(out))
    return out


def _jitter(w):
    seed = getattr(w, "jitter_seed", None)
    return (0, 0) if seed is None else (int(seed) & 0xFFFFFFFFFFFFFFFF, 1)


def ray_positions(w, ray_idx) -> np.ndarray:
    """float32 positions (n x 2) of the listed grid rays (cell centres or jittered)."""
    glo, ghi, gn, _, _, _ = _geom(w)
    idx = np.ascontiguousarray(ray_idx, dtype=np.int64)
    out = np.empty((len(idx), 2), dtype=np.float32)
    seed, jit = _jitter(w)
    lib().orc_ray_positions(_ptr(glo), _ptr(ghi), _ptr(gn), seed, jit, _ptr(idx), len(idx), _ptr(out))
    return out


def _geom(w):
    glo = np.array(w.grid_lo, dtype=np.float64)
    ghi = np.array(w.grid_hi, dtype=np.float64)
    gn = np.array(w.grid_n, dtype=np.int64)
    mlo = np.array(w.map_lo, dtype=np.float64)
    mhi = np.array(w.map_hi, dtype=np.float64)
    mn = np.array(w.map_n, dtype=np.int32)
    return glo, ghi, gn, mlo, mhi, mn


def trace(w, ray_idx) -> tuple[np.ndarray, np.ndarray]:
    """Source position y (n x 2, FP64) and pixel (-1 = lost) of the listed grid rays."""
    L = _lens(w.lenses)
    glo, ghi, gn, mlo, mhi, mn = _geom(w)
    idx = np.ascontiguousarray(ray_idx, dtype=np.int64)
    y = np.empty((len(idx), 2), dtype=np.float64)
    pix = np.empty(len(idx), dtype=np.int64)
    seed, jit = _jitter(w)
    lib().orc_trace(_ptr(L), L.shape[0], float(w.kappa_c), float(w.gamma), _ptr(glo), _ptr(ghi),
                    _ptr(gn), seed, jit, _ptr(mlo), _ptr(mhi), _ptr(mn), _ptr(idx), len(idx), _ptr(y), _ptr(pix))
    return y, pix


def trace_parallel(w, ray_idx, threads: int = 8) -> tuple[np.ndarray, np.ndarray]:
    """trace() over disjoint slices in parallel threads (each call is single-threaded)."""
    idx = np.ascontiguousarray(ray_idx, dtype=np.int64)
    parts = np.array_split(idx, max(1, min(threads, len(idx))))
    with ThreadPoolExecutor(max_workers=threads) as ex:
        res = list(ex.map(lambda p: trace(w, p), parts))
    return np.concatenate([r[0] for r in res]), np.concatenate([r[1] for r in res])


def shoot(w, window=None) -> tuple[np.ndarray, int]:
    """Counts (map_n[1] x map_n[0], uint32) and lost-ray count for a grid window.

    window = ((i1_lo, i2_lo), (n1, n2)); default: the whole grid.
    """
    L = _lens(w.lenses)
    glo, ghi, gn, mlo, mhi, mn = _geom(w)
    if window is None:
        window = ((0, 0), (w.grid_n[0], w.grid_n[1]))
    wlo = np.array(window[0], dtype=np.int64)
    wn = np.array(window[1], dtype=np.int64)
    counts = np.zeros((int(mn[1]), int(mn[0])), dtype=np.uint32)
    lost = np.zeros(1, dtype=np.uint64)
    seed, jit = _jitter(w)
    lib().orc_shoot(_ptr(L), L.shape[0], float(w.kappa_c), float(w.gamma), _ptr(glo), _ptr(ghi),
                    _ptr(gn), seed, jit, _ptr(wlo), _ptr(wn), _ptr(mlo), _ptr(mhi), _ptr(mn), _ptr(counts),
                    _ptr(lost))
    return counts, int(lost[0])


def shoot_parallel(w, window=None, threads: int = 8) -> tuple[np.ndarray, int]:
    """shoot() with the window's rows split over parallel threads; counts summed."""
    if window is None:
        window = ((0, 0), (w.grid_n[0], w.grid_n[1]))
    (a1, a2), (n1, n2) = window
    cuts = np.linspace(0, n2, max(1, min(threads, n2)) + 1).astype(np.int64)
    subs = [((a1, a2 + int(cuts[k])), (n1, int(cuts[k + 1] - cuts[k]))) for k in range(len(cuts) - 1)
            if cuts[k + 1] > cuts[k]]
    with ThreadPoolExecutor(max_workers=threads) as ex:
        res = list(ex.map(lambda s: shoot(w, s), subs))
    counts = np.zeros_like(res[0][0])
    lost = 0
    for c, l in res:
        counts += c
        lost += l
    return counts, lost


def lenses_at(lenses, velocities, t: float) -> np.ndarray:
    """Lens records of a moving field at time t (section 4: stars move between frames).

    Reading (the paper names the effect, not a motion model): each lens moves on a straight line
    at constant velocity, x_i(t) = x_i + v_i t, evaluated in FP64 from the float32 record and
    velocity, then rounded to the float32 record; masses do not change."""
    L = np.array(lenses, dtype=np.float32, copy=True).reshape(-1, 4)
    v = np.asarray(velocities, dtype=np.float32).reshape(-1, 2)
    for k in range(2):
        L[:, k] = (L[:, k].astype(np.float64) + v[:, k].astype(np.float64) * float(t)).astype(np.float32)
    return L


def n_av(w) -> float:
    """Rays per source pixel without lensing: pixel area over ray-cell area (eq. 4's N_av)."""
    dx1 = (w.grid_hi[0] - w.grid_lo[0]) / w.grid_n[0]
    dx2 = (w.grid_hi[1] - w.grid_lo[1]) / w.grid_n[1]
    dy1 = (w.map_hi[0] - w.map_lo[0]) / w.map_n[0]
    dy2 = (w.map_hi[1] - w.map_lo[1]) / w.map_n[1]
    return dy1 * dy2 / (dx1 * dx2)
