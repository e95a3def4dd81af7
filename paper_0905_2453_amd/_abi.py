"""ctypes mirror of the structs and functions declared in include/rs.h."""
from __future__ import annotations

import ctypes

c_double2 = ctypes.c_double * 2
c_int64_2 = ctypes.c_int64 * 2
c_int32_2 = ctypes.c_int32 * 2

RS_OK = 0
RS_EINVAL = -1
RS_ERANGE = -2
RS_EDEVICE = -3
RS_ESMALLBUF = -4
RS_ENOTFIT = -5
RS_EINTERNAL = -6

RS_FLAG_FAULT_INJECT = 0x1
RS_FLAG_NO_GRAPH = 0x2
RS_FLAG_AFFINE_ONLY = 0x4
N_PARAMS = 5378


class RayShootError(RuntimeError):
    def __init__(self, status: int, name: str, detail: str):
        super().__init__(f"{name} ({status}): {detail}")
        self.status = status
        self.name = name
        self.detail = detail


class Macro(ctypes.Structure):
    _fields_ = [("kappa_c", ctypes.c_double), ("gamma", ctypes.c_double)]


class RayGrid(ctypes.Structure):
    _fields_ = [("lo", c_double2), ("hi", c_double2), ("n", c_int64_2), ("win_lo", c_int64_2),
                ("win_n", c_int64_2), ("jitter_seed", ctypes.c_uint64), ("jitter", ctypes.c_int32),
                ("reserved", ctypes.c_int32)]


class Map(ctypes.Structure):
    _fields_ = [("lo", c_double2), ("hi", c_double2), ("n", c_int32_2)]


class Job(ctypes.Structure):
    _fields_ = [("lenses", ctypes.c_void_p), ("n_lens", ctypes.c_int64), ("macro", Macro),
                ("grid", RayGrid), ("map", Map), ("counts", ctypes.c_void_p), ("n_lost", ctypes.c_void_p),
                ("velocities", ctypes.c_void_p), ("time", ctypes.c_double)]


class Opts(ctypes.Structure):
    _fields_ = [("block_cols", ctypes.c_int32), ("block_rows", ctypes.c_int32), ("lens_tile", ctypes.c_int32),
                ("fp32_run", ctypes.c_int32), ("map_window", ctypes.c_int32), ("ray_y", ctypes.c_void_p),
                ("ray_pix", ctypes.c_void_p), ("flags", ctypes.c_uint32)]


class FFConfig(ctypes.Structure):
    _fields_ = [("tile_rays", c_int32_2), ("r_near", ctypes.c_double), ("n_samples", ctypes.c_int32),
                ("steps", ctypes.c_int32), ("batch", ctypes.c_int32), ("lr", ctypes.c_float),
                ("cell_size", ctypes.c_double), ("samples", ctypes.c_void_p), ("init_params", ctypes.c_void_p),
                ("debug_grad", ctypes.c_void_p), ("debug_targets", ctypes.c_void_p),
                ("eval_tiles", ctypes.c_void_p), ("n_eval_tiles", ctypes.c_int32), ("shared_x", ctypes.c_int32)]


class Zoom(ctypes.Structure):
    _fields_ = [("cell", ctypes.c_int32 * 2), ("margin", ctypes.c_double)]


class Source(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int32), ("size", ctypes.c_double), ("cutoff", ctypes.c_double),
                ("layout", ctypes.c_int32)]


# (name, restype, argtypes) of every exported function
EXPORTS = [
    ("rs_status_str", ctypes.c_char_p, [ctypes.c_int]),
    ("rs_last_error", ctypes.c_char_p, []),
    ("rs_version", ctypes.c_char_p, []),
    ("rs_workspace_bytes", ctypes.c_size_t, [ctypes.POINTER(Job), ctypes.POINTER(Opts)]),
    ("rs_shoot", ctypes.c_int, [ctypes.POINTER(Job), ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p,
                                ctypes.POINTER(Opts)]),
    ("rs_shoot_noalloc", ctypes.c_int, [ctypes.POINTER(Job), ctypes.c_void_p, ctypes.POINTER(Opts)]),
    ("rs_magnification", ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(RayGrid), ctypes.POINTER(Map),
                                        ctypes.c_void_p, ctypes.POINTER(ctypes.c_double), ctypes.c_void_p]),
    ("rs_batched_workspace_bytes", ctypes.c_size_t, [ctypes.POINTER(Job), ctypes.c_int32]),
    ("rs_shoot_batched", ctypes.c_int, [ctypes.POINTER(Job), ctypes.c_int32, ctypes.c_void_p, ctypes.c_size_t,
                                        ctypes.c_void_p, ctypes.POINTER(Opts)]),
    ("rs_autotune_batched", ctypes.c_int, [ctypes.POINTER(Job), ctypes.c_int32, ctypes.c_void_p, ctypes.c_size_t,
                                           ctypes.c_void_p, ctypes.c_char_p, ctypes.POINTER(Opts)]),
    ("rs_farfield_model_bytes", ctypes.c_size_t, [ctypes.POINTER(Job), ctypes.POINTER(FFConfig)]),
    ("rs_farfield_fit_workspace_bytes", ctypes.c_size_t, [ctypes.POINTER(Job), ctypes.POINTER(FFConfig)]),
    ("rs_farfield_eval_workspace_bytes", ctypes.c_size_t, [ctypes.POINTER(Job), ctypes.POINTER(FFConfig)]),
    ("rs_farfield_fit", ctypes.c_int, [ctypes.POINTER(Job), ctypes.POINTER(FFConfig), ctypes.c_void_p, ctypes.c_size_t,
                                       ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p]),
    ("rs_farfield_eval", ctypes.c_int, [ctypes.POINTER(Job), ctypes.POINTER(FFConfig), ctypes.c_void_p,
                                        ctypes.c_size_t, ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p,
                                        ctypes.POINTER(Opts)]),
    ("rs_plan_grid", ctypes.c_int, [ctypes.POINTER(Map), ctypes.POINTER(Macro), ctypes.c_double, ctypes.c_double,
                                    ctypes.c_double, ctypes.c_double, ctypes.POINTER(RayGrid),
                                    ctypes.POINTER(ctypes.c_double)]),
    ("rs_advance_lenses", ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64, ctypes.c_double,
                                         ctypes.c_void_p, ctypes.c_void_p]),
    ("rs_zoom_workspace_bytes", ctypes.c_size_t, [ctypes.POINTER(Job), ctypes.POINTER(Zoom), ctypes.POINTER(Opts)]),
    ("rs_shoot_zoom", ctypes.c_int, [ctypes.POINTER(Job), ctypes.POINTER(Zoom), ctypes.c_void_p, ctypes.c_size_t,
                                     ctypes.c_void_p, ctypes.POINTER(Opts)]),
    ("rs_zoom_stats", ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(ctypes.c_uint64 * 4), ctypes.c_void_p]),
    ("rs_light_curve", ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(Map), ctypes.c_double, ctypes.POINTER(Source),
                                      ctypes.c_void_p, ctypes.c_int32, ctypes.c_int32, ctypes.c_int64,
                                      ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]),
    ("rs_release_graphs", None, []),
    ("rs_probe_issue_rate", ctypes.c_int, [ctypes.c_int, ctypes.POINTER(ctypes.c_double),
                                           ctypes.POINTER(ctypes.c_double), ctypes.c_void_p]),
]


def bind(L: ctypes.CDLL) -> ctypes.CDLL:
    for name, res, args in EXPORTS:
        f = getattr(L, name)
        f.restype = res
        f.argtypes = args
    return L
