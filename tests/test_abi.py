"""Host-side checks of the C ABI (no GPU needed): exports, validation and error paths.

Every call here fails validation (or is the fault-injection path) before the
library makes any HIP call, so fake device addresses are safe.
"""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "rs.h")
HEADERS = sorted(os.path.join(ROOT, "include", f) for f in os.listdir(os.path.join(ROOT, "include")) if f.endswith(".h"))


def _lib():
    import paper_0905_2453_amd as P
    if not os.path.exists(P.LIB_PATH):
        pytest.skip("librs.so not built")
    return P, P.lib()


def _declared_functions():
    names = set()
    for h in HEADERS:
        txt = re.sub(r"/\*.*?\*/", "", open(h).read(), flags=re.S)
        names |= set(re.findall(r"\b(rs_[a-z_0-9]+)\s*\(", txt))
    return sorted(names)


def test_header_functions_exported():
    P, L = _lib()
    names = _declared_functions()
    assert "rs_shoot" in names and "rs_workspace_bytes" in names
    for n in names:
        assert hasattr(L, n), f"{n} declared in rs.h but not exported"
    from paper_0905_2453_amd import _abi
    assert sorted(e[0] for e in _abi.EXPORTS) == names


def test_struct_layout_matches_header(tmp_path):
    # compile the C header and compare every field offset and struct size with the ctypes mirror
    import subprocess
    from paper_0905_2453_amd import _abi
    structs = {"rs_macro": _abi.Macro, "rs_raygrid": _abi.RayGrid, "rs_map": _abi.Map, "rs_job": _abi.Job,
               "rs_opts": _abi.Opts, "rs_ff_config": _abi.FFConfig, "rs_source": _abi.Source, "rs_zoom": _abi.Zoom}
    lines = ["#include <stdio.h>", "#include <stddef.h>", '#include "rs.h"', "int main(void) {"]
    for cname, py in structs.items():
        lines.append(f'printf("{cname} sizeof() %zu\\n", sizeof({cname}));')
        for fname, _ in py._fields_:
            lines.append(f'printf("{cname} {fname} %zu\\n", offsetof({cname}, {fname}));')
    lines += ["return 0; }"]
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines))
    exe = tmp_path / "layout"
    subprocess.check_call(["gcc", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)])
    got = {}
    for line in subprocess.check_output([str(exe)], text=True).splitlines():
        a, b, c = line.split()
        got[(a, b)] = int(c)
    for cname, py in structs.items():
        assert got[(cname, "sizeof()")] == ctypes.sizeof(py), cname
        for fname, _ in py._fields_:
            assert got[(cname, fname)] == getattr(py, fname).offset, (cname, fname)


def _job(**kw):
    from paper_0905_2453_amd import _abi
    j = _abi.Job()
    j.lenses = ctypes.c_void_p(0x1000)
    j.n_lens = 10
    j.macro.kappa_c, j.macro.gamma = 0.0, 0.1
    for k in range(2):
        j.grid.lo[k], j.grid.hi[k], j.grid.n[k] = -1.0, 1.0, 64
        j.grid.win_lo[k], j.grid.win_n[k] = 0, 64
        j.map.lo[k], j.map.hi[k], j.map.n[k] = -1.0, 1.0, 16
    j.counts = ctypes.c_void_p(0x2000)
    j.n_lost = ctypes.c_void_p(0x3000)
    for key, v in kw.items():
        obj, attr = j, key
        if "." in key:
            a, attr = key.split(".")
            obj = getattr(j, a)
        if isinstance(v, tuple):
            getattr(obj, attr)[v[0]] = v[1]
        else:
            setattr(obj, attr, v)
    return j


def _shoot(L, job, ws_bytes=1 << 20, opts=None, ws=0x4000):
    return L.rs_shoot(ctypes.byref(job), ctypes.c_void_p(ws), ws_bytes, None,
                      ctypes.byref(opts) if opts is not None else None)


def test_workspace_query():
    P, L = _lib()
    j = _job()
    n = L.rs_workspace_bytes(ctypes.byref(j), None)
    assert n >= 8 * 16 * 16 * 4
    assert L.rs_workspace_bytes(ctypes.byref(_job(n_lens=-1)), None) == 0


@pytest.mark.parametrize("kw,code", [
    (dict(n_lens=-1), -1),
    (dict(lenses=None), -1),
    (dict(counts=None), -1),
    (dict(n_lost=None), -1),
    (dict(**{"grid.n": (0, 0)}), -1),
    (dict(**{"grid.hi": (1, -1.0)}), -1),
    (dict(**{"grid.lo": (0, float("nan"))}), -1),
    (dict(**{"grid.win_lo": (0, 10)}), -1),
    (dict(**{"grid.win_n": (1, 65)}), -1),
    (dict(**{"grid.win_lo": (1, -1)}), -1),
    (dict(**{"map.n": (0, -3)}), -1),
    (dict(**{"map.hi": (0, -2.0)}), -1),
    (dict(**{"macro.gamma": float("inf")}), -1),
    (dict(**{"grid.lo": (0, -1e13)}), -1),
    (dict(**{"map.lo": (0, 0.0), "map.hi": (0, 1e-310)}), -1),
])
def test_invalid_arguments_rejected(kw, code):
    P, L = _lib()
    st = _shoot(L, _job(**kw))
    assert st == code, L.rs_last_error()
    assert L.rs_status_str(st) == b"RS_EINVAL"
    assert len(L.rs_last_error()) > 0


def test_too_many_rays_is_range_error():
    P, L = _lib()
    j = _job()
    for k in range(2):
        j.grid.n[k] = 1 << 16
        j.grid.win_n[k] = 1 << 16
    assert _shoot(L, j) == -2


def test_map_too_large_is_range_error():
    P, L = _lib()
    j = _job()
    j.map.n[0] = 1 << 16
    j.map.n[1] = 1 << 15
    assert _shoot(L, j) == -2


def test_small_workspace_and_null_workspace():
    P, L = _lib()
    j = _job()
    need = L.rs_workspace_bytes(ctypes.byref(j), None)
    assert _shoot(L, j, ws_bytes=need - 1) == -4
    assert _shoot(L, j, ws=0) == -1


def test_bad_opts_rejected():
    P, L = _lib()
    from paper_0905_2453_amd import _abi
    for field, val in [("block_cols", 3), ("block_rows", 5), ("lens_tile", 100), ("fp32_run", 7),
                       ("map_window", 48)]:
        o = _abi.Opts()
        setattr(o, field, val)
        assert _shoot(L, _job(), opts=o) == -1
    o = _abi.Opts()
    o.block_cols, o.block_rows = 4, 8
    assert _shoot(L, _job(), opts=o) == -1
    o = _abi.Opts()
    o.ray_y = 0x5000  # without ray_pix
    assert _shoot(L, _job(), opts=o) == -1


def test_fault_injection_reports_device_error_without_launch():
    P, L = _lib()
    from paper_0905_2453_amd import _abi
    o = _abi.Opts()
    o.flags = _abi.RS_FLAG_FAULT_INJECT
    st = _shoot(L, _job(), opts=o)
    assert st == -3 and b"injected" in L.rs_last_error()
    with pytest.raises(P.RayShootError) as ei:
        P._check(st)
    assert ei.value.status == -3


def test_noalloc_validation_without_device():
    # rs_shoot_noalloc checks its arguments and the size of its fixed scratch before any HIP call
    P, L = _lib()
    from paper_0905_2453_amd import _abi

    def call(job, opts=None):
        return L.rs_shoot_noalloc(ctypes.byref(job), None, ctypes.byref(opts) if opts is not None else None)

    assert call(_job(n_lens=-1)) == -1
    big = _job()
    big.map.n[0], big.map.n[1] = 1025, 1024
    assert call(big) == -2 and b"at most" in L.rs_last_error()
    edge = _job(**{"grid.win_n": (0, 0)})
    edge.map.n[0], edge.map.n[1] = 1024, 1024
    assert call(edge) == 0                     # the largest map, empty window: nothing to launch
    o = _abi.Opts()
    o.flags = _abi.RS_FLAG_FAULT_INJECT
    assert call(_job(), o) == -3 and b"injected" in L.rs_last_error()
    o = _abi.Opts()
    o.block_cols, o.block_rows = 3, 3
    assert call(_job(), o) == -1


def test_magnification_validation_and_n_av_without_device():
    # rs_magnification computes N_av on the host before any HIP call: with NULL buffers it returns
    # RS_EINVAL after filling N_av, which must equal the oracle's pixel area / ray-cell area bit for bit
    import oracle
    import synth
    P, L = _lib()
    from paper_0905_2453_amd import _abi

    def grid_map(w):
        g, m = _abi.RayGrid(), _abi.Map()
        for k in range(2):
            g.lo[k], g.hi[k], g.n[k] = w.grid_lo[k], w.grid_hi[k], w.grid_n[k]
            m.lo[k], m.hi[k], m.n[k] = w.map_lo[k], w.map_hi[k], w.map_n[k]
        return g, m

    for w in (synth.workload_small(), synth.workload_paper(n_lens=10), synth.workload_farfield(n_lens=10)):
        g, m = grid_map(w)
        nav = ctypes.c_double(-1.0)
        st = L.rs_magnification(None, ctypes.byref(g), ctypes.byref(m), None, ctypes.byref(nav), None)
        assert st == -1 and nav.value == oracle.n_av(w), (w.name, nav.value, oracle.n_av(w))
    g, m = grid_map(synth.workload_small())
    assert L.rs_magnification(ctypes.c_void_p(0x1000), None, ctypes.byref(m), ctypes.c_void_p(0x2000), None, None) == -1
    bad = _abi.Map.from_buffer_copy(m)
    bad.n[1] = 0
    assert L.rs_magnification(ctypes.c_void_p(0x1000), ctypes.byref(g), ctypes.byref(bad), ctypes.c_void_p(0x2000),
                              None, None) == -1
    bad = _abi.RayGrid.from_buffer_copy(g)
    bad.hi[0] = bad.lo[0]
    assert L.rs_magnification(ctypes.c_void_p(0x1000), ctypes.byref(bad), ctypes.byref(m), ctypes.c_void_p(0x2000),
                              None, None) == -1
    big = _abi.Map.from_buffer_copy(m)
    big.n[0], big.n[1] = 65536, 32768
    assert L.rs_magnification(ctypes.c_void_p(0x1000), ctypes.byref(g), ctypes.byref(big), ctypes.c_void_p(0x2000),
                              None, None) == -2


def test_probe_validation_without_device():
    P, L = _lib()
    r = ctypes.c_double()
    assert L.rs_probe_issue_rate(99, ctypes.byref(r), None, None) == -1
    assert L.rs_probe_issue_rate(-1, ctypes.byref(r), None, None) == -1
    assert L.rs_probe_issue_rate(0, None, None, None) == -1


def test_version_string():
    P, L = _lib()
    assert b"gfx950" in L.rs_version()


def test_batched_validation_without_device():
    P, L = _lib()
    from paper_0905_2453_amd import _abi
    good = _job()
    bad = _job(n_lens=-1)
    arr = (_abi.Job * 2)(good, bad)
    assert L.rs_batched_workspace_bytes(arr, 2) == 0
    arr_ok = (_abi.Job * 2)(good, good)
    need = L.rs_batched_workspace_bytes(arr_ok, 2)
    assert need > 0
    # invalid job is reported with its index before any HIP call
    st = L.rs_shoot_batched(arr, 2, ctypes.c_void_p(0x4000), 1 << 30, None, None)
    assert st == -1 and b"job 1" in L.rs_last_error()
    assert L.rs_shoot_batched(arr_ok, 2, ctypes.c_void_p(0x4000), need - 1, None, None) == -4
    assert L.rs_shoot_batched(arr_ok, -1, ctypes.c_void_p(0x4000), need, None, None) == -1
    o = _abi.Opts()
    o.ray_y, o.ray_pix = 0x10, 0x20
    assert L.rs_shoot_batched(arr_ok, 2, ctypes.c_void_p(0x4000), need, None, ctypes.byref(o)) == -1
    o = _abi.Opts()
    o.flags = _abi.RS_FLAG_FAULT_INJECT
    assert L.rs_shoot_batched(arr_ok, 2, ctypes.c_void_p(0x4000), need, None, ctypes.byref(o)) == -3
    assert L.rs_autotune_batched(arr_ok, 2, ctypes.c_void_p(0x4000), need, None, None, None) == -1


def _ffcfg(**kw):
    from paper_0905_2453_amd import _abi
    c = _abi.FFConfig()
    c.tile_rays[0], c.tile_rays[1] = 16, 16
    c.r_near, c.n_samples, c.steps, c.batch, c.lr = 8.0, 1024, 10, 512, 1e-2
    c.samples, c.init_params = 0x7000, 0x8000
    for k, v in kw.items():
        setattr(c, k, v)
    return c


def test_farfield_validation_without_device():
    P, L = _lib()
    j = _job()
    good = _ffcfg()
    assert L.rs_farfield_model_bytes(ctypes.byref(j), ctypes.byref(good)) > 256
    assert L.rs_farfield_fit_workspace_bytes(ctypes.byref(j), ctypes.byref(good)) > 0
    assert L.rs_farfield_eval_workspace_bytes(ctypes.byref(j), ctypes.byref(good)) > 0
    for bad in [dict(n_samples=1000), dict(batch=100), dict(batch=384), dict(batch=128), dict(steps=-1),
                dict(r_near=0.0),
                dict(r_near=float("nan")), dict(lr=float("inf")), dict(cell_size=-1.0)]:
        c = _ffcfg(**bad)
        assert L.rs_farfield_model_bytes(ctypes.byref(j), ctypes.byref(c)) == 0, bad
        st = L.rs_farfield_fit(ctypes.byref(j), ctypes.byref(c), ctypes.c_void_p(0x9000), 1 << 30,
                               ctypes.c_void_p(0xa000), 1 << 30, None)
        assert st == -1, bad
    c = _ffcfg(tile_rays=(ctypes.c_int32 * 2)(0, 16))
    assert L.rs_farfield_model_bytes(ctypes.byref(j), ctypes.byref(c)) == 0
    huge = _ffcfg(tile_rays=(ctypes.c_int32 * 2)(4097, 4096))       # more than 2^24 rays per tile
    assert L.rs_farfield_model_bytes(ctypes.byref(j), ctypes.byref(huge)) == 0
    st = L.rs_farfield_fit(ctypes.byref(j), ctypes.byref(huge), ctypes.c_void_p(0x9000), 1 << 30,
                           ctypes.c_void_p(0xa000), 1 << 30, None)
    assert st == -2
    assert L.rs_farfield_model_bytes(ctypes.byref(j), ctypes.byref(_ffcfg(tile_rays=(ctypes.c_int32 * 2)(4096, 4096)))) > 0
    for bad in (2, -1):
        assert L.rs_farfield_model_bytes(ctypes.byref(j), ctypes.byref(_ffcfg(shared_x=bad))) == 0
    assert L.rs_farfield_model_bytes(ctypes.byref(j), ctypes.byref(_ffcfg(shared_x=1))) > 0
    need = L.rs_farfield_model_bytes(ctypes.byref(j), ctypes.byref(good))
    st = L.rs_farfield_fit(ctypes.byref(j), ctypes.byref(good), ctypes.c_void_p(0x9000), need - 1,
                           ctypes.c_void_p(0xa000), 1 << 30, None)
    assert st == -4
    st = L.rs_farfield_fit(ctypes.byref(j), ctypes.byref(_ffcfg(samples=None)), ctypes.c_void_p(0x9000), need,
                           ctypes.c_void_p(0xa000), 1 << 30, None)
    assert st == -1
    from paper_0905_2453_amd import _abi
    o = _abi.Opts()
    o.flags = _abi.RS_FLAG_FAULT_INJECT
    ew = L.rs_farfield_eval_workspace_bytes(ctypes.byref(j), ctypes.byref(good))
    st = L.rs_farfield_eval(ctypes.byref(j), ctypes.byref(good), ctypes.c_void_p(0x9000), need,
                            ctypes.c_void_p(0xa000), ew, None, ctypes.byref(o))
    assert st == -3


def test_light_curve_validation_without_device():
    P, L = _lib()
    from paper_0905_2453_amd import _abi
    m = _abi.Map()
    for k in range(2):
        m.lo[k], m.hi[k], m.n[k] = -1.0, 1.0, 64

    def src(kind=0, size=0.1, cutoff=0.0):
        s = _abi.Source()
        s.kind, s.size, s.cutoff = kind, size, cutoff
        return s

    def call(mp=m, n_av=4.0, s=None, nt=3, npts=10, counts=0x1000, tracks=0x2000, stride=0):
        s = s if s is not None else src()
        return L.rs_light_curve(ctypes.c_void_p(counts), ctypes.byref(mp), n_av, ctypes.byref(s),
                                ctypes.c_void_p(tracks), nt, npts, stride, ctypes.c_void_p(0x3000), None, None)

    bad_map = _abi.Map()
    for k in range(2):
        bad_map.lo[k], bad_map.hi[k], bad_map.n[k] = 1.0, 1.0, 64
    for st in [call(n_av=0.0), call(n_av=float("nan")), call(s=src(kind=2)), call(s=src(size=0.0)),
               call(s=src(size=float("inf"))), call(s=src(cutoff=-1.0)), call(nt=-1), call(npts=0),
               call(mp=bad_map), call(counts=0), call(tracks=0), call(stride=64 * 64 - 1), call(stride=-5)]:
        assert st == -1
    assert call(npts=0) == -1 and b"n_points" in L.rs_last_error()
    assert call(nt=0, counts=0, tracks=0) == 0          # nothing to do: no launch, no device


def test_zoom_validation_without_device():
    P, L = _lib()
    from paper_0905_2453_amd import _abi
    j = _job()

    def z(c0=0, c1=0, margin=0.0):
        r = _abi.Zoom()
        r.cell[0], r.cell[1], r.margin = c0, c1, margin
        return r

    need = L.rs_zoom_workspace_bytes(ctypes.byref(j), ctypes.byref(z()), None)
    assert need > L.rs_workspace_bytes(ctypes.byref(j), None)
    for bad in (z(-1, 4), z(4, 0), z(0, 4), z(70000, 1), z(margin=-1.0), z(margin=float("nan"))):
        assert L.rs_zoom_workspace_bytes(ctypes.byref(j), ctypes.byref(bad), None) == 0
        st = L.rs_shoot_zoom(ctypes.byref(j), ctypes.byref(bad), ctypes.c_void_p(0x4000), need, None, None)
        assert st == -1
    assert L.rs_shoot_zoom(ctypes.byref(j), None, ctypes.c_void_p(0x4000), need, None, None) == -1
    assert L.rs_shoot_zoom(ctypes.byref(j), ctypes.byref(z()), ctypes.c_void_p(0x4000), need - 1, None, None) == -4
    assert L.rs_shoot_zoom(ctypes.byref(j), ctypes.byref(z()), None, need, None, None) == -1
    o = _abi.Opts()
    o.ray_y, o.ray_pix = 0x5000, 0x6000
    assert L.rs_shoot_zoom(ctypes.byref(j), ctypes.byref(z()), ctypes.c_void_p(0x4000), need, None,
                           ctypes.byref(o)) == -1
    o = _abi.Opts()
    o.flags = _abi.RS_FLAG_FAULT_INJECT
    assert L.rs_shoot_zoom(ctypes.byref(j), ctypes.byref(z()), ctypes.c_void_p(0x4000), need, None,
                           ctypes.byref(o)) == -3
    assert L.rs_zoom_stats(None, None, None) == -1


def test_moving_lens_validation_without_device():
    P, L = _lib()
    j = _job()
    j.velocities = ctypes.c_void_p(0x7000)
    j.time = float("nan")
    assert L.rs_workspace_bytes(ctypes.byref(j), None) == 0
    j.time = 2.0
    assert L.rs_workspace_bytes(ctypes.byref(j), None) > 0
    # the closure is fitted on a static field; evaluating it on a moving one is allowed
    c = _ffcfg()
    assert L.rs_farfield_fit_workspace_bytes(ctypes.byref(j), ctypes.byref(c)) == 0
    assert L.rs_farfield_eval_workspace_bytes(ctypes.byref(j), ctypes.byref(c)) > 0
    assert L.rs_farfield_model_bytes(ctypes.byref(j), ctypes.byref(c)) > 0
    assert L.rs_advance_lenses(None, None, 5, 1.0, None, None) == -1
    assert L.rs_advance_lenses(ctypes.c_void_p(0x1000), ctypes.c_void_p(0x2000), 5, float("inf"),
                               ctypes.c_void_p(0x3000), None) == -1
    assert L.rs_advance_lenses(None, None, 0, 1.0, None, None) == 0
