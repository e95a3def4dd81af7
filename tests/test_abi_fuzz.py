"""Property tests of the C ABI's argument validation (no device needed).

Random job descriptions (finite, non-finite, negative, inverted and oversized fields) go to
rs_workspace_bytes and rs_shoot.  Every call must return one of the documented statuses, never
crash; a job that validates must, under RS_FLAG_FAULT_INJECT, stop at the device-error path
before any HIP call, and one that does not must be refused with RS_EINVAL or RS_ERANGE.
"""
import ctypes
import math

import pytest

hyp = pytest.importorskip("hypothesis")
from hypothesis import given, settings, strategies as st  # noqa: E402

OK, EINVAL, ERANGE, EDEVICE, ESMALLBUF = 0, -1, -2, -3, -4

floats = st.one_of(st.floats(min_value=-1e13, max_value=1e13, allow_nan=False, allow_infinity=False),
                   st.sampled_from([math.nan, math.inf, -math.inf, 0.0, -0.0, 1e300]))
ints = st.one_of(st.integers(min_value=-5, max_value=5000), st.sampled_from([0, 1, 2**31, 2**40, -2**40]))


def _lib():
    import paper_0905_2453_amd as P
    return P, P.lib()


@settings(max_examples=400, deadline=None)
@given(glo=st.tuples(floats, floats), gspan=st.tuples(floats, floats), gn=st.tuples(ints, ints),
       wlo=st.tuples(ints, ints), wn=st.tuples(ints, ints), mlo=st.tuples(floats, floats),
       mspan=st.tuples(floats, floats), mn=st.tuples(st.integers(-3, 70000), st.integers(-3, 70000)),
       kappa=floats, gamma=floats, n_lens=st.integers(-3, 1000), jitter=st.integers(-1, 2),
       null_counts=st.booleans())
def test_shoot_validation_never_crashes(glo, gspan, gn, wlo, wn, mlo, mspan, mn, kappa, gamma, n_lens, jitter,
                                        null_counts):
    P, L = _lib()
    from paper_0905_2453_amd import _abi
    j = _abi.Job()
    j.lenses = ctypes.c_void_p(0x1000 if n_lens else 0)
    j.n_lens = n_lens
    j.macro.kappa_c, j.macro.gamma = kappa, gamma
    for k in range(2):
        j.grid.lo[k] = glo[k]
        j.grid.hi[k] = glo[k] + gspan[k] if math.isfinite(glo[k] + gspan[k]) else gspan[k]
        j.grid.n[k], j.grid.win_lo[k], j.grid.win_n[k] = gn[k], wlo[k], wn[k]
        j.map.lo[k] = mlo[k]
        j.map.hi[k] = mlo[k] + mspan[k] if math.isfinite(mlo[k] + mspan[k]) else mspan[k]
        j.map.n[k] = mn[k]
    j.grid.jitter = jitter
    j.counts = ctypes.c_void_p(0 if null_counts else 0x2000)
    j.n_lost = ctypes.c_void_p(0x3000)
    need = L.rs_workspace_bytes(ctypes.byref(j), None)
    o = _abi.Opts()
    o.flags = _abi.RS_FLAG_FAULT_INJECT
    st_ = L.rs_shoot(ctypes.byref(j), ctypes.c_void_p(0x4000), max(need, 1) << 1, None, ctypes.byref(o))
    assert st_ in (EINVAL, ERANGE, EDEVICE)
    if need:
        assert st_ == EDEVICE                    # valid: stopped at the injected device fault
    else:
        assert st_ in (EINVAL, ERANGE) and L.rs_last_error()
    # the zoom validates the same job plus its own fields
    z = _abi.Zoom()
    assert L.rs_shoot_zoom(ctypes.byref(j), ctypes.byref(z), ctypes.c_void_p(0x4000), 1 << 40, None,
                           ctypes.byref(o)) in (EINVAL, ERANGE, EDEVICE)


@settings(max_examples=300, deadline=None)
@given(n_av=floats, size=floats, cutoff=floats, kind=st.integers(-1, 3), layout=st.integers(-1, 3),
       nt=st.integers(-2, 3), npts=st.integers(-2, 3), mspan=floats)
def test_light_curve_validation_never_crashes(n_av, size, cutoff, kind, layout, nt, npts, mspan):
    P, L = _lib()
    from paper_0905_2453_amd import _abi
    m = _abi.Map()
    for k in range(2):
        m.lo[k], m.hi[k], m.n[k] = 0.0, mspan, 16
    s = _abi.Source()
    s.kind, s.size, s.cutoff, s.layout = kind, size, cutoff, layout
    valid = (math.isfinite(n_av) and n_av > 0 and kind in (0, 1) and math.isfinite(size) and size > 0
             and math.isfinite(cutoff) and cutoff >= 0 and layout in (0, 1, 2) and nt >= 0 and npts >= 1
             and math.isfinite(mspan) and mspan > 0)
    if valid and nt > 0:
        return                                   # would launch: not a host-only case
    r = L.rs_light_curve(ctypes.c_void_p(0x1000), ctypes.byref(m), n_av, ctypes.byref(s), ctypes.c_void_p(0x2000),
                         nt, npts, 0, None, None, None)
    assert r == (OK if valid else EINVAL)


@settings(max_examples=300, deadline=None)
@given(n_av=floats, ks=floats, kc=floats, g=floats, ext=floats, margin=floats, mspan=floats)
def test_plan_grid_never_crashes_and_meets_budget(n_av, ks, kc, g, ext, margin, mspan):
    P, L = _lib()
    from paper_0905_2453_amd import _abi
    m = _abi.Map()
    for k in range(2):
        m.lo[k], m.hi[k], m.n[k] = -1.0, -1.0 + mspan if math.isfinite(mspan) else mspan, 64
    mac = _abi.Macro()
    mac.kappa_c, mac.gamma = kc, g
    grid = _abi.RayGrid()
    nav = ctypes.c_double()
    r = L.rs_plan_grid(ctypes.byref(m), ctypes.byref(mac), ks, ext, n_av, margin, ctypes.byref(grid),
                       ctypes.byref(nav))
    assert r in (OK, EINVAL, ERANGE)
    if r == OK:
        assert nav.value >= n_av * (1 - 1e-12)
        assert grid.n[0] > 0 and grid.n[1] > 0 and grid.hi[0] > grid.lo[0] and grid.hi[1] > grid.lo[1]
        assert all(math.isfinite(v) for v in (grid.lo[0], grid.lo[1], grid.hi[0], grid.hi[1]))
        # the planned grid is one a job accepts (or, if it holds 2^62 rays or more, refuses by range)
        j = _abi.Job()
        j.grid, j.map = grid, m
        j.macro = mac
        j.counts, j.n_lost = ctypes.c_void_p(0x2000), ctypes.c_void_p(0x3000)
        o = _abi.Opts()
        o.flags = _abi.RS_FLAG_FAULT_INJECT
        if math.isfinite(kc) and math.isfinite(g):
            assert L.rs_shoot(ctypes.byref(j), ctypes.c_void_p(0x4000), 1 << 62, None, ctypes.byref(o)) in (EDEVICE, ERANGE)


def _valid_job(_abi):
    j = _abi.Job()
    j.lenses = ctypes.c_void_p(0x1000)
    j.n_lens = 10
    j.macro.kappa_c, j.macro.gamma = 0.0, 0.1
    for k in range(2):
        j.grid.lo[k], j.grid.hi[k], j.grid.n[k] = -1.0, 1.0, 256
        j.grid.win_lo[k], j.grid.win_n[k] = 0, 256
        j.map.lo[k], j.map.hi[k], j.map.n[k] = -1.0, 1.0, 32
    j.counts, j.n_lost = ctypes.c_void_p(0x2000), ctypes.c_void_p(0x3000)
    return j


@settings(max_examples=300, deadline=None)
@given(tx=st.integers(-2, 300), ty=st.integers(-2, 300), r_near=floats, ns=st.integers(-1, 9000),
       steps=st.integers(-2, 5000), batch=st.integers(-1, 5000), lr=floats, cell=floats,
       shared=st.integers(-1, 2))
def test_farfield_config_validation_never_crashes(tx, ty, r_near, ns, steps, batch, lr, cell, shared):
    P, L = _lib()
    from paper_0905_2453_amd import _abi
    j = _valid_job(_abi)
    c = _abi.FFConfig()
    c.tile_rays[0], c.tile_rays[1] = tx, ty
    c.r_near, c.n_samples, c.steps, c.batch = r_near, ns, steps, batch
    c.lr = lr if abs(lr) < 3e38 or not math.isfinite(lr) else 1.0
    c.cell_size, c.shared_x = cell, shared
    c.samples, c.init_params = 0x5000, 0x6000
    nb = L.rs_farfield_model_bytes(ctypes.byref(j), ctypes.byref(c))
    valid = (tx > 0 and ty > 0 and math.isfinite(r_near) and r_near > 0 and ns > 0 and ns % 1024 == 0
             and steps >= 0 and batch > 0 and batch % 256 == 0 and ns % batch == 0 and math.isfinite(c.lr)
             and c.lr >= 0 and math.isfinite(cell) and cell >= 0 and shared in (0, 1))
    assert (nb > 0) == valid
    o = _abi.Opts()
    o.flags = _abi.RS_FLAG_FAULT_INJECT
    ws = L.rs_farfield_eval_workspace_bytes(ctypes.byref(j), ctypes.byref(c))
    r = L.rs_farfield_eval(ctypes.byref(j), ctypes.byref(c), ctypes.c_void_p(0x7000), max(nb, 1) << 1,
                           ctypes.c_void_p(0x8000), max(ws, 1) << 1, None, ctypes.byref(o))
    assert r in ((EDEVICE,) if valid else (EINVAL, ERANGE))


@settings(max_examples=300, deadline=None)
@given(c1=st.integers(-2, 70000), c2=st.integers(-2, 70000), margin=floats)
def test_zoom_parameters_never_crash(c1, c2, margin):
    P, L = _lib()
    from paper_0905_2453_amd import _abi
    j = _valid_job(_abi)
    z = _abi.Zoom()
    z.cell[0], z.cell[1], z.margin = c1, c2, margin
    need = L.rs_zoom_workspace_bytes(ctypes.byref(j), ctypes.byref(z), None)
    valid = (0 <= c1 <= 65536 and 0 <= c2 <= 65536 and (c1 == 0) == (c2 == 0) and math.isfinite(margin)
             and margin >= 0)
    assert (need > 0) == valid
    o = _abi.Opts()
    o.flags = _abi.RS_FLAG_FAULT_INJECT
    r = L.rs_shoot_zoom(ctypes.byref(j), ctypes.byref(z), ctypes.c_void_p(0x4000), max(need, 1), None, ctypes.byref(o))
    assert r == (EDEVICE if valid else EINVAL)


@settings(max_examples=200, deadline=None)
@given(bad=st.lists(st.integers(0, 5), min_size=1, max_size=6))
def test_batched_validation_never_crashes(bad):
    # 0: valid job; 1: negative lenses; 2: inverted grid; 3: NULL counts; 4: window outside; 5: map too big
    P, L = _lib()
    from paper_0905_2453_amd import _abi
    jobs = []
    for b in bad:
        j = _valid_job(_abi)
        if b == 1:
            j.n_lens = -1
        elif b == 2:
            j.grid.hi[0] = -2.0
        elif b == 3:
            j.counts = ctypes.c_void_p(0)
        elif b == 4:
            j.grid.win_lo[1] = 200
        elif b == 5:
            j.map.n[0], j.map.n[1] = 65536, 65536
        jobs.append(j)
    arr = (_abi.Job * len(jobs))(*jobs)
    need = L.rs_batched_workspace_bytes(arr, len(jobs))
    assert (need > 0) == all(b == 0 for b in bad)
