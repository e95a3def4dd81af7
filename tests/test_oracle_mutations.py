"""Planted slips in the oracles must each fail at least one of their pins.

Each case rewrites one expression of an oracle module's source (a dropped half-pixel offset, a
swapped axis, a wrong sign or factor), loads the result as a separate module, points the pin
tests at it and runs them: at least one pin must fail.  The oracles themselves are untouched.
"""
import importlib.util
import inspect
import os
import sys
import types

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)


def _mutant(module_file: str, package: str, old: str, new: str) -> types.ModuleType:
    src = open(os.path.join(ROOT, "oracle", module_file)).read()
    assert src.count(old) >= 1, f"slip target not found: {old!r}"
    mod = types.ModuleType(f"oracle._mutant_{module_file[:-3]}")
    mod.__package__ = package
    mod.__file__ = os.path.join(ROOT, "oracle", module_file)
    exec(compile(src.replace(old, new, 1), mod.__file__, "exec"), mod.__dict__)
    return mod


def _load_tests(name: str) -> types.ModuleType:
    spec = importlib.util.spec_from_file_location(f"_pins_{name}", os.path.join(HERE, f"{name}.py"))
    mod = importlib.util.module_from_spec(spec)
    sys.modules[spec.name] = mod
    spec.loader.exec_module(mod)
    return mod


def _failures(pins: types.ModuleType, attr: str, mutant: types.ModuleType) -> list[str]:
    """Run every argument-free pin of `pins` with pins.<attr> replaced by the mutant."""
    saved = getattr(pins, attr)
    setattr(pins, attr, mutant)
    failed = []
    try:
        for name, fn in sorted(vars(pins).items()):
            if not name.startswith("test_") or not callable(fn):
                continue
            if inspect.signature(fn).parameters:
                continue
            try:
                fn()
            except (AssertionError, ValueError, FloatingPointError, IndexError):
                failed.append(name)
    finally:
        setattr(pins, attr, saved)
    return failed


LIGHT_CURVE_SLIPS = [
    ("c1 = map_lo[0] + (np.arange(map_n[0], dtype=np.float64) + 0.5) * w0",
     "c1 = map_lo[0] + (np.arange(map_n[0], dtype=np.float64) + 0.0) * w0"),       # no half-pixel offset
    ("d1 = c1[None, :] - y1", "d1 = c1[None, :] - y2"),                              # axes crossed
    ("np.exp(-r2 / (2.0 * size * size))", "np.exp(-r2 / (size * size))"),           # Gaussian width
    ("mag = -2.5 * np.log10(mu)", "mag = 2.5 * np.log10(mu)"),                        # magnitude sign
    ("mu[t, k] = num[t, k] / (den[t, k] * n_av)", "mu[t, k] = num[t, k] / den[t, k]"),  # N_av dropped
    ("f = k / (n_points - 1) if n_points > 1 else 0.0",
     "f = k / n_points if n_points > 1 else 0.0"),                                    # track parameter
    ("frames = [counts.reshape(int(map_n[1]), int(map_n[0])).astype(np.float64)] * n_points",
     "frames = [counts.reshape(int(map_n[1]), int(map_n[0])).T.copy().reshape(int(map_n[1]), int(map_n[0]))"
     ".astype(np.float64)] * n_points"),                                               # transposed map
]


@pytest.mark.parametrize("old,new", LIGHT_CURVE_SLIPS)
def test_light_curve_slips_are_caught(old, new):
    pins = _load_tests("test_oracle_lightcurve")
    failed = _failures(pins, "lc", _mutant("lightcurve.py", "oracle", old, new))
    assert failed, f"no pin catches {new!r}"


FARFIELD_SLIPS = [
    ("j12 = np.sum(-2.0 * m * d[:, 0] * d[:, 1] / r2 ** 2)",
     "j12 = np.sum(2.0 * m * d[:, 0] * d[:, 1] / r2 ** 2)"),                         # shear sign
    ("j11 = np.sum(m * (d[:, 1] ** 2 - d[:, 0] ** 2) / r2 ** 2)",
     "j11 = np.sum(m * (d[:, 0] ** 2 - d[:, 1] ** 2) / r2 ** 2)"),                   # convergence sign
    ("return lo, hi, 0.5 * (lo + hi), 0.5 * (hi - lo), (i0, n)",
     "return lo, hi, 0.5 * (lo + hi), (hi - lo), (i0, n)"),                           # full width as h
    ("p = (c[None, :] + samples.astype(np.float64) * h[None, :])",
     "p = (c[None, :] - samples.astype(np.float64) * h[None, :])"),                   # mirrored samples
    ("return ex * ex + ey * ey < r_near * r_near", "return ex * ex + ey * ey <= r_near * r_near"),
    ("n = (min(tile_rays[0], wl1 + wn1 - i0[0]), min(tile_rays[1], wl2 + wn2 - i0[1]))",
     "n = (tile_rays[0], tile_rays[1])"),                                             # ragged tiles
    ("res = af - (a0[None, :] + (p - c[None, :]) @ J.T)", "res = af - (a0[None, :] + p @ J.T)"),  # offset
]


@pytest.mark.parametrize("old,new", FARFIELD_SLIPS)
def test_farfield_slips_are_caught(old, new):
    pins = _load_tests("test_oracle_farfield")
    failed = _failures(pins, "ff", _mutant("farfield.py", "oracle", old, new))
    assert failed, f"no pin catches {new!r}"
