"""Pins of the moving-lens oracle (oracle.lenses_at) and of the velocity generator.

- time 0 leaves every record unchanged; masses never change;
- each position equals the exactly rounded x + v t (rational arithmetic) to within one float32
  ulp (double rounding through FP64 is the only allowed difference);
- a lone unit-mass lens with no macro model has its caustic, the map's brightest pixel, at the
  lens position (a point lens maps its caustic to y = x_i), so the brightest pixel of each frame
  follows x_i + v t: a sign, axis or scaling slip moves it elsewhere.
"""
from fractions import Fraction

import numpy as np

import oracle
import synth


def test_time_zero_and_masses():
    L, _ = synth.lens_field(3, 500, kappa_star=0.4)
    v = synth.lens_velocities(4, 500, 0.7)
    assert np.array_equal(oracle.lenses_at(L, v, 0.0), L)
    for t in (-3.5, 0.25, 11.0):
        M = oracle.lenses_at(L, v, t)
        assert np.array_equal(M[:, 2:], L[:, 2:])


def test_positions_are_rounded_exact_motion():
    L, _ = synth.lens_field(5, 200, kappa_star=0.4)
    v = synth.lens_velocities(6, 200, 2.0)
    t = 0.37
    M = oracle.lenses_at(L, v, t)
    for i in range(0, 200, 7):
        for k in range(2):
            exact = Fraction(float(L[i, k])) + Fraction(float(v[i, k])) * Fraction(t)
            got = Fraction(float(M[i, k]))
            ulp = np.spacing(np.float32(abs(float(exact))))
            assert abs(got - exact) <= Fraction(float(ulp)), (i, k)


def test_brightest_pixel_follows_a_moving_lens():
    lens = np.array([[0.33, -0.17, 1.0, 0.0]], np.float32)
    vel = np.array([[0.8, 0.5]], np.float32)
    for t in (0.0, 1.0, 2.0):
        w = synth.Workload("one-moving-lens", oracle.lenses_at(lens, vel, t), 0.0, 0.0, (-4.0, -4.0), (4.0, 4.0),
                           (400, 400), (-4.0, -4.0), (4.0, 4.0), (80, 80))
        counts, _ = oracle.shoot_parallel(w)
        p2, p1 = np.unravel_index(np.argmax(counts), counts.shape)
        want = (np.array([0.33, -0.17]) + t * np.array([0.8, 0.5]) + 4.0) / 0.1
        assert (p1, p2) == (int(want[0]), int(want[1])), (t, p1, p2, want)


def test_velocity_generator():
    v = synth.lens_velocities(7, 200000, 1.5)
    assert v.dtype == np.float32 and v.shape == (200000, 2)
    assert abs(v.mean()) < 0.01 and abs(v.std() / 1.5 - 1) < 0.01
    assert abs(np.corrcoef(v[:, 0], v[:, 1])[0, 1]) < 0.01
