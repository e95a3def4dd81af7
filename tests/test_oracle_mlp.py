"""Pins of the far-field network oracle (oracle/mlp.py): finite differences, closed forms,
bfloat16 rounding values and the Adam update."""
import math

import numpy as np

from oracle import mlp


def _rand_params(seed, scale=0.3):
    rng = np.random.default_rng(seed)
    return rng.normal(0, scale, mlp.N_PARAMS)


def test_layout_size():
    assert mlp.N_PARAMS == 5378
    W1, b1, W2, b2, W3, b3 = mlp.unpack(np.arange(mlp.N_PARAMS, dtype=float))
    assert W1.shape == (64, 16) and W2.shape == (64, 64) and W3.shape == (2, 64)
    assert b3[-1] == mlp.N_PARAMS - 1


def test_features_closed_form():
    u = np.array([[0.0, 0.0], [1.0, -1.0], [0.5, 0.25]])
    f = mlp.features(u)
    # u = 0: every sine 0, every cosine 1
    assert np.allclose(f[0, 0::2], 0) and np.allclose(f[0, 1::2], 1)
    # u1 = 1: sin(pi/2) = 1, cos(pi/2) = 0, sin(pi) = 0, cos(pi) = -1, sin(2pi) = 0, cos(2pi) = 1
    assert np.allclose(f[1, :6], [1, 0, 0, -1, 0, 1], atol=1e-15)
    # identity sin^2 + cos^2 = 1 for every frequency
    assert np.allclose(f[2, 0::2] ** 2 + f[2, 1::2] ** 2, 1)
    # features are not periodic over the tile: phi(-1) != phi(1) for the lowest frequency
    assert f[1, 0] == -mlp.features([[-1.0, 0.0]])[0, 0]


def test_zero_weights_output_bias():
    p = np.zeros(mlp.N_PARAMS)
    p[mlp.OFF_B3:] = [0.25, -1.5]
    p[mlp.OFF_B1:mlp.OFF_W2] = 3.0
    u = np.random.default_rng(1).uniform(-1, 1, (7, 2))
    o, _ = mlp.forward(p, u)
    assert np.array_equal(o, np.tile([0.25, -1.5], (7, 1)))


def test_silu_and_its_derivative():
    z = np.linspace(-8, 8, 33)
    assert np.allclose(mlp.silu(z), z * (0.5 + 0.5 * np.tanh(z / 2)), rtol=1e-13, atol=1e-15)
    h = 1e-6
    fd = (mlp.silu(z + h) - mlp.silu(z - h)) / (2 * h)
    assert np.allclose(mlp.silu_grad(z), fd, rtol=1e-8, atol=1e-10)


def test_gradient_matches_central_differences():
    rng = np.random.default_rng(2)
    p = _rand_params(3)
    u = rng.uniform(-1, 1, (24, 2))
    t = rng.normal(0, 1, (24, 2))
    g = mlp.gradient(p, u, t)
    idx = np.concatenate([rng.choice(mlp.N_PARAMS, 150, replace=False),
                          [mlp.OFF_B1, mlp.OFF_B2, mlp.OFF_B3, mlp.OFF_B3 + 1, mlp.OFF_W3]])
    for i in idx:
        e = np.zeros_like(p)
        h = 1e-5 * max(1.0, abs(p[i]))
        e[i] = h
        fd = (mlp.loss(p + e, u, t) - mlp.loss(p - e, u, t)) / (2 * h)
        assert abs(fd - g[i]) <= 1e-7 * max(1e-3, np.abs(g).max()), (i, fd, g[i])


def test_bf16_rounding_values():
    # exact bfloat16 values, ties to even, via float32
    assert mlp.bf16(1.0) == 1.0
    assert mlp.bf16(1.0 + 2 ** -8) == 1.0                  # tie, rounds to even
    assert mlp.bf16(1.0 + 3 * 2 ** -8) == 1.0 + 2 ** -6     # tie, rounds up to even
    assert mlp.bf16(1.0 + 2 ** -8 + 2 ** -12) == 1.0 + 2 ** -7
    assert mlp.bf16(-3.0e-3) == -mlp.bf16(3.0e-3)
    x = np.random.default_rng(4).normal(0, 5, 1000)
    r = mlp.bf16(x)
    assert np.all(np.abs(r - x) <= np.abs(x) * 2 ** -8)
    assert np.array_equal(mlp.bf16(r), r)


def test_bf16_forward_close_to_fp64():
    p = _rand_params(5)
    u = np.random.default_rng(6).uniform(-1, 1, (64, 2))
    o64, _ = mlp.forward(p, u)
    o16, _ = mlp.forward(p, u, bf=True)
    assert np.abs(o16 - o64).max() <= 0.05 * np.abs(o64).max()
    assert not np.array_equal(o16, o64)


def test_first_adam_step_closed_form():
    p = _rand_params(7)
    g = np.random.default_rng(8).normal(0, 1, mlp.N_PARAMS)
    p1, m, v = mlp.adam_step(p, g, np.zeros_like(p), np.zeros_like(p), 1, 0.01)
    # bias-corrected first moments are g and g^2, so the step is -lr g / (|g| + eps)
    assert np.allclose(p1, p - 0.01 * g / (np.abs(g) + mlp.EPS), rtol=1e-14, atol=1e-16)
    assert mlp.lr_at(0.01, 1, 100) == 0.01 and abs(mlp.lr_at(0.01, 51, 100) - 0.005) < 1e-15


def test_training_fits_a_smooth_residual():
    # a cubic field over the tile (what remains after an affine base) is learned to ~1%
    rng = np.random.default_rng(9)
    u = rng.uniform(-1, 1, (512, 2))
    t = np.stack([u[:, 0] ** 2 - u[:, 1] ** 2 + 0.3 * u[:, 0] ** 3, 2 * u[:, 0] * u[:, 1]], 1)
    t = t / np.sqrt(np.mean(t ** 2))
    a = math.sqrt(6 / (16 + 64))
    p0 = np.zeros(mlp.N_PARAMS)
    p0[mlp.OFF_W1:mlp.OFF_B1] = rng.uniform(-a, a, 1024)
    p0[mlp.OFF_W2:mlp.OFF_B2] = rng.uniform(-math.sqrt(6 / 128), math.sqrt(6 / 128), 4096)
    p0[mlp.OFF_W3:mlp.OFF_B3] = rng.uniform(-math.sqrt(6 / 66), math.sqrt(6 / 66), 128)
    l0 = mlp.loss(p0, u, t)
    p = mlp.train(p0, u, t, steps=400, batch=128, lr=1e-2)
    assert mlp.loss(p, u, t) < 2e-3 * l0


def test_training_sample_schedule():
    # Step t takes samples [(t - 1) B mod N, + B).  With W3 = 0 the output is b3, so the gradient of
    # b3_1 is b3_1 - mean(target) over the batch; targets equal to the sample index and a zero
    # learning rate (the parameters never move) read the batch of every step off the gradients.
    n, batch, steps = 512, 128, 9
    u = np.zeros((n, 2))
    t = np.stack([np.arange(n, dtype=float), np.zeros(n)], 1)
    p0 = np.zeros(mlp.N_PARAMS)
    rec = []
    p = mlp.train(p0, u, t, steps=steps, batch=batch, lr=0.0, record=rec)
    assert np.array_equal(p, p0) and [s for s, _ in rec] == list(range(1, steps + 1))
    for s, g in rec:
        start = ((s - 1) * batch) % n
        assert g[mlp.OFF_B3] == -(start + (batch - 1) / 2), (s, g[mlp.OFF_B3])
        assert g[mlp.OFF_B3 + 1] == 0.0
    # the cosine schedule reaches zero after the last step and is never negative
    assert mlp.lr_at(1.0, steps + 1, steps) == 0.0
    assert all(mlp.lr_at(1.0, s, steps) >= 0 for s in range(1, steps + 1))
