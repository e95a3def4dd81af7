"""FP64 oracle of the learned far-field closure's network -- TEST INFRASTRUCTURE ONLY.

The network maps tile-local coordinates u in [-1, 1]^2 to the far-field
deflection residual of a ray tile (the learned closure of the far field; the
paper's direct sum over distant lenses is what it stands in for):

  features  phi (16): for axis d in (1, 2) and k in 0..3,
            sin(w_k u_d), cos(w_k u_d) with w_k = (pi / 2) 2^k,
            ordered phi[8 d + 2 k] = sin, phi[8 d + 2 k + 1] = cos (d = 0, 1)
  layer 1   z1 = W1 phi + b1   (64 x 16),  h1 = silu(z1)
  layer 2   z2 = W2 h1 + b2    (64 x 64),  h2 = silu(z2)
  layer 3   o  = W3 h2 + b3    (2 x 64)
  silu(z) = z / (1 + exp(-z))

Flat parameter vector (5378 values): W1 (row-major [j][f]) at 0, b1 at 1024,
W2 ([j][i]) at 1088, b2 at 5184, W3 ([o][j]) at 5248, b3 at 5376.

Loss over a batch of B samples: L = sum_s sum_o (o - t)^2 / (2 B).
Adam (beta1 0.9, beta2 0.999, eps 1e-8) with bias correction; the learning
rate of step t (1-based) of S is lr * (1 + cos(pi (t - 1) / S)) / 2.  Step t
uses samples [(t - 1) B mod N, (t - 1) B mod N + B) of the N fit samples.

With ``bf16=True`` every GEMM operand (features, weights, activations and the
back-propagated deltas that enter a GEMM) is rounded to bfloat16 (round to
nearest even, via float32) exactly where the GPU kernels round; the sums are
still exact FP64.  With ``bf16=False`` the same code is plain FP64 and its
gradients are pinned by central finite differences.
"""
from __future__ import annotations

import numpy as np

N_FEAT = 16
HIDDEN = 64
N_OUT = 2
OFF_W1 = 0
OFF_B1 = OFF_W1 + HIDDEN * N_FEAT
OFF_W2 = OFF_B1 + HIDDEN
OFF_B2 = OFF_W2 + HIDDEN * HIDDEN
OFF_W3 = OFF_B2 + HIDDEN
OFF_B3 = OFF_W3 + N_OUT * HIDDEN
N_PARAMS = OFF_B3 + N_OUT  # 5378
BETA1, BETA2, EPS = 0.9, 0.999, 1e-8


def bf16(x):
    """Round to bfloat16 (via float32, ties to even) and return as float64."""
    f = np.asarray(x, dtype=np.float64).astype(np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000
    return u.astype(np.uint32).view(np.float32).astype(np.float64)


def unpack(p):
    p = np.asarray(p, dtype=np.float64)
    W1 = p[OFF_W1:OFF_B1].reshape(HIDDEN, N_FEAT)
    b1 = p[OFF_B1:OFF_W2]
    W2 = p[OFF_W2:OFF_B2].reshape(HIDDEN, HIDDEN)
    b2 = p[OFF_B2:OFF_W3]
    W3 = p[OFF_W3:OFF_B3].reshape(N_OUT, HIDDEN)
    b3 = p[OFF_B3:N_PARAMS]
    return W1, b1, W2, b2, W3, b3


def features(u):
    """phi(u): n x 16."""
    u = np.asarray(u, dtype=np.float64).reshape(-1, 2)
    cols = []
    for d in range(2):
        for k in range(4):
            w = 0.5 * np.pi * 2.0 ** k
            cols.append(np.sin(w * u[:, d]))
            cols.append(np.cos(w * u[:, d]))
    return np.stack(cols, 1)


def silu(z):
    return z / (1.0 + np.exp(-z))


def silu_grad(z):
    s = 1.0 / (1.0 + np.exp(-z))
    return s * (1.0 + z * (1.0 - s))


def forward(p, u, bf=False):
    """Network output (n x 2) and the intermediate values backward() needs."""
    q = bf16 if bf else (lambda x: np.asarray(x, dtype=np.float64))
    W1, b1, W2, b2, W3, b3 = unpack(p)
    phi = q(features(u))
    z1 = phi @ q(W1).T + b1
    h1 = q(silu(z1))
    z2 = h1 @ q(W2).T + b2
    h2 = q(silu(z2))
    o = h2 @ q(W3).T + b3
    return o, (phi, z1, h1, z2, h2)


def loss(p, u, t, bf=False):
    o, _ = forward(p, u, bf)
    return float(np.sum((o - t) ** 2) / (2.0 * len(o)))


def gradient(p, u, t, bf=False):
    """dL/dp (5378) by back-propagation through the forward pass above."""
    q = bf16 if bf else (lambda x: np.asarray(x, dtype=np.float64))
    W1, b1, W2, b2, W3, b3 = unpack(p)
    o, (phi, z1, h1, z2, h2) = forward(p, u, bf)
    n = len(o)
    d3 = (o - t) / n                     # dL/do
    g = np.zeros(N_PARAMS)
    g[OFF_W3:OFF_B3] = (d3.T @ h2).ravel()
    g[OFF_B3:N_PARAMS] = d3.sum(0)
    dh2 = d3 @ q(W3)
    dz2 = q(dh2 * silu_grad(z2))
    g[OFF_W2:OFF_B2] = (dz2.T @ h1).ravel()
    g[OFF_B2:OFF_W3] = dz2.sum(0)
    dh1 = dz2 @ q(W2)
    dz1 = q(dh1 * silu_grad(z1))
    g[OFF_W1:OFF_B1] = (dz1.T @ phi).ravel()
    g[OFF_B1:OFF_W2] = dz1.sum(0)
    return g


def lr_at(lr, t, steps):
    """Cosine-decayed learning rate of step t (1-based) of `steps`."""
    return lr * 0.5 * (1.0 + np.cos(np.pi * (t - 1) / steps))


def adam_step(p, g, m, v, t, lr_t):
    """One Adam update (returns new p, m, v)."""
    m = BETA1 * m + (1.0 - BETA1) * g
    v = BETA2 * v + (1.0 - BETA2) * g * g
    mh = m / (1.0 - BETA1 ** t)
    vh = v / (1.0 - BETA2 ** t)
    return p - lr_t * mh / (np.sqrt(vh) + EPS), m, v


def train(p0, u, t, steps, batch, lr, bf=False, record=None):
    """Mini-batch Adam over the fit samples in order; returns the final parameters.

    record: optional list receiving (step, gradient) of every step.
    """
    p = np.array(p0, dtype=np.float64)
    m = np.zeros_like(p)
    v = np.zeros_like(p)
    n = len(u)
    for s in range(1, steps + 1):
        i0 = ((s - 1) * batch) % n
        ub, tb = u[i0:i0 + batch], t[i0:i0 + batch]
        g = gradient(p, ub, tb, bf)
        if record is not None:
            record.append((s, g))
        p, m, v = adam_step(p, g, m, v, s, lr_at(lr, s, steps))
    return p
