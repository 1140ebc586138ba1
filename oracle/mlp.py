"""FP64 CPU reference of the learned-initialiser MLP -- TEST INFRASTRUCTURE ONLY.

A plain numpy forward pass and hand-written backpropagation of the
4 -> 64 -> 64 -> 64 -> 1 network with SiLU activations and a mean-squared-error
loss.  The GPU FP32 training kernels are checked against these gradients, and
these gradients are checked against central finite differences of the loss.

Flat parameter layout (shared by both sides as an interface, 8705 values):
W1 (64 x 4, row = output), b1 (64), W2 (64 x 64), b2 (64), W3 (64 x 64),
b3 (64), W4 (1 x 64), b4 (1).
"""
from __future__ import annotations

import numpy as np

SIZES = [4, 64, 64, 64, 1]


def n_params() -> int:
    return sum(SIZES[i + 1] * SIZES[i] + SIZES[i + 1] for i in range(len(SIZES) - 1))


def unpack(theta):
    theta = np.asarray(theta, dtype=np.float64)
    out, o = [], 0
    for i in range(len(SIZES) - 1):
        fi, fo = SIZES[i], SIZES[i + 1]
        W = theta[o:o + fo * fi].reshape(fo, fi); o += fo * fi
        b = theta[o:o + fo]; o += fo
        out.append((W, b))
    assert o == theta.size
    return out


def silu(z):
    return z / (1.0 + np.exp(-z))


def dsilu(z):
    s = 1.0 / (1.0 + np.exp(-z))
    return s * (1.0 + z * (1.0 - s))


def forward(theta, X):
    """X: (B, 4) -> y (B,), cache of pre-activations and activations."""
    layers = unpack(theta)
    h = np.asarray(X, dtype=np.float64)
    zs, hs = [], [h]
    for li, (W, b) in enumerate(layers):
        z = h @ W.T + b
        zs.append(z)
        h = silu(z) if li < len(layers) - 1 else z
        hs.append(h)
    return h[:, 0], (zs, hs)


def loss(theta, X, t):
    y, _ = forward(theta, X)
    return float(np.mean((y - t) ** 2))


def grad(theta, X, t):
    """Gradient of the mean-squared error by backpropagation (flat layout)."""
    layers = unpack(theta)
    y, (zs, hs) = forward(theta, X)
    B = y.shape[0]
    delta = (2.0 / B) * (y - np.asarray(t, dtype=np.float64))[:, None]   # dL/dz of the output layer
    grads = [None] * len(layers)
    for li in range(len(layers) - 1, -1, -1):
        W, _ = layers[li]
        gW = delta.T @ hs[li]
        gb = delta.sum(axis=0)
        grads[li] = (gW, gb)
        if li > 0:
            delta = (delta @ W) * dsilu(zs[li - 1])
    return np.concatenate([np.concatenate([gW.ravel(), gb]) for gW, gb in grads])


def init_params(seed: int = 0) -> np.ndarray:
    """He-style uniform initialisation (for tests and training starts)."""
    rng = np.random.default_rng(seed)
    parts = []
    for i in range(len(SIZES) - 1):
        fi, fo = SIZES[i], SIZES[i + 1]
        lim = np.sqrt(6.0 / fi)
        parts.append(rng.uniform(-lim, lim, fo * fi) * (0.5 if i == len(SIZES) - 2 else 1.0))
        parts.append(np.zeros(fo))
    return np.concatenate(parts)
