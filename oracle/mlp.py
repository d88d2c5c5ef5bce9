"""FP64 reference of the learned warm-start network (test infrastructure).

The network maps 12 per-contact features to a 3-vector (a scaled impulse):
  z1 = W1 x + b1,  h1 = gelu(z1)      (128)
  z2 = W2 h1 + b2, h2 = gelu(z2)      (128)
  y  = W3 h2 + b3                      (3)
with the exact GELU, gelu(z) = z Phi(z), and the loss L = mean over samples and
outputs of (y - t)^2.  Parameters use the padded shapes of the GPU kernels:
W1 (128, 16) whose last 4 input columns multiply zero features, W3 (16, 128) whose
rows 3..15 are unused, b3 (16,).  Pins: the backward pass is checked against central
differences of the loss.
"""
from __future__ import annotations

import math

import numpy as np
from scipy.special import erf

SHAPES = {"W1": (128, 16), "b1": (128,), "W2": (128, 128), "b2": (128,), "W3": (16, 128), "b3": (16,)}
ORDER = ["W1", "b1", "W2", "b2", "W3", "b3"]


def n_params():
    return sum(int(np.prod(SHAPES[k])) for k in ORDER)


def unflatten(flat):
    out, o = {}, 0
    for k in ORDER:
        n = int(np.prod(SHAPES[k]))
        out[k] = np.asarray(flat[o:o + n], np.float64).reshape(SHAPES[k])
        o += n
    return out


def flatten(p):
    return np.concatenate([np.asarray(p[k], np.float64).reshape(-1) for k in ORDER])


def gelu(z):
    return 0.5 * z * (1.0 + erf(z / math.sqrt(2.0)))


def gelu_grad(z):
    return 0.5 * (1.0 + erf(z / math.sqrt(2.0))) + z * np.exp(-0.5 * z * z) / math.sqrt(2.0 * math.pi)


def pad_features(X):
    X = np.asarray(X, np.float64)
    out = np.zeros((len(X), 16))
    out[:, :X.shape[1]] = X
    return out


def forward(p, X):
    x = pad_features(X)
    z1 = x @ p["W1"].T + p["b1"]
    h1 = gelu(z1)
    z2 = h1 @ p["W2"].T + p["b2"]
    h2 = gelu(z2)
    y = h2 @ p["W3"].T + p["b3"]
    return y[:, :3], (x, z1, h1, z2, h2)


def loss(p, X, T):
    y, _ = forward(p, X)
    return float(np.mean((y - T) ** 2))


def grad(p, X, T):
    """Gradient of the mean-squared loss with respect to every parameter (FP64)."""
    y, (x, z1, h1, z2, h2) = forward(p, X)
    B = len(X)
    dy = np.zeros((B, 16))
    dy[:, :3] = 2.0 * (y - T) / (B * 3)
    g = {"W3": dy.T @ h2, "b3": dy.sum(0)}
    dh2 = dy @ p["W3"]
    dz2 = dh2 * gelu_grad(z2)
    g["W2"] = dz2.T @ h1
    g["b2"] = dz2.sum(0)
    dh1 = dz2 @ p["W2"]
    dz1 = dh1 * gelu_grad(z1)
    g["W1"] = dz1.T @ x
    g["b1"] = dz1.sum(0)
    return g


def bf16_round(a):
    """Round float64 values to bfloat16 (round to nearest even) and back."""
    a32 = np.asarray(a, np.float32)
    u = a32.view(np.uint32).astype(np.uint64)
    r = ((u + 0x7FFF + ((u >> 16) & 1)) >> 16) << 16
    return r.astype(np.uint32).view(np.float32).astype(np.float64)
