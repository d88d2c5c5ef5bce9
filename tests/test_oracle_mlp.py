"""Pins of the FP64 warm-start network reference: its backward pass against central
differences of the loss, GELU against its defining integral form, bf16 rounding
against the bit pattern definition."""
import math

import numpy as np

from oracle import mlp


def _params(seed):
    rng = np.random.default_rng(seed)
    flat = rng.normal(0, 0.2, mlp.n_params())
    return mlp.unflatten(flat)


def test_gelu_definition():
    z = np.linspace(-4, 4, 41)
    # gelu(z) = z * P(N(0,1) <= z), Phi by numerical integration of the density
    grid = np.linspace(-12, 0, 200001)
    phi = np.exp(-0.5 * grid ** 2) / math.sqrt(2 * math.pi)
    base = np.trapezoid(phi, grid)
    Phi = []
    for zi in z:
        g = np.linspace(0, zi, 20001) if zi != 0 else np.zeros(2)
        Phi.append(base + (np.trapezoid(np.exp(-0.5 * g ** 2) / math.sqrt(2 * math.pi), g) if zi != 0 else 0.0))
    np.testing.assert_allclose(mlp.gelu(z), z * np.array(Phi), atol=1e-8)
    eps = 1e-6
    np.testing.assert_allclose(mlp.gelu_grad(z), (mlp.gelu(z + eps) - mlp.gelu(z - eps)) / (2 * eps), atol=1e-8)


def test_backward_matches_central_differences():
    rng = np.random.default_rng(0)
    p = _params(1)
    X = rng.normal(0, 1, (7, 12))
    T = rng.normal(0, 1, (7, 3))
    g = mlp.grad(p, X, T)
    flat = mlp.flatten(p)
    gflat = mlp.flatten(g)
    eps = 1e-6
    idx = rng.choice(len(flat), 300, replace=False)
    for i in idx:
        fp = flat.copy()
        fm = flat.copy()
        fp[i] += eps
        fm[i] -= eps
        fd = (mlp.loss(mlp.unflatten(fp), X, T) - mlp.loss(mlp.unflatten(fm), X, T)) / (2 * eps)
        assert abs(fd - gflat[i]) <= 1e-6 * max(1.0, abs(fd)), (i, fd, gflat[i])


def test_padding_is_inert():
    rng = np.random.default_rng(2)
    p = _params(3)
    X = rng.normal(0, 1, (5, 12))
    y1, _ = mlp.forward(p, X)
    p2 = {k: v.copy() for k, v in p.items()}
    p2["W1"][:, 12:] = 123.0          # multiplies zero padding
    p2["W3"][3:, :] = -7.0            # rows not part of the output
    y2, _ = mlp.forward(p2, X)
    np.testing.assert_allclose(y1, y2, atol=0)


def test_bf16_round():
    # bf16 spacing at 1 is 2^-7: 1 + 2^-8 ties down to even 1.0, 1 + 3*2^-8 ties up to 1 + 2^-6
    vals = np.array([1.0, 1.00390625, 1.01171875, -3.14159, 1e-3, 65504.0])
    r = mlp.bf16_round(vals)
    bits = r.astype(np.float32).view(np.uint32)
    assert np.all(bits & 0xFFFF == 0)
    assert r[0] == 1.0 and r[1] == 1.0 and r[2] == 1.015625
    assert np.all(np.abs(r - vals) <= np.abs(vals) * 2 ** -8)
