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


def test_mean_edge_length_of_one_voxel():
    """A unit voxel split into 5 tets: four corner tets with three unit edges and three
    face diagonals each, a central tet with six face diagonals: mean (12 + 18 sqrt 2)/30."""
    from paper_2503_15078_amd import scenes
    rest, tets = scenes.voxel_mesh(np.ones((1, 1, 1), bool), 1.0)
    assert len(tets) == 5
    assert abs(mlp.mean_edge_length(rest, tets) - (12 + 18 * math.sqrt(2)) / 30) < 1e-12


def test_features_worked_example():
    """A node above the plane z = 0 (normal +z, d_n = 0), moving with v = (0.2, 0, -0.1)
    m/s, h = 0.01, l = 0.025, K_jj = 50, previous impulse (2, 0.5, 0) in its frame."""
    h, ell, kjj = 0.01, 0.025, 50.0
    n = np.array([0.0, 0.0, 1.0])
    f1, f2 = np.array([1.0, 0.0, 0.0]), np.array([0.0, 1.0, 0.0])
    C = np.array([[n, f1, f2]])
    q_pred = np.array([[0.3, -0.2, 0.003]])
    v = np.array([[0.2, 0.0, -0.1]])
    F = mlp.features(C, [0.0], [0.4], [0], q_pred, v, np.zeros((1, 3)), [[2.0, 0.5, 0.0]], [kjj], h, ell)
    np.testing.assert_allclose(F[0, 0], 0.003 / ell)
    np.testing.assert_allclose(F[0, 1:4], n)
    np.testing.assert_allclose(F[0, 4:7], [h * -0.1 / ell, h * 0.2 / ell, 0.0])
    np.testing.assert_allclose(F[0, 7:10], [h * h * kjj * 2.0 / ell, h * h * kjj * 0.5 / ell, 0.0])
    np.testing.assert_allclose(F[0, 10], math.log(kjj))
    assert F[0, 11] == 0.4 and np.all(F[0, 12:] == 0)
    # a moving obstacle: only the relative velocity enters
    F2 = mlp.features(C, [0.0], [0.4], [0], q_pred, v + 0.7, np.full((1, 3), 0.7), [[2.0, 0.5, 0.0]], [kjj], h, ell)
    np.testing.assert_allclose(F2, F, atol=1e-15)
    # targets invert the impulse scaling
    np.testing.assert_allclose(mlp.targets([[2.0, 0.5, 0.0]], [kjj], h, ell), F[:, 7:10])


def test_adam_first_step_and_constant_gradient():
    """Bias correction makes every Adam step move a parameter by lr |g| / (|g| + eps)
    against its gradient sign while the gradient is constant."""
    rng = np.random.default_rng(4)
    p = rng.normal(0, 1, 50)
    g = rng.normal(0, 1, 50)
    m = np.zeros(50)
    v = np.zeros(50)
    lr = 1e-3
    q = p.copy()
    for t in range(1, 6):
        q_new, m, v = mlp.adam_step(q, g, m, v, t, lr)
        np.testing.assert_allclose(q - q_new, lr * g / (np.abs(g) + 1e-8), rtol=1e-9, atol=1e-15)
        q = q_new


def test_bf16_rounding_points_reduce_to_the_exact_network(monkeypatch):
    """Without rounding (bf16_round the identity) the device-precision forms are the
    exact network and its gradient; with rounding the output moves by at most the
    first-order effect of the two activation roundings."""
    rng = np.random.default_rng(5)
    p = _params(6)
    X = rng.normal(0, 1, (9, 12))
    T = rng.normal(0, 1, (9, 3))
    y, (x, z1, h1, z2, h2) = mlp.forward(p, X)
    yb, _ = mlp.forward_bf16(p, X)
    W2, W3 = np.abs(p["W2"]), np.abs(p["W3"])
    u = 2.0 ** -8
    bound = (np.abs(h2) @ W3.T + (np.abs(mlp.gelu_grad(z2)) * ((np.abs(h1) + np.abs(x) @ np.abs(p["W1"]).T) @ W2.T))
             @ W3.T) * u * 2
    assert np.all(np.abs(yb - y) <= bound[:, :3] + 1e-12)
    monkeypatch.setattr(mlp, "bf16_round", lambda a: np.asarray(a, np.float64))
    y2, _ = mlp.forward_bf16(p, X)
    np.testing.assert_allclose(y2, y, rtol=0, atol=1e-13)
    g = mlp.grad(p, X, T)
    g2 = mlp.grad_bf16(p, X, T)
    for k in mlp.ORDER:
        np.testing.assert_allclose(g2[k], g[k], rtol=0, atol=1e-13)
