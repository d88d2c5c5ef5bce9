"""Pins of the oracle's local step (Eq. PD local) against the mathematics.

* psi on signed singular values equals psi evaluated from the invariants of F
  (two independent definitions; SNH, MR), and COROT equals mu |F - R|^2 +
  lam/2 (det F - 1)^2 with R the polar rotation;
* analytic gradient / Hessian of psi against central differences of psi;
* the prox minimiser is stationary, checked with central differences of psi;
* rest shape F = I gives p = I for every model;
* rotation-variant SVD reconstructs F with det U = det V = +1;
* ARAP's projection is the polar rotation of F.
"""
import numpy as np
import pytest
import scipy.linalg as sla

from oracle import material as mat

MODELS = [mat.COROT, mat.SNH, mat.MR]
MU, LAM = 3.4e5, 3.1e6


def rand_F(rng, m, spread=0.3, allow_inverted=False):
    F = np.eye(3)[None] + spread * rng.standard_normal((m, 3, 3))
    if not allow_inverted:
        d = np.linalg.det(F)
        F[d < 0, :, 0] *= -1.0
    return F


@pytest.mark.parametrize("model", [mat.SNH, mat.MR])
def test_energy_singular_values_matches_invariants(model):
    rng = np.random.default_rng(1)
    F = rand_F(rng, 200)
    U, s, Vt = mat.svd_rv(F)
    e1 = mat.energy(model, s, MU, LAM)
    e2 = mat.energy_from_F(model, F, MU, LAM)
    np.testing.assert_allclose(e1, e2, rtol=1e-10, atol=1e-6)


def test_corot_energy_matches_polar_definition():
    rng = np.random.default_rng(2)
    F = rand_F(rng, 50)
    _, s, _ = mat.svd_rv(F)
    e1 = mat.energy(mat.COROT, s, MU, LAM)
    e2 = []
    for Fi in F:
        R, _ = sla.polar(Fi)
        e2.append(MU * np.sum((Fi - R) ** 2) + 0.5 * LAM * (np.linalg.det(Fi) - 1.0) ** 2)
    np.testing.assert_allclose(e1, e2, rtol=1e-9, atol=1e-6)


@pytest.mark.parametrize("model", MODELS)
def test_gradient_hessian_central_differences(model):
    rng = np.random.default_rng(3)
    s = 1.0 + 0.3 * rng.standard_normal((40, 3))
    if model == mat.MR:
        s = np.abs(s) + 0.2          # away from the J clamp
    g, H = mat.grad_hess(model, s, MU, LAM)
    eps = 1e-6
    for i in range(3):
        dp = s.copy()
        dm = s.copy()
        dp[:, i] += eps
        dm[:, i] -= eps
        fd = (mat.energy(model, dp, MU, LAM) - mat.energy(model, dm, MU, LAM)) / (2 * eps)
        np.testing.assert_allclose(g[:, i], fd, rtol=1e-6, atol=1e-3 * MU * eps / eps * 1e-6)
        gp, _ = mat.grad_hess(model, dp, MU, LAM)
        gm, _ = mat.grad_hess(model, dm, MU, LAM)
        np.testing.assert_allclose(H[:, :, i], (gp - gm) / (2 * eps), rtol=1e-5, atol=1e-2)


@pytest.mark.parametrize("model", MODELS)
def test_prox_stationary_by_finite_differences(model):
    rng = np.random.default_rng(4)
    F = rand_F(rng, 100, spread=0.25, allow_inverted=(model != mat.MR))
    _, sig, _ = mat.svd_rv(F)
    k = 2 * MU + LAM
    s = mat.prox_singular(np.full(len(sig), model), sig, MU, LAM, k)
    eps = 1e-6

    def obj(x):
        return 0.5 * k * ((x - sig) ** 2).sum(1) + mat.energy(model, x, MU, LAM)

    for i in range(3):
        dp = s.copy()
        dm = s.copy()
        dp[:, i] += eps
        dm[:, i] -= eps
        fd = (obj(dp) - obj(dm)) / (2 * eps)
        assert np.max(np.abs(fd)) <= 1e-6 * k
    # and it is a minimiser along random directions
    for _ in range(5):
        d = rng.standard_normal(s.shape) * 1e-3
        assert np.all(obj(s + d) >= obj(s) - 1e-9 * k)


@pytest.mark.parametrize("model", [mat.ARAP] + MODELS)
def test_rest_shape_projects_to_identity(model):
    F = np.repeat(np.eye(3)[None], 7, axis=0)
    mu, lam = MU, LAM
    k = 2 * mu if model == mat.ARAP else 2 * mu + lam
    P = mat.local_step(np.full(7, model), F, mu, lam, k)
    np.testing.assert_allclose(P, F, atol=1e-12)


def test_svd_rotation_variant():
    rng = np.random.default_rng(5)
    F = rand_F(rng, 300, spread=0.8, allow_inverted=True)
    U, s, Vt = mat.svd_rv(F)
    np.testing.assert_allclose(np.einsum("tij,tj,tjk->tik", U, s, Vt), F, atol=1e-12)
    np.testing.assert_allclose(np.linalg.det(U), 1.0, atol=1e-12)
    np.testing.assert_allclose(np.linalg.det(Vt), 1.0, atol=1e-12)
    inv = np.linalg.det(F) < 0
    assert np.all((s[inv] < 0).sum(1) == 1)
    assert np.all(s[~inv] >= 0)


def test_arap_is_polar_rotation():
    rng = np.random.default_rng(6)
    F = rand_F(rng, 30)
    P = mat.local_step(np.full(30, mat.ARAP), F, MU, LAM, 2 * MU)
    for Fi, Pi in zip(F, P):
        R, _ = sla.polar(Fi)
        np.testing.assert_allclose(Pi, R, atol=1e-10)
