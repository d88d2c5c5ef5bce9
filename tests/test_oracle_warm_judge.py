"""Pins of the oracle's judge of start impulses (OracleSim.linearized_residual) and of
the learned candidate's projection (oracle.mlp.learned_impulse).

The judge scores impulses by the NCP residual they leave in the frame start's linear
contact problem, x_v = q~_v + h^2 sum_k K_jk C_k^T lambda_k (Sec. 5.3).  It is pinned by
what fixes it independently of its own formula: every brute-force solution of that
linear problem (mode enumeration, oracle.brute_ncp) scores zero while the zero start
does not, and a single frictionless contact has closed-form scores: 2|g| at lambda = 0,
|g|/sqrt 2 at half the closing impulse, 0 at -g / (h^2 K_jj)."""
import math

import numpy as np
import pytest

from oracle import brute_ncp
from oracle import mlp as omlp
from oracle.sim import OracleSim
from paper_2503_15078_amd import scenes


def _problem(nodes, mu, seed):
    rest, tets = scenes.voxel_mesh(np.ones((2, 2, 2), bool), 0.025)
    ground = scenes.Obstacle.make(0, [0, 0, 0, 0, 0, 1], mu)
    sc = scenes.Scene("p", rest, tets, 1, 1e5, 0.3, 1000.0, 0.01, np.zeros(3), [ground], 0.006, 1, 10, 1)
    o = OracleSim(sc)
    rng = np.random.default_rng(seed)
    q_t = rest.copy()
    push = np.array([rng.uniform(-0.3, 0.3), rng.uniform(-0.3, 0.3), -0.5])
    q_pred = q_t + o.h * push + o.h * o.h * rng.standard_normal(q_t.shape) * 0.2
    fc = o.contacts_from_keys(np.array(nodes), np.zeros(len(nodes), np.int64), q_t)
    return o, fc, q_t, q_pred


@pytest.mark.parametrize("nodes,mu,seed", [
    ([0], 0.0, 0), ([0, 2], 0.0, 1), ([0, 2, 6], 0.0, 2),
    ([0], 0.5, 3), ([0, 8], 0.3, 4), ([0, 2, 18], 0.8, 5), ([2, 6], 0.1, 6),
])
def test_brute_force_solutions_score_zero(nodes, mu, seed):
    o, fc, q_t, q_pred = _problem(nodes, mu, seed)
    h = o.h
    Hu = o.H(fc, q_pred)
    a = np.empty((fc.c, 3))
    a[:, 0] = Hu[:, 0] - fc.d_n
    a[:, 1:] = Hu[:, 1:] - np.einsum("jai,ji->ja", fc.C[:, 1:], q_t[fc.node]) - h * fc.d_f
    sols = brute_ncp.solve_all(a.reshape(-1), h * h * fc.W, fc.mu)
    assert len(sols) >= 1
    gap0 = np.abs(a[:, 0]).max()
    for lam in sols:
        lam = lam.reshape(-1, 3).copy()
        # an open contact's impulse is zero; the enumeration's linear solves leave ~1e-38
        lam[np.abs(lam).max(1) <= 1e-12 * np.abs(lam).max()] = 0.0
        assert o.linearized_residual(fc, q_t, q_pred, lam) <= 1e-9 * max(1.0, gap0 / 1e-3)
    # the zero start leaves the penetration of the predicted state: not a solution
    assert o.linearized_residual(fc, q_t, q_pred, np.zeros((fc.c, 3))) >= 2.0 * max(0.0, -a[:, 0].min()) - 1e-15


def test_single_frictionless_contact_closed_form():
    o, fc, q_t, q_pred = _problem([0], 0.0, 11)
    g = float(fc.C[0, 0] @ q_pred[0] - fc.d_n[0])
    assert g < -1e-4
    kjj = fc.K[0, 0]
    close = -g / (o.h * o.h * kjj)
    score = lambda ln: o.linearized_residual(fc, q_t, q_pred, np.array([[ln, 0.0, 0.0]]))
    assert abs(score(0.0) - 2.0 * abs(g)) <= 1e-15
    assert abs(score(0.5 * close) - abs(g) / math.sqrt(2.0)) <= 1e-15
    assert score(close) <= 1e-15
    # the sign of the displacement matters: pulling instead of pushing leaves 2|g| + ...
    assert score(-close) > 2.0 * abs(g)


def test_learned_impulse_projection_and_fallbacks():
    K = np.array([2.0, 2.0, 2.0, 2.0, 2.0])
    h, ell = 0.01, 0.02
    scale = ell / (h * h * 2.0)            # lambda = y * scale
    mu = np.array([0.5, 0.5, 0.5, 0.5, 0.5])
    plain = np.arange(15, dtype=float).reshape(5, 3) * 0.1
    y = np.array([[1.0, 0.1, 0.0],          # inside the cone: kept as is
                  [1.0, 3.0, 4.0],          # outside: friction scaled to mu lambda_n
                  [-1.0, 0.2, 0.0],         # negative normal: 0, friction scaled to 0
                  [np.nan, 0.0, 0.0],       # not finite: plain start
                  [1.0, 0.0, 0.0]])
    comp = np.array([-1.0, -1.0, -1.0, -1.0, 0.0])  # last row bilateral: plain start
    lam = omlp.learned_impulse(y, K, h, ell, mu, plain, comp)
    np.testing.assert_allclose(lam[0], y[0] * scale, rtol=1e-15)
    assert lam[1, 0] == y[1, 0] * scale
    np.testing.assert_allclose(np.linalg.norm(lam[1, 1:]), 0.5 * lam[1, 0], rtol=1e-15)
    np.testing.assert_allclose(lam[1, 1:] / np.linalg.norm(lam[1, 1:]), [0.6, 0.8], rtol=1e-15)
    np.testing.assert_array_equal(lam[2], [0.0, 0.0, 0.0])
    np.testing.assert_array_equal(lam[3], plain[3])
    np.testing.assert_array_equal(lam[4], plain[4])
    # persisting-contacts mode: a contact whose plain start is zero keeps it
    plain2 = plain.copy()
    plain2[0] = 0.0
    lam2 = omlp.learned_impulse(y, K, h, ell, mu, plain2, comp, persist=True)
    np.testing.assert_array_equal(lam2[0], [0.0, 0.0, 0.0])
    np.testing.assert_array_equal(lam2[1], lam[1])
