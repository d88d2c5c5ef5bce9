"""Pins of the oracle's ADMM-PD form of the local-global iteration (the paper's
implementations are PD and ADMM-PD; the local step of the cited ADMM-PD method).

* its converged iterate is stationary for the backward-Euler incremental potential of
  the hyperelastic energy itself (directional derivatives by central differences vanish
  relative to those at q^0), while PD's converged iterate, which minimises the
  quadratic-penalty relaxation, is not (stable Neo-Hookean bar);
* for ARAP, where the relaxation is the energy, PD and ADMM-PD (with ARAP's energy and
  its prox in the ADMM form) reach the same stationary iterate;
* the potential vanishes at rest.
"""
import numpy as np
import pytest

from oracle.sim import OracleSim
from paper_2503_15078_amd import scenes


def _converged(model, form, iters):
    sc = scenes.twist_bar(0, model=model, E=1e5, nu=0.3, nodes=(8, 3, 3), frames=40, press=0.0, ground=False)
    o = OracleSim(sc, lg_form=form)
    o.step(12, iters=10)
    q_t = o.q.copy()
    q_pred = o.predict(q_t, o.v)
    t_next = o.t + o.h
    fc = o.contacts_from_keys([], [], q_t)
    o.dual = None
    q, lam = q_pred.copy(), np.zeros((0, 3))
    for _ in range(iters):
        q, lam, _ = o.iterate(fc, q, lam, q_t, q_pred, t_next)
    return o, q_pred, t_next, q


def _stationarity(o, q_pred, t_next, q, seed=0):
    rng = np.random.default_rng(seed)
    f = lambda x: o.potential(x, q_pred, t_next)
    eps = 1e-7
    worst = 0.0
    for _ in range(3):
        d = rng.standard_normal(q.shape)
        d0 = (f(q_pred + eps * d) - f(q_pred - eps * d)) / (2 * eps)
        d1 = (f(q + eps * d) - f(q - eps * d)) / (2 * eps)
        worst = max(worst, abs(d1 / d0))
    return worst


def test_admm_is_stationary_for_the_potential_pd_is_not():
    o, qp, tn, q = _converged(scenes.MODEL_SNH, "admm", 400)
    r_admm = _stationarity(o, qp, tn, q)
    o, qp, tn, q = _converged(scenes.MODEL_SNH, "pd", 400)
    r_pd = _stationarity(o, qp, tn, q)
    print(f"stationarity ratio ADMM-PD {r_admm:.2e}, PD {r_pd:.2e}")
    assert r_admm <= 1e-8
    assert r_pd >= 1e-5


def test_arap_pd_and_admm_agree():
    """ARAP in ADMM form uses its energy mu |F - R|^2 (prox (sigma + 1) / 2); both forms
    then converge to stationary points of the ARAP potential, the same one to 1e-4 of
    the frame's displacement."""
    o, qp, tn, q_pd = _converged(scenes.MODEL_ARAP, "pd", 300)
    o2, _, _, q_admm = _converged(scenes.MODEL_ARAP, "admm", 300)
    assert np.abs(q_pd - q_admm).max() <= 1e-4 * np.abs(q_pd - qp).max()
    assert _stationarity(o, qp, tn, q_pd) <= 1e-8
    assert _stationarity(o2, qp, tn, q_admm) <= 1e-7


def test_potential_zero_at_rest():
    sc = scenes.incline_block(mu=0.5, theta_deg=0.0, nodes=3, E=1e5, model=scenes.MODEL_COROT)
    sc.gravity = np.zeros(3)
    o = OracleSim(sc)
    q = np.asarray(sc.rest, np.float64)
    assert abs(o.potential(q, q, 0.01)) <= 1e-20
