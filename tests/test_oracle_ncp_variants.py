"""Pins of the oracle's minimum-map rows (App. B) and of the mass-inverse
complementarity preconditioner (the alternative that Sec. 7's stick-sliding test
compares against, Sec. 5.4).

* min-map normal row: the two cases and the tie at delta_n = r_n lambda_n, written out;
  phi_n vanishes exactly on the complementarity set {delta >= 0, lambda >= 0,
  delta lambda = 0} and nowhere else (sampled), as the FB row does;
* min-map friction rows: zero on Coulomb's solutions (sticking inside the cone at rest,
  sliding with lambda_f = -mu lambda_n vdot_f / |vdot_f|), non-zero off them, inactive
  rows for lambda_n <= 0 or mu = 0;
* mass preconditioner: for a one-voxel block split into five tets, the bottom nodes
  carry 5/24 or 1/24 of the block's mass (central tet of volume 1/3 plus three corner
  tets of 1/6, or one corner tet), so r_n = h^2 / m_v takes exactly those two values;
* stick-sliding test (10 degree slope, E = 1e8, 10 L-G and 24 CR iterations): with the
  mass-inverse preconditioner the block still sticks at mu* - 0.05 and slides at
  mu* - 0.1, the paper's 0.1 precision; the min-map rows with the Delassus
  preconditioner slide at mu* - 0.05 and stick at mu* + 0.01.
"""
import json
import math
import os

import numpy as np
import pytest

from oracle import contact as ct
from oracle.sim import OracleSim
from paper_2503_15078_amd import scenes

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def test_minmap_normal_cases_and_tie():
    d = np.array([-0.02, 0.03, 0.01, 0.0])
    lam = np.array([1.0, 1.0, 2.0, 0.0])
    r = np.array([0.01, 0.01, 0.005, 0.3])
    phi, om, E = ct.normal_terms_minmap(d, lam, r)
    np.testing.assert_array_equal(phi, [-0.02, 0.01, 0.01, 0.0])
    np.testing.assert_array_equal(om, [1.0, 0.0, 1.0, 1.0])
    np.testing.assert_array_equal(E, [0.0, 0.01, 0.0, 0.0])


def test_minmap_normal_zero_set():
    rng = np.random.default_rng(0)
    k = 2000
    r = rng.uniform(1e-3, 1.0, k)
    # on the complementarity set
    d_on = np.where(rng.random(k) < 0.5, 0.0, rng.uniform(0, 1, k))
    l_on = np.where(d_on == 0.0, rng.uniform(0, 1, k), 0.0)
    phi_on, _, _ = ct.normal_terms_minmap(d_on, l_on, r)
    np.testing.assert_array_equal(phi_on, 0.0)
    # off it: penetration, negative impulse, or both positive
    d_off = rng.uniform(-1, 1, k)
    l_off = rng.uniform(-1, 1, k)
    off = ~(((d_off >= 0) & (l_off >= 0)) & ((d_off == 0) | (l_off == 0)))
    phi_off, _, _ = ct.normal_terms_minmap(d_off[off], l_off[off], r[off])
    assert np.all(phi_off != 0.0)
    # the FB row vanishes on the same set
    phi_fb, _, _ = ct.normal_terms(d_on, l_on, r)
    assert np.abs(phi_fb).max() <= 1e-15


def test_minmap_friction_on_and_off_coulomb_solutions():
    mu = np.array([0.5, 0.5, 0.5, 0.5, 0.0])
    lam_n = np.array([1.0, 2.0, 1.0, 0.0, 1.0])
    r_f = np.full(5, 0.3)
    v = np.array([[0.0, 0.0], [0.2, -0.1], [0.2, -0.1], [0.1, 0.0], [0.1, 0.0]])
    lf = np.zeros((5, 2))
    lf[0] = [0.1, -0.05]                                   # stick, inside the cone
    lf[1] = -mu[1] * lam_n[1] * v[1] / np.linalg.norm(v[1])  # sliding solution
    lf[2] = [0.1, 0.1]                                     # moving, not opposing: no solution
    lf[3] = [0.2, 0.0]                                     # lambda_n = 0: inactive
    lf[4] = [0.2, 0.0]                                     # mu = 0: inactive
    om, Ef, phi = ct.friction_terms_minmap(v, lam_n, lf, r_f, mu)
    np.testing.assert_array_equal(om, [1.0, 1.0, 1.0, 0.0, 0.0])
    assert Ef[0] == 0.0 and np.abs(phi[0]).max() == 0.0
    # slide: E_f = |v| / (mu lambda_n) (the cone boundary: mu lambda_n - |lambda_f| = 0)
    assert abs(Ef[1] - np.linalg.norm(v[1]) / (mu[1] * lam_n[1])) <= 1e-15
    assert np.abs(phi[1]).max() <= 1e-15
    assert np.abs(phi[2]).max() > 1e-3
    np.testing.assert_array_equal(Ef[3:], [1.0, 1.0])
    np.testing.assert_array_equal(phi[3:], lf[3:])


def test_mass_preconditioner_closed_form():
    sc = scenes.incline_block(mu=0.5, nodes=2, E=1e8)
    o = OracleSim(sc, precond="mass")
    q_t, q_pred, fc, lam = o.begin_frame()
    assert fc.c == 4
    m_block = sc.rho * 0.1 ** 3
    expect = sorted([o.h ** 2 / (m_block * 5 / 24)] * 2 + [o.h ** 2 / (m_block / 24)] * 2)
    np.testing.assert_allclose(sorted(fc.r_n), expect, rtol=1e-12)
    np.testing.assert_allclose(np.asarray(fc.r_f) * o.h, fc.r_n, rtol=1e-12)
    # the method's preconditioner, the Delassus diagonal, is smaller: the stiffness
    # rather than the mass dominates A's diagonal for E = 1e8 (Sec. 5.4)
    od = OracleSim(sc)
    fcd = od.begin_frame()[2]
    assert np.all(fcd.r_n < 0.25 * fc.r_n)


def _incline_velocity(offset, ncp, precond):
    with open(os.path.join(GOLDEN, "paper_values.json")) as f:
        g = json.load(f)["stick_slide_threshold"]
    frames = 40
    mu = g["mu_star"] + offset
    sc = scenes.incline_block(mu=mu, theta_deg=g["theta_deg"], E=g["E"], nodes=2,
                              iters=g["lg_iters"], cr_iters=g["cr_iters"], frames=frames)
    o = OracleSim(sc, ncp=ncp, precond=precond)
    o.step(frames)
    th = math.radians(g["theta_deg"])
    v_an = 9.81 * (math.sin(th) - mu * math.cos(th)) * frames * o.h
    return float(np.mean(o.v[:, 0])), v_an


def test_mass_preconditioner_precision_is_coarse():
    """Sec. 7: the mass-inverse preconditioner captures the threshold only to about 0.1."""
    v, v_an = _incline_velocity(-0.05, "fb", "mass")
    assert abs(v) < 0.01 * v_an          # should slide, sticks
    v, v_an = _incline_velocity(-0.1, "fb", "mass")
    assert abs(v - v_an) < 0.1 * v_an    # slides at the analytic velocity


def test_minmap_delassus_incline():
    v, v_an = _incline_velocity(-0.05, "minmap", "delassus")
    assert abs(v - v_an) < 0.01 * v_an
    v, _ = _incline_velocity(+0.01, "minmap", "delassus")
    _, v_an = _incline_velocity(-0.01, "fb", "delassus")
    assert abs(v) < 0.01 * v_an
