"""Pins of the oracle's contact path (App. A, App. B, Sec. 5.2-5.4, Sec. 7.5).

* signed distances / normals of each obstacle type against brute-force
  distances to sampled surface points;
* Gram-Schmidt tangent frames are orthonormal and right-handed;
* FB normal derivatives omega_n, E_n against central differences of phi_n;
* the FB friction compliance reduces to Coulomb's s/|lambda_f| on the cone
  and to 0 when sticking (App. B, the friction E_f expression);
* the Delassus K is symmetric PSD, K_jj is the entry of a dense A_n^-1, and
  W built from K and the frames equals the generic H A^-1 H^T (A = A_n (x) I3);
* the iteration converged on a fixed elastic right-hand side matches the
  brute-force NCP solution for 1-3 contacts, frictionless (exact LCP) and
  frictional;
* a frictionless block resting on the ground carries sum lambda_n = m g;
* a stiff block on a 10 degree incline sticks iff mu > tan 10 deg (Sec. 7.5).
"""
import json
import math
import os

import numpy as np
import pytest

from oracle import brute_ncp, contact as ct
from oracle.sim import OracleSim
from paper_2503_15078_amd import scenes

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _surface_samples(ob, rng, k=4000):
    t, g = ob.type, ob.geom
    if t == ct.BOX:
        c, hs = g[:3], g[3:6]
        pts = rng.uniform(-1, 1, (k, 3)) * hs
        ax = rng.integers(0, 3, k)
        sgn = rng.choice([-1.0, 1.0], k)
        pts[np.arange(k), ax] = sgn * hs[ax]
        return pts + c
    if t == ct.CYLINDER:
        a, b, r = g[:3], g[3:6], g[6]
        u = (b - a) / np.linalg.norm(b - a)
        e1 = np.cross(u, [1.0, 0.0, 0.0] if abs(u[0]) < 0.9 else [0.0, 1.0, 0.0])
        e1 /= np.linalg.norm(e1)
        e2 = np.cross(u, e1)
        th = rng.uniform(0, 2 * np.pi, k)
        L = np.linalg.norm(b - a)
        side = a + rng.uniform(0, L, (k, 1)) * u + r * (np.cos(th)[:, None] * e1 + np.sin(th)[:, None] * e2)
        rr = r * np.sqrt(rng.uniform(0, 1, k))
        cap = np.where(rng.uniform(size=(k, 1)) < 0.5, a, b) + rr[:, None] * (np.cos(th)[:, None] * e1 + np.sin(th)[:, None] * e2)
        return np.concatenate([side, cap])
    raise ValueError


@pytest.mark.parametrize("ob", [
    scenes.Obstacle.make(1, [0.1, -0.2, 0.05, 0.2, 0.1, 0.3], 0.3),
    scenes.Obstacle.make(2, [0.0, 0.0, 0.0, 0.1, 0.3, 0.2, 0.05], 0.3),
])
def test_sdf_against_sampled_surface(ob):
    rng = np.random.default_rng(0)
    surf = _surface_samples(ob, rng, 20000)
    for _ in range(40):
        x = rng.uniform(-0.6, 0.6, 3)
        d, nrm = ct.sdf_normal(ob.type, ob.geom, x)
        dist = np.min(np.linalg.norm(surf - x, axis=1))
        if d > 0:
            assert abs(d - dist) < 6e-3
            # gradient by central differences of the distance
            eps = 1e-6
            gfd = [(ct.sdf_normal(ob.type, ob.geom, x + eps * e)[0] - ct.sdf_normal(ob.type, ob.geom, x - eps * e)[0]) / (2 * eps) for e in np.eye(3)]
            np.testing.assert_allclose(gfd, nrm, atol=1e-6)
        else:
            assert abs(-d - dist) < 6e-3
        np.testing.assert_allclose(np.linalg.norm(nrm), 1.0, atol=1e-12)


def test_halfspace_sdf():
    ob = scenes.Obstacle.make(0, [0, 0, 1.0, 0, 0, 2.0], 0.1)
    d, n = ct.sdf_normal(ob.type, ob.geom, np.array([0.3, -4.0, 1.25]))
    assert abs(d - 0.25) < 1e-15 and n == (0.0, 0.0, 1.0)


def test_tangent_basis_orthonormal():
    rng = np.random.default_rng(1)
    for _ in range(200):
        n = rng.standard_normal(3)
        n /= np.linalg.norm(n)
        f1, f2 = ct.tangent_basis(tuple(n))
        C = np.array([n, f1, f2])
        np.testing.assert_allclose(C @ C.T, np.eye(3), atol=1e-14)
        assert np.linalg.det(C) > 0


def test_fb_normal_derivatives():
    rng = np.random.default_rng(2)
    d = rng.standard_normal(100) * 1e-3
    lam = rng.standard_normal(100)
    r = np.abs(rng.standard_normal(100)) * 1e-3
    phi, om, E = ct.normal_terms(d, lam, r)
    np.testing.assert_allclose(phi, ct.fb(d, r * lam), atol=1e-18)
    eps = 1e-9
    fd_d = (ct.normal_terms(d + eps, lam, r)[0] - ct.normal_terms(d - eps, lam, r)[0]) / (2 * eps)
    fd_l = (ct.normal_terms(d, lam + eps * 1e3, r)[0] - ct.normal_terms(d, lam - eps * 1e3, r)[0]) / (2 * eps * 1e3)
    np.testing.assert_allclose(om, fd_d, rtol=1e-5, atol=1e-7)
    np.testing.assert_allclose(E, fd_l, rtol=1e-5, atol=1e-12)
    # the zero case takes the generalised-Jacobian element
    _, om0, E0 = ct.normal_terms(np.zeros(1), np.zeros(1), np.ones(1) * 2.0)
    assert abs(om0[0] - (1 - 1 / math.sqrt(2))) < 1e-15 and abs(E0[0] - 2 * (1 - 1 / math.sqrt(2))) < 1e-15


def test_friction_compliance_limits():
    mu, r = 0.4, 0.7
    lam_n = np.array([2.0])
    # sliding on the cone: |lam_f| = mu lam_n, velocity opposite -> E_f = s/|lam_f|
    lf = np.array([[0.6, 0.8 * 0.0]]) * 0 + np.array([[mu * 2.0 * 0.6, mu * 2.0 * 0.8]])
    v = -0.37 * lf / np.linalg.norm(lf)
    om, Ef, phi = ct.friction_terms(v, lam_n, lf, np.array([r]), mu)
    np.testing.assert_allclose(Ef, 0.37 / (mu * 2.0), rtol=1e-12)
    np.testing.assert_allclose(phi, 0.0, atol=1e-14)
    # sticking strictly inside the cone with zero velocity -> E_f = 0
    om, Ef, phi = ct.friction_terms(np.zeros((1, 2)), lam_n, np.array([[0.1, 0.2]]), np.array([r]), mu)
    assert Ef[0] == 0.0 and om[0] == 1.0
    # first touch: s = 0, lam_f = 0 -> 0/0 -> E_f = 0 (stick)
    om, Ef, phi = ct.friction_terms(np.zeros((1, 2)), lam_n, np.zeros((1, 2)), np.array([r]), mu)
    assert Ef[0] == 0.0 and om[0] == 1.0
    # frictionless: rows inactive
    om, Ef, phi = ct.friction_terms(np.ones((1, 2)), lam_n, np.zeros((1, 2)), np.array([r]), 0.0)
    assert om[0] == 0.0 and Ef[0] == 1.0
    # inactive contact -> omega_f = 0, E_f = 1
    om, Ef, phi = ct.friction_terms(np.ones((1, 2)), np.array([-1.0]), np.ones((1, 2)), np.array([r]), mu)
    assert om[0] == 0.0 and Ef[0] == 1.0


def _small_problem(nodes, mu, seed):
    rest, tets = scenes.voxel_mesh(np.ones((2, 2, 2), bool), 0.025)
    ground = scenes.Obstacle.make(0, [0, 0, 0, 0, 0, 1], mu)
    sc = scenes.Scene("p", rest, tets, 1, 1e5, 0.3, 1000.0, 0.01, np.zeros(3), [ground], 0.006, 1, 10, 1)
    o = OracleSim(sc)
    rng = np.random.default_rng(seed)
    q_t = rest.copy()
    push = np.array([rng.uniform(-0.3, 0.3), rng.uniform(-0.3, 0.3), -0.5])
    u = q_t + o.h * push + o.h * o.h * rng.standard_normal(q_t.shape) * 0.2
    b = o.A @ u
    o.rhs = lambda q, qp, t: b
    fc = o.contacts_from_keys(np.array(nodes), np.zeros(len(nodes), np.int64), q_t)
    return o, fc, q_t, u


@pytest.mark.parametrize("nodes,mu,seed", [
    ([0], 0.0, 0), ([0, 2], 0.0, 1), ([0, 2, 6], 0.0, 2),
    ([0], 0.5, 3), ([0, 8], 0.3, 4), ([0, 2, 18], 0.8, 5), ([2, 6], 0.1, 6),
])
def test_converged_iteration_matches_brute_force(nodes, mu, seed):
    o, fc, q_t, u = _small_problem(nodes, mu, seed)
    h = o.h
    lam = np.zeros((fc.c, 3))
    q = u.copy()
    for _ in range(200):
        q, lam, _ = o.iterate(fc, q, lam, q_t, u, h, cr="exact")
    res = o.residual(fc, q, q_t, lam)
    assert res <= 1e-10
    Hu = o.H(fc, u)
    a = np.empty((fc.c, 3))
    a[:, 0] = Hu[:, 0] - fc.d_n
    a[:, 1:] = Hu[:, 1:] - np.einsum("jai,ji->ja", fc.C[:, 1:], q_t[fc.node]) - h * fc.d_f
    sols = brute_ncp.solve_all(a.reshape(-1), h * h * fc.W, fc.mu)
    assert len(sols) >= 1
    if len(sols) == 1:
        np.testing.assert_allclose(lam.reshape(-1), sols[0], rtol=1e-6, atol=1e-8 * np.abs(sols[0]).max())
    else:
        assert min(np.abs(lam.reshape(-1) - s).max() for s in sols) <= 1e-6 * np.abs(lam).max()


def test_delassus_properties():
    sc = scenes.cube_drop(0)
    o = OracleSim(sc)
    q_t = sc.rest.copy()
    nodes = np.array([0, 3, 7, 7, 30, 99])
    obst = np.array([0, 0, 0, 0, 0, 0])
    fc = o.contacts_from_keys(nodes, obst, q_t)
    K = fc.K
    np.testing.assert_allclose(K, K.T, atol=0)
    assert np.linalg.eigvalsh(K).min() > -1e-12 * np.abs(K).max()
    Ainv = np.linalg.inv(o.A.toarray())
    np.testing.assert_allclose(K, Ainv[np.ix_(nodes, nodes)], rtol=1e-10)
    H = np.zeros((3 * len(nodes), 3 * o.n))
    for j, v in enumerate(nodes):
        H[3 * j:3 * j + 3, 3 * v:3 * v + 3] = fc.C[j]
    A3 = np.kron(o.A.toarray(), np.eye(3))
    W = H @ np.linalg.solve(A3, H.T)
    np.testing.assert_allclose(fc.W, W, rtol=1e-9, atol=1e-12 * np.abs(W).max())
    np.testing.assert_allclose(fc.r_n, o.h ** 2 * np.diag(W)[0::3], rtol=1e-12)


def test_resting_frictionless_block_carries_weight():
    sc = scenes.incline_block(mu=0.0, theta_deg=0.0, E=1e5, iters=10, cr_iters=24)
    o = OracleSim(sc)
    st = None
    for _ in range(30):
        q_t, q_pred, fc, lam = o.begin_frame()
        q = q_pred.copy()
        for _ in range(10):
            q, lam, _ = o.iterate(fc, q, lam, q_t, q_pred, o.t + o.h)
        o.end_frame(q_t, q, fc, lam)
    np.testing.assert_allclose(lam[:, 0].sum(), o.mass.sum() * 9.81, rtol=1e-4)


@pytest.mark.parametrize("delta", [+0.01, -0.01])
def test_incline_stick_slide(delta):
    """Stick iff mu > tan(10 deg): after 40 frames with the paper's 10 L-G / 24 CR
    iterations, the sliding block (mu* - 0.01) moves at the analytic velocity
    g (sin - mu cos) t within 10%, the sticking block (mu* + 0.01) at under 1% of it."""
    with open(os.path.join(GOLDEN, "paper_values.json")) as f:
        g = json.load(f)["stick_slide_threshold"]
    mu_star = g["mu_star"]
    assert abs(mu_star - math.tan(math.radians(g["theta_deg"]))) < 1e-8
    th = math.radians(g["theta_deg"])
    frames = 40
    sc = scenes.incline_block(mu=mu_star + delta, theta_deg=g["theta_deg"], E=g["E"], nodes=2,
                              iters=g["lg_iters"], cr_iters=g["cr_iters"], frames=frames)
    o = OracleSim(sc)
    o.step(frames)
    m = o.mass
    v = ((m[:, None] * o.v).sum(0) / m.sum())[0]
    v_slide = 9.81 * (math.sin(th) - (mu_star - abs(delta)) * math.cos(th)) * frames * o.h
    if delta > 0:
        assert abs(v) < 0.01 * v_slide
    else:
        assert abs(v - v_slide) < 0.1 * v_slide


# ---- NCP residual (reading of the Signorini-Coulomb conditions, Sec. 3.2 and App. B) at
# states off the solution: each case isolates one term and states its value worked out by
# hand from the definitions (FB(a, b) = a + b - sqrt(a^2 + b^2), s = |vdot_f|,
# gamma = mu lambda_n - |lambda_f|), so a dropped term, a missing h or a wrong sign fails.
H_STEP = 0.01


def _res(dn, vf, lam, rn=0.5, rf=0.1, mu=0.5, comp=None):
    return ct.ncp_residual(np.array([dn], float), np.array([vf], float), np.array([lam], float),
                           np.array([rn]), np.array([rf]), np.array([mu]), H_STEP,
                           None if comp is None else np.array([comp], float))


def test_ncp_residual_normal_term():
    # penetration with no impulse: FB(-0.01, 0) = -0.01 - 0.01
    assert _res(-0.01, [0.0, 0.0], [0.0, 0.0, 0.0]) == pytest.approx(0.02, rel=1e-14)
    # separated with an impulse: FB(0.003, 0.5 * 0.008) = 0.007 - 0.005
    assert _res(0.003, [0.0, 0.0], [0.008, 0.0, 0.0]) == pytest.approx(0.002, rel=1e-12)
    # complementary pairs are zero
    assert _res(0.0, [0.0, 0.0], [0.01, 0.0, 0.0]) == 0.0
    assert _res(0.02, [0.0, 0.0], [0.0, 0.0, 0.0]) == 0.0


def test_ncp_residual_friction_fb_term():
    # active contact (delta_n = 0, lambda_n = 4 > 0), slip s = 0.5 inside the cone with no
    # friction impulse: h FB(0.5, r_f gamma) with r_f gamma = 0.1 * (0.5 * 4) = 0.2
    expect = H_STEP * (0.7 - math.sqrt(0.25 + 0.04))
    assert _res(0.0, [0.3, 0.4], [4.0, 0.0, 0.0]) == pytest.approx(expect, rel=1e-13)
    # sticking on the cone interior with zero slip: zero
    assert _res(0.0, [0.0, 0.0], [4.0, 0.5, -0.5]) == 0.0


def test_ncp_residual_direction_term():
    # sliding on the cone boundary (|lambda_f| = mu lambda_n = 1, so FB(s, 0) = 0), but the
    # friction impulse is perpendicular to the slip instead of opposing it:
    # h |vdot_f + s lambda_f / |lambda_f|| = h |(0, 0.5) + 0.5 (1, 0)| = h sqrt(0.5)
    assert _res(0.0, [0.0, 0.5], [2.0, 1.0, 0.0]) == pytest.approx(H_STEP * math.sqrt(0.5), rel=1e-13)
    # opposing the slip, as Coulomb's law requires: zero
    assert _res(0.0, [-0.5, 0.0], [2.0, 1.0, 0.0]) == 0.0


def test_ncp_residual_off_cone_term():
    # no normal impulse (separated, delta_n > 0) but a friction impulse: h r_f |lambda_f|
    assert _res(0.01, [0.2, 0.0], [0.0, 0.3, -0.4]) == pytest.approx(H_STEP * 0.1 * 0.5, rel=1e-13)
    # negative normal impulse also counts as inactive (and its FB term is its own value):
    # FB(0.01, 0.5 * -0.002) = 0.009 - sqrt(1e-4 + 1e-6)
    fbn = 0.009 - math.sqrt(1e-4 + 1e-6)
    got = _res(0.01, [0.0, 0.0], [-0.002, 0.3, -0.4])
    assert got == pytest.approx(max(abs(fbn), H_STEP * 0.1 * 0.5), rel=1e-12)


def test_ncp_residual_binding_row():
    # bilateral row of compliance e = 0.2: |delta_b + e lambda_b| = |0.01 - 0.2 * 0.01|, and
    # its tangent impulses are off-cone terms h r_f |lambda_f|
    assert _res(0.01, [0.0, 0.0], [-0.01, 0.0, 0.0], comp=0.2) == pytest.approx(0.008, rel=1e-12)
    assert _res(0.01, [0.0, 0.0], [-0.01, 0.0, 0.6], comp=0.2) == pytest.approx(0.008, rel=1e-12)
    assert _res(0.0, [0.0, 0.0], [0.0, 8.0, 6.0], comp=0.0) == pytest.approx(H_STEP * 0.1 * 10.0, rel=1e-13)
    # a hard binding (e = 0) pulled 0.01 off its line: |delta_b| (a unilateral row would
    # give |FB(-0.01, 0)| = 0.02)
    assert _res(-0.01, [0.0, 0.0], [0.0, 0.0, 0.0], comp=0.0) == pytest.approx(0.01, rel=1e-14)
    # the bilateral residual replaces the unilateral one (which would be 0.02 here)
    assert _res(-0.01, [0.0, 0.0], [0.05, 0.0, 0.0], comp=0.2) == pytest.approx(0.0, abs=1e-15)


def test_ncp_residual_is_the_max_over_contacts():
    dn = np.array([-0.01, 0.0, 0.01])
    vf = np.array([[0.0, 0.0], [0.0, 0.5], [0.2, 0.0]])
    lam = np.array([[0.0, 0.0, 0.0], [2.0, 1.0, 0.0], [0.0, 0.3, -0.4]])
    one = np.ones(3)
    got = ct.ncp_residual(dn, vf, lam, 0.5 * one, 0.1 * one, 0.5 * one, H_STEP)
    assert got == pytest.approx(0.02, rel=1e-14)
    got = ct.ncp_residual(dn[1:], vf[1:], lam[1:], 0.5 * one[1:], 0.1 * one[1:], 0.5 * one[1:], H_STEP)
    assert got == pytest.approx(H_STEP * math.sqrt(0.5), rel=1e-13)
