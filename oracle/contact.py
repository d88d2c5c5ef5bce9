"""Contacts: obstacle distances, frames, Fischer-Burmeister and minimum-map terms, NCP
residual (FP64).

Paper: Sec. 3.2 (linearised constraints along n and tangents f built by
Gram-Schmidt; Signorini-Coulomb conditions), App. A (constraint
linearisation; interpenetration computed from positions only:
delta_n = H_n q - d_n, h delta_dot_f = H_f (q - q_t) - h d_f), App. B
(Fischer-Burmeister and minimum-map NCP functions and their derivatives), Sec. 5.4
(complementarity preconditioner r from the Delassus diagonal, or from the mass
inverse as in the comparison of Sec. 7, stick-sliding test).

Readings where the paper is silent:
* detection: pair (v, o) is a contact iff min(sdf_o(x_t), sdf_o(x~)) < margin,
  evaluated in float64 with plain IEEE operations in a fixed order; normal n
  and closest point p^ are taken at x_t; d_n = n . p^;
* tangents: f1 = normalise(e_k - (e_k . n) n) with k = argmin_i |n_i| (lowest
  index on ties), f2 = n x f1;
* canonical contact order: (node id, obstacle id);
* FB at rho = 0 uses the generalised-Jacobian element omega_n = 1 - 1/sqrt 2,
  E_n = (1 - 1/sqrt 2) r_n;
* friction E_f with a zero denominator: 0/0 (s = 0 and lambda_f = 0 at a first
  touch) gives E_f = 0 (stick); a non-zero numerator (infinite compliance) and
  mu = 0 (a cone that is the single point lambda_f = 0) make the friction rows
  inactive, as for lambda_n <= 0 (omega_f = 0, E_f = 1, which drives lambda_f to 0);
* the friction cone is isotropic, E_f is one scalar for both tangent rows.
"""
from __future__ import annotations

import math

import numpy as np

HALFSPACE, BOX, CYLINDER, BINDING = 0, 1, 2, 3
INV_SQRT2 = 1.0 / math.sqrt(2.0)


def sdf_normal(ob_type, geom, x):
    """Signed distance and outward unit normal of one obstacle at one point (floats).

    Written with scalar IEEE operations in a fixed order so that the result is
    reproducible bit for bit by any implementation that follows the same order.
    """
    x0, x1, x2 = float(x[0]), float(x[1]), float(x[2])
    g = [float(v) for v in geom]
    if ob_type == HALFSPACE:
        nn = math.sqrt(g[3] * g[3] + g[4] * g[4] + g[5] * g[5])
        n0, n1, n2 = g[3] / nn, g[4] / nn, g[5] / nn
        d = n0 * (x0 - g[0]) + n1 * (x1 - g[1]) + n2 * (x2 - g[2])
        return d, (n0, n1, n2)
    if ob_type == BOX:
        r = (x0 - g[0], x1 - g[1], x2 - g[2])
        q = (abs(r[0]) - g[3], abs(r[1]) - g[4], abs(r[2]) - g[5])
        sg = tuple(1.0 if ri >= 0.0 else -1.0 for ri in r)
        o = (max(q[0], 0.0), max(q[1], 0.0), max(q[2], 0.0))
        out = math.sqrt(o[0] * o[0] + o[1] * o[1] + o[2] * o[2])
        if out > 0.0:
            return out, (o[0] * sg[0] / out, o[1] * sg[1] / out, o[2] * sg[2] / out)
        ax = 0
        if q[1] > q[ax]:
            ax = 1
        if q[2] > q[ax]:
            ax = 2
        nrm = [0.0, 0.0, 0.0]
        nrm[ax] = sg[ax]
        return q[ax], tuple(nrm)
    if ob_type == CYLINDER:
        e0, e1, e2 = g[3] - g[0], g[4] - g[1], g[5] - g[2]
        L = math.sqrt(e0 * e0 + e1 * e1 + e2 * e2)
        u0, u1, u2 = e0 / L, e1 / L, e2 / L
        r0, r1, r2 = x0 - g[0], x1 - g[1], x2 - g[2]
        t = r0 * u0 + r1 * u1 + r2 * u2
        w0, w1, w2 = r0 - t * u0, r1 - t * u1, r2 - t * u2
        rho = math.sqrt(w0 * w0 + w1 * w1 + w2 * w2)
        dr = rho - g[6]
        if t < 0.0:
            da, s0, s1, s2 = -t, -u0, -u1, -u2
        else:
            da, s0, s1, s2 = t - L, u0, u1, u2
        if rho > 0.0:
            wh = (w0 / rho, w1 / rho, w2 / rho)
        else:
            wh = tangent_basis((u0, u1, u2))[0]
        if dr > 0.0 and da > 0.0:
            out = math.sqrt(dr * dr + da * da)
            return out, ((dr * wh[0] + da * s0) / out, (dr * wh[1] + da * s1) / out, (dr * wh[2] + da * s2) / out)
        if dr > 0.0:
            return dr, wh
        if da > 0.0:
            return da, (s0, s1, s2)
        if dr > da:
            return dr, wh
        return da, (s0, s1, s2)
    raise ValueError("unknown obstacle type")


def tangent_basis(n):
    """Gram-Schmidt tangents: f1 from the axis with the smallest |n_i|, f2 = n x f1."""
    n0, n1, n2 = n
    a = [abs(n0), abs(n1), abs(n2)]
    k = 0
    if a[1] < a[k]:
        k = 1
    if a[2] < a[k]:
        k = 2
    ek = [0.0, 0.0, 0.0]
    ek[k] = 1.0
    dot = n0 * ek[0] + n1 * ek[1] + n2 * ek[2]
    t0, t1, t2 = ek[0] - dot * n0, ek[1] - dot * n1, ek[2] - dot * n2
    tn = math.sqrt(t0 * t0 + t1 * t1 + t2 * t2)
    f1 = (t0 / tn, t1 / tn, t2 / tn)
    f2 = (n1 * f1[2] - n2 * f1[1], n2 * f1[0] - n0 * f1[2], n0 * f1[1] - n1 * f1[0])
    return f1, f2


def binding_frame(geom, x_t):
    """A bilateral (binding) constraint (Sec. 3.2, binding contact; App. A, bilateral items):
    geom = [p^ (3), direction c (3), compliance e, node].  Its row is n = c / |c| with the
    Gram-Schmidt tangents, d_b = n . p^, and its gap n . x_t - d_b; it is active at every
    frame for its node."""
    c = np.asarray(geom[3:6], np.float64)
    nrm = tuple(float(v) for v in c / math.sqrt(float(c @ c)))
    f1, f2 = tangent_basis(nrm)
    d_n = float(np.dot(nrm, np.asarray(geom[0:3], np.float64)))
    return nrm, f1, f2, d_n, float(np.dot(nrm, x_t)) - d_n


def binding_terms(delta_n, lam, comp):
    """Bilateral rows: phi_b = delta_b + e lambda_b with omega_b = 1, E_b = e (e = 0: hard;
    e > 0: a quadratic potential of stiffness 1/e), and the tangent rows inactive
    (omega = 0, E = 1, driving lambda_f to 0)."""
    phi_n = delta_n + comp * lam[:, 0]
    return phi_n, np.ones_like(delta_n), comp.copy()


def detect(q_t, q_pred, obstacles, margin):
    """Contact list in canonical (node, obstacle) order.

    Returns dict with keys: node (c,), obst (c,), C (c,3,3) rows n,f1,f2,
    d_n (c,), gap (c,) = sdf at x_t, mu (c,), uhat (c,3) obstacle velocity.
    """
    nodes, obs, frames, dn, gaps, mus, vels = [], [], [], [], [], [], []
    for v in range(len(q_t)):
        for o, ob in enumerate(obstacles):
            if ob.type == BINDING:
                if v != int(ob.geom[7]):
                    continue
                nrm, f1, f2, d_n, gap = binding_frame(ob.geom, q_t[v])
                nodes.append(v)
                obs.append(o)
                frames.append([nrm, f1, f2])
                dn.append(d_n)
                gaps.append(gap)
                mus.append(0.0)
                vels.append(np.zeros(3))
                continue
            d_t, nrm = sdf_normal(ob.type, ob.geom, q_t[v])
            d_p, _ = sdf_normal(ob.type, ob.geom, q_pred[v])
            if min(d_t, d_p) < margin:
                f1, f2 = tangent_basis(nrm)
                ph = q_t[v] - d_t * np.asarray(nrm)
                nodes.append(v)
                obs.append(o)
                frames.append([nrm, f1, f2])
                dn.append(float(np.dot(nrm, ph)))
                gaps.append(d_t)
                mus.append(ob.mu)
                vels.append(ob.vel)
    c = len(nodes)
    return dict(node=np.asarray(nodes, np.int64), obst=np.asarray(obs, np.int64),
                C=np.asarray(frames, np.float64).reshape(c, 3, 3), d_n=np.asarray(dn),
                gap=np.asarray(gaps), mu=np.asarray(mus, np.float64),
                uhat=np.asarray(vels, np.float64).reshape(c, 3))


def fb(a, b):
    """Fischer-Burmeister function a + b - sqrt(a^2 + b^2)."""
    return a + b - np.sqrt(a * a + b * b)


def normal_terms(delta_n, lam_n, r_n):
    """App. B FB normal row: phi_n, omega_n = dphi/d delta, E_n = dphi/d lambda."""
    rho = np.sqrt(delta_n * delta_n + r_n * r_n * lam_n * lam_n)
    phi = delta_n + r_n * lam_n - rho
    safe = rho > 0.0
    rs = np.where(safe, rho, 1.0)
    omega = np.where(safe, 1.0 - delta_n / rs, 1.0 - INV_SQRT2)
    E = np.where(safe, (1.0 - r_n * lam_n / rs) * r_n, (1.0 - INV_SQRT2) * r_n)
    return phi, omega, E


def friction_terms(vdot_f, lam_n, lam_f, r_f, mu):
    """App. B FB friction rows: omega_f, scalar E_f and phi_f = omega_f vdot_f + E_f lambda_f.

    vdot_f (c,2) tangential relative velocity, lam_f (c,2).
    """
    s = np.sqrt((vdot_f ** 2).sum(1))
    lf = np.sqrt((lam_f ** 2).sum(1))
    gamma = mu * lam_n - lf
    rho = np.sqrt(s * s + r_f * r_f * gamma * gamma)
    den = s + mu * r_f * lam_n - rho
    num = rho - r_f * gamma
    # inactive rows: lambda_n <= 0 (App. B), mu = 0 (the cone is the point lambda_f = 0),
    # or an infinite compliance (zero denominator, non-zero numerator)
    active = (lam_n > 0.0) & (mu > 0.0) & ~((den == 0.0) & (num != 0.0))
    with np.errstate(divide="ignore", invalid="ignore"):
        Ef_act = np.where(den != 0.0, num / np.where(den != 0.0, den, 1.0) * r_f, 0.0)
    omega = np.where(active, 1.0, 0.0)
    Ef = np.where(active, Ef_act, 1.0)
    phi = omega[:, None] * vdot_f + Ef[:, None] * lam_f
    return omega, Ef, phi


def normal_terms_minmap(delta_n, lam_n, r_n):
    """App. B minimum-map normal row: phi_n = delta_n with omega_n = 1, E_n = 0 where
    delta_n <= r_n lam_n (ties included), else phi_n = r_n lam_n with omega_n = 0, E_n = r_n."""
    first = delta_n <= r_n * lam_n
    phi = np.where(first, delta_n, r_n * lam_n)
    omega = np.where(first, 1.0, 0.0)
    E = np.where(first, 0.0, r_n)
    return phi, omega, E


def friction_terms_minmap(vdot_f, lam_n, lam_f, r_f, mu):
    """App. B minimum-map friction rows: phi_f = omega_f vdot_f + E_f lambda_f.

    lambda_n <= 0: omega_f = 0, E_f = 1 (drives lambda_f to 0).  lambda_n > 0: omega_f = 1
    and E_f = 0 while |vdot_f| <= r_f (mu lambda_n - |lambda_f|) (stick), else
    E_f = (|vdot_f| - r_f (mu lambda_n - |lambda_f|)) / (mu lambda_n) (slide).  Reading
    shared with the FB rows: mu = 0 (the cone is the point lambda_f = 0) is inactive.
    """
    s = np.sqrt((vdot_f ** 2).sum(1))
    lf = np.sqrt((lam_f ** 2).sum(1))
    gamma = mu * lam_n - lf
    active = (lam_n > 0.0) & (mu > 0.0)
    slide = s > r_f * gamma
    with np.errstate(divide="ignore", invalid="ignore"):
        Ef_slide = (s - r_f * gamma) / np.where(active, mu * lam_n, 1.0)
    Ef = np.where(active, np.where(slide, Ef_slide, 0.0), 1.0)
    omega = np.where(active, 1.0, 0.0)
    phi = omega[:, None] * vdot_f + Ef[:, None] * lam_f
    return omega, Ef, phi


def ncp_residual(delta_n, vdot_f, lam, r_n, r_f, mu, h, comp=None):
    """Max-norm NCP residual in metres (reading of the Signorini-Coulomb conditions).

    Per contact: |FB(delta_n, r_n lam_n)|; if lam_n > 0: h |FB(s, r_f gamma)| and,
    when |lam_f| > 0, h |vdot_f + s lam_f/|lam_f||; if lam_n <= 0: h r_f |lam_f|.
    """
    if len(delta_n) == 0:
        return 0.0
    lam_n = lam[:, 0]
    lam_f = lam[:, 1:]
    res = np.abs(fb(delta_n, r_n * lam_n))
    s = np.sqrt((vdot_f ** 2).sum(1))
    lf = np.sqrt((lam_f ** 2).sum(1))
    gamma = mu * lam_n - lf
    act = lam_n > 0.0
    t_act = h * np.abs(fb(s, r_f * gamma))
    with np.errstate(divide="ignore", invalid="ignore"):
        dirv = vdot_f + (s / np.where(lf > 0, lf, 1.0))[:, None] * lam_f
    e_dir = np.where(lf > 0, h * np.sqrt((dirv ** 2).sum(1)), 0.0)
    e_off = h * r_f * lf
    res = np.maximum(res, np.where(act, np.maximum(t_act, e_dir), e_off))
    if comp is not None:  # bilateral rows: |delta_b + e lambda_b| and the inactive tangents
        b = comp >= 0.0
        res = np.where(b, np.maximum(np.abs(delta_n + comp * lam_n), e_off), res)
    return float(res.max())
