"""Hyperelastic energies on signed singular values and the local prox (FP64).

Paper: Eq. PD local, p_i = argmin_p (w_i/2)|p - G_i q|^2 + zeta_i(p).  For an
isotropic energy the minimiser shares the singular vectors of F = G_i q, so
with the rotation-variant SVD F = U diag(sigma) V^T (det U = det V = +1, the
smallest singular value negated when det F < 0) the prox reduces to

    s* = argmin_s (k/2)|s - sigma|^2 + psi(s),   p = U diag(s*) V^T,

after dividing by the tet volume (w = k V).  ARAP uses the SO(3) indicator,
so s* = (1, 1, 1).

The paper names its models without formulas; the energies below are the
readings used on both sides:
  COROT  psi = mu sum (s_i - 1)^2 + lam/2 (J - 1)^2
  SNH    psi = mu/2 (I_C - 3) + lam/2 (J - alpha)^2 - mu/2 log(I_C + 1),
         alpha = 1 + 3 mu / (4 lam)  (zero stress at F = I)
  MR     psi = c10 (J^-2/3 I1 - 3) + c01 (J^-4/3 I2 - 3) + kappa/2 (J - 1)^2,
         c10 = c01 = mu/4, kappa = lam + 2 mu / 3, J in the isochoric terms
         clamped below at 1e-4
with J = s0 s1 s2, I_C = I1 = sum s_i^2, I2 = sum_{i<j} s_i^2 s_j^2.

The paper solves the local problem with a small L-BFGS; this oracle uses
Newton with a shifted Hessian and Armijo backtracking from s = sigma, to
tight tolerance.  Pins: tests check psi on singular values against psi on F
invariants, gradients against central differences of psi, stationarity
of the returned s* by central differences, and s* = (1,1,1) at F = I.
"""
from __future__ import annotations

import numpy as np

ARAP, COROT, SNH, MR = 0, 1, 2, 3
J_CLAMP = 1e-4


def svd_rv(F):
    """Rotation-variant SVD of (m,3,3): U diag(s) Vt with det U = det V = +1."""
    U, s, Vt = np.linalg.svd(F)
    U = U.copy()
    s = s.copy()
    Vt = Vt.copy()
    neg = np.linalg.det(U) < 0
    U[neg, :, 2] *= -1.0
    s[neg, 2] *= -1.0
    neg = np.linalg.det(Vt) < 0
    Vt[neg, 2, :] *= -1.0
    s[neg, 2] *= -1.0
    return U, s, Vt


def _J_terms(s):
    J = s[:, 0] * s[:, 1] * s[:, 2]
    Ji = np.stack([s[:, 1] * s[:, 2], s[:, 0] * s[:, 2], s[:, 0] * s[:, 1]], axis=1)
    Jij = np.zeros(s.shape + (3,))
    Jij[:, 0, 1] = Jij[:, 1, 0] = s[:, 2]
    Jij[:, 0, 2] = Jij[:, 2, 0] = s[:, 1]
    Jij[:, 1, 2] = Jij[:, 2, 1] = s[:, 0]
    return J, Ji, Jij


def energy(model, s, mu, lam):
    """psi(s) per row; model, mu, lam broadcast over rows of s (m,3)."""
    s = np.asarray(s, dtype=np.float64)
    model = np.broadcast_to(model, s.shape[:1])
    mu = np.broadcast_to(mu, s.shape[:1]).astype(np.float64)
    lam = np.broadcast_to(lam, s.shape[:1]).astype(np.float64)
    J = s[:, 0] * s[:, 1] * s[:, 2]
    I1 = (s * s).sum(1)
    I2 = (s[:, 0] * s[:, 1]) ** 2 + (s[:, 0] * s[:, 2]) ** 2 + (s[:, 1] * s[:, 2]) ** 2
    out = np.zeros(len(s))
    c = model == COROT
    out[c] = mu[c] * ((s[c] - 1.0) ** 2).sum(1) + 0.5 * lam[c] * (J[c] - 1.0) ** 2
    c = model == SNH
    alpha = 1.0 + 0.75 * mu[c] / lam[c]
    out[c] = 0.5 * mu[c] * (I1[c] - 3.0) + 0.5 * lam[c] * (J[c] - alpha) ** 2 - 0.5 * mu[c] * np.log(I1[c] + 1.0)
    c = model == MR
    Jh = np.maximum(J[c], J_CLAMP)
    c10 = 0.25 * mu[c]
    kap = lam[c] + 2.0 * mu[c] / 3.0
    out[c] = c10 * (Jh ** (-2.0 / 3.0) * I1[c] - 3.0) + c10 * (Jh ** (-4.0 / 3.0) * I2[c] - 3.0) + 0.5 * kap * (J[c] - 1.0) ** 2
    return out


def energy_from_F(model, F, mu, lam):
    """psi evaluated from the invariants of F itself (no SVD); used as a pin."""
    J = np.linalg.det(F)
    C = np.einsum("tki,tkj->tij", F, F)
    I1 = np.trace(C, axis1=1, axis2=2)
    I2 = 0.5 * (I1 ** 2 - np.einsum("tij,tji->t", C, C))
    m = len(F)
    model = np.broadcast_to(model, (m,))
    mu = np.broadcast_to(mu, (m,)).astype(float)
    lam = np.broadcast_to(lam, (m,)).astype(float)
    out = np.zeros(m)
    c = model == SNH
    alpha = 1.0 + 0.75 * mu[c] / lam[c]
    out[c] = 0.5 * mu[c] * (I1[c] - 3.0) + 0.5 * lam[c] * (J[c] - alpha) ** 2 - 0.5 * mu[c] * np.log(I1[c] + 1.0)
    c = model == MR
    Jh = np.maximum(J[c], J_CLAMP)
    c10 = 0.25 * mu[c]
    kap = lam[c] + 2.0 * mu[c] / 3.0
    out[c] = c10 * (Jh ** (-2.0 / 3.0) * I1[c] - 3.0) + c10 * (Jh ** (-4.0 / 3.0) * I2[c] - 3.0) + 0.5 * kap * (J[c] - 1.0) ** 2
    return out


def grad_hess(model, s, mu, lam):
    """Gradient (m,3) and Hessian (m,3,3) of psi with respect to s."""
    m = len(s)
    model = np.broadcast_to(model, (m,))
    mu = np.broadcast_to(mu, (m,)).astype(float)
    lam = np.broadcast_to(lam, (m,)).astype(float)
    J, Ji, Jij = _J_terms(s)
    I1 = (s * s).sum(1)
    g = np.zeros((m, 3))
    H = np.zeros((m, 3, 3))
    eye = np.eye(3)

    c = model == COROT
    if c.any():
        g[c] = 2.0 * mu[c, None] * (s[c] - 1.0) + lam[c, None] * (J[c] - 1.0)[:, None] * Ji[c]
        H[c] = (2.0 * mu[c, None, None] * eye
                + lam[c, None, None] * (Ji[c, :, None] * Ji[c, None, :])
                + (lam[c] * (J[c] - 1.0))[:, None, None] * Jij[c])
    c = model == SNH
    if c.any():
        alpha = 1.0 + 0.75 * mu[c] / lam[c]
        q = 1.0 / (I1[c] + 1.0)
        g[c] = (mu[c, None] * s[c] + lam[c, None] * (J[c] - alpha)[:, None] * Ji[c]
                - (mu[c] * q)[:, None] * s[c])
        H[c] = (mu[c, None, None] * eye
                + lam[c, None, None] * (Ji[c, :, None] * Ji[c, None, :])
                + (lam[c] * (J[c] - alpha))[:, None, None] * Jij[c]
                - (mu[c] * q)[:, None, None] * eye
                + (2.0 * mu[c] * q * q)[:, None, None] * (s[c, :, None] * s[c, None, :]))
    c = model == MR
    if c.any():
        sc = s[c]
        Jc, Jic, Jijc = J[c], Ji[c], Jij[c]
        c10 = 0.25 * mu[c]
        kap = lam[c] + 2.0 * mu[c] / 3.0
        I1c = (sc * sc).sum(1)
        X1, X1i, X1ij = I1c, 2.0 * sc, 2.0 * np.broadcast_to(eye, (len(sc), 3, 3))
        sq = sc * sc
        X2 = sq[:, 0] * sq[:, 1] + sq[:, 0] * sq[:, 2] + sq[:, 1] * sq[:, 2]
        X2i = 2.0 * sc * (I1c[:, None] - sq)
        X2ij = 4.0 * sc[:, :, None] * sc[:, None, :]
        X2ij[:, [0, 1, 2], [0, 1, 2]] = 2.0 * (I1c[:, None] - sq)
        active = Jc > J_CLAMP
        Jh = np.maximum(Jc, J_CLAMP)
        gc = kap[:, None] * (Jc - 1.0)[:, None] * Jic
        Hc = kap[:, None, None] * (Jic[:, :, None] * Jic[:, None, :]) + (kap * (Jc - 1.0))[:, None, None] * Jijc
        for a, X, Xi, Xij in ((-2.0 / 3.0, X1, X1i, X1ij), (-4.0 / 3.0, X2, X2i, X2ij)):
            Ja = Jh ** a
            f_i = Ja[:, None] * Xi
            f_ij = Ja[:, None, None] * Xij
            # terms from d(J^a)/dJ only where the clamp is inactive
            A1 = np.where(active, a * Jh ** (a - 1.0), 0.0)
            A2 = np.where(active, a * (a - 1.0) * Jh ** (a - 2.0), 0.0)
            f_i = f_i + (A1 * X)[:, None] * Jic
            f_ij = (f_ij + (A2 * X)[:, None, None] * (Jic[:, :, None] * Jic[:, None, :])
                    + (A1 * X)[:, None, None] * Jijc
                    + A1[:, None, None] * (Jic[:, :, None] * Xi[:, None, :] + Xi[:, :, None] * Jic[:, None, :]))
            gc = gc + c10[:, None] * f_i
            Hc = Hc + c10[:, None, None] * f_ij
        g[c] = gc
        H[c] = Hc
    return g, H


def prox_singular(model, sigma, mu, lam, k, tol=1e-12, max_iter=200):
    """s* = argmin (k/2)|s - sigma|^2 + psi(s) by safeguarded Newton from s = sigma.

    Shift rule (shared reading with the GPU solver): if K = k I + Hess psi is not
    positive definite, retry with K + tau I, tau = 1e-2 k, 1e-1 k, k, ...
    Armijo backtracking (c = 1e-4, halving, at most 30 halvings).
    """
    m = len(sigma)
    model = np.broadcast_to(model, (m,)).copy()
    mu = np.broadcast_to(mu, (m,)).astype(float)
    lam = np.broadcast_to(lam, (m,)).astype(float)
    k = np.broadcast_to(k, (m,)).astype(float)
    s = sigma.astype(np.float64).copy()
    arap = model == ARAP
    s[arap] = 1.0
    act = ~arap

    def f(idx, x):
        return 0.5 * k[idx] * ((x - sigma[idx]) ** 2).sum(1) + energy(model[idx], x, mu[idx], lam[idx])

    for _ in range(max_iter):
        idx = np.nonzero(act)[0]
        if len(idx) == 0:
            break
        gp, Hp = grad_hess(model[idx], s[idx], mu[idx], lam[idx])
        g = k[idx, None] * (s[idx] - sigma[idx]) + gp
        gn = np.linalg.norm(g, axis=1)
        done = gn <= tol * k[idx] * np.maximum(1.0, np.abs(sigma[idx]).max(1))
        act[idx[done]] = False
        idx, g, Hp = idx[~done], g[~done], Hp[~done]
        if len(idx) == 0:
            break
        K = Hp + k[idx, None, None] * np.eye(3)
        tau = np.zeros(len(idx))
        while True:
            lo = np.linalg.eigvalsh(K + tau[:, None, None] * np.eye(3))[:, 0]
            bad = lo <= 0.0
            if not bad.any():
                break
            tau = np.where(bad, np.where(tau == 0.0, 1e-2 * k[idx], 10.0 * tau), tau)
        d = -np.linalg.solve(K + tau[:, None, None] * np.eye(3), g[:, :, None])[:, :, 0]
        f0 = f(idx, s[idx])
        slope = (g * d).sum(1)
        t = np.ones(len(idx))
        for _ in range(30):
            trial = s[idx] + t[:, None] * d
            ok = f(idx, trial) <= f0 + 1e-4 * t * slope
            if ok.all():
                break
            t = np.where(ok, t, 0.5 * t)
        step = t[:, None] * d
        s[idx] = s[idx] + step
        tiny = np.abs(step).max(1) <= 1e-15 * np.maximum(1.0, np.abs(s[idx]).max(1))
        act[idx[tiny]] = False
    return s


def local_step(model, F, mu, lam, k):
    """p_t = U diag(s*) V^T for every tet (Eq. PD local).  F (m,3,3) -> P (m,3,3)."""
    U, sig, Vt = svd_rv(F)
    s = prox_singular(model, sig, mu, lam, k)
    return np.einsum("tij,tj,tjk->tik", U, s, Vt)
