"""Rest quantities, mass, weights and the constant system matrix (FP64).

Paper: Sec. 3.1 (implicit Euler objective, predicted state), Sec. 3.3
(Eq. PD local / PD global: A = M + h^2 sum_i w_i G_i^T G_i and
b = M q~ + h^2 sum_i w_i G_i^T p_i).

Readings (the paper names but does not define these):
* mass is lumped, rho V / 4 per tet corner;
* G_i maps nodal positions to the deformation gradient F = sum_a x_a d_a^T of
  tet i, acting identically on x, y and z, so A = A_n (x) I3 with an n x n
  node-level A_n;
* w_i = k_i V_i with k = 2 mu (ARAP) or 2 mu + lambda (other models);
* pinned nodes carry a positional constraint (w_pin/2)|x - target|^2 with
  h^2 w_pin = 1e3 [A_n]_vv (the node's own diagonal before pins, times a user
  scale), added to A_n and b; the target moves rigidly per pin group.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp

ARAP, COROT, SNH, MR = 0, 1, 2, 3


def lame(E, nu):
    """Lame parameters (mu, lambda) from Young's modulus and Poisson ratio."""
    E = np.asarray(E, dtype=np.float64)
    nu = np.asarray(nu, dtype=np.float64)
    mu = E / (2.0 * (1.0 + nu))
    lam = E * nu / ((1.0 + nu) * (1.0 - 2.0 * nu))
    return mu, lam


def rest_shape(rest, tets):
    """Per tet: volume V and the rows d_0..d_3 with F = sum_a x_a d_a^T.

    Dm = [X1-X0, X2-X0, X3-X0] (columns); d_1..d_3 are the rows of Dm^-1 and
    d_0 = -(d_1 + d_2 + d_3).  Returns V (m,), D (m,4,3).
    """
    X = rest[tets]                                   # (m,4,3)
    Dm = np.stack([X[:, 1] - X[:, 0], X[:, 2] - X[:, 0], X[:, 3] - X[:, 0]], axis=2)
    V = np.linalg.det(Dm) / 6.0
    Dinv = np.linalg.inv(Dm)                         # rows d_1..d_3
    D = np.empty((len(tets), 4, 3))
    D[:, 1:, :] = Dinv
    D[:, 0, :] = -Dinv.sum(axis=1)
    return V, D


def deformation_gradient(q, tets, D):
    """F_t = sum_a x_a d_a^T for every tet; q (n,3) -> (m,3,3)."""
    return np.einsum("tai,taj->tij", q[tets], D)


def material_arrays(scene, m):
    model = np.full(m, scene.model, dtype=np.int64) if scene.tet_model is None else np.asarray(scene.tet_model, np.int64)
    E = np.full(m, scene.E) if scene.tet_E is None else np.asarray(scene.tet_E, np.float64)
    nu = np.full(m, scene.nu) if scene.tet_nu is None else np.asarray(scene.tet_nu, np.float64)
    mu, lam = lame(E, nu)
    k = np.where(model == ARAP, 2.0 * mu, 2.0 * mu + lam)
    return model, mu, lam, k


def lumped_mass(n, tets, V, rho):
    m = np.zeros(n)
    np.add.at(m, tets.reshape(-1), np.repeat(rho * V / 4.0, 4))
    return m


def system_matrix(n, tets, D, w, mass, h, pin_nodes, pin_h2w):
    """Node-level A_n = diag(m) + h^2 sum_t w_t [d_a . d_b]_ab + diag(h^2 w_pin) (CSR)."""
    blocks = h * h * w[:, None, None] * np.einsum("tai,tbi->tab", D, D)      # (m,4,4)
    rows = np.repeat(tets, 4, axis=1).reshape(-1)
    cols = np.tile(tets, (1, 4)).reshape(-1)
    A = sp.coo_matrix((blocks.reshape(-1), (rows, cols)), shape=(n, n)).tocsr()
    diag = mass.copy()
    if len(pin_nodes):
        np.add.at(diag, pin_nodes, pin_h2w)
    A = A + sp.diags(diag)
    A.sum_duplicates()
    A.sort_indices()
    return A


def elastic_rhs(n, tets, D, w, P):
    """sum_t w_t G_t^T p_t : node a of tet t receives w_t p_t d_a.  P (m,3,3) -> (n,3)."""
    contrib = w[:, None, None] * np.einsum("tij,taj->tai", P, D)              # (m,4,3)
    out = np.zeros((n, 3))
    np.add.at(out, tets.reshape(-1), contrib.reshape(-1, 3))
    return out


def rodrigues(theta):
    """Rotation matrix for the rotation vector theta (3,)."""
    a = float(np.linalg.norm(theta))
    if a == 0.0:
        return np.eye(3)
    k = theta / a
    Kx = np.array([[0, -k[2], k[1]], [k[2], 0, -k[0]], [-k[1], k[0], 0]])
    return np.eye(3) + np.sin(a) * Kx + (1.0 - np.cos(a)) * (Kx @ Kx)


def pin_targets(x0, group, lin, ang, pivot, t):
    """target(t) = pivot + lin t + R(ang t)(x0 - pivot), per pin group."""
    out = np.empty_like(x0)
    for g in range(len(lin)):
        sel = group == g
        R = rodrigues(ang[g] * t)
        out[sel] = pivot[g] + lin[g] * t + (x0[sel] - pivot[g]) @ R.T
    return out
