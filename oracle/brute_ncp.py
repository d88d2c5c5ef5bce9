"""Brute-force solutions of one frame's linear frictional contact problem (pins only).

With the unconstrained positions u fixed, the contact-space state is affine in
the impulses: y = a + B lambda with y_j = (delta_n, h delta_dot_f1,
h delta_dot_f2), a = H u - (d_n, H_f q_t + h d_f) and B = h^2 W (App. A,
Sec. 5.3).  A solution satisfies the Signorini-Coulomb conditions (Sec. 3.2,
App. A "Frictional contact formulation").  Each contact is open, sticking or
sliding; every assignment of modes is enumerated:

  open   lambda_j = 0,                       needs delta_n >= 0
  stick  y_j = 0,                            needs lambda_n >= 0, |lambda_f| <= mu lambda_n
  slide  delta_n = 0, lambda_f = mu lambda_n d(theta),
         h delta_dot_f = -t d(theta),        needs lambda_n > 0, t > 0

Open/stick assignments are linear solves; sliding contacts add the unknowns
(theta, t) and are solved by a root finder from a grid of starting angles.
For mu = 0 the problem is an LCP and the enumeration over open/closed is exact.
"""
from __future__ import annotations

import itertools

import numpy as np
import scipy.optimize as so


def _check(lam, y, mu, modes, tl, ty):
    """Signorini-Coulomb conditions with tolerances tl (impulses) and ty (metres)."""
    c = len(mu)
    for j in range(c):
        ln, lf = lam[3 * j], lam[3 * j + 1:3 * j + 3]
        yn, yf = y[3 * j], y[3 * j + 1:3 * j + 3]
        if ln < -tl or yn < -ty:
            return False
        if ln > tl and abs(yn) > ty:
            return False
        if np.linalg.norm(lf) > mu[j] * max(ln, 0.0) + tl:
            return False
        if modes[j] == "open" and (ln > tl or np.linalg.norm(lf) > tl):
            return False
        if modes[j] == "slide":
            s = np.linalg.norm(yf)
            if s > ty and np.linalg.norm(lf) > 0:
                if np.linalg.norm(yf / s + lf / np.linalg.norm(lf)) > 1e-6:
                    return False
        if modes[j] == "stick" and np.linalg.norm(yf) > ty:
            return False
    return True


def solve_all(a, B, mu, tol=1e-10, n_starts=12):
    """All solutions found of the frictional contact NCP y = a + B lambda."""
    c = len(mu)
    sols = []
    # frictionless contacts have lambda_f = 0: their "stick" mode is y_n = 0, lambda_f = 0
    mode_sets = [("open", "stick", "slide") if mu[j] > 0 else ("open", "closed") for j in range(c)]
    scale = max(1.0, np.abs(np.linalg.solve(B, -a)).max())
    for modes in itertools.product(*mode_sets):
        sl = [j for j in range(c) if modes[j] == "slide"]
        if any(mu[j] == 0 for j in sl):
            continue

        def unpack(z):
            lam = z[:3 * c].copy()
            th = z[3 * c:3 * c + len(sl)]
            for k, j in enumerate(sl):
                d = np.array([np.cos(th[k]), np.sin(th[k])])
                lam[3 * j + 1:3 * j + 3] = mu[j] * lam[3 * j] * d
            return lam

        def F(z):
            lam = unpack(z)
            y = a + B @ lam
            eqs = []
            for j in range(c):
                if modes[j] == "open":
                    eqs += list(z[3 * j:3 * j + 3])
                elif modes[j] == "closed":
                    eqs += [y[3 * j], z[3 * j + 1], z[3 * j + 2]]
                elif modes[j] == "stick":
                    eqs += list(y[3 * j:3 * j + 3])
                else:
                    k = sl.index(j)
                    th, t = z[3 * c + k], z[3 * c + len(sl) + k]
                    d = np.array([np.cos(th), np.sin(th)])
                    eqs += [y[3 * j], *(y[3 * j + 1:3 * j + 3] + t * d)]
                    eqs += [z[3 * j + 1], z[3 * j + 2]]   # unused slots pinned to 0
            return np.asarray(eqs)

        nz = 3 * c + 2 * len(sl)
        starts = [np.zeros(nz)]
        if sl:
            starts = []
            rng = np.random.default_rng(0)
            for _ in range(n_starts):
                z0 = np.zeros(nz)
                z0[:3 * c] = np.linalg.lstsq(B, -a, rcond=None)[0]
                z0[3 * c:3 * c + len(sl)] = rng.uniform(0, 2 * np.pi, len(sl))
                z0[3 * c + len(sl):] = rng.uniform(0, 1, len(sl)) * np.abs(a).max()
                starts.append(z0)
        for z0 in starts:
            if not sl:
                # linear system
                M = np.zeros((3 * c, 3 * c))
                rhs = np.zeros(3 * c)
                for j in range(c):
                    r = slice(3 * j, 3 * j + 3)
                    if modes[j] == "open":
                        M[r, r] = np.eye(3)
                    elif modes[j] == "closed":
                        M[r, r] = np.eye(3)
                        M[3 * j, :] = B[3 * j, :]
                        rhs[3 * j] = -a[3 * j]
                    else:
                        M[r, :] = B[r, :]
                        rhs[r] = -a[r]
                try:
                    lam = np.linalg.solve(M, rhs)
                except np.linalg.LinAlgError:
                    continue
            else:
                sol = so.root(F, z0, method="hybr", tol=1e-14)
                if not sol.success or np.abs(F(sol.x)).max() > 1e-10 * scale:
                    continue
                if np.any(sol.x[3 * c + len(sl):] <= 0):
                    continue
                lam = unpack(sol.x)
            y = a + B @ lam
            if _check(lam, y, mu, modes, tol * scale, tol * max(1e-3, np.abs(a).max())):
                if not any(np.abs(lam - s).max() <= 1e-7 * scale for s in sols):
                    sols.append(lam)
    return sols
