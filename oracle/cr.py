"""Conjugate Residual for a symmetric system (FP64).

Paper: Sec. 6 names Conjugate Residual as the constraint-space solver (10
iterations in its examples, 24 in the stick-slide test).  Reading: start
from x = 0, run a fixed number of iterations with no early exit; stop only
on exact breakdown ((Ap,Ap) = 0 or (r,Ar) = 0).  This is the textbook
Conjugate Residual recurrence for symmetric matrices (Stiefel 1955; see
Saad, Iterative Methods for Sparse Linear Systems).
"""
from __future__ import annotations

import numpy as np


def conjugate_residual(matvec, b, iters, tol=0.0):
    """At most ``iters`` iterations; with tol > 0 also stop once |r| <= tol |b|
    (checked before each iteration)."""
    x = np.zeros_like(b)
    r = b.copy()
    Ar = matvec(r)
    p = r.copy()
    Ap = Ar.copy()
    rAr = float(r @ Ar)
    rr0 = float(b @ b)
    for _ in range(iters):
        ApAp = float(Ap @ Ap)
        if ApAp == 0.0 or rAr == 0.0:
            break
        if tol > 0.0 and float(r @ r) <= tol * tol * rr0:
            break
        alpha = rAr / ApAp
        x = x + alpha * p
        r = r - alpha * Ap
        Ar = matvec(r)
        rAr_new = float(r @ Ar)
        beta = rAr_new / rAr
        rAr = rAr_new
        p = r + beta * p
        Ap = Ar + beta * Ap
    return x
