"""Elimination tree and the inverse Cholesky factor on small matrices (FP64).

Paper: Sec. 4.2, Theorem 1 -- for SPD A with Cholesky factor L, the structure
of L^-1 is the set of (i, j) with i an ancestor of j (or i = j) in the
elimination tree of A; A^-1 = S^T S with S = L^-1 (Algorithm 2).

Everything here is written from the definitions, with dense arrays, for
meshes of a few hundred nodes:
* symbolic factorisation by boolean elimination (column j of L is the lower
  part of column j of A plus the columns k < j with L_jk != 0, below j);
* parent(j) = min{ i > j : L_ij structurally nonzero };
* L by numpy's dense Cholesky, S = L^-1 by a dense triangular inverse.
Pins: tests check the etree from this symbolic factorisation against the
nonzeros of the numeric L^-1 (Theorem 1) and S^T S A = I.
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla


def symbolic_pattern(A):
    """Boolean lower-triangular structure of L for dense or sparse symmetric A."""
    A = A.toarray() if hasattr(A, "toarray") else np.asarray(A)
    n = A.shape[0]
    P = np.tril(A != 0)
    for j in range(n):
        ks = np.nonzero(P[j, :j])[0]
        for k in ks:
            P[j + 1:, j] |= P[j + 1:, k]
    return P


def etree_from_pattern(P):
    n = P.shape[0]
    parent = -np.ones(n, dtype=np.int64)
    for j in range(n):
        below = np.nonzero(P[j + 1:, j])[0]
        if len(below):
            parent[j] = j + 1 + below[0]
    return parent


def ancestors_pattern(parent):
    """Boolean matrix M[i, j] = (i == j or i is an ancestor of j)."""
    n = len(parent)
    M = np.zeros((n, n), dtype=bool)
    for j in range(n):
        i = j
        while i != -1:
            M[i, j] = True
            i = parent[i]
    return M


def dense_sparse_inverse(A):
    """(L, S = L^-1) by dense Cholesky of A."""
    A = A.toarray() if hasattr(A, "toarray") else np.asarray(A)
    L = np.linalg.cholesky(A)
    S = sla.solve_triangular(L, np.eye(A.shape[0]), lower=True)
    return L, S


def depth(parent):
    n = len(parent)
    d = np.zeros(n, dtype=np.int64)
    for j in range(n - 1, -1, -1):
        if parent[j] != -1:
            d[j] = d[parent[j]] + 1
    return d
