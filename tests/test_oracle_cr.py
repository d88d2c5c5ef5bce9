"""Pins of the oracle's Conjugate Residual solver (Sec. 6: the constraint-space solver).

Conjugate Residual minimises the residual norm |b - A x| over the Krylov space
K_k(A, b) = span{b, A b, ..., A^(k-1) b} at step k (x_0 = 0).  Three consequences are
checked against references that share nothing with the recurrence:
* on an SPD system of order n the n-th iterate is the exact solution (the Krylov
  space is the whole space), compared with numpy's LU solve;
* the residual norms of successive iterates never increase (nested spaces);
* every iterate equals the minimiser of |b - A x| over K_k(A, b) computed from an
  orthonormal Krylov basis and a dense least-squares solve.
A wrong beta, a stale (r, A r) or a missing update of A p changes the iterates and
fails the last test already at k = 2.
"""
import numpy as np
import pytest

from oracle.cr import conjugate_residual


def spd(n, seed, cond=50.0):
    rng = np.random.default_rng(seed)
    Q, _ = np.linalg.qr(rng.standard_normal((n, n)))
    ev = np.geomspace(1.0, cond, n)
    return (Q * ev) @ Q.T, rng.standard_normal(n)


def krylov_minimiser(A, b, k):
    """argmin_{x in K_k(A, b)} |b - A x|, by an orthonormal Krylov basis (modified
    Gram-Schmidt) and a dense least-squares solve."""
    n = len(b)
    V = np.zeros((n, k))
    v = b / np.linalg.norm(b)
    for j in range(k):
        for i in range(j):
            v = v - (V[:, i] @ v) * V[:, i]
        v = v / np.linalg.norm(v)
        V[:, j] = v
        v = A @ v
    y, *_ = np.linalg.lstsq(A @ V, b, rcond=None)
    return V @ y


@pytest.mark.parametrize("n", [1, 2, 3, 4, 5, 6])
@pytest.mark.parametrize("seed", [0, 1, 2])
def test_n_steps_solve_spd_system(n, seed):
    A, b = spd(n, seed)
    x = conjugate_residual(lambda v: A @ v, b, n)
    ref = np.linalg.solve(A, b)
    assert np.abs(x - ref).max() <= 1e-10 * np.abs(ref).max()


@pytest.mark.parametrize("seed", [0, 1, 2, 3])
def test_residual_norm_never_increases(seed):
    A, b = spd(6, seed, cond=1e3)
    res = [np.linalg.norm(b - A @ conjugate_residual(lambda v: A @ v, b, k)) for k in range(7)]
    assert res[0] == pytest.approx(np.linalg.norm(b))
    for a, c in zip(res, res[1:]):
        assert c <= a * (1.0 + 1e-12)
    assert res[-1] <= 1e-6 * res[0]  # exact in 6 steps up to rounding (cond 1e3)


@pytest.mark.parametrize("seed", [0, 1, 2])
@pytest.mark.parametrize("k", [1, 2, 3, 4])
def test_iterates_are_krylov_residual_minimisers(seed, k):
    A, b = spd(6, seed)
    x = conjugate_residual(lambda v: A @ v, b, k)
    ref = krylov_minimiser(A, b, k)
    assert np.abs(x - ref).max() <= 1e-9 * np.abs(ref).max()


def test_symmetric_indefinite_still_minimises_residual():
    # CR needs symmetry only (Sec. 6 applies it to the Schur system, whose Omega blocks
    # may zero whole rows); on a non-singular indefinite matrix its iterates are still the
    # Krylov residual minimisers while no breakdown occurs
    rng = np.random.default_rng(7)
    Q, _ = np.linalg.qr(rng.standard_normal((5, 5)))
    A = (Q * np.array([-3.0, -1.0, 2.0, 4.0, 9.0])) @ Q.T
    b = rng.standard_normal(5)
    for k in (1, 2, 3):
        x = conjugate_residual(lambda v: A @ v, b, k)
        assert np.abs(x - krylov_minimiser(A, b, k)).max() <= 1e-9 * max(1.0, np.abs(x).max())


def test_tolerance_stops_early_and_zero_rhs():
    A, b = spd(6, 4, cond=1e4)
    full = conjugate_residual(lambda v: A @ v, b, 6)
    loose = conjugate_residual(lambda v: A @ v, b, 6, tol=0.5)
    assert np.linalg.norm(b - A @ loose) <= 0.5 * np.linalg.norm(b)
    assert np.linalg.norm(b - A @ loose) > np.linalg.norm(b - A @ full)
    assert np.all(conjugate_residual(lambda v: A @ v, np.zeros(6), 6) == 0.0)
