"""The oracle's own float64 error at one L-G iteration of a frame (test infrastructure).

For the state (q_t, q^0 = q~, lambda^0, contact list) at a frame start, one iteration of
Algorithm 4 is taken and every intermediate result that parity tests compare against is
checked against its own defining equation:

* global step u = A^-1 b (Eq. PD global, solved by sparse LU): normwise backward error
  |A u - b|_inf / (|A|_inf |u|_inf + |b|_inf), and the change of u under one step of
  iterative refinement u' = u + A^-1 (b - A u), relative to |u|_inf (an estimate of the
  forward error);
* Delassus solves Z = A_n^-1 B (Sec. 5.3): backward error |A_n Z - B|_inf /
  (|A_n|_inf |Z|_inf + 1) over all contact columns;
* exact Schur solve (M dlambda = rhs, Sec. 5.2; dense LU): backward error
  |M x - rhs|_inf / (|M|_inf |x|_inf + |rhs|_inf), the 2-norm condition number of M, and
  the refinement change of x relative to |x|_inf;
* positions after the iteration, q^1 = A^-1 (b + h^2 H^T Omega lambda^1): the
  refinement change relative to |q^1|_inf;
* NCP residual (metres): the rounding bound of its evaluation, eps_64 times the largest
  magnitude entering it (|delta_n|, r_n |lambda_n|, h s, h r_f |lambda|), against the
  residual itself.

Run as a module to print the table for the 5^3-node cube drop at its first frame with
contacts and for the 800-contact teaser-scale state.
"""
from __future__ import annotations

import json
import sys

import numpy as np
import scipy.sparse.linalg as spla

from .sim import OracleSim

EPS64 = float(np.finfo(np.float64).eps)


def _inf(a):
    return float(np.abs(a).max()) if a.size else 0.0


def _sparse_inf(A):
    return float(abs(A).sum(axis=1).max())


def frame_errors(o: OracleSim):
    """Errors of the first iteration of the oracle's next frame (state unchanged)."""
    h = o.h
    q_t, q_pred, fc, lam = o.begin_frame()
    t_next = o.t + h
    out = {"nodes": o.n, "tets": o.m, "contacts": int(fc.c)}
    b = o.rhs(q_pred, q_pred, t_next)
    A = o.A
    An = _sparse_inf(A)
    u = o.solve(b)
    out["global_backward"] = _inf(A @ u - b) / (An * _inf(u) + _inf(b))
    du = o.solve(b - A @ u)
    out["global_refine_rel"] = _inf(du) / _inf(u)
    if fc.c:
        B = np.zeros((o.n, fc.c))
        B[fc.node, np.arange(fc.c)] = 1.0
        Z = o.lu.solve(B)
        out["delassus_backward"] = _inf(A @ Z - B) / (An * _inf(Z) + 1.0)
        q1, lam1, info = o.iterate(fc, q_pred.copy(), lam, q_t, q_pred, t_next, cr="exact")
        M, r = info["cr_matrix"], info["cr_rhs"]
        x = np.linalg.solve(M, r)
        out["schur_backward"] = _inf(M @ x - r) / (np.abs(M).sum(1).max() * _inf(x) + _inf(r))
        out["schur_cond2"] = float(np.linalg.cond(M))
        out["schur_refine_rel"] = _inf(np.linalg.solve(M, r - M @ x)) / max(_inf(x), 1e-300)
        rhs1 = b + h * h * o.H_T(fc, info["Omega"] * lam1)
        out["positions_refine_rel"] = _inf(o.solve(rhs1 - A @ q1)) / _inf(q1)
        res = o.residual(fc, q1, q_t, lam1)
        x = q1[fc.node]
        dn = np.einsum("ji,ji->j", fc.C[:, 0, :], x) - fc.d_n
        mag = max(_inf(dn), _inf(fc.r_n * lam1[:, 0]), h * _inf(fc.r_f[:, None] * lam1),
                  _inf(np.einsum("jai,ji->ja", fc.C[:, 1:, :], x - q_t[fc.node])))
        out["ncp_residual"] = float(res)
        out["ncp_eval_bound"] = 8.0 * EPS64 * mag
    else:
        q1, _, _ = o.iterate(fc, q_pred.copy(), lam, q_t, q_pred, t_next)
        out["positions_refine_rel"] = _inf(o.solve(o.rhs(q_pred, q_pred, t_next) - A @ q1)) / _inf(q1)
    return out


def cube_case(seed=0):
    from paper_2503_15078_amd import scenes
    o = OracleSim(scenes.cube_drop(seed))
    o.step(14)  # the cube reaches the ground: its first frames with contacts
    return frame_errors(o)


def teaser_case(seed=0):
    from paper_2503_15078_amd import scenes
    return frame_errors(OracleSim(scenes.teaser_scene(seed)))


def main(argv):
    cases = {"cube_drop_5x5x5": cube_case}
    if "--teaser" in argv:
        cases["teaser_800_contacts"] = teaser_case
    table = {k: f() for k, f in cases.items()}
    print(json.dumps(table, indent=1))


if __name__ == "__main__":
    spla.use_solver(useUmfpack=False)
    main(sys.argv[1:])
