"""Pins of bilateral (binding) constraints in the oracle (Sec. 3.2 binding contact;
App. A bilateral items; compliance as a quadratic potential of stiffness 1/e).

* a hard point anchor (three hard rows along x, y, z at the top corner) holds its node at
  the anchor while the rest of the block swings;
* with a compliant vertical row the anchor stretches by e times the row's force at every
  frame (phi_b = delta_b + e lambda_b = 0 at the converged constraint solve);
* the binding's frame is its normalised direction with the Gram-Schmidt tangents.
"""
import numpy as np

from oracle import contact as ct
from oracle.sim import OracleSim
from paper_2503_15078_amd import scenes


def _run(sc, frames, cr="exact"):
    o = OracleSim(sc)
    top = int(sc.obstacles[0].geom[7])
    out = []
    for _ in range(frames):
        q_t, q_pred, fc, lam = o.begin_frame()
        q = q_pred.copy()
        for _ in range(sc.iters):
            q, lam, _ = o.iterate(fc, q, lam, q_t, q_pred, o.t + o.h, cr=cr)
        o.end_frame(q_t, q, fc, lam)
        out.append((o.q[top].copy(), fc, lam.copy(), o.q.copy()))
    return o, top, out


def test_hard_anchor_holds_while_block_swings():
    sc = scenes.hanging_block(e_z=0.0, swing=0.5)
    o, top, out = _run(sc, 20)
    p = sc.obstacles[0].geom[:3]
    assert max(np.abs(x - p).max() for x, _, _, _ in out) <= 1e-9
    moved = np.abs(out[-1][3] - np.asarray(sc.rest)).max()
    assert moved > 5e-3


def test_compliant_row_stretches_by_e_times_force():
    e = 1e-4
    sc = scenes.hanging_block(e_z=e)
    o, top, out = _run(sc, 20)
    p = sc.obstacles[0].geom[:3]
    for x, fc, lam, _ in out:
        j = int(np.nonzero((fc.comp >= 0) & (fc.C[:, 0, 2] == 1.0))[0][0])  # the z row
        assert abs((x[2] - p[2]) + e * lam[j, 0]) <= 1e-9
        assert abs(x[0] - p[0]) <= 1e-9 and abs(x[1] - p[1]) <= 1e-9
    assert out[-1][2][:, 0].max() > 1.0  # the rows carry the block's weight


def test_binding_frame():
    nrm, f1, f2, d_n, gap = ct.binding_frame(np.array([1.0, 2.0, 3.0, 0.0, 0.0, 2.0, 0.0, 5.0]),
                                             np.array([1.0, 2.0, 2.5]))
    np.testing.assert_allclose(nrm, [0.0, 0.0, 1.0])
    assert abs(d_n - 3.0) < 1e-15 and abs(gap + 0.5) < 1e-15
    F = np.array([nrm, f1, f2])
    np.testing.assert_allclose(F @ F.T, np.eye(3), atol=1e-15)
