"""Failure paths forced from the host, through the C-ABI.

Non-finite input is refused at the boundary (SIM_E_ARG). A finite state can still produce a
non-finite one: a velocity of 1e30 m/s at one node gives deformation gradients near 1e29, whose
F^T F in the local step's SVD overflows float32. Such a frame is reported as SIM_E_DIVERGED (-7)
and rolled back. Frame-start positions, velocities and the saved contacts stay as they were, so a
finite state set afterwards steps exactly as on a handle that never failed.

Inverted elements are a state the method has to survive. Pushing a corner node 1.3 voxels into
the cube inverts four tets. The oracle un-inverts them within one frame for ARAP and stable
Neo-Hookean (checked here on the CPU), and the device's frame from the same state matches the
oracle's.

Every kernel on the frame path stays in bounds with non-finite values: no position becomes an
index, and every loop has a fixed count."""
import numpy as np
import pytest

from oracle.sim import OracleSim
from paper_2503_15078_amd import lgsim, scenes

torch = pytest.importorskip("torch")


def _volumes(x, tets):
    a, b, c, d = (x[tets[:, k]] for k in range(4))
    return np.einsum("ij,ij->i", np.cross(b - a, c - a), d - a) / 6.0


def _inverted_state(sc):
    q = sc.q0().astype(np.float64)
    corner = int(np.argmin(q.sum(1)))
    q[corner] += 1.3 * 0.025  # the 5-node cube's voxel is 0.025 m
    return q


@pytest.mark.parametrize("model", [scenes.MODEL_ARAP, scenes.MODEL_SNH])
def test_oracle_uninverts_within_one_frame(model):
    sc = scenes.cube_drop(0, model=model)
    q = _inverted_state(sc)
    assert (_volumes(q, sc.tets) <= 0).sum() == 4
    o = OracleSim(sc)
    o.q = q
    o.step(1)
    assert np.isfinite(o.q).all() and (_volumes(o.q, sc.tets) > 0).all()


@pytest.mark.gpu
@pytest.mark.parametrize("model", [scenes.MODEL_ARAP, scenes.MODEL_SNH])
def test_inverted_tets_frame_matches_oracle(model):
    sc = scenes.cube_drop(0, model=model)
    q = _inverted_state(sc)
    o = OracleSim(sc)
    o.q = q.copy()
    o.step(1)
    sim = lgsim.Sim(sc)
    sim.set_iterate_state(q, sc.v0(), None, 0.0, [], [], [])
    sim.step(1)
    x, _, _ = sim.read_state()
    sim.close()
    err = np.abs(x - o.q).max()
    print(f"model {model}: |x - oracle| {err:.2e} m")
    assert np.isfinite(x).all() and (_volumes(x, sc.tets) > 0).all()
    assert err <= 1e-4


@pytest.mark.gpu
def test_non_finite_state_is_reported_and_the_frame_rolled_back():
    sc = scenes.cube_drop(0)
    a, b = lgsim.Sim(sc), lgsim.Sim(sc)
    for s in (a, b):
        s.step(5)
    x5, v5, _ = a.read_state()
    t5 = 5 * sc.h
    nan = v5.copy()
    nan[3, 0] = np.nan
    with pytest.raises(lgsim.SimError) as e:
        a.set_iterate_state(x5, nan, None, t5, [], [], [])
    assert e.value.code == -1  # SIM_E_ARG: refused before any device work
    bad = v5.copy()
    bad[3, 0] = 1e30
    a.set_iterate_state(x5, bad, None, t5, [], [], [])
    with pytest.raises(lgsim.SimError) as e:
        a.step(1)
    assert e.value.code == -7  # SIM_E_DIVERGED
    x, v, _ = a.read_state()
    np.testing.assert_array_equal(x, x5)  # not advanced
    np.testing.assert_array_equal(v, bad.astype(np.float32).astype(np.float64))  # as set
    for s in (a, b):
        s.set_iterate_state(x5, v5, None, t5, [], [], [])
        s.step(3)
    (xa, va, _), (xb, vb, _) = a.read_state(), b.read_state()
    a.close()
    b.close()
    np.testing.assert_array_equal(xa, xb)
    np.testing.assert_array_equal(va, vb)
