"""Pins of the oracle's iteration loop without contact (Algorithm 4 / Eq. PD global).

* rest shape is a fixed point: with q_t = rest, v = 0 and no gravity every
  iteration returns the rest positions (zero elastic force at F = I);
* linear momentum: since sum_a d_a = 0, 1^T A = 1^T M and 1^T sum w G^T p = 0,
  so sum m v_{t+h} = sum m v_t + h sum m g exactly, for any iteration count;
* free fall: the centre of mass follows the implicit-Euler recursion
  v_{n+1} = v_n + h g, x_{n+1} = x_n + h v_{n+1};
* pins: a pinned node of a body at rest follows its target.
"""
import numpy as np
import pytest

from oracle.sim import OracleSim
from paper_2503_15078_amd import scenes


@pytest.mark.parametrize("model", [0, 1, 2, 3])
def test_rest_is_fixed_point(model):
    sc = scenes.free_block(0, model=model, gravity=(0.0, 0.0, 0.0))
    sc.init_pos = sc.rest.copy()
    sc.init_vel = np.zeros_like(sc.rest)
    o = OracleSim(sc)
    o.step(2, iters=3)
    np.testing.assert_allclose(o.q, sc.rest, atol=1e-13)
    np.testing.assert_allclose(o.v, 0.0, atol=1e-11)


@pytest.mark.parametrize("model,iters", [(1, 1), (2, 3), (3, 5), (0, 2)])
def test_linear_momentum(model, iters):
    sc = scenes.free_block(1 + model, model=model, spin=2.0)
    o = OracleSim(sc)
    m = o.mass
    for _ in range(3):
        p0 = (m[:, None] * o.v).sum(0)
        o.step(1, iters=iters)
        p1 = (m[:, None] * o.v).sum(0)
        np.testing.assert_allclose(p1, p0 + o.h * m.sum() * o.g, rtol=0, atol=1e-12 * max(1.0, np.abs(p0).max()))


def test_free_fall_centre_of_mass():
    sc = scenes.free_block(3, model=2)
    o = OracleSim(sc)
    m = o.mass
    x = (m[:, None] * o.q).sum(0) / m.sum()
    v = (m[:, None] * o.v).sum(0) / m.sum()
    for _ in range(5):
        o.step(1, iters=2)
        v = v + o.h * o.g
        x = x + o.h * v
        np.testing.assert_allclose((m[:, None] * o.q).sum(0) / m.sum(), x, atol=1e-12)


def test_pins_follow_targets():
    sc = scenes.twist_bar(0, nodes=(8, 4, 4), E=1e5, frames=40)
    sc.obstacles = []
    sc.gravity = np.zeros(3)
    o = OracleSim(sc)
    o.step(10, iters=5)
    tgt = o.pin_target(o.t)
    err = np.abs(o.q[o.pin_nodes] - tgt).max()
    # positional constraints are penalties 1e3 x the node's own stiffness; they lag slightly
    assert err < 5e-3 * np.abs(tgt - o.pin_x0).max() + 1e-9
