"""Pins of moving obstacles in the oracle (App. A: the obstacle velocity enters the
tangential relative velocity; the obstacle geometry can move between frames).

* conveyor: a block at rest on a plane whose surface moves at 0.2 m/s is carried up to
  belt speed by static friction (mu = 0.8, mu g far above what is needed), and with
  mu = 0.02 it slides, accelerated at mu g (Coulomb), reaching mu g t;
* a plane rising at 0.1 m/s (geometry moved every frame) lifts the block at its speed
  and the block does not sink into it.
"""
import numpy as np

from oracle.sim import OracleSim
from paper_2503_15078_amd import scenes


def test_conveyor_carries_block_to_belt_speed():
    o = OracleSim(scenes.conveyor_block(mu=0.8))
    o.step(40)
    v = o.v.mean(0)
    assert abs(v[0] - 0.2) <= 0.01 * 0.2
    assert abs(v[1]) <= 1e-6 and abs(v[2]) <= 1e-4


def test_conveyor_slip_accelerates_at_mu_g():
    mu = 0.02
    o = OracleSim(scenes.conveyor_block(mu=mu))
    o.step(40)
    v_an = mu * 9.81 * 40 * o.h
    assert abs(o.v.mean(0)[0] - v_an) <= 0.01 * v_an


def test_rising_plane_lifts_block():
    w = 0.1
    o = OracleSim(scenes.conveyor_block(mu=0.5, belt=(0.0, 0.0, 0.0)))
    for _ in range(40):
        o.obstacles = [scenes.moving_plane(w * (o.t + o.h), mu=0.5)]
        o.step(1)
    assert abs(o.v.mean(0)[2] - w) <= 0.01 * w
    assert o.q[:, 2].min() >= w * o.t - 1e-4
