"""Stick-sliding precision of the complementarity preconditioner (Sec. 7, stick-sliding
test; Sec. 5.4; App. B).

A stiff block (E = 1e8, rho = 1000) rests on a plane inclined by 10 degrees; the
analytic threshold is mu* = tan(10 deg).  For each offset d of a ladder, the block is
simulated with mu = mu* - d (it must slide, at g (sin - mu cos) t) and mu = mu* + d (it
must stick) with the paper's 10 L-G iterations and 24 CR iterations per frame.  The
precision of a configuration (NCP function x preconditioner) is the smallest offset of
the ladder from which on every larger offset is classified correctly, by two criteria:
"strict", sliding at no less than half the analytic velocity and sticking at under a
tenth of it; "moves", the paper's distinction of a block that slides from one that
sticks, read as sliding at no less than a tenth of the analytic velocity and sticking at
under a tenth of it.  Each row also gives the slide velocity as a fraction of the
analytic one.
"""
from __future__ import annotations

import math

import numpy as np

from . import lgsim, scenes

THETA_DEG = 10.0
MU_STAR = math.tan(math.radians(THETA_DEG))
LADDER = (0.1, 0.05, 0.02, 0.01, 0.005, 0.002, 0.001)
CONFIGS = {"fb_delassus": (lgsim.SIM_NCP_FB, lgsim.SIM_PRECOND_DELASSUS),
           "fb_mass": (lgsim.SIM_NCP_FB, lgsim.SIM_PRECOND_MASS),
           "minmap_delassus": (lgsim.SIM_NCP_MINMAP, lgsim.SIM_PRECOND_DELASSUS),
           "minmap_mass": (lgsim.SIM_NCP_MINMAP, lgsim.SIM_PRECOND_MASS)}


def analytic_velocity(mu, frames, h):
    th = math.radians(THETA_DEG)
    return max(0.0, 9.81 * (math.sin(th) - mu * math.cos(th)) * frames * h)


def block_velocity(mu, ncp, precond, frames=40, nodes=2):
    """Mean downhill node velocity of the block after `frames` frames on the GPU."""
    sc = scenes.incline_block(mu=mu, theta_deg=THETA_DEG, E=1e8, nodes=nodes, frames=frames)
    sim = lgsim.Sim(sc, ncp=ncp, precond=precond)
    sim.step(frames, stats=False)
    _, v1, _ = sim.read_state()
    sim.close()
    return float(np.mean(v1[:, 0]))


def scan(config, frames=40, nodes=2, ladder=LADDER):
    """Per-offset velocities and the precision of one configuration."""
    ncp, precond = CONFIGS[config]
    h = 0.01
    rows = []
    for d in ladder:
        v_an = analytic_velocity(MU_STAR - d, frames, h)
        v_slide = block_velocity(MU_STAR - d, ncp, precond, frames, nodes)
        v_stick = block_velocity(MU_STAR + d, ncp, precond, frames, nodes)
        stuck = abs(v_stick) <= 0.1 * v_an
        rows.append({"offset": d, "v_analytic": v_an, "v_slide": v_slide, "v_stick": v_stick,
                     "slide_fraction": v_slide / v_an, "correct": v_slide >= 0.5 * v_an and stuck,
                     "correct_moves": v_slide >= 0.1 * v_an and stuck})

    def precision(key):
        out = None
        for r in rows:  # ladder in decreasing order: stop at the first miss
            if not r[key]:
                break
            out = r["offset"]
        return out

    return {"config": config, "precision": precision("correct"), "precision_moves": precision("correct_moves"),
            "rows": rows}
