"""Complete vs incomplete global steps (Sec. 7, performance and accuracy evaluation).

A bar is twisted by rotating its pinned ends (the twisting test, no contact).  At a
frame where it is largely deformed, the next frame's local-global iterations run on the
GPU with the direct global step (S^T S, the method) and with one Jacobi sweep per
iteration (the incomplete baseline).  The relative error of iterate q^k is
(eps(q^k) - eps(q*)) / (eps(q^0) - eps(q*)), with eps the objective the iteration
minimises (sim_lg_energy, float64 sums on the GPU), q^0 the predicted state with the
pinned ends at their targets (start_state) and q* the converged solution.  Reading: q* is the direct iteration run to convergence (its objective changes
by less than the reported floor), in place of the paper's Newton solve of the same
objective.
"""
from __future__ import annotations

import time

import numpy as np

from . import lgsim, scenes

MODEL = scenes.MODEL_ARAP
CHECKPOINTS = (1, 2, 5, 10, 20, 50, 100, 200, 500, 1000)


def bar(E, frames_total=400):
    return scenes.twist_bar(0, model=MODEL, E=E, nu=0.3, nodes=(40, 10, 10), frames=frames_total, iters=10,
                            turns=1.0, press=0.0, ground=False)


def twisted_state(sc, frames):
    """(q_t, v_t, t) after `frames` frames of the direct solver (10 iterations each)."""
    sim = lgsim.Sim(sc)
    sim.step(frames, iters=10, stats=False)
    q, v, _ = sim.read_state()
    t = frames * sc.h
    sim.close()
    return q, v, t


def energies(sc, q_t, v_t, t, global_step, checkpoints, q0=None):
    """Objective at q^0 (q0, or q~ when None) and at the iterates q^k of one frame, k in
    checkpoints, and the last iterate."""
    sim = lgsim.Sim(sc, global_step=global_step)
    sim.set_iterate_state(q_t, v_t, q0, t, [], [], np.zeros((0, 3)))
    out, done = {0: sim.lg_energy()}, 0
    for k in checkpoints:
        sim.run_iterations(k - done)
        done = k
        out[k] = sim.lg_energy()
    q_last = sim.read_iterate(0)[0]
    sim.close()
    return out, q_last


def start_state(sc, q_t, v_t, t, q_star):
    """q^0: the predicted state q~ with the pinned nodes already at their targets (taken
    from the converged iterate), as hard boundary conditions would place them; the
    comparison then measures how each global step propagates the boundary motion and
    the elastic response, not how fast it pulls the pins (a penalty 1e3 times stiffer
    than the rest of the system) onto their targets."""
    sim = lgsim.Sim(sc)
    sim.set_iterate_state(q_t, v_t, None, t, [], [], np.zeros((0, 3)))
    q_pred = sim.read_iterate(0)[0]
    sim.close()
    q0 = q_pred.copy()
    q0[sc.pin_nodes] = q_star[sc.pin_nodes]
    return q0


def ms_per_iteration(sc, q_t, v_t, t, global_step, k=200):
    """GPU time per L-G iteration: graph-replayed frames of 10 and 10 + k iterations."""
    import torch
    sim = lgsim.Sim(sc, global_step=global_step)
    sim.step(1, iters=10, stats=False)
    sim.save_state()
    res = {}
    for iters in (10, 10 + k):
        sim.restore_state()
        sim.step(1, iters=iters, stats=False)  # capture
        torch.cuda.synchronize()
        best = float("inf")
        for _ in range(3):
            sim.restore_state()
            torch.cuda.synchronize()
            a = time.perf_counter()
            sim.step(1, iters=iters, stats=False)
            torch.cuda.synchronize()
            best = min(best, time.perf_counter() - a)
        res[iters] = best
    sim.close()
    return 1e3 * (res[10 + k] - res[10]) / k


def compare(E, frame=300, checkpoints=CHECKPOINTS, truth_iters=3000):
    sc = bar(E)
    q_t, v_t, t = twisted_state(sc, frame)
    _, q_star = energies(sc, q_t, v_t, t, lgsim.SIM_GLOBAL_DIRECT, (truth_iters,))
    q0 = start_state(sc, q_t, v_t, t, q_star)
    direct, _ = energies(sc, q_t, v_t, t, lgsim.SIM_GLOBAL_DIRECT, tuple(checkpoints) + (truth_iters,), q0)
    jac, _ = energies(sc, q_t, v_t, t, lgsim.SIM_GLOBAL_JACOBI, checkpoints, q0)
    e_star, e0 = direct[truth_iters], direct[0]
    rel = lambda e: (e - e_star) / (e0 - e_star)
    return {"E": E, "frame": frame, "truth_iters": truth_iters,
            "floor": abs(direct[checkpoints[-1]] - e_star) / (e0 - e_star),
            "direct": {k: rel(direct[k]) for k in checkpoints},
            "jacobi": {k: rel(jac[k]) for k in checkpoints},
            "ms_per_iter": {"direct": ms_per_iteration(sc, q_t, v_t, t, lgsim.SIM_GLOBAL_DIRECT),
                            "jacobi": ms_per_iteration(sc, q_t, v_t, t, lgsim.SIM_GLOBAL_JACOBI)}}
