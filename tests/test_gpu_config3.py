"""GPU parity on the stiffness and model sweep (Sec. 7, hyperelastic material evaluation:
the twisting bar): the 40x10x10-node bar (12k DoFs) of stable Neo-Hookean and
Mooney-Rivlin material (c10 = c01), E in {1e4, 1e6, 1e8}, nu = 0.4, twisted by 720 degrees
end to end and pressed into the ground plane, friction mu in {0, 0.8}.

From the same float32 state (the twisted, pressed bar with its contacts) one L-G iteration
on the GPU and in the oracle: positions within 1e-5 with the paper's 10 CR steps and with
the constraint system solved to convergence; impulses in converged mode within 1e-4."""
import math

import numpy as np
import pytest

from oracle.sim import OracleSim
from paper_2503_15078_amd import lgsim, scenes
from tests.parity_util import f32, iterate_pair, rel_inf

pytestmark = pytest.mark.gpu


def twisted_pressed(sc, turns=2.0, press=0.002, seed=0):
    """Rest shape twisted about the bar's axis by `turns` full turns (linear along x, the
    ends at -turns/2 and +turns/2), then lowered so that its lowest node is `press` below
    the plane z = 0; a small seeded perturbation and velocity."""
    X = sc.rest
    x0, x1 = X[:, 0].min(), X[:, 0].max()
    th = 2.0 * math.pi * turns * ((X[:, 0] - x0) / (x1 - x0) - 0.5)
    cy, cz = X[:, 1].mean(), X[:, 2].mean()
    y, z = X[:, 1] - cy, X[:, 2] - cz
    q = X.copy()
    q[:, 1] = cy + np.cos(th) * y - np.sin(th) * z
    q[:, 2] = cz + np.sin(th) * y + np.cos(th) * z
    rng = np.random.default_rng(seed)
    q += rng.uniform(-2e-5, 2e-5, q.shape)
    q[:, 2] += -press - q[:, 2].min()
    v = rng.normal(0.0, 0.01, q.shape)
    return q, v


@pytest.mark.parametrize("model", [scenes.MODEL_SNH, scenes.MODEL_MR])
@pytest.mark.parametrize("E", [1e4, 1e6, 1e8])
@pytest.mark.parametrize("mu", [0.0, 0.8])
def test_twisted_pressed_bar_iteration(model, E, mu):
    sc = scenes.twist_bar(0, model=model, E=E, nu=0.4, mu=mu)
    q_t, v_t = twisted_pressed(sc, seed=int(math.log10(E)))
    q_t, v_t = f32(q_t), f32(v_t)
    o = OracleSim(sc)
    q_pred = o.predict(q_t, v_t)
    node, obst = o.detect(q_t, q_pred)
    assert 10 <= len(node) <= 2048
    lam = np.zeros((len(node), 3))
    qg, _, qo, _, _, _ = iterate_pair(lgsim.Sim, sc, q_t, v_t, q_pred, 0.0, node, obst, lam, k=1)
    paper_pos = rel_inf(qg, qo)
    qg, lg_, qo, lo, o2, _ = iterate_pair(lgsim.Sim, sc, q_t, v_t, q_pred, 0.0, node, obst, lam, k=1,
                                          cr="exact", gpu_cr_iters=1000)
    lam_scale = max(np.abs(lo).max(), 1e-3 * o2.mass.sum() * 9.81)
    gap = rel_inf(lg_, lo, lam_scale)
    print(f"model {model} E {E:.0e} mu {mu}: {len(node)} contacts, positions {paper_pos:.2e} (10 CR) "
          f"{rel_inf(qg, qo):.2e} (converged), impulses {gap:.2e}")
    assert paper_pos <= 1e-5
    assert rel_inf(qg, qo) <= 1e-5
    assert gap <= 1e-4
