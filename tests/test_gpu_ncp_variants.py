"""GPU parity of the minimum-map rows and the mass-inverse preconditioner against the
FP64 oracle (App. B; Sec. 5.4; Sec. 7, stick-sliding test), through the C-ABI, and the
stick-sliding precision of the four combinations on the GPU.

Tolerances as in test_gpu_parity: positions 1e-5 relative per iteration, impulses of the
converged constraint solve 1e-4.  The min-map rows switch on delta_n <= r_n lambda_n and
|vdot_f| <= r_f (mu lambda_n - |lambda_f|); the tests check that the state keeps every
contact at least 1e-3 (relative) away from those switches, so float32 and float64 take
the same branch."""
import numpy as np
import pytest

from oracle.sim import OracleSim
from paper_2503_15078_amd import lgsim, scenes, stick_slide
from tests.parity_util import impulse_rounding_bound, iterate_pair, rel_inf

pytestmark = pytest.mark.gpu

VARIANTS = [
    (lgsim.SIM_NCP_MINMAP, lgsim.SIM_PRECOND_DELASSUS, "minmap", "delassus"),
    (lgsim.SIM_NCP_FB, lgsim.SIM_PRECOND_MASS, "fb", "mass"),
    (lgsim.SIM_NCP_MINMAP, lgsim.SIM_PRECOND_MASS, "minmap", "mass"),
]


def _state(frames=14):
    sc = scenes.cube_drop(0)
    o = OracleSim(sc)
    o.step(frames)
    q_t, q_pred, fc, lam = o.begin_frame()
    return sc, o, q_t, q_pred, fc, lam


def _switch_margin(o, fc, q, q_t, lam):
    """Smallest relative distance of the state to the min-map switches."""
    ev = o.contact_eval(fc, q, q_t, lam)
    dn, vf = ev["delta_n"], ev["vdot_f"]
    a = np.abs(dn - fc.r_n * lam[:, 0]) / np.maximum(np.abs(dn) + np.abs(fc.r_n * lam[:, 0]), 1e-30)
    s = np.sqrt((vf ** 2).sum(1))
    gam = fc.mu * lam[:, 0] - np.sqrt((lam[:, 1:] ** 2).sum(1))
    act = lam[:, 0] > 0
    b = np.abs(s - fc.r_f * gam) / np.maximum(s + np.abs(fc.r_f * gam), 1e-30)
    return float(min(a.min(), b[act].min() if act.any() else 1.0))


@pytest.mark.parametrize("ncp,pre,oncp,opre", VARIANTS)
def test_one_iteration_matches_oracle(ncp, pre, oncp, opre):
    sc, o, q_t, q_pred, fc, lam = _state()
    sopt, oopt = dict(ncp=ncp, precond=pre), dict(ncp=oncp, precond=opre)
    qg, _, qo, _, o2, fc2 = iterate_pair(lgsim.Sim, sc, q_t, o.v, q_pred, o.t, fc.node, fc.obst, lam, k=1,
                                         sim_opt=sopt, oracle_opt=oopt)
    f32 = lambda a: np.asarray(a).astype(np.float32).astype(np.float64)
    if oncp == "minmap":
        m = _switch_margin(o2, fc2, f32(q_pred), f32(q_t), f32(lam))
        print(f"switch margin {m:.2e}")
        assert m >= 1e-3
    assert rel_inf(qg, qo) <= 1e-5, rel_inf(qg, qo)
    _, lg, _, lo, o3, _ = iterate_pair(lgsim.Sim, sc, q_t, o.v, q_pred, o.t, fc.node, fc.obst, lam, k=1,
                                       cr="exact", gpu_cr_iters=100, sim_opt=sopt, oracle_opt=oopt)
    scale = max(np.abs(lo).max(), 1e-3 * o3.mass.sum() * 9.81)
    err = np.abs(lg - lo).max() / scale
    print(f"{oncp}/{opre}: position gap {rel_inf(qg, qo):.2e}, impulse gap {err:.2e} (float32 right-hand-side "
          f"rounding bound {impulse_rounding_bound(o3, scale):.2e})")
    assert err <= 1e-4


@pytest.mark.parametrize("ncp,pre,oncp,opre", VARIANTS)
def test_drop_trajectory_follows_oracle(ncp, pre, oncp, opre):
    """30 frames of the cube drop (impact and settling): the GPU trajectory stays within
    1e-3 m of the oracle's with the same rows and preconditioner."""
    sc = scenes.cube_drop(0)
    sim = lgsim.Sim(sc, ncp=ncp, precond=pre)
    o = OracleSim(sc, ncp=oncp, precond=opre)
    worst = 0.0
    for f in range(30):
        sim.step(1, stats=False)
        o.step(1)
        q, _, _ = sim.read_state()
        worst = max(worst, np.abs(q - o.q).max())
    sim.close()
    print(f"{oncp}/{opre}: worst position gap over 30 frames {worst:.2e} m")
    assert worst <= 1e-3


def test_stick_slide_precision_on_gpu():
    """Sec. 7's stick-sliding test on the GPU: the method's preconditioner (Delassus
    diagonal) with FB rows separates sticking from sliding at offsets down to 0.01 from
    mu* (the paper reports 0.001), the mass-inverse one only from 0.1 (the paper's 0.1)."""
    res = {k: stick_slide.scan(k, ladder=(0.1, 0.05, 0.02, 0.01)) for k in ("fb_delassus", "fb_mass")}
    for k, r in res.items():
        print(k, r["precision"], [(x["offset"], round(x["v_slide"], 5), round(x["v_stick"], 6)) for x in r["rows"]])
    assert res["fb_delassus"]["precision"] is not None and res["fb_delassus"]["precision"] <= 0.01
    assert res["fb_mass"]["precision"] == 0.1
