"""Shared helpers of the GPU parity tests: run the HIP solver and the FP64 oracle from
the same input state (rounded to float32-representable values) and compare."""
import numpy as np

from oracle.sim import OracleSim


def f32(a):
    return np.asarray(a, np.float64).astype(np.float32).astype(np.float64)


def rel_inf(a, b, scale=None):
    s = np.abs(b).max() if scale is None else scale
    return float(np.abs(a - b).max() / max(s, 1e-300))


def oracle_state_after(scene, frames, iters=None):
    """Oracle state (q_t, v_t, t, contacts, lambda) at the start of frame `frames`:
    runs `frames` frames, then detects the next frame's contacts."""
    o = OracleSim(scene)
    if frames:
        o.step(frames, iters=iters)
    q_t, q_pred, fc, lam = o.begin_frame()
    return o, q_t, o.v.copy(), o.t, fc, lam


def iterate_pair(sim_factory, scene, q_t, v_t, q_k, t, node, obst, lam, k=1, cr="fixed", cr_iters=None,
                 gpu_cr_iters=None, sim_opt=None, oracle_opt=None):
    """k iterations from the same state on the GPU and in the oracle.

    cr="fixed": both run the scene's (or cr_iters) CR iterations; cr="exact": the oracle
    solves the Schur system exactly and the GPU runs gpu_cr_iters iterations (converged
    mode).  Returns (q_gpu, lam_gpu, q_oracle, lam_oracle, oracle, fc)."""
    q_t, v_t, q_k, lam = f32(q_t), f32(v_t), f32(q_k), f32(lam)
    opt = dict(sim_opt or {})
    if gpu_cr_iters is not None:
        opt["cr_iters"] = gpu_cr_iters
    elif cr_iters is not None:
        opt["cr_iters"] = cr_iters
    sim = sim_factory(scene, **opt)
    sim.set_iterate_state(q_t, v_t, q_k, t, node, obst, lam)
    sim.run_iterations(k)
    qg, lg = sim.read_iterate(len(node))
    o = OracleSim(scene, cr_iters=cr_iters, **(oracle_opt or {}))
    o.t = t
    q_pred = o.predict(q_t, v_t)
    fc = o.contacts_from_keys(node, obst, q_t)
    q, lo = q_k.copy(), lam.copy()
    for _ in range(k):
        q, lo, info = o.iterate(fc, q, lo, q_t, q_pred, t + o.h, cr=cr)
    o.last_info = info
    sim.close()
    return qg, lg, q, lo, o, fc


def impulse_rounding_bound(o, lam_scale, ops=1):
    """First-order bound on the impulse error that float32 evaluation of the constraint
    right-hand side (h - Omega H u) / h^2 causes in the last oracle iteration: each of its
    two terms carries `ops` float32 roundings of relative size u = 2^-24 (storing it), and
    the solve propagates it by |M^-1| componentwise.  The terms cancel (they are large next
    to their difference at first impact), which is what makes this bound exceed 1e-4."""
    info = getattr(o, "last_info", None)
    if not info or "cr_matrix" not in info:
        return 0.0
    h2 = o.h * o.h
    M = info["cr_matrix"]
    hv = info["hvec"].reshape(-1)
    rhs = info["cr_rhs"]
    om_hu = hv - h2 * rhs                           # Omega H u, recovered from rhs
    d = ops * 2.0 ** -24 * (np.abs(hv) + np.abs(om_hu)) / h2
    return float((np.abs(np.linalg.inv(M)) @ d).max() / lam_scale)


def ulp_sensitivity(scene, t, fc, q_t, v_t, lam, draws=3, seed=0):
    """Largest relative change of the oracle's one-iteration impulses (exact constraint
    solve, iterate q^0 = q~) when its float32 inputs q_t, v_t and lambda each move by one
    float32 ulp in random directions: how strongly the iteration map amplifies rounding
    of the contact state.  At a resting contact the Fischer-Burmeister Jacobians make
    this amplification large (about 250 ulp per input ulp on a one-voxel cube)."""
    rng = np.random.default_rng(seed)

    def run(qt, vt, lm):
        o = OracleSim(scene)
        o.t = t
        q_pred = o.predict(qt, vt)
        fc2 = o.contacts_from_keys(fc.node, fc.obst, qt)
        _, lo, _ = o.iterate(fc2, f32(q_pred), lm.copy(), qt, q_pred, t + o.h, cr="exact")
        return lo

    q_t, v_t, lam = f32(q_t), f32(v_t), f32(lam)
    base = run(q_t, v_t, lam)
    scale = max(np.abs(base).max(), 1e-30)
    worst = 0.0
    for _ in range(draws):
        bump = lambda a: f32(a * (1.0 + rng.choice([-1.0, 1.0], a.shape) * 2.0 ** -23))
        worst = max(worst, float(np.abs(run(bump(q_t), bump(v_t), bump(lam)) - base).max() / scale))
    return worst



def _cr_float32(M, b, iters):
    """The Conjugate Residual recurrence of oracle.cr in float32 arithmetic (float32 M,
    b, vectors and inner products): a model of what any float32 solver computes."""
    M = np.asarray(M, np.float32)
    b = np.asarray(b, np.float32)
    x = np.zeros_like(b)
    r = b.copy()
    Ar = M @ r
    p, Ap = r.copy(), Ar.copy()
    rAr = np.float32(r @ Ar)
    for _ in range(iters):
        ApAp = np.float32(Ap @ Ap)
        if ApAp == 0.0 or rAr == 0.0:
            break
        a = rAr / ApAp
        x = x + a * p
        r = r - a * Ap
        Ar = M @ r
        rn = np.float32(r @ Ar)
        beta = rn / rAr
        rAr = rn
        p = r + beta * p
        Ap = Ar + beta * Ap
    return x.astype(np.float64)


def float32_cr_position_gap(o, q_k, q_pred, t, fc, lam):
    """Relative change of the oracle's positions after one iteration with the paper's
    fixed CR count when that CR runs in float32 arithmetic instead of float64 (same
    Schur system, rounded to float32).  A fixed-count Krylov iterate of an
    ill-conditioned system (Fischer-Burmeister compliances span many decades when
    contacts slide or separate) moves this much with float32 rounding alone; two float32
    solvers with different summation orders are each about this far from the float64
    iterate, so the device's paper-mode positions are held to 1e-5 plus twice this gap."""
    info = o.last_info
    if "cr_matrix" not in info:
        return 0.0
    from oracle.cr import conjugate_residual
    M, rhs, Om = info["cr_matrix"], info["cr_rhs"], info["Omega"]
    b = o.rhs(q_k, q_pred, t + o.h)

    def positions(dl):
        return o.solve(b + o.h * o.h * o.H_T(fc, Om * (lam + dl.reshape(-1, 3))))

    q64 = positions(conjugate_residual(lambda x: M @ x, rhs, o.cr_iters))
    return rel_inf(positions(_cr_float32(M, rhs, o.cr_iters)), q64)
