"""Thin ctypes binding of liblgsim_hip.so (argument marshalling only).

Every step of the solver runs in the library's HIP kernels; this module only
converts numpy arrays / scene descriptions into the C structures declared in
``include/lgsim.h`` and back.  PyTorch is used only to pass device memory and
streams (``read_state_device``).  Loading fails loudly if the library is missing.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_NAME = "liblgsim_hip.so"
LIB_PATH = os.path.join(_HERE, LIB_NAME)

SIM_OK = 0
SIM_WARM_ZERO, SIM_WARM_PREV, SIM_WARM_MLP, SIM_WARM_MLP_PERSIST = 0, 1, 2, 3
SIM_CR_TEXTBOOK, SIM_CR_PIPELINED = 0, 1
SIM_NCP_FB, SIM_NCP_MINMAP = 0, 1
SIM_PRECOND_DELASSUS, SIM_PRECOND_MASS = 0, 1
SIM_GLOBAL_DIRECT, SIM_GLOBAL_JACOBI = 0, 1
SIM_LG_PD, SIM_LG_ADMM = 0, 1
ERRORS = {-1: "SIM_E_ARG", -2: "SIM_E_MESH", -3: "SIM_E_NOT_SPD", -4: "SIM_E_NOMEM",
          -5: "SIM_E_DEVICE", -6: "SIM_E_STATE", -7: "SIM_E_DIVERGED", -8: "SIM_E_CAPACITY"}


class SimError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{ERRORS.get(code, code)}: {msg}")
        self.code = code


class sim_mesh(C.Structure):
    _fields_ = [("n_nodes", C.c_int32), ("n_tets", C.c_int32),
                ("rest_xyz", C.POINTER(C.c_double)), ("tets", C.POINTER(C.c_int32)),
                ("init_xyz", C.POINTER(C.c_double)), ("init_vel", C.POINTER(C.c_double)),
                ("n_pins", C.c_int32), ("pin_nodes", C.POINTER(C.c_int32)),
                ("pin_group", C.POINTER(C.c_int32))]


class sim_material(C.Structure):
    _fields_ = [("model", C.c_int32), ("E", C.c_double), ("nu", C.c_double), ("rho", C.c_double),
                ("tet_model", C.POINTER(C.c_int32)), ("tet_E", C.POINTER(C.c_double)),
                ("tet_nu", C.POINTER(C.c_double))]


class sim_options(C.Structure):
    _fields_ = [("gravity", C.c_double * 3), ("pin_weight_scale", C.c_double),
                ("contact_margin", C.c_double), ("cr_iters", C.c_int32), ("warm", C.c_int32),
                ("ncp_tol", C.c_double), ("max_iters", C.c_int32), ("max_contacts", C.c_int32),
                ("hip_stream", C.c_void_p), ("cr_tol", C.c_double), ("cr_variant", C.c_int32),
                ("graph", C.c_int32), ("ncp", C.c_int32), ("precond", C.c_int32),
                ("global_step", C.c_int32), ("lg_form", C.c_int32), ("self_contact", C.c_int32),
                ("self_mu", C.c_double)]


class sim_tuning(C.Structure):
    _fields_ = [("cr_blocks", C.c_int32), ("cr_variant", C.c_int32), ("seg_floats", C.c_int32),
                ("elem_block", C.c_int32), ("row_group", C.c_int32), ("col_group", C.c_int32),
                ("ms_frame", C.c_float)]


class sim_obstacle(C.Structure):
    _fields_ = [("type", C.c_int32), ("geom", C.c_double * 10), ("mu", C.c_double),
                ("vel", C.c_double * 3)]


class sim_stats(C.Structure):
    _fields_ = [("iters_done", C.c_int32), ("n_contacts", C.c_int32), ("ncp_res", C.c_double),
                ("ms_frame", C.c_float), ("ms_phase", C.c_float * 8)]


class sim_contact(C.Structure):
    _fields_ = [("node", C.c_int32), ("obstacle", C.c_int32), ("frame", C.c_double * 9),
                ("lambda_", C.c_double * 3), ("gap", C.c_double)]


_lib = None


def load():
    """Load the built library (raises if it was not built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with __graft_entry__.build()")
    try:
        # share torch's HIP runtime: torch links the runtime by file name, the library
        # by soname; loading torch first makes both resolve to one runtime instance
        import torch  # noqa: F401
    except ImportError:
        pass
    lib = C.CDLL(LIB_PATH)
    P = C.POINTER
    d, i32, i64 = C.c_double, C.c_int32, C.c_int64
    sig = {
        "sim_options_default": [P(sim_options)],
        "sim_create": [P(sim_mesh), P(sim_material), d, P(sim_options), P(C.c_void_p)],
        "sim_set_obstacles": [C.c_void_p, i32, P(sim_obstacle)],
        "sim_set_pin_motion": [C.c_void_p, i32, P(d), P(d), P(d)],
        "sim_step": [C.c_void_p, i32, i32, P(sim_stats)],
        "sim_read_state": [C.c_void_p, P(d), P(d), P(sim_contact), i32, P(i32)],
        "sim_read_state_device": [C.c_void_p, C.c_void_p, C.c_void_p],
        "sim_destroy": [C.c_void_p],
        "sim_set_solver": [C.c_void_p, i32, d, i32],
        "sim_set_warm_model": [C.c_void_p, P(C.c_float), i32],
        "sim_set_graph": [C.c_void_p, i32],
        "sim_time_kernel": [C.c_void_p, i32, i32, P(C.c_float)],
        "sim_profile_cr": [C.c_void_p, i32, P(C.c_float)],
        "sim_read_cr_stamps": [C.c_void_p, P(C.c_uint64), i32, P(i32)],
        "sim_get_tuning": [C.c_void_p, P(sim_tuning)],
        "sim_set_tuning": [C.c_void_p, P(sim_tuning)],
        "sim_autotune": [C.c_void_p, i32, i32, i32, P(sim_tuning)],
        "sim_set_warm_mode": [C.c_void_p, i32],
        "sim_record_training_pairs": [C.c_void_p, i32],
        "sim_read_training_pairs": [C.c_void_p, P(i32), P(i32), P(C.c_float), P(C.c_float), i32, P(i32)],
        "sim_read_warm_judge": [C.c_void_p, P(C.c_float), P(C.c_float), i32, P(i32)],
        "sim_surface_triangles": [C.c_void_p, P(i32), i32, P(i32)],
        "mlp_create": [P(C.c_float), i32, P(C.c_void_p)],
        "mlp_set_params": [C.c_void_p, P(C.c_float), i32],
        "mlp_get_params": [C.c_void_p, P(C.c_float), i32],
        "mlp_forward": [C.c_void_p, C.c_void_p, C.c_void_p, i32, C.c_void_p],
        "mlp_train_step": [C.c_void_p, C.c_void_p, C.c_void_p, i32, C.c_float, C.c_void_p, P(C.c_float)],
        "mlp_gradient": [C.c_void_p, C.c_void_p, C.c_void_p, i32, C.c_void_p, P(C.c_float), P(C.c_float)],
        "mlp_destroy": [C.c_void_p],
        "mlp_gradient_noalloc": [C.c_void_p, C.c_void_p, C.c_void_p, i32, C.c_void_p, C.c_void_p],
        "sim_save_state": [C.c_void_p],
        "sim_restore_state": [C.c_void_p],
        "sim_create_batch": [i32, P(sim_mesh), P(sim_material), P(i32), P(P(sim_obstacle)), d,
                             P(sim_options), P(C.c_void_p)],
        "sim_batch_info": [C.c_void_p, P(i32), P(i32)],
        "sim_set_iterate_state": [C.c_void_p, P(d), P(d), P(d), d, i32, P(sim_contact)],
        "sim_run_iterations": [C.c_void_p, i32],
        "sim_read_iterate": [C.c_void_p, P(d), P(d)],
        "sim_global_solve": [C.c_void_p, P(d), P(d)],
        "sim_lg_energy": [C.c_void_p, P(d)],
        "sim_debug_rhs": [C.c_void_p, P(d)],
        "sim_debug_delassus": [C.c_void_p, P(d)],
        "lg_host_create": [P(sim_mesh), P(sim_material), d, d, i32, P(C.c_void_p)],
        "lg_host_info": [C.c_void_p, P(i64)],
        "lg_host_ordering": [C.c_void_p, P(i32), P(i32)],
        "lg_host_dense_A": [C.c_void_p, P(d)],
        "lg_host_dense_S": [C.c_void_p, P(d)],
        "lg_host_apply_StS": [C.c_void_p, P(d), P(d)],
        "lg_host_destroy": [C.c_void_p],
    }
    for name, args in sig.items():
        if not hasattr(lib, name):
            continue
        f = getattr(lib, name)
        f.argtypes = args
        f.restype = C.c_int
    lib.sim_last_error.argtypes = []
    lib.sim_last_error.restype = C.c_char_p
    _lib = lib
    return lib


def _check(rc):
    if rc != SIM_OK:
        raise SimError(rc, _lib.sim_last_error().decode())


def _dp(a):
    return a.ctypes.data_as(C.POINTER(C.c_double)) if a is not None else None


def _fp(a):
    return a.ctypes.data_as(C.POINTER(C.c_float)) if a is not None else None


def _ip(a):
    return a.ctypes.data_as(C.POINTER(C.c_int32)) if a is not None else None


class _Marshal:
    """Keeps the numpy buffers of one scene alive while the C structs point at them."""

    def __init__(self, scene):
        self.rest = np.ascontiguousarray(scene.rest, np.float64)
        self.tets = np.ascontiguousarray(scene.tets, np.int32)
        self.init = None if scene.init_pos is None else np.ascontiguousarray(scene.init_pos, np.float64)
        self.vel = None if scene.init_vel is None else np.ascontiguousarray(scene.init_vel, np.float64)
        self.pins = np.ascontiguousarray(scene.pin_nodes, np.int32)
        self.groups = np.ascontiguousarray(scene.pin_group, np.int32)
        self.mesh = sim_mesh(len(self.rest), len(self.tets), _dp(self.rest), _ip(self.tets),
                             _dp(self.init), _dp(self.vel), len(self.pins),
                             _ip(self.pins) if len(self.pins) else None,
                             _ip(self.groups) if len(self.pins) else None)
        self.tm = None if scene.tet_model is None else np.ascontiguousarray(scene.tet_model, np.int32)
        self.tE = None if scene.tet_E is None else np.ascontiguousarray(scene.tet_E, np.float64)
        self.tnu = None if scene.tet_nu is None else np.ascontiguousarray(scene.tet_nu, np.float64)
        self.mat = sim_material(scene.model, scene.E, scene.nu, scene.rho, _ip(self.tm), _dp(self.tE),
                                _dp(self.tnu))
        obs = (sim_obstacle * max(1, len(scene.obstacles)))()
        for k, ob in enumerate(scene.obstacles):
            obs[k].type = ob.type
            for q in range(10):
                obs[k].geom[q] = float(ob.geom[q])
            obs[k].mu = ob.mu
            for q in range(3):
                obs[k].vel[q] = float(ob.vel[q])
        self.obs = obs
        self.n_obs = len(scene.obstacles)


def options_for(scene, **kw):
    lib = load()
    o = sim_options()
    _check(lib.sim_options_default(C.byref(o)))
    for q in range(3):
        o.gravity[q] = float(scene.gravity[q])
    o.pin_weight_scale = scene.pin_weight_scale
    o.contact_margin = scene.margin
    o.cr_iters = scene.cr_iters
    o.self_contact = int(bool(getattr(scene, "self_contact", False)))
    o.self_mu = float(getattr(scene, "self_mu", 0.0))
    for k, v in kw.items():
        setattr(o, k, v)
    return o


class HostPrecompute:
    """Host-only products of sim_create (ordering, S) for inspection on the CPU."""

    def __init__(self, scene, want_dense_S=False):
        lib = load()
        self._m = _Marshal(scene)
        h = C.c_void_p()
        _check(lib.lg_host_create(C.byref(self._m.mesh), C.byref(self._m.mat), scene.h,
                                  scene.pin_weight_scale, int(want_dense_S), C.byref(h)))
        self.h = h
        info = np.zeros(8, np.int64)
        _check(lib.lg_host_info(h, info.ctypes.data_as(C.POINTER(C.c_int64))))
        self.n, self.m, self.nnz_S, self.nnz_L, self.row_floats, self.max_depth, self.chains = map(int, info[:7])

    def ordering(self):
        perm = np.zeros(self.n, np.int32)
        parent = np.zeros(self.n, np.int32)
        _check(_lib.lg_host_ordering(self.h, _ip(perm), _ip(parent)))
        return perm, parent

    def dense_A(self):
        A = np.zeros((self.n, self.n))
        _check(_lib.lg_host_dense_A(self.h, _dp(A)))
        return A

    def dense_S(self):
        S = np.zeros((self.n, self.n))
        _check(_lib.lg_host_dense_S(self.h, _dp(S)))
        return S

    def apply_StS(self, b):
        b = np.ascontiguousarray(b, np.float64)
        u = np.zeros_like(b)
        _check(_lib.lg_host_apply_StS(self.h, _dp(b), _dp(u)))
        return u

    def __del__(self):
        if getattr(self, "h", None) and _lib is not None:
            _lib.lg_host_destroy(self.h)
            self.h = None


class Sim:
    """One solver handle (a single scene or a batch)."""

    def __init__(self, scene=None, batch=None, stream=None, **opt):
        lib = load()
        self.scenes = [scene] if scene is not None else list(batch)
        self._ms = [_Marshal(s) for s in self.scenes]
        s0 = self.scenes[0]
        self.opt = options_for(s0, **opt)
        if stream is not None:
            self.opt.hip_stream = C.c_void_p(stream)
        h = C.c_void_p()
        if scene is not None:
            _check(lib.sim_create(C.byref(self._ms[0].mesh), C.byref(self._ms[0].mat), s0.h,
                                  C.byref(self.opt), C.byref(h)))
            self.h = h
            if self._ms[0].n_obs:
                _check(lib.sim_set_obstacles(h, self._ms[0].n_obs, self._ms[0].obs))
        else:
            k = len(self.scenes)
            meshes = (sim_mesh * k)(*[m.mesh for m in self._ms])
            mats = (sim_material * k)(*[m.mat for m in self._ms])
            nobs = np.array([m.n_obs for m in self._ms], np.int32)
            obsp = (C.POINTER(sim_obstacle) * k)(*[C.cast(m.obs, C.POINTER(sim_obstacle)) for m in self._ms])
            _check(lib.sim_create_batch(k, meshes, mats, _ip(nobs), obsp, s0.h, C.byref(self.opt),
                                        C.byref(h)))
            self.h = h
        self.n = sum(s.n for s in self.scenes)
        groups = [s for s in self.scenes if len(s.pin_lin_vel)]
        if scene is not None and len(s0.pin_lin_vel):
            lin = np.ascontiguousarray(s0.pin_lin_vel, np.float64)
            ang = np.ascontiguousarray(s0.pin_ang_vel, np.float64)
            piv = np.ascontiguousarray(s0.pin_pivot, np.float64)
            _check(lib.sim_set_pin_motion(h, len(lin), _dp(lin), _dp(ang), _dp(piv)))
        del groups

    def set_obstacles(self, obstacles):
        """Replace the obstacle set (single-scene handles), e.g. to move obstacles between
        frames."""
        obs = (sim_obstacle * max(1, len(obstacles)))()
        for k, ob in enumerate(obstacles):
            obs[k].type = ob.type
            for q in range(10):
                obs[k].geom[q] = float(ob.geom[q])
            obs[k].mu = ob.mu
            for q in range(3):
                obs[k].vel[q] = float(ob.vel[q])
        _check(_lib.sim_set_obstacles(self.h, len(obstacles), obs))

    def step(self, frames=1, iters=None, stats=True):
        iters = self.scenes[0].iters if iters is None else iters
        st = (sim_stats * frames)() if stats else None
        _check(_lib.sim_step(self.h, frames, iters, st))
        if not stats:
            return None
        return [dict(iters=s.iters_done, contacts=s.n_contacts, ncp=s.ncp_res, ms=s.ms_frame,
                     phases=list(s.ms_phase)) for s in st]

    def read_state(self, cap=0):
        q = np.zeros((self.n, 3))
        v = np.zeros((self.n, 3))
        nc = C.c_int32(0)
        _check(_lib.sim_read_state(self.h, _dp(q), _dp(v), None, 0, C.byref(nc)))
        contacts = None
        if nc.value > 0:
            buf = (sim_contact * nc.value)()
            _check(_lib.sim_read_state(self.h, None, None, buf, nc.value, C.byref(nc)))
            contacts = dict(node=np.array([c.node for c in buf], np.int64),
                            obst=np.array([c.obstacle for c in buf], np.int64),
                            frame=np.array([list(c.frame) for c in buf]).reshape(-1, 3, 3),
                            lam=np.array([list(c.lambda_) for c in buf]),
                            gap=np.array([c.gap for c in buf]))
        else:
            contacts = dict(node=np.zeros(0, np.int64), obst=np.zeros(0, np.int64),
                            frame=np.zeros((0, 3, 3)), lam=np.zeros((0, 3)), gap=np.zeros(0))
        return q, v, contacts

    def set_solver(self, cr_iters, cr_tol=0.0, cr_variant=0):
        _check(_lib.sim_set_solver(self.h, int(cr_iters), float(cr_tol), int(cr_variant)))

    # ---- launch configuration
    def set_graph(self, on):
        _check(_lib.sim_set_graph(self.h, int(bool(on))))

    def time_kernel(self, which, reps=50):
        """Average ms of `reps` back-to-back launches of the S pass (0), the S^T pass (1) or
        the local step (2) on the current buffers (sim_time_kernel)."""
        ms = C.c_float(0.0)
        _check(_lib.sim_time_kernel(self.h, int(which), int(reps), C.byref(ms)))
        return float(ms.value)

    def profile_cr(self, reps=20):
        """Constraint-solve launch profile: ms per launch (HIP events), in-kernel us,
        set-up us, us per exchange, us of barrier wait per exchange, exchanges."""
        out = np.zeros(6, np.float32)
        _check(_lib.sim_profile_cr(self.h, int(reps), _fp(out)))
        keys = ("ms_per_launch", "kernel_us", "setup_us", "exchange_us", "barrier_wait_us", "exchanges")
        return {k: float(v) for k, v in zip(keys, out)}

    def cr_stamps(self):
        """Wall-clock stamps (ticks) of the last profile_cr's stamped launch: start, end,
        then per barrier (entry, exit, data read, products done; 0 where none)."""
        n = C.c_int32(0)
        _check(_lib.sim_read_cr_stamps(self.h, None, 0, C.byref(n)))
        out = np.zeros(n.value, np.uint64)
        if n.value:
            _check(_lib.sim_read_cr_stamps(self.h, out.ctypes.data_as(C.POINTER(C.c_uint64)), n.value, C.byref(n)))
        return out

    def tuning(self):
        t = sim_tuning()
        _check(_lib.sim_get_tuning(self.h, C.byref(t)))
        return {k: getattr(t, k) for k, _ in sim_tuning._fields_}

    def set_tuning(self, **kw):
        t = sim_tuning()
        _check(_lib.sim_get_tuning(self.h, C.byref(t)))
        for k, v in kw.items():
            setattr(t, k, v)
        _check(_lib.sim_set_tuning(self.h, C.byref(t)))

    def autotune(self, frames=3, iters=5, allow_pipelined=True):
        t = sim_tuning()
        _check(_lib.sim_autotune(self.h, int(frames), int(iters), int(bool(allow_pipelined)), C.byref(t)))
        return {k: getattr(t, k) for k, _ in sim_tuning._fields_}

    # ---- learned warm start
    def set_warm_model(self, params):
        p = np.ascontiguousarray(params, np.float32)
        _check(_lib.sim_set_warm_model(self.h, _fp(p), int(p.size)))

    def set_warm_mode(self, warm):
        _check(_lib.sim_set_warm_mode(self.h, int(warm)))

    def record_training_pairs(self, on=True):
        _check(_lib.sim_record_training_pairs(self.h, int(bool(on))))

    def read_training_pairs(self, cap=None):
        """(node, obstacle, features [c][16], scaled impulses [c][3]) of the last frame's
        contacts, canonical order."""
        cap = int(self.opt.max_contacts) if cap is None else cap
        node = np.zeros(cap, np.int32)
        obst = np.zeros(cap, np.int32)
        feat = np.zeros((cap, 16), np.float32)
        tgt = np.zeros((cap, 3), np.float32)
        n = C.c_int32(0)
        _check(_lib.sim_read_training_pairs(self.h, _ip(node), _ip(obst), _fp(feat), _fp(tgt), cap, C.byref(n)))
        c = n.value
        return node[:c].copy(), obst[:c].copy(), feat[:c].copy(), tgt[:c].copy()

    def read_warm_judge(self, cap=None):
        """Scores of the last frame's two start candidates per scene (previous-frame,
        network's: the NCP residual each leaves in the frame start's linear contact
        problem) and the network's candidate impulses [c][3] (canonical order)."""
        cap = int(self.opt.max_contacts) if cap is None else cap
        k = len(self.scenes)
        res = np.zeros(2 * k, np.float32)
        lam = np.zeros((max(cap, 1), 3), np.float32)
        n = C.c_int32(0)
        _check(_lib.sim_read_warm_judge(self.h, _fp(res), _fp(lam), cap, C.byref(n)))
        return res[:k].astype(np.float64), res[k:].astype(np.float64), lam[:n.value].astype(np.float64)

    def surface_triangles(self):
        """Surface triangles of a self-contact handle [T][3] (caller node ids)."""
        n = C.c_int32(0)
        _check(_lib.sim_surface_triangles(self.h, None, 0, C.byref(n)))
        tris = np.zeros((max(n.value, 1), 3), np.int32)
        _check(_lib.sim_surface_triangles(self.h, _ip(tris), n.value, C.byref(n)))
        return tris[:n.value].astype(np.int64)

    def save_state(self):
        _check(_lib.sim_save_state(self.h))

    def restore_state(self):
        _check(_lib.sim_restore_state(self.h))

    def read_state_device(self, out_tensor, stream=None):
        """Copy positions (float32 [3][n], caller order) into a device tensor."""
        _check(_lib.sim_read_state_device(self.h, C.c_void_p(out_tensor.data_ptr()),
                                          C.c_void_p(stream) if stream else None))

    def set_iterate_state(self, q_t, v_t, q_k, t, node, obst, lam):
        c = len(node)
        buf = (sim_contact * max(1, c))()
        for j in range(c):
            buf[j].node = int(node[j])
            buf[j].obstacle = int(obst[j])
            for q in range(3):
                buf[j].lambda_[q] = float(lam[j][q])
        qk = None if q_k is None else _dp(np.ascontiguousarray(q_k, np.float64))  # None: q^0 = q~
        _check(_lib.sim_set_iterate_state(self.h, _dp(np.ascontiguousarray(q_t, np.float64)),
                                          _dp(np.ascontiguousarray(v_t, np.float64)), qk, float(t), c, buf))

    def run_iterations(self, k=1):
        _check(_lib.sim_run_iterations(self.h, k))

    def read_iterate(self, c):
        q = np.zeros((self.n, 3))
        lam = np.zeros((max(c, 1), 3))
        _check(_lib.sim_read_iterate(self.h, _dp(q), _dp(lam)))
        return q, lam[:c]

    def lg_energy(self):
        """The L-G objective at the current iterate (sim_lg_energy)."""
        e = C.c_double(0.0)
        _check(_lib.sim_lg_energy(self.h, C.byref(e)))
        return e.value

    def global_solve(self, b):
        b = np.ascontiguousarray(b, np.float64)
        u = np.zeros_like(b)
        _check(_lib.sim_global_solve(self.h, _dp(b), _dp(u)))
        return u

    def debug_rhs(self):
        r = np.zeros((self.n, 3))
        _check(_lib.sim_debug_rhs(self.h, _dp(r)))
        return r

    def debug_delassus(self, c):
        K = np.zeros((max(c, 1), max(c, 1)))
        _check(_lib.sim_debug_delassus(self.h, _dp(K)))
        return K[:c, :c]

    def close(self):
        if getattr(self, "h", None) and _lib is not None:
            _lib.sim_destroy(self.h)
            self.h = None

    def __del__(self):
        self.close()


MLP_N_PARAMS = 20752
MLP_MAX_BATCH = 16384
MLP_NOALLOC_MAX_BATCH = 4096


def _stream_ptr():
    import torch
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


class Mlp:
    """Trainer of the warm-start network (device-resident parameters and Adam state).
    Batches are float32 torch tensors on the device: x [n][16], t [n][3]."""

    def __init__(self, params):
        load()
        p = np.ascontiguousarray(params, np.float32)
        h = C.c_void_p()
        _check(_lib.mlp_create(_fp(p), int(p.size), C.byref(h)))
        self.h = h

    def set_params(self, params):
        p = np.ascontiguousarray(params, np.float32)
        _check(_lib.mlp_set_params(self.h, _fp(p), int(p.size)))

    def params(self):
        p = np.zeros(MLP_N_PARAMS, np.float32)
        _check(_lib.mlp_get_params(self.h, _fp(p), MLP_N_PARAMS))
        return p

    def forward(self, x):
        import torch
        assert x.is_cuda and x.dtype == torch.float32 and x.is_contiguous() and x.shape[1] == 16
        y = torch.empty((x.shape[0], 3), dtype=torch.float32, device=x.device)
        _check(_lib.mlp_forward(self.h, C.c_void_p(x.data_ptr()), C.c_void_p(y.data_ptr()), int(x.shape[0]),
                                _stream_ptr()))
        return y

    def _batch(self, x, t):
        import torch
        assert x.is_cuda and t.is_cuda and x.dtype == torch.float32 and t.dtype == torch.float32
        assert x.is_contiguous() and t.is_contiguous() and x.shape[1] == 16 and t.shape[1] == 3
        assert x.shape[0] == t.shape[0]
        return C.c_void_p(x.data_ptr()), C.c_void_p(t.data_ptr()), int(x.shape[0])

    def train_step(self, x, t, lr, want_loss=False):
        xp, tp, n = self._batch(x, t)
        loss = C.c_float(0.0)
        _check(_lib.mlp_train_step(self.h, xp, tp, n, float(lr), _stream_ptr(),
                                   C.byref(loss) if want_loss else None))
        return float(loss.value) if want_loss else None

    def gradient(self, x, t):
        xp, tp, n = self._batch(x, t)
        g = np.zeros(MLP_N_PARAMS, np.float32)
        loss = C.c_float(0.0)
        _check(_lib.mlp_gradient(self.h, xp, tp, n, _stream_ptr(), _fp(g), C.byref(loss)))
        return g, float(loss.value)

    def close(self):
        if self.h:
            _check(_lib.mlp_destroy(self.h))
            self.h = None


def mlp_gradient_noalloc(params, x, t, out):
    """Gradient and loss of the network into out [MLP_N_PARAMS + 1] (float32 device
    tensors params [MLP_N_PARAMS], x [n][16], t [n][3]), on the current stream, with no
    device allocation in the library (its fixed scratch array)."""
    import torch
    load()
    for a in (params, x, t, out):
        assert a.is_cuda and a.dtype == torch.float32 and a.is_contiguous()
    assert x.shape[0] == t.shape[0] and params.numel() == MLP_N_PARAMS and out.numel() == MLP_N_PARAMS + 1
    _check(_lib.mlp_gradient_noalloc(C.c_void_p(params.data_ptr()), C.c_void_p(x.data_ptr()),
                                     C.c_void_p(t.data_ptr()), int(x.shape[0]), C.c_void_p(out.data_ptr()),
                                     _stream_ptr()))
