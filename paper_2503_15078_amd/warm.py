"""Learned warm start of the contact impulses: parameter initialisation, data from the
solver itself, training on the device with the library's own kernels, and the
comparison with the previous-frame warm start.

The network, its 16 input features and its target (the frame's converged impulse
scaled by h^2 K_jj / l) are defined in the library header next to sim_set_warm_model.
Inputs and targets are standardised for training; the standardisation is folded into
the first and last layers afterwards, so the device evaluates raw features.
"""
from __future__ import annotations

import time

import numpy as np

from . import lgsim, scenes

N_PARAMS = lgsim.MLP_N_PARAMS
SHAPES = [("W1", (128, 16)), ("b1", (128,)), ("W2", (128, 128)), ("b2", (128,)), ("W3", (16, 128)),
          ("b3", (16,))]
N_FEAT = 12  # used inputs (16 with padding)
N_OUT = 3
MODES = ((lgsim.SIM_WARM_PREV, "plain"), (lgsim.SIM_WARM_MLP, "learned"),
         (lgsim.SIM_WARM_MLP_PERSIST, "learned_persist"))


def split(flat):
    out, o = {}, 0
    for k, shp in SHAPES:
        n = int(np.prod(shp))
        out[k] = np.asarray(flat[o:o + n], np.float64).reshape(shp)
        o += n
    return out


def join(p):
    return np.concatenate([np.asarray(p[k], np.float64).reshape(-1) for k, _ in SHAPES]).astype(np.float32)


def init_params(seed=0):
    """He-normal hidden layers, small output layer, zero biases; padding entries zero."""
    rng = np.random.default_rng(seed)
    p = {k: np.zeros(s) for k, s in SHAPES}
    p["W1"][:, :N_FEAT] = rng.normal(0.0, np.sqrt(2.0 / N_FEAT), (128, N_FEAT))
    p["W2"] = rng.normal(0.0, np.sqrt(2.0 / 128), (128, 128))
    p["W3"][:N_OUT] = rng.normal(0.0, np.sqrt(0.1 / 128), (N_OUT, 128))
    return join(p)


def standardiser(feat, tgt):
    """Per-feature mean/std of the used inputs and per-output std of the targets."""
    mu = feat[:, :N_FEAT].mean(0)
    sd = feat[:, :N_FEAT].std(0)
    sd = np.where(sd > 1e-6, sd, 1.0)
    ts = tgt.std(0)
    ts = np.where(ts > 1e-9, ts, 1.0)
    return mu, sd, ts


def standardise(feat, tgt, mu, sd, ts):
    x = np.zeros((len(feat), 16), np.float32)
    x[:, :N_FEAT] = (feat[:, :N_FEAT] - mu) / sd
    return x, (tgt / ts).astype(np.float32)


def fold(flat, mu, sd, ts):
    """Parameters acting on raw features and producing raw targets."""
    p = split(flat)
    W1 = p["W1"].copy()
    W1[:, :N_FEAT] = p["W1"][:, :N_FEAT] / sd
    b1 = p["b1"] - W1[:, :N_FEAT] @ mu
    W3 = p["W3"].copy()
    b3 = p["b3"].copy()
    W3[:N_OUT] *= ts[:, None]
    b3[:N_OUT] *= ts
    return join({"W1": W1, "b1": b1, "W2": p["W2"], "b2": p["b2"], "W3": W3, "b3": b3})


# ------------------------------------------------------------------ data
def training_scenes(seeds):
    """(kind, seed, scene, frames) by seed mod 4: 0 small cube drops (model, E,
    mu, nodes and drop height varied per seed; whole drops), 1 and 2 the first frames of
    teaser-scale stars, 3 blobs resting on tilted planes.  Only
    frames whose NCP residual reaches 1e-6 m contribute samples."""
    out = []
    for s in seeds:
        rng = np.random.default_rng(s)
        k = s % 4
        if k == 0:
            sc = scenes.cube_drop(s, model=[1, 2][int(rng.integers(2))], nodes=int(rng.integers(4, 8)),
                                  mu=float(rng.uniform(0.1, 0.9)), E=float(10 ** rng.uniform(4.5, 6)),
                                  height=float(rng.uniform(0.01, 0.08)))
            out.append(("cube", s, sc, 60))
        elif k in (1, 2):
            out.append(("teaser", s, scenes.teaser_scene(s), 2))
        else:
            for i, b in enumerate(scenes.batch_scenes(s, count=4, hi=6000)):
                out.append(("blob", 100 * s + i, b, 3))
    return out


def generate(seeds, frames=None, cr_iters=300, cr_tol=1e-3, log=print):
    """Run each scene frame by frame until the NCP residual is <= 1e-6 m (at most 100
    iterations), with the previous-frame warm start, and keep (features, converged
    impulse) of every frame that converged."""
    feats, tgts = [], []
    for kind, seed, sc, nf in training_scenes(seeds):
        nf = nf if frames is None else min(nf, frames)
        t0 = time.perf_counter()
        sim = lgsim.Sim(sc, cr_iters=cr_iters, cr_tol=cr_tol, max_iters=100)
        sim.record_training_pairs(True)
        kept = conv = 0
        for f in range(nf):
            try:
                st = sim.step(1, iters=0)[0]
            except lgsim.SimError as e:
                log(f"  {kind} {seed}: stop at frame {f}: {e}")
                break
            if st["ncp"] <= 1e-6 and st["contacts"] > 0:
                _, _, x, t = sim.read_training_pairs()
                feats.append(x)
                tgts.append(t)
                kept += len(x)
                conv += 1
        sim.close()
        log(f"  {kind} seed {seed}: {conv}/{nf} frames converged, {kept} samples, {time.perf_counter() - t0:.1f} s")
    return np.concatenate(feats), np.concatenate(tgts)


# ------------------------------------------------------------------ training
def train(feat, tgt, epochs=30, batch=8192, lr=2e-3, seed=0, log=print):
    """Adam on the device (library kernels); returns folded parameters and the history."""
    import torch
    mu, sd, ts = standardiser(feat, tgt)
    x, t = standardise(feat, tgt, mu, sd, ts)
    n = len(x)
    rng = np.random.default_rng(seed)
    perm = rng.permutation(n)
    n_val = max(1, n // 20)
    val, tr = perm[:n_val], perm[n_val:]
    dev = torch.device("cuda:0")
    X = torch.from_numpy(x[tr]).to(dev)
    T = torch.from_numpy(t[tr]).to(dev)
    Xv = torch.from_numpy(x[val]).to(dev)
    Tv = torch.from_numpy(t[val]).to(dev)
    net = lgsim.Mlp(init_params(seed))
    steps_per_epoch = max(1, len(tr) // batch)
    total = epochs * steps_per_epoch
    hist = []
    step = 0
    g = torch.Generator(device="cpu").manual_seed(seed)
    for ep in range(epochs):
        order = torch.randperm(len(tr), generator=g).to(dev)
        for b in range(steps_per_epoch):
            idx = order[b * batch:(b + 1) * batch]
            rate = lr * 0.5 * (1.0 + np.cos(np.pi * step / total))  # cosine decay
            net.train_step(X[idx].contiguous(), T[idx].contiguous(), rate)
            step += 1
        vl = val_loss(net, Xv, Tv)
        hist.append(vl)
        log(f"  epoch {ep + 1}/{epochs}: validation loss {vl:.4e} (standardised)")
    params = fold(net.params(), mu, sd, ts)
    net.close()
    return params, {"val_loss": hist, "n_train": int(len(tr)), "n_val": int(n_val), "steps": step}


def val_loss(net, Xv, Tv):
    tot, n = 0.0, 0
    for b in range(0, len(Xv), lgsim.MLP_MAX_BATCH):
        xb, tb = Xv[b:b + lgsim.MLP_MAX_BATCH].contiguous(), Tv[b:b + lgsim.MLP_MAX_BATCH].contiguous()
        _, loss = net.gradient(xb, tb)
        tot += loss * len(xb)
        n += len(xb)
    return tot / max(n, 1)


# ------------------------------------------------------------------ evaluation
def compare(scene, params, frames, cr_iters=300, cr_tol=1e-3, max_iters=100, cr_variant=0):
    """Frames to NCP residual <= 1e-6 m (at most max_iters iterations) from the same start
    with the previous-frame warm start ("plain"), the learned one on every contact
    ("learned") and the learned one on persisting contacts only ("learned_persist"):
    per-frame iterations, ms (device-synchronised) and residual reached."""
    import torch
    out = {}
    for mode, name in MODES:
        sim = lgsim.Sim(scene, cr_iters=cr_iters, cr_tol=cr_tol, cr_variant=cr_variant, max_iters=max_iters)
        sim.set_warm_model(params)
        sim.set_warm_mode(mode)
        its, ms, res, kept = [], [], [], 0
        for _ in range(frames):
            torch.cuda.synchronize()
            a = time.perf_counter()
            st = sim.step(1, iters=0)[0]
            torch.cuda.synchronize()
            ms.append(1e3 * (time.perf_counter() - a))
            its.append(st["iters"])
            res.append(st["ncp"])
            if mode != lgsim.SIM_WARM_PREV and st["contacts"]:
                jp, jl, _ = sim.read_warm_judge(cap=0)
                kept += int(np.sum(jl < jp))
        sim.close()
        out[name] = {"iters": its, "ms": ms, "ncp": res, "learned_start_kept": kept}
    return out


def trajectory(scene, params, frames, modes=MODES, cr_iters=300, cr_tol=1e-3, max_iters=100, log=None):
    """One handle runs `frames` frames of the scene from its initial state once per warm
    start mode (restored between modes), every frame until the NCP residual is <= 1e-6 m
    or max_iters iterations.  Per mode: per-frame iterations, ms (device-synchronised),
    residual, and the frames whose judge kept the network's start."""
    import torch
    sim = lgsim.Sim(scene, cr_iters=cr_iters, cr_tol=cr_tol, max_iters=max_iters)
    if params is not None:
        sim.set_warm_model(params)
    sim.save_state()
    out = {}
    for mode, name in modes:
        sim.restore_state()
        sim.set_warm_mode(mode)
        its, ms, res, kept = [], [], [], 0
        for f in range(frames):
            torch.cuda.synchronize()
            a = time.perf_counter()
            st = sim.step(1, iters=0)[0]
            torch.cuda.synchronize()
            ms.append(1e3 * (time.perf_counter() - a))
            its.append(int(st["iters"]))
            res.append(float(st["ncp"]))
            if mode != lgsim.SIM_WARM_PREV and st["contacts"]:
                jp, jl, _ = sim.read_warm_judge(cap=0)
                kept += int(np.sum(jl < jp))
        out[name] = {"iters": its, "ms": ms, "ncp": res, "learned_start_kept": kept}
        if log:
            log(f"  {name}: {np.mean(its):.2f} iterations/frame, {np.mean(ms):.3f} ms/frame")
    sim.close()
    return out


def summarise(runs, tol=1e-6):
    """Converged fraction, mean / median / p90 of ms and iterations per frame."""
    out = {}
    for name, r in runs.items():
        ms, its, res = np.asarray(r["ms"]), np.asarray(r["iters"]), np.asarray(r["ncp"])
        out[name] = {"frames": int(len(ms)), "converged_fraction": round(float(np.mean(res <= tol)), 4),
                     "ms_per_frame_mean": round(float(ms.mean()), 4),
                     "ms_per_frame_median": round(float(np.median(ms)), 4),
                     "ms_per_frame_p90": round(float(np.percentile(ms, 90)), 4),
                     "iters_per_frame_mean": round(float(its.mean()), 3),
                     "iters_per_frame_median": float(np.median(its)),
                     "iters_per_frame_p90": float(np.percentile(its, 90)),
                     "frames_network_start_kept": int(r.get("learned_start_kept", 0))}
    return out
