#!/usr/bin/env python
"""Benchmark of the local-global solver with frictional contact on one MI355X.

Workload: the teaser-scale scene (seeded extruded star, 19,472 nodes = 58,416 DoFs,
82,875 tets, stable Neo-Hookean E = 1e6, nu = 0.45, h = 0.01 s) in its canonical
state with exactly 800 contacts, 5 local-global iterations per frame and 10 CR
iterations.  One step = one whole frame of the hot path (predicted state, collision
detection + compaction, Delassus operator, warm start, 5 iterations of local step /
S pass / contact evaluation / CR / force update / S^T pass, integration), restarted
from the same device-resident state each time so that every timed frame sees exactly
800 contacts.  value = ms per local-global iteration = frame time / 5 (as the paper's
per-iteration figure, which includes the once-per-frame Schur complement).

Before timing, the library's autotuner picks the launch configuration (CR grid and
form, S-pass segment length, S / S^T group sizes, element block size) on this state; timed frames replay
a captured hipGraph.  Also reported: per-kernel times from HIP events on the solver's
stream in an eagerly launched pass (graph replays hide kernel boundaries), the
roofline of the dominant S-pass kernel, ms/frame when iterating until the NCP residual
is <= 1e-6 m with the previous-frame and with the learned warm start, throughput of a
64-scene batch, and the FP64 oracle timed on the host cores on one frame of the same
state (cpu_baseline).
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
PAPER_MS_PER_ITER = 11.95  # Table 3, Gingerbread Man 19.5k, RTX 4090 + i9-13900KF (context only)
ITERS = 5
TOL_CR, TOL_CR_ITERS, TOL_MAX_ITERS = 1e-3, 300, 100

COUNTER_PASS_LAUNCHES = 20
# HBM bytes per launch from rocprofv3 counters (FETCH_SIZE + WRITE_SIZE, scaled by a plain
# copy of known size; profiles/ holds the runs), per kernel and workload, or absent
# FETCH_SIZE is scaled by 2.0 and WRITE_SIZE by 1.0: on this GPU each TCC->EA read request
# moves 128 bytes (a plain 256 MiB copy makes 2,097,320 requests) while FETCH_SIZE counts 64,
# and WRITE_SIZE of the copy equals its bytes (profiles/hbm_counters.md)
TRAFFIC = {
    "k_cr<0>, 16 blocks, teaser": 4.7e6,
    "k_cr<0>, 32 blocks, teaser": 9.2e6,
    "k_cr<0>, 48 blocks, teaser": 10.6e6,
    "k_cr<0>, 64 blocks, teaser": 11.0e6,
    "k_cr<0>, 96 blocks, teaser": 11.1e6,
    "k_cr<0>, 128 blocks, teaser": 10.9e6,
    "k_cr<0>, 192 blocks, teaser": 12.2e6,
    "k_cr<0>, 256 blocks, teaser": 13.6e6,
    "k_cr<1>, 16 blocks, teaser": 5.5e6,
    "k_cr<1>, 32 blocks, teaser": 9.9e6,
    "k_cr<1>, 48 blocks, teaser": 11.1e6,
    "k_cr<1>, 64 blocks, teaser": 11.4e6,
    "k_cr<1>, 96 blocks, teaser": 11.2e6,
    "k_cr<1>, 128 blocks, teaser": 10.7e6,
    "k_cr<1>, 192 blocks, teaser": 11.4e6,
    "k_cr<1>, 256 blocks, teaser": 12.2e6,
    "k_spmv_S (+k_spmv_S_finish), batch": 2.2152e9,
    "k_spmv_St, batch": 2.2281e9,
    "k_element (local step), batch": 269.5e6,
    "k_element (local step), teaser": 12.7e6,
}
TRAFFIC_NOTE = ("rocprofv3 FETCH_SIZE x 2.0 + WRITE_SIZE x 1.0 per launch (profiles/hbm_counters.md); null where the "
                "launch configuration differs from the counted one")


def log(msg):
    print(msg, file=sys.stderr, flush=True)


CR_STEPS = 10
# local step: 4 node indices + 9 Dm^-1 entries + 4 material values in, 12 corner forces out;
# about 1.2 kflop per tet: the SVD's Jacobi sweeps and QR about 650, two Newton steps on the
# singular values about 330, deformation gradients, P = U s V^T and the corner forces about
# 200 (counters on the batch: 64 x SQ_INSTS_VALU_FLOPS_FP32 x lane utilisation / tets = 1181)
ELEM_BYTES_PER_TET = 4 * (4 + 9 + 4) + 4 * 12
ELEM_FLOP_PER_TET = 1200.0
FP32_PEAK_TFLOPS = 157.3


def _hbm_entry(kernel, nbytes, ms, note):
    ach = nbytes / (ms * 1e-3) / 1e9
    return {"kernel": kernel, "bound": "hbm", "achieved": round(ach, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(ach / HBM_PEAK_GBS, 4), "bytes_per_launch": int(nbytes), "avg_launch_ms": round(ms, 5),
            "note": note}


def _element_entry(kernel, tets, ms):
    gbs = tets * ELEM_BYTES_PER_TET / (ms * 1e-3) / 1e9
    tfl = tets * ELEM_FLOP_PER_TET / (ms * 1e-3) / 1e12
    return {"kernel": kernel, "bound": "alu", "achieved": round(tfl, 2), "peak": FP32_PEAK_TFLOPS, "unit": "TFLOP/s",
            "frac": round(tfl / FP32_PEAK_TFLOPS, 4), "hbm_GBps": round(gbs, 1),
            "hbm_frac": round(gbs / HBM_PEAK_GBS, 4), "tets": int(tets), "avg_launch_ms": round(ms, 5),
            "note": (f"{ELEM_BYTES_PER_TET} B and about {ELEM_FLOP_PER_TET:.0f} flop per tet; one thread per tet "
                     f"runs the SVD and a Newton solve on the singular values; VALU counters (profiles/"
                     f"element_valu_counters.md): VALU busy 0.69, lane utilisation 0.77")}


def _with_traffic(entry):
    """The counter-measured HBM bytes per launch of the entry's kernel and workload, and the
    rate they give at the entry's launch time (null where not counted)."""
    t = TRAFFIC.get(entry["kernel"])
    entry["traffic"] = t
    if t:
        entry["traffic_GBps"] = round(t / (entry["avg_launch_ms"] * 1e-3) / 1e9, 1)
        entry["traffic_frac"] = round(entry["traffic_GBps"] / HBM_PEAK_GBS, 4)
    return entry


def algorithmic_bytes(n, nnz_s):
    """Bytes one launch of each S-pass kernel must move (float32 values, index-free
    skyline rows / column paths): S values once, the input vector once, the output once."""
    s_pass = 4 * nnz_s + 12 * n + 12 * n
    st_pass = 4 * nnz_s + 12 * n + 12 * n + 12 * n  # y, q~ (base) in, q out
    return s_pass, st_pass


def copy_probe(torch, mib=256):
    """A plain float32 copy of `mib` MiB, three times: the reference kernel whose counter
    readings scale FETCH_SIZE / WRITE_SIZE to bytes."""
    a = torch.ones(mib << 18, dtype=torch.float32, device="cuda:0")
    b = torch.empty_like(a)
    for _ in range(3):
        torch.neg(a, out=b)
    torch.cuda.synchronize()
    out = {"kernel": "torch neg (elementwise)", "read_bytes": 4 * a.numel(), "write_bytes": 4 * a.numel()}
    del a, b
    return out


def counter_pass(sim):
    """Fixed launch sequence for counter collection: for each S-pass configuration (row
    group 1, 2, 4, 8 x segment 1024, 2048, 4096 floats) and then each S^T-pass column group
    (1, 2, 4, 8), 1 + COUNTER_PASS_LAUNCHES back-to-back launches; then the local step and
    the constraint solve; then the copy probes."""
    from paper_2503_15078_amd import lgsim
    seq = []
    for rg in (1, 2, 4, 8):
        for seg in (1024, 2048, 4096):
            sim.set_tuning(row_group=rg, seg_floats=seg)
            sim.time_kernel(0, COUNTER_PASS_LAUNCHES)
            seq.append(("S", rg, seg))
    for cg in (1, 2, 4, 8):
        sim.set_tuning(col_group=cg)
        sim.time_kernel(1, COUNTER_PASS_LAUNCHES)
        seq.append(("St", cg))
    sim.time_kernel(2, COUNTER_PASS_LAUNCHES)
    seq.append(("local_step",))
    # both CR forms at every grid the autotuner may choose (those the contact capacity allows)
    grids = sorted({sim.tuning()["cr_blocks"], 16, 32, 48, 64, 96, 128, 192, 256})
    for variant in (0, 1):
        sim.set_solver(CR_STEPS, 0.0, variant)
        for blocks in grids:
            try:
                sim.set_tuning(cr_blocks=blocks, cr_variant=variant)
            except lgsim.SimError:  # fewer blocks than the contact capacity needs
                continue
            sim.profile_cr(COUNTER_PASS_LAUNCHES)
            seq.append(("cr", variant, blocks, "then one stamped launch after an impulse-restoring copy"))
    return seq


def cpu_baseline(scene):
    """The FP64 oracle as it stands, one frame of the same state (bounded sample)."""
    from oracle.sim import OracleSim
    try:
        from threadpoolctl import threadpool_info
        cores = max([p.get("num_threads", 1) for p in threadpool_info()] + [1])
    except Exception:  # noqa: BLE001
        cores = 1
    t0 = time.perf_counter()
    o = OracleSim(scene)
    t_create = time.perf_counter() - t0
    t0 = time.perf_counter()
    q_t, q_pred, fc, lam = o.begin_frame()
    q = q_pred.copy()
    for _ in range(ITERS):
        q, lam, _ = o.iterate(fc, q, lam, q_t, q_pred, o.t + o.h)
    t_frame = time.perf_counter() - t0
    return {"value": round(1e3 * t_frame / ITERS, 3), "unit": "ms/iter", "cores": int(cores),
            "kind": "oracle",
            "sample": (f"one frame of the benchmark state ({fc.c} contacts): float64 collision detection, "
                       f"Delassus by {fc.c} sparse LU solves, {ITERS} L-G iterations with LU global solves; "
                       f"frame {t_frame:.2f} s, factorisation at creation {t_create:.2f} s not included; "
                       f"SuperLU solves single-threaded, dense BLAS on {cores} threads")}


def phase_pass(sim, frames):
    """Per-phase ms per launch from HIP events of eagerly launched frames (each from the
    saved state)."""
    import numpy as np
    sim.set_graph(False)
    ph = np.zeros(8)
    for _ in range(frames):
        sim.restore_state()
        st = sim.step(1, iters=ITERS, stats=True)
        ph += np.asarray(st[0]["phases"])
    sim.set_graph(True)
    ph /= frames
    ph[1:6] /= ITERS
    return ph


def warm_compare(sim, params):
    """Frame to NCP residual <= 1e-6 m from the benchmark state with the previous-frame
    warm start (none exists at this state: zero), the learned one on every contact and the
    learned one on persisting contacts only (every contact is new at this state: zero)."""
    import torch
    from paper_2503_15078_amd import lgsim, warm
    sim.set_warm_model(params)
    for mode, _ in warm.MODES:  # load every kernel of the learned start before timing
        sim.set_warm_mode(mode)
        sim.restore_state()
        sim.step(1, iters=1)
    out = {}
    for mode, name in warm.MODES:
        sim.set_warm_mode(mode)
        sim.restore_state()
        torch.cuda.synchronize()
        a = time.perf_counter()
        s = sim.step(1, iters=0)[0]
        torch.cuda.synchronize()
        out[name] = {"ms_per_frame": round(1e3 * (time.perf_counter() - a), 3), "iters": int(s["iters"]),
                     "ncp_res": float(s["ncp"])}
        if mode != lgsim.SIM_WARM_PREV:
            jp, jl, _ = sim.read_warm_judge(cap=0)
            out[name]["judge"] = {"score_previous_frame_start": float(jp[0]), "score_network_start": float(jl[0]),
                                  "kept": "network" if jl[0] < jp[0] else "previous_frame"}
    sim.set_warm_mode(lgsim.SIM_WARM_PREV)
    return out


def warm_drops(params, seeds=(1001, 1002, 1003), frames=60):
    """Held-out cube drops (5^3-node cubes), every frame to NCP residual <= 1e-6 m."""
    import numpy as np
    from paper_2503_15078_amd import scenes, warm
    agg = {name: [[], []] for _, name in warm.MODES}
    kept = {}
    for s in seeds:
        res = warm.compare(scenes.cube_drop(s), params, frames, cr_iters=TOL_CR_ITERS, cr_tol=TOL_CR,
                           max_iters=TOL_MAX_ITERS)
        for k, v in res.items():
            agg[k][0] += v["ms"]
            agg[k][1] += v["iters"]
            if k != "plain":
                kept[k] = kept.get(k, 0) + v["learned_start_kept"]
    out = {k: {"ms_per_frame": round(float(np.mean(v[0])), 4), "iters_per_frame": round(float(np.mean(v[1])), 3)}
           for k, v in agg.items()}
    for k in out:
        if k in kept:
            out[k]["frames_network_start_kept"] = kept[k]
    out["workload"] = f"cube drops, seeds {list(seeds)}, {frames} frames each"
    return out


def stiffness_sweep(frames):
    """The stiffness and model sweep: the 40x10x10-node bar (stable Neo-Hookean and
    Mooney-Rivlin with c10 = c01, E 1e4..1e8, nu 0.4) whose ends turn by +-360 degrees over 400
    frames while pressed 20% of its height into the plane, mu 0 / 0.2 / 0.8, 10 L-G
    iterations per frame: ms per frame over `frames` frames, the most contacts at the frames
    sampled every 50 (and the last), the NCP residual of the last frame, and whether every
    frame stayed finite."""
    import numpy as np
    import torch
    from paper_2503_15078_amd import lgsim, scenes
    rows = []
    for model, mname in ((scenes.MODEL_SNH, "stable_nh"), (scenes.MODEL_MR, "mooney_rivlin")):
        for E in (1e4, 1e5, 1e6, 1e7, 1e8):
            for mu in (0.0, 0.2, 0.8):
                sc = scenes.twist_bar(0, model=model, E=E, nu=0.4, mu=mu)
                sim = lgsim.Sim(sc)
                most, ok = 0, True
                torch.cuda.synchronize()
                a = time.perf_counter()
                try:
                    for f in range(frames):
                        st = sim.step(1, iters=10, stats=(f % 50 == 49 or f == frames - 1))
                        if st:
                            most = max(most, int(st[0]["contacts"]))
                            res = float(st[0]["ncp"])
                except lgsim.SimError as e:
                    ok, res = False, str(e)
                torch.cuda.synchronize()
                dt = time.perf_counter() - a
                q, v, _ = sim.read_state()
                sim.close()
                rows.append({"model": mname, "E": E, "mu": mu, "ms_per_frame": round(1e3 * dt / frames, 3),
                             "contacts_max": most, "ncp_res_last": res, "finite": ok and bool(np.isfinite(q).all()),
                             "speed_max": round(float(np.abs(v).max()), 4)})
    return {"workload": (f"bar 40x10x10 nodes (4000 nodes, 15795 tets), ends turned +-360 deg over 400 frames and "
                         f"pressed 20% into the plane, 10 L-G iterations/frame, {frames} frames per configuration"),
            "rows": rows}


def batch_throughput(count, steps):
    """A batch of `count` blobs on tilted planes in one handle: scenes x iterations / s, and the
    S-pass bandwidth at a size that does not fit the infinity cache."""
    import torch
    from paper_2503_15078_amd import lgsim, scenes
    scs = scenes.batch_scenes(0, count=count)
    t0 = time.perf_counter()
    sim = lgsim.Sim(batch=scs, max_contacts=32768)
    t_create = time.perf_counter() - t0
    sim.save_state()
    tune = sim.autotune(frames=1, iters=ITERS, allow_pipelined=True)
    nnz = sum(lgsim.HostPrecompute(s).nnz_S for s in scs)
    for _ in range(2):
        sim.restore_state()
        sim.step(1, iters=ITERS)
    torch.cuda.synchronize()
    a = time.perf_counter()
    for _ in range(steps):
        sim.restore_state()
        sim.step(1, iters=ITERS)
    torch.cuda.synchronize()
    dt = time.perf_counter() - a
    ph = phase_pass(sim, 2)
    n = sum(s.n for s in scs)
    b_s, b_st = algorithmic_bytes(n, nnz)
    sim.restore_state()
    sim.step(1, iters=ITERS)
    k_s, k_st, k_el = sim.time_kernel(0, 20), sim.time_kernel(1, 20), sim.time_kernel(2, 20)
    m = sum(len(s.tets) for s in scs)
    rl = [_hbm_entry("k_spmv_S (+k_spmv_S_finish), batch", b_s, k_s, "S (2.0 GB) streams from HBM every launch"),
          _hbm_entry("k_spmv_St, batch", b_st, k_st, "the column copy of S (2.0 GB) streams from HBM"),
          _element_entry("k_element (local step), batch", m, k_el)]
    rl = [_with_traffic(e) for e in rl]
    out = {"metric": "scenes x L-G iterations / s", "value": round(count * ITERS * steps / dt, 1),
           "scenes": count, "nodes": int(n), "tets": int(sum(len(s.tets) for s in scs)), "nnz_S": int(nnz),
           "ms_per_frame": round(1e3 * dt / steps, 3), "create_s": round(t_create, 1), "launch": tune,
           "S_pass_GBps": round(b_s / (ph[2] * 1e-3) / 1e9, 1),
           "St_pass_GBps": round(b_st / (ph[5] * 1e-3) / 1e9, 1),
           "St_pass_frac_of_hbm_peak": round(b_st / (ph[5] * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
           "rooflines": rl,
           "phases_ms_per_launch": [round(float(x), 5) for x in ph]}
    sim.close()
    return out


def mlp_throughput(steps=50):
    """Warm-start network on random features: Adam training steps (forward, backward, the
    gradient reduction and the update over the whole batch) and forward passes, per call
    and in samples/s, timed with events on the stream the calls run on."""
    import numpy as np
    import torch
    from paper_2503_15078_amd import lgsim, warm
    rng = np.random.default_rng(0)
    out = []
    for n in (8192, lgsim.MLP_MAX_BATCH):
        x = np.zeros((n, 16), np.float32)
        x[:, :12] = rng.normal(0, 1, (n, 12))
        X = torch.from_numpy(x).cuda()
        T = torch.from_numpy(rng.normal(0, 0.3, (n, 3)).astype(np.float32)).cuda()
        net = lgsim.Mlp(warm.init_params(0))
        res = {"batch": n}
        for name, call in (("train_step", lambda: net.train_step(X, T, 1e-3)), ("forward", lambda: net.forward(X))):
            for _ in range(5):
                call()
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            torch.cuda.synchronize()
            e0.record()
            for _ in range(steps):
                call()
            e1.record()
            torch.cuda.synchronize()
            us = 1e3 * e0.elapsed_time(e1) / steps
            res[f"{name}_us"] = round(us, 1)
            res[f"{name}_Msamples_per_s"] = round(n / us, 2)
        net.close()
        out.append(res)
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=40)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--tol-frames", type=int, default=3)
    ap.add_argument("--frame-dist", type=int, default=300,
                    help="frames of the per-frame median / p90 pass (after 20 warm-up frames; 0 skips it)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-tune", action="store_true", help="keep the default launch configuration")
    ap.add_argument("--launch", default=None,
                    help="fixed launch configuration cr_blocks,cr_variant,seg_floats,elem_block,row_group,"
                         "col_group (no autotuning)")
    ap.add_argument("--no-extras", action="store_true", help="skip the warm-start comparison and the batch")
    ap.add_argument("--batch-scenes", type=int, default=64)
    ap.add_argument("--traj-frames", type=int, default=100,
                    help="frames of each to-tolerance trajectory (held-out teaser seeds; 0: none)")
    ap.add_argument("--traj-seeds", type=int, default=1, help="held-out teaser seeds 1000, 1001, ...")
    ap.add_argument("--sweep-frames", type=int, default=400,
                    help="frames of each stiffness/model sweep configuration (0: none)")
    ap.add_argument("--batch-only", action="store_true", help="only the batch measurement (for profiling)")
    ap.add_argument("--mlp-only", action="store_true", help="only the warm-start network's training and "
                                                             "inference throughput")
    ap.add_argument("--counter-pass", action="store_true",
                    help="only the fixed S-pass launch sequence for rocprofv3 counters (teaser, or the batch "
                         "with --batch-only), then copy probes of 256 MiB and 4 GiB")
    ap.add_argument("--copy-probe", action="store_true",
                    help="after the benchmark, run a plain float32 copy of 256 MiB three times "
                         "(reference kernel for scaling the HBM byte counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "the solver runs on one GPU; a scene batch is the unit of work and "
                                   "multi-GPU sharding is not implemented",
                          "n_gpus": args.gpus}))
        sys.exit(2)

    import numpy as np
    import torch

    from paper_2503_15078_amd import lgsim, scenes

    torch.cuda.init()
    if args.batch_only and args.counter_pass:
        sim = lgsim.Sim(batch=scenes.batch_scenes(0, count=args.batch_scenes), max_contacts=32768)
        sim.step(1, iters=ITERS)
        seq = counter_pass(sim)
        sim.close()
        print(json.dumps({"counter_pass": seq, "launches_per_config": 1 + COUNTER_PASS_LAUNCHES,
                          "copy_probe": [copy_probe(torch, 256), copy_probe(torch, 4096)]}))
        return
    if args.batch_only:
        print(json.dumps({"batch": batch_throughput(args.batch_scenes, 10)}))
        return
    if args.mlp_only:
        print(json.dumps({"warm_mlp_throughput": mlp_throughput()}))
        return
    log("building scene")
    sc = scenes.teaser_scene(0)
    hp = lgsim.HostPrecompute(sc)
    nnz_s = hp.nnz_S
    del hp
    log(f"n={sc.n} m={sc.m} nnz(S)={nnz_s}; creating solver")
    sim = lgsim.Sim(sc)
    sim.save_state()
    if args.counter_pass:
        sim.step(1, iters=ITERS)
        seq = counter_pass(sim)
        sim.close()
        print(json.dumps({"counter_pass": seq, "launches_per_config": 1 + COUNTER_PASS_LAUNCHES,
                          "copy_probe": [copy_probe(torch, 256), copy_probe(torch, 4096)]}))
        return
    if args.launch:
        cb, cv, sf, eb, rg, cg = (int(x) for x in args.launch.split(","))
        sim.set_tuning(cr_blocks=cb, cr_variant=cv, seg_floats=sf, elem_block=eb, row_group=rg, col_group=cg)
        tune = sim.tuning()
    else:
        tune = sim.tuning() if args.no_tune else sim.autotune(frames=3, iters=ITERS, allow_pipelined=True)
    log(f"launch configuration: {tune}")

    def frame():
        sim.restore_state()
        sim.step(1, iters=ITERS)

    log("warmup")
    for _ in range(args.warmup):
        frame()
    torch.cuda.synchronize()
    log(f"timed: {args.steps} frames")
    t0 = time.perf_counter()
    for _ in range(args.steps):
        frame()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ms_frame = 1e3 * (t1 - t0) / args.steps
    ms_iter = ms_frame / ITERS
    # per-frame distribution: 20 more warm-up frames, then 300 frames each followed by a
    # device synchronisation (so each time includes one host round trip, which the
    # back-to-back figure above does not)
    per_frame = []
    if args.frame_dist > 0:
        log(f"per-frame times: {args.frame_dist} frames, each synchronised")
        for i in range(20 + args.frame_dist):
            a = time.perf_counter()
            frame()
            torch.cuda.synchronize()
            if i >= 20:
                per_frame.append(1e3 * (time.perf_counter() - a))
    sim.restore_state()
    contacts = sim.step(1, iters=ITERS, stats=True)[0]["contacts"]

    log("per-kernel pass (eager launches)")
    per_launch = phase_pass(sim, max(5, args.steps // 4))
    names = ["frame_setup", "local_step_rhs", "S_pass", "contact_eval", "cr_and_force_update", "St_pass",
             "integrate", "residual"]
    phase_ms = {k: round(float(v), 5) for k, v in zip(names, per_launch)}
    b_s, b_st = algorithmic_bytes(sc.n, nnz_s)
    # Kernel durations for the rooflines: the constraint solve (the dominant kernel) with
    # a pair of HIP events around each launch on the solver's stream, plus its in-kernel
    # stamps; the S / S^T passes and the local step as back-to-back launches between one
    # pair of events (per-launch events would add their own overhead to these short ones)
    sim.restore_state()
    sim.step(1, iters=ITERS)
    crp = sim.profile_cr(20)
    k_ms = {"S_pass": sim.time_kernel(0, 100), "St_pass": sim.time_kernel(1, 100),
            "local_step": sim.time_kernel(2, 100)}
    cr_bytes = CR_STEPS * 4 * contacts * contacts  # K once per CR step, per launch
    cr_ms = crp["ms_per_launch"]
    cr_share = ITERS * cr_ms / ms_frame
    cr_ach = cr_bytes / (cr_ms * 1e-3) / 1e9
    exch = crp["exchange_us"] * crp["exchanges"]
    roofline = {
        "bound": "hbm", "kernel": f"k_cr<{tune.get('cr_variant', 0)}> (constraint solve, {CR_STEPS} CR steps)",
        "dominant_share_of_frame": round(cr_share, 3),
        "achieved": round(cr_ach, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": round(cr_ach / HBM_PEAK_GBS, 4),
        "traffic": TRAFFIC.get(f"k_cr<{tune.get('cr_variant', 0)}>, {tune.get('cr_blocks')} blocks, teaser"),
        "traffic_note": TRAFFIC_NOTE,
        "bytes_per_launch": int(cr_bytes), "avg_launch_ms": round(cr_ms, 5),
        "note": ("latency-bound: the Delassus rows (4 c^2 B) stay in LDS, so HBM bytes are not what limits it; "
                 "each CR step needs a device-wide exchange of the step's vectors and inner products"),
        "per_launch_us": {"kernel": round(crp["kernel_us"], 2), "setup_before_first_exchange": round(crp["setup_us"], 2),
                          "exchanges": int(crp["exchanges"]), "per_exchange": round(crp["exchange_us"], 3),
                          "barrier_wait_per_exchange": round(crp["barrier_wait_us"], 3),
                          "all_exchanges": round(exch, 2),
                          "compute_rest": round(crp["kernel_us"] - crp["setup_us"] - exch, 2)}}
    tets_per_launch = sc.m
    rooflines = [
        _hbm_entry("k_spmv_S (+k_spmv_S_finish), teaser", b_s, k_ms["S_pass"],
                   "S (108 MB) stays in the 256 MB infinity cache across launches: not an HBM figure"),
        _hbm_entry("k_spmv_St, teaser", b_st, k_ms["St_pass"], "infinity-cache resident, as the S pass"),
        _element_entry("k_element (local step), teaser", tets_per_launch, k_ms["local_step"]),
    ]
    rooflines = [_with_traffic(e) for e in rooflines]
    log("to-tolerance frames")
    # iterate until the NCP residual is <= 1e-6 m; the constraint solve runs CR to a
    # relative residual of TOL_CR (at most TOL_CR_ITERS iterations) instead of 10
    sim.set_solver(TOL_CR_ITERS, TOL_CR, tune.get("cr_variant", 0))
    tol = []
    for _ in range(args.tol_frames):
        sim.restore_state()
        torch.cuda.synchronize()
        a = time.perf_counter()
        s = sim.step(1, iters=0, stats=True)[0]
        torch.cuda.synchronize()
        tol.append((1e3 * (time.perf_counter() - a), s["iters"], s["ncp"]))

    extras = {}
    weights = os.path.join(ROOT, "paper_2503_15078_amd", "warm_mlp.npz")
    if not args.no_extras and os.path.exists(weights):
        log("learned vs previous-frame warm start")
        params = np.load(weights)["params"]
        extras["warm_start_benchmark_state"] = warm_compare(sim, params)
        extras["warm_start_held_out_drops"] = warm_drops(params)
    if not args.no_extras:
        extras["warm_mlp_throughput"] = mlp_throughput()
    sim.close()
    if not args.no_extras and args.traj_frames > 0:
        seeds = [1000 + k for k in range(args.traj_seeds)]
        log(f"to-tolerance trajectories: held-out teaser seeds {seeds}, {args.traj_frames} frames")
        from paper_2503_15078_amd import warm
        params = np.load(weights)["params"] if os.path.exists(weights) else None
        modes = warm.MODES if params is not None else warm.MODES[:1]
        runs = {}
        for sd in seeds:
            r = warm.trajectory(scenes.teaser_scene(sd), params, args.traj_frames, modes=modes, cr_iters=TOL_CR_ITERS,
                                cr_tol=TOL_CR, max_iters=TOL_MAX_ITERS, log=log)
            for k, v in r.items():
                agg = runs.setdefault(k, {"iters": [], "ms": [], "ncp": [], "learned_start_kept": 0})
                for q in ("iters", "ms", "ncp"):
                    agg[q] += v[q]
                agg["learned_start_kept"] += v["learned_start_kept"]
        extras["to_tolerance_trajectories"] = {
            "workload": (f"teaser-scale stars, held-out seeds {seeds}, {args.traj_frames} frames each from rest, "
                         f"every frame until NCP residual <= 1e-6 m or {TOL_MAX_ITERS} L-G iterations; CR to "
                         f"relative {TOL_CR} (at most {TOL_CR_ITERS} steps)"),
            **warm.summarise(runs)}
    if not args.no_extras:
        log("stick-sliding precision (NCP rows x preconditioner)")
        from paper_2503_15078_amd import stick_slide
        extras["stick_slide_precision"] = {
            "test": ("stiff block (E=1e8) on a 10 deg slope, mu* = tan 10 deg, 10 L-G / 24 CR iterations, 40 frames; "
                     "precision = smallest offset from mu* above which sliding (>= 0.5 x analytic velocity) "
                     "and sticking (< 0.1 x) are both classified correctly; precision_moves: sliding >= 0.1 x "
                     "analytic (the block moves) and sticking < 0.1 x; slide velocity / analytic per offset"),
            **{k: {"precision": r["precision"], "precision_moves": r["precision_moves"],
                   "slide_fraction_by_offset": {str(x["offset"]): round(x["slide_fraction"], 4) for x in r["rows"]}}
               for k, r in ((k, stick_slide.scan(k)) for k in stick_slide.CONFIGS)}}
    if not args.no_extras and args.sweep_frames > 0:
        log(f"stiffness and model sweep ({args.sweep_frames} frames each)")
        extras["stiffness_sweep"] = stiffness_sweep(args.sweep_frames)
    if not args.no_extras and args.batch_scenes > 0:
        log(f"batch of {args.batch_scenes} scenes")
        extras["batch"] = batch_throughput(args.batch_scenes, 10)

    out = {
        "metric": "ms/local-global iter @58.5k DoFs,800 contacts; ms/frame to NCP res<=1e-6",
        "value": round(ms_iter, 4),
        "unit": "ms/iter",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_frame, 4),
        "per_frame_ms": {"median": round(float(np.median(per_frame)), 4),
                         "p90": round(float(np.percentile(per_frame, 90)), 4), "frames": len(per_frame),
                         "warmup": 20, "timing": "wall clock around each frame and a device synchronisation"}
        if per_frame else None,
        "higher_is_better": False,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": (f"teaser-scale seeded extruded star, {sc.n} nodes ({3 * sc.n} DoFs), {sc.m} tets, "
                                f"stable Neo-Hookean E=1e6 nu=0.45, h=0.01 s, {contacts} contacts, "
                                f"{ITERS} L-G iterations/frame, 10 CR iterations; one step = one frame"),
                   "nodes": sc.n, "tets": sc.m, "contacts": contacts, "nnz_S": nnz_s,
                   "iters_per_frame": ITERS, "launch": tune, "graph_replay": True},
        "phases_ms_per_launch": phase_ms,
        "s_pass_kernels_ms": {k: round(v, 5) for k, v in k_ms.items()},
        "ms_per_frame_to_ncp_1e-6": round(float(np.median([t[0] for t in tol])), 3) if tol else None,
        "to_tolerance_solver": (f"CR to relative residual {TOL_CR} (at most {TOL_CR_ITERS} iterations), "
                                f"previous-frame warm start (zero at this state)"),
        "iters_to_ncp_1e-6": [int(t[1]) for t in tol],
        "ncp_res_reached": [float(t[2]) for t in tol],
        "paper_context_ms_per_iter": PAPER_MS_PER_ITER,
        "roofline": roofline,
        "rooflines": rooflines,
    }
    out.update(extras)
    if args.copy_probe:
        out["copy_probe"] = copy_probe(torch)
    if not args.no_cpu_baseline:
        log("cpu baseline (oracle)")
        out["cpu_baseline"] = cpu_baseline(sc)
    print(json.dumps(out))


if __name__ == "__main__":
    main()
