"""Train the learned warm start on data the solver generates, on the GPU.

  python -m paper_2503_15078_amd.train_warm --out warm_mlp.npz

1. Runs seeded training scenes (cube drops, the first frames of teaser-scale stars and of
   resting blobs) frame by frame until the NCP residual is <= 1e-6 m, with the
   previous-frame warm start, and keeps the features and converged impulses of every
   converged frame.
2. Trains the network with the library's own kernels (Adam, cosine learning rate).
3. Compares learned and previous-frame warm starts on held-out scenes: the first frame
   of teaser-scale stars (800 contacts) and whole cube drops; iterations and ms per
   frame to NCP residual <= 1e-6 m.
Writes the parameters (float32, the layout of sim_set_warm_model) and a summary.
"""
import argparse
import json
import sys
import time

import numpy as np


def _range(s):
    a, b = s.split("-") if "-" in s else (s, s)
    return list(range(int(a), int(b) + 1))


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--out", default="warm_mlp.npz")
    ap.add_argument("--seeds", default="100-179")
    ap.add_argument("--frames", type=int, default=None, help="cap on frames per scene")
    ap.add_argument("--epochs", type=int, default=30)
    ap.add_argument("--batch", type=int, default=8192)
    ap.add_argument("--lr", type=float, default=2e-3)
    ap.add_argument("--eval-seeds", default="1000-1003")
    args = ap.parse_args(argv)

    import torch

    from . import scenes, warm

    torch.cuda.init()

    def log(m):
        print(m, flush=True)

    t0 = time.perf_counter()
    log(f"generating data: seeds {args.seeds}")
    feat, tgt = warm.generate(_range(args.seeds), args.frames, log=log)
    log(f"{len(feat)} samples in {time.perf_counter() - t0:.0f} s")
    t1 = time.perf_counter()
    params, info = warm.train(feat, tgt, epochs=args.epochs, batch=args.batch, lr=args.lr, log=log)
    log(f"trained in {time.perf_counter() - t1:.0f} s")
    np.savez(args.out, params=params.astype(np.float32), n_samples=np.int64(len(feat)),
             val_loss=np.asarray(info["val_loss"], np.float64), feature_version=np.int64(1))
    summary = {"samples": int(len(feat)), "train": info, "eval": {}}
    for s in _range(args.eval_seeds):
        for kind, sc, nf in (("teaser", scenes.teaser_scene(s), 1), ("cube", scenes.cube_drop(s), 60)):
            res = warm.compare(sc, params, nf)
            row = {k: {"iters_mean": float(np.mean(v["iters"])), "ms_mean": float(np.mean(v["ms"])),
                       "frames_converged": int(np.sum(np.asarray(v["ncp"]) <= 1e-6))} for k, v in res.items()}
            summary["eval"][f"{kind}{s}"] = row
            log(f"eval {kind} seed {s} ({nf} frames): " + json.dumps(row))
    log(json.dumps(summary))
    return 0


if __name__ == "__main__":
    sys.exit(main())
