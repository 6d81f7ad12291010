#!/usr/bin/env python3
"""Train the learned contact-time bracket and write the package's model file.

Samples: every primitive candidate whose polynomial F (Eq. 3.1) is not
excluded by its Bernstein coefficients on [0,1] (the candidates the root
search sees), labelled by the oracle with the first root of F in [0,1]
(candidates without a root get the target 1).  Scenes: the 58 % packing
generator (1440 vesicles) and the random-packing and two-sphere generators,
all with seeds 100 and up, so no training scene is a test or benchmark
scene.  Training runs on the GPU in the library's kernels (bf16 matrix-core
forward/backward, Adam).

  python tests/train_toi_mlp.py [--samples 2000000] [--steps 4000] [--out PATH]
"""
import argparse
import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
sys.path.insert(0, ROOT)
sys.path.insert(0, HERE)

import numpy as np  # noqa: E402

import oracle  # noqa: E402
from paper_1812_04719_amd import scenes as S  # noqa: E402


def collect(n_target, threads, log):
    feats, targets, parts = [], [], []
    total = 0
    # dense packings dominate (they are the workload the search runs on);
    # a share of sparse packings and sphere pairs widens the input range
    plan = [("fcc", 100), ("fcc", 101), ("rsa", 100), ("rsa", 101), ("rsa", 102), ("rsa", 103),
            ("spheres", 100), ("spheres", 101), ("spheres", 102), ("spheres", 103), ("fcc", 102), ("fcc", 103)]
    for kind, sd in plan:
        if total >= n_target:
            break
        t0 = time.time()
        if kind == "fcc":
            sc = S.make_fcc_scene(seed=sd)
        elif kind == "rsa":
            sc = S.make_rsa_scene(seed=sd, n=64, vf=0.30)
        else:
            sc = S.make_two_spheres(seed=sd)
        f, r, h = oracle.toi_samples(sc, threads=threads)
        f, r = f[h], r[h]
        t = np.where(r >= 0.0, r, 1.0).astype(np.float32)
        feats.append(f)
        targets.append(t)
        total += len(t)
        parts.append(dict(kind=kind, seed=sd, samples=int(len(t)), with_root=int((r >= 0).sum())))
        log("%s seed %d: %d samples (%d with a root) in %.1fs; total %d"
            % (kind, sd, len(t), (r >= 0).sum(), time.time() - t0, total))
    x = np.concatenate(feats)
    y = np.concatenate(targets)
    rng = np.random.default_rng(0)
    if len(y) > n_target:
        keep = rng.choice(len(y), n_target, replace=False)
        x, y = x[keep], y[keep]
    return x, y, parts


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--samples", type=int, default=2_000_000)
    ap.add_argument("--steps", type=int, default=4000)
    ap.add_argument("--batch", type=int, default=8192)
    ap.add_argument("--lr", type=float, default=2e-3)
    ap.add_argument("--kwidth", type=float, default=3.0)
    ap.add_argument("--threads", type=int, default=16)
    ap.add_argument("--holdout", type=float, default=0.05)
    ap.add_argument("--out", default=None)
    args = ap.parse_args()

    def log(m):
        print(m, flush=True)

    import torch
    from paper_1812_04719_amd import stiv, toi_model
    out = args.out or toi_model.DEFAULT_WEIGHTS
    t0 = time.time()
    x, y, parts = collect(args.samples, args.threads, log)
    log("samples: %d (%.1fs)" % (len(y), time.time() - t0))
    n_hold = int(len(y) * args.holdout)
    xh, yh = x[:n_hold], y[:n_hold]
    xt, yt = x[n_hold:], y[n_hold:]
    ctx = stiv.Context(0)
    t1 = time.time()
    params, hist = toi_model.train(ctx, xt, yt, steps=args.steps, batch=args.batch, lr=args.lr, seed=0,
                                   log_every=max(1, args.steps // 20))
    torch.cuda.synchronize()
    t_train = time.time() - t1
    mu, sd = toi_model.predict(ctx, params, xh)
    z = np.abs(yh - mu) / sd
    cover = float(np.mean(z <= args.kwidth))
    width = float(np.median(np.minimum(1.0, mu + args.kwidth * sd) - np.maximum(0.0, mu - args.kwidth * sd)))
    mae = float(np.median(np.abs(yh - mu)))
    log("held-out: median |s - mu| %.4f, coverage of mu +- %.1f sd %.3f, median bracket width %.4f"
        % (mae, args.kwidth, cover, width))
    meta = dict(name="toi_mlp_18_64_64_2", samples=int(len(yt)), holdout=int(n_hold), steps=args.steps,
                batch=args.batch, lr=args.lr, train_seconds=round(t_train, 1), loss=hist[-1][1] if hist else None,
                holdout_median_abs_err=mae, holdout_coverage=cover, holdout_median_width=width, sources=parts,
                device=torch.cuda.get_device_name(0))
    toi_model.save(out, params, args.kwidth, meta)
    log("wrote %s" % out)
    log(json.dumps(meta))
    ctx.close()


if __name__ == "__main__":
    main()
