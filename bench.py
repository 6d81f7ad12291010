#!/usr/bin/env python3
"""Benchmark of the contact-detection path on one MI355X.

One step = one stiv_detect call over the whole 1440-vesicle scene (57.66 %
volume fraction, reduced volume 0.91, order-32 contact meshes: 3.04M
vertices, 6.08M triangles) with positions resident in HBM: boxes, Morton
vesicle broad phase, primitive broad phase, FP64 narrow phase, volumes and
gradients, aggregation.  Prints one JSON line.

  python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu-baseline]
"""
import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "candidate pairs/s & contacts/s, 1440 vesicles 58% vf; learned-TOI vs plain"
HBM_PEAK_GBS = 8000.0
FP64_PEAK_TFLOPS = 78.6

# Algorithmic work per unit (derivations in the design doc):
BYTES_PER_VERTEX_BOXES = 48.0       # X0 and X1, 3 doubles each, read once by the box kernel
BYTES_PER_BOX_OUT = 48.0            # 6 doubles per vesicle or patch box written
FLOPS_PER_CANDIDATE = 152.0         # coefficients of F = g^2 - d^2 q (counted from the formulas)
FLOPS_PER_VT_CONTACT = 300.0        # volume and gradient of one vertex-triangle contact


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--config", type=int, default=3)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-reps", type=int, default=3)
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only: the contact path here runs on a single MI355X "
              "(multi-GPU sharding is a design note, not a measured mode); use --gpus 1", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    from paper_1812_04719_amd import scenes, stiv

    t0 = time.time()
    sc = scenes.make_config(args.config)
    log("scene: %d vesicles, %d vertices, %d triangles (%.1fs)" % (sc.n_ves, sc.n_vtx, sc.n_tri(), time.time() - t0))
    dev = torch.device("cuda:0")
    ctx = stiv.Context(0)
    ds = stiv.DeviceScene(sc, dev)
    outs = None
    res, outs = stiv.detect(ctx, ds, sc.d, sc.eps, sc.dt, outputs=outs, to_numpy=False)
    # stage times measured by the library with HIP events on the same stream
    stage_sum = np.zeros(7)
    for _ in range(args.warmup):
        res, outs = stiv.detect(ctx, ds, sc.d, sc.eps, sc.dt, outputs=outs, to_numpy=False)
    torch.cuda.synchronize()
    t_start = time.perf_counter()
    for _ in range(args.steps):
        res, outs = stiv.detect(ctx, ds, sc.d, sc.eps, sc.dt, outputs=outs, to_numpy=False)
        stage_sum += np.array(ctx.stage_times())
    torch.cuda.synchronize()
    t_total = time.perf_counter() - t_start
    ms_step = 1e3 * t_total / args.steps
    stages = stage_sum / args.steps
    n_cand = res["n_cand_vt"] + res["n_cand_ee"]
    n_ct = res["n_ct"]
    pairs_per_s = n_cand / (ms_step * 1e-3)
    contacts_per_s = n_ct / (ms_step * 1e-3)
    names = ["boxes", "vesicle_broad_phase", "patch_pair_cull", "primitive_candidates", "narrow_volume_gradient",
             "aggregation", "device_total"]
    stage_ms = {n: round(float(v), 4) for n, v in zip(names, stages)}
    log("stages (ms): %s" % stage_ms)
    work = ctx.stats()
    log("work: %s" % work)

    # roofline of the dominant kernel
    n_patches = int(sum(ctx_patch for ctx_patch in [0]))  # patch boxes: counted below
    per_topo_patches = None
    dom = int(np.argmax(stages[:6]))
    if dom == 0:
        n_patch_boxes = sc.n_ves * math.ceil(sc.topos[0].nt / 64)
        bytes_alg = BYTES_PER_VERTEX_BOXES * sc.n_vtx + BYTES_PER_BOX_OUT * (sc.n_ves + n_patch_boxes)
        achieved = bytes_alg / (stages[0] * 1e-3) / 1e9
        roof = {"kernel": "k_boxes", "bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": None}
    else:
        flops = FLOPS_PER_CANDIDATE * n_cand + FLOPS_PER_VT_CONTACT * res["n_ct_vt"]
        t_k = stages[4] * 1e-3
        achieved = flops / t_k / 1e12
        roof = {"kernel": "k_narrow", "stage": names[dom], "bound": "alu", "achieved": round(achieved, 3),
                "peak": FP64_PEAK_TFLOPS, "unit": "TFLOP/s", "frac": round(achieved / FP64_PEAK_TFLOPS, 4),
                "traffic": None}

    out = {
        "metric": METRIC,
        "value": round(pairs_per_s, 1),
        "unit": "candidate pairs/s",
        "contacts_per_s": round(contacts_per_s, 1),
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "1440 vesicles, v=0.91, 57.66% vf periodic box, order-32 contact grid",
                   "n_vesicles": sc.n_ves, "n_vertices": sc.n_vtx, "n_triangles": sc.n_tri(),
                   "vesicle_pairs": int(res["n_pairs"]), "candidates_vt": int(res["n_cand_vt"]),
                   "candidates_ee": int(res["n_cand_ee"]), "contacts_vt": int(res["n_ct_vt"]),
                   "contacts_ee": int(res["n_ct_ee"]), "contact_volumes": int(res["n_vol"]),
                   "jacobian_rows": int(res["n_jrow"])},
        "stages_ms": stage_ms,
        "work": work,
        "roofline": roof,
    }
    if not args.no_cpu_baseline:
        import oracle
        ts = []
        r = None
        for _ in range(args.cpu_reps):
            t1 = time.perf_counter()
            r = oracle.detect(sc)
            ts.append(time.perf_counter() - t1)
        tmed = float(np.median(ts))
        oc = r["n_cand_vt"] + r["n_cand_ee"]
        out["cpu_baseline"] = {"value": round(oc / tmed, 1), "unit": "candidate pairs/s",
                               "contacts_per_s": round(r["n_ct"] / tmed, 1), "cores": int(r["threads_used"]),
                               "kind": "oracle",
                               "sample": "whole 1440-vesicle scene, median of %d runs (%.2f s each)"
                                         % (args.cpu_reps, tmed)}
        log("oracle: %.2f s per run on %d threads" % (tmed, r["threads_used"]))
    ctx.close()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
