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

# Algorithmic work per unit, counted from the formulas of the method:
BYTES_PER_VERTEX_BOXES = 48.0       # X0 and X1, 3 doubles each, read once by the box kernel
BYTES_PER_BOX_OUT = 48.0            # 6 doubles per vesicle or patch box written
FLOPS_PER_CANDIDATE = 152.0         # coefficients of F = g^2 - d^2 q (counted from the formulas)
# per candidate in the primitive kernel: exact FP64 box test (66: min/max of 4 vertices at both
# times, inflation and shift, 6 comparisons) + coefficients of F (152) + Bernstein screen (35)
OPS_PER_CANDIDATE_SCREEN = 253.0
FLOPS_PER_VT_CONTACT = 300.0        # volume and gradient of one vertex-triangle contact
OPS_PER_BOX_TEST = 6.0              # 3 axes x 2 interval-end comparisons of two FP32 boxes
LDS_BYTES_PER_BOX_TEST = 48.0       # two 6-float boxes read from LDS
# One VALU lane-operation per lane per clock: 256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz
# (an FP32 compare or an FP64 add/mul each take one; FMA and packed FP32 double it).
VALU_PEAK_TOPS = 256 * 64 * 2.4e9 / 1e12
# LDS: 128 bytes per clock per CU
LDS_PEAK_TBS = 256 * 128 * 2.4e9 / 1e12
# Algorithmic bytes and flops of the whole path (what the method must move and compute):
# X0 and X1 read once, 16 B per vesicle pair, 128 B per vertex-triangle contact (key, tau, V,
# 12-gradient), 32 B per edge-edge contact, 8 B per volume, 32 B per Jacobian row; F's
# coefficients per candidate (170 flops) and V with its gradient per vertex-triangle contact.
ALG_BYTES = {"vertex": 48.0, "pair": 16.0, "vt": 128.0, "ee": 32.0, "vol": 8.0, "jrow": 32.0}
ALG_FLOPS_PER_CANDIDATE = 170.0
FLUSH_BYTES = 1 << 30               # written before each cold-cache step (larger than the 256 MB MALL)
# HBM bytes per launch from rocprofv3 --pmc FETCH_SIZE + WRITE_SIZE on this workload,
# each scaled by the counter's reading for a plain 1 GiB copy (factors 2.0 and 1.0),
# keyed by a hash of the sources the kernel is built from: a figure taken on another
# build of the kernel no longer matches and is reported as null.
TRAFFIC_BYTES = {"k_prim_cand": {"sources": ("k_prim.hip", "narrow_math.h", "stiv_common.h"),
                                 "sha16": "a6d44364bb153495", "bytes": 652835413}}


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def sources_sha16(names):
    """First 16 hex digits of the SHA-256 of the kernel sources, in order."""
    import hashlib
    h = hashlib.sha256()
    for n in names:
        with open(os.path.join(ROOT, "paper_1812_04719_amd", "csrc", n), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def traffic_for(kernel):
    """Measured HBM bytes per launch of `kernel`, or None when the figure was
    taken on other sources than the ones built now."""
    t = TRAFFIC_BYTES.get(kernel)
    if not t or t["bytes"] is None or t["sha16"] != sources_sha16(t["sources"]):
        return None
    return t["bytes"]


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--config", type=int, default=3)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-reps", type=int, default=3)
    ap.add_argument("--cold-reps", type=int, default=50,
                    help="cold-cache steps (each after a 1 GiB write that evicts the MALL); median reported")
    ap.add_argument("--plain-only", action="store_true", help="skip the learned-bracket timing")
    ap.add_argument("--no-batch", action="store_true", help="skip the 256-scene batch measurement")
    ap.add_argument("--no-single-thread", action="store_true", help="skip the single-thread oracle run")
    ap.add_argument("--batch-only", action="store_true",
                    help="only the 256-scene batch measurement (for profiling it); prints its JSON object")
    ap.add_argument("--copy-probe", action="store_true",
                    help="only run a 1 GiB device-to-device copy (HBM counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only: the contact path here runs on a single MI355X "
              "(multi-GPU sharding is a design note, not a measured mode); use --gpus 1", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    from paper_1812_04719_amd import scenes, stiv

    if args.copy_probe:
        x = torch.empty(1 << 27, dtype=torch.float64, device="cuda:0").fill_(1.0)
        y = torch.empty_like(x)
        for _ in range(3):
            y.copy_(x)
        torch.cuda.synchronize()
        print(json.dumps({"copy_probe_bytes_read": x.numel() * 8, "copy_probe_bytes_written": y.numel() * 8,
                          "launches": 3}), flush=True)
        return

    if args.batch_only:
        ctx = stiv.Context(0)
        print(json.dumps(measure_batch(ctx, scenes, stiv, torch, np, args)), flush=True)
        ctx.close()
        return

    t0 = time.time()
    sc = scenes.make_config(args.config)
    log("scene: %d vesicles, %d vertices, %d triangles (%.1fs)" % (sc.n_ves, sc.n_vtx, sc.n_tri(), time.time() - t0))
    dev = torch.device("cuda:0")
    ctx = stiv.Context(0)
    ds = stiv.DeviceScene(sc, dev)
    outs = None
    res, outs = stiv.detect(ctx, ds, sc.d, sc.eps, sc.dt, outputs=outs, to_numpy=False)
    # stage times measured by the library with HIP events on the same stream
    def timed(learned):
        st_sum = np.zeros(7)
        r = None
        for _ in range(args.warmup):
            r, _o = stiv.detect(ctx, ds, sc.d, sc.eps, sc.dt, outputs=outs, to_numpy=False, learned_bracket=learned)
        torch.cuda.synchronize()
        t_a = time.perf_counter()
        for _ in range(args.steps):
            r, _o = stiv.detect(ctx, ds, sc.d, sc.eps, sc.dt, outputs=outs, to_numpy=False, learned_bracket=learned)
            st_sum += np.array(ctx.stage_times())
        torch.cuda.synchronize()
        return r, time.perf_counter() - t_a, st_sum / args.steps, ctx.stats()

    res, t_total, stages, work = timed(False)
    learned = None
    from paper_1812_04719_amd import toi_model
    if os.path.exists(toi_model.DEFAULT_WEIGHTS) and not args.plain_only:
        toi_model.install(ctx)
        res_l, t_l, stages_l, work_l = timed(True)
        same = bool(torch.equal(res_l["ct_key"], res["ct_key"]))
        learned = {"ms_per_step": round(1e3 * t_l / args.steps, 4),
                   "narrow_ms": round(float(stages_l[4]), 4), "narrow_ms_plain": round(float(stages[4]), 4),
                   "narrow_speedup": round(float(stages[4] / stages_l[4]), 4),
                   "bracket_certified": int(work_l["bracket_certified"]),
                   "root_searches": int(work_l["root_searches"]), "same_contacts": same}
        log("learned bracket: %s" % learned)
        if not same:
            raise SystemExit("learned bracket changed the contact set")
        if t_l < t_total:
            res, t_total, stages, work = res_l, t_l, stages_l, work_l
    mode = "learned" if (learned and t_total == t_l) else "plain"
    eager_ms = 1e3 * t_total / args.steps
    n_cand = res["n_cand_vt"] + res["n_cand_ee"]
    n_ct = res["n_ct"]
    # the same detect captured once as a HIP graph and replayed once per step (the way a
    # time-stepping caller runs it): W untimed replays, then K replays between synchronizations
    g_ms, g_wall, _ = graph_replay_ms(ctx, ds, sc, res, stiv, torch, np, args.steps, args.warmup,
                                      learned=(mode == "learned"))
    ms_step = 1e3 * g_wall
    pairs_per_s = n_cand / (ms_step * 1e-3)
    contacts_per_s = n_ct / (ms_step * 1e-3)
    eager = {"ms_per_step": round(eager_ms, 4), "candidate_pairs_per_s": round(n_cand / (eager_ms * 1e-3), 1),
             "contacts_per_s": round(n_ct / (eager_ms * 1e-3), 1),
             "note": "one stiv_detect call per step (enqueue, one synchronization to read the counts)"}
    log("graph replay: %.4f ms per step (events %.4f); eager %.4f ms" % (ms_step, g_ms, eager_ms))
    names = ["boxes", "vesicle_broad_phase", "patch_pair_cull", "primitive_candidates", "narrow_volume_gradient",
             "aggregation", "device_total"]
    stage_ms = {n: round(float(v), 4) for n, v in zip(names, stages)}
    log("stages (ms): %s" % stage_ms)
    log("work: %s" % work)

    # roofline of the dominant kernel, counted from the method's algorithmic work
    # (FP64 flops of F's coefficients per candidate the kernel examines, of V and its
    # gradient per vertex-triangle contact; bytes of X0 and X1 for the box kernel)
    dom = int(np.argmax(stages[:6]))
    t_dom = float(stages[dom]) * 1e-3
    b_alg_path = (ALG_BYTES["vertex"] * sc.n_vtx + ALG_BYTES["pair"] * res["n_pairs"]
                  + ALG_BYTES["vt"] * res["n_ct_vt"] + ALG_BYTES["ee"] * res["n_ct_ee"]
                  + ALG_BYTES["vol"] * res["n_vol"] + ALG_BYTES["jrow"] * res["n_jrow"])
    if dom == 0:
        n_patch_boxes = sc.n_ves * math.ceil(sc.topos[0].nt / 64)
        bytes_alg = BYTES_PER_VERTEX_BOXES * sc.n_vtx + BYTES_PER_BOX_OUT * (sc.n_ves + n_patch_boxes)
        achieved = bytes_alg / t_dom / 1e9
        roof = {"kernel": "k_boxes", "stage": names[0], "bound": "hbm", "achieved": round(achieved, 1),
                "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                "traffic": traffic_for("k_boxes"), "alg_bytes_per_launch": int(bytes_alg),
                "avg_launch_ms": round(float(stages[0]), 4)}
    else:
        kern = {3: "k_prim_cand", 4: "k_narrow"}.get(dom, names[dom])
        if dom == 3:
            flops = ALG_FLOPS_PER_CANDIDATE * n_cand
            per = "170 FP64 flops (coefficients of F) x %d candidates" % n_cand
        elif dom == 4:
            flops = ALG_FLOPS_PER_CANDIDATE * work["root_searches"] + FLOPS_PER_VT_CONTACT * res["n_ct_vt"]
            per = "170 x %d searched candidates + 300 x %d VT contacts" % (work["root_searches"], res["n_ct_vt"])
        else:
            flops = 0.0
            per = "no FP64 work counted for this stage"
        achieved = flops / t_dom / 1e12
        roof = {"kernel": kern, "stage": names[dom], "bound": "alu", "achieved": round(achieved, 4),
                "peak": FP64_PEAK_TFLOPS, "unit": "TFLOP/s", "frac": round(achieved / FP64_PEAK_TFLOPS, 5),
                "traffic": traffic_for(kern), "alg_flops_per_launch": int(flops), "alg_work": per,
                "avg_launch_ms": round(float(stages[dom]), 4),
                "peak_note": "FP64 vector datasheet peak of MI355X"}
        # the whole path's algorithmic bytes credited to this one launch, against HBM
        roof["alg_bytes_hbm_frac"] = round(b_alg_path / t_dom / (HBM_PEAK_GBS * 1e9), 5)
        if roof["traffic"]:
            roof["hbm_gbs"] = round(roof["traffic"] / t_dom / 1e9, 1)
            roof["hbm_frac"] = round(roof["hbm_gbs"] / HBM_PEAK_GBS, 4)
        if dom == 3:
            # the implementation's own operation count (box tests of the sweep, exact box
            # test and screens per candidate) against one VALU lane-operation per clock
            ops = OPS_PER_BOX_TEST * work["box_tests"] + OPS_PER_CANDIDATE_SCREEN * n_cand
            roof["impl_valu"] = {"ops_per_launch": int(ops),
                                 "achieved_tops": round(ops / t_dom / 1e12, 4), "peak_tops": VALU_PEAK_TOPS,
                                 "frac": round(ops / t_dom / 1e12 / VALU_PEAK_TOPS, 4)}
            lds = LDS_BYTES_PER_BOX_TEST * work["box_tests"] / t_dom / 1e12
            roof["lds_tbs"] = round(lds, 3)
            roof["lds_frac"] = round(lds / LDS_PEAK_TBS, 4)

    # measured copy bandwidth (1 GiB device-to-device) beside the datasheet peak
    src = torch.empty(FLUSH_BYTES // 8, dtype=torch.float64, device=dev).fill_(1.0)
    dst = torch.empty_like(src)
    for _ in range(2):
        dst.copy_(src)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(5):
        dst.copy_(src)
    e1.record()
    torch.cuda.synchronize()
    copy_gbs = 2.0 * FLUSH_BYTES * 5 / (e0.elapsed_time(e1) * 1e-3) / 1e9
    roof["copy_gbs"] = round(copy_gbs, 1)
    if roof.get("hbm_gbs"):
        roof["hbm_frac_of_copy"] = round(roof["hbm_gbs"] / copy_gbs, 4)
    # cold cache: before every step a 1 GiB write evicts the input from the 256 MB MALL;
    # each step is timed alone with events (the write is outside the timed window)
    cold = []
    for k in range(args.cold_reps):
        dst.fill_(float(k))
        torch.cuda.synchronize()
        e0.record()
        stiv.detect(ctx, ds, sc.d, sc.eps, sc.dt, outputs=outs, to_numpy=False, learned_bracket=(mode == "learned"))
        e1.record()
        torch.cuda.synchronize()
        cold.append(e0.elapsed_time(e1))
    del src, dst
    cold_ms = float(np.median(cold))
    cold_cache = {"ms_per_step": round(cold_ms, 4), "candidate_pairs_per_s": round(n_cand / (cold_ms * 1e-3), 1),
                  "contacts_per_s": round(n_ct / (cold_ms * 1e-3), 1), "steps": len(cold),
                  "flush_bytes": FLUSH_BYTES, "statistic": "median"}
    log("cold cache: %s" % cold_cache)
    # algorithmic fractions of the whole path
    b_alg = b_alg_path
    f_alg = ALG_FLOPS_PER_CANDIDATE * n_cand + FLOPS_PER_VT_CONTACT * res["n_ct_vt"]
    t_fp = float(stages[3] + stages[4] + stages[5]) * 1e-3  # screens, root search, volumes, aggregation
    algorithmic = {"bytes": int(b_alg), "hbm_frac": round(b_alg / (ms_step * 1e-3) / (HBM_PEAK_GBS * 1e9), 5),
                   "flops": int(f_alg), "fp64_frac": round(f_alg / t_fp / (FP64_PEAK_TFLOPS * 1e12), 5),
                   "fp64_time": "primitive_candidates + narrow_volume_gradient + aggregation"}

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
        "launch": "one HIP graph replay per step (stiv_detect_async captured once)",
        "protocol": ("value and ms_per_step: mean over K warm graph replays (wall clock between two "
                     "synchronizations); cold_cache: median of cold_reps eager steps, each timed with events "
                     "after a 1 GiB write that evicts the 256 MB MALL"),
        "eager": eager,
        "cold_cache": cold_cache,
        "algorithmic": algorithmic,
        "toi_search": mode,
        "learned_vs_plain": learned,
    }
    if not args.no_batch and not args.plain_only:
        out["batch"] = measure_batch(ctx, scenes, stiv, torch, np, args)
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
        cpu_model = ""
        try:
            with open("/proc/cpuinfo") as f:
                cpu_model = next((l.split(":", 1)[1].strip() for l in f if l.startswith("model name")), "")
        except OSError:
            pass
        out["cpu_baseline"] = {"value": round(oc / tmed, 1), "unit": "candidate pairs/s",
                               "contacts_per_s": round(r["n_ct"] / tmed, 1), "cores": int(r["threads_used"]),
                               "kind": "oracle", "cpu_model": cpu_model, "nproc": os.cpu_count(),
                               "sample": "whole 1440-vesicle scene, median of %d runs (%.2f s each)"
                                         % (args.cpu_reps, tmed)}
        log("oracle: %.2f s per run on %d threads" % (tmed, r["threads_used"]))
        if not args.no_single_thread:
            t1 = time.perf_counter()
            r1 = oracle.detect(sc, threads=1)
            t_one = time.perf_counter() - t1
            out["cpu_baseline"]["single_thread"] = {"value": round((r1["n_cand_vt"] + r1["n_cand_ee"]) / t_one, 1),
                                                    "seconds": round(t_one, 2), "cores": int(r1["threads_used"])}
            log("oracle: %.2f s on 1 thread" % t_one)
    ctx.close()
    print(json.dumps(out), flush=True)


def graph_replay_ms(ctx, ds, sc, eager, stiv, torch, np, steps, warmup, learned=False):
    """The whole detect captured once in a HIP graph (stiv_detect_async) and
    replayed: (ms per replay from events, wall ms per replay, result of the
    last replay), checked equal to the eager result."""
    outs = stiv.Outputs(ds.x0.device, cap_pairs=2 * int(eager["n_pairs"]) + 16, cap_ct=2 * int(eager["n_ct"]) + 16,
                        cap_vol=2 * int(eager["n_vol"]) + 16, cap_jrow=2 * int(eager["n_jrow"]) + 16)
    job = stiv.AsyncDetect(ctx, ds, sc.d, sc.eps, sc.dt, outs, learned_bracket=learned)
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        job.enqueue()
        job.collect()
    torch.cuda.current_stream().wait_stream(side)
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        job.enqueue()
    for _ in range(max(1, warmup)):
        g.replay()
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    t_a = time.perf_counter()
    e0.record()
    for _ in range(steps):
        g.replay()
    e1.record()
    torch.cuda.synchronize()
    wall = (time.perf_counter() - t_a) / steps
    ms = e0.elapsed_time(e1) / steps
    r = job.collect(to_numpy=True)
    # reference: a fresh eager call in the same mode (bit-identical results expected)
    ref, _ = stiv.detect(ctx, ds, sc.d, sc.eps, sc.dt, learned_bracket=learned)
    if not (np.array_equal(r["ct_key"], ref["ct_key"]) and np.array_equal(r["vol_V"], ref["vol_V"])
            and np.array_equal(r["ct_tau"], ref["ct_tau"])):
        raise SystemExit("graph replay differs from the eager result")
    return ms, wall, r


def measure_batch(ctx, scenes, stiv, torch, np, args):
    """256 independent scenes of 8-128 vesicles (orders 16/24/32, 10-60 % vf) in one
    call: autotuned launch configuration, then the whole detect captured in a HIP
    graph and replayed; checked equal to the eager result."""
    from paper_1812_04719_amd import autotune
    t0 = time.time()
    b = scenes.make_config(4)
    log("batch: %d scenes, %d vesicles, %d vertices (%.1fs)" % (b.n_scenes, b.n_ves, b.n_vtx, time.time() - t0))
    ds = stiv.DeviceScene(b)
    cfg, table = autotune.tune(ctx, ds, b.d, b.eps, b.dt, cache_file=None, reps=2)
    log("batch autotune: %s" % cfg)
    eager, _ = stiv.detect(ctx, ds, b.d, b.eps, b.dt)
    ms, wall, r = graph_replay_ms(ctx, ds, b, eager, stiv, torch, np, max(1, args.steps // 2), args.warmup)
    same = True
    n_cand = int(eager["n_cand_vt"] + eager["n_cand_ee"])
    res = {"workload": "256 scenes of 8-128 vesicles, orders 16/24/32, 10-60% vf, one graph-captured call",
           "scenes": int(b.n_scenes), "vesicles": int(b.n_ves), "vertices": int(b.n_vtx),
           "candidates": n_cand, "contacts": int(eager["n_ct"]), "volumes": int(eager["n_vol"]),
           "ms_per_batch": round(ms, 4), "wall_ms_per_batch": round(1e3 * wall, 4),
           "candidate_pairs_per_s": round(n_cand / (ms * 1e-3), 1),
           "contacts_per_s": round(eager["n_ct"] / (ms * 1e-3), 1), "tuned": cfg, "replay_equals_eager": same}
    log("batch: %s" % res)
    return res


if __name__ == "__main__":
    main()
