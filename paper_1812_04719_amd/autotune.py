"""Autotuner for the launch configuration of the contact path.

Tunes the patch size of the primitive broad phase (16, 32 or 64 triangles)
and the widths of the two persistent kernels (primitive candidates, root
search).  None of these change results; they change speed, and the best
choice depends on the mesh orders and the packing density.  Measurements
use the library's own HIP-event timers on the call's stream (median of a few
repetitions); the winner is cached in a JSON file keyed by
(device, mesh orders, density bucket, size bucket).
"""
import json
import math
import os
import statistics

from . import stiv

DEFAULT_CACHE = os.environ.get("STIV_AUTOTUNE_CACHE",
                               os.path.join(os.path.expanduser("~"), ".cache", "stiv", "autotune.json"))

CANDIDATES = [dict(tile=t, prim_blocks=pb, narrow_blocks=nb)
              for t in (64, 32, 16) for pb in (4096, 8192, 16384) for nb in (4096, 8192)]


def workload_key(device_name, scene):
    """Workload class of a scene: device, mesh orders, density and size buckets."""
    orders = sorted({t.order for t in scene.topos})
    ntri = scene.n_tri()
    vol = 0.0
    for s in range(scene.n_scenes):
        L = scene.box_len[s]
        if all(L > 0):
            vol += float(L[0] * L[1] * L[2])
        else:
            lo = scene.x0[:, scene.vtx_off[scene.scene_off[s]]:scene.vtx_off[scene.scene_off[s + 1]]].min(axis=1)
            hi = scene.x0[:, scene.vtx_off[scene.scene_off[s]]:scene.vtx_off[scene.scene_off[s + 1]]].max(axis=1)
            vol += float(max(1e-9, (hi - lo).prod()))
    density = ntri / max(vol, 1e-9)
    return "%s|orders=%s|dens=%d|size=%d" % (device_name, ",".join(map(str, orders)),
                                            int(round(math.log2(max(density, 1e-9)))),
                                            int(round(math.log2(max(scene.n_ves, 1)))))


def apply(ctx, cfg):
    ctx.set_option(stiv.STIV_OPT_PATCH_TRI, cfg["tile"])
    ctx.set_option(stiv.STIV_OPT_PRIM_BLOCKS, cfg["prim_blocks"])
    ctx.set_option(stiv.STIV_OPT_NARROW_BLOCKS, cfg["narrow_blocks"])


def _load(path):
    try:
        with open(path) as f:
            return json.load(f)
    except (OSError, ValueError):
        return {}


def _save(path, data):
    os.makedirs(os.path.dirname(os.path.abspath(path)), exist_ok=True)
    tmp = path + ".tmp%d" % os.getpid()
    with open(tmp, "w") as f:
        json.dump(data, f, indent=1, sort_keys=True)
    os.replace(tmp, path)


def tune(ctx, dscene, d, eps, dt, cache_file=DEFAULT_CACHE, reps=3, candidates=None, force=False):
    """Pick and apply the fastest configuration for this workload class.

    Returns (config, table) where table lists the median device time (ms) of
    every configuration tried (empty when the cache answered)."""
    import torch
    dev_name = torch.cuda.get_device_name(dscene.x0.device)
    key = workload_key(dev_name, dscene.scene)
    cache = _load(cache_file) if cache_file else {}
    if not force and key in cache:
        cfg = cache[key]["config"]
        apply(ctx, cfg)
        return cfg, []
    table = []
    outs = None
    for cfg in (candidates or CANDIDATES):
        apply(ctx, cfg)
        _, outs = stiv.detect(ctx, dscene, d, eps, dt, outputs=outs, to_numpy=False)
        times = []
        for _ in range(reps):
            _, outs = stiv.detect(ctx, dscene, d, eps, dt, outputs=outs, to_numpy=False)
            times.append(ctx.stage_times()[6])
        table.append(dict(cfg, ms=statistics.median(times)))
    best = min(table, key=lambda r: r["ms"])
    cfg = {k: best[k] for k in ("tile", "prim_blocks", "narrow_blocks")}
    apply(ctx, cfg)
    if cache_file:
        cache[key] = {"config": cfg, "ms": best["ms"], "tried": len(table)}
        _save(cache_file, cache)
    return cfg, table
