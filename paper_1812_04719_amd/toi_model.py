"""Learned contact-time bracket: model file, installation and GPU training.

The model (perceptron 18 -> 64 -> 64 -> 2, layout and features in
include/stiv.h) predicts where the first root of F (Eq. 3.1) lies for a
primitive pair, so the root search can start there.  The search verifies the
prediction (a Bernstein certificate that F has no root before the bracket),
so the model only changes speed, never the contacts.

Training runs entirely in the library's kernels (bf16 matrix-core forward and
backward, fixed-order gradient reduction, Adam on FP32 master weights);
samples (features, first root) come from the caller.  Checkpoints keep the
step count and the optimizer moments.
"""
import json
import os

import numpy as np

from . import stiv

DEFAULT_WEIGHTS = os.path.join(os.path.dirname(os.path.abspath(__file__)), "weights", "toi_mlp.npz")
N_IN, N_H, N_OUT = 18, 64, 2


def layout():
    """Offsets of W1, b1, W2, b2, W3, b3 in the flat parameter vector."""
    sizes = [N_IN * N_H, N_H, N_H * N_H, N_H, N_H * N_OUT, N_OUT]
    off = np.concatenate([[0], np.cumsum(sizes)])
    names = ["W1", "b1", "W2", "b2", "W3", "b3"]
    shapes = [(N_IN, N_H), (N_H,), (N_H, N_H), (N_H,), (N_H, N_OUT), (N_OUT,)]
    return {n: (int(off[i]), shapes[i]) for i, n in enumerate(names)}, int(off[-1])


def init_params(seed=0):
    """He-initialised weights, zero biases except b3 (mu ~ 0.5, sd ~ 0.1)."""
    lay, n = layout()
    rng = np.random.default_rng(seed)
    p = np.zeros(n, dtype=np.float32)
    for name, fan_in in (("W1", N_IN), ("W2", N_H), ("W3", N_H)):
        o, shp = lay[name]
        p[o:o + int(np.prod(shp))] = (rng.standard_normal(int(np.prod(shp))) * np.sqrt(2.0 / fan_in)).astype(np.float32)
    o, _ = lay["W3"]
    p[o:o + N_H * N_OUT] *= 0.1
    o, _ = lay["b3"]
    p[o:o + 2] = [0.0, np.log(np.expm1(0.1))]
    return p


def load(path=DEFAULT_WEIGHTS):
    """(params float32, kwidth, meta dict) of a saved model."""
    with np.load(path, allow_pickle=False) as z:
        params = np.asarray(z["params"], dtype=np.float32)
        kwidth = float(z["kwidth"])
        meta = json.loads(str(z["meta"])) if "meta" in z else {}
    return params, kwidth, meta


def save(path, params, kwidth, meta):
    os.makedirs(os.path.dirname(os.path.abspath(path)), exist_ok=True)
    np.savez(path, params=np.asarray(params, dtype=np.float32), kwidth=np.float64(kwidth),
             meta=np.array(json.dumps(meta, sort_keys=True)))


def install(ctx, path=DEFAULT_WEIGHTS, kwidth=None):
    """Load a saved model into a context (for STIV_LEARNED_BRACKET)."""
    params, kw, meta = load(path)
    ctx.set_toi_model(params, kw if kwidth is None else kwidth)
    return meta


def train(ctx, feats, roots, steps=3000, batch=8192, lr=2e-3, seed=0, params=None, log_every=0, checkpoint=None,
          lr_final=1e-4):
    """Fit the bracket model on the GPU.

    feats [n,18] float32, roots [n] in [0,1] (first root of F of each
    sample).  Mini-batches are drawn with a seeded permutation; the step size
    decays geometrically from lr to lr_final.  Returns (params, history)."""
    import torch
    dev = torch.device("cuda:%d" % ctx.device)
    x_all = torch.from_numpy(np.ascontiguousarray(feats, dtype=np.float32)).to(dev)
    y_all = torch.from_numpy(np.ascontiguousarray(roots, dtype=np.float32)).to(dev)
    n = x_all.shape[0]
    p0 = init_params(seed) if params is None else np.asarray(params, dtype=np.float32)
    p = torch.from_numpy(p0.copy()).to(dev)
    m = torch.zeros_like(p)
    v = torch.zeros_like(p)
    g = torch.empty_like(p)
    loss = torch.empty(1, dtype=torch.float32, device=dev)
    gen = torch.Generator(device="cpu")
    gen.manual_seed(seed)
    perm = torch.randperm(n, generator=gen).to(dev)
    pos = 0
    hist = []
    decay = (lr_final / lr) ** (1.0 / max(steps - 1, 1))
    for step in range(1, steps + 1):
        if pos + batch > n:
            perm = torch.randperm(n, generator=gen).to(dev)
            pos = 0
        idx = perm[pos:pos + batch]
        pos += batch
        xb = x_all.index_select(0, idx).contiguous()
        yb = y_all.index_select(0, idx).contiguous()
        ctx.mlp_grad(p, xb, yb, grad=g, loss=loss)
        ctx.mlp_adam(p, g, m, v, step, lr=lr * decay ** (step - 1))
        if log_every and (step % log_every == 0 or step == steps):
            hist.append((step, float(loss.item())))
            print("step %d loss %.4f" % hist[-1], flush=True)
        if checkpoint and log_every and step % (10 * log_every) == 0:
            np.savez(checkpoint, params=p.cpu().numpy(), m=m.cpu().numpy(), v=v.cpu().numpy(), step=step)
    return p.cpu().numpy(), hist


def predict(ctx, params, feats):
    """(mu, sd) of the model for features [n,18] (runs the library's forward kernel)."""
    import torch
    dev = torch.device("cuda:%d" % ctx.device)
    x = torch.from_numpy(np.ascontiguousarray(feats, dtype=np.float32)).to(dev)
    pt = torch.from_numpy(np.ascontiguousarray(params, dtype=np.float32)).to(dev)
    o = ctx.mlp_forward(pt, x).cpu().numpy().astype(np.float64)
    mu = 1.0 / (1.0 + np.exp(-o[:, 0]))
    sd = np.logaddexp(0.0, o[:, 1]) + 1e-3
    return mu, sd
