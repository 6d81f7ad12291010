"""GPU tests of the learned contact-time bracket: the bf16 matrix-core
perceptron kernels against the CPU FP64 reference (same bf16 rounding
points), Adam, and the bracketed root search, which must return exactly the
contacts of the plain search (and of the oracle)."""
import os

import numpy as np
import pytest

import mlp_ref
import oracle
import parity
import tinyscenes as T
from paper_1812_04719_amd import scenes as S

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    import torch
    from paper_1812_04719_amd import stiv
    assert torch.cuda.is_available()
    c = stiv.Context(0)
    yield c
    c.close()


def _rand_params(seed, scale=1.0):
    from paper_1812_04719_amd import toi_model
    rng = np.random.default_rng(seed)
    p = toi_model.init_params(seed).astype(np.float64)
    p += rng.normal(0, 0.05, p.shape)
    lay, _ = toi_model.layout()
    o, _ = lay["W3"]
    p[o:o + 128] *= 10.0 * scale  # make the outputs O(1)
    return p.astype(np.float32)


@pytest.mark.parametrize("n", [1, 15, 16, 17, 1000, 40000])
def test_mlp_forward_vs_reference(ctx, n):
    """Ragged tile tails and many workgroups; checks the MFMA operand layout."""
    import torch
    print("mlp forward n=%d" % n, flush=True)
    rng = np.random.default_rng(n)
    p = _rand_params(n)
    x = rng.normal(0, 1, (n, 18)).astype(np.float32)
    out = ctx.mlp_forward(torch.from_numpy(p).cuda(), torch.from_numpy(x).cuda()).cpu().numpy()
    ref, _ = mlp_ref.forward(p, x)
    # FP32 accumulation vs FP64 and a few hidden units landing on the other
    # side of a bf16 rounding boundary: errors of a few bf16 ulps of |o|
    scale = np.abs(ref).max() + 1.0
    err = np.abs(out - ref).max()
    assert err <= 2e-2 * scale, (err, scale)
    # a wrong operand layout gives O(scale) errors; typical errors are far below the bound
    assert np.median(np.abs(out - ref)) <= 2e-3 * scale


def test_mlp_forward_exact_small_integers(ctx):
    """Weights and inputs that are small dyadic numbers keep every sum exact
    in FP32 and bf16: the kernel must then agree bit for bit."""
    import torch
    from paper_1812_04719_amd import toi_model
    rng = np.random.default_rng(7)
    lay, npar = toi_model.layout()
    p = np.zeros(npar, dtype=np.float32)
    o, _ = lay["W1"]
    p[o:o + 18 * 64] = rng.integers(-2, 3, 18 * 64) / 4.0
    o, _ = lay["b1"]
    p[o:o + 64] = rng.integers(-4, 5, 64) / 4.0
    o, _ = lay["W2"]
    w2 = np.zeros((64, 64))
    for j in range(64):  # two nonzeros per column keep h2 within 8 significant bits
        rows = rng.choice(64, 2, replace=False)
        w2[rows, j] = rng.integers(-2, 3, 2) / 2.0
    p[o:o + 4096] = w2.ravel()
    o, _ = lay["W3"]
    w3 = np.zeros((64, 2))
    w3[rng.choice(64, 3, replace=False), 0] = [1.0, -0.5, 0.25]
    w3[rng.choice(64, 3, replace=False), 1] = [0.5, 1.0, -1.0]
    p[o:o + 128] = w3.ravel()
    x = (rng.integers(-3, 4, (100, 18)) / 2.0).astype(np.float32)
    out = ctx.mlp_forward(torch.from_numpy(p).cuda(), torch.from_numpy(x).cuda()).cpu().numpy()
    ref, (xr, h1, h2) = mlp_ref.forward(p, x)
    assert np.array_equal(mlp_ref.bf16(h1), h1) and np.array_equal(mlp_ref.bf16(h2), h2)
    assert np.array_equal(out.astype(np.float64), ref), np.abs(out - ref).max()


@pytest.mark.parametrize("n", [37, 5000])
def test_mlp_grad_vs_reference(ctx, n):
    import torch
    print("mlp grad n=%d" % n, flush=True)
    rng = np.random.default_rng(100 + n)
    p = _rand_params(n, scale=0.2)
    x = rng.normal(0, 1, (n, 18)).astype(np.float32)
    s = rng.uniform(0, 1, n).astype(np.float32)
    g, loss = ctx.mlp_grad(torch.from_numpy(p).cuda(), torch.from_numpy(x).cuda(), torch.from_numpy(s).cuda())
    g = g.cpu().numpy().astype(np.float64)
    gr = mlp_ref.grad(p, x, s.astype(np.float64), round_bf16=True)
    lr = mlp_ref.loss(p, x, s.astype(np.float64), round_bf16=True)
    assert abs(float(loss.item()) - lr) <= 1e-2 * (abs(lr) + 1.0)
    # deltas are rounded to bf16 in the backward products: per-entry relative
    # error a few bf16 ulps; compare block by block against each block's scale
    from paper_1812_04719_amd import toi_model
    lay, _ = toi_model.layout()
    for name, (o, shp) in lay.items():
        k = int(np.prod(shp))
        a, b = g[o:o + k], gr[o:o + k]
        sc = np.abs(b).max() + 1e-12
        assert np.abs(a - b).max() <= 3e-2 * sc, (name, np.abs(a - b).max(), sc)
        if k > 8:
            c = np.corrcoef(a, b)[0, 1]
            assert c > 0.999, (name, c)
    # deterministic: same inputs, same bits
    g2, _ = ctx.mlp_grad(torch.from_numpy(p).cuda(), torch.from_numpy(x).cuda(), torch.from_numpy(s).cuda())
    assert np.array_equal(g2.cpu().numpy().astype(np.float64), g)


def test_adam_step(ctx):
    import torch
    rng = np.random.default_rng(9)
    n = 5506
    p = rng.normal(0, 1, n).astype(np.float32)
    g = rng.normal(0, 1, n).astype(np.float32)
    m = rng.normal(0, 0.1, n).astype(np.float32)
    v = rng.uniform(0, 0.1, n).astype(np.float32)
    tp, tg, tm, tv = (torch.from_numpy(a.copy()).cuda() for a in (p, g, m, v))
    ctx.mlp_adam(tp, tg, tm, tv, 3, lr=1e-2, beta1=0.9, beta2=0.999, eps=1e-8)
    # reference in FP32 with the kernel's FP32 constants (1 - 0.999f is not 0.001)
    f = np.float32
    b1, b2 = f(0.9), f(0.999)
    m2 = b1 * m + (f(1) - b1) * g
    v2 = b2 * v + (f(1) - b2) * g * g
    c1, c2 = f(1) - b1 ** 3, f(1) - b2 ** 3
    p2 = p - f(1e-2) * (m2 / c1) / (np.sqrt(v2 / c2) + f(1e-8))
    assert np.allclose(tm.cpu().numpy(), m2, rtol=1e-5, atol=1e-7)
    assert np.allclose(tv.cpu().numpy(), v2, rtol=1e-5, atol=1e-9)
    assert np.allclose(tp.cpu().numpy(), p2, rtol=1e-5, atol=1e-5)


def _const_model(mu, o1):
    """A model whose prediction is the same for every input."""
    from paper_1812_04719_amd import toi_model
    lay, npar = toi_model.layout()
    p = np.zeros(npar, dtype=np.float32)
    o, _ = lay["b3"]
    p[o] = np.log(mu / (1 - mu))
    p[o + 1] = o1
    return p


def _scenes():
    yield "two_spheres", S.make_two_spheres(seed=1)
    yield "rsa64", S.make_rsa_scene(seed=2, n=64)
    yield "planes", T.translating_planes()


@pytest.mark.parametrize("model", ["const_0.05", "const_0.5", "const_0.95", "wide", "random"])
def test_bracket_same_contacts(ctx, model):
    """Whatever the model predicts, the bracketed search returns the contacts
    of the plain search; both match the oracle."""
    from paper_1812_04719_amd import stiv
    if model.startswith("const"):
        p, kw = _const_model(float(model.split("_")[1]), -8.0), 3.0
    elif model == "wide":
        p, kw = _const_model(0.5, 4.0), 3.0
    else:
        p, kw = _rand_params(5), 2.0
    ctx.set_toi_model(p, kw)
    for name, sc in _scenes():
        print("bracket %s on %s" % (model, name), flush=True)
        ds = stiv.DeviceScene(sc)
        plain, _ = stiv.detect(ctx, ds, sc.d, sc.eps, sc.dt)
        learned, _ = stiv.detect(ctx, ds, sc.d, sc.eps, sc.dt, learned_bracket=True)
        st = ctx.stats()
        assert np.array_equal(plain["ct_key"], learned["ct_key"])
        assert np.all(np.abs(plain["ct_tau"] - learned["ct_tau"]) <= 1e-12 * sc.dt)
        assert np.array_equal(plain["vol_pair"], learned["vol_pair"])
        assert np.array_equal(plain["j_vtx"], learned["j_vtx"])
        o = oracle.detect(sc)
        parity.compare(learned, o, sc, sc.dt, sc.eps)
        assert 0 <= st["bracket_certified"] <= st["root_searches"]
    ctx.set_toi_model(None)


@pytest.mark.parametrize("model", ["const_0.3", "random", "trained"])
def test_bracket_same_contacts_d0(ctx, model):
    """The bracketed search of the coplanarity variant (d = 0: F = g, degree
    3) returns the plain search's contacts, and both match the oracle."""
    from paper_1812_04719_amd import stiv, toi_model
    if model == "trained":
        if not os.path.exists(toi_model.DEFAULT_WEIGHTS):
            pytest.skip("no trained bracket model in the package")
        toi_model.install(ctx)
    elif model == "random":
        ctx.set_toi_model(_rand_params(6), 2.0)
    else:
        ctx.set_toi_model(_const_model(0.3, -8.0), 3.0)
    for name, sc in [("two_spheres", S.make_two_spheres(seed=1)), ("rsa64", S.make_config(2))]:
        print("bracket d=0 %s on %s" % (model, name), flush=True)
        ds = stiv.DeviceScene(sc)
        plain, _ = stiv.detect(ctx, ds, 0.0, sc.eps, sc.dt)
        learned, _ = stiv.detect(ctx, ds, 0.0, sc.eps, sc.dt, learned_bracket=True)
        st = ctx.stats()
        assert np.array_equal(plain["ct_key"], learned["ct_key"])
        assert np.all(np.abs(plain["ct_tau"] - learned["ct_tau"]) <= 1e-12 * sc.dt)
        o = oracle.detect(sc, d=0.0)
        parity.compare(learned, o, sc, sc.dt, sc.eps)
        assert st["root_searches"] > 0 and 0 <= st["bracket_certified"] <= st["root_searches"]
    ctx.set_toi_model(None)


def test_learned_flag_without_model_is_an_error(ctx):
    from paper_1812_04719_amd import stiv
    ctx.set_toi_model(None)
    sc = T.translating_planes()
    ds = stiv.DeviceScene(sc)
    with pytest.raises(stiv.StivError, match="STIV_E_STATE"):
        stiv.detect(ctx, ds, sc.d, sc.eps, sc.dt, learned_bracket=True)
    with pytest.raises(stiv.StivError, match="STIV_E_ARG"):
        ctx.set_toi_model(np.zeros(10, dtype=np.float32))
    bad = _const_model(0.5, 0.0)
    bad[3] = np.nan
    with pytest.raises(stiv.StivError, match="STIV_E_ARG"):
        ctx.set_toi_model(bad)


def test_trained_model_same_contacts_and_speed(ctx):
    """The shipped model on the 1440-vesicle workload: identical contacts,
    and the speed of the narrow phase with the bracket relative to the plain
    search.  The bracket does not beat the plain search on this workload (the
    plain subdivision decides about half of the searches in one interval and
    needs 2.5 on average); the ratio is reported in the assertion message and
    only a collapse below 0.7 fails."""
    from paper_1812_04719_amd import stiv, toi_model
    if not os.path.exists(toi_model.DEFAULT_WEIGHTS):
        pytest.skip("no trained bracket model in the package")
    meta = toi_model.install(ctx)
    sc = S.make_config(3)
    ds = stiv.DeviceScene(sc)
    print("trained model %s on 1440 vesicles" % meta.get("name", "?"), flush=True)
    plain, outs = stiv.detect(ctx, ds, sc.d, sc.eps, sc.dt)
    learned, outs = stiv.detect(ctx, ds, sc.d, sc.eps, sc.dt, learned_bracket=True)
    assert np.array_equal(plain["ct_key"], learned["ct_key"])
    assert np.all(np.abs(plain["ct_tau"] - learned["ct_tau"]) <= 1e-12 * sc.dt)
    tp, tl = [], []
    for _ in range(5):
        stiv.detect(ctx, ds, sc.d, sc.eps, sc.dt, outputs=outs, to_numpy=False)
        tp.append(ctx.stage_times()[4])
        stiv.detect(ctx, ds, sc.d, sc.eps, sc.dt, outputs=outs, to_numpy=False, learned_bracket=True)
        tl.append(ctx.stage_times()[4])
    st = ctx.stats()
    ctx.set_toi_model(None)
    gain = float(np.median(tp) / np.median(tl))
    msg = ("narrow phase ms: plain %.4f learned %.4f, learned speed / plain speed = %.3f (bracket used in %d of %d "
           "searches)" % (np.median(tp), np.median(tl), gain, st["bracket_certified"], st["root_searches"]))
    print(msg, flush=True)
    assert gain > 0.7, msg
