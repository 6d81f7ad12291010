"""GPU backward pass (adjoint) against the oracle's complex-step backward and
against central finite differences of the forward."""
import numpy as np
import pytest

import oracle
import parity
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


def _gpu_backward(ctx, sc, seed):
    import torch
    from paper_1812_04719_amd import stiv
    print("backward case: n_ves=%d seed=%d" % (sc.n_ves, seed), flush=True)
    ds = stiv.DeviceScene(sc)
    res, outs = stiv.detect(ctx, ds, sc.d, sc.eps, sc.dt, to_numpy=False)
    rng = np.random.default_rng(seed)
    gV = rng.normal(size=int(res["n_vol"]))
    gG = rng.normal(size=(int(res["n_jrow"]), 3))
    dX0, dX1 = stiv.backward(ctx, ds, sc.d, sc.eps, sc.dt, res["_struct"],
                             torch.tensor(gV, device="cuda:0"), torch.tensor(gG, device="cuda:0"))
    return gV, gG, dX0.cpu().numpy(), dX1.cpu().numpy(), res


@pytest.mark.parametrize("d", [None, 0.0])
def test_backward_vs_oracle_two_spheres(ctx, d):
    sc = S.make_config(1)
    if d is not None:
        sc = sc.with_params(d=d)
    gV, gG, dX0, dX1, _ = _gpu_backward(ctx, sc, 5)
    ora = oracle.detect(sc)
    o0, o1 = parity.oracle_backward(sc, ora, gV, gG)
    for got, want in ((dX0, o0), (dX1, o1)):
        scale = np.abs(want).max()
        assert scale > 0
        assert np.abs(got - want).max() <= 1e-10 * scale, np.abs(got - want).max() / scale


def test_backward_vs_oracle_rsa(ctx):
    sc = S.make_config(2)
    gV, gG, dX0, dX1, _ = _gpu_backward(ctx, sc, 6)
    ora = oracle.detect(sc)
    o0, o1 = parity.oracle_backward(sc, ora, gV, gG)
    for got, want in ((dX0, o0), (dX1, o1)):
        scale = np.abs(want).max()
        assert np.abs(got - want).max() <= 1e-10 * scale


def test_backward_vs_oracle_1440(ctx):
    """The full 1440-vesicle scene: every vertex-triangle contact's adjoint
    (random cotangents on all volumes and J rows) against the oracle's
    complex-step backward, 1e-10 of the largest component."""
    sc = S.make_config(3)
    gV, gG, dX0, dX1, res = _gpu_backward(ctx, sc, 7)
    ora = oracle.detect(sc)
    assert np.array_equal(res["ct_key"].cpu().numpy(), ora["ct_key"])
    assert int(res["n_ct_vt"]) > 10000
    o0, o1 = parity.oracle_backward(sc, ora, gV, gG)
    for got, want in ((dX0, o0), (dX1, o1)):
        scale = np.abs(want).max()
        assert scale > 0
        assert np.abs(got - want).max() <= 1e-10 * scale, np.abs(got - want).max() / scale


def test_autograd_function_vs_finite_differences(ctx):
    """torch.autograd through the library backward vs central FD (h = 1e-6) of
    L = sum(a V) + sum(b G) on a sample of coordinates of X0 and X1."""
    import torch
    from paper_1812_04719_amd import autograd, stiv
    sc = S.make_config(1)
    ds = stiv.DeviceScene(sc)
    x0 = ds.x0.clone().requires_grad_(True)
    x1 = ds.x1.clone().requires_grad_(True)
    V, G, idx = autograd.contact_volumes(ctx, ds, x0, x1, sc.d, sc.eps, sc.dt)
    rng = np.random.default_rng(9)
    a = torch.tensor(rng.normal(size=V.shape[0]), device="cuda:0")
    bvec = torch.tensor(rng.normal(size=tuple(G.shape)), device="cuda:0")
    L = (a * V).sum() + (bvec * G).sum()
    g0, g1 = torch.autograd.grad(L, (x0, x1))
    keys = idx["ct_key"].cpu().numpy()
    jv = idx["j_vtx"].cpu().numpy()
    verts = np.unique(jv)
    pick = rng.choice(verts, 12, replace=False)
    h = 1e-6

    def loss(X0, X1):
        with torch.no_grad():
            Vh, Gh, ih = autograd.contact_volumes(ctx, ds, X0, X1, sc.d, sc.eps, sc.dt)
        assert np.array_equal(ih["ct_key"].cpu().numpy(), keys)  # same contact set
        assert np.array_equal(ih["j_vtx"].cpu().numpy(), jv)
        return float(((a * Vh).sum() + (bvec * Gh).sum()).item())

    for which, grad in ((0, g0), (1, g1)):
        for v in pick:
            for c in range(3):
                Xp = [x0.detach().clone(), x1.detach().clone()]
                Xm = [x0.detach().clone(), x1.detach().clone()]
                Xp[which][c, v] += h
                Xm[which][c, v] -= h
                fd = (loss(*Xp) - loss(*Xm)) / (2 * h)
                an = float(grad[c, v].item())
                assert abs(fd - an) <= 1e-5 * max(abs(an), 1e-3), (which, v, c, fd, an)
