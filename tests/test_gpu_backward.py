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


def test_backward_deterministic_1440(ctx):
    """Two backward calls on the same 1440-vesicle detect give the same bits:
    every vertex's sum runs in one fixed order (no floating-point atomics),
    also for vertices in several contact volumes."""
    import torch
    from paper_1812_04719_amd import stiv
    sc = S.make_config(3)
    ds = stiv.DeviceScene(sc)
    res, outs = stiv.detect(ctx, ds, sc.d, sc.eps, sc.dt, to_numpy=False)
    rng = np.random.default_rng(8)
    gV = torch.tensor(rng.normal(size=int(res["n_vol"])), device="cuda:0")
    gG = torch.tensor(rng.normal(size=(int(res["n_jrow"]), 3)), device="cuda:0")
    a0, a1 = stiv.backward(ctx, ds, sc.d, sc.eps, sc.dt, res["_struct"], gV, gG)
    b0, b1 = stiv.backward(ctx, ds, sc.d, sc.eps, sc.dt, res["_struct"], gV, gG)
    assert torch.equal(a0, b0) and torch.equal(a1, b1)
    # vertices in more than one volume exist in this scene
    jv = res["j_vtx"].cpu().numpy()
    _, counts = np.unique(jv, return_counts=True)
    print("vertices in >= 2 volumes: %d, >= 3: %d" % ((counts >= 2).sum(), (counts >= 3).sum()), flush=True)
    assert (counts >= 2).sum() > 0


def _fd_contact_adjoint(x0, x1, d, eps, dt, gV, w, h=1e-6):
    """Central differences (h) of L = gV V_k + sum_r w_r . dV_k/dX1_r with
    respect to X0 and X1 of the contact's four vertices, the contact time
    re-found at every perturbed position (oracle)."""
    def L(a, b):
        s = oracle.narrow(a, b, ee=False, d=d)
        assert s is not None
        V, _, g1 = oracle.vt_grad_full(a, b, s, d, eps, dt)
        return gV * V + float((w * g1).sum())

    out = []
    for which in (0, 1):
        fd = np.zeros((4, 3))
        for r in range(4):
            for c in range(3):
                ap, am = [x0.copy(), x1.copy()], [x0.copy(), x1.copy()]
                ap[which][r, c] += h
                am[which][r, c] -= h
                fd[r, c] = (L(*ap) - L(*am)) / (2 * h)
        out.append(fd)
    return out


@pytest.mark.timeout(900)
@pytest.mark.parametrize("case", ["two_spheres_all", "1440_sample"])
def test_backward_vs_finite_differences_config5(ctx, case):
    """Adjoint of V and dV/dX1 against central finite differences (h = 1e-6,
    FP64): every vertex-triangle contact of the two-sphere scene, and a seeded
    sample of about 10^4 contacts of the 1440-vesicle scene (whole volumes
    drawn at random until 10^4 contacts are covered; cotangents are zero on
    all other volumes and rows, so the GPU adjoint is the sum over exactly
    the sampled contacts)."""
    import torch
    from paper_1812_04719_amd import stiv
    sc = S.make_config(1) if case == "two_spheres_all" else S.make_config(3)
    ds = stiv.DeviceScene(sc)
    res, _ = stiv.detect(ctx, ds, sc.d, sc.eps, sc.dt)
    keys, vp = res["ct_key"], res["vol_pair"]
    vt = keys[:, 1] < 2
    rng = np.random.default_rng(51)
    vol_ids = np.arange(len(vp))
    if case == "1440_sample":
        order = rng.permutation(len(vp))
        n_of = np.bincount(keys[vt, 0], minlength=int(res["n_pairs"]))[vp]
        take = np.cumsum(n_of[order]) <= 10000
        vol_ids = np.sort(order[take])
    gV = np.zeros(len(vp))
    gV[vol_ids] = rng.normal(size=len(vol_ids))
    rows = np.isin(res["j_vol"], vol_ids)
    gG = np.zeros((int(res["n_jrow"]), 3))
    gG[rows] = rng.normal(size=(int(rows.sum()), 3))
    dX0, dX1 = stiv.backward(ctx, ds, sc.d, sc.eps, sc.dt, res["_struct"], torch.tensor(gV, device="cuda:0"),
                             torch.tensor(gG, device="cuda:0"))
    dX0, dX1 = dX0.cpu().numpy(), dX1.cpu().numpy()
    # finite differences per sampled contact, summed per vertex
    f0 = np.zeros_like(dX0)
    f1 = np.zeros_like(dX1)
    vol_of_pair = {int(p): v for v, p in enumerate(vp)}
    row_of = {(int(v), int(g)): r for r, (v, g) in enumerate(zip(res["j_vol"], res["j_vtx"]))}
    sel = set(vol_ids.tolist())
    n_done = 0
    for k in np.nonzero(vt)[0]:
        v = vol_of_pair[int(keys[k, 0])]
        if v not in sel:
            continue
        gid, x0, x1 = parity.contact_positions(sc, res["pair_ab"], res["pair_shift"], keys[k])
        w = np.array([gG[row_of[(v, int(g))]] for g in gid])
        a0, a1 = _fd_contact_adjoint(x0, x1, sc.d, sc.eps, sc.dt, gV[v], w)
        for r in range(4):
            f0[:, gid[r]] += a0[r]
            f1[:, gid[r]] += a1[r]
        n_done += 1
    print("FD-checked contacts: %d in %d volumes" % (n_done, len(vol_ids)), flush=True)
    assert n_done >= (79 if case == "two_spheres_all" else 9000)
    for got, want in ((dX0, f0), (dX1, f1)):
        scale = np.abs(want).max()
        assert scale > 0
        assert np.abs(got - want).max() <= 1e-6 * scale, np.abs(got - want).max() / scale
