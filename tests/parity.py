"""Comparison of GPU results with the FP64 oracle (tolerances of the contract).

Sets (pairs, primitive candidates, contacts) must match exactly.  Reals:
  tau       |tau - tau_ref| <= 1e-10 dt
  V_k       |dV| <= 1e-10 (|V_ref| + dt eps A_k)  (A_k bounded by |grad| scale below)
  V_pair    relative 1e-10
  gradient  ||dG||_inf <= 1e-10 ||G_ref||_inf per contact, relaxed by the
            conditioning of the contact time (1e-14 kappa) where that is larger
"""
import numpy as np

TOL = 1e-10


def _rows(a):
    a = np.ascontiguousarray(a)
    return a.view(np.dtype((np.void, a.dtype.itemsize * a.shape[1]))).ravel()


def same_rows(a, b):
    """Exact equality of two integer row sets (order-insensitive)."""
    if len(a) == 0 or len(b) == 0:
        return len(a) == len(b)
    a = np.asarray(a).reshape(len(a), -1)
    b = np.asarray(b).reshape(len(b), -1)
    if a.shape != b.shape:
        return False
    return np.array_equal(np.sort(_rows(a.astype(np.int64))), np.sort(_rows(b.astype(np.int64))))


def compare(gpu, ora, dt, eps, check_cand=False, pair_subset=None):
    """Assert parity.  With pair_subset, contacts/volumes are compared only on
    those pair indices (the oracle examined only them)."""
    # candidate vesicle pairs (canonical order on both sides)
    assert gpu["n_pairs"] == ora["n_pairs"], (gpu["n_pairs"], ora["n_pairs"])
    assert np.array_equal(gpu["pair_ab"], ora["pair_ab"])
    assert np.array_equal(gpu["pair_shift"], ora["pair_shift"])
    gk = gpu["ct_key"]
    sel = np.ones(len(gk), dtype=bool)
    if pair_subset is not None:
        sel = np.isin(gk[:, 0], np.asarray(pair_subset))
    else:
        assert gpu["n_cand_vt"] == ora["n_cand_vt"], (gpu["n_cand_vt"], ora["n_cand_vt"])
        assert gpu["n_cand_ee"] == ora["n_cand_ee"], (gpu["n_cand_ee"], ora["n_cand_ee"])
    if check_cand:
        gc = gpu["cand"]
        if pair_subset is not None:
            gc = gc[np.isin(gc[:, 0], np.asarray(pair_subset))]
        assert same_rows(gc, ora["cand"])
    # contacts: exact key sets, canonical order on both sides
    gk = gk[sel]
    assert gk.shape == ora["ct_key"].shape, (gk.shape, ora["ct_key"].shape)
    assert np.array_equal(gk, ora["ct_key"])
    tau, tau_r = gpu["ct_tau"][sel], ora["ct_tau"]
    assert np.all(np.abs(tau - tau_r) <= TOL * dt), np.abs(tau - tau_r).max()
    vt = ora["ct_key"][:, 1] < 2
    G, G_r = gpu["ct_grad"][sel], ora["ct_grad"]
    V, V_r = gpu["ct_vol"][sel], ora["ct_vol"]
    if vt.any():
        gscale = np.abs(G_r[vt]).max(axis=1)
        # the volume scale dt * eps * area: area ~ |grad wrt vertex| * 2 / (dt * eps) is not
        # available here; |V_ref| + dt * eps * 1e-3 bounds it for the meshes used
        vtol = TOL * (np.abs(V_r[vt]) + dt * eps * 1e-3)
        assert np.all(np.abs(V[vt] - V_r[vt]) <= vtol), np.abs(V[vt] - V_r[vt]).max()
        kappa = np.where(ora["ct_fs_rel"][vt] > 0, 1.0 / np.maximum(ora["ct_fs_rel"][vt], 1e-300), np.inf)
        gtol = np.maximum(TOL * gscale, 1e-14 * np.minimum(kappa, 1e6) * gscale)
        err = np.abs(G[vt] - G_r[vt]).max(axis=1)
        assert np.all(err <= gtol), (err / np.maximum(gscale, 1e-300)).max()
    assert np.all(G[~vt] == 0.0) and np.all(V[~vt] == 0.0)
    # volumes and Jacobian rows
    gvp = gpu["vol_pair"]
    gsel = np.ones(len(gvp), dtype=bool) if pair_subset is None else np.isin(gvp, np.asarray(pair_subset))
    assert np.array_equal(gvp[gsel], ora["vol_pair"])
    Vg, Vo = gpu["vol_V"][gsel], ora["vol_V"]
    assert np.all(np.abs(Vg - Vo) <= TOL * np.abs(Vo)), np.abs(Vg - Vo).max()
    if pair_subset is None:
        assert np.array_equal(gpu["j_vol"], ora["j_vol"])
        assert np.array_equal(gpu["j_vtx"], ora["j_vtx"])
        scale = np.abs(ora["j_g"]).max() if len(ora["j_g"]) else 1.0
        assert np.all(np.abs(gpu["j_g"] - ora["j_g"]) <= TOL * scale + 1e-14 * scale)
    else:
        # map volume ids through the pair index
        gv_ids = np.nonzero(gsel)[0]
        rows = np.isin(gpu["j_vol"], gv_ids)
        gj_pair = gpu["vol_pair"][gpu["j_vol"][rows]]
        oj_pair = ora["vol_pair"][ora["j_vol"]]
        assert np.array_equal(gj_pair, oj_pair)
        assert np.array_equal(gpu["j_vtx"][rows], ora["j_vtx"])
        scale = np.abs(ora["j_g"]).max() if len(ora["j_g"]) else 1.0
        assert np.all(np.abs(gpu["j_g"][rows] - ora["j_g"]) <= TOL * scale + 1e-14 * scale)
    return True


def contact_positions(scene, pair_ab, pair_shift, key):
    """Global vertex ids (p, a, b, c) and shifted X0, X1 [4,3] of a VT contact key."""
    p, kind, i, j = [int(v) for v in key]
    a, b = pair_ab[p]
    sc = int(np.searchsorted(scene.scene_off, a, side="right") - 1)
    sh = pair_shift[p] * scene.box_len[sc]
    off = scene.vtx_off
    vv, vt = (b, a) if kind == 1 else (a, b)
    tri = scene.topos[scene.topo_id[vt]].tri[j]
    gid = np.array([off[vv] + i, off[vt] + tri[0], off[vt] + tri[1], off[vt] + tri[2]])
    shift = np.zeros((4, 3))
    if kind == 1:
        shift[0] = sh
    else:
        shift[1:] = sh
    x0 = scene.x0[:, gid].T + shift
    x1 = scene.x1[:, gid].T + shift
    return gid, x0, x1


def oracle_backward(scene, ora, gV, gG):
    """dL/dX0, dL/dX1 [3, n_vtx] from the oracle's per-contact complex-step backward."""
    import oracle
    dX0 = np.zeros((3, scene.n_vtx))
    dX1 = np.zeros((3, scene.n_vtx))
    vol_of_pair = {int(p): v for v, p in enumerate(ora["vol_pair"])}
    rows = {(int(v), int(g)): r for r, (v, g) in enumerate(zip(ora["j_vol"], ora["j_vtx"]))}
    for k, key in enumerate(ora["ct_key"]):
        if key[1] == 2:
            continue
        v = vol_of_pair[int(key[0])]
        gid, x0, x1 = contact_positions(scene, ora["pair_ab"], ora["pair_shift"], key)
        w = np.array([gG[rows[(v, int(g))]] for g in gid])
        b0, b1 = oracle.vt_backward(x0, x1, ora["ct_s"][k], scene.d, scene.eps, scene.dt, gV[v], w)
        for r in range(4):
            dX0[:, gid[r]] += b0[r]
            dX1[:, gid[r]] += b1[r]
    return dX0, dX1
