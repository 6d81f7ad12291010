"""Comparison of GPU results with the FP64 oracle (tolerances of the contract).

Sets (pairs, primitive candidates, contacts) must match exactly, and so must
the diagnostic counters (contacts already within d at s = 0, degenerate
skips).  Reals, per contact or per row:
  tau       |tau - tau_ref| <= 1e-10 dt
  V_k       |dV| <= 1e-10 (|V_ref| + dt eps A_k), A_k the triangle's area at s*
  V_pair    |dV| <= 1e-10 * (sum of |V_k| of the pair)
  gradient  ||dG||_inf <= 1e-10 ||G_ref||_inf per contact; a contact whose
            contact time is ill conditioned, kappa = ||dF/dX1|| l / |F_s| > 1e4
            (l its mean edge length), is compared at 1e-14 kappa instead
            (kappa capped at 1e6) and counted; a contact at s* = 0 has no
            contact-time term and keeps 1e-10
  J row     per row and component, 1e-10 times the sum of the absolute
            values of the contact gradients added into that row (each
            contribution taken at its own contact's tolerance factor)
"""
import numpy as np

TOL = 1e-10
KAPPA_ILL = 1e4


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


def vt_vertices(scene, pair_ab, keys):
    """Global vertex ids [n, 4] (p, a, b, c) of vertex-triangle contact keys."""
    keys = np.asarray(keys)
    if len(keys) == 0:
        return np.zeros((0, 4), dtype=np.int64)
    ab = np.asarray(pair_ab)[keys[:, 0]]
    kind = keys[:, 1]
    vv = np.where(kind == 1, ab[:, 1], ab[:, 0])
    vt = np.where(kind == 1, ab[:, 0], ab[:, 1])
    off = np.asarray(scene.vtx_off, dtype=np.int64)
    out = np.zeros((len(keys), 4), dtype=np.int64)
    out[:, 0] = off[vv] + keys[:, 2]
    tid = np.asarray(scene.topo_id)[vt]
    for t, topo in enumerate(scene.topos):
        m = tid == t
        if m.any():
            out[m, 1:] = off[vt[m]][:, None] + np.asarray(topo.tri)[keys[m, 3]]
    return out


def _area_and_edge(scene, gid, s):
    """Triangle area and mean edge length at s of each VT contact (translation
    invariant, so the image shift is not needed)."""
    P = [scene.x0[:, gid[:, r]].T + s[:, None] * (scene.x1[:, gid[:, r]].T - scene.x0[:, gid[:, r]].T)
         for r in range(4)]
    e1, e2, e3 = P[2] - P[1], P[3] - P[1], P[3] - P[2]
    area = 0.5 * np.linalg.norm(np.cross(e1, e2), axis=1)
    ell = (np.linalg.norm(e1, axis=1) + np.linalg.norm(e2, axis=1) + np.linalg.norm(e3, axis=1)) / 3.0
    return area, ell


def compare(gpu, ora, scene, dt, eps, check_cand=False, pair_subset=None, counters=True):
    """Assert parity.  With pair_subset, contacts/volumes are compared only on
    those pair indices (the oracle examined only them).  Returns a dict of
    statistics (number of ill-conditioned contacts, largest relative errors)."""
    stats = {}
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
        if counters:
            assert gpu["n_initially_within_d"] == ora["n_initially_within_d"], \
                (gpu["n_initially_within_d"], ora["n_initially_within_d"])
            assert gpu["n_degenerate_skipped"] == ora["n_degenerate_skipped"], \
                (gpu["n_degenerate_skipped"], ora["n_degenerate_skipped"])
    if "n_search_exhausted" in gpu:
        assert gpu["n_search_exhausted"] == 0
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
    gid = vt_vertices(scene, ora["pair_ab"], ora["ct_key"][vt])
    tf = np.zeros(0)
    if vt.any():
        area, ell = _area_and_edge(scene, gid, ora["ct_s"][vt])
        vtol = TOL * (np.abs(V_r[vt]) + dt * eps * area)
        assert np.all(np.abs(V[vt] - V_r[vt]) <= vtol), np.abs(V[vt] - V_r[vt]).max()
        fs = ora["ct_fs_rel"][vt]
        kappa = np.where(fs > 0, ell / np.maximum(fs, 1e-300), np.inf)
        # a contact clamped at s* = 0 (within d at t_n) has no contact-time term
        kappa = np.where(ora["ct_s"][vt] == 0.0, 0.0, kappa)
        tf = np.where(kappa > KAPPA_ILL, 1e-14 * np.minimum(kappa, 1e6), TOL)
        stats["ill_conditioned"] = int((kappa > KAPPA_ILL).sum())
        stats["kappa_max"] = float(kappa.max())
        gscale = np.abs(G_r[vt]).max(axis=1)
        err = np.abs(G[vt] - G_r[vt]).max(axis=1)
        assert np.all(err <= tf * gscale), (err / np.maximum(gscale, 1e-300)).max()
        stats["grad_rel_max"] = float((err / np.maximum(gscale, 1e-300)).max())
    assert np.all(G[~vt] == 0.0) and np.all(V[~vt] == 0.0)
    # volumes: per pair, relative to the sum of its |V_k|
    gvp = gpu["vol_pair"]
    gsel = np.ones(len(gvp), dtype=bool) if pair_subset is None else np.isin(gvp, np.asarray(pair_subset))
    assert np.array_equal(gvp[gsel], ora["vol_pair"])
    Vg, Vo = gpu["vol_V"][gsel], ora["vol_V"]
    vabs = np.zeros(len(Vo))
    if vt.any():
        vol_of_pair = np.full(int(ora["ct_key"][:, 0].max()) + 1, -1, dtype=np.int64)
        vol_of_pair[ora["vol_pair"]] = np.arange(len(ora["vol_pair"]))
        np.add.at(vabs, vol_of_pair[ora["ct_key"][vt, 0]], np.abs(V_r[vt]))
    assert np.all(np.abs(Vg - Vo) <= TOL * vabs), np.abs(Vg - Vo).max()
    # J rows: the tolerance of each row adds up those of its contributions
    rtol = np.zeros((len(ora["j_vol"]), 3))
    if vt.any():
        row_of = {(int(v), int(g)): r for r, (v, g) in enumerate(zip(ora["j_vol"], ora["j_vtx"]))}
        vols = vol_of_pair[ora["ct_key"][vt, 0]]
        Gv = G_r[vt].reshape(-1, 4, 3)
        for k in range(len(gid)):
            for r in range(4):
                rr = row_of[(int(vols[k]), int(gid[k, r]))]
                rtol[rr] += tf[k] * np.abs(Gv[k, r]).max()
    if pair_subset is None:
        assert np.array_equal(gpu["j_vol"], ora["j_vol"])
        assert np.array_equal(gpu["j_vtx"], ora["j_vtx"])
        jg = gpu["j_g"]
    else:
        # map volume ids through the pair index
        gv_ids = np.nonzero(gsel)[0]
        rows = np.isin(gpu["j_vol"], gv_ids)
        gj_pair = gpu["vol_pair"][gpu["j_vol"][rows]]
        oj_pair = ora["vol_pair"][ora["j_vol"]]
        assert np.array_equal(gj_pair, oj_pair)
        assert np.array_equal(gpu["j_vtx"][rows], ora["j_vtx"])
        jg = gpu["j_g"][rows]
    jerr = np.abs(jg - ora["j_g"])
    assert np.all(jerr <= rtol), (jerr - rtol).max()
    return stats


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
