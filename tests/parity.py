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
