"""FP64 CPU oracle of the contact-detection path -- TEST INFRASTRUCTURE ONLY.

Only the tests, the smoke check and the benchmark's CPU-baseline leg may
import this package.  The product (the GPU library and its binding) never
imports, links or executes anything here, and shares no code with it.

``detect(scene, ...)`` runs the brute-force reference in ``stiv_oracle.c``
on a scene produced by the seeded generator and returns numpy arrays.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
import threading

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "stiv_oracle.c")
_LIB = os.path.join(_HERE, "libstiv_oracle.so")
_lock = threading.Lock()
_lib = None


def build(force: bool = False) -> str:
    """Compile the oracle with gcc: FP64, no contraction, OpenMP."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-std=c99", "-ffp-contract=off", "-fno-fast-math", "-fopenmp",
                               "-fPIC", "-shared", "-Wall", "-Wno-unknown-pragmas", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


class _Scene(C.Structure):
    _fields_ = [("n_ves", C.c_int32), ("n_vtx", C.c_int32), ("n_scenes", C.c_int32), ("n_topo", C.c_int32),
                ("vtx_off", C.c_void_p), ("topo_id", C.c_void_p), ("scene_off", C.c_void_p),
                ("box_len", C.c_void_p), ("x0", C.c_void_p), ("x1", C.c_void_p),
                ("topo_nv", C.c_void_p), ("tri", C.c_void_p), ("tri_off", C.c_void_p),
                ("edge", C.c_void_p), ("edge_off", C.c_void_p)]


class _Result(C.Structure):
    _fields_ = [("n_pairs", C.c_int64), ("pair_ab", C.c_void_p), ("pair_shift", C.c_void_p),
                ("ves_box", C.c_void_p),
                ("n_cand_vt", C.c_int64), ("n_cand_ee", C.c_int64),
                ("n_cand_list", C.c_int64), ("cand", C.c_void_p),
                ("n_ct", C.c_int64), ("n_ct_vt", C.c_int64), ("n_ct_ee", C.c_int64),
                ("ct_key", C.c_void_p), ("ct_s", C.c_void_p), ("ct_tau", C.c_void_p), ("ct_vol", C.c_void_p),
                ("ct_grad", C.c_void_p), ("ct_fs_rel", C.c_void_p),
                ("n_vol", C.c_int64), ("vol_pair", C.c_void_p), ("vol_V", C.c_void_p),
                ("n_jrow", C.c_int64), ("j_vol", C.c_void_p), ("j_vtx", C.c_void_p), ("j_g", C.c_void_p),
                ("n_initially_within_d", C.c_int64), ("n_degenerate_skipped", C.c_int64),
                ("n_flag", C.c_int64 * 4), ("min_margin", C.c_double * 4), ("threads_used", C.c_int32)]


def lib():
    global _lib
    with _lock:
        if _lib is None:
            L = C.CDLL(build())
            L.oracle_detect.restype = C.POINTER(_Result)
            L.oracle_detect.argtypes = [C.POINTER(_Scene), C.c_double, C.c_double, C.c_double, C.c_int,
                                        C.c_void_p, C.c_int64, C.c_int]
            L.oracle_free.argtypes = [C.POINTER(_Result)]
            L.oracle_narrow.restype = C.c_int
            L.oracle_narrow.argtypes = [C.c_void_p, C.c_void_p, C.c_int, C.c_double, C.c_void_p, C.c_void_p]
            L.oracle_vt_volume.argtypes = [C.c_void_p, C.c_void_p, C.c_double, C.c_double, C.c_double,
                                           C.c_double, C.c_void_p, C.c_void_p]
            L.oracle_poly.argtypes = [C.c_void_p, C.c_void_p, C.c_int, C.c_double, C.c_void_p]
            L.oracle_roots01.restype = C.c_int
            L.oracle_roots01.argtypes = [C.c_void_p, C.c_int, C.c_void_p]
            L.oracle_sort_scatter.argtypes = [C.c_int64, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p]
            L.oracle_vt_grad_full.argtypes = [C.c_void_p, C.c_void_p, C.c_double, C.c_double, C.c_double, C.c_double,
                                              C.c_void_p, C.c_void_p, C.c_void_p]
            L.oracle_toi_samples.argtypes = [C.POINTER(_Scene), C.c_double, C.c_void_p, C.c_int64, C.c_void_p,
                                             C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_int]
            L.oracle_vt_backward.argtypes = [C.c_void_p, C.c_void_p, C.c_double, C.c_double, C.c_double, C.c_double,
                                             C.c_double, C.c_void_p, C.c_void_p, C.c_void_p]
            _lib = L
    return _lib


def _ptr(a):
    return a.ctypes.data_as(C.c_void_p)


def _arr(ptr, n, dtype, shape=None):
    n = int(n)
    if n == 0:
        out = np.zeros(0, dtype=dtype)
    else:
        buf = (C.c_char * (n * np.dtype(dtype).itemsize)).from_address(ptr)
        out = np.frombuffer(buf, dtype=dtype).copy()
    if shape is not None:
        out = out.reshape(shape)
    return out


class OracleResult(dict):
    __getattr__ = dict.__getitem__


def _scene_struct(scene):
    keep = {}
    keep["x0"] = np.ascontiguousarray(scene.x0, dtype=np.float64)
    keep["x1"] = np.ascontiguousarray(scene.x1, dtype=np.float64)
    keep["vtx_off"] = np.ascontiguousarray(scene.vtx_off, dtype=np.int32)
    keep["topo_id"] = np.ascontiguousarray(scene.topo_id, dtype=np.int32)
    keep["scene_off"] = np.ascontiguousarray(scene.scene_off, dtype=np.int32)
    keep["box_len"] = np.ascontiguousarray(scene.box_len, dtype=np.float64)
    keep["topo_nv"] = np.array([t.nv for t in scene.topos], dtype=np.int32)
    keep["tri"] = np.ascontiguousarray(np.concatenate([t.tri for t in scene.topos]), dtype=np.int32)
    keep["tri_off"] = np.concatenate([[0], np.cumsum([t.nt for t in scene.topos])]).astype(np.int32)
    keep["edge"] = np.ascontiguousarray(np.concatenate([t.edge for t in scene.topos]), dtype=np.int32)
    keep["edge_off"] = np.concatenate([[0], np.cumsum([t.ne for t in scene.topos])]).astype(np.int32)
    s = _Scene(scene.n_ves, scene.n_vtx, scene.n_scenes, len(scene.topos),
               _ptr(keep["vtx_off"]), _ptr(keep["topo_id"]), _ptr(keep["scene_off"]), _ptr(keep["box_len"]),
               _ptr(keep["x0"]), _ptr(keep["x1"]), _ptr(keep["topo_nv"]), _ptr(keep["tri"]),
               _ptr(keep["tri_off"]), _ptr(keep["edge"]), _ptr(keep["edge_off"]))
    return s, keep


def detect(scene, d=None, eps=None, dt=None, emit_candidates=False, pair_subset=None, threads=0):
    """Brute-force FP64 detection.  Returns an OracleResult of numpy arrays.

    pair_subset: optional ascending indices into the canonical pair list; only
    those vesicle pairs are examined beyond the pair stage.
    """
    L = lib()
    d = scene.d if d is None else d
    eps = scene.eps if eps is None else eps
    dt = scene.dt if dt is None else dt
    s, keep = _scene_struct(scene)
    sub = None
    nsub = 0
    if pair_subset is not None:
        sub = np.ascontiguousarray(pair_subset, dtype=np.int64)
        nsub = sub.size
    rp = L.oracle_detect(C.byref(s), d, eps, dt, 1 if emit_candidates else 0,
                         _ptr(sub) if sub is not None else None, nsub, int(threads))
    r = rp.contents
    out = OracleResult(
        n_pairs=r.n_pairs,
        pair_ab=_arr(r.pair_ab, 2 * r.n_pairs, np.int32, (-1, 2)),
        pair_shift=_arr(r.pair_shift, 3 * r.n_pairs, np.int32, (-1, 3)),
        ves_box=_arr(r.ves_box, 6 * scene.n_ves, np.float64, (-1, 6)),
        n_cand_vt=r.n_cand_vt, n_cand_ee=r.n_cand_ee,
        cand=_arr(r.cand, 4 * r.n_cand_list, np.int32, (-1, 4)),
        n_ct=r.n_ct, n_ct_vt=r.n_ct_vt, n_ct_ee=r.n_ct_ee,
        ct_key=_arr(r.ct_key, 4 * r.n_ct, np.int32, (-1, 4)),
        ct_s=_arr(r.ct_s, r.n_ct, np.float64), ct_tau=_arr(r.ct_tau, r.n_ct, np.float64),
        ct_vol=_arr(r.ct_vol, r.n_ct, np.float64), ct_grad=_arr(r.ct_grad, 12 * r.n_ct, np.float64, (-1, 12)),
        ct_fs_rel=_arr(r.ct_fs_rel, r.n_ct, np.float64),
        n_vol=r.n_vol, vol_pair=_arr(r.vol_pair, r.n_vol, np.int32), vol_V=_arr(r.vol_V, r.n_vol, np.float64),
        n_jrow=r.n_jrow, j_vol=_arr(r.j_vol, r.n_jrow, np.int32), j_vtx=_arr(r.j_vtx, r.n_jrow, np.int32),
        j_g=_arr(r.j_g, 3 * r.n_jrow, np.float64, (-1, 3)),
        n_initially_within_d=r.n_initially_within_d, n_degenerate_skipped=r.n_degenerate_skipped,
        n_flag=list(r.n_flag), min_margin=list(r.min_margin), threads_used=r.threads_used,
    )
    L.oracle_free(rp)
    del keep
    return out


def narrow(x0, x1, ee=False, d=0.0):
    """Earliest contact parameter s* of one primitive pair, or None.

    x0, x1: [4,3] positions of (vertex p, triangle a, b, c) or of
    (edge a-b, edge c-e).
    """
    a = np.ascontiguousarray(x0, dtype=np.float64).reshape(12)
    b = np.ascontiguousarray(x1, dtype=np.float64).reshape(12)
    s = C.c_double(0.0)
    w = C.c_int64(0)
    hit = lib().oracle_narrow(_ptr(a), _ptr(b), 1 if ee else 0, float(d), C.byref(s), C.byref(w))
    return s.value if hit else None


def vt_volume(x0, x1, s, d, eps, dt):
    """(V, grad[4,3]) of a vertex-triangle contact at parameter s."""
    a = np.ascontiguousarray(x0, dtype=np.float64).reshape(12)
    b = np.ascontiguousarray(x1, dtype=np.float64).reshape(12)
    V = C.c_double(0.0)
    g = np.zeros(12)
    lib().oracle_vt_volume(_ptr(a), _ptr(b), float(s), float(d), float(eps), float(dt), C.byref(V), _ptr(g))
    return V.value, g.reshape(4, 3)


def poly(x0, x1, ee=False, d=0.0):
    a = np.ascontiguousarray(x0, dtype=np.float64).reshape(12)
    b = np.ascontiguousarray(x1, dtype=np.float64).reshape(12)
    f = np.zeros(7)
    lib().oracle_poly(_ptr(a), _ptr(b), 1 if ee else 0, float(d), _ptr(f))
    return f


def roots01(coef):
    c = np.zeros(7)
    coef = np.asarray(coef, dtype=np.float64)
    c[: coef.size] = coef
    out = np.zeros(8)
    n = lib().oracle_roots01(_ptr(c), int(coef.size - 1), _ptr(out))
    return out[:n].copy()


def sort_scatter(keys, idx):
    keys = np.ascontiguousarray(keys, dtype=np.uint64)
    idx = np.ascontiguousarray(idx, dtype=np.int64)
    ko = np.zeros_like(keys)
    po = np.zeros_like(idx)
    lib().oracle_sort_scatter(keys.size, _ptr(keys), _ptr(idx), _ptr(ko), _ptr(po))
    return ko, po


def vt_grad_full(x0, x1, s, d, eps, dt):
    """(V, dV/dX0 [4,3], dV/dX1 [4,3]) of a vertex-triangle contact at parameter s."""
    a = np.ascontiguousarray(x0, dtype=np.float64).reshape(12)
    b = np.ascontiguousarray(x1, dtype=np.float64).reshape(12)
    V = C.c_double(0.0)
    g0 = np.zeros(12)
    g1 = np.zeros(12)
    lib().oracle_vt_grad_full(_ptr(a), _ptr(b), float(s), float(d), float(eps), float(dt), C.byref(V), _ptr(g0),
                              _ptr(g1))
    return V.value, g0.reshape(4, 3), g1.reshape(4, 3)


def vt_backward(x0, x1, s, d, eps, dt, gV, w):
    """Vector-Jacobian product of (V_k, dV_k/dX1) with cotangents (gV, w[4,3]):
    returns (dL/dX0 [4,3], dL/dX1 [4,3]) by the complex-step method."""
    a = np.ascontiguousarray(x0, dtype=np.float64).reshape(12)
    b = np.ascontiguousarray(x1, dtype=np.float64).reshape(12)
    ww = np.ascontiguousarray(w, dtype=np.float64).reshape(12)
    g0 = np.zeros(12)
    g1 = np.zeros(12)
    lib().oracle_vt_backward(_ptr(a), _ptr(b), float(s), float(d), float(eps), float(dt), float(gV), _ptr(ww),
                             _ptr(g0), _ptr(g1))
    return g0.reshape(4, 3), g1.reshape(4, 3)


def toi_samples(scene, d=None, threads=0):
    """Training samples of the learned contact-time bracket for every
    primitive candidate of the scene: (features [n,18] float32, first root of
    F in [0,1] [n] float64, -1 none; hard [n] bool: the
    Bernstein coefficients of F on [0,1] do not exclude a root)."""
    d = scene.d if d is None else d
    r = detect(scene, d=d, emit_candidates=True, threads=threads)
    keys = np.ascontiguousarray(r["cand"], dtype=np.int32)
    n = keys.shape[0]
    feat = np.zeros((n, 18), dtype=np.float32)
    root = np.zeros(n, dtype=np.float64)
    hard = np.zeros(n, dtype=np.int8)
    s, keep = _scene_struct(scene)
    pab = np.ascontiguousarray(r["pair_ab"], dtype=np.int32)
    psh = np.ascontiguousarray(r["pair_shift"], dtype=np.int32)
    lib().oracle_toi_samples(C.byref(s), float(d), _ptr(keys), n, _ptr(pab), _ptr(psh), _ptr(feat), _ptr(root),
                             _ptr(hard), int(threads))
    del keep
    return feat, root, hard.astype(bool)


# ---------------------------------------------------------------------------
# LCP matrix (Sec. 3.3.3, Alg. 3): B(j,k) = sum over vesicles i of
# g_j,i . M_i g_k,i, with g_j,i the Jacobian row of volume j restricted to
# vesicle i's points and M_i the vesicle's operator block on its active
# points (the points that appear in J).
# ---------------------------------------------------------------------------
def lcp_layout(vtx_off, j_vtx):
    """Active points per vesicle: (act_off [n_ves+1], act_vtx, m_off [n_ves+1])
    with blocks M_i of size [3 a_i]^2 at m_off[i] (doubles)."""
    vtx_off = np.asarray(vtx_off, dtype=np.int64)
    act = np.unique(np.asarray(j_vtx, dtype=np.int64))
    act_off = np.searchsorted(act, vtx_off).astype(np.int64)
    a = np.diff(act_off)
    m_off = np.concatenate([[0], np.cumsum(9 * a * a)]).astype(np.int64)
    return act_off, act.astype(np.int32), m_off


def lcp_matrix(n_vol, vtx_off, vol_pair, pair_ab, j_vol, j_vtx, j_g, act_off, act_vtx, m_off, M):
    """Dense B [n_vol, n_vol] by the loop of Alg. 3 (per vesicle, per pair of
    its volumes), and the structural pattern (bool) of pairs sharing a vesicle."""
    vtx_off = np.asarray(vtx_off, dtype=np.int64)
    n_ves = len(vtx_off) - 1
    j_vol = np.asarray(j_vol, dtype=np.int64)
    j_vtx = np.asarray(j_vtx, dtype=np.int64)
    B = np.zeros((n_vol, n_vol))
    S = np.zeros((n_vol, n_vol), dtype=bool)
    ves_of_row = np.searchsorted(vtx_off, j_vtx, side="right") - 1
    # volumes of each vesicle (a volume belongs to its vesicle pair) and rows of each volume
    vols_of = {}
    for j in range(n_vol):
        a, b = int(pair_ab[vol_pair[j]][0]), int(pair_ab[vol_pair[j]][1])
        for i in {a, b}:
            vols_of.setdefault(i, []).append(j)
    rows_of = {}
    for r in range(len(j_vol)):
        rows_of.setdefault(int(j_vol[r]), []).append(r)
    for i in range(n_ves):
        vols = vols_of.get(i, [])
        if not vols:
            continue
        a = int(act_off[i + 1] - act_off[i])
        Mi = np.asarray(M[m_off[i]:m_off[i + 1]], dtype=np.float64).reshape(3 * a, 3 * a)
        loc = {int(v): q for q, v in enumerate(act_vtx[act_off[i]:act_off[i + 1]])}
        g = {}
        for j in vols:
            gj = np.zeros(3 * a)
            for r in rows_of.get(j, []):
                if ves_of_row[r] == i:
                    q = loc[int(j_vtx[r])]
                    gj[3 * q:3 * q + 3] += j_g[r]
            g[j] = gj
        for j in vols:
            for k in vols:
                B[j, k] += g[j] @ Mi @ g[k]
                S[j, k] = True
    return B, S
