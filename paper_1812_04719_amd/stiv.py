"""Python binding of libstiv (ctypes).  Argument marshalling only.

Every step of the contact path runs in the library's HIP kernels; PyTorch
supplies device memory and the current stream.  The names follow the C ABI in
include/stiv.h.  If the library is not built this module raises on first use
-- there is no fallback path.
"""
from __future__ import annotations

import ctypes as C
import os
import threading

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libstiv.so")

STIV_OK, STIV_E_ARG, STIV_E_CAPACITY, STIV_E_HIP, STIV_E_NUMERIC, STIV_E_STATE = 0, -1, -2, -3, -4, -5
STIV_EMIT_CANDIDATES, STIV_LEARNED_BRACKET = 1, 2
STIV_OPT_PATCH_TRI, STIV_OPT_PRIM_BLOCKS, STIV_OPT_NARROW_BLOCKS, STIV_OPT_QUEUE_CAPACITY = 1, 2, 3, 4
_STATUS = {0: "STIV_OK", -1: "STIV_E_ARG", -2: "STIV_E_CAPACITY", -3: "STIV_E_HIP", -4: "STIV_E_NUMERIC",
           -5: "STIV_E_STATE"}

EXPORTS = ("stiv_create", "stiv_destroy", "stiv_set_topology", "stiv_reserve", "stiv_detect",
           "stiv_get_stage_times", "stiv_get_stats", "stiv_set_patch_size", "stiv_backward", "stiv_backward_static",
           "stiv_detect_async",
           "stiv_collect", "stiv_set_option", "stiv_sort_pairs_u64", "stiv_mlp_nparam", "stiv_set_toi_model",
           "stiv_mlp_forward", "stiv_mlp_grad", "stiv_mlp_adam", "stiv_lcp_layout", "stiv_form_lcp",
           "stiv_last_error")
STAT_NAMES = ("check_points", "vesicle_pairs", "work_items", "pre_candidates", "candidates_vt", "candidates_ee",
              "root_searches", "contacts", "box_tests", "bracket_certified")


class StivError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__("%s: %s" % (_STATUS.get(status, status), msg))
        self.status = status


class stiv_topology(C.Structure):
    _fields_ = [("n_topo", C.c_int32), ("nv", C.c_void_p), ("tri", C.c_void_p), ("tri_off", C.c_void_p),
                ("edge", C.c_void_p), ("edge_off", C.c_void_p)]


class stiv_scene(C.Structure):
    _fields_ = [("n_ves", C.c_int32), ("n_vtx", C.c_int32), ("n_scenes", C.c_int32),
                ("vtx_off", C.c_void_p), ("topo_id", C.c_void_p), ("scene_off", C.c_void_p),
                ("box_len", C.c_void_p), ("x0", C.c_void_p), ("x1", C.c_void_p)]


class stiv_params(C.Structure):
    _fields_ = [("d", C.c_double), ("eps", C.c_double), ("dt", C.c_double), ("flags", C.c_uint32)]


class stiv_result(C.Structure):
    _fields_ = [("cap_pairs", C.c_int64), ("n_pairs", C.c_int64), ("pair_ab", C.c_void_p),
                ("pair_shift", C.c_void_p),
                ("cap_cand", C.c_int64), ("n_cand_vt", C.c_int64), ("n_cand_ee", C.c_int64), ("cand", C.c_void_p),
                ("cap_ct", C.c_int64), ("n_ct_vt", C.c_int64), ("n_ct_ee", C.c_int64), ("ct_key", C.c_void_p),
                ("ct_tau", C.c_void_p), ("ct_vol", C.c_void_p), ("ct_grad", C.c_void_p),
                ("cap_vol", C.c_int64), ("n_vol", C.c_int64), ("vol_pair", C.c_void_p), ("vol_V", C.c_void_p),
                ("cap_jrow", C.c_int64), ("n_jrow", C.c_int64), ("j_vol", C.c_void_p), ("j_vtx", C.c_void_p),
                ("j_g", C.c_void_p),
                ("n_initially_within_d", C.c_int64), ("n_degenerate_skipped", C.c_int64),
                ("ct_s", C.c_void_p), ("n_search_exhausted", C.c_int64)]


_lock = threading.Lock()
_lib = None


def lib():
    """Load libstiv.so (raises if it has not been built)."""
    global _lib
    with _lock:
        if _lib is None:
            if not os.path.exists(LIB_PATH):
                raise ImportError("libstiv.so is not built; run paper_1812_04719_amd/build.py "
                                  "(or __graft_entry__.build())")
            L = C.CDLL(LIB_PATH)
            L.stiv_create.argtypes = [C.POINTER(C.c_void_p), C.c_int]
            L.stiv_destroy.argtypes = [C.c_void_p]
            L.stiv_set_topology.argtypes = [C.c_void_p, C.POINTER(stiv_topology)]
            L.stiv_reserve.argtypes = [C.c_void_p, C.POINTER(stiv_scene), C.POINTER(stiv_params)]
            L.stiv_detect.argtypes = [C.c_void_p, C.POINTER(stiv_scene), C.POINTER(stiv_params),
                                      C.POINTER(stiv_result), C.c_void_p]
            L.stiv_get_stage_times.argtypes = [C.c_void_p, C.POINTER(C.c_float), C.c_int]
            L.stiv_get_stats.argtypes = [C.c_void_p, C.POINTER(C.c_int64), C.c_int]
            L.stiv_set_patch_size.argtypes = [C.c_void_p, C.c_int]
            L.stiv_set_option.argtypes = [C.c_void_p, C.c_int, C.c_int64]
            L.stiv_detect_async.argtypes = [C.c_void_p, C.POINTER(stiv_scene), C.POINTER(stiv_params),
                                            C.POINTER(stiv_result), C.c_void_p]
            L.stiv_collect.argtypes = [C.c_void_p, C.POINTER(stiv_params), C.POINTER(stiv_result), C.c_void_p]
            L.stiv_backward.argtypes = [C.c_void_p, C.POINTER(stiv_scene), C.POINTER(stiv_params),
                                        C.POINTER(stiv_result), C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p,
                                        C.c_void_p]
            L.stiv_backward_static.argtypes = [C.c_void_p, C.POINTER(stiv_scene), C.POINTER(stiv_params),
                                        C.POINTER(stiv_result), C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p,
                                        C.c_void_p]
            L.stiv_sort_pairs_u64.argtypes = [C.c_void_p, C.c_void_p, C.c_void_p, C.c_int64, C.c_void_p]
            L.stiv_mlp_nparam.argtypes = []
            L.stiv_set_toi_model.argtypes = [C.c_void_p, C.c_void_p, C.c_int, C.c_float]
            L.stiv_mlp_forward.argtypes = [C.c_void_p, C.c_void_p, C.c_void_p, C.c_int64, C.c_void_p, C.c_void_p]
            L.stiv_mlp_grad.argtypes = [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_int64, C.c_void_p,
                                        C.c_void_p, C.c_void_p]
            L.stiv_mlp_adam.argtypes = [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_int64,
                                        C.c_float, C.c_float, C.c_float, C.c_float, C.c_void_p]
            L.stiv_lcp_layout.argtypes = [C.c_void_p, C.POINTER(stiv_scene), C.POINTER(stiv_result), C.c_void_p,
                                          C.c_void_p, C.c_void_p, C.c_int64, C.POINTER(C.c_int64),
                                          C.POINTER(C.c_int64), C.c_void_p]
            L.stiv_form_lcp.argtypes = [C.c_void_p, C.POINTER(stiv_scene), C.POINTER(stiv_result), C.c_void_p,
                                        C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p,
                                        C.c_int64, C.POINTER(C.c_int64), C.c_void_p]
            L.stiv_last_error.argtypes = [C.c_void_p]
            L.stiv_last_error.restype = C.c_char_p
            for n in EXPORTS:
                if n != "stiv_last_error":
                    getattr(L, n).restype = C.c_int
            _lib = L
    return _lib


def _torch():
    import torch
    return torch


def _ptr(t):
    return C.c_void_p(t.data_ptr()) if t is not None and t.numel() > 0 else C.c_void_p(0 if t is None else t.data_ptr())


class Context:
    """One library context on one HIP device (owns the scratch arena)."""

    def __init__(self, device=0):
        self._h = C.c_void_p()
        st = lib().stiv_create(C.byref(self._h), int(device))
        if st != STIV_OK:
            raise StivError(st, "stiv_create failed on device %d" % device)
        self.device = device
        self._topo_key = None

    def close(self):
        if self._h:
            lib().stiv_destroy(self._h)
            self._h = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _check(self, st):
        if st != STIV_OK:
            raise StivError(st, lib().stiv_last_error(self._h).decode())

    def set_topology(self, topos):
        key = tuple((t.nv, t.nt, t.ne, id(t)) for t in topos)
        if key == self._topo_key:
            return
        nv = np.array([t.nv for t in topos], dtype=np.int32)
        tri = np.ascontiguousarray(np.concatenate([t.tri for t in topos]), dtype=np.int32)
        tri_off = np.concatenate([[0], np.cumsum([t.nt for t in topos])]).astype(np.int32)
        edge = np.ascontiguousarray(np.concatenate([t.edge for t in topos]), dtype=np.int32)
        edge_off = np.concatenate([[0], np.cumsum([t.ne for t in topos])]).astype(np.int32)
        tp = stiv_topology(len(topos), nv.ctypes.data, tri.ctypes.data, tri_off.ctypes.data, edge.ctypes.data,
                           edge_off.ctypes.data)
        self._check(lib().stiv_set_topology(self._h, C.byref(tp)))
        self._topo_key = key

    def set_patch_size(self, tri_per_patch):
        self._check(lib().stiv_set_patch_size(self._h, int(tri_per_patch)))
        self._topo_key = None

    def set_option(self, option, value):
        self._check(lib().stiv_set_option(self._h, int(option), int(value)))
        if option == STIV_OPT_PATCH_TRI:
            self._topo_key = None

    def stage_times(self):
        ms = (C.c_float * 7)()
        self._check(lib().stiv_get_stage_times(self._h, ms, 7))
        return list(ms)

    def stats(self):
        v = (C.c_int64 * len(STAT_NAMES))()
        self._check(lib().stiv_get_stats(self._h, v, len(STAT_NAMES)))
        return dict(zip(STAT_NAMES, list(v)))

    # -- learned contact-time bracket ------------------------------------
    def set_toi_model(self, params, kwidth=3.0):
        """Install the bracket model (host FP32 array of stiv_mlp_nparam()
        values), or remove it with params=None."""
        if params is None:
            self._check(lib().stiv_set_toi_model(self._h, None, 0, 1.0))
            return
        p = np.ascontiguousarray(params, dtype=np.float32).ravel()
        self._check(lib().stiv_set_toi_model(self._h, C.c_void_p(p.ctypes.data), int(p.size), float(kwidth)))

    def mlp_forward(self, params, x, out=None):
        """Raw model outputs [n,2] for features x [n,18] (float32 device tensors)."""
        torch = _torch()
        n = x.shape[0]
        if out is None:
            out = torch.empty((n, 2), dtype=torch.float32, device=x.device)
        st = torch.cuda.current_stream(x.device).cuda_stream
        self._check(lib().stiv_mlp_forward(self._h, _ptr(params), _ptr(x), int(n), _ptr(out), C.c_void_p(st)))
        return out

    def mlp_grad(self, params, x, target, grad=None, loss=None):
        """Gradient of the mean bracket loss (device tensors); returns (grad, loss)."""
        torch = _torch()
        n = x.shape[0]
        if grad is None:
            grad = torch.empty_like(params)
        if loss is None:
            loss = torch.empty(1, dtype=torch.float32, device=x.device)
        st = torch.cuda.current_stream(x.device).cuda_stream
        self._check(lib().stiv_mlp_grad(self._h, _ptr(params), _ptr(x), _ptr(target), int(n), _ptr(grad),
                                        _ptr(loss), C.c_void_p(st)))
        return grad, loss

    def mlp_adam(self, params, grad, m, v, step, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8):
        torch = _torch()
        st = torch.cuda.current_stream(params.device).cuda_stream
        self._check(lib().stiv_mlp_adam(self._h, _ptr(params), _ptr(grad), _ptr(m), _ptr(v), int(step), float(lr),
                                        float(beta1), float(beta2), float(eps), C.c_void_p(st)))

    def sort_pairs_u64(self, keys, vals):
        """Stable sort of device uint64 keys (as int64 tensor bits) with uint32 values (as int32)."""
        torch = _torch()
        st = torch.cuda.current_stream(keys.device).cuda_stream
        self._check(lib().stiv_sort_pairs_u64(self._h, _ptr(keys), _ptr(vals), keys.numel(), C.c_void_p(st)))


class DeviceScene:
    """A scene uploaded to device memory (torch tensors) + its ABI struct."""

    def __init__(self, scene, device="cuda:0"):
        torch = _torch()
        self.scene = scene
        dev = torch.device(device)
        self.x0 = torch.from_numpy(np.ascontiguousarray(scene.x0, dtype=np.float64)).to(dev)
        self.x1 = torch.from_numpy(np.ascontiguousarray(scene.x1, dtype=np.float64)).to(dev)
        self.vtx_off = torch.from_numpy(np.ascontiguousarray(scene.vtx_off, dtype=np.int32)).to(dev)
        self.topo_id = torch.from_numpy(np.ascontiguousarray(scene.topo_id, dtype=np.int32)).to(dev)
        self.scene_off = torch.from_numpy(np.ascontiguousarray(scene.scene_off, dtype=np.int32)).to(dev)
        self.box_len = torch.from_numpy(np.ascontiguousarray(scene.box_len, dtype=np.float64)).to(dev)
        self.n_ves, self.n_vtx, self.n_scenes = scene.n_ves, scene.n_vtx, scene.n_scenes

    def struct(self):
        return stiv_scene(self.n_ves, self.n_vtx, self.n_scenes, self.vtx_off.data_ptr(), self.topo_id.data_ptr(),
                          self.scene_off.data_ptr(), self.box_len.data_ptr(), self.x0.data_ptr(),
                          self.x1.data_ptr())


class Outputs:
    """Caller-owned device output arrays with capacities."""

    def __init__(self, device, cap_pairs=1 << 14, cap_ct=1 << 16, cap_vol=1 << 12, cap_jrow=1 << 16, cap_cand=0):
        torch = _torch()
        self.device = device
        self.alloc(cap_pairs, cap_ct, cap_vol, cap_jrow, cap_cand)

    def alloc(self, cap_pairs, cap_ct, cap_vol, cap_jrow, cap_cand):
        torch = _torch()
        d = self.device
        self.cap = dict(pairs=cap_pairs, ct=cap_ct, vol=cap_vol, jrow=cap_jrow, cand=cap_cand)
        i32, f64 = torch.int32, torch.float64
        self.pair_ab = torch.empty((cap_pairs, 2), dtype=i32, device=d)
        self.pair_shift = torch.empty((cap_pairs, 3), dtype=i32, device=d)
        self.cand = torch.empty((max(cap_cand, 1), 4), dtype=i32, device=d)
        self.ct_key = torch.empty((cap_ct, 4), dtype=i32, device=d)
        self.ct_tau = torch.empty(cap_ct, dtype=f64, device=d)
        self.ct_s = torch.empty(cap_ct, dtype=f64, device=d)
        self.ct_vol = torch.empty(cap_ct, dtype=f64, device=d)
        self.ct_grad = torch.empty((cap_ct, 12), dtype=f64, device=d)
        self.vol_pair = torch.empty(cap_vol, dtype=i32, device=d)
        self.vol_V = torch.empty(cap_vol, dtype=f64, device=d)
        self.j_vol = torch.empty(cap_jrow, dtype=i32, device=d)
        self.j_vtx = torch.empty(cap_jrow, dtype=i32, device=d)
        self.j_g = torch.empty((cap_jrow, 3), dtype=f64, device=d)

    def struct(self):
        c = self.cap
        r = stiv_result()
        r.cap_pairs, r.pair_ab, r.pair_shift = c["pairs"], self.pair_ab.data_ptr(), self.pair_shift.data_ptr()
        r.cap_cand, r.cand = c["cand"], self.cand.data_ptr()
        r.cap_ct, r.ct_key = c["ct"], self.ct_key.data_ptr()
        r.ct_tau, r.ct_vol, r.ct_grad = self.ct_tau.data_ptr(), self.ct_vol.data_ptr(), self.ct_grad.data_ptr()
        r.ct_s = self.ct_s.data_ptr()
        r.cap_vol, r.vol_pair, r.vol_V = c["vol"], self.vol_pair.data_ptr(), self.vol_V.data_ptr()
        r.cap_jrow, r.j_vol, r.j_vtx, r.j_g = c["jrow"], self.j_vol.data_ptr(), self.j_vtx.data_ptr(), \
            self.j_g.data_ptr()
        return r


class DetectResult(dict):
    __getattr__ = dict.__getitem__


def mlp_nparam():
    return int(lib().stiv_mlp_nparam())


def detect(ctx: Context, dscene: DeviceScene, d, eps, dt, outputs: Outputs = None, emit_candidates=False,
           stream=None, to_numpy=True, learned_bracket=False):
    """Run stiv_detect; grows the output arrays and retries on STIV_E_CAPACITY."""
    torch = _torch()
    ctx.set_topology(dscene.scene.topos)
    if outputs is None:
        outputs = Outputs(dscene.x0.device, cap_cand=(1 << 20) if emit_candidates else 0)
    flags = (STIV_EMIT_CANDIDATES if emit_candidates else 0) | (STIV_LEARNED_BRACKET if learned_bracket else 0)
    p = stiv_params(float(d), float(eps), float(dt), flags)
    s = dscene.struct()
    st_ptr = stream if stream is not None else torch.cuda.current_stream(dscene.x0.device).cuda_stream
    for _ in range(3):
        r = outputs.struct()
        st = lib().stiv_detect(ctx._h, C.byref(s), C.byref(p), C.byref(r), C.c_void_p(st_ptr))
        if st == STIV_E_CAPACITY:
            nct = r.n_ct_vt + r.n_ct_ee
            outputs.alloc(max(r.n_pairs, 1) * 2, max(nct, 1) * 2, max(r.n_vol, 1) * 2, max(r.n_jrow, 1) * 2,
                          (r.n_cand_vt + r.n_cand_ee) * 2 if emit_candidates else 0)
            continue
        ctx._check(st)
        break
    else:
        raise StivError(STIV_E_CAPACITY, "outputs did not fit after growing")
    res = _collect(r, outputs, emit_candidates, to_numpy)
    res["_struct"] = r
    return res, outputs


class AsyncDetect:
    """Graph-capturable detect: enqueue() only launches kernels (capture it in
    a torch.cuda.CUDAGraph / hipGraph and replay), collect() synchronises and
    reads the counts.  Needs one synchronous detect on the same scene first."""

    def __init__(self, ctx, dscene, d, eps, dt, outputs, learned_bracket=False):
        self.ctx, self.dscene, self.outputs = ctx, dscene, outputs
        self.params = stiv_params(float(d), float(eps), float(dt), STIV_LEARNED_BRACKET if learned_bracket else 0)
        self.scene_struct = dscene.struct()
        self.result = outputs.struct()

    def enqueue(self, stream=None):
        torch = _torch()
        st_ptr = stream if stream is not None else torch.cuda.current_stream(self.dscene.x0.device).cuda_stream
        self.ctx._check(lib().stiv_detect_async(self.ctx._h, C.byref(self.scene_struct), C.byref(self.params),
                                                C.byref(self.result), C.c_void_p(st_ptr)))

    def collect(self, stream=None, to_numpy=True):
        torch = _torch()
        st_ptr = stream if stream is not None else torch.cuda.current_stream(self.dscene.x0.device).cuda_stream
        self.ctx._check(lib().stiv_collect(self.ctx._h, C.byref(self.params), C.byref(self.result),
                                           C.c_void_p(st_ptr)))
        res = _collect(self.result, self.outputs, False, to_numpy)
        res["_struct"] = self.result
        return res


def backward(ctx: Context, dscene: DeviceScene, d, eps, dt, result_struct, dL_dV=None, dL_dG=None, stream=None,
             static_scratch=False, out=None):
    """dL/dX0, dL/dX1 ([3, n_vtx] float64 tensors) for cotangents of V and G.
    static_scratch: call stiv_backward_static (no device allocation in the
    library); out: optional preallocated (dX0, dX1)."""
    torch = _torch()
    dev = dscene.x0.device
    if out is not None:
        dX0, dX1 = out
    else:
        dX0 = torch.empty_like(dscene.x0)
        dX1 = torch.empty_like(dscene.x1)
    p = stiv_params(float(d), float(eps), float(dt), 0)
    s = dscene.struct()
    st_ptr = stream if stream is not None else torch.cuda.current_stream(dev).cuda_stream
    gv = dL_dV.contiguous() if dL_dV is not None else None
    gg = dL_dG.contiguous() if dL_dG is not None else None
    fn = lib().stiv_backward_static if static_scratch else lib().stiv_backward
    st = fn(ctx._h, C.byref(s), C.byref(p), C.byref(result_struct),
            C.c_void_p(gv.data_ptr() if gv is not None else 0), C.c_void_p(gg.data_ptr() if gg is not None else 0),
            C.c_void_p(dX0.data_ptr()), C.c_void_p(dX1.data_ptr()), C.c_void_p(st_ptr))
    ctx._check(st)
    return dX0, dX1


def _collect(r, o, emit, to_numpy):
    nct = r.n_ct_vt + r.n_ct_ee
    out = DetectResult(
        n_pairs=r.n_pairs, n_cand_vt=r.n_cand_vt, n_cand_ee=r.n_cand_ee, n_ct_vt=r.n_ct_vt, n_ct_ee=r.n_ct_ee,
        n_ct=nct, n_vol=r.n_vol, n_jrow=r.n_jrow, n_initially_within_d=r.n_initially_within_d,
        n_degenerate_skipped=r.n_degenerate_skipped, n_search_exhausted=r.n_search_exhausted,
        pair_ab=o.pair_ab[: r.n_pairs], pair_shift=o.pair_shift[: r.n_pairs],
        ct_key=o.ct_key[:nct], ct_tau=o.ct_tau[:nct], ct_s=o.ct_s[:nct], ct_vol=o.ct_vol[:nct], ct_grad=o.ct_grad[:nct],
        vol_pair=o.vol_pair[: r.n_vol], vol_V=o.vol_V[: r.n_vol],
        j_vol=o.j_vol[: r.n_jrow], j_vtx=o.j_vtx[: r.n_jrow], j_g=o.j_g[: r.n_jrow],
    )
    if emit:
        out["cand"] = o.cand[: r.n_cand_vt + r.n_cand_ee]
    if to_numpy:
        for k, v in list(out.items()):
            if hasattr(v, "cpu"):
                out[k] = v.cpu().numpy()
    return out


def lcp_layout(ctx: Context, dscene: DeviceScene, result_struct, stream=None):
    """Active points of every vesicle for the LCP matrix: (act_off, m_off,
    act_vtx) device tensors (layout of the operator blocks in include/stiv.h)."""
    torch = _torch()
    dev = dscene.x0.device
    nv = dscene.n_ves
    act_off = torch.empty(nv + 1, dtype=torch.int64, device=dev)
    m_off = torch.empty(nv + 1, dtype=torch.int64, device=dev)
    cap = max(int(result_struct.n_jrow), 1)
    act_vtx = torch.empty(cap, dtype=torch.int32, device=dev)
    n_act, n_m = C.c_int64(), C.c_int64()
    s = dscene.struct()
    st_ptr = stream if stream is not None else torch.cuda.current_stream(dev).cuda_stream
    ctx._check(lib().stiv_lcp_layout(ctx._h, C.byref(s), C.byref(result_struct), _ptr(act_off), _ptr(m_off),
                                     _ptr(act_vtx), cap, C.byref(n_act), C.byref(n_m), C.c_void_p(st_ptr)))
    return act_off, m_off, act_vtx[: n_act.value]


def form_lcp(ctx: Context, dscene: DeviceScene, result_struct, act_off, m_off, act_vtx, M, cap_b=None,
             stream=None):
    """Sparse B = J M J^T (Alg. 3) as COO device tensors (rows, cols, vals),
    sorted by (row, col); grows the output and retries on STIV_E_CAPACITY."""
    torch = _torch()
    dev = dscene.x0.device
    cap = cap_b or max(4 * int(result_struct.n_vol), 16)
    s = dscene.struct()
    st_ptr = stream if stream is not None else torch.cuda.current_stream(dev).cuda_stream
    Mc = M.contiguous()
    for _ in range(3):
        rows = torch.empty(cap, dtype=torch.int32, device=dev)
        cols = torch.empty(cap, dtype=torch.int32, device=dev)
        vals = torch.empty(cap, dtype=torch.float64, device=dev)
        n_b = C.c_int64()
        st = lib().stiv_form_lcp(ctx._h, C.byref(s), C.byref(result_struct), _ptr(act_off), _ptr(m_off),
                                 _ptr(act_vtx), _ptr(Mc), _ptr(rows), _ptr(cols), _ptr(vals), cap, C.byref(n_b),
                                 C.c_void_p(st_ptr))
        if st == STIV_E_CAPACITY and n_b.value > cap:
            cap = n_b.value
            continue
        ctx._check(st)
        n = n_b.value
        return rows[:n], cols[:n], vals[:n]
    raise StivError(STIV_E_CAPACITY, "LCP output did not fit after growing")
