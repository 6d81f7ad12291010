"""Seeded synthetic scenes: vesicle surface meshes at t_n and t_{n+1}.

This module only *builds inputs*.  It holds none of the contact method's
arithmetic (no boxes, no roots, no volumes); both the FP64 oracle and the GPU
library consume exactly the arrays produced here.

Geometry follows the paper's surface description:

* Each vesicle surface is a map from the unit sphere, sampled on an order-p
  grid: p+1 Gauss-Legendre nodes in the polar angle times 2p uniform azimuths
  (Sec. 3.1.1).  Two pole vertices close the mesh.
* Each grid quad is split along one diagonal into two triangles (Sec. 3.1.2,
  Fig. 3); the pole caps are triangle fans.  Triangles are oriented with
  outward normals (counter-clockwise seen from outside).
* Shapes are prolate spheroids of reduced volume v = 0.91 and equivalent
  radius R0 = 1.34 (Sec. 4.3, the 1440-vesicle Taylor-vortex run), with a
  small smooth spherical-harmonic perturbation of degree <= 16 evaluated
  directly on the order-32 contact grid (the "upsampling" of Sec. 3.1.2 is
  exact for band-limited fields).
* Vertex trajectories are linear in time between x_n and x_{n+1}
  (Sec. 3.1.2, text after Eq. 3.1); x_{n+1} = seeded rigid motion of each
  vesicle plus a fresh smooth perturbation.

Layout handed to the library: positions are SoA float64 ``[3][n_vtx]``;
vesicle ``v`` owns vertices ``vtx_off[v]:vtx_off[v+1]`` and uses mesh
topology ``topo_id[v]``; scenes own vesicle ranges ``scene_off``; each scene
has a periodic box ``box_len[s]`` (0 on an axis means free space).
"""
from __future__ import annotations

import dataclasses
import functools
import hashlib
import json
import math
from typing import List, Optional

import numpy as np
import scipy.special as _sps
from scipy.optimize import brentq
from scipy.spatial import cKDTree
from scipy.spatial.transform import Rotation

# Separation parameters: d_m = 0.009 (Sec. 4.1, 4.5); mesh separation
# (1 + 2 alpha) d_m with alpha = 0.05 (Sec. 3.1.2).
D_M = 0.009
ALPHA = 0.05
D_MESH = (1.0 + 2.0 * ALPHA) * D_M
EPS_DEFAULT = 1.0
DT_DEFAULT = 0.1          # time step of the Taylor-vortex run (Sec. 4.3)
R0_PAPER = 1.34           # equivalent radius (Sec. 4.3)
REDUCED_VOLUME = 0.91


# ---------------------------------------------------------------------------
# Mesh topology of an order-p grid
# ---------------------------------------------------------------------------
@dataclasses.dataclass
class Topology:
    order: int
    nv: int
    tri: np.ndarray    # int32 [nt, 3] local vertex ids, outward CCW
    edge: np.ndarray   # int32 [ne, 2] local ids, lo < hi, sorted lexicographically

    @property
    def nt(self):
        return int(self.tri.shape[0])

    @property
    def ne(self):
        return int(self.edge.shape[0])


_TOPO_CACHE = {}


def grid_topology(p: int) -> Topology:
    """Triangle mesh of the order-p grid.

    Vertex ``i*2p + j`` is polar node i (0 = nearest the north pole) and
    azimuth j; vertex ``(p+1)*2p`` is the north pole and ``+1`` the south
    pole.  Quad (i,j),(i,j+1),(i+1,j+1),(i+1,j) is split on the diagonal
    (i,j)-(i+1,j+1).
    """
    if p in _TOPO_CACHE:
        return _TOPO_CACHE[p]
    nphi = 2 * p
    nv = (p + 1) * nphi + 2
    north, south = (p + 1) * nphi, (p + 1) * nphi + 1
    tris = []
    for i in range(p):
        for j in range(nphi):
            jn = (j + 1) % nphi
            a, b = i * nphi + j, i * nphi + jn
            c, d = (i + 1) * nphi + jn, (i + 1) * nphi + j
            tris.append((a, d, c))     # first edge points south, second south-east
            tris.append((a, c, b))     # first edge south-east, second east
    for j in range(nphi):
        jn = (j + 1) % nphi
        tris.append((north, j, jn))
        tris.append((south, p * nphi + jn, p * nphi + j))
    tri = np.asarray(tris, dtype=np.int32)
    e = np.concatenate([tri[:, [0, 1]], tri[:, [1, 2]], tri[:, [2, 0]]])
    e = np.sort(e, axis=1)
    e = np.unique(e, axis=0).astype(np.int32)
    topo = Topology(order=p, nv=nv, tri=tri, edge=e)
    assert nv - e.shape[0] + tri.shape[0] == 2          # sphere: V - E + F = 2
    _TOPO_CACHE[p] = topo
    return topo


@functools.lru_cache(maxsize=None)
def grid_angles(p: int):
    """(theta, phi) of every vertex of the order-p grid (poles last)."""
    x, _ = np.polynomial.legendre.leggauss(p + 1)
    theta_rows = np.arccos(x[::-1])                   # north -> south
    phi_cols = 2.0 * np.pi * np.arange(2 * p) / (2 * p)
    th = np.repeat(theta_rows, 2 * p)
    ph = np.tile(phi_cols, p + 1)
    th = np.concatenate([th, [0.0, np.pi]])
    ph = np.concatenate([ph, [0.0, 0.0]])
    return th, ph


_SH_CACHE = {}


def real_sh_basis(p: int, lmax: int) -> np.ndarray:
    """Orthonormal real spherical harmonics up to degree lmax on the order-p grid.

    Returns [nv, (lmax+1)^2]; column l*l + l + m holds Y_lm (m in -l..l).
    """
    key = (p, lmax)
    if key in _SH_CACHE:
        return _SH_CACHE[key]
    th, ph = grid_angles(p)
    cols = np.zeros((th.size, (lmax + 1) ** 2))
    for l in range(lmax + 1):
        for m in range(0, l + 1):
            y = _sps.sph_harm_y(l, m, th, ph)
            if m == 0:
                cols[:, l * l + l] = y.real
            else:
                s = math.sqrt(2.0) * (-1.0) ** m
                cols[:, l * l + l + m] = s * y.real
                cols[:, l * l + l - m] = s * y.imag
    _SH_CACHE[key] = cols
    return cols


def sh_perturbation_coeffs(rng, lmax: int, sigma: float, n: int) -> np.ndarray:
    """[n, (lmax+1)^2, 3] coefficients ~ N(0, sigma^2) / (l+1)^2."""
    ls = np.concatenate([[l] * (2 * l + 1) for l in range(lmax + 1)])
    c = rng.standard_normal((n, ls.size, 3)) * sigma
    return c / ((ls + 1.0) ** 2)[None, :, None]


# ---------------------------------------------------------------------------
# Shapes
# ---------------------------------------------------------------------------
def spheroid_axes(reduced_volume=REDUCED_VOLUME, r0=R0_PAPER):
    """Semi-axes (a, b) of the prolate spheroid with given reduced volume.

    Reduced volume = V / (4/3 pi R0^3) with R0 = sqrt(A / 4 pi).
    """
    if reduced_volume >= 1.0:
        return r0, r0

    def v_of(ar):
        a, b = ar, 1.0
        e = math.sqrt(1.0 - b * b / (a * a))
        area = 2.0 * math.pi * b * b * (1.0 + a / (b * e) * math.asin(e))
        vol = 4.0 / 3.0 * math.pi * a * b * b
        req = math.sqrt(area / (4.0 * math.pi))
        return vol / (4.0 / 3.0 * math.pi * req ** 3), req

    ar = brentq(lambda x: v_of(x)[0] - reduced_volume, 1.0 + 1e-9, 20.0, xtol=1e-15)
    req = v_of(ar)[1]
    b = r0 / req
    return ar * b, b


@functools.lru_cache(maxsize=None)
def spheroid_body_points(p: int, a: float, b: float) -> np.ndarray:
    """[nv, 3] body-frame points of the spheroid with semi-axes (b, b, a)."""
    th, ph = grid_angles(p)
    st = np.sin(th)
    return np.stack([b * st * np.cos(ph), b * st * np.sin(ph), a * np.cos(th)], axis=1)


# ---------------------------------------------------------------------------
# Ellipsoid overlap (Perram-Wertheim contact function), used for packing only
# ---------------------------------------------------------------------------
_LAM = np.linspace(0.0, 1.0, 65)[1:-1]


def _pw_max(r, Ainv, Binv):
    """max over lambda of lambda(1-lambda) r^T [(1-l)A^-1 + l B^-1]^-1 r.

    r: [k,3]; Ainv: [3,3] or [k,3,3]; Binv: [k,3,3].  The max over a grid is
    below the true max, so "overlap" (value < 1) is reported conservatively.
    The 3x3 systems are solved in closed form (adjugate / determinant).
    """
    lam = _LAM[None, :, None, None]
    A = np.broadcast_to(Ainv, Binv.shape)[:, None]
    C = (1.0 - lam) * A + lam * Binv[:, None]
    a, b, c = C[..., 0, 0], C[..., 0, 1], C[..., 0, 2]
    d, e, f = C[..., 1, 1], C[..., 1, 2], C[..., 2, 2]
    # adjugate of the symmetric matrix [[a b c] [b d e] [c e f]]
    A00, A01, A02 = d * f - e * e, c * e - b * f, b * e - c * d
    A11, A12, A22 = a * f - c * c, b * c - a * e, a * d - b * b
    det = a * A00 + b * A01 + c * A02
    x, y, z = r[:, None, 0], r[:, None, 1], r[:, None, 2]
    quad = (A00 * x * x + A11 * y * y + A22 * z * z + 2.0 * (A01 * x * y + A02 * x * z + A12 * y * z)) / det
    f_l = _LAM[None, :] * (1.0 - _LAM[None, :]) * quad
    return f_l.max(axis=1)


def _shape_inv(R, a, b, inflate):
    # ellipsoid interior: x^T (R diag(ax^2) R^T)^-1 x <= 1
    ax = np.array([b + inflate, b + inflate, a + inflate])
    return R @ np.diag(ax * ax) @ R.T


# ---------------------------------------------------------------------------
# Scene container
# ---------------------------------------------------------------------------
@dataclasses.dataclass
class Scene:
    x0: np.ndarray            # float64 [3, n_vtx]
    x1: np.ndarray            # float64 [3, n_vtx]
    vtx_off: np.ndarray       # int32 [N+1]
    topo_id: np.ndarray       # int32 [N]
    scene_off: np.ndarray     # int32 [S+1]
    box_len: np.ndarray       # float64 [S, 3]
    topos: List[Topology]
    d: float = D_MESH
    eps: float = EPS_DEFAULT
    dt: float = DT_DEFAULT
    meta: dict = dataclasses.field(default_factory=dict)

    @property
    def n_ves(self):
        return int(self.vtx_off.size - 1)

    @property
    def n_vtx(self):
        return int(self.x0.shape[1])

    @property
    def n_scenes(self):
        return int(self.scene_off.size - 1)

    def n_tri(self):
        return int(sum(self.topos[t].nt for t in self.topo_id))

    def sha256(self):
        h = hashlib.sha256()
        for arr in (self.x0, self.x1, self.vtx_off, self.topo_id, self.scene_off, self.box_len):
            h.update(np.ascontiguousarray(arr).tobytes())
        h.update(json.dumps([self.d, self.eps, self.dt]).encode())
        return h.hexdigest()

    def with_params(self, **kw):
        return dataclasses.replace(self, **kw)


def _assemble(shapes0, shapes1, orders, box_len, d=D_MESH, eps=EPS_DEFAULT, dt=DT_DEFAULT, meta=None):
    order_list = sorted(set(orders))
    topos = [grid_topology(p) for p in order_list]
    tid = np.array([order_list.index(p) for p in orders], dtype=np.int32)
    counts = np.array([s.shape[0] for s in shapes0], dtype=np.int64)
    off = np.zeros(len(shapes0) + 1, dtype=np.int32)
    off[1:] = np.cumsum(counts)
    x0 = np.ascontiguousarray(np.concatenate(shapes0, axis=0).T)
    x1 = np.ascontiguousarray(np.concatenate(shapes1, axis=0).T)
    return Scene(x0=x0, x1=x1, vtx_off=off, topo_id=tid,
                 scene_off=np.array([0, len(shapes0)], dtype=np.int32),
                 box_len=np.asarray(box_len, dtype=np.float64).reshape(1, 3),
                 topos=topos, d=d, eps=eps, dt=dt, meta=dict(meta or {}))


def concat_scenes(scenes: List[Scene]) -> Scene:
    """Batch independent scenes into one multi-scene input (pairs stay inside a scene)."""
    orders = sorted({t.order for s in scenes for t in s.topos})
    topos = [grid_topology(p) for p in orders]
    x0, x1, tid, counts, soff, blen = [], [], [], [], [0], []
    for s in scenes:
        x0.append(s.x0)
        x1.append(s.x1)
        tid.append(np.array([orders.index(s.topos[t].order) for t in s.topo_id], dtype=np.int32))
        counts.append(np.diff(s.vtx_off))
        soff.append(soff[-1] + s.n_ves)
        blen.append(s.box_len)
    counts = np.concatenate(counts)
    off = np.zeros(counts.size + 1, dtype=np.int32)
    off[1:] = np.cumsum(counts)
    p0 = scenes[0]
    return Scene(x0=np.ascontiguousarray(np.concatenate(x0, axis=1)),
                 x1=np.ascontiguousarray(np.concatenate(x1, axis=1)),
                 vtx_off=off, topo_id=np.concatenate(tid), scene_off=np.array(soff, dtype=np.int32),
                 box_len=np.concatenate(blen, axis=0), topos=topos, d=p0.d, eps=p0.eps, dt=p0.dt,
                 meta={"scenes": [s.meta for s in scenes]})


# ---------------------------------------------------------------------------
# Motion
# ---------------------------------------------------------------------------
def _rigid_motion(rng, pts, center, max_disp):
    """Rotation about `center` plus translation; every point moves <= max_disp."""
    t_dir = rng.standard_normal(3)
    t_dir /= np.linalg.norm(t_dir)
    t = t_dir * max_disp * (0.5 + 0.4 * rng.random())
    axis = rng.standard_normal(3)
    axis /= np.linalg.norm(axis)
    rmax = np.max(np.linalg.norm(pts - center, axis=1))
    ang = rng.random() * 0.1 * max_disp / max(rmax, 1e-30)
    # chord length of a rotation by ang at radius r is 2 r sin(ang/2) <= r ang
    Rm = Rotation.from_rotvec(axis * ang).as_matrix()
    return (pts - center) @ Rm.T + center + t


# ---------------------------------------------------------------------------
# Configurations
# ---------------------------------------------------------------------------
def make_two_spheres(seed=1, p=32, gap=0.02, step=0.05, sigma=1e-3, perturb=True,
                     lmax=32, d=D_MESH, eps=EPS_DEFAULT, dt=DT_DEFAULT):
    """Two unit spheres on the x axis, each moving `step` toward the other.

    x_{n+1} = x_n + rigid translation + seeded smooth perturbation with
    SH coefficients ~ N(0, sigma^2)/(l+1)^2, l <= lmax.
    """
    rng = np.random.default_rng(np.random.SeedSequence(seed))
    unit = spheroid_body_points(p, 1.0, 1.0)
    c = 1.0 + gap / 2.0
    # Each sphere's grid gets its own seeded orientation: the smooth surfaces
    # are still exact unit spheres, but the two meshes are no longer
    # translates of each other (which would make every edge of one parallel
    # to an edge of the other, a degenerate input for edge-edge tests).
    rots = Rotation.random(2, random_state=rng).as_matrix()
    s0 = [unit @ rots[0].T + np.array([-c, 0, 0]), unit @ rots[1].T + np.array([c, 0, 0])]
    s1 = [s0[0] + np.array([step, 0, 0]), s0[1] - np.array([step, 0, 0])]
    if perturb:
        Y = real_sh_basis(p, lmax)
        coef = sh_perturbation_coeffs(rng, lmax, sigma, 2)
        s1 = [s1[k] + Y @ coef[k] for k in range(2)]
    return _assemble(s0, s1, [p, p], [0.0, 0.0, 0.0], d=d, eps=eps, dt=dt,
                     meta={"config": "two_spheres", "seed": seed, "p": p, "gap": gap, "step": step,
                           "sigma": sigma, "perturb": perturb})


def _place_rsa(rng, n, a, b, L, g_min, max_tries=200000):
    """Random sequential addition of n spheroids in a periodic cube of side L."""
    infl = 0.5 * g_min * (a / b)     # axis inflation that contains the g_min/2 offset body
    centers, rots, invs = [], [], []
    tries = 0
    while len(centers) < n:
        tries += 1
        if tries > max_tries:
            raise RuntimeError("RSA did not reach the requested packing")
        c = rng.random(3) * L
        R = Rotation.random(random_state=rng).as_matrix()
        Ai = _shape_inv(R, a, b, infl)
        if centers:
            C = np.asarray(centers)
            r = C - c
            r -= L * np.round(r / L)
            near = np.linalg.norm(r, axis=1) < 2.0 * (a + infl) + 1e-9
            if near.any():
                if (_pw_max(r[near], Ai, np.asarray(invs)[near]) < 1.0).any():
                    continue
        centers.append(c)
        rots.append(R)
        invs.append(Ai)
    return np.asarray(centers), np.asarray(rots)


def make_rsa_scene(seed=2, n=64, vf=0.30, p=32, lmax=16, sigma=1e-3, max_disp=0.1,
                   g_min=0.03, d=D_MESH, eps=EPS_DEFAULT, dt=DT_DEFAULT, reduced_volume=REDUCED_VOLUME):
    """n spheroids at volume fraction vf in a periodic cube (random sequential addition)."""
    rng = np.random.default_rng(np.random.SeedSequence(seed))
    a, b = spheroid_axes(reduced_volume)
    vol = 4.0 / 3.0 * math.pi * a * b * b
    L = (n * vol / vf) ** (1.0 / 3.0)
    centers, rots = _place_rsa(rng, n, a, b, L, g_min)
    s0, s1 = _shapes_with_motion(rng, centers, rots, a, b, p, lmax, sigma, max_disp)
    return _assemble(s0, s1, [p] * n, [L, L, L], d=d, eps=eps, dt=dt,
                     meta={"config": "rsa", "seed": seed, "n": n, "vf": vf, "L": L, "p": p,
                           "lmax": lmax, "max_disp": max_disp})


def _shapes_with_motion(rng, centers, rots, a, b, p, lmax, sigma, max_disp, orders=None):
    n = len(centers)
    orders = [p] * n if orders is None else orders
    s0, s1 = [], []
    streams = rng.spawn(n)
    for k in range(n):
        r = streams[k]
        q = orders[k]
        Y = real_sh_basis(q, lmax)
        body = spheroid_body_points(q, a, b)
        coef = sh_perturbation_coeffs(r, lmax, sigma, 2)
        shape0 = body + Y @ coef[0]
        x0 = shape0 @ rots[k].T + centers[k]
        moved = _rigid_motion(r, x0, centers[k], max_disp * 0.97)
        x1 = moved + (Y @ coef[1]) @ rots[k].T
        s0.append(x0)
        s1.append(x1)
    return s0, s1


def make_fcc_scene(seed=3, cells=(8, 9, 5), box_volume=28.4 ** 3, p=32, lmax=16, sigma=1e-3,
                   max_disp=0.1, theta_max=math.radians(30.0), g_min=0.015, vacancies=0, rattle=0.0,
                   plane_gap=0.015,
                   d=D_MESH, eps=EPS_DEFAULT, dt=DT_DEFAULT, reduced_volume=REDUCED_VOLUME,
                   orders=None):
    """Spheroids on an affinely stretched FCC lattice with seeded rotations.

    The stretch along z equals the spheroid aspect ratio, so unrotated
    spheroids reproduce the contact graph of an FCC sphere packing.  With the
    default 8x9x5 cells (1440 sites) in a box of volume 28.4^3 the volume
    fraction is 57.66 %, the paper's 1440-vesicle configuration (Sec. 4.3).
    """
    rng = np.random.default_rng(np.random.SeedSequence(seed))
    a, b = spheroid_axes(reduced_volume)
    ar = a / b
    nx, ny, nz = cells
    c = (box_volume / (nx * ny * nz * ar)) ** (1.0 / 3.0)
    # Volume-preserving squeeze: scale x and y by f and z by 1/f^2 so the four
    # in-plane neighbours of every site sit `plane_gap` apart (equator to
    # equator) while the other eight move farther away.
    f = 1.0
    if plane_gap is not None:
        f = min(1.0, (2.0 * b + plane_gap) * math.sqrt(2.0) / c)
    cell = np.array([c * f, c * f, c * ar / (f * f)])
    L = cell * np.array([nx, ny, nz])
    basis = np.array([[0, 0, 0], [0.5, 0.5, 0], [0.5, 0, 0.5], [0, 0.5, 0.5]])
    g = np.stack(np.meshgrid(np.arange(nx), np.arange(ny), np.arange(nz), indexing="ij"), -1).reshape(-1, 3)
    sites = ((g[:, None, :] + basis[None]) * cell).reshape(-1, 3) + 0.25 * cell
    if vacancies:
        keep = np.sort(rng.permutation(sites.shape[0])[: sites.shape[0] - vacancies])
        sites = sites[keep]
    n = sites.shape[0]
    infl = 0.5 * g_min * (a / b)
    rots = np.repeat(np.eye(3)[None], n, axis=0)
    invs = np.array([_shape_inv(np.eye(3), a, b, infl) for _ in range(1)] * n)
    tree = cKDTree(sites % L, boxsize=L)
    nbrs = tree.query_ball_point(sites % L, r=2.0 * (a + infl) + 1e-9)
    angles = np.zeros(n)
    for k in rng.permutation(n):
        axis = rng.standard_normal(3)
        axis /= np.linalg.norm(axis)
        ang = rng.random() * theta_max
        nb = [j for j in nbrs[k] if j != k]
        r = sites[nb] - sites[k]
        r -= L * np.round(r / L)
        for _ in range(9):
            R = Rotation.from_rotvec(axis * ang).as_matrix()
            Ai = _shape_inv(R, a, b, infl)
            if not nb or not (_pw_max(r, Ai, invs[nb]) < 1.0).any():
                rots[k], invs[k], angles[k] = R, Ai, ang
                break
            ang *= 0.5
    # Rattle: move each site by up to `rattle` in a random direction while the
    # inflated spheroids stay disjoint.  A snapshot of a dense suspension has
    # many neighbours close to the minimum separation; the perfect lattice
    # has none, so this sets how many pairs the step's motion brings into
    # contact.
    moved = 0
    if rattle > 0.0:
        for k in rng.permutation(n):
            u = rng.standard_normal(3)
            u /= np.linalg.norm(u)
            step = rattle * rng.random()
            nb = [j for j in nbrs[k] if j != k]
            for _ in range(5):
                c_new = sites[k] + step * u
                r = sites[nb] - c_new
                r -= L * np.round(r / L)
                if not nb or not (_pw_max(r, invs[k], invs[nb]) < 1.0).any():
                    sites[k] = c_new
                    moved += 1
                    break
                step *= 0.5
    s0, s1 = _shapes_with_motion(rng, sites, rots, a, b, p, lmax, sigma, max_disp, orders=orders)
    return _assemble(s0, s1, orders or [p] * n, L, d=d, eps=eps, dt=dt,
                     meta={"config": "fcc", "seed": seed, "cells": list(cells), "n": n, "p": p,
                           "box": L.tolist(), "vf": n * 4 / 3 * math.pi * a * b * b / float(np.prod(L)),
                           "max_disp": max_disp, "rot_deg_mean": float(np.degrees(angles).mean()),
                           "rot_unrotated": int((angles == 0).sum()), "rattle": rattle, "plane_gap": plane_gap, "squeeze": f,
                           "rattled": moved})


def make_batch(seed=4, n_scenes=256, n_range=(8, 128), orders=(16, 24, 32), vf_range=(0.10, 0.60),
               max_disp=0.1, d=D_MESH, eps=EPS_DEFAULT, dt=DT_DEFAULT):
    """Many independent scenes of uneven size, order and density."""
    rng = np.random.default_rng(np.random.SeedSequence(seed))
    a, b = spheroid_axes()
    vol = 4.0 / 3.0 * math.pi * a * b * b
    out = []
    for s, sub in enumerate(rng.spawn(n_scenes)):
        n = int(sub.integers(n_range[0], n_range[1] + 1))
        vf = float(sub.uniform(*vf_range))
        ords = [int(orders[i]) for i in sub.integers(0, len(orders), n)]
        sseed = int(sub.integers(0, 2 ** 31))
        if vf <= 0.30:
            L = (n * vol / vf) ** (1.0 / 3.0)
            r2 = np.random.default_rng(sseed)
            centers, rots = _place_rsa(r2, n, a, b, L, 0.03)
            s0, s1 = _shapes_with_motion(r2, centers, rots, a, b, 32, 16, 1e-3, max_disp, orders=ords)
            sc = _assemble(s0, s1, ords, [L, L, L], d=d, eps=eps, dt=dt,
                           meta={"config": "rsa", "n": n, "vf": vf})
        else:
            sc = _fcc_for(sseed, n, vf, ords, max_disp, d, eps, dt)
        out.append(sc)
    return concat_scenes(out)


def _fcc_for(seed, n, vf, ords, max_disp, d, eps, dt):
    """Stretched-FCC scene with >= n sites, vacancies down to n, box scaled to vf."""
    a, b = spheroid_axes()
    vol = 4.0 / 3.0 * math.pi * a * b * b
    k = 1
    while 4 * k * k * k < n:
        k += 1
    cells = (k, k, k)
    sites = 4 * k ** 3
    # box volume so that n spheroids occupy vf; never denser than the lattice allows
    box_volume = n * vol / vf
    ar = a / b
    c = (box_volume / (k ** 3 * ar)) ** (1.0 / 3.0)
    c_min = (2.0 * b + 0.06) * math.sqrt(2.0)
    if c < c_min:
        box_volume = k ** 3 * ar * c_min ** 3
    sc = make_fcc_scene(seed=seed, cells=cells, box_volume=box_volume, vacancies=sites - n,
                        max_disp=max_disp, d=d, eps=eps, dt=dt, orders=ords)
    return sc


CONFIGS = {
    1: dict(fn="make_two_spheres", kw=dict(seed=1)),
    2: dict(fn="make_rsa_scene", kw=dict(seed=2)),
    3: dict(fn="make_fcc_scene", kw=dict(seed=3)),
    4: dict(fn="make_batch", kw=dict(seed=4)),
}


def make_config(k: int, **overrides) -> Scene:
    spec = CONFIGS[k]
    kw = dict(spec["kw"])
    kw.update(overrides)
    return globals()[spec["fn"]](**kw)


def lcp_blocks(x, vtx_off, act_off, act_vtx, ell=0.5, seed=11):
    """Synthetic operator blocks for the LCP matrix, one per vesicle on its
    active points (layout of the LCP matrix entry points): a Gaussian kernel
    of width ell between the points (x [3][n_vtx]) times a seeded random SPD
    3x3 matrix, plus a small diagonal shift; symmetric positive definite,
    smooth in space like a mobility operator.  Returns a flat float64 array."""
    rng = np.random.default_rng(seed)
    act_off = np.asarray(act_off, dtype=np.int64)
    out = []
    for i in range(len(act_off) - 1):
        ids = np.asarray(act_vtx[act_off[i]:act_off[i + 1]], dtype=np.int64)
        a = ids.size
        if a == 0:
            continue
        P = np.asarray(x)[:, ids].T
        d2 = ((P[:, None, :] - P[None, :, :]) ** 2).sum(-1)
        K = np.exp(-d2 / (2.0 * ell * ell))
        Q = rng.normal(size=(3, 3))
        C3 = Q @ Q.T + 0.5 * np.eye(3)
        Mi = np.kron(K, C3) + 1e-3 * np.eye(3 * a)
        out.append(Mi.ravel())
    return np.concatenate(out) if out else np.zeros(0)
