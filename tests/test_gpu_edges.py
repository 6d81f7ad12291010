"""Edge cases of the GPU path against the oracle: empty and single-vesicle
scenes, separated bodies, a static scene starting within d, one vesicle pair
with thousands of contacts, a finer mesh, and the error for a periodic box
too small for the image-shift range."""
import numpy as np
import pytest

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


def _check(ctx, sc, emit=True):
    from paper_1812_04719_amd import stiv
    print("edge case: n_ves=%d n_vtx=%d" % (sc.n_ves, sc.n_vtx), flush=True)
    g, _ = stiv.detect(ctx, stiv.DeviceScene(sc), sc.d, sc.eps, sc.dt, emit_candidates=emit)
    o = oracle.detect(sc, emit_candidates=emit)
    parity.compare(g, o, sc, sc.dt, sc.eps, check_cand=emit)
    return g, o


def test_no_vesicles(ctx):
    from paper_1812_04719_amd import stiv
    two = S.make_two_spheres(seed=1)
    sc = S.Scene(x0=np.zeros((3, 0)), x1=np.zeros((3, 0)), vtx_off=np.zeros(1, dtype=np.int32),
                 topo_id=np.zeros(0, dtype=np.int32), scene_off=np.array([0, 0], dtype=np.int32),
                 box_len=np.zeros((1, 3)), topos=two.topos)
    g, _ = stiv.detect(ctx, stiv.DeviceScene(sc), sc.d, sc.eps, sc.dt)
    assert g["n_pairs"] == 0 and g["n_ct"] == 0 and g["n_vol"] == 0 and g["n_jrow"] == 0


def test_single_vesicle(ctx):
    two = S.make_two_spheres(seed=1)
    n0 = two.vtx_off[1]
    sc = S.Scene(x0=two.x0[:, :n0].copy(), x1=two.x1[:, :n0].copy(), vtx_off=two.vtx_off[:2].copy(),
                 topo_id=two.topo_id[:1].copy(), scene_off=np.array([0, 1], dtype=np.int32),
                 box_len=np.zeros((1, 3)), topos=two.topos)
    g, o = _check(ctx, sc)
    assert g["n_pairs"] == 0 and g["n_ct"] == 0


def test_separated_bodies(ctx):
    sc = S.make_two_spheres(seed=1, gap=0.5)
    g, o = _check(ctx, sc)
    assert g["n_ct"] == 0 and g["n_vol"] == 0


def test_static_scene_within_d(ctx):
    """Two parallel squares 0.004 apart (d = 0.01) that do not move: every
    vertex over the other square is in contact at s = 0; volumes follow the
    static closed form V = eps * area * dt."""
    sc = T.translating_planes(gap=0.004, closing=0.0, d=0.01)
    g, o = _check(ctx, sc)
    assert g["n_ct_vt"] > 0
    assert np.all(g["ct_tau"] == 0.0)
    assert g["n_initially_within_d"] > 0


@pytest.mark.parametrize("n, contacts, paths", [
    (14, 1624, "contacts and J entries sorted in LDS, 2048 keys each (the largest LDS buckets)"),
    (16, 2115, "contacts sorted in a global slice, J entries in LDS"),
    (18, 2657, "contacts and J entries sorted in global slices"),
])
def test_one_pair_large_buckets(ctx, n, contacts, paths):
    """Two n x n grids closing through each other: one vesicle pair holds thousands of contacts,
    so the aggregation takes its paths for large buckets (named in `paths`)."""
    sc = T.translating_planes(gap=0.05, closing=0.1, d=0.01, n=n)
    g, o = _check(ctx, sc, emit=False)
    assert int(g["n_pairs"]) == 1 and int(g["n_ct_vt"]) + int(g["n_ct_ee"]) == contacts, paths


def test_finer_mesh_two_spheres(ctx):
    """Order-48 grids: more patches per vesicle and longer patch tables."""
    sc = S.make_two_spheres(seed=7, p=48)
    g, o = _check(ctx, sc, emit=False)
    assert g["n_ct"] > 0


def test_periodic_box_too_small(ctx):
    """A periodic box much smaller than the vesicles needs image shifts beyond
    the supported range: a clear error, not wrong pairs."""
    from paper_1812_04719_amd import stiv
    sc = S.make_two_spheres(seed=1)
    small = sc.with_params(box_len=np.full((1, 3), 0.2))
    with pytest.raises(stiv.StivError) as e:
        stiv.detect(ctx, stiv.DeviceScene(small), small.d, small.eps, small.dt)
    assert e.value.status == stiv.STIV_E_ARG


def _hub_scene(n_sat=20, p=16, r_sat=0.3, gap=0.01, step=0.03, seed=5):
    """Vesicle 0 (unit sphere) with n_sat small spheres around it, each moving
    toward it: every pair (0, k) is a vesicle pair, so the pair list of
    vesicle 0 is longer than the in-register sort of a pair bucket holds."""
    from scipy.spatial.transform import Rotation
    rng = np.random.default_rng(seed)
    unit = S.spheroid_body_points(p, 1.0, 1.0)
    rots = Rotation.random(n_sat + 1, random_state=rng).as_matrix()
    k = np.arange(n_sat) + 0.5
    polar = np.arccos(1.0 - 2.0 * k / n_sat)
    azim = np.pi * (1.0 + 5.0 ** 0.5) * k
    dirs = np.stack([np.sin(polar) * np.cos(azim), np.sin(polar) * np.sin(azim), np.cos(polar)], axis=1)
    s0 = [unit @ rots[0].T]
    s1 = [s0[0].copy()]
    for i in range(n_sat):
        c = dirs[i] * (1.0 + r_sat + gap)
        pts = r_sat * (unit @ rots[i + 1].T) + c
        s0.append(pts)
        s1.append(pts - step * dirs[i])
    return S._assemble(s0, s1, [p] * (n_sat + 1), [0.0, 0.0, 0.0],
                       meta={"config": "hub", "n_sat": n_sat, "seed": seed})


def test_vesicle_with_many_pairs(ctx):
    """More than 16 pairs share their first vesicle: the pair bucket is sorted
    by the general path instead of in registers."""
    sc = _hub_scene()
    g, o = _check(ctx, sc)
    first = np.asarray(g["pair_ab"])[: g["n_pairs"], 0]
    assert np.count_nonzero(first == 0) > 16
    assert g["n_ct_vt"] > 0 and g["n_vol"] >= 17


def test_vertex_in_many_patches(ctx):
    """Order-48 grids tiled into 16-triangle patches: each pole vertex lies in
    all 96 triangles of its fan, so in at least 6 patches (more than the four
    packed per vertex in the box kernel's incidence table)."""
    ctx.set_patch_size(16)
    try:
        sc = S.make_two_spheres(seed=7, p=48)
        g, o = _check(ctx, sc, emit=False)
        assert g["n_ct"] > 0
    finally:
        ctx.set_patch_size(64)
