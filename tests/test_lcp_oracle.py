"""Pins of the oracle's LCP matrix (Alg. 3) against closed forms."""
import numpy as np
import pytest

import oracle
from paper_1812_04719_amd import scenes as S


@pytest.fixture(scope="module")
def dense():
    # a small 58 % packing (72 vesicles, about 60 contact volumes)
    sc = S.make_fcc_scene(seed=5, cells=(3, 3, 2), box_volume=22906.304 * 18 / 360)
    r = oracle.detect(sc)
    return sc, r


def _identity_blocks(act_off):
    a = np.diff(act_off)
    return np.concatenate([np.eye(3 * k).ravel() for k in a if k > 0] or [np.zeros(0)])


def test_identity_operator_gives_J_JT(dense):
    """With M_i = I on every vesicle, B(j,k) is the dot product of the full
    Jacobian rows j and k: sum over shared vertices of g_jv . g_kv."""
    sc, r = dense
    act_off, act_vtx, m_off = oracle.lcp_layout(sc.vtx_off, r.j_vtx)
    B, Sp = oracle.lcp_matrix(len(r.vol_pair), sc.vtx_off, r.vol_pair, r.pair_ab, r.j_vol, r.j_vtx, r.j_g,
                              act_off, act_vtx, m_off, _identity_blocks(act_off))
    n = len(r.vol_pair)
    assert n >= 30
    rows = {}
    for v, x, g in zip(r.j_vol, r.j_vtx, r.j_g):
        rows.setdefault(int(v), {})[int(x)] = np.asarray(g)
    want = np.zeros((n, n))
    for j in range(n):
        for k in range(n):
            want[j, k] = sum(float(rows[j][x] @ rows[k][x]) for x in rows[j] if x in rows[k])
    assert np.allclose(B, want, rtol=1e-13, atol=1e-30)
    assert np.all(Sp[want != 0])


def test_spd_operator_gives_symmetric_psd(dense):
    sc, r = dense
    act_off, act_vtx, m_off = oracle.lcp_layout(sc.vtx_off, r.j_vtx)
    M = S.lcp_blocks(sc.x1, sc.vtx_off, act_off, act_vtx)
    B, Sp = oracle.lcp_matrix(len(r.vol_pair), sc.vtx_off, r.vol_pair, r.pair_ab, r.j_vol, r.j_vtx, r.j_g,
                              act_off, act_vtx, m_off, M)
    assert np.allclose(B, B.T, rtol=1e-12, atol=1e-14 * np.abs(B).max())
    w = np.linalg.eigvalsh(0.5 * (B + B.T))
    assert w.min() >= -1e-10 * w.max()
    assert np.all(B[~Sp] == 0.0)
    # diagonal entries are g_j^T M g_j summed over the two vesicles: positive
    assert np.all(np.diag(B) > 0)


def test_hand_example_two_vesicles():
    """One volume shared by vesicles 0 and 1, two volumes on vesicle 1:
    B written out by hand from the rows."""
    vtx_off = np.array([0, 3, 6])
    pair_ab = np.array([[0, 1], [1, 1]])
    vol_pair = np.array([0, 1])
    # volume 0: rows at vertices 1 (ves 0), 4 (ves 1); volume 1: rows at 4 and 5 (ves 1)
    j_vol = np.array([0, 0, 1, 1])
    j_vtx = np.array([1, 4, 4, 5])
    j_g = np.array([[1.0, 0, 0], [0, 2.0, 0], [0, 0, 1.0], [1.0, 1.0, 0]])
    act_off, act_vtx, m_off = oracle.lcp_layout(vtx_off, j_vtx)
    assert act_off.tolist() == [0, 1, 3] and act_vtx.tolist() == [1, 4, 5]
    M0 = np.diag([2.0, 3.0, 4.0])
    M1 = np.arange(36, dtype=float).reshape(6, 6) / 10.0
    M = np.concatenate([M0.ravel(), M1.ravel()])
    B, _ = oracle.lcp_matrix(2, vtx_off, vol_pair, pair_ab, j_vol, j_vtx, j_g, act_off, act_vtx, m_off, M)
    g0_v0 = np.array([1.0, 0, 0])
    g0_v1 = np.array([0, 2.0, 0, 0, 0, 0])
    g1_v1 = np.array([0, 0, 1.0, 1.0, 1.0, 0])
    want = np.array([[g0_v0 @ M0 @ g0_v0 + g0_v1 @ M1 @ g0_v1, g0_v1 @ M1 @ g1_v1],
                     [g1_v1 @ M1 @ g0_v1, g1_v1 @ M1 @ g1_v1]])
    assert np.allclose(B, want, rtol=0, atol=1e-14)
    assert B[0, 0] == pytest.approx(2.0 + 4.0 * M1[1, 1])
