"""GPU parity of the LCP matrix assembly (Alg. 3) against the oracle."""
import numpy as np
import pytest

import oracle
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


def _scene(name):
    if name == "spheres":
        return S.make_two_spheres(seed=1)
    if name == "small_dense":
        return S.make_fcc_scene(seed=5, cells=(3, 3, 2), box_volume=22906.304 * 18 / 360)
    if name == "rsa":
        return S.make_rsa_scene(seed=2, n=64)
    return S.make_config(3)


@pytest.mark.parametrize("name", ["spheres", "rsa", "small_dense", "c1440"])
def test_lcp_matrix_parity(ctx, name):
    import torch
    from paper_1812_04719_amd import stiv
    sc = _scene(name)
    print("lcp parity on %s (%d vesicles)" % (name, sc.n_ves), flush=True)
    ds = stiv.DeviceScene(sc)
    res, outs = stiv.detect(ctx, ds, sc.d, sc.eps, sc.dt)
    r = res["_struct"]
    act_off, m_off, act_vtx = stiv.lcp_layout(ctx, ds, r)
    o = oracle.detect(sc)
    o_act_off, o_act_vtx, o_m_off = oracle.lcp_layout(sc.vtx_off, o["j_vtx"])
    # the active sets are integer data: bit-exact
    assert np.array_equal(act_off.cpu().numpy(), o_act_off)
    assert np.array_equal(act_vtx.cpu().numpy(), o_act_vtx)
    assert np.array_equal(m_off.cpu().numpy(), o_m_off)
    M = S.lcp_blocks(sc.x1, sc.vtx_off, o_act_off, o_act_vtx)
    rows, cols, vals = stiv.form_lcp(ctx, ds, r, act_off, m_off, act_vtx, torch.from_numpy(M).cuda())
    rows, cols, vals = rows.cpu().numpy(), cols.cpu().numpy(), vals.cpu().numpy()
    n_vol = len(o["vol_pair"])
    B, Sp = oracle.lcp_matrix(n_vol, sc.vtx_off, o["vol_pair"], o["pair_ab"], o["j_vol"], o["j_vtx"], o["j_g"],
                              o_act_off, o_act_vtx, o_m_off, M)
    # structure: exactly the pairs of volumes that share a vesicle, sorted by (row, col)
    want_r, want_c = np.nonzero(Sp)
    assert np.array_equal(rows, want_r) and np.array_equal(cols, want_c)
    # values: J rows agree to 1e-10 relative; B is bilinear in them
    scale = np.abs(B).max() if B.size else 1.0
    assert np.all(np.abs(vals - B[rows, cols]) <= 1e-9 * scale + 1e-300)
    # reproducible
    _, _, vals2 = stiv.form_lcp(ctx, ds, r, act_off, m_off, act_vtx, torch.from_numpy(M).cuda())
    assert np.array_equal(vals2.cpu().numpy(), vals)


def test_lcp_empty_result(ctx):
    """A scene without contacts: no active points, empty B."""
    import torch
    from paper_1812_04719_amd import stiv
    sc = S.make_two_spheres(seed=1, gap=0.5)
    ds = stiv.DeviceScene(sc)
    res, outs = stiv.detect(ctx, ds, sc.d, sc.eps, sc.dt)  # outs keeps the result arrays alive
    assert res["n_vol"] == 0
    act_off, m_off, act_vtx = stiv.lcp_layout(ctx, ds, res["_struct"])
    assert act_vtx.numel() == 0 and int(act_off[-1]) == 0 and int(m_off[-1]) == 0
    rows, cols, vals = stiv.form_lcp(ctx, ds, res["_struct"], act_off, m_off, act_vtx,
                                     torch.zeros(1, dtype=torch.float64, device="cuda:0"))
    assert rows.numel() == 0
