"""stiv_backward_static: the backward pass with its scratch in the library's
static device array (no allocation), against stiv_backward on the same
detect results, bit for bit: two calls in a row, the second on a smaller
input; a request beyond the array is refused; a graph-captured call replays
to the same result."""
import ctypes as C

import numpy as np
import pytest

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


def _case(ctx, sc, seed):
    import torch
    from paper_1812_04719_amd import stiv
    ds = stiv.DeviceScene(sc)
    res, outs = stiv.detect(ctx, ds, sc.d, sc.eps, sc.dt, to_numpy=False)
    rng = np.random.default_rng(seed)
    gV = torch.tensor(rng.normal(size=int(res["n_vol"])), device="cuda:0")
    gG = torch.tensor(rng.normal(size=(int(res["n_jrow"]), 3)), device="cuda:0")
    return ds, res, outs, gV, gG


def test_static_backward_matches_backward(ctx):
    import torch
    from paper_1812_04719_amd import stiv
    for k, (sc, seed) in enumerate([(S.make_config(2), 3), (S.make_config(1), 4)]):
        print("static backward call %d: n_ves=%d" % (k, sc.n_ves), flush=True)
        ds, res, outs, gV, gG = _case(ctx, sc, seed)
        assert int(res["n_ct_vt"]) > 0
        want0, want1 = stiv.backward(ctx, ds, sc.d, sc.eps, sc.dt, res["_struct"], gV, gG)
        got0, got1 = stiv.backward(ctx, ds, sc.d, sc.eps, sc.dt, res["_struct"], gV, gG, static_scratch=True)
        torch.cuda.synchronize()
        assert torch.equal(got0, want0) and torch.equal(got1, want1)
        assert float(want1.abs().max()) > 0


def test_static_backward_refuses_oversized_request(ctx):
    """A result with more contacts than the static array can serve is refused
    before anything is launched (the counts are raised in a copy of the
    result struct; no kernel reads them)."""
    from paper_1812_04719_amd import stiv
    sc = S.make_config(1)
    ds, res, outs, gV, gG = _case(ctx, sc, 5)
    big = stiv.stiv_result()
    C.pointer(big)[0] = res["_struct"]
    big.n_ct_ee = 1 << 20
    big.cap_ct = big.n_ct_vt + big.n_ct_ee
    with pytest.raises(stiv.StivError, match="STIV_E_CAPACITY") as e:
        stiv.backward(ctx, ds, sc.d, sc.eps, sc.dt, big, gV, gG, static_scratch=True)
    assert "bytes of scratch" in str(e.value)


def test_static_backward_needs_validated_scene(ctx):
    from paper_1812_04719_amd import stiv
    sc = S.make_config(1)
    ds, res, outs, gV, gG = _case(ctx, sc, 6)
    other = stiv.DeviceScene(sc)  # same data, other (unvalidated) device arrays
    with pytest.raises(stiv.StivError, match="STIV_E_STATE"):
        stiv.backward(ctx, other, sc.d, sc.eps, sc.dt, res["_struct"], gV, gG, static_scratch=True)


def test_static_backward_graph_replay(ctx):
    """Captured once in a graph, every replay (with eager work in between)
    gives the eager stiv_backward result."""
    import torch
    from paper_1812_04719_amd import stiv
    sc = S.make_config(2)
    ds, res, outs, gV, gG = _case(ctx, sc, 7)
    want0, want1 = stiv.backward(ctx, ds, sc.d, sc.eps, sc.dt, res["_struct"], gV, gG)
    out = (torch.empty_like(ds.x0), torch.empty_like(ds.x1))
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        stiv.backward(ctx, ds, sc.d, sc.eps, sc.dt, res["_struct"], gV, gG, static_scratch=True, out=out)
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        stiv.backward(ctx, ds, sc.d, sc.eps, sc.dt, res["_struct"], gV, gG, static_scratch=True, out=out)
    for rep in range(3):
        out[0].fill_(float(rep + 1))
        out[1].fill_(-float(rep + 1))
        stiv.backward(ctx, ds, sc.d, sc.eps, sc.dt, res["_struct"], gV * 0.5, gG, static_scratch=True)
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        assert torch.equal(out[0], want0) and torch.equal(out[1], want1), rep
