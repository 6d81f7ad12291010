"""Batched multi-scene detection, graph capture/replay, autotuner."""
import numpy as np
import pytest

import oracle
import parity
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


@pytest.fixture(scope="module")
def batch():
    # 12 independent scenes of uneven size, order (16/24/32) and density (10-60 %)
    return S.make_batch(seed=44, n_scenes=12)


def test_batch_parity(ctx, batch):
    from paper_1812_04719_amd import stiv
    print("batch: scenes=%d vesicles=%d" % (batch.n_scenes, batch.n_ves), flush=True)
    g, _ = stiv.detect(ctx, stiv.DeviceScene(batch), batch.d, batch.eps, batch.dt, emit_candidates=True)
    o = oracle.detect(batch, emit_candidates=True)
    assert len({t.order for t in batch.topos}) >= 2
    parity.compare(g, o, batch, batch.dt, batch.eps, check_cand=True)
    # pairs never cross scenes
    sc_of = np.searchsorted(batch.scene_off, np.arange(batch.n_ves), side="right") - 1
    assert np.all(sc_of[g["pair_ab"][:, 0]] == sc_of[g["pair_ab"][:, 1]])


def test_graph_capture_replay(ctx, batch):
    """Capture the async detect in a graph; every replay (with eager work in
    between) equals the eager result bit for bit."""
    import torch
    from paper_1812_04719_amd import stiv
    ds = stiv.DeviceScene(batch)
    eager, outs_e = stiv.detect(ctx, ds, batch.d, batch.eps, batch.dt)
    outs = stiv.Outputs(ds.x0.device, cap_pairs=2 * eager["n_pairs"] + 16, cap_ct=2 * eager["n_ct"] + 16,
                        cap_vol=2 * eager["n_vol"] + 16, cap_jrow=2 * eager["n_jrow"] + 16)
    job = stiv.AsyncDetect(ctx, ds, batch.d, batch.eps, batch.dt, outs)
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        job.enqueue()  # warm-up on the capture stream
        job.collect()
    torch.cuda.current_stream().wait_stream(side)
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        job.enqueue()
    keys = ("pair_ab", "ct_key", "ct_tau", "ct_vol", "ct_grad", "vol_pair", "vol_V", "j_vtx", "j_g")
    for rep in range(3):
        # eager work between replays
        stiv.detect(ctx, ds, batch.d, batch.eps, batch.dt)
        torch.cuda.synchronize()
        g.replay()
        r = job.collect()
        for k in keys:
            assert np.array_equal(r[k], eager[k]), (rep, k)


def test_autotune(ctx, tmp_path):
    from paper_1812_04719_amd import autotune, stiv
    sc = S.make_config(2)
    ds = stiv.DeviceScene(sc)
    cand = [dict(tile=64, prim_blocks=8192, narrow_blocks=8192), dict(tile=32, prim_blocks=4096, narrow_blocks=4096)]
    cache = str(tmp_path / "tune.json")
    cfg, table = autotune.tune(ctx, ds, sc.d, sc.eps, sc.dt, cache_file=cache, candidates=cand, reps=2)
    assert cfg in [{k: c[k] for k in ("tile", "prim_blocks", "narrow_blocks")} for c in cand]
    assert len(table) == 2 and all(r["ms"] > 0 for r in table)
    cfg2, table2 = autotune.tune(ctx, ds, sc.d, sc.eps, sc.dt, cache_file=cache, candidates=cand)
    assert cfg2 == cfg and table2 == []
    g, _ = stiv.detect(ctx, ds, sc.d, sc.eps, sc.dt)
    parity.compare(g, oracle.detect(sc), sc, sc.dt, sc.eps)
    autotune.apply(ctx, dict(tile=64, prim_blocks=8192, narrow_blocks=8192))


@pytest.fixture(scope="module")
def batch_256():
    return S.make_config(4)


@pytest.mark.timeout(900)
def test_batch_config_256_scenes(ctx, batch_256):
    """The full batching configuration: 256 independent scenes of 8-128
    vesicles, orders 16/24/32, 10-60 % volume fraction, in one call; every
    set exact against the oracle (pairs, the primitive candidate set,
    contacts, volumes, J rows, counters)."""
    from paper_1812_04719_amd import stiv
    b = batch_256
    print("batch config: scenes=%d vesicles=%d vertices=%d" % (b.n_scenes, b.n_ves, b.n_vtx), flush=True)
    g, _ = stiv.detect(ctx, stiv.DeviceScene(b), b.d, b.eps, b.dt, emit_candidates=True)
    o = oracle.detect(b, emit_candidates=True)
    assert b.n_scenes == 256
    st = parity.compare(g, o, b, b.dt, b.eps, check_cand=True)
    print("parity statistics: %s" % st, flush=True)


@pytest.mark.timeout(900)
def test_batch_config_256_scenes_d0(ctx, batch_256):
    """The 256-scene batch with d = 0 (coplanarity cubic)."""
    from paper_1812_04719_amd import stiv
    b = batch_256
    print("batch config d=0", flush=True)
    g, _ = stiv.detect(ctx, stiv.DeviceScene(b), 0.0, b.eps, b.dt)
    o = oracle.detect(b, d=0.0)
    st = parity.compare(g, o, b, b.dt, b.eps)
    print("parity statistics: %s" % st, flush=True)
