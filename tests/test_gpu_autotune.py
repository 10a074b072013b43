"""The autotuner and its knobs: tuned values are in range, cached once and
read back, and no knob setting changes the graph."""
import numpy as np
import pytest

from gpu_util import dev, empty_u32
from paper_2609_30493_amd import datagen as gen

pytestmark = pytest.mark.gpu


def _build_hash(F, data, params, n):
    ws = F.alloc_workspace(data, params)
    G = F.make_graph(empty_u32(n, params.R), empty_u32(n, fill=0), empty_u32(n), empty_u32(params.T), params.T)
    F.build_graph(data, 42, params, G, ws)
    return F.graph_hash(G)


def test_autotune_caches_and_never_changes_the_graph(tmp_path):
    from paper_2609_30493_amd import fgraft as F
    x = gen.workload_data(gen.SIFT_1M, 60000)
    n = x.shape[0]
    data = F.make_data(dev(x))
    params = F.make_params(8, 64, 32, 1.2, 8)
    ws = F.alloc_workspace(data, params)
    cache = tmp_path / "tune.txt"
    t1 = F.autotune(data, params, ws, cache)
    assert t1.beam_table_slots in (512, 1024, 2048, 4096) and 0 <= t1.waves_per_cu <= 64
    assert (t1.T, t1.ef_h, t1.R, t1.B) == (8, 64, 32, 8)
    lines = cache.read_text().splitlines()
    assert len(lines) == 1 and "table=" in lines[0]
    t2 = F.autotune(data, params, ws, cache)
    assert (t2.beam_table_slots, t2.waves_per_cu) == (t1.beam_table_slots, t1.waves_per_cu)
    assert len(cache.read_text().splitlines()) == 1
    h0 = _build_hash(F, data, params, n)
    assert _build_hash(F, data, t1, n) == h0
    assert _build_hash(F, data, F.make_params(8, 64, 32, 1.2, 8, beam_table_slots=4096, waves_per_cu=1), n) == h0


def test_autotune_float32_screened():
    from paper_2609_30493_amd import fgraft as F
    x = gen.powerlaw_f32(8000, 192, 30, 3)
    data = F.make_data(dev(x))
    params = F.make_params(8, 128, 32, 1.2, 4, screen=F.SCREEN_BF16)
    ws = F.alloc_workspace(data, params)
    t = F.autotune(data, params, ws)
    assert t.screen == F.SCREEN_BF16 and t.beam_table_slots in (1024, 2048, 4096)
    assert _build_hash(F, data, t, 8000) == _build_hash(F, data, F.make_params(8, 128, 32, 1.2, 4), 8000)


@pytest.mark.parametrize("name", ["u8-d128", "f32-d64", "cos-d100"])
def test_lanes_per_row_never_changes_the_graph(fgo, name):
    """Every lanes-per-row shape (the library's, 4, 8, 16) gives the oracle's
    graph and counters: the declared order's bits do not depend on it."""
    from paper_2609_30493_amd import fgraft as F
    if name == "u8-d128":
        x, metric = gen.workload_data(gen.SIFT_1M, 5000), "l2"
    elif name == "f32-d64":
        x, metric = gen.isotropic_f32(4000, 64, 16, 0.2, 8), "l2"
    else:
        x, metric = gen.workload_data(gen.GLOVE_1183514, 4000), "cosine"
    n = x.shape[0]
    T, ef, R, B = 8, 64, 32, 4
    want = fgo.build_graph(fgo.Data(x, metric=metric), 42, fgo.params(T, ef, R, 1.2, B, 0, 8))
    data = F.make_data(dev(x), metric)
    for lanes in (0, 4, 8, 16):
        for table in (0, 4096):
            params = F.make_params(T, ef, R, 1.2, B, beam_table_slots=table, lanes_per_row=lanes)
            ws = F.alloc_workspace(data, params)
            G = F.make_graph(empty_u32(n, R), empty_u32(n, fill=0), empty_u32(n), empty_u32(T), T)
            c, _ = F.build_graph(data, 42, params, G, ws, timings=True)
            assert F.graph_hash(G) == want["hash"], (lanes, table)
            for k in ("harvest_evals", "prune_evals", "expansions", "scaffold_evals", "finalize_evals"):
                assert c[k] == want["counters"][k], (lanes, table, k)


def test_autotune_picks_lanes_and_batched_autotune_keeps_graphs():
    """The tuner's choice includes lanes_per_row; a batched build with
    FG_BATCH_AUTOTUNE gives every instance its own build's graph and the
    plain batched counters (the timing launches are not counted)."""
    from paper_2609_30493_amd import fgraft as F
    x = gen.workload_data(gen.GLOVE_1183514, 30000)
    data = F.make_data(dev(x), "cosine")
    params = F.make_params(8, 128, 64, 1.2, 8)
    ws = F.alloc_workspace(data, params)
    t = F.autotune(data, params, ws)
    assert t.lanes_per_row in (0, 8) and t.beam_table_slots in (512, 1024, 2048, 4096)
    insts = gen.batched_instances(count=8, seed0=7700, n_lo=500, n_hi=8000)
    datas = [F.make_data(dev(i["x"])) for i in insts]
    ps = [F.make_params(i["T"], i["ef_h"], i["R"], i["alpha"], i["B"]) for i in insts]

    def graphs():
        return [F.make_graph(empty_u32(i["x"].shape[0], i["R"]), empty_u32(i["x"].shape[0], fill=0),
                             empty_u32(i["x"].shape[0]), empty_u32(i["T"]), i["T"]) for i in insts]

    g0, g1 = graphs(), graphs()
    c0, ws_b = F.build_graph_batched(datas, ps, [i["seed"] for i in insts], g0)
    c1, _ = F.build_graph_batched(datas, ps, [i["seed"] for i in insts], g1, ws=ws_b, autotune=True)
    assert [F.graph_hash(g) for g in g1] == [F.graph_hash(g) for g in g0]
    for k in ("harvest_evals", "prune_evals", "expansions", "scaffold_evals", "finalize_evals"):
        assert c1[k] == c0[k], k
    # a second call reuses the tuned knobs of this batch shape, with graph capture
    g2 = graphs()
    c2, _ = F.build_graph_batched(datas, ps, [i["seed"] for i in insts], g2, ws=ws_b, autotune=True,
                                  use_hipgraph=True)
    assert [F.graph_hash(g) for g in g2] == [F.graph_hash(g) for g in g0]
    assert c2["harvest_evals"] == c0["harvest_evals"]
