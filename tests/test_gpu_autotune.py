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
    x = gen.workload_data(gen.CFG2, 60000)
    n = x.shape[0]
    data = F.make_data(dev(x))
    params = F.make_params(8, 64, 32, 1.2, 8)
    ws = F.alloc_workspace(data, params)
    cache = tmp_path / "tune.txt"
    t1 = F.autotune(data, params, ws, cache)
    assert t1.beam_table_slots in (1024, 2048, 4096) and 0 <= t1.waves_per_cu <= 64
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
    assert t.screen == F.SCREEN_BF16 and t.beam_table_slots in (2048, 4096)
    assert _build_hash(F, data, t, 8000) == _build_hash(F, data, F.make_params(8, 128, 32, 1.2, 4), 8000)
