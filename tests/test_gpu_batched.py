"""Batched builds: every instance of a batch must get exactly the graph its
own build gives (rows, counts, spine, roots, hash), eager and under HIP
graph capture, and the oracle's on small instances."""
import numpy as np
import pytest
import torch

from gpu_util import dev, empty_u32, host_u32, say
from paper_2609_30493_amd import datagen as gen

pytestmark = pytest.mark.gpu


def _lib():
    from paper_2609_30493_amd import fgraft as F
    return F


def _graph(F, n, R, T):
    arrs = (empty_u32(n, R), empty_u32(n, fill=0), empty_u32(n), empty_u32(T))
    return F.make_graph(*arrs, T), arrs


def _single(F, inst, metric="l2"):
    n, R, T = inst["x"].shape[0], inst["R"], inst["T"]
    data = F.make_data(dev(inst["x"]), metric)
    params = F.make_params(T, inst["ef_h"], R, inst["alpha"], inst["B"])
    ws = F.alloc_workspace(data, params)
    G, arrs = _graph(F, n, R, T)
    c, _ = F.build_graph(data, inst["seed"], params, G, ws, timings=True)
    return F.graph_hash(G), [host_u32(a) for a in arrs], c


def _batched(F, insts, use_graph, metric="l2"):
    datas = [F.make_data(dev(i["x"]), metric) for i in insts]
    params = [F.make_params(i["T"], i["ef_h"], i["R"], i["alpha"], i["B"]) for i in insts]
    gs = [_graph(F, i["x"].shape[0], i["R"], i["T"]) for i in insts]
    c, _ = F.build_graph_batched(datas, params, [i["seed"] for i in insts], [g for g, _ in gs],
                                 use_hipgraph=use_graph)
    return [F.graph_hash(g) for g, _ in gs], [[host_u32(a) for a in arrs] for _, arrs in gs], c


def _insts_f32():
    out = gen.batched_instances(count=6, seed0=7100, n_lo=300, n_hi=6000)
    out[2]["x"] = out[2]["x"][:701]  # n not a multiple of B
    out[2]["n"] = 701
    return out


@pytest.mark.parametrize("use_graph", [False, True])
def test_batched_f32_equals_single_builds(use_graph):
    F = _lib()
    insts = _insts_f32()
    say(f"batched f32 x{len(insts)} graph={use_graph}: n={[i['x'].shape[0] for i in insts]} "
        f"d={[i['d'] for i in insts]} ef={[i['ef_h'] for i in insts]}")
    hs, arrs, c = _batched(F, insts, use_graph)
    tot = {k: 0 for k in ("harvest_evals", "prune_evals", "expansions", "scaffold_evals", "finalize_evals")}
    for i, inst in enumerate(insts):
        h1, a1, c1 = _single(F, inst)
        assert hs[i] == h1, i
        for a, b in zip(arrs[i], a1):
            assert np.array_equal(a, b), i
        for k in tot:
            tot[k] += c1[k]
    for k in tot:
        assert c[k] == tot[k], k


def test_batched_matches_oracle_small(fgo):
    F = _lib()
    insts = gen.batched_instances(count=3, seed0=7300, n_lo=200, n_hi=900)
    hs, _, _ = _batched(F, insts, True)
    for i, inst in enumerate(insts):
        want = fgo.build_graph(fgo.Data(inst["x"]), inst["seed"],
                               fgo.params(inst["T"], inst["ef_h"], inst["R"], inst["alpha"], inst["B"], 0, 8))
        assert hs[i] == want["hash"], i


def test_batched_u8_and_cosine():
    F = _lib()
    u8 = []
    for i, (n, d, ef) in enumerate(((1200, 16, 32), (2600, 128, 64), (900, 32, 16))):
        x = gen.small_u8(n, d, 40 + i, hi=256)
        u8.append(dict(x=x, n=n, d=d, ef_h=ef, T=4, B=3, R=16, alpha=1.2, seed=9 + i))
    hs, _, _ = _batched(F, u8, True)
    for i, inst in enumerate(u8):
        assert hs[i] == _single(F, inst)[0], i
    cos = []
    for i, (n, d) in enumerate(((1500, 100), (800, 68))):
        cos.append(dict(x=gen.anisotropic_unit_f32(n, d, 10, 60 + i), n=n, d=d, ef_h=64, T=8, B=4, R=32,
                        alpha=1.2, seed=3 + i))
    hs, _, _ = _batched(F, cos, False, "cosine")
    for i, inst in enumerate(cos):
        assert hs[i] == _single(F, inst, "cosine")[0], i


@pytest.mark.parametrize("use_graph", [False, True])
def test_batched_hub_rows_beyond_the_on_chip_merge(use_graph):
    """A hub (every point's nearest neighbour) receives ~n/B reverse edges
    per merge, far beyond the 2048 a wave merges on chip: the captured
    blocks finish such rows on the device alone, the eager ones on the
    host-planned path; both must give the single build's graph."""
    F = _lib()
    insts = [dict(x=gen.hub_f32(12000, 32, 2), n=12000, d=32, ef_h=32, T=4, B=2, R=16, alpha=1.2, seed=42),
             dict(x=gen.isotropic_f32(1000, 32, 8, 0.1, 5), n=1000, d=32, ef_h=32, T=4, B=2, R=16, alpha=1.2,
                  seed=1)]
    hs, arrs, _ = _batched(F, insts, use_graph)
    assert int(arrs[0][1].max()) > 0
    for i, inst in enumerate(insts):
        assert hs[i] == _single(F, inst)[0], i


def test_batched_argument_errors():
    F = _lib()
    a = gen.isotropic_f32(500, 32, 4, 0.1, 1)
    datas = [F.make_data(dev(a)), F.make_data(dev(a))]
    gs = [_graph(F, 500, 16, 4)[0], _graph(F, 500, 16, 4)[0]]
    bad_T = [F.make_params(4, 32, 16, 1.2, 2), F.make_params(3, 32, 16, 1.2, 2)]
    assert F.batched_workspace_size(datas, bad_T) == 0
    with pytest.raises(F.FgError) as e:
        F.build_graph_batched(datas, bad_T, [1, 2], gs, ws=torch.empty(1 << 20, dtype=torch.uint8, device="cuda"))
    assert e.value.code == F.FG_EINVAL
    scr = [F.make_params(4, 32, 16, 1.2, 2, screen=1)] * 2
    assert F.batched_workspace_size(datas, scr) == 0
