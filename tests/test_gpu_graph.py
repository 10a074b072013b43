"""Parity of the HIP scaffold, merge, finalize, search and whole build with
the CPU oracle: element by element and by graph hash."""
import numpy as np
import pytest
import torch

from gpu_util import dev, empty_u32, host_u32, host_u64, say
from paper_2609_30493_amd import datagen as gen

pytestmark = pytest.mark.gpu


def _lib():
    from paper_2609_30493_amd import fgraft as F
    return F


DATASETS = {
    "u8-d16-3000": lambda: (gen.small_u8(3000, 16, 3, hi=256), "l2"),
    "u8-ties-2000": lambda: (gen.small_u8(2000, 32, 5, hi=3), "l2"),
    "u8-sift-9000": lambda: (gen.workload_data(gen.SIFT_1M, 9000), "l2"),
    "f32-d32-2500": lambda: (gen.workload_data(gen.MIX_10K, 2500), "l2"),
    "f32-cos-d100-1500": lambda: (gen.anisotropic_unit_f32(1500, 100, 20, 3), "cosine"),
    "f32-d960-600": lambda: (gen.powerlaw_f32(600, 960, 10, 4), "l2"),
    "collinear-400": lambda: (gen.degenerate_f32("collinear", 400, 4, 5), "l2"),
    "duplicates-900": lambda: (np.rint(gen.degenerate_f32("duplicates", 900, 8, 6) * 4), "l2"),
    "identical-50": lambda: (np.ones((50, 4), np.float32), "l2"),
    "single-1": lambda: (np.zeros((1, 16), np.uint8), "l2"),
    "pair-2": lambda: (np.array([[1] * 16, [3] * 16], np.uint8), "l2"),
    # a centre point that is every point's nearest neighbour: rows of
    # thousands of entries in S0, in the merges and in finalize
    "hub-u8-6000": lambda: (gen.hub_u8(6000, 128, 1), "l2"),
    "hub-f32-6000": lambda: (gen.hub_f32(6000, 32, 2), "l2"),
    # a hub with ~1500 finalize candidates: finalize's second on-chip tier
    "hub-f32-1500": lambda: (gen.hub_f32(1500, 32, 3), "l2"),
    # the longest rows each kind takes, and a set for every parameter at its bound
    "f32-d1024-400": lambda: (gen.powerlaw_f32(400, 1024, 8, 7), "l2"),
    "u8-d256-1500": lambda: (gen.small_u8(1500, 256, 8, hi=256), "l2"),
    "f32-d32-600": lambda: (gen.workload_data(gen.MIX_10K, 600), "l2"),
}


def _data(name):
    x, metric = DATASETS[name]()
    x = x if x.dtype == np.uint8 else x.astype(np.float32)
    return np.ascontiguousarray(x), metric


@pytest.mark.parametrize("name,T", [("u8-d16-3000", 4), ("u8-ties-2000", 3), ("u8-sift-9000", 8),
                                    ("f32-d32-2500", 4), ("f32-cos-d100-1500", 8),
                                    ("f32-d960-600", 2), ("collinear-400", 3),
                                    ("duplicates-900", 4), ("identical-50", 2), ("pair-2", 2),
                                    ("hub-u8-6000", 4)])
def test_scaffold_matches_oracle(fgo, name, T):
    F = _lib()
    say(f"scaffold parity {name} T={T}")
    x, metric = _data(name)
    n = x.shape[0]
    D = fgo.Data(x, metric=metric)
    r, parents, off, ids, ev = fgo.scaffold(D, 42, T)
    xd = dev(x)
    data = F.make_data(xd, metric)
    params = F.make_params(T, 8, 8)
    ws = F.alloc_workspace(data, params)
    off_d = torch.zeros(n + 1, dtype=torch.int64, device="cuda")
    ids_d = torch.zeros(max(1, 2 * T * (n - 1)), dtype=torch.int32, device="cuda")
    S0 = F.csr(off_d, ids_d, 0)
    tp = empty_u32(T, n)
    c = F.build_scaffold(data, dev(r), T, S0, tp, ws)
    assert np.array_equal(host_u32(tp), parents)
    assert np.array_equal(host_u64(off_d), off)
    assert np.array_equal(host_u32(ids_d)[:S0.nnz], ids)
    assert c["scaffold_evals"] == ev


@pytest.mark.parametrize("name,T,R,B,b", [("u8-d16-3000", 4, 16, 4, 2), ("f32-d32-2500", 4, 24, 3, 0),
                                          ("u8-sift-9000", 8, 32, 8, 6), ("hub-u8-6000", 4, 16, 2, 0),
                                          ("hub-f32-6000", 4, 16, 2, 1)])
def test_merge_matches_oracle(fgo, name, T, R, B, b):
    F = _lib()
    say(f"merge parity {name} R={R} B={B} b={b}")
    x, metric = _data(name)
    n = x.shape[0]
    D = fgo.Data(x, metric=metric)
    r, parents, off, ids, _ = fgo.scaffold(D, 42, T)
    P = fgo.params(T, 32, R, 1.2, B, 0, 8)
    rows = np.full((n, R), fgo.NONE, np.uint32)
    cnt = np.zeros(n, np.uint32)
    fgo.harvest_block(D, off, ids, r, P, b, rows, cnt)
    off2, ids2 = fgo.merge_block(n, off, ids, rows, cnt, R, B, b)
    data = F.make_data(dev(x), metric)
    params = F.make_params(T, 32, R, 1.2, B)
    ws = F.alloc_workspace(data, params)
    o1 = torch.zeros(n + 1, dtype=torch.int64, device="cuda")
    i1 = torch.zeros(len(ids2) + 8, dtype=torch.int32, device="cuda")
    S1 = F.csr(o1, i1, 0)
    nnz = F.merge_block(F.csr(dev(off), dev(ids)), dev(rows), dev(cnt), params, b, S1, ws)
    assert nnz == len(ids2)
    assert np.array_equal(host_u64(o1), off2)
    assert np.array_equal(host_u32(i1)[:nnz], ids2)
    # capacity too small is reported, not overrun
    S_small = F.csr(o1, i1[: nnz - 1], 0)
    with pytest.raises(F.FgError) as e:
        F.merge_block(F.csr(dev(off), dev(ids)), dev(rows), dev(cnt), params, b, S_small, ws)
    assert e.value.code == F.FG_ECAPACITY


@pytest.mark.parametrize("name,T,R,B,reprune", [("u8-d16-3000", 3, 8, 2, 0), ("f32-d32-2500", 4, 24, 1, 0),
                                                ("f32-cos-d100-1500", 4, 12, 2, 1), ("hub-u8-6000", 4, 16, 2, 0),
                                                ("hub-f32-6000", 4, 16, 2, 1), ("hub-u8-6000", 4, 1, 2, 0)])
def test_finalize_matches_oracle(fgo, name, T, R, B, reprune):
    F = _lib()
    say(f"finalize parity {name} R={R} reprune_all={reprune}")
    x, metric = _data(name)
    n = x.shape[0]
    D = fgo.Data(x, metric=metric)
    r, parents, off, ids, _ = fgo.scaffold(D, 42, T)
    P = fgo.params(T, 24, R, 1.2, B, reprune, 8)
    rows = np.full((n, R), fgo.NONE, np.uint32)
    cnt = np.zeros(n, np.uint32)
    so, si = off, ids
    for b in range(max(B, 1)):
        fgo.harvest_block(D, so, si, r, P, b, rows, cnt)
        if b + 1 < B:
            so, si = fgo.merge_block(n, so, si, rows, cnt, R, B, b)
    g, gc, fc = fgo.finalize(D, rows, cnt, P)
    data = F.make_data(dev(x), metric)
    params = F.make_params(T, 24, R, 1.2, B, reprune)
    ws = F.alloc_workspace(data, params)
    gn = empty_u32(n, R)
    gcnt = empty_u32(n, fill=0)
    sp = empty_u32(n)
    rt = dev(r)
    G = F.make_graph(gn, gcnt, sp, rt, T)
    c = F.finalize(data, dev(rows), dev(cnt), params, G, ws)
    assert np.array_equal(host_u32(gn), g)
    assert np.array_equal(host_u32(gcnt), gc)
    assert c["finalize_evals"] == fc["finalize_evals"]


BUILDS = [
    # name, T, ef, R, alpha, B
    ("u8-sift-9000", 8, 64, 32, 1.2, 8),
    ("f32-d32-2500", 4, 32, 24, 1.2, 1),
    ("f32-cos-d100-1500", 8, 128, 64, 1.2, 4),
    ("u8-ties-2000", 3, 16, 10, 1.0, 0),
    ("f32-d960-600", 4, 48, 16, 1.2, 2),
    ("collinear-400", 2, 8, 4, 1.2, 3),
    ("identical-50", 2, 64, 8, 1.2, 64),
    ("single-1", 1, 4, 4, 1.2, 2),
    ("pair-2", 2, 4, 4, 1.2, 1),
    ("hub-u8-6000", 4, 32, 16, 1.2, 2),
    ("hub-f32-6000", 4, 32, 16, 1.2, 3),
    ("hub-f32-1500", 4, 32, 16, 1.2, 2),
    ("f32-d1024-400", 4, 32, 16, 1.2, 2),
    ("u8-d256-1500", 4, 32, 16, 1.2, 2),
    # T, ef_h and R at their largest (64, 256, 1024): rows wider than every
    # on-chip tier of the merge and finalize
    ("f32-d32-600", 64, 256, 1024, 1.2, 4),
]


def _gpu_build(F, x, metric, T, ef, R, alpha, B, seed=42):
    n = x.shape[0]
    data = F.make_data(dev(x), metric)
    params = F.make_params(T, ef, R, alpha, B)
    ws = F.alloc_workspace(data, params)
    gn = empty_u32(n, R)
    gcnt = empty_u32(n, fill=0)
    sp = empty_u32(n)
    rt = empty_u32(T)
    G = F.make_graph(gn, gcnt, sp, rt, T)
    c, t = F.build_graph(data, seed, params, G, ws, timings=True)
    return data, params, ws, G, (gn, gcnt, sp, rt), c, t


@pytest.mark.parametrize("case", BUILDS, ids=[b[0] for b in BUILDS])
def test_build_graph_matches_oracle(fgo, case):
    F = _lib()
    name, T, ef, R, alpha, B = case
    say(f"build parity {name} T={T} ef={ef} R={R} B={B}")
    x, metric = _data(name)
    D = fgo.Data(x, metric=metric)
    want = fgo.build_graph(D, 42, fgo.params(T, ef, R, alpha, B, 0, 8))
    data, params, ws, G, (gn, gcnt, sp, rt), c, t = _gpu_build(F, x, metric, T, ef, R, alpha, B)
    assert np.array_equal(host_u32(rt), want["roots"])
    assert np.array_equal(host_u32(sp), want["parent0"])
    assert np.array_equal(host_u32(gcnt), want["cnt"])
    assert np.array_equal(host_u32(gn), want["nbrs"])
    assert F.graph_hash(G) == want["hash"]
    wc = want["counters"]
    for k in ("scaffold_evals", "harvest_evals", "prune_evals", "expansions", "finalize_evals"):
        assert c[k] == wc[k], k
    assert sum(t["block_evals"]) == wc["harvest_evals"]


def test_build_graph_repeatable_and_b0_equals_b1(fgo):
    F = _lib()
    x, metric = _data("u8-d16-3000")
    hs = []
    for B in (0, 1, 1):
        _, _, _, G, arrs, c, _ = _gpu_build(F, x, metric, 4, 32, 16, 1.2, B)
        hs.append(F.graph_hash(G))
    assert hs[0] == hs[1] == hs[2]


@pytest.mark.parametrize("L", [10, 32, 100, 512])
def test_search_matches_oracle(fgo, L):
    F = _lib()
    say(f"search parity L={L}")
    w = gen.MIX_10K
    x = gen.workload_data(w, 4000)
    q = gen.workload_queries(w, 150)
    D = fgo.Data(x)
    G = fgo.build_graph(D, 42, fgo.params(w.T, w.ef_h, w.R, w.alpha, 2, 0, 8))
    ids_o, d_o, ev_o = fgo.search(D, G, q, 10, L, threads=8)
    data = F.make_data(dev(x))
    params = F.make_params(w.T, w.ef_h, w.R, w.alpha, 2)
    ws = F.alloc_workspace(data, params)
    Gd = F.make_graph(dev(G["nbrs"]), dev(G["cnt"]), dev(G["parent0"]), dev(G["roots"]), w.T)
    qd = dev(q)
    oi = empty_u32(150, 10)
    od = torch.empty(150, 10, dtype=torch.float32, device="cuda")
    oe = empty_u32(150, fill=0)
    F.search(data, Gd, qd, 10, L, oi, od, oe, ws)
    torch.cuda.synchronize()
    assert np.array_equal(host_u32(oi), ids_o)
    assert np.array_equal(od.cpu().numpy().astype(np.float64), d_o)
    assert np.array_equal(host_u32(oe), ev_o)


def test_u8_search_distances_and_recall_mix10k_gpu_graph(fgo):
    """The GPU-built frozen-Graft graph reaches recall@10 >= 0.95."""
    import checkers as ck
    F = _lib()
    w = gen.MIX_10K
    x = gen.workload_data(w)
    q = gen.workload_queries(w)
    data, params, ws, G, arrs, c, t = _gpu_build(F, x, "l2", w.T, w.ef_h, w.R, w.alpha, w.B)
    tid, td = ck.knn_exact(x, q, 10)
    qd = dev(q)
    best = 0.0
    for L in (16, 32, 64):
        oi = empty_u32(len(q), 10)
        od = torch.empty(len(q), 10, dtype=torch.float32, device="cuda")
        F.search(data, G, qd, 10, L, oi, od, None, ws)
        ids = host_u32(oi).astype(np.int64)
        d64 = ((q.astype(np.float64)[:, None, :] - x.astype(np.float64)[ids]) ** 2).sum(-1)
        best = max(best, float(np.mean(d64 <= td[:, -1:] * (1 + 1e-6))))
    assert best >= 0.95
