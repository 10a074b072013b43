"""The harvest's on-chip bounds against the oracle, which has none: every
visited-table size (1024 / 2048 / 4096 slots) element by element, and
expanded sets longer than the on-chip sort space (sorted and pruned in the
search's device buffer), up to the stated capacity, beyond which the call
fails with FG_ECAPACITY instead of writing a wrong row."""
import numpy as np
import pytest
import torch

from gpu_util import dev, empty_u32, host_u32, say
from paper_2609_30493_amd import datagen as gen

pytestmark = pytest.mark.gpu


def _path(n):
    """Points on a line (x_i = (i, 0, 0, 0)) and the path graph i -- i+1 as
    the substrate: a search from root 0 for point p walks the whole path to
    p, so it expands about p vertices."""
    x = np.zeros((n, 4), np.float32)
    x[:, 0] = np.arange(n, dtype=np.float32)
    deg = np.full(n, 2, np.uint64)
    deg[0] = deg[-1] = 1
    off = np.concatenate([[0], np.cumsum(deg)]).astype(np.uint64)
    ids = np.empty(int(off[-1]), np.uint32)
    for v in range(n):
        nb = [u for u in (v - 1, v + 1) if 0 <= u < n]
        ids[int(off[v]):int(off[v + 1])] = nb
    return x, off, ids


@pytest.mark.parametrize("table", [1024, 2048, 4096])
def test_long_expanded_sets_match_oracle(fgo, table):
    from paper_2609_30493_amd import fgraft as F
    n, ef, R = 6000, 4, 4
    say(f"long expanded sets: path graph n={n} ef={ef} table={table}")
    x, off, ids = _path(n)
    D = fgo.Data(x)
    r = np.zeros(1, np.uint32)
    P = fgo.params(1, ef, R, 1.2, 1, 0, 8)
    rows_o = np.full((n, R), fgo.NONE, np.uint32)
    cnt_o = np.zeros(n, np.uint32)
    co = fgo.harvest_block(D, off, ids, r, P, 0, rows_o, cnt_o)
    # the longest searches expand several thousand vertices: past every
    # table's on-chip sort space (half its slots)
    assert co["expansions"] > n * (n - 1) // 2
    data = F.make_data(dev(x))
    params = F.make_params(1, ef, R, 1.2, 1, beam_table_slots=table)
    ws = F.alloc_workspace(data, params)
    rows, cnt = empty_u32(n, R), empty_u32(n, fill=0)
    cg = F.harvest_block(data, F.csr(dev(off), dev(ids)), dev(r), params, 0, rows, cnt, ws)
    assert np.array_equal(host_u32(rows), rows_o)
    assert np.array_equal(host_u32(cnt), cnt_o)
    for k in ("harvest_evals", "expansions", "prune_evals"):
        assert cg[k] == co[k], k


def test_expanded_set_beyond_capacity_is_an_error(fgo):
    """A search that expands 8192 vertices or more fails the call with
    FG_ECAPACITY (reported after the kernel, through the counters' sync and
    through fg_sync_status); the points whose searches fit still get the
    oracle's rows."""
    from paper_2609_30493_amd import fgraft as F
    n = 9000
    say(f"expanded-set capacity: path graph n={n}")
    x, off, ids = _path(n)
    rows_o = np.full((n, 4), fgo.NONE, np.uint32)
    cnt_o = np.zeros(n, np.uint32)
    fgo.harvest_block(fgo.Data(x), off, ids, np.zeros(1, np.uint32), fgo.params(1, 4, 4, 1.2, 1, 0, 8), 0,
                      rows_o, cnt_o)
    data = F.make_data(dev(x))
    params = F.make_params(1, 4, 4, 1.2, 1)
    ws = F.alloc_workspace(data, params)
    rows, cnt = empty_u32(n, 4), empty_u32(n, fill=0)
    r = dev(np.zeros(1, np.uint32))
    with pytest.raises(F.FgError) as e:
        F.harvest_block(data, F.csr(dev(off), dev(ids)), r, params, 0, rows, cnt, ws)
    assert e.value.code == F.FG_ECAPACITY
    F.harvest_block(data, F.csr(dev(off), dev(ids)), r, params, 0, rows, cnt, ws, counters=False)
    with pytest.raises(F.FgError) as e:
        F.sync_status(ws)
    assert e.value.code == F.FG_ECAPACITY
    # searches of p below 8180 expand fewer than 8192 vertices
    assert np.array_equal(host_u32(rows)[:8180], rows_o[:8180])
    assert np.array_equal(host_u32(cnt)[:8180], cnt_o[:8180])


@pytest.mark.parametrize("table", [512, 1024, 2048, 4096])
def test_harvest_table_sizes_match_oracle(fgo, table):
    """The uint8 workload's shape at every table size that applies
    (ef_h = 64, one 16-byte chunk per lane)."""
    from paper_2609_30493_amd import fgraft as F
    T, ef, R, B, b = 8, 64, 32, 8, 5
    x = gen.workload_data(gen.SIFT_1M, 6000)
    n = x.shape[0]
    say(f"harvest parity u8 sift-shape n={n} table={table}")
    D = fgo.Data(x)
    r, parents, off, ids, _ = fgo.scaffold(D, 42, T)
    P = fgo.params(T, ef, R, 1.2, B, 0, 8)
    rows_o = np.full((n, R), fgo.NONE, np.uint32)
    cnt_o = np.zeros(n, np.uint32)
    co = fgo.harvest_block(D, off, ids, r, P, b, rows_o, cnt_o)
    data = F.make_data(dev(x))
    params = F.make_params(T, ef, R, 1.2, B, beam_table_slots=table)
    ws = F.alloc_workspace(data, params)
    rows, cnt = empty_u32(n, R), empty_u32(n, fill=0)
    cg = F.harvest_block(data, F.csr(dev(off), dev(ids)), dev(r), params, b, rows, cnt, ws)
    assert np.array_equal(host_u32(rows), rows_o)
    assert np.array_equal(host_u32(cnt), cnt_o)
    for k in ("harvest_evals", "expansions", "prune_evals"):
        assert cg[k] == co[k], k
    if table <= 1024:
        assert cg["spilled_queries"] > 0  # the visited table overflowed into the bitset


@pytest.mark.parametrize("name,table", [("u8-sift-9000", 1024), ("u8-sift-9000", 512),
                                        ("f32-cos-d100-3000", 512), ("f32-cos-d100-3000", 1024),
                                        ("f32-cos-d100-3000", 2048), ("f32-cos-d100-3000", 4096),
                                        ("f32-d960-1500", 512)])
def test_build_table_sizes_match_oracle(fgo, name, table):
    """Whole builds at each table size: the uint8 workload's parameters at
    512 and 1024 slots, the GloVe-shaped cosine workload's (T=8, B=8,
    ef_h=128, R=64) at every size, and the GIST-shaped rows (d = 960, the
    matrix-core prune) at 512 (expanded sets beyond 256 go to the device)."""
    from paper_2609_30493_amd import fgraft as F
    if name == "u8-sift-9000":
        x, metric, T, ef, R, B = gen.workload_data(gen.SIFT_1M, 9000), "l2", 8, 64, 32, 8
    elif name == "f32-d960-1500":
        x, metric, T, ef, R, B = gen.workload_data(gen.GIST_1M, 1500), "l2", 8, 128, 64, 8
    else:
        x, metric, T, ef, R, B = gen.workload_data(gen.GLOVE_1183514, 3000), "cosine", 8, 128, 64, 8
    n = x.shape[0]
    say(f"build parity {name} table={table}")
    want = fgo.build_graph(fgo.Data(x, metric=metric), 42, fgo.params(T, ef, R, 1.2, B, 0, 8))
    data = F.make_data(dev(x), metric)
    params = F.make_params(T, ef, R, 1.2, B, beam_table_slots=table)
    ws = F.alloc_workspace(data, params)
    gn, gc, sp, rt = empty_u32(n, R), empty_u32(n, fill=0), empty_u32(n), empty_u32(T)
    G = F.make_graph(gn, gc, sp, rt, T)
    c, _ = F.build_graph(data, 42, params, G, ws, timings=True)
    assert np.array_equal(host_u32(gn), want["nbrs"])
    assert np.array_equal(host_u32(gc), want["cnt"])
    assert F.graph_hash(G) == want["hash"]
    for k in ("scaffold_evals", "harvest_evals", "prune_evals", "expansions", "finalize_evals"):
        assert c[k] == want["counters"][k], k
