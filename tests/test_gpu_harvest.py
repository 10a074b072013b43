"""Parity of the HIP harvest (beam + occlusion prune of one block) with the
CPU oracle, element by element, on the oracle's own scaffold."""
import numpy as np
import pytest
import torch

from gpu_util import dev, empty_u32, host_u32, say
from paper_2609_30493_amd import datagen as gen

pytestmark = pytest.mark.gpu


def _case(name):
    if name == "u8-d16":
        return gen.small_u8(3000, 16, 3, hi=256), "l2"
    if name == "u8-d128-ties":
        return gen.small_u8(2500, 128, 4, hi=3), "l2"
    if name == "u8-sift-shape":
        return gen.workload_data(gen.SIFT_1M, 6000), "l2"
    if name == "f32-d32":
        return gen.workload_data(gen.MIX_10K, 4000), "l2"
    if name == "f32-d100-cos":
        return gen.anisotropic_unit_f32(2500, 100, 20, 3), "cosine"
    if name == "f32-d960":
        return gen.powerlaw_f32(700, 960, 10, 4), "l2"
    if name == "f32-d64":
        return gen.isotropic_f32(2000, 64, 8, 0.2, 11), "l2"
    raise KeyError(name)


CASES = [
    # name, T, ef, R, alpha, B, b
    ("u8-d16", 3, 32, 16, 1.2, 3, 1),
    ("u8-d128-ties", 4, 24, 12, 1.0, 2, 0),
    ("u8-sift-shape", 8, 64, 32, 1.2, 8, 5),
    ("f32-d32", 4, 32, 24, 1.2, 1, 0),
    ("f32-d100-cos", 8, 128, 64, 1.2, 4, 3),
    ("f32-d960", 8, 64, 32, 1.2, 2, 1),
    ("f32-d64", 2, 256, 8, 1.5, 5, 4),
]


@pytest.mark.parametrize("case", CASES, ids=[c[0] for c in CASES])
def test_harvest_block_matches_oracle(fgo, case):
    from paper_2609_30493_amd import fgraft as F
    name, T, ef, R, alpha, B, b = case
    say(f"harvest parity case={name} T={T} ef={ef} R={R} B={B} b={b}")
    x, metric = _case(name)
    n = x.shape[0]
    D = fgo.Data(x, metric=metric)
    r, parents, off, ids, _ = fgo.scaffold(D, 42, T)
    P = fgo.params(T, ef, R, alpha, B, 0, 8)
    rows_o = np.full((n, R), fgo.NONE, np.uint32)
    cnt_o = np.zeros(n, np.uint32)
    co = fgo.harvest_block(D, off, ids, r, P, b, rows_o, cnt_o)

    xd = dev(x)
    data = F.make_data(xd, metric)
    params = F.make_params(T, ef, R, alpha, B)
    off_d, ids_d, r_d = dev(off), dev(ids), dev(r)
    rows = empty_u32(n, R)
    cnt = empty_u32(n, fill=0)
    ws = F.alloc_workspace(data, params)
    cg = F.harvest_block(data, F.csr(off_d, ids_d), r_d, params, b, rows, cnt, ws)
    torch.cuda.synchronize()
    rows_g, cnt_g = host_u32(rows), host_u32(cnt)
    bad = np.nonzero((rows_g != rows_o).any(1) | (cnt_g != cnt_o))[0]
    assert bad.size == 0, f"{bad.size} rows differ, first {bad[:5]}: gpu {rows_g[bad[0]][:8]} oracle {rows_o[bad[0]][:8]}"
    assert cg["harvest_evals"] == co["harvest_evals"]
    assert cg["expansions"] == co["expansions"]
    assert cg["prune_evals"] == co["prune_evals"]


def test_harvest_spill_path_and_full_width(fgo):
    """ef >= n: the search visits every point, overflowing the on-chip
    visited table into the device bitset; rows must still match."""
    from paper_2609_30493_amd import fgraft as F
    n = 5000
    say(f"harvest spill case n={n} ef=256")
    x = gen.small_u8(n, 16, 9, hi=256)
    D = fgo.Data(x)
    r, parents, off, ids, _ = fgo.scaffold(D, 1, 2)
    P = fgo.params(2, 256, 10, 1.2, 40, 0, 8)
    rows_o = np.full((n, 10), fgo.NONE, np.uint32)
    cnt_o = np.zeros(n, np.uint32)
    co = fgo.harvest_block(D, off, ids, r, P, 7, rows_o, cnt_o)
    xd = dev(x)
    data = F.make_data(xd)
    params = F.make_params(2, 256, 10, 1.2, 40)
    rows = empty_u32(n, 10)
    cnt = empty_u32(n, fill=0)
    ws = F.alloc_workspace(data, params)
    cg = F.harvest_block(data, F.csr(dev(off), dev(ids)), dev(r), params, 7, rows, cnt, ws)
    assert np.array_equal(host_u32(rows), rows_o) and np.array_equal(host_u32(cnt), cnt_o)
    assert cg["harvest_evals"] == co["harvest_evals"]
    # run again on the same workspace: the spill bitsets must have been left clean
    cg2 = F.harvest_block(data, F.csr(dev(off), dev(ids)), dev(r), params, 7, rows, cnt, ws)
    assert cg2["harvest_evals"] == co["harvest_evals"]
    # without counters the call returns at once; fg_sync_status waits and
    # reports the device status (clean here)
    rows.fill_(-1)
    F.harvest_block(data, F.csr(dev(off), dev(ids)), dev(r), params, 7, rows, cnt, ws, counters=False)
    F.sync_status(ws)
    assert np.array_equal(host_u32(rows), rows_o)
    with pytest.raises(F.FgError) as e:
        F._check(F.lib().fg_sync_status(None, None))
    assert e.value.code == F.FG_EINVAL


def test_harvest_rejects_bad_arguments():
    from paper_2609_30493_amd import fgraft as F
    x = dev(gen.small_u8(100, 16, 1))
    data = F.make_data(x)
    params = F.make_params(2, 300, 8)   # ef_h above the bound
    off = torch.zeros(101, dtype=torch.int64, device="cuda")
    ids = torch.zeros(1, dtype=torch.int32, device="cuda")
    r = dev(np.array([0, 1], np.uint32))
    rows = empty_u32(100, 8)
    cnt = empty_u32(100, fill=0)
    ws = F.alloc_workspace(data, params)
    with pytest.raises(F.FgError) as e:
        F.harvest_block(data, F.csr(off, ids), r, params, 0, rows, cnt, ws)
    assert e.value.code == F.FG_EINVAL
    params = F.make_params(2, 16, 8, B=4)
    with pytest.raises(F.FgError):
        F.harvest_block(data, F.csr(off, ids), r, params, 4, rows, cnt, ws)  # b >= B
