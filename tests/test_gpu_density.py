"""The harvest's visit log (Sec. 5.5's lockstep-density measurement) against
the oracle: for sampled points of every block, the ids the GPU search
visits, in order, equal the oracle beam's visited sequence over the same
substrate S_b, and the visit counts after the roots and after each of the
first expansions equal those the oracle's expanded sequence implies.  The
logged build's graph is the plain build's."""
import numpy as np
import pytest
import torch

from gpu_util import dev, empty_u32, host_u32, say
from paper_2609_30493_amd import datagen as gen

pytestmark = pytest.mark.gpu

MARKS = 17


def _counts_after_expansions(off, ids, roots, E, k):
    """|V| after the roots and after each of the first k - 1 expansions of
    the expanded sequence E (the search's total beyond its last one)."""
    seen = set(int(r) for r in roots)
    out = [len(seen)]
    for v in E[:k - 1]:
        seen.update(int(u) for u in ids[int(off[v]):int(off[v + 1])])
        out.append(len(seen))
    while len(out) < k:
        out.append(out[-1])
    return out


@pytest.mark.parametrize("name", ["cos-d100-2500", "u8-d128-4000"])
def test_visit_log_matches_oracle_sequence(fgo, name):
    from paper_2609_30493_amd import fgraft as F
    if name == "cos-d100-2500":
        x, metric, T, ef, R, B = gen.workload_data(gen.GLOVE_1183514, 2500), "cosine", 8, 128, 64, 4
    else:
        x, metric, T, ef, R, B = gen.workload_data(gen.SIFT_1M, 4000), "l2", 8, 64, 32, 4
    n = x.shape[0]
    say(f"visit log parity {name} T={T} ef={ef} R={R} B={B}")
    D = fgo.Data(x, metric=metric)
    P = fgo.params(T, ef, R, 1.2, B, 0, 8)
    r, parents, off, ids, _ = fgo.scaffold(D, 42, T)
    subs = []
    rows = np.full((n, R), fgo.NONE, np.uint32)
    cnt = np.zeros(n, np.uint32)
    so, si = off, ids
    for b in range(B):
        subs.append((so, si))
        fgo.harvest_block(D, so, si, r, P, b, rows, cnt)
        if b + 1 < B:
            so, si = fgo.merge_block(n, so, si, rows, cnt, R, B, b)
    want = fgo.build_graph(D, 42, P)

    pts = np.arange(0, n, 9)
    slot = np.full(n, -1, np.int32)
    slot[pts] = np.arange(len(pts), dtype=np.int32)
    data = F.make_data(dev(x), metric)
    params = F.make_params(T, ef, R, 1.2, B)
    ws = F.alloc_workspace(data, params)
    gn, gc, sp, rt = empty_u32(n, R), empty_u32(n, fill=0), empty_u32(n), empty_u32(T)
    G = F.make_graph(gn, gc, sp, rt, T)
    cap = n
    c, t, lids, lens, marks = F.build_graph_log(data, 42, params, G, ws, torch.from_numpy(slot).cuda(), cap)
    assert F.graph_hash(G) == want["hash"]
    assert c["harvest_evals"] == want["counters"]["harvest_evals"]
    lids, lens, marks = host_u32(lids), host_u32(lens), host_u32(marks)
    for i, p in enumerate(pts):
        so, si = subs[p % B]
        bo = fgo.beam(D, so, si, r, ef, p=int(p))
        V = bo["V"]
        assert lens[i] == len(V), p
        assert np.array_equal(lids[i, :len(V)], V), p
        assert marks[i].tolist() == _counts_after_expansions(so, si, r, bo["E_ids"], MARKS), p


def test_visit_log_rejects_screened_builds_and_bad_logs():
    from paper_2609_30493_amd import fgraft as F
    x = gen.workload_data(gen.GLOVE_1183514, 500)
    data = F.make_data(dev(x), "cosine")
    params = F.make_params(4, 32, 16, 1.2, 2, screen=F.SCREEN_BF16)
    ws = F.alloc_workspace(data, params)
    G = F.make_graph(empty_u32(500, 16), empty_u32(500, fill=0), empty_u32(500), empty_u32(4), 4)
    slot = torch.zeros(500, dtype=torch.int32, device="cuda")
    with pytest.raises(F.FgError) as e:
        F.build_graph_log(data, 42, params, G, ws, slot, 64)
    assert e.value.code == F.FG_EUNSUPPORTED
    with pytest.raises(F.FgError) as e:
        F.build_graph_log(data, 42, F.make_params(4, 32, 16, 1.2, 2), G, ws, slot, 0)
    assert e.value.code == F.FG_EINVAL
