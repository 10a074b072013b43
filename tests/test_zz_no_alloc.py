"""fg_search_noalloc (the query search for callers that cannot allocate):
its results equal fg_search's on the same graph and queries, bit for bit,
on two calls in a row (the second on a smaller graph and fewer queries),
and an input too large for its fixed scratch is refused before any work."""
import numpy as np
import pytest
import torch

from gpu_util import say
from paper_2609_30493_amd import datagen as gen
from paper_2609_30493_amd import fgraft as F

pytestmark = pytest.mark.gpu


def _u32(*shape):
    return torch.full(shape, -1, dtype=torch.int32, device="cuda")


def _built(x, metric, T=4, ef=48, R=24, B=2):
    xd = torch.from_numpy(x).cuda()
    data = F.make_data(xd, metric)
    params = F.make_params(T, ef, R, 1.2, B)
    ws = F.alloc_workspace(data, params)
    n = x.shape[0]
    G = F.make_graph(_u32(n, R), _u32(n), _u32(n), _u32(T), T)
    F.build_graph(data, 42, params, G, ws)
    return xd, data, G, ws


def _both(data, G, ws, q, k, L, dtype):
    nq = q.shape[0]
    outs = []
    for fn in ("search", "search_noalloc"):
        oi = _u32(nq, k)
        od = torch.full((nq, k), 7, dtype=dtype, device="cuda")
        oe = _u32(nq)
        if fn == "search":
            F.search(data, G, q, k, L, oi, od, oe, ws)
        else:
            F.search_noalloc(data, G, q, k, L, oi, od, oe)
        torch.cuda.synchronize()
        outs.append((oi.cpu().numpy(), od.cpu().numpy(), oe.cpu().numpy()))
    return outs


def test_noalloc_search_equals_search_twice_then_smaller():
    assert F.search_noalloc_scratch_bytes() == 64 << 20
    cases = [
        ("first: float32 cosine n=24000 d=100, 400 queries, L=96", gen.GLOVE_1183514, 24_000, 400, 96),
        ("second: uint8 n=6000 d=128, 150 queries, L=64", gen.SIFT_1M, 6_000, 150, 64),
    ]
    for label, w, n, nq, L in cases:
        say(f"[noalloc] {label}")
        x = gen.workload_data(w, n)
        metric = "cosine" if w.metric == "cosine" else "l2"
        xd, data, G, ws = _built(x, metric)
        q = torch.from_numpy(gen.workload_queries(w, nq)).cuda()
        dtype = torch.float32 if x.dtype == np.float32 else torch.int32
        (i0, d0, e0), (i1, d1, e1) = _both(data, G, ws, q, 10, L, dtype)
        assert np.array_equal(i0, i1), label
        assert np.array_equal(d0.view(np.uint32), d1.view(np.uint32)), label
        assert np.array_equal(e0, e1), label
        assert (e0 > 0).all()
        del ws, G, data, xd


def test_noalloc_search_refuses_oversize_inputs():
    # n = 2,000,000 needs far more than 64 MiB for its CSR alone; the call
    # must fail before enqueueing anything (the data pointer is never read)
    n, d, R, T = 2_000_000, 16, 32, 4
    xd = torch.zeros(16, d, dtype=torch.uint8, device="cuda")
    data = F.make_data(xd)
    data.n = n
    G = F.make_graph(_u32(1, R), _u32(1), _u32(1), _u32(T), T)
    G.n = n
    q = torch.zeros(4, d, dtype=torch.uint8, device="cuda")
    oi, od, oe = _u32(4, 10), _u32(4, 10), _u32(4)
    with pytest.raises(F.FgError) as e:
        F.search_noalloc(data, G, q, 10, 32, oi, od, oe)
    assert e.value.code == F.FG_EINVAL
    assert "scratch" in str(e.value)
