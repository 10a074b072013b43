"""The blocked dense leaf k-NN on matrix cores against brute force.

On small-integer data every product and partial sum is an exact float32
(and bfloat16 holds the inputs exactly), so ids and distances must match the
brute force exactly; on random floats the distances are checked within the
float32 error of the expansion |x|^2 + |y|^2 - 2<x,y>."""
import numpy as np
import pytest
import torch

from gpu_util import dev, host_u32, say

pytestmark = pytest.mark.gpu


def brute_leaf_knn(x: np.ndarray, S: int, R: int):
    n = x.shape[0]
    ids = np.full((n, R), 0xFFFFFFFF, np.uint32)
    dd = np.full((n, R), np.inf)
    xf = x.astype(np.float64)
    for l0 in range(0, n, S):
        l1 = min(n, l0 + S)
        blk = xf[l0:l1]
        D = ((blk[:, None, :] - blk[None, :, :]) ** 2).sum(-1)
        np.fill_diagonal(D, np.inf)
        m = l1 - l0
        for i in range(m):
            order = np.lexsort((np.arange(m), D[i]))[: min(R, m - 1)]
            ids[l0 + i, :len(order)] = l0 + order
            dd[l0 + i, :len(order)] = D[i, order]
    return ids, dd


@pytest.mark.parametrize("d,bf16", [(32, False), (96, False), (960, False), (32, True), (128, True),
                                    (960, True)])
def test_leaf_knn_exact_on_integers(d, bf16):
    from paper_2609_30493_amd import fgraft as F
    say(f"leaf knn exact d={d} bf16={bf16}")
    rng = np.random.default_rng(d)
    n, S, R = 2600, 1024, 16
    x = rng.integers(-8, 9, size=(n, d)).astype(np.float32)
    want_ids, want_d = brute_leaf_knn(x, S, R)
    data = F.make_data(dev(x))
    oi = torch.empty(n, R, dtype=torch.int32, device="cuda")
    od = torch.empty(n, R, dtype=torch.float32, device="cuda")
    F.leaf_knn(data, S, R, bf16, oi, od)
    torch.cuda.synchronize()
    got_d = od.cpu().numpy().astype(np.float64)
    assert np.array_equal(got_d, want_d)
    assert np.array_equal(host_u32(oi), want_ids)


@pytest.mark.parametrize("R,n,S,bf16", [(40, 2200, 1024, False), (64, 2048 + 20, 1024, False),
                                        (64, 1500, 512, True), (1, 700, 256, False), (33, 900, 128, True)])
def test_leaf_knn_list_lengths(R, n, S, bf16):
    """Lists spanning one or two keys per lane, and a last leaf shorter than
    R + 1 (padded rows)."""
    from paper_2609_30493_amd import fgraft as F
    say(f"leaf knn R={R} n={n} S={S} bf16={bf16}")
    rng = np.random.default_rng(R * 7 + n)
    d = 48
    x = rng.integers(-6, 7, size=(n, d)).astype(np.float32)
    want_ids, want_d = brute_leaf_knn(x, S, R)
    data = F.make_data(dev(x))
    oi = torch.empty(n, R, dtype=torch.int32, device="cuda")
    od = torch.empty(n, R, dtype=torch.float32, device="cuda")
    F.leaf_knn(data, S, R, bf16, oi, od)
    torch.cuda.synchronize()
    assert np.array_equal(od.cpu().numpy().astype(np.float64), want_d)
    assert np.array_equal(host_u32(oi), want_ids)


@pytest.mark.parametrize("bf16", [False, True])
def test_leaf_knn_random_floats(bf16):
    from paper_2609_30493_amd import fgraft as F
    rng = np.random.default_rng(5)
    n, d, S, R = 3000, 64, 2048, 32
    x = rng.standard_normal((n, d)).astype(np.float32)
    data = F.make_data(dev(x))
    oi = torch.empty(n, R, dtype=torch.int32, device="cuda")
    od = torch.empty(n, R, dtype=torch.float32, device="cuda")
    F.leaf_knn(data, S, R, bf16, oi, od)
    torch.cuda.synchronize()
    ids = host_u32(oi).astype(np.int64)
    got = od.cpu().numpy().astype(np.float64)
    xr = x.astype(np.float64)
    if bf16:  # the kernel computes with the bfloat16-rounded rows
        xr = torch.from_numpy(x).bfloat16().float().numpy().astype(np.float64)
    want_ids, want_d = brute_leaf_knn(xr, S, R)
    true_of_got = ((xr[:, None, :] - xr[ids]) ** 2).sum(-1)
    scale = (xr ** 2).sum(1).max() * 2
    tol = 64 * 2.0 ** -24 * scale
    assert np.all(np.abs(got - true_of_got) <= tol)
    assert np.all(np.abs(np.sort(got, 1) - want_d) <= 2 * tol)
    assert np.all(np.diff(got, axis=1) >= 0)
