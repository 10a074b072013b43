"""Host logic of the quality columns (Sec. 2): distances per query at a
matched recall, interpolated between adjacent beam widths, with no value
where the ladder does not bracket the target; and the coherent blocks of
Sec. 5.5 (maximal tree-0 subtrees of bounded size) from a spine."""
import importlib

import numpy as np
import pytest


@pytest.fixture(scope="module")
def bench():
    return importlib.import_module("bench")


def _ladder(points):
    return [{"L": 10 * (i + 1), "recall": r, "evals_per_query": e} for i, (r, e) in enumerate(points)]


def test_interpolates_between_the_bracketing_widths(bench):
    lad = _ladder([(0.80, 1000.0), (0.90, 2000.0), (0.96, 3200.0), (0.99, 5000.0)])
    # 0.95 lies 5/6 of the way from 0.90 to 0.96
    assert bench.d_at_recall(lad, 0.95) == pytest.approx(2000.0 + 5 / 6 * 1200.0, rel=1e-12)
    # 0.97 lies 1/3 of the way from 0.96 to 0.99
    assert bench.d_at_recall(lad, 0.97) == pytest.approx(3200.0 + 1 / 3 * 1800.0, rel=1e-12)
    # a target met exactly by a width takes that width's distances
    assert bench.d_at_recall(lad, 0.96) == pytest.approx(3200.0, rel=1e-12)


def test_no_value_when_not_bracketed(bench):
    lad = _ladder([(0.96, 900.0), (0.98, 1500.0)])
    assert bench.d_at_recall(lad, 0.95) is None  # the first width already reaches it
    assert bench.d_at_recall(lad, 0.99) is None  # no width reaches it
    assert bench.d_at_recall(lad, 0.97) == pytest.approx(1200.0, rel=1e-12)


def test_flat_recall_step_takes_the_upper_width(bench):
    lad = _ladder([(0.90, 1000.0), (0.95, 1500.0), (0.95, 1900.0)])
    assert bench.d_at_recall(lad, 0.95) == pytest.approx(1500.0, rel=1e-12)


def test_monotone_in_the_target(bench):
    lad = _ladder([(0.5, 100.0), (0.7, 250.0), (0.85, 600.0), (0.93, 1400.0), (0.97, 3000.0),
                   (0.99, 7000.0)])
    vals = [bench.d_at_recall(lad, r / 100) for r in range(51, 100)]
    assert all(v is not None for v in vals)
    assert all(a <= b for a, b in zip(vals, vals[1:]))


def test_coherent_blocks_hand_tree(bench):
    """Root 0 -> {1, 2}; 1 -> {3, 4, 5}; 2 -> {6}; 3 -> {7}: subtree sizes
    0:8 1:5 2:2 3:2, the rest 1.  At cap 3 the maximal subtrees of at most 3
    points are rooted at 2, 3, 4, 5 (their parents' subtrees hold 8 and 5)."""
    N = 0xFFFFFFFF
    parent = np.array([N, 0, 0, 1, 1, 1, 2, 3], dtype=np.uint32)
    assert sorted(bench.coherent_blocks(parent, 3).tolist()) == [1, 1, 2, 2]
    assert bench.coherent_blocks(parent, 8).tolist() == [8]  # the whole tree
    assert sorted(bench.coherent_blocks(parent, 1).tolist()) == [1, 1, 1, 1]  # the leaves 4, 5, 6, 7


def test_coherent_blocks_brute_force():
    """Random trees against subtree sizes counted from every node's ancestor
    chain."""
    bench = importlib.import_module("bench")
    rng = np.random.default_rng(9)
    for trial in range(20):
        n = int(rng.integers(1, 300))
        perm = rng.permutation(n)
        parent = np.full(n, 0xFFFFFFFF, dtype=np.uint32)
        for i in range(1, n):  # each node hangs below an earlier one in a random order
            parent[perm[i]] = perm[int(rng.integers(0, i))]
        size = np.zeros(n, dtype=np.int64)
        for v in range(n):
            u = v
            while True:
                size[u] += 1
                if parent[u] == 0xFFFFFFFF:
                    break
                u = int(parent[u])
        cap = int(rng.integers(1, n + 2))
        want = sorted(int(size[v]) for v in range(n)
                      if size[v] <= cap and (parent[v] == 0xFFFFFFFF or size[parent[v]] > cap))
        assert sorted(bench.coherent_blocks(parent, cap).tolist()) == want, trial


def test_coherent_block_members_hand_tree(bench):
    # 0 is the root; 1 and 2 its children; 3, 4 under 1; 5 under 2; 6 under 5
    N = 0xFFFFFFFF
    parent = np.array([N, 0, 0, 1, 1, 2, 5], np.uint32)
    blocks = bench.coherent_block_members(parent, 3)
    got = sorted(b.tolist() for b in blocks)
    # subtree(1) = {1, 3, 4} and subtree(2) = {2, 5, 6}: each of size 3 under a root of size 7
    assert got == [[1, 3, 4], [2, 5, 6]]
    # sizes agree with coherent_blocks on random trees, and blocks are disjoint
    rng = np.random.default_rng(4)
    for trial in range(20):
        n = int(rng.integers(2, 300))
        par = np.full(n, N, np.uint32)
        for v in range(1, n):
            par[v] = rng.integers(0, v)
        cap = int(rng.integers(1, 40))
        mem = bench.coherent_block_members(par, cap)
        assert sorted(len(b) for b in mem) == sorted(bench.coherent_blocks(par, cap).tolist())
        allp = np.concatenate(mem) if mem else np.zeros(0, np.int64)
        assert len(set(allp.tolist())) == len(allp)
        for b in mem:  # preorder from the block's root: every point's parent precedes it
            pos = {int(v): i for i, v in enumerate(b)}
            for v in b[1:]:
                assert int(par[v]) in pos and pos[int(par[v])] < pos[int(v)]


def test_lockstep_stats_hand_example(bench):
    import torch
    t = lambda *v: torch.tensor(v, dtype=torch.long)  # noqa: E731
    V = [t(1, 2, 3, 4), t(3, 4, 5, 6), t(4, 6, 7, 8)]
    W = [t(2, 3), t(3, 5, 6), t(6, 8)]
    st = bench.lockstep_stats(V, W, repeat=2)
    # union {1..8}: density 12 / (3 * 8)
    assert st["union"] == 8 and st["density"] == pytest.approx(12 / 24)
    assert st["mean_V"] == pytest.approx(4.0)
    # adjacent pairs: (W0, W1) share {3}, (W1, W2) share {6}; mean sizes 2.5 and 2.5
    assert st["shared_exp_1_10"] == pytest.approx(2 / 5)
    # targets seen by >= 2 points: 3 (x2), 4 (x3), 6 (x2): 7 of 12 evaluations
    assert st["evals_to_targets_seen_by_2_or_more"] == pytest.approx(7 / 12)
    # identical visited sets: density 1
    assert bench.lockstep_stats([t(1, 2), t(1, 2)], [t(1), t(1)])["density"] == pytest.approx(1.0)
