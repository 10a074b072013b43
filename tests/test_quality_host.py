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
