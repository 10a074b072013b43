"""Independent characterisations used to pin the oracle and to check the HIP
path at sizes the oracle cannot finish.

Nothing here calls the oracle: every check recomputes what it needs in numpy
from definitions (exact integer or float64 distances, set algebra, sorting).
Integer-valued inputs make every distance exact, so the checks agree with the
oracle's arithmetic bit for bit on them.
"""
from __future__ import annotations

import numpy as np

NONE = 0xFFFFFFFF


def exact_dist_matrix(x: np.ndarray, metric: str = "l2") -> np.ndarray:
    """All-pairs distances in float64 (exact for small-integer data)."""
    xf = x.astype(np.float64)
    if metric == "cosine":
        return (1.0 - (xf[:, None, :] * xf[None, :, :]).sum(-1))
    if np.issubdtype(x.dtype, np.integer) or np.all(xf == np.rint(xf)):
        xi = x.astype(np.int64)   # integer data: exact
        return ((xi[:, None, :] - xi[None, :, :]) ** 2).sum(-1).astype(np.float64)
    return ((xf[:, None, :] - xf[None, :, :]) ** 2).sum(-1)


def f32_mul(alpha: float, d: float) -> float:
    """alpha * d rounded once to float32 (the prune's scaled distance)."""
    return float(np.float32(alpha) * np.float32(d))


# --------------------------------------------------------------------------
# SAT tree: the classic SAT is determined node by node by three conditions.
# --------------------------------------------------------------------------

def check_sat(DM: np.ndarray, root: int, parent: np.ndarray) -> None:
    """Raise AssertionError unless `parent` is the classic SAT of the points
    under DM rooted at `root`:
      * a tree spanning every point, rooted at `root`;
      * for each node a with descendants S and children N (ranked by
        (d(v,a), v)): every child c beats every earlier child b
        (d(c,a) < d(c,b)); every non-child v has an earlier child b with
        d(v,b) <= d(v,a); and v lies below the child minimising (d(v,b), b).
    The first two conditions fix N as the greedy acceptance set; the third
    fixes the bags."""
    n = DM.shape[0]
    assert parent[root] == NONE
    children = [[] for _ in range(n)]
    for v in range(n):
        if v == root:
            continue
        p = int(parent[v])
        assert p != NONE and 0 <= p < n, f"node {v} has no parent"
        children[p].append(v)
    # reachability and descendant sets (iterative post-order)
    order = []
    stack = [root]
    seen = np.zeros(n, bool)
    while stack:
        a = stack.pop()
        assert not seen[a], "cycle"
        seen[a] = True
        order.append(a)
        stack.extend(children[a])
    assert seen.all(), "not spanning"
    desc = [None] * n
    for a in reversed(order):
        s = set()
        for c in children[a]:
            s.add(c)
            s |= desc[c]
        desc[a] = s
    for a in range(n):
        S = desc[a]
        if not S:
            continue
        N = children[a]
        rank = {v: r for r, v in enumerate(sorted(S, key=lambda v: (DM[v, a], v)))}
        Ns = sorted(N, key=lambda v: rank[v])
        for i, c in enumerate(Ns):
            for b in Ns[:i]:
                assert DM[c, a] < DM[c, b], f"child {c} of {a} occluded by {b}"
        for v in S:
            if v in N:
                continue
            earlier = [b for b in Ns if rank[b] < rank[v]]
            assert any(DM[v, b] <= DM[v, a] for b in earlier), \
                f"{v} should have been a neighbour of {a}"
            best = min(Ns, key=lambda b: (DM[v, b], b))
            assert v in desc[best], f"{v} not in the bag of its closest neighbour"


def tree_edges(parents: np.ndarray) -> set:
    T, n = parents.shape
    e = set()
    for t in range(T):
        for v in range(n):
            p = int(parents[t, v])
            if p != NONE:
                e.add((p, v))
                e.add((v, p))
    return e


def csr_edges(off, ids) -> set:
    e = set()
    for v in range(len(off) - 1):
        for u in ids[int(off[v]):int(off[v + 1])]:
            e.add((v, int(u)))
    return e


def csr_rows_sorted_unique(off, ids) -> bool:
    for v in range(len(off) - 1):
        r = ids[int(off[v]):int(off[v + 1])]
        if r.size and not np.all(np.diff(r.astype(np.int64)) > 0):
            return False
    return True


# --------------------------------------------------------------------------
# Beam search: a declarative restatement.  Before expansion i the beam holds
# the ef best (by key) of V_i = roots u N(E_0..E_{i-1}); the vertex expanded
# is the best beam entry not yet expanded; the search ends when none is left.
# --------------------------------------------------------------------------

def check_beam(dq: np.ndarray, off, ids, roots, ef: int, E, V, beam_ids) -> None:
    """dq[v] = distance of the query to vertex v."""
    key = lambda v: (dq[v], v)  # noqa: E731
    visited = []
    vset = set()
    for r in roots:
        r = int(r)
        if r not in vset:
            vset.add(r)
            visited.append(r)
    expanded = []
    eset = set()
    while True:
        top = sorted(vset, key=key)[:ef]
        nxt = [v for v in top if v not in eset]
        if not nxt:
            break
        v = nxt[0]
        assert len(expanded) < len(E) and int(E[len(expanded)]) == v, \
            f"expansion {len(expanded)}: expected {v}"
        expanded.append(v)
        eset.add(v)
        for u in ids[int(off[v]):int(off[v + 1])]:
            u = int(u)
            if u not in vset:
                vset.add(u)
                visited.append(u)
    assert len(expanded) == len(E), "extra expansions"
    assert set(int(v) for v in V) == vset and len(V) == len(vset)
    assert [int(v) for v in beam_ids] == sorted(vset, key=key)[:ef]


# --------------------------------------------------------------------------
# Occlusion prune: sorted, at most R, occlusion between kept pairs never
# fires, and every dropped candidate ranked before the R-th kept one (all of
# them when fewer than R are kept) is killed by an earlier kept one.  These
# three properties fix the greedy result.
# --------------------------------------------------------------------------

def check_prune(DM_p: dict, DM: np.ndarray, cand: list, kept: list, R: int,
                alpha: float, f32: bool = True) -> None:
    """cand: candidate ids; DM_p[c] = d(p, c); DM = pairwise distances."""
    key = lambda c: (DM_p[c], c)  # noqa: E731
    C = sorted(set(cand), key=key)
    rank = {c: i for i, c in enumerate(C)}
    kept = [int(k) for k in kept]
    assert len(kept) <= R and len(set(kept)) == len(kept)
    assert all(k in rank for k in kept)
    assert kept == sorted(kept, key=key)

    def kills(a, c):
        if f32:
            return f32_mul(alpha, DM[a, c]) <= DM_p[c]
        return alpha * DM[a, c] <= DM_p[c]

    for i, a in enumerate(kept):
        for c in kept[i + 1:]:
            assert not kills(a, c), f"kept {c} is occluded by kept {a}"
    limit = rank[kept[-1]] if len(kept) == R else len(C)
    kset = set(kept)
    for c in C[:limit]:
        if c in kset:
            continue
        assert any(kills(a, c) for a in kept if rank[a] < rank[c]), \
            f"dropped {c} is not occluded"


def hsp_neighbours(DM: np.ndarray, p: int) -> list:
    """Half-space proximal neighbours of p (Chavez et al. 2005) with the
    non-strict boundary: repeatedly take the closest remaining point c and
    discard every remaining v with d(c, v) <= d(p, v)."""
    rest = [v for v in range(DM.shape[0]) if v != p]
    out = []
    while rest:
        c = min(rest, key=lambda v: (DM[p, v], v))
        out.append(c)
        rest = [v for v in rest if v != c and not (DM[c, v] <= DM[p, v])]
    return out


def fnv1a64_graph(nbrs, cnt, parent0, roots, T: int) -> int:
    """FNV-1a-64 of the graph's little-endian byte image (n, R, T, rows,
    parent0, roots), written from the byte layout alone."""
    n, R = nbrs.shape
    parts = [np.uint64(n).tobytes(), np.uint32(R).tobytes(), np.uint32(T).tobytes()]
    for p in range(n):
        c = int(cnt[p])
        parts.append(np.uint32(c).tobytes())
        parts.append(np.ascontiguousarray(nbrs[p, :c], dtype="<u4").tobytes())
    parts.append(np.ascontiguousarray(parent0, dtype="<u4").tobytes())
    parts.append(np.ascontiguousarray(roots, dtype="<u4").tobytes())
    h = 0xCBF29CE484222325
    for b in b"".join(parts):
        h ^= b
        h = (h * 0x100000001B3) & 0xFFFFFFFFFFFFFFFF
    return h


def knn_exact(x: np.ndarray, q: np.ndarray, k: int, metric: str = "l2"):
    """Brute-force k nearest in float64 (ties by id)."""
    xf = x.astype(np.float64)
    qf = q.astype(np.float64)
    if metric == "cosine":
        d = 1.0 - qf @ xf.T
    else:
        d = (qf * qf).sum(1)[:, None] + (xf * xf).sum(1)[None, :] - 2 * qf @ xf.T
    idx = np.lexsort((np.broadcast_to(np.arange(x.shape[0]), d.shape), d), axis=1)[:, :k]
    return idx, np.take_along_axis(d, idx, 1)


# --------------------------------------------------------------------------
# Work counts (Sec. 2: every distance evaluation counts), restated from the
# finished structures that the characterisations above pin, per candidate
# rather than by replaying the loops that produced them.
# --------------------------------------------------------------------------

def prune_pair_count(DM_p: dict, DM: np.ndarray, cand: list, kept: list, R: int, alpha: float) -> int:
    """Pair distances of the lazy greedy prune, from its kept list: the
    kept candidates test later live ones, except the R-th kept, after which
    the prune stops.  So each candidate c is tested by the testing kept
    candidates ranked before it, in rank order, up to and including the first
    one whose float32-scaled distance reaches d(p, c) (that one kills it)."""
    key = lambda c: (DM_p[c], c)  # noqa: E731
    C = sorted(set(int(c) for c in cand), key=key)
    rank = {c: i for i, c in enumerate(C)}
    kept = [int(k) for k in kept]
    testers = kept[:-1] if len(kept) == R else kept
    total = 0
    for c in C:
        for a in testers:
            if rank[a] >= rank[c]:
                break
            total += 1
            if f32_mul(alpha, DM[a, c]) <= DM_p[c]:
                break
    return total


def sat_eval_count(DM: np.ndarray, root: int, parent: np.ndarray) -> int:
    """Distance evaluations of the classic SAT construction, from the tree:
    at every node a with descendants S and children N ranked by (d(v,a), v),
    |S| distances to a; each v of S is tested against the children ranked
    before it, in that order, up to and including the first b with
    d(v,b) <= d(v,a) (all of them when v is a child); and each descendant
    that is not a child takes its distance to every child (closest-child
    assignment)."""
    n = DM.shape[0]
    children = [[] for _ in range(n)]
    for v in range(n):
        if v != root:
            children[int(parent[v])].append(v)
    desc = [None] * n
    order, stack = [], [root]
    while stack:
        a = stack.pop()
        order.append(a)
        stack.extend(children[a])
    for a in reversed(order):
        s = set()
        for c in children[a]:
            s.add(c)
            s |= desc[c]
        desc[a] = s
    total = 0
    for a in range(n):
        S = desc[a]
        if not S:
            continue
        ranked = sorted(S, key=lambda v: (DM[v, a], v))
        rank = {v: r for r, v in enumerate(ranked)}
        N = sorted(children[a], key=lambda v: rank[v])
        Nset = set(N)
        total += len(S)
        for v in S:
            for b in N:
                if rank[b] >= rank[v]:
                    break
                total += 1
                if DM[v, b] <= DM[v, a]:
                    break
        total += (len(S) - len(N)) * len(N)
    return total


def finalize_eval_count(DM: np.ndarray, rows: np.ndarray, cnt: np.ndarray, g: np.ndarray, gc: np.ndarray,
                        R: int, alpha: float, reprune_all: bool = False) -> int:
    """Finalize's distance evaluations, from its input rows and output graph:
    one distance per distinct symmetrised candidate of every point, plus the
    prune's pair count (from the point's output row) where the candidates
    exceed R or every row is re-pruned."""
    n = rows.shape[0]
    cand = [set(int(u) for u in rows[p, :cnt[p]]) for p in range(n)]
    for u in range(n):
        for v in rows[u, :cnt[u]]:
            cand[int(v)].add(u)
    total = 0
    for p in range(n):
        C = sorted(cand[p])
        total += len(C)
        if len(C) > R or reprune_all:
            total += prune_pair_count({c: DM[p, c] for c in C}, DM, C, g[p, :gc[p]].tolist(), R, alpha)
    return total
