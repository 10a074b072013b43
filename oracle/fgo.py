"""ctypes binding of the CPU oracle (TEST INFRASTRUCTURE ONLY).

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this module.  The product library never does.
Build with :func:`build` (plain gcc, no GPU needed).
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB = os.path.join(HERE, "libfgo.so")
NONE = 0xFFFFFFFF


def build(sanitize: str | None = None, out: str | None = None) -> str:
    """Compile fgo.c into a shared library (optionally with a host sanitizer)."""
    target = out or LIB
    cmd = ["gcc", "-O2", "-std=c11", "-Wall", "-ffp-contract=off",
           "-fno-fast-math", "-fPIC", "-shared", "-pthread"]
    if sanitize:
        cmd += [f"-fsanitize={sanitize}", "-fno-omit-frame-pointer", "-g"]
    cmd += ["-o", target, os.path.join(HERE, "fgo.c"), "-lm"]
    subprocess.run(cmd, check=True)
    return target


class _Data(C.Structure):
    _fields_ = [("x", C.c_void_p), ("n", C.c_int64), ("d", C.c_int32),
                ("dtype", C.c_int32), ("metric", C.c_int32), ("prec", C.c_int32),
                ("stride", C.c_int64)]


class _Params(C.Structure):
    _fields_ = [("T", C.c_uint32), ("ef_h", C.c_uint32), ("R", C.c_uint32),
                ("alpha", C.c_float), ("B", C.c_uint32),
                ("reprune_all", C.c_uint32), ("threads", C.c_uint32)]


class _Counters(C.Structure):
    _fields_ = [("scaffold_evals", C.c_uint64), ("harvest_evals", C.c_uint64),
                ("prune_evals", C.c_uint64), ("finalize_evals", C.c_uint64),
                ("expansions", C.c_uint64), ("t_scaffold", C.c_double),
                ("t_harvest", C.c_double), ("t_merge", C.c_double),
                ("t_finalize", C.c_double)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB):
            build()
        L = C.CDLL(LIB)
        P = C.c_void_p
        L.fgo_splitmix64.restype = C.c_uint64
        L.fgo_splitmix64.argtypes = [C.c_uint64, C.c_uint64]
        L.fgo_roots.argtypes = [C.c_uint64, C.c_int64, C.c_uint32, P]
        L.fgo_dist.restype = C.c_double
        L.fgo_dist.argtypes = [P, C.c_int64, C.c_int64]
        L.fgo_dist_vec.restype = C.c_double
        L.fgo_dist_vec.argtypes = [P, P, C.c_int64]
        L.fgo_fnv1a64.restype = C.c_uint64
        L.fgo_fnv1a64.argtypes = [P, C.c_size_t]
        L.fgo_sat_tree.argtypes = [P, C.c_uint32, P, P]
        L.fgo_scaffold_csr.restype = C.c_int64
        L.fgo_scaffold_csr.argtypes = [C.c_int64, C.c_uint32, P, P, P]
        L.fgo_beam.restype = C.c_int64
        L.fgo_beam.argtypes = [P, P, C.c_int64, P, P, P, C.c_uint32, C.c_uint32,
                               P, P, P, P, P, P, P, P]
        L.fgo_prune.restype = C.c_int32
        L.fgo_prune.argtypes = [P, C.c_int64, P, P, C.c_uint32, C.c_uint32,
                                C.c_float, P, P]
        L.fgo_harvest_block.argtypes = [P, P, P, P, P, C.c_uint32, P, C.c_int64,
                                        P, P, P]
        L.fgo_merge_block.restype = C.c_int64
        L.fgo_merge_block.argtypes = [C.c_int64, P, P, P, P, C.c_uint32,
                                      C.c_uint32, C.c_uint32, P, P, C.c_uint64]
        L.fgo_finalize.argtypes = [P, P, P, P, P, P, P]
        L.fgo_graph_hash.restype = C.c_uint64
        L.fgo_graph_hash.argtypes = [C.c_int64, C.c_uint32, C.c_uint32, P, P, P, P]
        L.fgo_build_graph.argtypes = [P, C.c_uint64, P, P, P, P, P, P, P]
        L.fgo_search.argtypes = [P, P, P, C.c_uint32, P, P, C.c_uint32, P,
                                 C.c_int64, C.c_uint32, C.c_uint32, C.c_uint32,
                                 P, P, P]
        L.fgo_knn_brute.argtypes = [P, P, C.c_int64, C.c_uint32, C.c_uint32, P, P]
        _lib = L
    return _lib


def _p(a):
    return None if a is None else a.ctypes.data_as(C.c_void_p)


class Data:
    """A data matrix as the oracle sees it.  prec=0: float32 in the declared
    order (or exact integers for uint8); prec=1: float64."""

    def __init__(self, x: np.ndarray, metric: str = "l2", prec: int = 0):
        x = np.ascontiguousarray(x)
        if x.dtype == np.float32:
            dt = 0
        elif x.dtype == np.uint8:
            dt = 1
        else:
            raise TypeError(x.dtype)
        self.x = x
        self.n, self.d = x.shape
        self.metric = metric
        self.prec = prec
        self.s = _Data(x.ctypes.data, self.n, self.d, dt,
                       1 if metric == "cosine" else 0, prec, x.strides[0])

    @property
    def ref(self):
        return C.byref(self.s)


def params(T, ef_h, R, alpha=1.2, B=1, reprune_all=0, threads=1):
    return _Params(T, ef_h, R, alpha, B, reprune_all, threads)


def splitmix64(seed: int, k: int) -> int:
    return lib().fgo_splitmix64(seed, k)


def roots(seed: int, n: int, T: int) -> np.ndarray:
    r = np.zeros(T, np.uint32)
    assert lib().fgo_roots(seed, n, T, _p(r)) == 0
    return r


def dist(D: Data, i: int, j: int) -> float:
    return lib().fgo_dist(D.ref, i, j)


def dist_vec(D: Data, q: np.ndarray, j: int) -> float:
    q = np.ascontiguousarray(q, dtype=D.x.dtype)
    return lib().fgo_dist_vec(D.ref, _p(q), j)


def fnv1a64(b: bytes) -> int:
    buf = np.frombuffer(b, dtype=np.uint8).copy() if b else np.zeros(1, np.uint8)
    return lib().fgo_fnv1a64(_p(buf), len(b))


def sat_tree(D: Data, root: int):
    parent = np.zeros(D.n, np.uint32)
    ev = C.c_uint64(0)
    assert lib().fgo_sat_tree(D.ref, root, _p(parent), C.byref(ev)) == 0
    return parent, ev.value


def scaffold_csr(n: int, parents: np.ndarray):
    parents = np.ascontiguousarray(parents, dtype=np.uint32)
    T = parents.size // n
    off = np.zeros(n + 1, np.uint64)
    ids = np.zeros(max(1, 2 * T * (n - 1)), np.uint32)
    nnz = lib().fgo_scaffold_csr(n, T, _p(parents), _p(off), _p(ids))
    assert nnz >= 0
    return off, ids[:nnz].copy()


def scaffold(D: Data, seed: int, T: int):
    """Roots, per-tree parent arrays (T x n) and S0 as CSR."""
    r = roots(seed, D.n, T)
    parents = np.zeros((T, D.n), np.uint32)
    ev = 0
    for t in range(T):
        parents[t], e = sat_tree(D, int(r[t]))
        ev += e
    off, ids = scaffold_csr(D.n, parents)
    return r, parents, off, ids, ev


def beam(D: Data, off, ids, roots_, ef: int, p: int | None = None, q=None):
    n = D.n
    bi = np.zeros(max(ef, 1), np.uint32)
    bd = np.zeros(max(ef, 1), np.float64)
    bn = C.c_uint32(0)
    Ei = np.zeros(n, np.uint32)
    Ed = np.zeros(n, np.float64)
    En = C.c_uint32(0)
    Vi = np.zeros(n, np.uint32)
    Vn = C.c_uint32(0)
    qq = None if q is None else np.ascontiguousarray(q, dtype=D.x.dtype)
    ev = lib().fgo_beam(D.ref, _p(qq), -1 if p is None else p, _p(off), _p(ids),
                        _p(roots_), len(roots_), ef, _p(bi), _p(bd), C.byref(bn),
                        _p(Ei), _p(Ed), C.byref(En), _p(Vi), C.byref(Vn))
    assert ev >= 0
    return dict(beam_ids=bi[:bn.value], beam_d=bd[:bn.value],
                E_ids=Ei[:En.value], E_d=Ed[:En.value], V=Vi[:Vn.value],
                evals=ev)


def prune(D: Data, p: int, cand_ids, cand_d, R: int, alpha: float):
    cand_ids = np.ascontiguousarray(cand_ids, dtype=np.uint32)
    cand_d = np.ascontiguousarray(cand_d, dtype=np.float64)
    out = np.zeros(max(R, 1), np.uint32)
    pe = C.c_uint64(0)
    k = lib().fgo_prune(D.ref, p, _p(cand_ids), _p(cand_d), len(cand_ids), R,
                        alpha, _p(out), C.byref(pe))
    assert k >= 0
    return out[:k].copy(), pe.value


def harvest_block(D: Data, off, ids, roots_, P: _Params, b: int, rows, cnt,
                  order=None):
    cnt_ = _Counters()
    o = None if order is None else np.ascontiguousarray(order, dtype=np.uint32)
    rc = lib().fgo_harvest_block(D.ref, _p(off), _p(ids), _p(roots_), C.byref(P),
                                 b, _p(o), 0 if o is None else len(o), _p(rows),
                                 _p(cnt), C.byref(cnt_))
    assert rc == 0
    return cnt_.as_dict()


def merge_block(n, off, ids, rows, cnt, R, B, b):
    cap = int(ids.size + 2 * int(cnt.sum()) + 1)
    off2 = np.zeros(n + 1, np.uint64)
    ids2 = np.zeros(cap, np.uint32)
    nnz = lib().fgo_merge_block(n, _p(off), _p(ids), _p(rows), _p(cnt), R, B, b,
                                _p(off2), _p(ids2), cap)
    assert nnz >= 0
    return off2, ids2[:nnz].copy()


def finalize(D: Data, rows, cnt, P: _Params):
    g = np.full((D.n, P.R), NONE, np.uint32)
    gc = np.zeros(D.n, np.uint32)
    c = _Counters()
    assert lib().fgo_finalize(D.ref, _p(rows), _p(cnt), C.byref(P), _p(g), _p(gc),
                              C.byref(c)) == 0
    return g, gc, c.as_dict()


def graph_hash(g, gc, parent0, roots_, T: int) -> int:
    n, R = g.shape
    return lib().fgo_graph_hash(n, R, T, _p(g), _p(gc), _p(parent0), _p(roots_))


def build_graph(D: Data, seed: int, P: _Params):
    n = D.n
    g = np.full((n, P.R), NONE, np.uint32)
    gc = np.zeros(n, np.uint32)
    parent0 = np.zeros(n, np.uint32)
    r = np.zeros(P.T, np.uint32)
    c = _Counters()
    h = C.c_uint64(0)
    rc = lib().fgo_build_graph(D.ref, seed, C.byref(P), _p(g), _p(gc), _p(parent0),
                               _p(r), C.byref(c), C.byref(h))
    assert rc == 0
    return dict(nbrs=g, cnt=gc, parent0=parent0, roots=r, counters=c.as_dict(),
                hash=h.value)


def search(D: Data, graph: dict, queries: np.ndarray, k: int, L: int,
           threads: int = 1):
    q = np.ascontiguousarray(queries, dtype=D.x.dtype)
    nq = q.shape[0]
    ids = np.zeros((nq, k), np.uint32)
    dd = np.zeros((nq, k), np.float64)
    ev = np.zeros(nq, np.uint32)
    g = graph["nbrs"]
    rc = lib().fgo_search(D.ref, _p(g), _p(graph["cnt"]), g.shape[1],
                          _p(graph["parent0"]), _p(graph["roots"]),
                          len(graph["roots"]), _p(q), nq, k, L, threads, _p(ids),
                          _p(dd), _p(ev))
    assert rc == 0
    return ids, dd, ev


def knn_brute(D: Data, queries: np.ndarray, k: int, threads: int = 1):
    q = np.ascontiguousarray(queries, dtype=D.x.dtype)
    nq = q.shape[0]
    ids = np.zeros((nq, k), np.uint32)
    dd = np.zeros((nq, k), np.float64)
    assert lib().fgo_knn_brute(D.ref, _p(q), nq, k, threads, _p(ids), _p(dd)) == 0
    return ids, dd


def recall_at_k(found_d: np.ndarray, true_d: np.ndarray) -> float:
    """Tie-aware recall: a returned result counts when its distance is no
    larger than the true k-th distance."""
    kth = true_d[:, -1:]
    return float(np.mean(found_d <= kth))
