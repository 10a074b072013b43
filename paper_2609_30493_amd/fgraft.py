"""Thin Python binding of libfgraft.so (the C-ABI in include/fgraft.h).

Argument marshalling only: every step runs in the library's HIP kernels.
PyTorch supplies device memory and the stream.  If the library has not been
built, every call raises -- there is no fallback.
"""
from __future__ import annotations

import ctypes as C
import os

import torch

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libfgraft.so")
NONE = 0xFFFFFFFF

FG_OK, FG_EINVAL, FG_ENOMEM, FG_EHIP, FG_ECAPACITY, FG_EUNSUPPORTED = 0, -1, -2, -3, -4, -5
F32, U8 = 0, 1
L2SQ, COSINE = 0, 1


class FgError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"fgraft error {code}: {msg}")
        self.code = code


class fg_data(C.Structure):
    _fields_ = [("x_dev", C.c_void_p), ("n", C.c_int64), ("d", C.c_int32),
                ("dtype", C.c_int32), ("metric", C.c_int32), ("reserved", C.c_int32),
                ("row_stride_bytes", C.c_int64)]


class fg_params(C.Structure):
    _fields_ = [("T", C.c_uint32), ("ef_h", C.c_uint32), ("R", C.c_uint32),
                ("alpha", C.c_float), ("B", C.c_uint32), ("reprune_all", C.c_uint32),
                ("beam_table_slots", C.c_uint32), ("screen", C.c_uint32),
                ("waves_per_cu", C.c_uint32), ("lanes_per_row", C.c_uint32)]


SCREEN_NONE, SCREEN_BF16, SCREEN_FP8E4M3, SCREEN_BF16_PRUNE, SCREEN_INT8 = 0, 1, 2, 3, 4


class fg_csr(C.Structure):
    _fields_ = [("off_dev", C.c_void_p), ("ids_dev", C.c_void_p), ("n", C.c_int64),
                ("nnz", C.c_uint64), ("cap", C.c_uint64)]


class fg_graph(C.Structure):
    _fields_ = [("nbrs_dev", C.c_void_p), ("cnt_dev", C.c_void_p),
                ("spine_parent_dev", C.c_void_p), ("roots_dev", C.c_void_p),
                ("n", C.c_int64), ("R", C.c_uint32), ("T", C.c_uint32)]


class fg_counters(C.Structure):
    _fields_ = [("scaffold_evals", C.c_uint64), ("harvest_evals", C.c_uint64),
                ("prune_evals", C.c_uint64), ("expansions", C.c_uint64),
                ("finalize_evals", C.c_uint64), ("spilled_queries", C.c_uint64),
                ("screen_rejected", C.c_uint64), ("prune_rechecks", C.c_uint64)]

    def as_dict(self):
        return {k: int(getattr(self, k)) for k, _ in self._fields_}


class fg_timings(C.Structure):
    _fields_ = [("scaffold_ms", C.c_float), ("harvest_ms", C.c_float),
                ("merge_ms", C.c_float), ("finalize_ms", C.c_float), ("screen_ms", C.c_float),
                ("block_harvest_ms", C.c_float * 64), ("block_evals", C.c_uint64 * 64),
                ("nblocks", C.c_uint32)]

    def as_dict(self):
        nb = int(self.nblocks)
        return dict(scaffold_ms=self.scaffold_ms, harvest_ms=self.harvest_ms,
                    merge_ms=self.merge_ms, finalize_ms=self.finalize_ms, screen_ms=self.screen_ms,
                    block_harvest_ms=list(self.block_harvest_ms)[:nb],
                    block_evals=[int(v) for v in list(self.block_evals)[:nb]])


_lib = None
P = C.c_void_p
_SIGS = {
    "fg_last_error": (C.c_char_p, []),
    "fg_workspace_size": (C.c_size_t, [P, P]),
    "fg_roots": (C.c_int, [C.c_uint64, C.c_int64, C.c_uint32, P]),
    "fg_build_scaffold": (C.c_int, [P, P, C.c_uint32, P, P, P, C.c_size_t, P, P]),
    "fg_harvest_block": (C.c_int, [P, P, P, P, C.c_uint32, P, P, P, C.c_size_t, P, P]),
    "fg_merge_block": (C.c_int, [P, P, P, P, C.c_uint32, P, P, C.c_size_t, P]),
    "fg_finalize": (C.c_int, [P, P, P, P, P, P, C.c_size_t, P, P]),
    "fg_build_graph": (C.c_int, [P, C.c_uint64, P, P, P, C.c_size_t, P, P, P]),
    "fg_build_graph_log": (C.c_int, [P, C.c_uint64, P, P, P, C.c_size_t, P, P, P, P]),
    "fg_search": (C.c_int, [P, P, P, C.c_int64, C.c_uint32, C.c_uint32, P, P, P, P,
                            C.c_size_t, P]),
    "fg_search_noalloc": (C.c_int, [P, P, P, C.c_int64, C.c_uint32, C.c_uint32, P, P, P, P]),
    "fg_search_noalloc_scratch_bytes": (C.c_size_t, []),
    "fg_graph_hash": (C.c_int, [P, P, P]),
    "fg_sync_status": (C.c_int, [P, P]),
    "fg_autotune": (C.c_int, [P, P, C.c_char_p, P, C.c_size_t, P, P]),
    "fg_batched_workspace_size": (C.c_size_t, [P, P, C.c_uint32]),
    "fg_build_graph_batched": (C.c_int, [P, P, P, C.c_uint32, P, P, C.c_size_t, P, C.c_int, P]),
    "fg_screen_row_bytes": (C.c_int64, [C.c_int32, C.c_uint32]),
    "fg_screen_copy": (C.c_int, [P, C.c_uint32, P, P, P, P, P]),
    "fg_leaf_knn_workspace_size": (C.c_size_t, [P]),
    "fg_leaf_knn": (C.c_int, [P, C.c_uint32, C.c_uint32, C.c_int, P, P, P, C.c_size_t, P]),
}


def lib():
    """Load libfgraft.so; raise if it is missing (never fall back)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is not built: run __graft_entry__.build()")
        L = C.CDLL(LIB_PATH)
        for name, (res, args) in _SIGS.items():
            f = getattr(L, name, None)
            if f is not None:
                f.restype = res
                f.argtypes = args
        _lib = L
    return _lib


def exported_symbols():
    L = lib()
    return [n for n in _SIGS if getattr(L, n, None) is not None]


def _check(rc: int):
    if rc != FG_OK:
        raise FgError(rc, lib().fg_last_error().decode())


def _ptr(t):
    return None if t is None else C.c_void_p(t.data_ptr())


def _stream(stream):
    if stream is None:
        stream = torch.cuda.current_stream()
    return C.c_void_p(stream.cuda_stream)


# The C structures hold raw device pointers; each one keeps a reference to
# the tensors it points into (attribute `_keep`), so a temporary passed to a
# constructor stays allocated as long as the structure does.

def make_data(x: torch.Tensor, metric: str = "l2") -> fg_data:
    if x.dim() != 2 or not x.is_cuda or x.stride(1) != 1:
        raise ValueError("x must be a 2-D row-major device tensor")
    if x.dtype == torch.float32:
        dt = F32
    elif x.dtype == torch.uint8:
        dt = U8
    else:
        raise TypeError(x.dtype)
    s = fg_data(x.data_ptr(), x.shape[0], x.shape[1], dt,
                COSINE if metric == "cosine" else L2SQ, 0,
                x.stride(0) * x.element_size())
    s._keep = (x,)
    return s


def make_params(T, ef_h, R, alpha=1.2, B=1, reprune_all=0, beam_table_slots=0, screen=0,
                waves_per_cu=0, lanes_per_row=0) -> fg_params:
    return fg_params(T, ef_h, R, alpha, B, reprune_all, beam_table_slots, screen, waves_per_cu, lanes_per_row)


def workspace_size(data: fg_data, params: fg_params) -> int:
    return int(lib().fg_workspace_size(C.byref(data), C.byref(params)))


def alloc_workspace(data: fg_data, params: fg_params, device="cuda") -> torch.Tensor:
    nb = workspace_size(data, params)
    return torch.empty(nb + 256, dtype=torch.uint8, device=device)


def _ws(ws: torch.Tensor):
    base = ws.data_ptr()
    pad = (-base) % 256
    return C.c_void_p(base + pad), ws.numel() - pad


def roots(seed: int, n: int, T: int):
    import numpy as np
    r = np.zeros(T, np.uint32)
    _check(lib().fg_roots(seed, n, T, r.ctypes.data_as(C.c_void_p)))
    return r


def csr(off: torch.Tensor, ids: torch.Tensor, nnz: int | None = None) -> fg_csr:
    for t in (off, ids):
        if not t.is_cuda or not t.is_contiguous():
            raise ValueError("CSR arrays must be contiguous device tensors")
    n = off.numel() - 1
    s = fg_csr(off.data_ptr(), ids.data_ptr(), n,
               int(nnz if nnz is not None else ids.numel()), ids.numel())
    s._keep = (off, ids)
    return s


def harvest_block(data: fg_data, Sb: fg_csr, roots_dev: torch.Tensor, params: fg_params,
                  b: int, rows: torch.Tensor, cnt: torch.Tensor, ws: torch.Tensor,
                  stream=None, counters: bool = True):
    c = fg_counters()
    wp, wn = _ws(ws)
    _check(lib().fg_harvest_block(C.byref(data), C.byref(Sb), _ptr(roots_dev),
                                  C.byref(params), b, _ptr(rows), _ptr(cnt), wp, wn,
                                  _stream(stream), C.byref(c) if counters else None))
    return c.as_dict()


def build_scaffold(data: fg_data, roots_dev: torch.Tensor, T: int, S0: fg_csr,
                   tree_parent: torch.Tensor | None, ws: torch.Tensor, stream=None):
    c = fg_counters()
    wp, wn = _ws(ws)
    _check(lib().fg_build_scaffold(C.byref(data), _ptr(roots_dev), T, C.byref(S0),
                                   _ptr(tree_parent), wp, wn, _stream(stream), C.byref(c)))
    return c.as_dict()


def merge_block(Sb: fg_csr, rows: torch.Tensor, cnt: torch.Tensor, params: fg_params, b: int,
                Sb1: fg_csr, ws: torch.Tensor, stream=None):
    wp, wn = _ws(ws)
    _check(lib().fg_merge_block(C.byref(Sb), _ptr(rows), _ptr(cnt), C.byref(params), b,
                                C.byref(Sb1), wp, wn, _stream(stream)))
    return int(Sb1.nnz)


def make_graph(nbrs, cnt, spine_parent, roots_dev, T: int) -> fg_graph:
    for t in (nbrs, cnt, spine_parent, roots_dev):
        if not t.is_cuda or not t.is_contiguous():
            raise ValueError("graph arrays must be contiguous device tensors")
    if cnt.numel() != nbrs.shape[0] or spine_parent.numel() != nbrs.shape[0] or roots_dev.numel() < T:
        raise ValueError("graph array sizes do not match")
    s = fg_graph(nbrs.data_ptr(), cnt.data_ptr(), spine_parent.data_ptr(),
                 roots_dev.data_ptr(), nbrs.shape[0], nbrs.shape[1], T)
    s._keep = (nbrs, cnt, spine_parent, roots_dev)
    return s


def finalize(data: fg_data, rows, cnt, params: fg_params, graph: fg_graph, ws, stream=None):
    c = fg_counters()
    wp, wn = _ws(ws)
    _check(lib().fg_finalize(C.byref(data), _ptr(rows), _ptr(cnt), C.byref(params),
                             C.byref(graph), wp, wn, _stream(stream), C.byref(c)))
    return c.as_dict()


def build_graph(data: fg_data, seed: int, params: fg_params, graph: fg_graph, ws,
                stream=None, timings: bool = False):
    c = fg_counters()
    t = fg_timings()
    wp, wn = _ws(ws)
    _check(lib().fg_build_graph(C.byref(data), seed, C.byref(params), C.byref(graph), wp, wn,
                                _stream(stream), C.byref(c), C.byref(t) if timings else None))
    return c.as_dict(), (t.as_dict() if timings else None)


LOG_MARKS = 17


class fg_visit_log(C.Structure):
    _fields_ = [("slot_dev", C.c_void_p), ("nslots", C.c_uint32), ("cap", C.c_uint32),
                ("ids_dev", C.c_void_p), ("len_dev", C.c_void_p), ("marks_dev", C.c_void_p)]


def build_graph_log(data: fg_data, seed: int, params: fg_params, graph: fg_graph, ws,
                    slot: torch.Tensor, cap: int, stream=None):
    """fg_build_graph_log: the build plus the visit log of the points with
    slot[p] >= 0 (int32, n entries).  Returns (counters, timings, ids
    (nslots x cap, int32 bits of uint32), lens (nslots), marks (nslots x
    LOG_MARKS))."""
    nslots = int(slot.max().item()) + 1 if slot.numel() else 0
    if nslots < 1:
        _check(FG_EINVAL)
    dev = slot.device
    ids = torch.full((nslots, cap), -1, dtype=torch.int32, device=dev)
    lens = torch.zeros(nslots, dtype=torch.int32, device=dev)
    marks = torch.zeros((nslots, LOG_MARKS), dtype=torch.int32, device=dev)
    log = fg_visit_log(slot.data_ptr(), nslots, cap, ids.data_ptr(), lens.data_ptr(), marks.data_ptr())
    c = fg_counters()
    t = fg_timings()
    wp, wn = _ws(ws)
    _check(lib().fg_build_graph_log(C.byref(data), seed, C.byref(params), C.byref(graph), wp, wn,
                                    _stream(stream), C.byref(c), C.byref(t), C.byref(log)))
    return c.as_dict(), t.as_dict(), ids, lens, marks


def search(data: fg_data, graph: fg_graph, queries: torch.Tensor, k: int, L: int,
           out_ids, out_d, out_evals, ws, stream=None):
    wp, wn = _ws(ws)
    _check(lib().fg_search(C.byref(data), C.byref(graph), _ptr(queries), queries.shape[0], k,
                           L, _ptr(out_ids), _ptr(out_d), _ptr(out_evals), wp, wn,
                           _stream(stream)))


def search_noalloc(data: fg_data, graph: fg_graph, queries: torch.Tensor, k: int, L: int,
                   out_ids, out_d, out_evals, stream=None):
    """fg_search without a workspace (the library's fixed per-GPU scratch)."""
    _check(lib().fg_search_noalloc(C.byref(data), C.byref(graph), _ptr(queries), queries.shape[0], k,
                                   L, _ptr(out_ids), _ptr(out_d), _ptr(out_evals), _stream(stream)))


def search_noalloc_scratch_bytes() -> int:
    return int(lib().fg_search_noalloc_scratch_bytes())


def autotune(data: fg_data, params: fg_params, ws, cache_path=None, stream=None) -> fg_params:
    """Tuned copy of params (visited-table size, searches per compute unit)."""
    out = fg_params()
    wp, wn = _ws(ws)
    _check(lib().fg_autotune(C.byref(data), C.byref(params),
                             None if cache_path is None else str(cache_path).encode(), wp, wn,
                             _stream(stream), C.byref(out)))
    return out


def _ptr_array(structs):
    arr = (C.c_void_p * len(structs))(*[C.addressof(x) for x in structs])
    return arr


def batched_workspace_size(datas, paramses) -> int:
    return int(lib().fg_batched_workspace_size(_ptr_array(datas), _ptr_array(paramses), len(datas)))


BATCH_HIPGRAPH, BATCH_AUTOTUNE = 1, 2


def build_graph_batched(datas, paramses, seeds, graphs, ws=None, use_hipgraph=False, stream=None,
                        autotune=False):
    """Build len(datas) independent graphs together (fg_build_graph_batched);
    returns the summed counters and the workspace (reusable)."""
    count = len(datas)
    if ws is None:
        nb = batched_workspace_size(datas, paramses)
        if nb == 0:
            _check(FG_EINVAL)
        ws = torch.empty(nb + 256, dtype=torch.uint8, device=datas[0]._keep[0].device)
    wp, wn = _ws(ws)
    sd = (C.c_uint64 * count)(*seeds)
    c = fg_counters()
    _check(lib().fg_build_graph_batched(_ptr_array(datas), _ptr_array(paramses), sd, count, _ptr_array(graphs),
                                        wp, wn, _stream(stream),
                                        (BATCH_HIPGRAPH if use_hipgraph else 0) | (BATCH_AUTOTUNE if autotune else 0),
                                        C.byref(c)))
    return c.as_dict(), ws


def sync_status(ws: torch.Tensor, stream=None) -> None:
    """Wait for the last call made with workspace ws; raise FgError if it
    overflowed a bounded device buffer."""
    _check(lib().fg_sync_status(_ptr(ws), _stream(stream)))


def graph_hash(graph: fg_graph, stream=None) -> int:
    h = C.c_uint64(0)
    _check(lib().fg_graph_hash(C.byref(graph), _stream(stream), C.byref(h)))
    return int(h.value)


def screen_copy(data: fg_data, screen: int, stream=None):
    """The narrow copy of the rows a screened harvest reads: returns
    (codes uint8 [n, row_bytes], err [n], norm [n], sinv [n]) on the data's
    device."""
    rb = int(lib().fg_screen_row_bytes(data.d, screen))
    if rb <= 0:
        raise FgError(FG_EINVAL, "bad screen kind or d")
    dev = data._keep[0].device
    xs = torch.zeros(data.n, rb, dtype=torch.uint8, device=dev)
    err = torch.empty(data.n, dtype=torch.float32, device=dev)
    nrm = torch.empty(data.n, dtype=torch.float32, device=dev)
    sinv = torch.empty(data.n, dtype=torch.float32, device=dev)
    _check(lib().fg_screen_copy(C.byref(data), screen, _ptr(xs), _ptr(err), _ptr(nrm), _ptr(sinv),
                                _stream(stream)))
    return xs, err, nrm, sinv


def leaf_knn(data: fg_data, leaf_size: int, R: int, use_bf16: bool, out_ids, out_d,
             ws=None, stream=None):
    """Every point's R nearest within its leaf of consecutive ids, on MFMA."""
    if ws is None:
        nb = int(lib().fg_leaf_knn_workspace_size(C.byref(data)))
        ws = torch.empty(nb + 256, dtype=torch.uint8, device=out_ids.device)
    wp, wn = _ws(ws)
    _check(lib().fg_leaf_knn(C.byref(data), leaf_size, R, 1 if use_bf16 else 0, _ptr(out_ids),
                             _ptr(out_d), wp, wn, _stream(stream)))
    return ws
