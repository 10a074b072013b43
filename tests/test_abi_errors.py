"""Argument checking at the C-ABI, without a GPU: every case below fails
validation before any device work, so the library returns its status code
and message on a host with no GPU.  Device pointers are stand-in addresses
that the library never dereferences on these paths."""
import ctypes as C

import pytest

from paper_2609_30493_amd import fgraft as F

FAKE = 0x100000  # 256-byte aligned stand-in for a device address


@pytest.fixture(scope="module")
def lib():
    return F.lib()


def data(n=1000, d=32, dtype=F.F32, metric=F.L2SQ, stride=None, x=FAKE):
    esz = 4 if dtype == 0 else 1
    return F.fg_data(x, n, d, dtype, metric, 0, stride if stride is not None else d * esz)


def params(T=4, ef=32, R=16, alpha=1.2, B=2, table=0, screen=0, waves=0, lanes=0):
    return F.fg_params(T, ef, R, alpha, B, 0, table, screen, waves, lanes)


def graph(n=1000, R=16, T=4):
    return F.fg_graph(FAKE, FAKE, FAKE, FAKE, n, R, T)


def build(lib, d, p, g, ws=FAKE, ws_bytes=1 << 40):
    rc = lib.fg_build_graph(C.byref(d) if d is not None else None, 42, C.byref(p), C.byref(g),
                            C.c_void_p(ws) if ws else None, ws_bytes, None, None, None)
    return rc, lib.fg_last_error().decode()


@pytest.mark.parametrize("kw,msg", [
    (dict(x=0), "x_dev is NULL"),
    (dict(n=0), "n out of range"),
    (dict(d=30), "d % 4"),
    (dict(dtype=1, d=20), "d % 16"),
    (dict(dtype=1, d=32, metric=1), "squared L2 only"),
    (dict(dtype=7), "bad dtype"),
    (dict(metric=5), "bad metric"),
    (dict(stride=64), "row_stride_bytes"),
    (dict(stride=136), "row_stride_bytes"),
    (dict(x=FAKE + 8), "16-byte aligned"),
])
def test_bad_data_is_rejected(lib, kw, msg):
    rc, err = build(lib, data(**kw), params(), graph(n=kw.get("n", 1000) or 1000))
    assert rc == F.FG_EINVAL and msg in err, (rc, err)


@pytest.mark.parametrize("kw,msg", [
    (dict(T=0), "T <= n"),
    (dict(T=65), "T > 64"),
    (dict(ef=0), "ef_h"),
    (dict(ef=257), "ef_h"),
    (dict(R=0), "R <= 1024"),
    (dict(R=1025), "R <= 1024"),
    (dict(alpha=0.9), "alpha"),
    (dict(alpha=float("nan")), "alpha"),
    (dict(alpha=float("inf")), "alpha"),
    (dict(table=3000), "beam_table_slots"),
    (dict(screen=9), "fg_screen"),
    (dict(waves=65), "waves_per_cu"),
    (dict(lanes=3), "lanes_per_row"),
])
def test_bad_params_are_rejected(lib, kw, msg):
    p = params(**kw)
    rc, err = build(lib, data(), p, graph(R=p.R, T=p.T))
    assert rc == F.FG_EINVAL and msg in err, (rc, err)


def test_graph_shape_must_match(lib):
    rc, err = build(lib, data(), params(), graph(n=999))
    assert rc == F.FG_EINVAL and "does not match" in err
    g = graph()
    g.roots_dev = None
    rc, err = build(lib, data(), params(), g)
    assert rc == F.FG_EINVAL and "required" in err


@pytest.mark.parametrize("dkw,screen,msg", [
    (dict(dtype=1, d=128), F.SCREEN_BF16, "FG_F32 data only"),
    (dict(d=64), F.SCREEN_FP8E4M3, "64 < d <= 1024"),
    (dict(d=1028), F.SCREEN_BF16, "64 < d <= 1024"),
    (dict(d=100), F.SCREEN_BF16_PRUNE, "256 < d <= 1024"),
    (dict(dtype=1, d=128), F.SCREEN_INT8, "FG_F32 data only"),
    (dict(d=64), F.SCREEN_INT8, "64 < d <= 1024"),
])
def test_unsupported_screens_are_refused(lib, dkw, screen, msg):
    rc, err = build(lib, data(**dkw), params(screen=screen), graph())
    assert rc == F.FG_EUNSUPPORTED and msg in err, (rc, err)


def test_workspace_is_checked(lib):
    d, p, g = data(), params(), graph()
    need = lib.fg_workspace_size(C.byref(d), C.byref(p))
    assert need > 0
    assert lib.fg_workspace_size(None, C.byref(p)) == 0
    rc, err = build(lib, d, p, g, ws=0)
    assert rc == F.FG_ENOMEM and "NULL" in err
    rc, err = build(lib, d, p, g, ws=FAKE + 64)
    assert rc == F.FG_ENOMEM and "256-byte aligned" in err
    rc, err = build(lib, d, p, g, ws_bytes=need - 1)
    assert rc == F.FG_ENOMEM and "too small" in err


def test_search_arguments_are_checked(lib):
    d, g = data(), graph()
    def search(k, L, q=FAKE):
        rc = lib.fg_search(C.byref(d), C.byref(g), C.c_void_p(q) if q else None, 10, k, L, C.c_void_p(FAKE),
                           C.c_void_p(FAKE), None, C.c_void_p(FAKE), 1 << 40, None)
        return rc, lib.fg_last_error().decode()
    assert search(0, 10)[0] == F.FG_EINVAL
    assert search(10, 5)[0] == F.FG_EINVAL
    assert search(10, 513)[0] == F.FG_EINVAL
    rc, err = search(10, 64, q=FAKE + 4)
    assert rc == F.FG_EINVAL and "16-byte aligned" in err
    rc, err = search(10, 64, q=0)
    assert rc == F.FG_EINVAL and "required" in err
