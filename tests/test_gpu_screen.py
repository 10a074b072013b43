"""The screened harvest (bfloat16 / fp8-e4m3 copies with a proven margin):
the narrow copy against host encodings written from the formats'
definitions, and whole builds whose graphs, counters and hashes must equal
the unscreened build's and the oracle's."""
import numpy as np
import pytest
import torch

from gpu_util import dev, empty_u32, host_u32, say
from paper_2609_30493_amd import datagen as gen

pytestmark = pytest.mark.gpu


def _lib():
    from paper_2609_30493_amd import fgraft as F
    return F


def e4m3_table() -> np.ndarray:
    """Values of the 256 OCP fp8 e4m3 codes (bias 7, no infinities, S.1111.111
    is NaN, exponent field 0 is subnormal: m * 2^-9)."""
    out = np.empty(256)
    for c in range(256):
        s, e, m = c >> 7, (c >> 3) & 15, c & 7
        if e == 15 and m == 7:
            v = np.nan
        elif e == 0:
            v = m * 2.0 ** -9
        else:
            v = (1 + m / 8) * 2.0 ** (e - 7)
        out[c] = -v if s else v
    return out


def _rows(n, d, seed):
    rng = np.random.default_rng(seed)
    x = rng.standard_normal((n, d)) * np.exp(rng.uniform(-6, 6, size=(n, 1)))
    x[0] = 0.0                                   # an all-zero row
    x[1, : d // 2] = 1e-30                       # tiny values
    x = x.astype(np.float32)
    # bfloat16 rounding ties: low 16 bits exactly 0x8000
    b = x[2].view(np.uint32)
    x[2] = ((b & 0xFFFF0000) | 0x8000).view(np.float32)
    return x


def _loosest(true, x):
    """The largest value the float32 bound may give for a true norm: the
    rounding factor (1 + 2 gamma_d), the root's 2^-22 and one unit in the
    last place, and the flush term sqrt(d 2^-125) at the row's scale (2^ex
    below twice its largest magnitude)."""
    d = x.shape[1]
    mx = np.abs(x.astype(np.float64)).max(1)
    rel = 1 + 2 * d * 2.0 ** -24 + 2.0 ** -20
    return true * rel + np.sqrt(d * 2.0 ** -124) * 2 * np.maximum(mx, 2.0 ** -126) * rel


def test_screen_copy_bf16_is_rne_with_true_error_norms():
    F = _lib()
    n, d = 300, 96
    x = _rows(n, d, 1)
    data = F.make_data(dev(x))
    xs, err, nrm, sinv = F.screen_copy(data, F.SCREEN_BF16)
    torch.cuda.synchronize()
    codes = xs.cpu().numpy()[:, : 2 * d].copy().view(np.uint16)
    want = torch.from_numpy(x).bfloat16().view(torch.int16).numpy().view(np.uint16)
    assert np.array_equal(codes, want)
    back = (codes.astype(np.uint32) << 16).view(np.float32).astype(np.float64)
    e_true = np.sqrt(((back - x.astype(np.float64)) ** 2).sum(1))
    n_true = np.sqrt((x.astype(np.float64) ** 2).sum(1))
    e_gpu, n_gpu = err.cpu().numpy().astype(np.float64), nrm.cpu().numpy().astype(np.float64)
    assert np.all(e_gpu >= e_true) and np.all(e_gpu <= _loosest(e_true, x))
    assert np.all(n_gpu >= n_true) and np.all(n_gpu <= _loosest(n_true, x))
    assert np.all(sinv.cpu().numpy() == 1.0)
    _check_row_layout(F, xs, err, nrm, sinv, d, F.SCREEN_BF16)


def _check_row_layout(F, xs, err, nrm, sinv, d, screen):
    """Rows are whole 128-byte lines; after the codes (padded to 16-element
    steps for bfloat16, 16 bytes for fp8) each holds the trailer
    (err, norm, sinv, 0), and bfloat16 rows are zero everywhere else."""
    rb = xs.shape[1]
    assert rb % 128 == 0
    tail = (2 * d + 31) // 32 * 32 if screen == F.SCREEN_BF16 else (d + 15) // 16 * 16
    assert tail + 16 <= rb < tail + 16 + 128
    host = xs.cpu().numpy()
    tr = host[:, tail:tail + 16].copy().view(np.float32)
    assert np.array_equal(tr[:, 0], err.cpu().numpy())
    assert np.array_equal(tr[:, 1], nrm.cpu().numpy())
    assert np.array_equal(tr[:, 2], sinv.cpu().numpy())
    assert np.all(tr[:, 3] == 0.0)
    if screen == F.SCREEN_BF16:
        assert not host[:, 2 * d:tail].any() and not host[:, tail + 16:].any()


def test_screen_copy_fp8_codes_decode_per_ocp_e4m3():
    F = _lib()
    n, d = 300, 128
    x = _rows(n, d, 2)
    data = F.make_data(dev(x))
    xs, err, nrm, sinv = F.screen_copy(data, F.SCREEN_FP8E4M3)
    torch.cuda.synchronize()
    tab = e4m3_table()
    codes = xs.cpu().numpy()[:, :d]
    assert not np.any(np.isnan(tab[codes]))
    xd = x.astype(np.float64)
    mx = np.abs(xd).max(1)
    k = np.zeros(n, np.int64)
    for i in range(n):
        if mx[i] > 0:
            k[i] = int(np.floor(np.log2(448.0 / mx[i])))
            while np.ldexp(mx[i], k[i]) > 448.0:
                k[i] -= 1
            while np.ldexp(mx[i], k[i] + 1) <= 448.0:
                k[i] += 1
            k[i] = min(max(k[i], -100), 100)
    assert np.array_equal(sinv.cpu().numpy().astype(np.float64), np.ldexp(1.0, -k))
    # each code is a nearest e4m3 value of x * 2^k
    fin = tab[np.isfinite(tab)]
    scaled = xd * np.ldexp(1.0, k)[:, None]
    got = tab[codes]
    best = np.abs(scaled[..., None] - fin[None, None, :]).min(-1)
    assert np.all(np.abs(got - scaled) <= best)
    back = got * np.ldexp(1.0, -k)[:, None]
    e_true = np.sqrt(((back - xd) ** 2).sum(1))
    e_gpu = err.cpu().numpy().astype(np.float64)
    assert np.all(e_gpu >= e_true) and np.all(e_gpu <= _loosest(e_true, x))
    _check_row_layout(F, xs, err, nrm, sinv, d, F.SCREEN_FP8E4M3)


def test_screen_copy_int8_codes_and_error_norms():
    """int8 codes rint(x / s) clamped to [-127, 127], s = fl(max|x| / 127)
    in float32, read back as fl(code * s); the trailer's factor is s."""
    F = _lib()
    n, d = 300, 100
    x = _rows(n, d, 3)
    data = F.make_data(dev(x))
    xs, err, nrm, sinv = F.screen_copy(data, F.SCREEN_INT8)
    torch.cuda.synchronize()
    codes = xs.cpu().numpy()[:, :d].view(np.int8).astype(np.int64)
    mx = np.abs(x).max(1).astype(np.float32)
    s = (mx / np.float32(127)).astype(np.float32)
    assert np.array_equal(sinv.cpu().numpy(), s)
    with np.errstate(divide="ignore", invalid="ignore"):
        want = np.where(s[:, None] > 0, np.clip(np.rint((x / s[:, None]).astype(np.float32)), -127, 127), 0)
    assert np.array_equal(codes, want.astype(np.int64))
    back = (codes.astype(np.float32) * s[:, None]).astype(np.float32).astype(np.float64)
    e_true = np.sqrt(((back - x.astype(np.float64)) ** 2).sum(1))
    n_true = np.sqrt((x.astype(np.float64) ** 2).sum(1))
    e_gpu, n_gpu = err.cpu().numpy().astype(np.float64), nrm.cpu().numpy().astype(np.float64)
    assert np.all(e_gpu >= e_true) and np.all(e_gpu <= _loosest(e_true, x))
    assert np.all(n_gpu >= n_true) and np.all(n_gpu <= _loosest(n_true, x))
    _check_row_layout(F, xs, err, nrm, sinv, d, F.SCREEN_INT8)


SCREEN_BUILDS = [
    # name, data, metric, T, ef, R, B
    ("powerlaw-d96-5000", lambda: gen.powerlaw_f32(5000, 96, 40, 11), "l2", 8, 64, 32, 4),
    ("powerlaw-d256-4000", lambda: gen.powerlaw_f32(4000, 256, 40, 12), "l2", 8, 128, 32, 8),
    ("powerlaw-d960-3000", lambda: gen.powerlaw_f32(3000, 960, 60, 13), "l2", 8, 128, 64, 8),
    # rows screened by the whole wave (more than 64 chunks): cosine, and a
    # last lane holding one chunk of its four
    ("cosine-d300-3000", lambda: gen.anisotropic_unit_f32(3000, 300, 40, 16), "cosine", 8, 128, 64, 8),
    ("powerlaw-d260-3000", lambda: gen.powerlaw_f32(3000, 260, 40, 17), "l2", 8, 64, 32, 4),
    # the largest rows (every lane holds four chunks) and the widest beam
    ("powerlaw-d1024-2000", lambda: gen.powerlaw_f32(2000, 1024, 30, 18), "l2", 8, 256, 32, 4),
    ("cosine-d100-5000", lambda: gen.anisotropic_unit_f32(5000, 100, 50, 14), "cosine", 8, 128, 64, 8),
    ("isotropic-d68-4000", lambda: gen.isotropic_f32(4000, 68, 8, 0.1, 15), "l2", 4, 256, 16, 2),
]


def _build(F, x, metric, T, ef, R, B, screen, table=0):
    n = x.shape[0]
    data = F.make_data(dev(x), metric)
    params = F.make_params(T, ef, R, 1.2, B, screen=screen, beam_table_slots=table)
    ws = F.alloc_workspace(data, params)
    gn, gcnt, sp, rt = empty_u32(n, R), empty_u32(n, fill=0), empty_u32(n), empty_u32(T)
    G = F.make_graph(gn, gcnt, sp, rt, T)
    c, t = F.build_graph(data, 42, params, G, ws, timings=True)
    return F.graph_hash(G), host_u32(gn), host_u32(gcnt), c


@pytest.mark.parametrize("case", SCREEN_BUILDS, ids=[c[0] for c in SCREEN_BUILDS])
def test_screened_builds_equal_unscreened_and_oracle(fgo, case):
    F = _lib()
    name, mk, metric, T, ef, R, B = case
    x = np.ascontiguousarray(mk().astype(np.float32))
    say(f"screened build {name}")
    h0, g0, c0, k0 = _build(F, x, metric, T, ef, R, B, F.SCREEN_NONE)
    want = fgo.build_graph(fgo.Data(x, metric=metric), 42, fgo.params(T, ef, R, 1.2, B, 0, 8))
    assert h0 == want["hash"]
    for scr in (F.SCREEN_BF16, F.SCREEN_FP8E4M3, F.SCREEN_INT8):
        h, g, c, k = _build(F, x, metric, T, ef, R, B, scr)
        say(f"  screen={scr} rejected {k['screen_rejected']} of {k['harvest_evals']}")
        assert h == h0
        assert np.array_equal(g, g0) and np.array_equal(c, c0)
        for key in ("harvest_evals", "expansions", "prune_evals", "finalize_evals", "scaffold_evals"):
            assert k[key] == k0[key], key
        assert 0 < k["screen_rejected"] < k["harvest_evals"]
        assert k0["screen_rejected"] == 0


@pytest.mark.parametrize("table", [512, 1024, 2048, 4096])
def test_screened_builds_at_every_table_size(table):
    """The screened kernels' tables (1024 for rows of up to 4 chunks per lane
    by default, a 512 request served by 1024, 2048 and 4096 on request):
    the same graph and counters as the unscreened build, which the test
    above ties to the oracle."""
    F = _lib()
    picked = ("powerlaw-d96-5000", "powerlaw-d256-4000", "cosine-d100-5000", "cosine-d300-3000")
    for name, mk, metric, T, ef, R, B in (c for c in SCREEN_BUILDS if c[0] in picked):
        x = np.ascontiguousarray(mk().astype(np.float32))
        say(f"screened build {name} table={table}")
        h0, g0, c0, k0 = _build(F, x, metric, T, ef, R, B, F.SCREEN_NONE)
        for scr in (F.SCREEN_BF16, F.SCREEN_FP8E4M3, F.SCREEN_INT8):
            h, g, c, k = _build(F, x, metric, T, ef, R, B, scr, table)
            assert h == h0 and np.array_equal(g, g0) and np.array_equal(c, c0), (name, scr)
            for key in ("harvest_evals", "expansions", "prune_evals", "finalize_evals", "scaffold_evals"):
                assert k[key] == k0[key], (name, scr, key)
            assert k["screen_rejected"] > 0


def test_screened_harvest_block_equals_unscreened(fgo):
    F = _lib()
    x = np.ascontiguousarray(gen.powerlaw_f32(3000, 192, 30, 21))
    n, T, ef, R, B, b = x.shape[0], 8, 96, 32, 4, 1
    D = fgo.Data(x)
    r, parents, off, ids, _ = fgo.scaffold(D, 42, T)
    data = F.make_data(dev(x))
    out = []
    for scr in (0, 1, 2, 4):
        params = F.make_params(T, ef, R, 1.2, B, screen=scr)
        ws = F.alloc_workspace(data, params)
        S = F.csr(dev(off.view(np.int64)), dev(ids.view(np.int32)), int(off[-1]))
        rows, cnt = empty_u32(n, R), empty_u32(n, fill=0)
        c = F.harvest_block(data, S, dev(r), params, b, rows, cnt, ws)
        out.append((host_u32(rows), host_u32(cnt), c))
    for rows, cnt, c in out[1:]:
        assert np.array_equal(rows, out[0][0]) and np.array_equal(cnt, out[0][1])
        assert c["harvest_evals"] == out[0][2]["harvest_evals"] and c["screen_rejected"] > 0


def test_screen_argument_errors():
    F = _lib()
    xu = dev(gen.small_u8(500, 128, 1))
    d8 = F.make_data(xu)
    p8 = F.make_params(4, 32, 16, 1.2, 2, screen=1)
    ws8 = F.alloc_workspace(d8, p8)
    g8 = F.make_graph(empty_u32(500, 16), empty_u32(500), empty_u32(500), empty_u32(4), 4)
    with pytest.raises(F.FgError) as e:
        F.build_graph(d8, 1, p8, g8, ws8)
    assert e.value.code == F.FG_EUNSUPPORTED
    x64 = dev(gen.isotropic_f32(500, 64, 4, 0.1, 2))
    d64 = F.make_data(x64)
    with pytest.raises(F.FgError) as e:
        F.screen_copy(d64, F.SCREEN_BF16)
    assert e.value.code == F.FG_EUNSUPPORTED
    x192 = dev(gen.isotropic_f32(500, 192, 4, 0.1, 2))
    p3 = F.make_params(4, 32, 16, 1.2, 2, screen=F.SCREEN_BF16_PRUNE)
    with pytest.raises(F.FgError) as e:  # the split tiles need 256 < d <= 1024
        F.build_graph(F.make_data(x192), 1, p3, F.make_graph(empty_u32(500, 16), empty_u32(500), empty_u32(500),
                                                             empty_u32(4), 4),
                      torch.empty(1 << 26, dtype=torch.uint8, device="cuda"))
    assert e.value.code == F.FG_EUNSUPPORTED
    p = F.make_params(4, 32, 16, 1.2, 2, screen=5)  # no such fg_screen
    with pytest.raises(F.FgError) as e:
        F.build_graph(d64, 1, p, F.make_graph(empty_u32(500, 16), empty_u32(500), empty_u32(500),
                                              empty_u32(4), 4), torch.empty(1 << 20, dtype=torch.uint8,
                                                                            device="cuda"))
    assert e.value.code == F.FG_EINVAL
