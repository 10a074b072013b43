"""Rows whose squared distances fall into (or below) float32's subnormal
range, at d > 256 where the occlusion prune and the scaffold decide tests
from matrix-core Gram tiles, and through every screened form: each build
equals the oracle's (hash, rows and every counter).  The oracle evaluates
the declared order with IEEE subnormals, so any flush to zero in the device
arithmetic, or a margin with no absolute term, would show up here."""
import numpy as np
import pytest

from gpu_util import dev, empty_u32, host_u32, say
from paper_2609_30493_amd import datagen as gen

pytestmark = pytest.mark.gpu


def _build(F, x, metric, T, ef, R, B, screen):
    n = x.shape[0]
    data = F.make_data(dev(x), metric)
    params = F.make_params(T, ef, R, 1.2, B, screen=screen)
    ws = F.alloc_workspace(data, params)
    gn, gc, sp, rt = empty_u32(n, R), empty_u32(n, fill=0), empty_u32(n), empty_u32(T)
    G = F.make_graph(gn, gc, sp, rt, T)
    c, _ = F.build_graph(data, 42, params, G, ws, timings=True)
    return F.graph_hash(G), host_u32(gn), host_u32(gc), c


# scale 2^-64: squared differences near 2^-128, sums across the normal /
# subnormal boundary; 2^-70: most squares subnormal, many distances zero
@pytest.mark.parametrize("d,log2scale", [(288, -64), (288, -70), (960, -66)])
def test_subnormal_square_rows_match_oracle_in_every_form(fgo, d, log2scale):
    from paper_2609_30493_amd import fgraft as F
    n, T, ef, R, B = 1200, 4, 64, 24, 2
    x = gen.powerlaw_f32(n, d, 20, 31 + d)
    x = np.ascontiguousarray(np.ldexp(x.astype(np.float64), log2scale).astype(np.float32))
    assert np.all(np.isfinite(x))
    sq = (x.astype(np.float64) ** 2).sum(1)
    say(f"subnormal-range rows d={d} scale 2^{log2scale}: median |x|^2 = {np.median(sq):.3e}")
    want = fgo.build_graph(fgo.Data(x), 42, fgo.params(T, ef, R, 1.2, B, 0, 8))
    forms = [F.SCREEN_NONE, F.SCREEN_BF16, F.SCREEN_FP8E4M3, F.SCREEN_INT8, F.SCREEN_BF16_PRUNE]
    for scr in forms:
        h, g, c, k = _build(F, x, "l2", T, ef, R, B, scr)
        say(f"  screen={scr}: rechecks {k['prune_rechecks']}, rejected {k['screen_rejected']}")
        assert h == want["hash"], scr
        assert np.array_equal(g, want["nbrs"]) and np.array_equal(c, want["cnt"]), scr
        for key in ("harvest_evals", "expansions", "prune_evals", "finalize_evals", "scaffold_evals"):
            assert k[key] == want["counters"][key], (scr, key)
