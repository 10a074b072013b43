"""The Gram-tile prune and the scaffold's matrix-core closest-neighbour
assignment (float32 rows of more than 256 elements): kept lists, trees and
evaluation counts must equal the oracle's exact ones, including data where
the matrix-core distances cancel catastrophically (every test then falls to
the exact recheck), rows repeated many times (ties everywhere) and candidate
sets beyond the Gram tile (exact fallback)."""
import numpy as np
import pytest

from gpu_util import dev, empty_u32, host_u32, say
from paper_2609_30493_amd import datagen as gen

pytestmark = pytest.mark.gpu


def _offset_near_duplicates(n, d, seed):
    rng = np.random.default_rng(seed)
    centres = rng.standard_normal((12, d))
    x = centres[rng.integers(0, 12, n)] * 1e-2 + rng.standard_normal((n, d)) * 1e-3 + 100.0
    return x.astype(np.float32)


CASES = [
    # name, data, metric, T, ef, R, B
    ("powerlaw-d384", lambda: gen.powerlaw_f32(3000, 384, 30, 21), "l2", 8, 128, 64, 4),
    ("cosine-d512", lambda: gen.anisotropic_unit_f32(2500, 512, 20, 22), "cosine", 8, 96, 32, 4),
    ("offset-near-duplicates-d320", lambda: _offset_near_duplicates(1500, 320, 23), "l2", 4, 64, 24, 2),
    ("powerlaw-d288-ef256", lambda: gen.powerlaw_f32(2500, 288, 25, 24), "l2", 8, 256, 32, 2),
    # 40 distinct rows, each 75 times: every distance ties many ways
    ("duplicates-d320", lambda: np.repeat(gen.powerlaw_f32(40, 320, 4, 25), 75, axis=0), "l2", 4, 64, 16, 2),
    # a hub at the origin with ~1500 finalize candidates: beyond the Gram
    # tile's 1024, the exact per-pair prune of the second tier
    ("hub-d288-1500", lambda: gen.hub_f32(1500, 288, 3), "l2", 4, 32, 16, 2),
]


@pytest.mark.parametrize("case", CASES, ids=[c[0] for c in CASES])
def test_gram_prune_builds_match_oracle(fgo, case):
    from paper_2609_30493_amd import fgraft as F
    name, mk, metric, T, ef, R, B = case
    x = np.ascontiguousarray(mk().astype(np.float32))
    n = x.shape[0]
    say(f"gram prune {name}")
    want = fgo.build_graph(fgo.Data(x, metric=metric), 42, fgo.params(T, ef, R, 1.2, B, 0, 8))
    data = F.make_data(dev(x), metric)
    params = F.make_params(T, ef, R, 1.2, B)
    ws = F.alloc_workspace(data, params)
    gn, gcnt, sp, rt = empty_u32(n, R), empty_u32(n, fill=0), empty_u32(n), empty_u32(T)
    G = F.make_graph(gn, gcnt, sp, rt, T)
    c, _ = F.build_graph(data, 42, params, G, ws, timings=True)
    assert np.array_equal(host_u32(gcnt), want["cnt"])
    assert np.array_equal(host_u32(gn), want["nbrs"])
    assert F.graph_hash(G) == want["hash"]
    for k in ("harvest_evals", "prune_evals", "expansions", "finalize_evals", "scaffold_evals"):
        assert c[k] == want["counters"][k], k


@pytest.mark.parametrize("case", CASES, ids=[c[0] for c in CASES])
def test_split_tile_builds_match_oracle(fgo, case):
    """FG_SCREEN_BF16_PRUNE: the same graph from the bfloat16 split tiles."""
    from paper_2609_30493_amd import fgraft as F
    name, mk, metric, T, ef, R, B = case
    x = np.ascontiguousarray(mk().astype(np.float32))
    n = x.shape[0]
    say(f"split-tile prune {name}")
    want = fgo.build_graph(fgo.Data(x, metric=metric), 42, fgo.params(T, ef, R, 1.2, B, 0, 8))
    data = F.make_data(dev(x), metric)
    out = {}
    for scr in (F.SCREEN_NONE, F.SCREEN_BF16_PRUNE):
        params = F.make_params(T, ef, R, 1.2, B, screen=scr)
        ws = F.alloc_workspace(data, params)
        gn, gcnt, sp, rt = empty_u32(n, R), empty_u32(n, fill=0), empty_u32(n), empty_u32(T)
        G = F.make_graph(gn, gcnt, sp, rt, T)
        c, _ = F.build_graph(data, 42, params, G, ws, timings=True)
        assert np.array_equal(host_u32(gcnt), want["cnt"])
        assert np.array_equal(host_u32(gn), want["nbrs"])
        assert F.graph_hash(G) == want["hash"]
        for k in ("harvest_evals", "prune_evals", "expansions", "finalize_evals", "scaffold_evals"):
            assert c[k] == want["counters"][k], k
        assert c["screen_rejected"] == 0
        out[scr] = c["prune_rechecks"]
    say(f"  rechecks float32 tiles {out[F.SCREEN_NONE]}, split tiles {out[F.SCREEN_BF16_PRUNE]}")
    if not name.startswith(("offset", "duplicates", "hub")):  # there most tests are rechecked either way
        assert out[F.SCREEN_BF16_PRUNE] <= 20 * out[F.SCREEN_NONE] + 200
