"""The Gram-tile prune's margin (Sec. 5.3's matrix-core form of the pair
tests, rounding-error analysis in the standard model): the distance the
prune derives from Gram entries, d~ = G_aa + G_cc - 2 G_ac (cosine 1 - G_ac),
never differs from the oracle's exact declared-order distance by more than
the margin, for Gram entries accumulated in several float32 orders, from the
float32 rows and from their bfloat16 split x = hi + lo + e.  The margin is
restated here from its derivation (the kernels use twice this value)."""
import numpy as np
import pytest
import torch

U = 2.0 ** -24


def margin(dt, gaa, gcc, d, metric, split):
    nk = 3 * d + 4 if split else d + 4
    gg = nk * 2 * U / (1 - nk * 2 * U)
    if split:
        gg = 3.1 * 2.0 ** -16 + 1.016 * gg
    gc = (d // 16 + 8) * U / (1 - (d // 16 + 8) * U)
    if metric == "l2":
        s2 = 2 * (abs(gaa) + abs(gcc)) / (1 - gg)
        b = (gg + 2 * U) * (1 + gg) * s2
        eps = b + gc * (abs(dt) + b)
    else:
        nn = np.sqrt(abs(gaa) * abs(gcc)) / (1 - gg)
        eps = (gg + gc) * nn + 4 * U * (1 + nn)
    # underflow: flushed operands (k products per element) and nk flushed or
    # underflowed partial results, at most 2^-126 each; the operands' term
    # 2^-126 sqrt(d) (|a| + |c|) is bounded by AM-GM,
    # sqrt(d) sqrt(y) <= (d + y) / 2 with y = |G| + 2^-120
    flushed = (3 if split else 1) * (d + 0.5 * (abs(gaa) + abs(gcc)) + 2.0 ** -120)
    if metric == "l2":
        eps += 2.0 ** -124 * (flushed + 2 * nk)
    else:
        eps += 2.0 ** -125 * (flushed + nk)
    return eps


def bf16_split(x):
    """hi = x rounded to bfloat16 (nearest even), lo = (x - hi) so rounded."""
    t = torch.from_numpy(np.ascontiguousarray(x, dtype=np.float32))
    hi = t.bfloat16().float()
    lo = (t - hi).bfloat16().float()
    return hi.numpy(), lo.numpy()


TINY = np.float32(2.0 ** -126)


def ftz(v):
    """Flush float32 values below the normal range to zero."""
    v = np.asarray(v, dtype=np.float32)
    return np.where(np.abs(v) < TINY, np.float32(0), v).astype(np.float32)


def fsum(terms, mode):
    """Float32 sum of float32 terms in a given order ("ftz": sequential,
    every partial sum flushed to zero below the normal range)."""
    terms = np.asarray(terms, dtype=np.float32)
    if mode == "ftz":
        acc = np.float32(0)
        for t in terms:
            acc = ftz(np.float32(acc + t))[()]
        return acc
    if mode == "seq":
        return np.cumsum(terms, dtype=np.float32)[-1]
    if mode == "rev":
        return np.cumsum(terms[::-1], dtype=np.float32)[-1]
    a = terms.copy()  # pairwise
    while a.size > 1:
        if a.size % 2:
            a = np.append(a, np.float32(0))
        a = (a[0::2] + a[1::2]).astype(np.float32)
    return a[0]


def gram_entry(a, c, split, mode):
    flush = ftz if mode == "ftz" else (lambda v: np.asarray(v, dtype=np.float32))
    if not split:
        return fsum(flush((flush(a).astype(np.float64) * flush(c).astype(np.float64)).astype(np.float32)), mode)
    ah, al = (flush(v) for v in bf16_split(a))
    ch, cl = (flush(v) for v in bf16_split(c))
    f = lambda u, v: flush((u.astype(np.float64) * v.astype(np.float64)).astype(np.float32))  # noqa: E731
    if mode == "steps":  # the tile's order: per 16 elements al*ch, ah*cl, ah*ch
        terms = []
        for k in range(0, a.size, 16):
            s = slice(k, k + 16)
            terms += [f(al[s], ch[s]), f(ah[s], cl[s]), f(ah[s], ch[s])]
        return fsum(np.concatenate(terms), "seq")
    return fsum(np.concatenate([f(ah, ch), f(ah, cl), f(al, ch)]), mode)


def pairs(metric, rng, d):
    out = []
    for _ in range(40):
        scale = np.exp(rng.uniform(-4, 4))
        a = (rng.standard_normal(d) * scale).astype(np.float32)
        c = (a + rng.standard_normal(d) * scale * np.exp(rng.uniform(-8, 1))).astype(np.float32)
        out.append((a, c))
    # adversarial: identical rows, one ulp apart, a large common offset
    # (catastrophic cancellation in G_aa + G_cc - 2 G_ac), mixed magnitudes
    a = (rng.standard_normal(d) * 1e4).astype(np.float32)
    out.append((a, a.copy()))
    c = a.copy()
    c[3] = np.nextafter(c[3], np.float32(np.inf))
    out.append((a, c))
    o = (rng.standard_normal(d) * 1e-3 + 100.0).astype(np.float32)
    out.append((o, (o + rng.standard_normal(d) * 1e-3).astype(np.float32)))
    m = (rng.standard_normal(d) * np.logspace(-20, 5, d)).astype(np.float32)
    out.append((m, (m * 1.001).astype(np.float32)))
    # rows whose squares and products fall below the normal range
    for e in (-64, -70, -75):
        t = np.ldexp(rng.standard_normal(d), e).astype(np.float32)
        out.append((t, (t + np.ldexp(rng.standard_normal(d), e - 2)).astype(np.float32)))
    z = np.ldexp(rng.standard_normal(d), -70)
    z[: d // 2] *= 2.0 ** 60
    out.append((z.astype(np.float32), (z * 0.999).astype(np.float32)))
    if metric == "cosine":
        out = [(a / np.linalg.norm(a.astype(np.float64)), c / np.linalg.norm(c.astype(np.float64)))
               for a, c in out if np.linalg.norm(a) > 0 and np.linalg.norm(c) > 0]
        out = [(a.astype(np.float32), c.astype(np.float32)) for a, c in out]
    return out


@pytest.mark.parametrize("metric", ["l2", "cosine"])
@pytest.mark.parametrize("split", [False, True], ids=["f32", "bf16split"])
@pytest.mark.parametrize("d", [260, 960])
def test_gram_margin_bounds_exact_distance(fgo, metric, split, d):
    rng = np.random.default_rng(d + 2 * split + 5 * (metric == "cosine"))
    worst = 0.0
    modes = ("seq", "rev", "pair", "steps", "ftz") if split else ("seq", "rev", "pair", "ftz")
    for a, c in pairs(metric, rng, d):
        D = fgo.Data(np.stack([a, c]), metric=metric)
        exact = float(fgo.dist(D, 0, 1))
        for mode in modes + (("norms",) if split else ()):
            if mode == "norms":  # the kernels' combination: split <a,c>, float32 |a|^2, |c|^2
                gaa, gcc = gram_entry(a, a, False, "seq"), gram_entry(c, c, False, "pair")
                gac = gram_entry(a, c, True, "steps")
            else:
                gaa, gcc, gac = (gram_entry(u, v, split, mode) for u, v in ((a, a), (c, c), (a, c)))
            if metric == "l2":
                dt = float(np.float32(np.float32(gaa + gcc) - np.float32(np.float32(2) * gac)))
            else:
                dt = float(np.float32(np.float32(1) - gac))
            eps = margin(dt, float(gaa), float(gcc), d, metric, split)
            assert abs(exact - dt) <= eps, (mode, exact, dt, eps)
            if eps > 0:
                worst = max(worst, abs(exact - dt) / eps)
    # sound, and the emulated sums do carry rounding error for it to bound
    assert 1e-3 < worst <= 1.0


def test_split_margin_is_not_vacuous_on_neighbours():
    """On clustered rows the split tiles' margin is a small fraction of a
    neighbour distance, so most pair tests are settled without a recheck."""
    from paper_2609_30493_amd import datagen as gen
    x = gen.powerlaw_f32(64, 960, 4, 3)
    rel = []
    for i in range(1, 64):
        gaa, gcc = float(x[0].astype(np.float64) @ x[0]), float(x[i].astype(np.float64) @ x[i])
        dt = float(((x[0].astype(np.float64) - x[i]) ** 2).sum())
        rel.append(margin(dt, gaa, gcc, 960, "l2", True) / dt)
    assert np.median(rel) < 0.02


def test_split_planes_carry_sixteen_bits():
    """|x - hi - lo| <= 2^-16 |x| elementwise (the margin's premise)."""
    rng = np.random.default_rng(5)
    x = (rng.standard_normal(20000) * np.exp(rng.uniform(-30, 30, 20000))).astype(np.float32)
    hi, lo = bf16_split(x)
    r = np.abs(x.astype(np.float64) - hi.astype(np.float64) - lo.astype(np.float64))
    assert np.all(r <= 2.0 ** -16 * np.abs(x.astype(np.float64)))


@pytest.mark.parametrize("d", [68, 260, 960])
def test_flush_term_dominates_operand_flush_bound(d):
    """The margin's operand-flush term, d + (|G_aa| + |G_cc|) / 2 + 2^-120,
    is at least sqrt(d) (sqrt(|G_aa| + 2^-120) + sqrt(|G_cc| + 2^-120)),
    the bound on sum_i |a_i c_i| over operands flushed below 2^-126 (per
    unit of 2^-126), for squared norms across the float32 range."""
    g = np.concatenate([[0.0], np.logspace(-45, 38, 400)])
    ga, gc = np.meshgrid(g, g)
    t = 2.0 ** -120
    root_form = np.sqrt(d) * (np.sqrt(ga + t) + np.sqrt(gc + t))
    amgm = d + 0.5 * (ga + gc) + t
    assert np.all(amgm >= root_form * (1 - 1e-12))
