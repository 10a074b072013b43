"""The screening margin (Sec. 5.3's narrow rows, rounding-error analysis in
the standard model, unit roundoff 2^-24) against the oracle's exact distance
in the declared float32 order: for random and adversarial pairs, the exact
distance is never below the screened value minus the margin.  The margin is
restated here from its derivation, underflow terms included (the kernel
raises it by 2^-20 of itself for its own roundings)."""
import numpy as np
import pytest
import torch

U = 2.0 ** -24


T149 = 2.0 ** -149  # the smallest float32 subnormal


def margin(dt, d, E, np_, nu, metric, f=1.0):
    """f: the fp8 copy's power-of-two factor, applied to the cosine sum."""
    gs = (d + 12) * U / (1 - (d + 12) * U)
    gc = (d // 16 + 8) * U / (1 - (d // 16 + 8) * U)
    t = d * T149
    if metric == "l2":
        dd = max(dt, 0.0)
        A = np.sqrt((dd + t) / (1 - gs)) * (1 + 4 * U)
        return (gs + gc) * dd + 2 * A * E + t
    pu = np_ * (nu + E)
    return np_ * E + (gs + gc) * pu + 4 * U * (1 + pu) + t * (1 + max(1.0, f) + np_)


def bf16_back(u):
    return torch.from_numpy(u).bfloat16().float().numpy()


def fp8_back(u):
    """Nearest-even e4m3 (OCP) of u * 2^k, read back as value * 2^-k."""
    vals = []
    for c in range(256):
        s_, e, m = c >> 7, (c >> 3) & 15, c & 7
        if e == 15 and m == 7:
            continue
        v = m * 2.0 ** -9 if e == 0 else (1 + m / 8) * 2.0 ** (e - 7)
        vals.append((-v if s_ else v, c))
    vals.sort()
    grid = np.array([v for v, _ in vals])
    mx = np.abs(u.astype(np.float64)).max()
    k = 0 if mx == 0 else int(np.floor(np.log2(448.0 / mx)))
    while mx and np.ldexp(mx, k) > 448.0:
        k -= 1
    x = u.astype(np.float64) * 2.0 ** k
    idx = np.abs(x[:, None] - grid[None, :]).argmin(1)
    return (grid[idx] * 2.0 ** -k).astype(np.float32)


def fp8_factor(u):
    """The power of two 2^-k that reads an fp8 code back (see fp8_back)."""
    mx = np.abs(u.astype(np.float64)).max()
    k = 0 if mx == 0 else int(np.floor(np.log2(448.0 / mx)))
    while mx and np.ldexp(mx, k) > 448.0:
        k -= 1
    return 2.0 ** -k


def int8_codes(u):
    """Codes rint(u / s) in [-127, 127] with s = fl(max|u| / 127), all in
    float32 as the copy kernel computes them."""
    u = u.astype(np.float32)
    s = np.float32(np.abs(u).max() / np.float32(127))
    if s == 0:
        return np.zeros(u.shape, np.int64), np.float32(0)
    q = np.clip(np.rint((u / s).astype(np.float32)), -127, 127).astype(np.int64)
    return q, s


def int8_back(u):
    q, s = int8_codes(u)
    return (q.astype(np.float32) * s).astype(np.float32)


def margin_i8(E_p, np_, E_u, nu, d):
    """Cosine over int8 codes of both rows (the kernel's exact integer dot)."""
    gc = (d // 16 + 8) * U / (1 - (d // 16 + 8) * U)
    fl = d * T149 / 2
    Epp, Eup = E_p + U * (np_ + E_p) + fl, E_u + U * (nu + E_u) + fl
    P, Uu = np_ + Epp, nu + Eup
    return Epp * nu + P * Eup + (gc + 4 * U) * P * Uu + 4 * U * (1 + P * Uu) + 8192 * d * T149


def screened_i8(p, u):
    """1 - fl(fl(s_p s_u) I), I the exact integer dot product of the codes."""
    qp, sp = int8_codes(p)
    qu, su = int8_codes(u)
    I = np.float32(int((qp * qu).sum()))
    return float(np.float32(np.float32(1) - np.float32(np.float32(sp * su) * I)))


def screened(p, ub, metric, mode):
    """Screened value in float32, several summation orders."""
    if metric == "l2":
        t = (p.astype(np.float32) - ub.astype(np.float32)).astype(np.float32)
        terms = (t * t).astype(np.float32)
    else:
        terms = (p.astype(np.float32) * ub.astype(np.float32)).astype(np.float32)
    if mode == "seq":
        acc = np.float32(0)
        for v in terms:
            acc = np.float32(acc + v)
    elif mode == "rev":
        acc = np.float32(0)
        for v in terms[::-1]:
            acc = np.float32(acc + v)
    else:  # pairwise
        a = terms.copy()
        while a.size > 1:
            if a.size % 2:
                a = np.append(a, np.float32(0))
            a = (a[0::2] + a[1::2]).astype(np.float32)
        acc = a[0]
    if metric == "cosine":
        acc = np.float32(np.float32(1) - acc)
    return float(acc)


def pairs(metric, rng, d):
    out = []
    for _ in range(150):
        scale = np.exp(rng.uniform(-4, 4))
        p = (rng.standard_normal(d) * scale).astype(np.float32)
        u = (p + rng.standard_normal(d) * scale * np.exp(rng.uniform(-8, 1))).astype(np.float32)
        out.append((p, u))
    # adversarial: identical rows, rows differing in one element by one ulp,
    # huge norms with tiny differences, mixed magnitudes, bfloat16 ties
    p = (rng.standard_normal(d) * 1e4).astype(np.float32)
    out.append((p, p.copy()))
    u = p.copy()
    u[3] = np.nextafter(u[3], np.float32(np.inf))
    out.append((p, u))
    out.append((p, (p + 1e-2).astype(np.float32)))
    m = (rng.standard_normal(d) * np.logspace(-20, 5, d)).astype(np.float32)
    out.append((m, (m * 1.001).astype(np.float32)))
    t = ((rng.standard_normal(d).astype(np.float32).view(np.uint32) & 0xFFFF0000) | 0x8000).view(np.float32)
    out.append((t, t.copy()))
    if metric == "cosine":
        out = [(p / np.linalg.norm(p.astype(np.float64)), u / np.linalg.norm(u.astype(np.float64)))
               for p, u in out if np.linalg.norm(p) > 0 and np.linalg.norm(u) > 0]
        out = [(p.astype(np.float32), u.astype(np.float32)) for p, u in out]
    # rows whose squares and products fall in the subnormal range (or below
    # it), where the sums' underflow, not their rounding, decides the error
    for ex in (-60, -64, -68, -72, -76):
        for _ in range(6):
            p = (rng.standard_normal(d) * 2.0 ** ex).astype(np.float32)
            u = (p + rng.standard_normal(d) * 2.0 ** (ex - rng.uniform(0, 6))).astype(np.float32)
            out.append((p, u))
    return out


@pytest.mark.parametrize("metric", ["l2", "cosine"])
@pytest.mark.parametrize("kind", ["bf16", "fp8", "int8"])
@pytest.mark.parametrize("d", [68, 100, 960])
def test_margin_bounds_exact_distance(fgo, metric, kind, d):
    rng = np.random.default_rng(d * 3 + (kind == "fp8") + 7 * (metric == "cosine") + 11 * (kind == "int8"))
    worst = 0.0
    for p, u in pairs(metric, rng, d):
        if kind == "int8" and metric == "cosine":
            # both rows' codes, integer dot product (the kernel's form)
            E_p = np.sqrt(((int8_back(p).astype(np.float64) - p.astype(np.float64)) ** 2).sum())
            E_u = np.sqrt(((int8_back(u).astype(np.float64) - u.astype(np.float64)) ** 2).sum())
            np_ = np.sqrt((p.astype(np.float64) ** 2).sum())
            nu = np.sqrt((u.astype(np.float64) ** 2).sum())
            exact = float(fgo.dist(fgo.Data(np.stack([p, u]), metric=metric), 0, 1))
            dt = screened_i8(p, u)
            eps = margin_i8(E_p, np_, E_u, nu, d)
            assert abs(exact - dt) <= eps, (exact, dt, eps)
            if eps > 0:
                worst = max(worst, abs(dt - exact) / eps)
            continue
        ub = {"bf16": bf16_back, "fp8": fp8_back, "int8": int8_back}[kind](u)
        E = np.sqrt(((ub.astype(np.float64) - u.astype(np.float64)) ** 2).sum())
        np_ = np.sqrt((p.astype(np.float64) ** 2).sum())
        nu = np.sqrt((u.astype(np.float64) ** 2).sum())
        D = fgo.Data(np.stack([p, u]), metric=metric)
        exact = float(fgo.dist(D, 0, 1))
        for mode in ("seq", "rev", "pair"):
            dt = screened(p, ub, metric, mode)
            eps = margin(dt, d, E, np_, nu, metric, fp8_factor(u) if kind == "fp8" else 1.0)
            assert exact >= dt - eps, (mode, exact, dt, eps)
            if eps > 0:
                worst = max(worst, (dt - exact) / eps)
    assert worst <= 1.0


def test_margin_is_not_vacuous_on_neighbours(fgo):
    """On clustered rows the bfloat16 margin is a few percent of a typical
    neighbour distance, so the screen can reject."""
    from paper_2609_30493_amd import datagen as gen
    x = gen.powerlaw_f32(64, 960, 4, 3)
    rel = []
    for i in range(1, 64):
        ub = bf16_back(x[i])
        E = np.sqrt(((ub.astype(np.float64) - x[i].astype(np.float64)) ** 2).sum())
        dt = screened(x[0], ub, "l2", "pair")
        rel.append(margin(dt, 960, E, 0, 0, "l2") / dt)
    assert np.median(rel) < 0.05
