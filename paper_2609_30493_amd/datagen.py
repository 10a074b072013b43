"""Seeded synthetic inputs for the FGraft harvest.

This module only draws numbers: it holds none of the method's arithmetic
(no distances, no search, no pruning), so both the CPU oracle and the HIP
path consume exactly the same arrays.  Every generator is a pure function of
its seed (numpy ``default_rng``), computes in float64 and casts once.

The mixtures stand in for the paper's corpora (Sec. 2, "Systems"): an
isotropic small-d mixture for the frozen-Graft case, a SIFT-128-shaped uint8
mixture, a GloVe-100-shaped unit-norm anisotropic mixture, a GIST-960-shaped
power-law mixture (Sec. 5.4, Tab. 5) and a batch of uneven instances.  None of
the public datasets is reproduced.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np


@dataclasses.dataclass(frozen=True)
class Workload:
    name: str
    n: int
    d: int
    dtype: str          # "f32" or "u8"
    metric: str         # "l2" or "cosine"
    T: int
    B: int
    ef_h: int
    R: int
    alpha: float
    nq: int
    data_seed: int
    recipe: str         # "isotropic", "clustered_u8", "anisotropic_unit", "powerlaw"
    build_seed: int = 42


# The five workloads the measurements are quoted on.
MIX_10K = Workload("frozen-graft n=10k d=32 f32 l2", 10_000, 32, "f32", "l2",
                T=4, B=1, ef_h=32, R=24, alpha=1.2, nq=200, data_seed=1,
                recipe="isotropic")
SIFT_1M = Workload("u8 n=1M d=128 l2 T8 B8 ef64 R32", 1_000_000, 128, "u8", "l2",
                T=8, B=8, ef_h=64, R=32, alpha=1.2, nq=10_000, data_seed=2,
                recipe="clustered_u8")
GLOVE_1183514 = Workload("unit f32 n=1183514 d=100 cosine T8 B8 ef128 R64", 1_183_514, 100,
                "f32", "cosine", T=8, B=8, ef_h=128, R=64, alpha=1.2, nq=10_000,
                data_seed=3, recipe="anisotropic_unit")
GIST_1M = Workload("f32 n=1M d=960 l2 T8 B8 ef128 R64", 1_000_000, 960, "f32", "l2",
                T=8, B=8, ef_h=128, R=64, alpha=1.2, nq=1_000, data_seed=4,
                recipe="powerlaw")


def _chunks(n: int, step: int):
    for s in range(0, n, step):
        yield s, min(n, s + step)


def isotropic_f32(n: int, d: int, k: int, sigma: float, seed: int,
                  centres_seed: int | None = None) -> np.ndarray:
    """x = c_z + sigma * N(0, I), centres ~ U[-1, 1]^d, z ~ U{0..k-1}."""
    crng = np.random.default_rng(seed if centres_seed is None else centres_seed)
    centres = crng.uniform(-1.0, 1.0, size=(k, d))
    rng = np.random.default_rng([seed, 7])
    out = np.empty((n, d), dtype=np.float32)
    for s, e in _chunks(n, 1 << 16):
        z = rng.integers(0, k, size=e - s)
        out[s:e] = (centres[z] + sigma * rng.standard_normal((e - s, d))).astype(np.float32)
    return out


def clustered_u8(n: int, d: int, k: int, sd: float, seed: int,
                 centres_seed: int | None = None) -> np.ndarray:
    """x = clip(rint(c_z + sd * N(0, I)), 0, 255), centres ~ U[0, 255]^d."""
    crng = np.random.default_rng(seed if centres_seed is None else centres_seed)
    centres = crng.uniform(0.0, 255.0, size=(k, d))
    rng = np.random.default_rng([seed, 7])
    out = np.empty((n, d), dtype=np.uint8)
    for s, e in _chunks(n, 1 << 16):
        z = rng.integers(0, k, size=e - s)
        v = np.rint(centres[z] + sd * rng.standard_normal((e - s, d)))
        out[s:e] = np.clip(v, 0, 255).astype(np.uint8)
    return out


def anisotropic_unit_f32(n: int, d: int, k: int, seed: int,
                         centres_seed: int | None = None) -> np.ndarray:
    """Unit rows from a k-component mixture with per-component covariance
    Q_k diag(lambda_k) Q_k^T, lambda ~ Exp(1), Q_k a sign-fixed orthogonal
    factor of a Gaussian matrix; centres ~ N(0, I).  Normalised in float64."""
    crng = np.random.default_rng(seed if centres_seed is None else centres_seed)
    centres = crng.standard_normal((k, d))
    factors = np.empty((k, d, d))
    for c in range(k):
        q, r = np.linalg.qr(crng.standard_normal((d, d)))
        q = q * np.sign(np.diag(r))[None, :]
        lam = crng.exponential(1.0, size=d)
        factors[c] = q * np.sqrt(lam)[None, :]
    rng = np.random.default_rng([seed, 7])
    out = np.empty((n, d), dtype=np.float32)
    for s, e in _chunks(n, 1 << 15):
        z = rng.integers(0, k, size=e - s)
        g = rng.standard_normal((e - s, d))
        v = centres[z] + np.einsum("nij,nj->ni", factors[z], g)
        v /= np.linalg.norm(v, axis=1, keepdims=True)
        out[s:e] = v.astype(np.float32)
    return out


def powerlaw_f32(n: int, d: int, k: int, seed: int, d_total: int | None = None,
                 centres_seed: int | None = None) -> np.ndarray:
    """Per-dimension variance j^-0.5 (j = 1..d_total); centres ~ N(0, diag var);
    x = c_z + N(0, diag var).  With d < d_total the first d dims are kept."""
    dt = d if d_total is None else d_total
    sd = np.arange(1, dt + 1, dtype=np.float64) ** -0.25
    crng = np.random.default_rng(seed if centres_seed is None else centres_seed)
    centres = crng.standard_normal((k, dt)) * sd
    rng = np.random.default_rng([seed, 7])
    out = np.empty((n, d), dtype=np.float32)
    for s, e in _chunks(n, 1 << 14):
        z = rng.integers(0, k, size=e - s)
        v = centres[z] + rng.standard_normal((e - s, dt)) * sd
        out[s:e] = v[:, :d].astype(np.float32)
    return out


def workload_data(w: Workload, n: int | None = None) -> np.ndarray:
    """Data matrix of a workload (optionally only its first n rows' recipe at
    size n, drawn with the same centres)."""
    m = w.n if n is None else n
    return _draw(w, m, w.data_seed, None)


def _draw(w: Workload, m: int, seed: int, centres_seed):
    if w.recipe == "isotropic":
        return isotropic_f32(m, w.d, 16, 0.1, seed, centres_seed)
    if w.recipe == "clustered_u8":
        return clustered_u8(m, w.d, 256, 20.0, seed, centres_seed)
    if w.recipe == "anisotropic_unit":
        return anisotropic_unit_f32(m, w.d, 1000, seed, centres_seed)
    if w.recipe == "powerlaw":
        return powerlaw_f32(m, w.d, 500, seed, None, centres_seed)
    raise ValueError(w.recipe)


def workload_queries(w: Workload, nq: int | None = None) -> np.ndarray:
    """Held-out queries: the same mixture (same centres) with seed + 1000."""
    m = w.nq if nq is None else nq
    return _draw(w, m, w.data_seed + 1000, w.data_seed)


def batched_instances(count: int = 64, seed0: int = 5000, n_lo: int = 5_000,
                      n_hi: int = 200_000, scale: float = 1.0):
    """Uneven instances: n log-uniform in [n_lo, n_hi], d in {32, 96, 128},
    ef_h in {32, 64, 128}, each a seeded 64-component isotropic mixture.
    ``scale`` shrinks every n (for tests)."""
    out = []
    for i in range(count):
        rng = np.random.default_rng(seed0 + i)
        n = int(round(math.exp(rng.uniform(math.log(n_lo), math.log(n_hi))) * scale))
        n = max(n, 16)
        d = int(rng.choice([32, 96, 128]))
        ef = int(rng.choice([32, 64, 128]))
        x = isotropic_f32(n, d, 64, 0.1, seed0 + i)
        out.append(dict(x=x, n=n, d=d, ef_h=ef, T=8, B=8, R=32, alpha=1.2,
                        seed=42 + i))
    return out


def degenerate_f32(kind: str, n: int, d: int, seed: int) -> np.ndarray:
    """Edge-case geometries: 'collinear' (points on a line, deep SAT),
    'duplicates' (many repeated rows), 'identical' (all rows equal)."""
    rng = np.random.default_rng(seed)
    if kind == "collinear":
        t = rng.permutation(n).astype(np.float64)
        v = np.zeros((n, d))
        v[:, 0] = t
        return v.astype(np.float32)
    if kind == "duplicates":
        base = rng.standard_normal((max(1, n // 4), d))
        return base[rng.integers(0, base.shape[0], size=n)].astype(np.float32)
    if kind == "identical":
        return np.tile(rng.standard_normal((1, d)), (n, 1)).astype(np.float32)
    raise ValueError(kind)


def small_u8(n: int, d: int, seed: int, hi: int = 4) -> np.ndarray:
    """Tiny-range integer data: many exact distance ties."""
    rng = np.random.default_rng(seed)
    return rng.integers(0, hi, size=(n, d)).astype(np.uint8)


def hub_u8(n: int, d: int, seed: int, radius: float = 50.0) -> np.ndarray:
    """Row 0 at the centre (128, ..., 128), every other row on a noisy shell
    of the given radius around it: the centre is every point's nearest
    neighbour, so its in-degree in a k-NN-like graph approaches n."""
    rng = np.random.default_rng(seed)
    g = rng.standard_normal((n, d))
    g /= np.linalg.norm(g, axis=1, keepdims=True)
    r = radius * (1.0 + 0.1 * rng.random((n, 1)))
    v = np.clip(np.rint(128.0 + r * g), 0, 255)
    v[0] = 128.0
    return v.astype(np.uint8)


def hub_f32(n: int, d: int, seed: int) -> np.ndarray:
    """Float version of hub_u8: centre at the origin, a noisy unit shell."""
    rng = np.random.default_rng(seed)
    g = rng.standard_normal((n, d))
    g /= np.linalg.norm(g, axis=1, keepdims=True)
    v = g * (1.0 + 0.1 * rng.random((n, 1)))
    v[0] = 0.0
    return v.astype(np.float32)
