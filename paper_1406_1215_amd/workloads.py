"""Seeded synthetic weight vectors (input generators only).

Every workload is a non-increasing float64 weight vector drawn from a
power law, the degree shape the experiments of Sec. 5 use (Table 1 "PL"
networks); none of the paper's real-world degree sequences is used.  This
module holds no part of the generator's arithmetic: it only draws inputs,
which the HIP path and the CPU oracle then receive unchanged.

Sorted samples are drawn as order statistics directly (cumulative sums of
exponential spacings give sorted uniforms), so no sort of 10^9 values is
needed.
"""
from __future__ import annotations

import math

import numpy as np

__all__ = [
    "sorted_uniforms", "powerlaw_truncated", "powerlaw_capped", "powerlaw_mean",
    "config_small", "config_plain", "config_share", "config_batch", "config_calib",
    "tiny_cases",
]


def sorted_uniforms(n: int, rng: np.random.Generator, chunk: int = 1 << 24) -> np.ndarray:
    """n iid U(0,1) values in ascending order (Renyi representation:
    partial sums of n+1 standard exponentials divided by their total)."""
    out = np.empty(n + 1, dtype=np.float64)
    carry = 0.0
    for lo in range(0, n + 1, chunk):
        hi = min(n + 1, lo + chunk)
        rng.standard_exponential(hi - lo, out=out[lo:hi])
        np.cumsum(out[lo:hi], out=out[lo:hi])
        out[lo:hi] += carry
        carry = float(out[hi - 1])
    total = out[n]
    u = out[:n]
    u /= total
    return u


def powerlaw_truncated(n, alpha, lo, hi, rng) -> np.ndarray:
    """Continuous power law with density ~ x^-alpha on [lo, hi], sorted
    non-increasing (inverse-CDF transform of ascending uniforms)."""
    u = sorted_uniforms(n, rng)
    b = 1.0 - alpha
    x = (lo ** b + u * (hi ** b - lo ** b)) ** (1.0 / b)
    return np.ascontiguousarray(x[::-1])


def powerlaw_capped(n, alpha, wmin, rng, max_iter=200) -> np.ndarray:
    """x = wmin U^(-1/(alpha-1)), clipped at c where c = sqrt(sum min(x, c))
    (the largest weight allowed by max_i w_i^2 <= S), sorted non-increasing."""
    u = sorted_uniforms(n, rng)                   # ascending -> x descending
    x = wmin * np.power(u, -1.0 / (alpha - 1.0))
    csum = np.cumsum(x[::-1])[::-1]               # suffix sums, x descending
    c = math.sqrt(float(csum[0]))
    for _ in range(max_iter):
        k = int(np.searchsorted(-x, -c, side="right"))   # #{x >= c}
        tail = float(csum[k]) if k < n else 0.0
        c_new = math.sqrt(k * c + tail)
        if abs(c_new - c) <= 1e-12 * c:
            c = c_new
            break
        c = c_new
    return np.minimum(x, c)


def powerlaw_mean(n, alpha, mean, rng, cap=None, sample_stride=None) -> np.ndarray:
    """w = min(lam * x, cap) with x = U^(-1/(alpha-1)) sorted non-increasing,
    lam chosen by bisection so that mean(w) ~ mean; cap defaults to
    sqrt(n * mean).  For large n, lam is fitted on a strided subsample of the
    sorted x (a stratified sample)."""
    if cap is None:
        cap = math.sqrt(n * mean)
    u = sorted_uniforms(n, rng)
    x = np.power(u, -1.0 / (alpha - 1.0), out=u)
    if sample_stride is None:
        sample_stride = max(1, n // 2_000_000)
    xs = x[::sample_stride]
    lo, hi = 1e-12, float(mean) * 10.0
    while np.minimum(hi * xs, cap).mean() < mean:
        hi *= 2.0
    for _ in range(100):
        mid = 0.5 * (lo + hi)
        if np.minimum(mid * xs, cap).mean() < mean:
            lo = mid
        else:
            hi = mid
    lam = 0.5 * (lo + hi)
    np.multiply(x, lam, out=x)
    np.minimum(x, cap, out=x)
    return x


# ------------------------------------------------------------ the workloads
def config_small(seed: int = 1, n: int = 10_000) -> np.ndarray:
    """Plain CL, n = 1e4, density ~ x^-2.5 on [2, 100]."""
    return powerlaw_truncated(n, 2.5, 2.0, 100.0, np.random.default_rng(seed))


def config_plain(seed: int = 2, n: int = 10_000_000) -> np.ndarray:
    """Plain CL, n = 1e7, exponent 2.1, w_min = 10, clipped at sqrt(S)."""
    return powerlaw_capped(n, 2.1, 10.0, np.random.default_rng(seed))


def config_share(seed: int = 3, n: int = 1_000_000_000) -> np.ndarray:
    """The paper's largest PL shape: n = 1e9, exponent 2.1, mean degree 500,
    cap sqrt(500 n).  8 GB of float64."""
    return powerlaw_mean(n, 2.1, 500.0, np.random.default_rng(seed))


def config_batch(seed: int = 4, G: int = 256):
    """G uneven graphs: n log-uniform in [1e3, 1e6], exponent U(2, 3), mean
    degree U(4, 64); returns a list of (w, philox_seed)."""
    rng = np.random.default_rng(seed)
    shapes = []
    for g in range(G):
        n = int(math.floor(math.exp(rng.uniform(math.log(1e3), math.log(1e6)))))
        alpha = float(rng.uniform(2.0, 3.0))
        dbar = float(rng.uniform(4.0, 64.0))
        shapes.append((n, alpha, dbar))
    out = []
    for g, (n, alpha, dbar) in enumerate(shapes):
        w = powerlaw_mean(n, alpha, dbar, np.random.default_rng(seed * 1_000_003 + g))
        out.append((w, g + 1))
    return out


def config_calib(seed: int = 5, n: int = 100_000) -> np.ndarray:
    """Target degrees: t = min(2 U^(-1/1.1), n^0.8), sorted non-increasing."""
    u = sorted_uniforms(n, np.random.default_rng(seed))
    t = 2.0 * np.power(u, -1.0 / 1.1)
    return np.minimum(t, n ** 0.8)


def tiny_cases(seed: int = 11, count: int = 64):
    """Small edge-case weight vectors: empty, single node, zero weights,
    ties, complete graphs, capped heads, ER (constant) vectors."""
    rng = np.random.default_rng(seed)
    cases = [
        np.zeros(0),
        np.array([3.0]),
        np.array([1.0, 1.0]),
        np.zeros(7),
        np.array([5.0, 3.0, 0.0, 0.0]),
        np.full(64, 64.0),              # w = n, n a power of two: p = 1 for every pair
        np.full(100, 3.0),               # ER with p = 0.03
        np.full(1000, 0.5),              # ER, sparse
        np.array([50.0] * 3 + [2.0] * 50),
    ]
    for _ in range(count):
        n = int(rng.integers(2, 400))
        kind = int(rng.integers(0, 4))
        if kind == 0:
            w = np.sort(rng.pareto(1.5, n) + 1.0)[::-1] * rng.uniform(0.5, 20.0)
        elif kind == 1:
            w = np.sort(rng.uniform(0.0, 30.0, n))[::-1]
        elif kind == 2:
            w = np.sort(rng.integers(0, 6, n).astype(np.float64))[::-1]   # many ties and zeros
        else:
            w = np.sort(rng.pareto(0.8, n) + 1.0)[::-1]                  # very heavy head: capped pairs
        cases.append(np.ascontiguousarray(w, dtype=np.float64))
    return cases
