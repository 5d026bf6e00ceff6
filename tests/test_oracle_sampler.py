"""The oracle's sampler against what Sec. 3 fixes: the exact law of the edge
set (independent pairs, each present with probability min(w_u w_v / S, 1)),
the naive O(n^2) algorithm, the Erdos-Renyi special case, complete graphs,
isolated zero-weight nodes, the invariants (u < v, no duplicates, sorted) and
z-score bounds on m and on the degrees."""
import itertools
import math

import numpy as np
import pytest

import oracle as O
from paper_1406_1215_amd import workloads as W


def _graph_law(w, S):
    """probability of every edge set of a tiny graph (bit masks over pairs)"""
    n = len(w)
    a = np.asarray(w, dtype=np.float64) / S
    pairs = [(u, v) for u in range(n) for v in range(u + 1, n)]
    p = np.array([min(a[u] * w[v], 1.0) for (u, v) in pairs])
    codes = np.arange(1 << len(pairs), dtype=np.int64)
    prob = np.ones(codes.size)
    for i, pi in enumerate(p):
        bit = (codes >> i) & 1
        prob *= np.where(bit == 1, pi, 1.0 - pi)
    return prob


def _chi2_pass(counts, prob, N):
    exp = prob * N
    keep = exp >= 5.0
    # cells with tiny expectation are pooled into one
    obs = np.concatenate([counts[keep], [counts[~keep].sum()]])
    ex = np.concatenate([exp[keep], [exp[~keep].sum()]])
    if ex[-1] < 5.0:
        obs[-2] += obs[-1]
        ex[-2] += ex[-1]
        obs, ex = obs[:-1], ex[:-1]
    # cells with zero probability must stay empty
    assert counts[prob == 0.0].sum() == 0
    chi2 = float(((obs - ex) ** 2 / ex).sum())
    dof = obs.size - 1
    return chi2, dof


@pytest.mark.parametrize("w,e_seg", [
    ([4.0, 3.0, 2.0, 1.5, 1.0], O.E_SEG),          # pair (0,1) capped: w0 w1 / S > 1
    ([4.0, 3.0, 2.0, 1.5, 1.0], 0.01),             # every candidate its own segment
    ([2.0, 2.0, 1.0, 0.5], O.E_SEG),               # ties
    ([3.0, 1.0, 1.0, 0.0], O.E_SEG),               # zero weight node
    ([0.9, 0.8, 0.3, 0.2, 0.1], 0.05),             # segmented, light
])
def test_exact_law_tiny_graphs(w, e_seg):
    w = np.asarray(w)
    S = O.exact_sum(w)
    N = 400_000
    codes = O.graph_codes(w, S, 1, N, e_seg=e_seg).astype(np.int64)
    prob = _graph_law(w, S)
    counts = np.bincount(codes, minlength=prob.size).astype(np.float64)
    chi2, dof = _chi2_pass(counts, prob, N)
    assert chi2 < dof + 5.0 * math.sqrt(2.0 * dof), (chi2, dof)


def test_pair_frequencies_match_naive_algorithm():
    # per-pair frequency against p(u,v) of the naive algorithm, n = 40 with a capped head
    rng = np.random.default_rng(8)
    w = np.sort(rng.pareto(0.9, 40) + 1.0)[::-1] * 3.0
    S = O.exact_sum(w)
    P = O.pair_prob_matrix(w, S)
    assert (P == 1.0).sum() > 0
    R = 4000
    freq = np.zeros_like(P)
    for s in range(R):
        e, m, _, _ = O.generate(w, S, 1000 + s)
        freq[e[:, 0], e[:, 1]] += 1
    iu = np.triu_indices(w.size, k=1)
    p = P[iu]
    f = freq[iu] / R
    assert np.all(f[p == 1.0] == 1.0)
    assert np.all(f[p == 0.0] == 0.0)
    mid = (p > 0) & (p < 1)
    z = (f[mid] - p[mid]) / np.sqrt(p[mid] * (1 - p[mid]) / R)
    assert np.abs(z).max() < 5.0
    assert abs(z.mean()) < 5.0 / math.sqrt(z.size)
    # the brute-force Bernoulli sampler gives the same frequencies (cross-check of the test itself)
    brute = np.zeros_like(P)
    brng = np.random.default_rng(9)
    for _ in range(R):
        e = O.bernoulli_sample(w, S, brng)
        brute[e[:, 0], e[:, 1]] += 1
    zb = (brute[iu][mid] / R - p[mid]) / np.sqrt(p[mid] * (1 - p[mid]) / R)
    assert np.abs(zb).max() < 5.0


def test_erdos_renyi_special_case():
    # constant weights: p = q for every candidate, so every visited candidate is kept
    n, c = 3000, 6.0
    w = np.full(n, c)
    S = O.exact_sum(w)
    p = (c / S) * c
    N = n * (n - 1) // 2
    ms = []
    for seed in range(1, 6):
        e, m, _, cand = O.generate(w, S, seed)
        assert cand == m
        ms.append(m)
    mean = N * p
    sd = math.sqrt(N * p * (1 - p))
    for m in ms:
        assert abs(m - mean) < 5 * sd
    # gaps between consecutive targets of one source are Geometric(p)
    gaps = []
    wb = np.full(200_000, 2000.0)           # p = 0.01
    Sb = O.exact_sum(wb)
    pb = (wb[0] / Sb) * wb[0]
    for seed in range(40):
        v, _ = O.segment_edges(wb, Sb, seed, 0, 0, 1, wb.size)
        prev = 0
        for x in v:
            gaps.append(int(x) - prev - 1)
            prev = int(x)
    gaps = np.array(gaps)
    # chi-square against the geometric law on 20 quantile bins
    qs = np.unique(np.floor(np.log1p(-np.linspace(0, 0.999, 21)[1:-1]) / math.log1p(-pb)).astype(int))
    edges = np.concatenate([[-1], qs, [np.iinfo(np.int64).max]])
    obs = np.array([((gaps > lo) & (gaps <= hi)).sum() for lo, hi in zip(edges[:-1], edges[1:])])
    cdf = lambda k: 1.0 - (1.0 - pb) ** (k + 1)
    probs = np.array([(cdf(hi) if hi < 10**15 else 1.0) - (cdf(lo) if lo >= 0 else 0.0)
                      for lo, hi in zip(edges[:-1], edges[1:])])
    exp = probs * gaps.size
    chi2 = ((obs - exp) ** 2 / exp).sum()
    dof = obs.size - 1
    assert chi2 < dof + 5 * math.sqrt(2 * dof)
    assert abs(gaps.mean() - (1 - pb) / pb) < 5 * math.sqrt((1 - pb) / pb ** 2 / gaps.size)


def test_complete_graph():
    # w_i = n with n a power of two: p = (n / n^2) * n = 1 exactly for every pair
    n = 64
    w = np.full(n, float(n))
    S = O.exact_sum(w)
    e, m, _, _ = O.generate(w, S, 5)
    want = np.array(list(itertools.combinations(range(n), 2)), dtype=np.uint32)
    assert m == n * (n - 1) // 2
    assert np.array_equal(e, want)


def test_zero_weight_nodes_are_isolated():
    rng = np.random.default_rng(10)
    w = np.concatenate([np.sort(rng.uniform(1, 40, 300))[::-1], np.zeros(200)])
    S = O.exact_sum(w)
    for seed in range(3):
        e, m, _, _ = O.generate(w, S, seed)
        assert m > 0
        assert e.max() < 300


def _check_invariants(e, n, u0=0, u1=None):
    if u1 is None:
        u1 = n
    if e.shape[0] == 0:
        return
    u = e[:, 0].astype(np.int64)
    v = e[:, 1].astype(np.int64)
    assert np.all(u < v)
    assert np.all(v < n)
    assert np.all((u >= u0) & (u < u1))
    key = u * (1 << 32) + v
    assert np.all(np.diff(key) > 0)          # sorted by (u,v), no duplicates


def test_invariants_on_edge_cases():
    for i, w in enumerate(W.tiny_cases()):
        if w.size == 0:
            S = 1.0
        else:
            S = O.exact_sum(w)
            if S == 0.0:
                S = 1.0
        e, m, h, _ = O.generate(w, S, 100 + i)
        assert e.shape[0] == m
        _check_invariants(e, w.size)
        assert O.hash_edges(e) == h


def test_node_ranges_are_slices_of_the_whole():
    w = W.config_small(n=3000)
    S = O.exact_sum(w)
    e, m, h, _ = O.generate(w, S, 77)
    for (u0, u1) in [(0, 1), (0, 500), (500, 1700), (2999, 3000), (1700, 1700)]:
        es, ms, hs, _ = O.generate(w, S, 77, u0, u1)
        sel = (e[:, 0] >= u0) & (e[:, 0] < u1)
        assert np.array_equal(es, e[sel])
        off = int(np.argmax(sel)) if sel.any() else 0
        assert O.hash_edges(es, off) == O.hash_edges(e[sel], off)


def test_thread_count_does_not_change_output():
    w = W.config_small(n=5000)
    S = O.exact_sum(w)
    e1, m1, h1, _ = O.generate(w, S, 3, nthreads=1)
    e4, m4, h4, _ = O.generate(w, S, 3, nthreads=4)
    assert m1 == m4 and h1 == h4 and np.array_equal(e1, e4)


def test_edge_count_and_degrees_within_z_bounds():
    w = W.config_small()
    S = O.exact_sum(w)
    E, V = O.expected_edges_closed(w, S)
    P_deg = O.expected_degrees(w, S)
    n = w.size
    # variance of each degree: sum_j p(1-p)
    a = w / S
    for seed in (1, 2, 3):
        e, m, _, _ = O.generate(w, S, seed)
        assert abs(m - E) / math.sqrt(V) < 5.0
        deg = np.bincount(e.ravel().astype(np.int64), minlength=n).astype(np.float64)
        var = np.zeros(n)
        for lo in range(0, n, 2000):
            hi = min(n, lo + 2000)
            # p(u,v) uses the lower index as the source
            Pm = np.minimum(np.where(np.arange(lo, hi)[:, None] < np.arange(n)[None, :],
                                     a[lo:hi, None] * w[None, :], a[None, :] * w[lo:hi, None]), 1.0)
            Pm[np.arange(hi - lo), np.arange(lo, hi)] = 0.0
            var[lo:hi] = (Pm * (1 - Pm)).sum(axis=1)
        ok = var > 0
        z = (deg[ok] - P_deg[ok]) / np.sqrt(var[ok])
        k = ok.sum()
        assert abs((z ** 2).sum() - k) < 5 * math.sqrt(2 * k)
        assert np.abs(z).max() < math.sqrt(2 * math.log(k)) + 3
