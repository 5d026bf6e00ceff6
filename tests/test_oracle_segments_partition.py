"""Pins of the oracle's task splitting and partitioning.

* the quantised prefix Q against the real running sum sigma of Eq. 6;
* e_u against Eq. 1 evaluated with an exactly rounded sum;
* segment starts against their definition, by a linear scan;
* Eq. 2/4 (cost = m + n), Lemma 1 (costs non-increasing), Eq. 5 (argmin,
  brute force in Python integers), and the ER observation of Sec. 4 (at most
  two boundaries per block)."""
import math

import numpy as np
import pytest

import oracle as O
from paper_1406_1215_amd import workloads as W


def _heavy_weights(n=3000, seed=12):
    rng = np.random.default_rng(seed)
    return np.sort(rng.pareto(1.1, n) + 1.0)[::-1] * 40.0


def test_q_prefix_tracks_running_sum():
    w = _heavy_weights()
    qs, Q = O.qscan(w)
    assert qs == 2.0 ** 32 / w[0]
    sigma = np.concatenate([[0.0], np.cumsum(w)])
    # each quantised weight loses less than one unit of 1/QSCALE
    err = sigma - Q.astype(np.float64) / qs
    idx = np.arange(w.size + 1)
    assert np.all(err >= -1e-9 * sigma - 1e-12)
    assert np.all(err <= idx / qs + 1e-9 * sigma + 1e-12)
    # and the increments are floor(w_v * QSCALE), at most 2^32
    q = np.diff(Q.astype(np.int64))
    assert q.max() <= 2 ** 32
    assert np.all(q == np.floor(w * qs).astype(np.int64))


def test_ehat_matches_eq1():
    w = _heavy_weights()
    S = O.exact_sum(w)
    qs, Q = O.qscan(w)
    n = w.size
    for u in [0, 1, 5, 100, 1000, n - 2, n - 1]:
        e_eq1 = (w[u] / S) * math.fsum(w[u + 1:].tolist())
        eh = O.ehat(w, S, u, Q, qs)
        # quantisation costs at most (n-u-1)/QSCALE of mass
        tol = (w[u] / S) * (n - u) / qs + 1e-12 * max(e_eq1, 1.0)
        assert abs(eh - e_eq1) <= tol


def test_segment_starts_follow_their_definition():
    w = _heavy_weights()
    S = O.exact_sum(w)
    qs, Q = O.qscan(w)
    n = w.size
    Qi = [int(x) for x in Q]
    heavy = 0
    for u in range(0, 400, 7):
        K, b = O.segments(w, S, u, Q=Q, qscale=qs)
        eh = O.ehat(w, S, u, Q, qs)
        if eh > O.E_SEG and u + 2 < n:
            heavy += 1
            assert K == min(math.ceil(eh / O.E_SEG), n - u - 1)
        else:
            assert K == 1
        assert b[0] == u + 1 and b[K] == n
        assert np.all(np.diff(b.astype(np.int64)) >= 0)
        D = Qi[n] - Qi[u + 1]
        for k in range(1, K):
            target = Qi[u + 1] + (k * D) // K        # Python big integers
            v = u + 1
            while Qi[v] < target:                   # linear scan, independent of the bisection
                v += 1
            assert b[k] == v
    assert heavy > 10


def test_segments_cover_each_source_once():
    # the union of a source's segments is [u+1, n) and the edges agree with a
    # per-segment run
    w = _heavy_weights(1500, 13)
    S = O.exact_sum(w)
    qs, Q = O.qscan(w)
    for u in (0, 3, 20):
        K, b = O.segments(w, S, u, Q=Q, qscale=qs)
        assert K > 1
        parts = [O.segment_edges(w, S, 9, u, k, int(b[k]), int(b[k + 1]))[0] for k in range(K)]
        got = np.concatenate(parts)
        assert np.array_equal(got, O.node_edges(w, S, 9, u, Q=Q, qscale=qs))
        for k in range(K):
            assert np.all((parts[k] >= b[k]) & (parts[k] < b[k + 1]))


def test_segmented_and_unsegmented_laws_agree():
    # restarting the memoryless skip at fixed points leaves the pair law unchanged:
    # per-pair frequencies of heavily segmented runs match p(u,v)
    rng = np.random.default_rng(14)
    w = np.sort(rng.pareto(1.0, 30) + 1.0)[::-1] * 2.5
    S = O.exact_sum(w)
    P = O.pair_prob_matrix(w, S)
    R = 4000
    for e_seg in (0.3, 1e300):
        freq = np.zeros_like(P)
        for s in range(R):
            e, m, _, _ = O.generate(w, S, 5000 + s, e_seg=e_seg)
            freq[e[:, 0], e[:, 1]] += 1
        iu = np.triu_indices(w.size, k=1)
        p, f = P[iu], freq[iu] / R
        mid = (p > 0) & (p < 1)
        z = (f[mid] - p[mid]) / np.sqrt(p[mid] * (1 - p[mid]) / R)
        assert np.abs(z).max() < 5.0
        assert np.all(f[p == 1.0] == 1.0)


# ----------------------------------------------------------------- partition
def test_costs_follow_eq2_and_eq4_and_lemma1():
    w = W.config_small()
    S = O.exact_sum(w)
    c = O.costs(w, S).astype(np.float64)
    n = w.size
    suffix = np.concatenate([np.cumsum(w[::-1])[::-1][1:], [0.0]])
    e = (w / S) * suffix                                   # Eq. 1
    assert np.all(np.abs(c / 256.0 - (e + 1.0)) <= 1.0 / 256 + 1e-6 * e)
    # Lemma 1: c_u >= c_v for u < v
    assert np.all(np.diff(c) <= 0)
    # Eq. 4: total cost = m + n with m = sum e_u = (S^2 - sum w^2) / (2S) uncapped
    m_unc = (S * S - float(np.dot(w, w))) / (2 * S)
    assert abs(c.sum() / 256.0 - (m_unc + n)) <= n / 256.0 + 1e-9 * m_unc


def _eq5_bruteforce(c, P):
    C = np.cumsum(c.astype(object))            # exact Python integers
    Z = int(C[-1])
    n = c.size
    bounds = [0]
    for k in range(1, P):
        u = 0
        while not (int(C[u]) * P >= k * Z):
            u += 1
        bounds.append(u)
    bounds.append(n)
    return bounds, Z


@pytest.mark.parametrize("P", [1, 2, 7, 64, 300])
def test_partition_is_eq5_argmin(P):
    w = W.config_small(n=4000)
    S = O.exact_sum(w)
    b, Z = O.partition(w, S, P)
    want, Zw = _eq5_bruteforce(O.costs(w, S), P)
    assert Z == Zw
    assert [int(x) for x in b] == want


def test_partition_with_jumps_and_empty_parts():
    # one source costlier than several average partitions: boundaries repeat
    w = np.array([1000.0, 900.0] + [1.0] * 60)
    S = O.exact_sum(w)
    P = 16
    b, Z = O.partition(w, S, P)
    want, _ = _eq5_bruteforce(O.costs(w, S), P)
    assert [int(x) for x in b] == want
    assert len(set(want)) < len(want)               # some partitions are empty


def test_partition_more_parts_than_nodes():
    w = np.array([3.0, 2.0, 1.0])
    S = O.exact_sum(w)
    b, Z = O.partition(w, S, 10)
    want, _ = _eq5_bruteforce(O.costs(w, S), 10)
    assert [int(x) for x in b] == want
    b1, _ = O.partition(np.zeros(0), 1.0, 4)
    assert [int(x) for x in b1] == [0, 0, 0, 0, 0]


def test_partition_balances_cost():
    w = W.config_small()
    S = O.exact_sum(w)
    c = O.costs(w, S)
    P = 32
    b, Z = O.partition(w, S, P)
    Zbar = Z / P
    for i in range(P):
        part = int(c[int(b[i]):int(b[i + 1])].sum())
        assert part <= Zbar + int(c.max())


def test_er_has_at_most_two_boundaries_per_block():
    # Sec. 4 (Fig. 3 discussion): for ER inputs no block of n/P nodes holds more
    # than two partition boundaries
    n = 20000
    w = np.full(n, 50.0)
    S = O.exact_sum(w)
    for P in (4, 16, 64, 256):
        b, _ = O.partition(w, S, P)
        inner = np.array([int(x) for x in b[1:-1]])
        for i in range(P):
            lo, hi = (i * n) // P, ((i + 1) * n) // P
            assert ((inner >= lo) & (inner < hi)).sum() <= 2
