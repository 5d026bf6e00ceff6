"""Pins of the oracle's model statistics: E[m], Var[m], expected degrees and
the expected-degree gradient, against brute-force sums, the uncapped closed
forms of Sec. 3 (expected degree w_i - w_i^2/S), central finite differences
and torch's autograd in float64."""
import math

import numpy as np
import pytest

import oracle as O
from paper_1406_1215_amd import workloads as W


def test_expected_edges_closed_matches_all_pairs():
    rng = np.random.default_rng(20)
    for trial in range(6):
        n = int(rng.integers(50, 1500))
        w = np.sort(rng.pareto(rng.uniform(0.6, 2.0), n) + 1.0)[::-1] * rng.uniform(0.5, 30)
        S = O.exact_sum(w)
        E1, V1 = O.expected_edges_brute(w, S)
        E2, V2 = O.expected_edges_closed(w, S)
        assert abs(E1 - E2) <= 1e-10 * E1
        assert abs(V1 - V2) <= 1e-9 * max(V1, 1.0)


def test_expected_edges_uncapped_identity():
    # sum_{u<v} w_u w_v / S = (S^2 - sum w^2) / (2S) when no pair is capped
    w = W.config_small()
    S = O.exact_sum(w)
    assert w[0] * w[0] < S
    E, _ = O.expected_edges_closed(w, S)
    assert abs(E - (S * S - float(np.dot(w, w))) / (2 * S)) <= 1e-9 * E


def test_expected_degree_closed_matches_brute_and_uncapped_form():
    w = W.config_small(n=3000)
    S = O.exact_sum(w)
    d1 = O.expdeg_brute(w, S)
    d2 = O.expdeg_closed(w, S)
    assert np.max(np.abs(d1 - d2) / d1) < 1e-10
    # no capped pair here: d_i = w_i - w_i^2 / S (Sec. 3)
    assert np.max(np.abs(d1 - (w - w * w / S)) / d1) < 1e-10
    # capped regime: targets of the calibration workload, shuffled order
    t = W.config_calib(n=2000)
    rng = np.random.default_rng(21)
    t = t[rng.permutation(t.size)]
    St = O.exact_sum(t)
    assert (t.max() ** 2) > St
    d1 = O.expdeg_brute(t, St)
    d2 = O.expdeg_closed(t, St)
    assert np.max(np.abs(d1 - d2) / d1) < 1e-10


def _loss_grad_fd(w, g, h_rel=1e-6):
    """central differences of L(w) = g . d(w) with S = sum(w)"""
    grad = np.zeros_like(w)
    for k in range(w.size):
        h = h_rel * w[k]
        wp = w.copy(); wp[k] += h
        wm = w.copy(); wm[k] -= h
        Lp = float(g @ O.expdeg_brute(wp, math.fsum(wp.tolist())))
        Lm = float(g @ O.expdeg_brute(wm, math.fsum(wm.tolist())))
        grad[k] = (Lp - Lm) / (2 * h)
    return grad


def test_expected_degree_gradient_fd_and_closed_form():
    rng = np.random.default_rng(22)
    n = 60
    w = rng.pareto(1.0, n) + 1.0
    w *= 3.0
    S = O.exact_sum(w)
    X = np.outer(w, w) / S
    # keep clear of the kink |x - 1| small, where a finite difference straddles it
    assert np.min(np.abs(X - 1.0)) > 1e-4
    assert (X >= 1.0).sum() > n    # capped pairs present
    g = rng.standard_normal(n)
    gb = O.expdeg_grad_brute(w, S, g)
    gc = O.expdeg_grad_closed(w, S, g)
    assert np.max(np.abs(gb - gc)) <= 1e-10 * np.max(np.abs(gb))
    fd = _loss_grad_fd(w, g)
    assert np.linalg.norm(gb - fd) <= 1e-6 * np.linalg.norm(fd)
    # S held fixed: drop the T term
    gfix = O.expdeg_grad_brute(w, S, g, s_depends_on_w=False)
    gfixc = O.expdeg_grad_closed(w, S, g, s_depends_on_w=False)
    assert np.max(np.abs(gfix - gfixc)) <= 1e-10 * np.max(np.abs(gfix))


def test_expected_degree_gradient_vs_torch_autograd():
    torch = pytest.importorskip("torch")
    rng = np.random.default_rng(23)
    n = 40
    w0 = (rng.pareto(1.2, n) + 1.0) * 2.5
    g = rng.standard_normal(n)

    def d_of(w):
        S = w.sum()
        X = torch.minimum(w[:, None] * w[None, :] / S, torch.ones(n, n, dtype=torch.float64))
        X = X - torch.diag(torch.diagonal(X))
        return X.sum(dim=1)

    wt = torch.tensor(w0, dtype=torch.float64, requires_grad=True)
    (d_of(wt) * torch.tensor(g)).sum().backward()
    S = O.exact_sum(w0)
    ref = O.expdeg_grad_brute(w0, S, g)
    assert np.linalg.norm(wt.grad.numpy() - ref) <= 1e-10 * np.linalg.norm(ref)
    w1 = torch.tensor(w0 * 0.3, dtype=torch.float64, requires_grad=True)
    assert torch.autograd.gradcheck(lambda x: d_of(x), (w1,), eps=1e-6, atol=1e-6)
