"""Oracle for the Chung-Lu generator -- TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  The product path (the HIP library and
its binding) never does.

Two halves:

* ``cl_oracle.c`` (loaded here through ctypes): the sampler of Sec. 3, Alg. 1
  with the fixed readings R1-R6 listed in that file, the segmentation of heavy
  sources, the position-keyed digest, and the uniform consecutive partition
  of Sec. 4 (Eq. 2, Eq. 5, Eq. 6, Alg. 2).
* plain numpy / Python below: the exact sum S of Alg. 1 (``math.fsum``), the
  expected edge count and its variance under the capped model
  p(u,v) = min(w_u w_v / S, 1), a brute-force O(n^2) Bernoulli sampler
  (the naive algorithm of Sec. 3), and the expected degree
  d_i = sum_{j != i} min(w_i w_j / S, 1) with its gradient, in float64.
"""
from __future__ import annotations

import ctypes
import math
import os

import numpy as np

from . import build as _build

_LIB = None

ERR = {
    0: "ok", -1: "invalid_arg", -2: "unsorted", -3: "negative",
    -4: "nonfinite", -5: "too_large", -7: "capacity",
}

E_SEG = 256.0  # expected edges per segment of a heavy source (fixed reading R6)

_u64p = ctypes.POINTER(ctypes.c_uint64)
_u32p = ctypes.POINTER(ctypes.c_uint32)
_f64p = ctypes.POINTER(ctypes.c_double)


def lib():
    """Load (building if needed) the C oracle."""
    global _LIB
    if _LIB is not None:
        return _LIB
    path = _build.LIB
    if not os.path.exists(path) or os.path.getmtime(path) < os.path.getmtime(_build.SRC):
        _build.build()
    L = ctypes.CDLL(path)
    L.orc_philox4x32_10.argtypes = [_u32p, _u32p, _u32p]
    L.orc_philox4x32_10.restype = None
    L.orc_u53.argtypes = [ctypes.c_uint64]
    L.orc_u53.restype = ctypes.c_double
    L.orc_poly.argtypes = [ctypes.c_double]
    L.orc_poly.restype = ctypes.c_double
    L.orc_log.argtypes = [ctypes.c_double]
    L.orc_log.restype = ctypes.c_double
    L.orc_log1m.argtypes = [ctypes.c_double]
    L.orc_log1m.restype = ctypes.c_double
    L.orc_validate.argtypes = [_f64p, ctypes.c_uint64, ctypes.c_double]
    L.orc_validate.restype = ctypes.c_int
    L.orc_qscale.argtypes = [_f64p, ctypes.c_uint64]
    L.orc_qscale.restype = ctypes.c_double
    L.orc_qscan.argtypes = [_f64p, ctypes.c_uint64, ctypes.c_double, _u64p]
    L.orc_qscan.restype = None
    L.orc_ehat.argtypes = [_f64p, ctypes.c_uint64, ctypes.c_double, _u64p, ctypes.c_double, ctypes.c_uint64]
    L.orc_ehat.restype = ctypes.c_double
    L.orc_nseg.argtypes = [ctypes.c_uint64, ctypes.c_uint64, ctypes.c_double, ctypes.c_double]
    L.orc_nseg.restype = ctypes.c_uint64
    L.orc_seg_bounds.argtypes = [_u64p, ctypes.c_uint64, ctypes.c_uint64, ctypes.c_uint64, _u32p]
    L.orc_seg_bounds.restype = None
    L.orc_segment.argtypes = [_f64p, ctypes.c_double, ctypes.c_uint64, ctypes.c_uint32, ctypes.c_uint32,
                              ctypes.c_uint32, ctypes.c_uint32, _u32p, ctypes.c_uint64, _u64p]
    L.orc_segment.restype = ctypes.c_uint64
    L.orc_node.argtypes = [_f64p, ctypes.c_uint64, ctypes.c_double, ctypes.c_uint64, _u64p, ctypes.c_double,
                           ctypes.c_double, ctypes.c_uint64, _u32p, ctypes.c_uint64, _u64p, _u64p]
    L.orc_node.restype = ctypes.c_uint64
    L.orc_mix64.argtypes = [ctypes.c_uint64]
    L.orc_mix64.restype = ctypes.c_uint64
    L.orc_hash_edges.argtypes = [_u32p, ctypes.c_uint64, ctypes.c_uint64]
    L.orc_hash_edges.restype = ctypes.c_uint64
    L.orc_generate.argtypes = [_f64p, ctypes.c_uint64, ctypes.c_double, ctypes.c_uint64, ctypes.c_uint64,
                               ctypes.c_uint64, ctypes.c_double, _u32p, ctypes.c_uint64, _u64p, _u64p,
                               ctypes.c_int]
    L.orc_generate.restype = ctypes.c_int64
    L.orc_partition.argtypes = [_f64p, ctypes.c_uint64, ctypes.c_double, ctypes.c_uint64, _u64p, _u64p]
    L.orc_partition.restype = ctypes.c_int
    L.orc_costs.argtypes = [_f64p, ctypes.c_uint64, ctypes.c_double, _u64p]
    L.orc_costs.restype = ctypes.c_int
    L.orc_graph_codes.argtypes = [_f64p, ctypes.c_uint64, ctypes.c_double, ctypes.c_uint64, ctypes.c_uint64,
                                  ctypes.c_double, _u64p]
    L.orc_graph_codes.restype = ctypes.c_int
    L.orc_exact_sum.argtypes = [_f64p, ctypes.c_uint64, _f64p]
    L.orc_exact_sum.restype = ctypes.c_int
    _LIB = L
    return L


def _f64(a):
    a = np.ascontiguousarray(a, dtype=np.float64)
    return a, a.ctypes.data_as(_f64p)


class OracleError(RuntimeError):
    def __init__(self, code):
        super().__init__(f"oracle error {code} ({ERR.get(code, '?')})")
        self.code = code


# ---------------------------------------------------------------- primitives
def philox4x32_10(ctr, key):
    c = (ctypes.c_uint32 * 4)(*[int(x) & 0xFFFFFFFF for x in ctr])
    k = (ctypes.c_uint32 * 2)(*[int(x) & 0xFFFFFFFF for x in key])
    o = (ctypes.c_uint32 * 4)()
    lib().orc_philox4x32_10(c, k, o)
    return tuple(int(x) for x in o)


def u53(x):
    return lib().orc_u53(int(x) & 0xFFFFFFFFFFFFFFFF)


def poly(z):
    return lib().orc_poly(float(z))


def LOG(x):
    return lib().orc_log(float(x))


def LOG1M(p):
    return lib().orc_log1m(float(p))


def mix64(x):
    return lib().orc_mix64(int(x) & 0xFFFFFFFFFFFFFFFF)


# ------------------------------------------------------------- exact sum S
def exact_sum(w) -> float:
    """S of Alg. 1, correctly rounded: the exact real sum of the weights
    rounded once to the nearest double (``math.fsum`` for up to a million
    weights, the C accumulation of the same algorithm beyond)."""
    w = np.asarray(w, dtype=np.float64)
    if w.size <= 1_000_000:
        return math.fsum(w.tolist())
    return exact_sum_c(w)


def exact_sum_c(w) -> float:
    w, wp = _f64(w)
    out = ctypes.c_double(0.0)
    st = lib().orc_exact_sum(wp, w.size, ctypes.byref(out))
    if st != 0:
        raise OracleError(st)
    return out.value


def validate(w, S) -> int:
    w, wp = _f64(w)
    return int(lib().orc_validate(wp, w.size, float(S)))


# -------------------------------------------------------- segmentation (R6)
def qscan(w):
    w, wp = _f64(w)
    L = lib()
    qs = L.orc_qscale(wp, w.size)
    Q = np.zeros(w.size + 1, dtype=np.uint64)
    L.orc_qscan(wp, w.size, qs, Q.ctypes.data_as(_u64p))
    return qs, Q


def segments(w, S, u, e_seg=E_SEG, Q=None, qscale=None):
    """(K_u, [b_0..b_K]) of source u."""
    w, wp = _f64(w)
    n = w.size
    if Q is None:
        qscale, Q = qscan(w)
    L = lib()
    if u + 1 >= n or qscale == 0.0:
        return 1, np.array([min(u + 1, n), n], dtype=np.uint32)
    eh = L.orc_ehat(wp, n, float(S), Q.ctypes.data_as(_u64p), qscale, u)
    K = int(L.orc_nseg(n, u, eh, float(e_seg)))
    b = np.zeros(K + 1, dtype=np.uint32)
    L.orc_seg_bounds(Q.ctypes.data_as(_u64p), n, u, K, b.ctypes.data_as(_u32p))
    return K, b


def ehat(w, S, u, Q=None, qscale=None):
    w, wp = _f64(w)
    if Q is None:
        qscale, Q = qscan(w)
    return lib().orc_ehat(wp, w.size, float(S), Q.ctypes.data_as(_u64p), qscale, u)


def segment_edges(w, S, seed, u, k, j0, end, cap=1 << 22):
    """v's accepted by segment (u,k) over [j0, end) (R1-R5)."""
    w, wp = _f64(w)
    out = np.zeros(cap, dtype=np.uint32)
    nc = ctypes.c_uint64(0)
    a = float(w[u]) / float(S)
    c = lib().orc_segment(wp, a, int(seed), int(u), int(k), int(j0), int(end),
                          out.ctypes.data_as(_u32p), cap, ctypes.byref(nc))
    if c > cap:
        return segment_edges(w, S, seed, u, k, j0, end, cap=int(c))
    return out[:c].copy(), int(nc.value)


def node_edges(w, S, seed, u, Q=None, qscale=None, e_seg=E_SEG, cap=1 << 22):
    w, wp = _f64(w)
    if Q is None:
        qscale, Q = qscan(w)
    out = np.zeros(cap, dtype=np.uint32)
    nc = ctypes.c_uint64(0)
    ks = ctypes.c_uint64(0)
    c = lib().orc_node(wp, w.size, float(S), int(seed), Q.ctypes.data_as(_u64p), qscale, float(e_seg), int(u),
                       out.ctypes.data_as(_u32p), cap, ctypes.byref(nc), ctypes.byref(ks))
    if c > cap:
        return node_edges(w, S, seed, u, Q, qscale, e_seg, cap=int(c))
    return out[:c].copy()


# ------------------------------------------------------------- generation
def generate(w, S, seed, u_begin=0, u_end=None, e_seg=E_SEG, want_edges=True, nthreads=0):
    """Create-Edges(w, S, [u_begin, u_end)).

    Returns (edges (m,2) uint32 or None, m, digest, candidates visited)."""
    w, wp = _f64(w)
    n = w.size
    if u_end is None:
        u_end = n
    L = lib()
    h = ctypes.c_uint64(0)
    nc = ctypes.c_uint64(0)
    m = L.orc_generate(wp, n, float(S), int(seed), int(u_begin), int(u_end), float(e_seg),
                       None, 0, ctypes.byref(h), ctypes.byref(nc), int(nthreads))
    if m < 0:
        raise OracleError(m)
    if not want_edges:
        return None, int(m), int(h.value), int(nc.value)
    edges = np.zeros((max(int(m), 1), 2), dtype=np.uint32)
    m2 = L.orc_generate(wp, n, float(S), int(seed), int(u_begin), int(u_end), float(e_seg),
                        edges.ctypes.data_as(_u32p), int(m), ctypes.byref(h), None, int(nthreads))
    if m2 < 0:
        raise OracleError(m2)
    assert m2 == m
    return edges[: int(m)], int(m), int(h.value), int(nc.value)


def graph_codes(w, S, seed0, nseeds, e_seg=E_SEG):
    """Edge sets of nseeds runs on a tiny graph (n <= 11) as pair bit masks."""
    w, wp = _f64(w)
    out = np.zeros(int(nseeds), dtype=np.uint64)
    st = lib().orc_graph_codes(wp, w.size, float(S), int(seed0), int(nseeds), float(e_seg),
                               out.ctypes.data_as(_u64p))
    if st != 0:
        raise OracleError(st)
    return out


def hash_edges(edges, index_base=0):
    e = np.ascontiguousarray(edges, dtype=np.uint32)
    return int(lib().orc_hash_edges(e.ctypes.data_as(_u32p), e.shape[0], int(index_base)))


# ------------------------------------------------------------ partition
def partition(w, S, P):
    """Uniform consecutive partition (Alg. 2 / Eq. 5): bounds n_0..n_P."""
    w, wp = _f64(w)
    b = np.zeros(int(P) + 1, dtype=np.uint64)
    z = ctypes.c_uint64(0)
    st = lib().orc_partition(wp, w.size, float(S), int(P), b.ctypes.data_as(_u64p), ctypes.byref(z))
    if st != 0:
        raise OracleError(st)
    return b, int(z.value)


def costs(w, S):
    """Per-source cost c_u = floor(256 e_u) + 256 (Eq. 2 in units of 1/256)."""
    w, wp = _f64(w)
    c = np.zeros(max(w.size, 1), dtype=np.uint64)
    st = lib().orc_costs(wp, w.size, float(S), c.ctypes.data_as(_u64p))
    if st != 0:
        raise OracleError(st)
    return c[: w.size]


# ------------------------------------------- model statistics (float64)
def pair_prob_matrix(w, S):
    """p(u,v) = min((w_u/S) w_v, 1) for u < v (the sampler's own rounding);
    zero on and below the diagonal.  O(n^2) memory: tiny n only."""
    w = np.asarray(w, dtype=np.float64)
    a = w / S
    P = np.minimum(a[:, None] * w[None, :], 1.0)
    return np.triu(P, k=1)


def expected_edges_brute(w, S, block=2048):
    """E[m] = sum_{u<v} p(u,v) and Var[m] = sum p(1-p), by summing all pairs."""
    w = np.asarray(w, dtype=np.float64)
    n = w.size
    a = w / S
    E = 0.0
    V = 0.0
    for lo in range(0, n, block):
        hi = min(n, lo + block)
        P = np.minimum(a[lo:hi, None] * w[None, :], 1.0)
        cols = np.arange(n)[None, :]
        rows = np.arange(lo, hi)[:, None]
        P = np.where(cols > rows, P, 0.0)
        E += float(P.sum())
        V += float((P * (1.0 - P)).sum())
    return E, V


def _first_uncapped(a, w):
    """J_u = first v > u with a_u * w_v < 1 (w non-increasing), by bisection on
    the sampler's own product a_u * w_v."""
    n = w.size
    lo = np.arange(n, dtype=np.int64) + 1
    hi = np.full(n, n, dtype=np.int64)
    while True:
        act = lo < hi
        if not act.any():
            break
        mid = (lo + hi) // 2
        midc = np.minimum(mid, n - 1)
        capped = (a * w[midc]) >= 1.0
        lo = np.where(act & capped, mid + 1, lo)
        hi = np.where(act & ~capped, mid, hi)
    return lo


def expected_edges_closed(w, S):
    """Sorted closed form: for each u the capped candidates u+1..J_u-1 count 1,
    the rest a_u * sum_{v >= J_u} w_v (Eq. 1 with the cap)."""
    w = np.asarray(w, dtype=np.float64)
    n = w.size
    if n == 0:
        return 0.0, 0.0
    a = w / S
    J = _first_uncapped(a, w)
    suf = np.concatenate([np.cumsum(w[::-1])[::-1], [0.0]])
    suf2 = np.concatenate([np.cumsum((w * w)[::-1])[::-1], [0.0]])
    cnt_cap = (J - np.arange(n) - 1).astype(np.float64)
    E = float(cnt_cap.sum() + (a * suf[J]).sum())
    V = float((a * suf[J] - a * a * suf2[J]).sum())
    return E, V


def expected_degrees(w, S):
    """Expected degree of every node under the capped model (sum over j != i)."""
    w = np.asarray(w, dtype=np.float64)
    return expdeg_closed(w, S)


def bernoulli_sample(w, S, rng):
    """The naive O(n^2) algorithm of Sec. 3: one trial per pair."""
    P = pair_prob_matrix(w, S)
    U = rng.random(P.shape)
    iu, iv = np.nonzero((U < P) & (np.triu(np.ones_like(P), k=1) > 0))
    return np.stack([iu, iv], axis=1).astype(np.uint32)


# ------------------------------------------ expected degree (float64)
def expdeg_brute(w, S, block=1024):
    """d_i = sum_{j != i} min(w_i w_j / S, 1), all pairs, float64."""
    w = np.asarray(w, dtype=np.float64)
    n = w.size
    d = np.zeros(n)
    for lo in range(0, n, block):
        hi = min(n, lo + block)
        X = np.minimum(w[lo:hi, None] * w[None, :] / S, 1.0)
        X[np.arange(hi - lo), np.arange(lo, hi)] = 0.0
        d[lo:hi] = X.sum(axis=1)
    return d


def expdeg_grad_brute(w, S, g, s_depends_on_w=True, block=1024):
    """dL/dw_k for L with dL/dd = g, d as in expdeg_brute, S = sum(w) when
    s_depends_on_w (then dS/dw_k = 1), else S held fixed.  Pairs with
    x_ij >= 1 are capped (zero derivative)."""
    w = np.asarray(w, dtype=np.float64)
    g = np.asarray(g, dtype=np.float64)
    n = w.size
    A = np.zeros(n)
    B = np.zeros(n)
    U = np.zeros(n)
    for lo in range(0, n, block):
        hi = min(n, lo + block)
        X = w[lo:hi, None] * w[None, :] / S
        M = (X < 1.0).astype(np.float64)
        M[np.arange(hi - lo), np.arange(lo, hi)] = 0.0
        A[lo:hi] = M @ w
        B[lo:hi] = M @ (g * w)
        U[lo:hi] = (M * X).sum(axis=1)
    T = float(g @ U) if s_depends_on_w else 0.0
    return (g * A + B - T) / S


def expdeg_closed(w, S):
    """Sorted closed form of the expected degree (any order of w accepted)."""
    w = np.asarray(w, dtype=np.float64)
    n = w.size
    order = np.argsort(-w, kind="stable")
    ws = w[order]
    a = ws / S
    J = _count_capped(a, ws)
    suf = np.concatenate([np.cumsum(ws[::-1])[::-1], [0.0]])
    idx = np.arange(n)
    own_capped = idx < J
    d = (J - own_capped) + a * (suf[J] - np.where(own_capped, 0.0, ws))
    out = np.empty(n)
    out[order] = d
    return out


def _count_capped(a, ws):
    """J_i = #{j : ws_i ws_j / S >= 1} for ws sorted non-increasing, with the
    product formed as (w_i/S) * w_j."""
    n = ws.size
    lo = np.zeros(n, dtype=np.int64)
    hi = np.full(n, n, dtype=np.int64)
    while True:
        act = lo < hi
        if not act.any():
            break
        mid = (lo + hi) // 2
        midc = np.minimum(mid, n - 1)
        capped = (a * ws[midc]) >= 1.0
        lo = np.where(act & capped, mid + 1, lo)
        hi = np.where(act & ~capped, mid, hi)
    return lo


def expdeg_grad_closed(w, S, g, s_depends_on_w=True):
    w = np.asarray(w, dtype=np.float64)
    g = np.asarray(g, dtype=np.float64)
    n = w.size
    order = np.argsort(-w, kind="stable")
    ws = w[order]
    gs = g[order]
    a = ws / S
    J = _count_capped(a, ws)
    idx = np.arange(n)
    own_unc = idx >= J
    sw = np.concatenate([np.cumsum(ws[::-1])[::-1], [0.0]])
    sgw = np.concatenate([np.cumsum((gs * ws)[::-1])[::-1], [0.0]])
    A = sw[J] - np.where(own_unc, ws, 0.0)
    B = sgw[J] - np.where(own_unc, gs * ws, 0.0)
    U = a * A
    T = float(gs @ U) if s_depends_on_w else 0.0
    gr = (gs * A + B - T) / S
    out = np.empty(n)
    out[order] = gr
    return out
