"""GPU parity of batched generation (many graphs in one plan, one captured
HIP graph) against the oracle.

* The 256-graph workload at full size (n log-uniform in [1e3, 1e6], exponent
  U(2, 3), mean degree U(4, 64), 6.1e8 edges): every graph's edge count and
  position-keyed digest equal the oracle's, stored in
  ``tests/golden/batch_256.json`` by ``tests/golden/make_golden.py`` (which
  calls only the oracle); sampled sources of several graphs are compared edge
  by edge with live oracle runs; both planners, through replays of the
  captured graph.
* A batch whose last task is large enough for graded tail units (only the
  last task of a batch gets them): edge lists bit-exact with the oracle, with
  graded and with uniform units, plain and captured.
* 200 seeded random small graphs of many kinds (ties, zero tails, capped
  heads, constant weights, random source ranges) in one plan, plain and
  captured, bit-exact with the oracle.
"""
import json
import os

import numpy as np
import pytest

import oracle as O
from paper_1406_1215_amd import workloads as W

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "batch_256.json")


@pytest.fixture(scope="module")
def cg():
    from conftest import gpu_available
    if not gpu_available():
        pytest.skip("no GPU")
    from paper_1406_1215_amd import clgen
    clgen.lib()
    return clgen


def _to_dev(w):
    import torch
    return torch.from_numpy(np.ascontiguousarray(w, dtype=np.float64)).to("cuda:0")


def _edges_np(t):
    return t.cpu().numpy().view(np.uint32).reshape(-1, 2)


_BATCH = {}


def _batch(cg):
    if not _BATCH:
        with open(GOLDEN) as f:
            gold = json.load(f)
        graphs = W.config_batch()
        tasks = []
        for (w, seed), gg in zip(graphs, gold["graphs"]):
            assert w.size == gg["n"] and seed == gg["seed"]
            wd = _to_dev(w)
            S = cg.cl_weight_sum(wd)
            assert S == float.fromhex(gg["S"]), gg["g"]
            tasks.append(cg.Task(wd, S, seed))
        _BATCH.update(gold=gold, graphs=graphs, tasks=tasks)
    return _BATCH


def _per_graph_digests(cg, edges, offsets):
    """Digest of each graph's slice of the batch output, positions counted
    from the graph's first edge."""
    import torch
    G = offsets.numel() - 1
    acc = torch.zeros(G, dtype=torch.int64, device=edges.device)
    off = offsets.cpu().numpy()
    for g in range(G):
        if off[g + 1] > off[g]:
            cg.cl_hash_edges(edges[off[g]:off[g + 1]], 0, acc[g:g + 1])
    return [int(x) & ((1 << 64) - 1) for x in acc.cpu().numpy()], off


@pytest.mark.parametrize("planner", ["cl_sample", "cl_count"])
def test_batch_256_graphs_match_oracle(cg, planner):
    import torch
    B = _batch(cg)
    gold, tasks, graphs = B["gold"], B["tasks"], B["graphs"]
    want_m = [g["m"] for g in gold["graphs"]]
    want_h = [g["digest"] for g in gold["graphs"]]
    plan = getattr(cg, planner)(tasks)
    assert plan.m == want_m
    assert plan.total == gold["total_edges"]
    s = torch.cuda.Stream()
    bg = cg.cl_batch_capture(plan, s, cap=plan.total)
    rng = np.random.default_rng(44)
    sample_graphs = [0, 1, 255] + [int(x) for x in rng.integers(0, 256, 3)]
    for rep in range(2):
        bg.edges.fill_(-1)
        bg.graph_offsets.fill_(-1)
        torch.cuda.synchronize()
        bg.launch(s)
        s.synchronize()
        h, off = _per_graph_digests(cg, bg.edges, bg.graph_offsets)
        assert list(np.diff(off)) == want_m, rep
        bad = [g for g in range(len(tasks)) if h[g] != want_h[g]]
        assert not bad, (rep, bad[:10])
        x = torch.ones(1000, device="cuda:0").sum()   # eager work between replays
        assert float(x) == 1000.0
    # sampled sources, edge by edge against single-source oracle runs
    e = _edges_np(bg.edges[: plan.total])
    for g in sample_graphs:
        w, seed = graphs[g]
        S = tasks[g].S
        qs, Q = O.qscan(w)
        ge = e[off[g]:off[g + 1]]
        us = ge[:, 0]
        for u in [0, 1, w.size - 2] + [int(x) for x in rng.integers(0, w.size, 5)]:
            want_v = O.node_edges(w, S, seed, int(u), Q=Q, qscale=qs)
            lo = np.searchsorted(us, u, side="left")
            hi = np.searchsorted(us, u, side="right")
            assert np.array_equal(ge[lo:hi, 1], want_v), (g, int(u))
    bg.close()


@pytest.mark.parametrize("planner", ["cl_sample", "cl_count"])
def test_graded_tail_units_inside_a_batch(cg, planner):
    """Small graphs first, then a power-law graph of several thousand units
    last (the only task that gets graded units): every graph bit-exact with
    the oracle, with graded and uniform units, plain and through a captured
    graph."""
    import torch
    rng = np.random.default_rng(81)
    ws_ = [W.config_small(seed=int(rng.integers(1 << 30)), n=int(rng.integers(50, 20000))) for _ in range(5)]
    ws_ += [W.config_plain(n=1_000_000)]
    tasks, wants = [], []
    for i, w in enumerate(ws_):
        S = O.exact_sum(w)
        wants.append(O.generate(w, S, 900 + i)[0])
        tasks.append(cg.Task(_to_dev(w), S, 900 + i))
    want = np.concatenate(wants)
    lanes = {}
    for tail in (0, 1):
        plan = getattr(cg, planner)(tasks, tuning={"tail_units": tail})
        assert plan.m == [x.shape[0] for x in wants]
        lanes[tail] = cg.cl_plan_info(plan)["lanes"]
        got = _edges_np(cg.cl_generate(plan))[: plan.total]
        assert np.array_equal(got, want), tail
        s = torch.cuda.Stream()
        bg = cg.cl_batch_capture(plan, s)
        for rep in range(2):
            bg.edges.fill_(-1)
            torch.cuda.synchronize()
            bg.launch(s)
            s.synchronize()
            assert np.array_equal(_edges_np(bg.edges)[: plan.total], want), (tail, rep)
        bg.close()
    # the last graph alone has >= 4096 uniform units, so grading applies to it
    assert lanes[1] >= 4096 and lanes[0] > lanes[1]


def _random_graphs(seed, count):
    """Seeded small weight vectors of many kinds: ties, zero tails, capped
    heads, constant (ER), single nodes, heavy Pareto heads; each with a
    random source range."""
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(count):
        n = int(rng.integers(1, 3000))
        kind = int(rng.integers(0, 6))
        if kind == 0:
            w = np.sort(rng.pareto(float(rng.uniform(0.6, 2.5)), n) + 1.0)[::-1] * rng.uniform(0.1, 50.0)
        elif kind == 1:
            w = np.sort(rng.integers(0, 5, n).astype(np.float64))[::-1]
        elif kind == 2:
            w = np.full(n, float(rng.uniform(0.5, 40.0)))
        elif kind == 3:
            k = int(rng.integers(0, n + 1))
            w = np.concatenate([np.sort(rng.uniform(1.0, 200.0, k))[::-1], np.zeros(n - k)])
        elif kind == 4:
            w = np.sort(rng.uniform(0.0, 1.0, n))[::-1] ** 3 * float(n)
        else:
            w = np.sort(rng.lognormal(2.0, 1.5, n))[::-1]
        w = np.ascontiguousarray(w, dtype=np.float64)
        u0 = int(rng.integers(0, n + 1))
        u1 = int(rng.integers(u0, n + 1))
        if rng.random() < 0.5:
            u0, u1 = 0, n
        out.append((w, u0, u1, int(rng.integers(0, 1 << 62))))
    return out


@pytest.mark.parametrize("planner", ["cl_sample", "cl_count"])
def test_many_random_small_graphs_in_one_batch(cg, planner):
    """200 seeded random graphs of every kind in one plan, plain and replayed
    from a captured graph: each graph's edge list equals the oracle's."""
    import torch
    cases = _random_graphs(123 if planner == "cl_sample" else 456, 200)
    tasks, wants = [], []
    for w, u0, u1, seed in cases:
        S = O.exact_sum(w)
        if S == 0.0:
            S = 1.0
        wants.append(O.generate(w, S, seed, u0, u1)[0])
        tasks.append(cg.Task(_to_dev(w), S, seed, u0, u1))
    plan = getattr(cg, planner)(tasks)
    assert plan.m == [x.shape[0] for x in wants]
    want = np.concatenate(wants)
    go = torch.zeros(len(tasks) + 1, dtype=torch.int64, device="cuda:0")
    got = _edges_np(cg.cl_generate(plan, graph_offsets=go))[: plan.total]
    assert np.array_equal(got, want)
    assert list(np.diff(go.cpu().numpy())) == plan.m
    s = torch.cuda.Stream()
    bg = cg.cl_batch_capture(plan, s)
    bg.edges.fill_(-1)
    torch.cuda.synchronize()
    bg.launch(s)
    s.synchronize()
    assert np.array_equal(_edges_np(bg.edges)[: plan.total], want)
    bg.close()
