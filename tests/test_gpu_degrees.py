"""GPU: degrees of generated graphs without storing edges (cl_degrees),
against the degree counts of the oracle's edge lists, bit-exact."""
import math

import numpy as np
import pytest

import oracle as O
from paper_1406_1215_amd import workloads as W

pytestmark = pytest.mark.gpu

PLANNERS = ["cl_count", "cl_sample", "cl_plan"]


@pytest.fixture(scope="module")
def cg():
    from conftest import gpu_available
    if not gpu_available():
        pytest.skip("no GPU")
    from paper_1406_1215_amd import clgen
    clgen.lib()
    return clgen


def _dev(w):
    import torch
    return torch.from_numpy(np.ascontiguousarray(w, dtype=np.float64)).to("cuda:0")


def _oracle_degrees(w, S, seed, u0=0, u1=None):
    edges, m, _, _ = O.generate(w, S, seed, u0, u1)
    return np.bincount(edges.ravel().astype(np.int64), minlength=w.size).astype(np.int64), m


@pytest.mark.parametrize("planner", PLANNERS)
def test_degrees_small_config(cg, planner):
    w = W.config_small()
    S = O.exact_sum(w)
    want, m = _oracle_degrees(w, S, 1)
    plan = getattr(cg, planner)([cg.Task(_dev(w), S, 1)])
    (deg,) = cg.cl_degrees(plan)
    got = deg.cpu().numpy().view(np.uint32).astype(np.int64)
    assert np.array_equal(got, want)
    assert got.sum() == 2 * m
    if planner != "cl_plan":
        assert plan.total == m


@pytest.mark.parametrize("n", [100_000, 1_000_000])
def test_degrees_plain_shapes_and_ranges(cg, n):
    w = W.config_plain(n=n)
    S = O.exact_sum(w)
    want, m = _oracle_degrees(w, S, 7)
    plan = cg.cl_sample([cg.Task(_dev(w), S, 7)])
    (deg,) = cg.cl_degrees(plan)
    assert np.array_equal(deg.cpu().numpy().view(np.uint32).astype(np.int64), want)
    # the parts of a partition accumulate into one array: same degrees
    bounds, _ = cg.cl_partition(_dev(w), S, 3)
    import torch
    acc = torch.zeros(n + 1, dtype=torch.int32, device="cuda:0")
    for a, b in zip(bounds[:-1], bounds[1:]):
        part = cg.cl_plan([cg.Task(_dev(w), S, 7, a, b)])
        cg.cl_degrees(part, deg=acc)
    assert np.array_equal(acc[:n].cpu().numpy().view(np.uint32).astype(np.int64), want)


def test_degrees_batch_of_uneven_graphs(cg):
    rng = np.random.default_rng(21)
    ws = [W.powerlaw_capped(int(n), a, 2.0, np.random.default_rng(int(n)))
          for n, a in zip(rng.integers(1, 30000, 6), rng.uniform(2.0, 3.0, 6))]
    ws.append(np.zeros(4))
    tasks, wants = [], []
    for i, w in enumerate(ws):
        S = O.exact_sum(w) if w.sum() > 0 else 1.0
        wants.append(_oracle_degrees(w, S, 100 + i)[0])
        tasks.append(cg.Task(_dev(w), S, 100 + i))
    plan = cg.cl_sample(tasks)
    degs = cg.cl_degrees(plan)
    for d, want in zip(degs, wants):
        assert np.array_equal(d.cpu().numpy().view(np.uint32).astype(np.int64), want)


def test_degrees_capacity_error(cg):
    import torch
    w = W.config_small(n=2000)
    S = O.exact_sum(w)
    plan = cg.cl_count([cg.Task(_dev(w), S, 1)])
    with pytest.raises(cg.ClError):
        cg.cl_degrees(plan, deg=torch.zeros(100, dtype=torch.int32, device="cuda:0"))


def test_plan_only_workspace_writes_no_edges(cg):
    import torch
    w = W.config_small(n=3000)
    S = O.exact_sum(w)
    plan = cg.cl_plan([cg.Task(_dev(w), S, 2)])
    out = torch.full((64, 2), -1, dtype=torch.int32, device="cuda:0")
    cg.cl_generate(plan, edges=out, cap=64)
    torch.cuda.synchronize()
    assert bool((out == -1).all())


def test_parts_give_the_whole_graph(cg):
    """Degrees accumulated over a 5-part partition (parts.degrees) equal the
    one-plan degrees and the degree counts of the oracle's edge list."""
    from paper_1406_1215_amd import parts
    w = W.config_plain(n=300_000)
    S = O.exact_sum(w)
    want, m = _oracle_degrees(w, S, 5)
    res = parts.degrees(_dev(w), S, 5, parts=5)
    assert res["edges"] == m
    assert np.array_equal(res["deg"].cpu().numpy().view(np.uint32).astype(np.int64), want)


@pytest.mark.parametrize("budget", [32, 192])
@pytest.mark.parametrize("policy", [1, 2])
def test_degrees_under_every_unit_policy(cg, policy, budget):
    """Units of equal source counts (1) and round-robin units (2, Sec. 4's
    RRP over segments: unit i takes segments i, i + L, ...) change only the
    schedule: the degrees equal the oracle's, bit for bit, on a workload
    with heavy (segmented) sources."""
    w = W.config_plain(n=200_000)
    S = O.exact_sum(w)
    want, _ = _oracle_degrees(w, S, 9)
    plan = cg.cl_plan([cg.Task(_dev(w), S, 9)], tuning={"partition": policy, "lane_budget": budget})
    assert cg.cl_plan_info(plan)["heavy_segments"] > 0
    (deg,) = cg.cl_degrees(plan)
    assert np.array_equal(deg.cpu().numpy().view(np.uint32).astype(np.int64), want)


def test_round_robin_batch_and_ranges(cg):
    """Round-robin units over a batch of uneven graphs and a source range."""
    rng = np.random.default_rng(31)
    ws = [W.powerlaw_capped(int(n), a, 2.0, np.random.default_rng(int(n)))
          for n, a in zip(rng.integers(1, 20000, 5), rng.uniform(2.0, 3.0, 5))]
    tasks, wants = [], []
    for i, w in enumerate(ws):
        S = O.exact_sum(w)
        u0, u1 = (w.size // 3, w.size) if i == 0 else (0, w.size)
        wants.append(_oracle_degrees(w, S, 200 + i, u0, u1)[0])
        tasks.append(cg.Task(_dev(w), S, 200 + i, u0, u1))
    plan = cg.cl_plan(tasks, tuning={"partition": 2})
    for d, want in zip(cg.cl_degrees(plan), wants):
        assert np.array_equal(d.cpu().numpy().view(np.uint32).astype(np.int64), want)


@pytest.mark.parametrize("planner", ["cl_count", "cl_sample"])
def test_round_robin_refused_where_edges_are_written(cg, planner):
    w = W.config_small()
    S = O.exact_sum(w)
    with pytest.raises(cg.ClError):
        getattr(cg, planner)([cg.Task(_dev(w), S, 1)], tuning={"partition": 2})
    with pytest.raises(cg.ClError):
        cg.cl_plan([cg.Task(_dev(w), S, 1)], tuning={"partition": 3})


@pytest.mark.parametrize("n", [1, 7, 1000, 4095, 4096, 4097, 70000])
def test_degrees_single_graph_sizes(cg, n):
    """One graph of sizes from a single node to several units' worth of
    sources, bit-exact."""
    w = W.powerlaw_capped(n, 2.2, 3.0, np.random.default_rng(n)) if n > 1 else np.array([5.0])
    S = O.exact_sum(w)
    want, _ = _oracle_degrees(w, S, 40 + n)
    plan = cg.cl_plan([cg.Task(_dev(w), S, 40 + n)])
    (deg,) = cg.cl_degrees(plan)
    assert np.array_equal(deg.cpu().numpy().view(np.uint32).astype(np.int64), want)


@pytest.mark.parametrize("nparts", [1, 3, 8])
def test_whole_graph_edges_part_by_part(cg, nparts):
    """parts.edges: every part generated into one reused buffer; the parts
    concatenate to the oracle's edge list, and the position-keyed digest of
    the whole list matches."""
    from paper_1406_1215_amd import parts
    w = W.config_plain(n=150_000)
    S = O.exact_sum(w)
    want, m, _, _ = O.generate(w, S, 12)
    got = []
    res = parts.edges(_dev(w), S, 12, nparts,
                      consume=lambda e, first: got.append((first, e.cpu().numpy().view(np.uint32).copy())))
    assert res["edges"] == m
    assert [f for f, _ in got] == list(np.cumsum([0] + [x.shape[0] for _, x in got])[:-1])
    assert np.array_equal(np.concatenate([x for _, x in got]), want)
    res2 = parts.edges(_dev(w), S, 12, nparts)
    assert res2["digest"] == O.hash_edges(want)


@pytest.mark.parametrize("policy", [0, 1, 2])
def test_unit_statistics_pass(cg, policy):
    """cl_unit_stats over plans of all three unit policies (equal cost, equal
    source counts, round robin): every unit has a record, the records add up
    to the plan's candidates and edges (the oracle's) and to its total plan
    cost, clocks are ordered; the plan's output is unchanged afterwards."""
    w = W.config_plain(n=200_000)
    S = O.exact_sum(w)
    want, m, _, cand = O.generate(w, S, 21)
    wd = _dev(w)
    planner = cg.cl_plan if policy == 2 else cg.cl_sample
    plan = planner([cg.Task(wd, S, 21)], tuning={"partition": policy})
    st = cg.cl_unit_stats(plan)
    info = cg.cl_plan_info(plan)
    assert st["t0"].size == info["lanes"]
    assert int(st["visits"].sum()) == cand
    assert int(st["edges"].sum()) == m
    assert bool((st["t1"] >= st["t0"]).all()) and bool((st["t0"] > 0).all())
    # the segments' shares c_u / K_u add up to the lane plan's total cost,
    # sum_u floor(16 e_u) + 16 K_u (rounded once per unit)
    qs, Q = O.qscan(w)
    Z = 0
    for u in range(w.size):
        e = O.ehat(w, S, u, Q=Q, qscale=qs)
        K = O.segments(w, S, u, Q=Q, qscale=qs)[0] if e > O.E_SEG else 1
        Z += math.floor(16.0 * e) + 16 * K
    assert abs(int(st["cost"].sum()) - Z) <= st["cost"].size
    if policy != 2:
        got = cg.cl_generate(plan).cpu().numpy().view(np.uint32).reshape(-1, 2)[: plan.total]
        assert np.array_equal(got, want)


def test_unit_statistics_errors(cg):
    """cl_unit_stats: too short a record buffer is refused with the unit count
    reported and nothing written; a workspace without a plan is refused."""
    import ctypes
    import torch
    w = W.config_small(n=3000)
    S = O.exact_sum(w)
    plan = cg.cl_sample([cg.Task(_dev(w), S, 2)])
    L = cg.lib()
    units = ctypes.c_uint64(0)
    buf = torch.full((8,), -1, dtype=torch.int64, device="cuda:0")
    code = L.cl_unit_stats(ctypes.c_void_p(plan.ws.data_ptr()), None, ctypes.c_void_p(buf.data_ptr()), 8,
                           ctypes.byref(units), None)
    assert code == -7 and units.value == cg.cl_plan_info(plan)["lanes"] and units.value * 4 > 8
    torch.cuda.synchronize()
    assert bool((buf == -1).all())
    empty = torch.zeros(1 << 16, dtype=torch.uint8, device="cuda:0")
    assert L.cl_unit_stats(ctypes.c_void_p(empty.data_ptr()), None, ctypes.c_void_p(buf.data_ptr()), 8, None,
                           None) == -9
