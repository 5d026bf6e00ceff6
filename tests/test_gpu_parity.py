"""GPU parity: the HIP path through the C ABI against the oracle, element by
element on seeded inputs; invariants and digests at full size."""
import math

import numpy as np
import pytest

import oracle as O
from paper_1406_1215_amd import workloads as W

pytestmark = pytest.mark.gpu


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


PLANNERS = ["cl_count", "cl_sample"]


def _gpu_edges(cg, w, S, seed, u0=0, u1=None, tuning=None, planner="cl_count"):
    wd = _to_dev(w)
    plan = getattr(cg, planner)([cg.Task(wd, S, seed, u0, u1)], tuning=tuning)
    e = cg.cl_generate(plan)
    return _edges_np(e)[: plan.total], plan


def test_weight_sum_is_exact(cg):
    rng = np.random.default_rng(30)
    cases = [W.config_small(), np.array([1.0]), np.array([1e16, 1.0, 1.0]), np.array([3e-310, 2e-310, 1e-320]),
             np.sort(rng.pareto(0.7, 100000) * 1e3)[::-1], np.zeros(5), np.array([1e308, 1e308]),
             # round half to even, with and without a sticky bit far below
             np.array([2.0 ** 53, 1.0]), np.array([2.0 ** 53 + 2, 1.0]), np.array([2.0 ** 53, 1.0, 2.0 ** -1000]),
             np.array([2.0 ** 1000, 2.0 ** 947, 5e-324]), np.array([2.0 ** 1000, 2.0 ** 947])]
    import torch
    shared = torch.empty(cg.cl_weight_sum_workspace(1 << 20), dtype=torch.uint8, device="cuda:0")
    for ws in (None, shared):   # a fresh workspace per call, then one reused by every case
        for w in cases:
            wd = _to_dev(w)
            if not np.all(np.isfinite(np.sum(w))):
                with pytest.raises(cg.ClError):
                    cg.cl_weight_sum(wd, ws=ws)
                continue
            assert cg.cl_weight_sum(wd, ws=ws) == O.exact_sum(w)


@pytest.mark.parametrize("planner", PLANNERS)
def test_small_config_bit_exact(planner, cg):
    w = W.config_small()
    S = O.exact_sum(w)
    want, m, h, _ = O.generate(w, S, 1)
    got, plan = _gpu_edges(cg, w, S, 1, planner=planner)
    assert plan.m == [m]
    assert np.array_equal(got, want)


@pytest.mark.parametrize("seed", [1, 2, 12345678901234567])
@pytest.mark.parametrize("planner", PLANNERS)
def test_edge_cases_bit_exact(planner, cg, seed):
    for i, w in enumerate(W.tiny_cases(seed=40 + seed % 7, count=24)):
        if w.size == 0 or O.exact_sum(w) == 0.0:
            continue
        S = O.exact_sum(w)
        want, m, _, _ = O.generate(w, S, seed + i)
        got, plan = _gpu_edges(cg, w, S, seed + i, planner=planner)
        assert plan.m == [m], (i, w.size)
        assert np.array_equal(got, want), (i, w.size)


def test_zero_weights_and_empty_range(cg):
    import torch
    w = np.zeros(10)
    wd = _to_dev(w)
    plan = cg.cl_count([cg.Task(wd, 1.0, 3)])
    assert plan.m == [0]
    w = W.config_small(n=500)
    S = O.exact_sum(w)
    plan = cg.cl_count([cg.Task(_to_dev(w), S, 3, 200, 200)])
    assert plan.m == [0]
    _ = torch.cuda.synchronize()


def _heavy(n, seed, scale):
    rng = np.random.default_rng(seed)
    return np.sort(rng.pareto(1.05, n) + 1.0)[::-1] * scale


@pytest.mark.parametrize("n,scale,seed", [(20000, 30.0, 1), (60000, 80.0, 2), (5000, 400.0, 3)])
@pytest.mark.parametrize("planner", PLANNERS)
def test_segmented_sources_bit_exact(planner, cg, n, scale, seed):
    w = _heavy(n, 50 + seed, scale)
    S = O.exact_sum(w)
    K0, _ = O.segments(w, S, 0)
    assert K0 > 1                      # the head is split into segments
    want, m, h, _ = O.generate(w, S, seed)
    got, plan = _gpu_edges(cg, w, S, seed, planner=planner)
    info = cg.cl_plan_info(plan)
    assert info["heavy_segments"] > 0
    assert plan.m == [m]
    assert np.array_equal(got, want)


@pytest.mark.parametrize("u0,u1", [(0, 1), (0, 777), (500, 4000), (9999, 10000), (3000, 3000)])
@pytest.mark.parametrize("planner", PLANNERS)
def test_source_ranges_bit_exact(planner, cg, u0, u1):
    w = W.config_small()
    S = O.exact_sum(w)
    want, m, _, _ = O.generate(w, S, 9, u0, u1)
    got, plan = _gpu_edges(cg, w, S, 9, u0, u1, planner=planner)
    assert plan.m == [m]
    assert np.array_equal(got, want)


@pytest.mark.parametrize("tuning", [{"lane_budget": 1}, {"lane_budget": 17}, {"lane_budget": 4096},
                                    {"lane_budget": 192, "blocks_per_cu": 1}, {"blocks_per_cu": 32},
                                    {"partition": 1}, {"partition": 1, "lane_budget": 1},
                                    {"partition": 1, "lane_budget": 1 << 20}, {"tail_units": 1},
                                    {"lane_budget": 17, "tail_units": 1}])
@pytest.mark.parametrize("planner", PLANNERS)
def test_schedule_does_not_change_output(planner, cg, tuning):
    w = _heavy(30000, 60, 40.0)
    S = O.exact_sum(w)
    want, m, _, _ = O.generate(w, S, 4)
    got, plan = _gpu_edges(cg, w, S, 4, tuning=tuning, planner=planner)
    assert np.array_equal(got, want)


@pytest.mark.parametrize("planner", PLANNERS)
def test_batched_tasks_equal_single_tasks(planner, cg):
    import torch
    rng = np.random.default_rng(70)
    ws = [W.config_small(seed=int(rng.integers(1 << 30)), n=int(rng.integers(2, 3000))) for _ in range(7)]
    ws += [np.zeros(4), _heavy(8000, 71, 50.0), np.full(64, 64.0)]
    tasks, wants = [], []
    for i, w in enumerate(ws):
        S = O.exact_sum(w) if O.exact_sum(w) > 0 else 1.0
        e, m, _, _ = O.generate(w, S, 100 + i)
        wants.append(e)
        tasks.append(cg.Task(_to_dev(w), S, 100 + i))
    plan = getattr(cg, planner)(tasks)
    assert plan.m == [x.shape[0] for x in wants]
    go = torch.zeros(len(tasks) + 1, dtype=torch.int64, device="cuda:0")
    e = _edges_np(cg.cl_generate(plan, graph_offsets=go))
    off = go.cpu().numpy()
    assert off[-1] == plan.total
    for i, want in enumerate(wants):
        assert np.array_equal(e[off[i]:off[i + 1]], want), i


@pytest.mark.parametrize("planner", PLANNERS)
def test_batched_heavy_graphs_bit_exact(planner, cg):
    """Several graphs with split sources in one plan: their heavy segments sit
    side by side in one table (wavefronts straddle graphs), and each graph's
    unit starts are placed on its own segments."""
    import torch
    shapes = [(3000, 60.0), (9000, 25.0), (700, 300.0), (15000, 40.0), (64, 64.0), (5000, 120.0)]
    tasks, wants = [], []
    for i, (n, scale) in enumerate(shapes):
        w = _heavy(n, 90 + i, scale)
        S = O.exact_sum(w)
        e, m, _, _ = O.generate(w, S, 300 + i)
        wants.append(e)
        tasks.append(cg.Task(_to_dev(w), S, 300 + i))
    plan = getattr(cg, planner)(tasks)
    assert cg.cl_plan_info(plan)["heavy_segments"] > 64
    assert plan.m == [x.shape[0] for x in wants]
    go = torch.zeros(len(tasks) + 1, dtype=torch.int64, device="cuda:0")
    e = _edges_np(cg.cl_generate(plan, graph_offsets=go))
    off = go.cpu().numpy()
    for i, want in enumerate(wants):
        assert np.array_equal(e[off[i]:off[i + 1]], want), i


@pytest.mark.parametrize("planner", PLANNERS)
def test_write_windows(planner, cg):
    import torch
    w = _heavy(40000, 80, 30.0)
    S = O.exact_sum(w)
    want, m, _, _ = O.generate(w, S, 6)
    plan = getattr(cg, planner)([cg.Task(_to_dev(w), S, 6)])
    cuts = [0, 1, m // 3, m // 3 + 1, (2 * m) // 3, m]
    parts = []
    for a, b in zip(cuts[:-1], cuts[1:]):
        parts.append(_edges_np(cg.cl_generate(plan, edge_begin=a, cap=b - a))[: b - a])
    assert np.array_equal(np.concatenate(parts), want)
    acc = torch.zeros(1, dtype=torch.int64, device="cuda:0")
    e = cg.cl_generate(plan)
    cg.cl_hash_edges(e, 0, acc)
    assert cg.hash_value(acc) == O.hash_edges(want)


def test_validation_errors_match_oracle(cg):
    bad = {
        "unsorted": (np.array([1.0, 2.0, 0.5]), None),
        "unsorted tie then rise": (np.array([3.0, 2.0, 2.0, 2.5]), None),
        "negative": (np.array([2.0, 1.0, -0.5]), None),
        "negative subnormal": (np.array([1.0, -5e-324]), None),
        "nonfinite": (np.array([np.inf, 1.0]), 5.0),
        "nan": (np.array([3.0, np.nan]), 5.0),
        "S below w0": (np.array([5.0, 1.0]), 4.0),
        "tiny head": (np.array([2.0 ** -961, 2.0 ** -962]), 1.0),
        "nan and negative": (np.array([1.0, np.nan, -1.0, 5.0]), None),
        "unsorted and negative": (np.array([1.0, 2.0, -1.0]), None),
        "unsorted and S below w0": (np.array([4.0, 5.0]), 1.0),
    }
    for name, (w, S) in bad.items():
        S = S if S is not None else 10.0
        oc = O.validate(w, S)
        assert oc != 0, name
        for planner in (cg.cl_count, cg.cl_sample):
            with pytest.raises(cg.ClError) as ei:
                planner([cg.Task(_to_dev(w), S, 1)])
            assert ei.value.code == oc, name
    # accepted by both: -0.0, S == w_0, the smallest allowed head
    for w, S in ((np.array([1.0, -0.0]), 1.0), (np.array([5.0]), 5.0),
                 (np.array([2.0 ** -960, 2.0 ** -961]), 1.0)):
        assert O.validate(w, S) == 0
        plan = cg.cl_count([cg.Task(_to_dev(w), S, 1)])
        assert plan.m == [O.generate(w, S, 1)[1]]


def test_capture_refuses_a_plan_without_counts(cg):
    """cl_batch_capture needs a counted plan (cl_count, cl_sample): a
    workspace planned by cl_plan, or never planned, is refused."""
    import torch
    w = W.config_small(n=2000)
    S = O.exact_sum(w)
    tasks = [cg.Task(_to_dev(w), S, 1)]
    s = torch.cuda.Stream()
    plan = cg.cl_plan(tasks)
    with pytest.raises(cg.ClError) as ei:
        cg.cl_batch_capture(plan, s)
    assert ei.value.code == -9
    plan.ws.zero_()
    with pytest.raises(cg.ClError) as ei:
        cg.cl_batch_capture(plan, s)
    assert ei.value.code == -9


def test_partition_matches_oracle(cg):
    w = W.config_small()
    S = O.exact_sum(w)
    for P in (1, 3, 64, 1000, 20000):
        b, Z = cg.cl_partition(_to_dev(w), S, P)
        bo, Zo = O.partition(w, S, P)
        assert Z == Zo
        assert b == [int(x) for x in bo]
    w = np.array([1000.0, 900.0] + [1.0] * 60)
    S = O.exact_sum(w)
    b, Z = cg.cl_partition(_to_dev(w), S, 16)
    bo, Zo = O.partition(w, S, 16)
    assert b == [int(x) for x in bo]


def test_expected_edges_matches_oracle(cg):
    for w in (W.config_small(), _heavy(20000, 90, 60.0)):
        S = O.exact_sum(w)
        E, V = cg.cl_expected_edges(_to_dev(w), S)
        Eo, Vo = O.expected_edges_closed(w, S)
        assert abs(E - Eo) <= 1e-10 * Eo
        assert abs(V - Vo) <= 1e-9 * Vo


@pytest.mark.parametrize("planner", PLANNERS)
def test_graph_capture_replays(planner, cg):
    import torch
    rng = np.random.default_rng(95)
    ws = [W.config_small(seed=int(rng.integers(1 << 30)), n=int(rng.integers(100, 5000))) for _ in range(5)]
    tasks, wants = [], []
    for i, w in enumerate(ws):
        S = O.exact_sum(w)
        wants.append(O.generate(w, S, 7 + i)[0])
        tasks.append(cg.Task(_to_dev(w), S, 7 + i))
    plan = getattr(cg, planner)(tasks)
    s = torch.cuda.Stream()
    bg = cg.cl_batch_capture(plan, s)
    want_all = np.concatenate(wants)
    for rep in range(3):
        bg.edges.fill_(-1)
        torch.cuda.synchronize()
        bg.launch(s)
        s.synchronize()
        e = _edges_np(bg.edges)[: plan.total]
        assert np.array_equal(e, want_all), rep
        off = bg.graph_offsets.cpu().numpy()
        assert list(np.diff(off)) == [x.shape[0] for x in wants]
        x = torch.ones(1000, device="cuda:0").sum()   # eager work between replays
        assert float(x) == 1000.0
    bg.close()


_FULL = {}


def _full_plain():
    if not _FULL:
        w = W.config_plain()
        S = O.exact_sum(w)
        _, m, h, _ = O.generate(w, S, 2, want_edges=False)
        _FULL.update(w=w, S=S, m=m, h=h)
    return _FULL


@pytest.mark.parametrize("planner", PLANNERS)
def test_plain_config_full_size_digest(planner, cg):
    """n = 1e7 power law: count and digest equal the oracle's; invariants."""
    import torch
    F = _full_plain()
    w, S = F["w"], F["S"]
    wd = _to_dev(w)
    assert cg.cl_weight_sum(wd) == S
    plan = getattr(cg, planner)([cg.Task(wd, S, 2)])
    e = cg.cl_generate(plan)
    acc = cg.cl_hash_edges(e)
    m, h = F["m"], F["h"]
    assert plan.m == [m]
    assert cg.hash_value(acc) == h
    # sampled windows compared edge by edge with single-source oracle runs
    en = _edges_np(e)
    rng = np.random.default_rng(3)
    qs, Q = O.qscan(w)
    us = en[:, 0]
    for u in list(rng.integers(0, 2000, 10)) + list(rng.integers(0, w.size, 20)):
        want_v = O.node_edges(w, S, 2, int(u), Q=Q, qscale=qs)
        lo = np.searchsorted(us, u, side="left")
        hi = np.searchsorted(us, u, side="right")
        assert np.array_equal(en[lo:hi, 1], want_v), int(u)


@pytest.mark.parametrize("n", [100_000, 1_000_000])
@pytest.mark.parametrize("planner", PLANNERS)
def test_plain_shapes_bit_exact(planner, cg, n):
    """Smaller instances of the n = 1e7 shape (many capped sources at the head);
    n = 1e5 is the input on which an earlier persistent-loop miscompilation
    (single-lane tail merged into the loop head) never terminated."""
    w = W.config_plain(n=n)
    S = O.exact_sum(w)
    want, m, _, _ = O.generate(w, S, 2)
    got, plan = _gpu_edges(cg, w, S, 2, planner=planner)
    assert plan.m == [m]
    assert np.array_equal(got, want)
    info = cg.cl_plan_info(plan)
    _, _, _, cand = O.generate(w, S, 2, want_edges=False)
    assert info["candidates"] == cand


@pytest.mark.parametrize("tuning", [{"slot_margin": 1}, {"slot_margin": 1, "lane_budget": 7}])
def test_one_pass_slot_overflow_replay(cg, tuning):
    """Slots without a margin: about half the lanes overflow and are replayed
    by the write kernel; the output is unchanged."""
    w = _heavy(30000, 61, 40.0)
    S = O.exact_sum(w)
    want, m, _, _ = O.generate(w, S, 5)
    got, plan = _gpu_edges(cg, w, S, 5, tuning=tuning, planner="cl_sample")
    assert plan.m == [m]
    assert np.array_equal(got, want)


@pytest.mark.parametrize("tuning", [None, {"slot_margin": 1}])
def test_sample_into_one_call(cg, tuning):
    """cl_sample_into: plan, one pass and expansion into the caller's buffer in
    one call.  Bit-exact with the oracle for a batch (graph offsets included,
    and with the overflow replay when slots have no margin); a buffer that is
    too small holds the first cap edges and the plan completes the output
    through cl_generate; a second call reuses workspace and buffer."""
    import torch
    ws_ = [_heavy(20000, 90, 30.0), W.config_small(), np.zeros(3), _heavy(5000, 91, 60.0)]
    tasks, wants = [], []
    for i, w in enumerate(ws_):
        S = O.exact_sum(w) if O.exact_sum(w) > 0 else 1.0
        wants.append(O.generate(w, S, 300 + i)[0])
        tasks.append(cg.Task(_to_dev(w), S, 300 + i))
    want = np.concatenate(wants)
    m = want.shape[0]
    edges = torch.full((m + 100, 2), -1, dtype=torch.int32, device="cuda:0")
    go = torch.zeros(len(tasks) + 1, dtype=torch.int64, device="cuda:0")
    plan, fits = cg.cl_sample_into(tasks, edges, cap=m + 100, graph_offsets=go, tuning=tuning)
    assert fits and plan.total == m
    assert np.array_equal(_edges_np(edges)[:m], want)
    off = go.cpu().numpy()
    assert list(np.diff(off)) == [x.shape[0] for x in wants]
    # too small: the first cap edges, then the rest from the same plan
    small = torch.zeros((m // 3, 2), dtype=torch.int32, device="cuda:0")
    plan2, fits2 = cg.cl_sample_into(tasks, small, tuning=tuning, ws=plan.ws)
    assert not fits2 and plan2.total == m
    assert np.array_equal(_edges_np(small), want[: m // 3])
    assert np.array_equal(_edges_np(cg.cl_generate(plan2))[:m], want)
    # the same buffer and workspace again
    edges.fill_(-1)
    plan3, fits3 = cg.cl_sample_into(tasks, edges, tuning=tuning, ws=plan.ws)
    assert fits3 and np.array_equal(_edges_np(edges)[:m], want)


@pytest.mark.parametrize("planner", PLANNERS)
def test_graded_units_change_only_the_schedule(planner, cg):
    """Graded units (the last eighth of the cost in units a quarter of the
    lane budget) against uniform units on a graph of several thousand units:
    more units, the same edges as the oracle."""
    w = W.config_plain(n=300_000)
    S = O.exact_sum(w)
    want, m, _, _ = O.generate(w, S, 13)
    lanes = {}
    for tail in (0, 1):
        got, plan = _gpu_edges(cg, w, S, 13, tuning={"tail_units": tail}, planner=planner)
        assert np.array_equal(got, want), tail
        lanes[tail] = cg.cl_plan_info(plan)["lanes"]
    assert lanes[1] >= 4096 and lanes[0] > lanes[1]


def _csr_of(edges, n, base=0):
    """Row offsets and columns of a (u, v)-sorted edge list."""
    u = edges[:, 0].astype(np.int64)
    rows = np.concatenate([[0], np.cumsum(np.bincount(u, minlength=n))]) + base
    return rows, edges[:, 1]


@pytest.mark.parametrize("planner,tuning", [("cl_sample", None), ("cl_count", None),
                                            ("cl_sample", {"slot_margin": 1}), ("cl_sample", {"tail_units": 1})])
def test_csr_output(cg, planner, tuning):
    """cl_generate_csr: targets at the edges' positions and row offsets per
    source, against the oracle's edge list, for a batch of uneven graphs (a
    source range included), from one-pass plans (with and without slot
    overflow) and two-pass plans."""
    ws_ = [W.config_plain(n=200_000), _heavy(20000, 95, 30.0), np.zeros(5), W.config_small()]
    tasks, wants, ranges = [], [], [(0, None), (0, None), (0, None), (1000, 7000)]
    for i, w in enumerate(ws_):
        S = O.exact_sum(w) if O.exact_sum(w) > 0 else 1.0
        u0, u1 = ranges[i]
        wants.append(O.generate(w, S, 500 + i, u0, u1)[0])
        tasks.append(cg.Task(_to_dev(w), S, 500 + i, u0, u1))
    plan = getattr(cg, planner)(tasks, tuning=tuning)
    assert plan.m == [x.shape[0] for x in wants]
    col, rows = cg.cl_generate_csr(plan)
    col = col.cpu().numpy().view(np.uint32)
    off = 0
    for i, (w, want) in enumerate(zip(ws_, wants)):
        r_want, c_want = _csr_of(want, w.size, off)
        assert np.array_equal(rows[i].cpu().numpy(), r_want), i
        assert np.array_equal(col[off: off + want.shape[0]], c_want), i
        off += want.shape[0]
    # too small a column array
    with pytest.raises(cg.ClError):
        cg.cl_generate_csr(plan, col=torch_empty_i32(plan.total - 1))


def torch_empty_i32(n):
    import torch
    return torch.empty(max(n, 1), dtype=torch.int32, device="cuda:0")


def _capped_inputs():
    rng = np.random.default_rng(77)
    out = {}
    # a capped clique at the head: 400 nodes with w^2 > S, then a power-law tail
    head = np.full(400, 3000.0)
    tail = np.minimum(np.sort(rng.pareto(1.5, 50000) + 1.0)[::-1] * 3.0, 2000.0)
    out["clique head"] = np.concatenate([head, tail])
    # the complete graph on 2048 nodes (w = n, every pair exactly capped), many segments per source
    out["complete 2048"] = np.full(2048, 2048.0)
    # the shape of the 1e9-node graph's head at a small size: mean 500, cap sqrt(500 n)
    out["share shape"] = W.powerlaw_mean(200_000, 2.1, 500.0, np.random.default_rng(3))
    # capped pairs that end inside segments: a slowly falling head
    out["falling head"] = np.sort(rng.uniform(500.0, 4000.0, 3000))[::-1]
    return out


_CAPPED = {}


def _capped_cases():
    if not _CAPPED:
        for name, w in _capped_inputs().items():
            S = O.exact_sum(w)
            want, m, _, cand = O.generate(w, S, 31)
            _CAPPED[name] = (w, S, want, m, cand)
    return _CAPPED


@pytest.mark.parametrize("planner", PLANNERS)
def test_capped_runs_bit_exact(planner, cg):
    """Inputs dominated by capped pairs (p = 1), where runs of capped
    candidates are taken without drawing random words: edge lists and the
    visited-candidate count equal the oracle's."""
    for name, (w, S, want, m, cand) in _capped_cases().items():
        assert (w[0] / S) * w[min(10, w.size - 1)] >= 1.0, name     # the head is capped
        got, plan = _gpu_edges(cg, w, S, 31, planner=planner)
        assert plan.m == [m], name
        assert np.array_equal(got, want), name
        assert cg.cl_plan_info(plan)["candidates"] == cand, name
