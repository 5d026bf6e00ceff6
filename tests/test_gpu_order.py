"""GPU: the processing order of the work units (cl_tuning.unit_order).

A single-graph plan hands its units out by the position of their first
candidate in the quantised prefix of w (the default for one graph, or 2);
index order is 1.  The order is a schedule: every output bit must equal the
oracle's under each order, with both planners, with uniform and graded units,
for source ranges, for the degree and statistics passes and through a
captured graph; and the candidates visited must be the oracle's (a unit
taken twice or never would change them).  Batches refuse order 2."""
import numpy as np
import pytest

import oracle as O
from paper_1406_1215_amd import workloads as W

pytestmark = pytest.mark.gpu

PLANNERS = ["cl_sample", "cl_count"]


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


def _edges_np(t):
    return t.cpu().numpy().view(np.uint32).reshape(-1, 2)


def _pareto(n, seed, scale, shape=1.05):
    rng = np.random.default_rng(seed)
    return np.sort(rng.pareto(shape, n) + 1.0)[::-1] * scale


def _capped_head(n, heads, seed):
    """`heads` sources of one equal weight at the cap sqrt(S) (their segments
    line up in v, as in the head of the 1e9-node graph), then a power-law tail."""
    tail = _pareto(n - heads, seed, 20.0, 1.3)
    c = float(np.sqrt(tail.sum()) * 2.0)
    return np.concatenate([np.full(heads, c), np.minimum(tail, c)])


CASES = {
    "heavy": lambda: (_pareto(30000, 60, 40.0), 0, None),
    "very_heavy": lambda: (_pareto(5000, 53, 400.0), 0, None),
    "capped_head": lambda: (_capped_head(40000, 300, 7), 0, None),
    "light_only": lambda: (W.config_small(), 0, None),
    "er": lambda: (np.full(3000, 30.0), 0, None),
    "zero_tail": lambda: (np.concatenate([_pareto(2000, 9, 60.0), np.zeros(500)]), 0, None),
    "range": lambda: (_pareto(30000, 61, 40.0), 17, 9000),
    "single": lambda: (np.array([5.0]), 0, None),
    "all_zero": lambda: (np.zeros(10), 0, None),
    "empty_range": lambda: (_pareto(3000, 62, 40.0), 500, 500),
    "last_sources": lambda: (_pareto(20000, 63, 40.0), 19990, 20000),
}
TUNINGS = [None, {"unit_order": 1}, {"unit_order": 2}, {"unit_order": 2, "lane_budget": 17},
           {"unit_order": 2, "tail_units": 1}]


@pytest.mark.parametrize("case", sorted(CASES))
@pytest.mark.parametrize("planner", PLANNERS)
def test_orders_bit_exact(cg, planner, case):
    w, u0, u1 = CASES[case]()
    u1 = w.size if u1 is None else u1
    S = O.exact_sum(w) or 1.0
    want, m, _, cand = O.generate(w, S, 4, u0, u1)
    wd = _dev(w)
    for tun in TUNINGS:
        plan = getattr(cg, planner)([cg.Task(wd, S, 4, u0, u1)], tuning=tun)
        assert plan.m == [m], tun
        got = _edges_np(cg.cl_generate(plan))[: plan.total]
        assert np.array_equal(got, want), tun
        assert cg.cl_plan_info(plan)["candidates"] == cand, tun


@pytest.mark.parametrize("planner", PLANNERS)
def test_graded_units_in_position_order(cg, planner):
    """n = 1e6 power law: more than 4096 units, so the last eighth of the cost
    is cut into graded units (their own run, after the others)."""
    w = W.config_plain(n=1_000_000)
    S = O.exact_sum(w)
    want, m, _, cand = O.generate(w, S, 31)
    wd = _dev(w)
    lanes = {}
    for tun in ({"unit_order": 2}, {"unit_order": 2, "tail_units": 1}):
        plan = getattr(cg, planner)([cg.Task(wd, S, 31)], tuning=tun)
        got = _edges_np(cg.cl_generate(plan))[: plan.total]
        assert np.array_equal(got, want), tun
        info = cg.cl_plan_info(plan)
        assert info["candidates"] == cand
        lanes[tun.get("tail_units", 0)] = info["lanes"]
    assert lanes[1] >= 4096 and lanes[0] > lanes[1]


def test_degrees_and_statistics_in_position_order(cg):
    """cl_degrees and cl_unit_stats on plans in position order: the degrees
    equal those of the oracle's edge list, every unit has one record and the
    records add up to the oracle's candidates and edges."""
    import torch
    w = _capped_head(60000, 400, 11)
    S = O.exact_sum(w)
    want, m, _, cand = O.generate(w, S, 8)
    deg_want = np.bincount(want.reshape(-1), minlength=w.size)
    wd = _dev(w)
    plan = cg.cl_plan([cg.Task(wd, S, 8)], tuning={"unit_order": 2})
    d = cg.cl_degrees(plan)[0].cpu().numpy().view(np.uint32)
    assert np.array_equal(d.astype(np.int64), deg_want)
    plan = cg.cl_sample([cg.Task(wd, S, 8)], tuning={"unit_order": 2})
    st = cg.cl_unit_stats(plan)
    assert st["t0"].size == cg.cl_plan_info(plan)["lanes"]
    assert int(st["visits"].sum()) == cand and int(st["edges"].sum()) == m
    assert bool((st["t0"] > 0).all()) and bool((st["t1"] >= st["t0"]).all())
    got = _edges_np(cg.cl_generate(plan))[: plan.total]
    assert np.array_equal(got, want)
    torch.cuda.synchronize()


def test_position_order_in_a_captured_graph(cg):
    """A single-graph plan (position order by default) captured and replayed
    three times, with eager work between the replays: every replay equals the
    oracle's edge list."""
    import torch
    w = _pareto(50000, 71, 50.0)
    S = O.exact_sum(w)
    want = O.generate(w, S, 12)[0]
    plan = cg.cl_sample([cg.Task(_dev(w), S, 12)])
    s = torch.cuda.Stream()
    bg = cg.cl_batch_capture(plan, s)
    for rep in range(3):
        bg.edges.fill_(-1)
        torch.cuda.synchronize()
        bg.launch(s)
        s.synchronize()
        assert np.array_equal(_edges_np(bg.edges)[: plan.total], want), rep
        x = torch.ones(1000, device="cuda:0").sum()
        assert float(x) == 1000.0
    bg.close()


def test_position_order_refused_for_batches(cg):
    w = _pareto(3000, 5, 30.0)
    S = O.exact_sum(w)
    tasks = [cg.Task(_dev(w), S, 1), cg.Task(_dev(w), S, 2)]
    with pytest.raises(cg.ClError):
        cg.cl_sample(tasks, tuning={"unit_order": 2})
    with pytest.raises(cg.ClError):
        cg.cl_sample(tasks[:1], tuning={"unit_order": 3})
    # the default and index order are accepted for batches
    for tun in (None, {"unit_order": 1}):
        plan = cg.cl_sample(tasks, tuning=tun)
        assert plan.m == [O.generate(w, S, 1)[1], O.generate(w, S, 2)[1]]
