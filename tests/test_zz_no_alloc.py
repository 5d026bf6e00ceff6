"""cl_sample_into_noalloc, the entry point for callers that cannot allocate
device memory (its workspace is the library's fixed per-GPU array), against
cl_sample_into through the C ABI, bit for bit: calls in a row on one GPU
(the second on a smaller input, so stale contents of the array from the
first must not leak into it), a batch with graph offsets, an input whose plan
exceeds the array (refused before any edge is written), then a small input
again."""
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


def _reference(cg, tasks, cap):
    """The existing entry point's output (own workspace)."""
    import torch
    edges = torch.full((cap, 2), -1, dtype=torch.int32, device="cuda:0")
    go = torch.full((len(tasks) + 1,), -1, dtype=torch.int64, device="cuda:0")
    plan, fits = cg.cl_sample_into(tasks, edges, graph_offsets=go)
    assert fits
    return plan.m, edges, go


def _noalloc(cg, tasks, cap):
    import torch
    edges = torch.full((cap, 2), -1, dtype=torch.int32, device="cuda:0")
    go = torch.full((len(tasks) + 1,), -1, dtype=torch.int64, device="cuda:0")
    m, fits, need = cg.cl_sample_into_noalloc(tasks, edges, graph_offsets=go)
    return m, fits, need, edges, go


def test_noalloc_matches_sample_into(cg):
    import torch
    cases = [
        [W.config_plain(n=100_000)],                                     # ~3e6 edges, heavy head
        [W.config_small()],                                              # smaller: 2.6e4 edges
        [W.config_small(seed=7, n=3000), np.zeros(4), W.config_plain(n=20_000)],   # a batch
    ]
    seeds = iter(range(40, 100))
    for ci, ws_ in enumerate(cases):
        tasks = []
        for w in ws_:
            S = O.exact_sum(w) if O.exact_sum(w) > 0 else 1.0
            tasks.append(cg.Task(_to_dev(w), S, next(seeds)))
        cap = sum(O.generate(w, t.S, t.seed, want_edges=False)[1] for w, t in zip(ws_, tasks)) + 100
        m_ref, e_ref, go_ref = _reference(cg, tasks, cap)
        m, fits, need, e, go = _noalloc(cg, tasks, cap)
        assert fits and m == m_ref, ci
        assert 0 < need <= cg.NOALLOC_SCRATCH_BYTES, ci
        assert torch.equal(e, e_ref), ci            # the whole buffer: nothing written past m
        assert torch.equal(go, go_ref), ci
        print(f"case {ci}: {sum(m)} edges, workspace {need} bytes", flush=True)
    # the small graph once more against the oracle itself
    w = W.config_small()
    S = O.exact_sum(w)
    want = O.generate(w, S, 3)[0]
    m, fits, _, e, _ = _noalloc(cg, [cg.Task(_to_dev(w), S, 3)], want.shape[0])
    assert fits and m == [want.shape[0]]
    assert np.array_equal(e.cpu().numpy().view(np.uint32), want)


def test_noalloc_refuses_a_plan_larger_than_the_array(cg):
    import torch
    w = W.config_plain(n=1_000_000)              # ~3.2e7 edges: about 250 MB of workspace
    S = O.exact_sum(w)
    edges = torch.full((1024, 2), -1, dtype=torch.int32, device="cuda:0")
    with pytest.raises(cg.ClError) as ei:
        cg.cl_sample_into_noalloc([cg.Task(_to_dev(w), S, 2)], edges)
    assert ei.value.code == -6
    assert bool((edges == -1).all())
    # too small an output buffer: the first cap edges, CL_ERR_CAPACITY reported as fits = False
    w = W.config_small()
    S = O.exact_sum(w)
    want = O.generate(w, S, 5)[0]
    m, fits, _, e, _ = _noalloc(cg, [cg.Task(_to_dev(w), S, 5)], 1000)
    assert not fits and m == [want.shape[0]]
    assert np.array_equal(e.cpu().numpy().view(np.uint32), want[:1000])
    # and a full call afterwards is exact again
    m, fits, _, e, _ = _noalloc(cg, [cg.Task(_to_dev(w), S, 5)], want.shape[0])
    assert fits and np.array_equal(e.cpu().numpy().view(np.uint32), want)
