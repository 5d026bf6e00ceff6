"""The C-ABI library loads and exports every function include/clgen.h
declares; host-side argument checks answer without a GPU."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "clgen.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(cl_[a-z_0-9]+)\s*\(", src)))


def test_header_declares_the_boundary():
    names = _declared()
    for want in ["cl_weight_sum", "cl_expected_edges", "cl_partition", "cl_count", "cl_generate",
                 "cl_expected_degree", "cl_expected_degree_backward", "cl_batch_capture", "cl_batch_launch",
                 "cl_hash_edges", "cl_degrees"]:
        assert want in names


def test_library_exports_every_declared_symbol():
    import torch  # noqa: F401  (loads the HIP runtime the library binds to)
    from paper_1406_1215_amd import clgen
    if not os.path.exists(clgen.LIB_PATH):
        pytest.skip("library not built")
    L = ctypes.CDLL(clgen.LIB_PATH)
    missing = [n for n in _declared() if not hasattr(L, n)]
    assert not missing, missing
    assert clgen.lib().cl_version().startswith(b"clgen")


def test_host_side_argument_checks():
    import torch  # noqa: F401
    from paper_1406_1215_amd import clgen
    if not os.path.exists(clgen.LIB_PATH):
        pytest.skip("library not built")
    L = clgen.lib()
    need = ctypes.c_uint64(0)
    assert L.cl_weight_sum_workspace(10, ctypes.byref(need)) == 0 and need.value > 0
    # invalid ranges / sizes are refused before any device work
    g = (clgen.cl_graph * 1)(clgen.cl_graph(0, 10, 1.0, 1, 5, 3))
    fixed = ctypes.c_uint64(0)
    est = ctypes.c_uint64(0)
    assert L.cl_workspace_size(g, 1, None, 0, ctypes.byref(fixed), ctypes.byref(est)) == -1
    g = (clgen.cl_graph * 1)(clgen.cl_graph(0, 1 << 32, 1.0, 1, 0, 0))
    assert L.cl_workspace_size(g, 1, None, 0, ctypes.byref(fixed), ctypes.byref(est)) == -5
    g = (clgen.cl_graph * 1)(clgen.cl_graph(0, 0, -1.0, 1, 0, 0))
    assert L.cl_workspace_size(g, 1, None, 0, ctypes.byref(fixed), ctypes.byref(est)) == -1
    g = (clgen.cl_graph * 1)(clgen.cl_graph(0, 0, 1.0, 1, 0, 0))
    assert L.cl_workspace_size(g, 1, None, 0, ctypes.byref(fixed), ctypes.byref(est)) == 0
    assert est.value >= fixed.value > 0
    m = (ctypes.c_uint64 * 1)()
    req = ctypes.c_uint64(0)
    # too small a workspace is reported with the required size
    assert L.cl_count(g, 1, None, None, 0, m, ctypes.byref(req), None) == -6
    assert req.value == fixed.value
    bounds = (ctypes.c_uint64 * 3)()
    assert L.cl_partition(None, 0, 1.0, 0, None, 0, bounds, None, None) == -1
    # round-robin units are for plans without edge output; unknown policies refused
    rr = ctypes.pointer(clgen.cl_tuning(0, 0, 0, 2))
    assert L.cl_count(g, 1, rr, None, 0, m, ctypes.byref(req), None) == -1
    assert L.cl_sample(g, 1, rr, None, 0, m, ctypes.byref(req), None) == -1
    bad = ctypes.pointer(clgen.cl_tuning(0, 0, 0, 3))
    assert L.cl_plan(g, 1, bad, None, 0, ctypes.byref(req), None) == -1
    assert L.cl_plan(g, 1, rr, None, 0, ctypes.byref(req), None) == -6   # accepted; workspace too small
    # a processing order by position (the default for one graph): single-graph
    # plans only; index order anywhere; unknown orders refused
    by_pos = ctypes.pointer(clgen.cl_tuning(0, 0, 0, 0, 0, 0, 0, 2))
    by_idx = ctypes.pointer(clgen.cl_tuning(0, 0, 0, 0, 0, 0, 0, 1))
    assert L.cl_sample(g, 1, by_pos, None, 0, m, ctypes.byref(req), None) == -6   # accepted
    g2 = (clgen.cl_graph * 2)(clgen.cl_graph(0, 0, 1.0, 1, 0, 0), clgen.cl_graph(0, 0, 1.0, 2, 0, 0))
    m2 = (ctypes.c_uint64 * 2)()
    assert L.cl_sample(g2, 2, by_pos, None, 0, m2, ctypes.byref(req), None) == -1
    assert L.cl_count(g2, 2, by_pos, None, 0, m2, ctypes.byref(req), None) == -1
    assert L.cl_sample(g2, 2, by_idx, None, 0, m2, ctypes.byref(req), None) == -6
    assert L.cl_sample(g2, 2, None, None, 0, m2, ctypes.byref(req), None) == -6
    odd = ctypes.pointer(clgen.cl_tuning(0, 0, 0, 0, 0, 0, 0, 3))
    assert L.cl_sample(g, 1, odd, None, 0, m, ctypes.byref(req), None) == -1
    assert L.cl_workspace_size(g, 1, odd, 1, ctypes.byref(fixed), ctypes.byref(est)) == -1
    # the ordered plan's workspace estimate covers the order's arrays
    est1 = ctypes.c_uint64(0)
    assert L.cl_workspace_size(g, 1, by_pos, 1, ctypes.byref(fixed), ctypes.byref(est1)) == 0
    assert L.cl_workspace_size(g, 1, None, 1, ctypes.byref(fixed), ctypes.byref(est)) == 0
    assert est1.value == est.value
    assert L.cl_workspace_size(g, 1, by_idx, 1, ctypes.byref(fixed), ctypes.byref(est)) == 0
    assert est1.value > est.value
