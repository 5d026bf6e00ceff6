"""Thin Python binding of libclgen.so (include/clgen.h): argument marshalling
only; every step of the computation runs in the HIP kernels.

PyTorch provides device memory and streams.  torch is imported before the
library is loaded so that libclgen binds to the HIP runtime torch already
loaded (one runtime per process).  The library must have been built
(``__graft_entry__.build()``); there is no fallback.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass, field
from typing import List, Optional, Sequence

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libclgen.so")

CL_OK = 0
ERRORS = {
    -1: "CL_ERR_INVALID_ARG", -2: "CL_ERR_UNSORTED", -3: "CL_ERR_NEGATIVE", -4: "CL_ERR_NONFINITE",
    -5: "CL_ERR_TOO_LARGE", -6: "CL_ERR_WORKSPACE", -7: "CL_ERR_CAPACITY", -8: "CL_ERR_DEVICE",
    -9: "CL_ERR_NOT_PLANNED",
}


class ClError(RuntimeError):
    def __init__(self, code: int, what: str = ""):
        super().__init__(f"{what}: {ERRORS.get(code, code)} ({code})")
        self.code = code


class cl_graph(ctypes.Structure):
    _fields_ = [("w", ctypes.c_void_p), ("n", ctypes.c_uint64), ("S", ctypes.c_double),
                ("seed", ctypes.c_uint64), ("u_begin", ctypes.c_uint64), ("u_end", ctypes.c_uint64)]


class cl_tuning(ctypes.Structure):
    _fields_ = [("lane_budget", ctypes.c_uint32), ("blocks_per_cu", ctypes.c_uint32),
                ("slot_margin", ctypes.c_uint32), ("partition", ctypes.c_uint32), ("tail_units", ctypes.c_uint32),
                ("ed_rows", ctypes.c_uint32), ("ed_cols", ctypes.c_uint32), ("unit_order", ctypes.c_uint32)]


_lib = None
_P = ctypes.c_void_p
_U64 = ctypes.c_uint64
_U64P = ctypes.POINTER(ctypes.c_uint64)
_DP = ctypes.POINTER(ctypes.c_double)


def lib():
    """Load libclgen.so; raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    path = os.environ.get("CLGEN_LIBRARY", LIB_PATH)   # another build of the same library
    if not os.path.exists(path):
        raise RuntimeError(f"{path} is missing: build it with __graft_entry__.build()")
    L = ctypes.CDLL(path)
    S = ctypes.c_int32
    sig = {
        "cl_weight_sum_workspace": (S, [_U64, _U64P]),
        "cl_weight_sum": (S, [_P, _U64, _P, _U64, _DP, _P]),
        "cl_expected_edges_workspace": (S, [_U64, _U64P]),
        "cl_expected_edges": (S, [_P, _U64, ctypes.c_double, _P, _U64, _DP, _DP, _P]),
        "cl_partition_workspace": (S, [_U64, ctypes.c_uint32, _U64P]),
        "cl_partition": (S, [_P, _U64, ctypes.c_double, ctypes.c_uint32, _P, _U64, _U64P, _U64P, _P]),
        "cl_workspace_size": (S, [ctypes.POINTER(cl_graph), ctypes.c_uint32, ctypes.POINTER(cl_tuning), ctypes.c_uint32,
                                  _U64P, _U64P]),
        "cl_sample": (S, [ctypes.POINTER(cl_graph), ctypes.c_uint32, ctypes.POINTER(cl_tuning), _P, _U64, _U64P,
                          _U64P, _P]),
        "cl_sample_into": (S, [ctypes.POINTER(cl_graph), ctypes.c_uint32, ctypes.POINTER(cl_tuning), _P, _U64, _P,
                               _U64, _P, _U64P, _U64P, _P]),
        "cl_count": (S, [ctypes.POINTER(cl_graph), ctypes.c_uint32, ctypes.POINTER(cl_tuning), _P, _U64, _U64P,
                         _U64P, _P]),
        "cl_sample_into_noalloc": (S, [ctypes.POINTER(cl_graph), ctypes.c_uint32, ctypes.POINTER(cl_tuning), _P,
                                       _U64, _P, _U64P, _U64P, _P]),
        "cl_generate": (S, [_P, ctypes.POINTER(cl_tuning), _P, _U64, _U64, _P, _P]),
        "cl_plan_info": (S, [_P, _U64P, _U64P, _U64P, _U64P, ctypes.POINTER(ctypes.c_float),
                              ctypes.POINTER(ctypes.c_uint32), _U64P, _P]),
        "cl_hash_edges": (S, [_P, _U64, _U64, _P, _P]),
        "cl_degrees": (S, [_P, ctypes.POINTER(cl_tuning), _P, _U64, _P]),
        "cl_generate_csr": (S, [_P, ctypes.POINTER(cl_tuning), _P, _U64, _P, _U64, _P]),
        "cl_unit_stats": (S, [_P, ctypes.POINTER(cl_tuning), _P, _U64, _U64P, _P]),
        "cl_plan": (S, [ctypes.POINTER(cl_graph), ctypes.c_uint32, ctypes.POINTER(cl_tuning), _P, _U64, _U64P,
                        _P]),
        "cl_batch_capture": (S, [ctypes.POINTER(cl_graph), ctypes.c_uint32, ctypes.POINTER(cl_tuning), _P, _P, _U64,
                                 _P, ctypes.POINTER(ctypes.c_void_p), _P]),
        "cl_batch_launch": (S, [_P, _P]),
        "cl_batch_destroy": (S, [_P]),
        "cl_expected_degree_workspace": (S, [_U64, _U64P]),
        "cl_expected_degree": (S, [_P, _U64, ctypes.c_double, _P, _P, _U64, ctypes.POINTER(cl_tuning), _P]),
        "cl_expected_degree_backward": (S, [_P, _U64, ctypes.c_double, _P, ctypes.c_int, _P, _P, _U64,
                                            ctypes.POINTER(cl_tuning), _P]),
        "cl_device_cus": (ctypes.c_uint32, []),
        "cl_version": (ctypes.c_char_p, []),
    }
    for name, (res, args) in sig.items():
        f = getattr(L, name)
        f.restype = res
        f.argtypes = args
    _lib = L
    return L


def _check(code: int, what: str):
    if code != CL_OK:
        raise ClError(code, what)


def _stream(stream=None):
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


def _ptr(t: Optional[torch.Tensor]):
    return ctypes.c_void_p(t.data_ptr()) if t is not None and t.numel() > 0 else ctypes.c_void_p(0)


def _ws(nbytes: int, device) -> torch.Tensor:
    return torch.empty(max(int(nbytes), 256), dtype=torch.uint8, device=device)


def _tuning(t: Optional[dict]):
    if t is None:
        return None
    return ctypes.pointer(cl_tuning(int(t.get("lane_budget", 0)), int(t.get("blocks_per_cu", 0)),
                                    int(t.get("slot_margin", 0)), int(t.get("partition", 0)),
                                    int(t.get("tail_units", 0)), int(t.get("ed_rows", 0)),
                                    int(t.get("ed_cols", 0)), int(t.get("unit_order", 0))))


def _f64(w: torch.Tensor) -> torch.Tensor:
    if w.dtype != torch.float64 or not w.is_cuda or not w.is_contiguous():
        raise ValueError("weights must be a contiguous float64 CUDA tensor")
    return w


# ---------------------------------------------------------------- exact sum
def cl_weight_sum_workspace(n: int) -> int:
    """Workspace bytes cl_weight_sum needs for n weights."""
    need = _U64(0)
    _check(lib().cl_weight_sum_workspace(int(n), ctypes.byref(need)), "cl_weight_sum_workspace")
    return int(need.value)


def cl_weight_sum(w: torch.Tensor, stream=None, ws: Optional[torch.Tensor] = None) -> float:
    """S = sum(w), exactly rounded (Alg. 1, first line).  ws: a uint8 device
    tensor to reuse as the workspace (allocated here when None or too small)."""
    L = lib()
    w = _f64(w)
    need = _U64(0)
    _check(L.cl_weight_sum_workspace(w.numel(), ctypes.byref(need)), "cl_weight_sum_workspace")
    if ws is None or ws.numel() < need.value or ws.device != w.device:
        ws = _ws(need.value, w.device)
    out = ctypes.c_double(0.0)
    _check(L.cl_weight_sum(_ptr(w), w.numel(), _ptr(ws), ws.numel(), ctypes.byref(out), _stream(stream)),
           "cl_weight_sum")
    return out.value


def cl_expected_edges(w: torch.Tensor, S: float, stream=None):
    """(E[m], Var[m]) under p(u,v) = min(w_u w_v / S, 1)."""
    L = lib()
    w = _f64(w)
    need = _U64(0)
    _check(L.cl_expected_edges_workspace(w.numel(), ctypes.byref(need)), "cl_expected_edges_workspace")
    ws = _ws(need.value, w.device)
    E = ctypes.c_double(0.0)
    V = ctypes.c_double(0.0)
    _check(L.cl_expected_edges(_ptr(w), w.numel(), float(S), _ptr(ws), ws.numel(), ctypes.byref(E), ctypes.byref(V),
                               _stream(stream)), "cl_expected_edges")
    return E.value, V.value


def cl_partition(w: torch.Tensor, S: float, P: int, stream=None):
    """Uniform consecutive partition bounds n_0..n_P (Eq. 5) and the total cost."""
    L = lib()
    w = _f64(w)
    need = _U64(0)
    _check(L.cl_partition_workspace(w.numel(), int(P), ctypes.byref(need)), "cl_partition_workspace")
    ws = _ws(need.value, w.device)
    bounds = (ctypes.c_uint64 * (int(P) + 1))()
    Z = _U64(0)
    _check(L.cl_partition(_ptr(w), w.numel(), float(S), int(P), _ptr(ws), ws.numel(), bounds, ctypes.byref(Z),
                          _stream(stream)), "cl_partition")
    return [int(x) for x in bounds], int(Z.value)


# ------------------------------------------------------------ generation
@dataclass
class Task:
    """Create-Edges(w, S, [u_begin, u_end)) with Philox key `seed`."""
    w: torch.Tensor
    S: float
    seed: int
    u_begin: int = 0
    u_end: Optional[int] = None


@dataclass
class Plan:
    ws: torch.Tensor
    graphs: object            # ctypes array of cl_graph (kept alive with the tensors)
    tasks: List[Task]
    m: List[int]
    tuning: Optional[dict] = None
    keep: list = field(default_factory=list)

    @property
    def total(self) -> int:
        return int(sum(self.m))


def _graph_array(tasks: Sequence[Task]):
    arr = (cl_graph * len(tasks))()
    for i, t in enumerate(tasks):
        w = _f64(t.w)
        n = w.numel()
        ue = n if t.u_end is None else int(t.u_end)
        arr[i] = cl_graph(w.data_ptr() if n > 0 else 0, n, float(t.S), int(t.seed) & ((1 << 64) - 1),
                          int(t.u_begin), ue)
    return arr


def _plan(fn_name: str, one_pass: int, tasks: Sequence[Task], tuning, ws, stream, into=None,
          ws_growth: float = 1.0) -> Plan:
    L = lib()
    tasks = list(tasks)
    arr = _graph_array(tasks)
    G = len(tasks)
    tun = _tuning(tuning)
    dev = tasks[0].w.device
    if ws is None:
        # the part known before the data is seen; the data-dependent rest is
        # reported by the first call (CL_ERR_WORKSPACE + required bytes)
        fixed = _U64(0)
        est = _U64(0)
        _check(L.cl_workspace_size(arr, G, tun, one_pass, ctypes.byref(fixed), ctypes.byref(est)),
               "cl_workspace_size")
        free = torch.cuda.mem_get_info(dev)[0]
        ws = _ws(est.value if est.value < free // 4 else fixed.value, dev)
    m = (ctypes.c_uint64 * G)()
    req = _U64(0)
    fn = getattr(L, fn_name)
    if fn_name == "cl_plan":   # no edge counts
        call = lambda: fn(arr, G, tun, _ptr(ws), ws.numel(), ctypes.byref(req), _stream(stream))
    elif fn_name == "cl_sample_into":
        edges, cap, offs = into
        call = lambda: fn(arr, G, tun, _ptr(ws), ws.numel(), _ptr(edges), int(cap), _ptr(offs), m,
                          ctypes.byref(req), _stream(stream))
    else:
        call = lambda: fn(arr, G, tun, _ptr(ws), ws.numel(), m, ctypes.byref(req), _stream(stream))
    code = call()
    for _ in range(2):   # a too small workspace: first the fixed part, then the data-dependent rest
        if code != -6:
            break
        ws = None   # release the old workspace before the larger one is allocated
        ws = _ws(int(req.value * ws_growth), dev)
        code = call()
    plan = Plan(ws=ws, graphs=arr, tasks=tasks, m=[int(x) for x in m], tuning=tuning)
    if into is not None and code == -7:   # the edges did not fit: m is known, the plan is kept
        plan.keep.append("over_capacity")
        return plan
    _check(code, fn_name)
    return plan


def cl_count(tasks: Sequence[Task], tuning: Optional[dict] = None, ws: Optional[torch.Tensor] = None,
             stream=None) -> Plan:
    """Plans the tasks and counts their edges (count pass + offsets)."""
    return _plan("cl_count", 0, tasks, tuning, ws, stream)


def cl_sample(tasks: Sequence[Task], tuning: Optional[dict] = None, ws: Optional[torch.Tensor] = None,
              stream=None) -> Plan:
    """Plans the tasks and generates them in one pass into per-lane slots of
    the workspace; cl_generate then expands the slots into the output."""
    return _plan("cl_sample", 1, tasks, tuning, ws, stream)


def cl_sample_into(tasks: Sequence[Task], edges: torch.Tensor, cap: Optional[int] = None,
                   graph_offsets: Optional[torch.Tensor] = None, tuning: Optional[dict] = None,
                   ws: Optional[torch.Tensor] = None, stream=None, ws_growth: float = 1.0):
    """cl_sample and cl_generate(plan, edges, 0, cap) in one call (no host
    round trip in between).  Returns (plan, fits): when the edges do not fit
    (plan.total > cap), edges hold the first cap of them and cl_generate
    with a larger buffer completes the output from the same plan."""
    if cap is None:
        cap = edges.numel() // 2
    assert edges.dtype == torch.int32 and edges.is_contiguous() and edges.numel() >= 2 * cap
    plan = _plan("cl_sample_into", 1, tasks, tuning, ws, stream, into=(edges, cap, graph_offsets),
                 ws_growth=ws_growth)
    return plan, "over_capacity" not in plan.keep


def cl_sample_into_noalloc(tasks: Sequence[Task], edges: torch.Tensor, cap: Optional[int] = None,
                           graph_offsets: Optional[torch.Tensor] = None, tuning: Optional[dict] = None,
                           stream=None):
    """cl_sample_into with the library's fixed device array as the workspace
    (no device allocation in the call).  Returns (m per task, fits,
    workspace bytes the plan needed).  Raises ClError(CL_ERR_WORKSPACE) when
    the plan would need more than the array holds."""
    L = lib()
    tasks = list(tasks)
    arr = _graph_array(tasks)
    if cap is None:
        cap = edges.numel() // 2
    assert edges.dtype == torch.int32 and edges.is_contiguous() and edges.numel() >= 2 * cap
    m = (ctypes.c_uint64 * len(tasks))()
    req = _U64(0)
    code = L.cl_sample_into_noalloc(arr, len(tasks), _tuning(tuning), _ptr(edges), int(cap), _ptr(graph_offsets), m,
                                    ctypes.byref(req), _stream(stream))
    if code != -7:
        _check(code, "cl_sample_into_noalloc")
    return [int(x) for x in m], code == CL_OK, int(req.value)


NOALLOC_SCRATCH_BYTES = 64 << 20   # CL_NOALLOC_SCRATCH_BYTES


def cl_plan(tasks: Sequence[Task], tuning: Optional[dict] = None, ws: Optional[torch.Tensor] = None,
            stream=None, ws_growth: float = 1.0) -> Plan:
    """The plan alone (no lane kernel, no counts: plan.m is zeros), for cl_degrees."""
    return _plan("cl_plan", 0, tasks, tuning, ws, stream, ws_growth=ws_growth)


def cl_generate(plan: Plan, edges: Optional[torch.Tensor] = None, edge_begin: int = 0, cap: Optional[int] = None,
                graph_offsets: Optional[torch.Tensor] = None, stream=None) -> torch.Tensor:
    """Write pass: edges with batch positions in [edge_begin, edge_begin + cap)
    into an (cap, 2) int32 tensor holding uint32 (u, v) pairs."""
    L = lib()
    if cap is None:
        cap = plan.total - edge_begin
    if edges is None:
        edges = torch.empty((max(int(cap), 1), 2), dtype=torch.int32, device=plan.ws.device)
    assert edges.dtype == torch.int32 and edges.is_contiguous() and edges.numel() >= 2 * cap
    _check(L.cl_generate(_ptr(plan.ws), _tuning(plan.tuning), _ptr(edges), int(edge_begin), int(cap),
                         _ptr(graph_offsets), _stream(stream)), "cl_generate")
    return edges[: int(cap)]


def cl_generate_csr(plan: Plan, col: Optional[torch.Tensor] = None, row_ptr: Optional[torch.Tensor] = None,
                    stream=None):
    """The planned edges as compressed sparse rows: col (int32 tensor holding
    uint32 targets, one per edge in batch order) and, per task, a view of
    row_ptr (int64, n_g + 1 entries: the batch position of each source's
    first edge, then the task's end).  Returns (col[:m], [row views])."""
    L = lib()
    sizes = [int(t.w.numel()) for t in plan.tasks]
    total = sum(n + 1 for n in sizes)
    m = plan.total
    dev = plan.ws.device
    if col is None:
        col = torch.empty(max(m, 1), dtype=torch.int32, device=dev)
    if row_ptr is None:
        row_ptr = torch.empty(max(total, 1), dtype=torch.int64, device=dev)
    assert col.dtype == torch.int32 and col.is_contiguous() and row_ptr.dtype == torch.int64
    _check(L.cl_generate_csr(_ptr(plan.ws), _tuning(plan.tuning), _ptr(col), int(col.numel()), _ptr(row_ptr),
                             int(row_ptr.numel()), _stream(stream)), "cl_generate_csr")
    rows, off = [], 0
    for n in sizes:
        rows.append(row_ptr[off: off + n + 1])
        off += n + 1
    return col[:m], rows


def cl_degrees(plan: Plan, deg: Optional[torch.Tensor] = None, stream=None) -> List[torch.Tensor]:
    """Degrees of the planned graphs without storing edges: adds into `deg`
    (an int32 tensor holding uint32 counts, sum(n_g + 1) entries; created
    zeroed when None) and returns one view of n_g entries per task."""
    L = lib()
    sizes = [int(t.w.numel()) for t in plan.tasks]
    total = sum(n + 1 for n in sizes)
    if deg is None:
        deg = torch.zeros(max(total, 1), dtype=torch.int32, device=plan.ws.device)
    assert deg.dtype == torch.int32 and deg.is_contiguous()
    _check(L.cl_degrees(_ptr(plan.ws), _tuning(plan.tuning), _ptr(deg), int(deg.numel()), _stream(stream)),
           "cl_degrees")
    out, off = [], 0
    for n in sizes:
        out.append(deg[off: off + n])
        off += n + 1
    return out


def cl_unit_stats(plan: Plan, tuning: Optional[dict] = None, stream=None) -> dict:
    """Per-unit records of a statistics pass over the plan (see clgen.h):
    numpy arrays t0, t1 (wave clock, 100 MHz ticks), cost (cost units of
    1/16 expected candidate), visits, edges and lane, one entry per unit
    (padding units included)."""
    import numpy as np
    L = lib()
    units = _U64(0)
    code = L.cl_unit_stats(_ptr(plan.ws), _tuning(tuning if tuning is not None else plan.tuning), None, 0,
                           ctypes.byref(units), _stream(stream))
    if code != -7 and code != CL_OK:
        _check(code, "cl_unit_stats")
    n = int(units.value)
    buf = torch.zeros(4 * max(n, 1), dtype=torch.int64, device=plan.ws.device)
    _check(L.cl_unit_stats(_ptr(plan.ws), _tuning(tuning if tuning is not None else plan.tuning), _ptr(buf),
                           buf.numel(), None, _stream(stream)), "cl_unit_stats")
    a = buf.cpu().numpy().view(np.uint64).reshape(-1, 4)[:n]
    w2 = a[:, 2]
    w3 = a[:, 3]
    return {"t0": a[:, 0], "t1": a[:, 1], "cost": (w2 & 0xFFFFFFFF), "visits": (w2 >> np.uint64(32)),
            "edges": (w3 & 0xFFFFFFFF), "lane": (w3 >> np.uint64(32))}


def cl_plan_info(plan_or_ws, stream=None) -> dict:
    L = lib()
    ws = plan_or_ws.ws if isinstance(plan_or_ws, Plan) else plan_or_ws
    lanes, nh, m, nc, sw = _U64(0), _U64(0), _U64(0), _U64(0), _U64(0)
    ms = ctypes.c_float(0.0)
    ov = ctypes.c_uint32(0)
    code = L.cl_plan_info(_ptr(ws), ctypes.byref(lanes), ctypes.byref(nh), ctypes.byref(m), ctypes.byref(nc),
                          ctypes.byref(ms), ctypes.byref(ov), ctypes.byref(sw), _stream(stream))
    return {"status": code, "lanes": int(lanes.value), "heavy_segments": int(nh.value), "edges": int(m.value),
            "candidates": int(nc.value), "lane_kernel_ms": float(ms.value), "overflow_lanes": int(ov.value),
            "slot_words": int(sw.value)}


def cl_hash_edges(edges: torch.Tensor, index_base: int = 0, acc: Optional[torch.Tensor] = None,
                  stream=None) -> torch.Tensor:
    """Adds the position-keyed digest of `edges` into acc (a 1-element int64
    CUDA tensor, created zeroed when None) and returns acc."""
    L = lib()
    if acc is None:
        acc = torch.zeros(1, dtype=torch.int64, device=edges.device)
    m = edges.shape[0] if edges.numel() else 0
    _check(L.cl_hash_edges(_ptr(edges), int(m), int(index_base), _ptr(acc), _stream(stream)), "cl_hash_edges")
    return acc


def hash_value(acc: torch.Tensor) -> int:
    return int(acc.item()) & ((1 << 64) - 1)


# --------------------------------------------------------------- batches
class BatchGraph:
    """A captured, replayable batch generation (cl_batch_capture)."""

    def __init__(self, exec_handle, plan: Plan, edges, graph_offsets):
        self.handle = exec_handle
        self.plan = plan
        self.edges = edges
        self.graph_offsets = graph_offsets

    def launch(self, stream=None):
        _check(lib().cl_batch_launch(self.handle, _stream(stream)), "cl_batch_launch")

    def close(self):
        if self.handle:
            lib().cl_batch_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def cl_batch_capture(plan: Plan, stream: torch.cuda.Stream, cap: Optional[int] = None,
                     edges: Optional[torch.Tensor] = None, graph_offsets: Optional[torch.Tensor] = None) -> BatchGraph:
    L = lib()
    if cap is None:
        cap = plan.total
    dev = plan.ws.device
    if edges is None:
        edges = torch.empty((max(int(cap), 1), 2), dtype=torch.int32, device=dev)
    if graph_offsets is None:
        graph_offsets = torch.zeros(len(plan.tasks) + 1, dtype=torch.int64, device=dev)
    h = ctypes.c_void_p(0)
    _check(L.cl_batch_capture(plan.graphs, len(plan.tasks), _tuning(plan.tuning), _ptr(plan.ws), _ptr(edges),
                              int(cap), _ptr(graph_offsets), ctypes.byref(h), _stream(stream)), "cl_batch_capture")
    return BatchGraph(h, plan, edges, graph_offsets)


# ------------------------------------------------------- expected degree
def _ed_ws(n: int, device) -> torch.Tensor:
    need = _U64(0)
    _check(lib().cl_expected_degree_workspace(int(n), ctypes.byref(need)), "cl_expected_degree_workspace")
    return _ws(need.value, device)


def cl_expected_degree(w32: torch.Tensor, S: float, ws: Optional[torch.Tensor] = None, stream=None,
                       tuning: Optional[dict] = None) -> torch.Tensor:
    """d_i = sum_{j != i} min(w_i w_j / S, 1) (float32 tiles, float64 rows);
    tuning may give the tile shape (ed_rows, ed_cols)."""
    assert w32.dtype == torch.float32 and w32.is_contiguous()
    n = w32.numel()
    if ws is None:
        ws = _ed_ws(n, w32.device)
    d = torch.empty(n, dtype=torch.float64, device=w32.device)
    _check(lib().cl_expected_degree(_ptr(w32), n, float(S), _ptr(d), _ptr(ws), ws.numel(), _tuning(tuning),
                                    _stream(stream)), "cl_expected_degree")
    return d


def cl_expected_degree_backward(w32: torch.Tensor, S: float, grad_d: torch.Tensor, s_depends_on_w: bool = True,
                                ws: Optional[torch.Tensor] = None, stream=None,
                                tuning: Optional[dict] = None) -> torch.Tensor:
    assert w32.dtype == torch.float32 and grad_d.dtype == torch.float64
    n = w32.numel()
    if ws is None:
        ws = _ed_ws(n, w32.device)
    g = torch.empty(n, dtype=torch.float32, device=w32.device)
    _check(lib().cl_expected_degree_backward(_ptr(w32), n, float(S), _ptr(grad_d.contiguous()),
                                             1 if s_depends_on_w else 0, _ptr(g), _ptr(ws), ws.numel(),
                                             _tuning(tuning), _stream(stream)), "cl_expected_degree_backward")
    return g


# ----------------------------------------------------------- convenience
def generate(w: torch.Tensor, seed: int, S: Optional[float] = None, u_begin: int = 0, u_end: Optional[int] = None,
             tuning: Optional[dict] = None) -> torch.Tensor:
    """Serial-CL(w) of Alg. 1 on the GPU: S (exact sum unless given), count,
    write.  Returns an (m, 2) int32 tensor of uint32 (u, v) pairs."""
    if S is None:
        S = cl_weight_sum(w)
    plan = cl_sample([Task(w, S, seed, u_begin, u_end)], tuning=tuning)
    return cl_generate(plan)
