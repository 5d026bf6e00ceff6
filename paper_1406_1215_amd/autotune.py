"""Autotuner of the generator's schedule knobs.

The knobs (cl_tuning: lane budget = expected candidates per lane, i.e. the
chunk size of the uniform-cost split of Eq. 5 across lanes, and the
persistent grid in blocks per compute unit) change only the launch schedule:
the edge list is a pure function of (w, S, seed, range).  The tile shape of
the expected-degree kernels (rows per thread, columns per tile) is tuned the
same way (``tune_expdeg``); it changes only the float32 summation order
inside a tile.  The tuner times
every candidate setting on the caller's tasks, checks that each produces the
same digest as the first, and keeps the fastest.  Results are cached per
(device, size bucket) in a JSON file.
"""
from __future__ import annotations

import json
import math
import os
import time
from typing import Dict, Iterable, List, Optional, Sequence

import torch

from . import clgen

CACHE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "tuned.json")
BUDGETS = (64, 96, 128, 192, 256, 384, 512)
BLOCKS_PER_CU = (2, 3, 4, 8)


def size_bucket(total_edges: float) -> str:
    """log2 bucket of the expected output size."""
    return f"e2^{int(math.floor(math.log2(max(total_edges, 1.0))))}"


def device_key() -> str:
    p = torch.cuda.get_device_properties(0)
    return f"{p.name}:{getattr(p, 'gcnArchName', '')}:{p.multi_processor_count}"


def _run(tasks, tuning, planner, edges=None):
    plan = getattr(clgen, planner)(tasks, tuning=tuning)
    m = plan.total
    if edges is None or edges.shape[0] < m:
        edges = torch.empty((max(m, 1) + 1024, 2), dtype=torch.int32, device=tasks[0].w.device)
    clgen.cl_generate(plan, edges=edges, cap=m)
    return plan, edges


def tune(tasks: Sequence[clgen.Task], planner: str = "cl_sample", budgets: Iterable[int] = BUDGETS,
         blocks: Iterable[int] = BLOCKS_PER_CU, reps: int = 2, save: bool = True) -> Dict:
    """Times every (budget, blocks_per_cu) pair; returns the fastest and the
    table.  Raises if any setting changes the output digest."""
    tasks = list(tasks)
    table = []
    ref_hash = None
    edges = None
    for b in budgets:
        for bpc in blocks:
            tun = {"lane_budget": int(b), "blocks_per_cu": int(bpc)}
            plan, edges = _run(tasks, tun, planner, edges)           # warm (and sizes the workspace)
            m = plan.total
            acc = clgen.cl_hash_edges(edges[:m])
            h = clgen.hash_value(acc)
            if ref_hash is None:
                ref_hash = (m, h)
            elif (m, h) != ref_hash:
                raise RuntimeError(f"tuning {tun} changed the output ({(m, h)} != {ref_hash})")
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(reps):
                plan, edges = _run(tasks, tun, planner, edges)
            torch.cuda.synchronize()
            dt = (time.perf_counter() - t0) / reps
            table.append({"lane_budget": int(b), "blocks_per_cu": int(bpc), "ms": dt * 1e3})
    best = min(table, key=lambda r: r["ms"])
    result = {"best": {"lane_budget": best["lane_budget"], "blocks_per_cu": best["blocks_per_cu"]},
              "best_ms": best["ms"], "table": table, "edges": ref_hash[0]}
    if save:
        store(size_bucket(ref_hash[0]), result["best"], best["ms"])
    return result


def tune_batch(tasks: Sequence[clgen.Task], budgets: Iterable[int] = (96, 128, 192, 256, 384),
               blocks: Iterable[int] = (2, 3, 4, 6), reps: int = 3, save: bool = True) -> Dict:
    """Tunes the batched path as it is measured: for every (budget,
    blocks_per_cu) pair, one plan of all tasks (cl_sample), the whole path
    captured in a HIP graph (cl_batch_capture) and the mean time of `reps`
    replays.  Raises if any setting changes the output digest."""
    tasks = list(tasks)
    table = []
    ref = None
    dev = tasks[0].w.device
    s = torch.cuda.Stream(device=dev)
    edges = None
    for b in budgets:
        for bpc in blocks:
            tun = {"lane_budget": int(b), "blocks_per_cu": int(bpc)}
            plan = clgen.cl_sample(tasks, tuning=tun)
            m = plan.total
            if edges is None or edges.shape[0] < m:
                edges = torch.empty((max(m, 1) + 1024, 2), dtype=torch.int32, device=dev)
            bg = clgen.cl_batch_capture(plan, s, cap=m, edges=edges)
            bg.launch(s)
            s.synchronize()
            with torch.cuda.stream(s):
                h = clgen.hash_value(clgen.cl_hash_edges(edges[:m], stream=s))
            if ref is None:
                ref = (m, h)
            elif (m, h) != ref:
                bg.close()
                raise RuntimeError(f"tuning {tun} changed the output ({(m, h)} != {ref})")
            s.synchronize()
            t0 = time.perf_counter()
            for _ in range(reps):
                bg.launch(s)
            s.synchronize()
            dt = (time.perf_counter() - t0) / reps
            bg.close()
            del plan
            table.append({"lane_budget": int(b), "blocks_per_cu": int(bpc), "ms": dt * 1e3})
    best = min(table, key=lambda r: r["ms"])
    result = {"best": {"lane_budget": best["lane_budget"], "blocks_per_cu": best["blocks_per_cu"]},
              "best_ms": best["ms"], "table": table, "edges": ref[0]}
    if save:
        store("batch:" + size_bucket(ref[0]), result["best"], best["ms"])
    return result


ED_SHAPES = tuple({"ed_rows": r, "ed_cols": c} for r in (1, 2, 4) for c in (512, 1024, 2048))


def tune_expdeg(w32: torch.Tensor, S: float, shapes: Iterable[Dict] = ED_SHAPES, reps: int = 3,
                save: bool = True) -> Dict:
    """Tile shape of the expected-degree kernels (rows per thread x columns
    per tile): times forward + adjoint for each shape on these weights.  The
    shape changes only the float32 summation order inside a tile, so each
    result is checked against the first shape's (d: relative 1e-5; gradient:
    normwise relative 1e-5), and a larger difference raises."""
    n = w32.numel()
    g = torch.ones(n, dtype=torch.float64, device=w32.device)
    ws = clgen._ed_ws(n, w32.device)
    table = []
    ref = None
    for sh in shapes:
        sh = dict(sh)
        d = clgen.cl_expected_degree(w32, S, ws=ws, tuning=sh)
        gr = clgen.cl_expected_degree_backward(w32, S, g, True, ws=ws, tuning=sh).double()
        if ref is None:
            ref = (d, gr)
        else:
            ed = float((torch.abs(d - ref[0]) / ref[0].clamp_min(1e-300)).max())
            eg = float(torch.linalg.norm(gr - ref[1]) / torch.linalg.norm(ref[1]).clamp_min(1e-300))
            if ed > 1e-5 or eg > 1e-5:
                raise RuntimeError(f"tile shape {sh} changed the result beyond rounding ({ed}, {eg})")
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            clgen.cl_expected_degree(w32, S, ws=ws, tuning=sh)
            clgen.cl_expected_degree_backward(w32, S, g, True, ws=ws, tuning=sh)
        torch.cuda.synchronize()
        table.append(dict(sh, ms=(time.perf_counter() - t0) / reps * 1e3))
    best = min(table, key=lambda r: r["ms"])
    result = {"best": {"ed_rows": best["ed_rows"], "ed_cols": best["ed_cols"]}, "best_ms": best["ms"],
              "table": table, "pairs": float(n) * float(n)}
    if save:
        store("expdeg:" + size_bucket(float(n) * float(n)), result["best"], best["ms"])
    return result


def load() -> Dict:
    try:
        with open(CACHE) as f:
            return json.load(f)
    except (OSError, ValueError):
        return {}


def store(bucket: str, best: Dict, ms: float) -> None:
    data = load()
    data.setdefault(device_key(), {})[bucket] = {"tuning": best, "ms": ms}
    tmp = CACHE + ".tmp"
    with open(tmp, "w") as f:
        json.dump(data, f, indent=1, sort_keys=True)
    os.replace(tmp, CACHE)


def lookup(expected_edges: float, kind: str = "") -> Optional[Dict]:
    """Cached tuning for about this many edges (nearest bucket), from the
    plain tuner (kind "") or the batched one (kind "batch")."""
    data = load().get(device_key() if torch.cuda.is_available() else "", {})
    prefix = kind + ":" if kind else ""
    data = {k[len(prefix):]: v for k, v in data.items() if k.startswith(prefix) and ":" not in k[len(prefix):]}
    if not data:
        return None
    want = int(math.floor(math.log2(max(expected_edges, 1.0))))
    best = min(data.items(), key=lambda kv: abs(int(kv[0].split("^")[1]) - want))
    return dict(best[1]["tuning"])
