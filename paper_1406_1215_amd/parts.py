"""Whole graphs too large for one plan, generated part by part.

The node range is cut by the uniform consecutive partition (Sec. 4, Eq. 5,
cl_partition) into parts of equal expected cost; each part is planned alone
(cl_plan) and its edges are consumed on the fly.  Draws are keyed by
(seed, u, segment, draw index), so the union of the parts is the edge set of
the whole graph, whatever the number of parts.
"""
from __future__ import annotations

import time
from typing import Optional

import torch

from . import clgen


def degrees(w: torch.Tensor, S: float, seed: int, parts: int, tuning: Optional[dict] = None,
            deg: Optional[torch.Tensor] = None, log=None) -> dict:
    """Degree sequence of the whole graph (no edge is stored): cl_degrees on
    every part of a `parts`-way uniform consecutive partition, accumulated in
    one uint32 array (held in an int32 tensor of n + 1 entries)."""
    n = w.numel()
    if deg is None:
        deg = torch.zeros(n + 1, dtype=torch.int32, device=w.device)
    torch.cuda.synchronize(w.device)
    t0 = time.perf_counter()
    bounds, Z = clgen.cl_partition(w, S, parts)
    ws = None
    for p in range(parts):
        a, b = bounds[p], bounds[p + 1]
        if a == b:
            continue
        plan = clgen.cl_plan([clgen.Task(w, S, seed, a, b)], tuning=tuning, ws=ws, ws_growth=1.5)
        ws = plan.ws
        clgen.cl_degrees(plan, deg=deg)
        if log:
            log(f"part {p}: sources [{a}, {b})")
    torch.cuda.synchronize(w.device)
    secs = time.perf_counter() - t0
    total = int(deg[:n].to(torch.int64).sum().item())   # counts are < 2^31 for n < 2^31 nodes of degree < n
    return {"deg": deg[:n], "edges": total // 2, "seconds": secs, "bounds": bounds, "cost": Z}


def edges(w: torch.Tensor, S: float, seed: int, parts: int, tuning: Optional[dict] = None, consume=None,
          log=None) -> dict:
    """Every edge of the whole graph, part by part: each part of a
    `parts`-way uniform consecutive partition is generated in one pass into
    one reused output buffer (cl_sample_into), then handed to
    consume(edges, first_position) while it is resident, and overwritten by
    the next part.  The parts are consecutive source ranges, so their
    concatenation is the whole (u, v)-sorted edge list.  The default consumer
    adds the position-keyed digest (cl_hash_edges) of every edge."""
    dev = w.device
    acc = torch.zeros(1, dtype=torch.int64, device=dev)
    if consume is None:
        def consume(e, first):
            clgen.cl_hash_edges(e, first, acc)
    torch.cuda.synchronize(dev)
    t0 = time.perf_counter()
    bounds, Z = clgen.cl_partition(w, S, parts)
    ws = None
    buf = torch.empty((1, 2), dtype=torch.int32, device=dev)
    total = 0
    largest = 0
    for p in range(parts):
        a, b = bounds[p], bounds[p + 1]
        if a == b:
            continue
        plan, fits = clgen.cl_sample_into([clgen.Task(w, S, seed, a, b)], buf, tuning=tuning, ws=ws, ws_growth=1.5)
        ws = plan.ws
        m = plan.total
        if not fits:   # grow the buffer (with some room for the next parts) and expand again
            buf = None
            buf = torch.empty((int(m * 1.1) + 1024, 2), dtype=torch.int32, device=dev)
            clgen.cl_generate(plan, edges=buf, cap=m)
        consume(buf[:m], total)
        total += m
        largest = max(largest, m)
        if log:
            log(f"part {p}: sources [{a}, {b}), {m} edges")
    torch.cuda.synchronize(dev)
    secs = time.perf_counter() - t0
    return {"edges": total, "seconds": secs, "digest": clgen.hash_value(acc), "largest_part": largest,
            "bounds": bounds, "cost": Z}
