#!/usr/bin/env python3
"""Throughput of the Chung-Lu generation path on one MI355X.

A step is one pass of the whole generation path over the n = 1e7 power-law
workload (exponent 2.1, w_min = 10, weights capped at sqrt(S), Philox seed 2),
inputs resident in HBM: exact sum S, plan (validation, quantised prefix,
segments, lane plan), one pass of every lane into its slot (counting and
writing), offsets, compaction of the slots into the contiguous edge list
(after the first step, which allocates the output, plan + one pass +
compaction are one call, cl_sample_into).  `value` is edges generated per
second.  Printed as one JSON line, with:

* roofline: the one-pass generation kernel (Alg. 1 per lane, edges staged
  into 64-byte chunks of per-lane slots), timed with HIP events on its stream.
  Its bound is the memory system: every visited candidate reads one weight
  w_v at an essentially random position (8 algorithmic bytes, one 128-byte
  line from HBM or the Infinity Cache on an L2 miss) and every kept edge
  writes a 4-byte slot word (v; a mark and u are added where the source
  changes).  achieved = (8 B x candidates + 4 B x slot words) / launch time
  against 8 TB/s; traffic = the kernel's measured HBM bytes (FETCH_SIZE +
  WRITE_SIZE, scaled by a copy kernel of known size) from the committed
  counter summary when it was taken on the current kernel source;
  alu_view gives the same launch against the VALU peak;
* hbm_write: bytes written per second by that kernel (slot words) and moved
  by the compaction (slot words read, 8-byte edges written), against 8 TB/s;
* two_pass: the count-then-replay path (count pass, offsets, write pass);
* expected_degree: the float32 tiled expected-degree kernel and its adjoint
  on n = 1e5 (1e10 pairs), against the VALU lane-operation peak;
* csr: the same plan written as compressed sparse rows (4-byte targets and
  row offsets) instead of (u, v) pairs;
* calibration: 200 Adam steps on log w against n = 1e5 capped targets, then
  generation from the calibrated weights;
* partition_ablation: generation-kernel time with work units of equal
  expected cost (Eq. 5) vs units of equal source counts (Sec. 4's naive
  consecutive partition), same number of units; and the degree kernel under
  those two and round-robin units (Sec. 4's RRP);
* batched: 256 uneven graphs in one captured HIP graph vs 256 plain calls;
* cpu_baseline: the CPU oracle on a bounded sample of the same workload.
"""
import argparse
import hashlib
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

OPS_PER_CANDIDATE = 145          # operation count of one candidate step of the sampling rule
# 7.86e13 lane-ops/s: the published fp32 vector peak (157.3 TFLOP/s) counts
# an FMA as two flops, i.e. 128 lanes per CU per clock x 256 CUs x 2.4 GHz.
# Without packed fp32 math an FMA issues at half this rate.
PEAK_LANE_OPS = 256 * 128 * 2.4e9
BYTES_PER_CANDIDATE = 8           # w_v gathered
BYTES_PER_SLOT_WORD = 4           # slot words written: v per edge, (mark, u) per change of source
BYTES_PER_EDGE = 8                # (u, v) uint32 pair of the edge list
HBM_PEAK = 8.0e12                 # bytes/s
METRIC = "edges/sec generated on 1 MI355X + % HBM write roofline; batched vs plain"
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_generation_plain_1e7.json")
KERNEL_SOURCES = ["cl_device.hpp", "cl_kernels.hpp", "cl_plan.hpp"]


def kernel_hash() -> str:
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, "paper_1406_1215_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def traffic_per_launch():
    """HBM bytes per launch of the write pass from the committed counter
    summary, if it was taken on the current kernel source."""
    try:
        with open(TRAFFIC_FILE) as f:
            t = json.load(f)
    except (OSError, ValueError):
        return None
    if t.get("kernel_hash") != kernel_hash():
        return None
    return t.get("bytes_per_launch")


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-batched", action="store_true")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-two-pass", action="store_true")
    ap.add_argument("--no-ablation", action="store_true")
    ap.add_argument("--no-expdeg", action="store_true")
    ap.add_argument("--no-calib", action="store_true")
    ap.add_argument("--no-csr", action="store_true")
    ap.add_argument("--full-graph-degrees", action="store_true",
                    help="instead of the step: the degree sequence of the whole n=1e9 graph (exponent 2.1, mean "
                         "degree 500), every edge generated and consumed on the fly, part by part")
    ap.add_argument("--full-graph-edges", action="store_true",
                    help="instead of the step: every edge of the whole n=1e9 graph written to device memory part "
                         "by part (one reused buffer) and digested")
    ap.add_argument("--parts", type=int, default=64)
    ap.add_argument("--batched-reps", type=int, default=3)
    ap.add_argument("--n", type=int, default=10_000_000, help="sources of the plain workload")
    ap.add_argument("--verbose", action="store_true")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="also run one plain device copy of 2 GiB (for counter scaling)")
    return ap.parse_args()


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py measures one GPU; --gpus {args.gpus} is not supported: the generator runs on a single "
              f"MI355X (across GPUs, each would take parts of the uniform consecutive partition, Eq. 5)",
              file=sys.stderr)
        sys.exit(2)
    import numpy as np
    import torch
    from paper_1406_1215_amd import clgen as cg
    from paper_1406_1215_amd import workloads as W

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(1)
    cg.lib()
    dev = torch.device("cuda:0")
    stream = torch.cuda.current_stream()
    if args.full_graph_degrees or args.full_graph_edges:
        print(json.dumps(bench_full_graph(args, cg, W, torch, np, dev)), flush=True)
        return

    log("bench: generating the n=1e7 workload")
    w_np = W.config_plain(n=args.n)
    w = torch.from_numpy(w_np).to(dev)
    seed = 2

    # one-pass path (the default): S, plan + one pass into slots, compaction
    edges = None
    plan = None
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    sum_ws = torch.empty(cg.cl_weight_sum_workspace(w.numel()), dtype=torch.uint8, device=dev)

    def step(fused=True):
        """One step; with an output buffer from an earlier step, the plan, the
        one pass and the expansion run in one call (cl_sample_into)."""
        nonlocal edges, plan
        S = cg.cl_weight_sum(w, ws=sum_ws)
        if fused and edges is not None:
            plan, fits = cg.cl_sample_into([cg.Task(w, S, seed)], edges, ws=plan.ws)
            if fits:
                return plan.total
        plan = cg.cl_sample([cg.Task(w, S, seed)], ws=plan.ws if plan is not None else None)
        m = plan.total
        if args.verbose:
            log(f"bench: S = {S}, {m} edges")
        if edges is None or edges.shape[0] < m:
            edges = torch.empty((int(m * 1.02) + 1024, 2), dtype=torch.int32, device=dev)
        ev0.record(stream)
        cg.cl_generate(plan, edges=edges, cap=m)
        ev1.record(stream)
        return m

    log(f"bench: warmup {args.warmup}")
    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    log(f"bench: timing {args.steps} steps")
    total_edges = 0
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        total_edges += step()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    elapsed = t1 - t0
    # kernel times of the same step, outside the timed region (reading them
    # back costs a host round trip per step)
    copy_ms, lane_ms = [], []
    for _ in range(max(3, min(args.steps, 10))):
        step(fused=False)
        ev1.synchronize()
        copy_ms.append(ev0.elapsed_time(ev1))
        lane_ms.append(cg.cl_plan_info(plan)["lane_kernel_ms"])
    m = plan.total
    info = cg.cl_plan_info(plan)
    cand = info["candidates"]
    words = info["slot_words"]
    t_gen = sum(lane_ms) / len(lane_ms) / 1e3
    t_copy = sum(copy_ms) / len(copy_ms) / 1e3
    ms_step = elapsed / args.steps * 1e3
    value = total_edges / elapsed
    achieved_ops = cand * OPS_PER_CANDIDATE / t_gen
    alg_bytes = BYTES_PER_CANDIDATE * cand + BYTES_PER_SLOT_WORD * words
    achieved_bw = alg_bytes / t_gen
    traffic = traffic_per_launch()
    result = {
        "metric": METRIC,
        "value": value,
        "unit": "edges/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"plain CL, n={args.n:.0e}, power law exponent 2.1, w_min=10, capped at sqrt(S), "
                               f"Philox seed 2",
                   "n": int(w_np.size), "edges": int(m), "candidates": int(cand), "lanes": info["lanes"],
                   "heavy_segments": info["heavy_segments"], "path": "one pass into slots + compaction"},
        "roofline": {
            "kernel": "one-pass generation (k_lanes<2>)",
            "bound": "hbm",
            "achieved": achieved_bw / 1e9,
            "peak": HBM_PEAK / 1e9,
            "unit": "GB/s",
            "frac": achieved_bw / HBM_PEAK,
            "traffic": traffic,
            "algorithmic_bytes_per_launch": int(alg_bytes),
            "per_unit": "8 B per visited candidate (w_v gather) + 4 B per slot word written "
                        "(v of each edge; a mark and u where the source changes)",
            "candidates_per_launch": int(cand),
            "slot_words_per_launch": int(words),
            "launch_ms": t_gen * 1e3,
        },
        "alu_view": {
            "achieved": achieved_ops / 1e12,
            "peak": PEAK_LANE_OPS / 1e12,
            "unit": "Top/s",
            "frac": achieved_ops / PEAK_LANE_OPS,
            "ops_per_candidate": OPS_PER_CANDIDATE,
        },
        "hbm_write": {
            "generation_GBps": 4.0 * words / t_gen / 1e9,
            "generation_frac_of_8TBps": 4.0 * words / t_gen / HBM_PEAK,
            "compaction_ms": t_copy * 1e3,
            "compaction_GBps_read_plus_write": (4.0 * words + 8.0 * m) / t_copy / 1e9,
            "whole_step_GBps": 8.0 * total_edges / elapsed / 1e9,
            "whole_step_frac_of_8TBps": 8.0 * total_edges / elapsed / HBM_PEAK,
        },
    }
    if not args.no_two_pass:
        result["two_pass"] = bench_two_pass(args, cg, torch, w, seed, dev, stream)
    if not args.no_csr:
        result["csr"] = bench_csr(cg, torch, w, seed, plan, t_copy)

    if not args.no_ablation:
        result["partition_ablation"] = bench_partition(cg, torch, w, seed)

    if not args.no_expdeg:
        result["expected_degree"] = bench_expdeg(cg, W, torch, dev)
    if not args.no_calib:
        result["calibration"] = bench_calibration(cg, W, torch, dev)

    if not args.no_batched:
        result["batched"] = bench_batched(args, cg, W, torch, np, dev)

    if args.copy_calibration:
        # a plain device copy of 2 GiB whose source is not in any cache (a
        # 2 GiB fill of another buffer runs in between): its FETCH_SIZE and
        # WRITE_SIZE read 2 GiB each when the counters are exact
        n8 = 1 << 28
        x = torch.empty(n8, dtype=torch.float64, device=dev)
        y = torch.empty_like(x)
        z = torch.empty_like(x)
        x.fill_(1.0)
        z.fill_(2.0)
        torch.cuda.synchronize()
        y.copy_(x)
        torch.cuda.synchronize()
        result["copy_calibration_bytes"] = n8 * 8
        del x, y, z

    if not args.no_cpu:
        result["cpu_baseline"] = bench_cpu(w_np, seed)

    print(json.dumps(result), flush=True)


def bench_full_graph(args, cg, W, torch, np, dev):
    """The paper's largest power-law shape (1e9 nodes, mean degree 500) on one
    GPU: all edges generated part by part (uniform consecutive partition) and
    either reduced to the degree sequence (--full-graph-degrees) or written
    to device memory, part after part into one buffer, and digested
    (--full-graph-edges); m checked against E[m] and Var[m]."""
    from paper_1406_1215_amd import parts
    log("bench: generating the n=1e9 weights")
    w_np = W.config_share()
    w = torch.from_numpy(w_np).to(dev)
    del w_np
    S = cg.cl_weight_sum(w)
    Em, Vm = cg.cl_expected_edges(w, S)
    log(f"bench: S = {S:.6g}, E[m] = {Em:.6g}; {args.parts} parts")
    seed = 3
    tail = w[-(1 << 20):].contiguous()   # warm-up on the lightest 2^20 nodes (a sparse graph)
    fn = parts.edges if args.full_graph_edges else parts.degrees
    fn(tail, float(tail.sum().item()), seed, 2)
    del tail
    res = fn(w, S, seed, args.parts, log=log if args.verbose else None)
    m = res["edges"]
    z = (m - Em) / math.sqrt(Vm)
    out = {"metric": ("edges/sec generated into device memory and digested, whole graph" if args.full_graph_edges
                      else "edges/sec generated and reduced to degrees, whole graph"),
           "value": m / res["seconds"], "unit": "edges/s", "n_gpus": 1, "higher_is_better": True,
           "data": "synthetic", "dtype": "f64",
           "config": {"workload": "power law, n=1e9, exponent 2.1, mean degree 500, cap sqrt(500 n), Philox seed 3",
                      "parts": args.parts},
           "edges": m, "seconds": res["seconds"], "expected_edges": Em, "z_score_of_m": z}
    if args.full_graph_edges:
        out["digest"] = res["digest"]
        out["largest_part_edges"] = res["largest_part"]
    else:
        deg = res["deg"]
        out["max_degree"] = int(deg.max().item())
        out["isolated_nodes"] = int((deg == 0).sum().item())
    return out


def bench_expdeg(cg, W, torch, dev, reps=5):
    """Expected degree d_i = sum_{j != i} min(w_i w_j / S, 1) and its adjoint
    on n = 1e5 float32 weights (1e10 pairs each), timed with events; ALU
    work 3 lane-operations per pair forward (multiply, min, add) and 3
    backward (the clamped multiply-add that forms the mask, and one
    multiply-add for each of the two sums; FMA-class, so at most half of
    the lane-operation peak without packed math)."""
    t = W.config_calib()
    w32 = torch.from_numpy(t.astype("float32")).to(dev)
    S = float(w32.double().sum().item())
    n = w32.numel()
    g = torch.randn(n, dtype=torch.float64, device=dev)
    ws = cg._ed_ws(n, dev)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    out = {"n": n, "pairs": n * n}
    for name, fn, ops in (("forward", lambda: cg.cl_expected_degree(w32, S, ws=ws), 3),
                          ("backward", lambda: cg.cl_expected_degree_backward(w32, S, g, True, ws=ws), 3)):
        fn()
        torch.cuda.synchronize()
        e0.record()
        for _ in range(reps):
            fn()
        e1.record()
        e1.synchronize()
        ms = e0.elapsed_time(e1) / reps
        out[f"{name}_ms"] = ms
        out[f"{name}_pairs_per_s"] = n * n / (ms * 1e-3)
        out[f"{name}_alu_frac"] = n * n * ops / (ms * 1e-3) / PEAK_LANE_OPS
    return out


def bench_csr(cg, torch, w, seed, plan, pairs_ms):
    """The same one-pass plan written as compressed sparse rows
    (cl_generate_csr: 4-byte targets plus row offsets) instead of (u, v)
    pairs; timed with events around the call (which first reads the plan's
    sizes back)."""
    m = plan.total
    col = torch.empty(m, dtype=torch.int32, device=w.device)
    rows = torch.empty(w.numel() + 1, dtype=torch.int64, device=w.device)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    ms = []
    for _ in range(4):
        e0.record()
        cg.cl_generate_csr(plan, col=col, row_ptr=rows)
        e1.record()
        e1.synchronize()
        ms.append(e0.elapsed_time(e1))
    t = min(ms[1:])
    return {"edges": m, "csr_ms": t, "pairs_expansion_ms": pairs_ms * 1e3,
            "bytes_written": 4 * m + 8 * (w.numel() + 1), "GBps_written": (4 * m + 8 * (w.numel() + 1)) / t / 1e6}


def bench_calibration(cg, W, torch, dev, steps=200):
    """The calibration loop on n = 1e5 capped targets: Adam on log w for 200
    steps (forward + adjoint kernels each step, plus torch's elementwise
    work and one scalar read for S), then generation from the sorted
    calibrated weights; wall time of each."""
    from paper_1406_1215_amd.calibrate import calibrate
    t = torch.from_numpy(W.config_calib()).to(dev)
    calibrate(t, steps=3)                          # warm-up
    res = calibrate(t, steps=steps, lr=0.05)
    S = cg.cl_weight_sum(res.w)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    plan = cg.cl_sample([cg.Task(res.w, S, 11)])
    edges = cg.cl_generate(plan)
    torch.cuda.synchronize()
    gen_s = time.perf_counter() - t0
    del edges
    return {"n": int(t.numel()), "adam_steps": steps, "seconds": res.seconds,
            "ms_per_step": res.seconds / steps * 1e3, "max_rel_err": res.max_rel_err,
            "generation_edges": int(plan.total), "generation_ms": gen_s * 1e3}


def bench_partition(cg, torch, w, seed):
    """Sec. 4's comparison on one GPU: work units of equal expected cost
    (Eq. 5 applied to lanes) vs units of equal numbers of sources, same unit
    count; generation-kernel time of each (same output).  Then the degree
    kernel under those two and round-robin units (RRP over segments), timed
    with events around cl_degrees (which includes one small header read)."""
    S = cg.cl_weight_sum(w)
    out = {}
    for name, pol in (("equal_cost_ms", 0), ("equal_sources_ms", 1)):
        plan = None
        ms = []
        for _ in range(3):
            plan = cg.cl_sample([cg.Task(w, S, seed)], tuning={"partition": pol},
                                ws=plan.ws if plan is not None else None)
            ms.append(cg.cl_plan_info(plan)["lane_kernel_ms"])
        out[name] = min(ms)
        out["edges"] = plan.total
        del plan
    out["slowdown_equal_sources"] = out["equal_sources_ms"] / out["equal_cost_ms"]
    # the degree kernel (same candidates, no edge output) under all three unit
    # policies, round robin included (its units do not give ordered edge runs)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    ref = None
    out["degrees_identical"] = True
    for name, pol in (("equal_cost", 0), ("equal_sources", 1), ("round_robin", 2)):
        plan = cg.cl_plan([cg.Task(w, S, seed)], tuning={"partition": pol})
        deg = torch.zeros(w.numel() + 1, dtype=torch.int32, device=w.device)
        ms = []
        for _ in range(3):
            deg.zero_()
            e0.record()
            cg.cl_degrees(plan, deg=deg)
            e1.record()
            e1.synchronize()
            ms.append(e0.elapsed_time(e1))
        out[f"degrees_{name}_ms"] = min(ms)
        if ref is None:
            ref = deg
        else:
            out["degrees_identical"] = out["degrees_identical"] and bool(torch.equal(deg, ref))
        del plan
    return out


def bench_two_pass(args, cg, torch, w, seed, dev, stream):
    """The count-then-replay path on the same workload: S, plan + count pass,
    write pass (replay with the same random words) into the output."""
    edges = None
    plan = None
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    write_ms, count_ms = [], []
    reps = max(2, args.steps // 2)
    total = 0
    for it in range(reps + 1):
        if it == 1:
            torch.cuda.synchronize()
            t0 = time.perf_counter()
        S = cg.cl_weight_sum(w)
        plan = cg.cl_count([cg.Task(w, S, seed)], ws=plan.ws if plan is not None else None)
        m = plan.total
        if edges is None:
            edges = torch.empty((int(m * 1.02) + 1024, 2), dtype=torch.int32, device=dev)
        ev0.record(stream)
        cg.cl_generate(plan, edges=edges, cap=m)
        ev1.record(stream)
        ev1.synchronize()
        if it >= 1:
            total += m
            write_ms.append(ev0.elapsed_time(ev1))
            count_ms.append(cg.cl_plan_info(plan)["lane_kernel_ms"])
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    return {"edges_per_s": total / el, "ms_per_step": el / reps * 1e3,
            "count_kernel_ms": sum(count_ms) / len(count_ms), "write_kernel_ms": sum(write_ms) / len(write_ms)}


def bench_batched(args, cg, W, torch, np, dev):
    """256 uneven graphs: one captured HIP graph (whole path, no host sync)
    vs 256 separate count + write calls, identical output checked by digest."""
    log("bench: generating the 256-graph batch")
    batch = W.config_batch()
    tasks = []
    for w_np, sd in batch:
        wd = torch.from_numpy(w_np).to(dev)
        tasks.append(cg.Task(wd, cg.cl_weight_sum(wd), sd))
    # plain: one task per call
    plans = [None] * len(tasks)
    bufs = [None] * len(tasks)
    acc_plain = torch.zeros(1, dtype=torch.int64, device=dev)

    def plain_pass(check=False):
        total = 0
        base = 0
        for i, t in enumerate(tasks):
            p = cg.cl_sample([t], ws=plans[i].ws if plans[i] is not None else None)
            plans[i] = p
            mi = p.total
            if bufs[i] is None or bufs[i].shape[0] < mi:
                bufs[i] = torch.empty((mi + 64, 2), dtype=torch.int32, device=dev)
            cg.cl_generate(p, edges=bufs[i], cap=mi)
            if check:
                cg.cl_hash_edges(bufs[i][:mi], base, acc_plain)
            base += mi
            total += mi
        return total

    plain_pass()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.batched_reps):
        m_plain = plain_pass()
    torch.cuda.synchronize()
    t_plain = (time.perf_counter() - t0) / args.batched_reps
    acc_plain.zero_()
    plain_pass(check=True)

    plan = cg.cl_sample(tasks)
    s = torch.cuda.Stream()
    bg = cg.cl_batch_capture(plan, s, cap=plan.total)
    with torch.cuda.stream(s):
        bg.launch(s)
    s.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.batched_reps):
        bg.launch(s)
    s.synchronize()
    t_batch = (time.perf_counter() - t0) / args.batched_reps
    acc_b = torch.zeros(1, dtype=torch.int64, device=dev)
    with torch.cuda.stream(s):
        cg.cl_hash_edges(bg.edges[: plan.total], 0, acc_b, stream=s)
    s.synchronize()
    same = cg.hash_value(acc_b) == cg.hash_value(acc_plain) and plan.total == m_plain
    bg.close()
    return {
        "workload": "256 graphs, n log-uniform in [1e3,1e6], exponent U(2,3), mean degree U(4,64)",
        "edges": int(plan.total),
        "plain_edges_per_s": m_plain / t_plain,
        "batched_edges_per_s": plan.total / t_batch,
        "plain_ms": t_plain * 1e3,
        "batched_ms": t_batch * 1e3,
        "speedup": t_plain / t_batch,
        "identical_output": bool(same),
    }


def bench_cpu(w_np, seed):
    """The oracle (as it stands) on the first half of the sources by cost
    (uniform consecutive partition, P = 2, part 0): count + write passes."""
    import oracle as O
    S = O.exact_sum(w_np)
    bounds, _ = O.partition(w_np, S, 2)
    u1 = int(bounds[1])
    threads = max(1, min(16, os.cpu_count() or 1))
    log(f"bench: cpu oracle on sources [0, {u1}) with {threads} threads")
    t0 = time.perf_counter()
    _, m, _, _ = O.generate(w_np, S, seed, 0, u1, want_edges=True, nthreads=threads)
    dt = time.perf_counter() - t0
    return {"value": m / dt, "unit": "edges/s", "cores": threads, "kind": "oracle",
            "sample": f"sources [0, {u1}) of the n=1e7 workload (first of 2 equal-cost partitions), "
                      f"{m} edges, {dt:.1f} s"}


if __name__ == "__main__":
    main()
