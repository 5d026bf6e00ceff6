#!/usr/bin/env python3
"""Throughput of the Chung-Lu generation path on one MI355X.

A step is one pass of the whole generation path over the n = 1e7 power-law
workload (exponent 2.1, w_min = 10, weights capped at sqrt(S), Philox seed 2),
inputs resident in HBM: exact sum S, plan (validation, quantised prefix,
segments, lane plan), one pass of every lane into its slot (counting and
writing), offsets, compaction of the slots into the contiguous edge list
(after the first step, which allocates the output, plan + one pass +
compaction are one call, cl_sample_into).  The schedule (lane budget, the
Eq. 5 chunk size, and the persistent grid) is the autotuner's choice for
this output size, tuned at the start when its cache has none
(config.tuning).  `value` is edges generated per second.  Printed as one
JSON line, with:

* roofline: the one-pass generation kernel (Alg. 1 per lane, edges staged
  into 64-byte chunks of per-lane slots), timed with HIP events on its stream.
  Every visited candidate reads one weight w_v at an essentially random
  position (8 algorithmic bytes, one 128-byte line from HBM or the Infinity
  Cache on an L2 miss) and every kept edge writes a 4-byte slot word (v; a
  mark and u are added where the source changes).  achieved = (8 B x
  candidates + 4 B x slot words) / launch time against 8 TB/s; traffic = the
  kernel's measured HBM bytes (FETCH_SIZE + WRITE_SIZE, scaled by a copy of
  known size) from the committed counter summary when it was taken on the
  current kernel source; ceilings = the same number of 8-byte gathers from
  the same array alone (uniform positions, and positions drawn with the
  candidates' density) and plain stores, measured in the same run
  (libclceil.so), with the kernel's fraction of each;
* alu_view: VALU wave-instructions of that kernel from the committed counter
  summary against the issue capacity, and the counters' busy fraction;
* hbm_write: bytes written per second by that kernel (slot words) and moved
  by the compaction (slot words read, 8-byte edges written), against 8 TB/s;
* two_pass: the count-then-replay path (count pass, offsets, write pass);
* csr: the same plan written as compressed sparse rows (4-byte targets and
  row offsets) instead of (u, v) pairs;
* partition_ablation: generation-kernel time with work units of equal
  expected cost (Eq. 5) vs units of equal source counts (Sec. 4's naive
  consecutive partition), same number of units; the degree kernel under
  those two and round-robin units (Sec. 4's RRP); and per-unit statistics
  of each (unit time against plan cost, wavefront balance);
* expected_degree: the float32 tiled expected-degree kernel and its adjoint
  on n = 1e5 (1e10 pairs), default and autotuned tile shape, against the
  VALU lane-operation peak, with their errors against a float64 evaluation;
* calibration: 200 Adam steps on log w against n = 1e5 capped targets, then
  generation from the calibrated weights;
* batched: 256 uneven graphs in one captured HIP graph (default and
  autotuned schedule) vs 256 plain calls;
* share: part 0 of 64 of the n = 1e9 graph (the paper's largest PL shape),
  one pass and 4 output slabs through one buffer, digest checked against
  the oracle's stored value;
* cpu_baseline: the CPU oracle on bounded samples of the same workload, on
  the process's CPU share and single-threaded, with the host's CPU model;
* inflight: the same steps with two in flight (two host threads, streams,
  workspaces and output buffers), whole-job edges per second; `value` stays
  the one-at-a-time figure.
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
# wave64 VALU instructions per second: 256 CUs x 4 SIMDs x 2.4 GHz / 4 cycles
VALU_ISSUE_PER_S = 256 * 4 * 2.4e9 / 4
BYTES_PER_CANDIDATE = 8           # w_v gathered
BYTES_PER_SLOT_WORD = 4           # slot words written: v per edge, (mark, u) per change of source
BYTES_PER_EDGE = 8                # (u, v) uint32 pair of the edge list
HBM_PEAK = 8.0e12                 # bytes/s
METRIC = "edges/sec generated on 1 MI355X + % HBM write roofline; batched vs plain"
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_generation_plain_1e7.json")
SHARE_TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_generation_share_part0.json")
VALU_FILE = os.path.join(ROOT, "profiles", "valu_generation_plain_1e7.json")
KERNEL_SOURCES = ["cl_device.hpp", "cl_kernels.hpp", "cl_plan.hpp", "cl_order.hpp"]


def kernel_hash() -> str:
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, "paper_1406_1215_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def expdeg_hash() -> str:
    h = hashlib.sha256()
    with open(os.path.join(ROOT, "paper_1406_1215_amd", "csrc", "cl_expdeg.hpp"), "rb") as fh:
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
    ap.add_argument("--no-ceilings", action="store_true")
    ap.add_argument("--no-order-ablation", action="store_true",
                    help="skip the index-order runs of the generation kernel (profiles of the default order)")
    ap.add_argument("--no-share", action="store_true")
    ap.add_argument("--batched-only", action="store_true",
                    help="only the 256-graph batch: the captured launch against 256 separate calls")
    ap.add_argument("--share-only", action="store_true",
                    help="only the leg of part 0 of the n=1e9 graph (for profiling that launch)")
    ap.add_argument("--no-tune", action="store_true", help="batched leg at the default schedule only")
    ap.add_argument("--inflight", type=int, default=2,
                    help="also time the same steps with this many in flight (one host thread, stream, "
                         "workspace and output buffer each); 1 = not at all")
    ap.add_argument("--no-expdeg-ref", action="store_true",
                    help="expected-degree leg without the float64 reference (for counter passes)")
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
    if args.batched_only:
        print(json.dumps(bench_batched(args, cg, W, torch, np, dev)), flush=True)
        return
    if args.share_only:
        out = bench_share(args, cg, W, torch, np, dev)
        if args.copy_calibration:
            out["copy_calibration_bytes"] = copy_calibration(torch, dev)
        print(json.dumps(out), flush=True)
        return

    log("bench: generating the n=1e7 workload")
    w_np = W.config_plain(n=args.n)
    w = torch.from_numpy(w_np).to(dev)
    seed = 2

    # the schedule (lane budget = the Eq. 5 chunk size, persistent grid): the
    # autotuner's cached choice for this output size, tuned here once (plan +
    # one pass + expansion per setting, digest checked) when it has none
    from paper_1406_1215_amd import autotune
    S0 = cg.cl_weight_sum(w)
    E0, _ = cg.cl_expected_edges(w, S0)
    tuning = autotune.lookup(E0)
    tune_s = 0.0
    if tuning is None and not args.no_tune:
        log("bench: tuning the plain step")
        t0 = time.perf_counter()
        tuning = autotune.tune([cg.Task(w, S0, seed)], planner="cl_sample", reps=4)["best"]
        tune_s = time.perf_counter() - t0
        torch.cuda.empty_cache()

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
            plan, fits = cg.cl_sample_into([cg.Task(w, S, seed)], edges, ws=plan.ws, tuning=tuning)
            if fits:
                return plan.total
        plan = cg.cl_sample([cg.Task(w, S, seed)], ws=plan.ws if plan is not None else None, tuning=tuning)
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
    inflight = None
    if args.inflight > 1:
        inflight = bench_inflight(args, cg, torch, w, seed, dev, tuning)
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
                   "heavy_segments": info["heavy_segments"], "path": "one pass into slots + compaction",
                   "tuning": tuning, "tuning_seconds": tune_s},
        "roofline": {
            "kernel": "one-pass generation (k_lanes<2>)",
            "bound": "hbm",
            "limiter": "memory side: random 8-byte gathers of w_v, one 128-byte line per L2 miss, served mostly "
                       "by the Infinity Cache; the rate of L2 line requests binds (see ceilings)",
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
        "alu_view": alu_view(cand, t_gen),
        "hbm_write": {
            "generation_GBps": 4.0 * words / t_gen / 1e9,
            "generation_frac_of_8TBps": 4.0 * words / t_gen / HBM_PEAK,
            "compaction_ms": t_copy * 1e3,
            "compaction_GBps_read_plus_write": (4.0 * words + 8.0 * m) / t_copy / 1e9,
            "whole_step_GBps": 8.0 * total_edges / elapsed / 1e9,
            "whole_step_frac_of_8TBps": 8.0 * total_edges / elapsed / HBM_PEAK,
        },
    }
    if inflight is not None:
        result["inflight"] = inflight
    if not args.no_order_ablation:
        result["unit_order"] = bench_unit_order(cg, w, seed, tuning, t_gen)
    if not args.no_ceilings:
        log("bench: memory ceilings")
        result["roofline"]["ceilings"] = bench_ceilings(cg, torch, w, float(cg.cl_weight_sum(w)), cand, words, t_gen)
    if not args.no_two_pass:
        result["two_pass"] = bench_two_pass(args, cg, torch, w, seed, dev, stream)
    if not args.no_csr:
        result["csr"] = bench_csr(cg, torch, w, seed, plan, t_copy)

    if not args.no_ablation:
        result["partition_ablation"] = bench_partition(cg, torch, np, w, seed)

    if not args.no_expdeg:
        result["expected_degree"] = bench_expdeg(cg, W, torch, dev, ref=not args.no_expdeg_ref,
                                                 tune=not args.no_tune)
    if not args.no_calib:
        result["calibration"] = bench_calibration(cg, W, torch, dev)

    if not args.no_batched:
        result["batched"] = bench_batched(args, cg, W, torch, np, dev)

    if args.copy_calibration:
        result["copy_calibration_bytes"] = copy_calibration(torch, dev)

    if not args.no_share:
        edges = None
        plan = None
        torch.cuda.empty_cache()
        result["share"] = bench_share(args, cg, W, torch, np, dev)

    if not args.no_cpu:
        result["cpu_baseline"] = bench_cpu(w_np, seed)

    print(json.dumps(result), flush=True)


def bench_inflight(args, cg, torch, w, seed, dev, tuning=None):
    """The same step (exact S, then plan + one pass + compaction in one
    cl_sample_into call) with several steps in flight: one host thread per
    pipeline, each with its own stream, workspaces and output buffer, the
    steps dealt round robin; the library's host calls release the
    interpreter while they wait, so the GPU runs one pipeline's plan and
    compaction beside another's generation.  Whole-job edges per second."""
    import threading
    k = args.inflight
    pipes = []
    for _ in range(k):
        st = torch.cuda.Stream()
        with torch.cuda.stream(st):
            S = cg.cl_weight_sum(w)
            plan = cg.cl_sample([cg.Task(w, S, seed)], tuning=tuning)
            edges = torch.empty((int(plan.total * 1.02) + 1024, 2), dtype=torch.int32, device=dev)
            sws = torch.empty(cg.cl_weight_sum_workspace(w.numel()), dtype=torch.uint8, device=dev)
        pipes.append({"stream": st, "plan": plan, "edges": edges, "sws": sws, "m": 0})

    def run(p, nsteps):
        with torch.cuda.stream(p["stream"]):
            for _ in range(nsteps):
                S = cg.cl_weight_sum(w, ws=p["sws"])
                plan, fits = cg.cl_sample_into([cg.Task(w, S, seed)], p["edges"], ws=p["plan"].ws, tuning=tuning)
                assert fits
                p["plan"] = plan
                p["m"] += plan.total

    def round_(nsteps_total):
        per = [nsteps_total // k + (1 if i < nsteps_total % k else 0) for i in range(k)]
        th = [threading.Thread(target=run, args=(p, n)) for p, n in zip(pipes, per)]
        for t in th:
            t.start()
        for t in th:
            t.join()

    round_(max(args.warmup, k))
    for p in pipes:
        p["m"] = 0
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    round_(args.steps)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    m = sum(p["m"] for p in pipes)
    return {"inflight": k, "steps": args.steps, "edges": m, "edges_per_s": m / el, "ms_per_step": el / args.steps * 1e3}


def copy_calibration(torch, dev):
    """A plain device copy of 2 GiB whose source is not in any cache (a
    2 GiB fill of another buffer runs in between): its FETCH_SIZE and
    WRITE_SIZE read 2 GiB each when the counters are exact, which scales the
    counters of the other kernels of the same run."""
    n8 = 1 << 28
    x = torch.empty(n8, dtype=torch.float64, device=dev)
    y = torch.empty_like(x)
    z = torch.empty_like(x)
    x.fill_(1.0)
    z.fill_(2.0)
    torch.cuda.synchronize()
    y.copy_(x)
    torch.cuda.synchronize()
    del x, y, z
    return n8 * 8


def alu_view(cand, t_gen):
    """The generation kernel against the vector ALU.  From the committed
    rocprofv3 counter summary (taken on the current kernel source): VALU
    wave-instructions per launch against the issue capacity of 256 CUs x 4
    SIMDs, one wave64 instruction per 4 cycles each (16 lanes per SIMD: the
    rate of float64 and of unpacked float32 operations) at 2.4 GHz, and the
    counters' own busy fraction.  Without it, only the operation count of
    one candidate step against the lane-operation peak."""
    out = {"ops_per_candidate_estimate": OPS_PER_CANDIDATE,
           "frac_estimate": cand * OPS_PER_CANDIDATE / t_gen / PEAK_LANE_OPS}
    vc = valu_counters()
    if vc:
        insts = vc["valu_insts_per_launch"]
        cap = VALU_ISSUE_PER_S
        out.update({"source": os.path.relpath(VALU_FILE, ROOT),
                    "valu_insts_per_launch": insts,
                    "valu_insts_per_candidate": insts / max(cand, 1),
                    "lane_ops_per_candidate": 64.0 * insts / max(cand, 1),
                    "achieved": insts / t_gen / 1e9, "peak": cap / 1e9, "unit": "G wave-instructions/s",
                    "frac": insts / t_gen / cap})
        for k in ("valu_busy", "f64_share_of_valu"):
            if k in vc:
                out[k] = vc[k]
    return out


def candidate_density(torch, w, S):
    """Expected candidate visits at each position v of a sorted weight
    vector: sum over the sources u < v of min(w_u w_v / S, 1) (the visits of
    kept edges; the rejected ones follow the same shape).  With w sorted,
    the capped sources of v are a prefix u < J_v, J_v = #{u < v : w_u w_v >=
    S}, so visits(v) = J_v + (w_v / S) (sum of w_u over J_v <= u < v)."""
    n = w.numel()
    P = torch.cumsum(w, 0)
    Pex = P - w
    thr = torch.where(w > 0, S / w, torch.full_like(w, float("inf")))
    J = torch.searchsorted(-w, -thr, right=True)             # #{u : w_u >= S / w_v}
    J = torch.minimum(J, torch.arange(n, device=w.device))
    PJ = torch.where(J > 0, P[(J - 1).clamp(min=0)], torch.zeros_like(w))
    return J.to(torch.float64) + (w / S) * (Pex - PJ)


def draw_positions(torch, density, count, seed, chunk=1 << 25):
    """count positions drawn independently with probability proportional to
    density (inverse CDF), as int32."""
    cdf = torch.cumsum(density, 0)
    total = float(cdf[-1])
    g = torch.Generator(device=density.device)
    g.manual_seed(seed)
    out = torch.empty(count, dtype=torch.int32, device=density.device)
    for lo in range(0, count, chunk):
        hi = min(count, lo + chunk)
        r = torch.rand(hi - lo, dtype=torch.float64, device=density.device, generator=g) * total
        out[lo:hi] = torch.searchsorted(cdf, r).clamp(max=density.numel() - 1).to(torch.int32)
    return out


def _time_ms(torch, fn, reps=3):
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    fn()
    best = float("inf")
    for _ in range(reps):
        e0.record()
        fn()
        e1.record()
        e1.synchronize()
        best = min(best, e0.elapsed_time(e1))
    return best


def lane_ms_of(cg, task, tuning, reps, ws=None):
    """Lane-kernel times (HIP events, ms) of `reps` one-pass plans of one task."""
    out = []
    for _ in range(reps):
        p = cg.cl_sample([task], tuning=tuning, ws=ws)
        out.append(cg.cl_plan_info(p)["lane_kernel_ms"])
        ws = p.ws
    return out


def bench_unit_order(cg, w, seed, tuning, t_gen):
    """The generation kernel with its units taken in index order against the
    default for one graph, by the position of their first candidate (the same
    plan otherwise; the output is the same)."""
    S = cg.cl_weight_sum(w)
    idx = lane_ms_of(cg, cg.Task(w, S, seed), dict(tuning or {}, unit_order=1), 4)
    pos_ms = t_gen * 1e3
    return {"default": "by position (single graph)", "position_ms": pos_ms, "index_ms": sum(idx) / len(idx),
            "index_over_position": sum(idx) / len(idx) / pos_ms}


def bench_ceilings(cg, torch, w, S, cand, words, t_gen):
    """Measured ceilings for the generation kernel (libclceil.so), on the same
    device and weight array: `cand` 8-byte loads at uniform random positions,
    the same number at positions drawn with the candidates' density
    (candidate_density), the same positions on half the bytes per weight
    (the footprint of a float32 copy) and the same positions visited band by
    band (32 bands of v), and plain 16-byte stores; each the best over a few
    grid sizes.  The kernel's fractions: ceiling time of its gathers (and of
    its slot-word stores) over its own time."""
    from paper_1406_1215_amd import ceilings as C
    cus = int(cg.lib().cl_device_cus()) or 256
    grids = [cus * k for k in (4, 8, 16)]
    out = C.out_buffer(max(grids), w.device)
    t_uni = min(_time_ms(torch, lambda b=b: C.gather_uniform(w, cand, 12345, b, out)) for b in grids)
    idx = draw_positions(torch, candidate_density(torch, w, S), cand, 6789)
    t_wgt = min(_time_ms(torch, lambda b=b: C.gather_list(w, idx, b, out)) for b in grids)
    # the same positions on an array of half the bytes per weight (float32):
    # load 8 bytes at position idx // 2, so that every line holds the weights
    # of twice as many candidate positions
    # the same positions visited band by band (32 bands of v, the order inside
    # a band unchanged): the gathers of a traversal that keeps the whole chip
    # in one band of w at a time
    band = (idx.to(torch.int64) * 32) // w.numel()
    banded = idx[torch.sort(band, stable=True).indices].contiguous()
    del band
    t_band = min(_time_ms(torch, lambda b=b: C.gather_list(w, banded, b, out)) for b in grids)
    del banded
    idx.floor_divide_(2)
    t_half = min(_time_ms(torch, lambda b=b: C.gather_list(w, idx, b, out)) for b in grids)
    del idx
    sbytes = 4 << 30
    buf = torch.empty(sbytes, dtype=torch.uint8, device=w.device)
    t_st = min(_time_ms(torch, lambda b=b: C.store(buf, b)) for b in grids)
    del buf
    store_bw = sbytes / (t_st * 1e-3)
    t_words = BYTES_PER_SLOT_WORD * words / store_bw
    return {
        "loads": int(cand),
        "gather_uniform_ms": t_uni,
        "gather_uniform_loads_per_s": cand / (t_uni * 1e-3),
        "gather_candidate_density_ms": t_wgt,
        "gather_candidate_density_loads_per_s": cand / (t_wgt * 1e-3),
        "gather_candidate_density_half_footprint_ms": t_half,
        "gather_candidate_density_32_bands_ms": t_band,
        "store_GBps": store_bw / 1e9,
        "store_frac_of_8TBps": store_bw / HBM_PEAK,
        "kernel_frac_of_gather_uniform": t_uni * 1e-3 / t_gen,
        "kernel_frac_of_gather_candidate_density": t_wgt * 1e-3 / t_gen,
        "kernel_write_frac_of_store": t_words / t_gen,
        "kernel_frac_of_memory_ceiling": (t_wgt * 1e-3 + t_words) / t_gen,
    }


def valu_counters():
    """VALU counters of the generation kernel from the committed rocprofv3
    summary, if it was taken on the current kernel source."""
    try:
        with open(VALU_FILE) as f:
            t = json.load(f)
    except (OSError, ValueError):
        return None
    if t.get("kernel_hash") != kernel_hash():
        return None
    return t


def bench_share(args, cg, W, torch, np, dev):
    """One GPU's share of the paper's largest PL shape: n = 1e9 weights
    (exponent 2.1, mean degree 500, cap sqrt(500 n), weight seed 3), exact S,
    the uniform consecutive partition into 64 parts (Eq. 5), part 0 (the
    heavy head) generated with Philox seed 3 in one pass and written out in 4
    slabs through one reused buffer.  Timed: plan + one pass + the 4 slab
    expansions (the digest of each slab, standing in for the I/O the paper
    leaves out, is outside the timed region).  The part's digest is compared
    with the stored value of the oracle (tests/golden/share_part0.json)."""
    log("bench: generating the n=1e9 weights")
    w_np = W.config_share()
    w = torch.from_numpy(w_np).to(dev)
    del w_np
    S = cg.cl_weight_sum(w)
    P = 64
    bounds, Z = cg.cl_partition(w, S, P)
    u1 = bounds[1]
    seed = 3
    task = [cg.Task(w, S, seed, 0, u1)]
    plan = cg.cl_sample(task)
    m = plan.total
    slab = (m + 3) // 4
    buf = torch.empty((slab + 8, 2), dtype=torch.int32, device=dev)
    acc = torch.zeros(1, dtype=torch.int64, device=dev)

    def run(digest=False):
        p = cg.cl_sample(task, ws=plan.ws)
        for k in range(4):
            b0 = k * slab
            c = min(slab, m - b0)
            cg.cl_generate(p, edges=buf, edge_begin=b0, cap=c)
            if digest:
                cg.cl_hash_edges(buf[:c], b0, acc)
        return p

    run()
    torch.cuda.synchronize()
    reps = 3
    t0 = time.perf_counter()
    for _ in range(reps):
        p = run()
    torch.cuda.synchronize()
    el = (time.perf_counter() - t0) / reps
    info = cg.cl_plan_info(p)
    lane_ms = info["lane_kernel_ms"]
    order = None
    if not args.no_order_ablation:
        pos_ms = lane_ms_of(cg, task[0], None, 2, ws=plan.ws)
        idx_ms = lane_ms_of(cg, task[0], {"unit_order": 1}, 2, ws=plan.ws)
        order = {"default": "by position (single graph)", "position_ms": sum(pos_ms) / len(pos_ms),
                 "index_ms": sum(idx_ms) / len(idx_ms), "index_over_position": sum(idx_ms) / sum(pos_ms)}
    acc.zero_()
    run(digest=True)
    digest = cg.hash_value(acc)
    gold = None
    try:
        with open(os.path.join(ROOT, "tests", "golden", "share_part0.json")) as f:
            gold = json.load(f)
    except (OSError, ValueError):
        pass
    cand, words = info["candidates"], info["slot_words"]
    alg = BYTES_PER_CANDIDATE * cand + BYTES_PER_SLOT_WORD * words
    out = {
        "workload": "n=1e9 power law, exponent 2.1, mean degree 500, cap sqrt(500 n), weight seed 3; part 0 of 64 "
                    "(uniform consecutive partition, Eq. 5), Philox seed 3, 4 slabs through one buffer",
        "sources": int(u1), "edges": int(m), "candidates": int(cand), "lanes": info["lanes"],
        "seconds": el, "edges_per_s": m / el,
        "lane_kernel_ms": lane_ms,
        "unit_order": order,
        "roofline": {"kernel": "one-pass generation (k_lanes<2>)", "bound": "hbm",
                     "achieved": alg / (lane_ms * 1e-3) / 1e9, "peak": HBM_PEAK / 1e9, "unit": "GB/s",
                     "frac": alg / (lane_ms * 1e-3) / HBM_PEAK, "algorithmic_bytes_per_launch": int(alg),
                     "traffic": share_traffic()},
        "digest": digest,
        "digest_matches_oracle": (gold is not None and digest == gold["digest"] and m == gold["m"]),
    }
    del plan, p, buf, w
    torch.cuda.empty_cache()
    return out


def share_traffic():
    try:
        with open(SHARE_TRAFFIC_FILE) as f:
            t = json.load(f)
    except (OSError, ValueError):
        return None
    if t.get("kernel_hash") != kernel_hash():
        return None
    return t.get("bytes_per_launch")


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


def expdeg_reference(torch, w32, S, g, block=512):
    """Float64 expected degrees and their gradient (S = sum of the weights,
    so dS/dw_k = 1) by the definition, over all pairs in blocks of rows on
    the GPU with plain torch float64 operations (no part of the kernels):
    d_i = sum_{j != i} min(x_ij, 1), x_ij = w_i w_j / S, and
    grad_k = (g_k A_k + B_k - T) / S with A_k = sum_{j != k, x_kj < 1} w_j,
    B_k = sum_{j != k, x_kj < 1} g_j w_j, T = sum_i g_i sum_{j != i, x_ij < 1} x_ij."""
    w = w32.double()
    n = w.numel()
    d = torch.empty(n, dtype=torch.float64, device=w.device)
    A = torch.empty_like(d)
    B = torch.empty_like(d)
    U = torch.empty_like(d)
    gw = g * w
    for lo in range(0, n, block):
        hi = min(n, lo + block)
        X = w[lo:hi, None] * w[None, :] / S
        r = torch.arange(hi - lo, device=w.device)
        X[r, r + lo] = 0.0
        d[lo:hi] = torch.clamp(X, max=1.0).sum(1)
        M = (X < 1.0).double()
        M[r, r + lo] = 0.0
        A[lo:hi] = M @ w
        B[lo:hi] = M @ gw
        U[lo:hi] = (M * X).sum(1)
    T = float(g @ U)
    return d, (g * A + B - T) / S


def bench_expdeg(cg, W, torch, dev, reps=5, ref=True, tune=True):
    """Expected degree d_i = sum_{j != i} min(w_i w_j / S, 1) and its adjoint
    on n = 1e5 float32 weights (1e10 pairs each), timed with events, at the
    default tile shape and at the autotuner's (tuned here once when its
    cache has none); ALU work 2 lane-operations per pair forward (the
    multiply with the clamp modifier, the add) and 3 backward (the clamped
    multiply-add that forms the mask, and one multiply-add for each of the
    two sums; FMA-class, so at most half of the lane-operation peak without
    packed math).  The errors of both
    against the float64 definition (expdeg_reference): maximum relative
    error of d, normwise relative error of the gradient."""
    from paper_1406_1215_amd import autotune
    t = W.config_calib()
    w32 = torch.from_numpy(t.astype("float32")).to(dev)
    S = float(w32.double().sum().item())
    n = w32.numel()
    g = torch.randn(n, dtype=torch.float64, device=dev, generator=torch.Generator(device=dev).manual_seed(17))
    ws = cg._ed_ws(n, dev)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    out = {"n": n, "pairs": n * n}

    def timed(fn):
        fn()
        torch.cuda.synchronize()
        e0.record()
        for _ in range(reps):
            fn()
        e1.record()
        e1.synchronize()
        return e0.elapsed_time(e1) / reps

    tuned = autotune.lookup(float(n) * n, kind="expdeg")
    if tuned is None and tune:
        log("bench: tuning the expected-degree tile shape")
        tuned = autotune.tune_expdeg(w32, S, reps=2)["best"]
    shapes = [("default", None)] + ([("tuned", tuned)] if tuned is not None else [])
    for label, sh in shapes:
        for name, fn, ops in (("forward", lambda: cg.cl_expected_degree(w32, S, ws=ws, tuning=sh), 2),
                              ("backward", lambda: cg.cl_expected_degree_backward(w32, S, g, True, ws=ws,
                                                                                  tuning=sh), 3)):
            ms = timed(fn)
            key = name if label == "default" else f"{name}_tuned"
            out[f"{key}_ms"] = ms
            out[f"{key}_pairs_per_s"] = n * n / (ms * 1e-3)
            out[f"{key}_alu_frac"] = n * n * ops / (ms * 1e-3) / PEAK_LANE_OPS
    out["tile_shape_tuned"] = tuned
    # the tile kernels against the vector ALU from the committed counter
    # summary (default tile shape, same kernel source): VALU wave-instructions
    # per 64 pairs and rocprofv3's VALUBusy
    vc = valu_counters()
    if vc and vc.get("expdeg_hash") == expdeg_hash():
        for name, key in (("forward", "expdeg_forward_tile"), ("backward", "expdeg_adjoint_tile")):
            c = vc.get(key)
            if c:
                out[f"{name}_valu_insts_per_64_pairs"] = c["counters"]["SQ_INSTS_VALU"] / (n * n / 64.0)
                out[f"{name}_valu_busy"] = c["valu_busy"]
    if not ref:
        return out
    d = cg.cl_expected_degree(w32, S, ws=ws, tuning=tuned)
    gr = cg.cl_expected_degree_backward(w32, S, g, True, ws=ws, tuning=tuned).double()
    d_ref, gr_ref = expdeg_reference(torch, w32, S, g)
    out["forward_max_rel_err_vs_f64"] = float((torch.abs(d - d_ref) / d_ref).max())
    out["backward_normwise_rel_err_vs_f64"] = float(torch.linalg.norm(gr - gr_ref) / torch.linalg.norm(gr_ref))
    out["backward_max_abs_err_over_max_abs"] = float(torch.abs(gr - gr_ref).max() / torch.abs(gr_ref).max())
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


def bench_partition(cg, torch, np, w, seed):
    """Sec. 4's comparison on one GPU: work units of equal expected cost
    (Eq. 5 applied to lanes) vs units of equal numbers of sources, same unit
    count; generation-kernel time of each (same output).  Then the degree
    kernel under those two and round-robin units (RRP over segments), timed
    with events around cl_degrees (which includes one small header read),
    and for each policy a statistics pass (unit_summary): unit time against
    plan cost and the balance of the wavefronts."""
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
        # per-unit times of a statistics pass (a count pass that records each
        # unit's wave clock, plan cost and candidates)
        out[f"units_{name}"] = unit_summary(cg.cl_unit_stats(plan), np)
        del plan
    return out


def unit_summary(st, np):
    """Sec. 4's quantities from one statistics pass: unit run time against
    plan cost and visited candidates (Pearson correlation, least-squares
    time per cost unit), and the balance of the wavefronts: each one's span
    from its first unit taken to its last unit finished, mean and maximum,
    and the whole pass's span."""
    t0 = st["t0"].astype(np.float64)
    t1 = st["t1"].astype(np.float64)
    cost = st["cost"].astype(np.float64)
    vis = st["visits"].astype(np.float64)
    work = cost > 0
    tau = (t1 - t0) / 100.0            # microseconds (100 MHz clock)
    out = {"units": int(work.sum())}
    if work.sum() > 2:
        c, v, t = cost[work], vis[work], tau[work]
        out["corr_time_cost"] = float(np.corrcoef(t, c)[0, 1])
        out["corr_time_candidates"] = float(np.corrcoef(t, v)[0, 1])
        out["us_per_expected_candidate"] = float((t @ c) / (c @ c)) * 16.0
        out["unit_us_mean"] = float(t.mean())
        out["unit_us_max"] = float(t.max())
        out["cost_max_over_mean"] = float(c.max() / c.mean())
    wave = (st["lane"] // 64).astype(np.int64)
    _, inv = np.unique(wave, return_inverse=True)
    w0 = np.full(inv.max() + 1, np.inf)
    w1 = np.zeros(inv.max() + 1)
    np.minimum.at(w0, inv, t0)
    np.maximum.at(w1, inv, t1)
    span = (w1 - w0) / 100.0
    out["waves"] = int(span.size)
    out["wave_span_us_mean"] = float(span.mean())
    out["wave_span_us_max"] = float(span.max())
    out["wave_span_max_over_mean"] = float(span.max() / span.mean())
    out["pass_span_us"] = float((t1.max() - t0.min()) / 100.0)
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
    vs 256 separate plain calls (cl_sample + cl_generate each), identical
    output checked by digest.  The captured batch runs at the default
    schedule and at the autotuner's choice (lane budget = chunk size of the
    Eq. 5 split, persistent grid), both reported."""
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

    # the captured batch, at the default schedule and at the autotuned one
    # (the tuner's cached choice for this output size, tuned here once when
    # the cache has none)
    from paper_1406_1215_amd import autotune
    tuned = autotune.lookup(m_plain, kind="batch")
    tune_s = 0.0
    if tuned is None and not args.no_tune:
        log("bench: tuning the batched launch")
        t0 = time.perf_counter()
        tuned = autotune.tune_batch(tasks)["best"]
        tune_s = time.perf_counter() - t0
    s = torch.cuda.Stream()
    times = {}
    same = True
    edges = None
    for name, tun in (("default", None), ("tuned", tuned)):
        if name == "tuned" and tun is None:
            continue
        plan = cg.cl_sample(tasks, tuning=tun)
        if edges is None:
            edges = torch.empty((plan.total + 1024, 2), dtype=torch.int32, device=dev)
        bg = cg.cl_batch_capture(plan, s, cap=plan.total, edges=edges)
        bg.launch(s)
        s.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.batched_reps):
            bg.launch(s)
        s.synchronize()
        times[name] = (time.perf_counter() - t0) / args.batched_reps
        acc_b = torch.zeros(1, dtype=torch.int64, device=dev)
        with torch.cuda.stream(s):
            cg.cl_hash_edges(edges[: plan.total], 0, acc_b, stream=s)
        s.synchronize()
        same = same and cg.hash_value(acc_b) == cg.hash_value(acc_plain) and plan.total == m_plain
        bg.close()
        del plan
    t_batch = times.get("tuned", times["default"])
    return {
        "workload": "256 graphs, n log-uniform in [1e3,1e6], exponent U(2,3), mean degree U(4,64)",
        "edges": int(m_plain),
        "plain_edges_per_s": m_plain / t_plain,
        "batched_edges_per_s": m_plain / t_batch,
        "plain_ms": t_plain * 1e3,
        "batched_ms": t_batch * 1e3,
        "batched_default_ms": times["default"] * 1e3,
        "batched_tuned_ms": times["tuned"] * 1e3 if "tuned" in times else None,
        "tuning": tuned,
        "tuning_seconds": tune_s,
        "speedup": t_plain / t_batch,
        "identical_output": bool(same),
    }


def cpu_info():
    """Host CPU: logical CPUs the OS reports, the CPUs this process may run
    on, and the model name."""
    model = ""
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        allowed = len(os.sched_getaffinity(0))
    except (AttributeError, OSError):
        allowed = os.cpu_count() or 1
    return {"nproc": os.cpu_count(), "allowed_cpus": allowed, "model": model}


def bench_cpu(w_np, seed):
    """The oracle (as it stands) on bounded samples of the same workload:
    with the process's CPU share (at most 16 threads, the host share of one
    GPU on this machine) the first half of the sources by cost (uniform
    consecutive partition, P = 2, part 0), and single-threaded the first
    sixteenth (P = 16, part 0); count + write passes, edges stored."""
    import oracle as O
    info = cpu_info()
    S = O.exact_sum(w_np)
    bounds, _ = O.partition(w_np, S, 2)
    u1 = int(bounds[1])
    threads = max(1, min(16, info["allowed_cpus"]))
    log(f"bench: cpu oracle on sources [0, {u1}) with {threads} threads")
    t0 = time.perf_counter()
    _, m, _, _ = O.generate(w_np, S, seed, 0, u1, want_edges=True, nthreads=threads)
    dt = time.perf_counter() - t0
    b16, _ = O.partition(w_np, S, 16)
    v1 = int(b16[1])
    log(f"bench: cpu oracle on sources [0, {v1}) with 1 thread")
    t0 = time.perf_counter()
    _, m1, _, _ = O.generate(w_np, S, seed, 0, v1, want_edges=True, nthreads=1)
    dt1 = time.perf_counter() - t0
    return {"value": m / dt, "unit": "edges/s", "cores": threads, "kind": "oracle",
            "sample": f"sources [0, {u1}) of the n=1e7 workload (first of 2 equal-cost partitions), "
                      f"{m} edges, {dt:.1f} s",
            "host": info,
            "single_thread": {"value": m1 / dt1, "unit": "edges/s", "cores": 1,
                              "sample": f"sources [0, {v1}) (first of 16 equal-cost partitions), {m1} edges, "
                                        f"{dt1:.1f} s"}}


if __name__ == "__main__":
    main()
