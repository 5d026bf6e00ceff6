#!/usr/bin/env python3
"""Writes the stored expected values of the full-size parity tests.

Calls only the oracle (``oracle/``) on inputs from the seeded generators
(``workloads.py``); nothing here touches the GPU path.

* ``batch_256.json``: for each of the 256 uneven graphs of the batched
  workload (n log-uniform in [1e3, 1e6], exponent U(2, 3), mean degree
  U(4, 64), Philox seed g + 1): the exact sum S, the edge count m and the
  position-keyed digest of the graph's own edge list (positions counted from
  the graph's first edge), i.e. Create-Edges(w_g, S_g, [0, n_g)) of Sec. 3,
  Alg. 1 under the fixed sampling rule.
* ``share_part0.json``: part 0 of the uniform consecutive partition into 64
  parts (Sec. 4, Eq. 5) of the n = 1e9 power-law graph (exponent 2.1, mean
  degree 500, weight seed 3, Philox seed 3): S, the partition bounds' first
  entries, the total cost Z, and m, digest and visited candidates of the
  part's edge list (positions counted from the part's first edge).

Usage: python tests/golden/make_golden.py [batch] [share]
"""
import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import oracle as O  # noqa: E402
from paper_1406_1215_amd import workloads as W  # noqa: E402


def _write(name, obj):
    path = os.path.join(HERE, name)
    # one line per top-level key (and per graph), so that the file diffs well
    lines = []
    for k, v in obj.items():
        if isinstance(v, list) and v and isinstance(v[0], dict):
            body = ",\n".join("  " + json.dumps(x) for x in v)
            lines.append(f" {json.dumps(k)}: [\n{body}\n ]")
        else:
            lines.append(f" {json.dumps(k)}: {json.dumps(v)}")
    with open(path + ".tmp", "w") as f:
        f.write("{\n" + ",\n".join(lines) + "\n}\n")
    os.replace(path + ".tmp", path)
    print(f"wrote {path}", flush=True)


def batch():
    t0 = time.time()
    graphs = []
    total = 0
    for g, (w, seed) in enumerate(W.config_batch()):
        S = O.exact_sum(w)
        _, m, digest, cand = O.generate(w, S, seed, want_edges=False)
        graphs.append({"g": g, "n": int(w.size), "seed": int(seed), "S": S.hex(), "m": int(m),
                       "digest": int(digest), "candidates": int(cand)})
        total += m
    _write("batch_256.json", {
        "workload": "256 graphs, n log-uniform in [1e3,1e6], exponent U(2,3), mean degree U(4,64), "
                    "shape seed 4, Philox seed g+1",
        "digest_rule": "sum over the graph's edges i of mix(mix(i) ^ (u_i 2^32 + v_i)) mod 2^64, i from 0 per graph",
        "total_edges": int(total), "graphs": graphs})
    print(f"batch: {total} edges in {time.time() - t0:.0f} s", flush=True)


def share():
    t0 = time.time()
    w = W.config_share()
    print(f"share: weights in {time.time() - t0:.0f} s", flush=True)
    S = O.exact_sum(w)
    P = 64
    bounds, Z = O.partition(w, S, P)
    u1 = int(bounds[1])
    print(f"share: S = {S!r}, part 0 = [0, {u1}), Z = {Z} ({time.time() - t0:.0f} s)", flush=True)
    _, m, digest, cand = O.generate(w, S, 3, 0, u1, want_edges=False)
    _write("share_part0.json", {
        "workload": "n=1e9 power law, exponent 2.1, mean degree 500, cap sqrt(500 n), weight seed 3, "
                    "Philox seed 3; part 0 of the 64-part uniform consecutive partition",
        "digest_rule": "sum over the part's edges i of mix(mix(i) ^ (u_i 2^32 + v_i)) mod 2^64, i from 0",
        "n": int(w.size), "S": S.hex(), "P": P, "bounds_head": [int(x) for x in bounds[:4]], "Z": int(Z),
        "u_begin": 0, "u_end": u1, "m": int(m), "digest": int(digest), "candidates": int(cand)})
    print(f"share: {m} edges, {time.time() - t0:.0f} s", flush=True)


if __name__ == "__main__":
    which = sys.argv[1:] or ["batch", "share"]
    for name in which:
        {"batch": batch, "share": share}[name]()
