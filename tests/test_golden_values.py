"""The stored expected values of the full-size GPU tests agree with the
oracle as it stands: every graph of the 256-graph batch with fewer than
1e5 edges is regenerated here (S, m, digest, candidates), and the share's
stored values are checked for consistency (increasing bounds, the edge count
within Theorem 2's factor of the part's cost share).  The stored files are
written by tests/golden/make_golden.py, which calls only the oracle."""
import json
import os

import oracle as O
from paper_1406_1215_amd import workloads as W

HERE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def test_batch_golden_small_graphs_regenerate():
    with open(os.path.join(HERE, "batch_256.json")) as f:
        gold = json.load(f)
    assert len(gold["graphs"]) == 256
    assert sum(g["m"] for g in gold["graphs"]) == gold["total_edges"]
    checked = 0
    for (w, seed), g in zip(W.config_batch(), gold["graphs"]):
        assert w.size == g["n"] and seed == g["seed"]
        if g["m"] >= 100_000:
            continue
        S = O.exact_sum(w)
        assert S.hex() == g["S"]
        _, m, digest, cand = O.generate(w, S, seed, want_edges=False)
        assert (m, digest, cand) == (g["m"], g["digest"], g["candidates"]), g["g"]
        checked += 1
    assert checked >= 40


def test_share_golden_is_consistent():
    with open(os.path.join(HERE, "share_part0.json")) as f:
        gold = json.load(f)
    b = gold["bounds_head"]
    assert b[0] == 0 < b[1] < b[2] < b[3]
    assert gold["u_end"] == b[1] and gold["P"] == 64 and gold["n"] == 10 ** 9
    # Theorem 2 of Sec. 4: a part's edge count is within a factor 3/2 of its
    # expected share Z / P (costs in units of 1/256, one unit of 256 per source)
    share = gold["Z"] / gold["P"] / 256.0
    assert 0.5 * share < gold["m"] < 1.5 * share
    assert gold["m"] <= gold["candidates"]
