"""Host-side logic of the benchmark and the autotuner cache, on the CPU:
the candidate density the gather ceiling draws from (against its definition
by brute force), the per-unit summary of the statistics pass, and the
autotuner's lookup (nearest size bucket, plain / batch / expdeg entries kept
apart)."""
import json
import os
import sys

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def test_candidate_density_matches_its_definition():
    import torch
    import bench
    rng = np.random.default_rng(4)
    for w in (np.sort(rng.pareto(1.2, 300) + 1.0)[::-1] * 5.0,    # capped head
              np.full(50, 3.0),                                     # ER
              np.array([40.0, 40.0, 40.0, 2.0, 1.0, 0.0, 0.0])):     # ties, zeros
        S = float(w.sum())
        got = bench.candidate_density(torch, torch.from_numpy(w), S).numpy()
        want = np.array([sum(min(w[u] * w[v] / S, 1.0) for u in range(v)) for v in range(w.size)])
        assert np.allclose(got, want, rtol=1e-12, atol=1e-12)


def test_draw_positions_follow_the_density():
    import torch
    import bench
    dens = torch.tensor([0.0, 1.0, 3.0, 0.0, 4.0], dtype=torch.float64)
    idx = bench.draw_positions(torch, dens, 200_000, 7, chunk=1 << 16).numpy()
    assert idx.dtype == np.int32 and idx.min() >= 0 and idx.max() <= 4
    freq = np.bincount(idx, minlength=5) / idx.size
    assert freq[0] == 0.0 and freq[3] == 0.0
    assert np.allclose(freq[[1, 2, 4]], [0.125, 0.375, 0.5], atol=0.005)


def test_unit_summary_of_a_known_schedule():
    import bench
    # two wavefronts; unit time = 3 ticks per cost unit exactly
    cost = np.array([10, 20, 30, 40, 0], dtype=np.uint64)
    t0 = np.array([100, 100, 200, 150, 100], dtype=np.uint64)
    t1 = t0 + cost * 3
    lane = np.array([0, 1, 64, 65, 2], dtype=np.uint64)
    st = {"t0": t0, "t1": t1, "cost": cost, "visits": cost, "edges": cost, "lane": lane}
    out = bench.unit_summary(st, np)
    assert out["units"] == 4 and out["waves"] == 2
    assert out["corr_time_cost"] == pytest.approx(1.0)
    assert out["us_per_expected_candidate"] == pytest.approx(3 / 100.0 * 16)
    # wave 0: [100, 160]; wave 1: [150, 290]
    assert out["wave_span_us_max"] == pytest.approx(1.4)
    assert out["wave_span_us_mean"] == pytest.approx(1.0)
    assert out["pass_span_us"] == pytest.approx(1.9)


def test_autotune_lookup_keeps_kinds_apart(tmp_path, monkeypatch):
    from paper_1406_1215_amd import autotune
    cache = tmp_path / "tuned.json"
    monkeypatch.setattr(autotune, "CACHE", str(cache))
    monkeypatch.setattr(autotune, "device_key", lambda: "dev")
    monkeypatch.setattr(autotune.torch.cuda, "is_available", lambda: True)
    assert autotune.lookup(1e6) is None
    autotune.store("e2^20", {"lane_budget": 128, "blocks_per_cu": 2}, 1.0)
    autotune.store("e2^30", {"lane_budget": 256, "blocks_per_cu": 4}, 2.0)
    autotune.store("batch:e2^29", {"lane_budget": 192, "blocks_per_cu": 3}, 3.0)
    autotune.store("expdeg:e2^33", {"ed_rows": 2, "ed_cols": 2048}, 4.0)
    assert autotune.lookup(2 ** 21) == {"lane_budget": 128, "blocks_per_cu": 2}
    assert autotune.lookup(2 ** 28) == {"lane_budget": 256, "blocks_per_cu": 4}
    assert autotune.lookup(6e8, kind="batch") == {"lane_budget": 192, "blocks_per_cu": 3}
    assert autotune.lookup(1e2, kind="batch") == {"lane_budget": 192, "blocks_per_cu": 3}
    assert autotune.lookup(1e10, kind="expdeg") == {"ed_rows": 2, "ed_cols": 2048}
    assert autotune.lookup(1e10, kind="nothing") is None
    data = json.loads(cache.read_text())
    assert set(data["dev"]) == {"e2^20", "e2^30", "batch:e2^29", "expdeg:e2^33"}
    assert autotune.size_bucket(2 ** 20) == "e2^20" and autotune.size_bucket(0.5) == "e2^0"
