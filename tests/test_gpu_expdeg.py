"""GPU: expected degree (float32 tiles, float64 rows) and its adjoint against
the float64 oracle; the autograd Function against torch autograd in float64;
calibration to a capped target sequence, then generation from the calibrated
weights with the unchanged generator."""
import math

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


def _w32(n, seed, heavy=True):
    rng = np.random.default_rng(seed)
    w = (rng.pareto(1.1 if heavy else 3.0, n) + 1.0).astype(np.float32) * np.float32(3.0)
    return w   # unsorted: the kernels take any order


def _dev32(w):
    import torch
    return torch.from_numpy(np.ascontiguousarray(w, dtype=np.float32)).to("cuda:0")


def _dev64(x):
    import torch
    return torch.from_numpy(np.ascontiguousarray(x, dtype=np.float64)).to("cuda:0")


@pytest.mark.parametrize("n", [1, 2, 255, 1000, 1025, 4097])
def test_forward_matches_float64(cg, n):
    w = _w32(n, n)
    w64 = w.astype(np.float64)
    S = float(np.sum(w64))
    d = cg.cl_expected_degree(_dev32(w), S).cpu().numpy()
    ref = O.expdeg_brute(w64, S)
    rel = np.abs(d - ref) / np.maximum(ref, 1e-300)
    assert rel.max() < 1e-5, rel.max()


@pytest.mark.parametrize("s_dep", [True, False])
@pytest.mark.parametrize("n", [300, 3000])
def test_backward_matches_float64(cg, n, s_dep):
    w = _w32(n, 100 + n)
    w64 = w.astype(np.float64)
    S = float(np.sum(w64))
    g = np.random.default_rng(n).standard_normal(n)
    got = cg.cl_expected_degree_backward(_dev32(w), S, _dev64(g), s_dep).cpu().numpy().astype(np.float64)
    ref = O.expdeg_grad_brute(w64, S, g, s_depends_on_w=s_dep)
    err = np.linalg.norm(got - ref) / np.linalg.norm(ref)
    assert err < 1e-4, err


@pytest.mark.parametrize("case", ["tiny_thresholds", "zero_weights"])
def test_backward_mask_edge_cases(cg, case):
    """The adjoint forms its mask w_j < t_i with a clamped multiply-add that
    is exact only for thresholds t_i >= 2^-100; a wave holding a smaller
    one takes the plain comparison.  tiny_thresholds: S far below sum(w), so
    rows with w_i ~ 1 have t_i ~ 1e-31 and share waves with rows of normal
    thresholds; zero_weights: t_i = inf, every column passes."""
    n = 1500
    rng = np.random.default_rng(77)
    if case == "tiny_thresholds":
        big = rng.random(n) < 0.3
        w = np.where(big, 1.0 + rng.random(n), 1e-33 * (1.0 + rng.random(n))).astype(np.float32)
        S, s_dep = 1e-31, False
    else:
        w = _w32(n, 78)
        w[rng.random(n) < 0.1] = 0.0
        S, s_dep = float(np.sum(w.astype(np.float64))), True
    w64 = w.astype(np.float64)
    d = cg.cl_expected_degree(_dev32(w), S).cpu().numpy()
    ref = O.expdeg_brute(w64, S)
    assert np.max(np.abs(d - ref) / np.maximum(ref, 1.0)) < 1e-5
    g = rng.standard_normal(n)
    got = cg.cl_expected_degree_backward(_dev32(w), S, _dev64(g), s_dep).cpu().numpy().astype(np.float64)
    gref = O.expdeg_grad_brute(w64, S, g, s_depends_on_w=s_dep)
    err = np.linalg.norm(got - gref) / np.linalg.norm(gref)
    assert err < 1e-4, err


def test_full_size_forward_backward(cg):
    """n = 1e5 capped targets, 1e10 pairs: against the float64 closed forms."""
    t = W.config_calib()
    w = t.astype(np.float32)
    w64 = w.astype(np.float64)
    S = float(np.sum(w64))
    d = cg.cl_expected_degree(_dev32(w), S).cpu().numpy()
    ref = O.expdeg_closed(w64, S)
    rel = np.abs(d - ref) / ref
    assert rel.max() < 1e-5, rel.max()
    g = 2.0 * (ref / t - 1.0) / (t * t.size)        # gradient of mean((d/t-1)^2)
    got = cg.cl_expected_degree_backward(_dev32(w), S, _dev64(g), True).cpu().numpy().astype(np.float64)
    gref = O.expdeg_grad_closed(w64, S, g)
    err = np.linalg.norm(got - gref) / np.linalg.norm(gref)
    assert err < 1e-4, err


def test_autograd_function_matches_torch_float64(cg):
    import torch
    from paper_1406_1215_amd.calibrate import expected_degree
    n = 400
    w = _w32(n, 7)
    theta = torch.tensor(np.log(w), dtype=torch.float32, device="cuda:0", requires_grad=True)
    t = torch.tensor(w.astype(np.float64) * 0.8 + 1.0, device="cuda:0")
    loss = torch.mean((expected_degree(torch.exp(theta)) / t - 1.0) ** 2)
    loss.backward()
    # float64 reference on the CPU with torch autograd
    th = torch.tensor(np.log(w).astype(np.float64), requires_grad=True)
    ww = torch.exp(th)
    S = ww.sum()
    X = torch.minimum(ww[:, None] * ww[None, :] / S, torch.ones(n, n, dtype=torch.float64))
    X = X - torch.diag(torch.diagonal(X))
    l2 = torch.mean((X.sum(1) / t.cpu() - 1.0) ** 2)
    l2.backward()
    a = theta.grad.cpu().numpy().astype(np.float64)
    b = th.grad.numpy()
    assert np.linalg.norm(a - b) / np.linalg.norm(b) < 1e-4
    assert abs(float(loss) - float(l2)) < 1e-5 * float(l2)


def test_calibration_hits_capped_targets_then_generates(cg):
    import torch
    from paper_1406_1215_amd.calibrate import calibrate
    t = W.config_calib(n=20000)
    assert t[0] ** 2 > t.sum()                    # capped regime
    td = _dev64(t)
    # without calibration the top node falls far short of its target
    d0 = O.expdeg_closed(t, O.exact_sum(t))
    assert d0[0] < 0.9 * t[0]
    res = calibrate(td, steps=200, lr=0.05)
    assert res.max_rel_err < 1e-3, res.max_rel_err
    w = res.w.cpu().numpy()
    assert np.all(np.diff(w) <= 0)
    S = O.exact_sum(w)
    d = O.expdeg_closed(w, S)
    # the float64 expected degrees of the calibrated weights are close to the targets
    ts = np.sort(t)[::-1]
    assert np.max(np.abs(d / ts - 1.0)) < 2e-3
    # the unchanged generator on the calibrated weights: bit-identical to the oracle
    want, m, _, _ = O.generate(w, S, 11)
    plan = cg.cl_sample([cg.Task(res.w, S, 11)])
    got = cg.cl_generate(plan).cpu().numpy().view(np.uint32).reshape(-1, 2)[: plan.total]
    assert np.array_equal(got, want)
    deg = np.bincount(want.ravel().astype(np.int64), minlength=w.size)
    # degree sums agree with the calibrated targets in aggregate
    assert abs(deg.sum() - d.sum()) < 6 * math.sqrt(d.sum())


def test_autotuner_keeps_output_and_picks_a_setting(cg, tmp_path, monkeypatch):
    import torch
    from paper_1406_1215_amd import autotune
    monkeypatch.setattr(autotune, "CACHE", str(tmp_path / "tuned.json"))
    w = W.config_small(n=50000)
    S = O.exact_sum(w)
    tasks = [cg.Task(_dev64(w), S, 3)]
    res = autotune.tune(tasks, budgets=(32, 192, 1024), blocks=(2, 8), reps=1)
    assert res["best"]["lane_budget"] in (32, 192, 1024)
    assert len(res["table"]) == 6
    assert autotune.lookup(res["edges"]) == res["best"]


def test_batch_autotuner_keeps_output_and_is_looked_up(cg, tmp_path, monkeypatch):
    """tune_batch times replays of the captured batch for every setting
    (raising if any changes the digest); its choice is what lookup returns
    for batches of that size, and a batch captured with it is bit-exact with
    the oracle."""
    import torch
    from paper_1406_1215_amd import autotune
    monkeypatch.setattr(autotune, "CACHE", str(tmp_path / "tuned.json"))
    rng = np.random.default_rng(12)
    ws = [W.config_small(seed=int(rng.integers(1 << 30)), n=int(rng.integers(500, 30000))) for _ in range(6)]
    tasks, wants = [], []
    for i, w in enumerate(ws):
        S = O.exact_sum(w)
        wants.append(O.generate(w, S, 60 + i)[0])
        tasks.append(cg.Task(_dev64(w), S, 60 + i))
    res = autotune.tune_batch(tasks, budgets=(48, 192), blocks=(2, 4), reps=2)
    assert len(res["table"]) == 4
    m = sum(x.shape[0] for x in wants)
    assert res["edges"] == m
    assert autotune.lookup(m, kind="batch") == res["best"]
    assert autotune.lookup(m) is None          # the plain tuner's entries are separate
    plan = cg.cl_sample(tasks, tuning=res["best"])
    s = torch.cuda.Stream()
    bg = cg.cl_batch_capture(plan, s)
    bg.launch(s)
    s.synchronize()
    got = bg.edges.cpu().numpy().view(np.uint32).reshape(-1, 2)[:m]
    assert np.array_equal(got, np.concatenate(wants))
    bg.close()


SHAPES = [{"ed_rows": r, "ed_cols": c} for r in (1, 2, 4) for c in (512, 1024, 2048)]


@pytest.mark.parametrize("shape", SHAPES, ids=lambda t: f"R{t['ed_rows']}C{t['ed_cols']}")
def test_every_tile_shape_matches_float64(cg, shape):
    """Every tile shape the tuner may pick: forward and adjoint against the
    float64 oracle at the same bars, on sizes with ragged row and column
    tiles."""
    for n in (2049, 5000):
        w = _w32(n, 7 * n)
        w64 = w.astype(np.float64)
        S = float(np.sum(w64))
        d = cg.cl_expected_degree(_dev32(w), S, tuning=shape).cpu().numpy()
        ref = O.expdeg_brute(w64, S)
        assert (np.abs(d - ref) / np.maximum(ref, 1e-300)).max() < 1e-5
        g = np.random.default_rng(n).standard_normal(n)
        got = cg.cl_expected_degree_backward(_dev32(w), S, _dev64(g), True, tuning=shape).cpu().numpy()
        want = O.expdeg_grad_closed(w64, S, g, True)
        assert np.linalg.norm(got.astype(np.float64) - want) / np.linalg.norm(want) < 1e-4


def test_tile_shape_outside_the_instantiations_is_refused(cg):
    w = _w32(100, 1)
    for bad in ({"ed_rows": 3}, {"ed_cols": 256}, {"ed_cols": 4096}):
        with pytest.raises(cg.ClError) as ei:
            cg.cl_expected_degree(_dev32(w), float(w.sum()), tuning=bad)
        assert ei.value.code == -1


def test_expdeg_tuner_picks_a_shape_and_is_looked_up(cg, tmp_path, monkeypatch):
    from paper_1406_1215_amd import autotune
    monkeypatch.setattr(autotune, "CACHE", str(tmp_path / "tuned.json"))
    w = _w32(20000, 5)
    res = autotune.tune_expdeg(_dev32(w), float(w.astype(np.float64).sum()), reps=1)
    assert len(res["table"]) == len(SHAPES)
    assert res["best"] in SHAPES
    assert autotune.lookup(20000.0 ** 2, kind="expdeg") == res["best"]
