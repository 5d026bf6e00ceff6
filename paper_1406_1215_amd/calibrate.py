"""Weight calibration by differentiating the expected degree.

The Chung-Lu model of Sec. 3 treats w as the expected degrees, which holds
only when no pair is capped (the expected degree is w_i - w_i^2/S without the
cap).  In the capped regime (max w^2 > S) the expected degree
d_i = sum_{j != i} min(w_i w_j / S, 1) falls short of w_i.  Calibration finds
weights whose expected degrees hit a target sequence: Adam on theta = log w
minimising mean((d/t - 1)^2), with d and its adjoint from the HIP kernels
(cl_expected_degree, cl_expected_degree_backward).  The calibrated weights are
then sorted and handed unchanged to the generator.
"""
from __future__ import annotations

import math
from dataclasses import dataclass
from typing import Optional

import torch

from . import clgen


class ExpectedDegree(torch.autograd.Function):
    """d = expected degrees of float32 weights w under S = sum(w) (float64).

    Forward and backward run in the HIP kernels; with s_from_w the backward
    includes dS/dw_k = 1 (S is the sum of the same weights)."""

    @staticmethod
    def forward(ctx, w: torch.Tensor, S: float, s_from_w: bool = True, tuning: Optional[dict] = None):
        w = w.contiguous()
        d = clgen.cl_expected_degree(w, S, tuning=tuning)
        ctx.save_for_backward(w)
        ctx.S = S
        ctx.s_from_w = s_from_w
        ctx.tuning = tuning
        return d

    @staticmethod
    def backward(ctx, g: torch.Tensor):
        (w,) = ctx.saved_tensors
        grad = clgen.cl_expected_degree_backward(w, ctx.S, g.to(torch.float64).contiguous(), ctx.s_from_w,
                                                 tuning=ctx.tuning)
        return grad, None, None, None


def expected_degree(w: torch.Tensor, tuning: Optional[dict] = None) -> torch.Tensor:
    """Expected degrees of float32 weights with S = sum(w), differentiable;
    tuning: the kernels' tile shape (ed_rows, ed_cols), defaults if None."""
    S = float(w.detach().to(torch.float64).sum())
    return ExpectedDegree.apply(w, S, True, tuning)


@dataclass
class CalibrationResult:
    w: torch.Tensor              # float64, sorted non-increasing (ready for the generator)
    max_rel_err: float           # max_i |d_i / t_i - 1| at the end
    loss: float
    losses: list
    seconds: float
    pair_evals: float            # pairs evaluated (forward + backward)


def calibrate(t: torch.Tensor, steps: int = 200, lr: float = 0.05, betas=(0.9, 0.999), eps: float = 1e-8,
              log_every: int = 0, w0: Optional[torch.Tensor] = None,
              tuning: Optional[dict] = None) -> CalibrationResult:
    """Adam on log w so that the expected degrees match the targets t.  The
    kernels' tile shape is `tuning`, else the autotuner's cached choice for
    n^2 pairs, else the defaults."""
    import time
    from . import autotune
    dev = t.device
    if tuning is None:
        tuning = autotune.lookup(float(t.numel()) ** 2, kind="expdeg")
    t64 = t.to(torch.float64)
    init = (w0 if w0 is not None else t).to(torch.float32).clamp_min(1e-30)
    theta = torch.nn.Parameter(torch.log(init).clone())
    opt = torch.optim.Adam([theta], lr=lr, betas=betas, eps=eps)
    n = t.numel()
    losses = []
    torch.cuda.synchronize(dev)
    t0 = time.perf_counter()
    for it in range(steps):
        opt.zero_grad(set_to_none=True)
        w = torch.exp(theta)
        d = expected_degree(w, tuning)
        loss = torch.mean((d / t64 - 1.0) ** 2)
        loss.backward()
        opt.step()
        if log_every and (it % log_every == 0 or it == steps - 1):
            losses.append((it, float(loss)))
    torch.cuda.synchronize(dev)
    secs = time.perf_counter() - t0
    with torch.no_grad():
        w = torch.exp(theta).to(torch.float32)
        d = expected_degree(w, tuning)
        rel = (d / t64 - 1.0).abs()
        final = float(torch.mean((d / t64 - 1.0) ** 2))
        w64 = torch.sort(w.to(torch.float64), descending=True).values.contiguous()
    return CalibrationResult(w=w64, max_rel_err=float(rel.max()), loss=final, losses=losses, seconds=secs,
                             pair_evals=2.0 * steps * float(n) * float(n))
