"""Differentiable fault-tolerant FFT layer.

``fft(x)`` is the forward DFT of each row of a complex CUDA tensor,
y_j = sum_n x_n w_N^{jn} (TurboFFT Section II), computed by the library's
HIP kernels with the two-sided checksum.  Its backward pass applies the
adjoint of that linear map, F^H = conj(W)^T, which is the unscaled inverse DFT:
for a real loss, PyTorch's complex gradient (d/dRe + i d/dIm) of x is
F^H applied to the gradient of y.  The backward transform runs through the
same kernels with its own two-sided checksum (a plan created with the
unscaled-inverse flag), so a fault in either direction is detected and
corrected.
"""
from __future__ import annotations

import torch

from . import Plan

_PLANS: dict = {}


def _plans(n: int, batch: int, dtype, device) -> tuple[Plan, Plan]:
    key = (n, batch, str(dtype), str(device))
    if key not in _PLANS:
        with torch.cuda.device(device):
            _PLANS[key] = (Plan(n, batch, dtype), Plan(n, batch, dtype, inverse_unscaled=True))
    return _PLANS[key]


def clear_plan_cache() -> None:
    for fwd, adj in _PLANS.values():
        fwd.close()
        adj.close()
    _PLANS.clear()


class UncorrectableError(RuntimeError):
    """A flagged checksum group of the layer's transform was not corrected."""


def _verify(plan: Plan, what: str) -> None:
    counts, _ = plan.report()
    if counts["uncorrectable"] or counts["dropped"]:
        raise UncorrectableError(f"{what}: {counts}")


class _FFTFunction(torch.autograd.Function):
    @staticmethod
    def forward(ctx, x, ft_mode, check):
        n = x.shape[-1]
        batch = x.numel() // n
        fwd, adj = _plans(n, batch, x.dtype, x.device)
        ctx.adj = adj
        ctx.ft_mode = ft_mode
        ctx.check = check
        xc = x.contiguous()
        y = fwd.forward(xc, ft_mode=ft_mode).view(x.shape)
        if check and ft_mode == "correct":
            _verify(fwd, "forward transform")
        return y

    @staticmethod
    def backward(ctx, gy):
        gx = ctx.adj.inverse(gy.contiguous(), ft_mode=ctx.ft_mode)
        if ctx.check and ctx.ft_mode == "correct":
            _verify(ctx.adj, "backward transform")
        return gx.view(gy.shape), None, None


def fft(x: torch.Tensor, ft_mode: str = "correct", check: bool = False) -> torch.Tensor:
    """Forward DFT along the last axis of a complex64/complex128 CUDA tensor,
    differentiable, fault tolerant in both directions.

    The outcome of the checks is in the plans' reports, which the layer does
    not read by default (reading one waits for the transform's stream): call
    ``last_reports()`` to see detected, corrected and uncorrectable groups.
    With ``check=True`` (CORRECT mode) every forward and backward transform
    reads its report and raises ``UncorrectableError`` when a flagged group
    could not be corrected or a record was dropped."""
    if not x.is_complex():
        raise TypeError("fft expects a complex tensor")
    return _FFTFunction.apply(x, ft_mode, check)


def last_reports():
    """Reports of the most recent forward and backward executions of each cached plan."""
    out = {}
    for key, (fwd, adj) in _PLANS.items():
        out[key] = {"forward": fwd.report(), "backward": adj.report()}
    return out
