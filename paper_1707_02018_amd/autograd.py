"""A = R W as a differentiable torch operator.

Sec. "Motivation": the gradient of l(A x + b) is A^* grad l(A x + b), so the
backward of A is the adjoint A^* = W^* R^* (and the backward of A^* is A).
Both directions run the library's kernels on the current stream.
"""
from __future__ import annotations

import torch

from . import ops


class _AFn(torch.autograd.Function):
    @staticmethod
    def forward(ctx, x, w, b):
        ctx.w, ctx.b = w, b
        return ops.apply_A(w, b, x.contiguous())

    @staticmethod
    def backward(ctx, g):
        return ops.apply_A_adjoint(ctx.w, ctx.b, g.contiguous()), None, None


class _AadjFn(torch.autograd.Function):
    @staticmethod
    def forward(ctx, y, w, b):
        ctx.w, ctx.b = w, b
        return ops.apply_A_adjoint(w, b, y.contiguous())

    @staticmethod
    def backward(ctx, g):
        return ops.apply_A(ctx.w, ctx.b, g.contiguous()), None, None


class _WFn(torch.autograd.Function):
    @staticmethod
    def forward(ctx, x, w):
        ctx.w = w
        return ops.wavelet_synth(w, x.contiguous())

    @staticmethod
    def backward(ctx, g):
        return ops.wavelet_synth_adjoint(ctx.w, g.contiguous()), None


class AOperator(torch.nn.Module):
    """x [..., ncoef] -> R W x [..., rows, cols]; differentiable (backward = A^*)."""

    def __init__(self, w: ops.WaveletSpec, b: ops.BlurSpec):
        super().__init__()
        if (w.rows, w.cols) != (b.rows, b.cols):
            raise ValueError("wavelet and blur sizes differ")
        self.w, self.b = w, b

    def forward(self, x: torch.Tensor) -> torch.Tensor:
        return _AFn.apply(x, self.w, self.b)

    def adjoint(self, y: torch.Tensor) -> torch.Tensor:
        return _AadjFn.apply(y, self.w, self.b)


def apply_A(x, w, b):
    return _AFn.apply(x, w, b)


def apply_A_adjoint(y, w, b):
    return _AadjFn.apply(y, w, b)


def wavelet_synth(x, w):
    return _WFn.apply(x, w)
