"""Differentiable objectives f1 and f2 as torch.autograd.Functions.

f1(X) = ||A + X X^T||_F^2 and f2(X) = tr((2I - X^T X) X^T A X) on the
shifted normalized Laplacian A of a graph (Introduction; Sections 2.1, 2.2).
The forward pass returns f(X) computed by the library from k x k products;
the backward pass returns grad_out * grad f(X) (scaled by the library), where the gradient
(eqs. gradientf1, gradientf2) is produced by the same fused HIP kernels the
iteration uses (SpMM with the direction epilogue for f1, SpMM then the
direction pass for f2), during the forward call.  No CPU fallback.
"""
from __future__ import annotations

import torch

from . import ofm


class _Objective(torch.autograd.Function):
    @staticmethod
    def forward(ctx, X, ws):
        X = X.contiguous()
        grad = torch.empty_like(X)
        f, _ = ws.objective(X, grad)
        ctx.save_for_backward(grad)
        return f[0]

    @staticmethod
    def backward(ctx, grad_out):
        (grad,) = ctx.saved_tensors
        s = grad_out.detach().to(torch.float64).reshape(1).contiguous()
        return ofm.scale(grad, s), None


class Objective(torch.nn.Module):
    """f1 ("f1") or f2 ("f2") of the graph of ``lap`` as a function of an
    N x k tensor (FP64 or FP32, on the GPU)."""

    def __init__(self, lap: "ofm.Laplacian", k: int, kind: str = "f1", dtype=torch.float64):
        super().__init__()
        if kind not in ("f1", "f2"):
            raise ValueError("the triangular directions are not gradients; use f1 or f2")
        prec = ofm.OFM_FP64 if dtype == torch.float64 else ofm.OFM_FP32
        self.ws = ofm.Workspace(lap, k, variant=kind, precision=prec)
        self.dtype = dtype

    def forward(self, X):
        if X.dtype != self.dtype:
            raise TypeError(f"expected {self.dtype}")
        return _Objective.apply(X, self.ws)


def f1(lap, X):
    return Objective(lap, X.shape[1], "f1", X.dtype)(X)


def f2(lap, X):
    return Objective(lap, X.shape[1], "f2", X.dtype)(X)
