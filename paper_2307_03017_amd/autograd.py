"""PyTorch autograd over the HIP kernels.

``HSGDRender``: MPI -> rendered views (Eq. render / Eq. over); backward is the library's
hand-written adjoint (``hsgd_grad_step`` with an upstream image gradient, no update).

``HSGDPhotometricLoss``: MPI -> the photometric loss 1/(2N) sum (C - I)^2 against target
views; forward and backward share one fused gradient kernel call.

Both accept an optional plane mask (``hsgd_select_active``) restricting the gradient to the
selected voxels (zero elsewhere). Gradients are accumulated in FP32. For BF16 storage pass an
FP32 master tensor as the differentiable input and its BF16 copy as ``storage``: the kernels
read the BF16 copy and the FP32 gradient (at the BF16 point) flows to the master, which
PyTorch would otherwise round to the input's dtype.
"""

from __future__ import annotations

import torch

from . import hsgd


class HSGDRender(torch.autograd.Function):
    @staticmethod
    def forward(ctx, rgba: torch.Tensor, warps, N: int, mask: torch.Tensor | None = None,
                kcap: int | None = None, storage: torch.Tensor | None = None):
        src = rgba if storage is None else storage
        out, _ = hsgd.hsgd_render(src, warps, N)
        ctx.save_for_backward(src)
        ctx.warps, ctx.N, ctx.mask, ctx.kcap = warps, N, mask, kcap
        return out

    @staticmethod
    def backward(ctx, grad_out: torch.Tensor):
        (src,) = ctx.saved_tensors
        g = grad_out.contiguous().to(torch.float32)
        grad, _ = hsgd.hsgd_grad_step(src, ctx.warps, ctx.N, dimg=g, mask=ctx.mask, kcap=ctx.kcap,
                                      want_grad=True)
        return grad, None, None, None, None, None


class HSGDPhotometricLoss(torch.autograd.Function):
    @staticmethod
    def forward(ctx, rgba: torch.Tensor, warps, images: torch.Tensor, mask: torch.Tensor | None = None,
                kcap: int | None = None, storage: torch.Tensor | None = None):
        N = images.shape[0]
        src = rgba if storage is None else storage
        grad, loss = hsgd.hsgd_grad_step(src, warps, N, images=images, mask=mask, kcap=kcap,
                                         want_grad=True, want_loss=True)
        ctx.save_for_backward(grad)
        return loss[0]

    @staticmethod
    def backward(ctx, g: torch.Tensor):
        (grad,) = ctx.saved_tensors
        return grad * g, None, None, None, None, None


def render(rgba, warps, N, mask=None, kcap=None, storage=None):
    """Differentiable rendering of N views: [N][H][W][3] float32."""
    return HSGDRender.apply(rgba, warps, N, mask, kcap, storage)


def photometric_loss(rgba, warps, images, mask=None, kcap=None, storage=None):
    """Differentiable photometric loss 1/(2N) sum (C - I)^2 (a 0-dim float32 tensor)."""
    return HSGDPhotometricLoss.apply(rgba, warps, images, mask, kcap, storage)
