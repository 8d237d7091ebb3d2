"""The SMoE render as a ``torch.autograd.Function`` backed by the hand-written adjoint.

Forward: raw parameters (mu, s1, l21, s2, rho, experts) -> materialized rows
(smoe_materialize) -> block lists (smoe_bin) -> image (smoe_render).  The context keeps the
materialized rows, the block lists, the image and the per-pixel denominator D.
Backward: smoe_render_backward in upstream-gradient mode, which recomputes every gate from
D (nothing per (pixel, kernel) is stored) and returns dL/draw directly (d/ds = l d/dl).

Reading of the truncation.  The default here is trunc="render": the ellipse test q <= r^2
applies to the render as well, and the backward is then the exact adjoint of the forward
(what torch.autograd and gradcheck assume).  trunc="gradient" is Sec. IV-B's literal reading
that the fit step uses -- the render takes every term of the block lists and out-of-ellipse
pixels are discarded in the gradient only -- so its backward is NOT the derivative of its own
forward: it is the sum of the in-ellipse (pixel, kernel) pairs' terms of that derivative.
"""
from __future__ import annotations

import torch

from . import core


class SMoERender(torch.autograd.Function):
    @staticmethod
    def forward(ctx, raw, C, order, width, height, scale=1, origin_x=0, origin_y=0, radius=3.0,
                mode="smoe", trunc="render"):
        if not (raw.is_cuda and raw.dtype == torch.float32):
            raise ValueError("raw must be a cuda float32 [K, NP] tensor")
        grid = core.make_grid(width, height, scale, origin_x, origin_y, radius, mode=mode,
                              trunc=trunc)
        model = core.materialize(raw.detach().contiguous(), C, order)
        bins = core.bin(model, C, order, grid)
        image, denom, _, _ = core.render(model, C, order, grid, bins=bins)
        ctx.save_for_backward(model, image, denom)
        ctx.bins, ctx.grid, ctx.C, ctx.order = bins, grid, C, order
        return image

    @staticmethod
    def backward(ctx, grad_image):
        model, image, denom = ctx.saved_tensors
        g = core.render_backward(model, ctx.C, ctx.order, ctx.grid, ctx.bins, image, denom,
                                 grad_image=grad_image.contiguous())
        return g, None, None, None, None, None, None, None, None, None, None


def smoe_render(raw: torch.Tensor, C: int, order: int, width: int, height: int, scale: int = 1,
                origin_x: int = 0, origin_y: int = 0, radius: float = 3.0, mode: str = "smoe",
                trunc: str = "render") -> torch.Tensor:
    """Differentiable render of raw kernel rows [K, 6 + C(1 + 2 order)] into [H, W, C];
    mode "rbf" renders the weighted sum of kernels of Eq. (1) instead of the gates.
    trunc "render" (default): exact adjoint; "gradient": the fit step's reading, whose
    backward drops out-of-ellipse pairs (not the forward's derivative; see the module
    docstring)."""
    return SMoERender.apply(raw, C, order, width, height, scale, origin_x, origin_y, radius,
                            mode, trunc)
