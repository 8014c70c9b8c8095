"""torch.autograd.Function over the library's forward model.

Forward: gm_model_image (the PSF-convolved model image, FP32, image layout of
the batch).  Backward: gm_model_vjp, the hand-written adjoint that contracts
the derivative images with the incoming gradient on the device without
storing the Jacobian.  Gradients flow to the FP64 parameter tensor [n][p] in
natural units; the batch and model are constants.
"""
from __future__ import annotations

import torch

from . import gmfit as G


class ModelImage(torch.autograd.Function):
    @staticmethod
    def forward(ctx, params: torch.Tensor, model: G.Model, batch: G.Batch):
        ctx.model = model
        ctx.batch = batch
        ctx.save_for_backward(params)
        return G.gm_model_image(model, batch, params.detach())

    @staticmethod
    def backward(ctx, grad_out: torch.Tensor):
        (params,) = ctx.saved_tensors
        if not ctx.needs_input_grad[0]:
            return None, None, None
        g = G.gm_model_vjp(ctx.model, ctx.batch, params.detach(), grad_out)
        return g.to(params.dtype).view_as(params), None, None


def model_image(params: torch.Tensor, model: G.Model, batch: G.Batch) -> torch.Tensor:
    """Differentiable model image of every galaxy of the batch."""
    return ModelImage.apply(params, model, batch)
