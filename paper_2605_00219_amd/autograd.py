"""Differentiable rendering through the C ABI as a torch.autograd.Function.

    image = render(params_block, frame, views_dev)       # [pixels, 3]
    loss = f(image); loss.backward()                      # params_block.grad

Forward runs gs_project -> gs_bin_sort -> gs_rasterize_fwd.  Backward runs
gs_rasterize_bwd with dL/dC = the incoming gradient (transmittance is
recomputed front to back inside the kernel, nothing per pair is stored) and
gs_project_bwd_adam in gradient-only mode (no optimiser step), which returns
dL/dparams in the parameter-block layout.  `render_gaussians` does the same
from separate per-attribute tensors; packing them into the parameter block is
plain tensor indexing, so their gradients follow by torch's own autograd.
"""
from __future__ import annotations

import torch

from . import pipeline as P


class RenderFunction(torch.autograd.Function):
    @staticmethod
    def forward(ctx, params: torch.Tensor, frame: P.Frame, views_dev: torch.Tensor,
                lds_batch: int = 64):
        if not params.is_contiguous():
            params = params.contiguous()
        P.project(params, frame, views_dev)
        P.bin_sort(frame)
        if frame.status_bits():
            P.fit_capacity(params, frame, views_dev)
            P.bin_sort(frame)
        P.rasterize_fwd(frame, views_dev, lds_batch)
        frame._generation = getattr(frame, "_generation", 0) + 1
        ctx.frame = frame
        ctx.generation = frame._generation
        ctx.views_dev = views_dev
        ctx.lds_batch = lds_batch
        ctx.save_for_backward(params)
        return frame.image.clone()

    @staticmethod
    def backward(ctx, grad_image: torch.Tensor):
        (params,) = ctx.saved_tensors
        frame = ctx.frame
        if frame._generation != ctx.generation:
            raise RuntimeError("the frame was reused by another forward before this backward; "
                               "give each pending render its own Frame")
        g = grad_image.to(torch.float32).contiguous().reshape(-1, 3)
        P.rasterize_bwd(frame, ctx.views_dev, dLdC=g, lds_batch=ctx.lds_batch)
        grads = torch.zeros_like(params)
        model = _GradOnly(params)
        P.project_bwd_adam(model, frame, ctx.views_dev, adam=False, grads_out=grads)
        return grads, None, None, None


class _GradOnly:
    """Minimal stand-in for pipeline.Model when no optimiser state exists."""

    def __init__(self, params):
        self.params = params
        self.adam = None


def render(params: torch.Tensor, frame: P.Frame, views_dev: torch.Tensor,
           lds_batch: int = 64) -> torch.Tensor:
    """Differentiable forward render of a parameter block [15, N, 4]."""
    return RenderFunction.apply(params, frame, views_dev, lds_batch)


def pack(means, log_scales, quats, opacity_logits, sh) -> torch.Tensor:
    """Differentiable packing of per-attribute tensors into the parameter block."""
    n = means.shape[0]
    flat = torch.cat([means, log_scales, quats, opacity_logits.reshape(n, 1), sh.reshape(n, 48)], 1)
    idx = torch.as_tensor(P._PLANE_INDEX, device=flat.device)
    blk = torch.zeros(n, P.PLANES * 4, dtype=flat.dtype, device=flat.device)
    blk = blk.index_put((torch.arange(n, device=flat.device)[:, None], idx[None, :]), flat)
    return blk.view(n, P.PLANES, 4).permute(1, 0, 2).contiguous()


def render_gaussians(means, log_scales, quats, opacity_logits, sh, frame: P.Frame,
                     views_dev: torch.Tensor, lds_batch: int = 64) -> torch.Tensor:
    return render(pack(means, log_scales, quats, opacity_logits, sh), frame, views_dev, lds_batch)
