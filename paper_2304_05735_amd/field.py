"""Differentiable surface of one object's radiance field for PyTorch.

``RomapFieldFn`` wraps romap_field_forward / romap_field_backward: the forward
renders caller-given object-frame rays (colour on black, depth, T_end) with
the library's kernels; the backward recomputes every per-sample activation
(encoding, MLP, compositing) instead of saving it, and returns the gradient
with respect to the parameter vector (grid level-major, then W1..W4).  Only
the parameter tensor and the rays are kept between the two passes.

The context must order its work on torch's current stream (create it with
``stream=torch.cuda.current_stream()``), so that the library's kernels and
torch's own operations on the same tensors are ordered.
"""
from __future__ import annotations

import torch

from . import Context


class RomapFieldFn(torch.autograd.Function):
    @staticmethod
    def forward(ctx, params: torch.Tensor, rays: torch.Tensor, rctx: Context, oid: int):
        assert params.is_cuda and params.dtype == torch.float32 and params.is_contiguous()
        assert rays.is_cuda and rays.dtype == torch.float32 and rays.shape[-1] == 8
        rays = rays.contiguous()
        rgb, depth, tend = rctx.field_forward(oid, rays, params)
        ctx.save_for_backward(params, rays)
        ctx.rctx = rctx
        ctx.oid = oid
        return rgb, depth, tend

    @staticmethod
    def backward(ctx, d_rgb, d_depth, d_tend):
        params, rays = ctx.saved_tensors
        n = rays.shape[0]
        dev = rays.device
        d_rgb = torch.zeros(n, 3, device=dev) if d_rgb is None else d_rgb.contiguous().float()
        d_depth = torch.zeros(n, device=dev) if d_depth is None else d_depth.contiguous().float()
        d_tend = torch.zeros(n, device=dev) if d_tend is None else d_tend.contiguous().float()
        dp = ctx.rctx.field_backward(ctx.oid, rays, d_rgb, d_depth, d_tend, params)
        return dp, None, None, None


class RomapField(torch.nn.Module):
    """One object's field as a module: its parameter vector is a torch
    Parameter initialised from the library's object."""

    def __init__(self, rctx: Context, oid: int):
        super().__init__()
        self.rctx = rctx
        self.oid = oid
        p = torch.from_numpy(rctx.get_params(oid)).cuda()
        self.params = torch.nn.Parameter(p)

    def forward(self, rays: torch.Tensor):
        return RomapFieldFn.apply(self.params, rays, self.rctx, self.oid)
