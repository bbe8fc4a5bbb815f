"""torch.autograd.Function over the HIP renderer.

The forward saves only rgb (12 B), depth (4 B) and nsamp (4 B) per ray; the
backward recomputes every sample position and transmittance in the kernel
(no per-sample state), so whole 1200x680 frames, or many of them, fit in
memory at O(rays).

Pose gradients use a tangent input: `xi` [F, 6] (float64, zero) stands for
the left, world-frame perturbation exp(xi^) c2w of each frame; its gradient
is dL/d(rho, phi) at xi = 0.  The forward renders at c2w and requires xi == 0.
"""
from __future__ import annotations

import torch

from . import pxm


class RenderFunction(torch.autograd.Function):
    @staticmethod
    def forward(ctx, data, xi, grid, rays, opts):
        rgb, depth, nsamp = pxm.render_forward(grid, rays, opts)
        ctx.save_for_backward(rgb, depth, nsamp)
        ctx.grid, ctx.rays, ctx.opts = grid, rays, opts
        ctx.mark_non_differentiable(nsamp)
        return rgb, depth, nsamp

    @staticmethod
    def backward(ctx, g_rgb, g_depth, _g_nsamp):
        rgb, depth, nsamp = ctx.saved_tensors
        grid, rays, opts = ctx.grid, ctx.rays, ctx.opts
        n = rays.n_rays
        g_rgb = (torch.zeros(n, 3, device=rgb.device) if g_rgb is None
                 else g_rgb.to(torch.float32).contiguous())
        g_depth = (torch.zeros(n, device=rgb.device) if g_depth is None
                   else g_depth.to(torch.float32).contiguous())
        grad_data = grad_xi = None
        if ctx.needs_input_grad[0]:
            grad_data = pxm.render_backward_grid(grid, rays, opts, rgb, depth, nsamp, g_rgb, g_depth)
        if ctx.needs_input_grad[1]:
            grad_xi = pxm.render_backward_pose(grid, rays, opts, rgb, depth, nsamp, g_rgb, g_depth)
        return grad_data, grad_xi, None, None, None


def render(grid: "pxm.DeviceGrid", rays: "pxm.DeviceRays", opts, data=None, xi=None):
    """Differentiable render.  `data` [n_alloc, 28] defaults to grid.data;
    pass a tensor with requires_grad for mapping gradients and/or a zero
    `xi` [F, 6] float64 with requires_grad for tracking gradients.
    Returns (rgb [n, 3], z-depth [n], nsamp [n])."""
    if data is None:
        data = grid.data
    if xi is None:
        xi = torch.zeros(rays.n_frames, 6, dtype=torch.float64, device=data.device)
    elif xi.requires_grad and bool((xi.detach() != 0).any()):
        raise ValueError("xi is a tangent at the current pose and must be zero; "
                         "apply the update to rays.c2w instead")
    g = grid if data is grid.data else grid.with_data(data.detach())
    return RenderFunction.apply(data, xi, g, rays, opts)


def tv_loss_grad(grid, data, lambda_density, lambda_sh, eps=1e-9):
    """Adds the TV gradient into data.grad (allocating it if needed)."""
    if data.grad is None:
        data.grad = torch.zeros_like(data)
    pxm.tv_grad(grid.with_data(data.detach()), lambda_density, lambda_sh, eps, data.grad)
    return data.grad
