"""Differentiable rendering: a torch.autograd.Function whose forward pass is
the renderer (plain and foveated views alike) and whose backward pass is
vrs_render_backward, through the periphery blur, the LOW group mean and the
HYBRID mix for foveated views (Sec. 4.1 fine-tunes the Gaussians by
backpropagation through the renderer with StopThePop ordering and Optimal
Projection).

The renderer keeps the state of its last forward pass (render records,
sorted instances, tile ranges) on the GPU, and the backward kernels replay
the blending from it, so a backward call must come before the renderer's
next forward pass; this is checked.
"""
from __future__ import annotations

import torch

from .render import Gaussians, Renderer


class VRSRasterize(torch.autograd.Function):
    @staticmethod
    def forward(ctx, renderer: Renderer, sh_degree: int, check: bool, means, log_scales, quats,
                opacity_logits, sh):
        g = Gaussians(means.detach(), log_scales.detach(), quats.detach(), opacity_logits.detach(),
                      sh.detach(), sh_degree)
        imgs = renderer.render(g)
        if check:
            # An instance-capacity overflow leaves the lists incomplete:
            # grow the buffers and render again.
            try:
                renderer.check()
            except RuntimeError:
                renderer.status.zero_()
                renderer.ensure_capacity(g)
                imgs = renderer.render(g)
                renderer.check()
        outs = tuple(im.clone() for im in imgs)
        ctx.renderer = renderer
        ctx.generation = renderer.generation
        ctx.g = g
        ctx.save_for_backward(*outs)
        return outs

    @staticmethod
    def backward(ctx, *grad_out):
        r = ctx.renderer
        if r.generation != ctx.generation:
            raise RuntimeError("the renderer ran another forward pass after this one; the state the "
                               "backward pass replays belongs to the newer pass")
        imgs = ctx.saved_tensors
        grads = [torch.zeros_like(im) if go is None else go for go, im in zip(grad_out, imgs)]
        out = r.backward(ctx.g, grads, imgs)
        return (None, None, None, out["means"], out["log_scales"], out["quats"], out["opacity_logits"],
                out["sh"])


def rasterize(renderer: Renderer, means, log_scales, quats, opacity_logits, sh, sh_degree: int = 3,
              check: bool = True):
    """Images (tuple of (4, H, W) tensors, one per view) of the Gaussians,
    differentiable with respect to the five parameter tensors (float32 CUDA,
    the SoA layouts of vrs_gaussians).  ``check`` synchronises once to detect
    an instance-buffer overflow and re-renders after growing the buffers."""
    return VRSRasterize.apply(renderer, sh_degree, check, means, log_scales, quats, opacity_logits, sh)
