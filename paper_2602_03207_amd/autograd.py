"""torch.autograd.Function over the library's forward and backward calls.

    images = render_gaussians(means, log_scales, quats, opacity_logits, sh, renderer)

returns the views' images packed back to back (as Renderer.images); calling
backward() on anything computed from them runs ws_render_backward and yields
gradients for all five parameter tensors.  The renderer keeps the state of
its last forward, so one renderer serves one forward/backward at a time.
"""
from __future__ import annotations

import torch

from .pipeline import GaussianTensors, Renderer


class RenderGaussians(torch.autograd.Function):
    @staticmethod
    def forward(ctx, means, log_scales, quats, opacity_logits, sh, renderer: Renderer):
        g = GaussianTensors(means.detach().contiguous(), log_scales.detach().contiguous(),
                            quats.detach().contiguous(), opacity_logits.detach().contiguous(),
                            sh.detach().contiguous(), renderer.opts.sh_degree)
        renderer.forward(g, stream=torch.cuda.current_stream())
        ctx.renderer = renderer
        ctx.g = g
        return renderer.images.clone()

    @staticmethod
    def backward(ctx, grad_images):
        r: Renderer = ctx.renderer
        grads = r.backward(ctx.g, grad_images.contiguous(), stream=torch.cuda.current_stream(), check=True)
        return grads["means"], grads["log_scales"], grads["quats"], grads["opacity_logits"], grads["sh"], None


def render_gaussians(means, log_scales, quats, opacity_logits, sh, renderer: Renderer):
    return RenderGaussians.apply(means, log_scales, quats, opacity_logits, sh, renderer)
