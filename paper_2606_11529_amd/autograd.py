"""Differentiation: torch.autograd.Function wrappers over the C-ABI.

The forward saves only what the backward needs: the projected splat
records, the sorted pair list and tile ranges, and per pixel the final
transmittance and the position of the last blended entry (n_contrib); the
backward recomputes everything else in its kernels.
"""
from __future__ import annotations

import torch

from . import renderer as R


class RasterizeGaussians(torch.autograd.Function):
    """image [3, H, W] = render(means [3,n], scales [3,n] (activated),
    quats [4,n], opacities [n] (activated), sh [K,3,n]; cam, cfg)."""

    @staticmethod
    def forward(ctx, means, scales, quats, opacities, sh, cam, cfg):
        scene = R.Scene(means.detach(), scales.detach(), quats.detach(), opacities.detach(),
                        sh.detach())
        views = R.Views([scene], [cam], [0], cfg)
        proj = R.xpr_project(views, cfg)
        bins = R.xpr_bin_sort(views, cfg, proj)
        frame = R.xpr_render_fwd(views, cfg, proj, bins)
        ctx.state = (views, cfg, proj, bins, frame)
        return views.image(frame.image, 0)

    @staticmethod
    def backward(ctx, dimage):
        views, cfg, proj, bins, frame = ctx.state
        grads, _ = R.xpr_render_bwd(views, cfg, proj, bins, frame, dimage.reshape(-1))
        g = grads[0]
        ctx.state = None
        return g["means"], g["scales"], g["quats"], g["opacities"], g["sh"], None, None


class RasterizeViews(torch.autograd.Function):
    """Several views of one scene in one batched launch; returns the
    view-planar concatenation of the images. Gradients are summed over the
    views inside the projection-backward kernel."""

    @staticmethod
    def forward(ctx, means, scales, quats, opacities, sh, cams, cfg):
        scene = R.Scene(means.detach(), scales.detach(), quats.detach(), opacities.detach(),
                        sh.detach())
        views = R.Views([scene], list(cams), [0] * len(cams), cfg)
        proj = R.xpr_project(views, cfg)
        bins = R.xpr_bin_sort(views, cfg, proj)
        frame = R.xpr_render_fwd(views, cfg, proj, bins)
        ctx.state = (views, cfg, proj, bins, frame)
        return frame.image

    @staticmethod
    def backward(ctx, dimage):
        views, cfg, proj, bins, frame = ctx.state
        grads, _ = R.xpr_render_bwd(views, cfg, proj, bins, frame, dimage.reshape(-1))
        g = grads[0]
        ctx.state = None
        return g["means"], g["scales"], g["quats"], g["opacities"], g["sh"], None, None


def rasterize(means, scales, quats, opacities, sh, cam, cfg):
    return RasterizeGaussians.apply(means, scales, quats, opacities, sh, cam, cfg)


class GaussianModel(torch.nn.Module):
    """Trainable raw parameters (SoA); activations exp / sigmoid / identity
    are applied in torch before the kernels, which take activated values."""

    def __init__(self, means, log_scales, quats, logits, sh):
        super().__init__()
        self.means = torch.nn.Parameter(means)
        self.log_scales = torch.nn.Parameter(log_scales)
        self.quats = torch.nn.Parameter(quats)
        self.logits = torch.nn.Parameter(logits)
        self.sh = torch.nn.Parameter(sh)

    @classmethod
    def from_host(cls, scene, device="cuda"):
        t = lambda a: torch.as_tensor(a).to(device).contiguous()
        return cls(t(scene.means), t(scene.log_scales), t(scene.quats), t(scene.logits),
                   t(scene.sh))

    def forward(self, cam, cfg):
        return rasterize(self.means, torch.exp(self.log_scales), self.quats,
                         torch.sigmoid(self.logits), self.sh, cam, cfg)
