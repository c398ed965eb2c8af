"""torch.autograd.Function around the HIP rasterizer.

The forward and the backward are the library's kernels (gsr_rasterize_forward
/ gsr_rasterize_backward); for the raw training parameters the kernels also
apply the activations (exp of the log-scales, logistic function of the
opacity logits) and their chain rule.  torch holds the buffers.  Frozen layers (the paper's consecutive layer
training, Sec. 3.2) get zero gradient through `trainable_layers`.
"""
from __future__ import annotations

import torch

from . import rasterizer as rz


class RenderContext:
    """Reusable buffers of one rendering configuration (pair capacity,
    workspace, per-Gaussian accumulators for pruning)."""

    def __init__(self, trainable_layers=0xFFFFFFFF, track_activity=False, sync=True, timer=None,
                 grad_activity=True):
        self.state = None
        # track_activity: the backward updates max_contrib and, with
        # grad_activity, adds the gradient-norm activity into `activity`
        self.grad_activity = grad_activity
        self.timer = timer
        self.trainable_layers = int(trainable_layers)
        self.track_activity = track_activity
        self.sync = sync
        self.max_contrib = None
        self.activity = None
        self.densify_stats = None  # (grad_sum, count) [n] accumulators of density control, or None

    def reset_accumulators(self, n, device):
        self.max_contrib = torch.zeros(n, dtype=torch.float32, device=device)
        self.activity = torch.zeros(n, dtype=torch.float32, device=device)


class _RasterizeFn(torch.autograd.Function):
    @staticmethod
    def forward(ctx, mean, scale, quat, opacity, sh, layer, sh_degree, cams, views, rctx, raw):
        model = {"mean": mean.contiguous(), "scale": scale.contiguous(), "quat": quat.contiguous(),
                 "opacity": opacity.contiguous(), "sh": sh.contiguous(), "layer": layer, "sh_degree": sh_degree,
                 "raw": raw}
        rgb, alpha, st = rz.rasterize_forward(model, cams, views, state=rctx.state, sync=rctx.sync, timer=rctx.timer)
        rctx.state = st
        ctx.model = model
        ctx.cams, ctx.views, ctx.rctx, ctx.state = cams, views, rctx, st
        ctx.generation = st.generation
        return rgb, alpha

    @staticmethod
    def backward(ctx, g_rgb, g_alpha):
        rctx = ctx.rctx
        if ctx.state.generation != ctx.generation:
            # the context's buffers (records, sorted pairs, checkpoints) now
            # hold a later forward's: this graph's backward would be wrong
            raise RuntimeError("render state overwritten by a later forward on the same RenderContext before "
                               "this backward; use one RenderContext per forward awaiting its backward")
        mc = act = None
        if rctx.track_activity:
            n = ctx.model["mean"].shape[1]
            if rctx.max_contrib is None or rctx.max_contrib.numel() != n:
                rctx.reset_accumulators(n, ctx.model["mean"].device)
            mc, act = rctx.max_contrib, (rctx.activity if rctx.grad_activity else None)
        g = rz.rasterize_backward(ctx.model, ctx.cams, ctx.views, ctx.state,
                                  g_rgb.contiguous() if g_rgb is not None else None,
                                  g_alpha.contiguous() if g_alpha is not None else None,
                                  trainable=rctx.trainable_layers, max_contrib=mc, activity=act, timer=rctx.timer,
                                  densify=rctx.densify_stats)
        return g["mean"], g["scale"], g["quat"], g["opacity"], g["sh"], None, None, None, None, None, None


def rasterize(mean, scale, quat, opacity, sh, layer, sh_degree, cams, views, rctx=None):
    """Differentiable render of len(cams) equal-size views; activated inputs.
    Returns rgb [V,3,H,W] and alpha [V,H,W]."""
    if rctx is None:
        rctx = RenderContext()
    return _RasterizeFn.apply(mean, scale, quat, opacity, sh, layer, sh_degree, cams, views, rctx, False)


def render_params(params, layer, sh_degree, cams, views, rctx=None):
    """Render from raw parameters {mean, log_scale, quat, opacity_logit, sh};
    the kernels apply the activations, and the gradients are with respect to
    the raw parameters."""
    if rctx is None:
        rctx = RenderContext()
    return _RasterizeFn.apply(params["mean"], params["log_scale"], params["quat"], params["opacity_logit"],
                              params["sh"], layer, sh_degree, cams, views, rctx, True)


class _L1AlphaLossFn(torch.autograd.Function):
    @staticmethod
    def forward(ctx, rgb, alpha, target_rgb, target_alpha, bgs):
        loss, _, _ = rz.l1_alpha_loss(rgb, alpha, target_rgb, target_alpha, bgs)
        ctx.save_for_backward(rgb, alpha, target_rgb, target_alpha)
        ctx.bgs = bgs
        return loss.reshape(())

    @staticmethod
    def backward(ctx, g):
        rgb, alpha, target_rgb, target_alpha = ctx.saved_tensors
        _, g_rgb, g_a = rz.l1_alpha_loss(rgb, alpha, target_rgb, target_alpha, ctx.bgs, loss=False, grads=True,
                                         g_loss=g.reshape(1).contiguous())
        return g_rgb, g_a, None, None, None


def l1_alpha_loss(rgb, alpha, target_rgb, target_alpha, bgs):
    """mean|rgb - (target_rgb + (1 - target_alpha) bg)| + mean|alpha - target_alpha|
    (alpha-channel training with a random background, Sec. 3.2.1) on the
    library's fused kernels; differentiable in rgb and alpha."""
    return _L1AlphaLossFn.apply(rgb.contiguous(), alpha.contiguous(), target_rgb.contiguous(),
                                target_alpha.contiguous(), bgs)

