"""Mirror alignment through the C ABI: a torch.autograd.Function over the segment parameters.

Forward runs rich_propagate at the given parameters and returns the detector
coordinates (u, v) of every photon (NaN for photons that do not reach the
pixel grid).  Backward runs rich_propagate_adjoint with the incoming gradient
of (u, v).  The derivative is the interior one: photons that would cross a
mirror or detector edge under a parameter change are not differentiated
through that change.
"""

from __future__ import annotations

import torch

from . import rich as R


class MirrorAlign(torch.autograd.Function):
    @staticmethod
    def forward(ctx, params, scene, src, n, seed):
        scene.set_params(params.detach())
        out = R.propagate(scene, src, n, seed)
        fate = out["fate"]
        ctx.scene, ctx.src, ctx.n, ctx.seed = scene, src, n, seed
        ctx.save_for_backward(fate)
        return out["hit_uv"], fate

    @staticmethod
    def backward(ctx, grad_uv, grad_fate):
        (fate,) = ctx.saved_tensors
        on = (fate == R.DETECTED) | (fate == R.QE_REJECTED)
        g = torch.where(on[:, None], grad_uv, torch.zeros_like(grad_uv)).nan_to_num(0.0)
        grad, _ = R.adjoint(ctx.scene, ctx.src, ctx.seed, n=ctx.n, grad_uv=g, mask=on.to(torch.uint8))
        return grad, None, None, None, None


def hits(params, scene, src, n, seed):
    """Differentiable (u, v) hits and fates at `params` ([n_segments, 6] float32 on the scene's GPU)."""
    return MirrorAlign.apply(params, scene, src, n, seed)


def alignment_loss(scene, src, seed, targets, mask, n=None, params=None):
    """Fused mean-squared hit residual and its gradient in one adjoint launch: (loss, grad)."""
    if params is not None:
        scene.set_params(params)
    grad, loss = R.adjoint(scene, src, seed, n=n, targets=targets, mask=mask)
    return loss, grad
