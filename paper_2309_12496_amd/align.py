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


# ------------------------------------------------------------------ alignment fit

# Normalising scale of each parameter column (tx, ty [rad], R, dx, dy, dz [mm]):
# Adam steps are taken in z = (p - p0) / scale.
PARAM_SCALE = (1e-3, 1e-3, 10.0, 1.0, 1.0, 1.0)
# Columns fitted by default.  The pivot shifts are left out: with tilts and
# radius free, a shift of an analytic segment's pivot is degenerate with them
# (only the centre of curvature and the radius are seen by the photons).
FIT_TILTS_RADII = (True, True, True, False, False, False)


class _Adam:
    """Adam state on one device; `step` uses tensor arithmetic only (the step
    count and the step size live on the device), so one step can be captured
    in a graph and replayed."""

    def __init__(self, p0, steps, lr, lr_final, scale, free, betas, eps):
        self.p0 = p0
        self.sc = torch.as_tensor(scale, dtype=p0.dtype, device=p0.device)[None, :]
        self.fm = torch.as_tensor(free, dtype=p0.dtype, device=p0.device)[None, :]
        self.z = torch.zeros_like(p0)
        self.m = torch.zeros_like(p0)
        self.v = torch.zeros_like(p0)
        self.p = p0.clone()                                            # p0 + z * scale
        self.t = torch.zeros((), dtype=p0.dtype, device=p0.device)     # steps taken
        self.k = torch.zeros(1, dtype=torch.long, device=p0.device)    # next loss slot
        self.losses = torch.zeros(steps, dtype=p0.dtype, device=p0.device)
        self.steps, self.lr, self.lr_final, self.betas, self.eps = steps, lr, lr_final, betas, eps

    def step(self, loss_and_grad):
        import math
        b1, b2 = self.betas
        loss, grad = loss_and_grad(self.p)
        self.losses.index_copy_(0, self.k, torch.as_tensor(loss).reshape(1).to(self.p0.dtype))
        self.k.add_(1)
        g = torch.as_tensor(grad).reshape(self.p0.shape).to(self.p0.dtype) * self.sc * self.fm
        self.m.mul_(b1).add_(g, alpha=1 - b1)
        self.v.mul_(b2).addcmul_(g, g, value=1 - b2)
        self.t.add_(1)
        size = self.lr_final + 0.5 * (self.lr - self.lr_final) * (1 + torch.cos(math.pi * (self.t - 1) / self.steps))
        mh = self.m / (1 - torch.pow(b1, self.t))
        vh = self.v / (1 - torch.pow(b2, self.t))
        self.z.sub_(size * mh / (vh.sqrt() + self.eps))
        torch.addcmul(self.p0, self.z, self.sc, out=self.p)


def adam_fit(loss_and_grad, p0, steps=300, lr=0.1, lr_final=1e-4, scale=PARAM_SCALE, free=FIT_TILTS_RADII,
             betas=(0.9, 0.999), eps=1e-12, graph=False):
    """Adam over the free columns of `p0` ([n_segments, 6]) with a cosine-decayed step size.

    `loss_and_grad(p)` returns (loss, dL/dp) as tensors on p0's device; the
    loop keeps everything there (no host synchronisation per step).  With
    `graph`, the first step runs eagerly and one step is captured in a GPU
    graph and replayed for the others (loss_and_grad must then launch its
    work on the current stream and reuse its buffers).  Returns the final
    parameters and the loss of every step (at the parameters before that
    step's update).
    """
    p0 = torch.as_tensor(p0)
    st = _Adam(p0, steps, lr, lr_final, scale, free, betas, eps)
    if not graph or steps < 2:
        for _ in range(steps):
            st.step(loss_and_grad)
        return st.p.clone(), st.losses
    st.step(loss_and_grad)
    torch.cuda.synchronize(p0.device)
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        st.step(loss_and_grad)
    for _ in range(steps - 1):
        g.replay()
    return st.p.clone(), st.losses


def fit_alignment(scene, src, seed, targets, target_mask, params0=None, n=None, steps=600, lr=0.3, lr_final=1e-4,
                  free=FIT_TILTS_RADII, outlier_cut=5.0, cut_floor=1e-3, graph=True):
    """Fit the segment parameters so that the photons' detector hits match `targets`.

    Every step moves the mirrors on the device (rich_set_mirror_params: cap
    centres, instance transforms and the top-level boxes are recomputed
    there, nothing is rebuilt on the host) and runs one fused adjoint launch
    that retraces the photons, forms the mean squared hit residual over the
    photons in `target_mask` that still reach the pixel grid, and returns its
    gradient.  Photon ids key the random numbers, so the same photons are
    compared at every step.  With `graph` (the default) one whole step, the
    parameter update, the adjoint, the cut and the Adam arithmetic, is
    captured once and replayed: the loop is launch-bound otherwise.

    Photons that cross onto another facet or segment than in the target run
    carry residual jumps that the interior derivative cannot remove; they
    would bias the fit.  With `outlier_cut` set, a step leaves out photons
    whose residual exceeds outlier_cut x the previous step's RMS residual
    + cut_floor (mm); the cut lives on the device, so the loop never waits
    for the host.  Returns (params, losses); the scene is left at the fitted
    parameters.
    """
    device = f"cuda:{scene.device}"
    if params0 is None:
        params0 = scene.params0
    p0 = torch.as_tensor(params0, dtype=torch.float32, device=device).contiguous()
    tgt = torch.as_tensor(targets, dtype=torch.float32, device=device).contiguous()
    mask = torch.as_tensor(target_mask, device=device).to(torch.uint8).contiguous()
    if src["kind"] == "batch":
        b, keep, nb = R.make_batch(src, device)
        s, n = None, nb if n is None else n
    else:
        s, keep = R.make_source(src, device)
        b = None
    if n is None:
        raise ValueError("n is required for single sources")
    cut = torch.full((1,), float("inf"), dtype=torch.float32, device=device) if outlier_cut else None
    grad = torch.empty((scene.n_segments, 6), dtype=torch.float32, device=device)
    loss = torch.empty(1, dtype=torch.float32, device=device)
    inf = torch.full_like(loss, float("inf"))

    def loss_and_grad(p):
        scene.set_params(p)
        R.rich_propagate_adjoint(scene.handle, s, b, n, seed, 0, None, tgt, mask, cut, grad, loss)
        if cut is not None:
            # no photon counted (loss exactly 0): open the cut again
            cut.copy_(torch.where(loss > 0, loss.sqrt() * outlier_cut + cut_floor, inf))
        return loss, grad

    p, losses = adam_fit(loss_and_grad, p0, steps=steps, lr=lr, lr_final=lr_final, free=free, graph=graph)
    scene.set_params(p)
    torch.cuda.synchronize(device)
    return p, losses
