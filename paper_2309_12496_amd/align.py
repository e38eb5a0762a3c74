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
        ctx.mark_non_differentiable(fate)
        ctx.scene, ctx.src, ctx.n, ctx.seed = scene, src, n, seed
        return out["hit_uv"], fate

    @staticmethod
    def backward(ctx, grad_uv, grad_fate):
        # the adjoint reads the upstream gradient only for photons that reach the
        # pixel grid, so the NaN hits of the others never enter the sum
        grad, _ = R.adjoint(ctx.scene, ctx.src, ctx.seed, n=ctx.n, grad_uv=grad_uv)
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
# the fit's Adam steps (rich_fit_step) are taken in z = (p - p0) / scale.
PARAM_SCALE = (1e-3, 1e-3, 10.0, 1.0, 1.0, 1.0)
# Columns fitted by default.  The pivot shifts are left out: with tilts and
# radius free, a shift of an analytic segment's pivot is degenerate with them
# (only the centre of curvature and the radius are seen by the photons).
FIT_TILTS_RADII = (True, True, True, False, False, False)


_CAPTURE_STREAMS = {}


def _capture_stream(device):
    key = torch.device(device)
    if key not in _CAPTURE_STREAMS:
        _CAPTURE_STREAMS[key] = torch.cuda.Stream(key)
    return _CAPTURE_STREAMS[key]


def fit_alignment(scene, src, seed, targets, target_mask, params0=None, n=None, steps=600, lr=0.3, lr_final=1e-4,
                  free=FIT_TILTS_RADII, outlier_cut=5.0, cut_floor=1e-3, graph=True, betas=(0.9, 0.999), eps=1e-12):
    """Fit the segment parameters so that the photons' detector hits match `targets`.

    Every step is two library calls on the device: one fused adjoint launch
    that retraces the photons at the current parameters, forms the mean
    squared hit residual over the photons in `target_mask` that still reach
    the pixel grid and returns its gradient; then rich_fit_step, which takes
    the Adam step (cosine-decayed step size, normalised columns), records the
    loss, sets the residual cut and moves the mirrors (cap centres, instance
    transforms and top-level boxes recomputed on the device, nothing rebuilt
    on the host).  Photon ids key the random numbers, so the same photons are
    compared at every step.  With `graph` (the default) one step is captured
    once and replayed: the loop is launch-bound otherwise.

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
    cfg = R.fit_config(steps, lr, lr_final, PARAM_SCALE, free, betas, eps,
                       outlier_cut if outlier_cut else 0.0, cut_floor)
    cut = torch.full((1,), float("inf"), dtype=torch.float32, device=device) if outlier_cut else None
    grad = torch.empty((scene.n_segments, 6), dtype=torch.float32, device=device)
    loss = torch.empty(1, dtype=torch.float32, device=device)
    state = torch.zeros(3 * p0.numel() + 1, dtype=torch.float32, device=device)
    params = p0.clone()
    losses = torch.zeros(steps, dtype=torch.float32, device=device)
    scene.set_params(p0)

    def step():
        R.rich_propagate_adjoint(scene.handle, s, b, n, seed, 0, None, tgt, mask, cut, grad, loss)
        R.rich_fit_step(scene.handle, cfg, p0, grad, loss, state, params, losses, cut)

    if not graph or steps < 2:
        for _ in range(steps):
            step()
    else:
        # the first step runs on the stream the graph is captured on, so that
        # the library's per-stream work buffer is grown before the capture;
        # one such stream per device keeps one workspace slot per scene
        cs = _capture_stream(device)
        cs.wait_stream(torch.cuda.current_stream(device))
        with torch.cuda.stream(cs):
            step()
        torch.cuda.synchronize(device)
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g, stream=cs):
            step()
        for _ in range(steps - 1):
            g.replay()
    torch.cuda.synchronize(device)
    return params.clone(), losses
