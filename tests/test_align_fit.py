"""The Adam alignment driver run on the oracle's FP64 loss and gradient (no GPU).

The targets are the oracle's hits at the seeded misalignment; starting from the
nominal geometry, the fit must land on that misalignment for every segment the
photons reach, and leave the others untouched (their gradient is zero).
"""

import numpy as np
import pytest
import torch

from paper_2309_12496_amd import inputs as I
from paper_2309_12496_amd.align import adam_fit


def _problem(orc, k, scene, n_tracks, per_track):
    rng = np.random.default_rng(1000 + k)
    src = I.batch_source(I.sample_tracks(rng, n_tracks), np.full(n_tracks, per_track))
    n, seed = n_tracks * per_track, I.SEED_BASE + k
    tp = I.perturbed_params(k, scene).astype(np.float64)
    tgt = orc.propagate(orc.Scene(scene, params=tp), src, n, seed, jacobian=True)
    on = np.isin(tgt["fate"], [orc.DETECTED, orc.QE_REJECTED])
    return src, n, seed, tp, tgt, on


def _oracle_loss_and_grad(orc, scene, src, n, seed, tgt, on, outlier_cut=None, floor=1e-3):
    """Mirror of the device driver's step: fused masked MSE, optional adaptive residual cut."""
    nseg = scene["params"].shape[0]
    state = {"cut": np.inf, "segment": None}

    def lg(p):
        r = orc.propagate(orc.Scene(scene, params=p.numpy()), src, n, seed, jacobian=True)
        cut = state["cut"] if outlier_cut else None
        loss, grad, _ = orc.mse_loss_and_grad(r, tgt["hit_uv"], on, nseg, residual_cut=cut)
        if outlier_cut:
            state["cut"] = outlier_cut * np.sqrt(loss) + floor if loss > 0 else np.inf
        state["segment"] = r["segment"]
        return torch.tensor(loss), torch.tensor(grad)
    return lg, state


def _lit(orc, tgt, on, nseg, min_photons):
    use = on & (tgt["segment"] >= 0)
    return np.bincount(tgt["segment"][use], minlength=nseg) >= min_photons


def test_adam_fit_recovers_analytic_misalignment(orc):
    """G4 analytic caps: tilts and radius of every imaged segment."""
    scene = I.scene_g4()
    src, n, seed, tp, tgt, on = _problem(orc, 4, scene, 1000, 10)
    lg, _ = _oracle_loss_and_grad(orc, scene, src, n, seed, tgt, on)
    p0 = torch.tensor(np.array(scene["params"], np.float64))
    p, losses = adam_fit(lg, p0, steps=300, lr=0.3)
    p = p.numpy()
    lit = _lit(orc, tgt, on, len(p), 50)
    assert lit.sum() >= 4
    assert losses[-1] < 1e-8 * losses[0]
    assert np.abs(p[lit, :2] - tp[lit, :2]).max() < 1e-8          # rad (sigma 5e-4)
    assert np.abs(p[lit, 2] - tp[lit, 2]).max() < 1e-2           # mm (sigma 5)
    assert np.array_equal(p[~lit], p0.numpy()[~lit])              # unseen segments do not move


def test_adam_fit_with_residual_cut_recovers_meshed_tilts(orc):
    """Meshed segments: photons that change facet between the two runs are cut; tilts are recovered.

    Uniform scaling about the pivot leaves facet normals unchanged, so a meshed
    segment's radius is nearly invisible to the photons; only tilts are fitted.
    """
    scene = I.scene_g5(seg_quads=(14, 23), flat_tiles=2)
    src, n, seed, tp, tgt, on = _problem(orc, 5, scene, 400, 10)
    lg, _ = _oracle_loss_and_grad(orc, scene, src, n, seed, tgt, on, outlier_cut=5.0)
    p0 = torch.tensor(np.array(scene["params"], np.float64))
    p, losses = adam_fit(lg, p0, steps=300, lr=0.3, free=(True, True, False, False, False, False))
    p = p.numpy()
    lit = _lit(orc, tgt, on, len(p), 20)
    assert lit.sum() >= 4
    assert np.abs(p[lit, :2] - tp[lit, :2]).max() < 1e-7
    assert np.array_equal(p[:, 2:], p0.numpy()[:, 2:])
