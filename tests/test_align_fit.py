"""The alignment fit's optimiser (the oracle's FP64 Adam) run on the oracle's FP64 loss and gradient (no GPU).

The targets are the oracle's hits at the seeded misalignment; starting from the
nominal geometry, the fit must land on that misalignment for every segment the
photons reach, and leave the others untouched (their gradient is zero).
"""

import numpy as np
import pytest

from paper_2309_12496_amd import inputs as I
from paper_2309_12496_amd.align import FIT_TILTS_RADII, PARAM_SCALE


def _problem(orc, k, scene, n_tracks, per_track):
    rng = np.random.default_rng(1000 + k)
    src = I.batch_source(I.sample_tracks(rng, n_tracks), np.full(n_tracks, per_track))
    n, seed = n_tracks * per_track, I.SEED_BASE + k
    tp = I.perturbed_params(k, scene).astype(np.float64)
    tgt = orc.propagate(orc.Scene(scene, params=tp), src, n, seed, jacobian=True)
    on = np.isin(tgt["fate"], [orc.DETECTED, orc.QE_REJECTED])
    return src, n, seed, tp, tgt, on


def _oracle_fit(orc, scene, src, n, seed, tgt, on, steps=300, lr=0.3, free=FIT_TILTS_RADII, outlier_cut=None,
                floor=1e-3):
    """The device fit's loop on the oracle: fused masked MSE at the current parameters (with the
    previous step's residual cut), then one Adam step.  Returns (params, losses)."""
    nseg = scene["params"].shape[0]
    p0 = np.array(scene["params"], np.float64)
    adam = orc.AdamFit(p0, steps, lr, 1e-4, PARAM_SCALE, free, outlier_cut=outlier_cut, cut_floor=floor)
    losses = []
    for _ in range(steps):
        r = orc.propagate(orc.Scene(scene, params=adam.p), src, n, seed, jacobian=True)
        loss, grad, _ = orc.mse_loss_and_grad(r, tgt["hit_uv"], on, nseg,
                                              residual_cut=adam.cut if outlier_cut else None)
        losses.append(loss)
        adam.step(grad, loss)
    return adam.p, np.array(losses), p0


def _lit(orc, tgt, on, nseg, min_photons):
    use = on & (tgt["segment"] >= 0)
    return np.bincount(tgt["segment"][use], minlength=nseg) >= min_photons


def test_adam_fit_recovers_analytic_misalignment(orc):
    """G4 analytic caps: tilts and radius of all 16 segments (every one is imaged), 600 steps."""
    scene = I.scene_g4()
    src, n, seed, tp, tgt, on = _problem(orc, 4, scene, 2000, 10)
    p, losses, p0 = _oracle_fit(orc, scene, src, n, seed, tgt, on, steps=600)
    assert _lit(orc, tgt, on, len(p), 20).sum() == 16
    assert losses[-1] < 1e-8 * losses[0]
    # the bottom corner cells send ~40 photons each over a narrow range of
    # angles, so their radius and tilts converge more slowly
    assert np.abs(p[:, :2] - tp[:, :2]).max() < 1e-6             # rad (sigma 5e-4)
    assert np.abs(p[:, 2] - tp[:, 2]).max() < 0.5                # mm (sigma 5)
    well = _lit(orc, tgt, on, len(p), 60)
    assert well.sum() >= 12
    assert np.abs(p[well, :2] - tp[well, :2]).max() < 1e-8
    assert np.abs(p[well, 2] - tp[well, 2]).max() < 1e-2
    assert np.array_equal(p[:, 3:], p0[:, 3:])                    # pivot shifts are not fitted


def test_adam_fit_leaves_unseen_segments_in_place(orc):
    """G1's 600 mm flat mirror and 208-pixel detector image only the four central cells of the
    4 x 4 split: the other twelve get no photon, hence a zero gradient, and must not move."""
    scene = I.scene_g4()
    g1 = I.scene_g1()
    scene["rects"], scene["detector"] = g1["rects"], g1["detector"]
    src, n, seed, tp, tgt, on = _problem(orc, 4, scene, 500, 10)
    p, losses, p0 = _oracle_fit(orc, scene, src, n, seed, tgt, on, steps=100)
    seen = _lit(orc, tgt, on, len(p), 1)
    assert seen.sum() == 4 and losses[-1] < 1e-2 * losses[0]
    assert np.array_equal(p[~seen], p0[~seen])


def test_adam_fit_with_residual_cut_recovers_meshed_tilts(orc):
    """Meshed segments: photons that change facet between the two runs are cut; tilts are recovered.

    Uniform scaling about the pivot leaves facet normals unchanged, so a meshed
    segment's radius is nearly invisible to the photons; only tilts are fitted.
    """
    scene = I.scene_g5(seg_quads=(14, 23), flat_tiles=2)
    src, n, seed, tp, tgt, on = _problem(orc, 5, scene, 400, 10)
    p, losses, p0 = _oracle_fit(orc, scene, src, n, seed, tgt, on, free=(True, True, False, False, False, False),
                                outlier_cut=5.0)
    lit = _lit(orc, tgt, on, len(p), 20)
    assert lit.sum() >= 4
    assert np.abs(p[lit, :2] - tp[lit, :2]).max() < 1e-7
    assert np.array_equal(p[:, 2:], p0[:, 2:])
