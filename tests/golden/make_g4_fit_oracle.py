"""Writes g4_fit_oracle.json: where the oracle's FP64 alignment fit lands on the G4 fit problem.

The problem is the one the GPU fit test solves: the 4 x 4 analytic segmented
mirror (every segment imaged), 1000 tracks x 100 photons of the seeded track
sampler, targets = the oracle's hits at the seeded misalignment, the fit
started from the nominal geometry: 600 Adam steps (step size 0.3 decaying to
1e-4 along a cosine, normalised columns, tilts and radius free) on the fused
masked mean-squared hit residual, with the residual cut at 5 x the RMS
residual + 1e-3 mm.  Everything here runs in the oracle (FP64 C tracer and
Jacobians, FP64 Adam); the HIP library is not called.

    python tests/golden/make_g4_fit_oracle.py      # ~40 s on 8 threads
"""

import json
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from oracle import oracle as orc                      # noqa: E402
from paper_2309_12496_amd import inputs as I          # noqa: E402

# the fit's settings (paper_2309_12496_amd/align.py: PARAM_SCALE, FIT_TILTS_RADII)
PARAM_SCALE = (1e-3, 1e-3, 10.0, 1.0, 1.0, 1.0)
FREE = (True, True, True, False, False, False)
STEPS, LR, LR_FINAL, CUT, FLOOR = 600, 0.3, 1e-4, 5.0, 1e-3
K, N_TRACKS, PER_TRACK = 4, 1000, 100


def main():
    scene = I.scene_g4()
    rng = np.random.default_rng(1000 + K)
    src = I.batch_source(I.sample_tracks(rng, N_TRACKS), np.full(N_TRACKS, PER_TRACK))
    n, seed = N_TRACKS * PER_TRACK, I.SEED_BASE + K
    tp = I.perturbed_params(K, scene).astype(np.float64)
    tgt = orc.propagate(orc.Scene(scene, params=tp), src, n, seed, jacobian=True)
    on = np.isin(tgt["fate"], [orc.DETECTED, orc.QE_REJECTED])
    nseg = scene["params"].shape[0]
    adam = orc.AdamFit(np.array(scene["params"], np.float64), STEPS, LR, LR_FINAL, PARAM_SCALE, FREE,
                       outlier_cut=CUT, cut_floor=FLOOR)
    losses = []
    for _ in range(STEPS):
        r = orc.propagate(orc.Scene(scene, params=adam.p), src, n, seed, jacobian=True)
        loss, grad, _ = orc.mse_loss_and_grad(r, tgt["hit_uv"], on, nseg, residual_cut=adam.cut)
        losses.append(loss)
        adam.step(grad, loss)
    use = on & (tgt["segment"] >= 0)
    out = {"problem": "G4 fit: 1000 tracks x 100 photons, seed SEED_BASE + 4, 600 Adam steps",
           "params": adam.p.tolist(), "target_params": tp.tolist(),
           "photons_per_segment": np.bincount(tgt["segment"][use], minlength=nseg).tolist(),
           "loss_first": losses[0], "loss_last": losses[-1]}
    with open(os.path.join(HERE, "g4_fit_oracle.json"), "w") as f:
        json.dump(out, f, indent=1)
        f.write("\n")


if __name__ == "__main__":
    main()
