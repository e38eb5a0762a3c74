"""Comparison of HIP outputs with the FP64 oracle, photon by photon.

Bars (from the project's tolerance): fate and pixel agree on >= 99.99 % of
photons; hit positions of photons that reach the detector in both within
5e-3 mm.  Every disagreement must also be *explained*: the oracle says the
photon passed within a rounding distance of a decision boundary (a mirror or
facet edge, a pixel edge, or a roulette threshold), where FP32 and FP64 may
legitimately decide differently.
"""

import numpy as np

HIT_TOL_MM = 5e-3
# arrival times: FP32 path sums and group index, ~1e-5 ns at 30 ns; 2e-5 ns is
# 6e-3 mm of light path, the hit tolerance's counterpart
TIME_TOL_NS = 2e-5
MIN_AGREE = 0.9999
EDGE_EPS_MM = 2e-3
PIXEL_EPS_MM = 5e-3
ROULETTE_EPS = 1e-5


def to_np(t):
    return t.detach().cpu().numpy() if hasattr(t, "detach") else np.asarray(t)


def compare(gpu, ref, min_agree=MIN_AGREE, tol=HIT_TOL_MM, label=""):
    fate = to_np(gpu["fate"]).astype(np.int64)
    pix = to_np(gpu["pixel"]).astype(np.int64)
    xyz = to_np(gpu["hit_xyz"]).astype(np.float64)
    uv = to_np(gpu["hit_uv"]).astype(np.float64)
    ofate = ref["fate"].astype(np.int64)
    opix = ref["pixel"].astype(np.int64)
    n = len(ofate)
    assert len(fate) == n
    agree = (fate == ofate) & (pix == opix)
    explained = ((ref["edge_margin"] < EDGE_EPS_MM) | (ref["pixel_margin"] < PIXEL_EPS_MM)
                 | (ref["roulette_margin"] < ROULETTE_EPS))
    unexplained = np.where(~agree & ~explained)[0]
    on = agree & np.isin(fate, [0, 1])
    err = np.abs(xyz[on] - ref["hit_xyz"][on]).max() if on.any() else 0.0
    err_uv = np.abs(uv[on] - ref["hit_uv"][on]).max() if on.any() else 0.0
    off = ~np.isin(fate, [0, 1])
    report = {"n": n, "agree": float(agree.mean()), "disagree": int((~agree).sum()),
              "unexplained": int(len(unexplained)), "max_hit_err_mm": float(err), "max_uv_err_mm": float(err_uv)}
    err_t = 0.0
    if "hit_time" in gpu and "hit_time" in ref:
        t = to_np(gpu["hit_time"]).astype(np.float64)
        err_t = np.abs(t[on] - ref["hit_time"][on]).max() if on.any() else 0.0
        report["max_time_err_ns"] = float(err_t)
        assert np.all(np.isnan(t[off])), f"{label} hit_time set off the detector"
    msg = f"{label} {report} first unexplained ids {unexplained[:8]}"
    assert agree.mean() >= min_agree, msg
    assert len(unexplained) == 0, msg
    assert err <= tol and err_uv <= tol and err_t <= TIME_TOL_NS, msg
    assert np.all(np.isnan(xyz[off])) and np.all(pix[off] == -1), msg
    return report
