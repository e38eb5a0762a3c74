"""GPU parity of rich_set_mirror_params and rich_propagate_adjoint against the FP64 oracle."""

import numpy as np
import pytest

from paper_2309_12496_amd import inputs as I
from parity import compare, to_np

pytestmark = pytest.mark.gpu

GRAD_RTOL = 1e-3


@pytest.fixture(scope="module")
def R():
    import torch
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a GPU")
    from paper_2309_12496_amd import rich
    return rich


@pytest.fixture(scope="module")
def orc():
    from oracle import oracle
    return oracle


def grad_close(g, ref, rtol=GRAD_RTOL, label=""):
    """|g - g*| / |g*| <= rtol overall and per component with |g*_j| >= 1e-2 max|g*|."""
    g = np.asarray(g, np.float64).reshape(-1)
    ref = np.asarray(ref, np.float64).reshape(-1)
    norm = np.linalg.norm(ref)
    assert norm > 0, label
    rel = np.linalg.norm(g - ref) / norm
    big = np.abs(ref) >= 1e-2 * np.abs(ref).max()
    per = np.abs(g[big] - ref[big]) / np.abs(ref[big])
    assert rel <= rtol and per.max() <= rtol, f"{label} rel {rel:.2e} worst component {per.max():.2e}"
    return rel, per.max()


def c4_problem(orc, n_tracks, per_track, meshed=False):
    if meshed:
        scene = I.scene_g5(seg_quads=(30, 50), flat_tiles=4)
        k = 5
    else:
        scene = I.scene_g4()
        k = 4
    rng = np.random.default_rng(1000 + k)
    src = I.batch_source(I.sample_tracks(rng, n_tracks), np.full(n_tracks, per_track))
    n = n_tracks * per_track
    seed = I.SEED_BASE + k
    tgt_params = I.perturbed_params(k, scene)
    target = orc.propagate(orc.Scene(scene, params=tgt_params), src, n, seed)
    cur = orc.propagate(orc.Scene(scene), src, n, seed, jacobian=True)
    on = lambda r: np.isin(r["fate"], [orc.DETECTED, orc.QE_REJECTED])
    mask = on(target) & on(cur) & (target["edge_margin"] > 0.05) & (cur["edge_margin"] > 0.05)
    loss, grad, nuse = orc.mse_loss_and_grad(cur, target["hit_uv"], mask, scene["params"].shape[0])
    return {"scene": scene, "src": src, "n": n, "seed": seed, "target": target, "cur": cur, "mask": mask,
            "loss": loss, "grad": grad, "nuse": nuse, "tgt_params": tgt_params}


@pytest.fixture(scope="module")
def c4small(orc):
    return c4_problem(orc, 100, 1000)


def test_perturbed_forward_matches_oracle(R, orc, c4small):
    """rich_set_mirror_params moves the caps exactly as the oracle does."""
    p = c4small
    gs = R.Scene(p["scene"])
    gs.set_params(p["tgt_params"])
    out = R.propagate_batch(gs, p["src"], p["seed"], tune=R.tuning(256, 256, 4))
    compare(out, p["target"], label="G4 perturbed")


def test_fused_loss_gradient_matches_oracle(R, orc, c4small):
    p = c4small
    gs = R.Scene(p["scene"])
    grad, loss = R.adjoint(gs, p["src"], p["seed"], targets=p["target"]["hit_uv"], mask=p["mask"])
    assert gs.status() == 0
    assert abs(float(loss) / p["loss"] - 1) < 1e-4
    grad_close(to_np(grad), p["grad"], label="fused")


def test_upstream_gradient_mode_matches_oracle(R, orc, c4small):
    p = c4small
    rng = np.random.default_rng(3)
    gin = rng.normal(size=(p["n"], 2))
    gs = R.Scene(p["scene"])
    grad, _ = R.adjoint(gs, p["src"], p["seed"], grad_uv=gin, mask=p["mask"])
    cur = p["cur"]
    want = np.zeros_like(p["grad"])
    use = p["mask"] & (cur["segment"] >= 0)
    np.add.at(want, cur["segment"][use], np.einsum("nk,nkp->np", I.f32(gin)[use], cur["jac"][use]))
    grad_close(to_np(grad), want, label="grad_uv")


def test_gradient_is_deterministic(R, c4small):
    p = c4small
    gs = R.Scene(p["scene"])
    g1, l1 = R.adjoint(gs, p["src"], p["seed"], targets=p["target"]["hit_uv"], mask=p["mask"])
    g2, l2 = R.adjoint(gs, p["src"], p["seed"], targets=p["target"]["hit_uv"], mask=p["mask"])
    assert np.array_equal(to_np(g1), to_np(g2)) and float(l1) == float(l2)


def test_mask_forms_give_the_same_sums(R, c4small):
    """The mask's count and scan read it with 16-byte loads when it is aligned, bytes otherwise: a
    mask one byte into its buffer gives bit for bit the sums of the aligned one; a mask of all ones
    gives those of no mask."""
    import torch
    p = c4small
    gs = R.Scene(p["scene"])
    tg = np.nan_to_num(p["target"]["hit_uv"])
    mask = torch.as_tensor(p["mask"].astype(np.uint8), device="cuda")
    g0, l0 = R.adjoint(gs, p["src"], p["seed"], targets=tg, mask=mask)
    buf = torch.zeros(mask.numel() + 1, dtype=torch.uint8, device="cuda")
    buf[1:] = mask
    shifted = buf[1:]
    assert shifted.data_ptr() % 16 != 0
    g1, l1 = R.adjoint(gs, p["src"], p["seed"], targets=tg, mask=shifted)
    assert np.array_equal(to_np(g0), to_np(g1)) and np.array_equal(to_np(l0), to_np(l1))
    ones = torch.ones_like(mask)
    g2, l2 = R.adjoint(gs, p["src"], p["seed"], targets=tg, mask=ones)
    g3, l3 = R.adjoint(gs, p["src"], p["seed"], targets=tg, mask=None)
    assert np.array_equal(to_np(g2), to_np(g3)) and np.array_equal(to_np(l2), to_np(l3))
    assert gs.status() == 0


def test_gpu_finite_differences_fp32(R, c4small):
    """Central differences of the GPU's own FP32 forward loss agree with its adjoint at 1e-2."""
    import torch
    p = c4small
    gs = R.Scene(p["scene"])
    grad, loss0 = R.adjoint(gs, p["src"], p["seed"], targets=p["target"]["hit_uv"], mask=p["mask"])
    g = to_np(grad)
    tgt = torch.as_tensor(I.f32(p["target"]["hit_uv"]), device="cuda", dtype=torch.float32)
    m = torch.as_tensor(p["mask"], device="cuda")

    def L(params):
        gs.set_params(params)
        out = R.propagate_batch(gs, p["src"], p["seed"], tune=R.tuning(256, 256, 4))
        d = out["hit_uv"].double() - tgt.double()
        ok = m & torch.isfinite(d).all(1)
        return float((d[ok] ** 2).sum() / m.sum())

    p0 = p["scene"]["params"].astype(np.float64)
    steps = np.array([1e-5, 1e-5, 0.02, 0.01, 0.01, 0.01])
    k = int(np.argmax(np.abs(g).sum(1)))
    for j in range(6):
        pp, pm = p0.copy(), p0.copy()
        pp[k, j] += steps[j]
        pm[k, j] -= steps[j]
        fd = (L(pp) - L(pm)) / (2 * steps[j])
        assert abs(fd - g[k, j]) <= 1e-2 * np.abs(g[k]).max(), (k, j, fd, g[k, j])


def test_autograd_function_matches_fused_mode(R, c4small):
    import torch
    from paper_2309_12496_amd import align
    p = c4small
    gs = R.Scene(p["scene"])
    b, keep, n = R.make_batch(p["src"])
    # the autograd path uses single-source calls: check on the batch track with the most detector hits
    offs = np.asarray(p["src"]["offsets"], np.int64)
    per_track = np.add.reduceat(p["mask"].astype(np.int64), offs[:-1])
    kt = int(np.argmax(per_track))
    assert per_track[kt] > 50
    tr = p["src"]["tracks"][kt]
    src = I.point_source(origin=tr[0:3], direction=tr[3:6], beta=tr[7], length=tr[6])
    cnt = int(offs[kt + 1] - offs[kt])
    params = torch.tensor(I.f32(p["scene"]["params"]), device="cuda", dtype=torch.float32, requires_grad=True)
    uv, fate = align.hits(params, gs, src, cnt, p["seed"])
    on = (fate == 0) | (fate == 1)
    # the photons of this single-source call are ids 0..cnt-1, so the batch targets serve as arbitrary targets
    tgt = torch.as_tensor(I.f32(p["target"]["hit_uv"][offs[kt]:offs[kt + 1]]), device="cuda", dtype=torch.float32)
    use = on & torch.isfinite(tgt).all(1)
    assert int(use.sum()) > 20
    loss = ((uv[use] - tgt[use]) ** 2).sum() / use.sum()
    loss.backward()
    gref, lref = R.adjoint(gs, src, p["seed"], n=cnt, targets=tgt.nan_to_num(0.0), mask=use.to(torch.uint8))
    assert abs(float(loss.detach()) - float(lref)) <= 1e-5 * abs(float(lref))
    grad_close(params.grad.cpu().numpy(), to_np(gref), rtol=1e-5, label="autograd")


def test_c4_full_size_gradient(R, orc):
    """The 1e6-photon adjoint (1000 tracks x 1000 photons, 96 parameters) against the oracle."""
    cfg = I.config(4)
    p = c4_problem(orc, 1000, 1000)
    gs = R.Scene(cfg["scene"])
    grad, loss = R.adjoint(gs, cfg["source"], cfg["seed"], targets=p["target"]["hit_uv"], mask=p["mask"])
    assert gs.status() == 0
    assert abs(float(loss) / p["loss"] - 1) < 1e-4
    rel, worst = grad_close(to_np(grad), p["grad"], label="C4 full")
    print({"nuse": p["nuse"], "rel": rel, "worst": worst})
    # the forward of every photon at the autotuned launch shape the benchmark times
    out = R.propagate_batch(gs, p["src"], p["seed"])
    compare(out, p["cur"], label="C4 forward, autotuned shape")


def test_meshed_segments_forward_and_gradient(R, orc):
    """Meshed mirror segments moved through their instance transforms; gradient through facets."""
    p = c4_problem(orc, 150, 400, meshed=True)
    gs = R.Scene(p["scene"])
    gs.set_params(p["tgt_params"])
    out = R.propagate_batch(gs, p["src"], p["seed"], tune=R.tuning(256, 256, 4))
    compare(out, p["target"], label="G5-small perturbed")
    gs.set_params(p["scene"]["params"])
    grad, loss = R.adjoint(gs, p["src"], p["seed"], targets=p["target"]["hit_uv"], mask=p["mask"])
    assert gs.status() == 0
    assert abs(float(loss) / p["loss"] - 1) < 1e-4
    grad_close(to_np(grad), p["grad"], label="meshed")


def test_paths_over_two_segments_match_oracle(R, orc):
    """Every detected photon reflects off a spherical cap segment and then the flat mirror, itself a
    parametrised mesh (segment 16): the forward at a misalignment of all 17 segments, and the
    fused-loss gradient, which takes one contribution per reflection, against the oracle's sum of
    both segments' Jacobians."""
    scene = I.scene_g4_moving_flat()
    rng = np.random.default_rng(1006)
    src = I.batch_source(I.sample_tracks(rng, 200), np.full(200, 500))
    n, seed = 100_000, I.SEED_BASE + 4
    params = I.perturbed_params(4, scene)
    cur = orc.propagate(orc.Scene(scene, params=params), src, n, seed, jacobian=True)
    target = orc.propagate(orc.Scene(scene), src, n, seed)
    on = lambda r: np.isin(r["fate"], [orc.DETECTED, orc.QE_REJECTED])
    mask = on(target) & on(cur) & (target["edge_margin"] > 0.05) & (cur["edge_margin"] > 0.05)
    assert np.all(cur["segments"][mask, 1] == 16) and len(np.unique(cur["segments"][mask, 0])) == 16
    loss_ref, grad_ref, nuse = orc.mse_loss_and_grad(cur, target["hit_uv"], mask, 17)
    assert nuse > 5000 and np.all(grad_ref[16, [0, 1, 3, 4, 5]] != 0.0)
    gs = R.Scene(scene)
    gs.set_params(params)
    out = R.propagate_batch(gs, src, seed, tune=R.tuning(256, 256, 4))
    compare(out, cur, label="G4 moving flat, perturbed")
    grad, loss = R.adjoint(gs, src, seed, targets=np.nan_to_num(target["hit_uv"]), mask=mask)
    assert gs.status() == 0
    assert abs(float(loss) / loss_ref - 1) < 1e-4
    g = to_np(grad)
    # the flat's radius only scales the plane about a point on it: no effect (0 on both sides up to rounding)
    assert abs(g[16, 2]) <= 1e-6 * np.abs(g).max()
    keep = np.ones(grad_ref.shape, bool)
    keep[16, 2] = False
    grad_close(g[keep], grad_ref[keep], label="two segments per path")


def _cut_in_gap(r, lo_q=0.3, hi_q=0.7, clearance=5e-3):
    """A residual cut between two FP64 residuals far enough apart that FP32 cannot flip a photon."""
    s = np.sort(r[np.isfinite(r)])
    lo, hi = int(lo_q * len(s)), int(hi_q * len(s))
    gaps = s[lo + 1:hi + 1] - s[lo:hi]
    j = lo + int(np.argmax(gaps))
    assert s[j + 1] - s[j] > 2 * clearance
    return 0.5 * (s[j] + s[j + 1])


def test_dispersive_source_gradient_matches_oracle(R, orc):
    """The adjoint retraces photons whose wavelength and cone come from the dispersive generator."""
    scene = I.scene_g4()
    rng = np.random.default_rng(1004)
    src = I.with_dispersion(I.batch_source(I.sample_tracks(rng, 100), np.full(100, 1000)))
    n, seed = 100_000, I.SEED_BASE + 4
    tp = I.perturbed_params(4, scene)
    target = orc.propagate(orc.Scene(scene, params=tp), src, n, seed)
    cur = orc.propagate(orc.Scene(scene), src, n, seed, jacobian=True)
    on = lambda r: np.isin(r["fate"], [orc.DETECTED, orc.QE_REJECTED])
    mask = on(target) & on(cur) & (target["edge_margin"] > 0.05) & (cur["edge_margin"] > 0.05)
    loss_ref, grad_ref, nuse = orc.mse_loss_and_grad(cur, target["hit_uv"], mask, scene["params"].shape[0])
    assert nuse > 1000
    gs = R.Scene(scene)
    grad, loss = R.adjoint(gs, src, seed, targets=target["hit_uv"], mask=mask)
    assert abs(float(loss) / loss_ref - 1) < 1e-4
    grad_close(to_np(grad), grad_ref, label="dispersive")


def test_residual_cut_matches_oracle(R, orc, c4small):
    """Fused loss with dev_residual_cut: photons beyond the cut are left out of loss, count and gradient."""
    import torch
    p = c4small
    r = np.linalg.norm(p["cur"]["hit_uv"] - p["target"]["hit_uv"], axis=1)
    cut = _cut_in_gap(np.where(p["mask"], r, np.nan))
    loss_ref, grad_ref, nuse = orc.mse_loss_and_grad(p["cur"], p["target"]["hit_uv"], p["mask"],
                                                     p["scene"]["params"].shape[0], residual_cut=cut)
    assert 0.2 * p["nuse"] < nuse < 0.8 * p["nuse"]
    gs = R.Scene(p["scene"])
    grad, loss = R.adjoint(gs, p["src"], p["seed"], targets=p["target"]["hit_uv"], mask=p["mask"], residual_cut=cut)
    assert abs(float(loss) / loss_ref - 1) < 1e-4
    grad_close(to_np(grad), grad_ref, label="residual cut")
    # a NaN cut admits no photon; the cut is refused in upstream-gradient mode
    grad, loss = R.adjoint(gs, p["src"], p["seed"], targets=p["target"]["hit_uv"], mask=p["mask"],
                           residual_cut=float("nan"))
    assert float(loss) == 0.0 and not to_np(grad).any()
    b, keep, n = R.make_batch(p["src"])
    g = torch.zeros((gs.n_segments, 6), device="cuda")
    one = torch.ones(1, device="cuda")
    gin = torch.zeros((n, 2), device="cuda")
    with pytest.raises(R.RichError) as e:
        R.rich_propagate_adjoint(gs.handle, None, b, n, p["seed"], 0, gin, None, None, one, g, None)
    assert e.value.code == R.RICH_EINVAL


def _fit_problem(orc, k, scene, n_tracks, per_track, min_photons):
    rng = np.random.default_rng(1000 + k)
    src = I.batch_source(I.sample_tracks(rng, n_tracks), np.full(n_tracks, per_track))
    n, seed = n_tracks * per_track, I.SEED_BASE + k
    tp = I.perturbed_params(k, scene)
    tgt = orc.propagate(orc.Scene(scene, params=tp), src, n, seed, jacobian=True)
    on = np.isin(tgt["fate"], [orc.DETECTED, orc.QE_REJECTED])
    seg = tgt["segment"][on & (tgt["segment"] >= 0)]
    lit = np.bincount(seg, minlength=tp.shape[0]) >= min_photons
    return src, seed, tp.astype(np.float64), tgt, on, lit


def test_alignment_fit_recovers_analytic_misalignment(R, orc):
    """Adam through the fused device adjoint on the 16 imaged G4 segments lands where the oracle's FP64
    fit of the same problem lands (tests/golden/g4_fit_oracle.json), and on the seeded tilts and radii
    of every well-lit segment.

    Targets are the oracle's FP64 hits at the misalignment; every step moves the
    caps on the device and retraces the same 1e5 photons.  The two bottom corner
    cells send ~150 photons over a narrow range of angles, where tilt and radius
    nearly trade off: after 600 steps the FP64 fit itself is still 1.8e-6 and
    7.5e-6 rad from their seeded tilts (and 1.0 and 4.4 mm in radius), so for
    them the bar is the FP64 fit's own end point.
    """
    import json
    import os
    from paper_2309_12496_amd.align import fit_alignment
    scene = I.scene_g4()
    src, seed, tp, tgt, on, lit = _fit_problem(orc, 4, scene, 1000, 100, 100)
    gold = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "g4_fit_oracle.json")))
    assert np.array_equal(np.array(gold["target_params"]), tp)
    counts = np.array(gold["photons_per_segment"])
    assert lit.all() and np.array_equal(lit, counts >= 100)
    gs = R.Scene(scene)
    p, losses = fit_alignment(gs, src, seed, tgt["hit_uv"], on, steps=600, lr=0.3)
    p, losses = to_np(p).astype(np.float64), to_np(losses)
    assert gs.status() == 0
    assert losses[-1] < 1e-6 * losses[0], (losses[0], losses[-1])
    well = counts >= 300
    assert well.sum() == 14
    assert np.abs(p[well, :2] - tp[well, :2]).max() < 0.5e-6      # rad; perturbation sigma 0.5e-3
    assert np.abs(p[well, 2] - tp[well, 2]).max() < 0.1           # mm; perturbation sigma 5
    fp64 = np.array(gold["params"])
    print({"tilt_vs_fp64_fit": np.abs(p[:, :2] - fp64[:, :2]).max(axis=1).tolist(),
           "radius_vs_fp64_fit": np.abs(p[:, 2] - fp64[:, 2]).tolist()})
    assert np.abs(p[:, :2] - fp64[:, :2]).max() < 2e-6            # rad
    assert np.abs(p[:, 2] - fp64[:, 2]).max() < 1.0               # mm
    assert np.array_equal(p[:, 3:], np.asarray(scene["params"], np.float32)[:, 3:].astype(np.float64))


def test_alignment_fit_recovers_meshed_tilts(R, orc):
    """Meshed segments through their instance transforms, outliers cut on the device: tilts recovered."""
    from paper_2309_12496_amd.align import fit_alignment
    scene = I.scene_g5(seg_quads=(30, 50), flat_tiles=4)
    src, seed, tp, tgt, on, lit = _fit_problem(orc, 5, scene, 1000, 100, 100)
    assert lit.sum() >= 4
    gs = R.Scene(scene)
    p, losses = fit_alignment(gs, src, seed, tgt["hit_uv"], on, steps=600, lr=0.3,
                              free=(True, True, False, False, False, False))
    p = to_np(p).astype(np.float64)
    assert gs.status() == 0
    assert np.abs(p[lit, :2] - tp[lit, :2]).max() < 0.5e-6


def test_graph_captured_fit_matches_eager(R, orc):
    """The fit's step captured once in a graph and replayed gives exactly the eager trajectory, every step:
    two graph fits with eager work and synchronisations between them against one eager fit."""
    import torch
    from paper_2309_12496_amd.align import fit_alignment
    scene = I.scene_g4()
    src, seed, tp, tgt, on, lit = _fit_problem(orc, 4, scene, 300, 100, 50)
    gs = R.Scene(scene)
    p_e, l_e = fit_alignment(gs, src, seed, tgt["hit_uv"], on, steps=120, lr=0.3, graph=False)
    runs = []
    for rep in range(2):
        p_g, l_g = fit_alignment(gs, src, seed, tgt["hit_uv"], on, steps=120, lr=0.3, graph=True)
        runs.append((to_np(p_g).copy(), to_np(l_g).copy()))
        x = torch.ones(1 << 20, device="cuda").cumsum(0)   # eager work between the graph fits
        torch.cuda.synchronize()
        assert float(x[-1]) == float(1 << 20)
    for p_g, l_g in runs:
        assert np.array_equal(l_g, to_np(l_e)), np.flatnonzero(l_g != to_np(l_e))[:5]
        assert np.array_equal(p_g, to_np(p_e))
    assert gs.status() == 0


def test_adjoint_with_nothing_to_differentiate(R):
    """An all-zero mask, or no photons at all, overwrites the gradient and the loss with zeros
    (no division by a zero photon count)."""
    import torch
    scene = I.scene_g4()
    src = I.batch_source(I.sample_tracks(np.random.default_rng(1004), 8), np.full(8, 500))
    gs = R.Scene(scene)
    b, keep, n = R.make_batch(src)
    g = torch.full((gs.n_segments, 6), 5.0, device="cuda")
    loss = torch.full((1,), 5.0, device="cuda")
    tg = torch.zeros((n, 2), device="cuda")
    for mask, count in ((torch.zeros(n, dtype=torch.uint8, device="cuda"), n), (None, 0)):
        R.rich_propagate_adjoint(gs.handle, None, b, count, I.SEED_BASE + 4, 0, None, tg, mask, None, g, loss)
        torch.cuda.synchronize()
        assert not to_np(g).any() and float(loss) == 0.0
        g.fill_(5.0)
        loss.fill_(5.0)
    # upstream-gradient mode with a zero upstream gradient
    gin = torch.zeros((n, 2), device="cuda")
    R.rich_propagate_adjoint(gs.handle, None, b, n, I.SEED_BASE + 4, 0, gin, None, None, None, g, None)
    torch.cuda.synchronize()
    assert not to_np(g).any()
    assert gs.status() == 0


def test_fit_step_matches_oracle_adam(R, orc):
    """rich_fit_step over 60 seeded gradient and loss steps (two with no photon counted) against the
    oracle's FP64 Adam: moments, normalised coordinates, parameters, loss record, residual cut and
    the parameters left in the scene."""
    import torch
    from paper_2309_12496_amd.align import PARAM_SCALE
    scene = I.scene_g4()
    gs = R.Scene(scene)
    nseg = gs.n_segments
    rng = np.random.default_rng(41)
    T = 60
    grads = (rng.normal(size=(T, nseg, 6)) * 10.0 ** rng.uniform(-2, 2, size=(T, nseg, 6))).astype(np.float32)
    losses = rng.uniform(0.1, 10.0, size=T).astype(np.float32)
    losses[[5, 17]] = 0.0
    p0 = np.array(scene["params"], np.float32)
    free = (True, True, True, False, True, False)
    lr, lrf = 0.3, 1e-3
    ref = orc.adam_fit_steps(p0.astype(np.float64), grads.astype(np.float64), losses.astype(np.float64), T, lr, lrf,
                             PARAM_SCALE, free, outlier_cut=5.0, cut_floor=1e-3)
    cfg = R.fit_config(T, lr, lrf, PARAM_SCALE, free, outlier_cut=5.0, cut_floor=1e-3)
    dev = lambda a: torch.as_tensor(a, device="cuda").contiguous()
    p0_d, grad_d, loss_d = dev(p0), torch.empty((nseg, 6), device="cuda"), torch.empty(1, device="cuda")
    n_par = 6 * nseg
    state = torch.zeros(3 * n_par + 1, device="cuda")
    params = torch.empty((nseg, 6), device="cuda")
    rec = torch.zeros(T, device="cuda")
    cut = torch.full((1,), float("inf"), device="cuda")
    sc = np.asarray(PARAM_SCALE)
    # FP32 error scales: a moment's rounding is relative to the running mean of |g| (m itself can cancel
    # to ~0), and every step adds an error of ~1e-6 of its step size to z
    gabs = np.zeros((nseg, 6))
    cum = 0.0
    for t in range(T):
        g = np.where(np.asarray(free), grads[t].astype(np.float64) * sc, 0.0)
        gabs = 0.9 * gabs + 0.1 * np.abs(g)
        cum += lrf + 0.5 * (lr - lrf) * (1 + np.cos(np.pi * t / T))
        grad_d.copy_(dev(grads[t]))
        loss_d.fill_(float(losses[t]))
        R.rich_fit_step(gs.handle, cfg, p0_d, grad_d, loss_d, state, params, rec, cut)
        st = to_np(state).astype(np.float64)
        z, m, v = (st[k * n_par:(k + 1) * n_par].reshape(nseg, 6) for k in range(3))
        assert st[-1] == t + 1
        assert np.all(np.abs(m - ref["m"][t]) <= 1e-5 * gabs + 1e-30), t
        np.testing.assert_allclose(v, ref["v"][t], rtol=2e-5, atol=1e-30)
        ztol = 1e-5 * cum + 1e-6 * np.abs(ref["z"][t])
        assert np.all(np.abs(z - ref["z"][t]) <= ztol), (t, float((np.abs(z - ref["z"][t]) / ztol).max()))
        tol = ztol * sc + np.spacing(np.abs(p0))    # z's tolerance, then FP32 rounding of p
        err = np.abs(to_np(params) - ref["params"][t])
        assert np.all(err <= tol), (t, float((err / tol).max()))
        c = float(to_np(cut)[0])
        assert (np.isinf(c) and np.isinf(ref["cut"][t])) or abs(c - ref["cut"][t]) <= 1e-6 * ref["cut"][t]
    assert np.array_equal(to_np(rec), losses)
    # the scene holds the last parameters: propagating it equals propagating after setting them
    src = I.batch_source(I.sample_tracks(np.random.default_rng(1004), 200), np.full(200, 100))
    a = to_np(R.propagate_batch(gs, src, 7, tune=R.tuning(256, 256, 4))["hit_uv"])
    gs.set_params(params.clone())
    b = to_np(R.propagate_batch(gs, src, 7, tune=R.tuning(256, 256, 4))["hit_uv"])
    assert np.array_equal(a, b, equal_nan=True)
    # argument checks
    for bad in (R.fit_config(0, lr, lrf, PARAM_SCALE, free), R.fit_config(T, lr, lrf, PARAM_SCALE, free, betas=(1.0, 0.9)),
                R.fit_config(T, lr, lrf, (0.0,) + tuple(PARAM_SCALE[1:]), free),
                R.fit_config(T, float("nan"), lrf, PARAM_SCALE, free)):
        with pytest.raises(R.RichError) as e:
            R.rich_fit_step(gs.handle, bad, p0_d, grad_d, loss_d, state, None, None, None)
        assert e.value.code == R.RICH_EINVAL
    with pytest.raises(R.RichError) as e:
        R.rich_fit_step(gs.handle, cfg, None, grad_d, loss_d, state, None, None, None)
    assert e.value.code == R.RICH_EINVAL
    plain = R.Scene(I.scene_coincident(True))
    with pytest.raises(R.RichError) as e:
        R.rich_fit_step(plain.handle, cfg, p0_d, grad_d, loss_d, state, None, None, None)
    assert e.value.code == R.RICH_ESTATE


def test_prefiltered_source_gradient_matches_oracle(R, orc):
    """Fused-loss adjoint with the paper's pre-propagation efficiency filter: rejected photons do
    not count, kept ones are retraced with the surface roulettes off; loss and gradient match the
    oracle's."""
    scene = I.scene_g4()
    rng = np.random.default_rng(1004)
    src = I.with_prefilter(I.batch_source(I.sample_tracks(rng, 100), np.full(100, 1000)))
    n, seed = 100_000, I.SEED_BASE + 4
    target = orc.propagate(orc.Scene(scene, params=I.perturbed_params(4, scene)), src, n, seed)
    cur = orc.propagate(orc.Scene(scene), src, n, seed, jacobian=True)
    on = lambda r: np.isin(r["fate"], [orc.DETECTED, orc.QE_REJECTED])
    mask = on(target) & on(cur) & (target["edge_margin"] > 0.05) & (cur["edge_margin"] > 0.05)
    assert (cur["fate"] == orc.PREFILTERED).mean() > 0.5
    loss_ref, grad_ref, nuse = orc.mse_loss_and_grad(cur, target["hit_uv"], mask, scene["params"].shape[0])
    assert nuse > 500
    gs = R.Scene(scene)
    grad, loss = R.adjoint(gs, src, seed, targets=np.nan_to_num(target["hit_uv"]), mask=mask)
    assert abs(float(loss) / loss_ref - 1) < 1e-4
    grad_close(to_np(grad), grad_ref, label="pre-filtered")
    assert gs.status() == 0


def test_largest_segment_count(R, orc):
    """RICH_MAX_SEGMENTS (256) analytic segments, 1,536 parameters: more than one thread block's
    worth in the fit step, the widest accumulator rows in the adjoint.  The fused-loss gradient and
    five fit steps match the oracle."""
    import torch
    from paper_2309_12496_amd.align import PARAM_SCALE
    cells = I.grid_cells(16, 16)
    scene = I.scene_g1()
    scene["segments"] = I._segments_for_cells(cells)
    scene["params"] = I._nominal_params(len(cells))
    scene["caps"] = I._caps_for_cells(cells, list(range(len(cells))))
    assert len(cells) == R.MAX_SEGMENTS
    rng = np.random.default_rng(1007)
    src = I.batch_source(I.sample_tracks(rng, 200), np.full(200, 500))
    n, seed = 100_000, I.SEED_BASE + 7
    tp = I.perturbed_params(7, scene)
    target = orc.propagate(orc.Scene(scene, params=tp), src, n, seed)
    cur = orc.propagate(orc.Scene(scene), src, n, seed, jacobian=True)
    on = lambda r: np.isin(r["fate"], [orc.DETECTED, orc.QE_REJECTED])
    mask = on(target) & on(cur) & (target["edge_margin"] > 0.05) & (cur["edge_margin"] > 0.05)
    loss_ref, grad_ref, nuse = orc.mse_loss_and_grad(cur, target["hit_uv"], mask, len(cells))
    assert nuse > 1000 and np.count_nonzero(np.abs(grad_ref).sum(1)) > 8
    gs = R.Scene(scene)
    assert gs.n_segments == len(cells)
    grad, loss = R.adjoint(gs, src, seed, targets=np.nan_to_num(target["hit_uv"]), mask=mask)
    assert abs(float(loss) / loss_ref - 1) < 1e-4
    grad_close(to_np(grad), grad_ref, label="256 segments")
    # five fit steps on synthetic gradients, against the FP64 Adam
    T = 5
    gr = (rng.normal(size=(T, len(cells), 6))).astype(np.float32)
    ls = rng.uniform(0.5, 2.0, size=T).astype(np.float32)
    p0 = np.array(scene["params"], np.float32)
    free = (True, True, True, False, False, False)
    ref = orc.adam_fit_steps(p0.astype(np.float64), gr.astype(np.float64), ls.astype(np.float64), T, 0.3, 1e-3,
                             PARAM_SCALE, free, outlier_cut=5.0, cut_floor=1e-3)
    cfg = R.fit_config(T, 0.3, 1e-3, PARAM_SCALE, free, outlier_cut=5.0, cut_floor=1e-3)
    p0_d = torch.as_tensor(p0, device="cuda")
    state = torch.zeros(3 * p0.size + 1, device="cuda")
    params = torch.empty_like(p0_d)
    g_d, l_d, cut = torch.empty_like(p0_d), torch.empty(1, device="cuda"), torch.empty(1, device="cuda")
    for t in range(T):
        g_d.copy_(torch.as_tensor(gr[t], device="cuda"))
        l_d.fill_(float(ls[t]))
        R.rich_fit_step(gs.handle, cfg, p0_d, g_d, l_d, state, params, None, cut)
    z = to_np(state)[:p0.size].reshape(p0.shape).astype(np.float64)
    np.testing.assert_allclose(z, ref["z"][-1], rtol=1e-5, atol=1e-5)
    assert to_np(state)[-1] == T
    assert abs(float(to_np(cut)[0]) - ref["cut"][-1]) <= 1e-6 * ref["cut"][-1]
    assert gs.status() == 0
