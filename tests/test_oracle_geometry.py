"""Pins of the oracle's geometry and physics against closed forms, invariants and brute force."""

import copy
import math

import numpy as np
import pytest
from scipy import integrate

from paper_2309_12496_amd import inputs as I


def no_box(scene):
    s = copy.deepcopy(scene)
    s["box"] = None
    return s


def cap_only(scene):
    s = no_box(scene)
    s["rects"] = I._empty_rects()
    return s


# ---------------------------------------------------------------- primitives

def test_sphere_cap_from_centre_hits_at_radius(orc):
    sc = cap_only(I.scene_g1())
    S = orc.Scene(sc)
    centre, u0, e1, e2 = I.mirror_frame()
    rng = np.random.default_rng(0)
    a = rng.uniform(-590, 590, 50)
    b = rng.uniform(-490, 490, 50)
    targets = I.sphere_point(a, b)
    d = targets - centre
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    o = np.tile(centre, (50, 1))
    prim, t = orc.closest_hit(S, o, d)
    assert np.all(prim == 0)
    assert np.allclose(t, I.R_MIRROR, rtol=1e-13)


def test_sphere_cap_aperture_bounds(orc):
    """Rays just inside the aperture cell hit the cap, rays just outside miss it."""
    sc = cap_only(I.scene_g1())
    S = orc.Scene(sc)
    centre, _, _, _ = I.mirror_frame()
    inside = I.sphere_point(np.array([-599.999, 599.999]), np.array([0.0, 0.0]))
    outside = I.sphere_point(np.array([-600.001, 600.001]), np.array([0.0, 0.0]))
    for pts, want in ((inside, 0), (outside, -1)):
        dd = pts - centre
        dd /= np.linalg.norm(dd, axis=1, keepdims=True)
        p2, _ = orc.closest_hit(S, np.tile(centre, (2, 1)), dd)
        assert np.all(p2 == want)


def test_rect_and_box_distances(orc):
    sc = I.scene_g1()
    S = orc.Scene(sc)
    c, n, u, v, _ = I.flat_frame()
    # perpendicular approach to the flat mirror from 123 mm in front of its active side
    o = c + 123.0 * n + 50.0 * u - 70.0 * v
    prim, t = orc.closest_hit(S, o[None], -n[None])
    assert prim[0] == 1 and abs(t[0] - 123.0) < 1e-10
    # along +x from the origin the first surface is the box wall at x = 1500
    prim, t = orc.closest_hit(S, np.zeros((1, 3)), np.array([[1.0, 0, 0]]))
    assert prim[0] == 3 and abs(t[0] - 1500.0) < 1e-12
    prim, t = orc.closest_hit(S, np.zeros((1, 3)), np.array([[0, -1.0, 0]]))
    assert prim[0] == 3 and abs(t[0] - 1000.0) < 1e-12


def _soup_scene(tris, material=I.ABSORBER):
    s = no_box(I.scene_g2())
    s["meshes"] = [{"vertices": np.asarray(tris, float), "material": material, "segment": -1}]
    return s


def test_triangle_hit_at_known_barycentrics(orc):
    v = np.array([[[0.0, 0, 100], [50.0, 0, 100], [0.0, 40, 100]]])
    S = orc.Scene(_soup_scene(v))
    o = np.array([[10.0, 10.0, 0.0]])
    prim, t = orc.closest_hit(S, o, np.array([[0, 0, 1.0]]))
    assert prim[0] == S.tri_base and abs(t[0] - 100.0) < 1e-12
    prim, _ = orc.closest_hit(S, np.array([[40.0, 30.0, 0.0]]), np.array([[0, 0, 1.0]]))
    assert prim[0] == -1


def test_exact_tie_goes_to_lowest_index(orc):
    tri = np.array([[0.0, 0, 100], [50.0, 0, 100], [0.0, 40, 100]])
    S = orc.Scene(_soup_scene(np.stack([tri, tri[[0, 2, 1]], tri])))
    prim, _ = orc.closest_hit(S, np.array([[5.0, 5.0, 0.0]]), np.array([[0, 0, 1.0]]))
    assert prim[0] == S.tri_base


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_bvh_equals_brute_force_on_random_soups(orc, seed):
    rng = np.random.default_rng(seed)
    n = int(rng.integers(1, 2000))
    c = rng.uniform(-500, 500, size=(n, 1, 3))
    tris = c + rng.normal(scale=rng.uniform(1, 80), size=(n, 3, 3))
    S = orc.Scene(_soup_scene(tris))
    o = rng.uniform(-700, 700, size=(3000, 3))
    d = rng.normal(size=(3000, 3))
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    # half of the rays aimed at triangle vertices and edges
    k = rng.integers(0, n, size=1500)
    w = rng.dirichlet([1, 1, 1], size=1500) * (rng.random((1500, 1)) < 0.5) + 0.0
    w[w.sum(1) == 0] = [0.5, 0.5, 0.0]
    aim = np.einsum("kj,kjx->kx", w / w.sum(1, keepdims=True), tris[k])
    d[:1500] = aim - o[:1500]
    d[:1500] /= np.linalg.norm(d[:1500], axis=1, keepdims=True)
    p1, t1 = orc.closest_hit(S, o, d, use_bvh=True)
    p0, t0 = orc.closest_hit(S, o, d, use_bvh=False)
    assert np.array_equal(p0, p1)
    assert np.array_equal(t0[p0 >= 0], t1[p1 >= 0])


def test_bvh_equals_brute_force_on_meshed_rich(orc):
    sc = I.scene_g2()
    S = orc.Scene(sc)
    rng = np.random.default_rng(5)
    o = rng.uniform(I.BOX_LO + 1, I.BOX_HI - 1, size=(400, 3))
    d = rng.normal(size=(400, 3))
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    p1, t1 = orc.closest_hit(S, o, d, use_bvh=True)
    p0, t0 = orc.closest_hit(S, o, d, use_bvh=False)
    assert np.array_equal(p0, p1) and np.array_equal(t0, t1)


def test_closed_tessellated_box_is_watertight(orc):
    """Rays from inside a closed triangle box never escape, also when aimed at mesh vertices and edges."""
    box = I.box_mesh(I.BOX_LO, I.BOX_HI, 29)
    S = orc.Scene(_soup_scene(box))
    rng = np.random.default_rng(9)
    o = rng.uniform(I.BOX_LO + 10, I.BOX_HI - 10, size=(4000, 3))
    verts = box.reshape(-1, 3)
    aim = verts[rng.integers(0, len(verts), 2000)]
    k = rng.integers(0, len(box), 2000)
    edge_mid = 0.5 * (box[k, 0] + box[k, 1])
    tgt = np.concatenate([aim, edge_mid])
    d = tgt - o
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    prim, _ = orc.closest_hit(S, o, d)
    assert np.all(prim >= 0)


# ---------------------------------------------------------------- reflection and detection

def _flat_and_plane_scene():
    """A single flat mirror and the detector: reflection tested by the mirror-image construction."""
    s = no_box(I.scene_g1(unit_efficiencies=True))
    s["caps"] = I._empty_caps()
    return s


def test_reflection_obeys_mirror_image_law(orc):
    sc = _flat_and_plane_scene()
    c, n, u, v, r1 = I.flat_frame()
    det = sc["detector"]
    rng = np.random.default_rng(1)
    m = 200
    hit = c + rng.uniform(-200, 200, (m, 1)) * u + rng.uniform(-200, 200, (m, 1)) * v
    src_pt = c - 2000.0 * r1 + rng.normal(scale=20.0, size=(m, 3))
    d = hit - src_pt
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    res = orc.propagate(sc, I.explicit_source(src_pt, d, np.full(m, 400.0)), m, seed=3)
    ok = res["fate"] == orc.DETECTED
    assert ok.sum() > 150
    # image of the source across the mirror plane; the reflected ray continues from the image through hit
    img = src_pt - 2.0 * ((src_pt - c) @ n)[:, None] * n
    dd = hit - img
    dd /= np.linalg.norm(dd, axis=1, keepdims=True)
    tt = ((det["center"] - hit) @ det["normal"]) / (dd @ det["normal"])
    want = hit + tt[:, None] * dd
    assert np.allclose(res["hit_xyz"][ok], want[ok], atol=1e-8)
    # the distance to the detector is preserved by the unit-length reflected direction
    path = np.linalg.norm(want - hit, axis=1)
    assert np.allclose(np.linalg.norm(res["hit_xyz"][ok] - hit[ok], axis=1), path[ok], atol=1e-8)


def test_pixel_ids_and_dead_border(orc):
    sc = _flat_and_plane_scene()
    sc["rects"] = I._empty_rects()
    det = sc["detector"]
    p, nx = det["pitch"], det["nx"]
    half_active = 0.5 * nx * p
    ii = np.array([0, 1, 103, 207, 50])
    jj = np.array([0, 207, 104, 207, 3])
    uu = -half_active + (ii + 0.5) * p
    vv = -half_active + (jj + 0.5) * p
    # plus two points in the 0.24 mm dead border and one off the plane
    uu = np.concatenate([uu, [half_active + 0.1, 0.0, 301.0]])
    vv = np.concatenate([vv, [0.0, -half_active - 0.2, 0.0]])
    target = det["center"] + uu[:, None] * det["axis_u"] + vv[:, None] * det["axis_v"]
    o = target + 500.0 * det["normal"]
    d = np.tile(-det["normal"], (len(o), 1))
    res = orc.propagate(sc, I.explicit_source(o, d, np.full(len(o), 400.0)), len(o), seed=1)
    assert list(res["fate"][:5]) == [orc.DETECTED] * 5
    assert list(res["pixel"][:5]) == list(jj * nx + ii)
    assert np.allclose(res["hit_uv"][:5], np.stack([uu[:5], vv[:5]], 1), atol=1e-9)
    assert list(res["fate"][5:7]) == [orc.ABSORBED, orc.ABSORBED]
    assert list(res["pixel"][5:7]) == [-1, -1]
    assert res["fate"][7] == orc.ESCAPED


def test_back_faces_absorb(orc):
    sc = _flat_and_plane_scene()
    c, n, u, v, _ = I.flat_frame()
    det = sc["detector"]
    o = np.stack([c - 100 * n, det["center"] - 100 * det["normal"]])
    d = np.stack([n, det["normal"]])
    res = orc.propagate(sc, I.explicit_source(o, d, np.full(2, 400.0)), 2, seed=1)
    assert list(res["fate"]) == [orc.ABSORBED, orc.ABSORBED]


def test_parallel_mirrors_reach_max_bounces(orc):
    s = no_box(I.scene_g1(unit_efficiencies=True))
    s["caps"] = I._empty_caps()
    s["rects"] = {"material": np.array([0, 0], np.int32),
                  "center": np.array([[0, 0, 100.0], [0, 0, -100.0]]),
                  "normal": np.array([[0, 0, -1.0], [0, 0, 1.0]]),
                  "axis_u": np.array([[1.0, 0, 0], [1.0, 0, 0]]),
                  "axis_v": np.array([[0, 1.0, 0], [0, -1.0, 0]]),
                  "half": np.array([[1e4, 1e4], [1e4, 1e4]])}
    s["detector"]["center"] = np.array([0, 0, 5000.0])
    for mb in (0, 1, 16):
        s["max_bounces"] = mb
        d = np.array([[0, 0, 1.0], [0, 0.01, 1.0], [0.02, 0, -1.0]])
        d /= np.linalg.norm(d, axis=1, keepdims=True)
        res = orc.propagate(s, I.explicit_source(np.zeros((3, 3)), d, np.full(3, 400.0)), 3, seed=1)
        assert np.all(res["fate"] == orc.MAX_BOUNCES)
        assert np.all(res["n_bounce"] == mb)


def test_on_axis_ring_radius_closed_form(orc):
    """Focal-plane ring radius of a spherical mirror: r = (R/2) theta_c (Section 3 cone, Section 5.1 rings)."""
    res = orc.propagate(I.scene_t0(), I.point_source(), 20000, seed=7)
    assert np.all(res["fate"] == orc.DETECTED)
    r = np.hypot(res["hit_uv"][:, 0], res["hit_uv"][:, 1])
    want = 0.5 * I.R_MIRROR * math.acos(1 / 1.0014)
    assert abs(r.mean() / want - 1) < 2e-4
    assert r.std() / want < 1e-9     # on axis every photon lands on the same circle


# ---------------------------------------------------------------- C1 statistics and conservation

def _expect(f):
    lam0, lam1 = I.LAMBDA_MIN, I.LAMBDA_MAX
    norm = 1 / lam0 - 1 / lam1
    qx, qy = I.qe_table()
    rx, ry = I.reflectivity_table()
    fun = lambda l: f(np.interp(l, rx, ry), np.interp(l, qx, qy)) / (l * l) / norm
    return integrate.quad(fun, lam0, lam1, points=[400.0], epsabs=1e-14, epsrel=1e-13)[0]


def test_c1_fate_fractions_match_efficiency_integrals(orc):
    """With every photon reaching the detector geometrically, P(DETECTED) = E[R(l)^2 QE(l)] etc. (Section 4.3)."""
    cfg = I.config(1)
    n = cfg["n_photons"]
    res = orc.propagate(cfg["scene"], cfg["source"], n, cfg["seed"])
    cnt = orc.fate_counts(res)
    assert cnt.sum() == n
    p_det = _expect(lambda R, Q: R * R * Q)
    p_rej = _expect(lambda R, Q: R * R * (1 - Q))
    p_abs = _expect(lambda R, Q: 1 - R * R)
    assert abs(p_det - 0.10947375674) < 1e-9
    for k, p in ((orc.DETECTED, p_det), (orc.QE_REJECTED, p_rej), (orc.ABSORBED_MIRROR, p_abs)):
        sigma = math.sqrt(n * p * (1 - p))
        assert abs(int(cnt[k]) - n * p) < 5 * sigma, (k, cnt[k], n * p)
    assert cnt[orc.ABSORBED] == 0 and cnt[orc.ESCAPED] == 0 and cnt[orc.MAX_BOUNCES] == 0
    hist = orc.histogram(res, 208, 208)
    assert int(hist.sum()) == int(cnt[orc.DETECTED])
    # ring on the tilted geometry: within 0.1 % of (R/2) theta_c
    uv = res["hit_uv"][np.isin(res["fate"], [orc.DETECTED, orc.QE_REJECTED])]
    r = np.hypot(uv[:, 0] - uv[:, 0].mean(), uv[:, 1] - uv[:, 1].mean())
    assert abs(r.mean() / (0.5 * I.R_MIRROR * math.acos(1 / 1.0014)) - 1) < 1e-3


def test_hits_lie_on_detector_and_nan_elsewhere(orc):
    cfg = I.config(1)
    res = orc.propagate(cfg["scene"], cfg["source"], 5000, cfg["seed"])
    det = cfg["scene"]["detector"]
    on = np.isin(res["fate"], [orc.DETECTED, orc.QE_REJECTED])
    dist = (res["hit_xyz"][on] - det["center"]) @ det["normal"]
    assert np.all(np.abs(dist) < 1e-9)
    assert np.all(np.isnan(res["hit_xyz"][~on])) and np.all(res["pixel"][~on] == -1)


def test_split_ranges_are_identical(orc):
    cfg = I.config(1)
    S = orc.Scene(cfg["scene"])
    full = orc.propagate(S, cfg["source"], 3000, cfg["seed"], 500)
    a = orc.propagate(S, cfg["source"], 1234, cfg["seed"], 500)
    b = orc.propagate(S, cfg["source"], 1766, cfg["seed"], 1734)
    for k in ("fate", "pixel"):
        assert np.array_equal(full[k], np.concatenate([a[k], b[k]]))
    assert np.array_equal(full["hit_xyz"], np.concatenate([a["hit_xyz"], b["hit_xyz"]]), equal_nan=True)


# ---------------------------------------------------------------- errors

def test_rejects_subluminal_track(orc):
    with pytest.raises(ValueError):
        orc.propagate(I.scene_g1(), I.point_source(beta=0.99), 10, seed=1)


def test_rejects_non_finite_vertex(orc):
    s = I.scene_g2(sphere_quads=(4, 4))
    s["meshes"][0]["vertices"][0, 0, 0] = np.nan
    with pytest.raises(ValueError):
        orc.Scene(s)


# ---------------------------------------------------------------- pre-propagation filter (Section 4.3)

def test_prefilter_matches_roulette_in_law(orc):
    """Accept-reject of QE x R x R before propagation and roulette at the surfaces give the same
    detected-photon law when every photon meets two mirrors (C1): same detected fraction
    E[R^2 QE], same wavelength distribution of detected photons."""
    from scipy import stats
    cfg = I.config(1)
    n = 200_000
    S = orc.Scene(cfg["scene"])
    rou = orc.propagate(S, cfg["source"], n, cfg["seed"])
    pre = orc.propagate(S, I.with_prefilter(cfg["source"]), n, cfg["seed"])
    p = _expect(lambda R, Q: R * R * Q)
    sigma = math.sqrt(n * p * (1 - p))
    for res in (rou, pre):
        assert abs(int((res["fate"] == orc.DETECTED).sum()) - n * p) < 5 * sigma
    # pre-filter mode: photons are either rejected up front or detected (no roulette afterwards)
    assert set(np.unique(pre["fate"])) <= {orc.DETECTED, orc.PREFILTERED}
    _, _, lam = orc.generate(cfg["source"], n, cfg["seed"])
    ks = stats.ks_2samp(lam[rou["fate"] == orc.DETECTED], lam[pre["fate"] == orc.DETECTED])
    assert ks.pvalue > 1e-3
    # kept photons land where roulette-mode photons that reach the detector land
    on_r = np.isin(rou["fate"], [orc.DETECTED, orc.QE_REJECTED])
    kept = pre["fate"] == orc.DETECTED
    assert np.allclose(pre["hit_xyz"][kept & on_r], rou["hit_xyz"][kept & on_r])


def test_prefilter_rejects_non_mirror_material(orc):
    src = I.with_prefilter(I.point_source(), mirror_materials=(I.ABSORBER,))
    with pytest.raises(ValueError):
        orc.propagate(I.scene_g1(), src, 10, seed=1)


def test_coincident_copies_decide_by_listing_order(orc):
    """Whole-path version of the tie rule on two coincident fan-triangulated squares (mirror and
    absorber): the first-listed copy decides every photon, photons along shared and outer edges
    included; photons sent straight up come straight back down under their start point."""
    src = I.coincident_photons()
    n = len(src["lambda"])
    up = src["d"][:, 2] == 1.0
    for mirror_first, fate in ((True, orc.DETECTED), (False, orc.ABSORBED)):
        r = orc.propagate(I.scene_coincident(mirror_first), src, n, 1)
        assert np.all(r["fate"] == fate)
        if mirror_first:
            # detector axes: u along +x, v along -y
            assert np.array_equal(r["hit_uv"][up], np.column_stack([src["o"][up, 0], -src["o"][up, 1]]))
