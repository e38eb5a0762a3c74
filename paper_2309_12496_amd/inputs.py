"""Seeded synthetic inputs: RICH-like scenes, photon sources and track batches.

This module holds geometry and random draws only. None of the propagation
arithmetic (photon generation, intersection, reflection, detection, roulette,
gradients) lives here: the FP64 oracle and the HIP library each implement that
on their own and both consume the plain dictionaries built here.

Units are mm, nm and rad. z is the beam axis, y points up and the emitter sits
at the origin. The paper's geometry (the simplified LHCb RICH of Section 4.1)
is only described qualitatively and its GDML is not public, so the numbers
below are a synthetic stand-in with the same structure: a tilted spherical
focusing mirror, a flat secondary mirror tilted 30 degrees, a pixelated
detector plane on the focal surface, and an absorbing enclosure.

Every floating-point value that reaches the device (track data, parameters)
is rounded to FP32 first and stored back as float64, so both implementations
see bit-identical inputs.

Scene dictionary layout (all arrays float64 unless noted):
  materials : list of {"kind": MIRROR|ABSORBER, "refl_lambda": [n], "refl_value": [n]}
  segments  : {"pivot","u0","e1","e2": [K,3], "radius0": [K]}
              pivot = point on the sphere, u0 = unit vector pivot->centre at
              zero tilt, e1/e2 = fixed tilt axes (Rot = R_e2(ty) R_e1(tx)).
  params    : [K,6] = (tilt_x, tilt_y, radius, dx, dy, dz); FP32-representable
  caps      : {"segment","material": int32 [S], "origin","axis_a","axis_b": [S,3],
               "bounds": [S,4] = (a_lo, a_hi, b_lo, b_hi)}; the aperture cell is
              half-open in the fixed frame (origin, axis_a, axis_b)
  rects     : {"material": int32 [Q], "center","normal","axis_u","axis_v": [Q,3],
               "half": [Q,2]}; normal marks the active (reflecting) side
  meshes    : list of {"vertices": [T,3,3], "material": int, "segment": int}
              with the geometric normal (v1-v0)x(v2-v0) on the active side;
              segment >= 0 moves the mesh rigidly with that segment's params
  detector  : {"center","normal","axis_u","axis_v": [3], "half": [2],
               "pitch": float, "nx","ny": int, "qe_lambda","qe_value": [m]}
  box       : None or {"lo": [3], "hi": [3]} analytic absorbing enclosure
  max_bounces, t_min
"""

from __future__ import annotations

import numpy as np

MIRROR = 0
ABSORBER = 1

SEED_BASE = 2309124960          # Philox seed for config k is SEED_BASE + k
N_RADIATOR = 1.0014             # gas radiator index used by every config
LAMBDA_MIN, LAMBDA_MAX = 200.0, 600.0

# Mirror geometry (synthetic stand-in for the RICH optics of Section 4.1).
R_MIRROR = 8000.0
ALPHA = 0.15                    # tilt of the spherical mirror about x
PIVOT = np.array([0.0, 0.0, 2500.0])
APERTURE = (-600.0, 600.0, -500.0, 500.0)
FLAT_SIZE = 600.0
DET_PITCH = 2.88
BOX_LO = np.array([-1500.0, -1000.0, -1000.0])
BOX_HI = np.array([1500.0, 3000.0, 3000.0])


def f32(x):
    """Round to FP32 and return float64 holding the same value."""
    return np.asarray(x, dtype=np.float32).astype(np.float64)


# ---------------------------------------------------------------------------
# Efficiency tables (Section 4.3).  The measured curves exist only as a figure
# in the paper; these piecewise-linear stand-ins keep the stated ranges.
# ---------------------------------------------------------------------------

def qe_table():
    """Detector quantum efficiency vs wavelength: 0 at 200 nm, 0.30 peak at 400 nm, 0 at 600 nm."""
    return np.array([200.0, 400.0, 600.0]), np.array([0.0, 0.30, 0.0])


def reflectivity_table():
    """Mirror reflectivity falling linearly from 0.94 at 200 nm to 0.89 at 600 nm (Section 4.3)."""
    return np.array([200.0, 600.0]), np.array([0.94, 0.89])


def unit_table():
    """Reflectivity 1 at all wavelengths (closed-form geometric tests)."""
    return np.array([200.0, 600.0]), np.array([1.0, 1.0])


# ---------------------------------------------------------------------------
# Frames
# ---------------------------------------------------------------------------

def mirror_frame():
    u0 = np.array([0.0, np.sin(ALPHA), -np.cos(ALPHA)])
    e1 = np.array([1.0, 0.0, 0.0])
    e2 = np.array([0.0, np.cos(ALPHA), np.sin(ALPHA)])
    centre = PIVOT + R_MIRROR * u0
    return centre, u0, e1, e2


def flat_frame():
    """Flat mirror centred 2000 mm from the pivot along the central reflected ray."""
    r1 = np.array([0.0, np.sin(2 * ALPHA), -np.cos(2 * ALPHA)])
    c = PIVOT + 2000.0 * r1
    n = np.array([0.0, 0.5, np.sqrt(3.0) / 2.0])      # tilted 30 degrees from the beam axis
    u = np.array([1.0, 0.0, 0.0])
    v = np.cross(n, u)
    return c, n, u, v, r1


def detector_frame():
    """Detector on the focal surface: a further 2000 mm along the twice-reflected central ray."""
    cf, n, _, _, r1 = flat_frame()
    r2 = r1 - 2.0 * np.dot(r1, n) * n
    c = cf + 2000.0 * r2
    normal = -r2
    u = np.array([1.0, 0.0, 0.0])
    v = np.cross(normal, u)
    return c, normal, u, v


def sphere_point(a, b):
    """Point of the nominal mirror sphere above (a, b) in the mirror's tangent frame."""
    _, u0, e1, e2 = mirror_frame()
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    h = R_MIRROR - np.sqrt(R_MIRROR * R_MIRROR - a * a - b * b)
    return (PIVOT + a[..., None] * e1 + b[..., None] * e2 + h[..., None] * u0)


# ---------------------------------------------------------------------------
# Meshes
# ---------------------------------------------------------------------------

def _grid_tris(P, active_point=None, active_dir=None):
    """Split a (na+1, nb+1, 3) vertex grid into triangles, oriented to the active side.

    The active side is toward ``active_point`` when given, else along ``active_dir``.
    """
    v00 = P[:-1, :-1].reshape(-1, 3)
    v10 = P[1:, :-1].reshape(-1, 3)
    v11 = P[1:, 1:].reshape(-1, 3)
    v01 = P[:-1, 1:].reshape(-1, 3)
    t1 = np.stack([v00, v10, v11], axis=1)
    t2 = np.stack([v00, v11, v01], axis=1)
    tris = np.stack([t1, t2], axis=1).reshape(-1, 3, 3)
    nrm = np.cross(tris[:, 1] - tris[:, 0], tris[:, 2] - tris[:, 0])
    cen = tris.mean(axis=1)
    if active_point is not None:
        want = active_point[None, :] - cen
    else:
        want = np.broadcast_to(active_dir, cen.shape)
    flip = np.einsum("ij,ij->i", nrm, want) < 0
    tris[flip] = tris[flip][:, [0, 2, 1]]
    return np.ascontiguousarray(tris)


def sphere_mesh(a_lo, a_hi, b_lo, b_hi, na, nb):
    a = np.linspace(a_lo, a_hi, na + 1)
    b = np.linspace(b_lo, b_hi, nb + 1)
    A, B = np.meshgrid(a, b, indexing="ij")
    P = sphere_point(A, B)
    centre, _, _, _ = mirror_frame()
    return _grid_tris(P, active_point=centre)


def rect_mesh(c, n, u, v, half_u, half_v, nu, nv):
    s = np.linspace(-half_u, half_u, nu + 1)
    t = np.linspace(-half_v, half_v, nv + 1)
    S, T = np.meshgrid(s, t, indexing="ij")
    P = c + S[..., None] * u + T[..., None] * v
    return _grid_tris(P, active_dir=n)


def box_mesh(lo, hi, nq=29):
    """Six faces of the enclosure, nq x nq quads each, active side inward."""
    lo = np.asarray(lo, float)
    hi = np.asarray(hi, float)
    mid = 0.5 * (lo + hi)
    half = 0.5 * (hi - lo)
    out = []
    for ax in range(3):
        a1, a2 = (ax + 1) % 3, (ax + 2) % 3
        for side in (-1.0, 1.0):
            c = mid.copy()
            c[ax] = lo[ax] if side < 0 else hi[ax]
            n = np.zeros(3)
            n[ax] = -side
            u = np.zeros(3)
            u[a1] = 1.0
            v = np.zeros(3)
            v[a2] = 1.0
            out.append(rect_mesh(c, n, u, v, half[a1], half[a2], nq, nq))
    return np.concatenate(out, axis=0)


# ---------------------------------------------------------------------------
# Scenes
# ---------------------------------------------------------------------------

def _materials(unit_reflectivity=False):
    lam, val = unit_table() if unit_reflectivity else reflectivity_table()
    return [
        {"kind": MIRROR, "refl_lambda": lam, "refl_value": val},
        {"kind": ABSORBER, "refl_lambda": np.array([200.0, 600.0]), "refl_value": np.zeros(2)},
    ]


def _detector(n_pix, unit_qe=False):
    c, n, u, v = detector_frame()
    lam, val = qe_table()
    if unit_qe:
        val = np.ones_like(val)
    half = 0.5 * max(FLAT_SIZE, n_pix * DET_PITCH)
    return {"center": c, "normal": n, "axis_u": u, "axis_v": v,
            "half": np.array([half, half]), "pitch": DET_PITCH, "nx": n_pix, "ny": n_pix,
            "qe_lambda": lam, "qe_value": val}


def _segments_for_cells(cells):
    """One segment per aperture cell: pivot at the cell centre on the nominal sphere."""
    centre, _, e1, e2 = mirror_frame()
    piv, u0s = [], []
    for (a0, a1, b0, b1) in cells:
        p = sphere_point(0.5 * (a0 + a1), 0.5 * (b0 + b1))
        piv.append(p)
        u0s.append((centre - p) / np.linalg.norm(centre - p))
    k = len(cells)
    return {"pivot": np.array(piv), "u0": np.array(u0s),
            "e1": np.tile(e1, (k, 1)), "e2": np.tile(e2, (k, 1)),
            "radius0": np.full(k, R_MIRROR)}


def _nominal_params(k):
    p = np.zeros((k, 6))
    p[:, 2] = R_MIRROR
    return p


def _empty_caps():
    return {"segment": np.zeros(0, np.int32), "material": np.zeros(0, np.int32),
            "origin": np.zeros((0, 3)), "axis_a": np.zeros((0, 3)), "axis_b": np.zeros((0, 3)),
            "bounds": np.zeros((0, 4))}


def _empty_rects():
    return {"material": np.zeros(0, np.int32), "center": np.zeros((0, 3)), "normal": np.zeros((0, 3)),
            "axis_u": np.zeros((0, 3)), "axis_v": np.zeros((0, 3)), "half": np.zeros((0, 2))}


def _flat_rect(half_u=0.5 * FLAT_SIZE, v_range=(-0.5 * FLAT_SIZE, 0.5 * FLAT_SIZE)):
    """The flat mirror in G1's flat plane: |u| <= half_u, v in v_range about G1's flat centre."""
    c, n, u, v, _ = flat_frame()
    cc = c + 0.5 * (v_range[0] + v_range[1]) * v
    hv = 0.5 * (v_range[1] - v_range[0])
    return {"material": np.array([MIRROR], np.int32), "center": cc[None], "normal": n[None],
            "axis_u": u[None], "axis_v": v[None], "half": np.array([[half_u, hv]])}


# G4's flat mirror and detector.  G1's 600 x 600 mm flat mirror intercepts the
# reflected light of the four central cells of a 4 x 4 split only: the beams
# of the outer cells land beyond its edges (the bottom row's below the lower
# edge, which cannot move down without shadowing the forward beam).  G4 keeps
# G1's flat plane but extends the mirror to 1400 mm along u and from 500 mm
# below to 800 mm above G1's flat centre along v, with the large scene's
# 512 x 512-pixel detector, so that every segment sends light to the detector.
# The lower edge then shadows the part of the forward cone above ~0.19 rad
# upward; those photons meet the flat mirror's back face and are absorbed.
G4_FLAT_HALF_U = 700.0
G4_FLAT_V = (-500.0, 800.0)
G4_DET_PIXELS = 512


def _caps_for_cells(cells, segment_ids):
    _, _, e1, e2 = mirror_frame()
    s = len(cells)
    return {"segment": np.asarray(segment_ids, np.int32), "material": np.full(s, MIRROR, np.int32),
            "origin": np.tile(PIVOT, (s, 1)), "axis_a": np.tile(e1, (s, 1)),
            "axis_b": np.tile(e2, (s, 1)), "bounds": np.array(cells, dtype=np.float64)}


def grid_cells(n_cols, n_rows, aperture=APERTURE):
    a_lo, a_hi, b_lo, b_hi = aperture
    da = (a_hi - a_lo) / n_cols
    db = (b_hi - b_lo) / n_rows
    cells = []
    for r in range(n_rows):
        for c in range(n_cols):
            cells.append((a_lo + c * da, a_lo + (c + 1) * da, b_lo + r * db, b_lo + (r + 1) * db))
    return cells


def scene_g1(unit_efficiencies=False):
    """Analytic RICH geometry: one spherical cap, flat mirror, 208x208-pixel detector, box."""
    cells = [APERTURE]
    return {
        "name": "G1-analytic",
        "materials": _materials(unit_efficiencies),
        "segments": _segments_for_cells(cells),
        "params": _nominal_params(1),
        "caps": _caps_for_cells(cells, [0]),
        "rects": _flat_rect(),
        "meshes": [],
        "detector": _detector(208, unit_qe=unit_efficiencies),
        "box": {"lo": BOX_LO.copy(), "hi": BOX_HI.copy()},
        "max_bounces": 16,
        "t_min": 1e-2,
    }


def scene_g1_segment_override(scene, params):
    s = dict(scene)
    s["params"] = np.array(params, dtype=np.float64)
    return s


def scene_g2(sphere_quads=(346, 289), box_quads=29):
    """G1 as triangle meshes: sphere 346x289 quads, flat 2 triangles, box 6x29x29 quads.

    The detector stays an analytic plane.  The sphere mesh is fixed (segment -1).
    """
    na, nb = sphere_quads
    sph = sphere_mesh(*APERTURE, na, nb)
    c, n, u, v, _ = flat_frame()
    flat = rect_mesh(c, n, u, v, 0.5 * FLAT_SIZE, 0.5 * FLAT_SIZE, 1, 1)
    box = box_mesh(BOX_LO, BOX_HI, box_quads)
    return {
        "name": "G2-meshed",
        "materials": _materials(),
        "segments": {"pivot": np.zeros((0, 3)), "u0": np.zeros((0, 3)), "e1": np.zeros((0, 3)),
                     "e2": np.zeros((0, 3)), "radius0": np.zeros(0)},
        "params": np.zeros((0, 6)),
        "caps": _empty_caps(),
        "rects": _empty_rects(),
        "meshes": [
            {"vertices": sph, "material": MIRROR, "segment": -1},
            {"vertices": flat, "material": MIRROR, "segment": -1},
            {"vertices": box, "material": ABSORBER, "segment": -1},
        ],
        "detector": _detector(208),
        "box": None,
        "max_bounces": 16,
        "t_min": 1e-2,
    }


def scene_g4():
    """G1's sphere split into 4 columns x 4 rows of analytic segments (300 x 250 mm), with the
    enlarged flat mirror and the 512 x 512-pixel detector that image every segment."""
    cells = grid_cells(4, 4)
    s = scene_g1()
    s["name"] = "G4-segmented"
    s["segments"] = _segments_for_cells(cells)
    s["params"] = _nominal_params(len(cells))
    s["caps"] = _caps_for_cells(cells, list(range(len(cells))))
    s["rects"] = _flat_rect(G4_FLAT_HALF_U, G4_FLAT_V)
    s["detector"] = _detector(G4_DET_PIXELS)
    return s


# The flat mirror of scene_g4_moving_flat as a segment: pivot at its centre,
# axis along its normal, tilt axes along its u and v; "radius" R scales the
# mirror about its centre by R / FLAT_R0.
FLAT_R0 = 2000.0


def scene_g4_moving_flat():
    """G4 with its flat mirror turned into a parametrised mesh (segment 16, two triangles).

    Every detected photon reflects off one spherical cap and then the flat, so
    its hit depends on two segments' parameters.
    """
    s = scene_g4()
    s["name"] = "G4-moving-flat"
    r = s["rects"]
    c, n, u, v = r["center"][0], r["normal"][0], r["axis_u"][0], r["axis_v"][0]
    hu, hv = r["half"][0]
    seg = s["segments"]
    s["segments"] = {"pivot": np.vstack([seg["pivot"], c]), "u0": np.vstack([seg["u0"], n]),
                     "e1": np.vstack([seg["e1"], u]), "e2": np.vstack([seg["e2"], v]),
                     "radius0": np.append(seg["radius0"], FLAT_R0)}
    p = np.zeros((17, 6))
    p[:16] = s["params"]
    p[16, 2] = FLAT_R0
    s["params"] = p
    s["rects"] = _empty_rects()
    s["meshes"] = [{"vertices": rect_mesh(c, n, u, v, hu, hv, 1, 1), "material": MIRROR, "segment": 16}]
    return s


def scene_g5(seg_quads=(137, 228), flat_tiles=16, n_pix=512):
    """4 rows x 8 columns of meshed mirror segments, 16x16 flat tiles, box mesh, 512x512 px."""
    cells = grid_cells(8, 4)
    meshes = []
    na, nb = seg_quads
    for k, (a0, a1, b0, b1) in enumerate(cells):
        meshes.append({"vertices": sphere_mesh(a0, a1, b0, b1, na, nb), "material": MIRROR, "segment": k})
    c, n, u, v, _ = flat_frame()
    step = FLAT_SIZE / flat_tiles
    for i in range(flat_tiles):
        for j in range(flat_tiles):
            cc = c + (-0.5 * FLAT_SIZE + (i + 0.5) * step) * u + (-0.5 * FLAT_SIZE + (j + 0.5) * step) * v
            meshes.append({"vertices": rect_mesh(cc, n, u, v, 0.5 * step, 0.5 * step, 1, 1),
                           "material": MIRROR, "segment": -1})
    meshes.append({"vertices": box_mesh(BOX_LO, BOX_HI, 29), "material": ABSORBER, "segment": -1})
    return {
        "name": "G5-large",
        "materials": _materials(),
        "segments": _segments_for_cells(cells),
        "params": _nominal_params(len(cells)),
        "caps": _empty_caps(),
        "rects": _empty_rects(),
        "meshes": meshes,
        "detector": _detector(n_pix),
        "box": None,
        "max_bounces": 16,
        "t_min": 1e-2,
    }


def scene_t0(detector_half=600.0, n_pix=400, pitch=3.0):
    """On-axis test scene: untilted mirror (pivot z=2000, centre z=-6000) and a detector
    plane at z=-2000 facing +z, i.e. on the focal plane R/2 in front of the mirror.
    Reflectivity and QE are 1, so every photon reaching the plane is detected."""
    R = R_MIRROR
    pivot = np.array([0.0, 0.0, 2000.0])
    u0 = np.array([0.0, 0.0, -1.0])
    e1 = np.array([1.0, 0.0, 0.0])
    e2 = np.array([0.0, 1.0, 0.0])
    seg = {"pivot": pivot[None], "u0": u0[None], "e1": e1[None], "e2": e2[None], "radius0": np.array([R])}
    caps = {"segment": np.array([0], np.int32), "material": np.array([MIRROR], np.int32),
            "origin": pivot[None], "axis_a": e1[None], "axis_b": e2[None],
            "bounds": np.array([[-300.0, 300.0, -300.0, 300.0]])}
    det = {"center": np.array([0.0, 0.0, -2000.0]), "normal": np.array([0.0, 0.0, 1.0]),
           "axis_u": np.array([1.0, 0.0, 0.0]), "axis_v": np.array([0.0, 1.0, 0.0]),
           "half": np.array([detector_half, detector_half]), "pitch": pitch, "nx": n_pix, "ny": n_pix,
           "qe_lambda": np.array([200.0, 600.0]), "qe_value": np.array([1.0, 1.0])}
    return {
        "name": "T0-on-axis",
        "materials": _materials(unit_reflectivity=True),
        "segments": seg,
        "params": _nominal_params(1),
        "caps": caps,
        "rects": _empty_rects(),
        "meshes": [],
        "detector": det,
        "box": {"lo": np.array([-3000.0, -3000.0, -3000.0]), "hi": np.array([3000.0, 3000.0, 3000.0])},
        "max_bounces": 16,
        "t_min": 1e-2,
    }


def scene_t1(radius=2000.0, detector_z=100.0, n_pix=200, pitch=3.0):
    """Isochronism test scene: a concave mirror of radius `radius` centred on the
    origin (pivot at z = -radius, facing +z) and a detector plane at
    z = detector_z facing -z.  Light from a point at the centre of curvature
    comes back through it after one reflection, so every photon's path is
    2 radius + detector_z / cos(angle to the axis).  Reflectivity and QE are 1."""
    pivot = np.array([0.0, 0.0, -radius])
    u0 = np.array([0.0, 0.0, 1.0])
    e1 = np.array([1.0, 0.0, 0.0])
    e2 = np.array([0.0, 1.0, 0.0])
    seg = {"pivot": pivot[None], "u0": u0[None], "e1": e1[None], "e2": e2[None], "radius0": np.array([radius])}
    caps = {"segment": np.array([0], np.int32), "material": np.array([MIRROR], np.int32),
            "origin": pivot[None], "axis_a": e1[None], "axis_b": e2[None],
            "bounds": np.array([[-300.0, 300.0, -300.0, 300.0]])}
    half = 0.5 * n_pix * pitch
    det = {"center": np.array([0.0, 0.0, detector_z]), "normal": np.array([0.0, 0.0, -1.0]),
           "axis_u": np.array([1.0, 0.0, 0.0]), "axis_v": np.array([0.0, 1.0, 0.0]),
           "half": np.array([half, half]), "pitch": pitch, "nx": n_pix, "ny": n_pix,
           "qe_lambda": np.array([200.0, 600.0]), "qe_value": np.array([1.0, 1.0])}
    params = np.zeros((1, 6))
    params[0, 2] = radius
    return {
        "name": "T1-isochronous",
        "materials": _materials(unit_reflectivity=True),
        "segments": seg,
        "params": params,
        "caps": caps,
        "rects": _empty_rects(),
        "meshes": [],
        "detector": det,
        "box": {"lo": np.array([-3000.0, -3000.0, -3000.0]), "hi": np.array([3000.0, 3000.0, 3000.0])},
        "max_bounces": 16,
        "t_min": 1e-2,
    }


def scene_coincident(mirror_first, half=200.0, plane_z=500.0, detector_z=100.0, n_pix=200, pitch=3.0):
    """Tie and watertightness scene: two copies of one flat square at z = plane_z, a fan of eight
    triangles around its centre facing -z, one copy a mirror and one an absorber, listed mirror
    first or absorber first; the mirror copy also carries zero-area triangles (three collinear
    vertices along a fan edge, a repeated vertex).  A detector at z = detector_z faces +z;
    reflectivity and QE are 1.  Every photon leaving from between them toward the square meets
    both copies at exactly the same distance, so the first-listed copy (lower primitive index)
    decides its fate."""
    c = np.array([0.0, 0.0, plane_z])
    ring = [(half, 0.0), (half, half), (0.0, half), (-half, half), (-half, 0.0), (-half, -half),
            (0.0, -half), (half, -half)]
    ring = [np.array([x, y, plane_z]) for x, y in ring]
    fan = np.array([[c, ring[(k + 1) % 8], ring[k]] for k in range(8)])   # normals along -z
    degenerate = np.array([[c, c + [0.5 * half, 0.0, 0.0], c + [half, 0.0, 0.0]],
                           [ring[2], ring[2], c]])
    mirror = {"vertices": np.concatenate([fan, degenerate]), "material": MIRROR, "segment": -1}
    absorber = {"vertices": fan.copy(), "material": ABSORBER, "segment": -1}
    h = 0.5 * n_pix * pitch
    det = {"center": np.array([0.0, 0.0, detector_z]), "normal": np.array([0.0, 0.0, 1.0]),
           "axis_u": np.array([1.0, 0.0, 0.0]), "axis_v": np.array([0.0, -1.0, 0.0]),
           "half": np.array([h, h]), "pitch": pitch, "nx": n_pix, "ny": n_pix,
           "qe_lambda": np.array([200.0, 600.0]), "qe_value": np.array([1.0, 1.0])}
    return {
        "name": "coincident-" + ("mirror" if mirror_first else "absorber") + "-first",
        "materials": _materials(unit_reflectivity=True),
        "segments": {"pivot": np.zeros((0, 3)), "u0": np.zeros((0, 3)), "e1": np.zeros((0, 3)),
                     "e2": np.zeros((0, 3)), "radius0": np.zeros(0)},
        "params": np.zeros((0, 6)),
        "caps": _empty_caps(),
        "rects": _empty_rects(),
        "meshes": [mirror, absorber] if mirror_first else [absorber, mirror],
        "detector": det,
        "box": {"lo": np.array([-3000.0, -3000.0, -3000.0]), "hi": np.array([3000.0, 3000.0, 3000.0])},
        "max_bounces": 16,
        "t_min": 1e-2,
    }


def coincident_photons(seed=77, start_z=200.0):
    """Explicit photons for scene_coincident: straight up through the fan's centre, through points
    on its inner edges and on its outer boundary, through random interior points, and slightly
    tilted from random interior points."""
    rng = np.random.default_rng(seed)
    exact = [(0, 0), (100, 0), (0, 100), (-100, 0), (0, -100), (100, 100), (-50, -50), (150, -150),
             (-70, 70), (200, 50), (-200, -120), (30, 200), (-10, -200), (200, 200)]
    xy = np.concatenate([np.array(exact, np.float64), rng.uniform(-190.0, 190.0, size=(200, 2)),
                         rng.uniform(-120.0, 120.0, size=(300, 2))])
    n = len(xy)
    o = np.column_stack([xy, np.full(n, start_z)])
    d = np.zeros((n, 3))
    d[:, 2] = 1.0
    tilt = rng.uniform(-0.1, 0.1, size=(300, 2))
    d[-300:, :2] = tilt
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    return explicit_source(o, d, np.full(n, 400.0))


def film_paper(width=1320, height=620, sigma=0.5, threshold=45.0):
    """The paper's camera and film (Section 4.4): 1320 x 620 pixels, camera 478.69 mm in front of the
    detector, 116.38 degree field of view, hit threshold 45 of 255.  The reconstruction filter is not
    given; a Gaussian of sigma 0.5 pixel (radius 4 sigma) is assumed."""
    return {"width": width, "height": height, "distance": 478.69, "fov": float(np.radians(116.38)),
            "sigma": sigma, "threshold": threshold}


def film_hits(n, seed, half=300.0, detected_fraction=0.8):
    """Seeded synthetic read-out input: fates (DETECTED with the given probability, else one of the
    other fates) and detector coordinates uniform over [-half, half]^2, FP32-representable."""
    rng = np.random.default_rng(seed)
    fate = np.where(rng.uniform(size=n) < detected_fraction, 0, rng.integers(1, 6, size=n)).astype(np.uint8)
    uv = f32(rng.uniform(-half, half, size=(n, 2)))
    return fate, uv


# ---------------------------------------------------------------------------
# Sources
# ---------------------------------------------------------------------------

def gas_dispersion(n_at_400=1.0014, pole_nm=73.6, step_nm=25.0, lambda_min=LAMBDA_MIN, lambda_max=LAMBDA_MAX):
    """A synthetic dispersion table for a fluorocarbon-like radiator gas: nodes every
    `step_nm`, (n - 1) from a one-pole form A / (pole^-2 - lambda^-2) scaled to
    n(400 nm) = n_at_400, rounded so that n - 1 is FP32-representable.  About
    +-7 % variation of n - 1 across 200..600 nm."""
    lam = np.arange(lambda_min, lambda_max + 0.5 * step_nm, step_nm)
    shape = 1.0 / (pole_nm ** -2 - lam ** -2)
    m = (n_at_400 - 1.0) * shape / (1.0 / (pole_nm ** -2 - 400.0 ** -2))
    return {"lambda": lam, "index": 1.0 + f32(m)}


def with_dispersion(src, table=None):
    """The same source with a wavelength-dependent refractive index (default: gas_dispersion())."""
    out = dict(src)
    out["dispersion"] = gas_dispersion() if table is None else table
    return out


def point_source(origin=(0.0, 0.0, 0.0), direction=(0.0, 0.0, 1.0), beta=1.0,
                 n_radiator=N_RADIATOR, lambda_min=LAMBDA_MIN, lambda_max=LAMBDA_MAX, length=0.0):
    """A Cherenkov emitter on a straight track segment (length 0 = a point)."""
    return {"kind": "track", "origin": f32(origin), "direction": f32(direction), "length": float(f32(length)),
            "beta": float(f32(beta)), "n_radiator": float(n_radiator),
            "lambda_min": float(lambda_min), "lambda_max": float(lambda_max)}


def with_prefilter(src, mirror_materials=(MIRROR, MIRROR)):
    """The same source with the paper's pre-propagation efficiency filter (Section 4.3):
    keep each photon with probability QE * reflectivity of each listed mirror."""
    out = dict(src)
    out["prefilter"] = list(mirror_materials)
    return out


def explicit_source(o, d, lam):
    """Photons given one by one as origin, unit direction and wavelength (Section 4.2)."""
    return {"kind": "explicit", "o": f32(o).reshape(-1, 3), "d": f32(d).reshape(-1, 3),
            "lambda": f32(lam).reshape(-1)}


def sample_tracks(rng, n_tracks, max_angle=0.3, length=1000.0):
    """Track directions uniform in solid angle within max_angle of +z, starting at the origin.

    Returns float64 [T, 8] rows (ox, oy, oz, tx, ty, tz, length, beta), FP32-representable.
    """
    cos_psi = rng.uniform(np.cos(max_angle), 1.0, size=n_tracks)
    phi = rng.uniform(0.0, 2.0 * np.pi, size=n_tracks)
    sin_psi = np.sqrt(1.0 - cos_psi * cos_psi)
    t = np.stack([sin_psi * np.cos(phi), sin_psi * np.sin(phi), cos_psi], axis=1)
    rows = np.zeros((n_tracks, 8))
    rows[:, 3:6] = t
    rows[:, 6] = length
    rows[:, 7] = 1.0
    return f32(rows)


def batch_source(tracks, counts, n_radiator=N_RADIATOR, lambda_min=LAMBDA_MIN, lambda_max=LAMBDA_MAX):
    counts = np.asarray(counts, dtype=np.uint64)
    offsets = np.zeros(len(counts) + 1, dtype=np.uint64)
    offsets[1:] = np.cumsum(counts, dtype=np.uint64)
    return {"kind": "batch", "tracks": np.ascontiguousarray(tracks, dtype=np.float64),
            "offsets": offsets, "n_radiator": float(n_radiator),
            "lambda_min": float(lambda_min), "lambda_max": float(lambda_max)}


def poisson_batch(k, n_tracks, mean, clip=None):
    rng = np.random.default_rng(1000 + k)
    tracks = sample_tracks(rng, n_tracks)
    counts = rng.poisson(mean, size=n_tracks)
    if clip is not None:
        counts = np.clip(counts, clip[0], clip[1])
    return batch_source(tracks, counts)


def perturbed_params(k, scene, sigma_tilt=0.5e-3, sigma_radius=5.0):
    """Seeded misalignment of every segment: tilts ~ N(0, sigma_tilt), radius ~ R0 + N(0, sigma_radius)."""
    rng = np.random.default_rng(2000 + k)
    nseg = scene["params"].shape[0]
    draws = rng.normal(size=(nseg, 3))
    p = np.array(scene["params"], dtype=np.float64)
    p[:, 0] = draws[:, 0] * sigma_tilt
    p[:, 1] = draws[:, 1] * sigma_tilt
    p[:, 2] = scene["segments"]["radius0"] + draws[:, 2] * sigma_radius
    return f32(p)


# ---------------------------------------------------------------------------
# The five workloads
# ---------------------------------------------------------------------------

def config(k):
    """Workload k in 1..5.  Returns a dict with scene, source, n_photons, seed."""
    if k == 1:
        return {"name": "C1 analytic point 1e5", "scene": scene_g1(), "source": point_source(),
                "n_photons": 100_000, "seed": SEED_BASE + 1}
    if k == 2:
        return {"name": "C2 meshed point 1e7", "scene": scene_g2(), "source": point_source(),
                "n_photons": 10_000_000, "seed": SEED_BASE + 2}
    if k == 3:
        src = poisson_batch(3, 4096, 1000.0, clip=(50, 5000))
        return {"name": "C3 batched 4096 tracks", "scene": scene_g2(), "source": src,
                "n_photons": int(src["offsets"][-1]), "seed": SEED_BASE + 3}
    if k == 4:
        rng = np.random.default_rng(1000 + 4)
        src = batch_source(sample_tracks(rng, 1000), np.full(1000, 1000))
        sc = scene_g4()
        return {"name": "C4 adjoint 4x4 segments 1e6", "scene": sc, "source": src,
                "n_photons": int(src["offsets"][-1]), "seed": SEED_BASE + 4,
                "target_params": perturbed_params(4, sc)}
    if k == 5:
        src = poisson_batch(5, 8192, 1e8 / 8192)
        sc = scene_g5()
        return {"name": "C5 large 1e8 2M triangles", "scene": sc, "source": src,
                "n_photons": int(src["offsets"][-1]), "seed": SEED_BASE + 5,
                "target_params": perturbed_params(5, sc)}
    raise ValueError(f"unknown config {k}")
