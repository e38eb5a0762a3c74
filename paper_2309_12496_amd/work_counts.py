"""Units of the method's work per photon, counted on the GPU by the measurement build.

librich_work.so is librich.so compiled with -DRICH_WORK_COUNTERS: every
active lane counts the units of work it does (the WorkUnit list in
csrc/trace.h: photons, Philox blocks, closest-hit queries, cap, rectangle and
box tests, BVH4 nodes whose four child boxes it tests, leaves, triangle
tests, instance entries, reflections, detector hits), summed per wave with
one atomic per counter.  Photons and outputs are those of the product build;
only the counters are added.  This script runs each workload once through it
and prints the counts per traced photon, the algorithmic VALU work per
photon formed from them (units x operations per unit, OPS_PER_UNIT), and each
unit's SIMD efficiency: the share of a wave's 64 lanes that did the unit
when the wave did it.

    python -m paper_2309_12496_amd.build_lib --work-counters   # on the CPU, once
    python -m paper_2309_12496_amd.work_counts [c1 c2 c3 c4 c5] # on the GPU
"""

from __future__ import annotations

import ctypes as C
import json
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
WORK_LIB = os.path.join(HERE, "librich_work.so")
UNITS = ("photons", "philox_blocks", "sort_keys", "queries", "cap_boxes", "caps", "rects", "boxes", "nodes",
         "leaves", "triangles", "instances", "moving_instances", "reflections", "detections", "back_detector",
         "back_caps", "back_facets", "back_planes")

# VALU operations per unit of work, counted on the method's own arithmetic in
# 32-bit lane operations (a 3-vector dot product is 3: a mul and two fma; a
# select, compare, min or max is 1).  Address arithmetic, loads and stores,
# stack and loop bookkeeping are not counted.
OPS_PER_UNIT = {
    # per traced photon: wavelength (fma, reciprocal), azimuth (scale, sin,
    # cos), cone direction from the track's basis (2 x (3 mul + 3 fma)),
    # emission point (mul, 3 fma)
    "photons": 2 + 3 + 12 + 4,
    # ten rounds of two 32x32->64 multiplies (lo and hi: 4), four XORs and two
    # key additions (no key step after the last round); four U24 conversions
    # (shift, convert, scale)
    "philox_blocks": 10 * 10 - 2 + 4 * 3,
    # per closest-hit query: reciprocal direction and scaled origin (6); the
    # detector plane: d.n, zero test, c - o, (c - o).n, reciprocal, mul, t test,
    # point (6), u and v (6), 4 range tests (29); the best-hit compare (2)
    "queries": 6 + 29 + 2,
    # a cap's bounding box: 6 plane distances, 6 min/max, near and far (5),
    # far scale and cap, hit select (3)
    "cap_boxes": 6 + 6 + 5 + 3 + 2,
    # a sphere cap: offset, b = f.d, the cancellation-free discriminant
    # (fma3, dot, fma, test, sqrt), c (dot, fma), q (3), zero test, the two
    # roots (reciprocal, mul, min, max): 28; each root: t test, point, side
    # of the centre plane (sub, dot, test), cell coordinates (sub, 2 dots),
    # 4 bounds (24, both roots counted); the best-hit compare (2)
    "caps": 28 + 2 * 24 + 2,
    # a rectangle: the plane test as for the detector (29) and the compare (2)
    "rects": 29 + 2,
    # the analytic box: 6 plane distances, 10 min/max, 3 tests, compare (2)
    "boxes": 6 + 10 + 3 + 2,
    # a BVH4 node: per child box 6 plane distances, near (3 max) and far (2
    # min) distances, far scale, cap at the closest hit, entry-or-exit select
    # and miss test (3): 16 x 4; key packing (4 x 2), the 5-exchange sorting
    # network (10), the miss test and the count of children to push (6)
    "nodes": 16 * 4 + 8 + 10 + 6,
    # a leaf: the ray's shear constants (dominant axis 7, two other axes 2,
    # reciprocal and two scale factors 3, component selects 3)
    "leaves": 15,
    # watertight test: 9 translations, 9 component selects, 6 shears, 3 edge
    # functions (2 mul + sub), sign tests (10), determinant (2), scaled
    # distance (6), reciprocal, mul, t test, best-hit compare (2)
    "triangles": 9 + 9 + 6 + 9 + 10 + 2 + 6 + 3 + 2,
    # entering and leaving a mesh instance's frame: the origin translated and
    # rescaled by the reciprocal direction, both ways (2 x 6)
    "instances": 12,
    # in addition, for a moving segment: origin and direction rotated and
    # scaled (2 x 9), a new reciprocal direction (3 + 3 on leaving)
    "moving_instances": 18 + 6 - 6 + 9,
    # hit point (3), normal (rotation of the facet normal, or the cap's
    # (C - P)/R: ~8), front test (4), reflectivity table (6), roulette (1),
    # reflection (dot, scale, fma3: 7), renormalisation (dot, rsqrt, 3 mul:
    # 7), path time (1)
    "reflections": 3 + 8 + 4 + 6 + 1 + 7 + 7 + 1,
    # back-face test (4), detector-frame point (6), u and v (6), pixel
    # indices (2 x (add, mul, floor), 4 range tests, mul + add: 12), global
    # point (3), arrival time (1), QE table (5), roulette (1)
    "detections": 4 + 6 + 6 + 12 + 3 + 1 + 5 + 1,
    # adjoint, per counted photon: residual and loss (7), the upstream
    # gradient on the detector plane (6), back through the plane (two dots,
    # divide, fma3: 11), the direction's adjoint (3)
    "back_detector": 7 + 6 + 11 + 3,
    # back through a reflection off a cap: the normal's and direction's
    # adjoints (two dots, 10), through the sphere (reciprocal, offset, the
    # hit's adjoint: 17), centre and radius adjoints (11), onto the six
    # parameters (3 dots and an add: 10), next point and direction (6), the
    # six sums (6)
    "back_caps": 10 + 4 + 17 + 11 + 10 + 6 + 6 + 3,
    # back through a moving facet: the normal's and direction's adjoints
    # (16), the facet point (rotation, fma3: 12), through the plane (11),
    # point and normal adjoints (9), the six parameters (two rotations of the
    # vertex and normal by each tilt derivative and their dots: 2 x 26; the
    # radius: 4), next point and direction (6), the six sums (6)
    "back_facets": 16 + 12 + 11 + 9 + 52 + 4 + 6 + 6,
    # back through a fixed plane (flat mirror): adjoints (10), through the
    # plane (11), next point and direction (6)
    "back_planes": 10 + 11 + 6,
}


def algorithmic_ops(per_photon):
    """VALU operations per traced photon: sum of units per photon x ops per unit.  The regrouping's
    second draw of Philox block 0 (its sort key) is left out: the method draws each block once."""
    per = dict(per_photon)
    per["philox_blocks"] = per["philox_blocks"] - per["sort_keys"]
    return sum(per[u] * OPS_PER_UNIT[u] for u in OPS_PER_UNIT)


def main(which):
    os.environ["RICH_LIBRARY"] = WORK_LIB
    if not os.path.exists(WORK_LIB):
        raise SystemExit(f"{WORK_LIB} is missing: python -m paper_2309_12496_amd.build_lib --work-counters")
    import torch
    sys.path.insert(0, os.path.dirname(HERE))
    from paper_2309_12496_amd import inputs as I
    from paper_2309_12496_amd import rich as R
    assert R.LIB_PATH == WORK_LIB
    lib = C.CDLL(WORK_LIB)
    lib.rich_work_counters.argtypes = [C.POINTER(C.c_ulonglong), C.c_int]
    lib.rich_work_counters_adjoint.argtypes = [C.POINTER(C.c_ulonglong), C.c_int]
    raw = (C.c_ulonglong * (2 * len(UNITS)))()

    def read(adjoint=False):
        """Lane counts per unit; the wave counts that follow them go to waves."""
        fn = lib.rich_work_counters_adjoint if adjoint else lib.rich_work_counters
        if fn(raw, 1) != 0:
            raise RuntimeError("rich_work_counters failed")
        waves.clear()
        waves.update(zip(UNITS, raw[len(UNITS):]))
        return list(raw[:len(UNITS)])

    waves = {}

    def efficiency(counts):
        """Per unit, the active lanes of the waves that did it: lanes / (64 x waves)."""
        return {u: round(counts[u] / (64 * waves[u]), 3) for u in UNITS if waves.get(u)}

    out = {}
    for name in which:
        k = int(name[1])
        cfg = I.config(k)
        scene = R.Scene(cfg["scene"])
        read()                                              # zero the counters
        if cfg["source"]["kind"] == "batch":
            res = R.propagate_batch(scene, cfg["source"], cfg["seed"], tune=R.tuning(256, 256, 4))
        else:
            res = R.propagate(scene, cfg["source"], cfg["n_photons"], cfg["seed"])
        torch.cuda.synchronize()
        counts = dict(zip(UNITS, read()))
        assert scene.status() == 0
        n = counts["photons"]
        per = {u: counts[u] / n for u in UNITS}
        out[cfg["name"]] = {"traced_photons": n, "per_photon": {u: round(v, 4) for u, v in per.items()},
                            "algorithmic_ops_per_photon": round(algorithmic_ops(per), 1),
                            "simd_efficiency": efficiency(counts)}
        print(json.dumps({cfg["name"]: out[cfg["name"]]}), flush=True)
        if k in (4, 5):
            # the adjoint of the forward + adjoint form: targets at the seeded
            # misalignment, mask = detected in both runs
            scene.set_params(cfg["target_params"])
            tgt = R.propagate_batch(scene, cfg["source"], cfg["seed"], tune=R.tuning(256, 256, 4))
            scene.set_params(cfg["scene"]["params"])
            mask = ((tgt["fate"] == 0) & (res["fate"] == 0)).to(torch.uint8)
            targets = tgt["hit_uv"].nan_to_num(0.0)
            del tgt
            read(adjoint=True)
            R.adjoint(scene, cfg["source"], cfg["seed"], targets=targets, mask=mask)
            torch.cuda.synchronize()
            counts = dict(zip(UNITS, read(adjoint=True)))
            m = counts["photons"]
            per = {u: counts[u] / m for u in UNITS}
            key = cfg["name"] + ", adjoint"
            out[key] = {"masked_photons": m, "per_photon": {u: round(v, 4) for u, v in per.items()},
                        "algorithmic_ops_per_photon": round(algorithmic_ops(per), 1),
                        "simd_efficiency": efficiency(counts)}
            print(json.dumps({key: out[key]}), flush=True)
            del mask, targets
        del res, scene
        torch.cuda.empty_cache()
    return out


if __name__ == "__main__":
    main(sys.argv[1:] or ["c1", "c2", "c3", "c4", "c5"])
