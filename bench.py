"""Throughput benchmark: photons propagated per second on one MI355X.

A step is one pass of the whole hot path over one batch of synthetic input:
photon generation, closest-hit traversal, interaction and every output
(fate, pixel, hit xyz and uv, histogram, fate counters), i.e. one
rich_propagate launch.  Inputs and outputs are resident in HBM; the scene is
built once outside the timed region (as the paper separates scene parsing and
kernel initialisation from rendering, Section 5.2).

Default workload: the meshed RICH scene (200k-triangle spherical mirror, flat
mirror, 10k-triangle enclosure) with 1e7 photons from one point emitter.
Prints one JSON line.
"""

from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# HBM peak and VALU peak of MI355X: 256 CUs x 4 SIMD x 16 lanes x 2.4 GHz
# = 3.93e13 32-bit lane operations per second without packed math.
HBM_PEAK_GBS = 8000.0
VALU_PEAK_LANE_OPS = 256 * 64 * 2.4e9

# Algorithmic VALU work per photon of the forward kernel (lane operations),
# measured as SQ_INSTS_VALU * 64 / photons on the default workload (see profiles/).
ALU_OPS_PER_PHOTON = {"c1": None, "c2": None}
# Compulsory HBM bytes per photon: fate 1 + pixel 4 + xyz 12 + uv 8, plus the
# histogram atomics of the detected photons (4 B each).
OUT_BYTES_PER_PHOTON = 25.0

WORKLOADS = {"c1": 1, "c2": 2, "c3": 3}


def parse():
    p = argparse.ArgumentParser()
    p.add_argument("--gpus", type=int, default=1)
    p.add_argument("--steps", type=int, default=20)
    p.add_argument("--warmup", type=int, default=3)
    p.add_argument("--workload", default="c2", choices=sorted(WORKLOADS))
    p.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    p.add_argument("--no-forms", action="store_true", help="skip the batched form")
    p.add_argument("--cpu-seconds", type=float, default=12.0, help="target CPU time of the oracle sample")
    return p.parse_args()


def time_steps(fn, steps, warmup, stream):
    import torch
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    start = torch.cuda.Event(enable_timing=True)
    stop = torch.cuda.Event(enable_timing=True)
    start.record(stream)
    for _ in range(steps):
        fn()
    stop.record(stream)
    torch.cuda.synchronize()
    return start.elapsed_time(stop) / steps


def cpu_baseline(cfg, target_seconds):
    """FP64 oracle on a bounded prefix of the same workload, all host threads."""
    import numpy as np
    from oracle import oracle as O
    threads = min(os.cpu_count() or 1, 16)
    sc = O.Scene(cfg["scene"])
    probe = 20000
    t0 = time.perf_counter()
    O.propagate(sc, cfg["source"], probe, cfg["seed"], threads=threads)
    rate = probe / max(time.perf_counter() - t0, 1e-6)
    n = int(min(cfg["n_photons"], max(probe, rate * target_seconds)))
    t0 = time.perf_counter()
    res = O.propagate(sc, cfg["source"], n, cfg["seed"], threads=threads)
    dt = time.perf_counter() - t0
    assert int(np.bincount(res["fate"], minlength=6).sum()) == n
    return {"value": n / dt, "unit": "photons/s", "cores": threads, "kind": "oracle",
            "sample": f"photon ids 0..{n - 1} of the same workload ({dt:.1f} s on {threads} threads)"}


def main():
    args = parse()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py runs on one GPU only: photons are sharded by id range across GPUs, "
              "but this build measures a single MI355X (use --gpus 1).", file=sys.stderr)
        sys.exit(2)
    import numpy as np
    import torch
    from paper_2309_12496_amd import inputs as I
    from paper_2309_12496_amd import rich as R

    k = WORKLOADS[args.workload]
    cfg = I.config(k)
    t0 = time.perf_counter()
    scene = R.Scene(cfg["scene"])
    build_s = time.perf_counter() - t0
    info = scene.info()
    stream = torch.cuda.current_stream()
    n = cfg["n_photons"]

    if cfg["source"]["kind"] == "batch":
        b, keep, n = R.make_batch(cfg["source"])
        t, o = R.alloc_outputs(scene, n)
        tune = R.rich_autotune(scene.handle, b, n, cfg["seed"])

        def step():
            R.rich_propagate_batch(scene.handle, b, n, cfg["seed"], o, tune, stream)
    else:
        s, keep = R.make_source(cfg["source"])
        t, o = R.alloc_outputs(scene, n)

        def step():
            R.rich_propagate(scene.handle, s, n, cfg["seed"], 0, o, stream)

    ms = time_steps(step, args.steps, args.warmup, stream)
    flags = scene.status()
    counts = t["fate_counts"].cpu().numpy()
    assert counts.sum() == n * (args.steps + args.warmup), "fate counts do not add up"
    assert flags == 0, f"device flags {flags}"
    value = n / (ms * 1e-3)

    det_frac = counts[0] / counts.sum()
    ops = ALU_OPS_PER_PHOTON.get(args.workload)
    if ops:
        achieved = ops * n / (ms * 1e-3)
        roof = {"bound": "alu", "achieved": achieved / 1e12, "peak": VALU_PEAK_LANE_OPS / 1e12,
                "unit": "Tlane-op/s", "frac": achieved / VALU_PEAK_LANE_OPS, "traffic": None}
    else:
        gbs = (OUT_BYTES_PER_PHOTON + 4.0 * det_frac) * n / (ms * 1e-3) / 1e9
        roof = {"bound": "hbm", "achieved": gbs, "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": gbs / HBM_PEAK_GBS,
                "traffic": None}

    line = {
        "metric": "photons propagated/sec on 1 MI355X (fwd, batched, fwd+adjoint) at stated tolerance",
        "value": value, "unit": "photons/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": ms, "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": cfg["name"], "photons_per_step": n, "triangles": info["n_triangles"],
                   "form": "batched" if cfg["source"]["kind"] == "batch" else "forward",
                   "scene_build_s": round(build_s, 3)},
        "roofline": roof,
    }

    if not args.no_forms and args.workload != "c3":
        c3 = I.config(3)
        s3 = R.Scene(c3["scene"])
        b3, keep3, n3 = R.make_batch(c3["source"])
        t3, o3 = R.alloc_outputs(s3, n3)
        tune3 = R.rich_autotune(s3.handle, b3, n3, c3["seed"])
        ms3 = time_steps(lambda: R.rich_propagate_batch(s3.handle, b3, n3, c3["seed"], o3, tune3, stream),
                         max(5, args.steps // 2), 2, stream)
        assert s3.status() == 0
        line["forms"] = {"batched": {"workload": c3["name"], "photons_per_step": n3, "ms_per_step": ms3,
                                     "photons_per_s": n3 / (ms3 * 1e-3),
                                     "tuning": [tune3.block, tune3.chunk, tune3.blocks_per_cu]}}
    if not args.no_cpu:
        line["cpu_baseline"] = cpu_baseline(cfg, args.cpu_seconds)
    print(json.dumps(line))


if __name__ == "__main__":
    main()
