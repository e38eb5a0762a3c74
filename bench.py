"""Throughput benchmark: photons propagated per second on one MI355X.

A step is one pass of the whole hot path over one batch of synthetic input:
photon generation, closest-hit traversal, interaction and every output
(fate, pixel, hit xyz and uv, histogram, fate counters), i.e. one
rich_propagate launch.  Inputs and outputs are resident in HBM; the scene is
built once outside the timed region (as the paper separates scene parsing and
kernel initialisation from rendering, Section 5.2).

Headline workload: the meshed RICH scene (200k-triangle spherical mirror,
flat mirror, 10k-triangle enclosure) with 1e7 photons from one point
emitter, plain forward.  The other forms of the metric are reported under
"forms": batched (4096 Poisson-sized tracks, one persistent launch replayed
from a HIP graph), forward+adjoint (4x4 segmented mirror, 1e6 photons, 96
parameters), an Adam alignment fit on the same scene, the headline workload
with the pre-propagation efficiency filter, the analytic scene (1e5 photons
per call, and 1e8 in one call), and the large scene (1e8 photons, 2M
triangles, 192 parameters).
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

# MI355X peaks: HBM3E 8 TB/s; VALU 256 CUs x 4 SIMD x 16 lanes x 2.4 GHz =
# 3.93e13 32-bit lane operations per second (no packed math).
HBM_PEAK_GBS = 8000.0
VALU_PEAK_LANE_OPS = 256 * 64 * 2.4e9

# Algorithmic VALU work per photon of the headline workload, in 32-bit lane
# operations: the method's units of work per photon counted on the GPU by the
# measurement build (23.85 BVH4 nodes, 7.43 triangle tests, 3.72 leaves,
# 2.78 instance entries, 2.78 closest-hit queries, 1.78 reflections, 0.85
# detector hits, 2 Philox blocks) times the operations each takes
# (paper_2309_12496_amd/work_counts.py; profiles/work_counts.md).
ALU_OPS_PER_PHOTON = 3046.2
# What the forward launch (sort_photons_kernel, then forward_kernel) executes
# per photon on the same workload (rocprofv3,
# profiles/forward_kernel_c2_counters.md): SQ_INSTS_VALU x 64 / photons =
# issued lane slots (inactive lanes of divergent waves included), and
# SQ_THREAD_CYCLES_VALU / photons = lane operations of active lanes (the
# counter reads 64 per instruction on a plain copy kernel).
ISSUED_SLOTS_PER_PHOTON = 5266.3
ACTIVE_LANE_OPS_PER_PHOTON = 4376.0
# Compulsory HBM bytes per photon: fate 1 + pixel 4 + xyz 12 + uv 8 + arrival time 4 (writes).
OUT_BYTES_PER_PHOTON = 29.0
# Bytes per photon out of L2 of the same launch, both kernels: (FETCH_SIZE x 1.9998 + WRITE_SIZE x
# 1.0) KiB per dispatch, scaled by the 256 MiB copy-kernel calibration (262,144 KiB copied: FETCH_SIZE
# reads 131,086, WRITE_SIZE 262,144), / 1e7 photons (profiles/forward_kernel_c2_counters.md).
TRAFFIC_BYTES_PER_PHOTON = ((20485.7 + 207.1) * 1.9998 + 389902.0 + 39063.5) * 1024 / 1e7


def parse():
    p = argparse.ArgumentParser()
    p.add_argument("--gpus", type=int, default=1)
    p.add_argument("--steps", type=int, default=20)
    p.add_argument("--warmup", type=int, default=3)
    p.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    p.add_argument("--no-forms", action="store_true", help="only the headline workload")
    p.add_argument("--forms", default="c1,batched,adjoint,fit,prefilter,large,largefit", help="comma list of extra forms (also: sizes)")
    p.add_argument("--cpu-seconds", type=float, default=12.0, help="target CPU time of the oracle sample")
    p.add_argument("--fixed-tuning", action="store_true",
                   help="batch forms use block 256, chunk 256, 4 blocks per CU instead of the autotuner "
                        "(for profiler runs, which would otherwise trace the autotuner's sweep)")
    p.add_argument("--copy-calibration", action="store_true",
                   help="only run a plain 256 MiB device copy (to scale FETCH_SIZE/WRITE_SIZE counters)")
    return p.parse_args()


def copy_calibration():
    """A plain copy kernel of known size: 256 MiB read and 256 MiB written, 3 times."""
    import torch
    x = torch.ones(64 * 1024 * 1024, dtype=torch.float32, device="cuda")
    y = torch.empty_like(x)
    for _ in range(3):
        y.copy_(x)
    torch.cuda.synchronize()
    print(json.dumps({"copy_bytes_read": x.numel() * 4, "copy_bytes_written": y.numel() * 4, "reps": 3}))


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
    """FP64 oracle on a bounded prefix of the same workload, all host threads (up to 16)."""
    import numpy as np
    from oracle import oracle as O
    from paper_2309_12496_amd import inputs as I
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
    assert int(np.bincount(res["fate"], minlength=7).sum()) == n
    # one thread, a quarter of the time budget
    n1 = int(max(2000, min(n, rate / threads * target_seconds / 4)))
    t0 = time.perf_counter()
    O.propagate(sc, cfg["source"], n1, cfg["seed"], threads=1)
    dt1 = time.perf_counter() - t0
    # the analytic workload: all of its 1e5 photons, on every thread and on one
    c1 = I.config(1)
    sc1 = O.Scene(c1["scene"])
    c1_rates = {}
    for th in (threads, 1):
        t0 = time.perf_counter()
        O.propagate(sc1, c1["source"], c1["n_photons"], c1["seed"], threads=th)
        c1_rates[th] = c1["n_photons"] / (time.perf_counter() - t0)
    return {"value": n / dt, "unit": "photons/s", "cores": threads, "kind": "oracle",
            "sample": f"photon ids 0..{n - 1} of the headline workload ({dt:.1f} s on {threads} threads)",
            "single_thread": {"value": n1 / dt1, "unit": "photons/s",
                              "sample": f"photon ids 0..{n1 - 1} ({dt1:.1f} s on 1 thread)"},
            "analytic": {"workload": c1["name"], "sample": f"all {c1['n_photons']} photons",
                         "photons_per_s": c1_rates[threads], "threads": threads,
                         "single_thread_photons_per_s": c1_rates[1]}}


def form_batched(R, I, stream, steps, fixed_tuning=False):
    cfg = I.config(3)
    t0 = time.perf_counter()
    sc = R.Scene(cfg["scene"])
    build_s = time.perf_counter() - t0
    b, keep, n = R.make_batch(cfg["source"])
    t, o = R.alloc_outputs(sc, n)
    tune = R.tuning(256, 256, 4) if fixed_tuning else R.rich_autotune(sc.handle, b, n, cfg["seed"])
    ms = time_steps(lambda: R.rich_propagate_batch(sc.handle, b, n, cfg["seed"], o, tune, stream), steps, 2, stream)
    assert sc.status() == 0
    return {"workload": cfg["name"], "photons_per_step": n, "ms_per_step": ms, "photons_per_s": n / (ms * 1e-3),
            "tuning": {"block": tune.block, "chunk": tune.chunk, "blocks_per_cu": tune.blocks_per_cu},
            "scene_build_s": round(build_s, 3)}


def _fwd_adjoint(R, I, cfg, stream, steps, fixed_tuning=False):
    """Forward (batched) plus fused-loss adjoint per step, targets from misaligned segments."""
    import torch
    t0 = time.perf_counter()
    sc = R.Scene(cfg["scene"])
    build_s = time.perf_counter() - t0
    b, keep, n = R.make_batch(cfg["source"])
    # the autotuned shape is what a caller gets with tune=NULL
    tune = R.tuning(256, 256, 4) if fixed_tuning else R.rich_autotune(sc.handle, b, n, cfg["seed"])
    sc.set_params(cfg["target_params"])
    tgt_out = R.propagate_batch(sc, cfg["source"], cfg["seed"], tune=tune)
    targets = tgt_out["hit_uv"].nan_to_num(0.0)
    tfate = tgt_out["fate"]
    del tgt_out
    sc.set_params(cfg["scene"]["params"])
    t, o = R.alloc_outputs(sc, n)
    R.rich_propagate_batch(sc.handle, b, n, cfg["seed"], o, tune, stream)
    mask = ((tfate == 0) & (t["fate"] == 0)).to(torch.uint8)
    grad = torch.zeros((sc.n_segments, 6), dtype=torch.float32, device="cuda")
    loss = torch.zeros(1, dtype=torch.float32, device="cuda")
    s_ms = time_steps(lambda: R.rich_propagate_batch(sc.handle, b, n, cfg["seed"], o, tune, stream), steps, 1, stream)
    a_ms = time_steps(lambda: R.rich_propagate_adjoint(sc.handle, None, b, n, cfg["seed"], 0, None, targets, mask,
                                                       None, grad, loss, stream), steps, 1, stream)
    assert sc.status() == 0
    n_mask = int(mask.sum())
    return {"workload": cfg["name"], "photons_per_step": n, "parameters": 6 * sc.n_segments,
            "forward_ms": s_ms, "adjoint_ms": a_ms, "ms_per_step": s_ms + a_ms,
            "photons_per_s": n / ((s_ms + a_ms) * 1e-3), "forward_photons_per_s": n / (s_ms * 1e-3),
            "loss_mm2": float(loss), "masked_photons": n_mask,
            "adjoint_masked_photons_per_s": n_mask / (a_ms * 1e-3), "scene_build_s": round(build_s, 3),
            "tuning": {"block": tune.block, "chunk": tune.chunk, "blocks_per_cu": tune.blocks_per_cu}}


def form_align_fit(R, I, stream, steps, k=4):
    """Adam alignment fit of the segmented mirror: one fused adjoint launch and one device Adam step
    (which also moves the mirrors) per step, captured once in a graph and replayed.

    Targets are the device hits at the seeded misalignment; the fit starts from
    the nominal geometry.  k = 4: the analytic 4 x 4 mirror on its 1e6 photons,
    tilts and radii; k = 5: the 2M-triangle large scene, its 8192 tracks thinned
    to 1221 photons each (1.0e7), tilts only (a meshed segment's radius scales it
    about its pivot, which keeps every facet normal).  Reports the step rate over
    the photons a step retraces (the mask: those the target run detected) and
    how far the fitted tilts and radii are from the misalignment, over the
    segments the photons reach (the only ones whose parameters move).
    """
    import numpy as np
    import torch
    from paper_2309_12496_amd.align import FIT_TILTS_RADII, fit_alignment
    cfg = I.config(k)
    if k == 5:
        src = I.batch_source(cfg["source"]["tracks"], np.full(len(cfg["source"]["tracks"]), 1221))
        free, what = (True, True, False, False, False, False), "tilts"
    else:
        src, free, what = cfg["source"], FIT_TILTS_RADII, "tilts and radii"
    sc = R.Scene(cfg["scene"])
    sc.set_params(cfg["target_params"])
    tgt = R.propagate_batch(sc, src, cfg["seed"], tune=R.tuning(256, 256, 4))
    on = tgt["fate"] <= R.QE_REJECTED
    uv = tgt["hit_uv"].nan_to_num(0.0)
    del tgt
    fit_alignment(sc, src, cfg["seed"], uv, on, steps=3, free=free)          # warm-up
    start, stop = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    start.record(stream)
    p, losses = fit_alignment(sc, src, cfg["seed"], uv, on, steps=steps, lr=0.3, free=free)
    stop.record(stream)
    torch.cuda.synchronize()
    ms = start.elapsed_time(stop) / steps
    assert sc.status() == 0
    p = p.cpu().numpy().astype(np.float64)
    p0 = np.asarray(cfg["scene"]["params"], np.float32).astype(np.float64)
    tp = np.asarray(cfg["target_params"], np.float64)
    moved = np.any(p != p0, axis=1)
    tilt_err = np.abs(p[moved, :2] - tp[moved, :2]).max(axis=1)
    traced = int(on.sum())
    out = {"workload": f"{cfg['name']}, Adam fit of {what} from the nominal geometry",
           "emitted_photons": int(src["offsets"][-1]), "traced_photons_per_step": traced, "steps": steps,
           "ms_per_step": ms, "traced_photons_per_s": traced / (ms * 1e-3),
           "loss_first_mm2": float(losses[0]), "loss_last_mm2": float(losses[-1]),
           "segments_fitted": int(moved.sum()), "max_tilt_error_rad": float(tilt_err.max()),
           "tilt_error_rad_by_segment": [float(f"{x:.3g}") for x in np.sort(tilt_err)[::-1]]}
    if free[2]:
        out["max_radius_error_mm"] = float(np.abs(p[moved, 2] - tp[moved, 2]).max())
    return out


def form_scene_sizes(R, I, stream, steps):
    """The large scene's batch forward against its triangle count: the same 8192 tracks (2442
    photons each, 2.0e7) on the 32-segment mirror meshed at 137x228, 68x114 and 34x57 quads per
    segment.  Not in the default forms (it builds three scenes)."""
    import numpy as np
    cfg = I.config(5)
    src = I.batch_source(cfg["source"]["tracks"], np.full(len(cfg["source"]["tracks"]), 2442))
    rows = []
    for quads in ((137, 228), (68, 114), (34, 57)):
        sc = R.Scene(I.scene_g5(seg_quads=quads))
        info = sc.info()
        b, keep, n = R.make_batch(src)
        t, o = R.alloc_outputs(sc, n)
        tune = R.rich_autotune(sc.handle, b, n, cfg["seed"])
        ms = time_steps(lambda: R.rich_propagate_batch(sc.handle, b, n, cfg["seed"], o, tune, stream), steps, 2,
                        stream)
        assert sc.status() == 0
        rows.append({"segment_quads": list(quads), "triangles": info["n_triangles"], "bvh_nodes": info["n_nodes"],
                     "device_mb": round(info["device_bytes"] / 1e6, 1), "ms_per_step": ms,
                     "photons_per_s": n / (ms * 1e-3)})
        del t, o, sc
    return {"workload": "large scene at three mesh resolutions, 2.0e7 photons", "rows": rows}


def form_prefilter(R, I, stream, steps):
    """The headline workload with the accept-reject of QE x R x R before propagation."""
    cfg = I.config(2)
    sc = R.Scene(cfg["scene"])
    s, keep = R.make_source(I.with_prefilter(cfg["source"]))
    n = cfg["n_photons"]
    t, o = R.alloc_outputs(sc, n)
    ms = time_steps(lambda: R.rich_propagate(sc.handle, s, n, cfg["seed"], 0, o, stream), steps, 2, stream)
    assert sc.status() == 0
    kept = n - int(t["fate_counts"][R.PREFILTERED]) // (steps + 2)
    return {"workload": cfg["name"] + ", pre-filtered", "photons_per_step": n, "ms_per_step": ms,
            "emitted_photons_per_s": n / (ms * 1e-3), "kept_photons_per_step": kept,
            "kept_photons_per_s": kept / (ms * 1e-3)}


def form_c1(R, I, stream, steps):
    cfg = I.config(1)
    sc = R.Scene(cfg["scene"])
    s, keep = R.make_source(cfg["source"])
    n = cfg["n_photons"]
    t, o = R.alloc_outputs(sc, n)
    ms = time_steps(lambda: R.rich_propagate(sc.handle, s, n, cfg["seed"], 0, o, stream), steps, 3, stream)
    # the same call captured once in a HIP graph and replayed (fate counts and
    # histogram accumulate over the replays; per-photon outputs are rewritten)
    import torch
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        R.rich_propagate(sc.handle, s, n, cfg["seed"], 0, o, torch.cuda.current_stream())
    msg = time_steps(graph.replay, steps, 3, stream)
    big = 100_000_000
    tb, ob = R.alloc_outputs(sc, big)
    msb = time_steps(lambda: R.rich_propagate(sc.handle, s, big, cfg["seed"], 0, ob, stream), max(3, steps // 4), 1,
                     stream)
    assert sc.status() == 0
    return {"workload": cfg["name"], "single_call": {"photons_per_step": n, "ms_per_step": ms,
                                                      "photons_per_s": n / (ms * 1e-3)},
            "graph_replay": {"photons_per_step": n, "ms_per_step": msg, "photons_per_s": n / (msg * 1e-3)},
            "steady_state": {"photons_per_step": big, "ms_per_step": msb, "photons_per_s": big / (msb * 1e-3)}}


def main():
    args = parse()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py runs on one GPU only: photons shard by id range across GPUs, "
              "but this benchmark measures a single MI355X (use --gpus 1).", file=sys.stderr)
        sys.exit(2)
    if args.copy_calibration:
        copy_calibration()
        return
    import torch
    from paper_2309_12496_amd import inputs as I
    from paper_2309_12496_amd import rich as R

    cfg = I.config(2)
    t0 = time.perf_counter()
    scene = R.Scene(cfg["scene"])
    build_s = time.perf_counter() - t0
    info = scene.info()
    stream = torch.cuda.current_stream()
    n = cfg["n_photons"]
    s, keep = R.make_source(cfg["source"])
    t, o = R.alloc_outputs(scene, n)

    ms = time_steps(lambda: R.rich_propagate(scene.handle, s, n, cfg["seed"], 0, o, stream), args.steps,
                    args.warmup, stream)
    flags = scene.status()
    counts = t["fate_counts"].cpu().numpy()
    assert counts.sum() == n * (args.steps + args.warmup), "fate counts do not add up"
    assert flags == 0, f"device flags {flags}"
    value = n / (ms * 1e-3)

    if ALU_OPS_PER_PHOTON:
        achieved = ALU_OPS_PER_PHOTON * n / (ms * 1e-3)
        rate = n / (ms * 1e-3)
        roof = {"bound": "alu", "achieved": achieved / 1e12, "peak": VALU_PEAK_LANE_OPS / 1e12,
                "unit": "TOP/s", "frac": achieved / VALU_PEAK_LANE_OPS,
                "algorithmic_ops_per_photon": ALU_OPS_PER_PHOTON,
                # the same peak in the datasheet's units: 78.6 TFLOP/s counting an FMA as two
                # operations, 157.3 with packed FP32 (not used: the build disables it)
                "fp32_fma_tflops_peak": 78.6, "fp32_packed_tflops_peak": 157.3,
                "issue_frac": ISSUED_SLOTS_PER_PHOTON * rate / VALU_PEAK_LANE_OPS,
                "active_lane_frac": ACTIVE_LANE_OPS_PER_PHOTON * rate / VALU_PEAK_LANE_OPS,
                "traffic": None if TRAFFIC_BYTES_PER_PHOTON is None else TRAFFIC_BYTES_PER_PHOTON * n}
    else:
        gbs = OUT_BYTES_PER_PHOTON * n / (ms * 1e-3) / 1e9
        roof = {"bound": "hbm", "achieved": gbs, "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": gbs / HBM_PEAK_GBS,
                "traffic": None}

    line = {
        "metric": "photons propagated/sec on 1 MI355X (fwd, batched, fwd+adjoint) at stated tolerance",
        "value": value, "unit": "photons/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": ms, "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": cfg["name"] + " (meshed RICH, 210,082 triangles, point emitter)",
                   "photons_per_step": n, "triangles": info["n_triangles"], "form": "forward",
                   "scene_build_s": round(build_s, 3), "scene_build_host_s": round(info["build_seconds"], 3)},
        "roofline": roof,
        # the paper's own rates: wall-clock of whole Mitsuba calls (parse, JIT, render) on its workload
        "paper_reference": {"per_cpu_thread": {"value": 2e5, "unit": "photons/s",
                                               "hardware": "Intel Xeon Silver 4210R (LLVM variant)"},
                            "per_gpu": {"value": 1.2e6, "unit": "photons/s",
                                        "hardware": "NVIDIA Tesla T4 (CUDA/OptiX variant)"}},
    }
    del t, o
    torch.cuda.empty_cache()

    if not args.no_forms:
        forms = {}
        want = set(args.forms.split(","))
        half = max(5, args.steps // 2)
        if "c1" in want:
            forms["analytic"] = form_c1(R, I, stream, args.steps)
        if "batched" in want:
            forms["batched"] = form_batched(R, I, stream, half, args.fixed_tuning)
        if "adjoint" in want:
            forms["fwd_adjoint"] = _fwd_adjoint(R, I, I.config(4), stream, half, args.fixed_tuning)
        if "fit" in want:
            forms["align_fit"] = form_align_fit(R, I, stream, 300)
        if "sizes" in want:
            forms["scene_sizes"] = form_scene_sizes(R, I, stream, 5)
        if "largefit" in want:
            forms["large_align_fit"] = form_align_fit(R, I, stream, 300, k=5)
        if "prefilter" in want:
            forms["prefilter"] = form_prefilter(R, I, stream, half)
        if "large" in want:
            forms["large_fwd_adjoint"] = _fwd_adjoint(R, I, I.config(5), stream, 3, args.fixed_tuning)
        line["forms"] = forms
        torch.cuda.empty_cache()
    if not args.no_cpu:
        line["cpu_baseline"] = cpu_baseline(cfg, args.cpu_seconds)
    print(json.dumps(line))


if __name__ == "__main__":
    main()
