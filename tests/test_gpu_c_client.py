"""A C program compiled against include/rich.h drives the device calls (build, propagate into its own
hipMalloc'd buffers, get_status, destroy) on the analytic workload; its outputs match the oracle."""

import os
import shutil
import subprocess

import numpy as np
import pytest

from conftest import ROOT
from paper_2309_12496_amd import inputs as I
from parity import compare

pytestmark = pytest.mark.gpu

CLIENT = os.path.join(ROOT, "tests", "c_client", "rich_client.c")
LIBDIR = os.path.join(ROOT, "paper_2309_12496_amd")
ROCM = os.environ.get("ROCM_PATH", "/opt/rocm")


def _nums(*xs):
    out = []
    for x in xs:
        out += [repr(float(v)) for v in np.atleast_1d(np.asarray(x, np.float64)).reshape(-1)]
    return " ".join(out)


def scene_text(scene, src):
    """The scene and source in the client's plain-text format (exact doubles)."""
    lines = [f"materials {len(scene['materials'])}"]
    for m in scene["materials"]:
        lines.append(f"{m['kind']} {len(m['refl_lambda'])} {_nums(m['refl_lambda'], m['refl_value'])}")
    sg = scene["segments"]
    k = len(sg["radius0"])
    lines.append(f"segments {k}")
    for i in range(k):
        lines.append(_nums(sg["pivot"][i], sg["u0"][i], sg["e1"][i], sg["e2"][i], sg["radius0"][i],
                           scene["params"][i]))
    cp = scene["caps"]
    lines.append(f"caps {len(cp['segment'])}")
    for i in range(len(cp["segment"])):
        lines.append(f"{cp['segment'][i]} {cp['material'][i]} "
                     + _nums(cp["origin"][i], cp["axis_a"][i], cp["axis_b"][i], cp["bounds"][i]))
    rc = scene["rects"]
    lines.append(f"rects {len(rc['material'])}")
    for i in range(len(rc["material"])):
        lines.append(f"{rc['material'][i]} "
                     + _nums(rc["center"][i], rc["normal"][i], rc["axis_u"][i], rc["axis_v"][i], rc["half"][i]))
    d = scene["detector"]
    lines.append("detector " + _nums(d["center"], d["normal"], d["axis_u"], d["axis_v"], d["half"], d["pitch"],
                                     d["nx"], d["ny"]) + f" {len(d['qe_lambda'])} " + _nums(d["qe_lambda"], d["qe_value"]))
    b = scene["box"]
    lines.append("box 1 " + _nums(b["lo"], b["hi"]))
    lines.append("limits " + _nums(scene["max_bounces"], scene["t_min"]))
    lines.append("source " + _nums(src["origin"], src["direction"], src["length"], src["beta"], src["n_radiator"],
                                   src["lambda_min"], src["lambda_max"]))
    return "\n".join(lines) + "\n"


@pytest.fixture(scope="module")
def client(tmp_path_factory):
    import torch
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a GPU")
    cc = shutil.which("gcc") or shutil.which("cc")
    assert cc, "a C compiler is needed"
    exe = str(tmp_path_factory.mktemp("c_client") / "rich_client")
    cmd = [cc, "-std=c11", "-O2", "-Wall", "-Werror", "-D__HIP_PLATFORM_AMD__", f"-I{ROCM}/include",
           f"-I{os.path.join(ROOT, 'include')}", CLIENT, "-o", exe, f"-L{LIBDIR}", "-lrich", f"-L{ROCM}/lib",
           "-lamdhip64", f"-Wl,-rpath,{LIBDIR}", f"-Wl,-rpath,{ROCM}/lib"]
    r = subprocess.run(cmd, capture_output=True, text=True, timeout=120)
    assert r.returncode == 0, r.stderr
    return exe


def run_client(exe, tmp_path, scene, src, n, seed):
    sfile = tmp_path / "scene.txt"
    sfile.write_text(scene_text(scene, src))
    ofile = tmp_path / "out.bin"
    print(f"c client: {n} photons, seed {seed}", flush=True)
    r = subprocess.run([exe, str(sfile), str(n), str(seed), str(ofile)], capture_output=True, text=True,
                       timeout=120)
    assert r.returncode == 0, f"client exit {r.returncode}: {r.stdout} {r.stderr}"
    raw = ofile.read_bytes()
    assert len(raw) == n * (1 + 4 + 8) + 8 * 8
    fate = np.frombuffer(raw, np.uint8, n, 0)
    pixel = np.frombuffer(raw, np.int32, n, n)
    uv = np.frombuffer(raw, np.float32, 2 * n, 5 * n).reshape(n, 2)
    counts = np.frombuffer(raw, np.uint64, 7, 13 * n)
    hist_total = int(np.frombuffer(raw, np.uint64, 1, 13 * n + 56)[0])
    return fate, pixel, uv, counts, hist_total, r.stdout


def test_c_client_propagates_the_analytic_workload(client, tmp_path, orc):
    cfg = I.config(1)
    n = 10_000
    fate, pixel, uv, counts, hist_total, log = run_client(client, tmp_path, cfg["scene"], cfg["source"], n,
                                                          cfg["seed"])
    ref = orc.propagate(cfg["scene"], cfg["source"], n, cfg["seed"])
    # the client keeps hit_xyz on the device: compare (u, v) in its place
    gpu = {"fate": fate, "pixel": pixel, "hit_xyz": uv, "hit_uv": uv}
    ref2 = dict(ref)
    ref2["hit_xyz"] = ref["hit_uv"]
    compare(gpu, ref2, label="C client, C1 photons 0..9999")
    assert np.array_equal(counts, np.bincount(fate, minlength=7).astype(np.uint64))
    assert hist_total == int((fate == 0).sum())
    assert "detected" in log
