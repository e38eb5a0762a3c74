"""Build librich.so for gfx950 with hipcc (every source, every call).

Usage: python -m paper_2309_12496_amd.build_lib
"""

from __future__ import annotations

import concurrent.futures as cf
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
BUILD = os.path.join(os.path.dirname(HERE), "_build")
LIB = os.path.join(HERE, "librich.so")
# measurement build: the same library with per-photon work counters
# (-DRICH_WORK_COUNTERS, read by rich_work_counters); see work_counts.py
WORK_LIB = os.path.join(HERE, "librich_work.so")

SOURCES = ["kernels.hip", "adjoint.hip", "film.hip", "fit.hip", "bvh_build.cpp", "scene.cpp", "capi.cpp"]
ARCH = "gfx950"
FLAGS = ["-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}",
         # no packed FP32 instructions anywhere in the device code
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-Wall", "-Wno-unused-function", "-Wno-unused-parameter"]


def _compile(src, build=BUILD, extra=()):
    obj = os.path.join(build, os.path.splitext(src)[0] + ".o")
    lang = ["-x", "hip"] if src.endswith(".hip") else []
    cmd = ["hipcc", *FLAGS, *extra, *lang, "-c", os.path.join(CSRC, src), "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"{' '.join(cmd)}\n{r.stdout}\n{r.stderr}")
    return obj, r.stderr


def build(verbose=False, work_counters=False):
    """librich.so, or with work_counters the measurement build librich_work.so."""
    build_dir = os.path.join(BUILD, "work") if work_counters else BUILD
    lib = WORK_LIB if work_counters else LIB
    extra = ("-DRICH_WORK_COUNTERS",) if work_counters else ()
    os.makedirs(build_dir, exist_ok=True)
    with cf.ThreadPoolExecutor(max_workers=min(8, len(SOURCES))) as ex:
        results = list(ex.map(lambda src: _compile(src, build_dir, extra), SOURCES))
    objs = [o for o, _ in results]
    if verbose:
        for _, err in results:
            if err.strip():
                print(err, file=sys.stderr)
    tmp = lib + ".tmp"
    cmd = ["hipcc", f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp, *objs]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"{' '.join(cmd)}\n{r.stdout}\n{r.stderr}")
    os.replace(tmp, lib)
    return lib


if __name__ == "__main__":
    print(build(verbose=True, work_counters="--work-counters" in sys.argv))
