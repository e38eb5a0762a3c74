"""The C ABI library loads and exports every call include/rich.h declares; host-side checks fail cleanly."""

import ctypes as C
import os
import re

import numpy as np
import pytest

from conftest import ROOT
from paper_2309_12496_amd import inputs as I

HEADER = os.path.join(ROOT, "include", "rich.h")
LIB = os.path.join(ROOT, "paper_2309_12496_amd", "librich.so")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"^\s*(?:rich_status|const char \*)\s*(rich_\w+)\s*\(", text, flags=re.M)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(LIB):
        pytest.fail("librich.so is not built (run __graft_entry__.build())")
    return C.CDLL(LIB)


def test_header_declares_the_four_calls():
    names = declared_functions()
    for f in ("rich_build_scene", "rich_propagate", "rich_propagate_batch", "rich_propagate_adjoint"):
        assert f in names


def test_library_exports_every_declared_symbol(lib):
    for name in declared_functions():
        assert hasattr(lib, name), name


def test_binding_names_match_the_header():
    from paper_2309_12496_amd import rich as R
    assert sorted(R.EXPORTED) == declared_functions()
    for name in R.EXPORTED:
        assert callable(getattr(R, name))


def test_version_and_null_arguments(lib):
    lib.rich_version.restype = C.c_char_p
    lib.rich_last_error.restype = C.c_char_p
    assert b"gfx950" in lib.rich_version()
    out = C.c_void_p()
    assert lib.rich_build_scene(None, 0, C.byref(out)) == -1
    assert b"NULL" in lib.rich_last_error()
    assert lib.rich_destroy_scene(None) == -1
    assert lib.rich_propagate(None, None, 0, 0, 0, None, None) == -1


def _desc_of(scene):
    from paper_2309_12496_amd import rich as R
    return R.scene_desc(scene)


@pytest.mark.parametrize("breaker", ["nan_vertex", "bad_qe", "bad_material", "zero_pitch", "bad_segment"])
def test_scene_validation_rejects_bad_input_before_any_device_work(lib, breaker):
    """Validation runs on the host before any HIP call, so it is checkable without a GPU."""
    from paper_2309_12496_amd import inputs as I
    from paper_2309_12496_amd import rich as R
    sc = I.scene_g2(sphere_quads=(4, 4))
    if breaker == "nan_vertex":
        sc["meshes"][0]["vertices"][1, 2, 0] = np.nan
    elif breaker == "bad_qe":
        sc["detector"]["qe_value"] = np.array([0.0, 1.5, 0.0])
    elif breaker == "bad_material":
        sc["meshes"][1]["material"] = 7
    elif breaker == "zero_pitch":
        sc["detector"]["pitch"] = 0.0
    elif breaker == "bad_segment":
        sc["meshes"][0]["segment"] = 3
    desc, keep = R.scene_desc(sc)
    out = C.c_void_p()
    code = R._L.rich_build_scene(C.byref(desc), 0, C.byref(out))
    assert code == R.RICH_EINVAL
    assert not out.value
    assert R.rich_last_error()


def test_cherenkov_yield_matches_oracle(orc):
    """rich_cherenkov_yield (host Gauss-Legendre) against the oracle's composite Simpson, and its checks."""
    from paper_2309_12496_amd import rich as R
    src = I.point_source()
    disp = I.with_dispersion(src)
    for s in (src, disp):
        for beta in (1.0, 0.99995, 1 / 1.00146):
            assert R.cherenkov_yield(s, beta) == pytest.approx(orc.cherenkov_yield(s, beta), rel=1e-10, abs=1e-15)
    assert R.cherenkov_yield(src, 0.99) == 0.0
    with pytest.raises(R.RichError):
        R.rich_cherenkov_yield(None, 1.0014, -1.0, 200.0, 600.0)
    with pytest.raises(R.RichError):
        R.cherenkov_yield(I.with_dispersion(src, {"lambda": [300.0, 200.0], "index": [1.001, 1.001]}), 1.0)


def test_header_is_plain_c_and_links(tmp_path):
    """include/rich.h compiles as C99 and a C program linked against librich.so runs its host-only calls."""
    import shutil
    import subprocess
    if shutil.which("gcc") is None:
        pytest.skip("no C compiler")
    prog = tmp_path / "abi.c"
    prog.write_text(
        '#include <stdio.h>\n#include "rich.h"\n'
        "int main(void) {\n"
        "    double y = 0.0;\n"
        "    if (rich_cherenkov_yield(NULL, 1.0014, 1.0, 200.0, 600.0, &y) != RICH_OK) return 1;\n"
        "    if (rich_cherenkov_yield(NULL, 1.0014, -1.0, 200.0, 600.0, &y) != RICH_EINVAL) return 2;\n"
        '    printf("%.9f %s\\n", y, rich_version());\n'
        "    return 0;\n"
        "}\n")
    libdir = os.path.join(ROOT, "paper_2309_12496_amd")
    exe = tmp_path / "abi"
    cmd = ["gcc", "-std=c99", "-Wall", "-Werror", "-D__HIP_PLATFORM_AMD__", "-I", os.path.join(ROOT, "include"),
           "-I", "/opt/rocm/include", str(prog), "-L", libdir, "-lrich", f"-Wl,-rpath,{libdir}", "-o", str(exe)]
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr
    r = subprocess.run([str(exe)], capture_output=True, text=True)
    assert r.returncode == 0, (r.returncode, r.stderr)
    assert r.stdout.startswith("0.4270421")


@pytest.mark.parametrize("counts", [(1 << 26,), (1 << 25, 1 << 25), (3, (1 << 26) - 2)])
def test_scene_triangle_limit_is_refused_before_vertices_are_read(lib, counts):
    """Traversal forms 32-bit byte offsets of 64-byte triangles and 128-byte nodes, so a scene
    holds at most 2^26 - 1 triangles.  The count is checked before any vertex is read: here the
    meshes claim more triangles than their arrays hold, and the build must refuse them."""
    from paper_2309_12496_amd import rich as R
    sc = I.scene_g2(sphere_quads=(4, 4))
    desc, keep = R.scene_desc(sc)
    assert desc.n_meshes >= len(counts)
    for k, c in enumerate(counts):
        desc.meshes[k].n_tri = c
    out = C.c_void_p()
    assert R._L.rich_build_scene(C.byref(desc), 0, C.byref(out)) == R.RICH_EINVAL
    assert not out.value
    assert "too many triangles" in R.rich_last_error()
