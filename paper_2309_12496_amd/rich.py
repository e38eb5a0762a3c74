"""Python binding of librich.so (the C ABI in include/rich.h).

Argument marshalling only: every step of photon propagation runs in the HIP
kernels of librich.so.  PyTorch provides device memory and streams.  Importing
this module fails loudly when the library has not been built.

Functions named rich_* mirror the C calls one to one; the lower-case helpers
(Scene, propagate, propagate_batch, adjoint, ...) allocate outputs with torch
and translate the plain dictionaries of ``paper_2309_12496_amd.inputs``.
"""

from __future__ import annotations

import ctypes as C
import os

import numpy as np
import torch  # loads the HIP runtime that librich shares with torch

HERE = os.path.dirname(os.path.abspath(__file__))
# RICH_LIBRARY selects another build of the same ABI (the work-counting
# measurement build, librich_work.so); the default is librich.so.
LIB_PATH = os.environ.get("RICH_LIBRARY") or os.path.join(HERE, "librich.so")

if not os.path.exists(LIB_PATH):
    raise ImportError(f"{LIB_PATH} is missing: build it with `python -m paper_2309_12496_amd.build_lib`")
_L = C.CDLL(LIB_PATH)

RICH_OK, RICH_EINVAL, RICH_ENOMEM, RICH_EDEVICE, RICH_ERANGE, RICH_EOVERFLOW, RICH_ESTATE = 0, -1, -2, -3, -4, -5, -6
DETECTED, QE_REJECTED, ABSORBED_MIRROR, ABSORBED, ESCAPED, MAX_BOUNCES, PREFILTERED = range(7)
N_FATES = 7
FLAG_HITLIST_OVERFLOW, FLAG_STACK_OVERFLOW, FLAG_PATH_OVERFLOW, FLAG_BATCH_SIZE = 1, 2, 4, 8
SRC_TRACK, SRC_EXPLICIT = 0, 2
MAX_TABLE = 32
MAX_SEGMENTS = 256

_dp = C.POINTER(C.c_double)
_d3 = C.c_double * 3


class RichError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"rich status {code}: {msg}")
        self.code = code


class rich_material(C.Structure):
    _fields_ = [("kind", C.c_int32), ("n_refl", C.c_int32), ("refl_lambda", _dp), ("refl_value", _dp)]


class rich_segment(C.Structure):
    _fields_ = [("pivot", _d3), ("u0", _d3), ("e1", _d3), ("e2", _d3), ("radius0", C.c_double)]


class rich_cap(C.Structure):
    _fields_ = [("segment", C.c_int32), ("material", C.c_int32), ("origin", _d3), ("axis_a", _d3),
                ("axis_b", _d3), ("bounds", C.c_double * 4)]


class rich_rect(C.Structure):
    _fields_ = [("material", C.c_int32), ("reserved", C.c_int32), ("center", _d3), ("normal", _d3),
                ("axis_u", _d3), ("axis_v", _d3), ("half", C.c_double * 2)]


class rich_mesh(C.Structure):
    _fields_ = [("vertices", _dp), ("n_tri", C.c_int64), ("material", C.c_int32), ("segment", C.c_int32)]


class rich_detector(C.Structure):
    _fields_ = [("center", _d3), ("normal", _d3), ("axis_u", _d3), ("axis_v", _d3), ("half", C.c_double * 2),
                ("pitch", C.c_double), ("nx", C.c_int32), ("ny", C.c_int32), ("n_qe", C.c_int32),
                ("qe_lambda", _dp), ("qe_value", _dp)]


class rich_scene_desc(C.Structure):
    _fields_ = [("n_materials", C.c_int32), ("materials", C.POINTER(rich_material)),
                ("n_segments", C.c_int32), ("segments", C.POINTER(rich_segment)), ("params", _dp),
                ("n_caps", C.c_int32), ("caps", C.POINTER(rich_cap)),
                ("n_rects", C.c_int32), ("rects", C.POINTER(rich_rect)),
                ("n_meshes", C.c_int32), ("meshes", C.POINTER(rich_mesh)),
                ("detector", rich_detector),
                ("has_box", C.c_int32), ("box_lo", _d3), ("box_hi", _d3),
                ("max_bounces", C.c_int32), ("t_min", C.c_double)]


class rich_scene_stats(C.Structure):
    _fields_ = [("n_triangles", C.c_int64), ("n_nodes", C.c_int64), ("n_instances", C.c_int32),
                ("max_depth", C.c_int32), ("device_bytes", C.c_int64), ("build_seconds", C.c_double)]


class rich_prefilter(C.Structure):
    _fields_ = [("enabled", C.c_int32), ("n_materials", C.c_int32), ("materials", C.c_int32 * 4)]


class rich_dispersion(C.Structure):
    _fields_ = [("n_nodes", C.c_int32), ("reserved", C.c_int32), ("lambda_", C.POINTER(C.c_double)),
                ("index", C.POINTER(C.c_double))]


class rich_source(C.Structure):
    _fields_ = [("kind", C.c_int32), ("reserved", C.c_int32), ("origin", _d3), ("direction", _d3),
                ("length", C.c_double), ("beta", C.c_double),
                ("dev_o", C.c_void_p), ("dev_d", C.c_void_p), ("dev_lambda", C.c_void_p),
                ("n_radiator", C.c_double), ("lambda_min", C.c_double), ("lambda_max", C.c_double),
                ("prefilter", rich_prefilter), ("dispersion", rich_dispersion)]


class rich_batch(C.Structure):
    _fields_ = [("dev_tracks", C.c_void_p), ("dev_offsets", C.c_void_p), ("n_tracks", C.c_int32),
                ("reserved", C.c_int32), ("n_radiator", C.c_double), ("lambda_min", C.c_double),
                ("lambda_max", C.c_double), ("prefilter", rich_prefilter), ("dispersion", rich_dispersion)]


class rich_outputs(C.Structure):
    _fields_ = [("fate", C.c_void_p), ("pixel", C.c_void_p), ("hit_xyz", C.c_void_p), ("hit_uv", C.c_void_p),
                ("histogram", C.c_void_p), ("fate_counts", C.c_void_p), ("hit_list", C.c_void_p),
                ("hit_list_capacity", C.c_uint64), ("hit_count", C.c_void_p), ("hit_time", C.c_void_p)]


class rich_film(C.Structure):
    _fields_ = [("width", C.c_int32), ("height", C.c_int32), ("distance", C.c_double), ("fov", C.c_double),
                ("sigma", C.c_double), ("threshold", C.c_double)]


class rich_fit(C.Structure):
    _fields_ = [("n_steps", C.c_int32), ("reserved", C.c_int32), ("lr", C.c_double), ("lr_final", C.c_double),
                ("beta1", C.c_double), ("beta2", C.c_double), ("eps", C.c_double), ("scale", C.c_double * 6),
                ("free", C.c_int32 * 6), ("outlier_cut", C.c_double), ("cut_floor", C.c_double)]


class rich_tuning(C.Structure):
    _fields_ = [("block", C.c_int32), ("chunk", C.c_int32), ("blocks_per_cu", C.c_int32), ("reserved", C.c_int32)]


_L.rich_build_scene.argtypes = [C.POINTER(rich_scene_desc), C.c_int, C.POINTER(C.c_void_p)]
_L.rich_destroy_scene.argtypes = [C.c_void_p]
_L.rich_scene_info.argtypes = [C.c_void_p, C.POINTER(rich_scene_stats)]
_L.rich_set_mirror_params.argtypes = [C.c_void_p, C.c_void_p, C.c_void_p]
_L.rich_propagate.argtypes = [C.c_void_p, C.POINTER(rich_source), C.c_uint64, C.c_uint64, C.c_uint64,
                              C.POINTER(rich_outputs), C.c_void_p]
_L.rich_propagate_batch.argtypes = [C.c_void_p, C.POINTER(rich_batch), C.c_uint64, C.c_uint64,
                                    C.POINTER(rich_outputs), C.POINTER(rich_tuning), C.c_void_p]
_L.rich_autotune.argtypes = [C.c_void_p, C.POINTER(rich_batch), C.c_uint64, C.c_uint64, C.POINTER(rich_tuning)]
_L.rich_propagate_adjoint.argtypes = [C.c_void_p, C.POINTER(rich_source), C.POINTER(rich_batch), C.c_uint64,
                                      C.c_uint64, C.c_uint64, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p,
                                      C.c_void_p, C.c_void_p, C.c_void_p]
_L.rich_propagate_adjoint_noalloc.argtypes = _L.rich_propagate_adjoint.argtypes
_L.rich_get_status.argtypes = [C.c_void_p, C.c_void_p, C.POINTER(C.c_uint32)]
_L.rich_film_readout.argtypes = [C.POINTER(rich_film), C.c_void_p, C.c_void_p, C.c_uint64, C.c_void_p, C.c_void_p,
                                 C.c_void_p]
_L.rich_fit_step.argtypes = [C.c_void_p, C.POINTER(rich_fit)] + [C.c_void_p] * 8
_L.rich_cherenkov_yield.argtypes = [C.POINTER(rich_dispersion), C.c_double, C.c_double, C.c_double, C.c_double,
                                    C.POINTER(C.c_double)]
_L.rich_last_error.restype = C.c_char_p
_L.rich_version.restype = C.c_char_p
for _f in ("rich_build_scene", "rich_destroy_scene", "rich_scene_info", "rich_set_mirror_params", "rich_propagate",
           "rich_propagate_batch", "rich_autotune", "rich_propagate_adjoint", "rich_propagate_adjoint_noalloc",
           "rich_get_status",
           "rich_cherenkov_yield", "rich_film_readout", "rich_fit_step"):
    getattr(_L, _f).restype = C.c_int32

EXPORTED = ("rich_build_scene", "rich_destroy_scene", "rich_scene_info", "rich_set_mirror_params",
            "rich_propagate", "rich_propagate_batch", "rich_autotune", "rich_propagate_adjoint",
            "rich_propagate_adjoint_noalloc",
            "rich_get_status", "rich_cherenkov_yield", "rich_film_readout", "rich_fit_step", "rich_last_error",
            "rich_version")


def _check(code):
    if code != RICH_OK:
        raise RichError(code, _L.rich_last_error().decode())


def _stream(stream):
    if stream is None:
        stream = torch.cuda.current_stream()
    return C.c_void_p(stream.cuda_stream if hasattr(stream, "cuda_stream") else int(stream))


def _ptr(t):
    return None if t is None else C.c_void_p(t.data_ptr())


# ------------------------------------------------------------------ C calls

def rich_version():
    return _L.rich_version().decode()


def rich_last_error():
    return _L.rich_last_error().decode()


def rich_build_scene(desc, device=0):
    h = C.c_void_p()
    _check(_L.rich_build_scene(C.byref(desc), int(device), C.byref(h)))
    return h


def rich_destroy_scene(handle):
    _check(_L.rich_destroy_scene(handle))


def rich_scene_info(handle):
    st = rich_scene_stats()
    _check(_L.rich_scene_info(handle, C.byref(st)))
    return {k: getattr(st, k) for k, _ in rich_scene_stats._fields_}


def rich_set_mirror_params(handle, dev_params, stream=None):
    _check(_L.rich_set_mirror_params(handle, _ptr(dev_params), _stream(stream)))


def rich_propagate(handle, source, n_photons, seed, first_photon_id, outputs, stream=None):
    _check(_L.rich_propagate(handle, C.byref(source), int(n_photons), int(seed), int(first_photon_id),
                             C.byref(outputs), _stream(stream)))


def rich_propagate_batch(handle, batch, n_photons, seed, outputs, tune=None, stream=None):
    _check(_L.rich_propagate_batch(handle, C.byref(batch), int(n_photons), int(seed), C.byref(outputs),
                                   None if tune is None else C.byref(tune), _stream(stream)))


def rich_autotune(handle, batch, n_photons, seed):
    t = rich_tuning()
    _check(_L.rich_autotune(handle, C.byref(batch), int(n_photons), int(seed), C.byref(t)))
    return t


def rich_propagate_adjoint(handle, source, batch, n_photons, seed, first_photon_id, dev_grad_uv, dev_targets,
                           dev_mask, dev_residual_cut, dev_grad_params, dev_loss, stream=None):
    _check(_L.rich_propagate_adjoint(handle, None if source is None else C.byref(source),
                                     None if batch is None else C.byref(batch), int(n_photons), int(seed),
                                     int(first_photon_id), _ptr(dev_grad_uv), _ptr(dev_targets), _ptr(dev_mask),
                                     _ptr(dev_residual_cut), _ptr(dev_grad_params), _ptr(dev_loss),
                                     _stream(stream)))


def rich_propagate_adjoint_noalloc(handle, source, batch, n_photons, seed, first_photon_id, dev_grad_uv,
                                   dev_targets, dev_mask, dev_residual_cut, dev_grad_params, dev_loss, stream=None):
    _check(_L.rich_propagate_adjoint_noalloc(handle, None if source is None else C.byref(source),
                                             None if batch is None else C.byref(batch), int(n_photons), int(seed),
                                             int(first_photon_id), _ptr(dev_grad_uv), _ptr(dev_targets),
                                             _ptr(dev_mask), _ptr(dev_residual_cut), _ptr(dev_grad_params),
                                             _ptr(dev_loss), _stream(stream)))


def rich_fit_step(handle, fit, dev_p0, dev_grad, dev_loss, dev_state, dev_params, dev_losses, dev_cut, stream=None):
    _check(_L.rich_fit_step(handle, C.byref(fit), _ptr(dev_p0), _ptr(dev_grad), _ptr(dev_loss), _ptr(dev_state),
                            _ptr(dev_params), _ptr(dev_losses), _ptr(dev_cut), _stream(stream)))


def fit_config(steps, lr, lr_final, scale, free, betas=(0.9, 0.999), eps=1e-12, outlier_cut=0.0, cut_floor=0.0):
    """rich_fit struct for rich_fit_step."""
    return rich_fit(int(steps), 0, float(lr), float(lr_final), float(betas[0]), float(betas[1]), float(eps),
                    (C.c_double * 6)(*[float(x) for x in scale]), (C.c_int32 * 6)(*[1 if f else 0 for f in free]),
                    float(outlier_cut), float(cut_floor))


def rich_cherenkov_yield(dispersion, n_radiator, beta, lambda_min, lambda_max):
    out = C.c_double()
    _check(_L.rich_cherenkov_yield(None if dispersion is None else C.byref(dispersion), float(n_radiator),
                                   float(beta), float(lambda_min), float(lambda_max), C.byref(out)))
    return out.value


def rich_film_readout(film, dev_fate, dev_hit_uv, n_photons, dev_image, dev_hits, stream=None):
    _check(_L.rich_film_readout(C.byref(film), _ptr(dev_fate), _ptr(dev_hit_uv), int(n_photons), _ptr(dev_image),
                                _ptr(dev_hits), _stream(stream)))


def film_readout(film, fate, hit_uv, image=None, stream=None):
    """Camera + film + threshold emulation (Section 4.4) of detected hits on the GPU; returns (image, hits)."""
    f = rich_film(int(film["width"]), int(film["height"]), float(film["distance"]), float(film["fov"]),
                  float(film["sigma"]), float(film["threshold"]))
    fate = torch.as_tensor(fate).to(device="cuda", dtype=torch.uint8).contiguous()
    uv = torch.as_tensor(hit_uv).to(device=fate.device, dtype=torch.float32).contiguous()
    if image is None:
        image = torch.zeros((f.height, f.width), dtype=torch.float32, device=fate.device)
    hits = torch.empty((f.height, f.width), dtype=torch.uint8, device=fate.device)
    rich_film_readout(f, fate, uv, fate.numel(), image, hits, stream)
    return image, hits


def rich_get_status(handle, stream=None):
    """Synchronise and return the device flags (does not raise on overflow flags)."""
    f = C.c_uint32(0)
    code = _L.rich_get_status(handle, _stream(stream), C.byref(f))
    if code not in (RICH_OK, RICH_EOVERFLOW):
        _check(code)
    return int(f.value)


# ------------------------------------------------------------------ scene marshalling

def _arr(a, keep):
    a = np.ascontiguousarray(a, dtype=np.float64)
    keep.append(a)
    return a.ctypes.data_as(_dp)


def scene_desc(scene, params=None):
    """rich_scene_desc from an ``inputs`` scene dict; returns (desc, keepalive list)."""
    keep = []
    mats = scene["materials"]
    mat_arr = (rich_material * len(mats))()
    for i, m in enumerate(mats):
        mat_arr[i].kind = int(m["kind"])
        mat_arr[i].n_refl = len(m["refl_lambda"])
        mat_arr[i].refl_lambda = _arr(m["refl_lambda"], keep)
        mat_arr[i].refl_value = _arr(m["refl_value"], keep)
    sg = scene["segments"]
    nseg = len(sg["radius0"])
    seg_arr = (rich_segment * max(nseg, 1))()
    for k in range(nseg):
        seg_arr[k].pivot[:] = list(map(float, sg["pivot"][k]))
        seg_arr[k].u0[:] = list(map(float, sg["u0"][k]))
        seg_arr[k].e1[:] = list(map(float, sg["e1"][k]))
        seg_arr[k].e2[:] = list(map(float, sg["e2"][k]))
        seg_arr[k].radius0 = float(sg["radius0"][k])
    p = np.asarray(scene["params"] if params is None else params, np.float64).reshape(-1, 6)
    cp = scene["caps"]
    ncap = len(cp["segment"])
    cap_arr = (rich_cap * max(ncap, 1))()
    for i in range(ncap):
        c = cap_arr[i]
        c.segment = int(cp["segment"][i])
        c.material = int(cp["material"][i])
        c.origin[:] = list(map(float, cp["origin"][i]))
        c.axis_a[:] = list(map(float, cp["axis_a"][i]))
        c.axis_b[:] = list(map(float, cp["axis_b"][i]))
        c.bounds[:] = list(map(float, cp["bounds"][i]))
    rc = scene["rects"]
    nrect = len(rc["material"])
    rect_arr = (rich_rect * max(nrect, 1))()
    for i in range(nrect):
        r = rect_arr[i]
        r.material = int(rc["material"][i])
        r.center[:] = list(map(float, rc["center"][i]))
        r.normal[:] = list(map(float, rc["normal"][i]))
        r.axis_u[:] = list(map(float, rc["axis_u"][i]))
        r.axis_v[:] = list(map(float, rc["axis_v"][i]))
        r.half[:] = list(map(float, rc["half"][i]))
    meshes = scene["meshes"]
    mesh_arr = (rich_mesh * max(len(meshes), 1))()
    for i, m in enumerate(meshes):
        mesh_arr[i].vertices = _arr(m["vertices"], keep)
        mesh_arr[i].n_tri = len(m["vertices"])
        mesh_arr[i].material = int(m["material"])
        mesh_arr[i].segment = int(m["segment"])
    det = scene["detector"]
    d = rich_scene_desc()
    d.n_materials = len(mats)
    d.materials = mat_arr
    d.n_segments = nseg
    d.segments = seg_arr
    d.params = _arr(p, keep) if nseg else None
    d.n_caps = ncap
    d.caps = cap_arr
    d.n_rects = nrect
    d.rects = rect_arr
    d.n_meshes = len(meshes)
    d.meshes = mesh_arr
    dd = d.detector
    dd.center[:] = list(map(float, det["center"]))
    dd.normal[:] = list(map(float, det["normal"]))
    dd.axis_u[:] = list(map(float, det["axis_u"]))
    dd.axis_v[:] = list(map(float, det["axis_v"]))
    dd.half[:] = list(map(float, det["half"]))
    dd.pitch = float(det["pitch"])
    dd.nx = int(det["nx"])
    dd.ny = int(det["ny"])
    dd.n_qe = len(det["qe_lambda"])
    dd.qe_lambda = _arr(det["qe_lambda"], keep)
    dd.qe_value = _arr(det["qe_value"], keep)
    box = scene["box"]
    d.has_box = 0 if box is None else 1
    if box is not None:
        d.box_lo[:] = list(map(float, box["lo"]))
        d.box_hi[:] = list(map(float, box["hi"]))
    d.max_bounces = int(scene["max_bounces"])
    d.t_min = float(scene["t_min"])
    keep += [mat_arr, seg_arr, cap_arr, rect_arr, mesh_arr]
    return d, keep


class Scene:
    """A device scene built by rich_build_scene from an ``inputs`` scene dict."""

    def __init__(self, scene, device=0, params=None):
        desc, keep = scene_desc(scene, params)
        self.handle = rich_build_scene(desc, device)
        self.device = device
        det = scene["detector"]
        self.nx, self.ny = int(det["nx"]), int(det["ny"])
        self.n_segments = len(scene["segments"]["radius0"])
        self.params0 = np.array(scene["params"] if params is None else params, np.float32)

    def info(self):
        return rich_scene_info(self.handle)

    def set_params(self, params, stream=None):
        t = torch.as_tensor(np.asarray(params, np.float32) if not torch.is_tensor(params) else params)
        t = t.to(device=f"cuda:{self.device}", dtype=torch.float32).contiguous()
        rich_set_mirror_params(self.handle, t, stream)
        return t

    def status(self, stream=None):
        return rich_get_status(self.handle, stream)

    def close(self):
        if getattr(self, "handle", None):
            rich_destroy_scene(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# ------------------------------------------------------------------ sources and outputs

def _set_prefilter(pf_struct, mats):
    if mats is None:
        return
    pf_struct.enabled = 1
    pf_struct.n_materials = len(mats)
    for k, m in enumerate(mats):
        pf_struct.materials[k] = int(m)


def _set_dispersion(d_struct, table, keep):
    if table is None:
        return
    x = np.ascontiguousarray(table["lambda"], np.float64)
    n = np.ascontiguousarray(table["index"], np.float64)
    if x.shape != n.shape:
        raise ValueError("dispersion: lambda and index differ in length")
    keep += [x, n]
    d_struct.n_nodes = len(x)
    d_struct.lambda_ = x.ctypes.data_as(C.POINTER(C.c_double))
    d_struct.index = n.ctypes.data_as(C.POINTER(C.c_double))


def cherenkov_yield(src, beta):
    """Cherenkov photons per mm of track at velocity beta for a source dict's radiator."""
    keep = []
    d = rich_dispersion()
    _set_dispersion(d, src.get("dispersion"), keep)
    return rich_cherenkov_yield(d, src.get("n_radiator", 1.0), beta, src.get("lambda_min", 200.0),
                                src.get("lambda_max", 600.0))


def make_source(src, device="cuda"):
    """rich_source for a 'track' or 'explicit' source dict; returns (source, keepalive)."""
    s = rich_source()
    keep = []
    _set_prefilter(s.prefilter, src.get("prefilter"))
    _set_dispersion(s.dispersion, src.get("dispersion"), keep)
    s.n_radiator = float(src.get("n_radiator", 1.0))
    s.lambda_min = float(src.get("lambda_min", 200.0))
    s.lambda_max = float(src.get("lambda_max", 600.0))
    if src["kind"] == "track":
        s.kind = SRC_TRACK
        s.origin[:] = list(map(float, src["origin"]))
        s.direction[:] = list(map(float, src["direction"]))
        s.length = float(src["length"])
        s.beta = float(src["beta"])
    elif src["kind"] == "explicit":
        s.kind = SRC_EXPLICIT
        o = torch.as_tensor(np.asarray(src["o"], np.float32), device=device).contiguous()
        d = torch.as_tensor(np.asarray(src["d"], np.float32), device=device).contiguous()
        lam = torch.as_tensor(np.asarray(src["lambda"], np.float32), device=device).contiguous()
        keep += [o, d, lam]
        s.dev_o, s.dev_d, s.dev_lambda = o.data_ptr(), d.data_ptr(), lam.data_ptr()
    else:
        raise ValueError(f"not a single source: {src['kind']}")
    return s, keep


def make_batch(src, device="cuda"):
    """rich_batch for a 'batch' source dict; returns (batch, keepalive, n_photons)."""
    tracks = torch.as_tensor(np.asarray(src["tracks"], np.float32), device=device).contiguous()
    offsets = torch.as_tensor(np.asarray(src["offsets"], np.uint64).view(np.int64), device=device).contiguous()
    b = rich_batch()
    b.dev_tracks = tracks.data_ptr()
    b.dev_offsets = offsets.data_ptr()
    b.n_tracks = int(tracks.shape[0])
    b.n_radiator = float(src["n_radiator"])
    b.lambda_min = float(src["lambda_min"])
    b.lambda_max = float(src["lambda_max"])
    _set_prefilter(b.prefilter, src.get("prefilter"))
    keep = [tracks, offsets]
    _set_dispersion(b.dispersion, src.get("dispersion"), keep)
    return b, keep, int(np.asarray(src["offsets"])[-1])


def alloc_outputs(scene, n, device="cuda", per_photon=True, hit_list_capacity=0):
    """Zeroed output tensors and the rich_outputs struct pointing at them."""
    t = {}
    if per_photon:
        t["fate"] = torch.empty(n, dtype=torch.uint8, device=device)
        t["pixel"] = torch.empty(n, dtype=torch.int32, device=device)
        t["hit_xyz"] = torch.empty((n, 3), dtype=torch.float32, device=device)
        t["hit_uv"] = torch.empty((n, 2), dtype=torch.float32, device=device)
        t["hit_time"] = torch.empty(n, dtype=torch.float32, device=device)
    t["histogram"] = torch.zeros(scene.nx * scene.ny, dtype=torch.int32, device=device)
    t["fate_counts"] = torch.zeros(N_FATES, dtype=torch.int64, device=device)
    if hit_list_capacity:
        t["hit_list"] = torch.zeros((hit_list_capacity, 24), dtype=torch.uint8, device=device)
        t["hit_count"] = torch.zeros(1, dtype=torch.int64, device=device)
    return t, outputs_struct(t)


def outputs_struct(t):
    o = rich_outputs()
    for k in ("fate", "pixel", "hit_xyz", "hit_uv", "histogram", "fate_counts", "hit_list", "hit_count", "hit_time"):
        if k in t and t[k] is not None:
            setattr(o, k, t[k].data_ptr())
    if "hit_list" in t and t["hit_list"] is not None:
        o.hit_list_capacity = int(t["hit_list"].shape[0])
    return o


def decode_hits(hit_list, count):
    """(photon id, pixel, xyz) arrays from a rich_hit byte tensor."""
    raw = hit_list[: int(count)].cpu().numpy()
    ids = raw[:, 0:8].copy().view(np.uint64).reshape(-1)
    pix = raw[:, 8:12].copy().view(np.int32).reshape(-1)
    xyz = raw[:, 12:24].copy().view(np.float32).reshape(-1, 3)
    return ids, pix, xyz


# ------------------------------------------------------------------ convenience calls

def propagate(scene, src, n, seed, first_id=0, hit_list_capacity=0, stream=None):
    device = f"cuda:{scene.device}"
    s, keep = make_source(src, device)
    t, o = alloc_outputs(scene, n, device, hit_list_capacity=hit_list_capacity)
    rich_propagate(scene.handle, s, n, seed, first_id, o, stream)
    t["_keep"] = keep
    return t


def propagate_batch(scene, src, seed, tune=None, hit_list_capacity=0, stream=None):
    device = f"cuda:{scene.device}"
    b, keep, n = make_batch(src, device)
    t, o = alloc_outputs(scene, n, device, hit_list_capacity=hit_list_capacity)
    rich_propagate_batch(scene.handle, b, n, seed, o, tune, stream)
    t["_keep"] = keep
    return t


def tuning(block, chunk, blocks_per_cu):
    return rich_tuning(int(block), int(chunk), int(blocks_per_cu), 0)


def adjoint(scene, src, seed, n=None, first_id=0, grad_uv=None, targets=None, mask=None, residual_cut=None,
            stream=None):
    """Reverse-mode gradient of the hits w.r.t. the segment parameters at the scene's current parameters.

    Exactly one of grad_uv ([N,2] upstream dL/d(u,v)) and targets ([N,2], fused mean-squared loss) is
    given; residual_cut (fused mode, mm) leaves out photons whose |uv - target| exceeds it.
    Returns (grad [n_segments, 6] float32 tensor, loss [1] tensor).
    """
    device = f"cuda:{scene.device}"
    keep = []
    if src["kind"] == "batch":
        b, keep, nb = make_batch(src, device)
        s = None
        n = nb if n is None else n
    else:
        s, keep = make_source(src, device)
        b = None
    if n is None:
        raise ValueError("n is required for single sources")

    def dev(x, dtype):
        if x is None:
            return None
        t = x if torch.is_tensor(x) else torch.as_tensor(np.asarray(x))
        return t.to(device=device, dtype=dtype).contiguous()

    gu = dev(grad_uv, torch.float32)
    tg = dev(targets, torch.float32)
    mk = dev(mask, torch.uint8)
    rc = None if residual_cut is None else dev(torch.as_tensor([float(residual_cut)]), torch.float32)
    grad = torch.zeros((scene.n_segments, 6), dtype=torch.float32, device=device)
    loss = torch.zeros(1, dtype=torch.float32, device=device)
    rich_propagate_adjoint(scene.handle, s, b, n, seed, first_id, gu, tg, mk, rc, grad, loss, stream)
    keep += [gu, tg, mk, rc]
    grad._keep = keep
    return grad, loss
