"""Thin Python binding of libdhr (include/dhr.h): argument marshalling only.

Every function carries the C name and forwards torch tensors as device
pointers on torch's current HIP stream.  Nothing here computes any step of
the method; if the library is missing the import fails loudly (there is no
CPU fallback).

torch is imported first so that libdhr resolves to the HIP runtime torch has
already loaded (both carry the same SONAME).
"""
from __future__ import annotations

import ctypes as C
import math
import os

import torch

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libdhr.so")

MAX_LIGHTS = 8
MAX_LEVELS = 8
MISS_ID = 0xFFFFFFFF
STATUS = {0: "OK", 1: "INVALID_ARG", 2: "OOM", 3: "DEVICE", 4: "UNSUPPORTED"}


class DhrError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{STATUS.get(status, status)}: {msg}")
        self.status = status


# ----------------------------------------------------------------------------
# structs (mirror include/dhr.h)
# ----------------------------------------------------------------------------

class dhr_bvh_opts(C.Structure):
    _fields_ = [("max_leaf", C.c_uint32), ("max_depth", C.c_uint32), ("sah_bins", C.c_uint32),
                ("threads", C.c_uint32)]


class dhr_bvh_info(C.Structure):
    _fields_ = [("n_nodes", C.c_uint64), ("n_tris", C.c_uint64), ("device_bytes", C.c_uint64),
                ("depth", C.c_uint32), ("max_leaf_size", C.c_uint32), ("sah_cost", C.c_double),
                ("build_ms", C.c_double)]


class dhr_camera(C.Structure):
    _fields_ = [("eye", C.c_float * 3), ("target", C.c_float * 3), ("fov_y", C.c_float)]


class dhr_light(C.Structure):
    _fields_ = [("kind", C.c_uint32), ("vec", C.c_float * 3), ("one_minus_cos", C.c_float),
                ("radius", C.c_float)]


class dhr_trace_params(C.Structure):
    _fields_ = [("W", C.c_uint32), ("H", C.c_uint32), ("frame", C.c_uint32), ("client_id", C.c_uint32),
                ("seed", C.c_uint32), ("n_ao", C.c_uint32), ("ao_sample_offset", C.c_uint32),
                ("ao_radius", C.c_float), ("n_shadow", C.c_uint32), ("n_lights", C.c_uint32),
                ("lights", dhr_light * MAX_LIGHTS), ("eps_origin_abs", C.c_float)]


class dhr_gbuffer_job(C.Structure):
    _fields_ = [("bvh", C.c_void_p), ("cur", dhr_camera), ("prev", dhr_camera), ("has_prev", C.c_uint32),
                ("W", C.c_uint32), ("H", C.c_uint32), ("pos", C.c_void_p), ("nz", C.c_void_p),
                ("dz", C.c_void_p), ("mv", C.c_void_p)]


class dhr_trace_job(C.Structure):
    _fields_ = [("bvh", C.c_void_p), ("params", dhr_trace_params), ("pos", C.c_void_p), ("nz", C.c_void_p),
                ("ao_count", C.c_void_p), ("shadow_count", C.c_void_p)]


class dhr_svgf_params(C.Structure):
    _fields_ = [("levels", C.c_uint32), ("alpha", C.c_float), ("alpha_moments", C.c_float),
                ("sigma_z", C.c_float * MAX_LEVELS), ("sigma_n", C.c_float * MAX_LEVELS),
                ("sigma_l", C.c_float * MAX_LEVELS), ("eps_z_rel", C.c_float), ("eps_l", C.c_float),
                ("cos_normal_min", C.c_float), ("plane_px", C.c_float), ("use_obj_id", C.c_uint32),
                ("var_min_history", C.c_uint32), ("fallback_radius", C.c_uint32),
                ("feedback_level", C.c_uint32), ("history_cap", C.c_float), ("kernel_width", C.c_uint32)]


class dhr_svgf_frame(C.Structure):
    _fields_ = [("W", C.c_uint32), ("H", C.c_uint32), ("n_ao", C.c_uint32), ("ao_count", C.c_void_p),
                ("pos", C.c_void_p), ("nz", C.c_void_p), ("dz", C.c_void_p), ("mv", C.c_void_p),
                ("prev_pos", C.c_void_p), ("prev_nz", C.c_void_p), ("hist_in", C.c_void_p),
                ("hist_out", C.c_void_p), ("out", C.c_void_p), ("save", C.c_void_p), ("work", C.c_void_p),
                ("pix", C.c_float)]


class dhr_svgf_spatial_frame(C.Structure):
    _fields_ = [("W", C.c_uint32), ("H", C.c_uint32), ("cv_in", C.c_void_p), ("nz", C.c_void_p),
                ("dz", C.c_void_p), ("out", C.c_void_p), ("save", C.c_void_p), ("work", C.c_void_p)]


class dhr_svgf_bwd_frame(C.Structure):
    _fields_ = [("W", C.c_uint32), ("H", C.c_uint32), ("save", C.c_void_p), ("nz", C.c_void_p),
                ("dz", C.c_void_p), ("grad_out", C.c_void_p), ("grad_cv", C.c_void_p), ("work", C.c_void_p)]


# every symbol include/dhr.h declares
EXPORTS = ["dhr_create", "dhr_destroy", "dhr_last_error", "dhr_sync", "dhr_version", "dhr_build_bvh",
           "dhr_bvh_get_info", "dhr_bvh_destroy", "dhr_gbuffer", "dhr_trace_visibility", "dhr_gbuffer_batch",
           "dhr_trace_visibility_batch", "dhr_svgf_default_params", "dhr_svgf_filter", "dhr_svgf_spatial_forward",
           "dhr_svgf_backward", "dhr_svgf_workspace_bytes", "dhr_philox4x32_10", "dhr_set_trace_counters",
           "dhr_encode_frame", "dhr_build_bvh_device", "dhr_refit_bvh", "dhr_bvh_export",
           "dhr_gbuffer_raster_workspace_bytes", "dhr_gbuffer_raster", "dhr_build_bvh_instanced",
           "dhr_gbuffer_trace", "dhr_gbuffer_trace_batch", "dhr_svgf_filter_noalloc"]

# bytes of the library-owned scratch of dhr_svgf_filter_noalloc (per GPU)
SVGF_NOALLOC_SCRATCH_BYTES = 64 << 20

_lib = None


def load(path: str = LIB_PATH):
    """Load libdhr.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"{path} is missing: build the HIP library first (__graft_entry__.build())")
    L = C.CDLL(path)
    missing = [name for name in EXPORTS if not hasattr(L, name)]
    if missing:
        raise RuntimeError(f"{path} lacks {missing}: rebuild the HIP library")
    vp, u32, u64, i32 = C.c_void_p, C.c_uint32, C.c_uint64, C.c_int
    L.dhr_create.argtypes = [i32, C.POINTER(vp)]
    L.dhr_destroy.argtypes = [vp]
    L.dhr_destroy.restype = None
    L.dhr_last_error.argtypes = [vp]
    L.dhr_last_error.restype = C.c_char_p
    L.dhr_sync.argtypes = [vp, vp]
    L.dhr_version.restype = C.c_char_p
    L.dhr_build_bvh.argtypes = [vp, vp, vp, u32, C.POINTER(dhr_bvh_opts), C.POINTER(vp)]
    L.dhr_bvh_get_info.argtypes = [vp, C.POINTER(dhr_bvh_info)]
    L.dhr_bvh_destroy.argtypes = [vp]
    L.dhr_bvh_destroy.restype = None
    L.dhr_gbuffer.argtypes = [vp, vp, C.POINTER(dhr_camera), C.POINTER(dhr_camera), u32, u32, vp, vp, vp, vp, vp]
    L.dhr_trace_visibility.argtypes = [vp, vp, C.POINTER(dhr_trace_params), vp, vp, vp, vp, vp, vp]
    L.dhr_gbuffer_batch.argtypes = [vp, C.POINTER(dhr_gbuffer_job), u32, vp]
    L.dhr_trace_visibility_batch.argtypes = [vp, C.POINTER(dhr_trace_job), u32, vp]
    L.dhr_gbuffer_trace.argtypes = [vp, vp, C.POINTER(dhr_camera), C.POINTER(dhr_camera), u32, u32,
                                    C.POINTER(dhr_trace_params), vp, vp, vp, vp, vp, vp, vp]
    L.dhr_gbuffer_trace_batch.argtypes = [vp, C.POINTER(dhr_gbuffer_job), C.POINTER(dhr_trace_job), u32, vp]
    L.dhr_svgf_default_params.argtypes = [C.POINTER(dhr_svgf_params)]
    L.dhr_svgf_default_params.restype = None
    L.dhr_svgf_filter.argtypes = [vp, C.POINTER(dhr_svgf_params), C.POINTER(dhr_svgf_frame), u32, vp]
    L.dhr_svgf_filter_noalloc.argtypes = [vp, C.POINTER(dhr_svgf_params), C.POINTER(dhr_svgf_frame), u32, vp]
    L.dhr_svgf_spatial_forward.argtypes = [vp, C.POINTER(dhr_svgf_params), C.POINTER(dhr_svgf_spatial_frame), u32, vp]
    L.dhr_svgf_backward.argtypes = [vp, C.POINTER(dhr_svgf_params), C.POINTER(dhr_svgf_bwd_frame), u32, vp, vp]
    L.dhr_svgf_workspace_bytes.argtypes = [u32, u32, C.POINTER(dhr_svgf_params), i32]
    L.dhr_svgf_workspace_bytes.restype = u64
    L.dhr_philox4x32_10.argtypes = [vp, u32, u32, vp, vp, u64, vp]
    L.dhr_set_trace_counters.argtypes = [vp, vp]
    L.dhr_encode_frame.argtypes = [vp, vp, vp, vp, u32, u32, vp, u64, vp]
    L.dhr_build_bvh_device.argtypes = [vp, vp, vp, u32, vp, vp]
    L.dhr_refit_bvh.argtypes = [vp, vp, vp, vp]
    L.dhr_bvh_export.argtypes = [vp, vp, vp, vp, vp]
    L.dhr_build_bvh_instanced.argtypes = [vp, vp, vp, u32, vp, u32, vp, vp, u32, C.POINTER(dhr_bvh_opts),
                                          C.POINTER(vp)]
    L.dhr_gbuffer_raster_workspace_bytes.argtypes = [u32, u32, u32]
    L.dhr_gbuffer_raster_workspace_bytes.restype = u64
    L.dhr_gbuffer_raster.argtypes = [vp, vp, C.POINTER(dhr_camera), C.POINTER(dhr_camera), u32, u32, vp, vp, vp, vp,
                                     vp, u64, vp]
    _lib = L
    return L


# ----------------------------------------------------------------------------
# handles
# ----------------------------------------------------------------------------

class Context:
    def __init__(self, handle, device):
        self.handle = handle
        self.device = device

    def close(self):
        if self.handle and _lib is not None:
            _lib.dhr_destroy(self.handle)
        self.handle = None

    def __del__(self):
        self.close()


class Bvh:
    def __init__(self, ctx: Context, handle):
        self.ctx = ctx
        self.handle = handle

    def info(self) -> dict:
        info = dhr_bvh_info()
        _check(self.ctx, load().dhr_bvh_get_info(self.handle, C.byref(info)), "dhr_bvh_get_info")
        return {k: getattr(info, k) for k, _ in dhr_bvh_info._fields_}

    def close(self):
        if self.handle and _lib is not None:
            _lib.dhr_bvh_destroy(self.handle)
        self.handle = None

    def __del__(self):
        self.close()


def _check(ctx, status, what):
    if status != 0:
        msg = load().dhr_last_error(ctx.handle if ctx is not None else None).decode()
        raise DhrError(status, f"{what}: {msg}")


def _ptr(t):
    if t is None:
        return None
    if not isinstance(t, torch.Tensor):
        raise TypeError("expected a torch tensor")
    if not t.is_cuda:
        raise ValueError("expected a device tensor")
    if not t.is_contiguous():
        raise ValueError("expected a contiguous tensor")
    return t.data_ptr()


def _stream(stream=None):
    s = stream if stream is not None else torch.cuda.current_stream()
    return s.cuda_stream


# ----------------------------------------------------------------------------
# parameter helpers
# ----------------------------------------------------------------------------

def camera(cam) -> dhr_camera:
    """dhr_camera from any object with eye, target, fov_y."""
    c = dhr_camera()
    for k in range(3):
        c.eye[k] = float(cam.eye[k])
        c.target[k] = float(cam.target[k])
    c.fov_y = float(cam.fov_y)
    return c


def trace_params(W, H, *, frame=0, client_id=0, seed=0, n_ao=1, ao_sample_offset=0, ao_radius=1.0,
                 n_shadow=1, lights=(), eps_origin_abs=0.0) -> dhr_trace_params:
    p = dhr_trace_params()
    p.W, p.H, p.frame, p.client_id, p.seed = W, H, frame, client_id, seed
    p.n_ao, p.ao_sample_offset, p.ao_radius = n_ao, ao_sample_offset, ao_radius
    p.n_shadow, p.n_lights = n_shadow, len(lights)
    for k, L in enumerate(lights):
        p.lights[k].kind = int(L.kind)
        for j in range(3):
            p.lights[k].vec[j] = float(L.vec[j])
        p.lights[k].one_minus_cos = float(L.one_minus_cos)
        p.lights[k].radius = float(L.radius)
    p.eps_origin_abs = eps_origin_abs
    return p


def svgf_params(**kw) -> dhr_svgf_params:
    """Defaults of dhr_svgf_default_params, with keyword overrides (sigma_* may be
    scalars or per-level sequences)."""
    p = dhr_svgf_params()
    load().dhr_svgf_default_params(C.byref(p))
    for k, v in kw.items():
        if k.startswith("sigma_"):
            arr = getattr(p, k)
            vals = list(v) if hasattr(v, "__len__") else [v] * MAX_LEVELS
            for i, x in enumerate(vals[:MAX_LEVELS]):
                arr[i] = float(x)
        else:
            setattr(p, k, v)
    return p


def pix_angle(cam, H) -> float:
    return 2.0 * math.tan(0.5 * float(cam.fov_y)) / H


# ----------------------------------------------------------------------------
# the C calls
# ----------------------------------------------------------------------------

def dhr_version() -> str:
    return load().dhr_version().decode()


def dhr_create(device: int = 0) -> Context:
    L = load()
    h = C.c_void_p()
    st = L.dhr_create(int(device), C.byref(h))
    if st != 0:
        raise DhrError(st, f"dhr_create(device={device}) failed")
    return Context(h, device)


def dhr_sync(ctx: Context, stream=None):
    _check(ctx, load().dhr_sync(ctx.handle, _stream(stream)), "dhr_sync")


def dhr_build_bvh(ctx: Context, tris, obj_id=None, max_leaf=4, max_depth=32, sah_bins=64, threads=0) -> Bvh:
    import numpy as np
    t = np.ascontiguousarray(tris, dtype=np.float32).reshape(-1, 9)
    ids = None if obj_id is None else np.ascontiguousarray(obj_id, dtype=np.uint32)
    opts = dhr_bvh_opts(max_leaf, max_depth, sah_bins, threads)
    h = C.c_void_p()
    st = load().dhr_build_bvh(ctx.handle, t.ctypes.data_as(C.c_void_p),
                              None if ids is None else ids.ctypes.data_as(C.c_void_p), t.shape[0],
                              C.byref(opts), C.byref(h))
    _check(ctx, st, "dhr_build_bvh")
    return Bvh(ctx, h)


def dhr_build_bvh_instanced(ctx: Context, base_tris, base_obj, mesh_tris, xforms, inst_obj=None, max_leaf=4,
                            max_depth=32, sah_bins=64, threads=0) -> Bvh:
    """Host arrays: base_tris [n,3,3], base_obj [n] or None, mesh_tris [m,3,3],
    xforms [k,3,4] (object to world), inst_obj [k] or None."""
    import numpy as np
    bt = np.ascontiguousarray(base_tris, dtype=np.float32).reshape(-1, 9)
    bo = None if base_obj is None else np.ascontiguousarray(base_obj, dtype=np.uint32)
    mt = np.ascontiguousarray(mesh_tris, dtype=np.float32).reshape(-1, 9)
    xf = np.ascontiguousarray(xforms, dtype=np.float32).reshape(-1, 12)
    io = None if inst_obj is None else np.ascontiguousarray(inst_obj, dtype=np.uint32)
    opts = dhr_bvh_opts(max_leaf, max_depth, sah_bins, threads)
    h = C.c_void_p()
    p = lambda a: None if a is None else a.ctypes.data_as(C.c_void_p)
    st = load().dhr_build_bvh_instanced(ctx.handle, p(bt), p(bo), bt.shape[0], p(mt), mt.shape[0], p(xf), p(io),
                                        xf.shape[0], C.byref(opts), C.byref(h))
    _check(ctx, st, "dhr_build_bvh_instanced")
    return Bvh(ctx, h)


def dhr_gbuffer(ctx, bvh, cur, prev, W, H, pos, nz, dz, mv, stream=None):
    c = camera(cur)
    p = camera(prev) if prev is not None else None
    st = load().dhr_gbuffer(ctx.handle, bvh.handle, C.byref(c), C.byref(p) if p is not None else None, W, H,
                            _ptr(pos), _ptr(nz), _ptr(dz), _ptr(mv), _stream(stream))
    _check(ctx, st, "dhr_gbuffer")


def dhr_gbuffer_raster_workspace_bytes(W, H, n_tris) -> int:
    return int(load().dhr_gbuffer_raster_workspace_bytes(W, H, n_tris))


def dhr_gbuffer_raster(ctx, bvh, cur, prev, W, H, pos, nz, dz, mv, work, stream=None):
    """work: a device tensor of at least dhr_gbuffer_raster_workspace_bytes bytes."""
    c = camera(cur)
    p = camera(prev) if prev is not None else None
    nbytes = work.numel() * work.element_size()
    st = load().dhr_gbuffer_raster(ctx.handle, bvh.handle, C.byref(c), C.byref(p) if p is not None else None, W, H,
                                   _ptr(pos), _ptr(nz), _ptr(dz), _ptr(mv), _ptr(work), nbytes, _stream(stream))
    _check(ctx, st, "dhr_gbuffer_raster")


def dhr_trace_visibility(ctx, bvh, params, pos, nz, ao_count, shadow_count, debug_ray_bits=None, stream=None):
    st = load().dhr_trace_visibility(ctx.handle, bvh.handle, C.byref(params), _ptr(pos), _ptr(nz), _ptr(ao_count),
                                     _ptr(shadow_count), _ptr(debug_ray_bits), _stream(stream))
    _check(ctx, st, "dhr_trace_visibility")


def _gbuffer_jobs(jobs):
    arr = (dhr_gbuffer_job * max(len(jobs), 1))()
    for k, j in enumerate(jobs):
        a = arr[k]
        a.bvh = j["bvh"].handle
        a.cur = camera(j["cur"])
        if j.get("prev") is not None:
            a.prev = camera(j["prev"])
            a.has_prev = 1
        a.W, a.H = j["W"], j["H"]
        a.pos, a.nz, a.dz, a.mv = _ptr(j["pos"]), _ptr(j["nz"]), _ptr(j["dz"]), _ptr(j["mv"])
    return arr


def _trace_jobs(jobs):
    arr = (dhr_trace_job * max(len(jobs), 1))()
    for k, j in enumerate(jobs):
        a = arr[k]
        a.bvh = j["bvh"].handle
        a.params = j["params"]
        a.pos, a.nz = _ptr(j["pos"]), _ptr(j["nz"])
        a.ao_count, a.shadow_count = _ptr(j["ao_count"]), _ptr(j.get("shadow_count"))
    return arr


def dhr_gbuffer_batch(ctx, jobs, stream=None):
    """jobs: list of dicts(bvh, cur, prev, W, H, pos, nz, dz, mv)."""
    _check(ctx, load().dhr_gbuffer_batch(ctx.handle, _gbuffer_jobs(jobs), len(jobs), _stream(stream)),
           "dhr_gbuffer_batch")


def dhr_trace_visibility_batch(ctx, jobs, stream=None):
    """jobs: list of dicts(bvh, params, pos, nz, ao_count, shadow_count)."""
    _check(ctx, load().dhr_trace_visibility_batch(ctx.handle, _trace_jobs(jobs), len(jobs), _stream(stream)),
           "dhr_trace_visibility_batch")


def dhr_gbuffer_trace(ctx, bvh, cur, prev, W, H, params, pos, nz, dz, mv, ao_count, shadow_count, stream=None):
    c = camera(cur)
    p = camera(prev) if prev is not None else None
    st = load().dhr_gbuffer_trace(ctx.handle, bvh.handle, C.byref(c), C.byref(p) if p is not None else None, W, H,
                                  C.byref(params), _ptr(pos), _ptr(nz), _ptr(dz), _ptr(mv), _ptr(ao_count),
                                  _ptr(shadow_count), _stream(stream))
    _check(ctx, st, "dhr_gbuffer_trace")


def dhr_gbuffer_trace_batch(ctx, gbuffer_jobs, trace_jobs, stream=None):
    """Two lists of the dicts dhr_gbuffer_batch and dhr_trace_visibility_batch take, job k of each one frame."""
    n = len(gbuffer_jobs)
    if len(trace_jobs) != n:
        raise ValueError("dhr_gbuffer_trace_batch: the two job lists differ in length")
    _check(ctx, load().dhr_gbuffer_trace_batch(ctx.handle, _gbuffer_jobs(gbuffer_jobs), _trace_jobs(trace_jobs), n,
                                               _stream(stream)), "dhr_gbuffer_trace_batch")


def dhr_svgf_workspace_bytes(W, H, params, which=0) -> int:
    return int(load().dhr_svgf_workspace_bytes(W, H, C.byref(params), which))


def svgf_frame(W, H, n_ao, ao_count, pos, nz, dz, mv, prev_pos, prev_nz, hist_in, hist_out, out, pix,
               save=None, work=None) -> dhr_svgf_frame:
    f = dhr_svgf_frame()
    f.W, f.H, f.n_ao = W, H, n_ao
    f.ao_count = _ptr(ao_count)
    f.pos, f.nz, f.dz, f.mv = _ptr(pos), _ptr(nz), _ptr(dz), _ptr(mv)
    f.prev_pos, f.prev_nz, f.hist_in = _ptr(prev_pos), _ptr(prev_nz), _ptr(hist_in)
    f.hist_out, f.out, f.save, f.work = _ptr(hist_out), _ptr(out), _ptr(save), _ptr(work)
    f.pix = pix
    return f


def dhr_svgf_filter(ctx, params, frames, stream=None):
    arr = (dhr_svgf_frame * max(len(frames), 1))(*frames)
    _check(ctx, load().dhr_svgf_filter(ctx.handle, C.byref(params), arr, len(frames), _stream(stream)),
           "dhr_svgf_filter")


def dhr_svgf_filter_noalloc(ctx, params, frames, stream=None):
    """dhr_svgf_filter with the library's own scratch (frames without work)."""
    arr = (dhr_svgf_frame * max(len(frames), 1))(*frames)
    _check(ctx, load().dhr_svgf_filter_noalloc(ctx.handle, C.byref(params), arr, len(frames), _stream(stream)),
           "dhr_svgf_filter_noalloc")


def spatial_frame(W, H, cv_in, nz, dz, out, save=None, work=None) -> dhr_svgf_spatial_frame:
    f = dhr_svgf_spatial_frame()
    f.W, f.H = W, H
    f.cv_in, f.nz, f.dz, f.out, f.save, f.work = _ptr(cv_in), _ptr(nz), _ptr(dz), _ptr(out), _ptr(save), _ptr(work)
    return f


def dhr_svgf_spatial_forward(ctx, params, frames, stream=None):
    arr = (dhr_svgf_spatial_frame * max(len(frames), 1))(*frames)
    _check(ctx, load().dhr_svgf_spatial_forward(ctx.handle, C.byref(params), arr, len(frames), _stream(stream)),
           "dhr_svgf_spatial_forward")


def bwd_frame(W, H, save, nz, dz, grad_out, grad_cv, work) -> dhr_svgf_bwd_frame:
    f = dhr_svgf_bwd_frame()
    f.W, f.H = W, H
    f.save, f.nz, f.dz, f.grad_out, f.grad_cv, f.work = (_ptr(save), _ptr(nz), _ptr(dz), _ptr(grad_out),
                                                          _ptr(grad_cv), _ptr(work))
    return f


def dhr_svgf_backward(ctx, params, frames, grad_sigma, stream=None):
    arr = (dhr_svgf_bwd_frame * max(len(frames), 1))(*frames)
    _check(ctx, load().dhr_svgf_backward(ctx.handle, C.byref(params), arr, len(frames), _ptr(grad_sigma),
                                         _stream(stream)), "dhr_svgf_backward")


def dhr_set_trace_counters(ctx, counters=None):
    """counters: device int64 tensor of 4 (rays, node visits, leaf visits,
    triangle tests) accumulated by later trace calls, or None to switch off."""
    _check(ctx, load().dhr_set_trace_counters(ctx.handle, _ptr(counters)), "dhr_set_trace_counters")


def dhr_philox4x32_10(ctx, key, ctr, out, stream=None):
    n = ctr.numel() // 4
    _check(ctx, load().dhr_philox4x32_10(ctx.handle, int(key[0]), int(key[1]), _ptr(ctr), _ptr(out), n,
                                         _stream(stream)), "dhr_philox4x32_10")


def dhr_build_bvh_device(ctx: Context, tris, obj_id=None, stream=None) -> Bvh:
    """tris: device float tensor [T, 9] (or [T, 3, 3]); obj_id: device uint32/int32 tensor [T] or None."""
    t = tris.reshape(-1, 9)
    h = C.c_void_p()
    _check(ctx, load().dhr_build_bvh_device(ctx.handle, _ptr(t), _ptr(obj_id), t.shape[0], C.byref(h),
                                            _stream(stream)), "dhr_build_bvh_device")
    return Bvh(ctx, h)


def dhr_bvh_export(ctx: Context, bvh: Bvh, stream=None):
    """(nodes float32 [n_nodes, 16], tris float32 [n_tris, 12]) device copies of the records."""
    info = bvh.info()
    nodes = torch.empty(max(info["n_nodes"], 1), 16, device="cuda")
    tris = torch.empty(info["n_tris"], 12, device="cuda")
    _check(ctx, load().dhr_bvh_export(ctx.handle, bvh.handle, _ptr(nodes), _ptr(tris), _stream(stream)),
           "dhr_bvh_export")
    return nodes[: info["n_nodes"]], tris


def dhr_refit_bvh(ctx: Context, bvh: Bvh, tris, stream=None):
    _check(ctx, load().dhr_refit_bvh(ctx.handle, bvh.handle, _ptr(tris.reshape(-1, 9)), _stream(stream)),
           "dhr_refit_bvh")


def dhr_encode_frame(ctx, value=None, q=None, shadow_count=None, n_shadow=1, mask=None, stream=None):
    """value: float tensor [n] -> q uint8 [n]; shadow_count uint8 [L, n] -> mask uint8 [n]."""
    n = value.numel() if value is not None else shadow_count.shape[1]
    L = shadow_count.shape[0] if shadow_count is not None else 0
    _check(ctx, load().dhr_encode_frame(ctx.handle, _ptr(value), _ptr(q), _ptr(shadow_count), L, n_shadow, _ptr(mask),
                                        n, _stream(stream)), "dhr_encode_frame")


# ----------------------------------------------------------------------------
# buffer helpers
# ----------------------------------------------------------------------------

def gbuffer_tensors(W, H, device="cuda"):
    HW = W * H
    return {"pos": torch.empty(HW, 4, device=device), "nz": torch.empty(HW, 4, device=device),
            "dz": torch.empty(HW, 2, device=device), "mv": torch.empty(HW, 2, device=device)}
