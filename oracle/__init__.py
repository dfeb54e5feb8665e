"""CPU oracle of the DHR+S hot path — TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may import this package.  It shares no code with the HIP
library and never imports the product package; inputs arrive as numpy arrays
(the seeded generators live in their own module and hold no method
arithmetic).

Every function returns FP64 results (the G-buffer and counts excepted, which
are the fp32 / uint8 buffers the method defines).

Parity status of each function (pins live in ``tests/test_oracle_*.py``):
  philox4x32_10      pinned: rocRAND run as a library, statistics
  sample_cosine/cone pinned: moments, support, orthonormality
  anyhit/closest     pinned: brute force over all triangles
  gbuffer            pinned: closed-form plane depth/normal/motion/dz
  trace              pinned: lone plane, plane+wall closed form, penumbra
                     quadrature, radius monotonicity, bitmask example
  svgf_temporal      pinned: running mean, integer shift, disocclusion,
                     fractional motion over a linear history (exact blend),
                     renormalisation over rejected taps, the h' max rule
  svgf_variance      pinned: moments identity, constant / two-level patches
  svgf_atrous        pinned: constant image, scipy normalised convolution
  svgf_spatial_vjp   pinned: dual-number JVP dot-product test, central differences
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liborc.so")
_lib = None


class Camera(C.Structure):
    _fields_ = [("eye", C.c_double * 3), ("target", C.c_double * 3), ("fov_y", C.c_double)]


class Light(C.Structure):
    _fields_ = [("kind", C.c_int32), ("vec", C.c_double * 3), ("one_minus_cos", C.c_double),
                ("radius", C.c_double)]


class TraceParams(C.Structure):
    _fields_ = [("W", C.c_int32), ("H", C.c_int32), ("frame", C.c_uint32), ("client_id", C.c_uint32),
                ("seed", C.c_uint32), ("n_ao", C.c_int32), ("ao_sample_offset", C.c_uint32),
                ("ao_radius", C.c_double), ("n_shadow", C.c_int32), ("n_lights", C.c_int32),
                ("lights", Light * 8), ("eps_origin_abs", C.c_double)]


class SvgfParams(C.Structure):
    _fields_ = [("levels", C.c_int32), ("alpha", C.c_double), ("alpha_moments", C.c_double),
                ("sigma_z", C.c_double * 8), ("sigma_n", C.c_double * 8), ("sigma_l", C.c_double * 8),
                ("eps_z_rel", C.c_double), ("eps_l", C.c_double),
                ("cos_normal_min", C.c_float), ("plane_px", C.c_float),
                ("use_obj_id", C.c_int32), ("var_min_history", C.c_int32),
                ("fallback_radius", C.c_int32), ("feedback_level", C.c_int32),
                ("history_cap", C.c_double), ("kernel_width", C.c_int32)]


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            from . import build as _b
            _b.build()
        _lib = C.CDLL(_LIB_PATH)
        _declare(_lib)
    return _lib


def _p(a):
    return None if a is None else a.ctypes.data_as(C.c_void_p)


def _declare(L):
    vp, i64, i32, u32, dbl = C.c_void_p, C.c_int64, C.c_int, C.c_uint32, C.c_double
    L.orc_philox4x32_10.argtypes = [u32, u32, vp, vp, i64]
    L.orc_sample_cosine.argtypes = [vp, vp, vp, i64]
    L.orc_sample_cone.argtypes = [vp, dbl, vp, vp, i64]
    L.orc_scene_create.argtypes = [vp, vp, i64]
    L.orc_scene_create.restype = vp
    L.orc_scene_destroy.argtypes = [vp]
    L.orc_scene_depth.argtypes = [vp]
    L.orc_anyhit.argtypes = [vp, vp, vp, vp, i64, vp, vp]
    L.orc_closest.argtypes = [vp, vp, vp, i64, vp, vp, i32]
    L.orc_gbuffer.argtypes = [vp, vp, vp, i32, i32, vp, vp, vp, vp]
    L.orc_trace.argtypes = [vp, vp, vp, vp, vp, i64, vp, vp, vp]
    L.orc_svgf_temporal.argtypes = [vp, i32, i32, i32, vp, vp, vp, vp, vp, vp, vp, C.c_float, vp]
    L.orc_svgf_variance.argtypes = [vp, i32, i32, vp, vp, vp, vp]
    L.orc_svgf_atrous.argtypes = [vp, i32, i32, i32, vp, vp, vp, vp]
    L.orc_svgf_filter.argtypes = [vp, i32, i32, i32, vp, vp, vp, vp, vp, vp, vp, vp, C.c_float,
                                  vp, vp, vp, vp]
    L.orc_svgf_spatial.argtypes = [vp, i32, i32, vp, vp, vp, vp, vp]
    L.orc_svgf_spatial_vjp.argtypes = [vp, i32, i32, vp, vp, vp, vp, vp, vp]
    L.orc_svgf_spatial_jvp.argtypes = [vp, i32, i32, vp, vp, vp, vp, vp, vp]
    L.orc_quantize_u8.argtypes = [vp, vp, i64]
    L.orc_light_mask.argtypes = [vp, i32, i32, i64, vp]
    L.orc_num_threads.restype = i32
    L.orc_set_num_threads.argtypes = [i32]


def num_threads() -> int:
    return lib().orc_num_threads()


def set_num_threads(n: int) -> None:
    lib().orc_set_num_threads(int(n))


# ----------------------------------------------------------------------------
# RNG and samplers
# ----------------------------------------------------------------------------

def philox4x32_10(key, ctr) -> np.ndarray:
    ctr = np.ascontiguousarray(ctr, dtype=np.uint32).reshape(-1, 4)
    out = np.empty_like(ctr)
    lib().orc_philox4x32_10(int(key[0]), int(key[1]), _p(ctr), _p(out), ctr.shape[0])
    return out


def sample_cosine(n, u) -> np.ndarray:
    n = np.ascontiguousarray(n, dtype=np.float64).reshape(-1, 3)
    u = np.ascontiguousarray(u, dtype=np.float64).reshape(-1, 2)
    out = np.empty((u.shape[0], 3))
    lib().orc_sample_cosine(_p(n), _p(u), _p(out), u.shape[0])
    return out


def sample_cone(axis, one_minus_cos, u) -> np.ndarray:
    a = np.ascontiguousarray(axis, dtype=np.float64).reshape(3)
    u = np.ascontiguousarray(u, dtype=np.float64).reshape(-1, 2)
    out = np.empty((u.shape[0], 3))
    lib().orc_sample_cone(_p(a), float(one_minus_cos), _p(u), _p(out), u.shape[0])
    return out


# ----------------------------------------------------------------------------
# scene
# ----------------------------------------------------------------------------

class Scene:
    """Oracle scene: own median-split BVH plus brute force."""

    def __init__(self, tris, obj_id=None):
        self.tris = np.ascontiguousarray(tris, dtype=np.float32).reshape(-1, 3, 3)
        self.obj_id = None if obj_id is None else np.ascontiguousarray(obj_id, dtype=np.uint32)
        self._h = lib().orc_scene_create(_p(self.tris), _p(self.obj_id), self.tris.shape[0])

    def __del__(self):
        if getattr(self, "_h", None) and _lib is not None:
            _lib.orc_scene_destroy(self._h)
            self._h = None

    @property
    def depth(self) -> int:
        return lib().orc_scene_depth(self._h)

    def anyhit(self, o, d, tmax, brute=True):
        o = np.ascontiguousarray(o, dtype=np.float64).reshape(-1, 3)
        d = np.ascontiguousarray(d, dtype=np.float64).reshape(-1, 3)
        tmax = np.ascontiguousarray(np.broadcast_to(tmax, (o.shape[0],)), dtype=np.float64)
        hb = np.zeros(o.shape[0], np.uint8)
        hf = np.zeros(o.shape[0], np.uint8) if brute else None
        lib().orc_anyhit(self._h, _p(o), _p(d), _p(tmax), o.shape[0], _p(hb), _p(hf))
        return (hb, hf) if brute else hb

    def closest(self, o, d, brute=False):
        o = np.ascontiguousarray(o, dtype=np.float64).reshape(-1, 3)
        d = np.ascontiguousarray(d, dtype=np.float64).reshape(-1, 3)
        t = np.empty(o.shape[0])
        tri = np.empty(o.shape[0], np.int64)
        lib().orc_closest(self._h, _p(o), _p(d), o.shape[0], _p(t), _p(tri), int(brute))
        return t, tri


def camera(cam) -> Camera:
    """From any object with eye, target, fov_y."""
    c = Camera()
    for k in range(3):
        c.eye[k] = float(cam.eye[k])
        c.target[k] = float(cam.target[k])
    c.fov_y = float(cam.fov_y)
    return c


def gbuffer(scene: Scene, cam, prev_cam, W: int, H: int):
    """Returns pos [H*W,4], nz [H*W,4], dz [H*W,2], mv [H*W,2] as float32."""
    HW = W * H
    pos = np.empty((HW, 4), np.float32)
    nz = np.empty((HW, 4), np.float32)
    dz = np.empty((HW, 2), np.float32)
    mv = np.empty((HW, 2), np.float32)
    c = camera(cam)
    pc = camera(prev_cam) if prev_cam is not None else None
    lib().orc_gbuffer(scene._h, C.byref(c), C.byref(pc) if pc is not None else None, W, H,
                      _p(pos), _p(nz), _p(dz), _p(mv))
    return pos, nz, dz, mv


def trace_params(W, H, *, frame=0, client_id=0, seed=0, n_ao=1, ao_sample_offset=0, ao_radius=1.0,
                 n_shadow=1, lights=(), eps_origin_abs=0.0) -> TraceParams:
    p = TraceParams()
    p.W, p.H, p.frame, p.client_id, p.seed = W, H, frame, client_id, seed
    p.n_ao, p.ao_sample_offset, p.ao_radius = n_ao, ao_sample_offset, float(np.float32(ao_radius))
    p.n_shadow, p.n_lights = n_shadow, len(lights)
    for k, L in enumerate(lights):
        p.lights[k].kind = int(L.kind)
        for j in range(3):
            p.lights[k].vec[j] = float(np.float32(L.vec[j]))
        p.lights[k].one_minus_cos = float(np.float32(L.one_minus_cos))
        p.lights[k].radius = float(np.float32(L.radius))
    p.eps_origin_abs = float(np.float32(eps_origin_abs))
    return p


def trace(scene: Scene, params: TraceParams, pos, nz, pix_list=None, ray_bits=False):
    """Returns (ao_count [n], shadow_count [n_lights, n], bits or None)."""
    pos = np.ascontiguousarray(pos, dtype=np.float32).reshape(-1, 4)
    nz = np.ascontiguousarray(nz, dtype=np.float32).reshape(-1, 4)
    pl = None if pix_list is None else np.ascontiguousarray(pix_list, dtype=np.int64)
    n = pos.shape[0] if pl is None else pl.shape[0]
    ao = np.empty(n, np.uint8)
    sh = np.empty((max(params.n_lights, 1), n), np.uint8)
    bits = np.empty((1 + params.n_lights, n), np.uint64) if ray_bits else None
    lib().orc_trace(scene._h, C.byref(params), _p(pos), _p(nz), _p(pl), n, _p(ao), _p(sh), _p(bits))
    return ao, sh[: params.n_lights], bits


# ----------------------------------------------------------------------------
# SVGF
# ----------------------------------------------------------------------------

def svgf_params(levels=5, alpha=0.2, alpha_moments=0.2, sigma_z=1.0, sigma_n=128.0, sigma_l=4.0,
                eps_z_rel=1e-4, eps_l=1e-4, cos_normal_min=0.9, plane_px=4.0, use_obj_id=1,
                var_min_history=4, fallback_radius=3, feedback_level=0, history_cap=255.0,
                kernel_width=5, fp32=True) -> SvgfParams:
    """Defaults of the filter.  With fp32=True every continuous constant is
    first rounded to fp32 (the values the GPU path receives)."""
    r = (lambda v: float(np.float32(v))) if fp32 else float
    p = SvgfParams()
    p.levels, p.alpha, p.alpha_moments = levels, r(alpha), r(alpha_moments)
    for name, v in (("sigma_z", sigma_z), ("sigma_n", sigma_n), ("sigma_l", sigma_l)):
        arr = np.broadcast_to(np.asarray(v, dtype=np.float64), (levels,))
        tgt = getattr(p, name)
        for k in range(8):
            tgt[k] = r(arr[k]) if k < levels else 1.0
    p.eps_z_rel, p.eps_l = r(eps_z_rel), r(eps_l)
    p.cos_normal_min, p.plane_px = cos_normal_min, plane_px
    p.use_obj_id, p.var_min_history, p.fallback_radius = use_obj_id, var_min_history, fallback_radius
    p.feedback_level, p.history_cap = feedback_level, float(history_cap)
    p.kernel_width = kernel_width
    return p


def _f32(a, shape):
    return None if a is None else np.ascontiguousarray(a, dtype=np.float32).reshape(shape)


def svgf_temporal(P, W, H, n_ao, ao_count, pos, nz, mv, prev_pos, prev_nz, hist_in, pix):
    HW = W * H
    out = np.empty((HW, 4))
    ao = np.ascontiguousarray(ao_count, dtype=np.uint8).reshape(HW)
    lib().orc_svgf_temporal(C.byref(P), W, H, n_ao, _p(ao), _p(_f32(pos, (HW, 4))), _p(_f32(nz, (HW, 4))),
                            _p(_f32(mv, (HW, 2))), _p(_f32(prev_pos, (HW, 4))), _p(_f32(prev_nz, (HW, 4))),
                            _p(_f32(hist_in, (HW, 4))), float(pix), _p(out))
    return out


def svgf_variance(P, W, H, hist, nz, dz):
    HW = W * H
    hist = np.ascontiguousarray(hist, dtype=np.float64).reshape(HW, 4)
    cv = np.empty((HW, 2))
    lib().orc_svgf_variance(C.byref(P), W, H, _p(hist), _p(_f32(nz, (HW, 4))), _p(_f32(dz, (HW, 2))), _p(cv))
    return cv


def svgf_atrous(P, W, H, level, cv, nz, dz):
    HW = W * H
    cv = np.ascontiguousarray(cv, dtype=np.float64).reshape(HW, 2)
    out = np.empty((HW, 2))
    lib().orc_svgf_atrous(C.byref(P), W, H, level, _p(cv), _p(_f32(nz, (HW, 4))), _p(_f32(dz, (HW, 2))), _p(out))
    return out


def svgf_filter(P, W, H, n_ao, ao_count, pos, nz, dz, mv, prev_pos, prev_nz, hist_in, pix, save=False):
    """Full frame.  Returns dict(hist_out, out, cv0, save)."""
    HW = W * H
    hist_out = np.empty((HW, 4))
    out = np.empty(HW)
    cv0 = np.empty((HW, 2))
    sv = np.empty((P.levels, HW, 2)) if save else None
    ao = np.ascontiguousarray(ao_count, dtype=np.uint8).reshape(HW)
    lib().orc_svgf_filter(C.byref(P), W, H, n_ao, _p(ao), _p(_f32(pos, (HW, 4))), _p(_f32(nz, (HW, 4))),
                          _p(_f32(dz, (HW, 2))), _p(_f32(mv, (HW, 2))), _p(_f32(prev_pos, (HW, 4))),
                          _p(_f32(prev_nz, (HW, 4))), _p(_f32(hist_in, (HW, 4))), float(pix),
                          _p(hist_out), _p(out), _p(cv0), _p(sv))
    return {"hist_out": hist_out, "out": out, "cv0": cv0, "save": sv}


def svgf_spatial(P, W, H, cv_in, nz, dz, save=False):
    HW = W * H
    cv = np.ascontiguousarray(cv_in, dtype=np.float64).reshape(HW, 2)
    out = np.empty(HW)
    sv = np.empty((P.levels, HW, 2)) if save else None
    lib().orc_svgf_spatial(C.byref(P), W, H, _p(cv), _p(_f32(nz, (HW, 4))), _p(_f32(dz, (HW, 2))), _p(out), _p(sv))
    return (out, sv) if save else out


def svgf_spatial_vjp(P, W, H, cv_in, nz, dz, grad_out):
    HW = W * H
    cv = np.ascontiguousarray(cv_in, dtype=np.float64).reshape(HW, 2)
    g = np.ascontiguousarray(grad_out, dtype=np.float64).reshape(HW)
    gcv = np.empty((HW, 2))
    gs = np.empty(3 * P.levels)
    lib().orc_svgf_spatial_vjp(C.byref(P), W, H, _p(cv), _p(_f32(nz, (HW, 4))), _p(_f32(dz, (HW, 2))), _p(g),
                               _p(gcv), _p(gs))
    return gcv, gs.reshape(3, P.levels)


def svgf_spatial_jvp(P, W, H, cv_in, nz, dz, dcv, dsigma):
    HW = W * H
    cv = np.ascontiguousarray(cv_in, dtype=np.float64).reshape(HW, 2)
    dcv = np.ascontiguousarray(dcv, dtype=np.float64).reshape(HW, 2)
    ds = np.ascontiguousarray(dsigma, dtype=np.float64).reshape(3 * P.levels)
    out = np.empty(HW)
    lib().orc_svgf_spatial_jvp(C.byref(P), W, H, _p(cv), _p(_f32(nz, (HW, 4))), _p(_f32(dz, (HW, 2))), _p(dcv),
                               _p(ds), _p(out))
    return out


def id_bits(pos) -> np.ndarray:
    """Object ids stored in pos.w."""
    return np.ascontiguousarray(pos[:, 3]).view(np.uint32)


def quantize_u8(x) -> np.ndarray:
    """One byte per value: floor(255 clamp(x, 0, 1) + 1/2) in fp32 (NaN -> 0)."""
    x = np.ascontiguousarray(x, dtype=np.float32).ravel()
    q = np.empty(x.size, np.uint8)
    lib().orc_quantize_u8(_p(x), _p(q), x.size)
    return q


def light_mask(shadow_count, n_shadow: int) -> np.ndarray:
    """Bit l set where at least half of light l's n_shadow rays reach it."""
    sc = np.ascontiguousarray(shadow_count, dtype=np.uint8)
    L, hw = sc.shape
    m = np.empty(hw, np.uint8)
    lib().orc_light_mask(_p(sc), L, n_shadow, hw, _p(m))
    return m
