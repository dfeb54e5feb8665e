"""Seeded inputs for the GPU parity tests, produced only by the workload
generators and the oracle (never by the HIP path).

Per frame: the oracle's G-buffer (rounded to fp32 once, the canonical input of
every downstream pass) and the oracle's noisy visibility counts.
"""
from __future__ import annotations

import functools
import math

import numpy as np

import oracle as orc
from paper_2406_06963_amd import workloads as wl


@functools.lru_cache(maxsize=None)
def scene(name):
    sc = wl.make_scene(name)
    return sc, orc.Scene(sc.tris, sc.obj_id)


def pix_of(cam, H):
    return np.float32(2.0 * math.tan(0.5 * cam.fov_y) / H)


def frames(preset, n: int, n_ao: int | None = None, n_shadow: int | None = None, cams=None):
    """(preset, [dict(pos, nz, dz, mv, ao, sh, cam, pix, params)]) for frames 0..n-1
    of a preset given by name (cached) or as a workloads.Preset; `cams`
    replaces the preset's camera path."""
    if isinstance(preset, str) and cams is None:
        return _frames_named(preset, n, n_ao, n_shadow)
    return _frames(wl.preset(preset) if isinstance(preset, str) else preset, n, n_ao, n_shadow, cams)


@functools.lru_cache(maxsize=None)
def _frames_named(name: str, n: int, n_ao, n_shadow):
    return _frames(wl.preset(name), n, n_ao, n_shadow)


def _frames(pr, n: int, n_ao, n_shadow, cams=None):
    sc, so = scene(pr.scene)
    cams = wl.camera_path(pr.camera, n, sc) if cams is None else cams
    lights = wl.lights_for(pr.scene)
    nao = pr.n_ao if n_ao is None else n_ao
    nsh = pr.n_shadow if n_shadow is None else n_shadow
    out = []
    for f in range(n):
        pos, nz, dz, mv = orc.gbuffer(so, cams[f], cams[f - 1] if f > 0 else None, pr.W, pr.H)
        kw = dict(frame=f, seed=pr.seed, n_ao=nao, ao_radius=pr.ao_radius, n_shadow=nsh, lights=lights)
        P = orc.trace_params(pr.W, pr.H, **kw)
        ao, sh, _ = orc.trace(so, P, pos, nz)
        out.append(dict(pos=pos, nz=nz, dz=dz, mv=mv, ao=ao, sh=sh, cam=cams[f], pix=pix_of(cams[f], pr.H),
                        trace_kw=kw))
    return pr, out


def popcount64(a: np.ndarray) -> int:
    a = np.ascontiguousarray(a, dtype=np.uint64)
    return int(np.unpackbits(a.view(np.uint8)).sum())
