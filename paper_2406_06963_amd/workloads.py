"""Seeded synthetic inputs: scenes, camera paths, lights and test scenes.

The paper evaluates on three artist scenes (Section 4.1) that are not
available; these procedural scenes stand in for them.  This module holds
none of the method's arithmetic: it only produces triangles, object ids,
cameras and light descriptions.  Both the HIP path and the CPU oracle are fed
from here, so nothing in it may trace rays or filter images.

Conventions
-----------
* Triangles: float32 ``[T, 3, 3]`` (vertex, xyz), world space, +y up.
* Object ids: uint32 ``[T]``.
* Camera: ``Camera(eye, target, fov_y)``, fov in radians, up = +y.
* Lights: ``Light(kind, vec, one_minus_cos, radius)``; kind 0 = directional
  (vec = unit direction towards the light, ``one_minus_cos`` = 1 - cos of the
  cone half-angle, computed here as 2 sin^2(theta/2)), kind 1 = sphere
  (vec = centre, radius R).
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

__all__ = [
    "Camera", "Light", "Scene", "make_scene", "camera_path", "lights_for",
    "preset", "Preset", "PRESETS", "directional_light", "sphere_light",
    "scene_plane", "scene_plane_wall", "scene_closed_box", "scene_edge_occluder",
    "random_triangles", "terrain_height",
]


def _f32(v) -> float:
    return float(np.float32(v))


@dataclass
class Camera:
    """Pinhole camera; every value is rounded to fp32 on construction (the
    C interface carries fp32 cameras, so the oracle sees the same camera)."""
    eye: tuple
    target: tuple
    fov_y: float = math.radians(60.0)

    def __post_init__(self):
        self.eye = tuple(_f32(v) for v in self.eye)
        self.target = tuple(_f32(v) for v in self.target)
        self.fov_y = _f32(self.fov_y)

    def as_array(self) -> np.ndarray:
        return np.array([*self.eye, *self.target, self.fov_y], dtype=np.float64)

    def pix_angle(self, H: int) -> float:
        """Angular size of one pixel row at unit depth: 2 tan(fov/2) / H."""
        return 2.0 * math.tan(0.5 * self.fov_y) / H


@dataclass
class Light:
    kind: int               # 0 directional, 1 sphere
    vec: tuple              # direction (kind 0) or centre (kind 1)
    one_minus_cos: float = 0.0
    radius: float = 0.0


def directional_light(direction, half_angle_deg: float) -> Light:
    d = np.asarray(direction, dtype=np.float64)
    d = d / np.linalg.norm(d)
    th = math.radians(half_angle_deg)
    return Light(0, tuple(float(v) for v in d), 2.0 * math.sin(0.5 * th) ** 2, 0.0)


def sphere_light(center, radius: float) -> Light:
    return Light(1, tuple(float(v) for v in center), 0.0, float(radius))


@dataclass
class Scene:
    name: str
    tris: np.ndarray            # float32 [T,3,3]
    obj_id: np.ndarray          # uint32 [T]
    meta: dict = field(default_factory=dict)

    @property
    def n_tris(self) -> int:
        return int(self.tris.shape[0])


# ----------------------------------------------------------------------------
# primitive meshes
# ----------------------------------------------------------------------------

def _quad(p0, p1, p2, p3):
    """Two triangles p0 p1 p2 and p0 p2 p3."""
    return [[p0, p1, p2], [p0, p2, p3]]


def _uv_sphere(center, radius, segs=16, rings=16):
    cx, cy, cz = center
    verts = {}
    for i in range(rings + 1):
        th = math.pi * i / rings
        for j in range(segs):
            ph = 2.0 * math.pi * j / segs
            verts[(i, j)] = (cx + radius * math.sin(th) * math.cos(ph),
                             cy + radius * math.cos(th),
                             cz + radius * math.sin(th) * math.sin(ph))
    tris = []
    for j in range(segs):
        j1 = (j + 1) % segs
        tris.append([verts[(0, 0)], verts[(1, j1)], verts[(1, j)]])
        tris.append([verts[(rings, 0)], verts[(rings - 1, j)], verts[(rings - 1, j1)]])
    for i in range(1, rings - 1):
        for j in range(segs):
            j1 = (j + 1) % segs
            a, b = verts[(i, j)], verts[(i, j1)]
            c, d = verts[(i + 1, j1)], verts[(i + 1, j)]
            tris.append([a, b, c])
            tris.append([a, c, d])
    return tris


def _icosphere(center, radius, subdiv=3):
    t = (1.0 + math.sqrt(5.0)) / 2.0
    v = [(-1, t, 0), (1, t, 0), (-1, -t, 0), (1, -t, 0),
         (0, -1, t), (0, 1, t), (0, -1, -t), (0, 1, -t),
         (t, 0, -1), (t, 0, 1), (-t, 0, -1), (-t, 0, 1)]
    v = [np.array(p, dtype=np.float64) / np.linalg.norm(p) for p in v]
    f = [(0, 11, 5), (0, 5, 1), (0, 1, 7), (0, 7, 10), (0, 10, 11),
         (1, 5, 9), (5, 11, 4), (11, 10, 2), (10, 7, 6), (7, 1, 8),
         (3, 9, 4), (3, 4, 2), (3, 2, 6), (3, 6, 8), (3, 8, 9),
         (4, 9, 5), (2, 4, 11), (6, 2, 10), (8, 6, 7), (9, 8, 1)]
    faces = [tuple(v[i] for i in tri) for tri in f]
    for _ in range(subdiv):
        nf = []
        for a, b, c in faces:
            ab = (a + b); ab /= np.linalg.norm(ab)
            bc = (b + c); bc /= np.linalg.norm(bc)
            ca = (c + a); ca /= np.linalg.norm(ca)
            nf += [(a, ab, ca), (b, bc, ab), (c, ca, bc), (ab, bc, ca)]
        faces = nf
    c = np.asarray(center, dtype=np.float64)
    return np.array([[c + radius * p for p in tri] for tri in faces])


def _box(center, ext, yaw):
    """Axis-aligned box of extents ext, rotated by yaw about +y, 12 triangles."""
    hx, hy, hz = 0.5 * ext[0], 0.5 * ext[1], 0.5 * ext[2]
    cs, sn = math.cos(yaw), math.sin(yaw)

    def P(x, y, z):
        return (center[0] + cs * x + sn * z, center[1] + y, center[2] - sn * x + cs * z)

    c = [P(x, y, z) for x in (-hx, hx) for y in (-hy, hy) for z in (-hz, hz)]
    # corner index = 4*ix + 2*iy + iz
    faces = [(0, 1, 3, 2), (4, 6, 7, 5), (0, 4, 5, 1), (2, 3, 7, 6), (0, 2, 6, 4), (1, 5, 7, 3)]
    tris = []
    for a, b, cc, d in faces:
        tris += _quad(c[a], c[b], c[cc], c[d])
    return tris


def _pack(groups):
    """groups: list of (triangle list/array, obj id)."""
    tri_list, ids = [], []
    for tris, oid in groups:
        arr = np.asarray(tris, dtype=np.float64).reshape(-1, 3, 3)
        tri_list.append(arr)
        ids.append(np.full(arr.shape[0], oid, dtype=np.uint32))
    return np.concatenate(tri_list).astype(np.float32), np.concatenate(ids)


# ----------------------------------------------------------------------------
# fBm terrain (value noise)
# ----------------------------------------------------------------------------

def _value_noise_fbm(xs, zs, seed, octaves=6, lacunarity=2.0, gain=0.5, base_freq=1.0 / 96.0):
    """Seeded fBm of smoothstep-interpolated lattice value noise, range ~[-1,1]."""
    rng = np.random.default_rng(seed)
    X, Z = np.meshgrid(xs, zs, indexing="xy")
    total = np.zeros_like(X)
    amp, freq, norm = 1.0, base_freq, 0.0
    for _ in range(octaves):
        lat = rng.uniform(-1.0, 1.0, size=(257, 257))
        u = X * freq + 128.0
        v = Z * freq + 128.0
        i0 = np.floor(u).astype(np.int64) % 256
        j0 = np.floor(v).astype(np.int64) % 256
        fu = u - np.floor(u)
        fv = v - np.floor(v)
        su = fu * fu * (3 - 2 * fu)
        sv = fv * fv * (3 - 2 * fv)
        a = lat[j0, i0]; b = lat[j0, i0 + 1]
        c = lat[j0 + 1, i0]; d = lat[j0 + 1, i0 + 1]
        total += amp * ((a * (1 - su) + b * su) * (1 - sv) + (c * (1 - su) + d * su) * sv)
        norm += amp
        amp *= gain
        freq *= lacunarity
    return total / norm


def terrain_height(scene: Scene, x: float, z: float) -> float:
    """Bilinear height of a terrain scene's vertex grid at (x, z)."""
    g = scene.meta["grid"]
    ext, n = scene.meta["extent"], scene.meta["cells"]
    fx = (x + ext) / (2 * ext) * n
    fz = (z + ext) / (2 * ext) * n
    i = int(min(max(math.floor(fx), 0), n - 1))
    j = int(min(max(math.floor(fz), 0), n - 1))
    tx, tz = fx - i, fz - j
    return float((g[j, i] * (1 - tx) + g[j, i + 1] * tx) * (1 - tz)
                 + (g[j + 1, i] * (1 - tx) + g[j + 1, i + 1] * tx) * tz)


# ----------------------------------------------------------------------------
# the three plain-method scenes
# ----------------------------------------------------------------------------

def _scene_spheres(seed=1):
    """Ground quad [-10,10]^2 at y=0 plus 8 non-overlapping UV spheres."""
    rng = np.random.default_rng(seed)
    groups = [(_quad((-10, 0, -10), (-10, 0, 10), (10, 0, 10), (10, 0, -10)), 0)]
    placed = []
    while len(placed) < 8:
        r = rng.uniform(0.3, 1.0)
        x, z = rng.uniform(-4, 4, size=2)
        if all((x - px) ** 2 + (z - pz) ** 2 > (r + pr + 0.05) ** 2 for px, pz, pr in placed):
            placed.append((x, z, r))
    for k, (x, z, r) in enumerate(placed):
        groups.append((_uv_sphere((x, r, z), r), k + 1))
    tris, ids = _pack(groups)
    return Scene("spheres", tris, ids, {"spheres": placed})


def _scene_room(seed=2):
    """Room [0,20]x[0,5]x[0,20] (inward faces), 120 boxes, 80 icospheres."""
    rng = np.random.default_rng(seed)
    X, Y, Z = 20.0, 5.0, 20.0
    room = []
    room += _quad((0, 0, 0), (X, 0, 0), (X, 0, Z), (0, 0, Z))           # floor
    room += _quad((0, Y, 0), (0, Y, Z), (X, Y, Z), (X, Y, 0))           # ceiling
    room += _quad((0, 0, 0), (0, 0, Z), (0, Y, Z), (0, Y, 0))           # x=0
    room += _quad((X, 0, 0), (X, Y, 0), (X, Y, Z), (X, 0, Z))           # x=X
    room += _quad((0, 0, 0), (0, Y, 0), (X, Y, 0), (X, 0, 0))           # z=0
    room += _quad((0, 0, Z), (X, 0, Z), (X, Y, Z), (0, Y, Z))           # z=Z
    groups = [(room, 0)]
    oid = 1
    for _ in range(120):
        ext = rng.uniform(0.2, 1.5, size=3)
        yaw = rng.uniform(0, 2 * math.pi)
        x, z = rng.uniform(1.0, 19.0, size=2)
        y = rng.uniform(0.5, 3.0) if rng.uniform() < 1 / 3 else 0.5 * ext[1]
        groups.append((_box((x, y, z), ext, yaw), oid)); oid += 1
    for _ in range(80):
        r = rng.uniform(0.2, 0.8)
        x, z = rng.uniform(1.0, 19.0, size=2)
        y = rng.uniform(0.5, 3.0) if rng.uniform() < 1 / 3 else r
        groups.append((_icosphere((x, y, z), r, 3), oid)); oid += 1
    tris, ids = _pack(groups)
    return Scene("room", tris, ids, {"size": (X, Y, Z)})


def _scene_terrain(seed=3, cells=1024, extent=256.0, amplitude=40.0, n_boxes=5000):
    """fBm heightfield (cells x cells quads over [-extent,extent]^2) plus boxes."""
    rng = np.random.default_rng(seed)
    coords = np.linspace(-extent, extent, cells + 1)
    grid = amplitude * _value_noise_fbm(coords, coords, seed)
    xs, zs = np.meshgrid(coords, coords, indexing="xy")
    P = np.stack([xs, grid, zs], axis=-1)
    a = P[:-1, :-1]; b = P[:-1, 1:]; c = P[1:, 1:]; d = P[1:, :-1]
    t0 = np.stack([a, d, c], axis=2).reshape(-1, 3, 3)
    t1 = np.stack([a, c, b], axis=2).reshape(-1, 3, 3)
    terrain = np.stack([t0, t1], axis=1).reshape(-1, 3, 3)
    scene = Scene("terrain", None, None, {"grid": grid, "extent": extent, "cells": cells})
    groups = [(terrain, 0)]
    box_tris = []
    bx = rng.uniform(-extent * 0.95, extent * 0.95, size=n_boxes)
    bz = rng.uniform(-extent * 0.95, extent * 0.95, size=n_boxes)
    sc = rng.uniform(0.5, 3.0, size=n_boxes)
    yaw = rng.uniform(0, 2 * math.pi, size=n_boxes)
    for k in range(n_boxes):
        y = terrain_height(scene, bx[k], bz[k]) + 0.45 * sc[k]
        box_tris.append(np.asarray(_box((bx[k], y, bz[k]), (sc[k], sc[k], sc[k]), yaw[k])))
    all_boxes = np.stack(box_tris)                          # [n_boxes, 12, 3, 3]
    tris = np.concatenate([terrain, all_boxes.reshape(-1, 3, 3)]).astype(np.float32)
    ids = np.concatenate([np.zeros(terrain.shape[0], np.uint32),
                          np.repeat(np.arange(1, n_boxes + 1, dtype=np.uint32), 12)])
    scene.tris, scene.obj_id = tris, ids
    # the same boxes as instances of one unit cube: object-to-world [A | t]
    # with A = R_yaw diag(s), t = the box centre (the flattened boxes above
    # are exactly these transforms applied to the cube's corners)
    cs, sn = np.cos(yaw), np.sin(yaw)
    xf = np.zeros((n_boxes, 3, 4))
    xf[:, 0, 0], xf[:, 0, 2], xf[:, 2, 0], xf[:, 2, 2] = cs * sc, sn * sc, -sn * sc, cs * sc
    xf[:, 1, 1] = sc
    xf[:, 0, 3], xf[:, 2, 3] = bx, bz
    xf[:, 1, 3] = [terrain_height(scene, bx[k], bz[k]) + 0.45 * sc[k] for k in range(n_boxes)]
    scene.meta["instances"] = {"n_base": int(terrain.shape[0]),
                               "mesh": np.asarray(_box((0.0, 0.0, 0.0), (1.0, 1.0, 1.0), 0.0), np.float32),
                               "xforms": xf.astype(np.float32),
                               "ids": np.arange(1, n_boxes + 1, dtype=np.uint32)}
    return scene


def instanced_form(scene: Scene):
    """(base_tris, base_obj, mesh_tris, xforms, inst_ids) of a scene built with
    instances (the terrain): the flattened scene is base + each instance's mesh."""
    inst = scene.meta["instances"]
    nb = inst["n_base"]
    return scene.tris[:nb], scene.obj_id[:nb], inst["mesh"], inst["xforms"], inst["ids"]


# ----------------------------------------------------------------------------
# analytic test scenes
# ----------------------------------------------------------------------------

def scene_plane(half=50.0, y=0.0) -> Scene:
    """A lone horizontal plane (two triangles) facing +y."""
    tris, ids = _pack([(_quad((-half, y, -half), (-half, y, half), (half, y, half), (half, y, -half)), 0)])
    return Scene("plane", tris, ids, {})


def scene_plane_wall(wall_x=0.0, half=60.0, height=40.0) -> Scene:
    """Floor y=0 plus a wall in the plane x=wall_x that is tall and wide."""
    floor = _quad((-half, 0, -half), (-half, 0, half), (half, 0, half), (half, 0, -half))
    wall = _quad((wall_x, 0, -half), (wall_x, height, -half), (wall_x, height, half), (wall_x, 0, half))
    tris, ids = _pack([(floor, 0), (wall, 1)])
    return Scene("plane_wall", tris, ids, {"wall_x": wall_x})


def scene_closed_box(size=4.0) -> Scene:
    """Closed cube [-s/2, s/2]^3 seen from inside (every ray hits it)."""
    h = size / 2
    tris = _box((0, 0, 0), (size, size, size), 0.0)
    tris, ids = _pack([(tris, 0)])
    return Scene("closed_box", tris, ids, {"size": size})


def scene_edge_occluder(height=1.0, half=50.0) -> Scene:
    """Floor y=0 plus a horizontal half-plane occluder at y=height covering x<0."""
    floor = _quad((-half, 0, -half), (-half, 0, half), (half, 0, half), (half, 0, -half))
    occ = _quad((-half, height, -half), (0, height, -half), (0, height, half), (-half, height, half))
    tris, ids = _pack([(floor, 0), (occ, 1)])
    return Scene("edge_occluder", tris, ids, {"height": height})


def random_triangles(n: int, seed: int, box=1.0, size=0.6) -> Scene:
    """n random triangles in [-box,box]^3, some sharing edges (for BVH tests)."""
    rng = np.random.default_rng(seed)
    c = rng.uniform(-box, box, size=(n, 1, 3))
    tris = c + rng.uniform(-size, size, size=(n, 3, 3))
    # make a quarter of them share an edge with their predecessor
    for i in range(1, n, 4):
        tris[i, 0] = tris[i - 1, 1]
        tris[i, 1] = tris[i - 1, 2]
    return Scene("random", tris.astype(np.float32), np.arange(n, dtype=np.uint32), {})


_SCENE_CACHE: dict = {}


def make_scene(name: str, seed: int | None = None) -> Scene:
    """Scenes of the plain-method workloads: 'spheres', 'room', 'terrain'."""
    key = (name, seed)
    if key not in _SCENE_CACHE:
        if name == "spheres":
            _SCENE_CACHE[key] = _scene_spheres(1 if seed is None else seed)
        elif name == "room":
            _SCENE_CACHE[key] = _scene_room(2 if seed is None else seed)
        elif name == "terrain":
            _SCENE_CACHE[key] = _scene_terrain(3 if seed is None else seed)
        else:
            raise ValueError(f"unknown scene {name!r}")
    return _SCENE_CACHE[key]


# ----------------------------------------------------------------------------
# camera paths and lights
# ----------------------------------------------------------------------------

def camera_path(name: str, n_frames: int, scene: Scene | None = None, phase: float = 0.0):
    """Per-frame cameras for the workloads (list of Camera)."""
    cams = []
    fx, fz = -60.0, -40.0               # flyover ground position, integrated below
    for f in range(n_frames):
        if name == "orbit":              # spheres scene: radius 8, height 3, 2 deg/frame
            a = math.radians(2.0 * f) + phase
            eye = (8.0 * math.cos(a), 3.0, 8.0 * math.sin(a))
            cams.append(Camera(eye, (0.0, 0.5, 0.0)))
        elif name == "walk":             # room: +x at 0.05/frame, lateral sway
            t = f + phase * 30.0
            x = 2.0 + 0.05 * t
            z = 10.0 + 0.5 * math.sin(2 * math.pi * t / 30.0)
            eye = (x, 1.6, z)
            cams.append(Camera(eye, (x + 1.0, 1.45, z + 0.15 * math.cos(2 * math.pi * t / 45.0))))
        elif name == "flyover":          # terrain: yaw 3 deg/frame, forward 0.5/frame, 10 above ground
            yaw = math.radians(3.0 * f) + phase
            if f > 0:
                fx += 0.5 * math.cos(yaw)
                fz += 0.5 * math.sin(yaw)
            x, z = fx, fz
            y = terrain_height(scene, x, z) + 10.0
            fwd = (math.cos(yaw), -0.3, math.sin(yaw))
            cams.append(Camera((x, y, z), (x + fwd[0], y + fwd[1], z + fwd[2])))
        else:
            raise ValueError(f"unknown camera path {name!r}")
    return cams


def lights_for(scene_name: str):
    if scene_name == "spheres":
        return [directional_light((0.4, 1.0, 0.3), 1.0)]
    if scene_name == "room":
        return [sphere_light((10.0, 4.2, 10.0), 0.5)]
    if scene_name == "terrain":
        return [directional_light((-0.5, 0.8, 0.3), 1.0)]
    raise ValueError(scene_name)


# ----------------------------------------------------------------------------
# presets of the workloads
# ----------------------------------------------------------------------------

@dataclass
class Preset:
    name: str
    scene: str
    camera: str
    W: int
    H: int
    frames: int
    n_ao: int
    ao_radius: float
    n_shadow: int
    seed: int = 1
    alpha: float = 0.2
    levels: int = 5


PRESETS = {
    # 64x64, 8 frames, orbit at 2 deg/frame, 1 AO (r=1) + 1 shadow, 1 deg half-angle sun
    "tiny": Preset("tiny", "spheres", "orbit", 64, 64, 8, 1, 1.0, 1, seed=1),
    # 1280x720 room, 60 frames, 1 AO (r=0.5) + 1 shadow towards a sphere light
    "room720": Preset("room720", "room", "walk", 1280, 720, 60, 1, 0.5, 1, seed=2),
    # 1920x1080 terrain, 120 frames, 1 AO (r=1) + 2 shadow rays
    "terrain1080": Preset("terrain1080", "terrain", "flyover", 1920, 1080, 120, 1, 1.0, 2, seed=3),
    # ragged sizes for edge cases: no side a multiple of any kernel tile
    "ragged": Preset("ragged", "room", "walk", 141, 77, 4, 3, 0.5, 2, seed=4),
    "sliver": Preset("sliver", "spheres", "orbit", 5, 131, 3, 1, 1.0, 4, seed=5),
}


def preset(name: str) -> Preset:
    return PRESETS[name]
