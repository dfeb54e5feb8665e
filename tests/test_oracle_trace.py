"""Pins of the oracle's visibility rays (no GPU).

* T2 lone plane: nothing can occlude, so every AO count equals N and every
  shadow count equals the number of shadow rays (self-intersection check).
* T3 plane beside an infinite wall: with cosine-weighted rays of length r the
  projected disk point is uniform, and the wall at distance d cuts a circular
  segment, so V = 1 - (acos a - a sqrt(1 - a^2)) / pi with a = min(d/r, 1)
  (eqs. (1)-(3) of the paper).
* T4 radius monotonicity: with the same random numbers a ray occluded at
  radius r1 is occluded at every r2 > r1 (Section 3.2, Fig. 3 discussion).
* T5 a zero-width cone is the hard shadow ray to the light centre
  (Section 2.2); the worked bitmask example of Fig. 1 (Section 3.1): hard
  shadows give 110, the soft cone uncovers a nearby occluder of light 2 and
  gives 010 (bit i = light i visible, light 0 the least significant bit);
  penumbra behind a straight edge equals the occluded fraction of the cone
  computed by quadrature.
"""
import math
import os

import numpy as np
import pytest

from paper_2406_06963_amd import workloads as wl


def wall_visibility(a):
    a = np.clip(a, 0.0, 1.0)
    return 1.0 - (np.arccos(a) - a * np.sqrt(1.0 - a * a)) / np.pi


def test_wall_closed_form_values():
    # values quoted with the pin: V(0)=0.5, V(0.25)=0.657481, V(0.5)=0.804499, V(0.75)=0.927853, V(1)=1
    np.testing.assert_allclose(wall_visibility(np.array([0, 0.25, 0.5, 0.75, 1.0])),
                               [0.5, 0.657481, 0.804499, 0.927853, 1.0], atol=1e-6)


def _gbuf(orc, scene, cam, W, H):
    s = orc.Scene(scene.tris, scene.obj_id)
    pos, nz, dz, mv = orc.gbuffer(s, cam, None, W, H)
    return s, pos, nz


def test_lone_plane_fully_visible(orc):
    sc = wl.scene_plane()
    W, H = 48, 32
    cam = wl.Camera((0.3, 2.0, 4.0), (0.0, 0.0, 0.0))
    s, pos, nz = _gbuf(orc, sc, cam, W, H)
    assert (nz[:, 3] > 0).mean() > 0.6
    lights = [wl.directional_light((0.2, 1.0, 0.1), 1.0), wl.sphere_light((1.0, 3.0, -1.0), 0.5),
              wl.directional_light((0.0, -1.0, 0.0), 1.0)]
    for r in (0.1, 1.0, 5.0, 100.0):
        P = orc.trace_params(W, H, seed=9, n_ao=32, ao_radius=r, n_shadow=4, lights=lights)
        ao, sh, _ = orc.trace(s, P, pos, nz)
        assert (ao == 32).all()
        assert (sh[0] == 4).all() and (sh[1] == 4).all()
        # light from below: every cone direction is below the surface -> occluded without tracing
        valid = nz[:, 3] > 0
        assert (sh[2][valid] == 0).all() and (sh[2][~valid] == 4).all()


def test_invalid_pixels_fully_visible(orc):
    sc = wl.scene_plane()
    s = orc.Scene(sc.tris, sc.obj_id)
    W, H = 8, 8
    pos = np.zeros((W * H, 4), np.float32)
    nz = np.zeros((W * H, 4), np.float32)
    P = orc.trace_params(W, H, n_ao=7, n_shadow=3, lights=[wl.directional_light((0, 1, 0), 1.0)])
    ao, sh, bits = orc.trace(s, P, pos, nz, ray_bits=True)
    assert (ao == 7).all() and (sh == 3).all()
    assert (bits[0] == 0x7F).all() and (bits[1] == 0x7).all()


def test_plane_wall_closed_form(orc):
    sc = wl.scene_plane_wall(wall_x=0.0)
    W, H = 48, 48
    cam = wl.Camera((-0.7, 2.5, 2.0), (-0.7, 0.0, -0.3))
    s, pos, nz = _gbuf(orc, sc, cam, W, H)
    floor = (orc.id_bits(pos) == 0) & (nz[:, 3] > 0)
    r = 1.0
    counts = np.zeros(W * H)
    frames = 4
    for f in range(frames):
        P = orc.trace_params(W, H, frame=f, seed=17, n_ao=255, ao_radius=r, n_shadow=0)
        ao, _, _ = orc.trace(s, P, pos, nz)
        counts += ao
    n = 255 * frames
    d = -pos[:, 0].astype(np.float64)
    Vp = wall_visibility(d / r)
    est = counts / n
    sel = floor & (d > 0.0)
    assert sel.sum() > 1000
    bins = np.clip((d / r / 0.1).astype(int), 0, 12)
    checked = 0
    for b in range(13):
        m = sel & (bins == b)
        if m.sum() < 20:
            continue
        sigma = np.sqrt((Vp[m] * (1 - Vp[m])).sum() / n) / m.sum()
        assert abs(est[m].mean() - Vp[m].mean()) <= 5 * sigma + 1e-12, (b, est[m].mean(), Vp[m].mean(), sigma)
        checked += 1
    assert checked >= 8
    # beyond the radius the wall is invisible: V == 1 exactly
    far = sel & (d > 1.01 * r)
    assert far.sum() > 0 and (est[far] == 1.0).all()


def test_radius_monotonicity(orc):
    sc = wl.make_scene("spheres")
    W, H = 64, 64
    cam = wl.camera_path("orbit", 1)[0]
    s, pos, nz = _gbuf(orc, sc, cam, W, H)
    prev = None
    for r in (0.1, 0.3, 1.0, 2.5):
        P = orc.trace_params(W, H, seed=4, n_ao=64, ao_radius=r, n_shadow=0, eps_origin_abs=1e-3)
        _, _, bits = orc.trace(s, P, pos, nz, ray_bits=True)
        if prev is not None:
            # unoccluded at the larger radius implies unoccluded at the smaller one
            assert ((bits[0] & ~prev) == 0).all()
            assert (bits[0] != prev).any()
        prev = bits[0]


def test_hard_shadow_is_zero_width_cone(orc):
    sc = wl.make_scene("spheres")
    W, H = 64, 64
    cam = wl.camera_path("orbit", 1)[0]
    s, pos, nz = _gbuf(orc, sc, cam, W, H)
    L = wl.directional_light((0.4, 1.0, 0.3), 0.0)
    assert L.one_minus_cos == 0.0
    P = orc.trace_params(W, H, seed=2, n_ao=0, ao_radius=1.0, n_shadow=8, lights=[L])
    _, sh, bits = orc.trace(s, P, pos, nz, ray_bits=True)
    assert set(np.unique(bits[1]).tolist()) <= {0, 0xFF}
    # the same decision by one ray straight to the light centre
    valid = nz[:, 3] > 0
    p = pos[valid, :3].astype(np.float64)
    n = nz[valid, :3].astype(np.float64)
    n /= np.linalg.norm(n, axis=1, keepdims=True)
    eps = np.maximum(1e-3 * 1.0, np.ldexp(np.abs(p).max(axis=1), -17))
    o = p + eps[:, None] * n
    axis = np.array(L.vec) / np.linalg.norm(L.vec)
    hit = s.anyhit(o, np.broadcast_to(axis, o.shape), np.inf, brute=False)
    facing = n @ axis > 0
    expect = np.where(facing & (hit == 0), 8, 0)
    np.testing.assert_array_equal(sh[0][valid], expect)
    assert 0 < (expect == 0).sum() < valid.sum()


def _fig1_scene(cone_deg):
    """One floor point at the origin and three directional lights (Fig. 1)."""
    L0 = np.array([-0.6, 0.8, 0.0])          # blocked by a wall at x = -2, 5 high
    L1 = np.array([0.0, 1.0, 0.0])           # open sky
    L2 = np.array([0.6, 0.8, 0.0])           # a nearby occluder covers part of its cone, not its centre
    tris = []
    tris += [[(-2, 0, -50), (-2, 5, -50), (-2, 5, 50)], [(-2, 0, -50), (-2, 5, 50), (-2, 0, 50)]]
    # quad perpendicular to L2 at distance 2, covering z in [0.05, 2] of the cone's cross-section
    c = 2.0 * L2
    u = np.array([-0.8, 0.6, 0.0])
    ez = np.array([0.0, 0.0, 1.0])
    q = [c - 0.6 * u + 0.05 * ez, c + 0.6 * u + 0.05 * ez, c + 0.6 * u + 2 * ez, c - 0.6 * u + 2 * ez]
    tris += [[q[0], q[1], q[2]], [q[0], q[2], q[3]]]
    lights = [wl.directional_light(L, cone_deg) for L in (L0, L1, L2)]
    return np.array(tris, np.float32), lights


def _fig1_golden():
    """The bitmasks Fig. 1 prints, from tests/golden/fig1_bitmasks.txt."""
    path = os.path.join(os.path.dirname(__file__), "golden", "fig1_bitmasks.txt")
    rows = [ln.split() for ln in open(path) if ln.strip() and not ln.startswith("#")]
    return {case: int(bits, 2) for case, bits in rows}


def test_fig1_bitmask_example(orc):
    golden = _fig1_golden()
    assert set(golden) == {"hard", "soft"}
    tris, hard = _fig1_scene(0.0)
    s = orc.Scene(tris)
    pos = np.array([[0.0, 0.0, 0.0, 0.0]], np.float32)
    nz = np.array([[0.0, 1.0, 0.0, 1.0]], np.float32)

    def mask(lights, frame):
        P = orc.trace_params(1, 1, frame=frame, seed=1, n_ao=0, n_shadow=1, lights=lights)
        _, sh, _ = orc.trace(s, P, pos, nz)
        return sum(int(sh[i, 0]) << i for i in range(3))

    assert all(mask(hard, f) == golden["hard"] for f in range(16))
    _, soft = _fig1_scene(10.0)
    masks = [mask(soft, f) for f in range(64)]
    # lights 0 and 1 never change; light 2 is sometimes revealed as occluded
    # (the rays that miss the occluder keep the hard-shadow mask)
    assert set(masks) == {golden["hard"], golden["soft"]}


def test_penumbra_matches_quadrature(orc):
    h = 1.0
    sc = wl.scene_edge_occluder(height=h)
    s = orc.Scene(sc.tris, sc.obj_id)
    half_deg = 5.0
    L = wl.directional_light((0.0, 1.0, 0.0), half_deg)
    xs = np.linspace(-0.12, 0.12, 13)
    npx = xs.size
    pos = np.zeros((npx, 4), np.float32)
    pos[:, 0] = xs
    nz = np.tile(np.array([0, 1, 0, 1], np.float32), (npx, 1))
    frames, nsh = 8, 255
    cnt = np.zeros(npx)
    for f in range(frames):
        P = orc.trace_params(npx, 1, frame=f, seed=3, n_ao=0, n_shadow=nsh, lights=[L], eps_origin_abs=1e-4)
        _, sh, _ = orc.trace(s, P, pos, nz)
        cnt += sh[0]
    vis = cnt / (frames * nsh)
    # FP64 quadrature of the unoccluded fraction of the cone (uniform in solid angle)
    k = L.one_minus_cos
    m = 1500
    ct = 1.0 - (np.arange(m) + 0.5) / m * k
    st = np.sqrt(1 - ct ** 2)
    phi = 2 * np.pi * (np.arange(2 * m) + 0.5) / (2 * m)
    wx = st[:, None] * np.cos(phi)[None, :]       # axis = +y, tangent x
    wy = ct[:, None] * np.ones_like(phi)[None, :]
    for j, x in enumerate(xs):
        xh = x + (h - 1e-4) / wy * wx
        q = (xh >= 0).mean()
        sigma = math.sqrt(max(q * (1 - q), 1e-4) / (frames * nsh))
        assert abs(vis[j] - q) <= 5 * sigma + 2e-3, (x, vis[j], q)
    assert vis[0] == 0.0 and vis[-1] == 1.0


def test_sphere_light_bounds(orc):
    # a ceiling above the sphere light does not occlude it; one between does
    pos = np.array([[0, 0, 0, 0]], np.float32)
    nz = np.array([[0, 1, 0, 1]], np.float32)
    L = wl.sphere_light((0.0, 3.0, 0.0), 0.5)
    ceiling = np.array([[(-9, 5, -9), (9, 5, 9), (-9, 5, 9)], [(-9, 5, -9), (9, 5, -9), (9, 5, 9)]], np.float32)
    s = orc.Scene(ceiling)
    P = orc.trace_params(1, 1, seed=1, n_ao=0, n_shadow=64, lights=[L])
    _, sh, _ = orc.trace(s, P, pos, nz)
    assert sh[0, 0] == 64
    s2 = orc.Scene(ceiling - np.array([0, 3.5, 0], np.float32))    # plane y = 1.5
    _, sh, _ = orc.trace(s2, P, pos, nz)
    assert sh[0, 0] == 0
    # a point inside the light sphere sees the light
    L_in = wl.sphere_light((0.0, 0.2, 0.0), 0.5)
    P = orc.trace_params(1, 1, seed=1, n_ao=0, n_shadow=16, lights=[L_in])
    _, sh, _ = orc.trace(s2, P, pos, nz)
    assert sh[0, 0] == 16
