"""Pins of the oracle's G-buffer (no GPU): closed forms of a pinhole camera
looking at planes.

The G-buffer carries the world position of each pixel (Section 2.2) and
motion vectors that back-project it into the previous frame (Section 3.3).
"""
import math

import numpy as np

from paper_2406_06963_amd import workloads as wl


def _screen(W, H, fov):
    th = math.tan(fov / 2)
    x = np.arange(W) + 0.5
    y = np.arange(H) + 0.5
    sx = (2 * x / W - 1) * th * W / H
    sy = (1 - 2 * y / H) * th
    return np.meshgrid(sx, sy, indexing="xy")


def _wall(z=-5.0, half=100.0, obj=0):
    return [[(-half, -half, z), (half, -half, z), (half, half, z)], [(-half, -half, z), (half, half, z), (-half, half, z)]]


def test_fronto_parallel_wall(orc):
    W, H = 40, 24
    tris = np.array(_wall(), np.float32)
    s = orc.Scene(tris, np.array([3, 3], np.uint32))
    cam = wl.Camera((0.0, 0.0, 0.0), (0.0, 0.0, -1.0))
    prev = wl.Camera((0.1, 0.0, 0.0), (0.1, 0.0, -1.0))
    pos, nz, dz, mv = orc.gbuffer(s, cam, prev, W, H)
    sx, sy = _screen(W, H, cam.fov_y)
    np.testing.assert_allclose(pos[:, 0], (5 * sx).ravel(), rtol=1e-6, atol=1e-6)
    np.testing.assert_allclose(pos[:, 1], (5 * sy).ravel(), rtol=1e-6, atol=1e-6)
    np.testing.assert_allclose(pos[:, 2], -5.0, rtol=1e-7)
    assert (orc.id_bits(pos) == 3).all()
    np.testing.assert_allclose(nz[:, :3], np.broadcast_to([0, 0, 1], (W * H, 3)), atol=1e-7)
    np.testing.assert_allclose(nz[:, 3], 5.0, rtol=1e-7)
    np.testing.assert_allclose(dz, 0.0, atol=1e-5)
    # previous camera 0.1 to the right: every point moves by -0.1/(5 tan(fov/2) aspect) * W/2 pixels
    shift = -0.1 / (5 * math.tan(cam.fov_y / 2) * W / H) * W / 2
    np.testing.assert_allclose(mv[:, 0], shift, rtol=1e-5)
    np.testing.assert_allclose(mv[:, 1], 0.0, atol=1e-5)


def test_floor_depth_gradient_and_misses(orc):
    W, H, h = 32, 48, 1.5
    half = 1e4
    tris = np.array([[(-half, 0, -half), (-half, 0, half), (half, 0, half)],
                     [(-half, 0, -half), (half, 0, half), (half, 0, -half)]], np.float32)
    s = orc.Scene(tris, np.array([0, 0], np.uint32))
    cam = wl.Camera((0.0, h, 0.0), (0.0, h, -1.0))
    pos, nz, dz, mv = orc.gbuffer(s, cam, None, W, H)
    sx, sy = _screen(W, H, cam.fov_y)
    below = (sy < -0.05).ravel()
    above = (sy > 0).ravel()
    # above the horizon: misses (invalid pixels, depth 0, id 0xFFFFFFFF)
    assert (orc.id_bits(pos)[above] == 0xFFFFFFFF).all()
    assert (nz[above, 3] == 0).all()
    z = (h / -sy).ravel()
    np.testing.assert_allclose(nz[below, 3], z[below], rtol=1e-6)
    np.testing.assert_allclose(nz[below, :3], np.broadcast_to([0, 1, 0], (below.sum(), 3)), atol=1e-7)
    # dz.y: the floor's depth through the pixel one row down, minus z
    y = np.arange(H) + 0.5
    sy1 = (1 - 2 * (y + 1) / H) * math.tan(cam.fov_y / 2)
    dzy = (h / -sy1[:, None] - h / -sy[:, :1]) * np.ones((1, W))
    np.testing.assert_allclose(dz[below, 1], dzy.ravel()[below], rtol=1e-5)
    np.testing.assert_allclose(dz[below, 0], 0.0, atol=1e-4)
    # no previous camera: motion is NaN
    assert np.isnan(mv[below]).all()


def test_occluder_ids_and_sentinel(orc):
    W, H = 16, 16
    wall = _wall()
    near = [[(-0.5, -0.5, -2), (0.5, -0.5, -2), (0.5, 0.5, -2)], [(-0.5, -0.5, -2), (0.5, 0.5, -2), (-0.5, 0.5, -2)]]
    tris = np.array(wall + near, np.float32)
    s = orc.Scene(tris, np.array([1, 1, 2, 2], np.uint32))
    cam = wl.Camera((0.0, 0.0, 0.0), (0.0, 0.0, -1.0))
    pos, nz, dz, mv = orc.gbuffer(s, cam, cam, W, H)
    sx, sy = _screen(W, H, cam.fov_y)
    inside = ((np.abs(2 * sx) < 0.49) & (np.abs(2 * sy) < 0.49)).ravel()
    outside = ((np.abs(2 * sx) > 0.51) | (np.abs(2 * sy) > 0.51)).ravel()
    ids = orc.id_bits(pos)
    assert (ids[inside] == 2).all() and (ids[outside] == 1).all()
    np.testing.assert_allclose(nz[inside, 3], 2.0, rtol=1e-7)
    # same camera: zero motion
    np.testing.assert_allclose(mv, 0.0, atol=1e-4)
    # the ceiling seen just above the horizon: the ray of the pixel one row
    # down meets the ceiling's plane behind the camera -> dz.y = 1e20 sentinel
    half = 1e4
    tris = np.array([[(-half, 1, -half), (half, 1, half), (-half, 1, half)],
                     [(-half, 1, -half), (half, 1, -half), (half, 1, half)]], np.float32)
    s = orc.Scene(tris)
    W, H = 8, 8
    cam = wl.Camera((0.0, 0.0, 0.0), (0.0, 0.0, -1.0))
    pos, nz, dz, mv = orc.gbuffer(s, cam, None, W, H)
    row = (H // 2 - 1) * W + np.arange(W)
    assert (nz[row, 3] > 0).all()
    assert (dz[row, 1] == np.float32(1e20)).all()
    assert (nz[(H // 2) * W:, 3] == 0).all()
