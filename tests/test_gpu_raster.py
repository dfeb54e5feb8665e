"""The rasterised G-buffer (needs an MI355X).

Its texels are defined as those of the ray-traced G-buffer (closest hit of
each pixel's primary ray, ties to the lowest input index), so the check is
bitwise equality with dhr_gbuffer on the same triangles, on every workload,
ragged and one-pixel images, with the BVH of either builder, for a camera
whose eye lies almost on a triangle's plane (those triangles propose the
whole frame), triangles crossing the camera plane and a degenerate sliver;
plus the oracle's G-buffer on the small workload, and argument errors.
"""
import numpy as np
import pytest

import oracle as orc
from paper_2406_06963_amd import workloads as wl
from oracle_inputs import scene

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def B():
    import torch
    assert torch.cuda.is_available(), "GPU test run without a GPU"
    from paper_2406_06963_amd import binding
    binding.load()
    return binding


@pytest.fixture(scope="module")
def ctx(B):
    return B.dhr_create(0)


def dev(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda")


def both(B, ctx, bvh, cur, prev, W, H, n_tris):
    import torch
    g1, g2 = B.gbuffer_tensors(W, H), B.gbuffer_tensors(W, H)
    work = torch.empty((B.dhr_gbuffer_raster_workspace_bytes(W, H, n_tris) + 15) // 16 * 4, dtype=torch.float32,
                       device="cuda")
    B.dhr_gbuffer(ctx, bvh, cur, prev, W, H, g1["pos"], g1["nz"], g1["dz"], g1["mv"])
    B.dhr_gbuffer_raster(ctx, bvh, cur, prev, W, H, g2["pos"], g2["nz"], g2["dz"], g2["mv"], work)
    torch.cuda.synchronize()
    return g1, g2


def assert_same(g1, g2, what):
    import torch
    for k in ("pos", "nz", "dz", "mv"):   # bitwise (a miss's id and motion are NaN patterns)
        a, b = g1[k].view(torch.int32), g2[k].view(torch.int32)
        bad = int((a != b).any(dim=1).sum().item())
        assert bad == 0, (what, k, bad)


@pytest.mark.parametrize("preset", ["tiny", "room720", "terrain1080", "ragged", "sliver"])
def test_raster_equals_ray_traced(B, ctx, preset):
    pr = wl.preset(preset)
    sc, _ = scene(pr.scene)
    cams = wl.camera_path(pr.camera, 3, sc)
    bvh = B.dhr_build_bvh(ctx, sc.tris, sc.obj_id)
    for f in (0, 2):
        g1, g2 = both(B, ctx, bvh, cams[f], cams[f - 1] if f else None, pr.W, pr.H, sc.n_tris)
        valid = float((g1["nz"][:, 3] > 0).float().mean().item())
        print(f"{preset} frame {f}: {valid:.3f} of the pixels hit", flush=True)
        assert_same(g1, g2, (preset, f))


def test_raster_on_device_built_hierarchy(B, ctx):
    pr = wl.preset("room720")
    sc, _ = scene(pr.scene)
    cams = wl.camera_path(pr.camera, 2, sc)
    bvh = B.dhr_build_bvh_device(ctx, dev(np.asarray(sc.tris, np.float32).reshape(-1, 9)),
                                 dev(np.asarray(sc.obj_id, np.uint32).view(np.int32)))
    g1, g2 = both(B, ctx, bvh, cams[1], cams[0], pr.W, pr.H, sc.n_tris)
    assert_same(g1, g2, "device bvh")


def test_raster_matches_the_oracle(B, ctx):
    pr = wl.preset("tiny")
    sc, so = scene(pr.scene)
    cams = wl.camera_path(pr.camera, 2, sc)
    bvh = B.dhr_build_bvh(ctx, sc.tris, sc.obj_id)
    _, g = both(B, ctx, bvh, cams[1], cams[0], pr.W, pr.H, sc.n_tris)
    pos, nz, dz, mv = orc.gbuffer(so, cams[1], cams[0], pr.W, pr.H)
    ids = g["pos"].cpu().numpy()[:, 3].view(np.uint32)
    assert (ids != orc.id_bits(pos)).mean() <= 1e-4
    ok = (ids == orc.id_bits(pos)) & (nz[:, 3] > 0)
    assert np.abs(g["pos"].cpu().numpy()[ok, :3] - pos[ok, :3]).max() <= 1e-3


def _grid_plane(n, half, y=0.0, z_plane=False):
    # an n x n grid of quads (two triangles each) on y = const (or z = const)
    xs = np.linspace(-half, half, n + 1)
    tris = []
    for i in range(n):
        for j in range(n):
            a, b, c, d = ((xs[i], xs[j]), (xs[i + 1], xs[j]), (xs[i + 1], xs[j + 1]), (xs[i], xs[j + 1]))
            for t in ((a, b, c), (a, c, d)):
                tris.append([(u, y, v) if not z_plane else (u, v, y) for u, v in t])
    return np.asarray(tris, np.float32)


def test_near_and_crossing_triangles(B, ctx):
    # ground grid, a wall grid crossing the camera plane, a sliver with two
    # equal vertices; the eye 1e-5 above the ground (closer than the clip
    # neighbourhood), looking along it and slightly down
    ground = _grid_plane(24, 6.0)
    wall = _grid_plane(8, 4.0, y=0.5, z_plane=True)
    sliver = np.asarray([[(0.5, 0.2, 2.0), (0.5, 0.2, 2.0), (0.9, 0.6, 2.5)]], np.float32)
    tris = np.concatenate([ground, wall, sliver])
    ids = np.arange(len(tris), dtype=np.uint32)
    bvh = B.dhr_build_bvh(ctx, tris, ids)
    for eye, target in (((0.13, 1e-5, -0.4), (2.0, -0.05, 3.0)),     # eye almost on the ground plane
                        ((0.3, 0.4, 0.5), (-1.0, 0.2, 1.7)),         # wall plane through the frame
                        ((0.1, 1.5, -3.0), (0.0, 0.0, 0.0))):
        cam = wl.Camera(eye=eye, target=target, fov_y=1.1)
        for W, H in ((96, 64), (37, 23)):
            g1, g2 = both(B, ctx, bvh, cam, None, W, H, len(tris))
            assert (g1["nz"][:, 3] > 0).any()
            assert_same(g1, g2, (eye, W, H))


def test_one_pixel_and_argument_errors(B, ctx):
    import torch
    pr = wl.preset("tiny")
    sc, _ = scene(pr.scene)
    cams = wl.camera_path(pr.camera, 1, sc)
    bvh = B.dhr_build_bvh(ctx, sc.tris, sc.obj_id)
    for W, H in ((1, 1), (1, 7), (9, 1)):
        g1, g2 = both(B, ctx, bvh, cams[0], None, W, H, sc.n_tris)
        assert_same(g1, g2, (W, H))
    g = B.gbuffer_tensors(8, 8)
    need = B.dhr_gbuffer_raster_workspace_bytes(8, 8, sc.n_tris)
    short = torch.empty(need // 4 - 4, dtype=torch.float32, device="cuda")
    with pytest.raises(B.DhrError):
        B.dhr_gbuffer_raster(ctx, bvh, cams[0], None, 8, 8, g["pos"], g["nz"], g["dz"], g["mv"], short)
    work = torch.empty(need // 4 + 8, dtype=torch.float32, device="cuda")
    with pytest.raises(B.DhrError):
        B.dhr_gbuffer_raster(ctx, bvh, cams[0], None, 0, 8, g["pos"], g["nz"], g["dz"], g["mv"], work)
    with pytest.raises(B.DhrError):
        B.dhr_gbuffer_raster(ctx, bvh, cams[0], None, 8, 8, g["pos"], g["nz"], g["dz"], g["mv"], work[1:])
