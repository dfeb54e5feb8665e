"""Two-level hierarchies for instanced geometry (needs an MI355X).

The reference is the flattened scene: the oracle traces every instance's
copy of the mesh as world triangles (computed in float64 and rounded once),
while the GPU transforms each ray into the mesh's space, so the two differ
only by rounding:
* visibility rays on the large terrain workload (5,000 instanced boxes)
  mismatch the oracle in at most 1e-4 of the rays; the G-buffer's object ids,
  and positions beyond 1e-4 (relative), differ in at most 1e-4 of the pixels;
* the same for a small scene of rotated, anisotropically scaled instances
  of a curved mesh over a plane;
* calls that do not take a two-level hierarchy say so; bad transforms are
  rejected.
"""
import numpy as np
import pytest

import oracle as orc
from paper_2406_06963_amd import workloads as wl
from oracle_inputs import frames, popcount64, scene

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


def check_against_oracle(B, ctx, bvh, so, W, H, cam, prev, kw, what):
    import torch
    pos, nz, dz, mv = orc.gbuffer(so, cam, prev, W, H)
    g = B.gbuffer_tensors(W, H)
    B.dhr_gbuffer(ctx, bvh, cam, prev, W, H, g["pos"], g["nz"], g["dz"], g["mv"])
    gp = g["pos"].cpu().numpy()
    ids = gp[:, 3].view(np.uint32)
    same = ids == orc.id_bits(pos)
    hit = same & (nz[:, 3] > 0)
    # same object, but the fp32 and FP64 rays may pass a silhouette on either
    # side (another surface of it): a bounded number of discrete choices
    perr = np.abs(gp[:, :3] - pos[:, :3]).max(1) / (np.abs(pos[:, :3]).max(1) + 1.0)
    other = hit & (perr > 1e-4)
    print(f"{what}: G-buffer ids differ at {(~same).sum()}, positions at {other.sum()} of {W * H} pixels",
          flush=True)
    assert (~same).mean() <= 1e-4 and other.mean() <= 1e-4
    assert np.abs(g["nz"].cpu().numpy()[hit & ~other, 3] - nz[hit & ~other, 3]).max() <= 1e-3 * nz[:, 3].max()
    L, HW = len(kw["lights"]), W * H
    ao = torch.empty(HW, dtype=torch.uint8, device="cuda")
    sh = torch.empty(max(L, 1), HW, dtype=torch.uint8, device="cuda")
    rb = torch.empty(1 + L, HW, dtype=torch.int64, device="cuda")
    B.dhr_trace_visibility(ctx, bvh, B.trace_params(W, H, **kw), dev(pos), dev(nz), ao, sh, rb)
    _, _, bits_o = orc.trace(so, orc.trace_params(W, H, **kw), pos, nz, ray_bits=True)
    bad = popcount64(rb.cpu().numpy().view(np.uint64) ^ bits_o)
    n_rays = HW * (kw["n_ao"] + L * kw["n_shadow"])
    print(f"{what}: {bad} of {n_rays} rays differ", flush=True)
    assert bad <= 1e-4 * n_rays


def test_terrain_instances_match_the_flattened_oracle(B, ctx):
    pr, fr = frames("terrain1080", 2)
    sc, so = scene(pr.scene)
    bt, bo, mesh, xf, ids = wl.instanced_form(sc)
    bvh = B.dhr_build_bvh_instanced(ctx, bt, bo, mesh, xf, ids)
    info = bvh.info()
    assert info["n_tris"] == len(bt) + len(mesh)
    kw = dict(fr[1]["trace_kw"], n_ao=1, n_shadow=2)
    check_against_oracle(B, ctx, bvh, so, pr.W, pr.H, fr[1]["cam"], fr[0]["cam"], kw, "terrain")


def _rotation(rng):
    q = rng.normal(size=4)
    q /= np.linalg.norm(q)
    w, x, y, z = q
    return np.array([[1 - 2 * (y * y + z * z), 2 * (x * y - z * w), 2 * (x * z + y * w)],
                     [2 * (x * y + z * w), 1 - 2 * (x * x + z * z), 2 * (y * z - x * w)],
                     [2 * (x * z - y * w), 2 * (y * z + x * w), 1 - 2 * (x * x + y * y)]])


def test_rotated_scaled_instances(B, ctx):
    rng = np.random.default_rng(21)
    ground = wl.scene_plane(half=20.0).tris
    mesh = np.asarray(wl.make_scene("spheres").tris[-480:], np.float32)   # one UV sphere's triangles
    mesh = mesh - mesh.reshape(-1, 3).mean(0)                              # centred
    K = 24
    xf = np.zeros((K, 3, 4))
    for k in range(K):
        xf[k, :, :3] = _rotation(rng) @ np.diag(rng.uniform(0.4, 2.0, 3))
        xf[k, :, 3] = (rng.uniform(-6, 6), rng.uniform(0.5, 3.0), rng.uniform(-6, 6))
    xf = xf.astype(np.float32)
    ids = np.arange(1, K + 1, dtype=np.uint32)
    flat = [ground.astype(np.float64)]
    for k in range(K):
        A = xf[k].astype(np.float64)
        flat.append(mesh.astype(np.float64) @ A[:, :3].T + A[:, 3])
    tris = np.concatenate(flat).astype(np.float32)
    obj = np.concatenate([np.zeros(len(ground), np.uint32), np.repeat(ids, len(mesh))])
    so = orc.Scene(tris, obj)
    bvh = B.dhr_build_bvh_instanced(ctx, ground, np.zeros(len(ground), np.uint32), mesh, xf, ids)
    cams = [wl.Camera(eye=(9.0, 6.0, -11.0), target=(0.0, 1.0, 0.0), fov_y=0.9),
            wl.Camera(eye=(8.5, 6.2, -11.4), target=(0.0, 1.0, 0.0), fov_y=0.9)]
    kw = dict(frame=3, seed=9, n_ao=4, ao_radius=2.0, n_shadow=2, lights=wl.lights_for("spheres"))
    check_against_oracle(B, ctx, bvh, so, 160, 120, cams[1], cams[0], kw, "instances")


def test_unsupported_calls_and_bad_transforms(B, ctx):
    import torch
    ground = wl.scene_plane(half=5.0).tris
    mesh = np.asarray(wl.make_scene("spheres").tris[-480:], np.float32)
    xf = np.tile(np.float32([[1, 0, 0, 0], [0, 1, 0, 1], [0, 0, 1, 0]]), (2, 1, 1))
    bvh = B.dhr_build_bvh_instanced(ctx, ground, None, mesh, xf)
    cam = wl.Camera(eye=(0.0, 3.0, -6.0), target=(0.0, 0.5, 0.0))
    g = B.gbuffer_tensors(16, 16)
    work = torch.empty(B.dhr_gbuffer_raster_workspace_bytes(16, 16, 1000) // 4 + 64, device="cuda")
    with pytest.raises(B.DhrError):
        B.dhr_gbuffer_raster(ctx, bvh, cam, None, 16, 16, g["pos"], g["nz"], g["dz"], g["mv"], work)
    with pytest.raises(B.DhrError):
        B.dhr_refit_bvh(ctx, bvh, dev(np.zeros((len(ground), 9), np.float32)))
    with pytest.raises(B.DhrError):
        B.dhr_bvh_export(ctx, bvh)
    cnt = torch.zeros(4, dtype=torch.int64, device="cuda")
    B.dhr_set_trace_counters(ctx, cnt)
    try:
        B.dhr_gbuffer(ctx, bvh, cam, None, 16, 16, g["pos"], g["nz"], g["dz"], g["mv"])
        ao = torch.empty(256, dtype=torch.uint8, device="cuda")
        with pytest.raises(B.DhrError):
            B.dhr_trace_visibility(ctx, bvh, B.trace_params(16, 16, n_ao=1, ao_radius=1.0, n_shadow=0, lights=[]),
                                   g["pos"], g["nz"], ao, None)
    finally:
        B.dhr_set_trace_counters(ctx, None)
    singular = xf.copy()
    singular[1, :, :3] = 0.0
    with pytest.raises(B.DhrError):
        B.dhr_build_bvh_instanced(ctx, ground, None, mesh, singular)
    nan = xf.copy()
    nan[0, 0, 3] = np.nan
    with pytest.raises(B.DhrError):
        B.dhr_build_bvh_instanced(ctx, ground, None, mesh, nan)
    with pytest.raises(B.DhrError):
        B.dhr_build_bvh_instanced(ctx, ground, None, mesh, xf[:0])
