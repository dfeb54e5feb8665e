"""Limits of the batched calls and of the ray parameters (needs an MI355X).

* Batches longer than one launch holds (trace 12 jobs, G-buffer 16, filter
  24 frames), mixing single- and two-level hierarchies, equal the per-job
  calls bitwise.
* Eight lights (directional and sphere), 255 AO rays and 3 rays per light
  on one frame: the per-pixel counts agree with the oracle's to within the
  visibility mismatch budget.
"""
import numpy as np
import pytest

import oracle as orc
from paper_2406_06963_amd import workloads as wl
from oracle_inputs import frames, scene

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


def _instanced_spheres(B, ctx):
    # the tiny scene's ground and its first sphere placed twice more
    sc, _ = scene("spheres")
    ground, mesh = sc.tris[:2], sc.tris[2:482]
    xf = np.float32([[[1, 0, 0, 0], [0, 1, 0, 0], [0, 0, 1, 0]], [[0.5, 0, 0, 2.0], [0, 0.5, 0, 0.3], [0, 0, 0.5, -1.0]]])
    return B.dhr_build_bvh_instanced(ctx, ground, sc.obj_id[:2], mesh, xf, np.uint32([1, 9]))


def test_batches_beyond_one_launch(B, ctx):
    import torch
    pr, fr = frames("tiny", 2)
    sc, _ = scene("spheres")
    flat = B.dhr_build_bvh(ctx, sc.tris, sc.obj_id)
    inst = _instanced_spheres(B, ctx)
    n = 30
    sizes = [(64, 64), (48, 40), (33, 17), (64, 8)]
    cams = wl.camera_path(pr.camera, n + 1, sc)
    # G-buffers: 30 jobs, two hierarchy kinds, ragged sizes
    gj = []
    for k in range(n):
        W, H = sizes[k % 4]
        gj.append(dict(bvh=flat if k % 3 else inst, cur=cams[k + 1], prev=cams[k], W=W, H=H, **B.gbuffer_tensors(W, H)))
    B.dhr_gbuffer_batch(ctx, gj)
    for j in gj:
        g = B.gbuffer_tensors(j["W"], j["H"])
        B.dhr_gbuffer(ctx, j["bvh"], j["cur"], j["prev"], j["W"], j["H"], g["pos"], g["nz"], g["dz"], g["mv"])
        for key in ("pos", "nz", "dz", "mv"):
            assert torch.equal(g[key].view(torch.int32), j[key].view(torch.int32)), key
    # visibility: 30 jobs on those G-buffers
    lights = wl.lights_for("spheres")
    tj, singles = [], []
    for k, j in enumerate(gj):
        W, H = j["W"], j["H"]
        tp = B.trace_params(W, H, frame=k, seed=3, n_ao=3, ao_radius=1.0, n_shadow=2, lights=lights)
        ao = torch.empty(W * H, dtype=torch.uint8, device="cuda")
        sh = torch.empty(1, W * H, dtype=torch.uint8, device="cuda")
        B.dhr_trace_visibility(ctx, j["bvh"], tp, j["pos"], j["nz"], ao, sh)
        singles.append((ao, sh))
        tj.append(dict(bvh=j["bvh"], params=tp, pos=j["pos"], nz=j["nz"],
                       ao_count=torch.empty_like(ao), shadow_count=torch.empty_like(sh)))
    B.dhr_trace_visibility_batch(ctx, tj)
    for j, (ao, sh) in zip(tj, singles):
        assert torch.equal(j["ao_count"], ao) and torch.equal(j["shadow_count"], sh)
    # filter: 30 frames in one call (no history) against one call per frame
    P = B.svgf_params()
    outs, ones = [], []
    frs = []
    for k, (j, (ao, _)) in enumerate(zip(gj, singles)):
        W, H = j["W"], j["H"]
        work = torch.empty(B.dhr_svgf_workspace_bytes(W, H, P, 0) // 4, device="cuda")
        hist = torch.empty(W * H, 4, device="cuda")
        out = torch.empty(W * H, device="cuda")
        frs.append(B.svgf_frame(W, H, 3, ao, j["pos"], j["nz"], j["dz"], j["mv"], None, None, None, hist, out,
                                B.pix_angle(j["cur"], H), work=work))
        outs.append((out, hist, work))
    B.dhr_svgf_filter(ctx, P, frs)
    for fr_, (out, hist, work) in zip(frs, outs):
        o1, h1 = out.clone(), hist.clone()
        B.dhr_svgf_filter(ctx, P, [fr_])
        assert torch.equal(out, o1) and torch.equal(hist, h1)


def test_eight_lights_and_many_rays(B, ctx):
    import torch
    pr, fr = frames("tiny", 1)
    sc, so = scene("spheres")
    f = fr[0]
    lights = [wl.directional_light((0.4, 1.0, 0.3), 1.0), wl.directional_light((-0.5, 0.8, 0.1), 3.0),
              wl.directional_light((0.0, 1.0, -0.6), 0.25), wl.directional_light((0.7, 0.4, 0.7), 5.0),
              wl.sphere_light((2.0, 4.0, 1.0), 0.5), wl.sphere_light((-3.0, 2.5, -2.0), 1.0),
              wl.sphere_light((0.5, 1.2, 3.0), 0.2), wl.sphere_light((-1.0, 6.0, 4.0), 2.0)]
    kw = dict(frame=2, seed=11, n_ao=255, ao_radius=1.0, n_shadow=3, lights=lights)
    W, H = pr.W, pr.H
    ao = torch.empty(W * H, dtype=torch.uint8, device="cuda")
    sh = torch.empty(8, W * H, dtype=torch.uint8, device="cuda")
    B.dhr_trace_visibility(ctx, B.dhr_build_bvh(ctx, sc.tris, sc.obj_id), B.trace_params(W, H, **kw), dev(f["pos"]),
                           dev(f["nz"]), ao, sh)
    ao_o, sh_o, _ = orc.trace(so, orc.trace_params(W, H, **kw), f["pos"], f["nz"])
    n_rays = W * H * (255 + 8 * 3)
    diff = int(np.abs(ao.cpu().numpy().astype(int) - ao_o.astype(int)).sum()
               + np.abs(sh.cpu().numpy().astype(int) - sh_o.reshape(8, -1).astype(int)).sum())
    print(f"eight lights, 255 AO rays: count differences sum to {diff} over {n_rays} rays", flush=True)
    assert diff <= 1e-4 * n_rays
    assert ao.cpu().numpy().max() <= 255 and (sh.cpu().numpy() <= 3).all()
