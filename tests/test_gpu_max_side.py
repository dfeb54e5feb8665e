"""Frames at the largest side the calls accept (needs an MI355X).

A 16384 x 8 and an 8 x 16384 frame of the small scene: the tall one through
the scene's own orbit camera (60 degree vertical field, a thin vertical
strip), the wide one seen from above with a 0.047 degree vertical field, so
that its 80 degree horizontal field spans the ground and the spheres:
* the fused G-buffer + visibility call's texel ids against the oracle's;
* per-ray visibility bits traced from the oracle's G-buffer against the
  oracle's;
* one filtered frame (frame 1 on the oracle's history of frame 0) against
  the oracle's, within the filter tolerance;
* a side of 16385 is refused before anything is launched.
"""
import dataclasses
import math

import numpy as np
import pytest

import oracle as orc
from paper_2406_06963_amd import workloads as wl
from oracle_inputs import frames, popcount64, scene

pytestmark = pytest.mark.gpu

MISMATCH_RATE = 1e-4   # visibility rays and texel ids that may differ
ATOL = 1e-4            # filtered AO


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
    return None if a is None else torch.from_numpy(np.ascontiguousarray(a)).to("cuda")


@pytest.mark.parametrize("W,H", [(16384, 8), (8, 16384)])
def test_maximum_side(B, ctx, W, H):
    import torch
    cams = None
    if W > H:
        cams = [wl.Camera((0.0, 12.0, 3.0 + 0.01 * f), (0.0, 0.0, 0.0), math.radians(0.0466)) for f in range(2)]
    pr, fr = frames(dataclasses.replace(wl.preset("tiny"), W=W, H=H), 2, cams=cams)
    sc, so = scene(pr.scene)
    bvh = B.dhr_build_bvh(ctx, sc.tris, sc.obj_id)
    f, f0 = fr[1], fr[0]
    HW, L = W * H, len(f["trace_kw"]["lights"])
    # fused G-buffer + visibility: texel ids
    g = B.gbuffer_tensors(W, H)
    ao = torch.empty(HW, dtype=torch.uint8, device="cuda")
    sh = torch.empty(L, HW, dtype=torch.uint8, device="cuda")
    B.dhr_gbuffer_trace(ctx, bvh, f["cam"], f0["cam"], W, H, B.trace_params(W, H, **f["trace_kw"]),
                        g["pos"], g["nz"], g["dz"], g["mv"], ao, sh)
    ids = g["pos"].cpu().numpy()[:, 3].view(np.uint32)
    id_bad = int((ids != orc.id_bits(f["pos"])).sum())
    # visibility rays from the oracle's G-buffer
    rb = torch.empty(1 + L, HW, dtype=torch.int64, device="cuda")
    B.dhr_trace_visibility(ctx, bvh, B.trace_params(W, H, **f["trace_kw"]), dev(f["pos"]), dev(f["nz"]), ao, sh, rb)
    _, _, bits_o = orc.trace(so, orc.trace_params(W, H, **f["trace_kw"]), f["pos"], f["nz"], ray_bits=True)
    rays = int((f["nz"][:, 3] > 0).sum()) * (pr.n_ao + L * pr.n_shadow)
    ray_bad = popcount64(rb.cpu().numpy().view(np.uint64) ^ bits_o)
    # frame 1 filtered on the oracle's history of frame 0
    P, Po = B.svgf_params(levels=pr.levels, alpha=pr.alpha), orc.svgf_params(levels=pr.levels, alpha=pr.alpha)
    h0 = orc.svgf_filter(Po, W, H, pr.n_ao, f0["ao"], f0["pos"], f0["nz"], f0["dz"], f0["mv"], None, None, None,
                         f0["pix"])["hist_out"].astype(np.float32)
    ref = orc.svgf_filter(Po, W, H, pr.n_ao, f["ao"], f["pos"], f["nz"], f["dz"], f["mv"], f0["pos"], f0["nz"], h0,
                          f["pix"])
    hist = torch.empty(HW, 4, device="cuda")
    out = torch.empty(HW, device="cuda")
    work = torch.empty(B.dhr_svgf_workspace_bytes(W, H, P, 0) // 4, device="cuda")
    B.dhr_svgf_filter(ctx, P, [B.svgf_frame(W, H, pr.n_ao, dev(f["ao"]), dev(f["pos"]), dev(f["nz"]), dev(f["dz"]),
                                            dev(f["mv"]), dev(f0["pos"]), dev(f0["nz"]), dev(h0), hist, out,
                                            float(f["pix"]), work=work)])
    err = float(np.abs(out.cpu().numpy() - ref["out"]).max())
    valid = int((f["nz"][:, 3] > 0).sum())
    assert valid >= HW // 2
    print(f"{W}x{H}: {valid} valid pixels; ids differ at {id_bad} of {HW} pixels, {ray_bad} of {rays} rays differ, "
          f"max |out - oracle| {err:.2e}", flush=True)
    assert id_bad <= MISMATCH_RATE * HW
    assert ray_bad <= max(1, MISMATCH_RATE * rays)
    assert err <= ATOL


def test_side_beyond_the_maximum_is_refused(B, ctx):
    sc, _ = scene("spheres")
    bvh = B.dhr_build_bvh(ctx, sc.tris, sc.obj_id)
    cam = wl.camera_path(wl.preset("tiny").camera, 1, sc)[0]
    for W, H in ((16385, 1), (1, 16385)):
        g = B.gbuffer_tensors(W, H)
        with pytest.raises(B.DhrError):
            B.dhr_gbuffer(ctx, bvh, cam, None, W, H, g["pos"], g["nz"], g["dz"], g["mv"])
