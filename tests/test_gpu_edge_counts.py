"""Degenerate ray counts and a one-pixel frame (needs an MI355X).

* No AO rays, no lights (shadow_count NULL), no shadow rays with a light:
  every stream's per-ray bits against the oracle's, the counts of an empty
  stream exactly 0 (invalid pixels count as fully visible: n rays = 0), and
  the fused G-buffer + visibility call equal to the two separate calls.
* A 1 x 1 frame: the texel's object id against the oracle's, and the fused
  call equal to the two separate calls.
* Non-default client id (the generator's key), AO sample offset (its
  counter) and absolute origin offset: per-ray bits against the oracle's.
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


def _counts(B, L, HW):
    import torch
    ao = torch.full((HW,), 0xAB, dtype=torch.uint8, device="cuda")
    sh = torch.full((L, HW), 0xCD, dtype=torch.uint8, device="cuda") if L else None
    return ao, sh


@pytest.mark.parametrize("n_ao,n_shadow,n_lights", [(0, 2, 1), (3, 1, 0), (0, 1, 0), (2, 0, 1)])
def test_empty_streams(B, ctx, n_ao, n_shadow, n_lights):
    import torch
    pr, fr = frames("tiny", 2)
    sc, so = scene(pr.scene)
    bvh = B.dhr_build_bvh(ctx, sc.tris, sc.obj_id)
    f = fr[1]
    kw = dict(f["trace_kw"], n_ao=n_ao, n_shadow=n_shadow, lights=f["trace_kw"]["lights"][:n_lights])
    W, H, L = pr.W, pr.H, n_lights
    HW = W * H
    ao, sh = _counts(B, L, HW)
    rb = torch.empty(1 + L, HW, dtype=torch.int64, device="cuda")
    B.dhr_trace_visibility(ctx, bvh, B.trace_params(W, H, **kw), dev(f["pos"]), dev(f["nz"]), ao, sh, rb)
    ao_o, sh_o, bits_o = orc.trace(so, orc.trace_params(W, H, **kw), f["pos"], f["nz"], ray_bits=True)
    bits = rb.cpu().numpy().view(np.uint64)
    rays = int((f["nz"][:, 3] > 0).sum()) * (n_ao + L * n_shadow)
    bad = popcount64(bits ^ bits_o)
    print(f"n_ao {n_ao}, n_shadow {n_shadow}, lights {L}: {bad} of {rays} rays differ", flush=True)
    assert bad <= max(1, 1e-4 * rays)
    if n_ao == 0:
        assert not ao.cpu().numpy().any() and not bits[0].any()
    if L and n_shadow == 0:
        assert not sh.cpu().numpy().any() and not bits[1:].any()
    # the fused call on the device's own G-buffer equals the two calls
    tp = B.trace_params(W, H, **kw)
    cams = wl.camera_path(pr.camera, 2, sc)
    out = []
    for fused in (False, True):
        g = B.gbuffer_tensors(W, H)
        a, s = _counts(B, L, HW)
        if fused:
            B.dhr_gbuffer_trace(ctx, bvh, cams[1], cams[0], W, H, tp, g["pos"], g["nz"], g["dz"], g["mv"], a, s)
        else:
            B.dhr_gbuffer(ctx, bvh, cams[1], cams[0], W, H, g["pos"], g["nz"], g["dz"], g["mv"])
            B.dhr_trace_visibility(ctx, bvh, tp, g["pos"], g["nz"], a, s)
        # bit patterns: a missed pixel's pos.w holds the miss id, a NaN as float
        out.append([g["pos"].view(torch.int32), g["nz"].view(torch.int32), a] + ([s] if L else []))
    for x, y in zip(*out):
        assert torch.equal(x, y)


def test_one_pixel_frame(B, ctx):
    import torch
    pr = wl.preset("tiny")
    sc, so = scene(pr.scene)
    bvh = B.dhr_build_bvh(ctx, sc.tris, sc.obj_id)
    cams = wl.camera_path(pr.camera, 2, sc)
    lights = wl.lights_for(pr.scene)
    tp = B.trace_params(1, 1, frame=1, seed=pr.seed, n_ao=4, ao_radius=1.0, n_shadow=2, lights=lights)
    out = []
    for fused in (False, True):
        g = B.gbuffer_tensors(1, 1)
        a, s = _counts(B, len(lights), 1)
        if fused:
            B.dhr_gbuffer_trace(ctx, bvh, cams[1], cams[0], 1, 1, tp, g["pos"], g["nz"], g["dz"], g["mv"], a, s)
        else:
            B.dhr_gbuffer(ctx, bvh, cams[1], cams[0], 1, 1, g["pos"], g["nz"], g["dz"], g["mv"])
            B.dhr_trace_visibility(ctx, bvh, tp, g["pos"], g["nz"], a, s)
        out.append((g, a, s))
    (g1, a1, s1), (g2, a2, s2) = out
    for k in ("pos", "nz", "dz", "mv"):
        assert torch.equal(g1[k].view(torch.int32), g2[k].view(torch.int32)), k
    assert torch.equal(a1, a2) and torch.equal(s1, s2)
    assert int(a1[0]) <= 4 and int(s1[0, 0]) <= 2
    pos, nz, dz, mv = orc.gbuffer(so, cams[1], cams[0], 1, 1)
    assert g1["pos"].cpu().numpy()[0, 3].view(np.uint32) == orc.id_bits(pos)[0]


@pytest.mark.parametrize("kw", [dict(client_id=7, ao_sample_offset=100, seed=12345),
                                dict(client_id=65535, eps_origin_abs=1e-3, seed=3),
                                dict(ao_sample_offset=65530, seed=9)])
def test_rng_key_counter_and_origin_parameters(B, ctx, kw):
    # the client id keys the generator, the sample offset moves the AO counter,
    # eps_origin_abs replaces the relative origin offset: per-ray bits against
    # the oracle's
    import torch
    pr, fr = frames("tiny", 2)
    sc, so = scene(pr.scene)
    bvh = B.dhr_build_bvh(ctx, sc.tris, sc.obj_id)
    f = fr[1]
    args = dict(f["trace_kw"], n_ao=6, n_shadow=3, **kw)
    W, H, L = pr.W, pr.H, len(args["lights"])
    HW = W * H
    ao, sh = _counts(B, L, HW)
    rb = torch.empty(1 + L, HW, dtype=torch.int64, device="cuda")
    B.dhr_trace_visibility(ctx, bvh, B.trace_params(W, H, **args), dev(f["pos"]), dev(f["nz"]), ao, sh, rb)
    _, _, bits_o = orc.trace(so, orc.trace_params(W, H, **args), f["pos"], f["nz"], ray_bits=True)
    bits = rb.cpu().numpy().view(np.uint64)
    rays = int((f["nz"][:, 3] > 0).sum()) * (6 + L * 3)
    bad = popcount64(bits ^ bits_o)
    print(f"{kw}: {bad} of {rays} rays differ", flush=True)
    assert bad <= max(1, 1e-4 * rays)
    # and the parameters matter: the default key and counter give other rays
    rb0 = torch.empty_like(rb)
    B.dhr_trace_visibility(ctx, bvh, B.trace_params(W, H, **dict(f["trace_kw"], n_ao=6, n_shadow=3)),
                           dev(f["pos"]), dev(f["nz"]), ao, sh, rb0)
    assert not torch.equal(rb, rb0)
