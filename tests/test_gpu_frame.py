"""G-buffer and visibility in one launch (needs an MI355X).

dhr_gbuffer_trace must write exactly the bytes of dhr_gbuffer followed by
dhr_trace_visibility, whose texels and counts the other GPU tests pin to the
oracle; here the fused call is compared with them bit for bit:
* every preset size (ragged and one-pixel-wide images included), with and
  without a previous camera, several frames;
* two-level (instanced) and device-built hierarchies;
* a batch longer than one launch holds, mixing sizes and hierarchy kinds;
* its texels against the oracle's on the small scene, as for dhr_gbuffer;
* mismatched jobs are refused; the counting variant writes the same bytes
  and counts one primary ray per pixel beyond the visibility rays;
* a context whose walks address records by 64-bit offsets (the path of
  trees beyond 2^26 nodes or triangles, forced by DHR_WIDE_RECORDS=1) writes
  the same bytes and counts the same work as the 32-bit one.
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


def buffers(B, W, H, n_lights):
    import torch
    g = B.gbuffer_tensors(W, H)
    g["ao"] = torch.full((W * H,), 0xAB, dtype=torch.uint8, device="cuda")
    g["sh"] = torch.full((max(n_lights, 1), W * H), 0xCD, dtype=torch.uint8, device="cuda")
    for k in ("pos", "nz", "dz", "mv"):
        g[k].fill_(float("nan"))
    return g


def separate(B, ctx, bvh, cur, prev, W, H, tp, n_lights):
    g = buffers(B, W, H, n_lights)
    B.dhr_gbuffer(ctx, bvh, cur, prev, W, H, g["pos"], g["nz"], g["dz"], g["mv"])
    B.dhr_trace_visibility(ctx, bvh, tp, g["pos"], g["nz"], g["ao"], g["sh"] if n_lights else None)
    return g


def fused(B, ctx, bvh, cur, prev, W, H, tp, n_lights):
    g = buffers(B, W, H, n_lights)
    B.dhr_gbuffer_trace(ctx, bvh, cur, prev, W, H, tp, g["pos"], g["nz"], g["dz"], g["mv"], g["ao"],
                        g["sh"] if n_lights else None)
    return g


def assert_same(a, b, what):
    import torch
    for k in ("pos", "nz", "dz", "mv"):
        assert torch.equal(a[k].view(torch.int32), b[k].view(torch.int32)), f"{what}: {k}"
    assert torch.equal(a["ao"], b["ao"]), f"{what}: ao counts"
    assert torch.equal(a["sh"], b["sh"]), f"{what}: shadow counts"


@pytest.mark.parametrize("preset", ["tiny", "ragged", "sliver", "room720", "terrain1080"])
def test_fused_equals_the_two_calls(B, ctx, preset):
    pr = wl.preset(preset)
    sc, _ = scene(pr.scene)
    bvh = B.dhr_build_bvh(ctx, sc.tris, sc.obj_id)
    cams = wl.camera_path(pr.camera, 3, sc)
    lights = wl.lights_for(pr.scene)
    for f in range(3):
        prev = cams[f - 1] if f else None
        tp = B.trace_params(pr.W, pr.H, frame=f, seed=pr.seed, n_ao=pr.n_ao, ao_radius=pr.ao_radius,
                            n_shadow=pr.n_shadow, lights=lights)
        a = separate(B, ctx, bvh, cams[f], prev, pr.W, pr.H, tp, len(lights))
        b = fused(B, ctx, bvh, cams[f], prev, pr.W, pr.H, tp, len(lights))
        assert_same(a, b, f"{preset} frame {f}")
    print(f"{preset}: fused texels and counts equal the two calls on 3 frames", flush=True)


def test_fused_texels_match_the_oracle(B, ctx):
    pr = wl.preset("tiny")
    sc, so = scene(pr.scene)
    bvh = B.dhr_build_bvh(ctx, sc.tris, sc.obj_id)
    cams = wl.camera_path(pr.camera, 2, sc)
    lights = wl.lights_for(pr.scene)
    tp = B.trace_params(pr.W, pr.H, frame=1, seed=pr.seed, n_ao=pr.n_ao, ao_radius=pr.ao_radius,
                        n_shadow=pr.n_shadow, lights=lights)
    g = fused(B, ctx, bvh, cams[1], cams[0], pr.W, pr.H, tp, len(lights))
    pos, nz, dz, mv = orc.gbuffer(so, cams[1], cams[0], pr.W, pr.H)
    gp = g["pos"].cpu().numpy()
    same = gp[:, 3].view(np.uint32) == orc.id_bits(pos)
    hit = same & (nz[:, 3] > 0)
    perr = np.abs(gp[:, :3] - pos[:, :3]).max(1) / (np.abs(pos[:, :3]).max(1) + 1.0)
    print(f"fused texels: ids differ at {(~same).sum()}, positions beyond 1e-4 at {(perr[hit] > 1e-4).sum()} "
          f"of {pr.W * pr.H} pixels", flush=True)
    assert (~same).mean() <= 1e-4 and (perr[hit] > 1e-4).mean() <= 1e-4


def _instanced(B, ctx):
    sc, _ = scene("spheres")
    ground, mesh = sc.tris[:2], sc.tris[2:482]
    xf = np.float32([[[1, 0, 0, 0], [0, 1, 0, 0], [0, 0, 1, 0]], [[0.5, 0, 0, 2.0], [0, 0.5, 0, 0.3], [0, 0, 0.5, -1.0]]])
    return B.dhr_build_bvh_instanced(ctx, ground, sc.obj_id[:2], mesh, xf, np.uint32([1, 9]))


def test_fused_two_level_and_device_built(B, ctx):
    import torch
    pr = wl.preset("tiny")
    sc, _ = scene(pr.scene)
    cams = wl.camera_path(pr.camera, 2, sc)
    lights = wl.lights_for(pr.scene)
    tp = B.trace_params(pr.W, pr.H, frame=1, seed=5, n_ao=4, ao_radius=1.0, n_shadow=2, lights=lights)
    dev = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to("cuda")
    dev_bvh = B.dhr_build_bvh_device(ctx, dev(np.asarray(sc.tris, np.float32).reshape(-1, 9)),
                                     dev(np.asarray(sc.obj_id, np.uint32).view(np.int32)))
    for what, bvh in (("two-level", _instanced(B, ctx)), ("device-built", dev_bvh)):
        a = separate(B, ctx, bvh, cams[1], cams[0], pr.W, pr.H, tp, len(lights))
        b = fused(B, ctx, bvh, cams[1], cams[0], pr.W, pr.H, tp, len(lights))
        assert_same(a, b, what)


def test_fused_batch_beyond_one_launch(B, ctx):
    pr = wl.preset("tiny")
    sc, _ = scene(pr.scene)
    flat = B.dhr_build_bvh(ctx, sc.tris, sc.obj_id)
    inst = _instanced(B, ctx)
    lights = wl.lights_for("spheres")
    sizes = [(64, 64), (48, 40), (33, 17), (64, 8), (1, 9)]
    n = 14
    cams = wl.camera_path(pr.camera, n + 1, sc)
    gj, tj, ref = [], [], []
    for k in range(n):
        W, H = sizes[k % len(sizes)]
        bvh = flat if k % 3 else inst
        tp = B.trace_params(W, H, frame=k, seed=3, n_ao=3, ao_radius=1.0, n_shadow=2, lights=lights)
        g = buffers(B, W, H, len(lights))
        gj.append(dict(bvh=bvh, cur=cams[k + 1], prev=cams[k], W=W, H=H, pos=g["pos"], nz=g["nz"], dz=g["dz"],
                       mv=g["mv"]))
        tj.append(dict(bvh=bvh, params=tp, pos=g["pos"], nz=g["nz"], ao_count=g["ao"], shadow_count=g["sh"]))
        ref.append((g, separate(B, ctx, bvh, cams[k + 1], cams[k], W, H, tp, len(lights))))
    B.dhr_gbuffer_trace_batch(ctx, gj, tj)
    for k, (g, r) in enumerate(ref):
        assert_same(g, r, f"batch job {k}")


def test_fused_rejects_mismatched_jobs_and_counters(B, ctx):
    import torch
    pr = wl.preset("tiny")
    sc, _ = scene(pr.scene)
    bvh = B.dhr_build_bvh(ctx, sc.tris, sc.obj_id)
    other = B.dhr_build_bvh(ctx, sc.tris, sc.obj_id)
    cam = wl.camera_path(pr.camera, 1, sc)[0]
    lights = wl.lights_for("spheres")
    W, H = 32, 16
    g = buffers(B, W, H, len(lights))
    gjob = dict(bvh=bvh, cur=cam, prev=None, W=W, H=H, pos=g["pos"], nz=g["nz"], dz=g["dz"], mv=g["mv"])
    tp = B.trace_params(W, H, n_ao=1, ao_radius=1.0, n_shadow=1, lights=lights)
    tjob = dict(bvh=bvh, params=tp, pos=g["pos"], nz=g["nz"], ao_count=g["ao"], shadow_count=g["sh"])
    B.dhr_gbuffer_trace_batch(ctx, [gjob], [tjob])
    h = buffers(B, W, H, len(lights))
    for bad in (dict(bvh=other), dict(pos=h["pos"]), dict(nz=h["nz"]),
                dict(params=B.trace_params(W + 1, H, n_ao=1, ao_radius=1.0, n_shadow=1, lights=lights))):
        with pytest.raises(B.DhrError):
            B.dhr_gbuffer_trace_batch(ctx, [gjob], [dict(tjob, **bad)])
    with pytest.raises(B.DhrError):
        B.dhr_gbuffer_trace(ctx, bvh, cam, None, W, H, B.trace_params(W, H - 1, n_ao=1, ao_radius=1.0, n_shadow=1,
                                                                       lights=lights),
                            g["pos"], g["nz"], g["dz"], g["mv"], g["ao"], g["sh"])
    with pytest.raises(ValueError):
        B.dhr_gbuffer_trace_batch(ctx, [gjob, gjob], [tjob])


def test_fused_counting_variant(B, ctx):
    import torch
    pr = wl.preset("tiny")
    sc, _ = scene(pr.scene)
    bvh = B.dhr_build_bvh(ctx, sc.tris, sc.obj_id)
    cams = wl.camera_path(pr.camera, 2, sc)
    lights = wl.lights_for(pr.scene)
    W, H = pr.W, pr.H
    tp = B.trace_params(W, H, frame=1, seed=pr.seed, n_ao=2, ao_radius=1.0, n_shadow=2, lights=lights)
    ref = fused(B, ctx, bvh, cams[1], cams[0], W, H, tp, len(lights))
    c_fused = torch.zeros(4, dtype=torch.int64, device="cuda")
    c_trace = torch.zeros(4, dtype=torch.int64, device="cuda")
    B.dhr_set_trace_counters(ctx, c_fused)
    try:
        g = fused(B, ctx, bvh, cams[1], cams[0], W, H, tp, len(lights))
        B.dhr_set_trace_counters(ctx, c_trace)
        B.dhr_trace_visibility(ctx, bvh, tp, g["pos"], g["nz"], g["ao"], g["sh"])
        with pytest.raises(B.DhrError):
            fused(B, ctx, _instanced(B, ctx), cams[1], cams[0], W, H, tp, len(lights))
    finally:
        B.dhr_set_trace_counters(ctx, None)
    assert_same(g, ref, "counting variant")
    cf, ct = c_fused.cpu().tolist(), c_trace.cpu().tolist()
    print(f"fused counts {cf}, visibility alone {ct}", flush=True)
    # one primary ray per pixel on top of the visibility rays; primary walks add node visits
    assert cf[0] == ct[0] + W * H
    assert cf[1] > ct[1] and cf[3] >= ct[3]


@pytest.fixture(scope="module")
def wide_ctx(B):
    import os
    os.environ["DHR_WIDE_RECORDS"] = "1"
    try:
        return B.dhr_create(0)
    finally:
        del os.environ["DHR_WIDE_RECORDS"]


@pytest.mark.parametrize("preset", ["tiny", "ragged", "room720", "terrain1080"])
def test_wide_record_addressing_gives_the_same_bytes(B, ctx, wide_ctx, preset):
    import torch
    pr = wl.preset(preset)
    sc, _ = scene(pr.scene)
    cams = wl.camera_path(pr.camera, 2, sc)
    lights = wl.lights_for(pr.scene)
    tp = B.trace_params(pr.W, pr.H, frame=1, seed=pr.seed, n_ao=pr.n_ao, ao_radius=pr.ao_radius,
                        n_shadow=pr.n_shadow, lights=lights)
    res, counts = [], []
    for c in (ctx, wide_ctx):
        bvh = B.dhr_build_bvh(c, sc.tris, sc.obj_id)
        a = separate(B, c, bvh, cams[1], cams[0], pr.W, pr.H, tp, len(lights))
        cnt = torch.zeros(4, dtype=torch.int64, device="cuda")
        B.dhr_set_trace_counters(c, cnt)
        try:
            b = fused(B, c, bvh, cams[1], cams[0], pr.W, pr.H, tp, len(lights))
        finally:
            B.dhr_set_trace_counters(c, None)
        assert_same(a, b, f"{preset}: fused against the two calls")
        res.append(b)
        counts.append(cnt.cpu().tolist())
    if preset == "tiny":
        dev = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to("cuda")
        for c in (ctx, wide_ctx):
            bvh = B.dhr_build_bvh_device(c, dev(np.asarray(sc.tris, np.float32).reshape(-1, 9)),
                                         dev(np.asarray(sc.obj_id, np.uint32).view(np.int32)))
            res.append(fused(B, c, bvh, cams[1], cams[0], pr.W, pr.H, tp, len(lights)))
        assert_same(res[2], res[3], "device-built tree, 32- and 64-bit record offsets")
    assert_same(res[0], res[1], f"{preset}: 32- and 64-bit record offsets")
    assert counts[0] == counts[1]
    print(f"{preset}: 64-bit record offsets give the same texels, counts and work {counts[0]}", flush=True)
