"""Edge cases of the tilings on the GPU (needs an MI355X): frames whose sides
are multiples of no tile (141 x 77, and a 5 x 131 sliver narrower than one
tile), odd and even ray counts (the packed and the per-lane ray layouts),
every level count of the filter and the adjoint, against the oracle."""
import numpy as np
import pytest

import oracle as orc
from oracle_inputs import frames, popcount64, scene

pytestmark = pytest.mark.gpu

ATOL = 1e-4


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


@pytest.mark.parametrize("preset", ["ragged", "sliver"])
def test_gbuffer_ids_ragged(B, ctx, preset):
    pr, fr = frames(preset, 2)
    sc, _ = scene(pr.scene)
    bvh = B.dhr_build_bvh(ctx, sc.tris, sc.obj_id)
    g = B.gbuffer_tensors(pr.W, pr.H)
    B.dhr_gbuffer(ctx, bvh, fr[1]["cam"], fr[0]["cam"], pr.W, pr.H, g["pos"], g["nz"], g["dz"], g["mv"])
    ids = g["pos"].cpu().numpy()[:, 3].view(np.uint32)
    assert (ids != orc.id_bits(fr[1]["pos"])).sum() <= 1


@pytest.mark.parametrize("preset,n_ao,n_shadow", [("ragged", 3, 2), ("ragged", 4, 6), ("ragged", 2, 1),
                                                  ("sliver", 1, 4), ("sliver", 8, 3)])
def test_visibility_ragged(B, ctx, preset, n_ao, n_shadow):
    import torch
    pr, fr = frames(preset, 2)
    sc, so = scene(pr.scene)
    bvh = B.dhr_build_bvh(ctx, sc.tris, sc.obj_id)
    bad = rays = 0
    for f in fr:
        kw = dict(f["trace_kw"], n_ao=n_ao, n_shadow=n_shadow)
        L, HW = len(kw["lights"]), pr.W * pr.H
        ao = torch.empty(HW, dtype=torch.uint8, device="cuda")
        sh = torch.empty(L, HW, dtype=torch.uint8, device="cuda")
        rb = torch.empty(1 + L, HW, dtype=torch.int64, device="cuda")
        B.dhr_trace_visibility(ctx, bvh, B.trace_params(pr.W, pr.H, **kw), dev(f["pos"]), dev(f["nz"]), ao, sh, rb)
        bits = rb.cpu().numpy().view(np.uint64)
        ao_o, sh_o, bits_o = orc.trace(so, orc.trace_params(pr.W, pr.H, **kw), f["pos"], f["nz"], ray_bits=True)
        bad += popcount64(bits ^ bits_o)
        rays += int((f["nz"][:, 3] > 0).sum()) * (n_ao + L * n_shadow)
        # the counts are the popcounts of the bits, stream by stream
        for st, cnt in enumerate([ao.cpu().numpy()] + list(sh.cpu().numpy())):
            assert np.array_equal(cnt, np.unpackbits(bits[st].view(np.uint8).reshape(-1, 8), axis=1).sum(1))
    print(f"{preset} ao {n_ao} shadow {n_shadow}: {bad} of {rays} rays differ", flush=True)
    assert bad <= max(1, 1e-4 * rays)


@pytest.mark.parametrize("preset", ["ragged", "sliver"])
def test_filter_ragged(B, ctx, preset):
    import torch
    pr, fr = frames(preset, 3)
    P, Po = B.svgf_params(), orc.svgf_params()
    W, H, HW = pr.W, pr.H, pr.W * pr.H
    hist_in = None
    for k, f in enumerate(fr):
        prev = fr[k - 1] if k else None
        ref = orc.svgf_filter(Po, W, H, pr.n_ao, f["ao"], f["pos"], f["nz"], f["dz"], f["mv"],
                              prev["pos"] if prev else None, prev["nz"] if prev else None, hist_in, f["pix"])
        hist = torch.empty(HW, 4, device="cuda")
        out = torch.empty(HW, device="cuda")
        work = torch.empty(B.dhr_svgf_workspace_bytes(W, H, P, 0) // 4, device="cuda")
        fr_ = B.svgf_frame(W, H, pr.n_ao, dev(f["ao"]), dev(f["pos"]), dev(f["nz"]), dev(f["dz"]), dev(f["mv"]),
                           dev(prev["pos"]) if prev else None, dev(prev["nz"]) if prev else None,
                           dev(hist_in) if hist_in is not None else None, hist, out, float(f["pix"]), work=work)
        B.dhr_svgf_filter(ctx, P, [fr_])
        err = np.abs(out.cpu().numpy() - ref["out"]).max()
        assert err <= ATOL, (k, err)
        hist_in = ref["hist_out"].astype(np.float32)


@pytest.mark.parametrize("preset,levels", [("ragged", 5), ("ragged", 8), ("sliver", 5), ("sliver", 7)])
def test_spatial_and_adjoint_ragged(B, ctx, preset, levels):
    import torch
    pr, fr = frames(preset, 1)
    f = fr[0]
    W, H, HW = pr.W, pr.H, pr.W * pr.H
    Po = orc.svgf_params(levels=levels)
    P = B.svgf_params(levels=levels)
    ref = orc.svgf_filter(Po, W, H, pr.n_ao, f["ao"], f["pos"], f["nz"], f["dz"], f["mv"], None, None, None,
                          f["pix"])
    rng = np.random.default_rng(21)
    cv = ref["cv0"].copy()
    cv[:, 0] += rng.uniform(-0.02, 0.02, HW)
    cv[:, 1] += rng.uniform(2e-4, 2e-3, HW)
    cv = cv.astype(np.float32)
    out = torch.empty(HW, device="cuda")
    save = torch.empty(levels, HW, 2, device="cuda")
    work = torch.empty(B.dhr_svgf_workspace_bytes(W, H, P, 0) // 4, device="cuda")
    B.dhr_svgf_spatial_forward(ctx, P, [B.spatial_frame(W, H, dev(cv), dev(f["nz"]), dev(f["dz"]), out, save=save,
                                                        work=work)])
    out_o = orc.svgf_spatial(Po, W, H, cv.astype(np.float64), f["nz"], f["dz"])
    assert np.abs(out.cpu().numpy() - out_o).max() <= ATOL
    go = rng.normal(size=HW).astype(np.float32)
    bwork = torch.empty(B.dhr_svgf_workspace_bytes(W, H, P, 1) // 4, device="cuda")
    gcv = torch.empty(HW, 2, device="cuda")
    gs = torch.empty(3 * levels, device="cuda")
    B.dhr_svgf_backward(ctx, P, [B.bwd_frame(W, H, save, dev(f["nz"]), dev(f["dz"]), dev(go), gcv, bwork)], gs)
    gcv_o, gs_o = orc.svgf_spatial_vjp(Po, W, H, cv.astype(np.float64), f["nz"], f["dz"], go.astype(np.float64))
    g = gcv.cpu().numpy()
    for c in range(2):
        rel = np.linalg.norm(g[:, c] - gcv_o[:, c]) / np.linalg.norm(gcv_o[:, c])
        print(f"{preset} L={levels}: grad component {c} rel err {rel:.2e}", flush=True)
        assert rel <= 1e-3
    gs = gs.cpu().numpy().reshape(3, levels)
    assert (np.abs(gs - gs_o) <= 1e-3 * np.abs(gs_o) + 1e-6).all(), (gs, gs_o)


def test_empty_batches(B, ctx):
    """Zero frames: the filter and the spatial forward launch nothing and
    succeed; the adjoint's sigma gradient is the empty sum, zero."""
    import torch
    P = B.svgf_params()
    B.dhr_svgf_filter(ctx, P, [])
    B.dhr_svgf_spatial_forward(ctx, P, [])
    gs = torch.full((3 * P.levels,), 7.0, device="cuda")
    B.dhr_svgf_backward(ctx, P, [], gs)
    torch.cuda.synchronize()
    assert bool((gs == 0.0).all())
