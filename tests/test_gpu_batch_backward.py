"""GPU parity of the adjoint on batches of frames (needs an MI355X).

The differentiation workload is a batch of 16 frames at 1280 x 720 of the
room scene whose 15 per-level edge-stopping parameters are shared by every
frame, so their gradient is the sum over frames of each frame's gradient.
These tests run the spatial stack forward and its adjoint on such batches in
one call each and compare every frame with the oracle:

* 16 room frames at 1280 x 720 (one backward call): each frame's gradient
  with respect to (c, var) within rel 1e-3 of the oracle's FP64
  vector-Jacobian product of that frame, and the sigma gradient within rel
  1e-3 (absolute floor 1e-8) of the sum of the oracle's per-frame sigma
  gradients; the autograd binding gives the same numbers;
* 30 frames, beyond the 24 frames one launch holds, so the sigma gradient of
  the later chunk is accumulated onto the first: the same comparisons.

(c, var) of every frame is the oracle's variance-pass output of a
teacher-forced frame sequence, jittered off the kinks of the stack (ties of
|c_p - c_q| and zero variance under the prefilter's square root).
"""
import os
from concurrent.futures import ThreadPoolExecutor

import numpy as np
import pytest

import oracle as orc
from oracle_inputs import frames

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


def _batch_inputs(preset, F, seed):
    """Per frame: (c, var) of the oracle's teacher-forced variance pass,
    jittered, and the frame's geometry; plus a random loss gradient."""
    pr, fr = frames(preset, F)
    Po = orc.svgf_params()
    rng = np.random.default_rng(seed)
    hist, out = None, []
    for k, f in enumerate(fr):
        prev = fr[k - 1] if k else None
        ref = orc.svgf_filter(Po, pr.W, pr.H, pr.n_ao, f["ao"], f["pos"], f["nz"], f["dz"], f["mv"],
                              prev["pos"] if prev else None, prev["nz"] if prev else None, hist, f["pix"])
        hist = ref["hist_out"].astype(np.float32)
        cv = ref["cv0"].copy()
        cv[:, 0] += rng.uniform(-0.02, 0.02, cv.shape[0])
        cv[:, 1] += rng.uniform(2e-4, 2e-3, cv.shape[0])
        go = rng.normal(size=pr.W * pr.H).astype(np.float32)
        out.append(dict(cv=cv.astype(np.float32), nz=f["nz"], dz=f["dz"], go=go))
    return pr, out


def _oracle_vjps(Po, W, H, items):
    """The oracle's VJP of each frame, frames side by side on the host cores
    (one OpenMP thread per frame; the foreign calls release the GIL)."""
    def one(it):
        orc.set_num_threads(1)
        return orc.svgf_spatial_vjp(Po, W, H, it["cv"].astype(np.float64), it["nz"], it["dz"],
                                    it["go"].astype(np.float64))
    workers = max(1, min(len(items), 16, os.cpu_count() or 1))
    with ThreadPoolExecutor(workers) as ex:
        return list(ex.map(one, items))


def _check(preset, F, gcv_all, gs, items, W, H, Po):
    refs = _oracle_vjps(Po, W, H, items)
    gs_ref = np.zeros_like(refs[0][1])
    worst = 0.0
    for k, (gcv_o, gs_o) in enumerate(refs):
        gs_ref += gs_o
        for c in range(2):
            rel = np.linalg.norm(gcv_all[k][:, c] - gcv_o[:, c]) / np.linalg.norm(gcv_o[:, c])
            worst = max(worst, rel)
            assert rel <= 1e-3, (preset, k, c, rel)
    err = np.abs(gs - gs_ref)
    print(f"{preset} x {F}: worst per-frame grad rel err {worst:.2e}; sigma grads gpu {gs.ravel()} "
          f"oracle sum {gs_ref.ravel()}; worst rel {(err / (np.abs(gs_ref) + 1e-8)).max():.2e}", flush=True)
    assert (err <= 1e-3 * np.abs(gs_ref) + 1e-8).all(), err / (np.abs(gs_ref) + 1e-8)


def _gpu_batch(B, ctx, P, W, H, items):
    import torch
    F, L, HW = len(items), P.levels, W * H
    cv = dev(np.stack([it["cv"] for it in items]))
    nz = dev(np.stack([it["nz"] for it in items]))
    dz = dev(np.stack([it["dz"] for it in items]))
    go = dev(np.stack([it["go"] for it in items]))
    out = torch.empty(F, HW, device="cuda")
    save = torch.empty(F, L, HW, 2, device="cuda")
    nbf = (B.dhr_svgf_workspace_bytes(W, H, P, 0) + 15) // 16 * 4
    fwork = torch.empty(F, nbf, device="cuda")
    B.dhr_svgf_spatial_forward(ctx, P, [B.spatial_frame(W, H, cv[k], nz[k], dz[k], out[k], save=save[k],
                                                        work=fwork[k]) for k in range(F)])
    nbb = (B.dhr_svgf_workspace_bytes(W, H, P, 1) + 15) // 16 * 4
    work = torch.empty(F, nbb, device="cuda")
    gcv = torch.empty(F, HW, 2, device="cuda")
    gs = torch.full((3 * L,), float("nan"), device="cuda")
    B.dhr_svgf_backward(ctx, P, [B.bwd_frame(W, H, save[k], nz[k], dz[k], go[k], gcv[k], work[k])
                                 for k in range(F)], gs)
    torch.cuda.synchronize()
    return cv, nz, dz, go, out, gcv.cpu().numpy(), gs.cpu().numpy().reshape(3, L)


@pytest.mark.timeout(900)
def test_backward_16_frames_720p(B, ctx):
    import torch

    from paper_2406_06963_amd.autograd import svgf_stack
    print("case: room720 x 16, one forward and one backward call", flush=True)
    pr, items = _batch_inputs("room720", 16, 77)
    W, H = pr.W, pr.H
    P, Po = B.svgf_params(), orc.svgf_params()
    cv, nz, dz, go, out, gcv, gs = _gpu_batch(B, ctx, P, W, H, items)
    # forward of a few frames against the oracle's spatial stack
    for k in (0, 7, 15):
        ref = orc.svgf_spatial(Po, W, H, items[k]["cv"].astype(np.float64), items[k]["nz"], items[k]["dz"])
        assert np.abs(out[k].cpu().numpy() - ref).max() <= 1e-4, k
    _check("room720", 16, gcv, gs, items, W, H, Po)
    # the autograd binding runs the same kernels on the same batch
    c = cv[..., 0].clone().requires_grad_(True)
    v = cv[..., 1].clone().requires_grad_(True)
    sz = torch.full((5,), 1.0, device="cuda", requires_grad=True)
    sn = torch.full((5,), 128.0, device="cuda", requires_grad=True)
    sl = torch.full((5,), 4.0, device="cuda", requires_grad=True)
    o2 = svgf_stack(c, v, nz, dz, sz, sn, sl, ctx, P, W, H)
    assert torch.equal(o2, out)
    (o2 * go).sum().backward()
    assert np.array_equal(c.grad.cpu().numpy(), gcv[..., 0])
    assert np.array_equal(v.grad.cpu().numpy(), gcv[..., 1])
    for fam, t in enumerate((sz, sn, sl)):
        assert np.array_equal(t.grad.cpu().numpy(), gs[fam]), fam


@pytest.mark.timeout(600)
def test_backward_30_frames_crosses_the_launch_chunk(B, ctx):
    print("case: tiny x 30 (two launch chunks), one backward call", flush=True)
    pr, items = _batch_inputs("tiny", 30, 78)
    W, H = pr.W, pr.H
    sz = np.float32([0.8, 1.3, 1.0, 1.7, 0.6])
    sn = np.float32([64, 100, 128, 40, 90])
    sl = np.float32([3, 5, 4, 7, 2.5])
    P = B.svgf_params(sigma_z=sz, sigma_n=sn, sigma_l=sl)
    Po = orc.svgf_params(sigma_z=sz, sigma_n=sn, sigma_l=sl)
    *_, gcv, gs = _gpu_batch(B, ctx, P, W, H, items)
    _check("tiny", 30, gcv, gs, items, W, H, Po)
    # the two chunks called separately add up to the one call
    *_, gcv_a, gs_a = _gpu_batch(B, ctx, P, W, H, items[:24])
    *_, gcv_b, gs_b = _gpu_batch(B, ctx, P, W, H, items[24:])
    assert np.array_equal(np.concatenate([gcv_a, gcv_b]), gcv)
    np.testing.assert_allclose(gs_a.astype(np.float64) + gs_b, gs, rtol=2e-6, atol=1e-10)
