"""dhr_svgf_filter_noalloc (the filter with the library's own scratch, for
callers that cannot allocate) against dhr_svgf_filter with a caller-owned
workspace: identical outputs, histories and saved levels on two calls in a
row, the second with a smaller batch; frames beyond the scratch are refused
before anything is launched.  Needs an MI355X."""
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
    return None if a is None else torch.from_numpy(np.ascontiguousarray(a)).to("cuda")


def _inputs(preset, k):
    """Frame k of a workload with the oracle's history of frame k - 1."""
    pr, fr = frames(preset, k + 1)
    f, prev = fr[k], fr[k - 1]
    ref = orc.svgf_filter(orc.svgf_params(), pr.W, pr.H, pr.n_ao, prev["ao"], prev["pos"], prev["nz"], prev["dz"],
                          prev["mv"], None, None, None, prev["pix"])
    t = [dev(a) for a in (f["ao"], f["pos"], f["nz"], f["dz"], f["mv"], prev["pos"], prev["nz"],
                          ref["hist_out"].astype(np.float32))]
    return pr, f, t


def _run(B, ctx, P, cases, noalloc):
    import torch
    outs, keep = [], []
    frs = []
    for pr, f, t in cases:
        W, H = pr.W, pr.H
        hist = torch.full((W * H, 4), float("nan"), device="cuda")
        out = torch.full((W * H,), float("nan"), device="cuda")
        save = torch.full((P.levels, W * H, 2), float("nan"), device="cuda")
        work = None if noalloc else torch.empty(B.dhr_svgf_workspace_bytes(W, H, P, 0) // 4, device="cuda")
        frs.append(B.svgf_frame(W, H, pr.n_ao, *t, hist, out, float(f["pix"]), save=save, work=work))
        outs.append((hist, out, save))
        keep.append(work)
    (B.dhr_svgf_filter_noalloc if noalloc else B.dhr_svgf_filter)(ctx, P, frs)
    torch.cuda.synchronize()
    return [tuple(x.cpu().numpy() for x in o) for o in outs]


def _same(a, b):
    for (h1, o1, s1), (h2, o2, s2) in zip(a, b):
        assert np.array_equal(h1, h2) and np.array_equal(o1, o2) and np.array_equal(s1, s2)


def test_noalloc_equals_the_workspace_call(B, ctx):
    P = B.svgf_params()
    print("case: room720 frame 1 + tiny frame 2 (one batch), then tiny frame 1 alone", flush=True)
    big = [_inputs("room720", 1), _inputs("tiny", 2)]
    small = [_inputs("tiny", 1)]
    ref_big = _run(B, ctx, P, big, noalloc=False)
    ref_small = _run(B, ctx, P, small, noalloc=False)
    _same(_run(B, ctx, P, big, noalloc=True), ref_big)
    # the second call, smaller, reuses the scratch the first one left behind
    _same(_run(B, ctx, P, small, noalloc=True), ref_small)
    # and the lighter kernel form through the same scratch
    P3 = B.svgf_params(levels=1, kernel_width=3)
    _same(_run(B, ctx, P3, small, noalloc=True), _run(B, ctx, P3, small, noalloc=False))


def test_noalloc_refuses_what_does_not_fit(B, ctx):
    import torch
    P = B.svgf_params()
    W, H = 1920, 1080
    need = 2 * ((B.dhr_svgf_workspace_bytes(W, H, P, 0) + 255) // 256 * 256)
    assert need > B.SVGF_NOALLOC_SCRATCH_BYTES
    HW = W * H
    f4 = lambda: torch.zeros(HW, 4, device="cuda")
    f2 = lambda: torch.zeros(HW, 2, device="cuda")
    outs = []
    frs = []
    for _ in range(2):
        out = torch.full((HW,), 5.0, device="cuda")
        t = [torch.zeros(HW, dtype=torch.uint8, device="cuda"), f4(), f4(), f2(), f2(), f4()]
        frs.append((B.svgf_frame(W, H, 1, *t[:5], None, None, None, t[5], out, 1e-3), t))
        outs.append(out)
    with pytest.raises(B.DhrError, match="scratch"):
        B.dhr_svgf_filter_noalloc(ctx, P, [f for f, _ in frs])
    # a frame that brings its own work buffer is refused too
    w = torch.empty(B.dhr_svgf_workspace_bytes(W, H, P, 0) // 4, device="cuda")
    t = frs[0][1]
    with pytest.raises(B.DhrError, match="work must be NULL"):
        B.dhr_svgf_filter_noalloc(ctx, P, [B.svgf_frame(W, H, 1, *t[:5], None, None, None, t[5], outs[0], 1e-3,
                                                        work=w)])
    torch.cuda.synchronize()
    assert all(bool((o == 5.0).all()) for o in outs)
