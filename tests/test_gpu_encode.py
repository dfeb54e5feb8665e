"""GPU parity of the wire form (needs an MI355X): quantised AO bytes and the
per-light visibility bits equal the oracle's bit for bit, including values
outside [0, 1], NaN, code boundaries and a length that is not a multiple of
the four pixels a lane handles."""
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


def test_quantize_bitexact(B, ctx):
    import torch
    rng = np.random.default_rng(11)
    k = np.arange(256)
    edges = np.concatenate([(k + 0.5) / 255.0, k / 255.0]).astype(np.float32)
    x = np.concatenate([rng.random(1_000_003).astype(np.float32), edges, np.nextafter(edges, 2.0),
                        np.nextafter(edges, -1.0), np.array([-1, -0.0, np.nan, 1.5, np.inf, -np.inf], np.float32)])
    q = torch.empty(x.size, dtype=torch.uint8, device="cuda")
    B.dhr_encode_frame(ctx, value=torch.from_numpy(x).cuda(), q=q)
    assert np.array_equal(q.cpu().numpy(), orc.quantize_u8(x))
    # an unaligned start (the scalar path) gives the same bytes
    q2 = torch.empty(x.size - 1, dtype=torch.uint8, device="cuda")
    B.dhr_encode_frame(ctx, value=torch.from_numpy(x).cuda()[1:], q=q2)
    assert np.array_equal(q2.cpu().numpy(), orc.quantize_u8(x[1:]))


@pytest.mark.parametrize("n_lights,n_shadow", [(1, 1), (3, 1), (2, 4), (8, 3)])
def test_light_mask_bitexact(B, ctx, n_lights, n_shadow):
    import torch
    rng = np.random.default_rng(n_lights * 10 + n_shadow)
    n = 100_001
    sc = rng.integers(0, n_shadow + 1, size=(n_lights, n)).astype(np.uint8)
    m = torch.empty(n, dtype=torch.uint8, device="cuda")
    B.dhr_encode_frame(ctx, shadow_count=torch.from_numpy(sc).cuda(), n_shadow=n_shadow, mask=m)
    assert np.array_equal(m.cpu().numpy(), orc.light_mask(sc, n_shadow))


def test_encode_served_frame(B, ctx):
    """The oracle's filtered AO and shadow counts of a workload frame."""
    import torch
    pr, fr = frames("room720", 1)
    f = fr[0]
    ref = orc.svgf_filter(orc.svgf_params(), pr.W, pr.H, pr.n_ao, f["ao"], f["pos"], f["nz"], f["dz"], f["mv"],
                          None, None, None, f["pix"])
    ao = ref["out"].astype(np.float32)
    HW = pr.W * pr.H
    q = torch.empty(HW, dtype=torch.uint8, device="cuda")
    m = torch.empty(HW, dtype=torch.uint8, device="cuda")
    B.dhr_encode_frame(ctx, value=torch.from_numpy(ao).cuda(), q=q, shadow_count=torch.from_numpy(f["sh"]).cuda(),
                       n_shadow=pr.n_shadow, mask=m)
    assert np.array_equal(q.cpu().numpy(), orc.quantize_u8(ao))
    assert np.array_equal(m.cpu().numpy(), orc.light_mask(f["sh"], pr.n_shadow))


def test_encode_invalid_arguments(B, ctx):
    import torch
    sc = torch.zeros(9, 16, dtype=torch.uint8, device="cuda")
    m = torch.empty(16, dtype=torch.uint8, device="cuda")
    with pytest.raises(B.DhrError):
        B.dhr_encode_frame(ctx, shadow_count=sc, n_shadow=1, mask=m)        # 9 lights
    with pytest.raises(B.DhrError):
        B.dhr_encode_frame(ctx, shadow_count=sc[:2], n_shadow=0, mask=m)    # no rays
