"""Consecutive frames overlapped on two streams (needs an MI355X).

FramePipeline runs the G-buffer + visibility launches of the next one to
three frames beside frame f's filter and beside each other (the schedule
bench.py times).  Over eight frames, in two runs (the second continuing the
first's history), the filtered output, both history buffers, every G-buffer
slot and the counts equal those of the same frames run one at a time, bit for
bit.
"""
import pytest

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


def _bits(t):
    import torch
    return t.view(torch.int32) if t.dtype == torch.float32 else t


@pytest.mark.parametrize("preset,depth", [("tiny", 1), ("ragged", 2), ("room720", 1), ("room720", 3),
                                          ("terrain1080", 1), ("terrain1080", 2)])
def test_overlapped_frames_equal_one_at_a_time(B, ctx, preset, depth):
    import torch
    from paper_2406_06963_amd.pipeline import FramePipeline
    pr = wl.preset(preset)
    sc, _ = scene(pr.scene)
    bvh = B.dhr_build_bvh(ctx, sc.tris, sc.obj_id)
    n = 8
    cams = wl.camera_path(pr.camera, n, sc)
    lights = wl.lights_for(pr.scene)
    tps = [B.trace_params(pr.W, pr.H, frame=f, seed=pr.seed, n_ao=pr.n_ao, ao_radius=pr.ao_radius,
                          n_shadow=pr.n_shadow, lights=lights) for f in range(n)]
    P = B.svgf_params(levels=pr.levels, alpha=pr.alpha)
    res = []
    for overlap in (False, True):
        pipe = FramePipeline(ctx, bvh, pr.W, pr.H, pr.n_ao, len(lights), P, frames_in_flight=depth)
        pipe.run(cams, tps, 0, 5, overlap=overlap)
        pipe.run(cams, tps, 5, n, overlap=overlap)
        torch.cuda.synchronize()
        res.append([pipe.out] + pipe.hist + [g[k] for g in pipe.gb for k in ("pos", "nz", "dz", "mv")]
                   + pipe.aos + pipe.shs)
    for k, (a, b) in enumerate(zip(*res)):
        assert torch.equal(_bits(a), _bits(b)), k
    print(f"{preset}, {depth} frame(s) in flight: {n} overlapped frames equal the frames run one at a time",
          flush=True)
