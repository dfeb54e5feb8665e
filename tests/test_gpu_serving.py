"""Serving on the GPU: every client's outputs in the continuously batched mix
equal its outputs alone (bitwise), and the served frames stay accurate."""
import numpy as np
import pytest

from paper_2406_06963_amd import serve as sv
from paper_2406_06963_amd import workloads as wl

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def setup():
    import torch
    assert torch.cuda.is_available(), "GPU test run without a GPU"
    from paper_2406_06963_amd import binding as B
    ctx = B.dhr_create(0)
    scenes = {}
    for name, r in (("spheres", 1.0), ("room", 0.5)):
        sc = wl.make_scene(name)
        scenes[name] = {"bvh": B.dhr_build_bvh(ctx, sc.tris, sc.obj_id), "lights": wl.lights_for(name),
                        "ao_radius": r}
    return B, ctx, scenes


def test_alone_equals_mix(setup):
    B, ctx, scenes = setup
    # 24 clients at reduced resolutions so every output can be kept for comparison
    specs = []
    rng = np.random.default_rng(3)
    for i in range(24):
        W, H = [(160, 90), (320, 180), (480, 270)][int(rng.integers(0, 3))]
        specs.append(sv.ClientSpec(i, W, H, ["spheres", "room"][int(rng.integers(0, 2))]))
    reqs = sv.request_trace(specs, duration_s=0.5, rate_hz=30.0)
    ex = sv.GpuExecutor(ctx, scenes, n_streams=3)
    server = sv.Server(ex, max_batch=12, max_inflight=3, keep_outputs=True, max_stale_s=10.0)
    for sp in specs:
        assert server.connect(sp)
    # virtual time in 25 ms windows: every client with a delivered request joins
    # the window's batches, so batches mix clients, scenes and resolutions
    i = 0
    for k in range(1, 40):
        t = 0.025 * k
        while i < len(reqs) and reqs[i].deliver_t <= t:
            server.offer(reqs[i])
            i += 1
        while server.tick(t):
            pass
        server.drain()
    st = server.stats.summary(1.0)
    print("mix:", st, flush=True)
    assert st["served"] >= 48 and st["mean_batch"] > 2.0
    checked = 0
    for sp in specs[:8]:
        mine = server.clients[sp.client_id].served
        seqs = [s for s, _ in mine]
        alone_ex = sv.GpuExecutor(ctx, scenes, n_streams=1)
        alone = sv.Server(alone_ex, max_batch=1, max_inflight=1, keep_outputs=True, max_stale_s=1e9)
        alone.connect(sp)
        for r in reqs:
            if r.client_id == sp.client_id and r.seq in seqs:
                alone.offer(sv.Request(r.client_id, r.seq, r.camera, 0.0, 0.0))
                alone.tick()
                alone.drain()
        a = alone.clients[sp.client_id].served
        assert [s for s, _ in a] == seqs
        for (s1, o1), (s2, o2) in zip(mine, a):
            import torch
            assert torch.equal(o1, o2), (sp.client_id, s1)
            checked += 1
    assert checked > 8
