"""Serving scheduler on the CPU: a fake executor renders with the oracle on a
simulated clock, so admission, eviction, superseding, out-of-order and stale
drops, the one-frame-in-flight rule, latency accounting and the alone-vs-mix
invariance are checked without a GPU."""
import numpy as np
import pytest

import oracle as orc
from paper_2406_06963_amd import serve as sv
from paper_2406_06963_amd import workloads as wl


class Clock:
    def __init__(self):
        self.t = 0.0

    def __call__(self):
        return self.t


class OracleExecutor:
    """Renders a batch with the oracle at launch; it completes `latency` later."""

    def __init__(self, clock, latency=0.004):
        self.clock = clock
        self.latency = latency
        self.scenes = {}
        self.launches = []

    def n_lights(self, scene):
        return 1

    def _scene(self, name):
        if name not in self.scenes:
            sc = wl.make_scene(name)
            self.scenes[name] = (orc.Scene(sc.tris, sc.obj_id), wl.lights_for(name))
        return self.scenes[name]

    def alloc(self, spec):
        return {"prev": None, "hist": None, "out": None}

    def free(self, res):
        res.clear()

    def launch(self, items):
        self.launches.append([(spec.client_id, req.seq) for _, spec, req, _ in items])
        for res, spec, req, prev_cam in items:
            so, lights = self._scene(spec.scene)
            W, H = spec.W, spec.H
            has_prev = prev_cam is not None and res["prev"] is not None
            pos, nz, dz, mv = orc.gbuffer(so, req.camera, prev_cam if has_prev else None, W, H)
            P = orc.trace_params(W, H, frame=req.seq, client_id=spec.client_id, seed=5, n_ao=1, ao_radius=1.0,
                                 n_shadow=1, lights=lights)
            ao, _, _ = orc.trace(so, P, pos, nz)
            pix = np.float32(2 * np.tan(0.5 * req.camera.fov_y) / H)
            r = orc.svgf_filter(orc.svgf_params(), W, H, 1, ao, pos, nz, dz, mv,
                                res["prev"][0] if has_prev else None, res["prev"][1] if has_prev else None,
                                res["hist"] if has_prev else None, pix)
            res["pending"] = ((pos, nz), r["hist_out"].astype(np.float32), r["out"])
        return self.clock() + self.latency

    def done(self, token):
        return self.clock() >= token

    def wait(self, token):
        self.clock.t = max(self.clock.t, token)
        return True

    def commit(self, res):
        res["prev"], res["hist"], res["out"] = res.pop("pending")

    def output(self, res):
        return res["out"].copy()


def _req(cid, seq, t, delay=0.0, phase=0.0):
    cam = wl.camera_path("orbit", seq + 1, phase=phase)[seq]
    return sv.Request(cid, seq, cam, t, t + delay)


def test_admission_budget_and_eviction():
    clock = Clock()
    ex = OracleExecutor(clock)
    per = sv.resident_bytes(32, 32)
    server = sv.Server(ex, budget_bytes=2.5 * per, clock=clock, idle_evict_s=1.0)
    assert server.connect(sv.ClientSpec(0, 32, 32, "spheres"))
    assert server.connect(sv.ClientSpec(1, 32, 32, "spheres"))
    # no room and nobody idle long enough: rejected
    assert not server.connect(sv.ClientSpec(2, 32, 32, "spheres"))
    assert server.stats.rejected_clients == 1
    # client 1 stays active, client 0 goes idle: client 0 is evicted for client 2
    clock.t = 2.0
    server.clients[1].last_active = 1.9
    assert server.connect(sv.ClientSpec(2, 32, 32, "spheres"))
    assert 0 not in server.clients and 1 in server.clients and 2 in server.clients
    assert server.stats.evicted_clients == 1
    assert server.used <= server.budget


def test_drops_and_one_in_flight():
    clock = Clock()
    ex = OracleExecutor(clock, latency=0.010)
    server = sv.Server(ex, clock=clock, max_batch=8, max_inflight=2, max_stale_s=0.25)
    server.connect(sv.ClientSpec(0, 16, 16, "spheres"))
    # three requests delivered before the first tick: only the newest is served
    for s in range(3):
        server.offer(_req(0, s, 0.0))
    assert server.tick(0.001) == 1
    assert ex.launches[-1] == [(0, 2)]
    assert server.stats.dropped_superseded == 2
    # while frame 2 is in flight nothing else launches for this client
    server.offer(_req(0, 3, 0.002))
    assert server.tick(0.003) == 0
    clock.t = 0.012
    server.tick(clock.t)                      # retires frame 2, launches frame 3
    assert ex.launches[-1] == [(0, 3)]
    clock.t = 0.030
    server.tick(clock.t)
    # a late duplicate of an older frame is out of order
    server.offer(_req(0, 1, 0.0, delay=0.031))
    clock.t = 0.032
    server.tick(clock.t)
    assert server.stats.dropped_out_of_order == 1
    # a request sent 0.3 s ago is too stale
    server.offer(_req(0, 9, 0.0, delay=0.33))
    clock.t = 0.34
    server.tick(clock.t)
    assert server.stats.dropped_stale == 1
    assert server.stats.served == 2
    # latency = completion - delivery (frame 2 delivered at 0, retired at 0.012)
    assert abs(server.stats.latencies_ms[0] - 12.0) < 1e-9


def test_max_batch_and_fifo():
    clock = Clock()
    ex = OracleExecutor(clock)
    server = sv.Server(ex, clock=clock, max_batch=2, max_inflight=4)
    for c in range(3):
        server.connect(sv.ClientSpec(c, 8, 8, "spheres"))
    server.offer(_req(2, 0, 0.0, delay=0.001))
    server.offer(_req(0, 0, 0.0, delay=0.002))
    server.offer(_req(1, 0, 0.0, delay=0.003))
    assert server.tick(0.01) == 2
    assert ex.launches[-1] == [(2, 0), (0, 0)]      # earliest deliveries first
    assert server.tick(0.01) == 1
    assert ex.launches[-1] == [(1, 0)]


def test_alone_equals_mix_on_the_oracle_backend():
    specs = [sv.ClientSpec(0, 24, 16, "spheres"), sv.ClientSpec(1, 16, 16, "spheres"), sv.ClientSpec(2, 20, 12, "room")]
    reqs = sv.request_trace(specs, duration_s=0.25, rate_hz=30.0)

    def serve(specs_, reqs_, max_batch, sequential=False):
        clock = Clock()
        ex = OracleExecutor(clock, latency=0.012)
        server = sv.Server(ex, clock=clock, max_batch=max_batch, keep_outputs=True)
        for sp in specs_:
            server.connect(sp)
        for r in sorted(reqs_, key=lambda r: r.deliver_t):
            clock.t = max(clock.t, r.deliver_t)
            server.offer(r)
            server.tick(clock.t)
            if sequential:
                server.drain()
        while server.inflight or any(c.pending for c in server.clients.values()):
            clock.t += 0.004
            server.tick(clock.t)
        return server

    mix = serve(specs, reqs, 8)
    assert mix.stats.served > 6
    for sp in specs:
        st = mix.clients[sp.client_id]
        served = [s for s, _ in st.served]
        alone_reqs = [r for r in reqs if r.client_id == sp.client_id and r.seq in served]
        alone = serve([sp], [sv.Request(r.client_id, r.seq, r.camera, r.send_t, r.send_t) for r in alone_reqs], 1,
                      sequential=True)
        a = alone.clients[sp.client_id].served
        assert [s for s, _ in a] == served
        for (s1, o1), (s2, o2) in zip(st.served, a):
            assert np.array_equal(o1, o2), (sp.client_id, s1)
