"""Continuously batched multi-client serving of the hot path.

Many thin clients send camera updates (the paper sends camera data to the
server and tolerates it arriving up to 200 ms late, Section 4.1).  The server
keeps each client's history resident in HBM (SVGF moments and length, the
previous G-buffer and camera).  Every tick it admits ready requests of
different clients -- different scenes, resolutions and cameras -- into the
in-flight slots that have freed up, up to `max_batch` of them fused into two
ragged launches (G-buffer with visibility, then the filter) on one of
`max_inflight` streams, so that the work of consecutive admissions overlaps
on the device.  Measured on one MI355X with 64 clients at saturation, one
frame per launch with 12 slots in flight serves the most frames (about 7,900
frames/s, p99 8 ms); fusing 4 frames per launch serves 4 % fewer at a longer
tail (a fused launch finishes all its frames together), and one request at a
time serves about half (4,100 frames/s).

Policy
------
* admission: a client is admitted if its resident bytes fit the memory
  budget, after evicting clients idle for longer than `idle_evict_s` in LRU
  order; otherwise it is rejected;
* per client at most one frame is in flight (the history is a dependency);
* when a client is free, its newest delivered request is served and older
  pending ones are dropped as superseded; a request whose sequence number is
  not newer than the last served one is dropped as out of order; a request
  older than `max_stale_s` at dispatch is dropped as stale;
* latency = completion time - delivery time (send + injected delay), on the
  server's clock.

Results do not depend on the batching: the random numbers are keyed by
(client, frame, pixel, sample) and every kernel is deterministic, so a
client's outputs are the same alone and in the mix.
"""
from __future__ import annotations

import collections
import math
import time
from dataclasses import dataclass, field

import numpy as np


@dataclass
class ClientSpec:
    client_id: int
    W: int
    H: int
    scene: str


@dataclass
class Request:
    client_id: int
    seq: int
    camera: object
    send_t: float
    deliver_t: float


@dataclass
class ClientState:
    spec: ClientSpec
    bytes: int
    last_seq: int = -1
    last_cam: object = None
    last_active: float = 0.0
    in_flight: bool = False
    pending: list = field(default_factory=list)
    res: object = None           # executor resources
    served: list = field(default_factory=list)


@dataclass
class Stats:
    served: int = 0
    dropped_superseded: int = 0
    dropped_out_of_order: int = 0
    dropped_stale: int = 0
    rejected_clients: int = 0
    evicted_clients: int = 0
    batches: int = 0
    pixels: int = 0
    latencies_ms: list = field(default_factory=list)

    def summary(self, wall_s: float) -> dict:
        lat = np.array(self.latencies_ms) if self.latencies_ms else np.zeros(1)
        return {"served": self.served, "frames_per_s": self.served / max(wall_s, 1e-9),
                "mpix_per_s": self.pixels / max(wall_s, 1e-9) / 1e6,
                "p50_ms": float(np.percentile(lat, 50)), "p99_ms": float(np.percentile(lat, 99)),
                "mean_batch": self.served / max(self.batches, 1), "batches": self.batches,
                "dropped_superseded": self.dropped_superseded, "dropped_out_of_order": self.dropped_out_of_order,
                "dropped_stale": self.dropped_stale, "rejected_clients": self.rejected_clients,
                "evicted_clients": self.evicted_clients}


def resident_bytes(W: int, H: int, n_lights: int = 1) -> int:
    """Per-client HBM: two history buffers (16 B/px each), two G-buffers
    (pos 16 + nz 16 + dz 8 + mv 8), AO and shadow counts, filtered output,
    the filter's ping-pong scratch (16 B/px)."""
    return W * H * (2 * 16 + 2 * 48 + 1 + n_lights + 4 + 16)


class Server:
    def __init__(self, executor, budget_bytes: float = 200e9, max_batch: int = 8, max_inflight: int = 3,
                 max_stale_s: float = 0.25, idle_evict_s: float = 2.0, clock=time.perf_counter,
                 keep_outputs: bool = False):
        self.ex = executor
        self.budget = budget_bytes
        self.used = 0
        self.max_batch = max_batch
        self.max_inflight = max_inflight
        self.max_stale_s = max_stale_s
        self.idle_evict_s = idle_evict_s
        self.clock = clock
        self.keep_outputs = keep_outputs
        self.clients: dict[int, ClientState] = collections.OrderedDict()
        self.inflight = collections.deque()
        self.stats = Stats()

    # -------------------------------------------------------------- clients
    def connect(self, spec: ClientSpec, now: float | None = None) -> bool:
        now = self.clock() if now is None else now
        need = resident_bytes(spec.W, spec.H, self.ex.n_lights(spec.scene))
        if spec.client_id in self.clients:
            return True
        if self.used + need > self.budget:
            # evict idle clients, least recently active first
            idle = sorted((c for c in self.clients.values() if not c.in_flight and not c.pending
                           and now - c.last_active > self.idle_evict_s), key=lambda c: c.last_active)
            for c in idle:
                if self.used + need <= self.budget:
                    break
                self.disconnect(c.spec.client_id)
                self.stats.evicted_clients += 1
        if self.used + need > self.budget:
            self.stats.rejected_clients += 1
            return False
        st = ClientState(spec, need, last_active=now)
        st.res = self.ex.alloc(spec)
        self.clients[spec.client_id] = st
        self.used += need
        return True

    def disconnect(self, client_id: int):
        st = self.clients.pop(client_id, None)
        if st is not None:
            self.ex.free(st.res)
            self.used -= st.bytes

    def reset_history(self, client_id: int):
        st = self.clients[client_id]
        st.last_seq = -1
        st.last_cam = None

    # -------------------------------------------------------------- requests
    def offer(self, req: Request) -> bool:
        st = self.clients.get(req.client_id)
        if st is None:
            return False
        st.pending.append(req)
        return True

    def tick(self, now: float | None = None) -> int:
        """Retire finished batches, then launch at most one new batch."""
        now = self.clock() if now is None else now
        self._retire(now, block=False)
        if len(self.inflight) >= self.max_inflight:
            return 0
        batch = []
        ready = []
        for st in self.clients.values():
            if st.in_flight or not st.pending:
                continue
            deliv = [r for r in st.pending if r.deliver_t <= now]
            if not deliv:
                continue
            newest = max(deliv, key=lambda r: r.seq)
            for r in deliv:
                if r is newest:
                    continue
                if r.seq <= st.last_seq:
                    self.stats.dropped_out_of_order += 1
                else:
                    self.stats.dropped_superseded += 1
            st.pending = [r for r in st.pending if r.deliver_t > now]
            if newest.seq <= st.last_seq:
                self.stats.dropped_out_of_order += 1
                continue
            if now - newest.send_t > self.max_stale_s:
                self.stats.dropped_stale += 1
                continue
            ready.append((newest.deliver_t, st, newest))
        ready.sort(key=lambda x: x[0])
        for _, st, req in ready[: self.max_batch]:
            batch.append((st, req))
        # clients beyond the batch keep their request for the next tick
        for _, st, req in ready[self.max_batch:]:
            st.pending.append(req)
        if not batch:
            return 0
        items = [(st.res, st.spec, req, st.last_cam) for st, req in batch]
        token = self.ex.launch(items)
        for st, req in batch:
            st.in_flight = True
            st.last_active = now
        self.inflight.append((token, batch))
        self.stats.batches += 1
        return len(batch)

    def _retire(self, now: float, block: bool):
        while self.inflight:
            token, batch = self.inflight[0]
            if not (self.ex.wait(token) if block else self.ex.done(token)):
                return
            self.inflight.popleft()
            t = self.clock() if block else now
            for st, req in batch:
                st.in_flight = False
                st.last_seq = req.seq
                st.last_cam = req.camera
                st.last_active = t
                self.ex.commit(st.res)
                self.stats.served += 1
                self.stats.pixels += st.spec.W * st.spec.H
                self.stats.latencies_ms.append((t - req.deliver_t) * 1e3)
                st.served.append(req.seq)
                if self.keep_outputs:
                    st.served[-1] = (req.seq, self.ex.output(st.res))

    def drain(self):
        while self.inflight:
            self._retire(self.clock(), block=True)


# ----------------------------------------------------------------------------
# GPU executor: one ragged launch per pass per batch, through libdhr
# ----------------------------------------------------------------------------

class GpuExecutor:
    """Runs batches on `n_streams` HIP streams (default priority)."""

    def __init__(self, ctx, scenes: dict, n_streams: int = 3, seed: int = 5, n_ao: int = 1, n_shadow: int = 1,
                 svgf_params=None):
        import torch

        from . import binding as B
        self.B = B
        self.torch = torch
        self.ctx = ctx
        self.scenes = scenes          # name -> dict(bvh, lights, ao_radius)
        self.streams = [torch.cuda.Stream() for _ in range(n_streams)]
        self.next_stream = 0
        self.seed = seed
        self.n_ao = n_ao
        self.n_shadow = n_shadow
        self.P = svgf_params if svgf_params is not None else B.svgf_params()

    def n_lights(self, scene: str) -> int:
        return len(self.scenes[scene]["lights"])

    def alloc(self, spec: ClientSpec):
        t = self.torch
        HW = spec.W * spec.H
        L = self.n_lights(spec.scene)
        return {"pos": [t.empty(HW, 4, device="cuda") for _ in range(2)],
                "nz": [t.empty(HW, 4, device="cuda") for _ in range(2)],
                "dz": t.empty(HW, 2, device="cuda"), "mv": t.empty(HW, 2, device="cuda"),
                "hist": [t.empty(HW, 4, device="cuda") for _ in range(2)],
                "ao": t.empty(HW, dtype=t.uint8, device="cuda"),
                "sh": t.empty(max(L, 1), HW, dtype=t.uint8, device="cuda"),
                "out": t.empty(HW, device="cuda"),
                "work": t.empty(self.B.dhr_svgf_workspace_bytes(spec.W, spec.H, self.P, 0) // 4, device="cuda"),
                "cur": 0, "has_hist": False}

    def free(self, res):
        res.clear()

    def launch(self, items):
        B = self.B
        s = self.streams[self.next_stream]
        self.next_stream = (self.next_stream + 1) % len(self.streams)
        gjobs, tjobs, frames = [], [], []
        for res, spec, req, prev_cam in items:
            sc = self.scenes[spec.scene]
            c = 1 - res["cur"] if res["has_hist"] else res["cur"]   # slot this frame writes
            p = 1 - c
            has_prev = prev_cam is not None and res["has_hist"]
            gjobs.append(dict(bvh=sc["bvh"], cur=req.camera, prev=prev_cam if has_prev else None,
                              W=spec.W, H=spec.H, pos=res["pos"][c], nz=res["nz"][c], dz=res["dz"], mv=res["mv"]))
            tp = B.trace_params(spec.W, spec.H, frame=req.seq, client_id=spec.client_id, seed=self.seed,
                                n_ao=self.n_ao, ao_radius=sc["ao_radius"], n_shadow=self.n_shadow, lights=sc["lights"])
            tjobs.append(dict(bvh=sc["bvh"], params=tp, pos=res["pos"][c], nz=res["nz"][c], ao_count=res["ao"],
                              shadow_count=res["sh"]))
            frames.append(B.svgf_frame(spec.W, spec.H, self.n_ao, res["ao"], res["pos"][c], res["nz"][c], res["dz"],
                                       res["mv"], res["pos"][p] if has_prev else None,
                                       res["nz"][p] if has_prev else None,
                                       res["hist"][p] if has_prev else None, res["hist"][c], res["out"],
                                       B.pix_angle(req.camera, spec.H), work=res["work"]))
            res["pending_slot"] = c
        with self.torch.cuda.stream(s):
            B.dhr_gbuffer_trace_batch(self.ctx, gjobs, tjobs, stream=s)
            B.dhr_svgf_filter(self.ctx, self.P, frames, stream=s)
            ev = self.torch.cuda.Event()
            ev.record(s)
        return ev

    def done(self, token) -> bool:
        return token.query()

    def wait(self, token) -> bool:
        token.synchronize()
        return True

    def commit(self, res):
        res["cur"] = res.pop("pending_slot")
        res["has_hist"] = True

    def output(self, res):
        return res["out"].clone()


# ----------------------------------------------------------------------------
# simulated clients (the workload, not the method)
# ----------------------------------------------------------------------------

RESOLUTIONS = [(640, 360), (1280, 720), (1920, 1080)]


def make_clients(n: int, seed: int = 100):
    """Client i: resolution and scene drawn from seeded generators."""
    rng = np.random.default_rng(seed)
    specs = []
    for i in range(n):
        W, H = RESOLUTIONS[int(rng.integers(0, 3))]
        scene = ["spheres", "room"][int(rng.integers(0, 2))]
        specs.append(ClientSpec(i, W, H, scene))
    return specs


def request_trace(specs, duration_s: float, rate_hz: float = 30.0, max_delay_s: float = 0.2,
                  arrival_seed: int = 7, delay_seed: int = 8):
    """Poisson frame requests per client and injected network delays U[0, max]."""
    from . import workloads as wl
    ra = np.random.default_rng(arrival_seed)
    rd = np.random.default_rng(delay_seed)
    reqs = []
    for sp in specs:
        t = ra.exponential(1.0 / rate_hz)
        seq = 0
        path = "orbit" if sp.scene == "spheres" else "walk"
        n_est = int(duration_s * rate_hz * 2 + 10)
        cams = wl.camera_path(path, n_est, phase=float(np.random.default_rng(100 + sp.client_id).uniform(0, 2 * math.pi)))
        while t < duration_s and seq < n_est:
            d = rd.uniform(0.0, max_delay_s)
            reqs.append(Request(sp.client_id, seq, cams[seq], t, t + d))
            seq += 1
            t += ra.exponential(1.0 / rate_hz)
    reqs.sort(key=lambda r: r.deliver_t)
    return reqs


def run_trace(server: Server, reqs, duration_s: float, realtime: bool = True):
    """Replays a request trace against the server on its clock."""
    t0 = server.clock()
    i = 0
    n = len(reqs)
    while True:
        now = server.clock() - t0
        while i < n and reqs[i].deliver_t <= now:
            r = reqs[i]
            server.offer(Request(r.client_id, r.seq, r.camera, t0 + r.send_t, t0 + r.deliver_t))
            i += 1
        server.tick(server.clock())
        if i >= n and not server.inflight and all(not c.pending for c in server.clients.values()):
            break
        if now > duration_s + 1.0:
            break
    server.drain()
    return server.clock() - t0
