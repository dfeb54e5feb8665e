"""One view's frames through the hot path, consecutive frames overlapped.

Frame f's G-buffer and visibility rays are one dhr_gbuffer_trace launch on
one stream; its filter (dhr_svgf_filter: temporal accumulation, variance,
a-trous levels, Section 3.3) runs on a second stream.  Frame f + 1's
G-buffer + visibility launch therefore runs beside frame f's filter, which
fills the device where one pass alone leaves it idle (the tail of the
traversal kernel, the filter's launch boundaries).  Three G-buffer / count
slots and two history buffers make the overlap safe: frame f + 1 writes slot
(f + 1) % 3 only after frame f - 1's filter, the last reader of that slot,
has finished.  The results are those of the frames run one at a time
(`overlap=False`), byte for byte.

Both streams have the default priority.  One pipeline object serves one view;
its buffers are reused by every run, so runs of one object must not overlap.
"""
from __future__ import annotations

from . import binding as B


class FramePipeline:
    """Buffers and streams for the frames of one W x H view.

    ctx, bvh: the context and the scene's hierarchy; n_ao: AO rays per pixel
    (the filter's denominator); n_lights: lights of the trace parameters;
    params: the filter's dhr_svgf_params."""

    def __init__(self, ctx, bvh, W: int, H: int, n_ao: int, n_lights: int, params, device: str = "cuda"):
        import torch
        self.torch = torch
        self.ctx, self.bvh, self.W, self.H, self.n_ao, self.P = ctx, bvh, W, H, n_ao, params
        HW = W * H
        self.gb = [B.gbuffer_tensors(W, H, device) for _ in range(3)]
        self.aos = [torch.empty(HW, dtype=torch.uint8, device=device) for _ in range(3)]
        self.shs = [torch.empty(max(n_lights, 1), HW, dtype=torch.uint8, device=device) for _ in range(3)]
        self.n_lights = n_lights
        self.hist = [torch.empty(HW, 4, device=device) for _ in range(2)]
        self.out = torch.empty(HW, device=device)
        self.work = torch.empty(B.dhr_svgf_workspace_bytes(W, H, params, 0) // 4, device=device)
        self.s_frame, self.s_filt = torch.cuda.Stream(), torch.cuda.Stream()

    def launch_frame(self, f: int, cams, tps, stream) -> None:
        """G-buffer and visibility of frame f (cams[f - 1] is its previous camera; frame 0 has none)."""
        g = self.gb[f % 3]
        B.dhr_gbuffer_trace(self.ctx, self.bvh, cams[f], cams[f - 1] if f > 0 else None, self.W, self.H, tps[f],
                            g["pos"], g["nz"], g["dz"], g["mv"], self.aos[f % 3],
                            self.shs[f % 3] if self.n_lights else None, stream=stream)

    def launch_filter(self, f: int, cams, stream) -> None:
        """The filter of frame f on its G-buffer and counts, with frame f - 1's as history."""
        g, p = self.gb[f % 3], self.gb[(f - 1) % 3]
        first = f == 0
        fr = B.svgf_frame(self.W, self.H, self.n_ao, self.aos[f % 3], g["pos"], g["nz"], g["dz"], g["mv"],
                          None if first else p["pos"], None if first else p["nz"],
                          None if first else self.hist[(f + 1) % 2], self.hist[f % 2], self.out,
                          B.pix_angle(cams[f], self.H), work=self.work)
        B.dhr_svgf_filter(self.ctx, self.P, [fr], stream=stream)

    def run(self, cams, tps, n0: int, n1: int, overlap: bool = True, events=None) -> None:
        """Frames n0 .. n1 - 1 (frame n0 > 0 continues from frame n0 - 1's
        history).  tps[f]: frame f's dhr_trace_params.  events: None, or a
        dict with "frame" and "svgf" lists of (start, end) timing events,
        indexed f - n0, recorded on the stream each pass runs on.  Returns
        with the work enqueued and torch's current stream ordered after it."""
        torch = self.torch
        cur = torch.cuda.current_stream()

        def rec(k, f, e, s):
            if events is not None:
                events[k][f - n0][e].record(s)

        if not overlap:
            for f in range(n0, n1):
                rec("frame", f, 0, cur)
                self.launch_frame(f, cams, tps, cur)
                rec("frame", f, 1, cur)
                rec("svgf", f, 0, cur)
                self.launch_filter(f, cams, cur)
                rec("svgf", f, 1, cur)
            return
        sf, sv = self.s_frame, self.s_filt
        sf.wait_stream(cur)
        sv.wait_stream(cur)
        done = {}

        def frame(f):
            rec("frame", f, 0, sf)
            self.launch_frame(f, cams, tps, sf)
            rec("frame", f, 1, sf)

        if n1 > n0:
            frame(n0)
        for f in range(n0, n1):
            ready = torch.cuda.Event()
            ready.record(sf)
            sv.wait_event(ready)                 # filter f after frame f
            rec("svgf", f, 0, sv)
            self.launch_filter(f, cams, sv)
            rec("svgf", f, 1, sv)
            if f + 1 < n1:
                if f > n0:
                    sf.wait_event(done[f - 1])   # slot (f + 1) % 3 is filter f - 1's previous frame
                frame(f + 1)
            d = torch.cuda.Event()
            d.record(sv)
            done[f] = d
        cur.wait_stream(sf)
        cur.wait_stream(sv)
