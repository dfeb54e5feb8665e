"""One view's frames through the hot path, consecutive frames overlapped.

Frame f's G-buffer and visibility rays are one dhr_gbuffer_trace launch;
its filter (dhr_svgf_filter: temporal accumulation, variance, a-trous levels,
Section 3.3) runs on a filter stream.  With `frames_in_flight` = D, the
G-buffer + visibility launches of frames f + 1 .. f + D run on D streams
beside frame f's filter and beside each other: a frame's rays do not depend
on any other frame, so the long primary walks at the end of one frame's
launch (grazing rays at the horizon) leave the device to the next frame's
rays instead of idling it, and the filter's launch boundaries are filled
the same way.  D + 2 G-buffer / count slots and two history buffers make the
overlap safe: frame f writes slot f % (D + 2) only after the filter of frame
f - D - 1, the last reader of that slot (as its previous frame), has
finished.  The results are those of the frames run one at a time
(`overlap=False`), byte for byte.

All streams have the default priority.  One pipeline object serves one view;
its buffers are reused by every run, so runs of one object must not overlap.
"""
from __future__ import annotations

from . import binding as B


class FramePipeline:
    """Buffers and streams for the frames of one W x H view.

    ctx, bvh: the context and the scene's hierarchy; n_ao: AO rays per pixel
    (the filter's denominator); n_lights: lights of the trace parameters;
    params: the filter's dhr_svgf_params."""

    def __init__(self, ctx, bvh, W: int, H: int, n_ao: int, n_lights: int, params, device: str = "cuda",
                 frames_in_flight: int = 1):
        import torch
        self.torch = torch
        self.ctx, self.bvh, self.W, self.H, self.n_ao, self.P = ctx, bvh, W, H, n_ao, params
        HW = W * H
        self.depth = max(1, int(frames_in_flight))
        self.slots = S = self.depth + 2
        self.gb = [B.gbuffer_tensors(W, H, device) for _ in range(S)]
        self.aos = [torch.empty(HW, dtype=torch.uint8, device=device) for _ in range(S)]
        self.shs = [torch.empty(max(n_lights, 1), HW, dtype=torch.uint8, device=device) for _ in range(S)]
        self.n_lights = n_lights
        self.hist = [torch.empty(HW, 4, device=device) for _ in range(2)]
        self.out = torch.empty(HW, device=device)
        self.work = torch.empty(B.dhr_svgf_workspace_bytes(W, H, params, 0) // 4, device=device)
        self.s_frames = [torch.cuda.Stream() for _ in range(self.depth)]
        self.s_filt = torch.cuda.Stream()

    def launch_frame(self, f: int, cams, tps, stream) -> None:
        """G-buffer and visibility of frame f (cams[f - 1] is its previous camera; frame 0 has none)."""
        k = f % self.slots
        g = self.gb[k]
        B.dhr_gbuffer_trace(self.ctx, self.bvh, cams[f], cams[f - 1] if f > 0 else None, self.W, self.H, tps[f],
                            g["pos"], g["nz"], g["dz"], g["mv"], self.aos[k],
                            self.shs[k] if self.n_lights else None, stream=stream)

    def launch_filter(self, f: int, cams, stream) -> None:
        """The filter of frame f on its G-buffer and counts, with frame f - 1's as history."""
        S = self.slots
        g, p = self.gb[f % S], self.gb[(f - 1) % S]
        first = f == 0
        fr = B.svgf_frame(self.W, self.H, self.n_ao, self.aos[f % S], g["pos"], g["nz"], g["dz"], g["mv"],
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
        D, S = self.depth, self.slots
        sfs, sv = self.s_frames, self.s_filt
        for s in sfs:
            s.wait_stream(cur)
        sv.wait_stream(cur)
        done, ready = {}, {}

        def frame(f):
            s = sfs[f % D]
            if f - S + 1 >= n0:
                s.wait_event(done[f - S + 1])    # slot f % S: filter f - S + 1 read it as its previous frame
            rec("frame", f, 0, s)
            self.launch_frame(f, cams, tps, s)
            rec("frame", f, 1, s)
            e = torch.cuda.Event()
            e.record(s)
            ready[f] = e

        for f in range(n0, min(n0 + D, n1)):
            frame(f)
        for f in range(n0, n1):
            sv.wait_event(ready[f])              # filter f after frame f
            rec("svgf", f, 0, sv)
            self.launch_filter(f, cams, sv)
            rec("svgf", f, 1, sv)
            d = torch.cuda.Event()
            d.record(sv)
            done[f] = d
            if f + D < n1:
                frame(f + D)
        for s in sfs:
            cur.wait_stream(s)
        cur.wait_stream(sv)
