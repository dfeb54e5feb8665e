"""Benchmark of the DHR+S server hot path on one MI355X.

One step = one frame of the 1920x1080 terrain workload through the whole
path: G-buffer of primary rays, 1 AO + 2 soft-shadow rays per pixel through
the BVH, and the modified SVGF (temporal, variance, 5 a-trous levels), with
history and the previous G-buffer resident in HBM between frames.

Prints one JSON line.  `value` is AO+shadow Mrays/s of the whole step (rays
traced per second of step time); per-pass rates, the roofline of the dominant
kernel and the oracle's CPU rate ride along.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
# VALU peak in lane operations (slots) per second: the published FP32 vector
# rate, 157.3 TFLOP/s with an FMA counted as two flops, is 78.64 T lane-ops/s
# (256 CUs x 4 SIMDs x 2.4 GHz x 32 lanes: one wave64 instruction per SIMD
# every two cycles).  An FMA is one slot, a transcendental (exp2, log2, rcp,
# sqrt) four (quarter rate).
VALU_PEAK_TSLOTS = 256 * 4 * 32 * 2.4e9 / 1e12
# Only FP32 FMA, MUL and ADD with VGPR, inline or literal operands issue at
# that rate (measured: 54-72 T lane-ops/s).  Min, max, max3, compare and
# select instructions, and any FP32 instruction with an SGPR operand, issue
# at half of it (measured: 36-43 T).  The traversal's node step is made of
# those: slab FMAs on node planes held in SGPRs (scalar loads) and the
# min/max/compare reductions.  Each VALU roofline therefore also reports its
# fraction of the half rate.
VALU_HALF_TSLOTS = VALU_PEAK_TSLOTS / 2
SLOT_UNIT = "T VALU lane-ops/s"


def valu_roof(ach, **extra):
    """A VALU roofline object: achieved slots/s against the published peak,
    with the fraction of the half issue rate beside it."""
    return {"bound": "alu", "achieved": ach, "peak": VALU_PEAK_TSLOTS, "unit": SLOT_UNIT,
            "frac": ach / VALU_PEAK_TSLOTS if ach else None,
            "frac_half_issue_rate": ach / VALU_HALF_TSLOTS if ach else None, **extra}


PEAK_NOTE = ("peak: the published FP32 vector rate (157.3 TFLOP/s, an FMA = 1 slot), reached by FMA/MUL/ADD on VGPR "
             "or constant operands; frac_half_issue_rate: against half of it, the measured issue rate of "
             "min/max/compare/select and of any instruction with an SGPR operand (the walk's whole mix)")
# algorithmic VALU slots per unit of work
SLOTS_PER_NODE = 40      # one node visit: two child slab tests (12 FMA, 12 min/max, entry/exit reductions) and
                         # the hit and order compares
SLOTS_PER_TRI = 35       # one ray-triangle test: Moller-Trumbore without division (2 cross, 4 dot, o - v0,
                         # u + v, t bound, 5 compares)
# one a-trous level per pixel: 24 non-centre taps x (13 plain slots: normal
# dot, clamp, the two differences, three exponent FMAs, four accumulations;
# plus exp2 and log2 at 4 each) = 24 x 21, one depth reciprocal per mirrored
# tap pair with its span (12 x 6), and the prefilter, its square root and
# reciprocal and the normalisation (34)
SLOTS_PER_LEVEL_PX = 24 * 21 + 12 * 6 + 34
# the adjoint of one level per pixel: pass A forms each tap weight (24 x 24)
# and its adjoint terms (24 x 18) plus the per-pixel terms (40); pass B forms
# each neighbour's weight again (24 x 24: storing 24 weights per pixel would
# cost more HBM time than forming them) and gathers (24 x 12, + 20)
SLOTS_PER_ADJ_LEVEL_PX = 24 * 24 + 24 * 18 + 40 + 24 * 24 + 24 * 12 + 20

# Hardware byte counters of the dominant kernels, per launch, from the
# committed rocprofv3 --pmc summary; each entry holds the SHA-256 of the
# kernel's sources when it was taken and is ignored once they change.
PMC_SUMMARY = os.path.join(ROOT, "profiles", "pmc_terrain1080.md")
KERNEL_SOURCES = {
    "frame_kernel": ["trace.hip", "device.h", "camera.h"],
    "trace_kernel": ["trace.hip", "device.h", "camera.h"],
    "gbuffer_kernel": ["trace.hip", "device.h", "camera.h"],
    "svgf_pass": ["svgf.hip", "svgf_common.h", "device.h"],
}


def sources_sha(kernel: str) -> str:
    import hashlib
    h = hashlib.sha256()
    for f in KERNEL_SOURCES[kernel]:
        with open(os.path.join(ROOT, "paper_2406_06963_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def pmc_traffic(kernel: str):
    """HBM bytes per launch (FETCH_SIZE + WRITE_SIZE, copy-calibrated) from the
    committed summary, or None if absent or taken on other sources."""
    try:
        with open(PMC_SUMMARY) as fh:
            lines = fh.read().splitlines()
    except OSError:
        return None
    sha = sources_sha(kernel)
    for ln in lines:
        f = ln.split()
        if len(f) == 4 and f[0] == "traffic:" and f[1] == kernel and f[2] == sha:
            return float(f[3])
    return None


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=30)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--preset", default="terrain1080")
    ap.add_argument("--cpu-frames", type=int, default=16,
                    help="frames of the oracle CPU baseline, about 10-30 s of host work (0 = skip)")
    ap.add_argument("--no-counters", action="store_true")
    ap.add_argument("--serve-seconds", type=float, default=6.0, help="serving run per mode (0 = skip)")
    ap.add_argument("--serve-clients", type=int, default=64)
    ap.add_argument("--bwd-frames", type=int, default=16, help="frames of the differentiation run (0 = skip)")
    ap.add_argument("--other-steps", type=int, default=20,
                    help="timed steps of the 64x64 and 720p workloads (0 = skip)")
    ap.add_argument("--frames-in-flight", type=int, default=1,
                    help="G-buffer + visibility launches of later frames run beside a frame's filter")
    ap.add_argument("--copy-mib", type=int, default=0,
                    help="before the steps, copy a buffer of this many MiB three times (a plain copy kernel of "
                         "known size, to calibrate hardware byte counters; 0 = skip)")
    return ap.parse_args()


def progress(msg: str) -> None:
    """A progress line on stderr (the JSON line alone goes to stdout)."""
    print(f"[bench {time.strftime('%H:%M:%S')}] {msg}", file=sys.stderr, flush=True)


def svgf_bytes_per_px(levels: int) -> int:
    """Algorithmic bytes of the filter per pixel: each pass reads its inputs
    and writes its outputs once (neighbourhoods from cache).
      temporal: ao 1 + pos 16 + nz 16 + mv 8 + history taps (prev pos, prev nz,
                hist: 48) + hist_out 16                      = 105
      variance: hist 16 + nz 16 + (c, var) 8                 =  40
      level l : (c, var) 8 + nz 16 + dz 8 + output 8         =  40
                (last level writes 4 bytes; level 0 also writes hist.c: +4)
    These are the method's passes; the implementation writes most pixels'
    level-0 input from the temporal kernel and runs the variance kernel on
    short-history tiles only, so it moves fewer bytes than this figure."""
    return 105 + 40 + 40 * levels - 4 + 4


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py measures one GPU (--gpus {args.gpus} requested): the path shards by client, one GPU "
              "per shard, and multi-GPU runs are not part of this benchmark", file=sys.stderr)
        sys.exit(2)
    import numpy as np
    import torch

    from paper_2406_06963_amd import binding as B
    from paper_2406_06963_amd import workloads as wl

    dev = "cuda"
    if args.copy_mib > 0:
        src = torch.ones(args.copy_mib << 18, device=dev)
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    pr = wl.preset(args.preset)
    W, H = pr.W, pr.H
    HW = W * H
    nfr = args.warmup + max(args.steps, args.cpu_frames) + 6   # + the batched-filter frames
    scene = wl.make_scene(pr.scene)
    cams = wl.camera_path(pr.camera, nfr, scene)
    lights = wl.lights_for(pr.scene)
    ctx = B.dhr_create(0)
    t0 = time.time()
    bvh = B.dhr_build_bvh(ctx, scene.tris, scene.obj_id)
    bvh_s = time.time() - t0
    info = bvh.info()
    P = B.svgf_params(levels=pr.levels, alpha=pr.alpha)

    from paper_2406_06963_amd.pipeline import FramePipeline

    # frame f + 1's G-buffer + visibility launch overlaps frame f's filter on a
    # second stream, as a renderer (or the serving loop) runs them
    pipe = FramePipeline(ctx, bvh, W, H, pr.n_ao, len(lights), P, dev, frames_in_flight=args.frames_in_flight)
    gb, hist, out, work = pipe.gb, pipe.hist, pipe.out, pipe.work
    ao, sh = pipe.aos[0], pipe.shs[0]          # the single-frame runs below

    # one event pair per pass and timed step, each on the stream its kernels run on
    ev = {k: [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
              for _ in range(args.steps)] for k in ("frame", "svgf", "frame_seq", "svgf_seq", "gbuf", "trace")}

    def tparams(f):
        return B.trace_params(W, H, frame=f, seed=pr.seed, n_ao=pr.n_ao, ao_radius=pr.ao_radius,
                              n_shadow=pr.n_shadow, lights=lights)

    tps = [tparams(f) for f in range(nfr)]
    w0, w1 = args.warmup, args.warmup + args.steps

    progress(f"{pr.name}: scene and BVH ready ({bvh_s:.2f} s); timed steps")
    pipe.run(cams, tps, 0, w0)
    torch.cuda.synchronize()
    t_start = time.perf_counter()
    pipe.run(cams, tps, w0, w1, events={"frame": ev["frame"], "svgf": ev["svgf"]})
    torch.cuda.synchronize()
    t_end = time.perf_counter()
    ms_per_step = (t_end - t_start) * 1e3 / args.steps

    # the same frames again, one at a time on one stream from the same
    # history (the per-pass times without overlap), then as two launches
    # (dhr_gbuffer, then dhr_trace_visibility): the per-pass breakdown and the
    # visibility kernel's own roofline
    pipe.run(cams, tps, 0, w0, overlap=False)
    torch.cuda.synchronize()
    t_seq = time.perf_counter()
    pipe.run(cams, tps, w0, w1, overlap=False, events={"frame": ev["frame_seq"], "svgf": ev["svgf_seq"]})
    torch.cuda.synchronize()
    ms_per_step_seq = (time.perf_counter() - t_seq) * 1e3 / args.steps
    for k, f in enumerate(range(args.warmup, args.warmup + args.steps)):
        g = gb[0]
        ev["gbuf"][k][0].record()
        B.dhr_gbuffer(ctx, bvh, cams[f], cams[f - 1], W, H, g["pos"], g["nz"], g["dz"], g["mv"])
        ev["gbuf"][k][1].record()
        ev["trace"][k][0].record()
        B.dhr_trace_visibility(ctx, bvh, tparams(f), g["pos"], g["nz"], ao, sh)
        ev["trace"][k][1].record()
    torch.cuda.synchronize()
    per = {k: sum(a.elapsed_time(b) for a, b in ev[k]) / args.steps for k in ev}
    per_median = {k: float(np.median([a.elapsed_time(b) for a, b in ev[k]])) for k in ev}

    # valid pixels of the timed frames (untimed recount)
    valid = 0
    for f in range(args.warmup, args.warmup + args.steps):
        g = gb[0]
        B.dhr_gbuffer(ctx, bvh, cams[f], cams[f - 1], W, H, g["pos"], g["nz"], g["dz"], g["mv"])
        valid += int((g["nz"][:, 3] > 0).sum().item())
    rays_per_step = valid / args.steps * (pr.n_ao + len(lights) * pr.n_shadow)

    # traversal work (instrumented kernel variants, untimed): the fused
    # launch (primary and visibility rays) and the visibility launch alone
    counts = counts_frame = None
    if not args.no_counters:
        c = torch.zeros(4, dtype=torch.int64, device=dev)
        cf = torch.zeros(4, dtype=torch.int64, device=dev)
        for f in range(args.warmup, args.warmup + args.steps):
            g = gb[0]
            B.dhr_set_trace_counters(ctx, cf)
            B.dhr_gbuffer_trace(ctx, bvh, cams[f], cams[f - 1], W, H, tparams(f), g["pos"], g["nz"], g["dz"],
                                g["mv"], ao, sh)
            B.dhr_set_trace_counters(ctx, c)
            B.dhr_trace_visibility(ctx, bvh, tparams(f), g["pos"], g["nz"], ao, sh)
        B.dhr_set_trace_counters(ctx, None)
        counts = [int(v) / args.steps for v in c.cpu().tolist()]
        counts_frame = [int(v) / args.steps for v in cf.cpu().tolist()]

    frame_s = per["frame"] / 1e3           # timed launches (overlapping the filter)
    trace_s = per["trace"] / 1e3
    svgf_s = per["svgf_seq"] / 1e3         # the filter alone (its timed span shares the device)
    svgf_bytes = svgf_bytes_per_px(pr.levels) * HW
    roof_svgf = {"bound": "hbm", "achieved": svgf_bytes / svgf_s / 1e9, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                 "frac": svgf_bytes / svgf_s / 1e9 / HBM_PEAK_GBS, "traffic": pmc_traffic("svgf_pass"),
                 "kernel": "svgf (temporal + variance + 5 a-trous levels)",
                 "algorithmic_bytes_per_px": svgf_bytes_per_px(pr.levels)}
    roof_trace = None
    if counts:
        slots = counts[1] * SLOTS_PER_NODE + counts[3] * SLOTS_PER_TRI
        ach = slots / trace_s / 1e12
        roof_trace = valu_roof(ach, traffic=pmc_traffic("trace_kernel"),
                               kernel="trace_kernel (dhr_trace_visibility)", launch_ms=per["trace"],
                               traced_rays=counts[0], node_visits=counts[1], leaf_visits=counts[2],
                               tri_tests=counts[3], slots_per_node=SLOTS_PER_NODE, slots_per_tri=SLOTS_PER_TRI,
                               slots_per_launch=slots)
    roof_frame = roof_frame_seq = None
    if counts_frame:
        slots = counts_frame[1] * SLOTS_PER_NODE + counts_frame[3] * SLOTS_PER_TRI
        ach = slots / frame_s / 1e12
        roof_frame = valu_roof(ach, traffic=pmc_traffic("frame_kernel"), peak_note=PEAK_NOTE,
                               kernel="frame_kernel (dhr_gbuffer_trace: primary + visibility rays; its timed "
                                      "launches overlap the previous frame's filter)", launch_ms=per["frame"],
                               traced_rays=counts_frame[0], node_visits=counts_frame[1],
                               leaf_visits=counts_frame[2], tri_tests=counts_frame[3],
                               slots_per_node=SLOTS_PER_NODE, slots_per_tri=SLOTS_PER_TRI, slots_per_launch=slots)
        ach_seq = slots / (per["frame_seq"] / 1e3) / 1e12
        roof_frame_seq = valu_roof(ach_seq, kernel="frame_kernel, launched alone", launch_ms=per["frame_seq"])
    # the dominant kernel: the larger of the two passes run one at a time
    dominant = "frame" if per["frame_seq"] >= per["svgf_seq"] else "svgf"
    roofline = (roof_frame if (dominant == "frame" and roof_frame) else roof_svgf)

    line = {
        "metric": "AO+shadow Mrays/s and SVGF Mpix/s at 1080p; p99 frame latency, 64 clients",
        "value": rays_per_step / (ms_per_step / 1e3) / 1e6,
        "unit": "Mrays/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "fp32", "data": "synthetic",
        "config": {"workload": f"{pr.name}: {W}x{H}, {pr.scene} scene ({scene.n_tris} tris), "
                               f"{pr.n_ao} AO ray (r={pr.ao_radius}) + {pr.n_shadow} soft-shadow rays/px, "
                               f"{pr.levels}-level SVGF", "frames": args.steps,
                   "timed_frames": f"{w0}-{w1 - 1} of the camera path (frames 0-{w0 - 1} untimed warmup)",
                   "frames_in_flight": args.frames_in_flight, "parallelism": "single GPU"},
        "trace_mrays_s": rays_per_step / trace_s / 1e6,
        "svgf_mpix_s": HW / svgf_s / 1e6,
        "pass_ms": per,
        "pass_ms_median": per_median,
        "ms_per_step_sequential": ms_per_step_seq,
        "pass_note": "timed steps: frame = dhr_gbuffer_trace on one stream, svgf = dhr_svgf_filter on a second, "
                     "frame f + 1 overlapping frame f's filter (so svgf is a span, not a kernel time); *_seq = "
                     "the same frames one at a time on one stream; gbuf and trace = the same frames as two "
                     "launches (untimed for value)",
        "valid_frac": valid / args.steps / HW,
        "bvh": {"nodes": info["n_nodes"], "depth": info["depth"], "build_s": bvh_s,
                "device_mb": info["device_bytes"] / 2 ** 20},
        "roofline": roofline,
        "roofline_svgf": roof_svgf,
        "roofline_trace": roof_trace,
        "roofline_frame": roof_frame,
        "roofline_frame_sequential": roof_frame_seq,
    }

    # the light's visibility filtered by the same SVGF as a second channel
    # (own history), batched with the AO channel in one call
    hist_s = [torch.empty(HW, 4, device=dev) for _ in range(2)]
    out_s = torch.empty(HW, device=dev)
    work_s = torch.empty(B.dhr_svgf_workspace_bytes(W, H, P, 0) // 4, device=dev)
    f_end = args.warmup + args.steps
    f_first = max(1, f_end - 12)          # two untimed frames, then up to 10 timed
    n2 = f_end - f_first - 2
    e2 = [[torch.cuda.Event(enable_timing=True) for _ in range(2)] for _ in range(max(n2, 0))]
    for k, f in enumerate(range(f_first, f_end)):
        cur, prv = gb[f % 2], gb[(f + 1) % 2]
        B.dhr_gbuffer(ctx, bvh, cams[f], cams[f - 1], W, H, cur["pos"], cur["nz"], cur["dz"], cur["mv"])
        B.dhr_trace_visibility(ctx, bvh, B.trace_params(W, H, frame=f, seed=pr.seed, n_ao=pr.n_ao,
                                                        ao_radius=pr.ao_radius, n_shadow=pr.n_shadow, lights=lights),
                               cur["pos"], cur["nz"], ao, sh)
        first = k == 0
        frs = [B.svgf_frame(W, H, pr.n_ao, ao, cur["pos"], cur["nz"], cur["dz"], cur["mv"], None if first else prv["pos"],
                            None if first else prv["nz"], None if first else hist[(f + 1) % 2], hist[f % 2], out,
                            B.pix_angle(cams[f], H), work=work),
               B.svgf_frame(W, H, pr.n_shadow, sh[0], cur["pos"], cur["nz"], cur["dz"], cur["mv"],
                            None if first else prv["pos"], None if first else prv["nz"],
                            None if first else hist_s[(f + 1) % 2], hist_s[f % 2], out_s, B.pix_angle(cams[f], H),
                            work=work_s)]
        if k >= 2:
            e2[k - 2][0].record()
        B.dhr_svgf_filter(ctx, P, frs)
        if k >= 2:
            e2[k - 2][1].record()
    torch.cuda.synchronize()
    if n2 > 0:
        two_ms = sum(a.elapsed_time(b) for a, b in e2) / n2
        line["svgf_ao_and_shadow"] = {"ms": two_ms, "mpix_s": 2 * HW / (two_ms / 1e3) / 1e6,
                                      "vs_ao_only": two_ms / per["svgf_seq"]}

    progress(f"step {ms_per_step:.4f} ms; filter levels and batch")
    line["svgf_levels"] = bench_svgf_levels(B, ctx, W, H, P, gb[f_end % 2], out_s)
    line["svgf_batch4"] = bench_svgf_batch(B, ctx, bvh, pr, cams, lights, P, f_end, 4)

    # the lighter filter (one level of the 3x3 kernel) beside the full one, each
    # with its own history over the same noisy frames; both scored against a
    # 64-ray AO estimate of the last frame
    lf = range(max(1, args.warmup + args.steps - 16), args.warmup + args.steps)
    if len(lf) >= 3:
        line["svgf_light"] = bench_light_filter(B, ctx, bvh, pr, cams, lights, gb, ao, sh, P, lf)

    progress("device BVH, instancing, rasterised G-buffer, wire form")
    # the hierarchy built on the device (linear BVH) and refitted, and the
    # ray passes on it, against the host SAH build used above
    tri_d = torch.from_numpy(np.ascontiguousarray(scene.tris, dtype=np.float32).reshape(-1, 9)).to(dev)
    obj_d = torch.from_numpy(np.ascontiguousarray(scene.obj_id, dtype=np.uint32).view(np.int32)).to(dev)
    B.dhr_build_bvh_device(ctx, tri_d, obj_d).close()
    torch.cuda.synchronize()
    tb = time.perf_counter()
    lbvh = B.dhr_build_bvh_device(ctx, tri_d, obj_d)
    build_ms = (time.perf_counter() - tb) * 1e3
    er = [torch.cuda.Event(enable_timing=True) for _ in range(6)]
    f = args.warmup + args.steps - 1
    cur = gb[f % 2]
    tp = B.trace_params(W, H, frame=f, seed=pr.seed, n_ao=pr.n_ao, ao_radius=pr.ao_radius, n_shadow=pr.n_shadow,
                        lights=lights)
    B.dhr_refit_bvh(ctx, lbvh, tri_d)
    er[0].record()
    for _ in range(5):
        B.dhr_refit_bvh(ctx, lbvh, tri_d)
    er[1].record()
    for _ in range(5):
        B.dhr_gbuffer(ctx, lbvh, cams[f], cams[f - 1], W, H, cur["pos"], cur["nz"], cur["dz"], cur["mv"])
    er[2].record()
    for _ in range(5):
        B.dhr_trace_visibility(ctx, lbvh, tp, cur["pos"], cur["nz"], ao, sh)
    er[3].record()
    torch.cuda.synchronize()
    li = lbvh.info()
    line["bvh_device"] = {"build_ms": build_ms, "refit_ms": er[0].elapsed_time(er[1]) / 5,
                          "gbuf_ms": er[1].elapsed_time(er[2]) / 5, "trace_ms": er[2].elapsed_time(er[3]) / 5,
                          "nodes": li["n_nodes"], "depth": li["depth"],
                          "host_sah_build_s": bvh_s, "host_sah_gbuf_ms": per["gbuf"], "host_sah_trace_ms": per["trace"]}
    lbvh.close()
    del tri_d, obj_d

    # the terrain's boxes as instances of one cube (two-level hierarchy)
    if "instances" in scene.meta:
        bt, bo, mesh, xf, iid = wl.instanced_form(scene)
        tb = time.perf_counter()
        ibvh = B.dhr_build_bvh_instanced(ctx, bt, bo, mesh, xf, iid)
        ib_s = time.perf_counter() - tb
        ii = ibvh.info()
        ei = [torch.cuda.Event(enable_timing=True) for _ in range(3)]
        B.dhr_gbuffer(ctx, ibvh, cams[f], cams[f - 1], W, H, cur["pos"], cur["nz"], cur["dz"], cur["mv"])
        ei[0].record()
        for _ in range(5):
            B.dhr_gbuffer(ctx, ibvh, cams[f], cams[f - 1], W, H, cur["pos"], cur["nz"], cur["dz"], cur["mv"])
        ei[1].record()
        for _ in range(5):
            B.dhr_trace_visibility(ctx, ibvh, tp, cur["pos"], cur["nz"], ao, sh)
        ei[2].record()
        torch.cuda.synchronize()
        line["instanced"] = {"instances": int(len(xf)), "build_s": ib_s, "device_mb": ii["device_bytes"] / 2 ** 20,
                             "flat_device_mb": info["device_bytes"] / 2 ** 20,
                             "gbuf_ms": ei[0].elapsed_time(ei[1]) / 5, "trace_ms": ei[1].elapsed_time(ei[2]) / 5,
                             "flat_gbuf_ms": per["gbuf"], "flat_trace_ms": per["trace"]}
        ibvh.close()

    # the G-buffer by rasterisation (same texels as the ray-traced one)
    rwork = torch.empty(B.dhr_gbuffer_raster_workspace_bytes(W, H, scene.n_tris) // 4 + 64, device=dev)
    B.dhr_gbuffer_raster(ctx, bvh, cams[f], cams[f - 1], W, H, cur["pos"], cur["nz"], cur["dz"], cur["mv"], rwork)
    er[4].record()
    for _ in range(5):
        B.dhr_gbuffer_raster(ctx, bvh, cams[f], cams[f - 1], W, H, cur["pos"], cur["nz"], cur["dz"], cur["mv"], rwork)
    er[5].record()
    torch.cuda.synchronize()
    line["gbuffer_raster"] = {"ms": er[4].elapsed_time(er[5]) / 5, "ray_traced_ms": per["gbuf"]}
    del rwork

    # wire form of the last frame: AO bytes + per-light bits (memory-bound)
    q8 = torch.empty(HW, dtype=torch.uint8, device=dev)
    m8 = torch.empty(HW, dtype=torch.uint8, device=dev)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    B.dhr_encode_frame(ctx, value=out, q=q8, shadow_count=sh, n_shadow=pr.n_shadow, mask=m8)
    e0.record()
    for _ in range(200):
        B.dhr_encode_frame(ctx, value=out, q=q8, shadow_count=sh, n_shadow=pr.n_shadow, mask=m8)
    e1.record()
    torch.cuda.synchronize()
    enc_s = e0.elapsed_time(e1) / 200 / 1e3
    enc_bytes = HW * (4 + len(lights) + 2)
    line["encode"] = {"us": enc_s * 1e6, "bytes_per_px": 4 + len(lights) + 2,
                      "roofline": {"bound": "hbm", "achieved": enc_bytes / enc_s / 1e9, "peak": HBM_PEAK_GBS,
                                   "unit": "GB/s", "frac": enc_bytes / enc_s / 1e9 / HBM_PEAK_GBS}}
    progress("other workloads, differentiation, serving, CPU baseline")
    if args.other_steps > 0:
        line["other_workloads"] = {name: bench_preset(B, ctx, name, args.other_steps) for name in ("tiny", "room720")}
    if args.bwd_frames > 0:
        line["differentiation"] = bench_backward(B, ctx, args.bwd_frames)
        progress("differentiation done")
    if args.serve_seconds > 0:
        line["serving"] = bench_serving(B, ctx, args)
        line["p99_ms"] = line["serving"]["continuous"]["p99_ms"]
        progress("serving done")
    if args.cpu_frames > 0:
        line["cpu_baseline"] = cpu_baseline(pr, scene, cams, lights, args)
    print(json.dumps(line), flush=True)


def _median_ms(fn, reps=10):
    import numpy as np
    import torch
    fn()
    ev = [[torch.cuda.Event(enable_timing=True) for _ in range(2)] for _ in range(reps)]
    for a, b in ev:
        a.record()
        fn()
        b.record()
    torch.cuda.synchronize()
    return float(np.median([a.elapsed_time(b) for a, b in ev]))


def bench_svgf_levels(B, ctx, W, H, P, g, scratch):
    """Each a-trous level's time on one 1080p frame: the spatial stack run
    with 1 .. L levels on the (c, var) the filter's variance pass produced,
    level l's time the difference of the medians of l + 1 and l levels; its
    VALU roofline in algorithmic slots (SLOTS_PER_LEVEL_PX per pixel)."""
    import torch
    HW = W * H
    L = P.levels
    cv = torch.rand(HW, 2, device="cuda")
    cv[:, 1] *= 0.05
    work = torch.empty(B.dhr_svgf_workspace_bytes(W, H, P, 0) // 4, device="cuda")
    t = [0.0]
    for n in range(1, L + 1):
        Pn = B.svgf_params(levels=n, alpha=P.alpha)
        fr = [B.spatial_frame(W, H, cv, g["nz"], g["dz"], scratch, work=work)]
        t.append(_median_ms(lambda: B.dhr_svgf_spatial_forward(ctx, Pn, fr)))
    lv = []
    for l in range(L):
        ms = t[l + 1] - t[l]
        ach = SLOTS_PER_LEVEL_PX * HW / (ms / 1e3) / 1e12 if ms > 0 else None
        lv.append({"level": l, "ms": ms, **valu_roof(ach),
                   "hbm_frac": 40 * HW / (ms / 1e3) / 1e9 / HBM_PEAK_GBS if ms > 0 else None})
    return {"note": "level l = median of the stack with l + 1 levels minus that with l (one 1080p frame, its "
                    "geometry, synthetic (c, var)); slots per pixel and level: " + str(SLOTS_PER_LEVEL_PX),
            "stack_ms": t[1:], "levels": lv}


def bench_svgf_batch(B, ctx, bvh, pr, cams, lights, P, f0, n):
    """The filter over a batch of n consecutive 1080p frames in one call (one
    launch per pass for all of them): the working set (about 0.3 GB per
    frame) exceeds the 256 MB last-level cache, so the passes stream from
    HBM."""
    import torch
    W, H, HW = pr.W, pr.H, pr.W * pr.H
    gb = [B.gbuffer_tensors(W, H) for _ in range(n + 1)]
    aos = [torch.empty(HW, dtype=torch.uint8, device="cuda") for _ in range(n + 1)]
    sh = torch.empty(max(len(lights), 1), HW, dtype=torch.uint8, device="cuda")
    hin = [torch.rand(HW, 4, device="cuda") for _ in range(n)]
    for h in hin:
        h[:, 3] = 8.0
    hout = [torch.empty(HW, 4, device="cuda") for _ in range(n)]
    outs = [torch.empty(HW, device="cuda") for _ in range(n)]
    works = [torch.empty(B.dhr_svgf_workspace_bytes(W, H, P, 0) // 4, device="cuda") for _ in range(n)]
    for k in range(n + 1):
        f = f0 + k
        g = gb[k]
        B.dhr_gbuffer_trace(ctx, bvh, cams[f], cams[f - 1], W, H,
                            B.trace_params(W, H, frame=f, seed=pr.seed, n_ao=pr.n_ao, ao_radius=pr.ao_radius,
                                           n_shadow=pr.n_shadow, lights=lights),
                            g["pos"], g["nz"], g["dz"], g["mv"], aos[k], sh)
    frs = [B.svgf_frame(W, H, pr.n_ao, aos[k + 1], gb[k + 1]["pos"], gb[k + 1]["nz"], gb[k + 1]["dz"],
                        gb[k + 1]["mv"], gb[k]["pos"], gb[k]["nz"], hin[k], hout[k], outs[k],
                        B.pix_angle(cams[f0 + k + 1], H), work=works[k]) for k in range(n)]
    ms = _median_ms(lambda: B.dhr_svgf_filter(ctx, P, frs))
    nb = svgf_bytes_per_px(P.levels) * HW * n
    slots = (SLOTS_PER_LEVEL_PX * P.levels) * HW * n
    return {"frames": n, "ms": ms, "mpix_s": n * HW / (ms / 1e3) / 1e6,
            "roofline_hbm": {"bound": "hbm", "unit": "GB/s", "peak": HBM_PEAK_GBS,
                             "achieved": nb / (ms / 1e3) / 1e9, "frac": nb / (ms / 1e3) / 1e9 / HBM_PEAK_GBS},
            "roofline_valu_levels": valu_roof(slots / (ms / 1e3) / 1e12,
                                              note="the a-trous levels' slots over the whole filter's time")}


def bench_light_filter(B, ctx, bvh, pr, cams, lights, gb, ao, sh, P, frames):
    import torch
    W, H, HW = pr.W, pr.H, pr.W * pr.H
    PL = B.svgf_params(levels=1, alpha=pr.alpha, kernel_width=3)
    res = {}
    for name, Pk in (("full", P), ("light", PL)):
        hist = [torch.empty(HW, 4, device="cuda") for _ in range(2)]
        out = torch.empty(HW, device="cuda")
        work = torch.empty(B.dhr_svgf_workspace_bytes(W, H, Pk, 0) // 4, device="cuda")
        ev = []
        for k, f in enumerate(frames):
            cur, prv = gb[f % 2], gb[(f + 1) % 2]
            B.dhr_gbuffer(ctx, bvh, cams[f], cams[f - 1], W, H, cur["pos"], cur["nz"], cur["dz"], cur["mv"])
            B.dhr_trace_visibility(ctx, bvh, B.trace_params(W, H, frame=f, seed=pr.seed, n_ao=pr.n_ao,
                                                            ao_radius=pr.ao_radius, n_shadow=pr.n_shadow,
                                                            lights=lights), cur["pos"], cur["nz"], ao, sh)
            first = k == 0
            fr = B.svgf_frame(W, H, pr.n_ao, ao, cur["pos"], cur["nz"], cur["dz"], cur["mv"],
                              None if first else prv["pos"], None if first else prv["nz"],
                              None if first else hist[(f + 1) % 2], hist[f % 2], out, B.pix_angle(cams[f], H),
                              work=work)
            e = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
            e[0].record()
            B.dhr_svgf_filter(ctx, Pk, [fr])
            e[1].record()
            if k >= 2:
                ev.append(e)
        torch.cuda.synchronize()
        res[name] = {"ms": sum(a.elapsed_time(b) for a, b in ev) / len(ev), "out": out}
    # reference: 64 AO rays per pixel of the last frame (another seed)
    n_ref = 64
    f = frames[-1]
    cur = gb[f % 2]
    ref = torch.empty(HW, dtype=torch.uint8, device="cuda")
    sh1 = torch.empty(len(lights), HW, dtype=torch.uint8, device="cuda")
    B.dhr_trace_visibility(ctx, bvh, B.trace_params(W, H, frame=f, seed=pr.seed + 1000, n_ao=n_ref,
                                                    ao_radius=pr.ao_radius, n_shadow=1, lights=lights),
                           cur["pos"], cur["nz"], ref, sh1)
    valid = cur["nz"][:, 3] > 0
    r = ref.float()[valid] / n_ref
    raw = ao.float()[valid] / pr.n_ao
    rmse = lambda x: float(torch.sqrt(((x - r) ** 2).mean()).item())
    return {"kernel": "temporal + variance + one 3x3 a-trous level", "frames": len(frames),
            "ms": res["light"]["ms"], "full_ms": res["full"]["ms"],
            "mpix_s": HW / (res["light"]["ms"] / 1e3) / 1e6,
            "rmse_vs_64spp": {"light": rmse(res["light"]["out"][valid]), "full": rmse(res["full"]["out"][valid]),
                              "unfiltered_1spp": rmse(raw), "reference_own_noise_rms": float(
                                  torch.sqrt((r * (1 - r) / n_ref).mean()).item())}}


def bench_preset(B, ctx, name, steps, warmup=5):
    """The same step (G-buffer, rays, SVGF with resident history) on another
    workload: per-pass device time from HIP events, rates of the ray and
    filter passes, and the step with later frames' rays overlapping a
    frame's filter (the main workload's schedule, at one and two frames in
    flight)."""
    import torch

    from paper_2406_06963_amd import workloads as wl
    pr = wl.preset(name)
    W, H, HW = pr.W, pr.H, pr.W * pr.H
    scene = wl.make_scene(pr.scene)
    cams = wl.camera_path(pr.camera, warmup + steps, scene)
    lights = wl.lights_for(pr.scene)
    bvh = B.dhr_build_bvh(ctx, scene.tris, scene.obj_id)
    P = B.svgf_params(levels=pr.levels, alpha=pr.alpha)
    gb = [B.gbuffer_tensors(W, H) for _ in range(2)]
    hist = [torch.empty(HW, 4, device="cuda") for _ in range(2)]
    ao = torch.empty(HW, dtype=torch.uint8, device="cuda")
    sh = torch.empty(max(len(lights), 1), HW, dtype=torch.uint8, device="cuda")
    out = torch.empty(HW, device="cuda")
    work = torch.empty(B.dhr_svgf_workspace_bytes(W, H, P, 0) // 4, device="cuda")
    ev = [[torch.cuda.Event(enable_timing=True) for _ in range(5)] for _ in range(steps)]
    valid = 0
    for f in range(warmup + steps):
        cur, prv = gb[f % 2], gb[(f + 1) % 2]
        e = ev[f - warmup] if f >= warmup else None
        tp = B.trace_params(W, H, frame=f, seed=pr.seed, n_ao=pr.n_ao, ao_radius=pr.ao_radius,
                            n_shadow=pr.n_shadow, lights=lights)
        prev = cams[f - 1] if f else None
        if e:
            e[0].record()
            B.dhr_gbuffer(ctx, bvh, cams[f], prev, W, H, cur["pos"], cur["nz"], cur["dz"], cur["mv"])
            e[1].record()
            B.dhr_trace_visibility(ctx, bvh, tp, cur["pos"], cur["nz"], ao, sh)
            e[4].record()
        B.dhr_gbuffer_trace(ctx, bvh, cams[f], prev, W, H, tp, cur["pos"], cur["nz"], cur["dz"], cur["mv"], ao, sh)
        if e:
            e[2].record()
        fr = B.svgf_frame(W, H, pr.n_ao, ao, cur["pos"], cur["nz"], cur["dz"], cur["mv"],
                          prv["pos"] if f else None, prv["nz"] if f else None, hist[(f + 1) % 2] if f else None,
                          hist[f % 2], out, B.pix_angle(cams[f], H), work=work)
        B.dhr_svgf_filter(ctx, P, [fr])
        if e:
            e[3].record()
            valid += int((cur["nz"][:, 3] > 0).sum().item())
    torch.cuda.synchronize()
    # e0-e1 G-buffer, e1-e4 visibility (two launches, for the breakdown); e4-e2
    # the same frame through dhr_gbuffer_trace; e2-e3 the filter
    el = lambda a, b: sum(x[a].elapsed_time(x[b]) for x in ev) / steps
    t_g, t_t, t_f, t_s = el(0, 1), el(1, 4), el(4, 2), el(2, 3)
    rays = valid / steps * (pr.n_ao + len(lights) * pr.n_shadow)
    # the fused kernel's traversal work on the timed frames (counting variant, untimed)
    c = torch.zeros(4, dtype=torch.int64, device="cuda")
    B.dhr_set_trace_counters(ctx, c)
    for f in range(warmup, warmup + steps):
        g = gb[0]
        B.dhr_gbuffer_trace(ctx, bvh, cams[f], cams[f - 1], W, H,
                            B.trace_params(W, H, frame=f, seed=pr.seed, n_ao=pr.n_ao, ao_radius=pr.ao_radius,
                                           n_shadow=pr.n_shadow, lights=lights),
                            g["pos"], g["nz"], g["dz"], g["mv"], ao, sh)
    B.dhr_set_trace_counters(ctx, None)
    cnt = [int(v) / steps for v in c.cpu().tolist()]
    slots = cnt[1] * SLOTS_PER_NODE + cnt[3] * SLOTS_PER_TRI
    ach = slots / (t_f / 1e3) / 1e12
    # the same frames through the overlapped schedule with one and with two
    # later frames' rays in flight beside a frame's filter, wall clock
    # around them
    from paper_2406_06963_amd.pipeline import FramePipeline
    tps = [B.trace_params(W, H, frame=f, seed=pr.seed, n_ao=pr.n_ao, ao_radius=pr.ao_radius,
                          n_shadow=pr.n_shadow, lights=lights) for f in range(warmup + steps)]
    t_pipe = {}
    for d in (1, 2):
        pipe = FramePipeline(ctx, bvh, W, H, pr.n_ao, len(lights), P, frames_in_flight=d)
        pipe.run(cams, tps, 0, warmup)
        torch.cuda.synchronize()
        tp0 = time.perf_counter()
        pipe.run(cams, tps, warmup, warmup + steps)
        torch.cuda.synchronize()
        t_pipe[d] = (time.perf_counter() - tp0) * 1e3 / steps
        del pipe
    return {"workload": f"{name}: {W}x{H}, {pr.scene} scene ({scene.n_tris} tris), {pr.n_ao} AO + {pr.n_shadow} "
                        f"shadow rays/px, {pr.levels}-level SVGF", "steps": steps,
            "pass_ms": {"frame": t_f, "svgf": t_s, "gbuf": t_g, "trace": t_t},
            "trace_mrays_s": rays / (t_t / 1e3) / 1e6, "svgf_mpix_s": HW / (t_s / 1e3) / 1e6,
            "step_mrays_s": rays / ((t_f + t_s) / 1e3) / 1e6,
            "overlapped_step_ms": {f"{d}_in_flight": t for d, t in t_pipe.items()},
            "overlapped_step_mrays_s": {f"{d}_in_flight": rays / (t / 1e3) / 1e6 for d, t in t_pipe.items()},
            "roofline_frame": valu_roof(ach, traced_rays=cnt[0], node_visits=cnt[1], tri_tests=cnt[3]),
            "roofline_svgf": {"bound": "hbm", "unit": "GB/s", "peak": HBM_PEAK_GBS,
                              "achieved": svgf_bytes_per_px(pr.levels) * HW / (t_s / 1e3) / 1e9,
                              "frac": svgf_bytes_per_px(pr.levels) * HW / (t_s / 1e3) / 1e9 / HBM_PEAK_GBS}}


def bench_backward(B, ctx, n_frames):
    """Forward + backward of the 5-level stack over a batch of 720p frames of
    the room workload (inputs from the path itself, MSE against 256-spp AO)."""
    import torch

    from paper_2406_06963_amd import workloads as wl
    pr = wl.preset("room720")
    W, H, HW = pr.W, pr.H, pr.W * pr.H
    scene = wl.make_scene(pr.scene)
    cams = wl.camera_path(pr.camera, n_frames, scene)
    lights = wl.lights_for(pr.scene)
    bvh = B.dhr_build_bvh(ctx, scene.tris, scene.obj_id)
    P = B.svgf_params()
    L = P.levels
    gb = [B.gbuffer_tensors(W, H) for _ in range(n_frames)]
    hist = [torch.empty(HW, 4, device="cuda") for _ in range(2)]
    save = torch.empty(n_frames, L, HW, 2, device="cuda")
    cv = torch.empty(n_frames, HW, 2, device="cuda")
    target = torch.empty(n_frames, HW, device="cuda")
    ao = torch.empty(HW, dtype=torch.uint8, device="cuda")
    sh = torch.empty(1, HW, dtype=torch.uint8, device="cuda")
    out = torch.empty(n_frames, HW, device="cuda")
    fwork = torch.empty(B.dhr_svgf_workspace_bytes(W, H, P, 0) // 4, device="cuda")
    for f in range(n_frames):
        g = gb[f]
        B.dhr_gbuffer(ctx, bvh, cams[f], cams[f - 1] if f else None, W, H, g["pos"], g["nz"], g["dz"], g["mv"])
        B.dhr_trace_visibility(ctx, bvh, B.trace_params(W, H, frame=f, seed=pr.seed, n_ao=1, ao_radius=pr.ao_radius,
                                                        n_shadow=1, lights=lights), g["pos"], g["nz"], ao, sh)
        fr = B.svgf_frame(W, H, 1, ao, g["pos"], g["nz"], g["dz"], g["mv"], gb[f - 1]["pos"] if f else None,
                          gb[f - 1]["nz"] if f else None, hist[(f + 1) % 2] if f else None, hist[f % 2], out[f],
                          B.pix_angle(cams[f], H), save=save[f], work=fwork)
        B.dhr_svgf_filter(ctx, P, [fr])
        cv[f] = save[f, 0]
        # 256-spp reference: two 128-sample calls (sample offsets 0 and 128), another seed
        acc = torch.zeros(HW, device="cuda")
        for off in (0, 128):
            B.dhr_trace_visibility(ctx, bvh, B.trace_params(W, H, frame=f, seed=9, n_ao=128, ao_sample_offset=off,
                                                            ao_radius=pr.ao_radius, n_shadow=0),
                                   g["pos"], g["nz"], ao, sh)
            acc += ao.float()
        target[f] = acc / 256.0
    fwork_f = torch.empty(n_frames, (B.dhr_svgf_workspace_bytes(W, H, P, 0) + 15) // 16 * 4, device="cuda")
    fwd = [B.spatial_frame(W, H, cv[f], gb[f]["nz"], gb[f]["dz"], out[f], save=save[f], work=fwork_f[f])
           for f in range(n_frames)]
    nb = B.dhr_svgf_workspace_bytes(W, H, P, 1)
    work = torch.empty(n_frames, (nb + 15) // 16 * 4, device="cuda")
    gcv = torch.empty(n_frames, HW, 2, device="cuda")
    gs = torch.empty(3 * L, device="cuda")
    valid = torch.stack([g["nz"][:, 3] > 0 for g in gb]).float()
    e = [torch.cuda.Event(enable_timing=True) for _ in range(4)]
    times = []
    loss0 = None
    for it in range(6):
        e[0].record()
        B.dhr_svgf_spatial_forward(ctx, P, fwd)
        e[1].record()
        go = (2.0 / valid.sum()) * (out - target) * valid
        if it == 0:
            loss0 = float(((out - target) ** 2 * valid).sum() / valid.sum())
        bwd = [B.bwd_frame(W, H, save[f], gb[f]["nz"], gb[f]["dz"], go[f], gcv[f], work[f]) for f in range(n_frames)]
        e[2].record()
        B.dhr_svgf_backward(ctx, P, bwd, gs)
        e[3].record()
        torch.cuda.synchronize()
        if it > 0:
            times.append((e[0].elapsed_time(e[1]), e[2].elapsed_time(e[3])))
    fw = sum(t[0] for t in times) / len(times)
    bw = sum(t[1] for t in times) / len(times)
    px = n_frames * HW
    # algorithmic bytes per pixel and level: the forward level reads (c, var),
    # nz, dz and writes (c, var) (40 B); its adjoint reads the saved (c, var),
    # nz, dz and the output's gradient and writes the input's gradient (48 B)
    fb = px * L * 40
    bb = px * L * 48
    rf = lambda nb, ms: {"bound": "hbm", "unit": "GB/s", "peak": HBM_PEAK_GBS, "achieved": nb / (ms / 1e3) / 1e9,
                         "frac": nb / (ms / 1e3) / 1e9 / HBM_PEAK_GBS}
    rv = lambda per_px, ms: valu_roof(per_px * px * L / (ms / 1e3) / 1e12, slots_per_px_level=per_px)
    return {"workload": f"{n_frames} x {W}x{H} room frames, 5 levels, MSE vs 256-spp AO",
            "forward_ms": fw, "backward_ms": bw, "fwd_bwd_ms": fw + bw,
            "fwd_bwd_mpix_s": px / ((fw + bw) / 1e3) / 1e6, "mse": loss0,
            "roofline_forward": rf(fb, fw), "roofline_backward": rf(bb, bw),
            "roofline_forward_valu": rv(SLOTS_PER_LEVEL_PX, fw),
            "roofline_backward_valu": rv(SLOTS_PER_ADJ_LEVEL_PX, bw),
            "grad_sigma": gs.cpu().tolist()}


def bench_serving(B, ctx, args):
    """64 simulated clients (Poisson 30 Hz, delays U[0, 200] ms) served with
    continuous batching (unfused and fused launches), and the same trace
    served by per-client plain launches (one request at a time)."""
    from paper_2406_06963_amd import serve as sv
    from paper_2406_06963_amd import workloads as wl
    scenes = {}
    for name, r in (("spheres", 1.0), ("room", 0.5)):
        sc = wl.make_scene(name)
        scenes[name] = {"bvh": B.dhr_build_bvh(ctx, sc.tris, sc.obj_id), "lights": wl.lights_for(name),
                        "ao_radius": r}
    specs = sv.make_clients(args.serve_clients)
    reqs = sv.request_trace(specs, args.serve_seconds)
    res = {"clients": len(specs), "seconds": args.serve_seconds, "requests": len(reqs),
           "offered_mpix_s": sum(s.W * s.H for s in specs) * 30.0 / 1e6}
    # continuous batching: a client's request is admitted as soon as one of
    # the in-flight slots frees, and the work of the admitted requests
    # overlaps on the device.  "continuous": one frame per launch, 12 in
    # flight (the best setting measured on this GPU); "continuous_fused": up
    # to 4 frames fused per launch, 8 in flight; "plain": per-client plain
    # launches, one request at a time.
    modes = (("continuous", dict(max_batch=1, max_inflight=12)),
             ("continuous_fused", dict(max_batch=4, max_inflight=8)),
             ("plain", dict(max_batch=1, max_inflight=1)))
    for mode, kw in modes:
        progress(f"serving: {mode} at 30 Hz")
        ex = sv.GpuExecutor(ctx, scenes, n_streams=kw["max_inflight"])
        server = sv.Server(ex, budget_bytes=200e9, **kw)
        for sp in specs:
            server.connect(sp)
        wall = sv.run_trace(server, reqs, args.serve_seconds)
        res[mode] = server.stats.summary(wall)
        res[mode]["resident_gb"] = server.used / 1e9
        for sp in specs:
            server.disconnect(sp.client_id)
    res["speedup_frames_per_s"] = res["continuous"]["frames_per_s"] / max(res["plain"]["frames_per_s"], 1e-9)
    # capacity: every client always has a fresh request (400 Hz, far above
    # what the device can serve, no network delay)
    sat_s = min(args.serve_seconds, 3.0)
    sat = sv.request_trace(specs, sat_s, rate_hz=400.0, max_delay_s=0.0)
    for mode, kw in modes:
        progress(f"serving: {mode} at saturation")
        ex = sv.GpuExecutor(ctx, scenes, n_streams=kw["max_inflight"])
        server = sv.Server(ex, budget_bytes=200e9, **kw)
        for sp in specs:
            server.connect(sp)
        wall = sv.run_trace(server, sat, sat_s)
        res["saturated_" + mode] = server.stats.summary(wall)
        for sp in specs:
            server.disconnect(sp.client_id)
    res["saturated_speedup_frames_per_s"] = (res["saturated_continuous"]["frames_per_s"]
                                             / max(res["saturated_plain"]["frames_per_s"], 1e-9))
    res["saturated_fused_vs_unfused"] = (res["saturated_continuous_fused"]["frames_per_s"]
                                         / max(res["saturated_continuous"]["frames_per_s"], 1e-9))
    # the same 400 Hz with the U[0, 200] ms delays and the staleness limit:
    # a request is servable only if it is newer than the last served one, so
    # the out-of-order arrivals cap the served rate below the device's
    satd = sv.request_trace(specs, sat_s, rate_hz=400.0, max_delay_s=0.2)
    ex = sv.GpuExecutor(ctx, scenes, n_streams=12)
    server = sv.Server(ex, budget_bytes=200e9, max_batch=1, max_inflight=12)
    for sp in specs:
        server.connect(sp)
    wall = sv.run_trace(server, satd, sat_s)
    res["saturated_delayed_continuous"] = server.stats.summary(wall)
    res["saturated_delayed_requests"] = len(satd)
    for sp in specs:
        server.disconnect(sp.client_id)
    return res


def cpu_baseline(pr, scene, cams, lights, args):
    """The oracle as it stands, timed on the host cores over a bounded sample."""
    import numpy as np

    import oracle as orc
    W, H = pr.W, pr.H
    so = orc.Scene(scene.tris, scene.obj_id)
    Po = orc.svgf_params(levels=pr.levels, alpha=pr.alpha)
    hist = None
    prev = None
    rays = 0
    t_trace = t_svgf = t_all = 0.0
    f0 = args.warmup

    def frame(f, hist, prev):
        ts = time.perf_counter()
        pos, nz, dz, mv = orc.gbuffer(so, cams[f], cams[f - 1], W, H)
        tt = time.perf_counter()
        P = orc.trace_params(W, H, frame=f, seed=pr.seed, n_ao=pr.n_ao, ao_radius=pr.ao_radius,
                             n_shadow=pr.n_shadow, lights=lights)
        ao, sh, _ = orc.trace(so, P, pos, nz)
        tf = time.perf_counter()
        pix = np.float32(2 * math.tan(0.5 * cams[f].fov_y) / H)
        ref = orc.svgf_filter(Po, W, H, pr.n_ao, ao, pos, nz, dz, mv, prev[0] if prev else None,
                              prev[1] if prev else None, hist, pix)
        te = time.perf_counter()
        n = int((nz[:, 3] > 0).sum()) * (pr.n_ao + len(lights) * pr.n_shadow)
        return ref["hist_out"].astype(np.float32), (pos, nz), n, tf - tt, te - tf, te - ts

    for f in range(f0, f0 + args.cpu_frames):
        hist, prev, n, dt_trace, dt_svgf, dt = frame(f, hist, prev)
        rays += n
        t_trace += dt_trace
        t_svgf += dt_svgf
        t_all += dt
    cores = orc.num_threads()
    # one more frame on one thread
    orc.set_num_threads(1)
    try:
        _, _, n1, _, _, dt1 = frame(f0 + args.cpu_frames, hist, prev)
    finally:
        orc.set_num_threads(cores)
    return {"value": rays / t_all / 1e6, "unit": "Mrays/s", "cores": cores, "kind": "oracle",
            "sample": f"{args.cpu_frames} full {W}x{H} frames of the same workload (G-buffer, rays, SVGF in FP64)",
            "trace_only_mrays_s": rays / t_trace / 1e6,
            "svgf_only_mpix_s": args.cpu_frames * W * H / t_svgf / 1e6,
            "single_thread": {"value": n1 / dt1 / 1e6, "unit": "Mrays/s", "frames": 1}}


if __name__ == "__main__":
    main()
