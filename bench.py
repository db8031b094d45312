#!/usr/bin/env python3
"""Forward + backward throughput of the Gaussian Mesh Renderer hot path on one MI355X.

One step = the whole hot path over one batch: per-face conversion + EWA projection, binning,
(tile | depth) radix sort, tile ranges, front-to-back compositing, the fused L2-loss backward
(reverse-order adjoint, projection and conversion backward, vertex gather); the 2M-face torus
workload also runs the captured Adam step with the lists rebuilt in the backward.  Inputs are
synthetic and resident in HBM before timing.  Prints one JSON line.

  python bench.py [--steps K] [--warmup W] [--config {1..5}] [--gpus 1]

The default workload is the largest single-GPU one: the 2M-face torus, 32 views at 1920x1080, the
100-step Adam vertex optimisation captured as a HIP graph with the lists rebuilt in the backward.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0          # MI355X HBM3E, vendor figure
FP32_VECTOR_TFLOPS_PUBLISHED = 157.3   # MI355X vector FP32, published: packed FP32 (two FMAs per lane)
# What the build can reach: it disables packed FP32, so a lane issues one FMA per clock:
# 256 CUs x 4 SIMDs x 16 lanes x 2 FLOP x 2.4 GHz = 78.6 TFLOP/s
FP32_VECTOR_TFLOPS = 256 * 4 * 16 * 2 * 2.4e9 / 1e12
# Arithmetic per (pixel, Gaussian) pair, counting an FMA as 2: forward = offsets 4, w1/w2 4,
# squared radius 3, exp2 2, clamp/cutoff 2, transmittance 3, weight 1, colour 6 -> 25;
# backward = the forward's 19 up to the cutoff + rcp, T_k, c.g (5), dL/dalpha (4), weight, S (2),
# clamp test, dL/dpower, 5 geometry partials (16), 3 colour partials (6) -> 52.
FLOPS_PER_PAIR = {"raster_fwd": 25, "raster_bwd": 52}


# Measured HBM bytes per launch of the dominant kernels: rocprofv3 --pmc FETCH_SIZE and WRITE_SIZE
# (KiB per dispatch, averaged over the dispatches of one run), each scaled by what the same counter
# reads for the plain copy of --copy-probe.  Keyed by workload, kernel and launch configuration
# (tile, pixels per lane, raster mode, lane lists); `src` is source_hash of the kernel's code when the
# counters were taken, and changed code reports null.
TRAFFIC = {
    ("torus_2M_32x1920x1080", "raster_bwd", "32x16", 1, 0, 1):
        {"fetch": 5748517158, "write": 1797968330, "src": "6ff199d478dfb5b8"},
    ("torus_2M_32x1920x1080", "raster_bwd", "32x32", 1, 0, 1):
        {"fetch": 5703783343, "write": 1797835751, "src": "6ff199d478dfb5b8"},
}
STAGE_SOURCE = {"raster_fwd": "k_raster.hip", "raster_bwd": "k_raster.hip", "sort_fv_pass": "k_sort.hip",
                "sort_pass": "k_sort.hip", "tile_ranges": "k_sort.hip",
                "project": "k_project.hip", "scan_emit": "k_bin.hip", "face_bwd": "k_grad.hip",
                "vertex_gather": "k_grad.hip", "fill": "k_grad.hip", "build_small": "k_project.hip",
                "raster_step": "k_raster.hip"}


def source_hash(stage):
    """Hash of the code (comments and trailing blanks stripped) of a stage's source file and the
    shared header: a change of code makes stored counters stale, a reworded comment does not."""
    import hashlib
    import re
    csrc = os.path.join(ROOT, "paper_2602_14493_amd", "csrc")
    h = hashlib.sha256()
    for f in (STAGE_SOURCE[stage], "gmr_common.h"):
        with open(os.path.join(csrc, f), encoding="utf-8") as fh:
            code = re.sub(r"/\*.*?\*/", "", fh.read(), flags=re.S)
        code = "\n".join(line.split("//", 1)[0].rstrip() for line in code.splitlines())
        h.update(re.sub(r"\n+", "\n", code).strip().encode())
    return h.hexdigest()[:16]


def measured_traffic(workload, stage, tile, px, mode, lanes):
    e = TRAFFIC.get((workload, stage, tile, px, mode, lanes))
    if e is None or e["src"] != source_hash(stage):
        return None
    return e["fetch"] + e["write"]


def copy_peak_gbps(torch, mib: int = 1024, reps: int = 5) -> float:
    """Streaming-copy bandwidth of this GPU (bytes read + written per second, HIP events), the
    measured counterpart of the 8 TB/s vendor figure."""
    n = (mib << 20) // 4
    x = torch.ones(n, device="cuda")
    y = torch.empty_like(x)
    y.copy_(x)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        y.copy_(x)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    del x, y
    return 2.0 * (mib << 20) / (ms * 1e-3) / 1e9


def copy_probe():
    """A plain device-to-device copy of 256 MiB, three launches: FETCH_SIZE / WRITE_SIZE of this copy
    against its known 2^28 bytes each way give the counters' scale."""
    import torch
    n = 64 << 20
    x = torch.ones(n, device="cuda")
    y = torch.empty_like(x)
    torch.cuda.synchronize()
    for _ in range(3):
        y.copy_(x)
    torch.cuda.synchronize()
    print(json.dumps({"copy_probe_bytes_read_per_launch": 4 * n, "copy_probe_bytes_written_per_launch": 4 * n,
                      "launches": 3}))


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--config", type=int, default=5, choices=[1, 2, 3, 4, 5])
    ap.add_argument("--adam-steps", type=int, default=100,
                    help="length of the timed optimisation runs of the Adam workload (each from the start)")
    ap.add_argument("--adam-runs", type=int, default=3)
    ap.add_argument("--no-autotune", action="store_true", help="keep the default tile / block shape")
    ap.add_argument("--tile", type=str, default=None, help="WxH binning tile, e.g. 16x16")
    ap.add_argument("--raster-mode", type=int, default=None)
    ap.add_argument("--px-per-lane", type=int, default=None, choices=[1, 2, 4])
    ap.add_argument("--lane-lists", type=int, default=None, choices=[0, 1])
    ap.add_argument("--sh-degree", type=int, default=0, choices=[0, 1, 2, 3],
                    help="view-dependent colour: coefficient 0 = the workload's colours, the rest N(0, 0.1)")
    ap.add_argument("--cov-mode", type=int, default=0, choices=[0, 1, 2],
                    help="conversion: 0 Eq. 13, 1 Eq. 15, 2 the 3DGS-based edge-frame baseline")
    ap.add_argument("--no-graph", action="store_true",
                    help="Adam workload: launch its step eagerly; others: skip timing the captured step")
    ap.add_argument("--copy-probe", action="store_true",
                    help="only run a plain 256 MiB device copy (calibrates the HBM byte counters)")
    ap.add_argument("--no-per-view", action="store_true")
    ap.add_argument("--no-recon", action="store_true", help="skip timing the full reconstruction step")
    ap.add_argument("--no-fused-step", action="store_true",
                    help="skip timing the optimisation rendered with gmr_render_step_l2 (one list build per step)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=10.0)
    return ap.parse_args()


def progress(msg):
    """One line on stderr per finished phase (stdout carries only the JSON line)."""
    print(f"[bench {time.strftime('%H:%M:%S')}] {msg}", file=sys.stderr, flush=True)


def stage_profile(r):
    import ctypes
    import numpy as np
    from paper_2602_14493_amd import _lib
    names = ctypes.create_string_buffer(32 * 16)
    ms = (ctypes.c_float * 16)()
    cnt = (ctypes.c_int32 * 16)()
    n = ctypes.c_int32()
    _lib.call("gmr_profile_read", r.handle.ptr, 16, names, ms, cnt, ctypes.byref(n))
    out = {}
    raw = names.raw
    for i in range(n.value):
        nm = raw[32 * i:32 * i + 32].split(b"\0")[0].decode()
        out[nm] = (float(ms[i]), int(cnt[i]))
    return out


def byte_model(stage, F, FV, V, P, I, tiles):
    """Algorithmic HBM bytes of one launch group of `stage` (what the stage must move at least)."""
    return {
        "project": F * (12 + 36 + 36) + FV * (48 + 16),        # gathers; records + sort elements
        "sort_fv_pass": FV * 32,                                # 16 B element read + written
        "scan_emit": FV * 16 + I * 8,                           # elements read once; instances written
        "sort_pass": I * 16,                                    # {tile, face-view} read + written
        "tile_ranges": I * 4 + tiles * 8,
        "raster_fwd": I * (4 + 48) + tiles * 8 + P * (12 + 4 + 8),
        "raster_bwd": I * (4 + 48) + tiles * 8 + P * (12 + 12 + 8) + FV * 32,
        "face_bwd": F * (12 + 36 + 48) + FV * 32,
        "vertex_gather": V * 4 + 3 * F * (4 + 12 + 12) + V * 24,
        "fill": FV * 32,
        # the one-launch build of small batches: projection writes, then keys, values and ranges
        "build_small": F * (12 + 36 + 36) + FV * (48 + 16 + 16) + I * 8 + tiles * 8,
    }.get(stage, 0)


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (asked for --gpus {args.gpus}); the path shards by view "
              f"across GPUs as a design, not a run.", file=sys.stderr)
        sys.exit(2)
    import numpy as np
    import torch
    if args.copy_probe:
        copy_probe()
        return

    import paper_2602_14493_amd as gmr
    import workloads as wl

    torch.cuda.set_device(0)
    W = wl.make_workload(args.config)
    progress(f"workload {W.name}: {W.num_views} views, {W.num_pixels} px")
    batch = gmr.Batch.from_workload(W)
    kw = {}
    if args.cov_mode:
        kw["cov_mode"] = args.cov_mode
    if args.sh_degree:
        kw["sh_degree"] = args.sh_degree
    if args.tile:
        tw, th = (int(x) for x in args.tile.lower().split("x"))
        kw.update(tile_w=tw, tile_h=th)
    if args.raster_mode is not None:
        kw["raster_mode"] = args.raster_mode
    if args.px_per_lane is not None:
        kw["px_per_lane"] = args.px_per_lane
    if args.lane_lists is not None:
        kw["lane_lists"] = args.lane_lists
    r = gmr.Renderer(batch, W.faces, gmr.default_options(**kw))
    verts = torch.from_numpy(W.verts).cuda()
    if args.sh_degree:
        K = (args.sh_degree + 1) ** 2
        C = np.zeros((len(W.verts), K, 3), np.float32)
        C[:, 0] = W.colors
        C[:, 1:] = np.random.default_rng(7).normal(0, 0.1, size=(len(W.verts), K - 1, 3))
        colors = torch.from_numpy(C).cuda()
    else:
        colors = torch.from_numpy(W.colors).cuda()
    tverts = torch.from_numpy(W.target_verts).cuda()
    with torch.no_grad():
        target, _, _, _ = r.forward(tverts, colors, check=True)
    target = target.clone()
    tuned_ms = None
    recompute = args.config in (3, 5)
    if not args.no_autotune and not any(k not in ("cov_mode", "sh_degree") for k in kw):
        # more timed iterations where a step is short (the ranking of close candidates is noisy);
        # the tuner times the backward in the form this workload runs (lists rebuilt or reused)
        iters = 10 if W.num_pixels < (1 << 23) else (5 if W.num_pixels < (1 << 25) else 3)
        _, tuned_ms = r.autotune(verts, colors, target, iters=iters, recompute=recompute)
        progress(f"autotuned: tile {r.opts.tile_w}x{r.opts.tile_h}, {tuned_ms:.3f} ms/step")
    use_graph = args.config == 5
    P = W.num_pixels

    # ---- batched form ------------------------------------------------------------------------
    adam_runs = None
    fused_step = None
    if use_graph:
        # the workload's optimiser: Adam on the vertices, lr 1e-3, betas (0.9, 0.999), eps 1e-8.
        # The whole optimisation run goes once, untimed, to size the instance capacity: the peak
        # counter covers every list build of the run; on overflow the capacity grows to the peak
        # plus headroom and the step is captured again
        for attempt in range(4):
            loop = gmr.GraphAdamLoop(r, verts, colors, target, lr=1e-3, recompute=True)
            if not args.no_graph:
                loop.capture()
            start = [t.clone() for t in loop._state()]
            loop.overflow()          # restarts the peak counter
            for _ in range(args.adam_steps):
                loop._step_body() if args.no_graph else loop.graph.replay()
            c = r.counters(loop.ws)
            adam_peak = c.peak_instances
            progress(f"sizing run of {args.adam_steps} optimisation steps: peak {c.peak_instances} instances, "
                     f"capacity {c.capacity}")
            if not (c.overflow or c.overflow_any):
                break
            r.opts.instance_capacity = min((1 << 30) - 1, int(c.peak_instances * r.headroom) + 1024)
            del loop
        else:
            raise RuntimeError("instance capacity did not converge over the optimisation run")

        def reset():
            for t, t0 in zip(loop._state(), start):
                t.copy_(t0)

        def step():
            if args.no_graph:
                loop._step_body()
            else:
                loop.graph.replay()

        def step_profiled():
            loop._step_body()

        reset()
    else:
        # forward + fused L2 backward (with recompute the backward rebuilds the lists into the
        # forward's workspace), launched eagerly; the same step captured as one HIP graph is timed
        # beside it (on these workloads a replay is no faster: the time is in the kernels and the
        # dependency between consecutive launches, not in the host's launch calls)
        gstep = gmr.GraphStep(r, verts, colors, target, recompute=recompute)
        ws = gstep.ws
        step = gstep._step_body
        step_profiled = gstep._step_body
    for _ in range(args.warmup):
        step()
    if use_graph:
        reset()       # the timed steps are the first steps of the optimisation run
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(args.steps):
        step()
    e1.record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms_step = e0.elapsed_time(e1) / args.steps
    value = P / (ms_step * 1e-3) / 1e6
    # per-step spread (a second pass of the same steps, one event pair per step)
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(args.steps)]
    for a_, b_ in ev:
        a_.record()
        step()
        b_.record()
    torch.cuda.synchronize()
    per_step = np.array([a_.elapsed_time(b_) for a_, b_ in ev])
    spread = {"p10": round(float(np.percentile(per_step, 10)), 4), "p50": round(float(np.median(per_step)), 4),
              "p90": round(float(np.percentile(per_step, 90)), 4)}
    # the same step replayed from a captured HIP graph
    ms_graph = None
    if not use_graph and not args.no_graph:
        gstep.capture()
        for _ in range(2):
            gstep.graph.replay()
        e0.record()
        for _ in range(args.steps):
            gstep.graph.replay()
        e1.record()
        torch.cuda.synchronize()
        ms_graph = round(e0.elapsed_time(e1) / args.steps, 4)
    if not use_graph and not args.no_fused_step:
        # the same step rendered with gmr_render_step_l2 (one list build, compositing and adjoint
        # in one launch), launched eagerly, reported beside the headline
        rgb_f, alpha_f, saved_f = r._alloc_outputs()
        ws_f = r.new_workspace()
        dv_f, dc_f = torch.empty_like(verts), torch.empty_like(colors)
        loss_f = torch.zeros((1,), dtype=torch.float32, device="cuda")

        def fstep():
            r.step_l2_raw(verts, colors, target, 1.0, rgb_f, alpha_f, saved_f, ws_f, dv_f, dc_f, loss_f)
        for _ in range(args.warmup):
            fstep()
        torch.cuda.synchronize()
        e0.record()
        for _ in range(args.steps):
            fstep()
        e1.record()
        torch.cuda.synchronize()
        cf = r.counters(ws_f)
        if cf.overflow or cf.overflow_any:
            raise RuntimeError("instance capacity overflowed during the fused-step timing")
        ms_f = e0.elapsed_time(e1) / args.steps
        fused_step = {"ms_per_step": round(ms_f, 4), "Mpixel_per_s": round(P / (ms_f * 1e-3) / 1e6, 2),
                      "list_builds_per_step": 1, "entry_point": "gmr_render_step_l2", "graph": False}
        progress(f"fused step: {ms_f:.4f} ms/step")
        del ws_f
    ws_ref = loop.ws if use_graph else ws
    cnt = r.counters(ws_ref)
    if cnt.overflow or cnt.overflow_any:
        raise RuntimeError("instance capacity overflowed during the timed steps")
    progress(f"timed {args.steps} steps: {ms_step:.4f} ms/step")
    if use_graph:
        # the workload's own protocol: the whole optimisation run from its start, replayed several
        # times; ms/step = replay time / steps
        runs = []
        for _ in range(args.adam_runs):
            reset()
            torch.cuda.synchronize()
            e0.record()
            for _ in range(args.adam_steps):
                step()
            e1.record()
            torch.cuda.synchronize()
            runs.append(e0.elapsed_time(e1) / args.adam_steps)
        c = r.counters(loop.ws)
        if c.overflow or c.overflow_any:
            raise RuntimeError("instance capacity overflowed during the optimisation runs")
        progress(f"optimisation runs: {[round(x, 4) for x in runs]} ms/step")
        adam_runs = {"steps": args.adam_steps, "runs": args.adam_runs,
                     "ms_per_step": [round(x, 4) for x in runs], "ms_per_step_median": round(float(np.median(runs)), 4),
                     "Mpixel_per_s_median": round(P / (float(np.median(runs)) * 1e-3) / 1e6, 2),
                     "loss_final": float(loop.loss.item()), "peak_instances": int(max(adam_peak, c.peak_instances)),
                     "capacity": int(c.capacity), "lr": 1e-3, "graph": not args.no_graph}
        reset()
        if not args.no_fused_step:
            # the same optimisation rendered with gmr_render_step_l2: one list build per step, the
            # compositing and its adjoint in one launch; first K steps from the start and the whole
            # run, as above (reported beside the headline, which rebuilds the lists in the backward)
            floop = gmr.GraphAdamLoop(r, verts, colors, target, lr=1e-3, recompute=True, fused=True)
            if not args.no_graph:
                floop.capture()
            fstart = [t.clone() for t in floop._state()]

            def freset():
                for t, t0 in zip(floop._state(), fstart):
                    t.copy_(t0)

            def fstep():
                floop._step_body() if args.no_graph else floop.graph.replay()
            floop.overflow()
            torch.cuda.synchronize()
            e0.record()
            for _ in range(args.steps):
                fstep()
            e1.record()
            torch.cuda.synchronize()
            ms_fk = e0.elapsed_time(e1) / args.steps
            fruns = []
            for _ in range(args.adam_runs):
                freset()
                torch.cuda.synchronize()
                e0.record()
                for _ in range(args.adam_steps):
                    fstep()
                e1.record()
                torch.cuda.synchronize()
                fruns.append(e0.elapsed_time(e1) / args.adam_steps)
            if floop.overflow():
                raise RuntimeError("instance capacity overflowed during the fused-step runs")
            fused_step = {"ms_per_step": round(ms_fk, 4), "Mpixel_per_s": round(P / (ms_fk * 1e-3) / 1e6, 2),
                          "adam_ms_per_step_median": round(float(np.median(fruns)), 4),
                          "loss_final": float(floop.loss.item()), "list_builds_per_step": 1,
                          "entry_point": "gmr_render_step_l2", "graph": not args.no_graph}
            progress(f"fused step: {ms_fk:.4f} ms/step (first {args.steps}), runs {[round(x, 4) for x in fruns]}")
            del floop
            reset()

    # ---- per-stage timing (HIP events on the library's stream), same steps ----------------------
    # (the Adam workload's state was reset to its start: these are again its first steps)
    from paper_2602_14493_amd import _lib
    _lib.call("gmr_profile_enable", r.handle.ptr, 1)
    for _ in range(args.steps):
        step_profiled()
    torch.cuda.synchronize()
    prof = stage_profile(r)
    progress("per-stage profile done")
    _lib.call("gmr_profile_enable", r.handle.ptr, 0)
    # instance and pair counts of the last profiled step, which the per-stage rates are taken over
    cnt = r.counters(ws_ref)
    if cnt.overflow or cnt.overflow_any:
        raise RuntimeError("instance capacity overflowed during the profiled steps")
    I = cnt.instances
    pairs = {"raster_fwd": cnt.pairs_fwd, "raster_bwd": cnt.pairs_bwd}
    F, V = batch.num_faces, batch.num_verts
    FV = int(sum(int(W.face_offsets[m + 1] - W.face_offsets[m]) for m in W.view_mesh))
    tiles = int(sum(((w + r.opts.tile_w - 1) // r.opts.tile_w) * ((h + r.opts.tile_h - 1) // r.opts.tile_h)
                    for w, h in batch.sizes))
    stages = {}
    for k, (ms, n) in prof.items():
        if n == 0:
            continue
        avg = ms / n
        b = byte_model(k, F, FV, V, P, I, tiles)
        stages[k] = {"ms_per_launch": round(avg, 4), "launches_per_step": n / args.steps,
                     "ms_per_step": round(ms / args.steps, 4), "alg_GBps": round(b / (avg * 1e-3) / 1e9, 1)}
        if k in FLOPS_PER_PAIR:
            stages[k]["pairs"] = pairs[k]
            stages[k]["alg_TFLOPs"] = round(pairs[k] * FLOPS_PER_PAIR[k] / (avg * 1e-3) / 1e12, 2)
    # model bytes of the whole step against the vendor peak and a measured streaming copy
    model_bytes = sum(byte_model(k, F, FV, V, P, I, tiles) * n / args.steps for k, (ms, n) in prof.items() if n)
    copy_gbps = copy_peak_gbps(torch)
    hbm_model = {"bytes_per_step": int(model_bytes), "GBps": round(model_bytes / (ms_step * 1e-3) / 1e9, 1),
                 "frac_vendor_peak": round(model_bytes / (ms_step * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
                 "copy_GBps": round(copy_gbps, 1),
                 "frac_copy_peak": round(model_bytes / (ms_step * 1e-3) / 1e9 / copy_gbps, 4)}
    dom = max(stages, key=lambda k: stages[k]["ms_per_step"])
    d = stages[dom]
    traffic = measured_traffic(W.name, dom, f"{r.opts.tile_w}x{r.opts.tile_h}", r.opts.px_per_lane,
                               r.opts.raster_mode, r.opts.lane_lists)
    if dom in FLOPS_PER_PAIR:   # compositing kernels: VALU-bound on LDS-broadcast data
        achieved = d["alg_TFLOPs"]
        roofline = {"bound": "alu", "kernel": dom, "achieved": achieved, "peak": round(FP32_VECTOR_TFLOPS, 2),
                    "unit": "TFLOP/s", "frac": round(achieved / FP32_VECTOR_TFLOPS, 6), "traffic": traffic,
                    "peak_note": "unpacked FP32 (packed FP32 is disabled in this build)",
                    "peak_published": FP32_VECTOR_TFLOPS_PUBLISHED,
                    "frac_published": round(achieved / FP32_VECTOR_TFLOPS_PUBLISHED, 6),
                    "flops_per_pair": FLOPS_PER_PAIR[dom], "pairs_per_launch": pairs[dom],
                    "hbm_alg_GBps": d["alg_GBps"], "hbm_frac": round(d["alg_GBps"] / HBM_PEAK_GBS, 4)}
    else:
        achieved = d["alg_GBps"]
        roofline = {"bound": "hbm", "kernel": dom, "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                    "frac": round(achieved / HBM_PEAK_GBS, 6), "traffic": traffic}

    # ---- per-view launches (same work, one launch set per view) -------------------------------
    per_view = None
    if not args.no_per_view and W.num_views > 1:
        rs = []
        for v in range(W.num_views):
            bv = batch.view(v)
            v0, v1, f0, f1 = bv.mesh_range
            rv = gmr.Renderer(bv, W.faces[f0:f1] - v0, gmr.copy_options(r.opts, instance_capacity=0),
                              handle=r.handle)
            vv, cc = verts[v0:v1].contiguous(), colors[v0:v1].contiguous()
            npx = bv.num_pixels
            po = int(W.pixel_offsets()[v])
            tg = target[po:po + npx].contiguous()
            o_rgb, o_a, o_s, o_ws = rv.forward(vv, cc, check=True)
            rs.append((rv, vv, cc, tg, o_rgb, o_a, o_s, o_ws, torch.empty_like(vv), torch.empty_like(cc)))

        def step_pv():
            for (rv, vv, cc, tg, o_rgb, o_a, o_s, o_ws, dv, dc) in rs:
                rv.fwd_raw(vv, cc, o_rgb, o_a, o_s, o_ws)
                rv.bwd_l2_raw(vv, cc, o_rgb, tg, 1.0, o_s, o_ws, 1 if recompute else 0, dv, dc)
        for _ in range(args.warmup):
            step_pv()
        torch.cuda.synchronize()
        e0.record()
        for _ in range(args.steps):
            step_pv()
        e1.record()
        torch.cuda.synchronize()
        ms_pv = e0.elapsed_time(e1) / args.steps
        progress(f"per-view launches: {ms_pv:.4f} ms/step")
        per_view = {"ms_per_step": round(ms_pv, 4), "Mpixel_per_s": round(P / (ms_pv * 1e-3) / 1e6, 2),
                    "batched_speedup": round(ms_pv / ms_step, 3)}

    # ---- the full reconstruction step (Sec. 3.1): colour + silhouette backward, regularisers, ----
    # ---- VectorAdam; captured and replayed like the hot-path step ----------------------------
    recon_step = None
    if not args.no_recon:
        with torch.no_grad():
            _, t_alpha, _, _ = r.forward(tverts, colors)
        sil = (t_alpha > 0.5).float()
        rl = gmr.ReconLoop(r, verts, colors, target, sil, lr=1e-3, recompute=recompute)
        rl.capture()
        for _ in range(args.warmup):
            rl.graph.replay()
        torch.cuda.synchronize()
        e0.record()
        for _ in range(args.steps):
            rl.graph.replay()
        e1.record()
        torch.cuda.synchronize()
        ms_rc = e0.elapsed_time(e1) / args.steps
        if rl.overflow():
            raise RuntimeError("instance capacity overflowed during the reconstruction steps")
        # the step's own kernels beyond the renderer: regularisers + VectorAdam, timed alone
        reg_losses = torch.empty((2,), dtype=torch.float32, device=verts.device)
        e0.record()
        for _ in range(args.steps):
            rl.graph_mesh.regularizers_raw(rl.verts, rl.dV, reg_losses)
            gmr.vector_adam_step(rl.verts, rl.dV, rl.m, rl.v, rl.step_count, 0.0)
        e1.record()
        torch.cuda.synchronize()
        ms_tail = e0.elapsed_time(e1) / args.steps
        progress(f"reconstruction step: {ms_rc:.4f} ms/step")
        recon_step = {"ms_per_step": round(ms_rc, 4), "Mpixel_per_s": round(P / (ms_rc * 1e-3) / 1e6, 2),
                      "overhead_vs_hot_path": round(ms_rc / ms_step, 3),
                      "regularizers_vector_adam_ms": round(ms_tail, 4),
                      "edges": rl.graph_mesh.num_edges, "graph": True,
                      "losses": [round(float(x), 6) for x in rl.losses.cpu().tolist()]}
        del rl
        if not args.no_fused_step:
            # the same step rendered with gmr_render_step_recon (one list build, one compositing launch)
            rf = gmr.ReconLoop(r, verts, colors, target, sil, lr=1e-3, recompute=recompute, fused=True)
            rf.capture()
            for _ in range(args.warmup):
                rf.graph.replay()
            torch.cuda.synchronize()
            e0.record()
            for _ in range(args.steps):
                rf.graph.replay()
            e1.record()
            torch.cuda.synchronize()
            if rf.overflow():
                raise RuntimeError("instance capacity overflowed during the fused reconstruction steps")
            ms_rf = e0.elapsed_time(e1) / args.steps
            recon_step["fused_ms_per_step"] = round(ms_rf, 4)
            progress(f"fused reconstruction step: {ms_rf:.4f} ms/step")
            del rf

    # ---- CPU baseline: the FP64 oracle, forward + adjoint -------------------------------------
    cpu = None
    if not args.no_cpu_baseline:
        import oracle
        views = list(range(W.num_views)) if args.config in (1, 2) else [0]
        sample_px = int(sum(W.cams[v].width * W.cams[v].height for v in views))
        Wsub = W if args.config in (1, 2) else wl._single(W.name, *W.mesh(int(W.view_mesh[0])), [W.cams[0]])
        tg_np = target[:sample_px].cpu().numpy().astype(np.float64) if args.config not in (1, 2) else \
            target.cpu().numpy().astype(np.float64)
        # the same colour model and conversion as the timed GPU step
        prm = oracle.Params(cov_mode=args.cov_mode, sh_degree=args.sh_degree)
        m0 = int(W.view_mesh[0])
        c_all = colors.cpu().numpy()
        c_sub = c_all if args.config in (1, 2) else c_all[int(W.vert_offsets[m0]):int(W.vert_offsets[m0 + 1])]
        t_cpu, reps = 0.0, 0
        while t_cpu < args.cpu_seconds or reps == 0:
            t1 = time.perf_counter()
            o_rgb, o_tf, _, _ = oracle.render_workload(Wsub, prm, colors=c_sub)
            _, g = oracle.l2_loss(o_rgb, tg_np)
            oracle.adjoint_workload(Wsub, g, None, prm, colors=c_sub)
            t_cpu += time.perf_counter() - t1
            reps += 1
            progress(f"oracle rep {reps}: {t_cpu:.1f} s")
        cpu = {"value": round(sample_px * reps / t_cpu / 1e6, 4), "unit": "Mpixel/s", "cores": oracle.num_threads(),
               "kind": "oracle",
               "sample": f"{'all' if args.config in (1, 2) else 'view 0 of'} {W.num_views} views, "
                         f"{sample_px} px, fwd+adjoint, {reps} reps, {t_cpu:.1f} s"}

    out = {
        "metric": "fwd+bwd Mpixel/s (batched)",
        "value": round(value, 3),
        "unit": "Mpixel/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_step, 4),
        "ms_per_step_spread": spread,
        "ms_per_step_graph_replay": ms_graph,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": W.name, "faces": F, "verts": V, "views": W.num_views, "pixels": P,
                   "instances": I, "tile": f"{r.opts.tile_w}x{r.opts.tile_h}", "px_per_lane": r.opts.px_per_lane,
                   "lane_lists": r.opts.lane_lists, "cov_mode": r.opts.cov_mode, "sh_degree": r.opts.sh_degree,
                   "raster_mode": r.opts.raster_mode, "autotune_ms": tuned_ms,
                   "recompute_lists": recompute, "adam_graph": use_graph,
                   "launch": "graph" if (use_graph and not args.no_graph) else "eager"},
        "roofline": roofline,
        "hbm_model": hbm_model,
        "cpu_baseline": cpu,
        "per_view": per_view,
        "adam_optimisation": adam_runs,
        "fused_step": fused_step,
        "recon_step": recon_step,
        "stages": stages,
        "wall_s": round(wall, 3),
    }
    print(json.dumps(out))


if __name__ == "__main__":
    main()
