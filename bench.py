"""Benchmark: forward + backward + Adam iterations per second of the splatting hot path on one MI355X.

Workload (default): 1M Gaussians (SH degree 3) initialised from a synthetic LiDAR scan, 8 keyframes of
mixed resolution (640x512 .. 1280x1024) each rendered as a 3-level image pyramid = 24 views, L1 colour +
0.1 L1 LiDAR-depth loss.  One step = every view forward and backward, then Adam over all parameters.
`value` is the batched step (one HIP-graph replay); the plain per-view launch sequence is timed beside it,
as is the 1M-Gaussian single-keyframe 1280x1024 pyramid.  Prints one JSON line.
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

METRIC = "fwd+bwd splat iters/sec at 1M Gaussians, 1280×1024; batched vs plain"

# Algorithmic VALU lane-operations per (pixel, record) pair of the compositing (the planning budget of the
# hot-path scope: 14 operations + one exp, counted at quarter rate as 4, per evaluated pair; 10 more per
# contributing pair in the forward; 55 + one exp per contributing pair in the backward).
OPS_EVAL = 14 + 4
OPS_CONTRIB_FWD = 10
OPS_CONTRIB_BWD = 55 + 4
# The same work counted from this build's own per-pair code (multiply-add as one, exp and reciprocal as
# four); evaluated pairs are evaluated in both sweeps of the fused kernel.
OWN_EVAL, OWN_CONTRIB_FWD, OWN_CONTRIB_BWD = 19, 9, 37
# MI355X: 256 CUs x 4 SIMD x 16 lanes at 2.4 GHz, one VALU lane-operation per lane per cycle.
ALU_PEAK = 256 * 4 * 16 * 2.4e9
HBM_PEAK = 8.0e12  # bytes/s


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def timed(fn, steps, stream):
    import torch

    start = torch.cuda.Event(enable_timing=True)
    end = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    start.record(stream)
    for _ in range(steps):
        fn()
    end.record(stream)
    end.synchronize()
    return start.elapsed_time(end) / steps


def timed_trials(fn, steps, stream, trials=5):
    """Time exactly `steps` calls as `trials` runs of consecutive calls (equal runs, the last one takes the
    remainder), each bracketed by events after a synchronize; returns the median run's ms per call and every
    run's."""
    if steps < trials:
        sizes = [1] * steps
    else:
        per = steps // trials
        sizes = [per] * (trials - 1) + [steps - per * (trials - 1)]
    runs = [timed(fn, k, stream) for k in sizes]
    return float(sorted(runs)[len(runs) // 2]), runs


def spatial_order(model) -> float:
    """Put the model's Gaussians in Morton order of their means (the library's memory layout for locality; both
    the batched and the plain step use it); returns the milliseconds it took on the device."""
    import torch

    torch.cuda.synchronize()
    s, e = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    s.record()
    model.reorder_spatially()
    e.record()
    e.synchronize()
    return s.elapsed_time(e)


def persistent_step_ms(sc, tile, steps, warmup):
    """The same batched step with the compositing backward's walking kernels launched as persistent grids
    (resident workgroups taking the work items from an atomic counter) instead of one workgroup per item."""
    import torch

    from paper_2411_02703_amd import binding as B
    from paper_2411_02703_amd.step import BatchedStep, GaussianModel

    model = GaussianModel(sc.params(), sc.sh_degree)
    spatial_order(model)
    opts = B.default_opts(tile_w=tile[0], tile_h=tile[1], batch_depth=tile[2], block_w=tile[3], seg_len=tile[4],
                          persistent=1)
    bat = BatchedStep(model, sc.cams, sc.tgt_rgb, sc.tgt_depth, opts=opts)
    bat.capture()
    for _ in range(warmup):
        bat.run()
    bat.finish()
    ms, _ = timed_trials(bat.run, steps, torch.cuda.current_stream())
    bat.finish()
    del bat, model
    torch.cuda.synchronize()
    torch.cuda.empty_cache()
    return ms


def measure(sc, steps, warmup, plain_steps, do_plain, tile=None, peak=False):
    """Autotune (unless tile is given), then time the batched step and optionally the plain sequence; with
    peak, also the peak device memory of each (torch allocations, which hold every library buffer)."""
    import torch

    from paper_2411_02703_amd import autotune
    from paper_2411_02703_amd import binding as B
    from paper_2411_02703_amd.step import BatchedStep, GaussianModel, PlainStep

    stream = torch.cuda.current_stream()
    if tile is None:
        tile, _ = autotune.tune_batched(
            lambda o: BatchedStep(GaussianModel(sc.params(), sc.sh_degree), sc.cams, sc.tgt_rgb, sc.tgt_depth, opts=o),
            sc.n, sc.cams, sc.sh_degree, log=log)
    tile = tuple(tile) + (1, 0, 0)[len(tile) - 2:] if len(tile) < 5 else tuple(tile)
    opts = B.default_opts(tile_w=tile[0], tile_h=tile[1], batch_depth=tile[2], block_w=tile[3], seg_len=tile[4])
    log(f"  configuration: {tile[0]}x{tile[1]} tiles, {tile[2]} records per thread per round, "
        f"block {tile[3]}, seg_len {tile[4]}")
    if peak:
        torch.cuda.synchronize()
        torch.cuda.empty_cache()
        torch.cuda.reset_peak_memory_stats()
    model = GaussianModel(sc.params(), sc.sh_degree)
    t_order = spatial_order(model)
    t0 = time.time()
    bat = BatchedStep(model, sc.cams, sc.tgt_rgb, sc.tgt_depth, opts=opts)
    bat.capture()
    log(f"  batched: capacity {bat.frame.capacity}, capture {time.time() - t0:.1f}s")
    for _ in range(warmup):
        bat.run()
    bat.finish()
    replans = bat.replans
    ms, trials = timed_trials(bat.run, steps, stream)
    bat.finish()
    if bat.replans != replans:
        # the capacity was re-planned inside the timed steps (the map grew): time again at the new capacity
        log(f"  batched: capacity re-planned during timing ({bat.frame.capacity}); timing again")
        replans = bat.replans
        ms, trials = timed_trials(bat.run, steps, stream)
        bat.finish()
        if bat.replans != replans:
            raise RuntimeError("instance capacity re-planned twice during timing")
    res = dict(ms=ms, trials=trials, n_instances=bat.n_instances(), loss=bat.loss(), frame=bat.frame, model=model,
               step=bat, tile=tile, order_ms=t_order)
    if peak:
        res["peak_gb"] = torch.cuda.max_memory_allocated() / 1e9
    log(f"  batched: {ms:.3f} ms/step ({1000 / ms:.2f} it/s), {res['n_instances']} instances")
    if do_plain:
        if peak:
            torch.cuda.synchronize()
            base = torch.cuda.memory_allocated()  # the batched step's buffers, still held
            torch.cuda.reset_peak_memory_stats()
        # the plain sequence starts from the map the batched step has reached, so both are timed on the same
        # state of the map (it changes as it trains); the rows are already in Morton order
        pm = GaussianModel({k: v.detach().cpu().numpy() for k, v in model.p.items()}, sc.sh_degree)
        plain = PlainStep(pm, sc.cams, sc.tgt_rgb, sc.tgt_depth, opts=opts)
        plain.run()
        pms = timed(plain.run, plain_steps, stream)
        res["plain_ms"] = pms
        if peak:
            res["plain_peak_gb"] = (torch.cuda.max_memory_allocated() - base) / 1e9
        log(f"  plain:   {pms:.3f} ms/step ({1000 / pms:.2f} it/s)")
    return res


TRAFFIC_PROFILE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "profiles", "fused_composite_cfg4_traffic.md")


def measured_traffic(tile):
    """HBM bytes per launch of the fused compositing group from the committed counter summary, if it was
    taken for this configuration and the compositing sources have not changed since; else None."""
    import hashlib
    import re

    try:
        text = open(TRAFFIC_PROFILE).read()
    except OSError:
        return None
    fields = dict(re.findall(r"^([\w\[\],-]+): (\S+)$", text, re.M))
    h = hashlib.sha256()
    csrc = os.path.join(os.path.dirname(os.path.abspath(__file__)), "paper_2411_02703_amd", "csrc")
    for f in ("render.hip", "common.h"):
        with open(os.path.join(csrc, f), "rb") as fh:
            h.update(fh.read())
    key = "traffic_bytes_per_launch[" + ",".join(str(x) for x in tile) + "]"
    if fields.get("source_sha256") != h.hexdigest() or key not in fields:
        return None
    return int(fields[key])


def kernel_label(tile):
    tw, th, dp, _, sg = tile
    if sg is not None and sg < 0:
        return f"k_render_bwd<{tw},{th},{dp},fused,loss> (forward sweep + loss + backward sweep)"
    return (f"k_fused_main<{tw},{th},{dp},loss> + k_seg_prefix + k_seg_stop + k_seg_combine + k_seg_bwd (forward "
            f"sweep + loss + backward sweep; tile lists split into depth segments)")


def dominant_kernel(res, steps):
    """Average duration of the fused forward + loss + backward compositing launch, timed with HIP events on
    its stream, and its algorithmic work from the pair counts."""
    import torch

    from paper_2411_02703_amd import binding as B

    fr = res["frame"]
    st = res["step"]
    ev, co = B.gs_count_pairs(fr)
    ms = timed(lambda: B.gs_composite_bwd(fr, None, tgt_rgb=st.tgt_rgb, tgt_depth=st.tgt_depth), steps,
               torch.cuda.current_stream())
    ops = ev * OPS_EVAL + co * (OPS_CONTRIB_FWD + OPS_CONTRIB_BWD)
    own = ev * 2 * OWN_EVAL + co * (OWN_CONTRIB_FWD + OWN_CONTRIB_BWD)
    return dict(ms=ms, evaluated=ev, contributing=co, ops=ops, achieved=ops / (ms * 1e-3), own_ops=own,
                own_achieved=own / (ms * 1e-3))


def stage_times(res, steps):
    """Per-stage launch times of the batched step (eager calls timed with HIP events on their stream) and the
    whole-step roofline: the sum over stages of max(algorithmic bytes / HBM peak, algorithmic lane-ops / ALU
    peak), divided by the measured step time."""
    import numpy as np
    import torch

    from paper_2411_02703_amd import binding as B

    fr, st, model = res["frame"], res["step"], res["model"]
    stream = torch.cuda.current_stream()
    n = model.n
    K = (model.sh_degree + 1) ** 2
    pbytes = 44 + 12 * K
    mask = B.frame_tensor(fr, "vis_mask", n, torch.int64).cpu().numpy().view(np.uint8)
    R = int(np.unpackbits(mask).sum())  # visible (view, Gaussian) records
    I = res["n_instances"]
    # the scope's binning budget: 12 B emitted, 24 B per 8-bit pass of the full (tile, depth) key, 8 B of ranges
    # per instance, whatever sort the implementation uses
    tile_bits = max(1, int(fr.f.n_tiles - 1).bit_length())
    passes = -(-(32 + tile_bits) // 8)
    loss = dict(tgt_rgb=st.tgt_rgb, tgt_depth=st.tgt_depth)
    t = {}
    t["project"] = timed(lambda: B.gs_project(model.ps, fr), steps, stream)
    t["bin"] = timed(lambda: B.gs_bin_tiles(fr, sync_count=False), steps, stream)
    t["composite"] = timed(lambda: B.gs_composite_bwd(fr, None, **loss), steps, stream)
    both = timed(lambda: B.gs_render_bwd_adam(model.ps, fr, None, model.ms, model.vs, model.adam, None, **loss),
                 steps, stream)
    t["project_bwd_adam"] = max(both - t["composite"], 0.0)
    dk = res["dominant"]
    work = {
        "project": dict(bytes=n * pbytes + R * 48, ops=0),
        "bin": dict(bytes=I * (12 + 24 * passes + 8), ops=0),
        "composite": dict(bytes=I * 52, ops=dk["ops"]),
        "project_bwd_adam": dict(bytes=R * (40 + 48) + n * 6 * pbytes, ops=0),
    }
    stages, t_roof = {}, 0.0
    for k, ms in t.items():
        w = work[k]
        roof = max(w["bytes"] / HBM_PEAK, w["ops"] / ALU_PEAK) * 1e3
        t_roof += roof
        stages[k] = {"ms": round(ms, 4), "roofline_ms": round(roof, 4), "frac": round(roof / ms, 4) if ms > 0 else None,
                     "algorithmic_GB": round(w["bytes"] / 1e9, 4), "GB_per_s": round(w["bytes"] / (ms * 1e6), 1)}
        if w["ops"]:
            stages[k]["valu_frac"] = round(w["ops"] / (ms * 1e-3) / ALU_PEAK, 4)
    return dict(stages=stages, t_roof_ms=t_roof, records=R, sort_passes=passes)


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(sc, kf_views, threads=None):
    """The FP32 oracle (tiled mode) on one keyframe pyramid of the 24-view workload against all Gaussians, scaled by
    pixel count to the full step; threads=None uses every host thread."""
    import numpy as np

    import oracle

    n_all = oracle.num_threads()
    if threads is not None:
        oracle.set_threads(threads)
    cams = [sc.cams[i] for i in kf_views]
    offs = np.cumsum([0] + [c.width * c.height for c in sc.cams])
    rgb = np.concatenate([sc.tgt_rgb[3 * offs[i]:3 * offs[i + 1]] for i in kf_views])
    dep = np.concatenate([sc.tgt_depth[offs[i]:offs[i + 1]] for i in kf_views])
    p_sample = sum(c.width * c.height for c in cams)
    used = oracle.num_threads()
    t0 = time.time()
    oracle.backward(32, sc.params(), sc.sh_degree, cams, tgt_rgb=rgb, tgt_depth=dep)
    dt = time.time() - t0
    oracle.set_threads(n_all)
    scale = sc.total_pixels / p_sample
    return dict(value=1.0 / (dt * scale), unit="iters/s", cores=used, kind="oracle", cpu=cpu_model(),
                sample=(f"FP32 oracle forward + loss + backward of views {list(kf_views)} "
                        f"({'+'.join(f'{c.width}x{c.height}' for c in cams)}) against all {sc.n} Gaussians on "
                        f"{used} thread(s): {dt:.2f} s, scaled x{scale:.2f} by pixel count to the full step"))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200, help="timed steps (five runs of steps/5; the median is reported)")
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--plain-steps", type=int, default=5)
    ap.add_argument("--no-plain", action="store_true")
    ap.add_argument("--no-persistent", action="store_true",
                    help="skip timing the persistent-grid variant of the compositing launches")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-cfg3", action="store_true")
    ap.add_argument("--no-cfg5", action="store_true",
                    help="skip the large map (4M Gaussians, 16 keyframes x 3 levels; about a minute of scene "
                         "generation on the host)")
    ap.add_argument("--n", type=int, default=None, help="override the Gaussian count (smaller trial runs)")
    ap.add_argument("--tile", type=str, default=None,
                    help="tile_w,tile_h[,batch_depth,block_w,seg_len] (skips the autotuner)")
    ap.add_argument("--copy-calib", type=int, default=0, metavar="MIB",
                    help="also run a plain copy kernel over MIB MiB three times (the known-size kernel that scales "
                         "FETCH_SIZE / WRITE_SIZE counters to bytes)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py measures one GPU: this build has no multi-GPU path (see DESIGN.md on sharding by view).",
              file=sys.stderr)
        sys.exit(2)

    import torch

    from paper_2411_02703_amd import binding as B
    from paper_2411_02703_amd import scenes

    B.load()
    log(f"device: {torch.cuda.get_device_name(0)}; host threads {os.cpu_count()}")
    t0 = time.time()
    sc4 = scenes.config(4, n=args.n)
    log(f"cfg4 scene: {sc4.n} Gaussians, {len(sc4.cams)} views, {sc4.total_pixels} px ({time.time() - t0:.1f}s)")
    tile = None
    if args.tile:
        parts = args.tile.split(",")
        tile = tuple(int(x) for x in parts)
    r4 = measure(sc4, args.steps, args.warmup, args.plain_steps, not args.no_plain, tile)
    dk = dominant_kernel(r4, args.steps)
    r4["dominant"] = dk
    log(f"  fused compositing kernel: {dk['ms']:.3f} ms, {dk['evaluated']} evaluated / {dk['contributing']} "
        f"contributing pairs, {dk['achieved'] / 1e12:.2f} T lane-ops/s")
    stg = stage_times(r4, args.steps)
    for k, v in stg["stages"].items():
        log(f"  stage {k}: {v['ms']:.3f} ms, roofline {v['roofline_ms']:.3f} ms ({v['frac']:.3f})")
    pers_ms = None
    if not args.no_persistent and r4["tile"][4] >= 0:
        pers_ms = persistent_step_ms(sc4, r4["tile"], args.steps, args.warmup)
        log(f"  persistent compositing launches: {pers_ms:.3f} ms/step (work-item grids {r4['ms']:.3f})")
    if args.copy_calib > 0:
        src = torch.ones(args.copy_calib << 18, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            torch.mul(src, 1.0, out=dst)  # one elementwise kernel: reads and writes MIB MiB
        torch.cuda.synchronize()
        log(f"  copy calibration: 3 x {args.copy_calib} MiB device copies")
        del src, dst
    out = {
        "metric": METRIC,
        "value": round(1000.0 / r4["ms"], 3),
        "unit": "iters/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(r4["ms"], 4),
        "ms_per_step_runs": [round(x, 4) for x in r4["trials"]],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": ("batched step: 1M Gaussians (SH degree 3) from a synthetic LiDAR scan, 8 keyframes "
                                "640x512..1280x1024 x 3-level pyramid = 24 views, L1 RGB + 0.1 L1 depth, Adam; "
                                "one HIP-graph replay per step"),
                   "gaussians": sc4.n, "views": len(sc4.cams), "pixels": sc4.total_pixels,
                   "instances": r4["n_instances"], "tile": list(r4["tile"][:2]), "batch_depth": r4["tile"][2],
                   "block_w": r4["tile"][3], "seg_len": r4["tile"][4],
                   "layout": "Gaussians in Morton order of their means (one-time reorder, "
                             f"{r4['order_ms']:.2f} ms, outside the timed steps)"},
    }
    if pers_ms is not None:
        out["persistent_launch"] = {"ms_per_step": round(pers_ms, 4), "over_work_item_grids": round(pers_ms / r4["ms"], 3),
                                    "scheme": "walking kernels as grids of resident workgroups taking work items "
                                              "from an atomic counter (timed as a departure check; not the default)"}
    if "plain_ms" in r4:
        out["plain"] = {"value": round(1000.0 / r4["plain_ms"], 3), "ms_per_step": round(r4["plain_ms"], 4),
                        "steps": args.plain_steps}
        out["batched_over_plain"] = round(r4["plain_ms"] / r4["ms"], 3)
    out["roofline"] = {"bound": "alu", "achieved": round(dk["achieved"] / 1e12, 3), "peak": round(ALU_PEAK / 1e12, 3),
                       "unit": "T lane-op/s", "frac": round(dk["achieved"] / ALU_PEAK, 4),
                       "traffic": measured_traffic(r4["tile"]),
                       "kernel": kernel_label(r4["tile"]),
                       "kernel_ms": round(dk["ms"], 4), "pairs_evaluated": dk["evaluated"],
                       "pairs_contributing": dk["contributing"],
                       "ops_per_pair": {"evaluated": OPS_EVAL, "contributing_fwd": OPS_CONTRIB_FWD,
                                        "contributing_bwd": OPS_CONTRIB_BWD},
                       "frac_own_count": round(dk["own_achieved"] / ALU_PEAK, 4)}
    out["step_roofline"] = {"t_roof_ms": round(stg["t_roof_ms"], 4), "frac": round(stg["t_roof_ms"] / r4["ms"], 4),
                            "hbm_peak_GB_s": HBM_PEAK / 1e9, "alu_peak_T_lane_op_s": round(ALU_PEAK / 1e12, 3),
                            "records": stg["records"], "budget_sort_passes": stg["sort_passes"], "stages": stg["stages"]}
    if not args.no_cfg3:
        sc3 = scenes.config(3, n=args.n)
        log(f"cfg3 scene: {len(sc3.cams)} views, {sc3.total_pixels} px")
        r3 = measure(sc3, args.steps, args.warmup, args.plain_steps, not args.no_plain, tile)
        out["single_keyframe_1280x1024_pyramid"] = {"batched": round(1000.0 / r3["ms"], 3)}
        if "plain_ms" in r3:
            out["single_keyframe_1280x1024_pyramid"]["plain"] = round(1000.0 / r3["plain_ms"], 3)
    if not args.no_cfg5:
        t0 = time.time()
        sc5 = scenes.config(5, n=None if args.n is None else 4 * args.n)
        log(f"cfg5 scene: {sc5.n} Gaussians, {len(sc5.cams)} views, {sc5.total_pixels} px ({time.time() - t0:.1f}s)")
        torch.cuda.empty_cache()
        r5 = measure(sc5, max(5, args.steps // 4), args.warmup, 3, not args.no_plain, r4["tile"], peak=True)
        out["large_map_4M"] = {
            "workload": "4M Gaussians (SH degree 3) over a 200 m x 200 m LiDAR scene, 16 keyframes 640x512..1280x1024 "
                        "x 3 levels = 48 views; per-pixel state recomputed in the backward",
            "pixels": sc5.total_pixels, "instances": r5["n_instances"], "tile": list(r5["tile"]),
            "batched": {"value": round(1000.0 / r5["ms"], 3), "ms_per_step": round(r5["ms"], 4),
                        "peak_memory_gb": round(r5["peak_gb"], 3)}}
        if "plain_ms" in r5:
            out["large_map_4M"]["plain"] = {"value": round(1000.0 / r5["plain_ms"], 3),
                                            "ms_per_step": round(r5["plain_ms"], 4),
                                            "peak_memory_gb": round(r5["plain_peak_gb"], 3)}
            out["large_map_4M"]["batched_over_plain"] = round(r5["plain_ms"] / r5["ms"], 3)
        del sc5, r5
    if not args.no_cpu:
        big = max(range(0, len(sc4.cams), 3), key=lambda i: sc4.cams[i].width)
        small = min(range(0, len(sc4.cams), 3), key=lambda i: sc4.cams[i].width * sc4.cams[i].height)
        out["cpu_baseline"] = cpu_baseline(sc4, [big, big + 1, big + 2])
        # one thread, on the smallest keyframe's pyramid (about a quarter of the pixels) to bound its time
        out["cpu_baseline"]["single_thread"] = cpu_baseline(sc4, [small, small + 1, small + 2], threads=1)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
