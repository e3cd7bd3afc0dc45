#!/usr/bin/env python3
"""Benchmark of the terrain ray caster on one MI355X.

Headline workload: the 2048x2048 two-layer map (30% two-layer cells, sharp
40-unit cliffs) and one 1920x1080 eye-level horizon view looking along +y.
A step is one frame: one tc_render_views call casting all 2,073,600 rays
with the map and pyramid already resident in HBM.  Prints one JSON line.

    python bench.py [--steps 40] [--warmup 5] [--mode hier|flat|persistent]
                    [--no-cpu] [--extra]
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

PEAK_HBM_GBS = 8000.0
MODES = {"hier": 0, "flat": 1, "persistent": 2}


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def time_renders(torch, ctx, tc, views, out, steps, warmup):
    """Per-step HIP event timings (ms) of tc_render_views on the current
    stream, plus the bracketed wall time of all timed steps."""
    for _ in range(warmup):
        ctx.tc_render_views(views, out.data_ptr())
    torch.cuda.synchronize()
    starts = [torch.cuda.Event(enable_timing=True) for _ in range(steps)]
    ends = [torch.cuda.Event(enable_timing=True) for _ in range(steps)]
    t0 = time.perf_counter()
    for k in range(steps):
        starts[k].record()
        ctx.tc_render_views(views, out.data_ptr())
        ends[k].record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms = np.array([s.elapsed_time(e) for s, e in zip(starts, ends)])
    return ms, wall


def cpu_baseline(oracle, F, B, T, views, rays_per_frame, budget_s=12.0):
    """The CPU oracle on the host cores, on repeated renders of the same
    view until about budget_s seconds of wall time have passed."""
    try:
        cores = len(os.sched_getaffinity(0))
    except AttributeError:
        cores = os.cpu_count() or 1
    done = 0
    t0 = time.perf_counter()
    while True:
        oracle.render(F, B, T, views, threads=cores)
        done += 1
        if time.perf_counter() - t0 >= budget_s:
            break
    dt = time.perf_counter() - t0
    return {"value": done * rays_per_frame / dt / 1e9, "unit": "Grays/s",
            "cores": cores, "kind": "oracle",
            "sample": "%d full renders of the 1920x1080 headline view (%.1f s)" % (done, dt)}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=40)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--mode", default="hier", choices=list(MODES))
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--extra", action="store_true",
                    help="also time every render mode")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU; --gpus %d is not supported (the method "
              "shards by replicating the map and splitting views across GPUs, "
              "which this build does not run)" % args.gpus, file=sys.stderr)
        sys.exit(2)

    import torch
    import paper_2608_17390_amd as tc
    import synth

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    log("[bench] generating the 2048x2048 map")
    F, B, T = synth.make_map_from_config(2)
    views = synth.config_views(2, F, B)
    rays = synth.view_rays(views)
    ctx = tc.Context(0)
    ctx.tc_load_columns(F, B, T)
    torch.cuda.synchronize()
    out = torch.empty((rays, 2), dtype=torch.int32, device="cuda")
    ctx.tc_set_option(tc.TC_OPT_RENDER_MODE, MODES[args.mode])

    # algorithmic bytes: node/cell reads counted by the library itself
    ctx.tc_set_option(tc.TC_OPT_COUNT_READS, 1)
    ctx.tc_render_views(views, out.data_ptr())
    reads = ctx.tc_read_counters()
    ctx.tc_set_option(tc.TC_OPT_COUNT_READS, 0)
    alg_bytes = 8 * rays + 4 * reads
    log("[bench] %d rays, %d node/cell reads (%.1f per ray)" % (rays, reads, reads / rays))

    log("[bench] timing %d steps after %d warmup, mode %s" % (args.steps, args.warmup, args.mode))
    ms, wall = time_renders(torch, ctx, tc, views, out, args.steps, args.warmup)
    ms_per_step = wall * 1e3 / args.steps
    med = float(np.median(ms))
    avg = float(ms.mean())
    achieved = alg_bytes / (avg * 1e-3) / 1e9
    res = {
        "metric": "Grays/s and ms/frame @1920x1080 eye-level; batched vs plain p99 latency",
        "value": rays / (ms_per_step * 1e-3) / 1e9,
        "unit": "Grays/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "int64",
        "data": "synthetic",
        "config": {"workload": "c2: 2048x2048 two-layer map (30% two-layer cells, "
                               "40-unit cliffs), one 1920x1080 eye-level horizon view",
                   "rays_per_frame": rays, "render_mode": args.mode,
                   "frame_ms_median": med, "frame_ms_p99": float(np.percentile(ms, 99))},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": PEAK_HBM_GBS,
                     "unit": "GB/s", "frac": achieved / PEAK_HBM_GBS, "traffic": None,
                     "kernel": "render_kernel<false>" if args.mode == "hier" else args.mode,
                     "alg_bytes_per_launch": alg_bytes,
                     "kernel_ms_avg": avg},
    }
    if args.extra:
        modes = {}
        for m in MODES:
            ctx.tc_set_option(tc.TC_OPT_RENDER_MODE, MODES[m])
            mm, _ = time_renders(torch, ctx, tc, views, out, 10, 2)
            modes[m] = float(np.median(mm))
        res["mode_ms_median"] = modes
    if not args.no_cpu:
        import oracle
        log("[bench] CPU oracle baseline")
        res["cpu_baseline"] = cpu_baseline(oracle, F, B, T, views, rays)
    print(json.dumps(res), flush=True)
    ctx.close()


if __name__ == "__main__":
    main()
