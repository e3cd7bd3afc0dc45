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
# the sources of the headline traversal kernels (the committed profiles
# record their hash)
RENDER_SRCS = [os.path.join(ROOT, "paper_2608_17390_amd", "csrc", f)
               for f in ("tc_walk.h", "tc_beam.h", "tc_packet.h", "tc_render.hip")]
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

PEAK_HBM_GBS = 8000.0
MODES = {"hier": 0, "flat": 1, "persistent": 2, "march": 3, "occupancy": 4}
# (render mode 5, the voxel-accelerated march, needs its pyramid: it is
# timed in occupancy_compare)
KERNEL_NAMES = {"hier": "render_hier_kernel + split_kernel (one traversal)",
                "flat": "render_flat_kernel", "persistent": "render_persistent_kernel",
                "march": "march_kernel", "occupancy": "render_occ_kernel"}
PROTOCOL_SEED = 6000      # poses of the twelve protocol views


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def profile_value(kernel_srcs, name, key):
    """A figure measured by rocprofv3 and committed under profiles/ (the
    line `key: value` of profiles/<name>.txt), if that profile was taken on
    the current render sources (its render_source_sha256 line matches the
    sha256 over the files in order); else None."""
    import hashlib
    path = os.path.join(ROOT, "profiles", "%s.txt" % name)
    if not os.path.exists(path):
        return None
    try:
        keys = {}
        for line in open(path):
            k, sep, v = line.partition(":")
            if sep and k.strip() in ("render_source_sha256", key):
                keys[k.strip()] = v.strip()
        h = hashlib.sha256()
        for f in kernel_srcs:
            h.update(open(f, "rb").read())
        if keys.get("render_source_sha256") != h.hexdigest():
            return None
        return float(keys[key])
    except (ValueError, KeyError, OSError):
        return None


def calib_copy(torch, mib=256, reps=3):
    """A plain device-to-device copy of known size, for counter scaling."""
    a = torch.empty(mib << 18, dtype=torch.float32, device="cuda").fill_(1.0)
    b = torch.empty_like(a)
    for _ in range(reps):
        b.copy_(a)
    torch.cuda.synchronize()
    return mib << 20


def time_renders(torch, ctx, tc, views, out, steps, warmup):
    """The timed region: `steps` back-to-back tc_render_views calls on the
    current stream, bracketed by synchronisations (wall time); then as many
    again with HIP events around each call (per-step ms, for the median and
    p99).  Views are converted to C structures once, outside both."""
    vs = tc.views_struct(views)
    for _ in range(warmup):
        ctx.tc_render_views(vs, out.data_ptr())
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        ctx.tc_render_views(vs, out.data_ptr())
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    starts = [torch.cuda.Event(enable_timing=True) for _ in range(steps)]
    ends = [torch.cuda.Event(enable_timing=True) for _ in range(steps)]
    for k in range(steps):
        starts[k].record()
        ctx.tc_render_views(vs, out.data_ptr())
        ends[k].record()
    torch.cuda.synchronize()
    ms = np.array([s.elapsed_time(e) for s, e in zip(starts, ends)])
    return ms, wall


def kernel_times(torch, ctx, tc, views, out, steps):
    """(traversal kernel ms, split pass ms) of each of `steps` renders,
    from the HIP events the library attaches to its kernels (or records
    around them, for calls whose tables are uploaded)."""
    ctx.tc_set_option(tc.TC_OPT_KERNEL_TIMING, 1)
    rows = []
    vs = tc.views_struct(views)
    for _ in range(steps):
        ctx.tc_render_views(vs, out.data_ptr())
        rows.append(ctx.tc_read_kernel_times())
    ctx.tc_set_option(tc.TC_OPT_KERNEL_TIMING, 0)
    torch.cuda.synchronize()
    return np.array(rows, dtype=np.float64)


def cpu_model():
    """The host CPU's model name (from /proc/cpuinfo), or None."""
    try:
        for line in open("/proc/cpuinfo"):
            if line.lower().startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def cpu_baseline(oracle, F, B, T, views, rays_per_frame, budget_s=12.0, single_s=5.0):
    """The CPU oracle on the host cores, on repeated renders of the same
    view until about budget_s seconds of wall time have passed; then on one
    thread for about single_s seconds."""
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
    # one thread: whole renders of the same view until single_s has passed
    done1 = 0
    t1 = time.perf_counter()
    while True:
        oracle.render(F, B, T, views, threads=1)
        done1 += 1
        if time.perf_counter() - t1 >= single_s:
            break
    dt1 = time.perf_counter() - t1
    return {"value": done * rays_per_frame / dt / 1e9, "unit": "Grays/s",
            "cores": cores, "kind": "oracle", "cpu_model": cpu_model(),
            "sample": "%d full renders of the 1920x1080 headline view on %d threads (%.1f s)"
                      % (done, cores, dt),
            "single_thread_value": done1 * rays_per_frame / dt1 / 1e9,
            "single_thread_sample": "%d full renders of the same view on one thread (%.1f s)"
                                    % (done1, dt1)}


def c3_frame(torch, tc, synth, steps, warmup):
    """Configuration 3: 64 size-32 craters, dirty pyramid update, then the
    2560x1440 grazing and 1920x1080 oblique views, as one captured frame,
    with the knobs the autotuner picks for the frame's views (the frame with
    the default knobs is timed first and reported beside it)."""
    from paper_2608_17390_amd import tune
    F, B, T = synth.make_map_from_config(3)
    H, W = F.shape
    views = synth.config_views(3, F, B)
    edits = synth.crater_list(synth.SEEDS[3]["edits"], W, H, 64, size=32)
    rays = synth.view_rays(views)
    ctx = tc.Context(0)
    ctx.tc_load_columns(F, B, T)
    out = torch.empty((rays, 2), dtype=torch.int32, device="cuda")

    def run():
        frame = ctx.tc_frame_create(views, edits, out.data_ptr())
        for _ in range(warmup):
            frame.launch()
        torch.cuda.synchronize()
        ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
              for _ in range(steps)]
        for a, b in ev:
            a.record()
            frame.launch()
            b.record()
        torch.cuda.synchronize()
        frame.close()
        return np.array([a.elapsed_time(b) for a, b in ev])

    ms_default = run()
    knobs, cached = tune.autotune(ctx, views, out.data_ptr(), "c3-frame")
    log("[bench] c3 knobs %s (cached %s)" % (knobs, cached))
    ms = run()
    ctx.close()
    return {"workload": "c3: 2048x16384 map, 64 craters + dirty update + 2560x1440 "
                        "grazing + 1920x1080 oblique views, one graph launch",
            "rays_per_frame": rays, "frame_ms_median": float(np.median(ms)),
            "frame_ms_p99": float(np.percentile(ms, 99)),
            "grays_per_s": rays / (np.median(ms) * 1e-3) / 1e9, "knobs": knobs,
            "default_knobs": {"frame_ms_median": float(np.median(ms_default)),
                              "frame_ms_p99": float(np.percentile(ms_default, 99))}}


def march_protocol(torch, tc, synth, steps, warmup):
    """The sampled march of Section 3.1 at the paper's setting (128 samples,
    4 halvings, far 600) on the views of its measurement protocol (Section
    4.3: twelve 1280x800 views, three per pitch 0, -30, -60, -90 degrees)
    over the 2048x16384 map.  Per view: march and exact render times, the
    time of a complete shaded frame (exact render + shading pass with a
    shadow ray per lit pixel), and the quality metrics of Section 4.2 of the
    march against the exact cast (a hit beyond the far limit counts as
    background), averaged per pitch as the paper reports them."""
    from paper_2608_17390_amd import metrics
    F, B, T = synth.make_map_from_config(3)
    views, pitches = synth.pitch_views(F, B, PROTOCOL_SEED)
    ctx = tc.Context(0)
    ctx.tc_load_columns(F, B, T)
    n = 1280 * 800
    outs = {m: [torch.empty((n, 2), dtype=torch.int32, device="cuda") for _ in views]
            for m in ("march", "hier")}
    times = {}
    kern = {}
    for m in ("march", "hier"):
        ctx.tc_set_option(tc.TC_OPT_RENDER_MODE, MODES[m])
        per_view = []
        kv = []
        for v, out in zip(views, outs[m]):
            ms, _ = time_renders(torch, ctx, tc, [v], out, steps, warmup)
            per_view.append(float(np.median(ms)))
            kv.append(kernel_times(torch, ctx, tc, [v], out, steps).sum(axis=1).mean())
        times[m] = per_view
        kern[m] = kv
    # a complete frame: exact render then the shading pass (shadow ray per
    # lit pixel, palette, gradient normal, fog), as the paper's frames shade
    # every method the same way
    pal = synth.default_palette()
    light = (1 << 16, 2 << 16, 2 << 16)
    rgba = torch.empty(n, dtype=torch.int32, device="cuda")
    ctx.tc_set_option(tc.TC_OPT_RENDER_MODE, MODES["hier"])
    shaded = []
    for v, out in zip(views, outs["hier"]):
        for _ in range(warmup):
            ctx.tc_render_views([v], out.data_ptr())
            ctx.tc_shade_views([v], out.data_ptr(), light, pal, rgba.data_ptr())
        torch.cuda.synchronize()
        ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
              for _ in range(steps)]
        for a0, b0 in ev:
            a0.record()
            ctx.tc_render_views([v], out.data_ptr())
            ctx.tc_shade_views([v], out.data_ptr(), light, pal, rgba.data_ptr())
            b0.record()
        torch.cuda.synchronize()
        shaded.append(float(np.median([a0.elapsed_time(b0) for a0, b0 in ev])))
    times["shaded"] = shaded
    # the shading kernel alone: HIP events the library records around it,
    # and its algorithmic bytes (8 B hit record in, 4 B colour out, 4 B per
    # column, gradient neighbour and shadow-ray node or cell read)
    ctx.tc_set_option(tc.TC_OPT_KERNEL_TIMING, 1)
    shade_k = []
    for v, out in zip(views, outs["hier"]):
        ctx.tc_render_views([v], out.data_ptr())
        for _ in range(steps):
            ctx.tc_shade_views([v], out.data_ptr(), light, pal, rgba.data_ptr())
            shade_k.append(ctx.tc_read_kernel_times()[0])
    ctx.tc_set_option(tc.TC_OPT_KERNEL_TIMING, 0)
    ctx.tc_set_option(tc.TC_OPT_COUNT_READS, 1)
    ctx.tc_read_counters()
    for v, out in zip(views, outs["hier"]):
        ctx.tc_render_views([v], out.data_ptr())
    ctx.tc_read_counters()
    for v, out in zip(views, outs["hier"]):
        ctx.tc_shade_views([v], out.data_ptr(), light, pal, rgba.data_ptr())
    shade_reads = ctx.tc_read_counters()
    ctx.tc_set_option(tc.TC_OPT_COUNT_READS, 0)
    shade_alg = (12 * n * len(views) + 4 * shade_reads) / len(views)
    shade_ms = float(np.mean(shade_k))
    # algorithmic bytes of the march: 8 B per hit record + 4 B per column
    # sample read over the map (the library's own count)
    ctx.tc_set_option(tc.TC_OPT_RENDER_MODE, MODES["march"])
    ctx.tc_set_option(tc.TC_OPT_COUNT_READS, 1)
    ctx.tc_read_counters()
    for v, out in zip(views, outs["march"]):
        ctx.tc_render_views([v], out.data_ptr())
    samples = ctx.tc_read_counters()
    ctx.tc_set_option(tc.TC_OPT_COUNT_READS, 0)
    torch.cuda.synchronize()
    q = []
    for k, v in enumerate(views):
        wm, dm = tc.split_hits(outs["march"][k])
        we, de = tc.split_hits(outs["hier"][k])
        q.append(metrics.quality(wm, dm, we, de, 1280, 800, far=600.0))
    per_pitch = {}
    for p in sorted(set(pitches), reverse=True):
        ks = [k for k, pk in enumerate(pitches) if pk == p]
        per_pitch[str(p)] = {
            "march_ms": float(np.mean([times["march"][k] for k in ks])),
            "exact_ms": float(np.mean([times["hier"][k] for k in ks])),
            "exact_shaded_frame_ms": float(np.mean([times["shaded"][k] for k in ks])),
            "see_through_pct": 100 * float(np.mean([q[k]["see_through"] for k in ks])),
            "covers_sky_pct": 100 * float(np.mean([q[k]["covers_sky"] for k in ks])),
            "coherence_pct": 100 * float(np.mean([q[k]["coherence"] for k in ks])),
            "depth_err_median": float(np.mean([q[k]["depth_err_median"] for k in ks])),
            "depth_err_p95": float(np.mean([q[k]["depth_err_p95"] for k in ks])),
        }
    alg = 8 * n * len(views) + 4 * samples
    kms = float(np.sum(kern["march"]))
    ctx.close()
    return {"workload": "protocol: 2048x16384 map, twelve 1280x800 views (3 per pitch "
                        "0/-30/-60/-90), march 128 samples + 4 halvings, far 600",
            "march_ms_per_view": float(np.mean(times["march"])),
            "exact_ms_per_view": float(np.mean(times["hier"])),
            "exact_shaded_frame_ms": float(np.mean(times["shaded"])),
            "march_grays_per_s": n / (np.mean(times["march"]) * 1e-3) / 1e9,
            "exact_grays_per_s": n / (np.mean(times["hier"]) * 1e-3) / 1e9,
            "samples_per_ray": samples / (n * len(views)),
            "march_roofline": {"bound": "hbm", "achieved": alg / (kms * 1e-3) / 1e9,
                               "peak": PEAK_HBM_GBS, "unit": "GB/s",
                               "frac": alg / (kms * 1e-3) / 1e9 / PEAK_HBM_GBS,
                               "alg_bytes_per_view": alg / len(views),
                               "kernel_ms_per_view": kms / len(views)},
            "shade_roofline": {"bound": "hbm", "achieved": shade_alg / (shade_ms * 1e-3) / 1e9,
                               "peak": PEAK_HBM_GBS, "unit": "GB/s",
                               "frac": shade_alg / (shade_ms * 1e-3) / 1e9 / PEAK_HBM_GBS,
                               "alg_bytes_per_view": shade_alg,
                               "kernel_ms_per_view": shade_ms,
                               "reads_per_pixel": shade_reads / (n * len(views))},
            "per_pitch": per_pitch}


CAVE_SEED = 6002          # the cave-heavy comparison map


def voxel_bytes(ctx):
    """Bytes of the context's voxel occupancy pyramid (Morton tiles of 64 B)."""
    n = ctx.tc_voxel_dims(0)[3]
    total = 0
    for k in range(n):
        nx, ny, nz, _ = ctx.tc_voxel_dims(k)
        total += ((nx + 7) // 8) * ((ny + 7) // 8) * ((nz + 7) // 8) * 64
    return total


def occupancy_compare(torch, tc, synth, steps, warmup):
    """The 2D min/max pyramid (render mode 0, with and without its split
    pass) against the same walk with occupancy masks (mode 4) and against
    the voxel-accelerated march over the voxel occupancy pyramid (mode 5,
    Section 3.2, voxels of 4x4 cells by 2 units and 2x2 by 1, the paper's
    coarse and shipping proportions with square footprints): frame time,
    node/cell/voxel-word reads per ray and structure size, on a cave-heavy
    2048x2048 map (half the cells two-layer) and on the headline map.  The
    packet beam (which reads the window levels) is on in every row, and off
    in the last two."""
    out = {}
    cases = {"cave": synth.cave_map(CAVE_SEED, 2048, 2048),
             "c2": synth.make_map_from_config(2)}
    rows = (("pyramid_split", 0, 128, 0, 4), ("pyramid", 0, 0, 0, 4), ("occupancy", 4, 0, 0, 4),
            ("rayvoxel_4x4x2", 5, 0, 4 | (2 << 8), 4), ("rayvoxel_2x2x1", 5, 0, 2 | (1 << 8), 4),
            ("pyramid_nobeam", 0, 0, 0, 0), ("rayvoxel_4x4x2_nobeam", 5, 0, 4 | (2 << 8), 0))
    for name, (F, B, T) in cases.items():
        ctx = tc.Context(0)
        ctx.tc_load_columns(F, B, T)
        views = ([synth.perspective_view(synth.eye_above_floor(F, B, 1024.5, 32.5), 0, 0, 1920, 1080),
                  synth.perspective_view((1024.5, 600.5, 330.0), 0, -40, 1920, 1080)]
                 if name == "cave" else synth.config_views(2, F, B))
        rays = synth.view_rays(views)
        buf = torch.empty((rays, 2), dtype=torch.int32, device="cuda")
        res = {}
        for label, mode, budget, vox, beam in rows:
            ctx.tc_set_option(tc.TC_OPT_VOXEL_SHAPE, vox)
            ctx.tc_set_option(tc.TC_OPT_RENDER_MODE, mode)
            ctx.tc_set_option(tc.TC_OPT_SPLIT_BUDGET, budget)
            ctx.tc_set_option(tc.TC_OPT_BEAM_PASSES, beam)
            ms, _ = time_renders(torch, ctx, tc, views, buf, steps, warmup)
            ctx.tc_set_option(tc.TC_OPT_COUNT_READS, 1)
            ctx.tc_read_counters()
            ctx.tc_render_views(views, buf.data_ptr())
            reads = ctx.tc_read_counters()
            ctx.tc_set_option(tc.TC_OPT_COUNT_READS, 0)
            res[label] = {"frame_ms_median": float(np.median(ms)),
                          "grays_per_s": rays / (np.median(ms) * 1e-3) / 1e9,
                          "reads_per_ray": reads / rays}
            if vox:
                res[label]["voxel_MiB"] = voxel_bytes(ctx) / 2**20
        ctx.tc_set_option(tc.TC_OPT_VOXEL_SHAPE, 0)
        res["map_MiB"] = ctx.tc_map_bytes() / 2**20
        ctx.close()
        out[name] = res
    out["workload"] = ("2048x2048 cave-heavy map (50% two-layer), a 1920x1080 eye-level and "
                       "a 1920x1080 oblique view; and the c2 headline view")
    return out


def c4_batched(torch, tc, synth, steps, warmup, knob_set="tuned"):
    """Configuration 4: 64 views of uneven sizes + 8 shadow passes + 16
    craters.  Plain: tc_apply_edit then one tc_render_views per view,
    serialized on one stream; a view's latency runs from the frame start to
    its render's end.  Batched: the same work as one captured frame; every
    view completes with the frame.  knob_set: the autotuner's choice
    (default), the persistent packet queue, or the hierarchical defaults."""
    from paper_2608_17390_amd import tune
    F, B, T = synth.make_map_from_config(4)
    H, W = F.shape
    views = synth.config_views(4, F, B)
    edits = synth.crater_list(synth.SEEDS[4]["edits"], W, H, 16, size=32)
    va = synth.views_array(views)
    sizes = va["width"].astype(np.int64) * va["height"]
    offs = np.concatenate([[0], np.cumsum(sizes)])
    rays = int(offs[-1])
    ctx = tc.Context(0)
    ctx.tc_load_columns(F, B, T)
    out = torch.empty((rays, 2), dtype=torch.int32, device="cuda")
    if knob_set == "tuned":
        knobs, cached = tune.autotune(ctx, views, out.data_ptr(), "c4-batched")
    else:
        ctx.tc_set_option(tc.TC_OPT_RENDER_MODE, 2 if knob_set == "persistent" else 0)
        knobs, cached = {k: ctx.tc_get_option(o) for k, o in tune.OPTS.items()}, None
    log("[bench] c4 knobs %s (cached %s)" % (knobs, cached))
    # plain
    nv = len(views)
    plain_lat, plain_frame = [], []
    for it in range(warmup + steps):
        e0 = torch.cuda.Event(enable_timing=True)
        evs = [torch.cuda.Event(enable_timing=True) for _ in range(nv)]
        e0.record()
        ctx.tc_apply_edit(edits)
        for i in range(nv):
            ptr = out.data_ptr() + int(offs[i]) * 8
            ctx.tc_render_views(views[i:i + 1], ptr)
            evs[i].record()
        torch.cuda.synchronize()
        if it >= warmup:
            lat = [e0.elapsed_time(e) for e in evs]
            plain_lat.extend(lat)
            plain_frame.append(lat[-1])
    # batched
    frame = ctx.tc_frame_create(views, edits, out.data_ptr())
    for _ in range(warmup):
        frame.launch()
    torch.cuda.synchronize()
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
          for _ in range(steps)]
    for a, b in ev:
        a.record()
        frame.launch()
        b.record()
    torch.cuda.synchronize()
    bms = np.array([a.elapsed_time(b) for a, b in ev])
    frame.close()
    ctx.close()
    batched_lat = np.repeat(bms, nv)
    pf = np.array(plain_frame)
    return {"workload": "c4: 2048x16384 map, 64 views (256^2/640x480/1280x720/1920x1080) "
                        "+ 8 x 2048^2 shadow passes + 16 craters per frame",
            "rays_per_frame": rays, "views": nv, "knobs": knobs,
            "plain": {"frame_ms_median": float(np.median(pf)),
                      "view_latency_ms_p50": float(np.percentile(plain_lat, 50)),
                      "view_latency_ms_p99": float(np.percentile(plain_lat, 99)),
                      "grays_per_s": rays / (np.median(pf) * 1e-3) / 1e9},
            "batched": {"frame_ms_median": float(np.median(bms)),
                        "view_latency_ms_p50": float(np.percentile(batched_lat, 50)),
                        "view_latency_ms_p99": float(np.percentile(batched_lat, 99)),
                        "grays_per_s": rays / (np.median(bms) * 1e-3) / 1e9}}


def _serve(tc, ctx, F, B, T, reqs, cs, arr, batch, streams):
    """Submit `reqs` (prebuilt C structures `cs`) at arrival times `arr`
    (seconds from the start) to a server of `batch` views per render on
    `streams` streams; wait for all.  Latency runs from submission to
    observed completion."""
    ctx.tc_load_columns(F, B, T)
    srv = ctx.tc_server_start(8 << 30, max_batch_views=batch, streams=streams,
                              flags=tc.TC_SERVER_AUTO_RELEASE)
    ids = []
    t0 = time.perf_counter()
    late = 0.0
    for (kind, x), c, t in zip(reqs, cs, arr):
        while time.perf_counter() - t0 < t:
            pass
        late = max(late, time.perf_counter() - t0 - t)
        ids.append(srv.tc_server_submit_view(c) if kind == "view"
                   else srv.tc_server_submit_edit(c))
    for rid in ids:
        srv.tc_server_wait(rid, 300.0)
    t_end = time.perf_counter()
    states, lats = srv.tc_server_poll_many(ids)
    isview = np.array([k == "view" for k, _ in reqs])
    lat = lats[isview] * 1e3
    rays = sum(int(x["width"]) * int(x["height"]) for k, x in reqs if k == "view")
    stats = srv.tc_server_get_stats()
    srv.tc_server_stop()
    nv = max(1, int(stats["views"]))
    return {"latency_ms_p50": float(np.percentile(lat, 50)),
            "latency_ms_p99": float(np.percentile(lat, 99)),
            "grays_per_s": rays / (t_end - t0) / 1e9,
            "batches": stats["batches"],
            # host side of a view's latency: submission to launch (admission,
            # batching, planning, upload, launch), then launch to observed
            # completion (GPU time plus completion polling)
            "queue_ms_mean": stats["queue_s"] / nv * 1e3,
            "run_ms_mean": stats["run_s"] / nv * 1e3,
            "max_submit_lag_ms": late * 1e3,
            "peak_inflight_MiB": stats["peak_bytes"] / 2**20}


def c5_served(torch, tc, synth, rates=(200, 500, 1000, 2000, 5000, 10000),
              n_per_rate=1500, min_seconds=1.5, burst=2000):
    """Configuration 5: Poisson request streams against the resident
    2048x16384 map; 90% views (sizes and poses as configuration 4), 10%
    craters of size 16-64; an 8 GiB in-flight hit-buffer budget.  Served:
    continuous batching (up to 8 views per batch, 2 streams).  FIFO plain:
    the same server with one view per render on one stream, i.e. each view
    in its own render, serialized, with the plain kernel's knobs.  Each rate
    gets at least n_per_rate requests and at least min_seconds of arrivals,
    so the p99 of the fast rates rests on thousands of requests.  Then two
    saturation legs, where arrivals outrun the FIFO form: `burst` requests
    of the same mix submitted at once, and `burst` // 2 1920x1080 views at
    once; delivered rays/s there is the sustained capacity of each form."""
    F, B, T = synth.make_map_from_config(5)
    H, W = F.shape
    seeds = synth.SEEDS[5]
    ctx = tc.Context(0)
    forms = (("served", 8, 2), ("fifo_plain", 1, 1))
    out = {"workload": "c5: 2048x16384 map resident, Poisson arrivals, 90% views "
                       "(256^2..1920x1080) / 10% craters (16..64), 8 GiB in-flight budget",
           "requests_per_rate": {}, "rates": {}, "saturation": {}}

    def mix(rng, n):
        reqs = []
        for _ in range(n):
            if rng.random() < 0.1:
                reqs.append(("edit", synth.crater_list(rng, W, H, 1, size=(16, 64))))
            else:
                reqs.append(("view", synth.request_view(rng, F, B)))
        return reqs

    def structs(reqs):
        return [tc.view_struct(x) if k == "view" else tc.edits_struct(x) for k, x in reqs]

    for rate in rates:
        nreq = max(n_per_rate, int(rate * min_seconds))
        out["requests_per_rate"][str(rate)] = nreq
        rng = np.random.default_rng(seeds["views"] * 10 + rate)
        arr = synth.poisson_arrivals(seeds["arrivals"] * 10 + rate, rate, nreq)
        reqs = mix(rng, nreq)
        cs = structs(reqs)      # C structures built before the timed submission loop
        res = {}
        for name, batch, streams in forms:
            res[name] = _serve(tc, ctx, F, B, T, reqs, cs, arr, batch, streams)
            log("[bench] c5 rate %d %s: %s" % (rate, name, res[name]))
        out["rates"][str(rate)] = res
    rng = np.random.default_rng(seeds["views"] * 10 + 7)
    legs = {"burst_mix": mix(rng, burst)}
    big = []
    while len(big) < burst // 2:
        v = synth.request_view(rng, F, B)
        if int(v["width"]) == 1920:
            big.append(("view", v))
    legs["burst_1920x1080"] = big
    for leg, reqs in legs.items():
        cs = structs(reqs)
        arr = np.zeros(len(reqs))
        res = {"requests": len(reqs)}
        for name, batch, streams in forms:
            res[name] = _serve(tc, ctx, F, B, T, reqs, cs, arr, batch, streams)
            log("[bench] c5 %s %s: %s" % (leg, name, res[name]))
        out["saturation"][leg] = res
    ctx.close()
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--mode", default="hier", choices=list(MODES))
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--extra", action="store_true",
                    help="also time every render mode")
    ap.add_argument("--calib-copy", action="store_true",
                    help="first run a 256 MiB device copy (counter calibration)")
    ap.add_argument("--no-march", action="store_true",
                    help="skip the sampled-march leg (protocol views)")
    ap.add_argument("--no-growth", action="store_true",
                    help="skip the edit frame (c3), batched frame (c4) and server (c5)")
    ap.add_argument("--beam-passes", type=int, default=None,
                    help="packet beam passes of the headline render (default: the "
                         "library's)")
    ap.add_argument("--legs", default="march,occupancy,c3,c4,c5",
                    help="comma-separated legs to run after the headline (march, "
                         "occupancy, c3, c4, c5)")
    ap.add_argument("--c4-knobs", default="tuned", choices=["tuned", "persistent", "hier"],
                    help="knobs of the c4 frames: the autotuner's, the persistent packet "
                         "queue's, or the hierarchical defaults")
    args = ap.parse_args()
    legs = set(x for x in args.legs.split(",") if x)
    if args.no_march:
        legs -= {"march", "occupancy"}
    if args.no_growth:
        legs -= {"c3", "c4", "c5"}
    if args.gpus != 1:
        print("bench.py measures one GPU; --gpus %d is not supported (the method "
              "shards by replicating the map and splitting views across GPUs, "
              "which this build does not run)" % args.gpus, file=sys.stderr)
        sys.exit(2)

    import torch
    import paper_2608_17390_amd as tc
    import synth

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    if args.calib_copy:
        log("[bench] calibration copy of %d bytes" % calib_copy(torch))
    log("[bench] generating the 2048x2048 map")
    F, B, T = synth.make_map_from_config(2)
    views = synth.config_views(2, F, B)
    rays = synth.view_rays(views)
    ctx = tc.Context(0)
    ctx.tc_load_columns(F, B, T)
    torch.cuda.synchronize()
    out = torch.empty((rays, 2), dtype=torch.int32, device="cuda")
    ctx.tc_set_option(tc.TC_OPT_RENDER_MODE, MODES[args.mode])
    if args.beam_passes is not None:
        ctx.tc_set_option(tc.TC_OPT_BEAM_PASSES, args.beam_passes)
    beam = ctx.tc_get_option(tc.TC_OPT_BEAM_PASSES)

    # algorithmic bytes: node/cell reads of the one-pass exact walk (split
    # pass off, so speculative segment walks are not counted), counted by
    # the library itself
    budget = ctx.tc_get_option(tc.TC_OPT_SPLIT_BUDGET)
    ctx.tc_set_option(tc.TC_OPT_SPLIT_BUDGET, 0)
    ctx.tc_set_option(tc.TC_OPT_COUNT_READS, 1)
    ctx.tc_render_views(views, out.data_ptr())
    reads = ctx.tc_read_counters()
    ctx.tc_set_option(tc.TC_OPT_COUNT_READS, 0)
    ctx.tc_set_option(tc.TC_OPT_SPLIT_BUDGET, budget)
    alg_bytes = 8 * rays + 4 * reads
    log("[bench] %d rays, %d node/cell reads (%.1f per ray)" % (rays, reads, reads / rays))

    log("[bench] timing %d steps after %d warmup, mode %s" % (args.steps, args.warmup, args.mode))
    ms, wall = time_renders(torch, ctx, tc, views, out, args.steps, args.warmup)
    ms_per_step = wall * 1e3 / args.steps
    med = float(np.median(ms))
    # the traversal kernels alone, timed by HIP events the library attaches
    # to each kernel's dispatch (its start and end), over as many renders
    # again
    kern = kernel_times(torch, ctx, tc, views, out, args.steps)
    kavg = float(kern.sum(axis=1).mean())
    achieved = alg_bytes / (kavg * 1e-3) / 1e9
    traffic = profile_value(RENDER_SRCS, "render_c2_traffic", "hbm_bytes_per_launch")
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
                   "rays_per_frame": rays, "render_mode": args.mode, "beam_passes": beam,
                   "frame_ms_median": med, "frame_ms_p99": float(np.percentile(ms, 99))},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": PEAK_HBM_GBS,
                     "unit": "GB/s", "frac": achieved / PEAK_HBM_GBS,
                     # HBM bytes per traversal (FETCH_SIZE + WRITE_SIZE, copy-calibrated)
                     "traffic": traffic,
                     "traffic_gb_per_s": (traffic / (kavg * 1e-3) / 1e9) if traffic else None,
                     # VALU issue against the ALU roof (one wave64 VALU instruction per
                     # SIMD every 2 cycles: 256 CUs x 4 SIMDs x 32 lanes x 2.4 GHz):
                     # SQ_INSTS_VALU over 1024 SIMDs x GRBM_GUI_ACTIVE per XCD x 0.5
                     "valu_issue_frac": profile_value(RENDER_SRCS, "render_c2_counters",
                                                      "valu_issue_frac"),
                     # share of lanes active per VALU instruction (SQ_THREAD_CYCLES_VALU
                     # over 64 x SQ_INSTS_VALU)
                     "valu_lane_util": profile_value(RENDER_SRCS, "render_c2_counters",
                                                     "valu_lane_util"),
                     # share of the launch's lifetime its shader engines hold waves
                     # (SQ_BUSY_CYCLES over 32 engines x GRBM_GUI_ACTIVE per XCD)
                     "sq_busy_frac": profile_value(RENDER_SRCS, "render_c2_counters",
                                                   "sq_busy_frac"),
                     # the counters' verdict: neither HBM (measured traffic a fifth of the
                     # algorithmic bytes, far below peak) nor VALU issue binds; each walk
                     # step waits on the load of the step before, and the launch's tail
                     # (its longest packets) leaves engines idle
                     "binding_roof": "load_latency",
                     "kernel": KERNEL_NAMES[args.mode],
                     "alg_bytes_per_launch": alg_bytes,
                     "kernel_ms_avg": kavg,
                     "traversal_ms_avg": float(kern[:, 0].mean()),
                     "split_pass_ms_avg": float(kern[:, 1].mean()),
                     "render_call_ms_avg": float(ms.mean())},
    }
    if args.extra:
        modes = {}
        for m in MODES:
            ctx.tc_set_option(tc.TC_OPT_RENDER_MODE, MODES[m])
            mm, _ = time_renders(torch, ctx, tc, views, out, 10, 2)
            modes[m] = float(np.median(mm))
        res["mode_ms_median"] = modes
    if "march" in legs:
        log("[bench] sampled march on the protocol views")
        res["march_protocol"] = march_protocol(torch, tc, synth, 10, 2)
    if "occupancy" in legs:
        log("[bench] 2D pyramid vs occupancy masks vs voxel occupancy pyramid")
        res["occupancy_compare"] = occupancy_compare(torch, tc, synth, 10, 2)
    if "c3" in legs:
        log("[bench] c3 edit frame")
        res["c3_frame"] = c3_frame(torch, tc, synth, 10, 2)
    if "c4" in legs:
        log("[bench] c4 batched vs plain")
        res["c4_batched"] = c4_batched(torch, tc, synth, 10, 2, args.c4_knobs)
    if "c5" in legs:
        log("[bench] c5 served vs FIFO plain")
        res["c5_served"] = c5_served(torch, tc, synth)
    if not args.no_cpu:
        import oracle
        log("[bench] CPU oracle baseline")
        res["cpu_baseline"] = cpu_baseline(oracle, F, B, T, views, rays)
    print(json.dumps(res), flush=True)
    ctx.close()


if __name__ == "__main__":
    main()
