"""Autotuning cache: the render knobs chosen by tc_autotune, stored as JSON
keyed by (GPU architecture, map size, workload name)."""
import json
import os

from . import _tc

OPTS = {"render_mode": _tc.TC_OPT_RENDER_MODE, "start_level": _tc.TC_OPT_START_LEVEL,
        "tile_order": _tc.TC_OPT_TILE_ORDER, "xcd_remap": _tc.TC_OPT_XCD_REMAP,
        "persist_waves": _tc.TC_OPT_PERSIST_WAVES, "refill_min": _tc.TC_OPT_REFILL_MIN,
        "refill_iters": _tc.TC_OPT_REFILL_ITERS, "split_budget": _tc.TC_OPT_SPLIT_BUDGET,
        "beam_passes": _tc.TC_OPT_BEAM_PASSES, "packet_width": _tc.TC_OPT_PACKET_WIDTH,
        "max_level": _tc.TC_OPT_MAX_LEVEL}


def default_cache_path():
    return os.environ.get("TC_TUNE_CACHE",
                          os.path.join(os.path.expanduser("~"), ".cache", "tc_autotune.json"))


def _arch():
    try:
        import torch
        return torch.cuda.get_device_properties(0).gcnArchName.split(":")[0]
    except Exception:
        return "unknown"


def autotune(ctx, views, out_ptr, workload, cache_path=None, reps=5, force=False):
    """Apply cached knobs for (arch, map size, workload) or tune and cache
    them.  Returns (knobs dict, from_cache)."""
    path = cache_path or default_cache_path()
    key = "%s|%dx%d|%s" % (_arch(), ctx.W, ctx.H, workload)
    cache = {}
    if os.path.exists(path):
        try:
            cache = json.load(open(path))
        except ValueError:
            cache = {}
    if key in cache and not force and all(k in cache[key] for k in OPTS):
        knobs = cache[key]
        for k, opt in OPTS.items():
            ctx.tc_set_option(opt, knobs[k])
        return knobs, True
    knobs = ctx.tc_autotune(views, out_ptr, reps=reps)
    cache[key] = knobs
    os.makedirs(os.path.dirname(path) or ".", exist_ok=True)
    tmp = path + ".tmp%d" % os.getpid()
    with open(tmp, "w") as f:
        json.dump(cache, f, indent=1, sort_keys=True)
    os.replace(tmp, path)
    return knobs, False
