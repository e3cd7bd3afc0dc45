"""Captured frames (edits -> dirty pyramid update -> render in one HIP
graph) and the autotuner, against the oracle."""
import numpy as np
import pytest

import oracle
import synth

tc = pytest.importorskip("paper_2608_17390_amd")
torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

from test_gpu_parity import assert_parity, load, gpu_render, MODES, c4_full_check  # noqa: E402
from oracle_cache import config_map, oracle_render  # noqa: E402


@pytest.fixture(scope="module")
def ctx():
    assert torch.cuda.is_available()
    c = tc.Context(0)
    yield c
    c.close()


def _outbuf(views):
    return torch.empty((synth.view_rays(views), 2), dtype=torch.int32, device="cuda")


@pytest.mark.parametrize("mode", ["hier", "persistent"])
def test_frame_replays_apply_edits_each_time(ctx, mode):
    F, B, T = synth.make_map_from_config(1)
    load(ctx, F, B, T)
    ctx.tc_set_option(tc.TC_OPT_RENDER_MODE, MODES[mode][0])
    ctx.tc_set_option(tc.TC_OPT_BEAM_PASSES, MODES[mode][1])
    rng = np.random.default_rng(50)
    views = synth.config_views(1, F, B) + [
        synth.shadow_view(30, 40, 64, 35.0, 70.0),
        synth.perspective_view(synth.eye_above_floor(F, B, 60.5, 200.5), 200, -20, 77, 45)]
    edits = (synth.crater_list(51, 256, 256, 6, size=(8, 40), depth=(10, 60)) +
             synth.random_set_patches(52, 256, 256, 3, max_size=20))
    out = _outbuf(views)
    frame = ctx.tc_frame_create(views, edits, out.data_ptr())
    assert frame.rays == synth.view_rays(views)
    Fk, Bk, Tk = F, B, T
    for k in range(3):
        frame.launch()
        torch.cuda.synchronize()
        wg, dg = tc.split_hits(out)
        Fk, Bk, Tk = oracle.apply_edits(Fk, Bk, Tk, edits)
        wo, do = oracle.render(Fk, Bk, Tk, views)
        assert_parity(wg, dg, wo, do, "frame replay %d" % k)
        # eager work between replays
        junk = torch.ones(1 << 20, device="cuda").sum()
        torch.cuda.synchronize()
        assert float(junk) == float(1 << 20)
    g = ctx.tc_read_columns(0, 0, 256, 256)
    assert np.array_equal(g[0], Fk) and np.array_equal(g[1], Bk)
    levels = ctx.tc_pyramid_info()
    for L in range(1, levels + 1):
        assert np.array_equal(ctx.tc_read_pyramid(L), oracle.pyramid_level_fast(Fk, Bk, Tk, L))
    for L in range(0, levels + 1):
        assert np.array_equal(ctx.tc_read_window(L), oracle.window_level_fast(Fk, Bk, Tk, L))
    frame.close()
    ctx.tc_set_option(tc.TC_OPT_RENDER_MODE, 0)
    ctx.tc_set_option(tc.TC_OPT_BEAM_PASSES, 6)


def test_frame_without_edits_and_reload_invalidates(ctx):
    F, B, T = synth.make_map_from_config(1)
    load(ctx, F, B, T)
    views = synth.config_views(1, F, B)
    out = _outbuf(views)
    frame = ctx.tc_frame_create(views, [], out.data_ptr())
    for _ in range(4):
        frame.launch()
    torch.cuda.synchronize()
    wo, do = oracle.render(F, B, T, views)
    wg, dg = tc.split_hits(out)
    assert_parity(wg, dg, wo, do, "frame no edits")
    load(ctx, F, B, T)
    with pytest.raises(tc.TCError) as e:
        frame.launch()
    assert e.value.status == tc.TC_INVALID_ARG
    frame.close()


def test_autotune_keeps_results(ctx):
    F, B, T = synth.make_map_from_config(2)
    load(ctx, F, B, T)
    views = synth.config_views(2, F, B)
    ref = gpu_render(ctx, views, "hier")
    out = _outbuf(views)
    best = ctx.tc_autotune(views, out.data_ptr(), reps=2)
    assert best["tried"] >= 72 and best["ms"] > 0
    assert best["render_mode"] in (0, 2)
    assert best["split_budget"] in (0, 96, 112, 120, 128, 160)
    assert ctx.tc_get_option(tc.TC_OPT_SPLIT_BUDGET) == best["split_budget"]
    assert best["beam_passes"] in (0, 2, 4, 6, 8)
    assert ctx.tc_get_option(tc.TC_OPT_BEAM_PASSES) == best["beam_passes"]
    assert best["packet_width"] in (4, 8, 16, 32)
    assert ctx.tc_get_option(tc.TC_OPT_PACKET_WIDTH) == best["packet_width"]
    assert ctx.tc_get_option(tc.TC_OPT_MAX_LEVEL) == best["max_level"]
    assert ctx.tc_get_option(tc.TC_OPT_RENDER_MODE) == best["render_mode"]
    out2 = tc.render(ctx, views)
    torch.cuda.synchronize()
    w, d = tc.split_hits(out2)
    assert np.array_equal(w, ref[0]) and np.array_equal(d.view(np.uint32), ref[1].view(np.uint32))
    ctx.tc_set_option(tc.TC_OPT_RENDER_MODE, 0)
    ctx.tc_set_option(tc.TC_OPT_START_LEVEL, 2)
    ctx.tc_set_option(tc.TC_OPT_TILE_ORDER, 2)
    ctx.tc_set_option(tc.TC_OPT_XCD_REMAP, 64)
    ctx.tc_set_option(tc.TC_OPT_SPLIT_BUDGET, 120)
    ctx.tc_set_option(tc.TC_OPT_PACKET_WIDTH, 8)
    ctx.tc_set_option(tc.TC_OPT_MAX_LEVEL, 15)
    ctx.tc_set_option(tc.TC_OPT_BEAM_PASSES, 6)


# Render knobs of the configuration-4 frame: the set the autotuner picks on
# this GPU (what the benchmark times), the set it picked on an earlier run
# (hierarchical walk from level 3, column-major packets, XCD groups of 64,
# no split pass, 4 beam passes), and the persistent packet queue.
C4_KNOBS = {
    "tuned": None,
    "hier_l3_colmajor": {"render_mode": 0, "start_level": 3, "tile_order": 1,
                         "xcd_remap": 64, "split_budget": 0, "beam_passes": 4},
    "persistent": {"render_mode": 2, "start_level": 2, "tile_order": 2,
                   "xcd_remap": 64, "split_budget": 128, "beam_passes": 4},
}


@pytest.mark.parametrize("knobs", list(C4_KNOBS))
def test_c4_frame_full(ctx, knobs):
    """Configuration 4: 64 views + 8 shadow passes + 16 craters, one graph
    launch, with the knob sets above; every record against the oracle's
    render of the edited map."""
    from paper_2608_17390_amd import tune
    F, B, T = config_map(4)
    H, W = F.shape
    load(ctx, F, B, T)
    views = synth.config_views(4, F, B)
    edits = synth.crater_list(synth.SEEDS[4]["edits"], W, H, 16, size=32)
    out = _outbuf(views)
    saved = {k: ctx.tc_get_option(o) for k, o in tune.OPTS.items()}
    try:
        if C4_KNOBS[knobs] is None:
            # the benchmark's call: cached knobs of this GPU, else a tuning run
            chosen, _ = tune.autotune(ctx, views, out.data_ptr(), "c4-batched")
            print("c4 tuned knobs:", chosen, flush=True)
        else:
            for k, v in C4_KNOBS[knobs].items():
                ctx.tc_set_option(tune.OPTS[k], v)
        frame = ctx.tc_frame_create(views, edits, out.data_ptr())
        try:
            frame.launch()
            torch.cuda.synchronize()
        finally:
            frame.close()
        wg, dg = tc.split_hits(out)
        del out
        wo, do = oracle_render(F, B, T, views, edits)
        c4_full_check(wg, dg, wo, do, views, "c4 frame " + knobs)
    finally:
        for k, v in saved.items():
            ctx.tc_set_option(tune.OPTS[k], v)
