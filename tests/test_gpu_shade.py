"""GPU parity of the shading pass (tc_shade_views) against the shading
oracle, through the C ABI: every pixel's RGBA word must match bit for bit
(both sides compute in single precision, one operation at a time, and cast
their shadow rays exactly)."""
import numpy as np
import pytest

import oracle
import synth
from oracle_cache import config_map

tc = pytest.importorskip("paper_2608_17390_amd")
torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

S = 65536
LIGHTS = [(0, 0, S), (S, 2 * S, 3 * S), (-3 * S, S, S // 2), (2 * S, -S, -S), (0, S, 0)]


@pytest.fixture(scope="module")
def ctx():
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    c = tc.Context(0)
    yield c
    c.close()


def load(ctx, F, B, T):
    ctx.tc_load_columns(F, B, T)
    torch.cuda.synchronize()


def gpu_shade(ctx, views, light, palette, mode=0, **kw):
    ctx.tc_set_option(tc.TC_OPT_RENDER_MODE, mode)
    hits = tc.render(ctx, views)
    out = torch.empty(synth.view_rays(views), dtype=torch.int32, device="cuda")
    ctx.tc_shade_views(views, hits.data_ptr(), light, palette, out.data_ptr(), **kw)
    torch.cuda.synchronize()
    ctx.tc_set_option(tc.TC_OPT_RENDER_MODE, 0)
    return out.cpu().numpy().view(np.uint32)


def assert_same(g, o, what):
    bad = np.nonzero(g != o)[0]
    assert bad.size == 0, "%s: %d of %d pixels differ, first %d: gpu %08x oracle %08x" % (
        what, bad.size, g.size, bad[0], g[bad[0]], o[bad[0]])


@pytest.mark.parametrize("li", range(len(LIGHTS)))
def test_c1_lights(ctx, li):
    F, B, T = synth.make_map_from_config(1)
    load(ctx, F, B, T)
    views = synth.config_views(1, F, B)
    pal = synth.default_palette()
    g = gpu_shade(ctx, views, LIGHTS[li], pal)
    o = oracle.shade(F, B, T, views, LIGHTS[li], pal)
    assert_same(g, o, "c1 light %d" % li)
    assert len(np.unique(g)) > 200


@pytest.mark.parametrize("mode", [0, 1, 2])
def test_ragged_views_params_and_modes(ctx, mode):
    """Shadow passes, a straight-down image, eyes outside the map and in
    caves, several ambient and fog settings; hit records from each exact
    render mode shade alike."""
    F, B, T = synth.make_map_from_config(1)
    load(ctx, F, B, T)
    rng = np.random.default_rng(21 + mode)
    views = [synth.perspective_view(synth.eye_above_floor(F, B, 60.5, 200.5, dz=7), 200, -20, 77, 45),
             synth.perspective_view((-20.5, 128.0, 90.0), 90, -25, 33, 17),
             synth.shadow_view(30, 40, 64, 35.0, rng.uniform(0, 360)),
             synth.ortho_view((0, 0, 270 * S), (S // 2, 0, 0), (0, S // 2, 0), (0, 0, -1), 40, 24),
             synth.perspective_view(synth.eye_above_floor(F, B, 128.5, 128.5, dz=2), 45, -10, 24, 24)]
    # an eye inside a cave: between a floor and its slab
    ys, xs = np.nonzero((B > 0) & (B.astype(int) - F.astype(int) > 3))
    if ys.size:
        x, y = int(xs[0]), int(ys[0])
        views.append(synth.perspective_view((x + 0.5, y + 0.5, (int(F[y, x]) + int(B[y, x])) / 2),
                                            rng.uniform(0, 360), -20, 16, 12))
    pal = synth.default_palette()
    for kw in (dict(), dict(ambient=0.0, cave_ambient=0.0, fog_far=50.0),
               dict(ambient=1.0, cave_ambient=0.5, fog_far=1e6, sky_rgba=0, fog_rgba=0xFFFFFFFF)):
        light = LIGHTS[int(rng.integers(0, len(LIGHTS)))]
        g = gpu_shade(ctx, views, light, pal, mode=mode, **kw)
        o = oracle.shade(F, B, T, views, light, pal, **kw)
        assert_same(g, o, "mode %d %r" % (mode, kw))


def test_after_edits(ctx):
    F, B, T = synth.make_map_from_config(1)
    load(ctx, F, B, T)
    edits = synth.crater_list(57, 256, 256, 6, size=(8, 40), depth=(10, 60))
    ctx.tc_apply_edit(edits)
    F2, B2, T2 = oracle.apply_edits(F, B, T, edits)
    views = synth.config_views(1, F, B)
    pal = synth.default_palette()
    g = gpu_shade(ctx, views, LIGHTS[1], pal)
    assert_same(g, oracle.shade(F2, B2, T2, views, LIGHTS[1], pal), "after edits")


def test_protocol_views_sampled(ctx):
    """The twelve 1280x800 protocol views on the 2048x16384 map, 20,000
    sampled pixels against the oracle."""
    F, B, T = config_map(3)
    load(ctx, F, B, T)
    views, _ = synth.pitch_views(F, B, 91)
    pal = synth.default_palette()
    light = (S, 2 * S, 2 * S)
    g = gpu_shade(ctx, views, light, pal)
    rng = np.random.default_rng(93)
    n = 20000
    vi = rng.integers(0, len(views), n).astype(np.int32)
    px = rng.integers(0, 1280, n).astype(np.int32)
    py = rng.integers(0, 800, n).astype(np.int32)
    o = oracle.shade_pixels(F, B, T, views, vi, px, py, light, pal)
    idx = vi.astype(np.int64) * 1280 * 800 + py.astype(np.int64) * 1280 + px
    assert_same(g[idx], o, "protocol")


def test_kernel_timing_and_read_count(ctx):
    F, B, T = synth.make_map_from_config(1)
    load(ctx, F, B, T)
    views = synth.config_views(1, F, B)
    pal = synth.default_palette()
    hits = tc.render(ctx, views)
    out = torch.empty(synth.view_rays(views), dtype=torch.int32, device="cuda")
    ctx.tc_set_option(tc.TC_OPT_KERNEL_TIMING, 1)
    ctx.tc_set_option(tc.TC_OPT_COUNT_READS, 1)
    try:
        ctx.tc_read_counters()
        ctx.tc_shade_views(views, hits.data_ptr(), LIGHTS[1], pal, out.data_ptr())
        t0, t1 = ctx.tc_read_kernel_times()
        reads = ctx.tc_read_counters()
    finally:
        ctx.tc_set_option(tc.TC_OPT_KERNEL_TIMING, 0)
        ctx.tc_set_option(tc.TC_OPT_COUNT_READS, 0)
    assert t0 > 0 and t1 == 0
    w, _ = tc.split_hits(hits)
    nhit = int(np.sum(w != oracle.MISS))
    assert nhit <= reads <= 64 * nhit


def test_errors(ctx):
    F, B, T = synth.make_map_from_config(1)
    load(ctx, F, B, T)
    views = synth.config_views(1, F, B)
    pal = synth.default_palette()
    hits = tc.render(ctx, views)
    out = torch.empty(synth.view_rays(views), dtype=torch.int32, device="cuda")
    for light, kw in (((0, 0, 0), {}), ((1 << 23, 0, 1), {}), ((0, 0, S), dict(fog_far=0.0)),
                      ((0, 0, S), dict(fog_far=float("inf"))), ((0, 0, S), dict(ambient=1.5))):
        with pytest.raises(tc.TCError) as e:
            ctx.tc_shade_views(views, hits.data_ptr(), light, pal, out.data_ptr(), **kw)
        assert e.value.status == tc.TC_INVALID_ARG
    with pytest.raises(ValueError):
        ctx.tc_shade_views(views, hits.data_ptr(), (0, 0, S), pal[:10], out.data_ptr())
    torch.cuda.synchronize()
