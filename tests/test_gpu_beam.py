"""GPU parity of the packet beam start (TC_OPT_BEAM_PASSES): each packet's
rays skip a common empty stretch found by testing bounding boxes of the
ray bundle against the pyramid, then walk exactly from the last cell line
they enter before its end.  The skip must never pass a hit, so every case compares the hit
records with the oracle bit for bit (depth within 1e-5): pass counts from
1 to 64, start levels, eyes grazing the floor, inside caves and far outside
the map, orthographic shadow passes, packets straddling map edges and
ragged views."""
import numpy as np
import pytest

import oracle
import synth
from oracle_cache import config_map

tc = pytest.importorskip("paper_2608_17390_amd")
torch = pytest.importorskip("torch")

from test_gpu_parity import assert_parity, load, _random_views  # noqa: E402

pytestmark = pytest.mark.gpu

S = 65536


@pytest.fixture(scope="module")
def ctx():
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    c = tc.Context(0)
    yield c
    c.close()


def render(ctx, views, passes, mode=0, start=2):
    ctx.tc_set_option(tc.TC_OPT_RENDER_MODE, mode)
    ctx.tc_set_option(tc.TC_OPT_BEAM_PASSES, passes)
    ctx.tc_set_option(tc.TC_OPT_START_LEVEL, start)
    try:
        out = tc.render(ctx, views)
        torch.cuda.synchronize()
    finally:
        ctx.tc_set_option(tc.TC_OPT_RENDER_MODE, 0)
        ctx.tc_set_option(tc.TC_OPT_BEAM_PASSES, 6)
        ctx.tc_set_option(tc.TC_OPT_START_LEVEL, 2)
    return tc.split_hits(out)


def _grazing_views(F, B, rng, n, size=(96, 64)):
    """eye-level views from just above the floor, pitched around the
    horizon: the long walks the beam is for"""
    H, W = F.shape
    out = []
    for _ in range(n):
        eye = synth.eye_above_floor(F, B, rng.uniform(0, W), rng.uniform(0, H),
                                    dz=float(rng.uniform(0.05, 3)))
        out.append(synth.perspective_view(eye, rng.uniform(0, 360), rng.uniform(-6, 3),
                                          size[0], size[1], vfov_deg=rng.uniform(30, 90)))
    return out


@pytest.mark.parametrize("passes", [1, 2, 3, 8, 64])
def test_pass_counts_c1(ctx, passes):
    F, B, T = synth.make_map_from_config(1)
    load(ctx, F, B, T)
    rng = np.random.default_rng(300 + passes)
    views = (synth.config_views(1, F, B) + _grazing_views(F, B, rng, 6) +
             _random_views(rng, F, B, 9, [(77, 53), (1, 1), (13, 40), (8, 9)]))
    wo, do = oracle.render(F, B, T, views)
    for mode in (0, 4):
        wg, dg = render(ctx, views, passes, mode)
        assert_parity(wg, dg, wo, do, "c1 passes %d mode %d" % (passes, mode))


@pytest.mark.parametrize("start", [0, 1, 4, 15])
def test_start_levels(ctx, start):
    F, B, T = synth.make_map_from_config(1)
    load(ctx, F, B, T)
    rng = np.random.default_rng(320 + start)
    views = _grazing_views(F, B, rng, 6) + _random_views(rng, F, B, 6, [(40, 30)])
    wo, do = oracle.render(F, B, T, views)
    wg, dg = render(ctx, views, 8, 0, start)
    assert_parity(wg, dg, wo, do, "start level %d" % start)


def test_eyes_outside_the_map_and_straddling_edges(ctx):
    """Eyes far outside looking in (the skip crosses the empty outside and
    the start line is clamped at the map's edge), looking away, and along
    the edges, so that packets straddle the map's border."""
    F, B, T = synth.make_map(97, 61, 330, dual=0.3, period=16)
    load(ctx, F, B, T)
    H, W = F.shape
    views = [
        synth.perspective_view((-2000.0, 30.5, 60.0), 90 - 90, -1, 64, 48),
        synth.perspective_view((-2000.0, 30.5, 60.0), 0, -1, 64, 48),
        synth.perspective_view((48.5, -3000.0, 90.0), 0, -1.5, 48, 40),
        synth.perspective_view((48.5, 5000.0, 200.0), 180, -2.2, 48, 40),
        synth.perspective_view((120.0, 80.0, 40.0), 225, -2, 64, 64),
        synth.perspective_view((120.0, 80.0, 40.0), 45, -2, 64, 64),      # away
        synth.perspective_view((0.0, 0.0, 30.0), 45, -4, 64, 64),         # from a corner
        synth.perspective_view((97.0, 30.0, 30.0), 90, 0, 32, 32),        # on the far edge
        synth.perspective_view((-0.01, 30.5, 20.0), 0, -2, 40, 40),       # along x = 0
        synth.shadow_view(-20, -20, 140, 20.0, 30.0),
        synth.shadow_view(40, 20, 64, 5.0, 200.0),
        synth.ortho_view((-50 * S, 10 * S, 120 * S), (0, S // 3, 0), (0, 0, S // 2), (3, 1, -1), 64, 40),
    ]
    rng = np.random.default_rng(331)
    for _ in range(6):
        views.append(synth.perspective_view(
            (rng.uniform(-400, 500), rng.uniform(-400, 460), rng.uniform(-50, 400)),
            rng.uniform(0, 360), rng.uniform(-30, 30), 33, 21))
    wo, do = oracle.render(F, B, T, views)
    for passes in (1, 8, 64):
        for mode in (0, 4):
            wg, dg = render(ctx, views, passes, mode)
            assert_parity(wg, dg, wo, do, "outside passes %d mode %d" % (passes, mode))


def test_caves_and_touching_heights(ctx):
    """Eyes inside caves (a slab just above), eyes at exactly a floor's or
    slab top's height, rays along flat floors at their height, and slabs
    touching 255."""
    F, B, T = synth.cave_map(340, 256, 256)
    B = B.copy()
    T = T.copy()
    T[B > 0] = np.maximum(T[B > 0], np.minimum(255, B[B > 0].astype(int) + 30)).astype(np.uint8)
    T[100:110, 100:110] = np.where(B[100:110, 100:110] > 0, 255, 0)
    load(ctx, F, B, T)
    rng = np.random.default_rng(341)
    views = []
    ys, xs = np.nonzero((B > 0) & (B.astype(int) - F.astype(int) > 4))
    for k in rng.choice(ys.size, 8, replace=False):
        x, y = int(xs[k]), int(ys[k])
        views.append(synth.perspective_view((x + 0.5, y + 0.5, int(F[y, x]) + 1.0),
                                            rng.uniform(0, 360), rng.uniform(-10, 15), 48, 32))
    for k in range(6):
        x, y = int(rng.integers(0, 256)), int(rng.integers(0, 256))
        if B[y, x]:
            continue
        # eye exactly at the column's floor height, looking level
        views.append(synth.perspective_view((x + 0.5, y + 0.5, float(F[y, x])),
                                            rng.uniform(0, 360), 0.0, 40, 24))
    flat = np.full((64, 64), 20, np.uint8)
    zero = np.zeros_like(flat)
    wo, do = oracle.render(F, B, T, views)
    for passes in (1, 8):
        wg, dg = render(ctx, views, passes, 0)
        assert_parity(wg, dg, wo, do, "caves passes %d" % passes)
    # a flat floor seen along its own height: every ray runs on the surface
    load(ctx, flat, zero, zero)
    views = [synth.perspective_view((-3.0, 32.5, 20.0), 0, 0, 64, 64),
             synth.ortho_view((-S, 0, 20 * S), (0, S // 2, 0), (0, 0, S // 64), (1, 0, 0), 64, 64)]
    wo, do = oracle.render(flat, zero, zero, views)
    wg, dg = render(ctx, views, 8, 0)
    assert_parity(wg, dg, wo, do, "flat floor at eye height")


def test_c2_view_and_read_count(ctx):
    """The 1920x1080 eye-level view: identical records with and without the
    beam; the beam reads far fewer nodes per ray."""
    budget0 = ctx.tc_get_option(tc.TC_OPT_SPLIT_BUDGET)
    F, B, T = synth.make_map_from_config(2)
    views = synth.config_views(2, F, B)
    load(ctx, F, B, T)
    wo, do = oracle.render(F, B, T, views)
    reads = {}
    ctx.tc_set_option(tc.TC_OPT_SPLIT_BUDGET, 0)
    ctx.tc_set_option(tc.TC_OPT_COUNT_READS, 1)
    try:
        for passes in (0, 8):
            ctx.tc_read_counters()
            wg, dg = render(ctx, views, passes, 0)
            reads[passes] = ctx.tc_read_counters()
            assert_parity(wg, dg, wo, do, "c2 passes %d" % passes)
    finally:
        ctx.tc_set_option(tc.TC_OPT_COUNT_READS, 0)
        ctx.tc_set_option(tc.TC_OPT_SPLIT_BUDGET, budget0)
    rays = synth.view_rays(views)
    print("reads per ray: no beam %.2f, beam %.2f" % (reads[0] / rays, reads[8] / rays))
    assert reads[8] < reads[0]


def test_large_map_batched_views_sampled(ctx):
    """Grazing, oblique and shadow views on the 2048x16384 map, 30,000
    sampled pixels against the oracle, beam on and off."""
    F, B, T = config_map(3)
    load(ctx, F, B, T)
    rng = np.random.default_rng(350)
    views = (_grazing_views(F, B, rng, 6, (640, 360)) +
             [synth.shadow_view(int(rng.integers(0, 1500)), int(rng.integers(0, 15000)), 512,
                                35.0, rng.uniform(0, 360)) for _ in range(2)] +
             [synth.perspective_view((rng.uniform(0, 2048), rng.uniform(0, 16384), 300.0),
                                     rng.uniform(0, 360), -45, 320, 240)])
    n = 30000
    sizes = np.array([int(v["width"]) * int(v["height"]) for v in views])
    base = np.concatenate([[0], np.cumsum(sizes)])
    vi = rng.integers(0, len(views), n).astype(np.int32)
    wv = np.array([int(views[i]["width"]) for i in vi])
    hv = np.array([int(views[i]["height"]) for i in vi])
    px = (rng.random(n) * wv).astype(np.int32)
    py = (rng.random(n) * hv).astype(np.int32)
    wo, do = oracle.cast_pixels(F, B, T, views, vi, px, py)
    idx = base[vi] + py.astype(np.int64) * wv + px
    for passes in (0, 8):
        wg, dg = render(ctx, views, passes, 0)
        assert_parity(wg[idx], dg[idx], wo, do, "large map passes %d" % passes)


def test_option_range(ctx):
    for bad in (-1, 65):
        with pytest.raises(tc.TCError):
            ctx.tc_set_option(tc.TC_OPT_BEAM_PASSES, bad)
    assert ctx.tc_get_option(tc.TC_OPT_BEAM_PASSES) == 6
    for bad in (0, 3, 8):
        with pytest.raises(tc.TCError):
            ctx.tc_set_option(tc.TC_OPT_SPLIT_WAVES, bad)
    assert ctx.tc_get_option(tc.TC_OPT_SPLIT_WAVES) == 4
