"""GPU parity of the sampled march (render mode 3, Section 3.1 RAYMARCH):
the HIP kernel against the single-precision oracle, through the C ABI.

Both sides decide every sample in IEEE single precision, one rounding per
operation, so hit words and depths must match bit for bit."""
import numpy as np
import pytest

import oracle
import synth
from oracle_cache import config_map
from paper_2608_17390_amd import metrics

tc = pytest.importorskip("paper_2608_17390_amd")
torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

MARCH = 3


@pytest.fixture(scope="module")
def ctx():
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    c = tc.Context(0)
    yield c
    c.close()


def load(ctx, F, B, T):
    ctx.tc_load_columns(F, B, T)
    torch.cuda.synchronize()


def set_march(ctx, far=600, steps=128, bisect=4):
    ctx.tc_set_option(tc.TC_OPT_RENDER_MODE, MARCH)
    ctx.tc_set_option(tc.TC_OPT_MARCH_FAR, far)
    ctx.tc_set_option(tc.TC_OPT_MARCH_STEPS, steps)
    ctx.tc_set_option(tc.TC_OPT_MARCH_BISECT, bisect)


@pytest.fixture(autouse=True)
def restore(ctx):
    yield
    set_march(ctx)
    ctx.tc_set_option(tc.TC_OPT_RENDER_MODE, 0)


def gpu_march(ctx, views):
    out = tc.render(ctx, views)
    torch.cuda.synchronize()
    return tc.split_hits(out)


def assert_same(wg, dg, wo, do, what=""):
    assert wg.shape == wo.shape
    bad = np.nonzero(wg != wo)[0]
    assert bad.size == 0, "%s: %d word mismatches, first at %d: gpu %08x oracle %08x" % (
        what, bad.size, bad[0], wg[bad[0]], wo[bad[0]])
    db = np.nonzero(dg.view(np.uint32) != do.astype(np.float32).view(np.uint32))[0]
    assert db.size == 0, "%s: %d depth mismatches, first at %d: gpu %r oracle %r" % (
        what, db.size, db[0], dg[db[0]], do[db[0]])


def test_c1_full_image_paper_setting(ctx):
    F, B, T = synth.make_map_from_config(1)
    load(ctx, F, B, T)
    views = synth.config_views(1, F, B)
    set_march(ctx)
    wg, dg = gpu_march(ctx, views)
    wo, do = oracle.march(F, B, T, views)
    assert_same(wg, dg, wo, do, "c1 march")
    assert np.mean(wg != oracle.MISS) > 0.3


@pytest.mark.parametrize("far,steps,bisect", [(600, 1, 0), (600, 7, 1), (50, 127, 4),
                                              (5000, 1000, 9), (300, 129, 30)])
def test_options_ragged_views(ctx, far, steps, bisect):
    """Sample counts that are not a multiple of the load group, far limits
    inside and beyond the map, many halvings; ragged views of several
    kinds, including shadow passes and views from outside the map."""
    F, B, T = synth.make_map_from_config(1)
    load(ctx, F, B, T)
    rng = np.random.default_rng(steps)
    views = [synth.perspective_view(synth.eye_above_floor(F, B, 60.5, 200.5, dz=7), 200, -20, 77, 45),
             synth.perspective_view((-20.5, 128.0, 90.0), 90, -25, 33, 17),
             synth.perspective_view((128.25, 300.5, 40.0), 180, -5, 19, 23),
             synth.shadow_view(30, 40, 64, 35.0, rng.uniform(0, 360)),
             synth.ortho_view((10 * 65536, 10 * 65536, 270 * 65536), (65536, 0, 0),
                              (0, 65536, 0), (0, 0, -1), 13, 11),
             synth.perspective_view(synth.eye_above_floor(F, B, 128.5, 128.5, dz=2), 0, 80, 24, 24)]
    set_march(ctx, far, steps, bisect)
    wg, dg = gpu_march(ctx, views)
    wo, do = oracle.march(F, B, T, views, far=far, steps=steps, bisect=bisect)
    assert_same(wg, dg, wo, do, "options %r" % ((far, steps, bisect),))


def test_read_count_matches_oracle(ctx):
    F, B, T = synth.make_map_from_config(1)
    load(ctx, F, B, T)
    views = synth.config_views(1, F, B) + [synth.shadow_view(10, 10, 100, 30.0, 45.0)]
    set_march(ctx)
    ctx.tc_set_option(tc.TC_OPT_COUNT_READS, 1)
    ctx.tc_read_counters()
    gpu_march(ctx, views)
    got = ctx.tc_read_counters()
    ctx.tc_set_option(tc.TC_OPT_COUNT_READS, 0)
    _, _, reads = oracle.march(F, B, T, views, with_reads=True)
    assert got == reads


def test_c2_full_image(ctx):
    F, B, T = synth.make_map_from_config(2)
    load(ctx, F, B, T)
    views = synth.config_views(2, F, B)
    set_march(ctx)
    wg, dg = gpu_march(ctx, views)
    wo, do = oracle.march(F, B, T, views)
    assert_same(wg, dg, wo, do, "c2 march")


def test_protocol_views_sampled_and_metrics(ctx):
    """The paper's protocol on the 2048x16384 map: twelve 1280x800 views,
    three per pitch; sampled pixels against the oracle, and the quality
    metrics of the GPU buffers against the exact render's."""
    F, B, T = config_map(3)
    load(ctx, F, B, T)
    views, pitches = synth.pitch_views(F, B, 91)
    set_march(ctx)
    wg, dg = gpu_march(ctx, views)
    va = synth.views_array(views)
    base = np.concatenate([[0], np.cumsum(va["width"].astype(np.int64) * va["height"])])
    rng = np.random.default_rng(92)
    n = 20000
    vi = rng.integers(0, len(views), n).astype(np.int32)
    px = rng.integers(0, 1280, n).astype(np.int32)
    py = rng.integers(0, 800, n).astype(np.int32)
    wo, do = oracle.march_pixels(F, B, T, views, vi, px, py)
    idx = base[vi] + py.astype(np.int64) * 1280 + px
    assert_same(wg[idx], dg[idx], wo, do, "protocol march")
    # metrics against the exact render of the same views
    ctx.tc_set_option(tc.TC_OPT_RENDER_MODE, 0)
    we, de = gpu_march(ctx, views)
    q = metrics.quality_views(wg, dg, we, de, views, far=600)
    for k, p in enumerate(pitches):
        assert 0 <= q[k]["see_through"] < 0.2, (p, q[k])
        assert q[k]["covers_sky"] < 0.01, (p, q[k])
    # a march hit is not in front of the exact hit, except where a sample
    # point, rounded to single precision (2^-9 units at y ~ 16000), lands in
    # a column the exact ray passes within that distance of
    hit = wg != oracle.MISS
    ahead = (we[hit] == oracle.MISS) | (dg[hit].astype(np.float64) < de[hit] * (1 - 1e-4) - 1e-2)
    assert np.mean(ahead) < 1e-3, np.mean(ahead)


def test_frame_with_edits_in_march_mode(ctx):
    F, B, T = synth.make_map_from_config(1)
    load(ctx, F, B, T)
    views = synth.config_views(1, F, B)
    edits = synth.crater_list(53, 256, 256, 5, size=(8, 40), depth=(10, 60))
    set_march(ctx, 400, 100, 4)
    out = torch.empty((synth.view_rays(views), 2), dtype=torch.int32, device="cuda")
    frame = ctx.tc_frame_create(views, edits, out.data_ptr())
    Fk, Bk, Tk = F, B, T
    for k in range(2):
        frame.launch()
        torch.cuda.synchronize()
        Fk, Bk, Tk = oracle.apply_edits(Fk, Bk, Tk, edits)
        wo, do = oracle.march(Fk, Bk, Tk, views, far=400, steps=100)
        wg, dg = tc.split_hits(out)
        assert_same(wg, dg, wo, do, "frame replay %d" % k)
    frame.close()
    with pytest.raises(tc.TCError):
        ctx.tc_autotune(views, out.data_ptr(), reps=1)


def test_kernel_timing_and_option_checks(ctx):
    F, B, T = synth.make_map_from_config(1)
    load(ctx, F, B, T)
    views = synth.config_views(1, F, B)
    set_march(ctx)
    ctx.tc_set_option(tc.TC_OPT_KERNEL_TIMING, 1)
    try:
        gpu_march(ctx, views)
        t0, t1 = ctx.tc_read_kernel_times()
        assert t0 > 0 and t1 == 0
    finally:
        ctx.tc_set_option(tc.TC_OPT_KERNEL_TIMING, 0)
    for key, bad in ((tc.TC_OPT_MARCH_STEPS, 0), (tc.TC_OPT_MARCH_STEPS, 65537),
                     (tc.TC_OPT_MARCH_BISECT, -1), (tc.TC_OPT_MARCH_BISECT, 65),
                     (tc.TC_OPT_MARCH_FAR, 0), (tc.TC_OPT_RENDER_MODE, 6)):
        with pytest.raises(tc.TCError) as e:
            ctx.tc_set_option(key, bad)
        assert e.value.status == tc.TC_INVALID_ARG
    assert ctx.tc_get_option(tc.TC_OPT_MARCH_STEPS) == 128
