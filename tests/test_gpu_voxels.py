"""The voxel occupancy pyramid and render mode 5 (the voxel-accelerated
march, Section 3.2) against the oracle: every level of the pyramid equals
its definition after a load and after edits (and a fresh build of the
edited map), and renders over it are bit-identical to the exact oracle."""
import numpy as np
import pytest

import oracle
import synth

tc = pytest.importorskip("paper_2608_17390_amd")
torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

from test_gpu_parity import assert_parity, load, _random_views  # noqa: E402

SHAPES = [(1, 1), (2, 2), (2, 4), (4, 2), (8, 8)]


@pytest.fixture(scope="module")
def ctx():
    assert torch.cuda.is_available()
    c = tc.Context(0)
    yield c
    c.tc_set_option(tc.TC_OPT_VOXEL_SHAPE, 0)
    c.close()


def shape_opt(v, vz):
    return v | (vz << 8)


def check_levels(ctx, F, B, T, v, vz):
    H, W = F.shape
    n = ctx.tc_voxel_dims(0)[3]
    expect = 1
    while oracle.voxel_dims(W, H, v, vz, expect - 1) != (1, 1, 1):
        expect += 1
    assert n == expect
    for k in range(n):
        got = ctx.tc_read_voxels(k)
        assert got.shape[::-1] == oracle.voxel_dims(W, H, v, vz, k), k
        assert np.array_equal(got, oracle.voxel_level_direct(F, B, T, v, vz, k)), (v, vz, k)
    assert ctx.tc_voxel_dims(n - 1)[:3] == (1, 1, 1)


def render(ctx, views, mode=5):
    ctx.tc_set_option(tc.TC_OPT_RENDER_MODE, mode)
    out = tc.render(ctx, views)
    torch.cuda.synchronize()
    ctx.tc_set_option(tc.TC_OPT_RENDER_MODE, 0)
    return tc.split_hits(out)


@pytest.mark.parametrize("v,vz", SHAPES)
def test_levels_and_renders_c1(ctx, v, vz):
    F, B, T = synth.make_map_from_config(1)
    load(ctx, F, B, T)
    ctx.tc_set_option(tc.TC_OPT_VOXEL_SHAPE, shape_opt(v, vz))
    check_levels(ctx, F, B, T, v, vz)
    rng = np.random.default_rng(40 + v * 10 + vz)
    views = synth.config_views(1, F, B) + _random_views(
        rng, F, B, 12, [(77, 53), (1, 1), (130, 9), (64, 64)])
    wo, do = oracle.render(F, B, T, views)
    for beam in (0, 4):
        ctx.tc_set_option(tc.TC_OPT_BEAM_PASSES, beam)
        wg, dg = render(ctx, views)
        assert_parity(wg, dg, wo, do, "voxels %dx%d beam %d" % (v, vz, beam))
    ctx.tc_set_option(tc.TC_OPT_BEAM_PASSES, 6)


@pytest.mark.parametrize("W,H", [(1, 1), (9, 1), (17, 3), (129, 65)])
def test_odd_maps(ctx, W, H):
    rng = np.random.default_rng(W * 7 + H)
    F, B, T = synth.make_map(W, H, 70 + W, dual=0.4, period=4)
    load(ctx, F, B, T)
    for v, vz in ((1, 1), (4, 2)):
        ctx.tc_set_option(tc.TC_OPT_VOXEL_SHAPE, shape_opt(v, vz))
        check_levels(ctx, F, B, T, v, vz)
        views = _random_views(rng, F, B, 5, [(23, 19), (8, 8)])
        wo, do = oracle.render(F, B, T, views)
        wg, dg = render(ctx, views)
        assert_parity(wg, dg, wo, do, "map %dx%d voxels %dx%d" % (W, H, v, vz))


@pytest.mark.parametrize("v,vz", SHAPES)
def test_rays_entering_below_ground(ctx, v, vz):
    """Steep rays from beside the map that are already below height 0 when
    they reach it: the floor is unbounded below, so the first wall they meet
    is a hit (regression: a height range wholly below 0 once tested no
    voxel)."""
    S = 65536
    F, B, T = synth.make_map(61, 45, 5, dual=0.35, period=16)
    load(ctx, F, B, T)
    ctx.tc_set_option(tc.TC_OPT_VOXEL_SHAPE, shape_opt(v, vz))
    views = [
        synth.ortho_view((0, 60 * S, 260 * S), (S // 2, 0, 0), (0, S // 2, 0),
                         (0.06, -0.01, -1.0), 120, 30),
        synth.ortho_view((-20 * S, 0, 100 * S), (0, S // 2, 0), (0, 0, S), (0.01, 0.003, -0.2), 90, 40),
        synth.ortho_view((70 * S, 50 * S, 30 * S), (-S // 2, 0, 0), (0, 0, S // 4),
                         (-0.1, -0.1, -0.5), 100, 60),
    ]
    wo, do = oracle.render(F, B, T, views)
    wg, dg = render(ctx, views)
    assert_parity(wg, dg, wo, do, "below ground voxels %dx%d" % (v, vz))
    assert np.count_nonzero(wo != oracle.MISS) > 1000


def test_edits_update_the_pyramid(ctx):
    """Craters and SET patches (some hanging over the map's edges): every
    voxel level equals the oracle's for the edited map and a fresh build;
    renders over the edited pyramid are exact; a captured frame replays the
    edits on the pyramid too."""
    F, B, T = synth.make_map_from_config(1)
    edits = (synth.crater_list(61, 256, 256, 12, size=(4, 64), depth=(0, 255)) +
             synth.random_set_patches(62, 256, 256, 8, max_size=40))
    edits += [dict(kind=2, x0=-10, y0=250, w=20, h=20, depth=30)]
    for v, vz in ((2, 2), (8, 4)):
        load(ctx, F, B, T)
        ctx.tc_set_option(tc.TC_OPT_VOXEL_SHAPE, shape_opt(v, vz))
        ctx.tc_apply_edit(edits)
        F2, B2, T2 = oracle.apply_edits(F, B, T, edits)
        check_levels(ctx, F2, B2, T2, v, vz)
        views = synth.config_views(1, F, B) + [synth.shadow_view(30, 40, 64, 35.0, 70.0)]
        wo, do = oracle.render(F2, B2, T2, views)
        wg, dg = render(ctx, views)
        assert_parity(wg, dg, wo, do, "edited voxels %dx%d" % (v, vz))
    # frames: edits, dirty updates (pyramid, windows, voxels) and a mode-5
    # render in one graph, replayed
    load(ctx, F, B, T)
    ctx.tc_set_option(tc.TC_OPT_VOXEL_SHAPE, shape_opt(2, 4))
    ctx.tc_set_option(tc.TC_OPT_RENDER_MODE, 5)
    views = synth.config_views(1, F, B)
    out = torch.empty((synth.view_rays(views), 2), dtype=torch.int32, device="cuda")
    frame = ctx.tc_frame_create(views, edits[:6], out.data_ptr())
    ctx.tc_set_option(tc.TC_OPT_RENDER_MODE, 0)
    Fk, Bk, Tk = F, B, T
    try:
        for k in range(2):
            frame.launch()
            torch.cuda.synchronize()
            Fk, Bk, Tk = oracle.apply_edits(Fk, Bk, Tk, edits[:6])
            wg, dg = tc.split_hits(out)
            wo, do = oracle.render(Fk, Bk, Tk, views)
            assert_parity(wg, dg, wo, do, "voxel frame replay %d" % k)
        check_levels(ctx, Fk, Bk, Tk, 2, 4)
    finally:
        frame.close()


def test_cave_map_and_c2(ctx):
    """Half the cells two-layer (the case an occupancy pyramid is for) and
    the headline view, with the paper's voxel proportions."""
    F, B, T = synth.cave_map(97, 512, 512)
    load(ctx, F, B, T)
    ctx.tc_set_option(tc.TC_OPT_VOXEL_SHAPE, shape_opt(2, 1))
    rng = np.random.default_rng(99)
    views = _random_views(rng, F, B, 8, [(96, 64), (64, 48)])
    ys, xs = np.nonzero((B > 0) & (B.astype(int) - F.astype(int) > 6))
    for k in rng.choice(ys.size, 4, replace=False):
        x, y = int(xs[k]), int(ys[k])
        views.append(synth.perspective_view((x + 0.5, y + 0.5, (int(F[y, x]) + int(B[y, x])) / 2),
                                            rng.uniform(0, 360), rng.uniform(-30, 10), 48, 32))
    wo, do = oracle.render(F, B, T, views)
    wg, dg = render(ctx, views)
    assert_parity(wg, dg, wo, do, "cave map voxels")
    F, B, T = synth.make_map_from_config(2)
    load(ctx, F, B, T)
    ctx.tc_set_option(tc.TC_OPT_VOXEL_SHAPE, shape_opt(4, 2))
    views = synth.config_views(2, F, B)
    wo, do = oracle.render(F, B, T, views)
    wg, dg = render(ctx, views)
    assert_parity(wg, dg, wo, do, "c2 voxels")


def test_errors(ctx):
    F, B, T = synth.make_map_from_config(1)
    load(ctx, F, B, T)
    ctx.tc_set_option(tc.TC_OPT_VOXEL_SHAPE, 0)
    views = synth.config_views(1, F, B)
    out = torch.empty((synth.view_rays(views), 2), dtype=torch.int32, device="cuda")
    ctx.tc_set_option(tc.TC_OPT_RENDER_MODE, 5)
    with pytest.raises(tc.TCError) as e:
        ctx.tc_render_views(views, out.data_ptr())
    assert e.value.status == tc.TC_INVALID_ARG
    ctx.tc_set_option(tc.TC_OPT_RENDER_MODE, 0)
    for bad in (3, 2 | (3 << 8), 16, 1 | (16 << 8)):
        with pytest.raises(tc.TCError):
            ctx.tc_set_option(tc.TC_OPT_VOXEL_SHAPE, bad)
    with pytest.raises(tc.TCError) as e:
        ctx.tc_voxel_dims(0)
    ctx.tc_set_option(tc.TC_OPT_VOXEL_SHAPE, shape_opt(2, 2))
    with pytest.raises(tc.TCError):
        ctx.tc_server_start(16 << 20)
    ctx.tc_set_option(tc.TC_OPT_VOXEL_SHAPE, 0)
    srv = ctx.tc_server_start(16 << 20)
    srv.tc_server_stop()
