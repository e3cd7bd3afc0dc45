"""GPU parity: the HIP library against the CPU oracle, through the C ABI.

Hit words (cell, face, layer) must match bit for bit; FP32 depth must be
within 1e-5 relative of the oracle's FP64 depth (exactly 0 for inside hits
and +inf for misses)."""
import numpy as np
import pytest

import oracle
import synth
from oracle_cache import config_map, oracle_render

tc = pytest.importorskip("paper_2608_17390_amd")
torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

S = 65536
# (render mode, packet beam passes): the hierarchical modes run with the
# beam start (the default) and without it
MODES = {"hier": (0, 6), "hier_nobeam": (0, 0), "flat": (1, 0), "persistent": (2, 0),
         "occupancy": (4, 6)}
DEPTH_RTOL = 1e-5


@pytest.fixture(scope="module")
def ctx():
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    c = tc.Context(0)
    yield c
    c.close()


def gpu_render(ctx, views, mode="hier"):
    ctx.tc_set_option(tc.TC_OPT_RENDER_MODE, MODES[mode][0])
    ctx.tc_set_option(tc.TC_OPT_BEAM_PASSES, MODES[mode][1])
    out = tc.render(ctx, views)
    torch.cuda.synchronize()
    ctx.tc_set_option(tc.TC_OPT_BEAM_PASSES, 6)
    return tc.split_hits(out)


def assert_parity(wg, dg, wo, do, what=""):
    """Every record: word bit-exact; depth +inf on a miss, exactly 0 where
    the oracle's is 0 (inside), else within DEPTH_RTOL relative.  Large
    buffers are checked in chunks to bound the memory used."""
    assert wg.shape == wo.shape, "%s: %s records vs %s" % (what, wg.shape, wo.shape)
    bad = np.nonzero(wg != wo)[0]
    assert bad.size == 0, "%s: %d word mismatches, first at %d: gpu %08x oracle %08x" % (
        what, bad.size, bad[0], wg[bad[0]], wo[bad[0]])
    step = 1 << 23
    for c0 in range(0, wo.size, step):
        w = wo[c0:c0 + step]
        d = dg[c0:c0 + step]
        ref_all = do[c0:c0 + step]
        miss = w == oracle.MISS
        assert np.all(np.isinf(d[miss])), "%s: a miss without +inf depth" % what
        hit = ~miss
        dg64 = d[hit].astype(np.float64)
        ref = ref_all[hit]
        err = np.abs(dg64 - ref)
        tol = DEPTH_RTOL * np.abs(ref)
        if not np.all(err <= tol):
            worst = np.argmax(err - tol)
            raise AssertionError("%s: depth off by %g at %g" % (what, err[worst], ref[worst]))
        assert np.all(dg64[ref == 0] == 0), "%s: inside hit with nonzero depth" % what


def load(ctx, F, B, T):
    ctx.tc_load_columns(F, B, T)
    torch.cuda.synchronize()


@pytest.mark.parametrize("mode", list(MODES))
def test_c1_full_image(ctx, mode):
    F, B, T = synth.make_map_from_config(1)
    views = synth.config_views(1, F, B)
    load(ctx, F, B, T)
    wo, do = oracle.render(F, B, T, views)
    wg, dg = gpu_render(ctx, views, mode)
    assert_parity(wg, dg, wo, do, "c1 " + mode)


def _random_views(rng, F, B, n, sizes):
    H, W = F.shape
    out = []
    for k in range(n):
        w, h = sizes[k % len(sizes)]
        if k % 3 == 2:
            x0 = int(rng.integers(-10, W))
            y0 = int(rng.integers(-10, H))
            el = rng.uniform(20, 89)
            out.append(synth.shadow_view(x0, y0, max(w, h), el, rng.uniform(0, 360)))
            continue
        try:
            eye = synth.eye_above_floor(F, B, rng.uniform(0, W), rng.uniform(0, H),
                                        dz=float(rng.uniform(0.5, 40)))
        except ValueError:   # every cell has a slab: look from above
            eye = (rng.uniform(0, W), rng.uniform(0, H), 300.0)
        out.append(synth.perspective_view(eye, rng.uniform(0, 360),
                                          rng.uniform(-89, 60), w, h,
                                          vfov_deg=rng.uniform(20, 120)))
    return out


@pytest.mark.parametrize("mode", list(MODES))
def test_ragged_multi_view_batch(ctx, mode):
    """Many views of ragged sizes (partial 8x8 tiles, 1x1, thin strips) in
    one call; views concatenated in order."""
    rng = np.random.default_rng(21)
    F, B, T = synth.make_map_from_config(1)
    load(ctx, F, B, T)
    sizes = [(77, 53), (1, 1), (8, 9), (13, 200), (300, 2), (64, 64), (9, 8)]
    views = _random_views(rng, F, B, 21, sizes)
    wo, do = oracle.render(F, B, T, views)
    wg, dg = gpu_render(ctx, views, mode)
    assert_parity(wg, dg, wo, do, "ragged " + mode)


@pytest.mark.parametrize("mode", ["hier", "persistent", "occupancy"])
def test_c2_full_image(ctx, mode):
    F, B, T = synth.make_map_from_config(2)
    views = synth.config_views(2, F, B)
    load(ctx, F, B, T)
    wo, do = oracle.render(F, B, T, views)
    wg, dg = gpu_render(ctx, views, mode)
    assert_parity(wg, dg, wo, do, "c2 " + mode)


def test_kernel_timing_leaves_results_unchanged(ctx):
    """TC_OPT_KERNEL_TIMING times the kernels with events (attached to the
    kernels when the tables travel in their arguments, markers on the stream
    otherwise): results are the same bytes, times are positive, the split
    pass time is 0 when that pass is off, and reading before any timed
    render is an error."""
    budget0 = ctx.tc_get_option(tc.TC_OPT_SPLIT_BUDGET)
    F, B, T = synth.make_map_from_config(2)
    load(ctx, F, B, T)
    views = synth.config_views(2, F, B)
    ref = gpu_render(ctx, views, "hier")
    ctx.tc_set_option(tc.TC_OPT_KERNEL_TIMING, 1)
    with pytest.raises(tc.TCError) as e:
        ctx.tc_read_kernel_times()
    assert e.value.status == tc.TC_INVALID_ARG
    try:
        for mode, budget, inline in (("hier", 128, 1), ("hier", 0, 1), ("hier", 128, 0),
                                     ("hier", 0, 0), ("flat", 128, 1), ("persistent", 128, 1)):
            ctx.tc_set_option(tc.TC_OPT_SPLIT_BUDGET, budget)
            ctx.tc_set_option(tc.TC_OPT_INLINE_TABLES, inline)
            w, d = gpu_render(ctx, views, mode)
            assert np.array_equal(w, ref[0]), mode
            assert np.array_equal(d.view(np.uint32), ref[1].view(np.uint32)), mode
            t0, t1 = ctx.tc_read_kernel_times()
            assert t0 > 0
            assert (t1 > 0) == (mode == "hier" and budget > 0), (mode, budget, t1)
    finally:
        ctx.tc_set_option(tc.TC_OPT_KERNEL_TIMING, 0)
        ctx.tc_set_option(tc.TC_OPT_SPLIT_BUDGET, budget0)
        ctx.tc_set_option(tc.TC_OPT_INLINE_TABLES, 1)
        ctx.tc_set_option(tc.TC_OPT_RENDER_MODE, 0)


def test_occupancy_mode_on_a_cave_heavy_map(ctx):
    """Half the cells two-layer, with slabs at scattered heights (the case
    the occupancy masks are for): the masks match their definition and the
    occupancy mode is bit-identical to the oracle on eye-level, cave and
    oblique views."""
    F, B, T = synth.cave_map(97, 512, 512)
    load(ctx, F, B, T)
    for L in range(1, ctx.tc_pyramid_info() + 1):
        assert np.array_equal(ctx.tc_read_occupancy(L), oracle.occupancy_level(F, B, T, L)), L
    rng = np.random.default_rng(98)
    views = _random_views(rng, F, B, 8, [(96, 64), (64, 48)])
    ys, xs = np.nonzero((B > 0) & (B.astype(int) - F.astype(int) > 6))
    for k in rng.choice(ys.size, 6, replace=False):
        x, y = int(xs[k]), int(ys[k])
        views.append(synth.perspective_view((x + 0.5, y + 0.5, (int(F[y, x]) + int(B[y, x])) / 2),
                                            rng.uniform(0, 360), rng.uniform(-30, 10), 48, 32))
    wo, do = oracle.render(F, B, T, views)
    for mode in ("occupancy", "hier"):
        wg, dg = gpu_render(ctx, views, mode)
        assert_parity(wg, dg, wo, do, "cave map " + mode)


def test_modes_identical_bytes(ctx):
    F, B, T = synth.make_map_from_config(2)
    load(ctx, F, B, T)
    rng = np.random.default_rng(5)
    views = _random_views(rng, F, B, 9, [(640, 480), (256, 256), (333, 97)])
    res = [gpu_render(ctx, views, m) for m in MODES]
    for w, d in res[1:]:
        assert np.array_equal(w, res[0][0])
        assert np.array_equal(d.view(np.uint32), res[0][1].view(np.uint32))
    # run-to-run determinism
    w2, d2 = gpu_render(ctx, views, "persistent")
    assert np.array_equal(w2, res[0][0])


def test_level_options_do_not_change_results(ctx):
    F, B, T = synth.make_map_from_config(1)
    load(ctx, F, B, T)
    rng = np.random.default_rng(8)
    views = _random_views(rng, F, B, 6, [(128, 96), (50, 70)])
    base = gpu_render(ctx, views, "flat")
    for start, top in [(0, 3), (4, 15), (8, 8), (15, 1), (2, 0)]:
        ctx.tc_set_option(tc.TC_OPT_START_LEVEL, start)
        ctx.tc_set_option(tc.TC_OPT_MAX_LEVEL, top)
        for mode in ("hier", "persistent"):
            w, d = gpu_render(ctx, views, mode)
            assert np.array_equal(w, base[0]), (start, top, mode)
    ctx.tc_set_option(tc.TC_OPT_START_LEVEL, 0)
    ctx.tc_set_option(tc.TC_OPT_MAX_LEVEL, 15)
    for rmin, iters, waves in [(1, 1, 4), (64, 3, 8), (7, 200, 32)]:
        ctx.tc_set_option(tc.TC_OPT_REFILL_MIN, rmin)
        ctx.tc_set_option(tc.TC_OPT_REFILL_ITERS, iters)
        ctx.tc_set_option(tc.TC_OPT_PERSIST_WAVES, waves)
        w, d = gpu_render(ctx, views, "persistent")
        assert np.array_equal(w, base[0]), (rmin, iters, waves)
    ctx.tc_set_option(tc.TC_OPT_REFILL_MIN, 16)
    ctx.tc_set_option(tc.TC_OPT_REFILL_ITERS, 16)
    ctx.tc_set_option(tc.TC_OPT_PERSIST_WAVES, 16)


def test_packet_orders_and_xcd_groups(ctx):
    """Every packet order and XCD grouping gives the same bytes."""
    F, B, T = synth.make_map_from_config(1)
    load(ctx, F, B, T)
    rng = np.random.default_rng(12)
    views = _random_views(rng, F, B, 12, [(77, 53), (130, 9), (8, 300), (64, 64)])
    wo, do = oracle.render(F, B, T, views)
    for order in (0, 1, 2):
        for remap in (0, 3, 64):
            ctx.tc_set_option(tc.TC_OPT_TILE_ORDER, order)
            ctx.tc_set_option(tc.TC_OPT_XCD_REMAP, remap)
            for mode in MODES:
                wg, dg = gpu_render(ctx, views, mode)
                assert_parity(wg, dg, wo, do, "order %d remap %d %s" % (order, remap, mode))
    ctx.tc_set_option(tc.TC_OPT_TILE_ORDER, 2)
    ctx.tc_set_option(tc.TC_OPT_XCD_REMAP, 64)


@pytest.mark.parametrize("width", [4, 16, 32])
def test_packet_widths(ctx, width):
    """Packets of 4x16, 16x4 and 32x2 pixels (one wave each): every mode,
    every packet order, ragged views (partial packets on both axes), the
    packet beam on, and the c2 image, against the oracle."""
    F, B, T = synth.make_map_from_config(1)
    load(ctx, F, B, T)
    rng = np.random.default_rng(30 + width)
    views = _random_views(rng, F, B, 12, [(77, 53), (1, 1), (130, 9), (8, 300), (33, 3), (64, 64)])
    wo, do = oracle.render(F, B, T, views)
    ctx.tc_set_option(tc.TC_OPT_PACKET_WIDTH, width)
    try:
        for order in (0, 1, 2):
            ctx.tc_set_option(tc.TC_OPT_TILE_ORDER, order)
            for mode in MODES:
                wg, dg = gpu_render(ctx, views, mode)
                assert_parity(wg, dg, wo, do, "width %d order %d %s" % (width, order, mode))
        ctx.tc_set_option(tc.TC_OPT_TILE_ORDER, 2)
        F, B, T = synth.make_map_from_config(2)
        load(ctx, F, B, T)
        views = synth.config_views(2, F, B)
        wo, do = oracle.render(F, B, T, views)
        wg, dg = gpu_render(ctx, views, "hier")
        assert_parity(wg, dg, wo, do, "c2 width %d" % width)
    finally:
        ctx.tc_set_option(tc.TC_OPT_PACKET_WIDTH, 8)
        ctx.tc_set_option(tc.TC_OPT_TILE_ORDER, 2)


@pytest.mark.parametrize("budget,queue,waves", [(1, 1 << 20, 4), (5, 1 << 20, 1), (5, 1 << 20, 2),
                                               (1, 7, 2), (30, 1000, 4)])
def test_split_pass(ctx, budget, queue, waves):
    """Rays still walking after `budget` steps are finished by 64 parallel
    segment walks per wave, `waves` waves per ray; a tiny budget sends
    nearly every ray there, a tiny queue leaves the overflow to the first
    pass.  Results must not change."""
    budget0 = ctx.tc_get_option(tc.TC_OPT_SPLIT_BUDGET)
    F, B, T = synth.make_map_from_config(1)
    load(ctx, F, B, T)
    rng = np.random.default_rng(13)
    views = synth.config_views(1, F, B) + _random_views(
        rng, F, B, 9, [(77, 53), (8, 9), (130, 64)])
    wo, do = oracle.render(F, B, T, views)
    ctx.tc_set_option(tc.TC_OPT_SPLIT_BUDGET, budget)
    ctx.tc_set_option(tc.TC_OPT_SPLIT_QUEUE, queue)
    ctx.tc_set_option(tc.TC_OPT_SPLIT_WAVES, waves)
    try:
        for order, start in ((0, 0), (2, 2), (2, 5)):
            ctx.tc_set_option(tc.TC_OPT_TILE_ORDER, order)
            ctx.tc_set_option(tc.TC_OPT_START_LEVEL, start)
            wg, dg = gpu_render(ctx, views, "hier")
            assert_parity(wg, dg, wo, do, "split budget %d queue %d waves %d start %d" % (
                budget, queue, waves, start))
    finally:
        ctx.tc_set_option(tc.TC_OPT_SPLIT_BUDGET, budget0)
        ctx.tc_set_option(tc.TC_OPT_SPLIT_QUEUE, 1 << 17)
        ctx.tc_set_option(tc.TC_OPT_SPLIT_WAVES, 4)
        ctx.tc_set_option(tc.TC_OPT_TILE_ORDER, 2)
        ctx.tc_set_option(tc.TC_OPT_START_LEVEL, 2)


def test_inline_tables(ctx):
    """A call whose tables fit in the kernels' arguments uploads nothing, and
    its split pass clears the ring slot's queue counters for the slot's next
    use.  Calls with and without inline tables, small and large split
    budgets and queues (overflowing ones too), and calls too large to travel
    inline are interleaved over more calls than the ring has slots; every
    record equals the oracle's."""
    budget0 = ctx.tc_get_option(tc.TC_OPT_SPLIT_BUDGET)
    F, B, T = synth.make_map_from_config(1)
    load(ctx, F, B, T)
    rng = np.random.default_rng(17)
    one = synth.config_views(1, F, B)
    two = one + _random_views(rng, F, B, 1, [(130, 64)])
    many = one + _random_views(rng, F, B, 13, [(77, 53), (8, 9), (130, 64)])   # > 1536 B
    sets = [(vs, oracle.render(F, B, T, vs)) for vs in (one, two, many)]
    plans = [(1, 128, 1 << 17), (1, 1, 1 << 17), (0, 1, 1 << 17), (1, 5, 7), (1, 0, 1 << 17),
             (1, 30, 1000)]
    try:
        for k in range(48):
            inline, budget, queue = plans[k % len(plans)]
            vs, (wo, do) = sets[(k // 2) % 3]
            ctx.tc_set_option(tc.TC_OPT_INLINE_TABLES, inline)
            ctx.tc_set_option(tc.TC_OPT_SPLIT_BUDGET, budget)
            ctx.tc_set_option(tc.TC_OPT_SPLIT_QUEUE, queue)
            wg, dg = gpu_render(ctx, vs, "hier")
            assert_parity(wg, dg, wo, do, "call %d: inline %d budget %d queue %d views %d" % (
                k, inline, budget, queue, len(vs)))
    finally:
        ctx.tc_set_option(tc.TC_OPT_INLINE_TABLES, 1)
        ctx.tc_set_option(tc.TC_OPT_SPLIT_BUDGET, budget0)
        ctx.tc_set_option(tc.TC_OPT_SPLIT_QUEUE, 1 << 17)
    for bad in (-1, 2):
        with pytest.raises(tc.TCError):
            ctx.tc_set_option(tc.TC_OPT_INLINE_TABLES, bad)
    assert ctx.tc_get_option(tc.TC_OPT_INLINE_TABLES) == 1


def test_split_pass_edge_rays_and_large_map(ctx):
    """Split walks on rays from outside the map, along cell edges and over
    the 2048x2048 map's long horizon rays."""
    budget0 = ctx.tc_get_option(tc.TC_OPT_SPLIT_BUDGET)
    F, B, T = synth.make_map(61, 45, 3, dual=0.35, period=16)
    load(ctx, F, B, T)
    views = [
        synth.ortho_view((0, -5 * S, 40 * S), (S, 0, 0), (0, S // 4, 0), (0, 3, -1), 62, 60),
        synth.ortho_view((-5 * S, 0, 80 * S), (0, S, 0), (0, 0, S // 2), (5, 0, -2), 46, 70),
        synth.ortho_view((0, 0, 60 * S), (S, 0, 0), (0, S, 0), (1, 1, -1), 61, 45),
        synth.perspective_view((-500.0, -300.0, 90.0), 45, -3, 64, 48),
        synth.perspective_view((30.5, 22.5, 400.0), 10, -89.9, 50, 50),
    ]
    wo, do = oracle.render(F, B, T, views)
    ctx.tc_set_option(tc.TC_OPT_SPLIT_BUDGET, 2)
    try:
        wg, dg = gpu_render(ctx, views, "hier")
        assert_parity(wg, dg, wo, do, "split edge")
        F, B, T = synth.make_map_from_config(2)
        load(ctx, F, B, T)
        v = synth.config_views(2, F, B)
        wo, do = oracle.render(F, B, T, v)
        for budget, waves in ((8, 4), (96, 1), (96, 2)):
            ctx.tc_set_option(tc.TC_OPT_SPLIT_BUDGET, budget)
            ctx.tc_set_option(tc.TC_OPT_SPLIT_WAVES, waves)
            wg, dg = gpu_render(ctx, v, "hier")
            assert_parity(wg, dg, wo, do, "split c2 budget %d waves %d" % (budget, waves))
    finally:
        ctx.tc_set_option(tc.TC_OPT_SPLIT_BUDGET, budget0)
        ctx.tc_set_option(tc.TC_OPT_SPLIT_WAVES, 4)


def test_straight_down_closed_form_large_map(ctx):
    """Straight-down orthographic image over the whole 2048x16384 map: each
    hit is the column's topmost solid, face top, depth 256 - height."""
    F, B, T = config_map(3)
    H, W = F.shape
    load(ctx, F, B, T)
    v = synth.ortho_view((0, 0, 256 * S), (S // 2, 0, 0), (0, S // 2, 0),
                         (0, 0, -1), W, H)
    wg, dg = gpu_render(ctx, [v], "hier")
    top = np.where(B > 0, T, F).reshape(-1).astype(np.float32)
    layer = (B > 0).reshape(-1).astype(np.uint32)
    exp = np.arange(W * H, dtype=np.uint32) | np.uint32(1 << 27) | (layer << np.uint32(30))
    assert np.array_equal(wg, exp)
    assert np.array_equal(dg, np.float32(256) - top)


def test_edge_rays(ctx):
    """Origins outside the map, vertical rays, zero directions, rays
    running exactly along cell edges and through lattice corners."""
    rng = np.random.default_rng(9)
    F, B, T = synth.make_map(61, 45, 3, dual=0.35, period=16)
    load(ctx, F, B, T)
    views = [
        # zero direction: every ray misses
        synth.ortho_view((S, S, 10 * S), (S // 2, 0, 0), (0, S // 2, 0), (0, 0, 0), 9, 9),
        # vertical up and down from cell corners and centres
        synth.ortho_view((0, 0, 3 * S), (S // 2, 0, 0), (0, S // 2, 0), (0, 0, 1), 61, 45),
        synth.ortho_view((-S, -S, 300 * S), (S, 0, 0), (0, S, 0), (0, 0, -7), 40, 30),
        # along cell edges (integer x, dx = 0) and along rows
        synth.ortho_view((0, -5 * S, 40 * S), (S, 0, 0), (0, S // 4, 0), (0, 3, -1), 62, 60),
        synth.ortho_view((-5 * S, 0, 80 * S), (0, S, 0), (0, 0, S // 2), (5, 0, -2), 46, 70),
        # 45 degree diagonals through lattice corners
        synth.ortho_view((0, 0, 60 * S), (S, 0, 0), (0, S, 0), (1, 1, -1), 61, 45),
        synth.ortho_view((61 * S, 45 * S, 60 * S), (-S, 0, 0), (0, -S, 0), (-1, -1, -1), 61, 45),
        # from far outside the map, toward it and away from it
        synth.perspective_view((-500.0, -300.0, 90.0), 45, -3, 64, 48),
        synth.perspective_view((700.0, 20.0, 50.0), 90, 0, 32, 32),
        synth.perspective_view((30.5, 22.5, 400.0), 10, -89.9, 50, 50),
    ]
    for _ in range(6):
        views.append(synth.perspective_view(
            (rng.uniform(-100, 160), rng.uniform(-100, 140), rng.uniform(-20, 300)),
            rng.uniform(0, 360), rng.uniform(-90, 90), 31, 17))
    wo, do = oracle.render(F, B, T, views)
    for mode in MODES:
        wg, dg = gpu_render(ctx, views, mode)
        assert_parity(wg, dg, wo, do, "edge " + mode)
    assert np.all(wo[:81] == oracle.MISS)


def test_wide_pixel_steps(ctx):
    """Views whose per-pixel origin or direction steps reach 2^22 and more
    (pixels 128 cells apart, directions swinging across the full range
    between neighbouring pixels), batched with ordinary views: the kernels
    form a lane's ray from its packet's first pixel with 24-bit
    multiply-adds only while every step of the view is below 2^22, and in
    32-bit wrapping arithmetic otherwise."""
    rng = np.random.default_rng(21)
    F, B, T = synth.make_map(300, 220, 22, dual=0.35, period=16)
    load(ctx, F, B, T)
    big = 1 << 22
    views = [
        # origins 2 * 2^22 / S = 128 cells apart, one step exactly -2^22
        synth.ortho_view((-60 * S, -40 * S, 200 * S), (big, 0, 0), (0, big + 4321, 0),
                         (0.3, 0.4, -1), 4, 3),
        synth.ortho_view((500 * S, 400 * S, 90 * S), (-big, S // 3, 0), (12345, -big - 7, 3 * S),
                         (-1, -0.7, -0.2), 5, 9),
        # one step just below the limit, the others tiny
        synth.ortho_view((-30 * S, 5 * S, 150 * S), (big - 1, 0, 0), (0, S, 0), (0.2, 1, -0.5), 3, 40),
    ]
    for _ in range(8):
        v = np.zeros((), synth.VIEW_DTYPE)
        w, h = int(rng.integers(1, 3)), int(rng.integers(1, 3))
        v["width"], v["height"] = w, h
        v["o0"] = [int(rng.integers(20, 280)) * S, int(rng.integers(20, 200)) * S,
                   int(rng.integers(30, 120)) * S]
        # D = d0 + a dpx + b dpy with a, b in {1, 3}: steps of 2^22 and more
        # still keep |D| within 2^23 - 1
        dpx = [int(rng.choice([-1, 1])) * int(rng.integers(big, big + 200)) for _ in range(2)] + [0]
        dpy = [0, 0, int(rng.choice([-1, 1])) * int(rng.integers(big // 2, big + 100))]
        v["d_px"], v["d_py"] = dpx, dpy
        v["d0"] = [-2 * dpx[0] if w == 2 else -dpx[0] // 2, -2 * dpx[1] if w == 2 else 0,
                   -2 * dpy[2] if h == 2 else -dpy[2] - int(rng.integers(1, 1000))]
        views.append(v)
    views += _random_views(rng, F, B, 3, [(20, 12), (9, 9)])
    wo, do = oracle.render(F, B, T, views)
    for mode in MODES:
        wg, dg = gpu_render(ctx, views, mode)
        assert_parity(wg, dg, wo, do, "wide steps " + mode)
    assert np.count_nonzero(wo != oracle.MISS) > 30


def test_single_cell_and_odd_maps(ctx):
    rng = np.random.default_rng(4)
    for (W, H) in [(1, 1), (1, 9), (9, 1), (17, 3), (129, 65)]:
        F, B, T = synth.make_map(W, H, 40 + W, dual=0.4, period=4)
        load(ctx, F, B, T)
        views = _random_views(rng, F, B, 5, [(23, 19), (8, 8)])
        wo, do = oracle.render(F, B, T, views)
        for mode in MODES:
            wg, dg = gpu_render(ctx, views, mode)
            assert_parity(wg, dg, wo, do, "map %dx%d %s" % (W, H, mode))


def test_widest_view(ctx):
    F, B, T = synth.make_map_from_config(1)
    load(ctx, F, B, T)
    v = synth.perspective_view(synth.eye_above_floor(F, B, 40.5, 10.5), 0, 0, 16384, 2,
                               vfov_deg=1.0)
    wo, do = oracle.render(F, B, T, [v])
    wg, dg = gpu_render(ctx, [v], "hier")
    assert_parity(wg, dg, wo, do, "16384x2")


@pytest.mark.parametrize("shape", [(256, 256), (2048, 2048), (77, 1000)])
def test_pyramid_matches_definition(ctx, shape):
    W, H = shape
    F, B, T = synth.make_map(W, H, 600 + W, dual=0.3, period=32)
    load(ctx, F, B, T)
    levels = ctx.tc_pyramid_info()
    assert (1 << levels) >= max(W, H) > (1 << (levels - 1)) or max(W, H) == 1
    for L in range(1, levels + 1):
        assert np.array_equal(ctx.tc_read_pyramid(L), oracle.pyramid_level_fast(F, B, T, L)), L
        assert np.array_equal(ctx.tc_read_occupancy(L), oracle.occupancy_level(F, B, T, L)), L
    for L in range(0, levels + 1):
        assert np.array_equal(ctx.tc_read_window(L), oracle.window_level_fast(F, B, T, L)), L
    f2, b2, t2 = ctx.tc_read_columns(0, 0, W, H)
    assert np.array_equal(f2, F) and np.array_equal(b2, B) and np.array_equal(t2, T)


def _edited_checks(ctx, F, B, T, edits, views, oracle_result=None):
    """Apply edits on the GPU; compare the map with the oracle's edit, the
    pyramid with a fresh build of the edited map, and renders with both the
    oracle and a fresh load."""
    H, W = F.shape
    load(ctx, F, B, T)
    ctx.tc_apply_edit(edits)
    F2, B2, T2 = oracle.apply_edits(F, B, T, edits)
    g = ctx.tc_read_columns(0, 0, W, H)
    assert np.array_equal(g[0], F2) and np.array_equal(g[1], B2) and np.array_equal(g[2], T2)
    levels = ctx.tc_pyramid_info()
    pyr_edit = [ctx.tc_read_pyramid(L) for L in range(1, levels + 1)]
    occ_edit = [ctx.tc_read_occupancy(L) for L in range(1, levels + 1)]
    win_edit = [ctx.tc_read_window(L) for L in range(0, levels + 1)]
    res_edit = {m: gpu_render(ctx, views, m) for m in ("hier", "persistent", "occupancy")}
    load(ctx, F2, B2, T2)
    for L in range(1, levels + 1):
        assert np.array_equal(ctx.tc_read_pyramid(L), pyr_edit[L - 1]), L
        assert np.array_equal(ctx.tc_read_occupancy(L), occ_edit[L - 1]), L
        assert np.array_equal(occ_edit[L - 1], oracle.occupancy_level(F2, B2, T2, L)), L
    for L in range(0, levels + 1):
        assert np.array_equal(ctx.tc_read_window(L), win_edit[L]), L
        assert np.array_equal(win_edit[L], oracle.window_level_fast(F2, B2, T2, L)), L
    w_fresh, d_fresh = gpu_render(ctx, views, "hier")
    for m, (w, d) in res_edit.items():
        assert np.array_equal(w, w_fresh), m
        assert np.array_equal(d.view(np.uint32), d_fresh.view(np.uint32)), m
    wo, do = oracle_result if oracle_result is not None else oracle.render(F2, B2, T2, views)
    assert_parity(w_fresh, d_fresh, wo, do, "edited")
    for m, (w, d) in res_edit.items():
        assert_parity(w, d, wo, do, "edited " + m)


def test_edits_small_map(ctx):
    F, B, T = synth.make_map_from_config(1)
    edits = (synth.crater_list(31, 256, 256, 20, size=(4, 64), depth=(0, 255)) +
             synth.random_set_patches(32, 256, 256, 15, max_size=40))
    rng = np.random.default_rng(33)
    rng.shuffle(edits)
    # overlapping edits on one spot, and patches hanging over every edge
    edits += [dict(kind=2, x0=100, y0=100, w=32, h=32, depth=50),
              dict(kind=2, x0=110, y0=104, w=16, h=16, depth=90),
              dict(kind=2, x0=-10, y0=250, w=20, h=20, depth=30),
              dict(kind=2, x0=250, y0=-7, w=12, h=12, depth=30)]
    edits += synth.random_set_patches(34, 256, 256, 3, max_size=12)
    views = synth.config_views(1, F, B) + _random_views(rng, F, B, 5, [(96, 64)])
    _edited_checks(ctx, F, B, T, edits, views)


@pytest.mark.parametrize("shape", [(1, 1), (2, 1), (3, 2), (5, 7), (16, 9), (17, 3), (33, 20),
                                   (65, 100), (129, 65), (300, 220), (77, 1000), (2049, 60)])
def test_edits_every_level_grouping(ctx, shape):
    """The dirty update climbs three pyramid levels per launch, each from the
    level below its group; maps whose top level is 0 to 12 cover every way
    the levels fall into groups (a last group of one, two or three levels,
    and a map with no pyramid level above the cells)."""
    W, H = shape
    F, B, T = synth.make_map(W, H, 700 + W + H, dual=0.4, period=4)
    rng = np.random.default_rng(W * 7 + H)
    m = max(W, H)
    edits = (synth.crater_list(rng, W, H, 12, size=(1, min(64, m)), depth=(0, 255)) +
             synth.random_set_patches(rng, W, H, 8, max_size=max(1, min(40, m))))
    rng.shuffle(edits)
    # one crater over the whole map, one hanging over its far corner
    edits += [dict(kind=2, x0=0, y0=0, w=min(W, H, 4096), h=min(W, H, 4096), depth=40),
              dict(kind=2, x0=W - 2, y0=H - 2, w=5, h=5, depth=90)]
    views = _random_views(rng, F, B, 3, [(24, 16), (8, 8)])
    _edited_checks(ctx, F, B, T, edits, views)


@pytest.mark.parametrize("case", ["scattered", "clustered"])
def test_long_edit_lists(ctx, case):
    """Long edit lists: a cell tests only the edits whose rectangles meet its
    edit's, listed on the host from a grid of 128-cell buckets (300 edits
    scattered over the map), or, with more than 512 edits in one bucket
    (700 edits within 96 x 96 cells), every edit against every other; the
    map and every pyramid level against the oracle's sequential edits."""
    F, B, T = synth.make_map_from_config(1)
    rng = np.random.default_rng(71 if case == "scattered" else 72)
    if case == "scattered":
        edits = (synth.crater_list(rng, 256, 256, 200, size=(1, 48), depth=(0, 255)) +
                 synth.random_set_patches(rng, 256, 256, 100, max_size=24))
    else:
        edits = (synth.crater_list(rng, 96, 96, 400, size=(1, 16), depth=(0, 255)) +
                 synth.random_set_patches(rng, 96, 96, 300, max_size=8, allow_outside=False))
    rng.shuffle(edits)
    load(ctx, F, B, T)
    ctx.tc_apply_edit(edits)
    F2, B2, T2 = oracle.apply_edits(F, B, T, edits)
    g = ctx.tc_read_columns(0, 0, 256, 256)
    assert np.array_equal(g[0], F2) and np.array_equal(g[1], B2) and np.array_equal(g[2], T2)
    for L in range(1, ctx.tc_pyramid_info() + 1):
        assert np.array_equal(ctx.tc_read_pyramid(L), oracle.pyramid_level_fast(F2, B2, T2, L)), L
        assert np.array_equal(ctx.tc_read_occupancy(L), oracle.occupancy_level(F2, B2, T2, L)), L
    for L in range(0, ctx.tc_pyramid_info() + 1):
        assert np.array_equal(ctx.tc_read_window(L), oracle.window_level_fast(F2, B2, T2, L)), L


def test_edit_sequences_accumulate(ctx):
    """Several apply calls in a row equal one call with the concatenated
    list, and equal the oracle's sequential application."""
    F, B, T = synth.make_map_from_config(1)
    e1 = synth.crater_list(41, 256, 256, 8)
    e2 = synth.random_set_patches(42, 256, 256, 8)
    e3 = synth.crater_list(43, 256, 256, 8, size=(16, 64))
    load(ctx, F, B, T)
    for e in (e1, e2, e3):
        ctx.tc_apply_edit(e)
    g = ctx.tc_read_columns(0, 0, 256, 256)
    F2, B2, T2 = oracle.apply_edits(F, B, T, e1 + e2 + e3)
    assert np.array_equal(g[0], F2) and np.array_equal(g[1], B2) and np.array_equal(g[2], T2)


def test_c3_edits_then_views_full(ctx):
    """Configuration 3: 64 craters of size 32 on the 2048x16384 map, dirty
    pyramid update, then the grazing and oblique views; every record of
    every render mode against the oracle's render of the edited map."""
    F, B, T = config_map(3)
    H, W = F.shape
    edits = synth.crater_list(synth.SEEDS[3]["edits"], W, H, 64, size=32)
    views = synth.config_views(3, F, B)
    _edited_checks(ctx, F, B, T, edits, views, oracle_result=oracle_render(F, B, T, views, edits))


DEFAULT_KNOBS = ((tc.TC_OPT_RENDER_MODE, 0), (tc.TC_OPT_START_LEVEL, 2), (tc.TC_OPT_TILE_ORDER, 2),
                 (tc.TC_OPT_XCD_REMAP, 64), (tc.TC_OPT_SPLIT_BUDGET, 120),
                 (tc.TC_OPT_PACKET_WIDTH, 8), (tc.TC_OPT_MAX_LEVEL, 15),
                 (tc.TC_OPT_BEAM_PASSES, 6), (tc.TC_OPT_PERSIST_WAVES, 16),
                 (tc.TC_OPT_REFILL_MIN, 16), (tc.TC_OPT_REFILL_ITERS, 16))


@pytest.mark.parametrize("knobs", ["default", "tuned"])
def test_c3_graph_frame_full(ctx, knobs):
    """The configuration-3 frame as the benchmark times it: one captured
    graph of the 64 craters, the dirty update and both views, with the
    default knobs (hierarchical walk, beam start, split pass) and with the
    knobs the autotuner picks for the two views on this machine, replayed
    twice; each replay digs again, and every record of each replay equals
    the oracle's render of the map edited that many times."""
    F, B, T = config_map(3)
    H, W = F.shape
    edits = synth.crater_list(synth.SEEDS[3]["edits"], W, H, 64, size=32)
    views = synth.config_views(3, F, B)
    load(ctx, F, B, T)
    out = torch.empty((synth.view_rays(views), 2), dtype=torch.int32, device="cuda")
    frame = None
    try:
        if knobs == "tuned":
            ctx.tc_autotune(views, out.data_ptr(), reps=2)
        frame = ctx.tc_frame_create(views, edits, out.data_ptr())
        for k in (1, 2):
            frame.launch()
            torch.cuda.synchronize()
            wg, dg = tc.split_hits(out)
            wo, do = oracle_render(F, B, T, views, edits * k)
            assert_parity(wg, dg, wo, do, "c3 graph frame (%s knobs) replay %d" % (knobs, k))
    finally:
        if frame is not None:
            frame.close()
        for opt, v in DEFAULT_KNOBS:
            ctx.tc_set_option(opt, v)


def c4_full_check(wg, dg, wo, do, views, what):
    """Full-buffer parity of a configuration-4 render, reported per view."""
    va = synth.views_array(views)
    base = np.concatenate([[0], np.cumsum(va["width"].astype(np.int64) * va["height"])])
    assert wg.size == base[-1]
    for i in range(len(views)):
        a, b = int(base[i]), int(base[i + 1])
        assert_parity(wg[a:b], dg[a:b], wo[a:b], do[a:b], "%s view %d (%dx%d)" % (
            what, i, int(va["width"][i]), int(va["height"][i])))


@pytest.mark.parametrize("mode", ["hier", "persistent"])
def test_c4_views_full(ctx, mode):
    """Configuration 4's 64 views of uneven sizes plus 8 shadow passes in
    one render call: every record against the oracle."""
    F, B, T = config_map(4)
    load(ctx, F, B, T)
    views = synth.config_views(4, F, B)
    assert len(views) == 72
    wg, dg = gpu_render(ctx, views, mode)
    wo, do = oracle_render(F, B, T, views)
    c4_full_check(wg, dg, wo, do, views, "c4 " + mode)


def test_renders_allocate_nothing(ctx):
    """After tc_create and tc_load_columns, renders (split pass on and off,
    every exact mode), edits and shading make no device or pinned
    allocation: the staging ring and its split queues exist from the start."""
    budget0 = ctx.tc_get_option(tc.TC_OPT_SPLIT_BUDGET)
    F, B, T = synth.make_map_from_config(2)
    load(ctx, F, B, T)
    views = synth.config_views(2, F, B)
    out = torch.empty((synth.view_rays(views), 2), dtype=torch.int32, device="cuda")
    rgba = torch.empty(synth.view_rays(views), dtype=torch.int32, device="cuda")
    pal = synth.default_palette()
    vs = tc.views_struct(views)
    crater = [dict(kind=2, x0=1000, y0=300, w=32, h=32, depth=5)]
    before = ctx.tc_get_option(tc.TC_INFO_ALLOCATIONS)
    for k in range(40):
        ctx.tc_set_option(tc.TC_OPT_RENDER_MODE, (0, 1, 2, 4)[k % 4])
        ctx.tc_set_option(tc.TC_OPT_SPLIT_BUDGET, 128 if k % 3 else 0)
        ctx.tc_render_views(vs, out.data_ptr())
        if k % 10 == 9:
            ctx.tc_apply_edit(crater)
            ctx.tc_shade_views(vs, out.data_ptr(), (1 << 16, 1 << 16, 1 << 16), pal,
                               rgba.data_ptr())
    torch.cuda.synchronize()
    ctx.tc_set_option(tc.TC_OPT_RENDER_MODE, 0)
    ctx.tc_set_option(tc.TC_OPT_SPLIT_BUDGET, budget0)
    assert ctx.tc_get_option(tc.TC_INFO_ALLOCATIONS) == before
    # a split queue longer than the ring's (earlier tests may have grown
    # it) re-sizes the ring's queues in tc_set_option, not in renders
    ctx.tc_set_option(tc.TC_OPT_SPLIT_QUEUE, (1 << 20) + 1)
    grown = ctx.tc_get_option(tc.TC_INFO_ALLOCATIONS)
    assert grown == before + 16
    for _ in range(3):
        ctx.tc_render_views(vs, out.data_ptr())
    torch.cuda.synchronize()
    assert ctx.tc_get_option(tc.TC_INFO_ALLOCATIONS) == grown
    ctx.tc_set_option(tc.TC_OPT_SPLIT_QUEUE, 1 << 17)


def test_error_paths(ctx):
    ctx2 = tc.Context(0)
    F = np.zeros((4, 4), np.uint8)
    v = synth.perspective_view((1.5, 1.5, 5.0), 0, 0, 8, 8)
    out = torch.empty((64, 2), dtype=torch.int32, device="cuda")
    with pytest.raises(tc.TCError) as e:
        ctx2.tc_render_views([v], out.data_ptr())
    assert e.value.status == tc.TC_NO_MAP
    with pytest.raises(tc.TCError) as e:
        ctx2.tc_apply_edit([dict(kind=2, x0=0, y0=0, w=4, h=4, depth=3)])
    assert e.value.status == tc.TC_NO_MAP
    bad = np.zeros((4, 4), np.uint8)
    bad[1, 1] = 3        # B > 0 but T < B and B <= F? F = 0 so B > F ok, T = 0 < B
    with pytest.raises(tc.TCError) as e:
        ctx2.tc_load_columns(F, bad, F)
    assert e.value.status == tc.TC_INVALID_ARG
    ctx2.tc_load_columns(F, F, F)
    big = v.copy()
    big["d0"] = [1 << 23, 0, 0]
    with pytest.raises(tc.TCError) as e:
        ctx2.tc_render_views([big], out.data_ptr())
    assert e.value.status == tc.TC_INVALID_ARG
    for ed in [dict(kind=2, x0=0, y0=0, w=0, h=0, depth=3),
               dict(kind=2, x0=0, y0=0, w=4, h=5, depth=3),
               dict(kind=2, x0=0, y0=0, w=4, h=4, depth=256),
               dict(kind=9, x0=0, y0=0, w=4, h=4, depth=3),
               dict(kind=1, x0=0, y0=0, w=2, h=2, depth=0,
                    F=np.array([[5, 5], [5, 5]], np.uint8),
                    B=np.array([[5, 0], [0, 0]], np.uint8),
                    T=np.array([[6, 0], [0, 0]], np.uint8))]:
        with pytest.raises(tc.TCError) as e:
            ctx2.tc_apply_edit([ed])
        assert e.value.status == tc.TC_INVALID_ARG
    # a failed call leaves the map unchanged
    g = ctx2.tc_read_columns(0, 0, 4, 4)
    assert not g[0].any() and not g[1].any()
    # empty inputs: no views is an error, an empty edit list does nothing
    with pytest.raises(tc.TCError) as e:
        ctx2.tc_render_views([], out.data_ptr())
    assert e.value.status == tc.TC_INVALID_ARG
    ctx2.tc_apply_edit([])
    g = ctx2.tc_read_columns(0, 0, 4, 4)
    assert not g[0].any() and not g[1].any()
    ctx2.tc_render_views([v], out.data_ptr())
    torch.cuda.synchronize()
    with pytest.raises(tc.TCError):
        ctx2.tc_set_option(tc.TC_OPT_RENDER_MODE, 7)
    ctx2.close()
