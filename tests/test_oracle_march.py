"""Pins of the sampled-march oracle (Section 3.1, RAYMARCH in single
precision) to facts that do not come from the oracle itself: hand-worked
straight-down cases whose samples are exact binary fractions, the error
bound of bisection on a single surface, the exact oracle (a different
algorithm) as a lower bound on every hit, and convergence to it as the
sample count grows."""
import math

import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.timeout(300)

S = 65536
MISS = oracle.MISS


def _col(F, B=0, T=0, w=3, h=3):
    """w x h map of one repeated column."""
    return (np.full((h, w), F, np.uint8), np.full((h, w), B, np.uint8),
            np.full((h, w), T, np.uint8))


def _down(F, B, T, steps, far=600.0, bisect=4, z=200):
    """Straight-down ray from (1.5, 1.5, z) with D = (0, 0, -S): every
    sample height z - i * dt * S is an exact binary fraction when z / (steps
    + 1) is one."""
    O = np.array([[3 * S // 2, 3 * S // 2, z * S]], np.int64)
    D = np.array([[0, 0, -S]], np.int64)
    w, d = oracle.march_rays(F, B, T, O, D, far=far, steps=steps, bisect=bisect)
    return int(w[0]), float(d[0])


def test_hand_cases_straight_down():
    """Eye at z = 200, 127 samples: the segment ends at z = 0 and the
    samples sit at z = 200 - 1.5625 i, i = 1..127 (all exact)."""
    # floor at 100: sample 64 is exactly 100 -> solid; bisection keeps it
    w, d = _down(*_col(100), steps=127)
    assert w == 4 and d == 100.0          # cell (1,1) of a 3x3 map, floor
    # a zero-thickness slab exactly on a sample height is found
    w, d = _down(*_col(100, 150, 150), steps=127)
    assert w == (4 | 1 << 30) and d == 50.0
    # one unit higher it falls between samples 31 (151.5625) and 32 (150):
    # stepped over, the march finds the floor (the method's trade-off)
    w, d = _down(*_col(100, 151, 151), steps=127)
    assert w == 4 and d == 100.0
    # a 2-unit slab [150, 152]: sample 31 (151.5625) is inside; bisection
    # against sample 30 (153.125): 152.34375 out, 151.953125 in,
    # 152.1484375 out, 152.05078125 out -> depth 200 - 151.953125
    w, d = _down(*_col(100, 150, 152), steps=127)
    assert w == (4 | 1 << 30) and d == 48.046875
    # floor at 5: sample 125 (4.6875) in; against 6.25: 5.46875 out,
    # 5.078125 out, 4.8828125 in, 4.98046875 in -> depth 195.01953125
    w, d = _down(*_col(5), steps=127)
    assert w == 4 and d == 195.01953125
    # the last sample is at z = 1.5625 and the end point z = 0 is never
    # tested: floors at 0 and 1 are missed, 2 is found (sample 127 in;
    # against 3.125: 2.34375 out, 1.953125 in, 2.1484375 out, 2.05078125
    # out -> depth 200 - 1.953125)
    for F in (0, 1):
        w, d = _down(*_col(F), steps=127)
        assert w == MISS and math.isinf(d)
    w, d = _down(*_col(2), steps=127)
    assert w == 4 and d == 198.046875


def test_hand_cases_far_limit_and_bisection_count():
    # far 100 along the ray, 127 samples: z = 200 - 0.78125 i
    w, d = _down(*_col(150), steps=127, far=100.0)
    assert w == 4 and d == 50.0            # sample 64 at exactly 150
    w, d = _down(*_col(99), steps=127, far=100.0)
    assert w == MISS                        # beyond the far limit
    # no bisection: the first solid sample itself
    w, d = _down(*_col(100, 150, 152), steps=127, bisect=0)
    assert d == 200 - 151.5625
    # one halving: 152.34375 is out -> the bracket keeps 151.5625
    w, d = _down(*_col(100, 150, 152), steps=127, bisect=1)
    assert d == 200 - 151.5625
    # two: then 151.953125 is in
    w, d = _down(*_col(100, 150, 152), steps=127, bisect=2)
    assert d == 200 - 151.953125


def test_hand_case_slab_underside_going_up():
    """A ray going up under a slab finds its underside (SOLID tests the
    slab interval in either vertical direction): eye z = 10, D = (0,0,S),
    far 128 and 127 samples put sample i at z = 10 + i."""
    F, B, T = _col(0, 20, 30)
    O = np.array([[3 * S // 2, 3 * S // 2, 10 * S]], np.int64)
    D = np.array([[0, 0, S]], np.int64)
    w, d = oracle.march_rays(F, B, T, O, D, far=128.0, steps=127)
    assert int(w[0]) == (4 | 1 << 30) and float(d[0]) == 10.0
    # no slab: nothing above, a miss
    F, B, T = _col(0)
    w, d = oracle.march_rays(F, B, T, O, D, far=128.0, steps=127)
    assert int(w[0]) == MISS


def test_degenerate_rays():
    F, B, T = _col(10)
    O = np.array([[S, S, 20 * S], [S, S, -S], [S, S, 20 * S]], np.int64)
    D = np.array([[0, 0, 0], [0, 0, -S], [5, 0, -S]], np.int64)
    w, d = oracle.march_rays(F, B, T, O, D)
    # zero direction; eye below z = 0 descending (empty segment); a normal ray
    assert w[0] == MISS and w[1] == MISS and w[2] != MISS


def _rays_of(views):
    O, D = [], []
    for v in views:
        for py in range(int(v["height"])):
            for px in range(int(v["width"])):
                a, b = 2 * px + 1, 2 * py + 1
                O.append([int(v["o0"][c]) + a * int(v["o_px"][c]) + b * int(v["o_py"][c])
                          for c in range(3)])
                D.append([int(v["d0"][c]) + a * int(v["d_px"][c]) + b * int(v["d_py"][c])
                          for c in range(3)])
    return np.array(O, np.int64), np.array(D, np.int64)


def test_flat_floor_bisection_error_bound():
    """On a flat floor the solid part of every ray is one interval
    [t*, inf): when a sample lands beyond t*, the bracket holds t* and four
    halvings leave the hit at most 1/16 of the sample spacing past it; the
    largest error over many rays comes close to that bound (so the halving
    count is four, not more)."""
    h = 37
    F = np.full((64, 64), h, np.uint8)
    Z = np.zeros_like(F)
    views = [synth.perspective_view((20.3, 3.7, h + 9.0), 12, -25, 48, 36),
             synth.perspective_view((40.5, 50.5, h + 30.0), 225, -60, 33, 29),
             synth.perspective_view((30.0, 30.0, h + 4.0), 90, -8, 40, 30)]
    O, D = _rays_of(views)
    far, steps = 300.0, 128
    w, d = oracle.march_rays(F, Z, Z, O, D, far=far, steps=steps)
    # closed form of the exact hit distance (world units)
    o = O.astype(np.float64) / S
    Dn = D.astype(np.float64)
    L = np.sqrt((Dn ** 2).sum(1))
    desc = Dn[:, 2] < 0
    t_star = np.where(desc, (h - o[:, 2]) / np.where(desc, Dn[:, 2], -1), np.inf)
    hx = o[:, 0] + t_star * Dn[:, 0]
    hy = o[:, 1] + t_star * Dn[:, 1]
    inside = desc & (hx >= 0) & (hx < 64) & (hy >= 0) & (hy < 64)
    d_star = t_star * L
    t_end = np.minimum(far / L, np.where(desc, -o[:, 2] / np.where(desc, Dn[:, 2], -1), np.inf))
    spacing = t_end * L / (steps + 1)
    last = spacing * steps
    # a sample lands within one spacing past t*: it must still be over the map
    t_next = t_star + spacing / L
    nx = o[:, 0] + t_next * Dn[:, 0]
    ny = o[:, 1] + t_next * Dn[:, 1]
    stays = (nx >= 0.01) & (nx < 63.99) & (ny >= 0.01) & (ny < 63.99)
    sure = inside & stays & (d_star < last - spacing * 1e-3)
    assert sure.sum() > 2000
    assert np.all(w[sure] != MISS)
    err = d[sure].astype(np.float64) - d_star[sure]
    tol = 1e-5 * d_star[sure] + 1e-4
    assert np.all(err >= -tol)                                # never before t*
    assert np.all(err <= spacing[sure] / 16 + tol)            # four halvings
    assert np.max(err / (spacing[sure] / 16)) > 0.75          # ... and no more
    # rays whose floor hit lies beyond the last sample miss
    beyond = inside & (d_star > last + spacing * 1e-3)
    assert np.all(w[beyond] == MISS)
    # the hit cell is the column under the returned point, the point at the
    # returned distance along the ray (up to rounding on a cell boundary)
    cell = (w[sure] & 0x07FFFFFF).astype(np.int64)
    tr = d[sure].astype(np.float64) / L[sure]
    rx = np.floor(o[sure, 0] + tr * Dn[sure, 0])
    ry = np.floor(o[sure, 1] + tr * Dn[sure, 1])
    assert np.mean(cell == (ry * 64 + rx).astype(np.int64)) > 0.999


def test_never_hits_before_the_exact_hit():
    """Every solid sample is a solid point of the ray, so a march hit is at
    or after the exact first hit (up to single-precision rounding), and a
    ray the exact cast misses is a march miss too."""
    F, B, T = synth.make_map_from_config(1)
    views = synth.config_views(1, F, B) + [
        synth.perspective_view(synth.eye_above_floor(F, B, 100.5, 30.5, dz=20), 30, -35, 96, 64),
        synth.perspective_view(synth.eye_above_floor(F, B, 200.5, 180.5, dz=3), 250, 5, 96, 64)]
    we, de = oracle.render(F, B, T, views)
    wm, dm = oracle.march(F, B, T, views, far=2000.0, steps=128)
    hit = wm != MISS
    assert hit.sum() > 50000
    assert np.all(we[hit] != MISS)
    dm64 = dm[hit].astype(np.float64)
    assert np.all(dm64 >= de[hit] * (1 - 1e-5) - 2e-3)
    # the march's layer bit names an interval of the hit column: a slab hit
    # only on a two-layer column
    cell = (wm[hit] & 0x07FFFFFF).astype(np.int64)
    slab = (wm[hit] >> 30) & 1
    assert np.all(B.reshape(-1)[cell[slab == 1]] > 0)
    assert np.all(((wm[hit] >> 27) & 7) == 0)


def test_converges_to_exact_cast():
    """As the spacing shrinks the march approaches the exact first hit:
    hit/miss agreement, hit-cell agreement and depth error all improve from
    128 to 1024 to 16384 samples, and at 16384 samples (spacing 0.024
    units) nearly every pixel agrees."""
    F, B, T = synth.make_map_from_config(1)
    v = synth.config_views(1, F, B)
    rows = (0, 240, 3)
    we, de = oracle.render(F, B, T, v, rows=rows)
    stats = []
    for steps, bisect in ((128, 4), (1024, 8), (16384, 16)):
        wm, dm = oracle.march(F, B, T, v, far=400.0, steps=steps, bisect=bisect, rows=rows)
        both = (we != MISS) & (wm != MISS)
        rel = np.abs(dm[both].astype(np.float64) - de[both]) / np.maximum(de[both], 1e-9)
        stats.append((np.mean((we == MISS) == (wm == MISS)),
                      np.mean((we[both] & 0x07FFFFFF) == (wm[both] & 0x07FFFFFF)),
                      np.median(rel)))
    for a, b in zip(stats, stats[1:]):
        assert b[0] > a[0] and b[1] > a[1] and b[2] < a[2], stats
    assert stats[-1][0] > 0.9995 and stats[-1][1] > 0.995 and stats[-1][2] < 1e-6, stats


def test_read_count_and_pixels_agree_with_rows():
    F, B, T = synth.make_map_from_config(1)
    v = synth.config_views(1, F, B)
    w, d, reads = oracle.march(F, B, T, v, with_reads=True)
    assert w.size <= reads <= w.size * (128 + 4)
    rng = np.random.default_rng(3)
    px = rng.integers(0, 320, 500).astype(np.int32)
    py = rng.integers(0, 240, 500).astype(np.int32)
    wp, dp = oracle.march_pixels(F, B, T, v, np.zeros(500, np.int32), px, py)
    idx = py.astype(np.int64) * 320 + px
    assert np.array_equal(wp, w[idx])
    assert np.array_equal(dp.view(np.uint32), d[idx].view(np.uint32))
