"""Pins of the shading oracle (palette, gradient normal, shadow ray, cave
ambient, fog) on hand-worked scenes whose colours follow from the
definition by arithmetic done here by hand: flat floors lit from the zenith
and from below, fog at its two limits, a ramp's gradient normal with the
clamped border, the shadow of a pillar, a lit and an unlit wall, and a
floor under a slab."""
import numpy as np
import pytest

import oracle
import synth

S = 65536
SKY = synth.rgba(1, 2, 3)
FOG = synth.rgba(250, 240, 230)


def _palette():
    """floor at height h: (h, 200, 100); slab top at height h: (255 - h, 50, h)."""
    h = np.arange(256, dtype=np.uint32)
    floor = h | (200 << 8) | (100 << 16) | (0xFF << 24)
    slab = (255 - h) | (50 << 8) | (h << 16) | (0xFF << 24)
    return np.concatenate([floor, slab]).astype(np.uint32)


def _down_view(W, H, z=250.0):
    """one straight-down ray over the centre of every cell"""
    return synth.ortho_view((0, 0, int(z * S)), (S // 2, 0, 0), (0, S // 2, 0),
                            (0, 0, -1), W, H)


def _rgb(v):
    v = int(v)
    return (v & 0xFF, (v >> 8) & 0xFF, (v >> 16) & 0xFF, v >> 24)


def _shade(F, B, T, views, light, **kw):
    args = dict(ambient=0.3, cave_ambient=0.1, fog_far=1e30, sky_rgba=SKY, fog_rgba=FOG)
    args.update(kw)
    return oracle.shade(F, B, T, views, light, _palette(), **args)


def test_flat_floor_zenith_light_is_the_palette():
    """n = l = +z: lambert 1, lit, I = min(0.3 + 1, 1) = 1, no fog: every
    pixel is its palette entry; rays past the map's edge see the sky."""
    F = np.full((4, 5), 37, np.uint8)
    Z = np.zeros_like(F)
    out = _shade(F, Z, Z, [_down_view(5, 4)], (0, 0, S))
    assert all(_rgb(o) == (37, 200, 100, 255) for o in out)
    v = synth.perspective_view((2.5, 2.0, 40.0), 0, 10, 8, 6)   # looking up: all sky
    assert np.all(_shade(F, Z, Z, [v], (0, 0, S)) == SKY)


def test_fog_limits():
    F = np.full((3, 3), 37, np.uint8)
    Z = np.zeros_like(F)
    # fog complete at any distance: the fog colour
    out = _shade(F, Z, Z, [_down_view(3, 3)], (0, 0, S), fog_far=1e-6)
    assert np.all(out == FOG)
    # fog_far = 2 x the distance (250 - 37 = 213): halfway, (37 + 250) / 2
    # = 143.5 -> 144, (200 + 240) / 2 = 220, (100 + 230) / 2 = 165
    out = _shade(F, Z, Z, [_down_view(3, 3)], (0, 0, S), fog_far=426.0)
    assert all(_rgb(o) == (144, 220, 165, 255) for o in out)


def test_light_from_below_leaves_ambient():
    """lambert -1: I = 0.3; 37*0.3 = 11.1 -> 11, 200*0.3 = 60, 100*0.3 = 30"""
    F = np.full((3, 3), 37, np.uint8)
    Z = np.zeros_like(F)
    out = _shade(F, Z, Z, [_down_view(3, 3)], (0, 0, -S))
    assert all(_rgb(o) == (11, 60, 30, 255) for o in out)


def test_ramp_gradient_normal_and_clamped_border():
    """F(x) = 10 + 2x: inside the ramp gx = 2, n = (-2, 0, 1)/sqrt(5); zenith
    light gives lambert = 1/sqrt(5) = 0.4472136, I = 0.7472136:
    red = 10+2x scaled, green 200*I = 149.44 -> 149, blue 74.72 -> 75.  At
    x = 0 the left neighbour clamps to x = 0: gx = 1, n = (-1, 0, 1)/sqrt(2),
    lambert 0.7071068, I = 1.0 (clamped), so the palette colour itself.
    A light along the normal's own direction, (-2, 0, 1), gives lambert 1."""
    F = np.tile((10 + 2 * np.arange(6)).astype(np.uint8), (3, 1))
    Z = np.zeros_like(F)
    out = _shade(F, Z, Z, [_down_view(6, 3)], (0, 0, S)).reshape(3, 6)
    for y in range(3):
        assert _rgb(out[y, 0]) == (10, 200, 100, 255)
        for x in range(1, 5):
            r = int(np.float32(10 + 2 * x) * np.float32(0.7472136) + np.float32(0.5))
            assert _rgb(out[y, x]) == (r, 149, 75, 255), (x, y)
    out = _shade(F, Z, Z, [_down_view(6, 3)], (-2 * S, 0, S)).reshape(3, 6)
    assert _rgb(out[1, 2]) == (14, 200, 100, 255)


def test_pillar_shadow():
    """Light from -x at 45 degrees (L = (-S, 0, S)): lambert on the floor is
    0.7071068; with ambient 0.2, I = 0.9071068.  A pillar of height 100 at
    x = 4 on a floor of 10 shadows the floor cells right of it within 90
    units; the cells left of it are lit.  Shadowed: I = 0.2 (x = 5 also
    faces away: its gradient leans the normal off the light)."""
    F = np.full((1, 12), 10, np.uint8)
    F[0, 4] = 100
    Z = np.zeros_like(F)
    out = _shade(F, Z, Z, [_down_view(12, 1)], (-S, 0, S), ambient=0.2)
    lit = (int(10 * np.float32(0.9071068) + np.float32(0.5)), 181, 91, 255)
    dark = (2, 40, 20, 255)
    for x in (0, 1, 2):              # x = 3 leans on the pillar (gradient)
        assert _rgb(out[x]) == lit, x
    for x in range(5, 12):
        assert _rgb(out[x]) == dark, x
    # the pillar top: lit, palette entry 100 scaled by 0.9071068
    assert _rgb(out[4]) == (91, 181, 91, 255)


def test_walls_face_toward_and_away_from_the_light():
    """A horizontal ray at z = 50 along +x meets the -X wall of a pillar
    (F = 100 at x = 5).  Light from -x (L = (-S, 0, 0)): n = (-1, 0, 0),
    lambert 1, the shadow ray leaves through empty cells: I = 1, the floor
    entry of height 100.  Light from +x: lambert -1, I = 0.3."""
    F = np.full((1, 10), 10, np.uint8)
    F[0, 5] = 100
    Z = np.zeros_like(F)
    v = synth.ortho_view((S // 2, S // 2, 50 * S), (0, 0, 0), (0, 0, 0), (1, 0, 0), 1, 1)
    assert _rgb(_shade(F, Z, Z, [v], (-S, 0, 0))[0]) == (100, 200, 100, 255)
    assert _rgb(_shade(F, Z, Z, [v], (S, 0, 0))[0]) == (30, 60, 30, 255)


def test_floor_under_a_slab_gets_cave_ambient():
    """Column x = 3 with floor 10 and slab [40, 60], floors of 5 around it.
    An eye inside the cave (z = 30) looking straight down meets the floor
    (top face, floor layer, flat neighbours): the zenith light's shadow ray
    meets the slab's underside, so the pixel is unlit with cave ambient:
    (10, 200, 100) * 0.1 -> (1, 20, 10).  From above, the slab top (slab
    entry 60 = (195, 50, 60)) is fully lit."""
    F = np.full((1, 6), 5, np.uint8)
    B = np.zeros_like(F)
    T = np.zeros_like(F)
    F[0, 3], B[0, 3], T[0, 3] = 10, 40, 60
    cave = synth.ortho_view((3 * S + S // 2, S // 2, 30 * S), (0, 0, 0), (0, 0, 0),
                            (0, 0, -1), 1, 1)
    assert _rgb(_shade(F, B, T, [cave], (0, 0, S))[0]) == (1, 20, 10, 255)
    down = synth.ortho_view((3 * S + S // 2, S // 2, 250 * S), (0, 0, 0), (0, 0, 0),
                            (0, 0, -1), 1, 1)
    assert _rgb(_shade(F, B, T, [down], (0, 0, S))[0]) == (195, 50, 60, 255)


def test_random_scene_consistency():
    """On the 256x256 map the face formula of every hit reproduces the exact
    caster's time (the oracle raises otherwise); lit pixels are never darker
    than the same pixel with the light blocked everywhere."""
    F, B, T = synth.make_map_from_config(1)
    views = synth.config_views(1, F, B)
    rows = [0, 240, 4]
    pal = synth.default_palette()
    a = oracle.shade(F, B, T, views, (S, 2 * S, 3 * S), pal, fog_far=1e30)
    b = oracle.shade(F, B, T, views, (S, 2 * S, 3 * S), pal, ambient=0.0, cave_ambient=0.0,
                     fog_far=1e30)
    ch = lambda x, c: (x >> (8 * c)) & 0xFF
    for c in range(3):
        assert np.all(ch(a, c) >= ch(b, c))
    assert len(set(a.tolist())) > 100
