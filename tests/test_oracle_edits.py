"""Pins of the oracle's edit semantics and pyramid definition."""
import json
import os

import numpy as np
import pytest

import oracle
import synth


def test_crater_hand_case(golden_dir):
    g = json.load(open(os.path.join(golden_dir, "crater_s4_d40.json")))
    W, H = g["W"], g["H"]
    F = np.full((H, W), g["F0"], np.uint8)
    B = np.full((H, W), g["B0"], np.uint8)
    T = np.full((H, W), g["T0"], np.uint8)
    F2, B2, T2 = oracle.apply_edits(F, B, T, [g["edit"]])
    assert np.array_equal(F2, np.array(g["F"], np.uint8))
    assert np.array_equal(B2, np.array(g["B"], np.uint8))
    assert np.array_equal(T2, np.where(B2 > 0, g["T0"], 0).astype(np.uint8))
    assert oracle.valid_columns(F2, B2, T2)


def test_crater_saturates_at_zero_and_clips():
    F = np.full((10, 10), 5, np.uint8)
    Z = np.zeros_like(F)
    F2, B2, T2 = oracle.apply_edits(F, Z, Z, [dict(kind=2, x0=-3, y0=7, w=8, h=8, depth=255)])
    assert F2.min() == 0
    # nothing outside the clipped patch changes
    assert np.all(F2[:7, :] == 5) and np.all(F2[:, 5:] == 5)


def test_set_patch_clipped_and_ordered():
    F = np.full((8, 8), 10, np.uint8)
    Z = np.zeros_like(F)
    p = dict(kind=1, x0=6, y0=-1, w=4, h=3, depth=0,
             F=np.full((3, 4), 50, np.uint8), B=np.full((3, 4), 60, np.uint8),
             T=np.full((3, 4), 70, np.uint8))
    c = dict(kind=2, x0=5, y0=0, w=4, h=4, depth=100)
    Fa, Ba, Ta = oracle.apply_edits(F, Z, Z, [p, c])
    Fb, Bb, Tb = oracle.apply_edits(F, Z, Z, [c, p])
    # the SET rectangle covers x 6..7, y 0..1 only
    assert np.all(Fb[0:2, 6:8] == 50) and np.all(Bb[0:2, 6:8] == 60)
    assert Fb[2, 6] != 50
    # order matters where they overlap
    assert not np.array_equal(Fa, Fb) or not np.array_equal(Ba, Bb)
    assert oracle.valid_columns(Fa, Ba, Ta) and oracle.valid_columns(Fb, Bb, Tb)


def test_pyramid_hand_case():
    F = np.array([[1, 2, 3, 4, 5],
                  [6, 7, 8, 9, 10],
                  [0, 0, 0, 0, 0]], np.uint8)
    B = np.zeros_like(F)
    T = np.zeros_like(F)
    B[0, 1], T[0, 1] = 20, 25
    B[1, 4], T[1, 4] = 30, 31
    B[2, 2], T[2, 2] = 9, 40
    p1 = oracle.pyramid_level(F, B, T, 1)
    assert p1.shape == (2, 3)
    node = lambda f, lo, hi: f | (lo << 8) | (hi << 16)
    assert p1[0, 0] == node(7, 20, 25)
    assert p1[0, 1] == node(9, 255, 0)
    assert p1[0, 2] == node(10, 30, 31)
    assert p1[1, 1] == node(0, 9, 40)
    assert p1[1, 2] == node(0, 255, 0)
    p2 = oracle.pyramid_level(F, B, T, 2)
    assert p2.shape == (1, 2)
    assert p2[0, 0] == node(9, 9, 40)
    assert p2[0, 1] == node(10, 30, 31)
    p3 = oracle.pyramid_level(F, B, T, 3)
    assert p3[0, 0] == node(10, 9, 40)


def test_window_hand_case():
    """The map of the pyramid hand case.  Window level 0 entry (i, j) covers
    cells (i..i+1, j..j+1); window level 1 entry (i, j) covers cells
    (2i..2i+3, 2j..2j+3), clipped to the 5 x 3 map."""
    F = np.array([[1, 2, 3, 4, 5],
                  [6, 7, 8, 9, 10],
                  [0, 0, 0, 0, 0]], np.uint8)
    B = np.zeros_like(F)
    T = np.zeros_like(F)
    B[0, 1], T[0, 1] = 20, 25
    B[1, 4], T[1, 4] = 30, 31
    B[2, 2], T[2, 2] = 9, 40
    node = lambda f, lo, hi: f | (lo << 8) | (hi << 16)
    w0 = oracle.window_level(F, B, T, 0)
    assert w0.shape == (3, 5)
    assert w0[0, 0] == node(7, 20, 25)     # cells (0..1, 0..1)
    assert w0[0, 1] == node(8, 20, 25)     # cells (1..2, 0..1)
    assert w0[0, 3] == node(10, 30, 31)    # cells (3..4, 0..1)
    assert w0[0, 4] == node(10, 30, 31)    # cells (4, 0..1): clipped
    assert w0[1, 1] == node(8, 9, 40)      # cells (1..2, 1..2)
    assert w0[1, 3] == node(10, 30, 31)
    assert w0[2, 0] == node(0, 255, 0)     # cells (0..1, 2)
    assert w0[2, 2] == node(0, 9, 40)      # cells (2..3, 2)
    assert w0[2, 4] == node(0, 255, 0)     # cell (4, 2)
    w1 = oracle.window_level(F, B, T, 1)
    assert w1.shape == (2, 3)
    assert w1[0, 0] == node(9, 9, 40)      # cells (0..3, 0..2)
    assert w1[0, 1] == node(10, 9, 40)     # cells (2..4, 0..2)
    assert w1[0, 2] == node(10, 30, 31)    # cells (4, 0..2)
    assert w1[1, 1] == node(0, 9, 40)      # cells (2..4, 2)
    # the top window covers everything
    w3 = oracle.window_level(F, B, T, 3)
    assert w3.shape == (1, 1) and w3[0, 0] == node(10, 9, 40)


@pytest.mark.parametrize("shape,L", [((1, 1), 0), ((3, 5), 1), ((17, 9), 0), ((17, 9), 2),
                                     ((40, 33), 1), ((40, 33), 3), ((40, 33), 6)])
def test_window_definitions_agree(shape, L):
    """Per-entry blocks of cells against the 2 x 2 combine of level-L
    nodes, on random two-layer maps of odd shapes."""
    import synth
    H, W = shape
    F, B, T = synth.make_map(W, H, 70 + W * 3 + L, dual=0.4, period=4)
    a = oracle.window_level(F, B, T, L)
    b = oracle.window_level_fast(F, B, T, L)
    assert a.dtype == b.dtype == np.uint32 and a.shape == b.shape
    assert np.array_equal(a, b)
    # every window bounds each of its cells: fmax >= F, and a two-layer
    # cell's slab lies inside [smin, smax]
    n = 1 << L
    for y in range(H):
        for x in range(W):
            e = int(a[y // n, x // n])
            assert (e & 0xFF) >= F[y, x]
            if B[y, x]:
                assert ((e >> 8) & 0xFF) <= B[y, x] and ((e >> 16) & 0xFF) >= T[y, x]


def test_occupancy_hand_case():
    """Slabs [20, 25], [30, 31], [9, 40] as in the pyramid hand case: the
    bands [4k, 4k+4] they meet are k = 4..6 ([20,25]: 16-20 touches 20,
    20-24, 24-28), k = 7 ([30,31]: 28-32), k = 2..10 ([9,40]: 8-12 .. 40-44
    touches 40).  A slab whose bottom sits on a band edge meets both
    neighbours: [8, 8] sets k = 1 and 2."""
    F = np.array([[1, 2, 3, 4, 5],
                  [6, 7, 8, 9, 10],
                  [0, 0, 0, 0, 0]], np.uint8)
    B = np.zeros_like(F)
    T = np.zeros_like(F)
    B[0, 1], T[0, 1] = 20, 25
    B[1, 4], T[1, 4] = 30, 31
    B[2, 2], T[2, 2] = 9, 40
    bits = lambda ks: sum(1 << k for k in ks)
    m1 = oracle.occupancy_level(F, B, T, 1)
    assert m1.shape == (2, 3) and m1.dtype == np.uint64
    assert int(m1[0, 0]) == bits(range(4, 7))
    assert int(m1[0, 1]) == 0
    assert int(m1[0, 2]) == bits([7])
    assert int(m1[1, 1]) == bits(range(2, 11))
    assert int(m1[1, 0]) == 0 and int(m1[1, 2]) == 0
    m2 = oracle.occupancy_level(F, B, T, 2)
    assert int(m2[0, 0]) == bits(range(2, 11))
    assert int(m2[0, 1]) == bits([7])
    m3 = oracle.occupancy_level(F, B, T, 3)
    assert int(m3[0, 0]) == bits(range(2, 11))
    one = np.zeros((1, 1), np.uint8)
    assert int(oracle.occupancy_level(one, one + 8, one + 8, 1)[0, 0]) == bits([1, 2])
    assert int(oracle.occupancy_level(one, one + 1, one + 255, 1)[0, 0]) == (1 << 64) - 1


def test_pyramid_two_definitions_agree():
    for seed, (W, H) in enumerate([(37, 23), (64, 64), (5, 130), (1, 1)]):
        F, B, T = synth.make_map(W, H, 500 + seed, dual=0.3, period=8)
        L = 0
        while (1 << L) < max(W, H):
            L += 1
            assert np.array_equal(oracle.pyramid_level(F, B, T, L),
                                  oracle.pyramid_level_fast(F, B, T, L))


def test_synthetic_edits_keep_invariants():
    F, B, T = synth.make_map_from_config(1)
    eds = synth.crater_list(1, 256, 256, 10) + synth.random_set_patches(2, 256, 256, 10)
    F2, B2, T2 = oracle.apply_edits(F, B, T, eds)
    assert oracle.valid_columns(F2, B2, T2)
