"""Pins of the oracle's voxel occupancy pyramid (the structure of the
voxel-accelerated march, Section 3.2): a hand-worked map, the union-of-eight
construction against the direct per-level definition, and the exact
caster's hits lying in occupied voxels at every level."""
import numpy as np
import pytest

import oracle
import synth


def test_voxel_hand_case():
    """3 x 2 map, voxels of 2 x 2 cells by 4 units.  Footprint X = 0 holds
    floors 3, 9, 1, 0: bits Z = 0, 1, 2 (4 Z <= 9).  Footprint X = 1 holds
    floors 0, 0 and the slab [5, 12] at (2, 1): Z = 0 from the floor, and
    Z = 1..3 from the slab (5 <= 4 Z + 4 and 12 >= 4 Z; Z = 3 touches it at
    12).  Level 1 is the union of pairs in X and Z."""
    F = np.array([[3, 9, 0], [1, 0, 0]], np.uint8)
    B = np.zeros_like(F)
    T = np.zeros_like(F)
    B[1, 2], T[1, 2] = 5, 12
    lv = oracle.voxel_levels(F, B, T, 2, 4)
    assert lv[0].shape == (64, 1, 2)
    assert list(np.nonzero(lv[0][:, 0, 0])[0]) == [0, 1, 2]
    assert list(np.nonzero(lv[0][:, 0, 1])[0]) == [0, 1, 2, 3]
    assert lv[1].shape == (32, 1, 1)
    assert list(np.nonzero(lv[1][:, 0, 0])[0]) == [0, 1]
    assert lv[-1].shape == (1, 1, 1) and lv[-1][0, 0, 0]
    assert len(lv) == 7     # nz 64 -> 1 in six halvings
    # a slab whose bottom sits on a voxel boundary touches the voxel below
    B[1, 2], T[1, 2] = 8, 8
    lv = oracle.voxel_levels(F, B, T, 2, 4)
    assert list(np.nonzero(lv[0][:, 0, 1])[0]) == [0, 1, 2]


@pytest.mark.parametrize("shape,v,vz", [((1, 1), 1, 1), ((5, 3), 2, 4), ((17, 9), 4, 2),
                                        ((40, 33), 2, 8), ((33, 40), 8, 1), ((24, 24), 1, 2)])
def test_union_of_children_equals_direct_definition(shape, v, vz):
    H, W = shape
    F, B, T = synth.make_map(W, H, 900 + W + v * 7 + vz, dual=0.5, period=4)
    lv = oracle.voxel_levels(F, B, T, v, vz)
    for k, a in enumerate(lv):
        assert a.shape[::-1] == oracle.voxel_dims(W, H, v, vz, k)
        assert np.array_equal(a, oracle.voxel_level_direct(F, B, T, v, vz, k)), k


@pytest.mark.parametrize("v,vz", [(1, 1), (2, 4), (4, 2)])
def test_exact_hits_lie_in_occupied_voxels(v, vz):
    """Every hit point of the exact caster is solid, so its voxel is set at
    every level (the structure only skips space known to be empty); points
    on a voxel boundary are checked in every voxel that holds them."""
    rng = np.random.default_rng(50 + v + vz)
    F, B, T = synth.make_map(23, 19, 60 + v, dual=0.45, period=4)
    H, W = F.shape
    n = 3000
    O = np.stack([rng.integers(0, W * 65536, n), rng.integers(0, H * 65536, n),
                  rng.integers(0, 300 * 65536, n)], 1)
    D = rng.integers(-(1 << 16), 1 << 16, (n, 3))
    D[:, 2] -= 1 << 15
    w, d, tn, td = oracle.cast_rays_exact(F, B, T, O, D)
    lv = oracle.voxel_levels(F, B, T, v, vz)
    hits = np.nonzero(w != oracle.MISS)[0]
    assert hits.size > 1000
    from fractions import Fraction
    for i in hits[:400]:
        t = Fraction(int(tn[i]), int(td[i]))
        p = [Fraction(int(O[i, c])) / 65536 + t * int(D[i, c]) / 65536 for c in range(3)]
        for k, a in enumerate(lv):
            nz, ny, nx = a.shape
            sx, sz = v << k, vz << k
            # every voxel whose closed box holds the point
            xs = {min(int(p[0] // sx), nx - 1)} | ({int(p[0] // sx) - 1} if p[0] % sx == 0 else set())
            ys = {min(int(p[1] // sx), ny - 1)} | ({int(p[1] // sx) - 1} if p[1] % sx == 0 else set())
            zq = max(p[2], 0)
            zs = {min(int(zq // sz), nz - 1)} | ({int(zq // sz) - 1} if zq % sz == 0 else set())
            cells = [(X, Y, Z) for X in xs for Y in ys for Z in zs
                     if 0 <= X < nx and 0 <= Y < ny and 0 <= Z < nz]
            assert any(a[Z, Y, X] for X, Y, Z in cells), (i, k, p)
