"""Definition of the per-layer min/max pyramid (test infrastructure).

The acceleration structure is the maximum-mipmap idea that Section 1.1
cites, extended to the two intervals of a column.  Level L >= 1 has one node
per 2^L x 2^L block of cells (blocks clipped to the map).  A node stores
  fmax = max F over the block,
  smin = min B over the block's two-layer cells (255 when there are none),
  smax = max T over the block's two-layer cells (0 when there are none),
packed as fmax | smin << 8 | smax << 16 (uint32), row-major [y][x].

A window level L >= 0 has one entry per level-L node (i, j) holding the
same three quantities over the 2^(L+1) x 2^(L+1) block of cells whose
corner is the node's, [i 2^L, (i + 2) 2^L) x [j 2^L, (j + 2) 2^L), clipped
to the map: a box narrower than a level-L node overlaps at most two nodes
per axis, all inside the window of the first, so one entry bounds the
solid of the whole box (Section 3.2's conservative test of a region against
the hierarchy, here for the boxes that bound a bundle of rays).
"""
import numpy as np


def pyramid_level(F, B, T, L):
    H, W = F.shape
    n = 1 << L
    HL = (H + n - 1) // n
    WL = (W + n - 1) // n
    out = np.zeros((HL, WL), np.uint32)
    for j in range(HL):
        for i in range(WL):
            f = F[j * n:(j + 1) * n, i * n:(i + 1) * n]
            b = B[j * n:(j + 1) * n, i * n:(i + 1) * n]
            t = T[j * n:(j + 1) * n, i * n:(i + 1) * n]
            two = b > 0
            fmax = int(f.max())
            smin = int(b[two].min()) if two.any() else 255
            smax = int(t[two].max()) if two.any() else 0
            out[j, i] = fmax | (smin << 8) | (smax << 16)
    return out


def pyramid_level_fast(F, B, T, L):
    """Same result as pyramid_level via padded reshapes (for large maps)."""
    H, W = F.shape
    n = 1 << L
    HL = (H + n - 1) // n
    WL = (W + n - 1) // n
    pad = ((0, HL * n - H), (0, WL * n - W))
    f = np.pad(F, pad, constant_values=0).reshape(HL, n, WL, n)
    two = B > 0
    b = np.pad(np.where(two, B, 255).astype(np.uint8), pad,
               constant_values=255).reshape(HL, n, WL, n)
    t = np.pad(np.where(two, T, 0).astype(np.uint8), pad,
               constant_values=0).reshape(HL, n, WL, n)
    fmax = f.max(axis=(1, 3)).astype(np.uint32)
    smin = b.min(axis=(1, 3)).astype(np.uint32)
    smax = t.max(axis=(1, 3)).astype(np.uint32)
    return fmax | (smin << 8) | (smax << 16)


def occupancy_level(F, B, T, L):
    """Occupancy masks of level L >= 1 (uint64, row-major [y][x]): bit k of a
    node is set iff some two-layer column of its 2^L x 2^L block has a slab
    [B, T] meeting the closed height band [4k, 4k + 4], i.e. B <= 4k + 4 and
    T >= 4k.  The union over the block follows the occupancy hierarchy of
    Section 3.2 (each level the union of its children)."""
    H, W = F.shape
    n = 1 << L
    HL = (H + n - 1) // n
    WL = (W + n - 1) // n
    b = B.astype(np.int64)
    t = T.astype(np.int64)
    cell = np.zeros((H, W), np.uint64)
    for k in range(64):
        meets = (b > 0) & (b <= 4 * k + 4) & (t >= 4 * k)
        cell |= meets.astype(np.uint64) << np.uint64(k)
    pad = ((0, HL * n - H), (0, WL * n - W))
    c = np.pad(cell, pad, constant_values=0).reshape(HL, n, WL, n)
    return np.bitwise_or.reduce(np.bitwise_or.reduce(c, axis=3), axis=1)


def window_level(F, B, T, L):
    """Window level L >= 0 (uint32, row-major [y][x], the shape of level L),
    written as its definition: per entry, the block of cells it covers."""
    H, W = F.shape
    n = 1 << L
    HL = (H + n - 1) // n
    WL = (W + n - 1) // n
    out = np.zeros((HL, WL), np.uint32)
    for j in range(HL):
        for i in range(WL):
            f = F[j * n:(j + 2) * n, i * n:(i + 2) * n]
            b = B[j * n:(j + 2) * n, i * n:(i + 2) * n]
            t = T[j * n:(j + 2) * n, i * n:(i + 2) * n]
            two = b > 0
            fmax = int(f.max())
            smin = int(b[two].min()) if two.any() else 255
            smax = int(t[two].max()) if two.any() else 0
            out[j, i] = fmax | (smin << 8) | (smax << 16)
    return out


def window_level_fast(F, B, T, L):
    """Same result as window_level, derived the other way round: the 2 x 2
    neighbourhood combine (max, min, max) of level-L nodes (i..i+1, j..j+1)
    that exist, level 0 being the cells themselves (for large maps)."""
    if L == 0:
        two = B > 0
        P = (F.astype(np.uint32) | (np.where(two, B, 255).astype(np.uint32) << 8) |
             (np.where(two, T, 0).astype(np.uint32) << 16))
    else:
        P = pyramid_level_fast(F, B, T, L)
    f = (P & 0xFF).astype(np.int64)
    lo = ((P >> 8) & 0xFF).astype(np.int64)
    hi = ((P >> 16) & 0xFF).astype(np.int64)
    fp = np.pad(f, ((0, 1), (0, 1)), constant_values=0)
    lp = np.pad(lo, ((0, 1), (0, 1)), constant_values=255)
    hp = np.pad(hi, ((0, 1), (0, 1)), constant_values=0)
    h, w = P.shape
    fm = np.maximum(np.maximum(fp[:h, :w], fp[1:, :w]), np.maximum(fp[:h, 1:], fp[1:, 1:]))
    lm = np.minimum(np.minimum(lp[:h, :w], lp[1:, :w]), np.minimum(lp[:h, 1:], lp[1:, 1:]))
    hm = np.maximum(np.maximum(hp[:h, :w], hp[1:, :w]), np.maximum(hp[:h, 1:], hp[1:, 1:]))
    return (fm | (lm << 8) | (hm << 16)).astype(np.uint32)


# ---- the occupancy pyramid of the voxel-accelerated march (Section 3.2) ----
#
# Voxels of v x v cells by vz height units.  The finest level holds one bit
# per voxel: set iff the solid set of some column of its footprint meets the
# voxel's closed height range [Z vz, (Z + 1) vz] (a floor (-inf, F] meets it
# iff Z vz <= F; a slab [B, T] iff B <= (Z + 1) vz and T >= Z vz).  Each
# higher level is the union of its eight children (2 x 2 x 2).  Heights run
# 0..256, so the finest level has 256 / vz voxels per column.  Arrays are
# indexed [Z][Y][X].


def voxel_dims(W, H, v, vz, k):
    """Voxel counts (nx, ny, nz) of level k."""
    nx, ny, nz = -(-W // v), -(-H // v), 256 // vz
    for _ in range(k):
        nx, ny, nz = -(-nx // 2), -(-ny // 2), -(-nz // 2)
    return nx, ny, nz


def voxel_levels(F, B, T, v, vz):
    """Every level, finest first, built the way the structure is defined:
    the finest from the columns, each next one as the union of eight
    children, until a single voxel remains."""
    H, W = F.shape
    nx, ny, nz = voxel_dims(W, H, v, vz, 0)
    leaf = np.zeros((nz, ny, nx), bool)
    for y in range(H):
        for x in range(W):
            f, b, t = int(F[y, x]), int(B[y, x]), int(T[y, x])
            for Z in range(nz):
                z0, z1 = Z * vz, (Z + 1) * vz
                if z0 <= f or (b > 0 and b <= z1 and t >= z0):
                    leaf[Z, y // v, x // v] = True
    levels = [leaf]
    while levels[-1].shape != (1, 1, 1):
        c = levels[-1]
        z, y, x = c.shape
        p = np.zeros((-(-z // 2), -(-y // 2), -(-x // 2)), bool)
        for Z in range(z):
            for Y in range(y):
                for X in range(x):
                    if c[Z, Y, X]:
                        p[Z // 2, Y // 2, X // 2] = True
        levels.append(p)
    return levels


def voxel_level_direct(F, B, T, v, vz, k):
    """Level k written directly: a voxel of level k covers the cells
    [X v 2^k, (X + 1) v 2^k) x [Y v 2^k, (Y + 1) v 2^k) and the closed
    heights [Z vz 2^k, (Z + 1) vz 2^k]; its bit is set iff a column of its
    footprint has solid in that range (vectorised, for large maps)."""
    H, W = F.shape
    nx, ny, nz = voxel_dims(W, H, v, vz, k)
    n, s = v << k, vz << k
    f = F.astype(np.int64)
    b = B.astype(np.int64)
    t = T.astype(np.int64)
    out = np.zeros((nz, ny, nx), bool)
    pad = ((0, ny * n - H), (0, nx * n - W))
    for Z in range(nz):
        z0, z1 = Z * s, (Z + 1) * s
        col = (z0 <= f) | ((b > 0) & (b <= z1) & (t >= z0))
        col = np.pad(col, pad, constant_values=False).reshape(ny, n, nx, n)
        out[Z] = col.any(axis=(1, 3))
    return out
