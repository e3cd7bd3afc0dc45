"""Seeded two-layer height-column maps.

A map is three uint8 planes of shape (H, W), indexed [y, x]:
  floor  F  -- top of the floor interval (the paper's `low`)
  sbot   B  -- bottom of the upper slab (`mid`), 0 when the cell has one layer
  stop   T  -- top of the upper slab (`high`), 0 when the cell has one layer
with the encoding invariants  B == 0 => T == 0  and  B > 0 => B > F, T >= B
(Section 2 describes the low/mid/high triple; a single-level texel carries no
upper interval).

Recipe (the stand-in for the paper's level, which is not available):
  * floor: fBm value noise, 6 octaves, gain 0.5, bilinear lattice
    interpolation, base period 64 cells (256 for the large maps), normalised
    to 0..215, plus sharp cliff features (half-discs and discs that raise or
    lower the floor by a constant step), clamped to 0..255;
  * slabs: connected blobs grown by randomised breadth-first (Eden) growth
    from uniform seed cells until the requested share of two-layer cells is
    reached; per blob B = min(254, max F in blob + U{4..48}),
    T = min(255, B + U{0..40}); per-cell jitter of +-2 on both (T >= B);
    cells whose floor reaches the slab bottom keep one layer.
"""
import numpy as np

from .configs import config as _config


def _value_noise(rng, H, W, period):
    gh = int(H // period) + 2
    gw = int(W // period) + 2
    lat = rng.random((gh, gw), dtype=np.float32)
    xs = (np.arange(W, dtype=np.float32) + 0.5) / period
    ys = (np.arange(H, dtype=np.float32) + 0.5) / period
    x0 = np.floor(xs).astype(np.int64)
    y0 = np.floor(ys).astype(np.int64)
    fx = (xs - x0).astype(np.float32)
    fy = (ys - y0).astype(np.float32)
    lx = lat[:, x0] * (1 - fx) + lat[:, x0 + 1] * fx          # (gh, W)
    out = lx[y0] * (1 - fy)[:, None] + lx[y0 + 1] * fy[:, None]
    return out


def _fbm(rng, H, W, period, octaves=6, gain=0.5):
    acc = np.zeros((H, W), np.float32)
    amp = 1.0
    p = float(period)
    for _ in range(octaves):
        acc += np.float32(amp) * _value_noise(rng, H, W, max(p, 1.0))
        amp *= gain
        p /= 2.0
    lo, hi = float(acc.min()), float(acc.max())
    return (acc - lo) / max(hi - lo, 1e-6)


def _cliffs(rng, H, W, kind, n):
    add = np.zeros((H, W), np.float32)
    ys = np.arange(H, dtype=np.float32)[:, None]
    xs = np.arange(W, dtype=np.float32)[None, :]
    scale = max(H, W)
    for _ in range(n):
        cx = rng.uniform(0, W)
        cy = rng.uniform(0, H)
        r = rng.uniform(0.05, 0.25) * min(scale, 2048)
        # only touch the bounding box of the feature
        x0, x1 = int(max(0, cx - r)), int(min(W, cx + r + 1))
        y0, y1 = int(max(0, cy - r)), int(min(H, cy + r + 1))
        if x0 >= x1 or y0 >= y1:
            continue
        dx = xs[:, x0:x1] - cx
        dy = ys[y0:y1, :] - cy
        inside = dx * dx + dy * dy <= r * r
        if kind == "terraces":
            delta = 40.0
            th = rng.uniform(0, 2 * np.pi)
            inside &= (dx * np.cos(th) + dy * np.sin(th)) > 0
        else:
            delta = float(rng.integers(8, 41)) * (1 if rng.random() < 0.5 else -1)
            if rng.random() < 0.5:
                th = rng.uniform(0, 2 * np.pi)
                inside &= (dx * np.cos(th) + dy * np.sin(th)) > 0
        add[y0:y1, x0:x1] += np.where(inside, np.float32(delta), np.float32(0))
    return add


def _grow_blobs(rng, sizes, R):
    """Eden growth of len(sizes) blobs, each inside its own RxR window."""
    nb = len(sizes)
    c = R // 2
    win = np.zeros((nb, R, R), bool)
    win[:, c, c] = True
    cnt = np.ones(nb, np.int64)
    sizes = np.asarray(sizes, np.int64)
    for _ in range(4 * R):
        act = np.nonzero(cnt < sizes)[0]
        if act.size == 0:
            break
        w = win[act]
        nbr = np.zeros_like(w)
        nbr[:, 1:, :] |= w[:, :-1, :]
        nbr[:, :-1, :] |= w[:, 1:, :]
        nbr[:, :, 1:] |= w[:, :, :-1]
        nbr[:, :, :-1] |= w[:, :, 1:]
        front = nbr & ~w
        fc = front.sum(axis=(1, 2))
        need = sizes[act] - cnt[act]
        p = np.where(fc > 0, np.minimum(0.5, need / np.maximum(fc, 1)), 0.0)
        acc = front & (rng.random(w.shape, dtype=np.float32) < p[:, None, None])
        w |= acc
        win[act] = w
        cnt[act] = w.sum(axis=(1, 2))
    return win


def _slabs(rng, F, dual, blob):
    H, W = F.shape
    target = int(round(dual * H * W))
    label = np.zeros((H, W), np.int32)
    lo, hi = blob
    R = 2 * int(np.ceil(np.sqrt(hi))) + 13
    c = R // 2
    nlab = 0
    for _ in range(8):
        have = int((label > 0).sum())
        if have >= 0.985 * target or target == 0:
            break
        mean = 0.5 * (lo + hi)
        nb = max(1, int(np.ceil((target - have) / mean * 1.05)))
        for s in range(0, nb, 4096):
            k = min(4096, nb - s)
            sizes = rng.integers(lo, hi + 1, size=k)
            sx = rng.integers(0, W, size=k)
            sy = rng.integers(0, H, size=k)
            win = _grow_blobs(rng, sizes, R)
            bi, v, u = np.nonzero(win)
            x = sx[bi] - c + u
            y = sy[bi] - c + v
            ok = (x >= 0) & (x < W) & (y >= 0) & (y < H)
            label[y[ok], x[ok]] = (nlab + 1 + bi[ok]).astype(np.int32)
            nlab += k
            if int((label > 0).sum()) >= target:
                break
    B = np.zeros((H, W), np.uint8)
    T = np.zeros((H, W), np.uint8)
    m = label > 0
    if not m.any():
        return B, T
    lab = label[m]
    maxf = np.zeros(nlab + 1, np.int32)
    np.maximum.at(maxf, lab, F[m].astype(np.int32))
    bb = np.minimum(254, maxf + rng.integers(4, 49, size=nlab + 1))
    tt = np.minimum(255, bb + rng.integers(0, 41, size=nlab + 1))
    jb = rng.integers(-2, 3, size=lab.size)
    jt = rng.integers(-2, 3, size=lab.size)
    bc = np.clip(bb[lab] + jb, 1, 254)
    tc = np.clip(tt[lab] + jt, bc, 255)
    f = F[m].astype(np.int32)
    keep = bc > f
    bc = np.where(keep, bc, 0)
    tc = np.where(keep, tc, 0)
    B[m] = bc.astype(np.uint8)
    T[m] = tc.astype(np.uint8)
    return B, T


def make_map(W, H, seed, dual=0.2, period=64, cliffs="steps", n_cliffs=6,
             blob=(8, 200)):
    """Return (F, B, T) uint8 planes of shape (H, W) for the given seed."""
    rng = np.random.default_rng(seed)
    base = _fbm(rng, H, W, period) * np.float32(215.0)
    base += _cliffs(rng, H, W, cliffs, n_cliffs)
    F = np.clip(np.rint(base), 0, 255).astype(np.uint8)
    B, T = _slabs(rng, F, dual, blob)
    return F, B, T


def cave_map(seed, W, H, dual=0.5):
    """A cave-heavy map: half the cells two-layer, in blobs whose slabs sit
    at heights set by their own surroundings, so one pyramid node often
    holds slabs at several heights with air between them."""
    return make_map(W, H, seed, dual=dual, period=64, cliffs="steps", n_cliffs=8)


_MAP_CACHE = {}


def make_map_from_config(k):
    """Map of workload configuration k (cached in-process)."""
    if k in _MAP_CACHE:
        return _MAP_CACHE[k]
    c = _config(k)
    F, B, T = make_map(c["W"], c["H"], c["seeds"]["map"], dual=c["dual"],
                       period=c["period"], cliffs=c["cliffs"],
                       n_cliffs=c["n_cliffs"], blob=c["blob"])
    _MAP_CACHE[k] = (F, B, T)
    return F, B, T


def pack_columns_check(F, B, T):
    """True iff every cell satisfies the column encoding invariants."""
    F = F.astype(np.int32)
    B = B.astype(np.int32)
    T = T.astype(np.int32)
    single = B == 0
    ok = np.where(single, T == 0, (B > F) & (T >= B))
    return bool(ok.all())
