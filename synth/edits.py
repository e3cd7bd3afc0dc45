"""Seeded edit lists.

An edit is a dict with keys kind, x0, y0, w, h, depth and, for SET patches,
three uint8 arrays F, B, T of shape (h, w).  The paper's game hands the
renderer a dirty rectangle plus the modified rows (Section 2, Section 4.4);
SET carries exactly that.  CRATER is the headless runner's dig operation
(Section 4.4) as a compact descriptor: a size x size patch at (x0, y0) whose
floor is lowered by a radial profile of the given depth and whose upper slab
is removed inside the radius.  What the descriptor does to the map is defined
by the edit semantics of the library and the oracle, not here.
"""
import numpy as np

EDIT_SET = 1
EDIT_CRATER = 2


def crater_list(seed, W, H, n, size=32, depth=(8, 64)):
    """n craters, fully inside the map. `size` is an int or an inclusive
    (lo, hi) range; `depth` an inclusive (lo, hi) range."""
    rng = np.random.default_rng(seed) if not isinstance(seed, np.random.Generator) else seed
    out = []
    for _ in range(n):
        s = size if isinstance(size, int) else int(rng.integers(size[0], size[1] + 1))
        s = min(s, W, H)
        x0 = int(rng.integers(0, W - s + 1))
        y0 = int(rng.integers(0, H - s + 1))
        d = int(rng.integers(depth[0], depth[1] + 1))
        out.append(dict(kind=EDIT_CRATER, x0=x0, y0=y0, w=s, h=s, depth=d))
    return out


def random_set_patches(seed, W, H, n, max_size=24, allow_outside=True):
    """n SET patches with valid column encodings; some may hang over the map
    edge (they are clipped by the consumer) when allow_outside is set."""
    rng = np.random.default_rng(seed) if not isinstance(seed, np.random.Generator) else seed
    out = []
    for _ in range(n):
        w = int(rng.integers(1, max_size + 1))
        h = int(rng.integers(1, max_size + 1))
        if allow_outside:
            x0 = int(rng.integers(-w + 1, W))
            y0 = int(rng.integers(-h + 1, H))
        else:
            w, h = min(w, W), min(h, H)
            x0 = int(rng.integers(0, W - w + 1))
            y0 = int(rng.integers(0, H - h + 1))
        F = rng.integers(0, 256, size=(h, w)).astype(np.int32)
        two = rng.random((h, w)) < 0.4
        Bv = F + rng.integers(1, 60, size=(h, w))
        two &= Bv <= 255
        B = np.where(two, Bv, 0)
        Tv = np.minimum(255, B + rng.integers(0, 40, size=(h, w)))
        T = np.where(two, Tv, 0)
        out.append(dict(kind=EDIT_SET, x0=x0, y0=y0, w=w, h=h, depth=0,
                        F=F.astype(np.uint8), B=B.astype(np.uint8),
                        T=T.astype(np.uint8)))
    return out
