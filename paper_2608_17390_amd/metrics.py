"""Image-quality metrics of the paper's evaluation (Section 4.2), comparing
a renderer's hit buffer with a reference's over one view.

  coverage   see-through: fraction of pixels where the reference has
             terrain and the renderer left background; covers-sky: the
             reverse.
  geometry   median and 95th percentile of |depth - reference depth| over
             the pixels where both have terrain.
  coherence  fraction of pixels whose distance disagrees with their own 3x3
             neighbourhood, in excess of the reference doing the same.

Readings where the paper gives no formula:
  * "terrain present" = a hit within the far limit when one is given (a
    reference hit beyond the renderer's far limit counts as background);
  * a pixel disagrees with its neighbourhood when its distance lies outside
    the range of its eight neighbours' distances by more than `rel` (1 %) of
    its own distance, background counting as infinitely far; border pixels
    (without eight neighbours) are not scored.  A pixel on a smooth surface
    lies between its neighbours and never counts; a speck, a hole or a crack
    one pixel wide does.

Host-side numpy on hit records already copied off the GPU (word uint32,
depth float); this module runs no render.
"""
import numpy as np

MISS = 0xFFFFFFFF


def present(word, depth, far=None):
    word = np.asarray(word, np.uint32)
    p = word != MISS
    if far is not None:
        p &= np.asarray(depth, np.float64) <= far
    return p


def incoherent_fraction(dist, rel=0.01):
    """Fraction of interior pixels of an (h, w) distance image (np.inf for
    background) lying outside their 8 neighbours' range by more than rel
    times their own distance."""
    d = np.asarray(dist, np.float64)
    h, w = d.shape
    if h < 3 or w < 3:
        return 0.0
    c = d[1:-1, 1:-1]
    nb = [d[1 + dy:h - 1 + dy, 1 + dx:w - 1 + dx]
          for dy in (-1, 0, 1) for dx in (-1, 0, 1) if dy or dx]
    lo = np.minimum.reduce(nb)
    hi = np.maximum.reduce(nb)
    tau = np.where(np.isfinite(c), rel * c, 0.0)
    with np.errstate(invalid="ignore"):
        bad = (c < lo - tau) | (c > hi + tau)
    return float(bad.mean())


def quality(word, depth, ref_word, ref_depth, width, height, far=None, rel=0.01):
    """Metrics of one view (buffers of width*height records, row-major)."""
    n = width * height
    word, depth = np.asarray(word)[:n], np.asarray(depth, np.float64)[:n]
    ref_word, ref_depth = np.asarray(ref_word)[:n], np.asarray(ref_depth, np.float64)[:n]
    p = present(word, depth, far)
    q = present(ref_word, ref_depth, far)
    both = p & q
    err = np.abs(depth[both] - ref_depth[both])
    dr = np.where(p, depth, np.inf).reshape(height, width)
    dq = np.where(q, ref_depth, np.inf).reshape(height, width)
    ir = incoherent_fraction(dr, rel)
    iq = incoherent_fraction(dq, rel)
    return {
        "see_through": float(np.mean(q & ~p)),
        "covers_sky": float(np.mean(p & ~q)),
        "depth_err_median": float(np.median(err)) if err.size else 0.0,
        "depth_err_p95": float(np.percentile(err, 95)) if err.size else 0.0,
        "coherence": ir - iq,
        "incoherent": ir,
        "incoherent_ref": iq,
    }


def quality_views(word, depth, ref_word, ref_depth, views, far=None, rel=0.01):
    """Per-view metrics of concatenated buffers of several views."""
    out = []
    off = 0
    for v in views:
        w, h = int(v["width"]), int(v["height"])
        sl = slice(off, off + w * h)
        out.append(quality(word[sl], depth[sl], ref_word[sl], ref_depth[sl], w, h, far, rel))
        off += w * h
    return out
