"""The evaluation metrics (Section 4.2) on hand-built images whose values
are known by counting."""
import numpy as np

from paper_2608_17390_amd import metrics

MISS = metrics.MISS


def _img(depth):
    d = np.asarray(depth, np.float64)
    w = np.where(np.isfinite(d), 7, MISS).astype(np.uint32)
    return w.reshape(-1), np.where(np.isfinite(d), d, np.inf).reshape(-1)


def test_identical_images_score_zero():
    d = np.add.outer(np.arange(6.0), np.arange(8.0)) + 10
    d[0, :3] = np.inf
    w, dd = _img(d)
    q = metrics.quality(w, dd, w, dd, 8, 6)
    assert q["see_through"] == 0 and q["covers_sky"] == 0
    assert q["depth_err_median"] == 0 and q["depth_err_p95"] == 0
    assert q["coherence"] == 0


def test_coverage_counts():
    ref = np.full((4, 5), 20.0)
    ref[0, :] = np.inf                       # 5 sky pixels in the reference
    r = ref.copy()
    r[2, 1:4] = np.inf                       # renderer drops 3 terrain pixels
    r[0, 0] = 50.0                           # and fills 1 sky pixel
    w, d = _img(r)
    rw, rd = _img(ref)
    q = metrics.quality(w, d, rw, rd, 5, 4)
    assert q["see_through"] == 3 / 20 and q["covers_sky"] == 1 / 20


def test_far_limit_turns_far_hits_into_background():
    ref = np.full((3, 3), 100.0)
    ref[1, 1] = 700.0
    r = ref.copy()
    r[1, 1] = np.inf
    w, d = _img(r)
    rw, rd = _img(ref)
    assert metrics.quality(w, d, rw, rd, 3, 3)["see_through"] == 1 / 9
    assert metrics.quality(w, d, rw, rd, 3, 3, far=600)["see_through"] == 0


def test_depth_error_percentiles():
    ref = np.full((1, 20), 10.0)
    r = ref + np.arange(20) / 10.0           # errors 0.0, 0.1, ..., 1.9
    w, d = _img(r)
    rw, rd = _img(ref)
    q = metrics.quality(w, d, rw, rd, 20, 1)
    assert abs(q["depth_err_median"] - 0.95) < 1e-12
    assert abs(q["depth_err_p95"] - np.percentile(np.arange(20) / 10.0, 95)) < 1e-12


def test_coherence_hole_speck_and_ramp():
    ramp = np.add.outer(np.arange(7.0), 2 * np.arange(9.0)) + 5   # smooth
    assert metrics.incoherent_fraction(ramp) == 0.0
    hole = ramp.copy()
    hole[3, 4] = np.inf                       # a one-pixel hole
    assert metrics.incoherent_fraction(hole) == 1 / 35      # 5 x 7 interior
    speck = np.full((5, 5), np.inf)
    speck[2, 2] = 30.0                         # a lone hit in the sky
    assert metrics.incoherent_fraction(speck) == 1 / 9
    spike = ramp.copy()
    spike[2, 2] = ramp[2, 2] * 1.5             # a depth spike
    assert metrics.incoherent_fraction(spike) == 1 / 35
    tiny = ramp.copy()
    tiny[2, 2] = ramp[1:4, 1:4].max() * 1.005  # within 1 % of the range
    assert metrics.incoherent_fraction(tiny) == 0.0
    # excess over the reference: the renderer's hole counts, the reference's
    # own speck is subtracted
    w, d = _img(hole)
    rw, rd = _img(ramp)
    assert metrics.quality(w, d, rw, rd, 9, 7)["coherence"] == 1 / 35
    assert metrics.quality(rw, rd, w, d, 9, 7)["coherence"] == -1 / 35


def test_quality_views_splits_concatenated_buffers():
    a = np.full((3, 4), 5.0)
    b = np.full((2, 2), 9.0)
    ra, rb = a.copy(), b.copy()
    ra[0, 0] = np.inf
    w = np.concatenate([_img(ra)[0], _img(rb)[0]])
    d = np.concatenate([_img(ra)[1], _img(rb)[1]])
    rw = np.concatenate([_img(a)[0], _img(b)[0]])
    rd = np.concatenate([_img(a)[1], _img(b)[1]])
    views = [{"width": 4, "height": 3}, {"width": 2, "height": 2}]
    q = metrics.quality_views(w, d, rw, rd, views)
    assert q[0]["see_through"] == 1 / 12 and q[1]["see_through"] == 0
