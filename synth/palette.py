"""Colour palettes for the shading pass: 512 RGBA words (R in the low
byte), entries 0..255 for a floor top at height h, 256..511 for a slab top
at height h.  Plain data; the synthetic maps carry no terrain types, so the
colour follows the layer and the height."""
import numpy as np


def _ramp(stops, n=256):
    xs = np.array([s[0] for s in stops], float)
    cols = np.array([s[1] for s in stops], float)
    h = np.arange(n, dtype=float)
    rgb = np.stack([np.interp(h, xs, cols[:, c]) for c in range(3)], axis=1)
    return np.rint(rgb).astype(np.uint32)


def default_palette():
    floor = _ramp([(0, (40, 70, 140)), (20, (194, 178, 128)), (60, (86, 140, 60)),
                   (140, (110, 100, 70)), (200, (150, 140, 130)), (255, (240, 240, 245))])
    slab = _ramp([(0, (90, 80, 75)), (128, (150, 120, 95)), (255, (210, 200, 185))])
    rgb = np.concatenate([floor, slab])
    return (rgb[:, 0] | (rgb[:, 1] << 8) | (rgb[:, 2] << 16) | (0xFF << 24)).astype(np.uint32)


def rgba(r, g, b, a=255):
    return (r | (g << 8) | (b << 16) | (a << 24)) & 0xFFFFFFFF
