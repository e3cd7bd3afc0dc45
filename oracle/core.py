"""ctypes front end of the C oracle (test infrastructure only)."""
import ctypes
import os

import numpy as np

from .build import LIB, SOURCES, build

_lib = None

# Same 84-byte record layout as the input generator's view dtype.
VIEW_FIELDS = [("width", "<i4"), ("height", "<i4"),
               ("o0", "<i4", 3), ("o_px", "<i4", 3), ("o_py", "<i4", 3),
               ("d0", "<i4", 3), ("d_px", "<i4", 3), ("d_py", "<i4", 3),
               ("flags", "<u4")]
VIEW_DT = np.dtype(VIEW_FIELDS)
MISS = 0xFFFFFFFF


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB) or os.path.getmtime(LIB) < max(
                os.path.getmtime(f) for f in SOURCES):
            build()
        L = ctypes.CDLL(LIB)
        p = ctypes.c_void_p
        L.or_render_rows.restype = ctypes.c_int64
        L.or_render_rows.argtypes = [ctypes.c_int32, ctypes.c_int32, p, p, p,
                                     p, ctypes.c_int, ctypes.c_int32,
                                     ctypes.c_int32, ctypes.c_int32, p, p,
                                     ctypes.c_int]
        L.or_cast_list.restype = None
        L.or_cast_list.argtypes = [ctypes.c_int32, ctypes.c_int32, p, p, p, p,
                                   p, ctypes.c_int64, p, p]
        L.or_cast_list_exact.restype = None
        L.or_cast_list_exact.argtypes = [ctypes.c_int32, ctypes.c_int32, p, p,
                                         p, p, p, ctypes.c_int64, p, p, p, p]
        L.or_cast_pixels.restype = None
        L.or_cast_pixels.argtypes = [ctypes.c_int32, ctypes.c_int32, p, p, p,
                                     p, p, p, p, ctypes.c_int64, p, p]
        f32, i32, i64 = ctypes.c_float, ctypes.c_int32, ctypes.c_int64
        L.om_march_rows.restype = i64
        L.om_march_rows.argtypes = [i32, i32, p, p, p, p, ctypes.c_int, i32, i32,
                                    i32, f32, ctypes.c_int, ctypes.c_int, p, p,
                                    ctypes.c_int, p]
        L.om_march_list.restype = None
        L.om_march_list.argtypes = [i32, i32, p, p, p, p, p, i64, f32,
                                    ctypes.c_int, ctypes.c_int, p, p]
        L.om_march_pixels.restype = None
        L.om_march_pixels.argtypes = [i32, i32, p, p, p, p, p, p, p, i64, f32,
                                      ctypes.c_int, ctypes.c_int, p, p]
        L.os_shade_views.restype = i64
        L.os_shade_views.argtypes = [i32, i32, p, p, p, p, ctypes.c_int, p, p, p]
        L.os_shade_pixels.restype = i64
        L.os_shade_pixels.argtypes = [i32, i32, p, p, p, p, p, p, p, i64, p, p, p]
        _lib = L
    return _lib


def default_threads():
    """Threads of a multi-threaded oracle call: the cores this process may
    run on, at most 16."""
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:
        n = os.cpu_count() or 1
    return max(1, min(n, 16))


def _ptr(a):
    return a.ctypes.data_as(ctypes.c_void_p)


def _map(F, B, T):
    F = np.ascontiguousarray(F, np.uint8)
    B = np.ascontiguousarray(B, np.uint8)
    T = np.ascontiguousarray(T, np.uint8)
    assert F.shape == B.shape == T.shape and F.ndim == 2
    return F, B, T


def _views(views):
    v = np.ascontiguousarray(np.asarray(views).astype(VIEW_DT))
    return v.reshape(-1)


def render(F, B, T, views, threads=None, rows=None):
    """Hit records of every pixel of every view, views concatenated, rows
    top-down.  Returns (word uint32[n], depth float64[n]).  `rows` =
    (row0, row1, step) restricts the rows cast in each view."""
    F, B, T = _map(F, B, T)
    v = _views(views)
    H, W = F.shape
    r0, r1, st = rows if rows is not None else (0, 1 << 30, 1)
    n = 0
    for x in v:
        hh = min(int(x["height"]), r1)
        n += int(x["width"]) * len(range(r0, hh, st)) if hh > r0 else 0
    word = np.empty(n, np.uint32)
    depth = np.empty(n, np.float64)
    th = threads if threads else default_threads()
    got = lib().or_render_rows(W, H, _ptr(F), _ptr(B), _ptr(T), _ptr(v),
                               len(v), r0, r1, st, _ptr(word), _ptr(depth), th)
    if got != n:
        raise RuntimeError("oracle render failed")
    return word, depth


def cast_rays(F, B, T, O, D):
    """Cast explicit rays: O, D int64 arrays of shape (n, 3)."""
    F, B, T = _map(F, B, T)
    H, W = F.shape
    O = np.ascontiguousarray(O, np.int64).reshape(-1, 3)
    D = np.ascontiguousarray(D, np.int64).reshape(-1, 3)
    n = O.shape[0]
    word = np.empty(n, np.uint32)
    depth = np.empty(n, np.float64)
    lib().or_cast_list(W, H, _ptr(F), _ptr(B), _ptr(T), _ptr(O), _ptr(D), n,
                       _ptr(word), _ptr(depth))
    return word, depth


def cast_rays_exact(F, B, T, O, D):
    """Like cast_rays, also returning the exact hit time numerator and
    denominator (tn = -1 on a miss)."""
    F, B, T = _map(F, B, T)
    H, W = F.shape
    O = np.ascontiguousarray(O, np.int64).reshape(-1, 3)
    D = np.ascontiguousarray(D, np.int64).reshape(-1, 3)
    n = O.shape[0]
    word = np.empty(n, np.uint32)
    depth = np.empty(n, np.float64)
    tn = np.empty(n, np.int64)
    td = np.empty(n, np.int64)
    lib().or_cast_list_exact(W, H, _ptr(F), _ptr(B), _ptr(T), _ptr(O), _ptr(D),
                             n, _ptr(word), _ptr(depth), _ptr(tn), _ptr(td))
    return word, depth, tn, td


def cast_pixels(F, B, T, views, vi, px, py):
    """Cast selected pixels (view index, column, row) of a list of views."""
    F, B, T = _map(F, B, T)
    H, W = F.shape
    v = _views(views)
    vi = np.ascontiguousarray(vi, np.int32)
    px = np.ascontiguousarray(px, np.int32)
    py = np.ascontiguousarray(py, np.int32)
    n = vi.size
    word = np.empty(n, np.uint32)
    depth = np.empty(n, np.float64)
    lib().or_cast_pixels(W, H, _ptr(F), _ptr(B), _ptr(T), _ptr(v), _ptr(vi),
                         _ptr(px), _ptr(py), n, _ptr(word), _ptr(depth))
    return word, depth


def _march_args(far, steps, bisect):
    if not (far > 0 and 1 <= steps and 0 <= bisect):
        raise ValueError("march needs far > 0, steps >= 1, bisect >= 0")
    return float(np.float32(far)), int(steps), int(bisect)


def march(F, B, T, views, far=600.0, steps=128, bisect=4, threads=None,
          rows=None, with_reads=False):
    """Sampled march (Section 3.1 RAYMARCH, single precision) of every pixel
    of every view.  Returns (word uint32[n], depth float32[n]) and, with
    with_reads, the number of in-map samples tested."""
    F, B, T = _map(F, B, T)
    v = _views(views)
    H, W = F.shape
    r0, r1, st = rows if rows is not None else (0, 1 << 30, 1)
    n = 0
    for x in v:
        hh = min(int(x["height"]), r1)
        n += int(x["width"]) * len(range(r0, hh, st)) if hh > r0 else 0
    word = np.empty(n, np.uint32)
    depth = np.empty(n, np.float32)
    reads = ctypes.c_int64(0)
    th = threads if threads else default_threads()
    got = lib().om_march_rows(W, H, _ptr(F), _ptr(B), _ptr(T), _ptr(v), len(v),
                              r0, r1, st, *_march_args(far, steps, bisect),
                              _ptr(word), _ptr(depth), th, ctypes.byref(reads))
    if got != n:
        raise RuntimeError("oracle march failed")
    return (word, depth, reads.value) if with_reads else (word, depth)


def march_rays(F, B, T, O, D, far=600.0, steps=128, bisect=4):
    """Sampled march of explicit rays: O, D int64 arrays of shape (n, 3)."""
    F, B, T = _map(F, B, T)
    H, W = F.shape
    O = np.ascontiguousarray(O, np.int64).reshape(-1, 3)
    D = np.ascontiguousarray(D, np.int64).reshape(-1, 3)
    n = O.shape[0]
    word = np.empty(n, np.uint32)
    depth = np.empty(n, np.float32)
    lib().om_march_list(W, H, _ptr(F), _ptr(B), _ptr(T), _ptr(O), _ptr(D), n,
                        *_march_args(far, steps, bisect), _ptr(word), _ptr(depth))
    return word, depth


def march_pixels(F, B, T, views, vi, px, py, far=600.0, steps=128, bisect=4):
    """Sampled march of selected pixels (view index, column, row)."""
    F, B, T = _map(F, B, T)
    H, W = F.shape
    v = _views(views)
    vi = np.ascontiguousarray(vi, np.int32)
    px = np.ascontiguousarray(px, np.int32)
    py = np.ascontiguousarray(py, np.int32)
    n = vi.size
    word = np.empty(n, np.uint32)
    depth = np.empty(n, np.float32)
    lib().om_march_pixels(W, H, _ptr(F), _ptr(B), _ptr(T), _ptr(v), _ptr(vi),
                          _ptr(px), _ptr(py), n, *_march_args(far, steps, bisect),
                          _ptr(word), _ptr(depth))
    return word, depth


SHADE_DT = np.dtype([("light", "<i4", 3), ("ambient", "<f4"), ("cave_ambient", "<f4"),
                     ("fog_far", "<f4"), ("sky_rgba", "<u4"), ("fog_rgba", "<u4")])


def _shade_params(light, ambient, cave_ambient, fog_far, sky_rgba, fog_rgba):
    p = np.zeros(1, SHADE_DT)
    p["light"] = np.asarray(light, np.int64)
    p["ambient"] = ambient
    p["cave_ambient"] = cave_ambient
    p["fog_far"] = fog_far
    p["sky_rgba"] = sky_rgba
    p["fog_rgba"] = fog_rgba
    return p


def shade(F, B, T, views, light, palette, ambient=0.3, cave_ambient=0.12,
          fog_far=600.0, sky_rgba=0xFFEBCE87, fog_rgba=0xFFD2C8B4):
    """Shaded RGBA (uint32 R | G<<8 | B<<16 | A<<24) of every pixel of every
    view: exact hit, shadow ray along `light` (integer direction toward the
    light), palette (512 uint32: floor by height, then slab top by
    height), gradient normal, ambient / cave ambient, linear fog."""
    F, B, T = _map(F, B, T)
    v = _views(views)
    H, W = F.shape
    pal = np.ascontiguousarray(palette, np.uint32)
    assert pal.size == 512
    prm = _shade_params(light, ambient, cave_ambient, fog_far, sky_rgba, fog_rgba)
    n = int((v["width"].astype(np.int64) * v["height"]).sum())
    out = np.empty(n, np.uint32)
    err = lib().os_shade_views(W, H, _ptr(F), _ptr(B), _ptr(T), _ptr(v), len(v),
                               _ptr(prm), _ptr(pal), _ptr(out))
    if err:
        raise RuntimeError("shading oracle: %d face times disagree with the cast" % err)
    return out


def shade_pixels(F, B, T, views, vi, px, py, light, palette, ambient=0.3,
                 cave_ambient=0.12, fog_far=600.0, sky_rgba=0xFFEBCE87,
                 fog_rgba=0xFFD2C8B4):
    """shade() of selected pixels (view index, column, row)."""
    F, B, T = _map(F, B, T)
    H, W = F.shape
    v = _views(views)
    vi = np.ascontiguousarray(vi, np.int32)
    px = np.ascontiguousarray(px, np.int32)
    py = np.ascontiguousarray(py, np.int32)
    pal = np.ascontiguousarray(palette, np.uint32)
    prm = _shade_params(light, ambient, cave_ambient, fog_far, sky_rgba, fog_rgba)
    out = np.empty(vi.size, np.uint32)
    err = lib().os_shade_pixels(W, H, _ptr(F), _ptr(B), _ptr(T), _ptr(v), _ptr(vi),
                                _ptr(px), _ptr(py), vi.size, _ptr(prm), _ptr(pal),
                                _ptr(out))
    if err:
        raise RuntimeError("shading oracle: %d face times disagree with the cast" % err)
    return out


def decode(word):
    """Split hit words into (cell, face, layer, miss) arrays."""
    word = np.asarray(word, np.uint32)
    miss = word == MISS
    cell = (word & 0x07FFFFFF).astype(np.int64)
    face = ((word >> 27) & 7).astype(np.int32)
    layer = ((word >> 30) & 1).astype(np.int32)
    return cell, face, layer, miss
