"""ctypes binding of libtc.so: the C ABI of include/tc.h, same names.

Argument marshalling only: every step of the ray cast, the edits and the
pyramid maintenance runs in the library's HIP kernels.  torch supplies
device memory (tensor data pointers) and streams (their HIP handles).  If
the library has not been built, importing the binding fails loudly; there
is no other execution path.
"""
import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libtc.so")

TC_OK = 0
TC_INVALID_ARG = -1
TC_OUT_OF_MEMORY = -2
TC_NO_MAP = -3
TC_DEVICE_ERROR = -4
TC_OVER_BUDGET = -5
TC_TIMEOUT = -6
TC_SERVER_AUTO_RELEASE = 1
TC_S = 65536
TC_MAX_DIM = 16384
TC_MAX_CELLS = 1 << 27
TC_MAX_DIR = (1 << 23) - 1
TC_MISS = 0xFFFFFFFF
TC_FACE_TOP = 1
TC_FACE_UNDER = 2
TC_FACE_WMX = 3
TC_FACE_WPX = 4
TC_FACE_WMY = 5
TC_FACE_WPY = 6
TC_FACE_INSIDE = 7
TC_EDIT_SET = 1
TC_EDIT_CRATER = 2

TC_OPT_RENDER_MODE = 1
TC_OPT_START_LEVEL = 2
TC_OPT_MAX_LEVEL = 3
TC_OPT_XCD_REMAP = 4
TC_OPT_PERSIST_WAVES = 5
TC_OPT_REFILL_MIN = 6
TC_OPT_REFILL_ITERS = 7
TC_OPT_COUNT_READS = 8
TC_OPT_TILE_ORDER = 9
TC_OPT_PRIORITY_BOOST = 10
TC_OPT_SPLIT_BUDGET = 11
TC_OPT_SPLIT_QUEUE = 12
TC_OPT_KERNEL_TIMING = 13
TC_OPT_MARCH_STEPS = 14
TC_OPT_MARCH_BISECT = 15
TC_OPT_MARCH_FAR = 16
TC_OPT_BEAM_PASSES = 17
TC_OPT_SPLIT_WAVES = 18
TC_INFO_ALLOCATIONS = 19
TC_OPT_PACKET_WIDTH = 20
TC_OPT_VOXEL_SHAPE = 21
TC_OPT_INLINE_TABLES = 22
TC_FACE_SAMPLED = 0

_STATUS = {0: "TC_OK", -1: "TC_INVALID_ARG", -2: "TC_OUT_OF_MEMORY",
           -3: "TC_NO_MAP", -4: "TC_DEVICE_ERROR", -5: "TC_OVER_BUDGET",
           -6: "TC_TIMEOUT"}


class tc_view(ctypes.Structure):
    _fields_ = [("width", ctypes.c_int32), ("height", ctypes.c_int32),
                ("o0", ctypes.c_int32 * 3), ("o_px", ctypes.c_int32 * 3),
                ("o_py", ctypes.c_int32 * 3), ("d0", ctypes.c_int32 * 3),
                ("d_px", ctypes.c_int32 * 3), ("d_py", ctypes.c_int32 * 3),
                ("flags", ctypes.c_uint32)]


class tc_edit(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int32), ("x0", ctypes.c_int32),
                ("y0", ctypes.c_int32), ("w", ctypes.c_int32),
                ("h", ctypes.c_int32), ("depth", ctypes.c_int32),
                ("floor_top", ctypes.c_void_p), ("slab_bottom", ctypes.c_void_p),
                ("slab_top", ctypes.c_void_p)]


class tc_tune_result(ctypes.Structure):
    _fields_ = [("render_mode", ctypes.c_int32), ("start_level", ctypes.c_int32),
                ("tile_order", ctypes.c_int32), ("xcd_remap", ctypes.c_int32),
                ("persist_waves", ctypes.c_int32), ("refill_min", ctypes.c_int32),
                ("refill_iters", ctypes.c_int32), ("ms", ctypes.c_float),
                ("tried", ctypes.c_int32), ("split_budget", ctypes.c_int32),
                ("beam_passes", ctypes.c_int32), ("packet_width", ctypes.c_int32),
                ("max_level", ctypes.c_int32)]


class tc_shade_params(ctypes.Structure):
    _fields_ = [("light", ctypes.c_int32 * 3), ("ambient", ctypes.c_float),
                ("cave_ambient", ctypes.c_float), ("fog_far", ctypes.c_float),
                ("sky_rgba", ctypes.c_uint32), ("fog_rgba", ctypes.c_uint32),
                ("palette", ctypes.c_void_p)]


class tc_server_stats(ctypes.Structure):
    _fields_ = [("batches", ctypes.c_uint64), ("edits", ctypes.c_uint64),
                ("views", ctypes.c_uint64), ("rays", ctypes.c_uint64),
                ("peak_bytes", ctypes.c_uint64), ("bytes_in_use", ctypes.c_uint64),
                ("queue_s", ctypes.c_double), ("run_s", ctypes.c_double)]


assert ctypes.sizeof(tc_view) == 84

# (name, restype, argtypes) of every exported symbol of include/tc.h
_P = ctypes.c_void_p
_I32 = ctypes.c_int32
SIGNATURES = [
    ("tc_create", _I32, [ctypes.c_int, ctypes.POINTER(_P)]),
    ("tc_destroy", None, [_P]),
    ("tc_last_error", ctypes.c_char_p, [_P]),
    ("tc_load_columns", _I32, [_P, _I32, _I32, _P, _P, _P, ctypes.c_size_t, _P]),
    ("tc_apply_edit", _I32, [_P, ctypes.POINTER(tc_edit), _I32, _P]),
    ("tc_render_views", _I32, [_P, ctypes.POINTER(tc_view), _I32, _P, _P]),
    ("tc_render_views_noalloc", _I32, [_P, ctypes.POINTER(tc_view), _I32, _P, _P]),
    ("tc_shade_views", _I32, [_P, ctypes.POINTER(tc_view), _I32, _P,
                              ctypes.POINTER(tc_shade_params), _P, _P]),
    ("tc_set_option", _I32, [_P, _I32, ctypes.c_int64]),
    ("tc_get_option", _I32, [_P, _I32, ctypes.POINTER(ctypes.c_int64)]),
    ("tc_read_columns", _I32, [_P, _I32, _I32, _I32, _I32, _P, _P, _P, _P]),
    ("tc_pyramid_info", _I32, [_P, ctypes.POINTER(_I32)]),
    ("tc_pyramid_dims", _I32, [_P, _I32, ctypes.POINTER(_I32), ctypes.POINTER(_I32)]),
    ("tc_read_pyramid", _I32, [_P, _I32, _P, _P]),
    ("tc_read_occupancy", _I32, [_P, _I32, _P, _P]),
    ("tc_read_window", _I32, [_P, _I32, _P, _P]),
    ("tc_voxel_dims", _I32, [_P, _I32, ctypes.POINTER(_I32), ctypes.POINTER(_I32),
                             ctypes.POINTER(_I32), ctypes.POINTER(_I32)]),
    ("tc_read_voxels", _I32, [_P, _I32, _P, _P]),
    ("tc_read_counters", _I32, [_P, ctypes.POINTER(ctypes.c_uint64), _P]),
    ("tc_read_kernel_times", _I32, [_P, ctypes.POINTER(ctypes.c_float)]),
    ("tc_map_bytes", _I32, [_P, ctypes.POINTER(ctypes.c_uint64)]),
    ("tc_frame_create", _I32, [_P, ctypes.POINTER(tc_view), _I32, ctypes.POINTER(tc_edit),
                               _I32, _P, _P, ctypes.POINTER(_P)]),
    ("tc_frame_launch", _I32, [_P, _P]),
    ("tc_frame_rays", _I32, [_P, ctypes.POINTER(ctypes.c_int64)]),
    ("tc_frame_destroy", None, [_P]),
    ("tc_server_start", _I32, [_P, ctypes.c_uint64, _I32, _I32, ctypes.c_uint32,
                               ctypes.POINTER(_P)]),
    ("tc_server_submit_view", _I32, [_P, ctypes.POINTER(tc_view), ctypes.POINTER(ctypes.c_uint64)]),
    ("tc_server_submit_edit", _I32, [_P, ctypes.POINTER(tc_edit), _I32,
                                     ctypes.POINTER(ctypes.c_uint64)]),
    ("tc_server_poll", _I32, [_P, ctypes.c_uint64, ctypes.POINTER(_I32),
                              ctypes.POINTER(ctypes.c_double)]),
    ("tc_server_poll_many", _I32, [_P, _P, _I32, _P, _P]),
    ("tc_server_wait", _I32, [_P, ctypes.c_uint64, ctypes.c_double]),
    ("tc_server_result", _I32, [_P, ctypes.c_uint64, ctypes.POINTER(_P),
                                ctypes.POINTER(ctypes.c_int64)]),
    ("tc_server_read", _I32, [_P, ctypes.c_uint64, _P, ctypes.c_int64]),
    ("tc_server_release", _I32, [_P, ctypes.c_uint64]),
    ("tc_server_get_stats", _I32, [_P, ctypes.POINTER(tc_server_stats)]),
    ("tc_server_stop", _I32, [_P]),
    ("tc_autotune", _I32, [_P, ctypes.POINTER(tc_view), _I32, _P, _I32, _P,
                           ctypes.POINTER(tc_tune_result)]),
]

_lib = None


def load_library(path=LIB_PATH):
    """Load libtc.so (after torch, so both share one HIP runtime)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise ImportError(
            "libtc.so is not built (%s); run `python -m paper_2608_17390_amd.build`"
            % path)
    try:
        import torch  # noqa: F401  -- load torch's HIP runtime first
    except ImportError:
        pass
    lib = ctypes.CDLL(path)
    for name, res, args in SIGNATURES:
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    _lib = lib
    return lib


class TCError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__("%s: %s" % (_STATUS.get(status, status), msg))
        self.status = status


def _check(ctx, st):
    if st != TC_OK:
        msg = load_library().tc_last_error(ctx)
        raise TCError(st, msg.decode() if msg else "")


def _stream_handle(stream):
    if stream is None:
        try:
            import torch
            if torch.cuda.is_available():
                return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
        except ImportError:
            pass
        return ctypes.c_void_p(0)
    if isinstance(stream, int):
        return ctypes.c_void_p(stream)
    return ctypes.c_void_p(stream.cuda_stream)


# numpy layout of tc_view (84 bytes, the field order of the C struct)
_VIEW_NP = np.dtype([("width", "<i4"), ("height", "<i4"), ("o0", "<i4", 3),
                     ("o_px", "<i4", 3), ("o_py", "<i4", 3), ("d0", "<i4", 3),
                     ("d_px", "<i4", 3), ("d_py", "<i4", 3), ("flags", "<u4")])


def _views_struct(views):
    """ctypes array of tc_view: an existing one as is, a numpy structured
    array (or list of records) with the tc_view fields copied in one go."""
    if isinstance(views, ctypes.Array) and views._type_ is tc_view:
        return views
    a = np.asarray(views)
    a = a.reshape(-1)
    if a.dtype.names is not None and set(a.dtype.names) == set(_VIEW_NP.names):
        b = np.zeros(len(a), _VIEW_NP)
        for f in _VIEW_NP.names:
            b[f] = a[f]
        return (tc_view * len(b)).from_buffer_copy(b.tobytes())
    arr = (tc_view * len(a))()
    for i, v in enumerate(a):
        t = arr[i]
        t.width = int(v["width"])
        t.height = int(v["height"])
        for f in ("o0", "o_px", "o_py", "d0", "d_px", "d_py"):
            src = v[f]
            dst = getattr(t, f)
            for c in range(3):
                dst[c] = int(src[c])
        t.flags = int(v["flags"])
    return arr


def _edits_struct(edits):
    arr = (tc_edit * max(1, len(edits)))()
    keep = []
    for i, e in enumerate(edits):
        t = arr[i]
        t.kind = int(e["kind"])
        t.x0 = int(e["x0"])
        t.y0 = int(e["y0"])
        t.w = int(e["w"])
        t.h = int(e["h"])
        t.depth = int(e.get("depth", 0))
        if t.kind == TC_EDIT_SET:
            planes = [np.ascontiguousarray(e[k], np.uint8) for k in ("F", "B", "T")]
            keep.extend(planes)
            t.floor_top = planes[0].ctypes.data
            t.slab_bottom = planes[1].ctypes.data
            t.slab_top = planes[2].ctypes.data
    return arr, keep


class Context:
    """One library context on one HIP device."""

    def __init__(self, device=0):
        lib = load_library()
        h = ctypes.c_void_p()
        st = lib.tc_create(int(device), ctypes.byref(h))
        if st != TC_OK:
            raise TCError(st, lib.tc_last_error(None).decode())
        self._h = h
        self.W = self.H = 0

    @property
    def handle(self):
        return self._h

    def close(self):
        if self._h:
            load_library().tc_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    # -- C ABI calls ------------------------------------------------------
    def tc_load_columns(self, F, B, T, stream=None):
        F = np.ascontiguousarray(F, np.uint8)
        B = np.ascontiguousarray(B, np.uint8)
        T = np.ascontiguousarray(T, np.uint8)
        H, W = F.shape
        st = load_library().tc_load_columns(
            self._h, W, H, F.ctypes.data, B.ctypes.data, T.ctypes.data, W,
            _stream_handle(stream))
        _check(self._h, st)
        self.W, self.H = W, H

    def tc_apply_edit(self, edits, stream=None):
        arr, keep = _edits_struct(list(edits))
        st = load_library().tc_apply_edit(self._h, arr, len(edits),
                                          _stream_handle(stream))
        del keep
        _check(self._h, st)

    def tc_render_views(self, views, out_ptr, stream=None):
        arr = _views_struct(views)
        st = load_library().tc_render_views(self._h, arr, len(arr),
                                            ctypes.c_void_p(int(out_ptr)),
                                            _stream_handle(stream))
        _check(self._h, st)

    def tc_render_views_noalloc(self, views, out_ptr, stream=None):
        arr = _views_struct(views)
        st = load_library().tc_render_views_noalloc(self._h, arr, len(arr),
                                                    ctypes.c_void_p(int(out_ptr)),
                                                    _stream_handle(stream))
        _check(self._h, st)

    def tc_shade_views(self, views, hits_ptr, light, palette, out_ptr, ambient=0.3,
                       cave_ambient=0.12, fog_far=600.0, sky_rgba=0xFFEBCE87,
                       fog_rgba=0xFFD2C8B4, stream=None):
        """Shade the hit records at hits_ptr (device) of `views` into
        out_ptr (device, one uint32 RGBA per pixel); `palette` is 512
        uint32 on the host."""
        arr = _views_struct(views)
        pal = np.ascontiguousarray(palette, np.uint32)
        if pal.size != 512:
            raise ValueError("palette needs 512 entries")
        p = tc_shade_params()
        for c in range(3):
            p.light[c] = int(light[c])
        p.ambient, p.cave_ambient, p.fog_far = ambient, cave_ambient, fog_far
        p.sky_rgba, p.fog_rgba = sky_rgba, fog_rgba
        p.palette = pal.ctypes.data
        st = load_library().tc_shade_views(self._h, arr, len(arr),
                                           ctypes.c_void_p(int(hits_ptr)), ctypes.byref(p),
                                           ctypes.c_void_p(int(out_ptr)),
                                           _stream_handle(stream))
        _check(self._h, st)

    def tc_set_option(self, key, value):
        _check(self._h, load_library().tc_set_option(self._h, int(key), int(value)))

    def tc_get_option(self, key):
        v = ctypes.c_int64()
        _check(self._h, load_library().tc_get_option(self._h, int(key), ctypes.byref(v)))
        return v.value

    def tc_read_columns(self, x0, y0, w, h, stream=None):
        F = np.empty((h, w), np.uint8)
        B = np.empty((h, w), np.uint8)
        T = np.empty((h, w), np.uint8)
        st = load_library().tc_read_columns(self._h, x0, y0, w, h, F.ctypes.data,
                                            B.ctypes.data, T.ctypes.data,
                                            _stream_handle(stream))
        _check(self._h, st)
        return F, B, T

    def tc_pyramid_info(self):
        n = ctypes.c_int32()
        _check(self._h, load_library().tc_pyramid_info(self._h, ctypes.byref(n)))
        return n.value

    def tc_pyramid_dims(self, level):
        w, h = ctypes.c_int32(), ctypes.c_int32()
        _check(self._h, load_library().tc_pyramid_dims(self._h, level, ctypes.byref(w),
                                                       ctypes.byref(h)))
        return w.value, h.value

    def tc_read_occupancy(self, level, stream=None):
        w, h = self.tc_pyramid_dims(level)
        out = np.empty((h, w), np.uint64)
        st = load_library().tc_read_occupancy(self._h, level, out.ctypes.data,
                                              _stream_handle(stream))
        _check(self._h, st)
        return out

    def tc_voxel_dims(self, level):
        """(nx, ny, nz, levels) of voxel level `level`."""
        a, b, c, n = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()
        _check(self._h, load_library().tc_voxel_dims(self._h, level, ctypes.byref(a),
                                                     ctypes.byref(b), ctypes.byref(c),
                                                     ctypes.byref(n)))
        return a.value, b.value, c.value, n.value

    def tc_read_voxels(self, level, stream=None):
        """Voxel level `level` as a bool array [z][y][x]."""
        nx, ny, nz, _ = self.tc_voxel_dims(level)
        out = np.empty((nz, ny, nx), np.uint8)
        st = load_library().tc_read_voxels(self._h, level, out.ctypes.data,
                                           _stream_handle(stream))
        _check(self._h, st)
        return out.astype(bool)

    def tc_read_window(self, level, stream=None):
        w, h = self.tc_pyramid_dims(level)
        out = np.empty((h, w), np.uint32)
        st = load_library().tc_read_window(self._h, level, out.ctypes.data,
                                           _stream_handle(stream))
        _check(self._h, st)
        return out

    def tc_read_pyramid(self, level, stream=None):
        w, h = self.tc_pyramid_dims(level)
        out = np.empty((h, w), np.uint32)
        st = load_library().tc_read_pyramid(self._h, level, out.ctypes.data,
                                            _stream_handle(stream))
        _check(self._h, st)
        return out

    def tc_read_counters(self, stream=None):
        v = ctypes.c_uint64()
        _check(self._h, load_library().tc_read_counters(self._h, ctypes.byref(v),
                                                        _stream_handle(stream)))
        return v.value

    def tc_read_kernel_times(self):
        """(traversal kernel ms, split pass ms) of the last timed render."""
        ms = (ctypes.c_float * 2)()
        _check(self._h, load_library().tc_read_kernel_times(self._h, ms))
        return float(ms[0]), float(ms[1])

    def tc_frame_create(self, views, edits, out_ptr, stream=None):
        varr = _views_struct(views)
        earr, keep = _edits_struct(list(edits))
        h = ctypes.c_void_p()
        st = load_library().tc_frame_create(self._h, varr, len(varr), earr, len(edits),
                                            ctypes.c_void_p(int(out_ptr)),
                                            _stream_handle(stream), ctypes.byref(h))
        del keep
        _check(self._h, st)
        rays = ctypes.c_int64()
        load_library().tc_frame_rays(h, ctypes.byref(rays))
        return Frame(self, h, rays.value)

    def tc_autotune(self, views, out_ptr, reps=5, stream=None):
        arr = _views_struct(views)
        r = tc_tune_result()
        st = load_library().tc_autotune(self._h, arr, len(arr), ctypes.c_void_p(int(out_ptr)),
                                        int(reps), _stream_handle(stream), ctypes.byref(r))
        _check(self._h, st)
        return {f: getattr(r, f) for f, _ in tc_tune_result._fields_}

    def tc_server_start(self, budget_bytes, max_batch_views=64, streams=4, flags=0):
        return Server(self, budget_bytes, max_batch_views, streams, flags)

    def tc_map_bytes(self):
        v = ctypes.c_uint64()
        _check(self._h, load_library().tc_map_bytes(self._h, ctypes.byref(v)))
        return v.value


class Frame:
    """A captured frame (edits, dirty update, render) replayed by launch()."""

    def __init__(self, ctx, handle, rays):
        self._ctx = ctx
        self._h = handle
        self.rays = rays

    def tc_frame_launch(self, stream=None):
        _check(self._ctx.handle, load_library().tc_frame_launch(self._h, _stream_handle(stream)))

    launch = tc_frame_launch

    def close(self):
        if self._h:
            load_library().tc_frame_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Server:
    """Continuous-batching request server over a context's map."""

    def __init__(self, ctx, budget_bytes, max_batch_views=64, streams=4, flags=0):
        self._ctx = ctx
        h = ctypes.c_void_p()
        st = load_library().tc_server_start(ctx.handle, int(budget_bytes), int(max_batch_views),
                                            int(streams), int(flags), ctypes.byref(h))
        _check(ctx.handle, st)
        self._h = h

    def _chk(self, st):
        _check(self._ctx.handle, st)

    def tc_server_submit_view(self, view):
        """view: a view record, or a prebuilt structure from view_struct()."""
        arr = view if isinstance(view, ctypes.Array) else _views_struct([view])
        rid = ctypes.c_uint64()
        self._chk(load_library().tc_server_submit_view(self._h, arr, ctypes.byref(rid)))
        return rid.value

    def tc_server_submit_edit(self, edits):
        """edits: a list of edit dicts, or a prebuilt (structure, keep) pair
        from edits_struct()."""
        if isinstance(edits, tuple):
            arr, keep = edits
            n = len(arr)
            rid = ctypes.c_uint64()
            self._chk(load_library().tc_server_submit_edit(self._h, arr, n, ctypes.byref(rid)))
            return rid.value
        arr, keep = _edits_struct(list(edits))
        rid = ctypes.c_uint64()
        st = load_library().tc_server_submit_edit(self._h, arr, len(edits), ctypes.byref(rid))
        del keep
        self._chk(st)
        return rid.value

    def tc_server_poll(self, rid):
        state, lat = ctypes.c_int32(), ctypes.c_double()
        self._chk(load_library().tc_server_poll(self._h, rid, ctypes.byref(state),
                                                ctypes.byref(lat)))
        return state.value, lat.value

    def tc_server_poll_many(self, rids):
        """(states int32[n], latencies float64[n]) of several requests."""
        ids = np.ascontiguousarray(rids, np.uint64)
        states = np.empty(ids.size, np.int32)
        lat = np.empty(ids.size, np.float64)
        self._chk(load_library().tc_server_poll_many(self._h, ids.ctypes.data, int(ids.size),
                                                     states.ctypes.data, lat.ctypes.data))
        return states, lat

    def tc_server_wait(self, rid, timeout_s=60.0):
        self._chk(load_library().tc_server_wait(self._h, rid, float(timeout_s)))

    def tc_server_read(self, rid, records):
        out = np.empty((records, 2), np.uint32)
        self._chk(load_library().tc_server_read(self._h, rid, out.ctypes.data, records))
        return out[:, 0].copy(), out[:, 1].view(np.float32).copy()

    def tc_server_release(self, rid):
        self._chk(load_library().tc_server_release(self._h, rid))

    def tc_server_get_stats(self):
        st = tc_server_stats()
        self._chk(load_library().tc_server_get_stats(self._h, ctypes.byref(st)))
        return {f: getattr(st, f) for f, _ in tc_server_stats._fields_}

    def tc_server_stop(self):
        if self._h:
            h, self._h = self._h, None
            self._chk(load_library().tc_server_stop(h))

    def __del__(self):
        try:
            self.tc_server_stop()
        except Exception:
            pass


def view_struct(view):
    """Prebuilt C view structure (for low-overhead repeated submission)."""
    return _views_struct([view])


def views_struct(views):
    """Prebuilt C array of several views, accepted wherever views are."""
    return _views_struct(views)


def edits_struct(edits):
    """Prebuilt C edit array plus the buffers it points into."""
    return _edits_struct(list(edits))


def tc_create(device=0):
    return Context(device)


def view_total_rays(views):
    a = np.asarray(views).reshape(-1)
    return int((a["width"].astype(np.int64) * a["height"].astype(np.int64)).sum())


def render(ctx, views, stream=None, out=None):
    """Render views into a (rays, 2) int32 torch tensor on the current
    device: column 0 the hit word (as int32 bits), column 1 the float depth
    bits.  Returns the tensor."""
    import torch
    n = view_total_rays(views)
    if out is None:
        out = torch.empty((n, 2), dtype=torch.int32, device="cuda")
    ctx.tc_render_views(views, out.data_ptr(), stream)
    return out


def split_hits(out):
    """(words uint32, depth float32) numpy arrays from a render tensor."""
    a = out.cpu().numpy()
    return a[:, 0].view(np.uint32).copy(), a[:, 1].view(np.float32).copy()
