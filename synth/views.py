"""Camera poses and their quantisation into integer ray parameters.

A view is W x H pixels. Pixel (px, py) (row py = 0 at the top) casts the ray
    O = o0 + (2px+1) * o_px + (2py+1) * o_py        (Q16 fixed point, S = 2^16)
    D = d0 + (2px+1) * d_px + (2py+1) * d_py        (integers, |D_c| < 2^23)
Perspective views have o_px = o_py = 0; orthographic views (shadow passes,
straight-down test images) have d_px = d_py = 0.

The camera convention fixes the three camera bugs the paper reports for its
reference (Section 4.1 and Section 5.6): the focal length is in pixels and is
derived from the vertical field of view at every resolution, rays go through
pixel centres, and the screen-X basis is the camera's right vector (a camera
turned toward +x sees the +y side of the world on its left).

World axes: x east (map width), y north (map height), z up.  yaw = 0 looks
along +y, yaw = 90 deg looks along +x; pitch > 0 looks up.

Floats are rounded to integers once, here, with round-half-even (numpy.rint),
so the CPU oracle and the GPU library consume identical integers.
"""
import numpy as np

S = 1 << 16                  # fixed-point scale of origins (cells per unit)
MAX_DIR = (1 << 23) - 1      # largest allowed |direction component|
_DIR_TARGET = float(1 << 22) # quantiser scales the largest corner to this

VIEW_DTYPE = np.dtype([
    ("width", "<i4"), ("height", "<i4"),
    ("o0", "<i4", 3), ("o_px", "<i4", 3), ("o_py", "<i4", 3),
    ("d0", "<i4", 3), ("d_px", "<i4", 3), ("d_py", "<i4", 3),
    ("flags", "<u4"),
])
assert VIEW_DTYPE.itemsize == 84


def _basis(yaw_deg, pitch_deg):
    y = np.deg2rad(yaw_deg)
    p = np.deg2rad(pitch_deg)
    fwd = np.array([np.sin(y) * np.cos(p), np.cos(y) * np.cos(p), np.sin(p)])
    right = np.array([np.cos(y), -np.sin(y), 0.0])
    up = np.cross(right, fwd)
    return fwd, right, up


def perspective_view(eye, yaw_deg, pitch_deg, width, height, vfov_deg=60.0,
                     flags=0):
    """Integer parameters of a pinhole camera at `eye` (world units)."""
    fwd, right, up = _basis(yaw_deg, pitch_deg)
    focal = (height / 2.0) / np.tan(np.deg2rad(vfov_deg) / 2.0)
    d0 = fwd * focal - right * (width / 2.0) + up * (height / 2.0)
    dpx = right / 2.0
    dpy = -up / 2.0
    corners = [d0 + (2 * px + 1) * dpx + (2 * py + 1) * dpy
               for px in (0, width - 1) for py in (0, height - 1)]
    scale = _DIR_TARGET / max(np.abs(c).max() for c in corners)
    v = np.zeros((), VIEW_DTYPE)
    v["width"] = width
    v["height"] = height
    v["o0"] = np.rint(np.asarray(eye, float) * S).astype(np.int64)
    v["d0"] = np.rint(d0 * scale).astype(np.int64)
    v["d_px"] = np.rint(dpx * scale).astype(np.int64)
    v["d_py"] = np.rint(dpy * scale).astype(np.int64)
    v["flags"] = flags
    return v


def ortho_view(o0, o_px, o_py, direction, width, height, flags=0):
    """Orthographic view: integer origin lattice, one float direction."""
    d = np.asarray(direction, float)
    m = np.abs(d).max()
    scale = _DIR_TARGET / m if m > 0 else 0.0
    v = np.zeros((), VIEW_DTYPE)
    v["width"] = width
    v["height"] = height
    v["o0"] = np.asarray(o0, np.int64)
    v["o_px"] = np.asarray(o_px, np.int64)
    v["o_py"] = np.asarray(o_py, np.int64)
    v["d0"] = np.rint(d * scale).astype(np.int64)
    v["flags"] = flags
    return v


def shadow_view(x0, y0, size, elevation_deg, azimuth_deg, z0=260, flags=0):
    """Directional shadow-ray pass over a size x size window of cells.

    One ray per cell centre of the window [x0, x0+size) x [y0, y0+size),
    starting at height z0 and travelling along -L, where L points toward the
    light (elevation above the horizon, azimuth measured from +y toward +x).
    Row py of the image is cell row y0 + py.
    """
    el = np.deg2rad(elevation_deg)
    az = np.deg2rad(azimuth_deg)
    L = np.array([np.cos(el) * np.sin(az), np.cos(el) * np.cos(az), np.sin(el)])
    return ortho_view((x0 * S, y0 * S, z0 * S), (S // 2, 0, 0), (0, S // 2, 0),
                      -L, size, size, flags=flags)


def views_array(views):
    a = np.zeros(len(views), VIEW_DTYPE)
    for i, v in enumerate(views):
        a[i] = v
    return a


def view_rays(views):
    a = views_array(views) if not isinstance(views, np.ndarray) else views
    return int((a["width"].astype(np.int64) * a["height"]).sum())


def _free_cell_near(F, B, x, y):
    """Nearest cell (by centre distance) to (x, y) with a single layer."""
    H, W = F.shape
    xi, yi = int(np.floor(x)), int(np.floor(y))
    for r in range(0, max(W, H)):
        x0, x1 = max(0, xi - r), min(W, xi + r + 1)
        y0, y1 = max(0, yi - r), min(H, yi + r + 1)
        sub = B[y0:y1, x0:x1]
        ys, xs = np.nonzero(sub == 0)
        if ys.size:
            cx = xs + x0 + 0.5
            cy = ys + y0 + 0.5
            d = (cx - x) ** 2 + (cy - y) ** 2
            j = int(np.argmin(d))
            return int(xs[j] + x0), int(ys[j] + y0)
    raise ValueError("map has no single-layer cell")


def eye_above_floor(F, B, x, y, dz=2.0):
    cx, cy = _free_cell_near(F, B, x, y)
    return (cx + 0.5, cy + 0.5, float(F[cy, cx]) + dz)


_SIZES = [(256, 256), (640, 480), (1280, 720), (1920, 1080)]


def _random_pose_views(rng, F, B, n):
    H, W = F.shape
    out = []
    eyes = []
    for _ in range(n):
        w, h = _SIZES[int(rng.integers(0, 4))]
        x = rng.uniform(0, W)
        y = rng.uniform(0, H)
        yaw = rng.uniform(0, 360)
        if rng.random() < 0.5:
            eye = eye_above_floor(F, B, x, y)
            pitch = rng.uniform(-15, 5)
        else:
            cx, cy = _free_cell_near(F, B, x, y)
            eye = (cx + 0.5, cy + 0.5, 255.0 + rng.uniform(16, 128))
            pitch = rng.uniform(-75, -30)
        eyes.append(eye)
        out.append(perspective_view(eye, yaw, pitch, w, h))
    return out, eyes


def batched_views(F, B, seed, n_views=64, shadow_every=8, shadow_size=2048):
    """Views of the batched frame: n_views random poses and, after every
    `shadow_every` of them, one shadow pass centred on their eyes."""
    rng = np.random.default_rng(seed)
    H, W = F.shape
    views, eyes = _random_pose_views(rng, F, B, n_views)
    out = []
    for g in range(0, n_views, shadow_every):
        out.extend(views[g:g + shadow_every])
        ex = np.mean([e[0] for e in eyes[g:g + shadow_every]])
        ey = np.mean([e[1] for e in eyes[g:g + shadow_every]])
        size = min(shadow_size, W, H)
        x0 = int(np.clip(np.floor(ex) - size // 2, 0, W - size))
        y0 = int(np.clip(np.floor(ey) - size // 2, 0, H - size))
        az = rng.uniform(0, 360)
        out.append(shadow_view(x0, y0, size, 35.0, az))
    return out


def request_view(rng, F, B):
    v, _ = _random_pose_views(rng, F, B, 1)
    return v[0]


def pitch_views(F, B, seed, width=1280, height=800, pitches=(0, -30, -60, -90),
                per_pitch=3, dz=40.0):
    """Views of the paper's measurement protocol (Section 4.3): per_pitch
    random poses at each pitch, width x height, each eye dz units above a
    single-layer column.  Returns (views, pitch of each view)."""
    rng = np.random.default_rng(seed)
    H, W = F.shape
    views, tags = [], []
    for pitch in pitches:
        for _ in range(per_pitch):
            eye = eye_above_floor(F, B, rng.uniform(0, W), rng.uniform(0, H), dz=dz)
            views.append(perspective_view(eye, rng.uniform(0, 360), pitch, width, height))
            tags.append(pitch)
    return views, tags


def config_views(k, F, B):
    """The fixed views of configurations 1-4 (list of VIEW_DTYPE scalars)."""
    from .configs import config as _config
    c = _config(k)
    if k == 1:
        # eye-level across the map from its west side (an eye at the centre
        # sits in a pit and sees only its walls)
        return [perspective_view(eye_above_floor(F, B, 32.5, 128.5), 0, 0,
                                 320, 240)]
    if k == 2:
        return [perspective_view(eye_above_floor(F, B, 1024.5, 32.5), 0, 0,
                                 1920, 1080)]
    if k == 3:
        H, W = F.shape
        graze = perspective_view(eye_above_floor(F, B, 1024.5, 64.5), 0, -2,
                                 2560, 1440)
        ob = perspective_view((1024.5, min(8192.5, H - 0.5), 319.0), 0, -45,
                              1920, 1080)
        return [graze, ob]
    if k in (4, 5):
        return batched_views(F, B, c["seeds"]["views"])
    raise KeyError(k)
