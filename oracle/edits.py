"""Edit semantics, written plainly on numpy planes (test infrastructure).

Section 2 describes edits as local game events that can change a column's
heights and whether it has an upper slab, handed to the renderer as a
changed rectangle with its new rows; Section 4.4's digging lowers the
ground and deletes the slab inside the crater.

  SET    overwrite the rectangle [x0, x0+w) x [y0, y0+h) (clipped to the map)
         with the given F, B, T patch.
  CRATER size s = w = h, depth d: for patch cell (i, j) let
         r2 = (2i+1-s)^2 + (2j+1-s)^2 and R2 = s^2.  If r2 < R2 the floor is
         lowered by floor(d * (R2 - r2) / R2), saturating at 0, and the upper
         slab is removed (B = T = 0).  Clipped to the map.
Edits apply one after another in list order.
"""
import numpy as np

EDIT_SET = 1
EDIT_CRATER = 2


def valid_columns(F, B, T):
    F = np.asarray(F, np.int32)
    B = np.asarray(B, np.int32)
    T = np.asarray(T, np.int32)
    return bool(np.where(B == 0, T == 0, (B > F) & (T >= B)).all())


def apply_edits(F, B, T, edits):
    """Return edited copies of the three planes."""
    F = np.array(F, np.uint8, copy=True)
    B = np.array(B, np.uint8, copy=True)
    T = np.array(T, np.uint8, copy=True)
    H, W = F.shape
    for e in edits:
        x0, y0, w, h = int(e["x0"]), int(e["y0"]), int(e["w"]), int(e["h"])
        if e["kind"] == EDIT_SET:
            for j in range(h):
                y = y0 + j
                if y < 0 or y >= H:
                    continue
                for i in range(w):
                    x = x0 + i
                    if 0 <= x < W:
                        F[y, x] = e["F"][j][i]
                        B[y, x] = e["B"][j][i]
                        T[y, x] = e["T"][j][i]
        elif e["kind"] == EDIT_CRATER:
            s = w
            d = int(e["depth"])
            R2 = s * s
            for j in range(s):
                y = y0 + j
                if y < 0 or y >= H:
                    continue
                for i in range(s):
                    x = x0 + i
                    if x < 0 or x >= W:
                        continue
                    r2 = (2 * i + 1 - s) ** 2 + (2 * j + 1 - s) ** 2
                    if r2 < R2:
                        drop = (d * (R2 - r2)) // R2
                        F[y, x] = max(0, int(F[y, x]) - drop)
                        B[y, x] = 0
                        T[y, x] = 0
        else:
            raise ValueError("unknown edit kind")
    return F, B, T
