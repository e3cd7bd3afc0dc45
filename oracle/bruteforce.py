"""Brute-force first hit over every solid box of every cell (test
infrastructure, tiny maps only).

Each column (x, y) contributes up to two closed boxes in S-scaled units:
  floor  [xS, (x+1)S] x [yS, (y+1)S] x (-inf, F*S]
  slab   [xS, (x+1)S] x [yS, (y+1)S] x [B*S, T*S]        (only when B > 0)
which is the solid set of the paper's SOLID predicate (Section 3.1) over the
column's footprint.  The ray P(t) = O + t D, t >= 0, is clipped against each
box with the slab method in exact rational arithmetic (fractions.Fraction).
Nothing here walks cells in order: every box is tested.

check_ray() compares one oracle result against this brute force:
  * the oracle's time must never precede the earliest box entry t*;
  * every box entered strictly before the oracle's time must lie in a
    column whose open square the ray never enters for t > 0 -- a lattice
    corner touch, a run exactly along a cell edge, or an origin on the
    boundary moving away.  A cell walk cannot visit such a column, and these
    are exactly the measure-zero ties the cell-boundary convention decides;
  * when the oracle hits at t*, its (cell, layer, face) must be one of the
    boxes entered at t*, through one of the faces achieving that entry.
    At t* = 0 (origin on a solid boundary) an interior start and a boundary
    entry are the same event, so the face is not compared there.
"""
from fractions import Fraction

S = 65536
FACE = {"x+": 3, "x-": 4, "y+": 5, "y-": 6}
TOP, UNDER, INSIDE = 1, 2, 7


def _axis(o, d, lo, hi):
    """Closed time interval of lo <= o + t d <= hi; None for empty.
    lo/hi None mean unbounded; returns (tlo, thi) with None = infinite."""
    if d == 0:
        if (lo is not None and o < lo) or (hi is not None and o > hi):
            return None
        return (None, None)
    a = None if lo is None else Fraction(lo - o, d)
    b = None if hi is None else Fraction(hi - o, d)
    if d < 0:
        a, b = b, a
    return (a, b)


def box_entry(O, D, x, y, zlo, zhi):
    """Entry of the ray into the closed box; returns (t, axes) where axes is
    the set of axis names achieving the entry ('x','y','z'; 'inside' when the
    origin is strictly inside on every bounded axis), or None."""
    ivs = {
        "x": _axis(O[0], D[0], x * S, (x + 1) * S),
        "y": _axis(O[1], D[1], y * S, (y + 1) * S),
        "z": _axis(O[2], D[2], zlo, zhi),
    }
    if any(v is None for v in ivs.values()):
        return None
    lo = None
    for v in ivs.values():
        if v[0] is not None and (lo is None or v[0] > lo):
            lo = v[0]
    hi = None
    for v in ivs.values():
        if v[1] is not None and (hi is None or v[1] < hi):
            hi = v[1]
    t = Fraction(0) if lo is None or lo < 0 else lo
    if hi is not None and t > hi:
        return None
    axes = set()
    if lo is None or lo < 0:
        axes.add("inside")
    else:
        for k, v in ivs.items():
            if v[0] is not None and v[0] == lo:
                axes.add(k)
    return t, axes


def _faces(axes, D, layer):
    out = set()
    for a in axes:
        if a == "inside":
            out.add(INSIDE)
        elif a == "x":
            out.add(FACE["x+"] if D[0] > 0 else FACE["x-"])
        elif a == "y":
            out.add(FACE["y+"] if D[1] > 0 else FACE["y-"])
        elif a == "z":
            out.add(TOP if D[2] < 0 else UNDER)
    return out


def all_entries(F, B, T, O, D):
    """Every box the ray enters: list of (t, x, y, layer, faces)."""
    H, W = len(F), len(F[0])
    out = []
    for y in range(H):
        for x in range(W):
            f, b, tt = int(F[y][x]), int(B[y][x]), int(T[y][x])
            e = box_entry(O, D, x, y, None, f * S)
            if e is not None:
                out.append((e[0], x, y, 0, _faces(e[1], D, 0)))
            if b > 0:
                e = box_entry(O, D, x, y, b * S, tt * S)
                if e is not None:
                    out.append((e[0], x, y, 1, _faces(e[1], D, 1)))
    return out


def open_square_never_entered(O, D, x, y):
    """True iff P(t) lies in the open square (x, x+1) x (y, y+1) for no
    t > 0."""
    lo, hi = Fraction(0), None
    for o, d, a in ((O[0], D[0], x), (O[1], D[1], y)):
        if d == 0:
            if not (a * S < o < (a + 1) * S):
                return True
            continue
        t1 = Fraction(a * S - o, d)
        t2 = Fraction((a + 1) * S - o, d)
        if t1 > t2:
            t1, t2 = t2, t1
        lo = max(lo, t1)
        hi = t2 if hi is None else min(hi, t2)
    return hi is not None and lo >= hi


def check_ray(F, B, T, O, D, word, tn, td):
    """Return None if the oracle result agrees with brute force, else a
    message."""
    W = len(F[0])
    if all(d == 0 for d in D):
        return None if word == 0xFFFFFFFF else "zero direction must miss"
    ents = all_entries(F, B, T, O, D)
    miss = word == 0xFFFFFFFF
    t_or = None if miss else Fraction(int(tn), int(td))
    if not miss and t_or < 0:
        return "negative hit time"
    early = [e for e in ents if t_or is None or e[0] < t_or]
    for e in early:
        if not open_square_never_entered(O, D, e[1], e[2]):
            return "missed box cell=(%d,%d) layer=%d at t=%s (oracle t=%s)" % (
                e[1], e[2], e[3], e[0], t_or)
    if miss:
        return None
    cell = word & 0x07FFFFFF
    face = (word >> 27) & 7
    layer = (word >> 30) & 1
    x, y = cell % W, cell // W
    same = [e for e in ents if e[0] == t_or and e[1] == x and e[2] == y
            and e[3] == layer]
    if not same:
        return "oracle hit cell=(%d,%d) layer=%d t=%s is not a box entry" % (
            x, y, layer, t_or)
    if t_or == 0:
        return None
    faces = set().union(*[e[4] for e in same])
    if face not in faces:
        return "face %d not in admissible %s" % (face, sorted(faces))
    return None
