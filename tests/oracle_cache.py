"""Test helpers: seeded configuration maps and oracle renders, cached.

The full-buffer parity tests of the large configurations compare tens of
millions of records, and the oracle takes seconds to tens of seconds per
frame on the host cores.  Each result is computed once per process and also
kept on disk under tests/.oracle_cache/ (not committed), keyed by a hash of
everything it depends on: the map planes, the views, the edits applied
first and the oracle's own sources.  Only the oracle writes these files.
"""
import functools
import hashlib
import os

import numpy as np

import oracle
import synth

CACHE_DIR = os.environ.get("TC_ORACLE_CACHE",
                           os.path.join(os.path.dirname(os.path.abspath(__file__)),
                                        ".oracle_cache"))
_ORACLE_SRCS = [os.path.join(os.path.dirname(os.path.abspath(oracle.__file__)), f)
                for f in ("oracle.c", "edits.py")]


def host_threads():
    """Threads for the oracle: the cores this process may run on, at most
    16 (the host share of one GPU on the test machines)."""
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:
        n = os.cpu_count() or 1
    return max(1, min(n, 16))


@functools.lru_cache(maxsize=None)
def config_map(k):
    """(F, B, T) of configuration k, generated once per process (read-only)."""
    planes = synth.make_map_from_config(k)
    for p in planes:
        p.setflags(write=False)
    return planes


def _key(F, B, T, views, edits):
    h = hashlib.sha256()
    for a in (F, B, T):
        h.update(np.ascontiguousarray(a).tobytes())
        h.update(repr(a.shape).encode())
    h.update(np.ascontiguousarray(synth.views_array(views)).tobytes())
    for e in edits or []:
        h.update(repr(sorted((k, v) for k, v in e.items()
                             if not isinstance(v, np.ndarray))).encode())
        for k in ("F", "B", "T"):
            if k in e:
                h.update(np.ascontiguousarray(e[k], np.uint8).tobytes())
    for f in _ORACLE_SRCS:
        h.update(open(f, "rb").read())
    return h.hexdigest()[:32]


_memo = {}


def oracle_render(F, B, T, views, edits=None):
    """oracle.render of `views` on the map after `edits` (applied in order
    by oracle.apply_edits), cached in memory and on disk."""
    key = _key(F, B, T, views, edits)
    if key in _memo:
        return _memo[key]
    path = os.path.join(CACHE_DIR, key + ".npz")
    if os.path.exists(path):
        try:
            with np.load(path) as z:
                res = (z["word"], z["depth"])
            _memo[key] = res
            return res
        except (OSError, ValueError, KeyError):
            pass
    if edits:
        F, B, T = oracle.apply_edits(F, B, T, edits)
    res = oracle.render(F, B, T, views, threads=host_threads())
    try:
        os.makedirs(CACHE_DIR, exist_ok=True)
        tmp = path + ".tmp%d.npz" % os.getpid()
        np.savez(tmp, word=res[0], depth=res[1])
        os.replace(tmp, path)
    except OSError:
        pass
    _memo.clear()          # keep one large result in memory at a time
    _memo[key] = res
    return res
