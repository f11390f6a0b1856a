"""Autotuner for the FE kernel configuration per length range: a thin binding of
``afs_autotune`` (``include/afsat.h``), which times the candidates on the device
-- the segment shape above length 16 and, with ``tiles=True``, the work tile of
every range and the restarts per lane of the one-lane kernel for each length up
to 16 -- and keeps a text cache keyed by GPU architecture, FE kernel revision,
restarts, range and size class.  The tile stage ranks configurations by their
time alone; in iterations of mixed lengths, where short buckets run beside long
ones, its choices made the iteration slower, so it is off by default.

``tune(inst, B)`` returns the list ``[(k_hi, J, S, tile, rpl)]`` that
``Instance(..., shapes=...)`` takes, and a report per range.  The package ships
the cache for the bench workloads (``tuned_shapes.txt``)."""
import ctypes
import os

import numpy as np

from . import afsat

DEFAULT_CACHE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "tuned_shapes.txt")
MAX_RANGES = 512


def _path(p):
    return None if p is None else os.fsencode(p)


def tune(inst, B, device=0, reps=7, cache_path=None, out_path=None, log=None, max_cons=None, tiles=False):
    """Configurations [(k_hi, J, S, tile, rpl)] for the lengths of ``inst`` (a
    workloads Instance or an afsat.Instance) at B restarts (J == 1: one-lane
    length k_hi, S == k_hi; tile and rpl 0: the defaults, always so unless
    ``tiles``).

    Cached results are read from ``cache_path`` and ``out_path`` (``cache_path``'s
    where both hold one for a range); ``out_path`` (default: ``cache_path``) is
    rewritten with them and the new ones.
    ``max_cons`` caps how many constraints of a range are timed (a sample is
    enough to rank shapes).  Returns (shapes, report)."""
    own = None
    if isinstance(inst, afsat.Instance):
        h = inst
    else:
        own = h = afsat.Instance.from_arrays(inst, device=-1)     # host tables only
    out_path = out_path or cache_path
    lo, hi, lanes, seg, tile, rpl = (np.zeros(MAX_RANGES, np.int32) for _ in range(6))
    ms = np.zeros(MAX_RANGES, np.float32)
    n = ctypes.c_int32(0)
    i32p = ctypes.POINTER(ctypes.c_int32)
    try:
        afsat._check(afsat.lib().afs_autotune(
            h._h, int(device), int(B), int(reps), int(max_cons or 0), int(bool(tiles)), _path(cache_path),
            _path(out_path),
            MAX_RANGES, lo.ctypes.data_as(i32p), hi.ctypes.data_as(i32p), lanes.ctypes.data_as(i32p),
            seg.ctypes.data_as(i32p), tile.ctypes.data_as(i32p), rpl.ctypes.data_as(i32p),
            ms.ctypes.data_as(ctypes.POINTER(ctypes.c_float)), ctypes.byref(n)))
    finally:
        if own is not None:
            own.close()
    if n.value > MAX_RANGES:
        raise RuntimeError("more length ranges than expected")
    shapes, report = [], []
    for i in range(n.value):
        shapes.append((int(hi[i]), int(lanes[i]), int(seg[i]), int(tile[i]), int(rpl[i])))
        cached, timed = bool(ms[i] < 0), bool(ms[i] > 0)
        report.append({"range": [int(lo[i]), int(hi[i])], "shape": [int(lanes[i]), int(seg[i])],
                       "tile": int(tile[i]), "rpl": int(rpl[i]), "cached": cached, "timed": timed,
                       "ms": float(ms[i]) if timed else None})
        if log and timed:
            log("autotune k %d-%d: %dx%d tile %d rpl %d  %.3f ms" % (lo[i], hi[i], lanes[i], seg[i], tile[i],
                                                                   rpl[i], ms[i]))
    return shapes, report
