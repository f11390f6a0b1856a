"""Autotuner for the kernel shape of long constraints (length > 16).

For each length range between consecutive kernel capacities, the constraints of
an instance in that range are packed alone into a sub-instance once per
candidate shape (J lanes per restart x S literals per lane, J*S >= the range's
upper length), the FE+gradient kernel of that bucket is timed on the device
(median of several launches, HIP events on the launch stream), and the fastest
shape wins.  Results are cached in JSON keyed by (GPU architecture, kernel
source revision, restarts, length range), so other instances with constraints
in the same ranges reuse them, and a change to the kernels invalidates them.  The chosen list is passed to ``Instance(..., shapes=...)``.
"""
import hashlib
import json
import os
import time

import numpy as np
import torch

from . import afsat

DEFAULT_CACHE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "tuned_shapes.json")

LANES = (2, 4, 8, 16, 32, 64)
SEGS = tuple(range(8, 33, 2))
SHORT_MAX = 16
MAX_LEN = 1024


def capacities():
    return sorted({j * s for j in LANES for s in SEGS if j * s <= MAX_LEN and j * s > SHORT_MAX})


def length_ranges():
    """[(k_lo, k_hi)] covering 17..1024, split at every candidate capacity."""
    out, lo = [], SHORT_MAX + 1
    for cap in capacities():
        if cap >= lo:
            out.append((lo, cap))
            lo = cap + 1
    return out


def _sub_instance(inst_arrays, cons):
    n, con_off, lits, types, params, weights = inst_arrays
    lens = np.diff(con_off)[cons]
    off = np.zeros(len(cons) + 1, dtype=np.int64)
    np.cumsum(lens, out=off[1:])
    sel = np.concatenate([np.arange(con_off[c], con_off[c + 1]) for c in cons])
    w = None if weights is None else np.asarray(weights)[cons]
    return n, off, np.asarray(lits)[sel], np.asarray(types)[cons], np.asarray(params)[cons], w


def _time_bucket(sub, shape, B, device, reps):
    n, off, lits, types, params, w = sub
    d = afsat.Instance(n, off, lits, types, params, w, device=device, shapes=[shape])
    x = torch.rand((n, B), device=torch.device("cuda", device)) * 2 - 1
    ws = d.workspace(B)
    stream = torch.cuda.current_stream(device)
    d.fe_grad(x, ws)                               # warm up
    times = []
    for _ in range(reps):
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        d.fe_grad(x, ws)
        e1.record(stream)
        e1.synchronize()
        times.append(e0.elapsed_time(e1))
    d.close()
    return float(np.median(times))


def kernel_revision():
    """First 12 hex digits of the SHA-256 of the FE kernels' source."""
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "csrc", "fe_kernels.hip")
    with open(path, "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()[:12]


def arch_name(device=0):
    return torch.cuda.get_device_properties(device).gcnArchName.split(":")[0]


def tune(inst, B, device=0, reps=7, cache_path=None, out_path=None, log=None, max_cons=None):
    """Shapes [(k_hi, J, S)] for the long constraints of ``inst`` at B restarts.

    Cached entries are read from ``cache_path`` and the updated cache is written to
    ``out_path`` (default: ``cache_path``).  ``max_cons`` caps how many constraints
    of a range are timed (a sample is enough to rank shapes).  Returns
    (shapes, report)."""
    arrays = (int(inst.n), np.asarray(inst.con_off, np.int64), np.asarray(inst.lits, np.int32),
              np.asarray(inst.types, np.int32), np.asarray(inst.params, np.int32),
              getattr(inst, "weights", None))
    lens = np.diff(arrays[1])
    cache = {}
    for path in (cache_path, out_path):
        if path and os.path.exists(path):
            with open(path) as f:
                cache.update(json.load(f))
    arch = arch_name(device)
    rev = kernel_revision()
    shapes, report = [], []
    for lo, hi in length_ranges():
        cons = np.nonzero((lens >= lo) & (lens <= hi))[0]
        if cons.size == 0:
            continue
        key = "%s|%s|B=%d|k=%d-%d" % (arch, rev, B, lo, hi)
        if key in cache:
            best = tuple(cache[key]["shape"])
            shapes.append((hi,) + best)
            report.append({"range": [lo, hi], "shape": list(best), "cached": True})
            continue
        if max_cons and cons.size > max_cons:
            cons = np.sort(np.random.default_rng(lo).choice(cons, size=max_cons, replace=False))
        sub = _sub_instance(arrays, cons)
        timings = {}
        for J in LANES:
            for S in SEGS:
                if J * S < hi or J * S >= 2 * hi + 64:   # too small, or mostly padding
                    continue
                t = _time_bucket(sub, (hi, J, S), B, device, reps)
                timings["%dx%d" % (J, S)] = t
        best = min(timings, key=timings.get)
        J, S = (int(v) for v in best.split("x"))
        shapes.append((hi, J, S))
        entry = {"shape": [J, S], "ms": timings, "n_cons_timed": int(cons.size), "when": time.time()}
        cache[key] = entry
        report.append({"range": [lo, hi], "shape": [J, S], "ms": timings})
        if log:
            log("autotune k %d-%d: %s  (%s)" % (lo, hi, best, ", ".join("%s %.3f" % kv for kv in sorted(timings.items(), key=lambda kv: kv[1]))))
    out_path = out_path or cache_path
    cache = {k: v for k, v in cache.items() if k.split("|")[1:2] == [rev]}   # drop stale revisions
    if out_path:
        tmp = out_path + ".tmp%d" % os.getpid()
        with open(tmp, "w") as f:
            json.dump(cache, f, indent=1, sort_keys=True)
        os.replace(tmp, out_path)
    return shapes, report
