"""FP64 CPU oracle for the Accelerated Fourier SAT hot path (test infrastructure).

Only the tests, the smoke check and the benchmark's CPU-baseline leg may import
this package.  It shares no code with the GPU library: it neither imports the
product package nor is imported by it.  Instances are passed as plain arrays
(any object with ``n, con_off, lits, types, params, weights`` attributes).

Functions follow the paper:
  * ``sat``    -- constraint predicates, Table 1 / Table 2 / Appendix A.
  * ``eval``   -- Walsh-Fourier expansion (Sec. 2.1, Eq. 1) of every constraint,
                  objective (Sec. 2.1.1, Eq. 2) and gradient, in FP64.
  * ``step``   -- the projected gradient step of Algorithm 1.
  * ``verify`` -- rounding and unsat_count of Algorithm 1, on FP32 points.
  * ``pgd``    -- Algorithm 1 with constant step length, FP64.
"""
import ctypes
import os

import numpy as np

from . import build as _build

_lib = None

OR, XOR, NAE, CARD_GE, CARD_LT, AMO, EO, EK = range(8)

_i64p = ctypes.POINTER(ctypes.c_int64)
_i32p = ctypes.POINTER(ctypes.c_int32)
_u32p = ctypes.POINTER(ctypes.c_uint32)
_u8p = ctypes.POINTER(ctypes.c_uint8)
_f32p = ctypes.POINTER(ctypes.c_float)
_f64p = ctypes.POINTER(ctypes.c_double)


def lib():
    global _lib
    if _lib is None:
        path = _build.LIB
        if not os.path.exists(path) or os.path.getmtime(path) < os.path.getmtime(_build.SRC):
            _build.build()
        L = ctypes.CDLL(path)
        L.orc_sat.argtypes = [ctypes.c_int] * 4
        L.orc_sat.restype = ctypes.c_int
        L.orc_eval.argtypes = [ctypes.c_int, ctypes.c_int, _i64p, _i32p, _i32p, _i32p, _f64p,
                               ctypes.c_int, _f64p, _f64p, _f64p, _f64p, _f64p, ctypes.c_int]
        L.orc_eval.restype = ctypes.c_int
        L.orc_step.argtypes = [ctypes.c_int, ctypes.c_int, _f64p, _f64p, ctypes.c_double,
                               _u8p, _u8p, _f64p]
        L.orc_step.restype = None
        L.orc_verify.argtypes = [ctypes.c_int, ctypes.c_int, _i64p, _i32p, _i32p, _i32p,
                                 ctypes.c_int, _f32p, _i32p, _u32p]
        L.orc_verify.restype = ctypes.c_int
        L.orc_pgd.argtypes = [ctypes.c_int, ctypes.c_int, _i64p, _i32p, _i32p, _i32p, _f64p,
                              ctypes.c_int, _f64p, ctypes.c_double, ctypes.c_int, _u8p,
                              _i32p, _i32p, _f64p, ctypes.c_int]
        L.orc_pgd.restype = ctypes.c_int
        _lib = L
    return _lib


def _p(a, t):
    return None if a is None else a.ctypes.data_as(t)


def _arrays(inst):
    con_off = np.ascontiguousarray(inst.con_off, dtype=np.int64)
    lits = np.ascontiguousarray(inst.lits, dtype=np.int32)
    types = np.ascontiguousarray(inst.types, dtype=np.int32)
    params = np.ascontiguousarray(inst.params, dtype=np.int32)
    w = getattr(inst, "weights", None)
    w = None if w is None else np.ascontiguousarray(w, dtype=np.float64)
    return int(inst.n), len(types), con_off, lits, types, params, w


def default_threads():
    try:
        return max(1, len(os.sched_getaffinity(0)))
    except AttributeError:  # pragma: no cover
        return os.cpu_count() or 1


def sat(ctype, k, param, t):
    """Truth predicate (Table 1, Table 2, Appendix A).  True if satisfied."""
    r = lib().orc_sat(int(ctype), int(k), int(param), int(t))
    if r < 0:
        raise ValueError("unknown constraint type %r" % (ctype,))
    return bool(r)


def eval(inst, x, fe=False, adj=False, grad=True, nthreads=None):
    """FE / objective / gradient at the columns of ``x`` (shape (n, B)).

    ``x`` is widened exactly to FP64.  Returns a dict with ``obj`` (B,),
    and optionally ``fe`` (C, B), ``adj`` (L, B) in input literal order, and
    ``grad`` (n, B)."""
    n, C, con_off, lits, types, params, w = _arrays(inst)
    x = np.ascontiguousarray(x, dtype=np.float64)
    if x.ndim != 2 or x.shape[0] != n:
        raise ValueError("x must have shape (n, B)")
    B = x.shape[1]
    L = int(con_off[-1])
    out = {"obj": np.zeros(B)}
    if fe:
        out["fe"] = np.zeros((C, B))
    if adj:
        out["adj"] = np.zeros((L, B))
    if grad:
        out["grad"] = np.zeros((n, B))
    rc = lib().orc_eval(n, C, _p(con_off, _i64p), _p(lits, _i32p), _p(types, _i32p),
                        _p(params, _i32p), _p(w, _f64p), B, _p(x, _f64p),
                        _p(out["obj"], _f64p), _p(out.get("fe"), _f64p),
                        _p(out.get("adj"), _f64p), _p(out.get("grad"), _f64p),
                        int(nthreads or default_threads()))
    if rc:
        raise ValueError("orc_eval failed with status %d" % rc)
    return out


def step(x, grad, lr, fixed=None, done=None):
    """Projected step of Algorithm 1: clip(x - lr*grad, -1, 1), FP64."""
    x = np.ascontiguousarray(x, dtype=np.float64)
    g = np.ascontiguousarray(grad, dtype=np.float64)
    n, B = x.shape
    out = np.empty_like(x)
    fx = None if fixed is None else np.ascontiguousarray(fixed, dtype=np.uint8)
    dn = None if done is None else np.ascontiguousarray(done, dtype=np.uint8)
    lib().orc_step(n, B, _p(x, _f64p), _p(g, _f64p), float(lr), _p(fx, _u8p),
                   _p(dn, _u8p), _p(out, _f64p))
    return out


def verify(inst, x, want_bits=False):
    """Rounding + exact unsat count per restart on FP32 ``x`` (n, B)."""
    n, C, con_off, lits, types, params, _ = _arrays(inst)
    x = np.ascontiguousarray(x, dtype=np.float32)
    B = x.shape[1]
    unsat = np.zeros(B, dtype=np.int32)
    bits = np.zeros((n, (B + 31) // 32), dtype=np.uint32) if want_bits else None
    rc = lib().orc_verify(n, C, _p(con_off, _i64p), _p(lits, _i32p), _p(types, _i32p),
                          _p(params, _i32p), B, _p(x, _f32p), _p(unsat, _i32p),
                          _p(bits, _u32p))
    if rc:
        raise ValueError("orc_verify failed with status %d" % rc)
    return (unsat, bits) if want_bits else unsat


def pgd(inst, x0, lr, steps, fixed=None, nthreads=None):
    """Algorithm 1 with constant step length ``lr``, FP64 throughout."""
    n, C, con_off, lits, types, params, w = _arrays(inst)
    x = np.array(x0, dtype=np.float64, order="C", copy=True)
    B = x.shape[1]
    unsat = np.zeros(B, dtype=np.int32)
    first = np.zeros(B, dtype=np.int32)
    obj = np.zeros(B)
    fx = None if fixed is None else np.ascontiguousarray(fixed, dtype=np.uint8)
    rc = lib().orc_pgd(n, C, _p(con_off, _i64p), _p(lits, _i32p), _p(types, _i32p),
                       _p(params, _i32p), _p(w, _f64p), B, _p(x, _f64p), float(lr),
                       int(steps), _p(fx, _u8p), _p(unsat, _i32p), _p(first, _i32p),
                       _p(obj, _f64p), int(nthreads or default_threads()))
    if rc:
        raise ValueError("orc_pgd failed with status %d" % rc)
    return {"x": x, "unsat": unsat, "first_sat": first, "obj": obj}
