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
  * ``pgd``    -- Algorithm 1 with constant step length, FP64 (with the
                  step-length rule delta and the location rule epsilon).
  * ``line_search_step`` / ``pgd_search`` -- Algorithm 1 with lineSearch taken
                  as backtracking from a maximum step s with the Armijo
                  sufficient-decrease test along the projection arc, FP64.
  * ``fixed_columns`` -- the partial-assignment slices of Sec. 3.4 (the restarts
                  divided evenly among the rows of a fixed mask).
  * ``pgd_momentum`` -- one of the other search algorithms Sec. 3.2 says can take
                  PGD's place: projected gradient descent with heavy-ball
                  momentum, FP64.
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


def fixed_columns(fixed, n, B):
    """Boolean (n, B) mask of held variables for a fixed mask shaped (n,) or
    (P, n): restart b uses row b*P//B (Sec. 3.4 divides the restarts evenly
    among the partial assignments)."""
    if fixed is None:
        return np.zeros((n, B), dtype=bool)
    f = np.asarray(fixed)
    if f.ndim == 1:
        f = f[None, :]
    P = f.shape[0]
    rows = (np.arange(B, dtype=np.int64) * P) // max(B, 1)
    return (f[rows, :] != 0).T.copy()


def _slices(fixed, B):
    """(columns, row) pairs of the restarts that share one row of ``fixed``."""
    f = np.asarray(fixed)
    P = 1 if f.ndim == 1 else f.shape[0]
    rows = (np.arange(B, dtype=np.int64) * P) // max(B, 1)
    out = []
    for p in range(P):
        cols = np.nonzero(rows == p)[0]
        if cols.size:
            out.append((cols, f if f.ndim == 1 else f[p]))
    return out


def pgd(inst, x0, lr, steps, fixed=None, nthreads=None, delta=0.0, epsilon=0.0):
    """Algorithm 1 with constant step length ``lr``, FP64 throughout.

    ``fixed`` may hold several partial assignments (P, n); the restarts are then
    run slice by slice (restarts are independent).  With ``delta`` > lr every
    restart that has not verified after the first iteration has converged
    (eta = lr < delta) and stops there.  With ``epsilon`` > 0 a restart that has
    not verified converges once its new point lies within epsilon of the
    previous one in every variable (Sec. 3.3's location test); the result then
    also holds ``done`` (0 running, 1 verified, 2 converged)."""
    if epsilon > 0:
        return _pgd_steps(inst, x0, lr, steps, fixed, delta, epsilon, nthreads)
    if fixed is not None and np.asarray(fixed).ndim == 2:
        x0 = np.asarray(x0)
        out = {"x": np.array(x0, dtype=np.float64), "unsat": np.zeros(x0.shape[1], np.int32),
               "first_sat": np.zeros(x0.shape[1], np.int32), "obj": np.zeros(x0.shape[1])}
        for cols, row in _slices(fixed, x0.shape[1]):
            r = pgd(inst, x0[:, cols], lr, steps, fixed=row, nthreads=nthreads, delta=delta)
            for k in out:
                if k == "x":
                    out[k][:, cols] = r[k]
                else:
                    out[k][cols] = r[k]
        return out
    if delta > 0 and lr < delta:
        steps = min(steps, 1)
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


def _pgd_steps(inst, x0, lr, steps, fixed, delta, epsilon, nthreads):
    """Algorithm 1 iteration by iteration (gradient, projected step, exact count),
    for the stopping rules that need the point of every iteration."""
    x = np.array(x0, dtype=np.float64, copy=True)
    B = x.shape[1]
    masks = None
    if fixed is not None:
        masks = np.zeros(x.shape, dtype=bool)
        f = np.asarray(fixed)
        if f.ndim == 1:
            masks[:] = f.astype(bool)[:, None]
        else:
            for cols, row in _slices(f, B):
                masks[:, cols] = np.asarray(row, dtype=bool)[:, None]
    unsat = unsat_count(inst, x)
    done = (unsat == 0).astype(np.uint8)
    first = np.where(unsat == 0, 0, -1).astype(np.int32)
    for t in range(1, steps + 1):
        if done.all():
            break
        g = eval(inst, x, grad=True, nthreads=nthreads)["grad"]
        xn = np.clip(x - lr * g, -1.0, 1.0)
        hold = done.astype(bool)[None, :] if masks is None else (masks | done.astype(bool)[None, :])
        xn = np.where(hold, x, xn)
        move = np.max(np.abs(xn - x), axis=0) if x.shape[0] else np.zeros(B)
        x = xn
        unsat = unsat_count(inst, x)
        newly = (done == 0) & (unsat == 0)
        first[newly] = t
        done[newly] = 1
        if delta > 0 and lr < delta:
            done[done == 0] = 2
        done[(done == 0) & (move < epsilon)] = 2
    obj = eval(inst, x, grad=False, nthreads=nthreads)["obj"]
    return {"x": x, "unsat": unsat, "first_sat": first, "obj": obj, "done": done}


def pgd_momentum(inst, x0, lr, mu, steps, fixed=None, v0=None, nthreads=None):
    """Projected gradient descent with heavy-ball momentum, FP64: per restart,
    v_t = mu v_(t-1) + grad F(x_(t-1)) and x_t = clip(x_(t-1) - lr v_t, -1, 1),
    with v_0 = ``v0`` (zero by default).  As in Algorithm 1 the point is rounded
    and counted after every step, and a restart that verifies stops there (its x
    and v no longer change); fixed variables (Sec. 3.4) keep x and v.  With
    mu = 0 this is Algorithm 1 with constant step length.

    Returns x, v, unsat, first_sat (-1: never verified; 0: the start point does),
    done (1 verified) and the objective at the final point."""
    x = np.array(x0, dtype=np.float64, copy=True)
    n, B = x.shape
    v = np.zeros((n, B)) if v0 is None else np.array(v0, dtype=np.float64, copy=True)
    held_fixed = fixed_columns(fixed, n, B)
    unsat = unsat_count(inst, x)
    done = (unsat == 0).astype(np.uint8)
    first = np.where(unsat == 0, 0, -1).astype(np.int32)
    for t in range(1, steps + 1):
        if done.all():
            break
        g = eval(inst, x, grad=True, nthreads=nthreads)["grad"]
        hold = held_fixed | done.astype(bool)[None, :]
        vn = mu * v + g
        xn = np.clip(x - lr * vn, -1.0, 1.0)
        v = np.where(hold, v, vn)
        x = np.where(hold, x, xn)
        unsat = unsat_count(inst, x)
        newly = (done == 0) & (unsat == 0)
        first[newly] = t
        done[newly] = 1
    obj = eval(inst, x, grad=False, nthreads=nthreads)["obj"]
    return {"x": x, "v": v, "unsat": unsat, "first_sat": first, "done": done, "obj": obj}


def unsat_count(inst, x):
    """unsat_count of Algorithm 1 on FP64 points (n, B): variable v True where
    x[v] < 0; a literal is true when its variable's truth differs from its sign."""
    n, C, con_off, lits, types, params, _ = _arrays(inst)
    tv = np.asarray(x, dtype=np.float64) < 0.0
    out = np.zeros(tv.shape[1], dtype=np.int32)
    for c in range(C):
        ls = lits[con_off[c]:con_off[c + 1]]
        t = np.zeros(tv.shape[1], dtype=np.int64)
        for l in ls:
            t += tv[abs(int(l)) - 1] ^ (l < 0)
        ok = np.array([sat(types[c], len(ls), params[c], tt) for tt in range(len(ls) + 1)])
        out += ~ok[t]
    return out


def line_search_step(inst, x, search, fixed=None, done=None, nthreads=None):
    """One iteration of Algorithm 1 with lineSearch as backtracking, FP64.

    search = (s, beta, c, T).  Per restart: f0 = F(x), g = grad F(x); trial j
    takes eta_j = s * beta^j and xt = clip(x - eta_j g, -1, 1) with the fixed
    variables held, and the first trial with F(xt) <= f0 + c * <g, xt - x> is
    taken; when none is, eta = 0.  Restarts with done != 0 keep eta = 0 and x.

    Returns x (the new point), eta (B,), f0 (B,), g (n, B), and for every trial
    (whether or not the restart had already decided) eta_trials (T,) and
    margin (T, B) = f0 + c * <g, xt - x> - F(xt), so a caller can see how close
    each decision was."""
    s_max, beta, c, T = float(search[0]), float(search[1]), float(search[2]), int(search[3])
    x = np.asarray(x, dtype=np.float64)
    n, B = x.shape
    held = fixed_columns(fixed, n, B)
    r0 = eval(inst, x, grad=True, nthreads=nthreads)
    f0, g = r0["obj"], r0["grad"]
    gm = np.where(held, 0.0, g)
    eta = np.zeros(B)
    decided = np.zeros(B, dtype=bool) if done is None else np.asarray(done).reshape(B) != 0
    etas, margins = [], []
    e = s_max
    for j in range(T):
        xt = np.where(held, x, np.clip(x - e * g, -1.0, 1.0))
        dot = np.sum(gm * (xt - x), axis=0)
        ft = eval(inst, xt, grad=False, nthreads=nthreads)["obj"]
        m = f0 + c * dot - ft
        take = ~decided & (m >= 0.0)
        eta[take] = e
        decided |= take
        etas.append(e)
        margins.append(m)
        e *= beta
    x_new = np.where(held, x, np.clip(x - eta[None, :] * g, -1.0, 1.0))
    if done is not None:
        x_new[:, np.asarray(done).reshape(B) != 0] = x[:, np.asarray(done).reshape(B) != 0]
    return {"x": x_new, "eta": eta, "f0": f0, "g": g, "eta_trials": np.array(etas),
            "margin": np.array(margins)}


def pgd_search(inst, x0, search, steps, fixed=None, delta=0.0, nthreads=None, epsilon=0.0):
    """Algorithm 1 with the backtracking lineSearch, FP64: at most ``steps``
    iterations; a restart stops when its point verifies (unsat_count = 0) or,
    with ``delta`` > 0, when its step length falls below delta, or, with
    ``epsilon`` > 0, when its new point lies within epsilon of the previous one
    in every variable."""
    x = np.array(x0, dtype=np.float64, copy=True)
    B = x.shape[1]
    unsat = unsat_count(inst, x)
    done = (unsat == 0).astype(np.uint8)
    first = np.where(unsat == 0, 0, -1).astype(np.int32)
    for t in range(1, steps + 1):
        if done.all():
            break
        r = line_search_step(inst, x, search, fixed=fixed, done=done, nthreads=nthreads)
        move = np.max(np.abs(r["x"] - x), axis=0) if x.shape[0] else np.zeros(B)
        x = r["x"]
        unsat = unsat_count(inst, x)
        newly = (done == 0) & (unsat == 0)
        first[newly] = t
        done[newly] = 1
        if delta > 0:
            done[(done == 0) & (r["eta"] < delta)] = 2
        if epsilon > 0:
            done[(done == 0) & (move < epsilon)] = 2
    return {"x": x, "unsat": unsat, "done": done, "first_sat": first}
