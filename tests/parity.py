"""Helpers for GPU-vs-oracle parity (tolerances per length bucket).

Both FE and the gradient can be arbitrarily close to 0 (a satisfied long
cardinality constraint has FE = -1 + 1e-30 and a gradient of that order), so a
per-element relative error is meaningless; the bars are relative to the largest
oracle value of the bucket, plus a relative-L2 bar over the bucket:

  FE      : max |FE_gpu - FE_orc|        <= max(1e-4 * max |FE_orc|, R_FE) (per bucket)
  adjoint : max |adj_gpu - adj_orc|      <= max(1e-4 * max |adj_orc|, R) (per bucket)
            ||adj_gpu - adj_orc||_2      <= max(1e-4 * ||adj_orc||_2, R * sqrt(count))
  obj     : max |F_gpu - F_orc|          <= 1e-4 * max_b sum_c |w_c FE_orc,c(b)|
  grad    : |grad_gpu - grad_orc|        <= max(1e-4 * max |grad_orc|, R_v)  (every entry)
            ||grad_gpu - grad_orc||_2    <= max(1e-4 * ||grad_orc||_2, ||R||_2)

R_FE = 4 * 2^-24 * sqrt(k_max) is the FP32 resolution of FE itself (a sum of
floor(k/2) + 1 root terms bounded by 1 whose total can be 1e-15, e.g. a long XOR
at a random point); it binds only when every FE of the bucket is that small.
R is the FP32 resolution of an adjoint: each one is a sum over the floor(k/2)
complex roots of terms bounded by the constraint weight |w|, whose exact total
can be 1e-30 (a constraint deep inside its satisfied region); FP32 rounds each
root's term at 2^-24 relative, so the sum carries an absolute error of order
2^-24 * sqrt(k) * |w| whatever its value.  R = 4 * 2^-24 * sqrt(k_max) * max|w|
over the bucket; it binds only in buckets whose oracle adjoints all lie below
about 1e-2 |w| (every constraint saturated), elsewhere the relative bar is the
larger one.  A variable's gradient sums its occurrences' adjoints, so its
floor R_v is the sum of theirs.  The objective sums terms w_c FE_c of either
sign, so its bar is relative to the sum of their magnitudes (the sum itself can
cancel to 0).  An array whose oracle values are all exactly zero is held to
ABS_FLOOR.
"""
import numpy as np
import torch

REL_TOL = 1e-4
ABS_FLOOR = 1e-6
EPS32 = 2.0 ** -24


def adj_resolution(k_max, w_max):
    """FP32 resolution floor R of one adjoint (see the module docstring)."""
    return 4.0 * EPS32 * np.sqrt(max(k_max, 1)) * max(w_max, 1e-30)


def to_dev(a, device=0):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).to(f"cuda:{device}")


def gpu_eval(dinst, x32):
    x = to_dev(x32)
    out = dinst.eval(x, obj=True, grad=True, fe=True, adj=True)
    torch.cuda.synchronize()
    return {k: v.cpu().numpy().astype(np.float64) for k, v in out.items()}


def bucket_of_literals(dinst):
    """Bucket index of every input literal (input order)."""
    smap = dinst.slot_map()
    out = np.empty(dinst.n_lits, dtype=np.int64)
    for i, b in enumerate(dinst.buckets()):
        out[smap[b.slot0:b.slot0 + b.n_lits]] = i
    return out


def bucket_of_constraints(inst, lit_bucket):
    return lit_bucket[np.asarray(inst.con_off[:-1], dtype=np.int64)]


def rel_max(got, want):
    """(max |got - want|, the bar it is held to, the error relative to max |want|
    or, when want is all zero, absolute)."""
    if got.size == 0:
        return 0.0, ABS_FLOOR, 0.0
    err = float(np.max(np.abs(got - want)))
    scale = float(np.max(np.abs(want)))
    if scale > 0:
        return err, REL_TOL * scale, err / scale
    return err, ABS_FLOOR, err


def rel_l2(got, want):
    """(||got - want||_2, the bar it is held to, the relative error)."""
    if got.size == 0:
        return 0.0, ABS_FLOOR, 0.0
    err = float(np.linalg.norm(got - want))
    ref = float(np.linalg.norm(want))
    if ref > 0:
        return err, REL_TOL * ref, err / ref
    return err, ABS_FLOOR * np.sqrt(got.size), err / np.sqrt(got.size)


def check_adjoints(adj_gpu, adj_orc, lit_bucket, buckets, label="", lit_w=None):
    """Per bucket: the adjoint bars (lit_w: |weight| of each literal's
    constraint, default 1).  Returns [(max err / max|orc|, L2 err / ||orc||)]."""
    out = []
    for i, b in enumerate(buckets):
        lm = lit_bucket == i
        g, w = adj_gpu[lm], adj_orc[lm]
        res = adj_resolution(b.k_hi, float(np.max(lit_w[lm])) if lit_w is not None and lm.any() else 1.0)
        e, bar, r = rel_max(g, w)
        assert e <= max(bar, res), (label, "adj max", b, e, bar, res)
        e2, bar2, r2 = rel_l2(g, w)
        assert e2 <= max(bar2, res * np.sqrt(max(g.size, 1))), (label, "adj l2", b, e2, bar2, res)
        out.append((r, r2))
    return out


def literal_weights(inst):
    """|w| of each literal's constraint (input literal order)."""
    w = np.ones(inst.n_cons) if getattr(inst, "weights", None) is None else np.asarray(inst.weights, np.float64)
    return np.repeat(np.abs(w), np.diff(np.asarray(inst.con_off)))


def compare(inst, dinst, gpu, orc, label=""):
    """Assert parity per bucket; return a per-bucket error table with errors
    relative to the bucket's largest oracle value (FE, adjoint) and its norm."""
    lb = bucket_of_literals(dinst)
    cb = bucket_of_constraints(inst, lb)
    buckets = dinst.buckets()
    adj_rel = check_adjoints(gpu["adj"], orc["adj"], lb, buckets, label, literal_weights(inst))
    rows = []
    for i, b in enumerate(buckets):
        cm = cb == i
        e, bar, r = rel_max(gpu["fe"][cm], orc["fe"][cm])
        assert e <= max(bar, 4.0 * EPS32 * np.sqrt(b.k_hi)), (label, "FE", b, e, bar)
        rows.append((b.k_lo, b.k_hi, b.lanes_per_restart, b.lits_per_lane, r) + adj_rel[i])
    check_obj(inst, gpu["obj"], orc["obj"], orc.get("fe"), label)
    check_grad(gpu["grad"], orc["grad"], label, inst)
    return rows


def check_obj(inst, got, want, fe_orc=None, label=""):
    """|F_gpu - F_orc| <= 1e-4 * max_b sum_c |w_c FE_c(b)| (sum_c |w_c| without fe)."""
    w = np.ones(inst.n_cons) if getattr(inst, "weights", None) is None else np.asarray(inst.weights, np.float64)
    if fe_orc is not None and fe_orc.size:
        scale = float(np.max((np.abs(w)[:, None] * np.abs(fe_orc)).sum(axis=0)))
    else:
        scale = float(np.sum(np.abs(w)))
    e = float(np.max(np.abs(got - want))) if got.size else 0.0
    bar = REL_TOL * scale if scale > 0 else ABS_FLOOR
    assert e <= bar, (label, "obj", e, bar)
    return e / max(scale, 1e-300)


def grad_floor(inst):
    """R_v per variable: the sum over its occurrences of the adjoint floor."""
    lens = np.diff(np.asarray(inst.con_off))
    lit_k = np.repeat(lens, lens)
    lw = literal_weights(inst)
    per_lit = 4.0 * EPS32 * np.sqrt(lit_k) * lw
    out = np.zeros(inst.n)
    np.add.at(out, np.abs(np.asarray(inst.lits)) - 1, per_lit)
    return out


def check_grad(got, want, label="", inst=None):
    """The gradient bars (with inst: the per-variable FP32 floor R_v)."""
    e, bar, r = rel_max(got, want)
    floor = grad_floor(inst)[:, None] if inst is not None else np.zeros((got.shape[0], 1))
    over = np.abs(got - want) > np.maximum(bar, floor)
    assert not over.any(), (label, "grad max", e, bar, int(over.sum()))
    e2, bar2, r2 = rel_l2(got, want)
    fl2 = float(np.linalg.norm(np.broadcast_to(floor, got.shape))) if inst is not None else 0.0
    assert e2 <= max(bar2, fl2), (label, "grad l2", e2, bar2, fl2)
    return r, r2


def format_rows(rows):
    lines = ["k_lo k_hi  J  S  max|dFE|/max|FE|  max|dadj|/max|adj|  rel-L2(adj)"]
    for r in rows:
        lines.append("%4d %4d %2d %2d  %14.2e  %18.2e  %11.2e" % r)
    return "\n".join(lines)
