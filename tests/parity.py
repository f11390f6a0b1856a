"""Helpers for GPU-vs-oracle parity (tolerances per length bucket).

Both FE and the gradient can be arbitrarily close to 0 (a satisfied long
cardinality constraint has FE = -1 + 1e-30 and a gradient of that order), so a
per-element relative error is meaningless; the bars are relative to the largest
oracle value of the bucket, plus a relative-L2 bar over the bucket:

  FE      : max |FE_gpu - FE_orc|        <= 1e-4 * max |FE_orc|         (per bucket)
  adjoint : max |adj_gpu - adj_orc|      <= 1e-4 * max |adj_orc|        (per bucket)
            ||adj_gpu - adj_orc||_2      <= 1e-4 * ||adj_orc||_2        (per bucket)
  obj     : max |F_gpu - F_orc|          <= 1e-4 * max |F_orc|
  grad    : max |grad_gpu - grad_orc|    <= 1e-4 * max |grad_orc|
            ||grad_gpu - grad_orc||_2    <= 1e-4 * ||grad_orc||_2

A bucket (or array) whose oracle values are all exactly zero is held to the
absolute bar ABS_FLOOR instead (a constant constraint has FE = -1 exactly and a
zero gradient; the kernels must return zeros to within FP32 rounding of the
table entries).
"""
import numpy as np
import torch

REL_TOL = 1e-4
ABS_FLOOR = 1e-6


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


def check_adjoints(adj_gpu, adj_orc, lit_bucket, buckets, label=""):
    """Per bucket: the adjoint bars.  Returns [(max err / max|orc|, L2 err / ||orc||)]."""
    out = []
    for i, b in enumerate(buckets):
        lm = lit_bucket == i
        g, w = adj_gpu[lm], adj_orc[lm]
        e, bar, r = rel_max(g, w)
        assert e <= bar, (label, "adj max", b, e, bar)
        e2, bar2, r2 = rel_l2(g, w)
        assert e2 <= bar2, (label, "adj l2", b, e2, bar2)
        out.append((r, r2))
    return out


def compare(inst, dinst, gpu, orc, label=""):
    """Assert parity per bucket; return a per-bucket error table with errors
    relative to the bucket's largest oracle value (FE, adjoint) and its norm."""
    lb = bucket_of_literals(dinst)
    cb = bucket_of_constraints(inst, lb)
    buckets = dinst.buckets()
    adj_rel = check_adjoints(gpu["adj"], orc["adj"], lb, buckets, label)
    rows = []
    for i, b in enumerate(buckets):
        cm = cb == i
        e, bar, r = rel_max(gpu["fe"][cm], orc["fe"][cm])
        assert e <= bar, (label, "FE", b, e, bar)
        rows.append((b.k_lo, b.k_hi, b.lanes_per_restart, b.lits_per_lane, r) + adj_rel[i])
    e, bar, _ = rel_max(gpu["obj"], orc["obj"])
    assert e <= bar, (label, "obj", e, bar)
    check_grad(gpu["grad"], orc["grad"], label)
    return rows


def check_grad(got, want, label=""):
    e, bar, r = rel_max(got, want)
    assert e <= bar, (label, "grad max", e, bar)
    e2, bar2, r2 = rel_l2(got, want)
    assert e2 <= bar2, (label, "grad l2", e2, bar2)
    return r, r2


def format_rows(rows):
    lines = ["k_lo k_hi  J  S  max|dFE|/max|FE|  max|dadj|/max|adj|  rel-L2(adj)"]
    for r in rows:
        lines.append("%4d %4d %2d %2d  %14.2e  %18.2e  %11.2e" % r)
    return "\n".join(lines)
