"""Helpers for GPU-vs-oracle parity (tolerances per length bucket).

Tolerances, per bucket (FE and every per-literal adjoint lie in [-1, 1] times the
constraint weight, and both may be arbitrarily close to 0, so errors are taken
relative to that range, with a relative-L2 test on top):
  FE      : max |FE_gpu - FE_orc|                         <= 1e-4
  adjoint : max |adj_gpu - adj_orc|                       <= 1e-4 * max|w|
            ||adj_gpu - adj_orc||_2                       <= 1e-4 * ||adj_orc||_2 + 1e-6 * sqrt(count)
  obj     : |F_gpu - F_orc| per restart                   <= 1e-4 * sum_c |w_c|
  grad    : max |grad_gpu - grad_orc| over (v, b)         <= 1e-4 * max_v sum_{occ of v} |w|
"""
import numpy as np
import torch

FE_TOL = 1e-4
ADJ_TOL = 1e-4


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


def compare(inst, dinst, gpu, orc, label=""):
    """Assert parity per bucket; return a per-bucket error table."""
    w = np.ones(inst.n_cons) if inst.weights is None else np.asarray(inst.weights, np.float64)
    lb = bucket_of_literals(dinst)
    cb = bucket_of_constraints(inst, lb)
    lit_w = np.repeat(np.abs(w), np.diff(inst.con_off))
    rows = []
    for i, b in enumerate(dinst.buckets()):
        cm = cb == i
        lm = lb == i
        fe_err = np.max(np.abs(gpu["fe"][cm] - orc["fe"][cm])) if cm.any() else 0.0
        d = gpu["adj"][lm] - orc["adj"][lm]
        adj_max = np.max(np.abs(d)) if d.size else 0.0
        adj_l2 = np.linalg.norm(d)
        ref_l2 = np.linalg.norm(orc["adj"][lm])
        wmax = np.max(lit_w[lm]) if lm.any() else 1.0
        rows.append((b.k_lo, b.k_hi, b.lanes_per_restart, b.lits_per_lane, fe_err, adj_max,
                     adj_l2 / max(ref_l2, 1e-30)))
        assert fe_err <= FE_TOL, (label, "FE", b, fe_err)
        assert adj_max <= ADJ_TOL * wmax, (label, "adj max", b, adj_max)
        assert adj_l2 <= ADJ_TOL * ref_l2 + 1e-6 * np.sqrt(d.size), (label, "adj l2", b, adj_l2, ref_l2)
    obj_tol = FE_TOL * max(np.sum(np.abs(w)), 1.0)
    assert np.max(np.abs(gpu["obj"] - orc["obj"])) <= obj_tol, (label, "obj")
    deg_w = np.zeros(inst.n)
    np.add.at(deg_w, np.abs(inst.lits) - 1, lit_w)
    assert np.max(np.abs(gpu["grad"] - orc["grad"])) <= ADJ_TOL * max(deg_w.max(), 1.0), (label, "grad")
    return rows


def format_rows(rows):
    lines = ["k_lo k_hi  J  S   max|dFE|   max|dadj|  rel-L2(adj)"]
    for r in rows:
        lines.append("%4d %4d %2d %2d  %9.2e  %9.2e  %9.2e" % r)
    return "\n".join(lines)
