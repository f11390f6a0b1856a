"""FP64 NumPy reference of the learned-initialisation network (test infrastructure).

Only the tests use it.  It shares no code with the GPU library: features,
message passing, head, loss and every gradient are written out here from the
network's definition:

  hv = relu(fv Wv0 + bv0),  hc = relu(fc Wc0 + bc0)
  for r = 1..R:  ac_c = (1/k_c) sum_{e in c} s_e hv_{v(e)}
                 hc   = relu([hc, ac] U_r + bu_r)
                 av_v = (1/deg_v) sum_{e of v} s_e hc_{c(e)}
                 hv   = relu([hv, av] V_r + bv_r)
  P = hv Wh + bh;  per (v, b): u = relu(P_v + x0_{v,b} wx), z = u.wo + bo, xhat = tanh z
  loss = mean_{v,b} [ y_v softplus(2z) + (1-y_v) softplus(-2z) ]   (y_v = 1: True)

With ``bf16=True`` the operands of every dense layer are rounded to BF16
(round to nearest even, via FP32) the way the GPU's matrix cores consume them;
accumulation stays FP64.  With ``bf16=False`` the network is a smooth function
of its parameters almost everywhere (checked against finite differences).
``acc`` (default FP64) is the precision every array, sum and elementwise step
is carried in; ``acc=np.float32`` evaluates the same definition with FP32
accumulation, as the device's layers accumulate, which the tests use to size
their tolerance (the rounding of FP32 sums moves values across BF16 rounding
boundaries and relu thresholds).

Flat parameter layout (the device layout): Wv0 [16][64], bv0 [64], Wc0 [16][64],
bc0 [64], U [R][128][64], bu [R][64], V [R][128][64], bv [R][64], Wh [64][64],
bh [64], wx [64], wo [64], bo [1].
"""
import numpy as np

H = 64
F = 16


def layout(R):
    sizes = [("Wv0", (F, H)), ("bv0", (H,)), ("Wc0", (F, H)), ("bc0", (H,)),
             ("U", (R, 2 * H, H)), ("bu", (R, H)), ("V", (R, 2 * H, H)), ("bv", (R, H)),
             ("Wh", (H, H)), ("bh", (H,)), ("wx", (H,)), ("wo", (H,)), ("bo", (1,))]
    out, o = {}, 0
    for name, shp in sizes:
        size = int(np.prod(shp))
        out[name] = (o, shp)
        o += size
    return out, o


def unpack(flat, R):
    lay, total = layout(R)
    assert flat.size == total
    return {k: np.asarray(flat[o:o + int(np.prod(s))], np.float64).reshape(s) for k, (o, s) in lay.items()}


def pack(p, R):
    lay, total = layout(R)
    flat = np.zeros(total)
    for k, (o, s) in lay.items():
        flat[o:o + int(np.prod(s))] = p[k].reshape(-1)
    return flat


def bf16(a):
    """Round to BF16 (nearest even) through FP32, returned as float64."""
    f = np.asarray(a, np.float64).astype(np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    nan = np.isnan(f)
    u = (u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000
    r = u.astype(np.uint32).view(np.float32).astype(np.float64)
    r[nan] = np.nan
    return r


def features(inst):
    """fc [C][16], fv [n][16] as described in the module docstring of the device code:
    constraint: one-hot type, log2(k+1)/10, K/(k+1) (CARD/EK) or parity (XOR), weight, 1;
    variable: log2(1+deg)/10, (positive - negative occurrences)/deg, 1."""
    n, C = int(inst.n), len(inst.types)
    lens = np.diff(np.asarray(inst.con_off))
    w = np.ones(C) if getattr(inst, "weights", None) is None else np.asarray(inst.weights, np.float64)
    fc = np.zeros((C, F))
    for c in range(C):
        t, k = int(inst.types[c]), int(lens[c])
        fc[c, t] = 1.0
        fc[c, 8] = np.log2(k + 1.0) / 10.0
        if t in (3, 4, 7):
            fc[c, 9] = inst.params[c] / (k + 1.0)
        elif t == 1:
            fc[c, 9] = inst.params[c] & 1
        fc[c, 10] = w[c]
        fc[c, 11] = 1.0
    lits = np.asarray(inst.lits)
    v = np.abs(lits) - 1
    pos = np.bincount(v[lits > 0], minlength=n).astype(np.float64)
    neg = np.bincount(v[lits < 0], minlength=n).astype(np.float64)
    deg = pos + neg
    fv = np.zeros((n, F))
    fv[:, 0] = np.log2(1.0 + deg) / 10.0
    fv[:, 1] = np.where(deg > 0, (pos - neg) / np.maximum(deg, 1), 0.0)
    fv[:, 2] = 1.0
    return fc.astype(np.float32).astype(np.float64), fv.astype(np.float32).astype(np.float64)


def _graph(inst):
    n, C = int(inst.n), len(inst.types)
    con_off = np.asarray(inst.con_off, np.int64)
    lits = np.asarray(inst.lits)
    e_con = np.repeat(np.arange(C), np.diff(con_off))
    e_var = np.abs(lits) - 1
    e_sgn = np.where(lits > 0, 1.0, -1.0)
    k = np.diff(con_off).astype(np.float64)
    deg = np.bincount(e_var, minlength=n).astype(np.float64)
    return e_con, e_var, e_sgn, k, np.maximum(deg, 1.0)


def _agg_c(h_v, g):
    e_con, e_var, e_sgn, k, deg = g
    out = np.zeros((len(k), h_v.shape[1]), h_v.dtype)
    np.add.at(out, e_con, e_sgn[:, None] * h_v[e_var])
    return out / k[:, None]


def _agg_v(h_c, g, n):
    e_con, e_var, e_sgn, k, deg = g
    out = np.zeros((n, h_c.shape[1]), h_c.dtype)
    np.add.at(out, e_var, e_sgn[:, None] * h_c[e_con])
    return out / deg[:, None]


def _agg_c_T(d_ac, g, n):       # adjoint of _agg_c
    e_con, e_var, e_sgn, k, deg = g
    out = np.zeros((n, d_ac.shape[1]), d_ac.dtype)
    np.add.at(out, e_var, e_sgn[:, None] * (d_ac / k[:, None])[e_con])
    return out


def _agg_v_T(d_av, g):          # adjoint of _agg_v
    e_con, e_var, e_sgn, k, deg = g
    out = np.zeros((len(k), d_av.shape[1]), d_av.dtype)
    np.add.at(out, e_con, e_sgn[:, None] * (d_av / deg[:, None])[e_var])
    return out


def _mm(a, b, q):
    if q:
        return bf16(a).astype(a.dtype) @ bf16(b).astype(b.dtype)
    return a @ b


def forward(flat, inst, x0, R=3, bf16_ops=True, acc=np.float64):
    p = {k: v.astype(acc) for k, v in unpack(np.asarray(flat, np.float64), R).items()}
    fc, fv = (a.astype(acc) for a in features(inst))
    g = tuple(a.astype(acc) if a.dtype.kind == "f" else a for a in _graph(inst))
    n = int(inst.n)
    q = bf16_ops
    cache = {"xv": [], "xc": [], "hv": [], "hc": []}
    hv = np.maximum(_mm(fv, p["Wv0"], q) + p["bv0"], 0)
    hc = np.maximum(_mm(fc, p["Wc0"], q) + p["bc0"], 0)
    cache["hv0"], cache["hc0"] = hv, hc
    for r in range(R):
        ac = _agg_c(hv, g)
        xc = np.concatenate([hc, ac], axis=1)
        hc = np.maximum(_mm(xc, p["U"][r], q) + p["bu"][r], 0)
        av = _agg_v(hc, g, n)
        xv = np.concatenate([hv, av], axis=1)
        hv = np.maximum(_mm(xv, p["V"][r], q) + p["bv"][r], 0)
        cache["xc"].append(xc); cache["xv"].append(xv); cache["hc"].append(hc); cache["hv"].append(hv)
    P = _mm(hv, p["Wh"], q) + p["bh"]
    x0 = np.asarray(x0, np.float64).astype(acc)
    pre = P[:, None, :] + x0[:, :, None] * p["wx"][None, None, :]      # (n, B, H)
    u = np.maximum(pre, 0)
    z = u @ p["wo"] + p["bo"][0]
    cache.update(P=P, pre=pre, u=u, z=z, g=g, fc=fc, fv=fv, p=p)
    return np.tanh(z), cache


def softplus(t):
    return np.where(t > 0, t + np.log1p(np.exp(-np.abs(t))), np.log1p(np.exp(t)))


def loss_and_grad(flat, inst, x0, target, R=3, bf16_ops=True, acc=np.float64):
    """Mean BCE and its gradient with respect to the flat parameters."""
    xhat, c = forward(flat, inst, x0, R, bf16_ops, acc)
    p, g, n, q = c["p"], c["g"], int(inst.n), bf16_ops
    y = np.asarray(target, np.float64).astype(acc)[:, None]
    z = c["z"]
    count = z.size
    loss = float(np.sum(y * softplus(2 * z) + (1 - y) * softplus(-2 * z)) / count)
    dz = 2.0 * (1.0 / (1.0 + np.exp(-2 * z)) - 1.0 + y) / count          # (n, B)
    gr = {k: np.zeros_like(v) for k, v in p.items()}
    du = dz[:, :, None] * p["wo"][None, None, :] * (c["pre"] > 0)         # (n, B, H)
    gr["wo"] = np.einsum("vb,vbj->j", dz, c["u"])
    gr["bo"] = np.array([dz.sum()])
    gr["wx"] = np.einsum("vbj,vb->j", du, np.asarray(x0, np.float64).astype(acc))
    dP = du.sum(axis=1)                                                    # (n, H)
    hv = c["hv"][-1]
    gr["Wh"] = _mm(hv.T, dP, q)
    gr["bh"] = dP.sum(axis=0)
    dhv = _mm(dP, p["Wh"].T, q)
    dhc = np.zeros_like(c["hc"][-1])
    for r in reversed(range(R)):
        hv_out, hc_out, xv, xc = c["hv"][r], c["hc"][r], c["xv"][r], c["xc"][r]
        dpre = dhv * (hv_out > 0)
        gr["V"][r] = _mm(xv.T, dpre, q)
        gr["bv"][r] = dpre.sum(axis=0)
        dxv = _mm(dpre, p["V"][r].T, q)
        dhv_prev, dav = dxv[:, :H], dxv[:, H:]
        dhc = dhc + _agg_v_T(dav, g)
        dpre = dhc * (hc_out > 0)
        gr["U"][r] = _mm(xc.T, dpre, q)
        gr["bu"][r] = dpre.sum(axis=0)
        dxc = _mm(dpre, p["U"][r].T, q)
        dhc_prev, dac = dxc[:, :H], dxc[:, H:]
        dhv = dhv_prev + _agg_c_T(dac, g, n)
        dhc = dhc_prev
    dpre = dhv * (c["hv0"] > 0)
    gr["Wv0"] = _mm(c["fv"].T, dpre, q)
    gr["bv0"] = dpre.sum(axis=0)
    dpre = dhc * (c["hc0"] > 0)
    gr["Wc0"] = _mm(c["fc"].T, dpre, q)
    gr["bc0"] = dpre.sum(axis=0)
    return loss, pack({k: v.astype(np.float64) for k, v in gr.items()}, R), xhat.astype(np.float64)
