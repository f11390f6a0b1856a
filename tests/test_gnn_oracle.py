"""Pins for the FP64 reference of the learned-initialisation network (CPU only):
its gradient against central finite differences of its own loss (FP64, without
BF16 rounding, where the network is smooth almost everywhere), the BF16 rounding
helper against exactly representable values, and the features against their
definition on a hand-built instance."""
import numpy as np

from oracle import gnn as G
from paper_2606_06641_amd import workloads as W


def small_instance(seed=0):
    rng = np.random.default_rng(seed)
    return W.random_instance(rng, n=14, count=18, k_lo=1, k_hi=6)


def test_gradient_matches_finite_differences():
    inst = small_instance()
    R = 2
    _, total = G.layout(R)
    rng = np.random.default_rng(1)
    flat = rng.normal(0, 0.3, size=total)
    x0 = rng.uniform(-1, 1, size=(inst.n, 3))
    target = rng.integers(0, 2, size=inst.n)
    loss, grad, _ = G.loss_and_grad(flat, inst, x0, target, R=R, bf16_ops=False)
    idx = rng.choice(total, size=120, replace=False)
    h = 1e-6
    bad = 0
    for i in idx:
        e = np.zeros(total)
        e[i] = h
        lp, _, _ = G.loss_and_grad(flat + e, inst, x0, target, R=R, bf16_ops=False)
        lm, _, _ = G.loss_and_grad(flat - e, inst, x0, target, R=R, bf16_ops=False)
        fd = (lp - lm) / (2 * h)
        if abs(fd - grad[i]) > 1e-6 * max(1.0, abs(fd)) + 1e-9:
            bad += 1
    assert bad == 0
    # every parameter group receives gradient
    lay, _ = G.layout(R)
    for name, (o, shp) in lay.items():
        assert np.any(grad[o:o + int(np.prod(shp))] != 0), name


def test_bf16_rounding():
    vals = np.array([1.0, -2.5, 3.0, 0.0, 1.0 + 2 ** -7, 1.0 + 2 ** -8, 1.0 + 3 * 2 ** -9, 65504.0])
    out = G.bf16(vals)
    # exactly representable values are unchanged; halfway cases go to even
    assert out[0] == 1.0 and out[1] == -2.5 and out[2] == 3.0 and out[3] == 0.0
    assert out[4] == 1.0 + 2 ** -7
    assert out[5] == 1.0                      # halfway between 1 and 1+2^-7: even (1.0)
    assert out[6] == 1.0 + 2 ** -7            # 1.5 ulp rounds up
    assert out[7] == 65536.0


def test_features_definition():
    inst = W.Instance(n=3, con_off=np.array([0, 2, 5]), lits=np.array([1, -2, 1, 2, 3], np.int32),
                      types=np.array([W.OR, W.CARD_GE], np.int32), params=np.array([0, 2], np.int32))
    fc, fv = G.features(inst)
    assert fc[0, 0] == 1 and fc[1, 3] == 1
    assert np.isclose(fc[1, 8], np.log2(4) / 10) and np.isclose(fc[1, 9], 2 / 4)
    assert np.all(fc[:, 10] == 1) and np.all(fc[:, 11] == 1)
    # variable 1: two positive occurrences; variable 2: one negative, one positive; variable 3: one positive
    assert np.isclose(fv[0, 1], 1.0) and np.isclose(fv[1, 1], 0.0) and np.isclose(fv[2, 1], 1.0)
    assert np.isclose(fv[0, 0], np.log2(3) / 10)


def _dense_forward(flat, inst, x0, R):
    """The network written with dense incidence matrices instead of scatter-adds."""
    p = G.unpack(np.asarray(flat, np.float64), R)
    fc, fv = G.features(inst)
    n, C = int(inst.n), len(inst.types)
    Ac = np.zeros((C, n))                 # Ac[c, v] = sum of signs of v in c, / k_c
    Av = np.zeros((n, C))                 # Av[v, c] = sum of signs of v in c, / deg_v
    off = np.asarray(inst.con_off)
    deg = np.zeros(n)
    for c in range(C):
        for l in inst.lits[off[c]:off[c + 1]]:
            v = abs(int(l)) - 1
            Ac[c, v] += np.sign(l) / (off[c + 1] - off[c])
            Av[v, c] += np.sign(l)
            deg[v] += 1
    Av /= np.maximum(deg, 1)[:, None]
    relu = lambda a: np.maximum(a, 0)
    hv = relu(fv @ p["Wv0"] + p["bv0"])
    hc = relu(fc @ p["Wc0"] + p["bc0"])
    for r in range(R):
        hc = relu(np.hstack([hc, Ac @ hv]) @ p["U"][r] + p["bu"][r])
        hv = relu(np.hstack([hv, Av @ hc]) @ p["V"][r] + p["bv"][r])
    P = hv @ p["Wh"] + p["bh"]
    z = relu(P[:, None, :] + np.asarray(x0)[:, :, None] * p["wx"]) @ p["wo"] + p["bo"][0]
    return np.tanh(z)


def test_forward_matches_dense_incidence_form():
    inst = small_instance(3)
    R = 3
    _, total = G.layout(R)
    rng = np.random.default_rng(5)
    flat = rng.normal(0, 0.3, size=total)
    x0 = rng.uniform(-1, 1, size=(inst.n, 4))
    got, _ = G.forward(flat, inst, x0, R=R, bf16_ops=False)
    assert np.allclose(got, _dense_forward(flat, inst, x0, R), rtol=1e-12, atol=1e-12)


def test_variable_relabelling_permutes_outputs():
    inst = small_instance(4)
    R = 2
    _, total = G.layout(R)
    rng = np.random.default_rng(6)
    flat = rng.normal(0, 0.3, size=total)
    x0 = rng.uniform(-1, 1, size=(inst.n, 3))
    perm = rng.permutation(inst.n)                 # new index of old variable v is perm[v]
    lits = np.asarray(inst.lits)
    relab = (np.sign(lits) * (perm[np.abs(lits) - 1] + 1)).astype(np.int32)
    inst2 = W.Instance(n=inst.n, con_off=inst.con_off, lits=relab, types=inst.types, params=inst.params)
    x2 = np.empty_like(x0)
    x2[perm] = x0
    a, _ = G.forward(flat, inst, x0, R=R, bf16_ops=False)
    b, _ = G.forward(flat, inst2, x2, R=R, bf16_ops=False)
    assert np.allclose(b[perm], a, rtol=1e-12, atol=1e-12)
