"""Pins for the FP64 CPU oracle (CPU only).

Each test checks the oracle against something other than itself: the paper's
worked examples (Appendix A truth tables), exact rational evaluation of Eq. (1)
and of the multilinear polynomial on all corners, closed forms, the binomial
special case, finite differences (exact for multilinear functions), invariants
and the planted witness.  A dropped term, a wrong sign or index, or a
transposed operand in the oracle fails at least one of them.
"""
import os
from fractions import Fraction
from math import comb

import numpy as np
import pytest

import oracle
import exact
from paper_2606_06641_amd import workloads as W

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "appendix_a_truth.txt")
ALL_TYPES = range(8)


def one_constraint(ctype, k, param, signs=None, n=None):
    n = n or k
    lits = np.arange(1, k + 1, dtype=np.int32)
    if signs is not None:
        lits = np.where(np.asarray(signs) < 0, -lits, lits).astype(np.int32)
    return W.Instance(n=n, con_off=np.array([0, k], dtype=np.int64), lits=lits,
                      types=np.array([ctype], dtype=np.int32),
                      params=np.array([param], dtype=np.int32))


def params_for(ctype, k):
    if ctype == W.XOR:
        return [0, 1]
    if ctype in (W.CARD_GE, W.CARD_LT, W.EK):
        return list(range(0, k + 2))
    return [0]


def fe_single(ctype, k, param, y):
    inst = one_constraint(ctype, k, param)
    x = np.asarray(y, dtype=np.float64).reshape(k, -1)
    return oracle.eval(inst, x, fe=True)["fe"][0]


# -- Appendix A worked examples -------------------------------------------------

def test_appendix_a_truth_tables():
    rows = 0
    with open(GOLDEN) as f:
        for line in f:
            line = line.split("|")[0].strip()
            if not line or line.startswith("#"):
                continue
            ctype, k, param, gs = line.split()
            ctype, k, param = int(ctype), int(k), int(param)
            want = [int(v) for v in gs.split(",")]
            assert len(want) == k + 1
            got = [-1 if oracle.sat(ctype, k, param, t) else 1 for t in range(k + 1)]
            assert got == want, line
            # and the oracle's FE at the corner with t true literals equals g(t)
            for t in range(k + 1):
                y = np.ones(k)
                y[:t] = -1.0
                assert fe_single(ctype, k, param, y)[0] == want[t]
            rows += 1
    assert rows == 11


# -- corners: FE is exactly the +-1 truth value -----------------------------------

@pytest.mark.parametrize("k", [1, 2, 3, 5, 8, 10])
def test_corners_exact(k):
    corners = np.array([[1 - 2 * ((m >> i) & 1) for m in range(1 << k)] for i in range(k)],
                       dtype=np.float64)               # (k, 2^k), -1 = True
    t = (corners < 0).sum(axis=0)
    for ctype in ALL_TYPES:
        for param in params_for(ctype, k):
            fe = fe_single(ctype, k, param, corners)
            want = np.array([exact.g(ctype, k, param, int(tt)) for tt in t], dtype=np.float64)
            assert np.array_equal(fe, want), (ctype, k, param)


# -- interior: exact multilinear polynomial (rational arithmetic) -----------------

@pytest.mark.parametrize("k", [1, 2, 3, 4, 6, 9])
def test_interior_matches_exact_multilinear(k):
    rng = np.random.default_rng(100 + k)
    pts = [[Fraction(int(rng.integers(-64, 65)), 64) for _ in range(k)] for _ in range(6)]
    x = np.array([[float(p[i]) for p in pts] for i in range(k)])
    for ctype in ALL_TYPES:
        for param in params_for(ctype, k):
            fe = fe_single(ctype, k, param, x)
            for j, p in enumerate(pts):
                want = float(exact.fe_by_corners(ctype, k, param, p))
                assert abs(fe[j] - want) <= 1e-14, (ctype, k, param, j)


@pytest.mark.parametrize("k", [1, 3, 5])
def test_interior_matches_eq1_fourier_coefficients(k):
    """Eq. (1) literally: coefficients by their definition, then sum_S f(S) prod y."""
    rng = np.random.default_rng(7 + k)
    pts = [[Fraction(int(rng.integers(-32, 33)), 32) for _ in range(k)] for _ in range(4)]
    x = np.array([[float(p[i]) for p in pts] for i in range(k)])
    for ctype in ALL_TYPES:
        for param in params_for(ctype, k):
            coef = exact.fourier_coefficients(ctype, k, param)
            fe = fe_single(ctype, k, param, x)
            for j, p in enumerate(pts):
                assert abs(fe[j] - float(exact.fe_by_coefficients(coef, p))) <= 1e-14


# -- closed forms at any length --------------------------------------------------

@pytest.mark.parametrize("k", [3, 17, 64, 200, 1024])
def test_closed_forms_long(k):
    rng = np.random.default_rng(k)
    y = rng.uniform(-1, 1, size=(k, 5))
    # keep products away from underflow for the long cases
    y[:, :2] = np.sign(y[:, :2]) * (1 - 1e-3 * rng.uniform(0, 1, size=(k, 2)))
    prod_plus = np.prod((1 + y) / 2, axis=0)
    prod_minus = np.prod((1 - y) / 2, axis=0)
    checks = {
        (W.OR, 0): -1 + 2 * prod_plus,
        (W.CARD_GE, k): 1 - 2 * prod_minus,             # AND of all literals
        (W.XOR, 1): np.prod(y, axis=0),
        (W.XOR, 0): -np.prod(y, axis=0),
        (W.NAE, 0): -1 + 2 * (prod_plus + prod_minus),
        (W.CARD_GE, 0): -np.ones(5),                    # trivially true
        (W.CARD_LT, 0): np.ones(5),                     # trivially false
    }
    for (ctype, param), want in checks.items():
        fe = fe_single(ctype, k, param, y)
        assert np.max(np.abs(fe - want)) <= 1e-12, (ctype, param)


@pytest.mark.parametrize("k", [5, 40, 120, 200])
def test_binomial_special_case(k):
    """All literals at the same dyadic value: FE = sum_t g(t) C(k,t) p^t (1-p)^(k-t)."""
    ys = [Fraction(-3, 4), Fraction(-1, 8), Fraction(1, 2), Fraction(15, 16)]
    for ctype in (W.CARD_GE, W.CARD_LT, W.EK, W.EO, W.AMO, W.NAE):
        for param in sorted({0, 1, k // 3, k // 2, k - 1, k}):
            x = np.array([[float(v) for v in ys]] * k)
            fe = fe_single(ctype, k, param, x)
            for j, yv in enumerate(ys):
                want = float(exact.fe_binomial(ctype, k, param, yv))
                assert abs(fe[j] - want) <= 1e-12, (ctype, k, param, yv)


@pytest.mark.parametrize("k", [1, 4, 33, 300])
def test_value_at_zero(k):
    x = np.zeros((k, 1))
    for ctype in ALL_TYPES:
        for param in sorted(set(params_for(ctype, k)) & {0, 1, 2, k // 2, k, k + 1}):
            want = float(exact.fe_at_zero(ctype, k, param))
            assert abs(fe_single(ctype, k, param, x)[0] - want) <= 1e-13


# -- gradient -----------------------------------------------------------------------

@pytest.mark.parametrize("k", [1, 2, 4, 7])
def test_gradient_exact_small(k):
    rng = np.random.default_rng(31 + k)
    pts = [[Fraction(int(rng.integers(-16, 17)), 16) for _ in range(k)] for _ in range(3)]
    x = np.array([[float(p[i]) for p in pts] for i in range(k)])
    signs = [(-1) ** i for i in range(k)]
    for ctype in ALL_TYPES:
        for param in params_for(ctype, k):
            inst = one_constraint(ctype, k, param, signs=signs)
            out = oracle.eval(inst, x, adj=True, grad=True)
            for j, p in enumerate(pts):
                y = [p[i] * signs[i] for i in range(k)]          # literal values
                dy = exact.grad_by_corners(ctype, k, param, y)
                for i in range(k):
                    want = float(dy[i]) * signs[i]              # dFE/dx_i
                    assert abs(out["adj"][i, j] - want) <= 1e-14
                    assert abs(out["grad"][i, j] - want) <= 1e-14


@pytest.mark.parametrize("k", [12, 96, 300])
def test_gradient_central_differences(k):
    """Central differences are exact for a function affine in each coordinate."""
    rng = np.random.default_rng(5 * k)
    signs = rng.choice([-1, 1], size=k)
    h = 1e-3
    for ctype, param in [(W.CARD_GE, k // 3), (W.EK, k // 2), (W.CARD_LT, 2 * k // 3),
                         (W.NAE, 0), (W.OR, 0)]:
        inst = one_constraint(ctype, k, param, signs=signs)
        x0 = rng.uniform(-0.9, 0.9, size=(k, 1))
        g = oracle.eval(inst, x0, grad=True)["grad"][:, 0]
        idx = rng.choice(k, size=min(k, 12), replace=False)
        xs = np.repeat(x0, 2 * len(idx), axis=1)
        for j, i in enumerate(idx):
            xs[i, 2 * j] += h
            xs[i, 2 * j + 1] -= h
        fe = oracle.eval(inst, xs, fe=True, grad=False)["fe"][0]
        fd = (fe[0::2] - fe[1::2]) / (2 * h)
        assert np.max(np.abs(fd - g[idx])) <= 1e-10, (ctype, param)


def test_or_gradient_closed_form():
    k = 50
    rng = np.random.default_rng(1)
    y = rng.uniform(-1, 1, size=(k, 3))
    g = oracle.eval(one_constraint(W.OR, k, 0), y, grad=True)["grad"]
    for i in range(k):
        want = 2 * np.prod((1 + np.delete(y, i, axis=0)) / 2, axis=0) / 2
        assert np.max(np.abs(g[i] - want)) <= 1e-15


# -- invariants ---------------------------------------------------------------------

def test_invariants():
    rng = np.random.default_rng(2)
    k = 23
    y = rng.uniform(-1, 1, size=(k, 8))
    perm = rng.permutation(k)
    for ctype in ALL_TYPES:
        for param in [0, 1, 7, 12, 23]:
            fe = fe_single(ctype, k, param, y)
            assert np.all(np.abs(fe) <= 1 + 1e-15)
            assert np.allclose(fe_single(ctype, k, param, y[perm]), fe, atol=1e-14, rtol=0)
            # negating literal i is the same as flipping y_i
            signs = np.ones(k)
            signs[3] = -1
            inst = one_constraint(ctype, k, param, signs=signs)
            y2 = y.copy()
            y2[3] = -y2[3]
            fe2 = oracle.eval(inst, y2, fe=True)["fe"][0]
            assert np.allclose(fe2, fe, atol=1e-14, rtol=0)


def test_objective_and_gradient_assembly():
    """obj = sum_c w_c FE_c and grad = per-variable sum of adjoints, per restart."""
    rng = np.random.default_rng(3)
    inst = W.random_instance(rng, n=30, count=40, k_lo=1, k_hi=12)
    inst.weights = rng.uniform(0.5, 2.0, size=inst.n_cons)
    x = rng.uniform(-1, 1, size=(inst.n, 5))
    out = oracle.eval(inst, x, fe=True, adj=True, grad=True)
    assert np.allclose(out["obj"], (inst.weights[:, None] * out["fe"]).sum(0), atol=1e-13, rtol=0)
    g = np.zeros_like(x)
    var = np.abs(inst.lits) - 1
    np.add.at(g, var, out["adj"])
    assert np.allclose(out["grad"], g, atol=1e-13, rtol=0)
    # restart columns are independent: evaluating one column alone gives the same
    for b in range(5):
        one = oracle.eval(inst, x[:, b:b + 1], fe=True, grad=True)
        assert np.allclose(one["fe"][:, 0], out["fe"][:, b], atol=0, rtol=0)
        assert np.allclose(one["grad"][:, 0], out["grad"][:, b], atol=0, rtol=0)
    # threads do not change the result
    out1 = oracle.eval(inst, x, fe=True, grad=True, nthreads=1)
    assert np.array_equal(out1["grad"], out["grad"])


# -- rounding and verification --------------------------------------------------------

def test_verify_planted_witness():
    for inst in [W.planted_3sat(instance=0), W.mixed_5k(instance=0)]:
        H = inst.hidden
        x = np.where(H, -1.0, 1.0).astype(np.float32)[:, None]
        x = np.concatenate([x, 0.5 * x, -x], axis=1)
        unsat = oracle.verify(inst, x)
        assert unsat[0] == 0 and unsat[1] == 0
        assert unsat[2] > 0


def test_verify_signed_zero_and_flips():
    # (x1 or not x2): x1 = +0 / -0 are False; x2 = 0 is False so "not x2" is True.
    inst = W.Instance(n=2, con_off=np.array([0, 2, 3]), lits=np.array([1, -2, 1], dtype=np.int32),
                      types=np.array([W.OR, W.OR], dtype=np.int32),
                      params=np.zeros(2, dtype=np.int32))
    x = np.array([[0.0, -0.0, -0.5, 0.5], [0.0, 0.0, 0.5, 0.5]], dtype=np.float32)
    unsat, bits = oracle.verify(inst, x, want_bits=True)
    # col0: x1 F, x2 F: c0 = F or T -> sat; c1 = x1 F -> unsat  => 1
    # col1: -0.0 is False as well => 1
    # col2: x1 T -> both sat => 0 ; col3: x1 F, x2 F -> c0 sat, c1 unsat => 1
    assert unsat.tolist() == [1, 1, 0, 1]
    assert bits[0, 0] == 0b0100 and bits[1, 0] == 0


def test_step_projection_fixed_done():
    x = np.array([[0.95, -0.2], [0.0, 0.5]])
    gr = np.array([[-1.0, 10.0], [2.0, -0.3]])
    out = oracle.step(x, gr, 0.1)
    assert np.allclose(out, [[1.0, -1.0], [-0.2, 0.53]])
    out = oracle.step(x, gr, 0.1, fixed=np.array([1, 0], np.uint8), done=np.array([0, 1], np.uint8))
    assert np.allclose(out, [[0.95, -0.2], [-0.2, 0.5]])


def test_pgd_solves_planted_3sat():
    inst = W.planted_3sat(instance=0)
    x0 = W.uniform_x0(inst.n, 32, workload=1)
    res = oracle.pgd(inst, x0, lr=0.1, steps=200)
    solved = res["first_sat"] >= 0
    assert solved.sum() >= 1
    assert np.all(res["unsat"][solved] == 0)
    xs = res["x"][:, solved].astype(np.float32)
    assert np.all(oracle.verify(inst, xs) == 0)
