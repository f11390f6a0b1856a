"""Tables of the two DFT evaluation forms (Sec. 2.1.2; precision study of
Sec. 3.5), on the CPU.

Pins: form A's coefficients carry the Walsh-Fourier coefficients computed by
brute force from their definition (an average over every corner of {-1,1}^k);
both forms' tables, evaluated in complex128 here, give the oracle's FE at
random points; form B's factor rows are the closed forms (1 +- omega^m)/2 and
its d the library's coefficient vector."""
import itertools
from fractions import Fraction

import numpy as np
import pytest

import oracle
from paper_2606_06641_amd import afsat

TYPES = [(afsat.OR, 0), (afsat.XOR, 1), (afsat.NAE, 0), (afsat.CARD_GE, 2), (afsat.CARD_LT, 3),
         (afsat.AMO, 0), (afsat.EO, 0), (afsat.EK, 2)]


def walsh_brute(ctype, k, param):
    """fhat_t = 2^-k sum over x in {-1,1}^k of g(#(x = -1)) * prod_{i<t} x_i."""
    out = []
    for t in range(k + 1):
        acc = Fraction(0)
        for x in itertools.product([1, -1], repeat=k):
            s = sum(1 for v in x if v < 0)
            g = -1 if oracle.sat(ctype, k, param, s) else 1
            acc += g * int(np.prod(x[:t]))
        out.append(acc / 2 ** k)
    return out


def one_constraint(ctype, k, param):
    class I:
        pass
    i = I()
    i.n, i.con_off, i.lits = k, np.array([0, k]), np.arange(1, k + 1, dtype=np.int32)
    i.types, i.params, i.weights = np.array([ctype]), np.array([param]), None
    return i


def eval_form(tables, y):
    alpha, beta, d = tables
    prods = np.prod(alpha[:, None, None] + beta[:, None, None] * y[None, :, :], axis=1)   # (N, B)
    return np.real(np.sum(d[:, None] * prods, axis=0))


@pytest.mark.parametrize("ctype,param", TYPES)
@pytest.mark.parametrize("k", [1, 3, 6])
def test_form_a_carries_the_walsh_coefficients(ctype, param, k):
    _, _, c = afsat.form_tables(ctype, k, param, afsat.FORM_A)
    N = k + 1
    w = np.exp(2j * np.pi * np.outer(np.arange(N), np.arange(N)) / N)
    fh_rev = c @ w                        # sum_m c_m omega^(m j) = fhat_(k-j)
    want = walsh_brute(ctype, k, param)
    np.testing.assert_allclose(fh_rev.real[::-1], [float(v) for v in want], rtol=0, atol=1e-14)
    np.testing.assert_allclose(fh_rev.imag, 0, atol=1e-14)


@pytest.mark.parametrize("ctype,param", TYPES)
@pytest.mark.parametrize("k", [2, 5, 12])
def test_both_forms_give_the_oracle_fe(ctype, param, k):
    rng = np.random.default_rng(k * 10 + ctype)
    y = rng.uniform(-1, 1, size=(k, 20))
    want = oracle.eval(one_constraint(ctype, k, param), y, fe=True, grad=False)["fe"][0]
    for form in (afsat.FORM_A, afsat.FORM_B):
        got = eval_form(afsat.form_tables(ctype, k, param, form), y)
        np.testing.assert_allclose(got, want, rtol=0, atol=1e-12)
    # at corners the FE is the truth value
    corners = np.where(rng.random((k, 16)) < 0.5, -1.0, 1.0)
    tv = np.array([-1.0 if oracle.sat(ctype, k, param, int((corners[:, b] < 0).sum())) else 1.0 for b in range(16)])
    np.testing.assert_allclose(eval_form(afsat.form_tables(ctype, k, param, afsat.FORM_A), corners), tv, atol=1e-12)


def test_form_b_rows_are_the_count_basis():
    k = 9
    alpha, beta, d = afsat.form_tables(afsat.CARD_GE, k, 4, afsat.FORM_B)
    w = np.exp(2j * np.pi * np.arange(k + 1) / (k + 1))
    np.testing.assert_allclose(alpha, (1 + w) / 2, atol=1e-15)
    np.testing.assert_allclose(beta, (1 - w) / 2, atol=1e-15)
    np.testing.assert_array_equal(d, afsat.coefficients(afsat.CARD_GE, k, 4))


def test_form_a_length_limit_and_errors():
    afsat.form_tables(afsat.AMO, 120, 0, afsat.FORM_A)
    with pytest.raises(afsat.AfsError):
        afsat.form_tables(afsat.AMO, 121, 0, afsat.FORM_A)
    afsat.form_tables(afsat.AMO, 1024, 0, afsat.FORM_B)
    with pytest.raises(afsat.AfsError):
        afsat.form_tables(afsat.AMO, 8, 0, 2)
