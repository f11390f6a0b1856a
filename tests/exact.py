"""Exact rational checks that pin the FP64 oracle to the mathematics.

Nothing here shares code with the oracle or the GPU library.  Every value is
computed in ``fractions.Fraction`` straight from a definition:

* ``truth``       -- constraint predicates restated from Table 1 / Table 2 /
                     Appendix A (True -> -1, False -> +1, Sec. 2.1).
* ``fourier_coefficients`` / ``fe_by_coefficients``
                  -- Eq. (1): f_hat(S) = 2^-k sum_z f(z) prod_{i in S} z_i and
                     FE(y) = sum_S f_hat(S) prod_{i in S} y_i  (tiny k only).
* ``fe_by_corners`` -- the same multilinear polynomial written as
                     sum_z f(z) prod_i (1 + y_i z_i)/2 (k <= 12).
* ``fe_binomial`` -- closed form when every literal has the same value y:
                     sum_t g(t) C(k,t) p^t (1-p)^(k-t), p = (1-y)/2.
"""
from fractions import Fraction
from itertools import product
from math import comb

OR, XOR, NAE, CARD_GE, CARD_LT, AMO, EO, EK = range(8)


def truth(ctype, k, param, t):
    """Satisfied? given t true literals out of k."""
    if ctype == OR:
        return t >= 1
    if ctype == XOR:
        return t % 2 == param % 2
    if ctype == NAE:
        return 0 < t < k
    if ctype == CARD_GE:
        return t >= param
    if ctype == CARD_LT:
        return t < param
    if ctype == AMO:
        return t <= 1
    if ctype == EO:
        return t == 1
    if ctype == EK:
        return t == param
    raise ValueError(ctype)


def g(ctype, k, param, t):
    return -1 if truth(ctype, k, param, t) else 1


def _f_of_corner(ctype, k, param, z):
    # z_i = -1 means literal i is True (Sec. 2.1)
    return g(ctype, k, param, sum(1 for zi in z if zi == -1))


def fourier_coefficients(ctype, k, param):
    """{S (tuple of indices): f_hat(S)} by the definition (2^k x 2^k sums)."""
    corners = list(product((1, -1), repeat=k))
    fz = [_f_of_corner(ctype, k, param, z) for z in corners]
    coef = {}
    for mask in range(1 << k):
        S = tuple(i for i in range(k) if mask >> i & 1)
        acc = 0
        for z, f in zip(corners, fz):
            s = f
            for i in S:
                s *= z[i]
            acc += s
        coef[S] = Fraction(acc, 1 << k)
    return coef


def fe_by_coefficients(coef, y):
    total = Fraction(0)
    for S, c in coef.items():
        term = c
        for i in S:
            term *= y[i]
        total += term
    return total


def fe_by_corners(ctype, k, param, y):
    y = [Fraction(v) for v in y]
    total = Fraction(0)
    for z in product((1, -1), repeat=k):
        w = Fraction(1)
        for yi, zi in zip(y, z):
            w *= (1 + yi * zi) / 2
        total += w * _f_of_corner(ctype, k, param, z)
    return total


def grad_by_corners(ctype, k, param, y):
    """dFE/dy_i of the multilinear polynomial: (FE(y_i=1) - FE(y_i=-1)) / 2."""
    out = []
    for i in range(k):
        hi = list(y)
        lo = list(y)
        hi[i] = Fraction(1)
        lo[i] = Fraction(-1)
        out.append((fe_by_corners(ctype, k, param, hi) - fe_by_corners(ctype, k, param, lo)) / 2)
    return out


def fe_binomial(ctype, k, param, y):
    p = (1 - Fraction(y)) / 2
    return sum(g(ctype, k, param, t) * comb(k, t) * p ** t * (1 - p) ** (k - t)
               for t in range(k + 1))


def fe_at_zero(ctype, k, param):
    """FE(0) = 1 - 2^(1-k) sum_{t satisfied} C(k, t)."""
    sat = sum(comb(k, t) for t in range(k + 1) if truth(ctype, k, param, t))
    return 1 - Fraction(2 * sat, 1 << k)
