"""Long-constraint decomposition (Sec. 5, constraint length ceiling), CPU only.

Pins of the oracle (oracle/decompose.py), independent of it: brute force over
every assignment of small constraints (the original holds exactly when some
values of the auxiliary variables satisfy every piece), judged with the
truth tables of tests/exact.py; the chain's shape (fewest pieces of at most
max_len literals, lengths within one, literals in order, every link shared by
two neighbouring pieces with the stated signs); and the DP completion of an
assignment at lengths brute force cannot reach.  Then the library's
afs_decompose (host code, called through the C ABI) equals the oracle array
for array, and rejects invalid input.
"""
import itertools
from types import SimpleNamespace

import numpy as np
import pytest

import exact
from oracle import decompose as odec
from paper_2606_06641_amd import afsat
from paper_2606_06641_amd.workloads import AMO, CARD_GE, CARD_LT, EK, EO, NAE, OR, XOR

CHAIN = [(OR, 0), (XOR, 0), (XOR, 1), (NAE, 0), (AMO, 0), (EO, 0)]


def _inst(n, rows, types, params, weights=None):
    off = np.zeros(len(rows) + 1, np.int64)
    off[1:] = np.cumsum([len(r) for r in rows])
    return SimpleNamespace(n=n, con_off=off, lits=np.array([v for r in rows for v in r], np.int32),
                           types=np.array(types, np.int32), params=np.array(params, np.int32),
                           weights=None if weights is None else np.array(weights, np.float32))


def _holds(ctype, param, row, value):
    """Truth of one constraint under value (dict var -> bool), from the tables."""
    t = sum(1 for l in row if value[abs(l)] == (l > 0))
    return exact.truth(ctype, len(row), param, t)


def _pieces(dec, c):
    idx = np.nonzero(dec["origin"] == c)[0]
    off, lits = dec["con_off"], dec["lits"]
    return [(list(map(int, lits[off[i]:off[i + 1]])), int(dec["types"][i]), int(dec["params"][i])) for i in idx]


@pytest.mark.parametrize("ctype,param", CHAIN)
@pytest.mark.parametrize("max_len", [3, 4, 5])
def test_brute_force_equivalence(ctype, param, max_len):
    rng = np.random.default_rng(100 * ctype + 10 * param + max_len)
    for k in range(max_len + 1, 10):
        for rep in range(2):
            n = k if rep == 0 else k - 2        # the second draw repeats variables
            vars_ = rng.permutation(n)[:k] + 1 if rep == 0 else rng.integers(1, n + 1, size=k)
            row = [int(v) if rng.random() < 0.5 else -int(v) for v in vars_]
            inst = _inst(n, [row], [ctype], [param])
            dec = odec.decompose(inst, max_len)
            pieces = _pieces(dec, 0)
            aux = list(range(n + 1, dec["n"] + 1))
            assert len(aux) == len(pieces) - 1
            for bits in itertools.product((False, True), repeat=n):
                value = {v + 1: b for v, b in enumerate(bits)}
                want = _holds(ctype, param, row, value)
                got = False
                for abits in itertools.product((False, True), repeat=len(aux)):
                    value.update(zip(aux, abits))
                    if all(_holds(t, p, r, value) for r, t, p in pieces):
                        got = True
                        break
                assert got == want, (k, row, bits)


@pytest.mark.parametrize("ctype,param", CHAIN)
def test_chain_shape(ctype, param):
    rng = np.random.default_rng(7 + ctype)
    for _ in range(40):
        max_len = int(rng.integers(3, 60))
        k = int(rng.integers(max_len + 1, 700))
        row = [int(v) for v in (rng.permutation(1000)[:k] + 1) * rng.choice([-1, 1], size=k)]
        dec = odec.decompose(_inst(1000, [row], [ctype], [param], [2.5]), max_len)
        pieces = _pieces(dec, 0)
        p = len(pieces)
        # fewest pieces: each link adds two literals in total
        assert p * max_len >= k + 2 * (p - 1) and (p - 1) * max_len < k + 2 * (p - 2)
        lens = [len(r) for r, _, _ in pieces]
        assert max(lens) <= max_len and max(lens) - min(lens) <= 1 and lens == sorted(lens, reverse=True)
        own = []
        for i, (r, t, prm) in enumerate(pieces):
            assert t == ctype
            body = r[(1 if i > 0 else 0):(len(r) - 1 if i < p - 1 else len(r))]
            assert body, "a piece without literals of its own"
            own += body
            if i > 0:
                assert r[0] == (1000 + i if ctype == XOR else -(1000 + i))
            if i < p - 1:
                assert r[-1] == 1000 + i + 1
            if ctype == XOR:
                assert prm == (param if i == p - 1 else 0)
        assert own == row
        assert dec["n"] == 1000 + p - 1
        assert np.all(dec["weights"] == np.float32(2.5))


def test_short_and_other_types_are_copied():
    rows = [[1, -2, 3, 4, 5], [1, 2, 3], [-1, 2, -3, 4, 5, 6], [1, 2, 3, 4, 5, 6], [2, 3, 4, 5, 6, 1]]
    inst = _inst(6, rows, [OR, NAE, EK, CARD_GE, CARD_LT], [0, 0, 2, 3, 4], [1, 2, 3, 4, 5])
    dec = odec.decompose(inst, 5)
    assert dec["n"] == 6
    assert np.array_equal(dec["lits"], inst.lits) and np.array_equal(dec["con_off"], inst.con_off)
    assert np.array_equal(dec["types"], inst.types) and np.array_equal(dec["params"], inst.params)
    assert np.array_equal(dec["origin"], np.arange(5))


@pytest.mark.parametrize("ctype,param", CHAIN)
def test_completion_at_length(ctype, param):
    """The DP completion satisfies every piece whenever the original holds, at
    lengths brute force cannot reach; and a violated original leaves a piece
    violated under it."""
    rng = np.random.default_rng(300 + 10 * ctype + param)
    n = 600
    for trial in range(12):
        k = int(rng.integers(60, 500))
        max_len = int(rng.integers(3, 48))
        row = [int(v) for v in (rng.permutation(n)[:k] + 1) * rng.choice([-1, 1], size=k)]
        inst = _inst(n, [row], [ctype], [param])
        dec = odec.decompose(inst, max_len)
        # assignments near the edge of the predicate: mostly false literals with a few true
        lit_true = np.zeros(k, bool)
        lit_true[rng.choice(k, size=int(rng.integers(0, 4)), replace=False)] = True
        if trial % 3 == 0:
            lit_true = rng.random(k) < 0.5
        if trial % 4 == 1:
            lit_true[:] = True
        bits = np.zeros(n, bool)
        for l, tv in zip(row, lit_true):
            bits[abs(l) - 1] = tv if l > 0 else not tv
        full = odec.aux_values(inst, dec, bits)
        value = {v + 1: bool(full[v]) for v in range(dec["n"])}
        ok = all(_holds(t, p, r, value) for r, t, p in _pieces(dec, 0))
        assert ok == _holds(ctype, param, row, value), (k, max_len, trial)


def _random_instance(rng, n, C):
    rows, types, params = [], [], []
    for _ in range(C):
        k = int(rng.integers(1, 200)) if rng.random() < 0.5 else int(rng.integers(1, 12))
        rows.append([int(v) for v in rng.integers(1, n + 1, size=k) * rng.choice([-1, 1], size=k)])
        t = int(rng.integers(0, 8))
        types.append(t)
        params.append(int(rng.integers(0, 2)) if t == XOR else int(rng.integers(0, k + 2)) if t in (3, 4, 7) else 0)
    return rows, types, params


@pytest.mark.parametrize("seed", range(6))
def test_library_equals_oracle(seed):
    rng = np.random.default_rng(seed)
    n = int(rng.integers(5, 400))
    rows, types, params = _random_instance(rng, n, int(rng.integers(0, 60)))
    w = rng.uniform(0.5, 3.0, size=len(rows)) if seed % 2 else None
    inst = _inst(n, rows, types, params, w)
    for max_len in (3, 8, 17, 48, 1024):
        want = odec.decompose(inst, max_len)
        got = afsat.decompose(inst, max_len)
        assert got.n == want["n"] and got.n_orig == n
        for key in ("con_off", "lits", "types", "params", "origin"):
            assert np.array_equal(getattr(got, key), want[key]), key
        if w is None:
            assert got.weights is None
        else:
            assert np.array_equal(got.weights, want["weights"])


def test_library_accepts_lengths_beyond_the_kernels():
    """A chain type longer than the kernels' 1,024 maximum decomposes to pieces they take."""
    row = list(range(1, 3001))
    got = afsat.decompose(_inst(3000, [row], [XOR], [1]), 64)
    assert np.diff(got.con_off).max() <= 64 and got.n == 3000 + len(got.types) - 1


@pytest.mark.parametrize("case", ["max_len_low", "max_len_high", "empty", "literal_zero", "literal_high",
                                  "type", "offsets"])
def test_library_rejects_invalid_input(case):
    inst = _inst(4, [[1, 2, 3, 4, -1]], [OR], [0])
    max_len = 4
    if case == "max_len_low":
        max_len = 2
    elif case == "max_len_high":
        max_len = 1025
    elif case == "empty":
        inst = _inst(4, [[1, 2], []], [OR, OR], [0, 0])
    elif case == "literal_zero":
        inst.lits[2] = 0
    elif case == "literal_high":
        inst.lits[2] = -5
    elif case == "type":
        inst.types[0] = 8
    elif case == "offsets":
        inst.con_off = np.array([1, 5], np.int64)     # the first offset must be 0
    with pytest.raises((afsat.AfsError, ValueError)) as e:
        afsat.decompose(inst, max_len)
    if isinstance(e.value, afsat.AfsError):
        assert e.value.status == afsat.AFS_EINVAL
