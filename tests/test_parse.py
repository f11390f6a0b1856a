"""Reader of DIMACS CNF and the hybrid symmetric-constraint format (App. A).

Pins: the paper's own example lines (tests/golden/appendix_a_*.cnf and the
source column of appendix_a_truth.txt) parse to the type, length and threshold
that App. A's table and CARD normalisation give; and on random small inputs,
brute force over every assignment shows that the kept constraints together with
the reported units accept exactly the assignments the input accepts, where the
input's meaning is computed straight from its written form (operator and
number), not from the normalised one.
"""
import itertools
import os

import numpy as np
import pytest

from paper_2606_06641_amd import afsat
from paper_2606_06641_amd.afsat import AFS_EINVAL, AFS_EUNSAT, AfsError
import oracle

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def _one(text):
    p = afsat.parse_text(text)
    assert len(p.types) == 1, text
    return int(p.types[0]), int(p.con_off[1] - p.con_off[0]), int(p.params[0]), p


def test_truth_fixture_lines_parse_to_their_type_and_threshold():
    """Each example line of App. A (source column of the truth-table fixture)
    reads as the (type, k, param) the fixture lists for it."""
    n = 0
    with open(os.path.join(GOLDEN, "appendix_a_truth.txt")) as f:
        for line in f:
            if line.startswith("#") or not line.strip():
                continue
            cols, src = line.split("|", 1)
            ty, k, prm = (int(v) for v in cols.split()[:3])
            got = _one(src.strip())
            assert got[:3] == (ty, k, prm), src
            n += 1
    assert n == 11


def test_hybrid_example_file():
    p = afsat.parse_file(os.path.join(GOLDEN, "appendix_a_hybrid.cnf"))
    assert p.n == 6 and p.declared_cons == 7 and p.n_dropped == 0
    assert list(p.types) == [afsat.OR, afsat.XOR, afsat.NAE, afsat.AMO, afsat.EO, afsat.EK, afsat.CARD_GE]
    assert list(p.params) == [0, 1, 0, 0, 0, 2, 2]
    assert list(p.con_off) == [0, 3, 6, 9, 12, 15, 18, 21]
    assert list(p.lits) == [1, -2, 3] + [1, 2, 3] * 3 + [4, 5, 6] + [1, 2, 3] * 2
    assert not p.units.any()


def test_plain_cnf_example_file():
    p = afsat.parse_file(os.path.join(GOLDEN, "appendix_a_cnf.cnf"))
    assert p.n == 4 and p.declared_cons == 2
    assert list(p.types) == [afsat.OR, afsat.OR]
    assert list(p.con_off) == [0, 3, 5] and list(p.lits) == [1, -2, 3, -1, 4]


@pytest.mark.parametrize("text,ty,prm", [
    ("card >= 2 1 2 3 0", afsat.CARD_GE, 2),      # operator apart from its number
    ("d > 1 1 2 3 0", afsat.CARD_GE, 2),
    ("d < 3 1 2 3 4 0", afsat.CARD_LT, 3),
    ("d <= 1 1 2 3 0", afsat.CARD_LT, 2),
    ("d <2 1 2 3 0", afsat.CARD_LT, 2),
    ("xor -1 2 0", afsat.XOR, 1),
    ("n 1 -2 0", afsat.NAE, 0),
    ("a 1 2 3 0", afsat.AMO, 0),
    ("e 1 2 0", afsat.EO, 0),
    ("k 2 1 2 3 0", afsat.EK, 2),
])
def test_type_spellings(text, ty, prm):
    assert _one(text)[0::2] == (ty, prm)


def test_simplifications():
    """Each rule of App. A's simplification list, one at a time."""
    p = afsat.parse_text("p cnf 9 9\n-1 0\ne 2 0\na 3 0\nd 1 4 5 0\nek 1 6 7 0\n"
                         "d >=2 8 -9 0\nk 0 4 -5 0\nd >=0 1 2 3 0\nd 0 1 2 0\n")
    assert p.n == 9 and p.declared_cons == 9
    # kept: CARD>=1 -> OR, EK 1 -> EO
    assert list(p.types) == [afsat.OR, afsat.EO]
    assert list(p.lits) == [4, 5, 6, 7]
    # units: -1 (x1 False), 2 True, CARD-n fixes 8 True and 9 False, EK-0 fixes 4 False and 5 True
    assert list(p.units) == [-1, 1, 0, -1, 1, 0, 0, 1, -1]
    assert p.n_dropped == 7  # unit OR, unit EO, unit AMO, CARD-n, EK-0, two CARD-0


def test_cardinality_beyond_length():
    p = afsat.parse_text("d <5 1 2 3 0\n1 2 0\n")  # always met: dropped
    assert p.n_dropped == 1 and list(p.types) == [afsat.OR]
    for text in ("d >=4 1 2 3 0\n", "k 4 1 2 3 0\n", "k -1 1 2 0\n", "d <0 1 2 0\n", "d <=-1 1 0\n"):
        with pytest.raises(AfsError) as e:
            afsat.parse_text(text)
        assert e.value.status in (AFS_EUNSAT, AFS_EINVAL), text
    for text in ("d >=4 1 2 3 0\n", "k 4 1 2 3 0\n", "k -1 1 2 0\n", "d <0 1 2 0\n"):
        with pytest.raises(AfsError) as e:
            afsat.parse_text(text)
        assert e.value.status == AFS_EUNSAT, text


@pytest.mark.parametrize("text", [
    "1 0\n-1 0\n",               # unit clauses both ways
    "e 2 0\nk 0 2 3 0\n",        # EO unit vs EK-0
    "d 2 1 -1 0\n",              # CARD-n over complementary literals
])
def test_conflicting_units_are_unsat(text):
    with pytest.raises(AfsError) as e:
        afsat.parse_text(text)
    assert e.value.status == AFS_EUNSAT
    assert "line" in str(e.value)


def test_layout_details():
    text = ("c comment\n* star comment\n\n"
            "h x 1 2\n  3 0 trailing words\n"      # a constraint over two lines, text after 0
            "card >=2\n1 2 3 0\n"                  # literals on the next line
            "-4 5 0\n%\n0\nignored after the end marker\n")
    p = afsat.parse_text(text)
    assert p.n == 5 and p.declared_cons == -1
    assert list(p.types) == [afsat.XOR, afsat.CARD_GE, afsat.OR]
    assert list(p.lits) == [1, 2, 3, 1, 2, 3, -4, 5]


@pytest.mark.parametrize("text,where", [
    ("1 2\n", "line 1"),                     # not terminated
    ("p cnf 2 1\n1 3 0\n", "exceeds"),       # variable beyond the problem line
    ("p cnf 2 1\n1 2000000000 0\n", "line 2"),  # reported where it appears, nothing sized to it
    ("p cnf 2 1\n-2000000000 0\n", "line 2"),
    ("p cnf 2 1\np cnf 2 1\n", "line 2"),    # second problem line
    ("p dnf 2 1\n", "line 1"),
    ("1 foo 0\n", "line 1"),
    ("x 0\n", "line 1"),                     # constraint without literals
    ("k two 1 2 0\n", "line 1"),
    ("d >= -2 1 2 0\n", "line 1"),           # operator with a negative number
    ("0\n", "line 1"),
    ("1 99999999999 0\n", "line 1"),
])
def test_malformed_input_rejected(text, where):
    with pytest.raises(AfsError) as e:
        afsat.parse_text(text)
    assert e.value.status == AFS_EINVAL
    assert where in str(e.value)


def test_missing_file():
    with pytest.raises(AfsError) as e:
        afsat.parse_file("/nonexistent/file.cnf")
    assert e.value.status == AFS_EINVAL


def test_empty_input():
    p = afsat.parse_text("")
    assert p.n == 0 and len(p.types) == 0 and len(p.con_off) == 1


# ---- brute force: input meaning == kept constraints + units ------------------------------

_SPELL = {"x": ("x", "xor"), "n": ("n", "nae"), "a": ("a", "amo"), "e": ("e", "eo"),
          "k": ("k", "ek"), "d": ("d", "card")}


def _written_meaning(kind, op, K, t, k):
    """Truth of the written constraint for t true literals out of k (Table 2 and
    the CARD operators as written, before any normalisation)."""
    if kind == "or":
        return t >= 1
    if kind == "x":
        return t % 2 == 1
    if kind == "n":
        return 0 < t < k
    if kind == "a":
        return t <= 1
    if kind == "e":
        return t == 1
    if kind == "k":
        return t == K
    return {">=": t >= K, ">": t > K, "<": t < K, "<=": t <= K,
            "+": t >= K, "-": t < -K, "0": True}[op]


def _random_input(rng, n):
    cons, lines = [], []
    for _ in range(int(rng.integers(1, 5))):
        kind = str(rng.choice(["or", "x", "n", "a", "e", "k", "d"]))
        k = int(rng.integers(1, 5))
        vs = rng.choice(n, size=k, replace=bool(k > n or rng.random() < 0.15)) + 1
        lits = [int(v) * (1 if rng.random() < 0.5 else -1) for v in vs]
        op, K, head = None, 0, []
        if kind == "k":
            K = int(rng.integers(0, k + 1)) if rng.random() < 0.95 else k + 1
            head = [str(rng.choice(_SPELL["k"])), str(K)]
        elif kind == "d":
            op = str(rng.choice([">=", ">", "<", "<=", "+", "-", "0"]))
            K = int(rng.integers(0, k + 2))
            if op == "+":
                K = max(K, 1)
                th = [str(K)]
            elif op == "-":
                K = -max(K, 1)
                th = [str(K)]
            elif op == "0":
                K = 0
                th = ["0"]
            else:
                if op == "<" and K == 0:
                    K = 1
                th = [op + str(K)] if rng.random() < 0.5 else [op, str(K)]
            head = [str(rng.choice(_SPELL["d"]))] + th
        elif kind != "or":
            head = [str(rng.choice(_SPELL[kind]))]
        toks = (["h"] if rng.random() < 0.3 else []) + head + [str(l) for l in lits] + ["0"]
        lines.append(" ".join(toks))
        cons.append((kind, op, K, lits))
    return cons, "p cnf %d %d\n" % (n, len(cons)) + "\n".join(lines) + "\n"


def _truth_of_lits(A, lits):
    cols = [A[:, abs(l) - 1] ^ (l < 0) for l in lits]
    return np.sum(cols, axis=0)


@pytest.mark.parametrize("seed", range(300))
def test_simplified_input_accepts_the_same_assignments(seed):
    rng = np.random.default_rng(seed)
    n = int(rng.integers(1, 7))
    cons, text = _random_input(rng, n)
    A = np.array(list(itertools.product([False, True], repeat=n)), dtype=bool)  # True = variable true
    want = np.ones(len(A), dtype=bool)
    for kind, op, K, lits in cons:
        t = _truth_of_lits(A, lits)
        want &= np.array([_written_meaning(kind, op, K, int(ti), len(lits)) for ti in t])
    try:
        p = afsat.parse_text(text)
    except AfsError as e:
        assert e.status == AFS_EUNSAT, (text, str(e))
        assert not want.any(), text
        return
    assert p.n == n
    got = np.ones(len(A), dtype=bool)
    for c in range(len(p.types)):
        lits = p.lits[p.con_off[c]:p.con_off[c + 1]]
        t = _truth_of_lits(A, [int(l) for l in lits])
        got &= np.array([oracle.sat(int(p.types[c]), len(lits), int(p.params[c]), int(ti)) for ti in t])
    for v in range(n):
        if p.units[v]:
            got &= A[:, v] == (p.units[v] > 0)
    assert np.array_equal(got, want), text


# ---- unit folding (Sec. 3.4) ------------------------------------------------------------

def test_units_become_a_universal_partial_assignment():
    p = afsat.parse_text("p cnf 5 3\n-2 0\ne 4 0\n1 3 5 0\n")
    vals = p.fold_units()
    assert vals.shape == (1, 5)
    assert list(vals[0]) == [0, -1, 0, 1, 0]


def test_units_fold_into_every_partial_assignment():
    p = afsat.parse_text("p cnf 4 2\n-2 0\n1 3 4 0\n")
    parts = np.array([[1, 0, 0, 0], [0, -1, 1, 0], [-1, 0, 0, -1]], dtype=np.int8)
    vals = p.fold_units(parts)
    np.testing.assert_array_equal(vals, [[1, -1, 0, 0], [0, -1, 1, 0], [-1, -1, 0, -1]])
    np.testing.assert_array_equal(parts[0], [1, 0, 0, 0])     # the input is not modified


def test_unit_contradicting_a_partial_assignment_is_unsat():
    p = afsat.parse_text("p cnf 3 2\n2 0\n1 3 0\n")
    with pytest.raises(AfsError) as e:
        p.fold_units([[0, 0, 1], [0, -1, 0]])
    assert e.value.status == AFS_EUNSAT and "partial assignment 1" in str(e.value)
    with pytest.raises(ValueError):
        p.fold_units([[0, 1]])
