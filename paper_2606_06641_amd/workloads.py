"""Seeded synthetic workloads: planted-solution instances and starting points.

This module only draws random inputs.  It holds none of the method's
arithmetic (no expansion, gradient, step or verification) and imports neither
the GPU library nor the oracle, so both sides can be fed the same arrays.

An instance is a list of symmetric constraints (Table 1 of the paper) over
variables 1..n.  Each constraint is a list of DIMACS-signed literals, a type
code and an integer parameter:

    type  code  param
    OR     0    unused
    XOR    1    parity (1 = odd number of true literals, the paper's XOR)
    NAE    2    unused
    CARD>= 3    K  (at least K true)
    CARD<  4    K  (fewer than K true; Appendix A normalisation)
    AMO    5    unused
    EO     6    unused
    EK     7    K  (exactly K true)

Planting: a hidden assignment H is drawn first; every constraint is drawn
until H satisfies it, so H is a witness that the instance is satisfiable.
Literal i is true under H when H[var] differs from the literal's negation.

Seeds: numpy PCG64 streams keyed by SeedSequence([workload, instance, purpose])
with purpose 0 = instance, 1 = starting points, 2 = learned-initialisation data.
"""
from dataclasses import dataclass, field
from typing import List, Optional, Sequence

import numpy as np

OR, XOR, NAE, CARD_GE, CARD_LT, AMO, EO, EK = range(8)
TYPE_NAMES = ["OR", "XOR", "NAE", "CARD_GE", "CARD_LT", "AMO", "EO", "EK"]

PURPOSE_INSTANCE, PURPOSE_X0, PURPOSE_GNN = 0, 1, 2


@dataclass
class Instance:
    """Constraint list in CSR form (``con_off`` int64 [C+1], ``lits`` int32 [L])."""
    n: int
    con_off: np.ndarray
    lits: np.ndarray
    types: np.ndarray
    params: np.ndarray
    weights: Optional[np.ndarray] = None
    hidden: Optional[np.ndarray] = None          # bool [n], True = variable true
    name: str = ""
    meta: dict = field(default_factory=dict)

    @property
    def n_cons(self) -> int:
        return int(len(self.types))

    @property
    def n_lits(self) -> int:
        return int(self.con_off[-1])

    def lengths(self) -> np.ndarray:
        return np.diff(self.con_off).astype(np.int64)


def rng_for(workload: int, instance: int, purpose: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(np.random.SeedSequence([workload, instance, purpose])))


def _true_counts(rows_vars: np.ndarray, rows_neg: np.ndarray, hidden: np.ndarray) -> np.ndarray:
    return (hidden[rows_vars] ^ rows_neg).sum(axis=1)


def _distinct_rows(rng, n: int, count: int, k: int) -> np.ndarray:
    """``count`` rows of ``k`` distinct variable indices in [0, n)."""
    if k * 4 > n:
        return np.stack([rng.choice(n, size=k, replace=False) for _ in range(count)])
    out = rng.integers(0, n, size=(count, k))
    for _ in range(64):
        s = np.sort(out, axis=1)
        bad = np.nonzero((s[:, 1:] == s[:, :-1]).any(axis=1))[0]
        if bad.size == 0:
            return out
        out[bad] = rng.integers(0, n, size=(bad.size, k))
    for i in np.nonzero((np.sort(out, axis=1)[:, 1:] == np.sort(out, axis=1)[:, :-1]).any(axis=1))[0]:
        out[i] = rng.choice(n, size=k, replace=False)
    return out


def _draw_group(rng, n: int, hidden: np.ndarray, count: int, k: int, ctype: int,
                k_param=None):
    """Draw ``count`` planted constraints of one type and one length ``k``.

    Returns (vars [count,k], neg [count,k], params [count])."""
    vars_ = np.empty((count, k), dtype=np.int64)
    neg = np.empty((count, k), dtype=bool)
    params = np.zeros(count, dtype=np.int64)
    todo = np.arange(count)
    for _ in range(10000):
        if todo.size == 0:
            break
        v = _distinct_rows(rng, n, todo.size, k)
        s = rng.integers(0, 2, size=(todo.size, k)).astype(bool)
        t = _true_counts(v, s, hidden)
        if ctype == OR:
            ok = t >= 1
            p = np.zeros(todo.size, dtype=np.int64)
        elif ctype == XOR:
            ok = np.ones(todo.size, dtype=bool)
            p = (t & 1).astype(np.int64)
        elif ctype == NAE:
            ok = (t > 0) & (t < k)
            p = np.zeros(todo.size, dtype=np.int64)
        elif ctype == CARD_GE:
            hi = max(1, k // 2)
            p = rng.integers(1, hi + 1, size=todo.size)
            ok = p <= t
        elif ctype in (AMO, EO):
            # a random draw almost never has t <= 1 at length: the signs are
            # chosen from H instead, every literal false but one (EO) or at
            # most one (AMO, a fair coin)
            s = hidden[v].copy()
            one = rng.integers(0, k, size=todo.size)
            flip = np.ones(todo.size, dtype=bool) if ctype == EO else rng.integers(0, 2, size=todo.size) == 1
            rows = np.nonzero(flip)[0]
            s[rows, one[rows]] = ~s[rows, one[rows]]
            ok = np.ones(todo.size, dtype=bool)
            p = np.zeros(todo.size, dtype=np.int64)
        else:
            raise ValueError("planted draw not defined for type %d" % ctype)
        keep = np.nonzero(ok)[0]
        vars_[todo[keep]] = v[keep]
        neg[todo[keep]] = s[keep]
        params[todo[keep]] = p[keep]
        todo = todo[~ok]
    if todo.size:
        raise RuntimeError("could not plant %d constraints" % todo.size)
    return vars_, neg, params


def _assemble(n: int, groups, hidden, name: str, rng, shuffle: bool = True) -> Instance:
    """groups: list of (ctype, vars [c,k], neg [c,k], params [c]).  The rows of all
    groups, in group order, are permuted by one draw of ``rng`` and concatenated."""
    lit_rows, row_len, row_type, row_par, row_src = [], [], [], [], []
    base = 0
    for ctype, v, s, p in groups:
        c, k = v.shape
        lit = (v + 1).astype(np.int32)
        lit[s] = -lit[s]
        lit_rows.append(lit.reshape(-1))
        row_len.append(np.full(c, k, dtype=np.int64))
        row_type.append(np.full(c, ctype, dtype=np.int32))
        row_par.append(np.asarray(p, dtype=np.int32))
        row_src.append(base + np.arange(c, dtype=np.int64) * k)    # start of each row in the flat lits
        base += c * k
    total_rows = sum(len(x) for x in row_len)
    flat = np.concatenate(lit_rows) if lit_rows else np.zeros(0, np.int32)
    lens_all = np.concatenate(row_len) if row_len else np.zeros(0, np.int64)
    src_all = np.concatenate(row_src) if row_src else np.zeros(0, np.int64)
    order = rng.permutation(total_rows) if shuffle else np.arange(total_rows)
    lens = lens_all[order]
    con_off = np.zeros(total_rows + 1, dtype=np.int64)
    np.cumsum(lens, out=con_off[1:])
    # every output literal's index in the flat array: its row's source start plus its position
    pos = np.arange(int(con_off[-1]), dtype=np.int64) - np.repeat(con_off[:-1], lens)
    lits = flat[np.repeat(src_all[order], lens) + pos].astype(np.int32)
    types = (np.concatenate(row_type) if row_type else np.zeros(0, np.int32))[order]
    params = (np.concatenate(row_par) if row_par else np.zeros(0, np.int32))[order]
    return Instance(n=n, con_off=con_off, lits=lits, types=types.astype(np.int32),
                    params=params.astype(np.int32), weights=None, hidden=hidden, name=name)


def _by_length(rng, count: int, lo: int, hi: int, log_uniform: bool = False) -> dict:
    if count <= 0:
        return {}
    if log_uniform:
        ks = np.floor(np.exp(rng.uniform(np.log(lo), np.log(hi + 1), size=count))).astype(np.int64)
        ks = np.clip(ks, lo, hi)
    else:
        ks = rng.integers(lo, hi + 1, size=count)
    vals, counts = np.unique(ks, return_counts=True)
    return {int(k): int(c) for k, c in zip(vals, counts)}


def planted_mixed(n: int, spec: Sequence[tuple], workload: int, instance: int = 0,
                  name: str = "") -> Instance:
    """Planted instance from ``spec`` = [(ctype, count, k_lo, k_hi, log_uniform)]."""
    rng = rng_for(workload, instance, PURPOSE_INSTANCE)
    hidden = rng.integers(0, 2, size=n).astype(bool)
    groups = []
    for ctype, count, lo, hi, logu in spec:
        for k, c in sorted(_by_length(rng, count, lo, hi, logu).items()):
            if k > n:
                raise ValueError("constraint length %d exceeds n=%d" % (k, n))
            v, s, p = _draw_group(rng, n, hidden, c, k, ctype)
            groups.append((ctype, v, s, p))
    inst = _assemble(n, groups, hidden, name, rng)
    inst.meta = {"workload": workload, "instance": instance, "spec": [tuple(x) for x in spec]}
    return inst


# ---------------------------------------------------------------------------
# Named workloads (the shapes of the paper's benchmark families: random 3-SAT
# near the 4.26 threshold, cardinality-heavy and parity/XOR instances).
# ---------------------------------------------------------------------------

def planted_3sat(n: int = 100, m: int = 426, instance: int = 0) -> Instance:
    """Planted random 3-SAT, n=100, m=426 by default."""
    return planted_mixed(n, [(OR, m, 3, 3, False)], workload=1, instance=instance,
                         name="planted-3sat-n%d-m%d" % (n, m))


def mixed_10k(instance: int = 0) -> Instance:
    """n=10,000: 30,000 clauses (k 3-8), 2,000 XOR (k 3-5), 500 CARD>=K (k 20-200)."""
    return planted_mixed(10000, [(OR, 30000, 3, 8, False), (XOR, 2000, 3, 5, False),
                                 (CARD_GE, 500, 20, 200, False)],
                         workload=2, instance=instance, name="mixed-n10k")


def long_card_50k(instance: int = 0) -> Instance:
    """n=50,000: 200,000 clauses (k 3-10), 1,000 CARD>=K (k 256-1024)."""
    return planted_mixed(50000, [(OR, 200000, 3, 10, False), (CARD_GE, 1000, 256, 1024, False)],
                         workload=4, instance=instance, name="longcard-n50k")


def long_chain_20k(instance: int = 0) -> Instance:
    """n=20,000: 60,000 clauses (k 3-8) and 150 each of OR, XOR, NAE, AMO and EO
    with k 64-1024: the types the chain decomposition of Sec. 5 applies to."""
    spec = [(OR, 60000, 3, 8, False)] + [(t, 150, 64, 1024, False) for t in (OR, XOR, NAE, AMO, EO)]
    return planted_mixed(20000, spec, workload=6, instance=instance, name="longchain-n20k")


def mixed_5k(instance: int = 0) -> Instance:
    """n=5,000: 15,000 clauses (k 3-8), 1,000 XOR (k 3-5), 250 CARD>=K (k 20-200)."""
    return planted_mixed(5000, [(OR, 15000, 3, 8, False), (XOR, 1000, 3, 5, False),
                                (CARD_GE, 250, 20, 200, False)],
                         workload=5, instance=instance, name="mixed-n5k")


def uneven_batch(count: int = 64, n_lo: int = 500, n_hi: int = 50000) -> List[Instance]:
    """``count`` planted instances with n log-uniform in [n_lo, n_hi], constraint/variable
    ratio uniform in [3.5, 4.2], mixing 70% clauses (k 2-8), 10% NAE (k 2-8),
    10% XOR (k 2-6) and 10% CARD>=K (k log-uniform 8-256)."""
    rng = rng_for(3, 0, PURPOSE_INSTANCE)
    ns = np.floor(np.exp(rng.uniform(np.log(n_lo), np.log(n_hi), size=count))).astype(int)
    ratios = rng.uniform(3.5, 4.2, size=count)
    out = []
    for i in range(count):
        m = int(round(ns[i] * ratios[i]))
        spec = [(OR, int(round(0.7 * m)), 2, 8, False), (NAE, int(round(0.1 * m)), 2, 8, False),
                (XOR, int(round(0.1 * m)), 2, 6, False),
                (CARD_GE, int(round(0.1 * m)), 8, min(256, int(ns[i])), True)]
        out.append(planted_mixed(int(ns[i]), spec, workload=3, instance=i + 1,
                                 name="uneven-%d-n%d" % (i, ns[i])))
    return out


def uniform_x0(n: int, B: int, workload: int, instance: int = 0, round_: int = 0) -> np.ndarray:
    """Starting points x ~ U[-1, 1], float32, layout [n][B] (restart index contiguous)."""
    rng = np.random.Generator(np.random.PCG64(
        np.random.SeedSequence([workload, instance, PURPOSE_X0, round_])))
    return rng.uniform(-1.0, 1.0, size=(n, B)).astype(np.float32)


def random_instance(rng: np.random.Generator, n: int, count: int, k_lo: int, k_hi: int,
                    types: Sequence[int] = (OR, XOR, NAE, CARD_GE, CARD_LT, AMO, EO, EK)
                    ) -> Instance:
    """Unplanted random instance with every type mixed (for parity tests): distinct
    variables per constraint, uniform signs, parameters drawn over their full range
    0..k+1 for the counted types."""
    lens = rng.integers(k_lo, k_hi + 1, size=count)
    con_off = np.zeros(count + 1, dtype=np.int64)
    np.cumsum(lens, out=con_off[1:])
    lits = np.empty(int(con_off[-1]), dtype=np.int32)
    tps = rng.choice(np.asarray(types, dtype=np.int32), size=count)
    params = np.zeros(count, dtype=np.int32)
    for c in range(count):
        k = int(lens[c])
        v = rng.choice(n, size=k, replace=False) + 1
        s = rng.integers(0, 2, size=k).astype(bool)
        v = v.astype(np.int32)
        v[s] = -v[s]
        lits[con_off[c]:con_off[c + 1]] = v
        if tps[c] == XOR:
            params[c] = rng.integers(0, 2)
        elif tps[c] in (CARD_GE, CARD_LT, EK):
            params[c] = rng.integers(0, k + 2)
    return Instance(n=n, con_off=con_off, lits=lits, types=tps.astype(np.int32), params=params)
