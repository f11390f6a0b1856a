"""Long-constraint decomposition, plain Python (test infrastructure).

Only the tests and the benchmark's CPU-baseline leg may import this module; it
shares no code with the GPU library.

Sec. 5 (constraint length ceiling) proposes replacing a long constraint by
O(k / 50) shorter equivalent constraints of the same type, available for every
type but EK and CARD.  The reading taken here: a chain.  A constraint of type OR,
XOR, NAE, AMO or EO with k > max_len literals gets p = ceil((k - 2) / (max_len - 2))
pieces -- the fewest of at most max_len literals, since the chain adds two
literals per link -- over consecutive groups G_1 .. G_p of its literals, joined
by new variables a_1 .. a_(p-1):

    OR, NAE, AMO, EO:  piece i = [-a_(i-1)] + G_i + [a_i]   (ends drop the missing link)
    XOR:               piece i = [ a_(i-1)] + G_i + [a_i],  parity 0 except the last

The k + 2(p - 1) literals are spread so that the pieces' lengths differ by at
most one, the longer pieces first.  Each piece keeps its constraint's weight.
EK, CARD and short constraints are copied.

``aux_values`` completes an assignment of the original variables to the
auxiliary ones by dynamic programming over each chain, judging every piece
with the oracle's own predicate (``sat``), so equivalence can be checked at any
length without trusting a per-type rule.
"""
import numpy as np

from . import AMO, EO, NAE, OR, XOR, sat

CHAIN_TYPES = (OR, XOR, NAE, AMO, EO)


def n_pieces(ctype, k, max_len):
    """Pieces of a constraint of type ``ctype`` and length ``k``."""
    if ctype not in CHAIN_TYPES or k <= max_len:
        return 1
    return -(-(k - 2) // (max_len - 2))


def _group_sizes(k, p):
    total = k + 2 * (p - 1)
    lengths = [total // p + (1 if i < total % p else 0) for i in range(p)]
    links = [(i > 0) + (i < p - 1) for i in range(p)]
    return [lengths[i] - links[i] for i in range(p)]


def decompose(inst, max_len):
    """Decomposed arrays of ``inst``: dict with n, con_off, lits, types, params,
    weights (None when inst has none) and origin."""
    if not 3 <= max_len <= 1024:
        raise ValueError("max_len must be in [3, 1024]")
    n = int(inst.n)
    con_off = np.asarray(inst.con_off, dtype=np.int64)
    lits = np.asarray(inst.lits, dtype=np.int64)
    types = np.asarray(inst.types, dtype=np.int64)
    params = getattr(inst, "params", None)
    params = np.zeros(len(types), np.int64) if params is None else np.asarray(params, dtype=np.int64)
    weights = getattr(inst, "weights", None)
    rows, out_types, out_params, out_w, origin = [], [], [], [], []
    next_var = n
    for c in range(len(types)):
        cl = [int(v) for v in lits[con_off[c]:con_off[c + 1]]]
        ctype, k = int(types[c]), len(cl)
        p = n_pieces(ctype, k, max_len)
        if p == 1:
            rows.append(cl)
            out_types.append(ctype)
            out_params.append(int(params[c]))
            origin.append(c)
            continue
        aux = list(range(next_var + 1, next_var + p))      # a_1 .. a_(p-1)
        next_var += p - 1
        groups, start = [], 0
        for size in _group_sizes(k, p):
            groups.append(cl[start:start + size])
            start += size
        for i, g in enumerate(groups):
            row = []
            if i > 0:
                row.append(aux[i - 1] if ctype == XOR else -aux[i - 1])
            row += g
            if i < p - 1:
                row.append(aux[i])
            rows.append(row)
            out_types.append(ctype)
            out_params.append((int(params[c]) & 1 if i == p - 1 else 0) if ctype == XOR else int(params[c]))
            origin.append(c)
    offs = np.zeros(len(rows) + 1, dtype=np.int64)
    offs[1:] = np.cumsum([len(r) for r in rows])
    flat = np.array([v for r in rows for v in r], dtype=np.int32)
    w = None
    if weights is not None:
        w = np.asarray(weights, dtype=np.float32)[np.array(origin, dtype=np.int64)]
    return dict(n=next_var, con_off=offs, lits=flat, types=np.array(out_types, np.int32),
                params=np.array(out_params, np.int32), weights=w, origin=np.array(origin, np.int32))


def _true_count(row, value):
    """Number of true literals of ``row`` under ``value`` (dict var -> bool)."""
    return sum(1 for l in row if value[abs(l)] == (l > 0))


def aux_values(inst, dec, bits):
    """Values of the auxiliary variables that satisfy every piece of each
    decomposed constraint whose original holds under ``bits`` (bool [n_orig],
    True = true), by a forward reachability pass over the two values of each
    link and a backward choice; links of violated constraints are set False.
    Returns bool [dec n]."""
    n0 = int(inst.n)
    out = np.zeros(dec["n"], dtype=bool)
    out[:n0] = np.asarray(bits, dtype=bool)[:n0]
    origin, offs, flat = dec["origin"], dec["con_off"], dec["lits"]
    c = 0
    while c < len(origin):
        e = c
        while e + 1 < len(origin) and origin[e + 1] == origin[c]:
            e += 1
        if e > c:
            _solve_chain(out, [list(flat[offs[i]:offs[i + 1]]) for i in range(c, e + 1)],
                         int(dec["types"][c]), [int(dec["params"][i]) for i in range(c, e + 1)])
        c = e + 1
    return out


def _solve_chain(out, rows, ctype, params):
    p = len(rows)
    links = [abs(int(rows[i][-1])) for i in range(p - 1)]      # a_i closes piece i

    def piece_ok(i, prev, cur):
        value = {abs(int(l)): bool(out[abs(int(l)) - 1]) for l in rows[i]}
        if i > 0:
            value[links[i - 1]] = prev
        if i < p - 1:
            value[links[i]] = cur
        return sat(ctype, len(rows[i]), params[i], _true_count([int(l) for l in rows[i]], value))

    # reach[i][v]: some values of a_1 .. a_i with a_i = v satisfy pieces 1 .. i
    reach = [[piece_ok(0, None, v) for v in (False, True)]]
    for i in range(1, p - 1):
        reach.append([any(reach[i - 1][u] and piece_ok(i, bool(u), v) for u in (0, 1)) for v in (False, True)])
    last = [reach[p - 2][u] and piece_ok(p - 1, bool(u), None) for u in (0, 1)]
    if not any(last):
        return
    v = 0 if last[0] else 1
    for i in range(p - 2, -1, -1):
        out[links[i] - 1] = bool(v)
        if i == 0:
            break
        v = next(u for u in (0, 1) if reach[i - 1][u] and piece_ok(i, bool(u), bool(v)))
