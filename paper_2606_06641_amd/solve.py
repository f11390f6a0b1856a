"""Command-line solver: read DIMACS CNF or the hybrid format (App. A), run
Algorithm 1 on the GPU over a batch of restarts, and print the result in the
DIMACS output convention.

    python -m paper_2606_06641_amd.solve FILE [--batch B] [--iters T] ...

Output: comment lines ("c ..."), then "s SATISFIABLE" with the assignment on
"v" lines ending in 0, or "s UNKNOWN" (the method is incomplete: it cannot
prove unsatisfiability, Sec. 5) with the best restart's unsatisfied-constraint
count -- with --best also an "o" line with that count and the best restart's
assignment, the best-effort answer of Sec. 5 -- or "s UNSATISFIABLE" when the
reader's simplifications already prove it (conflicting units).  Exit status
10 / 20 / 0 as is customary for SAT solvers.

Partial assignments (Sec. 3.4) come from --partial FILE: one assignment per
line, literals ending in 0 (a positive literal fixes its variable True); the
restarts are divided evenly among them and the units found by the reader are
folded into each.  --decompose L splits every OR, XOR, NAE, AMO and EO
constraint longer than L literals into a chain of pieces joined by auxiliary
variables (Sec. 5), so that such constraints longer than the kernels' 1,024
maximum can be solved too; the search runs on the decomposed instance and the
answer is its restriction to the input's variables.  Every step of the search
runs in the library's kernels.
"""
import argparse
import sys
import time

import numpy as np
import torch

from . import afsat


def read_partials(path, n):
    rows = []
    with open(path) as f:
        for ln, line in enumerate(f, 1):
            toks = line.split()
            if not toks or toks[0] in ("c", "*"):
                continue
            if toks[-1] != "0":
                raise ValueError("%s:%d: a partial assignment ends with 0" % (path, ln))
            row = np.zeros(n, dtype=np.int8)
            for t in toks[:-1]:
                lit = int(t)
                if lit == 0 or abs(lit) > n:
                    raise ValueError("%s:%d: literal %d out of range" % (path, ln, lit))
                if row[abs(lit) - 1] == (-1 if lit > 0 else 1):
                    raise ValueError("%s:%d: variable %d given both ways" % (path, ln, abs(lit)))
                row[abs(lit) - 1] = 1 if lit > 0 else -1
            rows.append(row)
    if not rows:
        raise ValueError("%s holds no partial assignment" % path)
    return np.stack(rows)


def assignment_lines(bits, width=20):
    lits = [(v + 1) if t else -(v + 1) for v, t in enumerate(bits)]
    out = []
    for i in range(0, len(lits), width):
        out.append("v " + " ".join(str(l) for l in lits[i:i + width]))
    out.append("v 0")
    return out


def main(argv=None, out=None):
    out = out or sys.stdout
    ap = argparse.ArgumentParser(prog="python -m paper_2606_06641_amd.solve", description=__doc__.split("\n\n")[0])
    ap.add_argument("file")
    ap.add_argument("--batch", type=int, default=1024, help="restarts searched together (B)")
    ap.add_argument("--iters", type=int, default=1000, help="iteration budget d")
    ap.add_argument("--lr", type=float, default=0.1, help="constant step length")
    ap.add_argument("--line-search", action="store_true", help="backtracking line search instead of the constant step")
    ap.add_argument("--max-step", type=float, default=1.0, help="line search: first trial step s")
    ap.add_argument("--shrink", type=float, default=0.5, help="line search: factor between trials")
    ap.add_argument("--armijo", type=float, default=1e-4, help="line search: sufficient-decrease constant")
    ap.add_argument("--trials", type=int, default=8, help="line search: trials per iteration")
    ap.add_argument("--momentum", type=float, default=0.0, metavar="MU",
                    help="heavy-ball momentum in [0, 1) in place of plain PGD steps")
    ap.add_argument("--delta", type=float, default=0.0, help="stop a restart once its step length < delta")
    ap.add_argument("--epsilon", type=float, default=0.0,
                    help="stop a restart once no variable of it moves by epsilon or more in an iteration")
    ap.add_argument("--poll", type=int, default=10, help="iterations between checks for a verified restart")
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--partial", help="file of partial assignments, one per line, ending in 0")
    ap.add_argument("--decompose", type=int, default=0, metavar="L",
                    help="split long OR/XOR/NAE/AMO/EO constraints into chains of pieces of at most L literals")
    ap.add_argument("--device", type=int, default=0)
    ap.add_argument("--no-graph", action="store_true", help="launch iterations one by one")
    ap.add_argument("--best", action="store_true",
                    help="when no restart verifies, print the best restart's assignment (best effort, "
                         "with its unsatisfied-constraint count on an 'o' line)")
    a = ap.parse_args(argv)
    if a.momentum and (a.line_search or a.delta or a.epsilon):
        raise SystemExit("--momentum takes a constant step (no --line-search, --delta or --epsilon)")
    if not 0.0 <= a.momentum < 1.0:
        raise SystemExit("--momentum must lie in [0, 1)")

    t0 = time.perf_counter()
    try:
        p = afsat.parse_file(a.file)
    except afsat.AfsError as e:
        if e.status == afsat.AFS_EUNSAT:
            print("c %s" % e, file=out)
            print("s UNSATISFIABLE", file=out)
            return 20
        raise
    print("c read %d variables, %d constraints (%d removed, %d units) in %.3f s"
          % (p.n, len(p.types), p.n_dropped, int((p.units != 0).sum()), time.perf_counter() - t0), file=out)
    try:
        vals = p.fold_units(read_partials(a.partial, p.n) if a.partial else None)
    except afsat.AfsError as e:
        print("c %s" % e, file=out)
        print("s UNSATISFIABLE" if not a.partial else "s UNKNOWN", file=out)
        return 20 if not a.partial else 0
    B = max(a.batch, vals.shape[0])
    if len(p.types) == 0:
        # every constraint was simplified away: the units alone satisfy the input
        bits = vals[0] > 0
        print("s SATISFIABLE", file=out)
        for line in assignment_lines(bits):
            print(line, file=out)
        return 10
    form = p
    if a.decompose:
        form = afsat.decompose(p, a.decompose)
        vals = np.ascontiguousarray(np.pad(vals, ((0, 0), (0, form.n - p.n))))    # links start free
        print("c decomposed into %d variables, %d constraints of at most %d literals"
              % (form.n, len(form.types), int(np.diff(form.con_off).max())), file=out)
    inst = afsat.Instance.from_arrays(form, device=a.device)
    dev = torch.device("cuda", a.device)
    vd = torch.from_numpy(vals).to(dev)
    fixed = vd if (vals != 0).any() else None
    x = inst.init_points(B, a.seed, vd if fixed is not None else None)
    search = afsat.LineSearch(a.max_step, a.shrink, a.armijo, a.trials) if a.line_search else None
    t1 = time.perf_counter()
    st = inst.pgd(x, a.lr, a.iters, fixed=fixed, poll=a.poll, stop_on_sat=True, graph=not a.no_graph,
                  search=search, delta=a.delta, epsilon=a.epsilon, momentum=a.momentum)
    torch.cuda.synchronize(dev)
    dt = time.perf_counter() - t1
    unsat = st["unsat"].cpu().numpy()
    done = st["done"].cpu().numpy()
    print("c %d iterations over %d restarts in %.3f s" % (st["iters"], B, dt), file=out)
    sat = np.nonzero(done == 1)[0]
    if sat.size:
        b = int(sat[np.argmin(st["first_sat"].cpu().numpy()[sat])])
        bits = (x[:p.n, b] < 0).cpu().numpy()
        print("c restart %d verified at iteration %d" % (b, int(st["first_sat"][b])), file=out)
        print("s SATISFIABLE", file=out)
        for line in assignment_lines(bits):
            print(line, file=out)
        return 10
    b = int(np.argmin(unsat))
    best = int(unsat[b])
    if a.decompose:
        print("c best restart %d leaves %d pieces unsatisfied" % (b, best), file=out)
        best = input_unsat(p, x[:p.n, b:b + 1].contiguous(), a.device)
        if best is None:
            print("c (the input has constraints beyond the kernels' length limit: its own count is not taken)",
                  file=out)
            best = int(unsat[b])
    if best is not None:
        print("c best restart %d leaves %d constraints unsatisfied" % (b, best), file=out)
    if a.best:
        print("o %d" % best, file=out)
    print("s UNKNOWN", file=out)
    if a.best:
        for line in assignment_lines((x[:p.n, b] < 0).cpu().numpy()):
            print(line, file=out)
    return 0


def input_unsat(p, xb, device):
    """Unsatisfied constraints of the parsed input under the points xb (n, 1),
    counted by the library's verification kernels, or None when the input holds
    a constraint longer than they take."""
    if len(p.types) and int(np.diff(p.con_off).max()) > afsat.MAX_LEN:
        return None
    return int(afsat.Instance.from_arrays(p, device=device).round_verify(xb)[0])


if __name__ == "__main__":
    sys.exit(main())
