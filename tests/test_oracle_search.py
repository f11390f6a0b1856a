"""Pins of the oracle's line search, partial-assignment slices and convergence
(Algorithm 1, Sec. 3.3, Sec. 3.4), and of the test-side Philox4x32-10 reference
that the GPU start-point test compares against.

The line search is pinned by hand-worked cases whose objective has a closed
form (a two-literal XOR has FE = y1*y2, a one-literal clause FE = y1, Sec. 2.1),
and by properties any correct backtracking search has: the chosen trial passes
the Armijo test, every earlier trial fails it, and the objective never rises.
"""
import numpy as np
import pytest

import oracle
from paper_2606_06641_amd import workloads

from philox_ref import philox4x32_10, uniform_pm1


class Inst:
    def __init__(self, n, cons, weights=None):
        self.n = n
        self.con_off = np.cumsum([0] + [len(c[2]) for c in cons]).astype(np.int64)
        self.lits = np.array([l for c in cons for l in c[2]], dtype=np.int32)
        self.types = np.array([c[0] for c in cons], dtype=np.int32)
        self.params = np.array([c[1] for c in cons], dtype=np.int32)
        self.weights = weights


XOR2 = Inst(2, [(oracle.XOR, 1, [1, 2])])          # F = x1 * x2
CLAUSE1 = Inst(1, [(oracle.OR, 0, [1])])           # F = x1


def test_xor2_objective_is_the_product():
    x = np.array([[0.5, -0.3, 0.9], [0.4, 0.7, -1.0]])
    np.testing.assert_allclose(oracle.eval(XOR2, x)["obj"], x[0] * x[1], rtol=0, atol=1e-15)


def test_hand_worked_backtracking():
    """From (0.5, 0.4) with s = 2, beta = 1/2, c = 1/2: the step 2 lands on
    (-0.3, -0.6) with F = 0.18 > 0.2 - 0.41, rejected; the step 1 lands on
    (0.1, -0.1) with F = -0.01 <= 0.2 - 0.205, accepted."""
    r = oracle.line_search_step(XOR2, np.array([[0.5], [0.4]]), (2.0, 0.5, 0.5, 4))
    assert r["eta"][0] == 1.0
    np.testing.assert_allclose(r["x"][:, 0], [0.1, -0.1], atol=1e-15)
    np.testing.assert_allclose(r["margin"][:2, 0], [-0.39, 0.005], atol=1e-15)


def test_no_trial_accepted_means_no_step():
    r = oracle.line_search_step(XOR2, np.array([[0.5], [0.4]]), (2.0, 0.5, 0.5, 1))
    assert r["eta"][0] == 0.0
    np.testing.assert_array_equal(r["x"][:, 0], [0.5, 0.4])


def test_projection_arc_accepts_the_clipped_step():
    """F = x1 from 0.5 with s = 4: the trial clips to -1, F drops by 1.5 and
    <g, xt - x> = -1.5, so the first trial passes for any c < 1."""
    r = oracle.line_search_step(CLAUSE1, np.array([[0.5]]), (4.0, 0.5, 0.9, 3))
    assert r["eta"][0] == 4.0 and r["x"][0, 0] == -1.0


def test_fixed_variable_is_held_and_left_out_of_the_test():
    """x2 fixed: only x1 moves (g1 = x2 = 0.4); from x1 = 0.5 with s = 2 the
    trial lands on -0.3 with F = -0.12 and <g, xt - x> = -0.32."""
    r = oracle.line_search_step(XOR2, np.array([[0.5], [0.4]]), (2.0, 0.5, 0.5, 3),
                                fixed=np.array([0, 1], dtype=np.uint8))
    assert r["eta"][0] == 2.0
    np.testing.assert_allclose(r["x"][:, 0], [-0.3, 0.4], atol=1e-15)
    np.testing.assert_allclose(r["margin"][0, 0], 0.2 - 0.16 + 0.12, atol=1e-15)


@pytest.mark.parametrize("seed", [1, 2, 3])
def test_backtracking_properties(seed):
    rng = np.random.default_rng(seed)
    inst = workloads.random_instance(rng, n=40, count=120, k_lo=2, k_hi=9)
    x = rng.uniform(-1, 1, size=(inst.n, 64))
    search = (4.0, 0.5, 1e-3, 10)
    r = oracle.line_search_step(inst, x, search)
    for b in range(x.shape[1]):
        j = np.nonzero(r["eta_trials"] == r["eta"][b])[0]
        if r["eta"][b] == 0.0:
            assert (r["margin"][:, b] < 0).all()
            continue
        j = int(j[0])
        assert r["margin"][j, b] >= 0 and (r["margin"][:j, b] < 0).all()
    # the objective never rises (the accepted step has <g, xt - x> <= 0)
    f1 = oracle.eval(inst, r["x"], grad=False)["obj"]
    assert (f1 <= r["f0"] + 1e-12).all()
    # eta_j = s * beta^j
    np.testing.assert_allclose(r["eta_trials"], 4.0 * 0.5 ** np.arange(10), rtol=0, atol=0)


def test_search_descent_solves_a_planted_instance():
    inst = workloads.planted_3sat(n=60, m=220, instance=5)
    rng = np.random.default_rng(5)
    res = oracle.pgd_search(inst, rng.uniform(-1, 1, size=(inst.n, 32)), (2.0, 0.5, 1e-4, 8), steps=60)
    assert (res["unsat"][res["done"] == 1] == 0).all()
    assert (res["done"] == 1).any()
    assert (oracle.unsat_count(inst, res["x"])[res["done"] == 1] == 0).all()


def test_unsat_count_matches_the_fp32_verifier():
    inst = workloads.planted_3sat(n=50, m=200, instance=7)
    x = np.random.default_rng(7).uniform(-1, 1, size=(inst.n, 70)).astype(np.float32)
    np.testing.assert_array_equal(oracle.unsat_count(inst, x.astype(np.float64)), oracle.verify(inst, x))


def test_fixed_columns_divides_restarts_evenly():
    f = np.array([[1, 0, 0], [0, 1, 0], [0, 0, 1]], dtype=np.uint8)
    m = oracle.fixed_columns(f, 3, 10)
    # rows used by restarts 0..9: 0,0,0,0,1,1,1,2,2,2
    np.testing.assert_array_equal(m[:, :4], np.repeat([[1], [0], [0]], 4, axis=1).astype(bool))
    np.testing.assert_array_equal(m[:, 4:7], np.repeat([[0], [1], [0]], 3, axis=1).astype(bool))
    np.testing.assert_array_equal(m[:, 7:], np.repeat([[0], [0], [1]], 3, axis=1).astype(bool))
    assert not oracle.fixed_columns(None, 3, 5).any()


def test_pgd_slices_hold_each_rows_variables():
    inst = workloads.planted_3sat(n=30, m=100, instance=9)
    x0 = np.random.default_rng(9).uniform(-1, 1, size=(inst.n, 12))
    f = np.zeros((3, inst.n), dtype=np.uint8)
    f[0, :5] = 1
    f[1, 5:10] = 1
    f[2, 10:15] = 1
    r = oracle.pgd(inst, x0, 0.1, 5, fixed=f)
    held = oracle.fixed_columns(f, inst.n, 12)
    np.testing.assert_array_equal(r["x"][held], x0[held])
    # same result as running each slice alone
    r1 = oracle.pgd(inst, x0[:, 4:8], 0.1, 5, fixed=f[1])
    np.testing.assert_array_equal(r["x"][:, 4:8], r1["x"])


def test_constant_step_converges_when_delta_exceeds_it():
    inst = workloads.planted_3sat(n=30, m=100, instance=11)
    x0 = np.random.default_rng(11).uniform(-1, 1, size=(inst.n, 8))
    a = oracle.pgd(inst, x0, 0.1, 20, delta=0.2)
    b = oracle.pgd(inst, x0, 0.1, 1)
    np.testing.assert_array_equal(a["x"], b["x"])


# ---- Philox4x32-10 reference (test side) -----------------------------------------------

def test_philox_known_answers():
    """Known-answer vectors of Philox4x32-10 published with the generator's
    reference implementation (Random123): zero counter and key, all-ones counter
    and key, and the hexadecimal digits of pi."""
    assert philox4x32_10((0, 0, 0, 0), (0, 0)) == (0x6627e8d5, 0xe169c58d, 0xbc57ac4c, 0x9b00dbd8)
    m = 0xffffffff
    assert philox4x32_10((m, m, m, m), (m, m)) == (0x408f276d, 0x41c83b0e, 0xa20bc7c6, 0x6d5451fd)
    assert philox4x32_10((0x243f6a88, 0x85a308d3, 0x13198a2e, 0x03707344), (0xa4093822, 0x299f31d0)) == \
        (0xd16cfe09, 0x94fdcceb, 0x5001e420, 0x24126ea1)


def test_uniform_map_is_exact_and_in_range():
    u = uniform_pm1(np.array([0, 255, 256, 0xffffffff], dtype=np.uint64))
    assert u.dtype == np.float32
    np.testing.assert_array_equal(u, np.array([-1.0, -1.0, -1.0 + 2.0 ** -23, 1.0 - 2.0 ** -23], dtype=np.float32))


def test_vectorised_philox_matches_scalar():
    from philox_ref import philox_first_words
    rng = np.random.default_rng(3)
    c0 = rng.integers(0, 2 ** 32, size=50, dtype=np.uint64)
    c1 = rng.integers(0, 2 ** 32, size=50, dtype=np.uint64)
    key = (0x12345678, 0x9abcdef0)
    got = philox_first_words(c0, c1, key)
    want = [philox4x32_10((int(a), int(b), 0, 0), key)[0] for a, b in zip(c0, c1)]
    np.testing.assert_array_equal(got, np.array(want, dtype=np.uint64))


# x1 alone in a clause (F = x1: it falls by lr per step until the bound -1);
# x2, x3 in an odd and an even XOR, one of which is always violated and whose
# expansions cancel (zero gradient): the input never verifies.
DRIFT = Inst(3, [(oracle.OR, 0, [1]), (oracle.XOR, 1, [2, 3]), (oracle.XOR, 0, [2, 3])])


@pytest.mark.parametrize("eps,t_conv", [(0.5, 1), (0.2, 7), (0.05, 8)])
def test_location_rule_by_hand(eps, t_conv):
    """From x1 = 0.9 with lr = 0.3 the moves are 0.3 six times (x1: 0.6 .. -0.9),
    then 0.1 onto the bound, then 0: the restart converges at the first
    iteration whose move is below epsilon, and its point stays there."""
    x0 = np.array([[0.9], [0.25], [-0.5]])
    for steps in (t_conv - 1, t_conv, t_conv + 5):
        r = oracle.pgd(DRIFT, x0, 0.3, steps, epsilon=eps)
        assert r["first_sat"][0] == -1 and r["unsat"][0] >= 1
        assert r["done"][0] == (2 if steps >= t_conv else 0)
        want = max(-1.0, 0.9 - 0.3 * min(steps, t_conv))
        np.testing.assert_allclose(r["x"][:, 0], [want, 0.25, -0.5], atol=1e-12)


def test_location_rule_off_and_fixed():
    """epsilon = 0 keeps the plain run; a held x1 means no move at all, so the
    restart converges at the first iteration."""
    x0 = np.array([[0.9], [0.25], [-0.5]])
    plain = oracle.pgd(DRIFT, x0, 0.3, 9)
    assert "done" not in plain and plain["x"][0, 0] == -1.0
    r = oracle.pgd(DRIFT, x0, 0.3, 9, fixed=np.array([1, 0, 0], np.uint8), epsilon=1e-9)
    assert r["done"][0] == 2
    np.testing.assert_array_equal(r["x"][:, 0], x0[:, 0])


def test_location_rule_agrees_with_the_plain_run_until_it_stops():
    inst = workloads.planted_3sat(n=60, m=240, instance=5)
    x0 = workloads.uniform_x0(inst.n, 12, workload=1, instance=5).astype(np.float64)
    a = oracle.pgd(inst, x0, 0.1, 40, epsilon=1e-12)       # moves of exactly 0 only
    b = oracle.pgd(inst, x0, 0.1, 40)
    running = a["done"] != 2
    np.testing.assert_allclose(a["x"][:, running], b["x"][:, running], atol=1e-12)
    np.testing.assert_array_equal(a["first_sat"], b["first_sat"])


def test_line_search_location_rule():
    """The line search on F = x1 from 0.5 with s = 4 lands on the bound at once
    (move 1.5); nothing moves after that, and the clause is then satisfied, so
    the restart verifies rather than converges; with the XOR pair beside it the
    second iteration's zero move converges it."""
    r = oracle.pgd_search(CLAUSE1, np.array([[0.5]]), (4.0, 0.5, 0.9, 3), 5, epsilon=0.1)
    assert r["done"][0] == 1 and r["first_sat"][0] == 1
    r = oracle.pgd_search(DRIFT, np.array([[0.5], [0.25], [-0.5]]), (4.0, 0.5, 0.9, 3), 5, epsilon=0.1)
    assert r["done"][0] == 2 and r["x"][0, 0] == -1.0


# Two one-literal clauses: x1 must be True (F gains x1) and x2 False (the
# negated literal gives -x2), so F = x1 - x2 and the gradient is (1, -1) at every
# point.  Every value below is a multiple of 1/4, so each step is exact in FP64.
UNITS2 = Inst(2, [(oracle.OR, 0, [1]), (oracle.OR, 0, [-2])])


@pytest.mark.parametrize("steps", [0, 1, 2, 3, 4, 9])
def test_constant_step_first_sat_by_hand(steps):
    """Algorithm 1 with lr = 1/4.  Restart 0 from x = (3/4, 1/2): x1 moves to 1/2,
    1/4, 0, -1/4 while x2 (False throughout) climbs to the bound 1; the point
    x1 = 0 is False (the rounding tie), so the restart first verifies at
    iteration 4, and then stays put (a finished candidate does no-ops).
    Restart 1 starts at a satisfying corner (first_sat 0, never moves).
    Restart 2 from (-1/4, -1/2): x1 is True from the start (and keeps falling),
    x2 is True at -1/2 and -1/4 and False at 0, so it verifies at iteration 2."""
    x0 = np.array([[0.75, -1.0, -0.25],
                   [0.5, 1.0, -0.5]])
    r = oracle.pgd(UNITS2, x0, 0.25, steps)
    want_first = [4 if steps >= 4 else -1, 0, 2 if steps >= 2 else -1]
    np.testing.assert_array_equal(r["first_sat"], want_first)
    x1 = [0.75 - 0.25 * min(steps, 4), -1.0, -0.25 - 0.25 * min(steps, 2)]
    x2 = [min(1.0, 0.5 + 0.25 * min(steps, 4)), 1.0, -0.5 + 0.25 * min(steps, 2)]
    np.testing.assert_array_equal(r["x"], np.array([x1, x2]))
    np.testing.assert_array_equal(r["unsat"], [0 if f >= 0 else 1 for f in want_first])


@pytest.mark.parametrize("steps", [0, 1, 2, 3, 6])
def test_momentum_by_hand(steps):
    """Heavy-ball momentum with lr = 1/4, mu = 1/2 on the clauses (x1), (not x2)
    (gradient (1, -1) everywhere), in exact dyadic arithmetic.  Restart 0 from
    (3/4, 1/2): v = (1, -1), (3/2, -3/2), (7/4, -7/4) and x1 = 1/2, 1/8, -5/16,
    so it verifies at iteration 3; x2 reaches the bound 1 at iteration 2 and stays
    there while its velocity keeps growing.  Restart 1 starts satisfied.
    Restart 2 from (1/4, 1): x1 = 0 (False, the rounding tie) after one step and
    -3/8 after two."""
    x0 = np.array([[0.75, -1.0, 0.25],
                   [0.5, 1.0, 1.0]])
    r = oracle.pgd_momentum(UNITS2, x0, 0.25, 0.5, steps)
    want_first = [3 if steps >= 3 else -1, 0, 2 if steps >= 2 else -1]
    np.testing.assert_array_equal(r["first_sat"], want_first)
    v0_traj = [0.0, 1.0, 1.5, 1.75]
    x0_traj = [0.75, 0.5, 0.125, -0.3125]
    x20_traj = [0.5, 0.75, 1.0, 1.0]
    v2_traj = [0.0, 1.0, 1.5]
    x2_traj = [0.25, 0.0, -0.375]
    t0, t2 = min(steps, 3), min(steps, 2)
    np.testing.assert_array_equal(r["x"], [[x0_traj[t0], -1.0, x2_traj[t2]],
                                           [x20_traj[t0], 1.0, 1.0]])
    np.testing.assert_array_equal(r["v"], [[v0_traj[t0], 0.0, v2_traj[t2]],
                                           [-v0_traj[t0], 0.0, -v2_traj[t2]]])
    np.testing.assert_array_equal(r["done"], [1 if f >= 0 else 0 for f in want_first])


def test_momentum_holds_fixed_variables():
    """A fixed variable keeps both its value and its velocity; the others move as
    without it (here their gradients do not depend on it)."""
    x0 = np.array([[0.75], [0.5]])
    free = oracle.pgd_momentum(UNITS2, x0, 0.25, 0.5, 3)
    held = oracle.pgd_momentum(UNITS2, x0, 0.25, 0.5, 3, fixed=np.array([0, 1], np.uint8))
    assert held["x"][1, 0] == 0.5 and held["v"][1, 0] == 0.0
    assert held["x"][0, 0] == free["x"][0, 0] and held["v"][0, 0] == free["v"][0, 0]
    assert held["first_sat"][0] == free["first_sat"][0] == 3


def test_momentum_zero_is_algorithm_1():
    """mu = 0 is PGD with a constant step: the same points, counts and first
    verifications as the C oracle's Algorithm 1 (exact FP64 equality), and the
    velocity is the last gradient taken."""
    rng = np.random.default_rng(77)
    inst = workloads.random_instance(rng, n=60, count=80, k_lo=2, k_hi=9)
    x0 = rng.uniform(-1, 1, size=(inst.n, 12))
    for steps in (1, 4, 15):
        a = oracle.pgd_momentum(inst, x0, 0.1, 0.0, steps)
        b = oracle.pgd(inst, x0, 0.1, steps)
        np.testing.assert_array_equal(a["x"], b["x"])
        np.testing.assert_array_equal(a["unsat"], b["unsat"])
        np.testing.assert_array_equal(a["first_sat"], b["first_sat"])
    one = oracle.pgd_momentum(inst, x0, 0.1, 0.9, 1)
    g = oracle.eval(inst, x0, grad=True)["grad"]
    running = one["first_sat"] != 0
    np.testing.assert_array_equal(one["v"][:, running], g[:, running])
