"""GPU parity: the HIP path through the C ABI against the FP64 oracle.

Every comparison feeds both sides the same FP32 points (the oracle widens them
exactly to FP64).  Tolerances are per length bucket (see parity.py); rounding,
verification and step bookkeeping are compared bit for bit.
"""
import os
import sys

import numpy as np
import pytest
import torch

import oracle
import parity
from paper_2606_06641_amd import afsat
from paper_2606_06641_amd import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    afsat.lib()          # raises if the HIP library is missing


def log(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def check(inst, x32, label):
    log("case:", label, "n=%d C=%d L=%d B=%d" % (inst.n, inst.n_cons, inst.n_lits, x32.shape[1]))
    d = afsat.Instance.from_arrays(inst)
    gpu = parity.gpu_eval(d, x32)
    orc = oracle.eval(inst, x32, fe=True, adj=True, grad=True)
    rows = parity.compare(inst, d, gpu, orc, label)
    log(parity.format_rows(rows))
    return d, gpu, orc


def adversarial_points(n, rng):
    cols = [np.ones(n), -np.ones(n), np.zeros(n),
            (1 - 1e-3) * np.ones(n), -(1 - 1e-3) * np.ones(n),
            rng.choice([-1.0, 1.0], size=n),
            rng.choice([-1.0, 1.0], size=n) * (1 - 1e-3),
            rng.choice([-1.0, 1.0], size=n) * (1 - rng.uniform(0, 1e-2, size=n))]
    c = rng.choice([-1.0, 1.0], size=n)
    c[rng.choice(n, size=max(1, n // 10), replace=False)] = rng.uniform(-1e-3, 1e-3, size=max(1, n // 10))
    cols.append(c)
    return np.stack(cols, axis=1).astype(np.float32)


@pytest.mark.parametrize("B", [37, 64, 300])
def test_short_all_types_ragged_batch(B):
    """Every type, lengths 1-16, weighted; B = 37 takes one restart per lane, B = 64
    and 300 four restarts per lane for k <= 8 (300 leaves a partial wave)."""
    rng = np.random.default_rng(10)
    inst = W.random_instance(rng, n=300, count=500, k_lo=1, k_hi=16)
    inst.weights = rng.uniform(0.5, 2.0, size=inst.n_cons).astype(np.float32)
    x = rng.uniform(-1, 1, size=(inst.n, B)).astype(np.float32)
    check(inst, x, "short k1-16 B=%d weighted" % B)


def test_long_every_bucket_shape():
    rng = np.random.default_rng(11)
    ks = [17, 24, 25, 32, 33, 48, 49, 64, 65, 96, 97, 128, 129, 192, 193, 256, 257, 384, 385, 512,
          513, 768, 769, 1000, 1024]
    parts = []
    for k in ks:
        parts.append(W.random_instance(rng, n=1500, count=3, k_lo=k, k_hi=k))
    inst = concat(parts, n=1500)
    inst.weights = rng.uniform(0.5, 2.0, size=inst.n_cons).astype(np.float32)
    x = rng.uniform(-1, 1, size=(inst.n, 70)).astype(np.float32)
    check(inst, x, "long k17-1024 B=70 weighted")


@pytest.mark.parametrize("J", [2, 4, 8, 16, 32, 64])
def test_every_segment_kernel_shape(J):
    """Each (lanes J, literals per lane S) instantiation, forced through the shape
    option, on lengths that fill it exactly, leave one lane short, and leave most
    lanes padding."""
    rng = np.random.default_rng(100 + J)
    for S in range(4, 33, 2):
        cap = J * S
        if cap > 1024 or cap <= 16:
            continue
        ks = sorted({cap, max(17, cap - 5), max(17, cap // 2 + 1)})
        parts = [W.random_instance(rng, n=1200, count=2, k_lo=k, k_hi=k) for k in ks]
        inst = concat(parts, n=1200)
        x = rng.uniform(-1, 1, size=(inst.n, 70)).astype(np.float32)
        x[:, :3] = np.sign(x[:, :3]) * (1 - 1e-3)
        log("case: forced shape J=%d S=%d lengths %s" % (J, S, ks))
        d = afsat.Instance.from_arrays(inst, shapes=[(cap, J, S)])
        assert all((b.lanes_per_restart, b.lits_per_lane) == (J, S) for b in d.buckets())
        gpu = parity.gpu_eval(d, x)
        orc = oracle.eval(inst, x, fe=True, adj=True, grad=True)
        parity.compare(inst, d, gpu, orc, "J=%d S=%d" % (J, S))


@pytest.mark.parametrize("J,S,tile", [(2, 12, 5), (4, 22, 4), (8, 26, 4), (8, 32, 2), (16, 14, 4), (32, 30, 2)])
def test_segment_kernel_uneven_tiles(J, S, tile):
    """Segment kernels with several constraints per work tile, the last tile
    ragged (7 constraints of each of three lengths), through the shape option's
    tile; B = 70 leaves a ragged last restart group."""
    rng = np.random.default_rng(300 + J + S)
    cap = J * S
    ks = sorted({cap, cap - 3, max(17, cap // 2 + 1)})
    inst = concat([W.random_instance(rng, n=1500, count=7, k_lo=k, k_hi=k) for k in ks], n=1500)
    x = rng.uniform(-1, 1, size=(inst.n, 70)).astype(np.float32)
    d = afsat.Instance.from_arrays(inst, shapes=[(cap, J, S, tile)])
    assert all((b.lanes_per_restart, b.lits_per_lane, b.tile) == (J, S, tile) for b in d.buckets())
    log("case: J=%d S=%d tile %d lengths %s" % (J, S, tile, ks))
    parity.compare(inst, d, parity.gpu_eval(d, x), oracle.eval(inst, x, fe=True, adj=True, grad=True),
                   "J=%d S=%d tile %d" % (J, S, tile))


def test_autotuner_shapes_are_valid_and_exact(tmp_path):
    """The tuned shapes cover their ranges, give results within the parity bar,
    and the cache file round-trips: a second call finds every range cached.
    With tiles the one-lane restarts per lane and every tile are tuned; without,
    they stay at the defaults (0) and one-lane lengths are not timed."""
    from paper_2606_06641_amd import autotune
    rng = np.random.default_rng(21)
    inst = concat([W.random_instance(rng, n=800, count=6, k_lo=20, k_hi=150),
                   W.random_instance(rng, n=800, count=50, k_lo=2, k_hi=8)], n=800)
    cache = str(tmp_path / "shapes.txt")
    shapes, report = autotune.tune(inst, 64, reps=2, log=log, out_path=cache, tiles=True)
    assert shapes and all((S == kh if J == 1 else J * S >= kh) for kh, J, S, _, _ in shapes)
    assert all(tile in (1, 2, 4, 8, 16) for _, _, _, tile, _ in shapes)
    assert all((rpl in (1, 2, 4) and 64 % rpl == 0) if J == 1 else rpl == 0 for _, J, _, _, rpl in shapes)
    assert [s[0] for s in shapes] == sorted(s[0] for s in shapes)
    lens = np.diff(inst.con_off)
    assert {kh for kh, J, _, _, _ in shapes if J == 1} == {int(k) for k in lens if k <= 16}
    assert not any(r["cached"] for r in report) and all(r["timed"] for r in report)
    shapes2, report2 = autotune.tune(inst, 64, reps=2, cache_path=cache, tiles=True)
    assert shapes2 == shapes and all(r["cached"] for r in report2)
    # shape only: the cached segment shapes at default tiles, one-lane lengths at
    # their defaults and not timed
    plain, report_p = autotune.tune(inst, 64, reps=2, cache_path=cache)
    assert plain == [(kh, J, S, 0, 0) for kh, J, S, _, _ in shapes]
    assert all(r["cached"] for r in report_p if r["shape"][0] != 1)
    assert not any(r["cached"] or r["timed"] for r in report_p if r["shape"][0] == 1)
    # an instance with more constraints in the same ranges: a range is taken from
    # the cache exactly when its constraint count has the same floor(log2) (size
    # class) as in the first instance, else tuned anew
    big = concat([W.random_instance(np.random.default_rng(22), n=800, count=24, k_lo=20, k_hi=150),
                  W.random_instance(np.random.default_rng(23), n=800, count=200, k_lo=2, k_hi=8)], n=800)
    _, report3 = autotune.tune(big, 64, reps=2, cache_path=cache, tiles=True)
    la, lb = np.diff(inst.con_off), np.diff(big.con_off)
    fresh = 0
    for r in report3:
        lo, hi = r["range"]
        ca, cb = int(((la >= lo) & (la <= hi)).sum()), int(((lb >= lo) & (lb <= hi)).sum())
        same = ca > 0 and int(np.log2(ca)) == int(np.log2(cb))
        assert r["cached"] == same, (r, ca, cb)
        fresh += not same
    assert fresh > 0
    # a shape-only tuning writes tile 0 for its segment ranges and nothing for
    # one-lane lengths; a later request for tiles tunes those ranges anew
    cache_p = str(tmp_path / "plain.txt")
    p1, r1 = autotune.tune(inst, 64, reps=2, out_path=cache_p)
    assert all(t == 0 and rp == 0 for _, _, _, t, rp in p1)
    assert all(r["timed"] for r in r1 if r["shape"][0] != 1)
    rows = [l.split() for l in open(cache_p) if not l.startswith("#")]
    assert rows and all(f[6] != "1" and f[8] == "0" and f[9] == "0" for f in rows)
    _, r2 = autotune.tune(inst, 64, reps=2, cache_path=cache_p, tiles=True)
    assert not any(r["cached"] for r in r2)
    # where the file read and the file written both hold a range, the file read
    # wins: a copy of the cache with every segment shape replaced by J = 64
    def wide(k_hi):
        S = max(4, -(-k_hi // 64))
        return 64, S + S % 2
    rows = [l.split() for l in open(cache) if not l.startswith("#")]
    other = str(tmp_path / "other.txt")
    with open(other, "w") as fh:
        for f in rows:
            if f[6] != "1":
                f[6], f[7] = (str(v) for v in wide(int(f[4])))
            fh.write(" ".join(f) + "\n")
    want = {kh: wide(kh) for kh, J, _, _, _ in shapes if J != 1}
    assert want and want != {kh: (J, S) for kh, J, S, _, _ in shapes if J != 1}
    got, report4 = autotune.tune(inst, 64, reps=2, cache_path=other, out_path=cache)
    assert all(r["cached"] for r in report4 if r["shape"][0] != 1)
    assert {kh: (J, S) for kh, J, S, _, _ in got if J != 1} == want
    x = rng.uniform(-1, 1, size=(inst.n, 64)).astype(np.float32)
    d = afsat.Instance.from_arrays(inst, shapes=shapes)
    conf = {kh: (tile, rpl) for kh, J, _, tile, rpl in shapes if J == 1}
    for b in d.buckets():
        if b.lanes_per_restart == 1:
            assert (b.tile, b.rpl) == conf[b.k_lo]
    orc = oracle.eval(inst, x, fe=True, adj=True, grad=True)
    parity.compare(inst, d, parity.gpu_eval(d, x), orc, "tuned")
    d = afsat.Instance.from_arrays(inst, shapes=got)
    parity.compare(inst, d, parity.gpu_eval(d, x), orc, "J = 64 shapes from the file read")


@pytest.mark.parametrize("rpl", [1, 2, 4])
def test_short_kernel_restarts_per_lane_and_tiles(rpl):
    """Every one-lane length at 1, 2 or 4 restarts per lane (4 only up to k = 8)
    with uneven tiles, against the oracle; B = 132 leaves a ragged last wave, and
    B = 130 (not a multiple of 4) makes the launch fall back to fewer restarts."""
    rng = np.random.default_rng(40 + rpl)
    ks = [k for k in range(1, 17) if rpl < 4 or k <= 8]
    inst = concat([W.random_instance(rng, n=300, count=13, k_lo=k, k_hi=k) for k in ks], n=300)
    shapes = [(k, 1, k, (1, 3, 16)[k % 3], rpl) for k in ks]
    d = afsat.Instance.from_arrays(inst, shapes=shapes)
    assert all(b.rpl == rpl for b in d.buckets())
    for B in (132, 130):
        x = rng.uniform(-1, 1, size=(inst.n, B)).astype(np.float32)
        orc = oracle.eval(inst, x, fe=True, adj=True, grad=True)
        parity.compare(inst, d, parity.gpu_eval(d, x), orc, "one-lane rpl=%d B=%d" % (rpl, B))


def test_adversarial_points():
    rng = np.random.default_rng(12)
    parts = [W.random_instance(rng, n=1200, count=60, k_lo=1, k_hi=16),
             W.random_instance(rng, n=1200, count=30, k_lo=17, k_hi=300),
             W.random_instance(rng, n=1200, count=6, k_lo=700, k_hi=1024)]
    inst = concat(parts, n=1200)
    x = adversarial_points(inst.n, rng)
    check(inst, x, "adversarial")


def test_single_restart_and_k1():
    rng = np.random.default_rng(13)
    inst = W.random_instance(rng, n=50, count=80, k_lo=1, k_hi=3)
    x = rng.uniform(-1, 1, size=(inst.n, 1)).astype(np.float32)
    check(inst, x, "B=1")
    x = rng.uniform(-1, 1, size=(inst.n, 65)).astype(np.float32)
    check(inst, x, "B=65")


def test_empty_instance():
    inst = W.Instance(n=7, con_off=np.zeros(1, np.int64), lits=np.zeros(0, np.int32),
                      types=np.zeros(0, np.int32), params=np.zeros(0, np.int32))
    d = afsat.Instance.from_arrays(inst)
    x = parity.to_dev(np.random.default_rng(0).uniform(-1, 1, size=(7, 5)))
    out = d.eval(x, obj=True, grad=True)
    assert torch.all(out["obj"] == 0) and torch.all(out["grad"] == 0)
    assert torch.all(d.round_verify(x) == 0)
    out = d.eval(x[:, :0].contiguous(), obj=True, grad=True)       # B = 0
    assert out["obj"].numel() == 0


def test_planted_3sat_n100_parity():
    inst = W.planted_3sat(instance=0)
    x = W.uniform_x0(inst.n, 32, workload=1)
    check(inst, x, "planted 3-SAT n=100 m=426 B=32")


def tuned_shapes(inst, B):
    """The kernel configurations bench.py runs: the package's tuned table (ranges
    missing from it are tuned on the device, into a temporary file so the shipped
    table stays as it is)."""
    import tempfile
    from paper_2606_06641_amd import autotune
    with tempfile.TemporaryDirectory() as tmp:
        shapes, _ = autotune.tune(inst, B, cache_path=autotune.DEFAULT_CACHE, out_path=os.path.join(tmp, "t.txt"),
                                  max_cons=400)
    return shapes


def test_mixed10k_full_size():
    """The mixed n = 10k instance at all 1,024 restarts with the tuned shapes the
    bench times: every FE, adjoint, gradient and objective entry."""
    inst = W.mixed_10k()
    B = 1024
    x = W.uniform_x0(inst.n, B, workload=2)
    shapes = tuned_shapes(inst, B)
    log("case: mixed n=10k B=1024 (all restarts), tuned shapes %s" % shapes)
    d = afsat.Instance.from_arrays(inst, shapes=shapes)
    gpu = parity.gpu_eval(d, x)
    orc = oracle.eval(inst, x, fe=True, adj=True, grad=True)
    rows = parity.compare(inst, d, gpu, orc, "mixed10k")
    log(parity.format_rows(rows))


def test_mixed10k_default_shapes():
    inst = W.mixed_10k()
    x = W.uniform_x0(inst.n, 256, workload=2, instance=1)
    check(inst, x, "mixed n=10k B=256, default shapes")


def test_longcard50k_sampled():
    """n=50k, 200k clauses, 1k CARD k 256-1024, B=512 on the GPU with the tuned
    shapes the bench times; the oracle checks 16 sampled restart columns
    (columns are independent)."""
    inst = W.long_card_50k()
    B = 512
    x = W.uniform_x0(inst.n, B, workload=4)
    shapes = tuned_shapes(inst, B)
    log("case: long-card n=50k B=512 sampled, tuned shapes %s" % shapes)
    d = afsat.Instance.from_arrays(inst, shapes=shapes)
    xd = parity.to_dev(x)
    out = d.eval(xd, obj=True, grad=True, fe=True, adj=True)
    cols = np.sort(np.random.default_rng(4).choice(B, size=16, replace=False))
    ci = torch.from_numpy(cols).cuda()
    sub = {k: v.index_select(v.dim() - 1, ci).cpu().numpy().astype(np.float64) for k, v in out.items()}
    del out
    torch.cuda.empty_cache()
    orc = oracle.eval(inst, x[:, cols], fe=True, adj=True, grad=True)
    rows = parity.compare(inst, d, sub, orc, "longcard50k sampled")
    log(parity.format_rows(rows))


def test_batch64_full_size_sampled():
    """The 64-instance uneven batch at full size (n log-uniform 500-50,000, 27.8M
    literal occurrences) and 256 restarts, packed block-diagonally with the tuned
    shapes exactly as the bench runs it; the oracle checks 8 sampled restart
    columns of FE, adjoints, gradient and objective (columns are independent), and
    the exact unsat counts of every part at those columns."""
    parts = W.uneven_batch()
    off = np.cumsum([0] + [p.n for p in parts])
    cat = concat([W.Instance(n=p.n, con_off=p.con_off, lits=np.where(p.lits > 0, p.lits + o, p.lits - o).astype(np.int32),
                             types=p.types, params=p.params) for p, o in zip(parts, off[:-1])], n=int(off[-1]))
    B = 256
    shapes = tuned_shapes(cat, B)
    Bt = afsat.Instance.batch(parts, shapes=shapes)
    x = W.uniform_x0(cat.n, B, workload=3)
    cols = np.sort(np.random.default_rng(33).choice(B, size=8, replace=False))
    log("case: batch64 full size, L=%d, B=%d, columns %s" % (cat.n_lits, B, cols.tolist()))
    xd = parity.to_dev(x)
    out = Bt.eval(xd, obj=True, grad=True, fe=True, adj=True)
    ci = torch.from_numpy(cols).cuda()
    gpu = {k: v.index_select(v.dim() - 1, ci).cpu().numpy().astype(np.float64) for k, v in out.items()}
    del out
    torch.cuda.empty_cache()
    orc = oracle.eval(cat, x[:, cols], fe=True, adj=True, grad=True)
    rows = parity.compare(cat, Bt, gpu, orc, "batch64 sampled")
    log(parity.format_rows(rows))
    u = Bt.round_verify(xd).cpu().numpy()
    for p, part in enumerate(parts):
        assert np.array_equal(u[p][cols], oracle.verify(part, x[off[p]:off[p + 1]][:, cols])), p


def test_verify_bit_exact():
    rng = np.random.default_rng(14)
    inst = W.random_instance(rng, n=200, count=900, k_lo=1, k_hi=40)
    x = rng.uniform(-1, 1, size=(inst.n, 77)).astype(np.float32)
    x[rng.random(x.shape) < 0.1] = 0.0
    x[rng.random(x.shape) < 0.05] = -0.0
    x[rng.random(x.shape) < 0.05] = 1.0
    x[rng.random(x.shape) < 0.05] = -1.0
    d = afsat.Instance.from_arrays(inst)
    unsat, bits = d.round_verify(parity.to_dev(x), want_bits=True)
    want_u, want_bits = oracle.verify(inst, x, want_bits=True)
    assert np.array_equal(unsat.cpu().numpy(), want_u)
    assert np.array_equal(bits.cpu().numpy().view(np.uint32), want_bits)


@pytest.mark.parametrize("B", [1, 33, 256, 2100])
def test_verify_word_layouts_and_parameters(B):
    """Restart counts that leave a partial 32-restart word, one word per lane group
    (B = 33), eight words (B = 256: eight constraints per wave) and more than 64
    words (B = 2100); lengths up to the maximum 1024; parameters outside 0..k
    (negative, k+1, huge) as well as inside."""
    rng = np.random.default_rng(B)
    n = 1100
    parts = [W.random_instance(rng, n=n, count=60, k_lo=1, k_hi=12),
             W.random_instance(rng, n=n, count=12, k_lo=200, k_hi=1024)]
    con_off = np.concatenate([parts[0].con_off, parts[1].con_off[1:] + parts[0].n_lits])
    inst = W.Instance(n=n, con_off=con_off, lits=np.concatenate([p.lits for p in parts]),
                      types=np.concatenate([p.types for p in parts]),
                      params=np.concatenate([p.params for p in parts]))
    lens = np.diff(inst.con_off)
    odd = rng.random(len(lens)) < 0.3
    inst.params[odd] = rng.choice([-5, -1, 0, 1, 2047, 4096, 1 << 30], size=int(odd.sum())).astype(np.int32)
    edge = rng.random(len(lens)) < 0.2
    inst.params[edge] = (lens[edge] + rng.integers(-1, 2, size=int(edge.sum()))).astype(np.int32)
    # points near the thresholds: mostly one sign, so long CARD counts land near k
    bias = rng.uniform(-1, 1, size=(n, 1))
    x = np.clip(bias + rng.normal(0, 0.4, size=(n, B)), -1, 1).astype(np.float32)
    d = afsat.Instance.from_arrays(inst)
    log("case: verify B=%d C=%d max k=%d" % (B, len(lens), lens.max()))
    unsat = d.round_verify(parity.to_dev(x)).cpu().numpy()
    want = oracle.verify(inst, x)
    assert np.array_equal(unsat, want)


def test_verify_planted_witness():
    for inst in [W.planted_3sat(instance=3), W.mixed_10k()]:
        H = np.where(inst.hidden, -1.0, 1.0).astype(np.float32)
        x = np.stack([H, 0.3 * H, -H], axis=1)
        d = afsat.Instance.from_arrays(inst)
        u = d.round_verify(parity.to_dev(x)).cpu().numpy()
        assert u[0] == 0 and u[1] == 0 and u[2] > 0
        assert np.array_equal(u, oracle.verify(inst, x))


def test_step_matches_oracle():
    rng = np.random.default_rng(15)
    n, B = 300, 90
    x = rng.uniform(-1, 1, size=(n, B)).astype(np.float32)
    g = rng.normal(0, 5, size=(n, B)).astype(np.float32)
    fixed = (rng.random(n) < 0.2).astype(np.uint8)
    done = (rng.random(B) < 0.3).astype(np.uint8)
    inst = W.random_instance(rng, n=n, count=10, k_lo=2, k_hi=3)
    d = afsat.Instance.from_arrays(inst)
    xd = parity.to_dev(x)
    d.step(xd, parity.to_dev(g), 0.1, fixed=torch.from_numpy(fixed).cuda(), done=torch.from_numpy(done).cuda())
    want = oracle.step(x, g, 0.1, fixed=fixed, done=done)
    got = xd.cpu().numpy()
    assert np.max(np.abs(got - want)) <= 1e-6
    frozen = fixed[:, None].astype(bool) | done[None, :].astype(bool)
    assert np.array_equal(got[frozen], x[frozen])
    assert got.min() >= -1 and got.max() <= 1


def test_pgd_step_is_eval_step_verify_and_deterministic():
    rng = np.random.default_rng(16)
    inst = concat([W.random_instance(rng, n=400, count=700, k_lo=1, k_hi=12),
                   W.random_instance(rng, n=400, count=20, k_lo=20, k_hi=200)], n=400)
    d = afsat.Instance.from_arrays(inst)
    B = 100
    x0 = parity.to_dev(rng.uniform(-1, 1, size=(inst.n, B)))
    # reference composition
    xa = x0.clone()
    g = d.eval(xa, obj=False, grad=True)["grad"]
    d.step(xa, g, 0.1)
    ua = d.round_verify(xa)
    # fused PGD step
    xb = x0.clone()
    st = d.pgd_state(B)
    d.pgd_init(xb, st)
    u0 = st["unsat"].clone()
    d.pgd_step(xb, st, 0.1)
    torch.cuda.synchronize()
    assert torch.equal(u0, d.round_verify(x0))
    assert torch.equal(xa, xb)
    assert torch.equal(ua, st["unsat"])
    assert int(st["counter"][0]) == 1
    # deterministic: same again bit for bit
    xc = x0.clone()
    st2 = d.pgd_state(B)
    d.pgd_init(xc, st2)
    d.pgd_step(xc, st2, 0.1)
    torch.cuda.synchronize()
    assert torch.equal(xb, xc)
    e1 = d.eval(x0, obj=True, grad=True)
    e2 = d.eval(x0, obj=True, grad=True)
    assert torch.equal(e1["grad"], e2["grad"]) and torch.equal(e1["obj"], e2["obj"])


def test_pgd_done_bookkeeping():
    inst = W.planted_3sat(instance=1)
    d = afsat.Instance.from_arrays(inst)
    H = np.where(inst.hidden, -1.0, 1.0).astype(np.float32)
    rng = np.random.default_rng(17)
    x = rng.uniform(-1, 1, size=(inst.n, 40)).astype(np.float32)
    x[:, 0] = H                                          # restart 0 starts satisfied
    xd = parity.to_dev(x)
    st = d.pgd_state(40)
    d.pgd_init(xd, st)
    assert int(st["done"][0]) == 1 and int(st["first_sat"][0]) == 0
    for t in range(1, 31):
        d.pgd_step(xd, st, 0.1)
    torch.cuda.synchronize()
    xs = xd.cpu().numpy()
    assert np.array_equal(xs[:, 0], H)                    # frozen
    done = st["done"].cpu().numpy().astype(bool)
    fs = st["first_sat"].cpu().numpy()
    u = st["unsat"].cpu().numpy()
    assert np.all(fs[done] >= 0) and np.all(fs[~done] == -1)
    assert np.all(u[done] == 0)
    assert np.array_equal(u, oracle.verify(inst, xs))
    assert int(st["counter"][0]) == 30 and int(st["counter"][1]) == done.sum()


@pytest.mark.parametrize("graph", [False, True])
def test_pgd_driver_stops_on_first_verified_restart(graph):
    """afs_pgd with stop_on_sat: it stops at the first counter read (every poll
    iterations) that finds a verified restart, the iteration count is a multiple
    of poll, every done restart verifies on the CPU, and the objective it returns
    is the one afs_eval gives at the final point."""
    inst = W.planted_3sat(n=100, m=340, instance=4)      # ratio 3.4: the oracle's PGD solves it
    d = afsat.Instance.from_arrays(inst)
    x0 = W.uniform_x0(inst.n, 64, workload=1, instance=4)
    xd = parity.to_dev(x0)
    res = d.pgd(xd, lr=0.1, steps=300, poll=5, stop_on_sat=True, graph=graph, obj=True)
    torch.cuda.synchronize()
    it, ndone = res["iters"], int(res["counter"][1])
    log("stopped after %d iterations with %d restarts done" % (it, ndone))
    assert ndone > 0 and it < 300 and it % 5 == 0 and int(res["counter"][0]) == it
    xs = xd.cpu().numpy()
    u = oracle.verify(inst, xs)
    done = res["done"].cpu().numpy().astype(bool)
    assert np.all(u[done] == 0) and np.array_equal(u, res["unsat"].cpu().numpy())
    fs = res["first_sat"].cpu().numpy()
    # the stop comes at the first read after a restart verifies: within the last poll window
    assert np.all((fs[done] > it - 5) & (fs[done] <= it))
    ev = d.eval(xd)
    assert torch.allclose(res["obj"], ev["obj"], rtol=0, atol=1e-5)


def test_pgd_driver_keeps_fixed_variables():
    """A partial assignment (Sec. 3.4): variables marked fixed keep their values
    through the driver's iterations; the others move."""
    inst = W.mixed_10k()
    d = afsat.Instance.from_arrays(inst)
    rng = np.random.default_rng(40)
    fixed = (rng.random(inst.n) < 0.3).astype(np.uint8)
    x0 = W.uniform_x0(inst.n, 64, workload=2, instance=1)
    xd = parity.to_dev(x0)
    d.pgd(xd, lr=0.1, steps=20, poll=5, stop_on_sat=False, fixed=torch.from_numpy(fixed).cuda())
    xs = xd.cpu().numpy()
    f = fixed.astype(bool)
    assert np.array_equal(xs[f], x0[f])
    assert np.mean(xs[~f] != x0[~f]) > 0.9


def test_planted_3sat_end_to_end_solves():
    """Algorithm 1 on planted 3-SAT (n=100, m=426, the 4.26 threshold ratio), 32
    restarts, lr 0.1, 200 steps.  Trajectories are chaotic, so success is compared
    per instance with the oracle's own FP64 PGD run, not restart by restart; every
    restart the GPU reports as done must verify on the CPU."""
    solved_gpu = solved_orc = 0
    for i in range(8):
        inst = W.planted_3sat(instance=i)
        x0 = W.uniform_x0(inst.n, 32, workload=1, instance=i)
        d = afsat.Instance.from_arrays(inst)
        xd = parity.to_dev(x0)
        res = d.pgd(xd, lr=0.1, steps=200, stop_on_sat=False)
        done = res["done"].cpu().numpy().astype(bool)
        xs = xd.cpu().numpy()
        if done.any():
            solved_gpu += 1
            assert np.all(oracle.verify(inst, xs[:, done]) == 0)
        ro = oracle.pgd(inst, x0, lr=0.1, steps=200)
        solved_orc += int((ro["first_sat"] >= 0).any())
        log("instance", i, "gpu restarts solved", int(done.sum()), "oracle", int((ro["first_sat"] >= 0).sum()))
    assert solved_gpu >= 1 and solved_gpu >= solved_orc - 2


def concat(parts, n):
    offs = [np.zeros(1, np.int64)]
    lits, types, params = [], [], []
    base = 0
    for p in parts:
        offs.append(p.con_off[1:] + base)
        base += p.n_lits
        lits.append(p.lits)
        types.append(p.types)
        params.append(p.params)
    return W.Instance(n=n, con_off=np.concatenate(offs), lits=np.concatenate(lits),
                      types=np.concatenate(types), params=np.concatenate(params))


def test_batch_of_uneven_instances():
    """A block-diagonal batch of instances of different sizes and types: FE and
    gradient match the oracle on the concatenation, verification is exact per
    (part, restart), and PGD freezes exactly the (part, restart) pairs that verify."""
    rng = np.random.default_rng(50)
    parts = [W.planted_3sat(n=60, m=250, instance=7),
             W.random_instance(rng, n=300, count=200, k_lo=2, k_hi=30),
             W.planted_3sat(n=100, m=426, instance=8),
             W.random_instance(rng, n=900, count=40, k_lo=17, k_hi=300),
             W.planted_3sat(n=40, m=120, instance=9)]
    Bt = afsat.Instance.batch(parts)
    off = Bt.var_offsets()
    cat = concat([W.Instance(n=p.n, con_off=p.con_off, lits=np.where(p.lits > 0, p.lits + o, p.lits - o).astype(np.int32),
                             types=p.types, params=p.params) for p, o in zip(parts, off[:-1])], n=int(off[-1]))
    B = 40
    x = rng.uniform(-1, 1, size=(cat.n, B)).astype(np.float32)
    parity.compare(cat, Bt, parity.gpu_eval(Bt, x), oracle.eval(cat, x, fe=True, adj=True, grad=True), "batch")
    xd = parity.to_dev(x)
    u = Bt.round_verify(xd).cpu().numpy()
    assert u.shape == (len(parts), B)
    for p, part in enumerate(parts):
        assert np.array_equal(u[p], oracle.verify(part, x[off[p]:off[p + 1]]))
    res = Bt.pgd(xd, lr=0.1, steps=60, stop_on_sat=False)
    xs = xd.cpu().numpy()
    done = res["done"].cpu().numpy().astype(bool)
    fs = res["first_sat"].cpu().numpy()
    assert done.shape == (len(parts), B) and np.all((fs >= 0) == done)
    for p, part in enumerate(parts):
        up = oracle.verify(part, xs[off[p]:off[p + 1]])
        assert np.array_equal(up, res["unsat"].cpu().numpy()[p])
        assert np.all(up[done[p]] == 0)
    assert done.sum() == int(res["counter"][1])
    assert done[0].any() or done[2].any() or done[4].any()     # small planted parts get solved


def test_bucket_set_call_equals_the_range_call():
    """afs_fe_grad_buckets over every bucket, listed in a shuffled order, writes
    the same adjoints and objective partials bit for bit as afs_fe_grad over the
    range (the long buckets then run two at a time on two streams, the short
    ones beside them); duplicates and bad indices are rejected."""
    rng = np.random.default_rng(44)
    inst = concat([W.random_instance(rng, n=500, count=900, k_lo=1, k_hi=12),
                   W.random_instance(rng, n=500, count=40, k_lo=17, k_hi=300)], n=500)
    d = afsat.Instance.from_arrays(inst)
    B = 96
    x = parity.to_dev(rng.uniform(-1, 1, size=(inst.n, B)))
    ws_a, ws_b = d.workspace(B), d.workspace(B).clone()
    d.fe_grad(x, ws_a, 0, d.n_buckets, want_obj=True)
    order = rng.permutation(d.n_buckets)
    d.fe_grad_buckets(x, ws_b, order, want_obj=True)
    ga = torch.empty((inst.n, B), device="cuda")
    gb = torch.empty_like(ga)
    oa = torch.empty(B, device="cuda")
    ob = torch.empty_like(oa)
    d.scatter(B, ws_a, obj=oa, grad=ga)
    d.scatter(B, ws_b, obj=ob, grad=gb)
    torch.cuda.synchronize()
    assert torch.equal(ga, gb) and torch.equal(oa, ob)
    log("buckets: %d (%d long)" % (d.n_buckets, sum(1 for b in d.buckets() if b.lanes_per_restart > 1)))
    for bad in ([0, 0], [d.n_buckets], [-1]):
        with pytest.raises(afsat.AfsError):
            d.fe_grad_buckets(x, ws_b, bad)
