"""Differentiation: the hand-written adjoint behind torch.autograd.Function
(forward = FE only, backward = recomputed products seeded by dL/dF per restart),
checked against the FP64 oracle's gradient and against central differences of
the oracle's objective (exact for a function affine in each coordinate)."""
import os
import sys
import tempfile

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
    afsat.lib()


def log(*a):
    print(*a, flush=True)


def test_forward_and_vjp_match_eval_and_oracle():
    """FEObjective's forward and backward against the oracle at the per-bucket
    bars of parity.py: the objective, the gradient, and every per-literal
    adjoint term of afs_eval_adjoint (seeded by a random dL/dF per restart)."""
    rng = np.random.default_rng(30)
    parts = [W.random_instance(rng, n=500, count=400, k_lo=1, k_hi=16),
             W.random_instance(rng, n=500, count=12, k_lo=17, k_hi=400)]
    inst = W.Instance(n=500, con_off=np.concatenate([parts[0].con_off, parts[1].con_off[1:] + parts[0].n_lits]),
                      lits=np.concatenate([p.lits for p in parts]), types=np.concatenate([p.types for p in parts]),
                      params=np.concatenate([p.params for p in parts]))
    B = 45
    x32 = rng.uniform(-1, 1, size=(inst.n, B)).astype(np.float32)
    d = afsat.Instance.from_arrays(inst)
    x = parity.to_dev(x32).requires_grad_(True)
    obj = afsat.FEObjective.apply(x, d)
    gobj = torch.from_numpy(rng.normal(size=B).astype(np.float32)).cuda()
    (obj * gobj).sum().backward()
    torch.cuda.synchronize()
    orc = oracle.eval(inst, x32, grad=True, adj=True)
    parity.check_obj(inst, obj.detach().cpu().numpy().astype(np.float64), orc["obj"], None, "forward")
    seed = gobj.cpu().numpy().astype(np.float64)[None, :]
    parity.check_grad(x.grad.cpu().numpy().astype(np.float64) / np.max(np.abs(seed)),
                      orc["grad"] * seed / np.max(np.abs(seed)), "vjp", inst)
    grad, adj = d.eval_adjoint(x.detach(), gobj, adj=True)
    torch.cuda.synchronize()
    lit_w = parity.literal_weights(inst) * float(np.max(np.abs(seed)))
    rel = parity.check_adjoints(adj.cpu().numpy().astype(np.float64), orc["adj"] * seed,
                                parity.bucket_of_literals(d), d.buckets(), "eval_adjoint", lit_w)
    log("per-bucket adjoint errors (max rel, L2 rel):", ["%.1e/%.1e" % r for r in rel])
    assert torch.equal(grad, x.grad)
    # the forward-only objective equals the full evaluation's, and the unseeded
    # adjoint equals the gradient of afs_eval bit for bit (same kernels, same order)
    e = d.eval(x.detach(), obj=True, grad=True)
    assert torch.allclose(obj.detach(), e["obj"], rtol=0, atol=1e-5)
    assert torch.equal(d.eval_adjoint(x.detach()), e["grad"])


def test_longcard50k_autograd():
    """n=50k, 200k clauses (k 3-10) and 1,000 CARD (k 256-1,024), 512 restarts,
    FE and gradient through FEObjective; at 8 sampled restarts, the gradient and
    every per-literal adjoint term against the oracle at the per-bucket bars, and
    the gradient against FP64 central differences of the oracle objective
    (h = 1e-3) at 48 sampled (variable, restart) pairs."""
    from paper_2606_06641_amd import autotune
    inst = W.long_card_50k()
    B = 512
    x32 = W.uniform_x0(inst.n, B, workload=4)
    with tempfile.TemporaryDirectory() as tmp:
        shapes, _ = autotune.tune(inst, B, cache_path=autotune.DEFAULT_CACHE, out_path=os.path.join(tmp, "t.txt"),
                                  max_cons=400)
    log("case: long-card autograd n=50k B=512, tuned shapes %s" % shapes)
    d = afsat.Instance.from_arrays(inst, shapes=shapes)
    x = parity.to_dev(x32).requires_grad_(True)
    obj = afsat.FEObjective.apply(x, d)
    obj.sum().backward()
    torch.cuda.synchronize()
    g = x.grad.cpu().numpy().astype(np.float64)
    rng = np.random.default_rng(40)
    cols = np.sort(rng.choice(B, size=8, replace=False))
    orc = oracle.eval(inst, x32[:, cols], grad=True, adj=True)
    r = parity.check_grad(g[:, cols], orc["grad"], "longcard50k grad", inst)
    log("gradient: max rel %.2e, L2 rel %.2e" % r)
    parity.check_obj(inst, obj.detach().cpu().numpy().astype(np.float64)[cols], orc["obj"], None, "forward")
    _, adj = d.eval_adjoint(x.detach(), adj=True)
    ci = torch.from_numpy(cols).cuda()
    adj_s = adj.index_select(1, ci).cpu().numpy().astype(np.float64)
    del adj
    rel = parity.check_adjoints(adj_s, orc["adj"], parity.bucket_of_literals(d), d.buckets(), "longcard50k adj",
                                parity.literal_weights(inst))
    log("per-bucket adjoint errors (max rel, L2 rel):")
    for b, rr in zip(d.buckets(), rel):
        log("  [%4d-%4d] J%-2d S%-2d  %.2e  %.2e" % (b.k_lo, b.k_hi, b.lanes_per_restart, b.lits_per_lane, *rr))
    # central differences of the oracle objective, variables of the long constraints first
    h = 1e-3
    card_vars = np.unique(np.abs(inst.lits[inst.con_off[np.nonzero(inst.types == W.CARD_GE)[0][0]]:
                                           inst.con_off[np.nonzero(inst.types == W.CARD_GE)[0][0] + 1]]) - 1)
    vs = np.concatenate([rng.choice(card_vars, size=24, replace=False), rng.choice(inst.n, size=24, replace=False)])
    bs = rng.choice(B, size=48)
    X = np.repeat(x32[:, bs].astype(np.float64), 2, axis=1)
    for j, v in enumerate(vs):
        X[v, 2 * j] += h
        X[v, 2 * j + 1] -= h
    F = oracle.eval(inst, X, grad=False)["obj"]
    fd = (F[0::2] - F[1::2]) / (2 * h)
    ferr = np.max(np.abs(fd - g[vs, bs]))
    scale = np.max(np.abs(orc["grad"]))
    log("max |grad - central difference| = %.3e (bar 1e-4 * %.3e)" % (ferr, scale))
    assert ferr <= parity.REL_TOL * scale


@pytest.mark.parametrize("kind", ["3sat", "mixed"])
def test_graph_replay_equals_eager(kind):
    """Algorithm 1 through the library's driver with and without its internal HIP
    graph gives the same bits; and afs_pgd_step captured by the caller (a torch
    CUDA graph) and replayed, with eager work and syncs between replays, matches
    eager steps at every replay.  The mixed instance has short and long buckets,
    whose launches fork to a second stream and join back inside the graphs."""
    inst = W.planted_3sat(instance=2) if kind == "3sat" else W.mixed_10k()
    log("case: graph replay %s" % kind)
    B = 32
    x0 = W.uniform_x0(inst.n, B, workload=1, instance=2)
    d = afsat.Instance.from_arrays(inst)
    xa = parity.to_dev(x0)
    ra = d.pgd(xa, lr=0.1, steps=40, poll=10, stop_on_sat=False, graph=False, obj=True)
    xb = parity.to_dev(x0)
    rb = d.pgd(xb, lr=0.1, steps=40, poll=10, stop_on_sat=False, graph=True, obj=True)
    torch.cuda.synchronize()
    assert ra["iters"] == rb["iters"] == 40
    assert torch.equal(xa, xb)
    for k in ("unsat", "done", "first_sat", "counter", "obj"):
        assert torch.equal(ra[k], rb[k]), k
    if kind == "3sat":
        # a poll period longer than one captured graph (64 iterations): two
        # replays and 22 eager iterations per period, then an eager tail
        xl = parity.to_dev(x0)
        rl = d.pgd(xl, lr=0.1, steps=160, poll=150, stop_on_sat=False, graph=True, obj=True)
        xe = parity.to_dev(x0)
        re_ = d.pgd(xe, lr=0.1, steps=160, poll=150, stop_on_sat=False, graph=False, obj=True)
        torch.cuda.synchronize()
        assert rl["iters"] == re_["iters"] == 160 and torch.equal(xl, xe)
        for k in ("unsat", "done", "first_sat", "counter", "obj"):
            assert torch.equal(rl[k], re_[k]), k
    # the driver (whose verification overlaps the next iteration's FE on a stream
    # of its own) equals 40 plain afs_pgd_step calls on one stream
    xs = parity.to_dev(x0)
    ss = d.pgd_state(B)
    d.pgd_init(xs, ss)
    for _ in range(40):
        d.pgd_step(xs, ss, 0.1)
    torch.cuda.synchronize()
    assert torch.equal(xa, xs)
    for k in ("unsat", "done", "first_sat", "counter"):
        assert torch.equal(ra[k], ss[k]), k
    # caller-side capture of afs_pgd_step
    ws_c, ws_e = d.workspace(B), d.workspace(B)
    xc, xe = parity.to_dev(x0), parity.to_dev(x0)
    sc, se = d.pgd_state(B), d.pgd_state(B)
    d.pgd_init(xc, sc, ws_c)
    d.pgd_init(xe, se, ws_e)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        for _ in range(10):
            d.pgd_step(xc, sc, 0.1, None, ws_c)
    for rep in range(3):
        for _ in range(10):
            d.pgd_step(xe, se, 0.1, None, ws_e)
        g.replay()
        torch.cuda.synchronize()
        assert torch.equal(xc, xe), rep
        for k in ("unsat", "done", "first_sat", "counter"):
            assert torch.equal(sc[k], se[k]), (rep, k)
