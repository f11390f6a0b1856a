"""afs_eval_noalloc (the evaluation with the library's static scratch in place of
a workspace) against afs_eval, through the C ABI: same outputs bit for bit,
on two calls in a row (the second with a smaller input, so it runs over what the
first left in the scratch), and a clear error with nothing launched when the
input needs more scratch than the array holds."""
import ctypes
import sys

import numpy as np
import pytest
import torch

import parity
from paper_2606_06641_amd import afsat
from paper_2606_06641_amd import workloads as W

pytestmark = pytest.mark.gpu

SCRATCH_BYTES = 64 << 20


@pytest.fixture(scope="module", autouse=True)
def need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    afsat.lib()


def log(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def mixed(seed, n, short, long_):
    rng = np.random.default_rng(seed)
    a = W.random_instance(rng, n=n, count=short, k_lo=1, k_hi=16)
    b = W.random_instance(rng, n=n, count=long_, k_lo=17, k_hi=300)
    inst = W.Instance(n=n, con_off=np.concatenate([a.con_off, b.con_off[1:] + a.n_lits]),
                      lits=np.concatenate([a.lits, b.lits]), types=np.concatenate([a.types, b.types]),
                      params=np.concatenate([a.params, b.params]))
    inst.weights = rng.uniform(0.5, 2.0, size=inst.n_cons).astype(np.float32)
    return inst


def noalloc(d, x, want):
    """afs_eval_noalloc through ctypes on preallocated outputs."""
    B = x.shape[1]
    out = {k: torch.full(shp, float("nan"), dtype=torch.float32, device=x.device) for k, shp in
           (("obj", (B,)), ("grad", (d.n, B)), ("fe", (d.n_cons, B)), ("adj", (d.n_lits, B))) if k in want}
    p = lambda k: ctypes.c_void_p(out[k].data_ptr()) if k in out else None
    rc = afsat.lib().afs_eval_noalloc(d._h, B, ctypes.c_void_p(x.data_ptr()), p("obj"), p("grad"), p("fe"),
                                      p("adj"), ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))
    return rc, out


def test_noalloc_equals_eval_twice_then_smaller():
    cases = [(mixed(1, 600, 900, 30), 200), (mixed(2, 300, 200, 6), 70)]
    for i, (inst, B) in enumerate(cases):
        log("case %d: n=%d C=%d L=%d B=%d" % (i, inst.n, inst.n_cons, inst.n_lits, B))
        d = afsat.Instance.from_arrays(inst)
        x = parity.to_dev(np.random.default_rng(10 + i).uniform(-1, 1, size=(inst.n, B)))
        want = d.eval(x, obj=True, grad=True, fe=True, adj=True)
        rc, got = noalloc(d, x, ("obj", "grad", "fe", "adj"))
        torch.cuda.synchronize()
        assert rc == afsat.AFS_OK, afsat.lib().afs_last_error()
        for k in want:
            assert torch.equal(got[k], want[k]), (i, k)
        # only some outputs requested
        rc, got = noalloc(d, x, ("grad",))
        torch.cuda.synchronize()
        assert rc == afsat.AFS_OK and torch.equal(got["grad"], want["grad"])
        d.close()


def test_noalloc_rejects_inputs_beyond_the_scratch():
    inst = mixed(3, 2000, 3000, 40)
    d = afsat.Instance.from_arrays(inst)
    B = (SCRATCH_BYTES // (4 * inst.n_lits) // 64 + 2) * 64          # adjoint rows alone exceed the array
    x = parity.to_dev(np.zeros((inst.n, B), np.float32))
    rc, out = noalloc(d, x, ("obj",))
    torch.cuda.synchronize()
    assert rc == afsat.AFS_EINVAL
    assert b"scratch" in afsat.lib().afs_last_error()
    assert torch.isnan(out["obj"]).all()                               # nothing was launched
    # the same instance at a size that fits still works after the refusal
    Bs = 64
    xs = parity.to_dev(np.random.default_rng(5).uniform(-1, 1, size=(inst.n, Bs)))
    rc, got = noalloc(d, xs, ("obj", "grad"))
    want = d.eval(xs, obj=True, grad=True)
    torch.cuda.synchronize()
    assert rc == afsat.AFS_OK
    assert torch.equal(got["obj"], want["obj"]) and torch.equal(got["grad"], want["grad"])
    d.close()
