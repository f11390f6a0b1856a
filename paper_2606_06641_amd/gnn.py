"""Learned initialisation: binding of the message-passing network (afs_gnn_* in
``include/afsat.h``) and the orchestration around it -- collecting training
targets from the solver's own runs, training with the network's kernels, and
proposing starting points for Algorithm 1 (uniform random as fallback).

Every numeric step (message passing, dense layers, head, loss, gradients, Adam)
runs in the library's kernels; this module moves arrays and loops over data.
"""
import ctypes
import time

import numpy as np
import torch

from . import afsat

_vp = ctypes.c_void_p
_f32p = ctypes.POINTER(ctypes.c_float)
_i32p = ctypes.POINTER(ctypes.c_int32)

GNN_SIGNATURES = [
    ("afs_gnn_last_error", ctypes.c_char_p, []),
    ("afs_gnn_create", ctypes.c_int, [ctypes.c_int32, ctypes.c_uint64, ctypes.c_int32, ctypes.POINTER(_vp)]),
    ("afs_gnn_destroy", None, [_vp]),
    ("afs_gnn_num_params", ctypes.c_int, [_vp, ctypes.POINTER(ctypes.c_int64)]),
    ("afs_gnn_get", ctypes.c_int, [_vp, ctypes.c_int32, _f32p]),
    ("afs_gnn_set", ctypes.c_int, [_vp, ctypes.c_int32, _f32p]),
    ("afs_gnn_features", ctypes.c_int, [_vp, _f32p, _f32p, _i32p, _i32p, _f32p]),
    ("afs_gnn_workspace_bytes", ctypes.c_int, [_vp, _vp, ctypes.c_int32, ctypes.POINTER(ctypes.c_size_t)]),
    ("afs_gnn_forward", ctypes.c_int, [_vp, _vp, ctypes.c_int32, _vp, _vp, ctypes.c_size_t, _vp, _vp]),
    ("afs_gnn_backward", ctypes.c_int, [_vp, _vp, ctypes.c_int32, _vp, _vp, _vp, ctypes.c_size_t, _vp, _vp]),
    ("afs_gnn_zero_grad", ctypes.c_int, [_vp, _vp]),
    ("afs_gnn_adam", ctypes.c_int, [_vp, ctypes.c_float, ctypes.c_float, ctypes.c_float, ctypes.c_float,
                                    ctypes.c_int32, _vp]),
    ("afs_gnn_gemm_bf16", ctypes.c_int, [ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, _vp, ctypes.c_int64,
                                         ctypes.c_int64, _vp, ctypes.c_int64, ctypes.c_int64, _vp,
                                         ctypes.c_int64, _vp]),
]

_bound = False


def lib():
    global _bound
    L = afsat.lib()
    if not _bound:
        for name, res, args in GNN_SIGNATURES:
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _bound = True
    return L


def _check(rc):
    if rc != afsat.AFS_OK:
        raise afsat.AfsError(rc, lib().afs_gnn_last_error().decode())


def _p(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _stream(device):
    return ctypes.c_void_p(torch.cuda.current_stream(device).cuda_stream)


def gemm_bf16(A, B):
    """C = A @ B on the network's BF16 MFMA kernel (A, B float32 CUDA, 2-D)."""
    M, K = A.shape
    K2, N = B.shape
    assert K == K2
    C = torch.empty((M, N), dtype=torch.float32, device=A.device)
    _check(lib().afs_gnn_gemm_bf16(M, N, K, _p(A), A.stride(0), A.stride(1), _p(B), B.stride(0), B.stride(1),
                                   _p(C), C.stride(0), _stream(A.device.index)))
    return C


def features(inst):
    """Host features (fcon [C][16], fvar [n][16]) of an Instance, as the device uses them."""
    fc = np.zeros((inst.n_cons, 16), np.float32)
    fv = np.zeros((inst.n, 16), np.float32)
    _check(lib().afs_gnn_features(inst._h, fc.ctypes.data_as(_f32p), fv.ctypes.data_as(_f32p), None, None, None))
    return fc, fv


class GNN:
    """Message-passing network over the variable-constraint graph (device-resident)."""

    def __init__(self, rounds=3, seed=0, device=0):
        h = ctypes.c_void_p()
        _check(lib().afs_gnn_create(int(rounds), int(seed), int(device), ctypes.byref(h)))
        self._h = h
        self.rounds = rounds
        self.device = device
        n = ctypes.c_int64()
        _check(lib().afs_gnn_num_params(h, ctypes.byref(n)))
        self.num_params = n.value
        self._ws = {}
        self.t = 0

    def close(self):
        if getattr(self, "_h", None):
            lib().afs_gnn_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def get(self, which=0):
        a = np.zeros(self.num_params, np.float32)
        _check(lib().afs_gnn_get(self._h, int(which), a.ctypes.data_as(_f32p)))
        return a

    def set(self, a, which=0):
        a = np.ascontiguousarray(a, np.float32)
        assert a.size == self.num_params
        _check(lib().afs_gnn_set(self._h, int(which), a.ctypes.data_as(_f32p)))

    def state_dict(self):
        return {"rounds": self.rounds, "t": self.t, "params": self.get(0), "m": self.get(2), "v": self.get(3)}

    def load_state_dict(self, sd):
        self.set(sd["params"], 0)
        self.set(sd["m"], 2)
        self.set(sd["v"], 3)
        self.t = int(sd["t"])

    def _workspace(self, inst, B):
        key = (id(inst), B)
        ws = self._ws.get(key)
        if ws is None:
            nb = ctypes.c_size_t()
            _check(lib().afs_gnn_workspace_bytes(self._h, inst._h, int(B), ctypes.byref(nb)))
            ws = torch.empty(max(nb.value, 256), dtype=torch.uint8, device=torch.device("cuda", self.device))
            self._ws = {key: ws}
        return ws

    def forward(self, inst, x0):
        """xhat (n, B) in (-1, 1) from x0 (n, B) float32 CUDA."""
        B = x0.shape[1]
        ws = self._workspace(inst, B)
        xhat = torch.empty_like(x0)
        _check(lib().afs_gnn_forward(self._h, inst._h, int(B), _p(x0), _p(ws), ws.numel(), _p(xhat),
                                     _stream(self.device)))
        return xhat

    def zero_grad(self):
        _check(lib().afs_gnn_zero_grad(self._h, _stream(self.device)))

    def loss_backward(self, inst, x0, target):
        """Mean BCE against target (n,) uint8 CUDA (1 = True); gradient accumulates."""
        B = x0.shape[1]
        ws = self._workspace(inst, B)
        loss = torch.empty(1, dtype=torch.float32, device=x0.device)
        _check(lib().afs_gnn_backward(self._h, inst._h, int(B), _p(x0), _p(target), _p(ws), ws.numel(),
                                      _p(loss), _stream(self.device)))
        return loss

    def adam(self, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8):
        self.t += 1
        _check(lib().afs_gnn_adam(self._h, float(lr), float(beta1), float(beta2), float(eps), int(self.t),
                                  _stream(self.device)))


# ---------------------------------------------------------------------------
# Orchestration
# ---------------------------------------------------------------------------

def solver_target(dinst, x0, steps, lr=0.1, poll=10):
    """Run Algorithm 1 from x0 (n, B) and return the rounded assignment of its best
    restart (a verified one if any, else the fewest unsatisfied constraints) as a
    uint8 CUDA tensor (1 = True), plus whether it verified."""
    x = x0.clone()
    st = dinst.pgd(x, lr=lr, steps=steps, poll=poll, stop_on_sat=True, graph=False)
    unsat = st["unsat"].reshape(-1)
    best = int(torch.argmin(unsat).item())
    return (x[:, best] < 0).to(torch.uint8).contiguous(), int(unsat[best].item()) == 0


def uniform_start(n, B, generator=None, device=0):
    dev = torch.device("cuda", device)
    return (torch.rand((n, B), generator=generator, device=dev) * 2 - 1).contiguous()


def learned_start(net, dinst, B, generator=None, temperature=1.0, mix=0.0, sample=False):
    """Starting points proposed by the network (uniform random if it yields
    non-finite values: fallback).

    The network maps noise x0 to xhat = tanh(z).  ``temperature`` T softens it to
    tanh(z / T) (= tanh(atanh(xhat) / T)); ``mix`` blends the result with the
    noise, (1 - mix) tanh(z/T) + mix x0; with ``sample`` each restart instead draws
    the sign of every variable from the softened marginal P(True) = (1 - tanh(z/T))/2
    and keeps |x0| as magnitude."""
    x0 = uniform_start(dinst.n, B, generator, net.device)
    xhat = net.forward(dinst, x0)
    if not bool(torch.isfinite(xhat).all()):
        return x0, False
    if temperature != 1.0:
        xhat = torch.tanh(torch.atanh(xhat.clamp(-0.999999, 0.999999)) / temperature)
    if sample:
        u = torch.rand(x0.shape, generator=generator, device=x0.device)
        true = u < (1 - xhat) / 2
        out = torch.where(true, -x0.abs(), x0.abs())
    else:
        out = (1 - mix) * xhat + mix * x0
    return out.clamp(-1, 1).contiguous(), True


def time_to_sat(dinst, make_start, B, max_steps, lr=0.1, poll=10):
    """Seconds from the start of init generation to the first verified restart
    (None if none verifies within max_steps), and the best unsat count seen."""
    torch.cuda.synchronize(dinst.device)
    t0 = time.perf_counter()
    x0 = make_start()
    st = dinst.pgd(x0, lr=lr, steps=max_steps, poll=poll, stop_on_sat=True, graph=False)
    solved = int(st["counter"][1].item()) > 0
    torch.cuda.synchronize(dinst.device)
    t1 = time.perf_counter()
    return (t1 - t0) if solved else None, int(st["unsat"].min().item()), st["iters"]


# ---------------------------------------------------------------------------
# Train-and-compare experiment (learned vs uniform random initialisation)
# ---------------------------------------------------------------------------

def collect_targets(parts, B=256, steps=150, lr=0.1, chunk=32):
    """Solver-produced targets for each instance: the rounded best restart of
    Algorithm 1 from uniform random starts (instances solved together in batches).
    Returns (list of uint8 CUDA tensors, number verified)."""
    targets, verified = [], 0
    for i in range(0, len(parts), chunk):
        group = parts[i:i + chunk]
        bt = afsat.Instance.batch(group)
        x = uniform_start(bt.n, B)
        st = bt.pgd(x, lr=lr, steps=steps, poll=10, stop_on_sat=False, graph=False)
        unsat = st["unsat"].reshape(len(group), B)
        best = torch.argmin(unsat, dim=1)
        off = bt.var_offsets()
        for p in range(len(group)):
            b = int(best[p].item())
            verified += int(unsat[p, b].item()) == 0
            targets.append((x[off[p]:off[p + 1], b] < 0).to(torch.uint8).contiguous())
    return targets, verified


def train(net, parts, targets, steps, lr=2e-3, chunk=32, restarts=16, seed=0, log=None):
    """Adam on the mean BCE, cycling over batches of ``chunk`` instances."""
    batches = []
    for i in range(0, len(parts), chunk):
        batches.append((afsat.Instance.batch(parts[i:i + chunk]), torch.cat(targets[i:i + chunk])))
    gen = torch.Generator(device="cuda").manual_seed(seed)
    losses = []
    for step in range(steps):
        bt, tg = batches[step % len(batches)]
        net.zero_grad()
        loss = net.loss_backward(bt, uniform_start(bt.n, restarts, gen), tg)
        net.adam(lr=lr)
        if step % 50 == 0 or step == steps - 1:
            losses.append((step, float(loss.item())))
            if log:
                log("train step %d loss %.4f" % losses[-1])
    return losses


def run_arm(dinst, make_start, max_steps, lr=0.1, poll=10):
    """One arm on one instance: (seconds to the first verified restart or None,
    first verifying iteration or None, best unsat at the end, wall seconds spent).
    The clock starts before the starting points are generated."""
    torch.cuda.synchronize(dinst.device)
    t0 = time.perf_counter()
    x0 = make_start()
    st = dinst.pgd(x0, lr=lr, steps=max_steps, poll=poll, stop_on_sat=True, graph=False)
    torch.cuda.synchronize(dinst.device)
    t1 = time.perf_counter()
    fs = st["first_sat"].reshape(-1)
    ok = fs >= 0
    if bool(ok.any()):
        return t1 - t0, int(fs[ok].min().item()), 0, t1 - t0
    return None, None, int(st["unsat"].min().item()), t1 - t0


def compare(net, tests, B, max_steps, variant, seed=0, timeout_s=None, lr=0.1):
    """Learned vs uniform random starts on each test instance (same noise seed per
    instance for both arms).  Returns per-arm lists of (seconds, iteration, best_unsat)."""
    out = {"random": [], "learned": []}
    for i, p in enumerate(tests):
        d = afsat.Instance.from_arrays(p)
        net.forward(d, uniform_start(p.n, 1))           # build the instance's graph tensors once
        for arm in ("random", "learned"):
            g = torch.Generator(device="cuda").manual_seed(seed * 100003 + i)
            if arm == "random":
                make = lambda: uniform_start(p.n, B, g)
            else:
                make = lambda: learned_start(net, d, B, g, **variant)[0]
            out[arm].append(run_arm(d, make, max_steps, lr))
        d.close()
    return out


def summarize(res, max_steps, timeout_s=None):
    """Median time / iterations to a verified assignment (censored runs count twice
    the timeout, PAR-2), solved counts.  The default timeout is the longest wall time
    any run of either arm spent (an unsolved run spends the full iteration budget)."""
    if timeout_s is None:
        timeout_s = max(r[3] for rows in res.values() for r in rows)
    out = {"timeout_s": timeout_s}
    for arm, rows in res.items():
        t = [r[0] for r in rows]
        it = [r[1] for r in rows]
        solved = [x is not None for x in t]
        par2 = [x if x is not None else 2 * timeout_s for x in t]
        it_c = [x if x is not None else 2 * max_steps for x in it]
        out[arm] = {"solved": int(sum(solved)), "of": len(rows),
                    "median_s": float(np.median(par2)), "par2_mean_s": float(np.mean(par2)),
                    "median_iters": float(np.median(it_c)),
                    "mean_best_unsat_unsolved": float(np.mean([r[2] for r in rows if r[0] is None]))
                    if not all(solved) else 0.0}
    return out
