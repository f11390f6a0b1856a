"""Learned initialisation: binding of the message-passing network (afs_gnn_* in
``include/afsat.h``) and the orchestration around it -- collecting training
targets from the solver's own runs, training with the network's kernels, and
proposing starting points for Algorithm 1 (uniform random as fallback).

Every numeric step (message passing, dense layers, head, loss, gradients, Adam)
runs in the library's kernels; this module moves arrays and loops over data.
"""
import ctypes
import time
import weakref

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
    ("afs_gnn_starts", ctypes.c_int, [ctypes.c_int32, ctypes.c_int32, _vp, _vp, ctypes.c_uint64, ctypes.c_float,
                                      ctypes.c_float, ctypes.c_int32, _vp, _vp]),
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
        self._ws = None
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
        # one cached workspace, for the instance object it was sized for (held by a
        # weak reference, so a later instance at the same address is not mistaken
        # for it) and B
        ref, b, ws = self._ws or (None, None, None)
        if ws is None or b != B or ref() is not inst:
            nb = ctypes.c_size_t()
            _check(lib().afs_gnn_workspace_bytes(self._h, inst._h, int(B), ctypes.byref(nb)))
            ws = torch.empty(max(nb.value, 256), dtype=torch.uint8, device=torch.device("cuda", self.device))
            self._ws = (weakref.ref(inst), B, ws)
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

def uniform_start(dinst, B, seed):
    """Uniform starting points (n, B) on [-1, 1) from the library's counter-based
    generator (afs_init_points) keyed by seed."""
    return dinst.init_points(B, seed)


def learned_start(net, dinst, B, seed, temperature=1.0, mix=0.0, sample=False):
    """Starting points proposed by the network: noise x0 = uniform_start(seed)
    through the network (xhat = tanh(z)), then afs_gnn_starts: softened to
    tanh(z / T); with ``sample`` every variable's sign drawn from the softened
    marginal P(True) = (1 - tanh(z/T))/2 with |x0| as magnitude, else
    (1 - mix) tanh(z/T) + mix x0; a non-finite output falls back to x0."""
    x0 = uniform_start(dinst, B, seed)
    xhat = net.forward(dinst, x0)
    out = torch.empty_like(x0)
    _check(lib().afs_gnn_starts(dinst.n, B, _p(xhat), _p(x0), (int(seed) * 0x9E3779B97F4A7C15 + 1) % (1 << 64),
                                float(temperature), float(mix), int(bool(sample)), _p(out), _stream(net.device)))
    return out


def collect_targets(parts, B=256, steps=200, lr=0.1, chunk=32, seed=0):
    """Solver-produced targets for each instance: the rounded best restart of
    Algorithm 1 from uniform random starts (instances solved together in
    block-diagonal batches of ``chunk``), a verified restart when there is one,
    else the fewest unsatisfied constraints.  Returns (list of uint8 CUDA
    tensors, number verified, unsat count of each target)."""
    targets, verified, unsat_of = [], 0, []
    for i in range(0, len(parts), chunk):
        group = parts[i:i + chunk]
        bt = afsat.Instance.batch(group)
        x = uniform_start(bt, B, seed * 1000003 + i)
        st = bt.pgd(x, lr=lr, steps=steps, poll=10, stop_on_sat=False)
        unsat = st["unsat"].reshape(len(group), B)
        best = torch.argmin(unsat, dim=1)
        off = bt.var_offsets()
        for p in range(len(group)):
            b = int(best[p].item())
            u = int(unsat[p, b].item())
            verified += u == 0
            unsat_of.append(u)
            targets.append((x[off[p]:off[p + 1], b] < 0).to(torch.uint8).contiguous())
        bt.close()
    return targets, verified, unsat_of


def train(net, parts, targets, steps, lr=2e-3, chunk=32, restarts=16, seed=0, log=None):
    """Adam on the mean BCE, cycling over batches of ``chunk`` instances; the
    noise given to the network is drawn by afs_init_points, fresh every step."""
    batches = []
    for i in range(0, len(parts), chunk):
        batches.append((afsat.Instance.batch(parts[i:i + chunk]), torch.cat(targets[i:i + chunk])))
    losses = []
    for step in range(steps):
        bt, tg = batches[step % len(batches)]
        net.zero_grad()
        loss = net.loss_backward(bt, uniform_start(bt, restarts, seed * 1000003 + step), tg)
        net.adam(lr=lr)
        if step % 50 == 0 or step == steps - 1:
            losses.append((step, float(loss.item())))
            if log:
                log("train step %d loss %.4f" % losses[-1])
    for bt, _ in batches:
        bt.close()
    return losses


def run_arm(dinst, make_start, round_steps, timeout_s, lr=0.1, poll=10, search=None, max_rounds=0):
    """One arm on one instance: Algorithm 1 in rounds of ``round_steps``
    iterations, each from fresh starting points (``make_start()``), until a
    restart verifies, ``timeout_s`` has passed or (``max_rounds`` > 0) that many
    rounds have run.  The clock starts before the
    first starting points are generated, so the learned arm's time includes the
    network's first use on the instance (its graph build) and every round's
    inference.  Returns (seconds to the first verified restart or None, rounds,
    iterations run, best unsat count seen, wall seconds spent)."""
    torch.cuda.synchronize(dinst.device)
    t0 = time.perf_counter()
    rounds = iters = 0
    best = None
    while True:
        x0 = make_start()
        st = dinst.pgd(x0, lr=lr, steps=round_steps, poll=poll, stop_on_sat=True, search=search)
        rounds += 1
        iters += st["iters"]
        u = int(st["unsat"].min().item())
        best = u if best is None else min(best, u)
        solved = int(st["counter"][1].item()) > 0
        el = time.perf_counter() - t0
        if solved:
            return el, rounds, iters, 0, el
        if el >= timeout_s or (max_rounds and rounds >= max_rounds):
            return None, rounds, iters, best, el


def compare(net, tests, B, round_steps, timeout_s, variant, seed=0, lr=0.1, search=None, log=None, max_rounds=0,
            arms=("random", "learned"), index0=0):
    """Learned vs uniform random starts on each test instance.  Before either arm
    is timed, one untimed two-iteration run on the instance pays the solver's
    first-use costs (its workspace, state and driver streams); the arms then take
    turns going first (even instances random first, odd ones learned first), each
    with its own noise generator seeded per instance (tests[j] counts as instance
    index0 + j, so a test set split over several calls draws the same noise as one
    call).  Returns per-arm lists of run_arm results."""
    out = {arm: [] for arm in arms}
    for i, p in enumerate(tests, start=index0):
        d = afsat.Instance.from_arrays(p)
        d.pgd(uniform_start(d, B, (seed << 40) + (i << 20) + 0xFFFFF), lr=lr, steps=2, poll=1, stop_on_sat=False,
              search=search)
        order = tuple(arms) if i % 2 == 0 else tuple(reversed(arms))
        for arm in order:
            rounds = iter(range(1 << 20))
            base = (seed << 40) + (i << 20)          # round r of either arm draws noise with seed base + r
            if arm == "random":
                make = lambda: uniform_start(d, B, base + next(rounds))
            else:
                make = lambda: learned_start(net, d, B, base + next(rounds), **variant)
            out[arm].append(run_arm(d, make, round_steps, timeout_s, lr, search=search, max_rounds=max_rounds))
        if log:
            log("instance %d: %s" % (i, " | ".join("%s %s" % (arm, _fmt(out[arm][-1])) for arm in arms)))
        d.close()
    return out


def _fmt(r):
    return ("%.3f s, %d iterations" % (r[0], r[2])) if r[0] is not None else \
        ("unsolved after %.1f s, %d iterations, best unsat %d" % (r[4], r[2], r[3]))


def summarize(res, timeout_s):
    """Per arm: solved count, median time to a verified assignment and mean PAR-2
    (an unsolved run counts twice the timeout), median iterations to it (an
    unsolved run counts its iterations twice), mean best unsat of the unsolved."""
    out = {"timeout_s": timeout_s}
    for arm, rows in res.items():
        t = [r[0] for r in rows]
        solved = [x is not None for x in t]
        par2 = [x if x is not None else 2 * timeout_s for x in t]
        it_c = [r[2] if r[0] is not None else 2 * r[2] for r in rows]
        out[arm] = {"solved": int(sum(solved)), "of": len(rows),
                    "median_s": float(np.median(par2)), "par2_mean_s": float(np.mean(par2)),
                    "median_iters": float(np.median(it_c)),
                    "mean_best_unsat_unsolved": float(np.mean([r[3] for r in rows if r[0] is None]))
                    if not all(solved) else 0.0}
    return out
