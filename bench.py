"""Throughput of the Accelerated Fourier SAT hot path on one MI355X.

One step is one iteration of Algorithm 1 over the whole batch: FE + gradient of
every constraint at every restart (all length buckets), the per-variable
gradient sum, the projected step, rounding and the exact unsat count.  The
headline workload is the largest single-GPU one: 64 planted instances of uneven
size (n log-uniform 500-50,000; 27.8M literal occurrences) packed into one
block-diagonal batch with 256 restarts each, all resident in HBM before timing
starts.  After the headline line, the same measurement runs on the mixed
n = 10,000 instance (1,024 restarts) and, as a forward + adjoint pass through
the autograd function, on the long-cardinality n = 50,000 instance (512
restarts); their lines go to stderr.

value = B * L / step time  (literal-evaluations per second; L = literal
occurrences).  The JSON line also carries the roofline of the dominant kernel
(timed with HIP events on the stream it runs on, inside the timed region), the
per-bucket roofline fractions, the peak probes, and the FP64 CPU oracle timed on
this host on a bounded sample.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload NAME]
                       [--no-extra] [--no-cpu-baseline]
"""
import argparse
import hashlib
import json
import os
import sys
import tempfile
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_HBM_GBS = 8000.0          # MI355X HBM3E, GB/s
PEAK_FP32_TFLOPS = 157.3       # MI355X FP32 vector, TFLOP/s
PEAK_BF16_TFLOPS = 2500.0      # MI355X dense BF16 MFMA, TFLOP/s

WORKLOAD_SEED = {"mixed10k": 2, "batch64": 3, "longcard50k": 4, "longchain20k": 6}
# oracle baseline sample: restart columns (0 = all of them)
CPU_RESTARTS = {"mixed10k": 0, "batch64": 16, "longcard50k": 16, "longchain20k": 16}


def flops_per_literal_eval(k):
    """Algorithmic FP32 flops of one literal-eval (one literal of a length-k
    constraint at one restart, FE + gradient) in the complex-product form: per
    complex root, forward 10 (factor 4, complex multiply 6) and backward 16
    (suffix update 6, leave-one-out product 6, contraction 4); per literal of the
    real root (k odd) 1 + 4.  F_k = 26 floor(k/2) + 5 (k mod 2)."""
    return 26 * (k // 2) + 5 * (k % 2)


def algorithmic_flops(k):
    """F_k flops for the k literal-evals of one constraint at one restart."""
    return k * flops_per_literal_eval(k)


def executed_flops(k):
    """Flops the kernels execute for one constraint at one restart in the
    rotated-factor form (each factor alpha (1 + i z) with the alpha powers in the
    tables): per complex root and literal z = -tan(h) y (1), one prefix and one
    suffix step by (1 + i z) (2 FMA each), the adjoint contraction (2 FMA): 13;
    per literal of the real root 4.  Cross-lane products, rescaling and padding
    are not counted."""
    return 13 * (k // 2) * k + 4 * k * (k % 2)


def kernel_source_hash():
    with open(os.path.join(ROOT, "paper_2606_06641_amd", "csrc", "fe_kernels.hip"), "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()[:16]


def stored_traffic(kernel_name, workload):
    """HBM traffic per launch from the committed rocprofv3 counter summary, or None
    when it is missing or the kernel source changed since it was taken."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    try:
        with open(path) as f:
            t = json.load(f)
    except (OSError, ValueError):
        return None
    e = t.get("%s@%s" % (kernel_name, workload))
    if not e or e.get("fe_kernels_sha256_16") != kernel_source_hash():
        return None
    return e.get("bytes_per_launch")


def cpu_baseline(inst, x0, lr, budget_s=12.0, threads=0, restarts=0, pgd=True):
    """The FP64 oracle timed on this host's cores (or `threads` of them), on all
    restarts or the first `restarts`: FE + gradient, and with `pgd` the step and
    the verification too (one Algorithm 1 iteration), repeated until budget_s."""
    import numpy as np
    import oracle
    threads = threads or oracle.default_threads()
    x = x0.astype(np.float64)
    if restarts:
        x = np.ascontiguousarray(x[:, :restarts])
    B = x.shape[1]
    reps, t_used = 0, 0.0
    t0 = time.perf_counter()
    while True:
        g = oracle.eval(inst, x, grad=True, nthreads=threads)["grad"]
        if pgd:
            x = oracle.step(x, g, lr)
            oracle.verify(inst, x.astype(np.float32))
        reps += 1
        t_used = time.perf_counter() - t0
        if t_used >= budget_s or reps >= 50:
            break
    value = B * inst.n_lits * reps / t_used
    what = "full PGD iterations (FE+grad, step, verify)" if pgd else "FE + gradient passes"
    return {"value": value, "unit": "literal-evals/s", "cores": threads, "kind": "oracle",
            "sample": "same instance, %s %d restarts, %d %s in FP64, %.1f s" % (
                "the first" if restarts else "all", B, reps, what, t_used)}


def timed(fn, reps):
    """Mean milliseconds of `reps` calls of fn (one launch each) on the current stream."""
    import torch
    fn()
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        work = fn()
    e1.record()
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / reps, work


def run_probes():
    """The peak probes (afs_probe_*): plain FP32 FMA issue, dense BF16 MFMA and a
    streaming copy, each timed over several launches with HIP events."""
    from paper_2606_06641_amd import afsat
    blocks = 256 * 8 * 4                   # 32 waves per CU
    names = ["fma_uniform", "fmac_vector", "mul", "complex_step", "fma_3address", "mul_uniform", "fmac_uniform"]
    fp32 = {}
    for v, name in enumerate(names):
        ms, fl = timed(lambda: afsat.probe("fma", blocks, iters=4096, variant=v), 5)
        fp32[name] = fl / (ms * 1e-3) / 1e12
    fma = max(fp32[n] for n in names if not n.startswith("mul"))
    ms, fl = timed(lambda: afsat.probe("mfma_bf16", blocks, iters=512), 5)
    mfma = fl / (ms * 1e-3) / 1e12
    nbytes = 1 << 30
    ms, by = timed(lambda: afsat.probe("copy", 256 * 16, nbytes=nbytes), 10)
    copy = by / (ms * 1e-3) / 1e9
    afsat.probe._bufs = None
    out = {"fp32_fma_tflops": fma, "fp32_by_form_tflops": fp32, "bf16_mfma_tflops": mfma, "hbm_copy_gbs": copy,
           "note": "measured on this device by afs_probe_fma (16 independent plain FP32 chains per lane, no packed "
                   "instructions: v_fma_f32 with uniform operands, v_fmac_f32 with per-lane operands, v_mul_f32, "
                   "the FE kernels' complex product step, three-address v_fma_f32 with per-lane operands, and "
                   "v_mul_f32 / v_fmac_f32 with a uniform (scalar-register) operand; "
                   "fp32_fma_tflops is the best FMA form), "
                   "afs_probe_mfma_bf16 (8 independent v_mfma_f32_16x16x32_bf16 accumulators per wave) and "
                   "afs_probe_copy (1 GiB, 16-byte non-temporal loads/stores; read + write bytes)"}
    print("probes: %s" % json.dumps(out), file=sys.stderr, flush=True)
    return out


def gemm_probe(rows, reps=20):
    """The learned-initialisation network's dense-layer kernel (BF16 MFMA, FP32
    accumulation) at its layer shape [rows x 64] . [64 x 64]: 2*rows*64*64 flops
    against rows*64*4 bytes read and rows*64*4 written (16 flops per byte, so
    HBM-bound on MI355X).  Prints one JSON line with the kernel's mean time from
    HIP events on its stream."""
    import torch
    from paper_2606_06641_amd import gnn
    dev = torch.device("cuda", 0)
    g = torch.Generator(device=dev).manual_seed(0)
    A = torch.rand((rows, 64), device=dev, generator=g) - 0.5
    W = torch.rand((64, 64), device=dev, generator=g) - 0.5
    for _ in range(3):
        gnn.gemm_bf16(A, W)
    stream = torch.cuda.current_stream(dev)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(reps):
        gnn.gemm_bf16(A, W)
    e1.record(stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    flops = 2.0 * rows * 64 * 64
    bytes_ = rows * 64 * 4 * 2.0 + 64 * 64 * 4
    print(json.dumps({"gemm_probe_rows": rows, "ms_per_launch": ms, "TFLOP/s": flops / ms / 1e9,
                      "GB/s": bytes_ / ms / 1e6, "hbm_frac": bytes_ / ms / 1e6 / PEAK_HBM_GBS,
                      "mfma_frac": flops / ms / 1e9 / PEAK_BF16_TFLOPS}), flush=True)


def copy_probe(mib):
    """A plain device-to-device copy of known size (reads and writes mib MiB each)."""
    import torch
    n = mib * (1 << 20) // 4
    a = torch.ones(n, dtype=torch.float32, device="cuda:0")
    b = torch.empty_like(a)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(5):
        b.copy_(a)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / 5
    print(json.dumps({"copy_probe_bytes": n * 4, "launches": 5, "ms_per_launch": ms,
                      "GB/s (read + write)": 2 * n * 4 / ms / 1e6}), flush=True)


def build_workload(name, W):
    """(instance or parts, restarts, description) of a named workload."""
    if name == "mixed10k":
        return W.mixed_10k(), 1024, ("planted mixed n=10000: 30000 clauses k3-8, 2000 XOR k3-5, "
                                     "500 CARD>=K k20-200; 1024 restarts; one PGD iteration per step")
    if name == "batch64":
        return W.uneven_batch(64), 256, ("64 planted instances, n log-uniform 500-50000, constraints/n "
                                         "3.5-4.2, 70% clauses k2-8, 10% NAE k2-8, 10% XOR k2-6, 10% "
                                         "CARD>=K k8-256 log-uniform; 256 restarts each, one block-diagonal "
                                         "batch; one PGD iteration per step")
    if name == "longcard50k":
        return W.long_card_50k(), 512, ("planted n=50000: 200000 clauses k3-10, 1000 CARD>=K k256-1024; "
                                        "512 restarts; one forward + adjoint (autograd) pass per step")
    if name == "longchain20k":
        return W.long_chain_20k(), 512, ("planted n=20000: 60000 clauses k3-8, 150 each of OR, XOR, NAE, AMO "
                                         "and EO k64-1024; 512 restarts; one PGD iteration per step")
    raise SystemExit("unknown workload %r" % name)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--workload", default="batch64",
                    choices=["mixed10k", "batch64", "longcard50k", "longchain20k", "learned3sat", "learned5k"])
    ap.add_argument("--no-extra", action="store_true",
                    help="only the chosen workload (by default the batch64 headline is followed by mixed10k "
                         "and longcard50k lines on stderr)")
    ap.add_argument("--train", type=int, default=0, help="learned-init workloads: training instances")
    ap.add_argument("--test", type=int, default=-1,
                    help="learned-init workloads: held-out test instances (default 100; 0: train only)")
    ap.add_argument("--test-offset", type=int, default=0, help="learned-init workloads: first test instance")
    ap.add_argument("--val", type=int, default=8, help="learned-init workloads: validation instances")
    ap.add_argument("--timeout", type=float, default=0.0, help="learned-init workloads: seconds per arm and instance")
    ap.add_argument("--val-timeout", type=float, default=2.0, help="learned-init workloads: validation timeout")
    ap.add_argument("--round-steps", type=int, default=200,
                    help="learned-init workloads: Algorithm 1 iterations per round of fresh starting points")
    ap.add_argument("--target-steps", type=int, default=200, help="learned-init workloads: solver iterations per target")
    ap.add_argument("--train-steps", type=int, default=1000, help="learned-init workloads: Adam steps")
    ap.add_argument("--ls-trials", type=int, default=0,
                    help="learned-init workloads: backtracking line search with this many trials (0: constant step)")
    ap.add_argument("--ls-step", type=float, default=4.0, help="learned-init workloads: line search maximum step")
    ap.add_argument("--save-net", default=None, help="learned-init workloads: save the trained network (.npz)")
    ap.add_argument("--load-net", default=None, help="learned-init workloads: load a trained network and only test")
    ap.add_argument("--select", action="store_true",
                    help="learned-init workloads: with --load-net, choose the inference variant again on validation")
    ap.add_argument("--restarts", type=int, default=0, help="override the workload's restart count")
    ap.add_argument("--lr", type=float, default=0.1)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-probes", action="store_true")
    ap.add_argument("--tune-out", default=None,
                    help="file receiving the shape cache with any newly tuned ranges (default: the temp directory)")
    ap.add_argument("--no-autotune", action="store_true",
                    help="use the default kernel shapes instead of the tuned ones")
    ap.add_argument("--shapes-cache", default=None,
                    help="tuned-shape cache to read (default: the package's tuned_shapes.txt)")
    ap.add_argument("--tune-tiles", action="store_true",
                    help="also tune work tiles and one-lane restarts per lane (slower iterations on mixed lengths)")
    ap.add_argument("--tune-max-cons", type=int, default=400,
                    help="constraints of a length range timed by the tuner when a range is not cached (0: all)")
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    ap.add_argument("--cpu-threads", type=int, default=0, help="oracle baseline threads (0: every host core)")
    ap.add_argument("--cpu-restarts", type=int, default=-1,
                    help="oracle baseline on the first R restarts only (default: per workload)")
    ap.add_argument("--search", type=int, default=0,
                    help="mixed10k only: time Algorithm 1 iterations with the backtracking line search "
                         "of this many trials instead of the constant-step hot path")
    ap.add_argument("--chain", default="",
                    help="comma-separated piece lengths: run Algorithm 1 on the long-constraint workload "
                         "(longchain20k) as given for --steps iterations, and decomposed into chains of "
                         "pieces of at most each length for --steps iterations and then to the same wall "
                         "time; compare time per iteration and the input's unsatisfied constraints")
    ap.add_argument("--gemm-probe", type=int, default=0,
                    help="only time the learned-initialisation network's dense-layer kernel on this many rows")
    ap.add_argument("--copy-probe-mib", type=int, default=0,
                    help="only run a plain device copy of this size (to calibrate byte counters)")
    args = ap.parse_args()
    if args.gemm_probe:
        gemm_probe(args.gemm_probe)
        return
    if args.copy_probe_mib:
        copy_probe(args.copy_probe_mib)
        return
    if args.gpus != 1:
        print("bench.py measures one GPU: the restart-sharded multi-GPU path is not built "
              "(--gpus must be 1)", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2606_06641_amd import workloads as W

    dev = torch.device("cuda", 0)
    torch.cuda.set_device(dev)
    if args.workload.startswith("learned"):
        learned_init_bench(args, W)
        return
    if args.chain:
        chain_bench(args, W)
        return
    if args.search:
        if args.workload != "mixed10k":
            raise SystemExit("--search takes --workload mixed10k")
        throughput(args, "mixed10k", W, None)
        return
    probes = None if args.no_probes else run_probes()
    line = throughput(args, args.workload, W, probes)
    print(json.dumps(line), flush=True)
    if args.workload == "batch64" and not args.no_extra:
        for name in ("mixed10k", "longcard50k"):
            extra = throughput(args, name, W, probes)
            print("extra config line: " + json.dumps(extra), file=sys.stderr, flush=True)


def throughput(args, name, W, probes):
    """One workload: setup, per-bucket timing, warm-up, exactly args.steps timed
    steps, the dominant kernel's roofline, the oracle baseline.  Returns the line."""
    import numpy as np
    import torch
    from paper_2606_06641_amd import afsat

    dev = torch.device("cuda", 0)
    t_setup = time.perf_counter()
    work, B, desc = build_workload(name, W)
    B = args.restarts or B
    parts = work if isinstance(work, list) else None
    inst = _concat(parts, W) if parts is not None else work   # the block-diagonal instance
    x0 = W.uniform_x0(inst.n, B, workload=WORKLOAD_SEED[name])
    shapes = []
    if not args.no_autotune:
        from paper_2606_06641_amd import autotune
        out = args.tune_out or os.path.join(tempfile.gettempdir(), "afsat_tuned_shapes.txt")
        os.makedirs(os.path.dirname(os.path.abspath(out)), exist_ok=True)
        shapes, _ = autotune.tune(inst, B, cache_path=args.shapes_cache or autotune.DEFAULT_CACHE, out_path=out,
                                  log=lambda m: print(m, file=sys.stderr, flush=True), max_cons=args.tune_max_cons,
                                  tiles=args.tune_tiles)
    if parts is not None:
        d = afsat.Instance.batch(parts, device=0, shapes=shapes)
    else:
        d = afsat.Instance.from_arrays(inst, device=0, shapes=shapes)
    print("[%s] setup %.1f s: n=%d C=%d L=%d B=%d parts=%d" % (name, time.perf_counter() - t_setup, d.n, d.n_cons,
          d.n_lits, B, d.n_inst), file=sys.stderr, flush=True)
    x = torch.from_numpy(x0).to(dev)
    ws = d.workspace(B)
    st = d.pgd_state(B)
    d.pgd_init(x, st, ws)
    if args.search:
        return search_bench(args, d, x, st, ws, B, desc)
    stream = torch.cuda.current_stream(dev)
    buckets = d.buckets()
    nb = len(buckets)
    autograd = name == "longcard50k"
    if autograd:
        x.requires_grad_(True)

    def step(ev=None, dom=None):
        if autograd:
            # forward (FE only) + backward (adjoint, recomputed) through FEObjective;
            # the bracketed region is the whole adjoint pass
            obj = afsat.FEObjective.apply(x, d)
            if ev is not None:
                ev[0].record(stream)
            x.grad = None
            obj.sum().backward()
            if ev is not None:
                ev[1].record(stream)
            return
        if ev is None:
            d.fe_grad(x, ws, 0, nb)
        else:
            # the dominant bucket first, alone between the events (its duration is
            # the kernel's own); then every other bucket in one call, where the
            # library runs the short ones beside the long ones and the long ones
            # two at a time
            ev[0].record(stream)
            d.fe_grad(x, ws, dom, dom + 1)
            ev[1].record(stream)
            if rest:
                d.fe_grad_buckets(x, ws, rest)
        d.pgd_update(x, st, args.lr, None, ws)

    # per-bucket timing (outside the timed region) to find the dominant kernel;
    # each bucket is launched alone once first (code loading), and the warm-up
    # steps come after, in the timed steps' layout, so that every launch of the
    # dominant kernel in the run is a solo one (as in a profile of the run)
    xd = x.detach()
    for i in range(nb):
        d.fe_grad(xd, ws, i, i + 1)
    torch.cuda.synchronize()
    per_bucket = []
    for i in range(nb):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(3):
            d.fe_grad(xd, ws, i, i + 1)
        e1.record(stream)
        torch.cuda.synchronize()
        per_bucket.append(e0.elapsed_time(e1) / 3)
    dom = int(np.argmax(per_bucket))
    bk = buckets[dom]
    rest = [i for i in range(nb) if i != dom]
    warm = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
            for _ in range(max(1, args.warmup))]
    for ev in warm:
        step(ev, dom)
    torch.cuda.synchronize()

    # timed region: exactly K steps, events around the dominant kernel's launch
    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
           for _ in range(args.steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(args.steps):
        step(evs[k], dom)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ms_per_step = (t1 - t0) * 1e3 / args.steps
    dom_ms = float(np.mean([a.elapsed_time(b) for a, b in evs]))
    value = B * d.n_lits / (ms_per_step * 1e-3)

    # roofline of the dominant kernel
    lens = np.diff(np.asarray(inst.con_off))
    smap = d.slot_map()
    slot_of_lit = np.empty_like(smap)
    slot_of_lit[smap] = np.arange(len(smap))
    first_slot = slot_of_lit[np.asarray(inst.con_off[:-1])]
    in_b = (first_slot >= bk.slot0) & (first_slot < bk.slot0 + bk.n_lits)
    kb = lens[in_b]
    table = bucket_roofline(name, buckets, per_bucket, lens, first_slot, B)
    kname = "fe_grad_seg<%d,%d>" % (bk.lanes_per_restart, bk.lits_per_lane) if bk.lanes_per_restart > 1 \
        else "fe_grad_short<%d>" % bk.k_hi
    if autograd:
        # the bracketed region is the whole adjoint pass (every bucket + gradient sum)
        flops = float(B * sum(algorithmic_flops(int(k)) for k in lens))
        exe = float(B * sum(executed_flops(int(k)) for k in lens))
        roof = {"bound": "alu", "achieved": flops / (dom_ms * 1e-3) / 1e12, "peak": PEAK_FP32_TFLOPS,
                "unit": "TFLOP/s", "kernel": "adjoint pass (all fe_grad buckets + gradient sum)",
                "flops_per_launch": flops, "executed_tflops": exe / (dom_ms * 1e-3) / 1e12}
    elif bk.lanes_per_restart == 1 and bk.k_hi <= 8:
        bytes_per_launch = 8.0 * B * kb.sum()
        roof = {"bound": "hbm", "achieved": bytes_per_launch / (dom_ms * 1e-3) / 1e9, "peak": PEAK_HBM_GBS,
                "unit": "GB/s", "kernel": kname, "bytes_per_launch": bytes_per_launch}
    else:
        flops = float(B * sum(algorithmic_flops(int(k)) for k in kb))
        exe = float(B * sum(executed_flops(int(k)) for k in kb))
        roof = {"bound": "alu", "achieved": flops / (dom_ms * 1e-3) / 1e12, "peak": PEAK_FP32_TFLOPS,
                "unit": "TFLOP/s", "kernel": kname, "k_range": [bk.k_lo, bk.k_hi], "flops_per_launch": flops,
                "evals_per_launch": float(B * kb.sum()), "executed_tflops": exe / (dom_ms * 1e-3) / 1e12}
    roof["frac"] = roof["achieved"] / roof["peak"]
    roof["ms_per_launch"] = dom_ms
    if roof["bound"] == "alu":
        roof["flop_model"] = "F_k = 26 floor(k/2) + 5 (k mod 2) per literal-eval"
    if probes:
        p = probes["fp32_fma_tflops"] if roof["bound"] == "alu" else probes["hbm_copy_gbs"]
        roof["peak_probe"] = p
        roof["frac_probe"] = roof["achieved"] / p
    roof["traffic"] = None if autograd else stored_traffic(kname, name)

    line = {
        "metric": "FE+grad literal-evals/s",
        "value": value,
        "unit": "literal-evals/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": name + ": " + desc, "n_vars": d.n, "n_cons": d.n_cons, "n_lits": d.n_lits,
                   "restarts": B, "parts": d.n_inst, "lr": args.lr,
                   "shapes": [list(sh) for sh in shapes]},
        "roofline": roof,
        "buckets": table,
    }
    if probes:
        line["probes"] = probes
    if not autograd:
        print("[%s] (part, restart) pairs verified after %d iterations: %d" % (
            name, int(st["counter"][0].item()), int(st["counter"][1].item())), file=sys.stderr, flush=True)
    del ws, st, x, xd
    d.close()
    torch.cuda.empty_cache()
    if not args.no_cpu_baseline:
        r = CPU_RESTARTS[name] if args.cpu_restarts < 0 else args.cpu_restarts
        line["cpu_baseline"] = cpu_baseline(inst, x0, args.lr, args.cpu_seconds, args.cpu_threads, r,
                                            pgd=not autograd)
    return line


def chain_bench(args, W):
    """Long-constraint decomposition as a comparison point (Sec. 5): Algorithm 1
    (constant step, the library's graph-captured driver) on the planted
    long-constraint workload as given, where every constraint is evaluated whole
    by the count-basis kernels, and on the same instance decomposed into chains
    of pieces of at most L literals (afs_decompose).  Per form: milliseconds per
    iteration over --steps iterations from uniform starting points, and the
    input's unsatisfied constraints under the points restricted to its own
    variables, in total and per constraint class (exact counts by the library's
    verification kernels on per-class sub-instances); a decomposed form then
    continues to the wall time the form as given took, and is counted again.
    One JSON line per form."""
    import numpy as np
    import torch
    from paper_2606_06641_amd import afsat, autotune

    inst = W.long_chain_20k()
    B = args.restarts or 512
    dev = torch.device("cuda", 0)
    lens_in = np.diff(np.asarray(inst.con_off))
    types_in = np.asarray(inst.types)

    def subset(sel):
        ks = lens_in[sel]
        off = np.zeros(len(sel) + 1, np.int64)
        np.cumsum(ks, out=off[1:])
        lits = np.concatenate([inst.lits[inst.con_off[c]:inst.con_off[c + 1]] for c in sel])
        return W.Instance(n=inst.n, con_off=off, lits=lits, types=types_in[sel], params=np.asarray(inst.params)[sel])

    classes = {}
    for t in sorted(set(types_in.tolist())):
        for long_ in (False, True):
            sel = np.nonzero((types_in == t) & ((lens_in > 16) == long_))[0]
            if sel.size:
                name = "%s k%d-%d" % (W.TYPE_NAMES[t], lens_in[sel].min(), lens_in[sel].max())
                classes[name] = afsat.Instance.from_arrays(subset(sel), device=0)
    native = afsat.Instance.from_arrays(inst, device=0)

    def input_unsat(x, iters):
        xs = x[:inst.n].contiguous()
        tot = native.round_verify(xs).cpu().numpy()
        by = {name: round(float(h.round_verify(xs).float().mean()), 2) for name, h in classes.items()}
        return {"iterations": iters, "best": int(tot.min()), "mean": round(float(tot.mean()), 2),
                "mean_by_class": by}

    poll = max(1, min(args.steps, 100))
    native_ms = None
    for L in [0] + [int(v) for v in args.chain.split(",") if v]:
        t_setup = time.perf_counter()
        form = inst if L == 0 else afsat.decompose(inst, L)
        shapes = []
        if not args.no_autotune:
            out = args.tune_out or os.path.join(tempfile.gettempdir(), "afsat_tuned_shapes.txt")
            shapes, _ = autotune.tune(form, B, cache_path=autotune.DEFAULT_CACHE, out_path=out,
                                      log=lambda m: print(m, file=sys.stderr, flush=True), max_cons=400)
        d = afsat.Instance.from_arrays(form, device=0, shapes=shapes)
        setup = time.perf_counter() - t_setup
        x = torch.from_numpy(W.uniform_x0(d.n, B, workload=6)).to(dev)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        d.pgd(x, args.lr, args.steps, poll=poll, stop_on_sat=False)
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t0) * 1e3 / args.steps
        line = {"metric": "PGD iterations/s", "value": 1e3 / ms, "unit": "iterations/s", "n_gpus": 1,
                "steps": args.steps, "warmup": 0, "ms_per_step": ms, "higher_is_better": True,
                "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
                "config": {"workload": "planted n=20000: 60000 clauses k3-8, 150 each of OR, XOR, NAE, AMO and "
                                       "EO k64-1024; %d restarts; " % B
                                       + ("as given" if L == 0 else
                                          "decomposed into chains of pieces of at most %d literals" % L),
                           "max_len": L or int(lens_in.max()), "n_vars": d.n, "n_cons": d.n_cons,
                           "n_lits": d.n_lits, "restarts": B, "lr": args.lr, "setup_s": round(setup, 2),
                           "shapes": [list(sh) for sh in shapes]},
                "input_literal_evals_per_s": B * int(inst.con_off[-1]) / (ms * 1e-3),
                "input_unsat": [input_unsat(x, args.steps)]}
        if L == 0:
            native_ms = ms
        elif native_ms is not None:
            more = int(args.steps * native_ms / ms) - args.steps
            if more > 0:
                d.pgd(x, args.lr, more, poll=poll, stop_on_sat=False)
                line["input_unsat"].append(input_unsat(x, args.steps + more))
        print(json.dumps(line), flush=True)
        if d is not native:
            d.close()


def search_bench(args, d, x, st, ws, B, desc):
    """Iterations of Algorithm 1 with the backtracking line search (one FE +
    gradient pass, `--search` forward-only FE passes and trial points, the step,
    rounding and verification per iteration): iterations per second."""
    import torch
    from paper_2606_06641_amd import afsat
    if d.n_inst != 1:
        raise SystemExit("the line search takes a plain instance (--workload mixed10k)")
    ls = afsat.LineSearch(1.0, 0.5, 1e-4, args.search)
    eta = torch.empty(B, dtype=torch.float32, device=x.device)
    for _ in range(args.warmup):
        d.search_step(x, st, ls, eta=eta, ws=ws)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        d.search_step(x, st, ls, eta=eta, ws=ws)
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3 / args.steps
    e = eta.cpu()
    print("step lengths after the last iteration: %s" % {float(v): int((e == v).sum()) for v in e.unique()},
          file=sys.stderr, flush=True)
    print(json.dumps({"metric": "line-search PGD iterations/s", "value": 1e3 / ms, "unit": "iterations/s",
                      "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms,
                      "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
                      "data": "synthetic",
                      "config": {"workload": desc, "restarts": B, "trials": args.search, "max_step": 1.0,
                                 "shrink": 0.5, "armijo": 1e-4}}), flush=True)


def bucket_roofline(name, buckets, per_bucket_ms, lens, first_slot, B):
    """Per length bucket (each timed alone, outside the timed region): literal-evals
    per second against the bucket's own roofline min(P_VALU / F, BW / Q), with F
    the algorithmic flops per literal-eval of its lengths (F_k) and Q = 8 B (x
    gather and adjoint write).  Printed to stderr and returned as rows
    [k_lo, k_hi, J, S, constraints, ms, bound, fraction, tile, restarts per lane]."""
    print("[%s] bucket roofline (alone): k range, shape, constraints, ms, literal-evals/s, TFLOP/s (F_k), "
          "GB/s, bound, fraction" % name, file=sys.stderr)
    rows = []
    for b, t in zip(buckets, per_bucket_ms):
        sel = (first_slot >= b.slot0) & (first_slot < b.slot0 + b.n_lits)
        ks = lens[sel]
        evals = float(B * ks.sum())
        flops = float(B * sum(algorithmic_flops(int(k)) for k in ks))
        sec = t * 1e-3
        rate = evals / sec
        alu_ceiling = PEAK_FP32_TFLOPS * 1e12 / (flops / evals)
        hbm_ceiling = PEAK_HBM_GBS * 1e9 / 8.0
        bound = "alu" if alu_ceiling < hbm_ceiling else "hbm"
        frac = rate / min(alu_ceiling, hbm_ceiling)
        rows.append([b.k_lo, b.k_hi, b.lanes_per_restart, b.lits_per_lane, int(sel.sum()), round(t, 4), bound,
                     round(frac, 3), b.tile, b.rpl])
        print("  [%4d-%4d] J%-2d S%-2d t%-2d r%d %6d %8.3f ms %10.3e %7.2f %8.1f %s %.3f" % (
            b.k_lo, b.k_hi, b.lanes_per_restart, b.lits_per_lane, b.tile, b.rpl, int(sel.sum()), t, rate,
            flops / sec / 1e12, 8.0 * evals / sec / 1e9, bound, frac), file=sys.stderr, flush=True)
    return rows


def _gen_instances(make, seeds, workers=8):
    """Instances make(seed) for every seed, generated in worker processes."""
    from concurrent.futures import ProcessPoolExecutor
    if len(seeds) < 64:
        return [make(i) for i in seeds]
    with ProcessPoolExecutor(max_workers=workers) as ex:
        return list(ex.map(make, seeds, chunksize=16))


def _make_3sat(i):
    from paper_2606_06641_amd import workloads as W
    return W.planted_3sat(n=100, m=426, instance=i)


def _make_5k(i):
    from paper_2606_06641_amd import workloads as W
    return W.mixed_5k(instance=i)


def learned_init_bench(args, W):
    """Time to a verified assignment from learned vs uniform random starting
    points (the learned-initialisation row).

    learned5k: planted mixed instances of the n = 10k workload's shape at
    n = 5,000 (15,000 clauses k3-8, 1,000 XOR k3-5, 250 CARD>=K k20-200);
    learned3sat: planted random 3-SAT, n = 100, 426 clauses.  The network
    (3 rounds, width 64) trains on targets the solver itself produces on the
    training instances (its best restart: a verified one where there is one,
    else the fewest unsatisfied constraints); the way its output becomes starting
    points (sign-sampling temperature, or a blend with the noise) is chosen on
    separate validation instances; both arms then run on held-out test
    instances, 1,024 restarts each, Algorithm 1 with lr 0.1 in rounds of
    --round-steps iterations from fresh starting points, until a restart
    verifies or --timeout seconds pass.  --save-net / --load-net split training
    and testing across runs."""
    import numpy as np
    import torch
    from paper_2606_06641_amd import gnn
    log = lambda m: print(m, file=sys.stderr, flush=True)
    t0 = time.perf_counter()
    five = args.workload == "learned5k"
    make = _make_5k if five else _make_3sat
    n_train = args.train or (2000 if five else 512)
    n_val, n_test = args.val, (100 if args.test < 0 else args.test)
    B = args.restarts or 1024
    timeout = args.timeout or (20.0 if five else 3.0)
    desc = ("planted mixed n=5000: 15000 clauses k3-8, 1000 XOR k3-5, 250 CARD>=K k20-200" if five
            else "planted 3-SAT n=100 m=426")
    search = (args.ls_step, 0.5, 1e-4, args.ls_trials) if args.ls_trials else None
    net = gnn.GNN(rounds=3, seed=1)
    info = {}
    if args.load_net:
        z = np.load(args.load_net, allow_pickle=False)
        net.load_state_dict({k: z[k] for k in ("params", "m", "v", "t")})
        info = json.loads(str(z["info"]))
        log("loaded network from %s: %s" % (args.load_net, info))
    else:
        train_set = _gen_instances(make, [10000 + i for i in range(n_train)])
        log("generated %d training instances (%.1f s)" % (n_train, time.perf_counter() - t0))
        targets, verified, unsat_of = gnn.collect_targets(train_set, B=256, steps=args.target_steps)
        info = {"train": n_train, "target_steps": args.target_steps, "targets_verified": verified,
                "target_unsat_median": float(np.median(unsat_of)), "target_unsat_max": int(max(unsat_of)),
                "train_steps": args.train_steps}
        log("targets: %d of %d verified, median unsat %.1f (%.1f s)" % (
            verified, n_train, np.median(unsat_of), time.perf_counter() - t0))
        losses = gnn.train(net, train_set, targets, args.train_steps, log=log)
        info["final_loss"] = losses[-1][1] if losses else None
        del train_set, targets
        log("trained (%.1f s)" % (time.perf_counter() - t0))
    if not args.load_net or args.select:
        # how the network's output becomes starting points: chosen on validation
        # instances (learned arm only) by solved count, then by the mean best
        # unsatisfied count (solves are rare on the mixed shape, so the count of
        # constraints left is the finer signal)
        val_set = [make(20000 + i) for i in range(n_val)]
        variants = [dict(sample=True, temperature=T) for T in (1.0, 2.0, 4.0)] + [dict(mix=0.8), dict(mix=0.5)]
        best_key = None
        info["validation"] = []
        for v in variants:
            res = gnn.compare(net, val_set, B, args.round_steps, args.val_timeout, v, seed=1, lr=args.lr,
                              search=search, arms=("learned",))
            rows = res["learned"]
            solved = sum(r[0] is not None for r in rows)
            mean_best = float(np.mean([r[3] for r in rows]))
            key = (-solved, mean_best)
            log("validation %s: solved %d of %d, mean best unsat %.2f" % (v, solved, len(rows), mean_best))
            info["validation"].append({"variant": v, "solved": solved, "mean_best_unsat": mean_best})
            if best_key is None or key < best_key:
                info["inference"], best_key = v, key
        info["validation_instances"], info["validation_timeout_s"] = n_val, args.val_timeout
    if args.save_net:
        sd = net.state_dict()
        np.savez(args.save_net, params=sd["params"], m=sd["m"], v=sd["v"], t=sd["t"], info=json.dumps(info))
        log("saved network to %s" % args.save_net)
    if not n_test:
        print(json.dumps({"trained": info, "wall_s": time.perf_counter() - t0}), flush=True)
        return
    test_set = [make(30000 + i) for i in range(args.test_offset, args.test_offset + n_test)]
    res = gnn.compare(net, test_set, B, args.round_steps, timeout, info["inference"], seed=2, lr=args.lr,
                      search=search, log=log, index0=args.test_offset)
    summ = gnn.summarize(res, timeout)
    rm, lm = summ["random"]["median_s"], summ["learned"]["median_s"]
    solved_any = summ["random"]["solved"] + summ["learned"]["solved"] > 0
    line = {"metric": "median time to a verified assignment, learned init",
            "value": lm if summ["learned"]["solved"] * 2 > n_test else None,
            "unit": "s", "higher_is_better": False, "n_gpus": 1, "dtype": "f32 (solver), bf16 MFMA (network)",
            "data": "synthetic",
            "config": {"workload": desc, "test": n_test, "test_offset": args.test_offset, "restarts": B,
                       "round_iterations": args.round_steps, "timeout_s": timeout, "lr": args.lr,
                       "line_search": list(search) if search else None, "network": info},
            "learned": summ["learned"], "random": summ["random"],
            "vs_random_median": (lm / rm) if solved_any else None,
            "per_instance": {arm: [[None if r[0] is None else round(r[0], 4), r[2], r[3]] for r in rows]
                             for arm, rows in res.items()},
            "wall_s": time.perf_counter() - t0}
    print(json.dumps(line), flush=True)


def _concat(parts, W):
    import numpy as np
    offs, lits, types, params = [np.zeros(1, np.int64)], [], [], []
    base = v0 = 0
    for p in parts:
        offs.append(np.asarray(p.con_off[1:], np.int64) + base)
        base += p.n_lits
        lits.append(np.where(p.lits > 0, p.lits + v0, p.lits - v0).astype(np.int32))
        types.append(p.types)
        params.append(p.params)
        v0 += p.n
    return W.Instance(n=v0, con_off=np.concatenate(offs), lits=np.concatenate(lits),
                      types=np.concatenate(types), params=np.concatenate(params))


if __name__ == "__main__":
    main()
