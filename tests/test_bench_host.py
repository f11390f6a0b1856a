"""Host-side logic of bench.py, on the CPU: the flop model, the lookup of the
committed traffic counters, and the one-GPU guard."""
import json
import os
import subprocess
import sys
from fractions import Fraction

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


def complex_form_flops(k):
    """F_k counted operation by operation from the complex-product form (FE +
    gradient of one literal-eval): per complex root a factor (4), a complex
    multiply into the prefix (6), then backward a suffix update (6), the
    leave-one-out product (6) and the contraction (4); per literal of the real
    root of an odd length one multiply forward and 4 backward."""
    per_root = 4 + 6 + 6 + 6 + 4
    return per_root * (k // 2) + (1 + 4) * (k % 2)


@pytest.mark.parametrize("k", [1, 2, 3, 16, 17, 255, 256, 1024])
def test_flop_model(k):
    assert bench.flops_per_literal_eval(k) == complex_form_flops(k)
    assert bench.algorithmic_flops(k) == k * complex_form_flops(k)
    # the kernels execute exactly half of F_k's complex-root work (13 of 26 per
    # root and literal) and 4 of the real root's 5
    ex = bench.executed_flops(k)
    assert ex == 13 * (k // 2) * k + 4 * k * (k % 2)
    if k % 2 == 0:
        assert Fraction(ex, bench.algorithmic_flops(k)) == Fraction(1, 2)
    assert ex <= bench.algorithmic_flops(k)


def test_stored_traffic_follows_the_kernel_source():
    with open(os.path.join(ROOT, "profiles", "traffic.json")) as f:
        table = json.load(f)
    current = bench.kernel_source_hash()
    for key, entry in table.items():
        kernel, workload = key.split("@")
        got = bench.stored_traffic(kernel, workload)
        if entry.get("fe_kernels_sha256_16") == current:
            assert got == entry["bytes_per_launch"] and got > 0
        else:
            assert got is None
    assert bench.stored_traffic("no_such_kernel", "batch64") is None


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr and r.stdout == ""
