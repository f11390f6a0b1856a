"""Host code of the library under AddressSanitizer and UndefinedBehaviorSanitizer.

The reader (csrc/parse.cpp), the packing (csrc/host.cpp) and the long-constraint
decomposition (csrc/decompose.cpp) are built with g++ and the two sanitizers
into small programs (tests/sanitize/*.cpp) that feed them random and mutated
inputs and check the structure of what comes back: the reader's arrays and
units; the packed buckets, slots, variable-to-slot transpose and
coefficient-table rows the kernels index; and the decomposition's announced
sizes, piece lengths, literal order, and that its result packs.  Host code only: no HIP
source is compiled here, and nothing runs on a GPU.
"""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2606_06641_amd", "csrc")
HERE = os.path.join(ROOT, "tests", "sanitize")
FLAGS = ["-std=c++17", "-O1", "-g", "-fsanitize=address,undefined", "-fno-sanitize-recover=undefined",
         "-I" + os.path.join(ROOT, "include"), "-I" + CSRC]
# instance.hpp (included by the reader) declares HIP runtime types
HIP_INC = ["-I/opt/rocm/include", "-D__HIP_PLATFORM_AMD__"]


def _build(tmp_path_factory, name, sources, extra=()):
    if shutil.which("g++") is None:
        pytest.skip("g++ not found")
    out = str(tmp_path_factory.mktemp("sanitize") / name)
    cmd = ["g++"] + FLAGS + list(extra) + ["-o", out] + sources
    r = subprocess.run(cmd, capture_output=True, text=True, timeout=300)
    if r.returncode != 0:
        if "cannot find" in r.stderr and ("asan" in r.stderr or "ubsan" in r.stderr):
            pytest.skip("sanitizer runtime not installed")
        raise AssertionError("build failed:\n" + r.stderr[-3000:])
    return out


def _run(exe, *args):
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
    r = subprocess.run([exe] + [str(a) for a in args], capture_output=True, text=True, timeout=600, env=env)
    assert r.returncode == 0, "exit %d\n%s\n%s" % (r.returncode, r.stdout[-2000:], r.stderr[-6000:])
    assert "runtime error" not in r.stderr, r.stderr[-6000:]
    fields = r.stdout.split()
    assert fields[0] == "ok", r.stdout
    return int(fields[1]), int(fields[2])


@pytest.fixture(scope="module")
def reader_exe(tmp_path_factory):
    return _build(tmp_path_factory, "reader_fuzz",
                  [os.path.join(HERE, "reader_fuzz.cpp"), os.path.join(CSRC, "parse.cpp")], HIP_INC)


@pytest.fixture(scope="module")
def pack_exe(tmp_path_factory):
    return _build(tmp_path_factory, "pack_fuzz",
                  [os.path.join(HERE, "pack_fuzz.cpp"), os.path.join(CSRC, "host.cpp")])


@pytest.fixture(scope="module")
def decompose_exe(tmp_path_factory):
    return _build(tmp_path_factory, "decompose_fuzz",
                  [os.path.join(HERE, "decompose_fuzz.cpp"), os.path.join(CSRC, "decompose.cpp"),
                   os.path.join(CSRC, "host.cpp")], HIP_INC)


@pytest.mark.parametrize("seed", [12345, 2024])
def test_reader_under_sanitizers(reader_exe, seed):
    accepted, rejected = _run(reader_exe, 60000, seed)
    # both the accepting and the rejecting paths are exercised in bulk
    assert accepted > 2000 and rejected > 2000


@pytest.mark.parametrize("seed", [777, 31337])
def test_packing_under_sanitizers(pack_exe, seed):
    packed, _ = _run(pack_exe, 200, seed)
    assert packed > 100


@pytest.mark.parametrize("seed", [99, 4242])
def test_decomposition_under_sanitizers(decompose_exe, seed):
    done, rejected = _run(decompose_exe, 200, seed)
    assert done > 150 and rejected > 0
