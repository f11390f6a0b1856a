"""Build ``libafsat.so`` (HIP kernels for gfx950 + host packing + C ABI) in-tree.

Run ``python -m paper_2606_06641_amd.build``.  hipcc cross-compiles the device
code without a GPU.  Translation units are compiled in parallel and linked into
one shared library beside this file.
"""
import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
INCLUDE = os.path.join(ROOT, "include")
OBJDIR = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libafsat.so")
ARCH = os.environ.get("AFS_OFFLOAD_ARCH", "gfx950")

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
COMMON = ["-O3", "-std=c++17", "-fPIC", "-Wall", "-I", INCLUDE, "-I", CSRC]
# Device code is built without packed-FP32 instructions.
DEVICE = ["--offload-arch=" + ARCH, "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
          "-munsafe-fp-atomics"]



def fe_revision():
    """First 12 hex digits of the SHA-256 of the FE kernels' source: the revision
    that keys the autotuner's cache."""
    import hashlib
    with open(os.path.join(CSRC, "fe_kernels.hip"), "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()[:12]


HOST_HIP = [HIPCC] + COMMON + ["-x", "c++", "-D__HIP_PLATFORM_AMD__", "-I", "/opt/rocm/include"]
SOURCES = [
    ("host.cpp", ["g++"] + COMMON),
    ("api.cpp", HOST_HIP),
    ("autotune.cpp", HOST_HIP + ['-DAFS_FE_REV="%s"' % fe_revision()]),
    ("parse.cpp", HOST_HIP),
    ("forms.cpp", HOST_HIP),
    ("decompose.cpp", HOST_HIP),
    ("fe_kernels.hip", [HIPCC] + COMMON + DEVICE),
    ("update_kernels.hip", [HIPCC] + COMMON + DEVICE),
    ("search_kernels.hip", [HIPCC] + COMMON + DEVICE),
    ("forms.hip", [HIPCC] + COMMON + DEVICE),
    ("gnn.hip", [HIPCC] + COMMON + DEVICE),
    ("probes.hip", [HIPCC] + COMMON + DEVICE),
    ("noalloc.hip", [HIPCC] + COMMON + DEVICE),
]


def _compile(item, verbose):
    name, cmd = item
    src = os.path.join(CSRC, name)
    obj = os.path.join(OBJDIR, name + ".o")
    full = cmd + ["-c", src, "-o", obj]
    if verbose:
        print(" ".join(full), flush=True)
    r = subprocess.run(full, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("compile failed: %s\n%s%s" % (" ".join(full), r.stdout, r.stderr))
    return obj


def build(verbose: bool = False) -> str:
    os.makedirs(OBJDIR, exist_ok=True)
    with ThreadPoolExecutor(max_workers=len(SOURCES)) as ex:
        objs = list(ex.map(lambda it: _compile(it, verbose), SOURCES))
    tmp = LIB + ".tmp%d" % os.getpid()
    link = [HIPCC, "-shared", "-fPIC", "--offload-arch=" + ARCH, "-o", tmp] + objs + ["-lamdhip64"]
    if verbose:
        print(" ".join(link), flush=True)
    r = subprocess.run(link, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("link failed:\n%s%s" % (r.stdout, r.stderr))
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    build(verbose=True)
    print("built", LIB)
    sys.exit(0)
