"""The ctypes structures of the binding against the C structures of
include/afsat.h: a small C program compiled here prints every structure's size
and each field's offset, and the binding's ctypes classes must agree field by
field (a mismatch would make the library read or write the wrong bytes)."""
import ctypes
import os
import shutil
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
from paper_2606_06641_amd import afsat  # noqa: E402

STRUCTS = {
    "afs_info": afsat._Info,
    "afs_bucket_info": afsat._BucketInfo,
    "afs_options": afsat._Options,
    "afs_pgd_state": afsat._PgdState,
    "afs_line_search": afsat._LineSearch,
    "afs_pgd_params": afsat._PgdParams,
    "afs_parsed_info": afsat._ParsedInfo,
}


def c_layout(tmp_path):
    if shutil.which("gcc") is None:
        pytest.skip("gcc not found")
    lines = ["#include <stdio.h>", "#include <stddef.h>", '#include "afsat.h"', "int main(void) {"]
    for cname, cls in STRUCTS.items():
        lines.append('    printf("%s size %%zu\\n", sizeof(%s));' % (cname, cname))
        for fname, _ in cls._fields_:
            lines.append('    printf("%s.%s %%zu\\n", offsetof(%s, %s));' % (cname, fname, cname, fname))
    lines += ["    return 0;", "}"]
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines) + "\n")
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-std=c11", "-I", os.path.join(ROOT, "include"), "-o", str(exe), str(src)],
                   check=True, capture_output=True, timeout=120)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True, timeout=60).stdout
    layout = {}
    for line in out.splitlines():
        parts = line.split()
        if parts[1] == "size":                 # "<struct> size <bytes>"
            layout[parts[0] + ".__size__"] = int(parts[2])
        else:                                  # "<struct>.<field> <offset>"
            layout[parts[0]] = int(parts[1])
    return layout


def test_ctypes_structures_match_the_header(tmp_path):
    got = c_layout(tmp_path)
    for cname, cls in STRUCTS.items():
        assert got[cname + ".__size__"] == ctypes.sizeof(cls), cname
        for fname, _ in cls._fields_:
            assert got["%s.%s" % (cname, fname)] == getattr(cls, fname).offset, (cname, fname)
