"""The Python binding's ctypes structures against the C header: every field
at the offset and of the size the C compiler gives it, and the same total
size (compiled with gcc from include/amg_p2.h; no GPU needed)."""
import ctypes
import os
import shutil
import subprocess

import pytest

from paper_1503_01287_amd import _lib as C

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
STRUCTS = {"amg_system": C.AmgSystem, "amg_params": C.AmgParams, "amg_result": C.AmgResult,
           "amg_level_info": C.AmgLevelInfo}


@pytest.mark.skipif(shutil.which("gcc") is None, reason="needs gcc")
def test_struct_layouts_match_the_header(tmp_path):
    lines = ["#include <stdio.h>", "#include <stddef.h>", '#include "amg_p2.h"', "int main(void) {"]
    for cname, py in STRUCTS.items():
        lines.append(f'printf("{cname} size %zu\\n", sizeof({cname}));')
        for f in py._fields_:
            lines.append(f'printf("{cname} {f[0]} %zu %zu\\n", offsetof({cname}, {f[0]}), '
                         f'sizeof((({cname} *)0)->{f[0]}));')
    lines += ["return 0;", "}"]
    src = tmp_path / "abi.c"
    src.write_text("\n".join(lines) + "\n")
    exe = tmp_path / "abi"
    subprocess.check_call(["gcc", "-std=c99", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)])
    out = subprocess.check_output([str(exe)], text=True).split("\n")
    seen = 0
    for line in out:
        if not line:
            continue
        parts = line.split()
        py = STRUCTS[parts[0]]
        if parts[1] == "size":
            assert ctypes.sizeof(py) == int(parts[2]), line
        else:
            field = getattr(py, parts[1])
            assert (field.offset, field.size) == (int(parts[2]), int(parts[3])), line
        seen += 1
    assert seen == sum(len(p._fields_) + 1 for p in STRUCTS.values())
