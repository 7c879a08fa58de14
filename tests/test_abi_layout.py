"""The ctypes mirrors of the C-ABI structs against the header itself: a
small C program, compiled with the host compiler against include/ptflash.h,
prints sizeof and the offset of every field, which must equal what ctypes
lays out (a field added to the header and not to the binding, or in another
order, fails here)."""
import ctypes
import os
import shutil
import subprocess

import pytest

from paper_2205_03090_amd import _capi

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
STRUCTS = {"ptflash_problem": _capi.Problem, "ptflash_ragged_problem": _capi.RaggedProblem,
           "ptflash_options": _capi.Options, "ptflash_result": _capi.Result}


def test_struct_layout_matches_header(tmp_path):
    cc = shutil.which("gcc") or shutil.which("cc")
    if cc is None or not os.path.isdir("/opt/rocm/include"):
        pytest.skip("no host C compiler or HIP headers")
    lines = ["#include <stdio.h>", "#include <stddef.h>", '#include "ptflash.h"',
             "int main(void) {"]
    for cn, py in STRUCTS.items():
        lines.append(f'printf("{cn} %zu\\n", sizeof({cn}));')
        for f in py._fields_:
            lines.append(f'printf("{cn}.{f[0]} %zu\\n", offsetof({cn}, {f[0]}));')
    lines.append("return 0; }")
    src, exe = tmp_path / "layout.c", tmp_path / "layout"
    src.write_text("\n".join(lines) + "\n")
    subprocess.run([cc, "-D__HIP_PLATFORM_AMD__", "-I", os.path.join(ROOT, "include"),
                    "-I", "/opt/rocm/include", str(src), "-o", str(exe)], check=True)
    out = dict(l.rsplit(" ", 1) for l in
               subprocess.run([str(exe)], check=True, capture_output=True,
                              text=True).stdout.split("\n") if l)
    for cn, py in STRUCTS.items():
        assert int(out[cn]) == ctypes.sizeof(py), cn
        for f in py._fields_:
            assert int(out[f"{cn}.{f[0]}"]) == getattr(py, f[0]).offset, (cn, f[0])

