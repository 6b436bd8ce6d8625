"""The ctypes mirrors of the C-ABI structs in the binding have the C
compiler's size and field offsets (compiled from include/mxl.h with gcc),
so a field added on one side only fails here, on the CPU."""
import ctypes as C
import os
import shutil
import subprocess
import tempfile

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

PAIRS = [("mxl_format_params", "FormatParams"), ("mxl_criteria", "Criteria"),
         ("mxl_solve_info", "SolveInfo"), ("mxl_op_desc", "OpDesc"), ("mxl_ir_params", "IrParams"),
         ("mxl_tuning", "Tuning"), ("mxl_kernel_class", "KernelClass"), ("mxl_select_info", "SelectInfo")]


def _binding_structs():
    """The binding's ctypes classes (importing the package loads libmxl.so
    with ctypes only; no GPU call is made)."""
    import paper_2006_16852_amd as m
    return {p: getattr(m, p) for _, p in PAIRS}


@pytest.mark.skipif(shutil.which("gcc") is None, reason="needs gcc")
def test_struct_layouts_match_header():
    ns = _binding_structs()
    lines = ['#include <stddef.h>', '#include <stdio.h>', '#include "mxl.h"', "int main(void) {"]
    for cname, pname in PAIRS:
        lines.append(f'printf("{pname} size %zu\\n", sizeof({cname}));')
        for f, _ in ns[pname]._fields_:
            lines.append(f'printf("{pname} {f} %zu\\n", offsetof({cname}, {f}));')
    lines.append("return 0; }")
    with tempfile.TemporaryDirectory() as d:
        c = os.path.join(d, "layout.c")
        exe = os.path.join(d, "layout")
        open(c, "w").write("\n".join(lines) + "\n")
        subprocess.check_call(["gcc", "-std=c99", "-I", os.path.join(ROOT, "include"), "-o", exe, c])
        out = subprocess.check_output([exe], text=True).split("\n")
    got = {}
    for ln in out:
        if ln:
            name, field, val = ln.split()
            got[(name, field)] = int(val)
    for _, pname in PAIRS:
        cls = ns[pname]
        assert got[(pname, "size")] == C.sizeof(cls), pname
        for f, _ in cls._fields_:
            assert got[(pname, f)] == getattr(cls, f).offset, (pname, f)
