"""The binding's ctypes mirrors of the public structs have the C layout.

A C program compiled against include/ctof.h (host compiler only, no GPU
code) prints sizeof and offsetof of every field; each ctypes Structure in
the binding must agree field by field, so that a field added to the header
but not to the binding (or in another place) fails here rather than
corrupting a call.
"""

import ctypes
import os
import shutil
import subprocess

import pytest

from paper_2101_11680_amd import ctof

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

# C struct -> (ctypes mirror, renamed fields: Python name -> C name)
STRUCTS = {
    "ctof_geometry": (ctof._Geometry, {}),
    "ctof_fluorescence": (ctof._Fluorescence, {}),
    "ctof_mux": (ctof._Mux, {}),
    "ctof_solver_opts": (ctof._SolverOpts, {}),
    "ctof_solver_report": (ctof._SolverReport, {"lambda_": "lambda"}),
    "ctof_tuning": (ctof._Tuning, {}),
    "ctof_conv_desc": (ctof._ConvDesc, {}),
    "ctof_tensor": (ctof._Tensor, {}),
}


def _c_layout(tmp_path):
    cc = shutil.which("gcc") or shutil.which("cc")
    if cc is None:
        pytest.skip("no host C compiler")
    lines = ["#include <stdio.h>", "#include <stddef.h>", '#include "ctof.h"', "int main(void) {"]
    for cname, (cls, ren) in STRUCTS.items():
        lines.append(f'  printf("{cname} . %zu %zu\\n", sizeof({cname}), (size_t)0);')
        for f, _ in cls._fields_:
            cf = ren.get(f, f)
            lines.append(f'  printf("{cname} {f} %zu %zu\\n", sizeof((({cname} *)0)->{cf}), offsetof({cname}, {cf}));')
    lines += ["  return 0;", "}"]
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines) + "\n")
    exe = tmp_path / "layout"
    rocm = os.environ.get("ROCM_PATH", "/opt/rocm")
    res = subprocess.run([cc, "-D__HIP_PLATFORM_AMD__", "-I", os.path.join(ROOT, "include"), "-I",
                          os.path.join(rocm, "include"), str(src), "-o", str(exe)], capture_output=True, text=True)
    assert res.returncode == 0, res.stderr
    out = subprocess.run([str(exe)], capture_output=True, text=True, check=True).stdout
    layout = {}
    for line in out.splitlines():
        s, f, size, off = line.split()
        layout[(s, f)] = (int(size), int(off))
    return layout


def test_ctypes_mirrors_match_the_header(tmp_path):
    layout = _c_layout(tmp_path)
    for cname, (cls, _) in STRUCTS.items():
        assert ctypes.sizeof(cls) == layout[(cname, ".")][0], cname
        for f, _ in cls._fields_:
            d = getattr(cls, f)
            assert (d.size, d.offset) == layout[(cname, f)], (cname, f)
