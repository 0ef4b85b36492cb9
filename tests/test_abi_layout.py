"""The ctypes mirrors of the C structs have the C layout (CPU only).

A small C program built with gcc against include/stokes.h prints sizeof and the offset of every
field; the ctypes structures of the binding must agree field by field and in total size, so that
a field added to, removed from or reordered in the header without the binding (or the other way
round) fails here rather than as corrupted arguments at run time.
"""
import ctypes
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

STRUCTS = {"stk_mesh_desc": "MeshDesc", "stk_solver_params": "SolverParams", "stk_report": "Report",
           "stk_temp_params": "TempParams", "stk_temp_report": "TempReport"}


def _c_layout(tmp_path):
    from paper_2506_04157_amd import _lib
    lines = ["#include <stdio.h>", "#include <stddef.h>", '#include "stokes.h"', "int main(void) {"]
    for cname, pyname in STRUCTS.items():
        lines.append(f'  printf("{cname} size %zu\\n", sizeof({cname}));')
        for f, _ in getattr(_lib, pyname)._fields_:
            lines.append(f'  printf("{cname} {f} %zu\\n", offsetof({cname}, {f}));')
    lines += ["  return 0;", "}"]
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines) + "\n")
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-std=c99", "-Wall", "-Werror", "-I", os.path.join(ROOT, "include"),
                    str(src), "-o", str(exe)], check=True, capture_output=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout
    lay = {}
    for line in out.splitlines():
        s, f, v = line.split()
        lay[(s, f)] = int(v)
    return lay


@pytest.mark.skipif(shutil.which("gcc") is None, reason="gcc not available")
def test_ctypes_structs_match_header(tmp_path):
    from paper_2506_04157_amd import _lib
    lay = _c_layout(tmp_path)
    for cname, pyname in STRUCTS.items():
        cls = getattr(_lib, pyname)
        assert ctypes.sizeof(cls) == lay[(cname, "size")], cname
        for f, _ in cls._fields_:
            assert getattr(cls, f).offset == lay[(cname, f)], (cname, f)
