"""The binding's ctypes structures against the layout the C header gives them
(sizeof and offsetof of every field, from a small program compiled with gcc
against include/morx.h), so that a field added or reordered on one side only
is caught without a GPU."""
import ctypes
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
STRUCTS = ["morx_opts", "morx_col_stats", "morx_trace_entry", "morx_serve_config", "morx_tune",
           "morx_factor_spec", "morx_serve_counts"]


def test_struct_layouts_match_the_header(tmp_path):
    gcc = shutil.which("gcc")
    if gcc is None:
        pytest.skip("gcc not found")
    from paper_2003_12759_amd import morx

    lines = ["#include <stdio.h>", "#include <stddef.h>", '#include "morx.h"', "int main(void) {"]
    for sname in STRUCTS:
        cls = getattr(morx, sname)
        lines.append(f'  printf("{sname} . %zu\\n", sizeof({sname}));')
        for fname, _ in cls._fields_:
            lines.append(f'  printf("{sname} {fname} %zu\\n", offsetof({sname}, {fname}));')
    lines += ["  return 0;", "}"]
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines) + "\n")
    exe = tmp_path / "layout"
    subprocess.run([gcc, "-std=c11", "-Wall", "-I", os.path.join(ROOT, "include"), str(src),
                    "-o", str(exe)], check=True)
    out = subprocess.run([str(exe)], capture_output=True, text=True, check=True).stdout
    got = {}
    for line in out.splitlines():
        sname, fname, value = line.split()
        got[(sname, fname)] = int(value)
    for sname in STRUCTS:
        cls = getattr(morx, sname)
        assert got[(sname, ".")] == ctypes.sizeof(cls), sname
        for fname, _ in cls._fields_:
            assert got[(sname, fname)] == getattr(cls, fname).offset, (sname, fname)
