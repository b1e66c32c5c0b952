"""The ctypes mirrors of the C ABI's option structs have the C compiler's
layout: a C program built with gcc from include/feastband.h prints sizeof
and every field's offsetof, which must equal the Structure's size and field
offsets (a field added on one side only would shift every later one)."""
import os
import shutil
import subprocess

import pytest

from paper_2012_00506_amd import _native as N

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
STRUCTS = [N.fb_band, N.fb_solve_opts, N.fb_feast_opts, N.fb_plan_opts, N.fb_prev_opts]


@pytest.mark.skipif(shutil.which("gcc") is None, reason="no gcc")
def test_struct_layouts_match_c(tmp_path):
    lines = ["#include <stddef.h>", "#include <stdio.h>", '#include "feastband.h"',
             "int main(void) {"]
    for S in STRUCTS:
        name = S.__name__
        lines.append(f'  printf("{name} size %zu\\n", sizeof({name}));')
        for f, _ in S._fields_:
            lines.append(f'  printf("{name} {f} %zu\\n", offsetof({name}, {f}));')
    lines += ["  return 0;", "}"]
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines) + "\n")
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-std=c11", "-I", os.path.join(ROOT, "include"), str(src), "-o",
                    str(exe)], check=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout
    got = {}
    for line in out.splitlines():
        s, f, v = line.split()
        got[(s, f)] = int(v)
    for S in STRUCTS:
        name = S.__name__
        assert got[(name, "size")] == N.C.sizeof(S), name
        for f, _ in S._fields_:
            assert got[(name, f)] == getattr(S, f).offset, (name, f)
