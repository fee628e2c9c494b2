"""The ctypes mirrors of the public structs match the C header: every field's
offset and every struct's size, as a C compiler lays them out from
include/tgs.h (a small program built with the host compiler, no GPU)."""
import ctypes as C
import os
import shutil
import subprocess

import pytest

from paper_2412_13547_amd import api

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
STRUCTS = ("tgs_camera", "tgs_dilation", "tgs_gaussians", "tgs_options", "tgs_grads",
           "tgs_sizes", "tgs_state", "tgs_adam_group", "tgs_view_io")


def _c_layout(tmp_path):
    cc = shutil.which("gcc") or shutil.which("cc")
    if cc is None:
        pytest.skip("no host C compiler")
    lines = ["#include <stddef.h>", "#include <stdio.h>", '#include "tgs.h"', "int main(void) {"]
    for s in STRUCTS:
        lines.append(f'    printf("{s} sizeof %zu\\n", sizeof({s}));')
        for name, *_ in getattr(api, s)._fields_:
            lines.append(f'    printf("{s} {name} %zu\\n", offsetof({s}, {name}));')
    lines += ["    return 0;", "}"]
    src = tmp_path / "layout.c"
    exe = tmp_path / "layout"
    src.write_text("\n".join(lines) + "\n")
    subprocess.run([cc, "-std=c11", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)],
                   check=True, capture_output=True, text=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout
    got = {}
    for line in out.splitlines():
        s, field, val = line.split()
        got[(s, field)] = int(val)
    return got


def test_ctypes_structs_match_header(tmp_path):
    c = _c_layout(tmp_path)
    for s in STRUCTS:
        cls = getattr(api, s)
        assert C.sizeof(cls) == c[(s, "sizeof")], s
        for name, *_ in cls._fields_:
            assert getattr(cls, name).offset == c[(s, name)], (s, name)
