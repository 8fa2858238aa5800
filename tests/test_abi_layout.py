"""The binding's ctypes structures match the C header field by field: the
header is compiled with gcc and every field's offset and every structure's
size is compared (a mismatch would silently shift arguments)."""
import os
import shutil
import subprocess

import pytest

from paper_2305_07636_amd import _binding as B

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
STRUCTS = [B.mcdc_problem_desc, B.mcdc_run_options, B.mcdc_result]


@pytest.mark.skipif(shutil.which("gcc") is None, reason="gcc not available")
def test_ctypes_layout_matches_header(tmp_path):
    lines = ["#include <stddef.h>", "#include <stdio.h>", '#include "mcdc.h"', "int main(void) {"]
    for S in STRUCTS:
        n = S.__name__
        lines.append(f'    printf("{n} %zu\\n", sizeof({n}));')
        for f in S._fields_:
            lines.append(f'    printf("{n}.{f[0]} %zu\\n", offsetof({n}, {f[0]}));')
    lines += ["    return 0;", "}"]
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines) + "\n")
    exe = tmp_path / "layout"
    subprocess.check_call(["gcc", "-std=c11", "-I", os.path.join(ROOT, "include"), "-o", str(exe), str(src)])
    got = dict(l.rsplit(" ", 1) for l in subprocess.check_output([str(exe)], text=True).splitlines())
    for S in STRUCTS:
        n = S.__name__
        assert int(got[n]) == B.C.sizeof(S), (n, got[n], B.C.sizeof(S))
        for f in S._fields_:
            assert int(got[f"{n}.{f[0]}"]) == getattr(S, f[0]).offset, (n, f[0])
