"""The ctypes structures of the Python binding against the C headers: a small C program,
built with the host compiler from include/*.h alone, prints sizeof and offsetof of every
field the binding declares; a field missing from the header fails the build."""
import ctypes
import os
import shutil
import subprocess

import pytest

from paper_2303_01471_amd import qhd as q

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
STRUCTS = [q.qhd_instance, q.qhd_plan_opts, q.qhd_observables, q.qhd_kernel_timing, q.qhd_class_info,
           q.qhd_sno_desc, q.qhd_rqp_desc, q.qhd_rqp_obs]


def test_ctypes_layouts_match_the_headers(tmp_path):
    cc = shutil.which("gcc") or shutil.which("cc")
    if not cc:
        pytest.skip("no host C compiler")
    lines = ['#include <stddef.h>', '#include <stdio.h>', '#include "qhd.h"', '#include "qhd_sno.h"',
             '#include "qhd_rqp.h"', "int main(void) {"]
    for st in STRUCTS:
        name = st.__name__
        lines.append(f'  printf("{name} %zu\\n", sizeof({name}));')
        for field, _ in st._fields_:
            lines.append(f'  printf("{name}.{field} %zu\\n", offsetof({name}, {field}));')
    lines += ["  return 0;", "}"]
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines) + "\n")
    exe = tmp_path / "layout"
    subprocess.run([cc, "-std=c99", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True,
                   capture_output=True)
    got = dict(line.rsplit(" ", 1) for line in subprocess.run([str(exe)], check=True, capture_output=True,
                                                                   text=True).stdout.splitlines())
    for st in STRUCTS:
        name = st.__name__
        assert int(got[name]) == ctypes.sizeof(st), name
        for field, _ in st._fields_:
            assert int(got[f"{name}.{field}"]) == getattr(st, field).offset, f"{name}.{field}"


def test_option_bits_match_the_header():
    text = open(os.path.join(ROOT, "include", "qhd.h")).read()
    for name in ("QHD_OPT_TIME_PASSES", "QHD_OPT_AUTOTUNE", "QHD_OPT_NO_GRAPH", "QHD_OPT_MFMA_DFT",
                 "QHD_OPT_RESIDENT"):
        tok = text.split(f"#define {name} ", 1)[1].split()[0].rstrip("u")
        assert int(tok, 16) == getattr(q, name), name
