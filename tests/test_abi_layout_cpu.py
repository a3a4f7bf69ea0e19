"""The ctypes structures of the binding match the C header's layout.

A small C program built with the host compiler against include/kkt_lu.h
prints sizeof and offsetof of every field of kkt_options, kkt_report and
kkt_info; the binding's ctypes fields must sit at the same offsets (a field
added to one side only would shift every later option silently).
"""
import ctypes
import os
import shutil
import subprocess

import pytest

from paper_2306_14337_amd import binding

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
STRUCTS = [("kkt_options", binding.Options), ("kkt_report", binding.Report),
           ("kkt_info", binding.Info)]


@pytest.mark.skipif(shutil.which("gcc") is None, reason="no host C compiler")
def test_ctypes_layout_matches_header(tmp_path):
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "kkt_lu.h"', 'int main(void) {']
    for cname, py in STRUCTS:
        lines.append(f'  printf("{cname} size %zu\\n", sizeof({cname}));')
        for fname, _ in py._fields_:
            lines.append(f'  printf("{cname} {fname} %zu\\n", offsetof({cname}, {fname}));')
    lines += ['  return 0;', '}']
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines) + "\n")
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-std=c99", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)],
                   check=True, capture_output=True, text=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout.split("\n")
    got = {}
    for line in out:
        if line:
            cname, key, val = line.split()
            got[(cname, key)] = int(val)
    for cname, py in STRUCTS:
        assert got[(cname, "size")] == ctypes.sizeof(py), cname
        for fname, _ in py._fields_:
            assert got[(cname, fname)] == getattr(py, fname).offset, (cname, fname)
