"""Host-side checks of the C-ABI that need no GPU:

* every ctypes mirror of a public struct has the header's fields, in order,
  at the header's offsets and with its size (a shorter mirror lets the
  library's `*_opts_default` and stats writes run past the Python object);
* the thick-restart Lanczos solver's host bookkeeping (Sec. 2.5 and Sec. 3:
  T = V^T rho V block by block, the Ritz residuals read from T, the kept
  count and T after a restart) against a dense computation, built with
  bounds-checked containers and the address and undefined-behaviour
  sanitisers.
"""
import ctypes
import os
import re
import shutil
import subprocess

import pytest

from paper_1902_07041_amd import _capi

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "pfeig.h")
CSRC = os.path.join(ROOT, "paper_1902_07041_amd", "csrc")

MIRRORS = {
    "pfe_filter_opts": _capi.CFilterOpts,
    "pfe_filter": _capi.CFilter,
    "pfe_solve_opts": _capi.CSolveOpts,
    "pfe_solve_stats": _capi.CSolveStats,
    "pfe_dirac_filter": _capi.CDiracFilter,
    "pfe_lanczos_opts": _capi.CLanczosOpts,
    "pfe_slice_opts": _capi.CSliceOpts,
}


def header_structs():
    """{typedef name: [field names in order]} from the header's text."""
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", " ", text, flags=re.S)
    text = re.sub(r"//[^\n]*", " ", text)
    out = {}
    for body, name in re.findall(r"typedef\s+struct\s*\{(.*?)\}\s*(\w+)\s*;", text, flags=re.S):
        fields = []
        for decl in body.split(";"):
            decl = " ".join(decl.split())
            if not decl:
                continue
            first, *rest = [p.strip() for p in decl.split(",")]
            fields.append(re.findall(r"\w+", first)[-1])
            fields.extend(re.findall(r"\w+", r)[-1] for r in rest)
        out[name] = fields
    return out


def test_every_public_struct_has_a_mirror():
    assert set(header_structs()) == set(MIRRORS)


@pytest.mark.skipif(shutil.which("gcc") is None, reason="gcc not available")
def test_ctypes_mirrors_match_the_header(tmp_path):
    hs = header_structs()
    lines = ["#include <stddef.h>", "#include <stdio.h>", '#include "pfeig.h"', "int main(void) {"]
    for name, fields in hs.items():
        lines.append(f'  printf("{name} size %zu\\n", sizeof({name}));')
        for f in fields:
            lines.append(f'  printf("{name} {f} %zu\\n", offsetof({name}, {f}));')
    lines += ["  return 0;", "}"]
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines) + "\n")
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-std=c11", "-I", os.path.dirname(HEADER), str(src), "-o", str(exe)],
                   check=True)
    got = {}
    for ln in subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout.splitlines():
        name, field, val = ln.split()
        got[(name, field)] = int(val)
    for name, cls in MIRRORS.items():
        names = [f for f, _ in cls._fields_]
        assert names == hs[name], (name, names, hs[name])
        assert ctypes.sizeof(cls) == got[(name, "size")], name
        for f in names:
            assert getattr(cls, f).offset == got[(name, f)], (name, f)


@pytest.mark.skipif(shutil.which("g++") is None, reason="g++ not available")
def test_lanczos_host_bookkeeping_sanitized(tmp_path):
    exe = tmp_path / "lanczos_host_check"
    cmd = ["g++", "-std=c++17", "-O1", "-g", "-fsanitize=address,undefined",
           "-fno-sanitize-recover=all", "-D_GLIBCXX_ASSERTIONS", "-I", CSRC,
           os.path.join(ROOT, "tests", "lanczos_host_check.cpp"),
           os.path.join(CSRC, "lanczos_host.cpp"), "-o", str(exe)]
    subprocess.run(cmd, check=True)
    r = subprocess.run([str(exe)], capture_output=True, text=True, timeout=300,
                       env=dict(os.environ, ASAN_OPTIONS="detect_leaks=1"))
    print(r.stdout)
    assert r.returncode == 0, r.stdout + r.stderr
    assert "b=8 m=48" in r.stdout and r.stdout.rstrip().endswith("ALL OK")


@pytest.mark.skipif(shutil.which("g++") is None, reason="g++ not available")
def test_tile_row_orders_sanitized(tmp_path):
    exe = tmp_path / "reorder_check"
    cmd = ["g++", "-std=c++17", "-O1", "-g", "-fsanitize=address,undefined",
           "-fno-sanitize-recover=all", "-D_GLIBCXX_ASSERTIONS", "-I", CSRC,
           os.path.join(ROOT, "tests", "reorder_check.cpp"),
           os.path.join(CSRC, "reorder.cpp"), "-o", str(exe)]
    subprocess.run(cmd, check=True)
    r = subprocess.run([str(exe)], capture_output=True, text=True, timeout=300,
                       env=dict(os.environ, ASAN_OPTIONS="detect_leaks=1"))
    print(r.stdout)
    assert r.returncode == 0, r.stdout + r.stderr
    assert "window holes n=2121 W=4096 R=4" in r.stdout and r.stdout.rstrip().endswith("ALL OK")
