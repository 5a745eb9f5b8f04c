"""The ctypes mirror of the C-ABI structs (paper_1110_1328_amd/_abi.py) has
the header's layout: a small C program built against include/bayeslsh.h with
the host compiler prints each struct's size and every field's offset, and the
mirror must agree field by field."""
import ctypes
import os
import shutil
import subprocess

import pytest

from paper_1110_1328_amd import _abi as A

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

STRUCTS = {
    "blsh_prior": A.Prior,
    "blsh_sigs": A.Sigs,
    "blsh_candidates": A.Candidates,
    "blsh_tile": A.Tile,
    "blsh_vectors": A.Vectors,
    "blsh_result": A.Result,
    "blsh_tuning": A.Tuning,
    "blsh_list_desc": A.ListDesc,
    "blsh_server_config": A.ServerConfig,
    "blsh_request_result": A.RequestResult,
}


def c_layout(tmp_path):
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "bayeslsh.h"', 'int main(void) {']
    for cname, py in STRUCTS.items():
        lines.append('  printf("%s size %%zu\\n", sizeof(%s));' % (cname, cname))
        for fname, _ in py._fields_:
            lines.append('  printf("%s %s %%zu\\n", offsetof(%s, %s));' % (cname, fname, cname, fname))
    lines += ['  return 0;', '}']
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines) + "\n")
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-std=c11", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout
    return {tuple(l.split()[:2]): int(l.split()[2]) for l in out.splitlines()}


@pytest.mark.skipif(shutil.which("gcc") is None, reason="needs a host C compiler")
def test_ctypes_mirror_matches_header(tmp_path):
    got = c_layout(tmp_path)
    for cname, py in STRUCTS.items():
        assert got[(cname, "size")] == ctypes.sizeof(py), cname
        for fname, _ in py._fields_:
            assert got[(cname, fname)] == getattr(py, fname).offset, (cname, fname)
