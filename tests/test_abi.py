"""The C-ABI library loads and exports every function include/dgthermo.h declares
(no compute call: runs without a GPU)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    names = set()
    for fn in os.listdir(os.path.join(ROOT, "include")):
        if fn.endswith(".h"):
            text = open(os.path.join(ROOT, "include", fn)).read()
            text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
            names |= set(re.findall(r"\b(dg_[a-z0-9_]+)\s*\(", text))
    return names


def test_library_exports_every_declared_symbol():
    import paper_2306_01085_amd as pkg
    lib = ctypes.CDLL(pkg.library_path())
    declared = _declared()
    assert {"dg_mesh_create", "dg_residual", "dg_jvp", "dg_implicit_step"} <= declared
    missing = [n for n in sorted(declared) if not hasattr(lib, n)]
    assert not missing, missing
    assert set(pkg.EXPORTED) >= declared
    assert pkg.version() >= 1


def test_struct_layout_matches_header(tmp_path):
    """the ctypes mirrors have the sizes the C compiler gives the header's structs"""
    import shutil
    import subprocess
    import paper_2306_01085_amd as pkg
    cc = shutil.which("gcc") or shutil.which("cc")
    if cc is None:
        pytest.skip("no C compiler")
    src = tmp_path / "sizes.c"
    src.write_text('#include <stdio.h>\n#include "dgthermo.h"\n'
                   'int main(void) { printf("%zu %zu %zu %zu", sizeof(dg_mesh_desc_t), sizeof(dg_physics_t), '
                   'sizeof(dg_solver_opts_t), sizeof(dg_step_stats_t)); return 0; }\n')
    exe = tmp_path / "sizes"
    subprocess.run([cc, "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    sizes = [int(x) for x in subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout.split()]
    assert sizes == [ctypes.sizeof(pkg.MeshDesc), ctypes.sizeof(pkg.Physics), ctypes.sizeof(pkg.SolverOpts),
                     ctypes.sizeof(pkg.StepStats)]
