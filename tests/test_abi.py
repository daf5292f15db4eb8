"""The C-ABI library loads and exports every symbol include/rw.h declares
(no GPU needed: nothing is computed)."""
import ctypes
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "rw.h")


def _declared():
    txt = open(HEADER).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    names = set(re.findall(r"\b(rw_[a-z_0-9]+)\s*\(", txt))
    return sorted(names)


def test_header_declares_the_boundary():
    names = _declared()
    for n in ("rw_build_weights", "rw_solve", "rw_solve_bricks", "rw_solve_backward"):
        assert n in names


def test_library_exports_every_declared_symbol():
    from paper_2509_26213_amd import rw
    lib = rw.lib()
    for n in _declared():
        assert hasattr(lib, n), n
    assert sorted(rw.EXPORTS) == _declared()
    out = subprocess.run(["nm", "-D", "--defined-only", rw.LIB_PATH], capture_output=True,
                         text=True).stdout
    exported = set(re.findall(r" T (rw_[a-z_0-9]+)$", out, flags=re.M))
    assert set(_declared()) <= exported


def test_host_side_validation_without_gpu():
    """Calls that fail validation return before touching the device."""
    from paper_2509_26213_amd import rw
    L = rw.lib()
    assert L.rw_status_string(-2) == b"RW_ERR_NO_SEEDS"
    o = rw.Options()
    L.rw_default_options(ctypes.byref(o))
    assert o.tol == 1e-6 and o.max_iter == 20000 and o.check_interval == 16
    # NULL context / volume
    assert L.rw_solve(None, None, None, None, None, None, None, 0, None, None) == -1
    assert L.rw_build_weights(None, None, 1.0, 0.0, 0, None, None, None, None) == -1
    assert L.rw_solve_workspace_bytes(rw.Dims(0, 4, 4), 2, 0, 0) == 0
    n = L.rw_solve_workspace_bytes(rw.Dims(64, 64, 64), 2, 0, 0)
    assert n >= 64 ** 3 * 8 * 4
    # grids the kernels cannot address are refused: a plane above 2^29 voxels
    # (32-bit in-plane byte offsets), more than 2^40 voxels, a side above 2^30
    assert L.rw_solve_workspace_bytes(rw.Dims(1 << 15, 1 << 14, 1), 2, 0, 0) > 0
    assert L.rw_solve_workspace_bytes(rw.Dims(1 << 15, (1 << 14) + 1, 1), 2, 0, 0) == 0
    assert L.rw_solve_workspace_bytes(rw.Dims(1 << 14, 1 << 14, (1 << 13) + 1), 2, 0, 0) == 0
    assert L.rw_solve_workspace_bytes(rw.Dims((1 << 30) + 1, 1, 1), 2, 0, 0) == 0
    assert L.rw_operator_workspace_bytes(rw.Dims(1 << 20, 1 << 10, 1), 1) == 0
    assert L.rw_backward_workspace_bytes(rw.Dims(1 << 20, 1 << 10, 1)) == 0


def test_oracle_is_not_imported_by_the_product_path():
    pkg = os.path.join(ROOT, "paper_2509_26213_amd")
    for dirpath, _, files in os.walk(pkg):
        for f in files:
            if f.endswith((".py", ".hip", ".h", ".cpp", ".c")):
                txt = open(os.path.join(dirpath, f)).read()
                assert "oracle" not in txt.replace("oracle is", ""), os.path.join(dirpath, f)


def test_binding_structs_match_the_header_layout(tmp_path):
    """Every struct the binding mirrors has the header's size and field
    offsets (compiled by the host C compiler)."""
    from paper_2509_26213_amd import rw
    pairs = [("rw_dims", rw.Dims), ("rw_volume", rw.Volume), ("rw_seeds", rw.Seeds),
             ("rw_options", rw.Options), ("rw_stats", rw.Stats), ("rw_brick", rw.Brick),
             ("rw_subvolume", rw.SubVolume)]
    lines = ["#include <stdio.h>", "#include <stddef.h>", '#include "rw.h"', "int main(void) {"]
    for cname, py in pairs:
        lines.append(f'printf("{cname} sizeof %zu\\n", sizeof({cname}));')
        for f, _ in py._fields_:
            lines.append(f'printf("{cname} {f} %zu\\n", offsetof({cname}, {f}));')
    lines += ["return 0;", "}"]
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines) + "\n")
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-std=c99", "-I", os.path.dirname(HEADER), str(src), "-o", str(exe)],
                   check=True)
    got = {}
    for line in subprocess.run([str(exe)], capture_output=True, text=True,
                               check=True).stdout.splitlines():
        c, f, v = line.split()
        got[(c, f)] = int(v)
    for cname, py in pairs:
        assert got[(cname, "sizeof")] == ctypes.sizeof(py), cname
        for f, _ in py._fields_:
            assert got[(cname, f)] == getattr(py, f).offset, (cname, f)
