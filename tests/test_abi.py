"""CPU checks of the C ABI boundary: the HIP library loads and exports every
function declared in include/swe_nh.h (no compute call: no GPU here)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "swe_nh.h")
LIB = os.path.join(ROOT, "paper_2505_17025_amd", "_build", "libswe_nh.so")


def declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(swe_nh_[a-z0-9_]+)\s*\(", src)))


def test_header_declares_the_entry_points():
    names = declared_functions()
    for must in ("swe_nh_init", "swe_nh_step", "swe_nh_solve_pressure", "swe_nh_mask",
                 "swe_nh_workspace_bytes", "swe_nh_destroy"):
        assert must in names


@pytest.mark.skipif(not os.path.exists(LIB), reason="HIP library not built")
def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(LIB)
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing


@pytest.mark.skipif(not os.path.exists(LIB), reason="HIP library not built")
def test_binding_names_match_header():
    from paper_2505_17025_amd import swe_nh as B
    assert sorted(B.EXPORTED) == sorted(n for n in declared_functions())


@pytest.mark.skipif(not os.path.exists(LIB), reason="HIP library not built")
def test_workspace_query_rejects_bad_config():
    from paper_2505_17025_amd import swe_nh as B
    cfg = B.swe_nh_config()
    cfg.dim = 3
    assert B.LIB.swe_nh_workspace_bytes(ctypes.byref(cfg)) == 0


@pytest.mark.skipif(not os.path.exists(LIB), reason="HIP library not built")
def test_binding_structures_match_the_header_layout(tmp_path):
    """every ctypes structure of the binding has the size and field offsets
    that a C compiler gives the header's struct of the same name"""
    import subprocess
    from paper_2505_17025_amd import swe_nh as B
    structs = [B.swe_nh_body, B.swe_nh_config, B.swe_nh_dg1d_config, B.swe_nh_stats]
    lines = ['#include <stddef.h>', '#include <stdio.h>', '#include "swe_nh.h"', "int main(void) {"]
    want = []
    for T in structs:
        lines.append(f'  printf("%zu\\n", sizeof({T.__name__}));')
        want.append(ctypes.sizeof(T))
        for name, *_ in T._fields_:
            lines.append(f'  printf("%zu\\n", offsetof({T.__name__}, {name}));')
            want.append(getattr(T, name).offset)
    lines += ["  return 0;", "}"]
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines) + "\n")
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-std=c99", "-I", os.path.join(ROOT, "include"), str(src), "-o",
                    str(exe)], check=True)
    got = [int(v) for v in subprocess.run([str(exe)], check=True, capture_output=True,
                                          text=True).stdout.split()]
    assert got == want
