"""The C-ABI library builds, loads and exports every symbol that
include/lbddc.h declares; without a GPU, creating a context fails cleanly
with LBDDC_E_ARG (no compute call is made here)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def header_functions():
    text = open(os.path.join(ROOT, "include", "lbddc.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(lbddc_[a-z0-9_]+)\s*\(", text)))


def test_header_matches_binding():
    from paper_2604_09113_amd import lbddc
    assert header_functions() == sorted(lbddc.FUNCTIONS)


def test_library_exports_every_symbol():
    from paper_2604_09113_amd import lbddc
    if not os.path.exists(lbddc.LIB_PATH):
        pytest.skip("library not built")
    lib = ctypes.CDLL(lbddc.LIB_PATH)
    for name in header_functions():
        assert hasattr(lib, name), name


def test_status_codes_and_no_device_path():
    from paper_2604_09113_amd import lbddc
    if not os.path.exists(lbddc.LIB_PATH):
        pytest.skip("library not built")
    lib = lbddc.library()
    assert lib.lbddc_version() == 2
    assert lib.lbddc_last_error(None) == b"null context"
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present; the no-device path is not reachable")
    ctx = ctypes.c_void_p()
    assert lib.lbddc_create(0, None, ctypes.byref(ctx)) == lbddc.E_ARG
    assert lib.lbddc_create(0, None, None) == lbddc.E_ARG
    # every call rejects a null context without touching a device
    assert lib.lbddc_assemble(None, 0) == lbddc.E_ARG
    assert lib.lbddc_setup(None, 0) == lbddc.E_ARG
    assert lib.lbddc_solve(None, 1e-8, 10, None) == lbddc.E_ARG
    assert lib.lbddc_query(None, 0, None) == lbddc.E_ARG


def test_struct_layouts_match_header(tmp_path):
    """The ctypes mirrors of the descriptor structs have the sizes and field
    offsets that a C compiler gives the header's structs."""
    import shutil
    import subprocess
    from paper_2604_09113_amd import lbddc
    cc = shutil.which("gcc") or shutil.which("cc")
    if cc is None:
        pytest.skip("no C compiler")
    structs = {"lbddc_problem_desc": lbddc.ProblemDesc, "lbddc_rom_desc": lbddc.RomDesc,
               "lbddc_solve_info": lbddc.SolveInfo}
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "lbddc.h"', "int main(void) {"]
    for cname, py in structs.items():
        lines.append(f'printf("{cname} size %zu\\n", sizeof({cname}));')
        for fname, _ in py._fields_:
            lines.append(f'printf("{cname} {fname} %zu\\n", offsetof({cname}, {fname}));')
    lines.append("return 0; }")
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines))
    exe = tmp_path / "layout"
    subprocess.run([cc, "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout.split("\n")
    got = {tuple(l.split()[:2]): int(l.split()[2]) for l in out if l}
    import ctypes as C
    for cname, py in structs.items():
        assert got[(cname, "size")] == C.sizeof(py), cname
        for fname, _ in py._fields_:
            assert got[(cname, fname)] == getattr(py, fname).offset, (cname, fname)
