"""CPU checks of the C ABI: the library loads, exports every function that
include/agc.h declares, and rejects bad host arguments without a GPU."""
import ctypes
import os
import re
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "agc.h")
LIB = os.path.join(ROOT, "paper_2605_04773_amd", "libagc.so")


def declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(agc_[a-z0-9_]+)\s*\(", text)))


needs_lib = pytest.mark.skipif(not os.path.exists(LIB), reason="libagc.so not built")


def test_header_declares_the_five_calls():
    names = declared()
    for n in ("agc_aggregate", "agc_assemble_coarse", "agc_pcg", "agc_prolongate", "agc_solve"):
        assert n in names


@needs_lib
def test_every_declared_symbol_is_exported():
    lib = ctypes.CDLL(LIB)
    missing = [n for n in declared() if not hasattr(lib, n)]
    assert not missing, missing


@needs_lib
def test_binding_covers_the_header():
    from paper_2605_04773_amd import agc
    assert sorted(agc.EXPORTS) == declared()
    assert os.path.samefile(agc.library_path(), LIB)
    assert "gfx950" in agc.version()


@needs_lib
def test_host_argument_checks():
    from paper_2605_04773_amd import agc
    lib = agc._lib
    assert lib.agc_create(None, 0, None) == agc.AGC_ERR_INVALID_ARG
    assert lib.agc_destroy(None) == agc.AGC_ERR_INVALID_ARG
    assert lib.agc_set_stream(None, None) == agc.AGC_ERR_INVALID_ARG
    assert lib.agc_mesh_info(None, None, None, None) == agc.AGC_ERR_INVALID_ARG
    assert lib.agc_matrix_info(None, None, None, None) == agc.AGC_ERR_INVALID_ARG
    assert lib.agc_last_error(None) == b"null context"
    n = ctypes.c_int32()
    assert lib.agc_aggregate(None, 1, 0, None, None, None, ctypes.byref(n)) == agc.AGC_ERR_INVALID_ARG
    assert lib.agc_solve(None, None, None, None, None, None) == agc.AGC_ERR_INVALID_ARG


@pytest.mark.skipif(not shutil.which("gcc"), reason="gcc not available")
def test_struct_layouts_match_header(tmp_path):
    """ctypes mirrors of the ABI structs have the C compiler's sizes and offsets."""
    from paper_2605_04773_amd import agc
    structs = {"agc_problem": agc.agc_problem, "agc_solve_opts": agc.agc_solve_opts,
               "agc_solve_info": agc.agc_solve_info, "agc_pcg_info": agc.agc_pcg_info}
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "agc.h"', "int main(void) {"]
    expect = []
    for name, cls in structs.items():
        lines.append(f'printf("%zu\\n", sizeof({name}));')
        expect.append(ctypes.sizeof(cls))
        for field, _ in cls._fields_:
            lines.append(f'printf("%zu\\n", offsetof({name}, {field}));')
            expect.append(getattr(cls, field).offset)
    lines.append("return 0; }")
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines))
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    got = [int(v) for v in subprocess.run([str(exe)], capture_output=True, text=True, check=True).stdout.split()]
    assert got == expect
