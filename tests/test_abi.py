"""Host-side checks of the C ABI (no GPU needed): the library loads, exports every entry point the
header declares, reports status strings, and fails cleanly when no device is present."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "lsq.h")


def declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(lsq_[a-z_]+)\s*\(", src)))


def test_header_declares_the_boundary():
    names = declared_functions()
    for req in ("lsq_sketch", "lsq_pcg_solve", "lsq_ihs_solve", "lsq_pcg_solve_batched", "lsq_create",
                "lsq_destroy", "lsq_status_string", "lsq_last_error"):
        assert req in names


def test_library_exports_every_declared_symbol():
    from paper_1911_02675_amd import lsq
    lib = lsq.load()
    for name in declared_functions():
        assert hasattr(lib, name), name
    assert set(lsq.EXPORTED) == set(declared_functions())


def test_status_strings_and_version():
    from paper_1911_02675_amd import lsq
    lib = lsq.load()
    assert lib.lsq_version().startswith(b"liblsq")
    for code in range(8):
        assert lib.lsq_status_string(code)
    assert lsq.status_string(lsq.LSQ_ERR_RANK).startswith("rank")


def test_struct_layouts_match_header():
    from paper_1911_02675_amd import lsq
    # sizes follow from the header (all 8-byte aligned, no implicit tail padding)
    assert ctypes.sizeof(lsq.Problem) == 48
    assert ctypes.sizeof(lsq.SketchDesc) == 40
    assert ctypes.sizeof(lsq.PcgOpts) == 40
    assert ctypes.sizeof(lsq.IhsOpts) == 40
    assert ctypes.sizeof(lsq.Info) == 80


def test_null_arguments_rejected_without_device():
    from paper_1911_02675_amd import lsq
    lib = lsq.load()
    assert lib.lsq_create(None, None) == lsq.LSQ_ERR_INVALID_ARG
    assert lib.lsq_sketch(None, None, None, None, 0, 0) == lsq.LSQ_ERR_INVALID_ARG
    assert lib.lsq_pcg_solve(None, None, None, None, None, None, None) == lsq.LSQ_ERR_INVALID_ARG
    assert lib.lsq_ihs_solve(None, None, None, None, None, None, None) == lsq.LSQ_ERR_INVALID_ARG
    assert lib.lsq_factor(None, None, 4, 4, 4, None, None) == lsq.LSQ_ERR_INVALID_ARG
    assert lib.lsq_pcg_solve_batched(None, 1, None, None, None, None, None, None) == lsq.LSQ_ERR_INVALID_ARG
    assert b"null" in lib.lsq_last_error()
    assert lib.lsq_tune(b"batched_slots", -1) == lsq.LSQ_ERR_INVALID_ARG
    assert lib.lsq_tune(b"batched_slots", 0) == lsq.LSQ_OK


def test_c_header_compiles_standalone(tmp_path):
    # the header is plain C: compile a translation unit that includes it with gcc
    src = tmp_path / "t.c"
    src.write_text('#include "lsq.h"\nint main(void){ lsq_problem p; lsq_sketch_desc s; lsq_pcg_opts o;'
                   ' lsq_ihs_opts i; lsq_info f; (void)p;(void)s;(void)o;(void)i;(void)f;'
                   ' return (int)sizeof(lsq_problem) - 48 + (int)sizeof(lsq_info) - 80; }\n')
    import subprocess
    r = subprocess.run(["gcc", "-std=c99", "-Wall", "-Werror", "-I", os.path.join(ROOT, "include"),
                        str(src), "-o", str(tmp_path / "t")], capture_output=True, text=True)
    assert r.returncode == 0, r.stderr
    assert subprocess.run([str(tmp_path / "t")]).returncode == 0
