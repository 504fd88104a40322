"""CPU checks of the C ABI library: it loads and exports every symbol that
include/fcw.h declares (no compute call is made without a GPU)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "fcw.h")


def declared_symbols():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(fcw_[a-z_]+)\s*\(", text)))


def test_header_declares_the_boundary():
    names = declared_symbols()
    for required in ("fcw_assemble_cells", "fcw_stabilize_cut_cells", "fcw_critical_dt",
                     "fcw_step_explicit", "fcw_imex_prepare", "fcw_step_imex"):
        assert required in names


def test_library_exports_every_declared_symbol():
    from paper_2501_19013_amd import fcw
    if not os.path.exists(fcw.LIB_PATH):
        pytest.fail("libfcw.so is not built (run __graft_entry__.build())")
    lib = ctypes.CDLL(fcw.LIB_PATH)
    for name in declared_symbols():
        assert hasattr(lib, name), name
    assert set(fcw.EXPORTS) == set(declared_symbols())


def test_error_path_without_gpu():
    # argument errors are reported without touching the device
    from paper_2501_19013_amd import fcw
    lib = fcw.load()
    ctx = ctypes.c_void_p()
    assert lib.fcw_assemble_cells(None, ctypes.byref(ctx)) == fcw.FCW_E_ARG
    assert b"null" in lib.fcw_last_error()
    desc = fcw.ProblemDesc()
    desc.dim = 4
    assert lib.fcw_assemble_cells(ctypes.byref(desc), ctypes.byref(ctx)) == fcw.FCW_E_ARG
    assert lib.fcw_stabilize_cut_cells(None, 1e-4, 1e-4) == fcw.FCW_E_ARG
    assert lib.fcw_step_imex(None, 1, None, None, None, None, None, 0.0, 0.0, 1, 0) == fcw.FCW_E_ARG
    n = ctypes.c_int64()
    assert lib.fcw_imex_prepare(None, 1e-3, ctypes.byref(n)) == fcw.FCW_E_ARG
