"""The C-ABI library loads and exports every entry point that include/rtsvd.h declares (CPU only)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "rtsvd.h")
LIB = os.path.join(ROOT, "paper_2110_02485_amd", "librtsvd.so")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"^\s*(?:const\s+)?(?:int|void|char\s*\*|const char\s*\*)\s*\*?\s*(\w+)\s*\(", text, flags=re.M)
    return sorted(set(names))


def test_header_declares_entry_points():
    names = declared_functions()
    for n in ["rtsvd_factor", "rtsvd_solve", "tprod", "tprod_adjoint", "tgkb_solve", "ttsvd_factor",
              "rtsvd_factor_info", "rtsvd_factor_destroy", "rtsvd_status_string", "rtsvd_last_error"]:
        assert n in names, n


@pytest.mark.skipif(not os.path.exists(LIB), reason="librtsvd.so not built")
def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(LIB)
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing


@pytest.mark.skipif(not os.path.exists(LIB), reason="librtsvd.so not built")
def test_status_strings_without_gpu():
    lib = ctypes.CDLL(LIB)
    lib.rtsvd_status_string.restype = ctypes.c_char_p
    assert lib.rtsvd_status_string(0) == b"ok"
    assert b"invalid" in lib.rtsvd_status_string(-1)


@pytest.mark.skipif(not os.path.exists(LIB), reason="librtsvd.so not built")
def test_argument_errors_without_gpu():
    # argument checks run before any device call
    from paper_2110_02485_amd import rtsvd as rt
    lib = rt.load()
    h = ctypes.c_void_p()
    opts = rt._Opts(5, 2, 0, 0, 0, None, 0.0)
    assert lib.rtsvd_factor(None, 4, 4, 4, 0, ctypes.byref(opts), None, ctypes.byref(h)) == rt.E_ARG
    assert lib.rtsvd_factor(ctypes.c_void_p(16), 3, 4, 4, 0, ctypes.byref(opts), None, ctypes.byref(h)) == rt.E_ARG
    bad = rt._Opts(0, 2, 0, 0, 0, None, 0.0)
    assert lib.rtsvd_factor(ctypes.c_void_p(16), 8, 4, 4, 0, ctypes.byref(bad), None, ctypes.byref(h)) == rt.E_ARG
    big = rt._Opts(300, 10, 0, 0, 0, ctypes.c_void_p(16), 0.0)
    assert lib.rtsvd_factor(ctypes.c_void_p(16), 400, 400, 4, 0, ctypes.byref(big), None, ctypes.byref(h)) == rt.E_UNSUPPORTED
    assert lib.tprod(None, None, None, 1, 1, 1, 1, 0, None) == rt.E_ARG
    assert lib.tprod(ctypes.c_void_p(16), ctypes.c_void_p(16), ctypes.c_void_p(16), 1, 1, 1, 1, 7, None) == rt.E_ARG
    assert b"dtype" in lib.rtsvd_last_error()
