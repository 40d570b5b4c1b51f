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
    grp = rt._Opts(5, 2, 0, 0, 0, ctypes.c_void_p(16), 0.0, 0, 4)
    assert lib.rtsvd_factor(ctypes.c_void_p(16), 8, 8, 4, 0, ctypes.byref(grp), None, ctypes.byref(h)) == rt.E_ARG
    assert b"face_groups" in lib.rtsvd_last_error()
    tile = rt._Opts(5, 2, 0, 0, 0, ctypes.c_void_p(16), 0.0, 0, 0, 3)
    assert lib.rtsvd_factor(ctypes.c_void_p(16), 8, 8, 4, 0, ctypes.byref(tile), None, ctypes.byref(h)) == rt.E_ARG
    assert b"sketch_tile" in lib.rtsvd_last_error()
    assert lib.tprod(None, None, None, 1, 1, 1, 1, 0, None) == rt.E_ARG
    assert lib.tprod(ctypes.c_void_p(16), ctypes.c_void_p(16), ctypes.c_void_p(16), 1, 1, 1, 1, 7, None) == rt.E_ARG
    assert b"dtype" in lib.rtsvd_last_error()


@pytest.mark.skipif(not os.path.exists(LIB), reason="librtsvd.so not built")
def test_argument_errors_of_the_krylov_and_symmetric_entry_points():
    # argument checks run before any device call
    from paper_2110_02485_amd import rtsvd as rt
    lib = rt.load()
    p16 = ctypes.c_void_p(16)
    k = (ctypes.c_int32 * 4)()
    one = (ctypes.c_double * 1)(0.1)
    two = (ctypes.c_double * 2)(0.1, 0.1)
    neg = (ctypes.c_double * 1)(-1.0)
    # nested_tgkb_solve(A, B, l, m, n, p, dtype, delta, n_delta, eta, k_max, k_init, X, k, resid, status, stream)
    f = lib.nested_tgkb_solve
    assert f(None, p16, 8, 4, 4, 1, 0, one, 1, 1.1, 2, 2, p16, k, None, None, None) == rt.E_ARG
    assert f(p16, p16, 3, 4, 4, 1, 0, one, 1, 1.1, 2, 2, p16, k, None, None, None) == rt.E_ARG      # l < m
    assert f(p16, p16, 8, 4, 4, 1, 0, one, 1, 1.1, 5, 2, p16, k, None, None, None) == rt.E_ARG      # k_max > m
    assert f(p16, p16, 8, 4, 4, 1, 0, one, 1, 1.1, 2, 0, p16, k, None, None, None) == rt.E_ARG      # k_init < 1
    assert f(p16, p16, 8, 4, 4, 1, 0, one, 1, 1.0, 2, 2, p16, k, None, None, None) == rt.E_ARG      # eta <= 1
    assert f(p16, p16, 8, 4, 4, 3, 0, two, 2, 1.1, 2, 2, p16, k, None, None, None) == rt.E_ARG      # n_delta
    assert f(p16, p16, 8, 4, 4, 1, 0, neg, 1, 1.1, 2, 2, p16, k, None, None, None) == rt.E_ARG      # delta < 0
    assert f(p16, p16, 9000, 4, 4, 1, 0, one, 1, 1.1, 2, 2, p16, k, None, None, None) == rt.E_UNSUPPORTED
    assert b"nested_tgkb_solve" in lib.rtsvd_last_error()
    # nested_tgkt_solve(A, B, l, m, n, p, dtype, delta, n_delta, eta, k_max, k_init, mu_lo, mu_hi, X, k, mu,
    #                   resid, status, stream): the nested checks, then the mu interval
    mu = (ctypes.c_double * 4)()
    nt = lib.nested_tgkt_solve
    assert nt(p16, p16, 8, 4, 4, 1, 0, one, 1, 1.1, 2, 2, 1e1, 1e7, p16, k, None, None, None, None) == rt.E_ARG  # mu_out
    assert nt(p16, p16, 3, 4, 4, 1, 0, one, 1, 1.1, 2, 2, 1e1, 1e7, p16, k, mu, None, None, None) == rt.E_ARG    # l < m
    assert nt(p16, p16, 8, 4, 4, 1, 0, one, 1, 1.1, 2, 0, 1e1, 1e7, p16, k, mu, None, None, None) == rt.E_ARG    # k_init
    assert nt(p16, p16, 8, 4, 4, 1, 0, one, 1, 1.1, 2, 2, 1e7, 1e1, p16, k, mu, None, None, None) == rt.E_ARG    # mu_lo >= mu_hi
    assert nt(p16, p16, 8, 4, 4, 1, 0, one, 1, 1.1, 2, 2, 0.0, 1e1, p16, k, mu, None, None, None) == rt.E_ARG    # mu_lo <= 0
    assert nt(p16, p16, 8, 4, 4, 1, 0, one, 1, 1.0, 2, 2, 1e1, 1e7, p16, k, mu, None, None, None) == rt.E_ARG    # eta <= 1
    assert nt(p16, p16, 9000, 4, 4, 1, 0, one, 1, 1.1, 2, 2, 1e1, 1e7, p16, k, mu, None, None, None) == rt.E_UNSUPPORTED
    assert b"nested_tgkt_solve" in lib.rtsvd_last_error()
    # tlanczos_solve(A, B, m, n, p, dtype, delta, n_delta, eta, k_max, X, k, resid, status, stream)
    g = lib.tlanczos_solve
    assert g(None, p16, 4, 4, 1, 0, one, 1, 1.1, 2, p16, k, None, None, None) == rt.E_ARG
    assert g(p16, p16, 4, 4, 1, 0, one, 1, 1.1, 5, p16, k, None, None, None) == rt.E_ARG         # k_max > m
    assert g(p16, p16, 4, 4, 1, 9, one, 1, 1.1, 2, p16, k, None, None, None) == rt.E_ARG         # dtype
    assert g(p16, p16, 9000, 4, 1, 0, one, 1, 1.1, 2, p16, k, None, None, None) == rt.E_UNSUPPORTED
    # ttevd_factor(A, m, n, dtype, precision, k_max, stream, out)
    h = ctypes.c_void_p()
    t = lib.ttevd_factor
    assert t(None, 4, 4, 0, 0, 2, None, ctypes.byref(h)) == rt.E_ARG
    assert t(p16, 4, 4, 0, 2, 2, None, ctypes.byref(h)) == rt.E_ARG                               # bf16
    assert t(p16, 4, 4, 0, 0, 5, None, ctypes.byref(h)) == rt.E_ARG                               # k_max > m
    assert t(p16, 300, 4, 0, 0, 5, None, ctypes.byref(h)) == rt.E_UNSUPPORTED                     # m > 256


def test_bench_refuses_several_gpus():
    import subprocess
    import sys
    out = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                         text=True, timeout=60)
    assert out.returncode == 2
    assert "one GPU" in out.stdout


@pytest.mark.skipif(not os.path.exists(LIB), reason="librtsvd.so not built")
def test_gaussian_argument_errors_without_gpu():
    from paper_2110_02485_amd import rtsvd as rt
    lib = rt.load()
    assert lib.rtsvd_gaussian(1, 4, 4, 4, 0, None, None) == rt.E_ARG
    assert lib.rtsvd_gaussian(1, 0, 4, 4, 0, ctypes.c_void_p(16), None) == rt.E_ARG
    assert lib.rtsvd_gaussian(1, 4, 4, 4, 9, ctypes.c_void_p(16), None) == rt.E_ARG
    assert lib.rtsvd_gaussian(1, 1 << 20, 1 << 12, 1 << 10, 0, ctypes.c_void_p(16), None) == rt.E_UNSUPPORTED
    assert lib.rtsvd_status_string(rt.E_NOTFINITE) is not None


def test_solve_arguments_are_checked_before_the_call():
    # Factor.solve validates B and the output buffers against the factor's sizes (the library reads
    # l p n elements of B and writes m p n of X with the factor's l, m, n): mismatches raise before
    # any launch
    import torch
    from paper_2110_02485_amd import rtsvd as rt
    f = rt.Factor.__new__(rt.Factor)
    f._h = None
    f.dtype, f.device = torch.float64, torch.device("cuda", 0)
    f.l, f.m, f.n, f.k_max, f.r, f.oversample = 40, 32, 16, 10, 14, 4
    dev = torch.device("cuda", 0)
    f.check_solve_args((16, 3, 40), torch.float64, dev, 1, 1)            # fits
    f.check_solve_args((16, 3, 40), torch.float64, dev, 3, 0)
    with pytest.raises(ValueError):
        f.check_solve_args((8, 3, 40), torch.float64, dev, 1, 1)         # fewer tubes than the factor's n
    with pytest.raises(ValueError):
        f.check_solve_args((16, 3, 39), torch.float64, dev, 1, 1)        # rows differ from l
    with pytest.raises(ValueError):
        f.check_solve_args((16, 3, 40), torch.float32, dev, 1, 1)        # dtype
    with pytest.raises(ValueError):
        f.check_solve_args((16, 3, 40), torch.float64, torch.device("cuda", 1), 1, 1)
    with pytest.raises(ValueError):
        f.check_solve_args((16, 3, 40), torch.float64, dev, 2, 1)        # 2 bounds for 3 slices
    with pytest.raises(ValueError):
        f.check_solve_args((16, 3, 40), torch.float64, dev, 1, 11)       # k_start > min(k_max, r)

    class Out:
        pass
    out = Out()
    out.X = torch.empty((16, 3, 31), dtype=torch.float64)                # m is 32
    out.k = torch.empty(1, dtype=torch.int32)
    out.resid = torch.empty((1, 10), dtype=torch.float64)
    out.status = torch.empty(1, dtype=torch.int32)
    with pytest.raises(ValueError):
        f.check_solve_args((16, 3, 40), torch.float64, dev, 1, 1, out)
