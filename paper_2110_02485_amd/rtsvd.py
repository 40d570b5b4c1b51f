"""Python binding of librtsvd (argument marshalling only; every step runs in the HIP library).

Tensors are torch tensors on a ROCm device in storage order: a tensor A in R^{l x m x n} is a
contiguous torch tensor of shape (n, m, l) (column-major l x m x n, frontal slices contiguous),
float64 or float32.  Work is ordered on torch's current stream.  The library must be built
(``python -m paper_2110_02485_amd.build``); a missing library raises, there is no fallback.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "librtsvd.so")

F64, F32 = 0, 1
P_FP64, P_FP32, P_BF16 = 0, 1, 2
OK, W_DP_NOT_MET, W_RANK_DEFICIENT = 0, 1, 2
E_ARG, E_NOTFINITE, E_HIP, E_NOMEM, E_UNSUPPORTED = -1, -2, -3, -4, -5

PRECISIONS = {"fp64": P_FP64, "fp32": P_FP32, "bf16": P_BF16, "mixed": P_BF16}

EXPORTS = ["rtsvd_factor", "ttsvd_factor", "rtsvd_factor_info", "rtsvd_factor_destroy", "rtsvd_solve",
           "tprod", "tprod_adjoint", "tgkb_solve", "nested_tgkb_solve", "ttevd_factor", "tlanczos_solve", "rtsvd_status_string", "rtsvd_last_error",
           "rtsvd_timer_enable", "rtsvd_timer_read", "rtsvd_solve_vjp", "rtsvd_trim", "rtsvd_gaussian",
           "rtsvd_solve_noalloc", "tgkt_solve", "tlanczos_tik_solve", "nested_tgkt_solve"]


class RtsvdError(RuntimeError):
    def __init__(self, code: int, where: str, detail: str):
        super().__init__(f"{where}: status {code}: {detail}")
        self.code = code


class _Opts(ctypes.Structure):
    _fields_ = [("k_max", ctypes.c_int32), ("oversample", ctypes.c_int32), ("power_iters", ctypes.c_int32),
                ("precision", ctypes.c_int32), ("seed", ctypes.c_uint64), ("omega", ctypes.c_void_p),
                ("eps", ctypes.c_double), ("adaptive", ctypes.c_int32), ("face_groups", ctypes.c_int32),
                ("sketch_tile", ctypes.c_int32)]


_lib = None


def load(path: str = LIB_PATH) -> ctypes.CDLL:
    """Load librtsvd.so once; raises FileNotFoundError when it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise FileNotFoundError(f"{path} not built: run `python -m paper_2110_02485_amd.build`")
    lib = ctypes.CDLL(path)
    vp, i64, i32, dbl = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32, ctypes.c_double
    pi32, pdbl = ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_double)
    lib.rtsvd_factor.argtypes = [vp, i64, i64, i64, ctypes.c_int, ctypes.POINTER(_Opts), vp, ctypes.POINTER(vp)]
    lib.ttsvd_factor.argtypes = [vp, i64, i64, i64, ctypes.c_int, i32, i32, vp, ctypes.POINTER(vp)]
    lib.rtsvd_factor_info.argtypes = [vp, pi32, pi32, pdbl, pi32, pdbl, pi32]
    lib.rtsvd_factor_destroy.argtypes = [vp]
    lib.rtsvd_factor_destroy.restype = None
    lib.rtsvd_solve.argtypes = [vp, vp, i64, ctypes.c_int, pdbl, i32, dbl, i32, vp, vp, vp, vp, vp]
    lib.rtsvd_solve_noalloc.argtypes = [vp, vp, i64, ctypes.c_int, pdbl, i32, dbl, i32, vp, vp, vp, vp, vp]
    lib.tprod.argtypes = [vp, vp, vp, i64, i64, i64, i64, ctypes.c_int, vp]
    lib.tprod_adjoint.argtypes = [vp, vp, vp, i64, i64, i64, i64, ctypes.c_int, vp]
    if hasattr(lib, "tgkb_solve"):
        lib.tgkb_solve.argtypes = [vp, vp, i64, i64, i64, i64, ctypes.c_int, pdbl, i32, dbl, i32, vp, vp, vp, vp, vp]
    if hasattr(lib, "ttevd_factor"):
        lib.ttevd_factor.argtypes = [vp, i64, i64, ctypes.c_int, i32, i32, vp, ctypes.POINTER(vp)]
    if hasattr(lib, "tlanczos_solve"):
        lib.tlanczos_solve.argtypes = [vp, vp, i64, i64, i64, ctypes.c_int, pdbl, i32, dbl, i32, vp, vp, vp, vp, vp]
    if hasattr(lib, "nested_tgkb_solve"):
        lib.nested_tgkb_solve.argtypes = [vp, vp, i64, i64, i64, i64, ctypes.c_int, pdbl, i32, dbl, i32, i32, vp, vp, vp,
                                          vp, vp]
    lib.rtsvd_status_string.restype = ctypes.c_char_p
    lib.rtsvd_status_string.argtypes = [ctypes.c_int]
    lib.rtsvd_last_error.restype = ctypes.c_char_p
    lib.rtsvd_solve_vjp.argtypes = [vp, vp, vp, vp, vp, i64, i64, i64, i64, i32, i32, ctypes.c_int, vp, vp, vp]
    lib.rtsvd_timer_enable.argtypes = [ctypes.c_int]
    lib.rtsvd_timer_read.argtypes = [ctypes.c_int, pdbl, pi32]
    lib.rtsvd_trim.argtypes = []
    lib.rtsvd_gaussian.argtypes = [ctypes.c_uint64, i64, i64, i64, ctypes.c_int, vp, vp]
    lib.tgkt_solve.argtypes = [vp, vp, i64, i64, i64, i64, ctypes.c_int, pdbl, i32, dbl, i32, dbl, dbl, vp, vp, vp, vp,
                               vp, vp]
    lib.tlanczos_tik_solve.argtypes = [vp, vp, i64, i64, i64, ctypes.c_int, pdbl, i32, dbl, i32, dbl, dbl, vp, vp, vp,
                                       vp, vp, vp]
    lib.nested_tgkt_solve.argtypes = [vp, vp, i64, i64, i64, i64, ctypes.c_int, pdbl, i32, dbl, i32, i32, dbl, dbl, vp,
                                      vp, vp, vp, vp, vp]
    _lib = lib
    return lib


def _check(rc: int, where: str) -> int:
    if rc < 0:
        lib = load()
        raise RtsvdError(rc, where, lib.rtsvd_last_error().decode())
    return rc


def _dtype_code(t: torch.Tensor) -> int:
    if t.dtype == torch.float64:
        return F64
    if t.dtype == torch.float32:
        return F32
    raise TypeError(f"unsupported dtype {t.dtype}")


def _dev(t: torch.Tensor, name: str) -> torch.Tensor:
    if not t.is_cuda:
        raise ValueError(f"{name} must be a device tensor")
    if t.dim() != 3:
        raise ValueError(f"{name} must be 3-D in storage order (n, cols, rows)")
    return t.contiguous()


def _stream() -> ctypes.c_void_p:
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def gaussian(seed: int, m: int, r: int, n: int, dtype=torch.float64, device="cuda") -> torch.Tensor:
    """The Gaussian test tensor (m x r x n, storage shape (n, r, m)) that rtsvd_factor draws on the
    device from `seed` when no omega is given (Philox4x32-10 + Box-Muller, see include/rtsvd.h)."""
    lib = load()
    out = torch.empty((n, r, m), dtype=dtype, device=device)
    code = F64 if dtype == torch.float64 else F32 if dtype == torch.float32 else None
    if code is None:
        raise TypeError(f"unsupported dtype {dtype}")
    _check(lib.rtsvd_gaussian(int(seed) & ((1 << 64) - 1), m, r, n, code, out.data_ptr(), _stream()),
           "rtsvd_gaussian")
    return out


def tprod(A: torch.Tensor, B: torch.Tensor) -> torch.Tensor:
    """C = A * B (storage order: A (n, m, l), B (n, p, m) -> C (n, p, l))."""
    lib = load()
    A, B = _dev(A, "A"), _dev(B, "B")
    n, m, l = A.shape
    n2, p, m2 = B.shape
    if n2 != n or m2 != m or B.dtype != A.dtype:
        raise ValueError("tprod: shape/dtype mismatch")
    C = torch.empty((n, p, l), dtype=A.dtype, device=A.device)
    _check(lib.tprod(A.data_ptr(), B.data_ptr(), C.data_ptr(), l, m, p, n, _dtype_code(A), _stream()), "tprod")
    return C


def tprod_adjoint(A: torch.Tensor, C: torch.Tensor) -> torch.Tensor:
    """B = A^T * C (storage order: A (n, m, l), C (n, p, l) -> B (n, p, m))."""
    lib = load()
    A, C = _dev(A, "A"), _dev(C, "C")
    n, m, l = A.shape
    n2, p, l2 = C.shape
    if n2 != n or l2 != l or C.dtype != A.dtype:
        raise ValueError("tprod_adjoint: shape/dtype mismatch")
    B = torch.empty((n, p, m), dtype=A.dtype, device=A.device)
    _check(lib.tprod_adjoint(A.data_ptr(), C.data_ptr(), B.data_ptr(), l, m, p, n, _dtype_code(A), _stream()),
           "tprod_adjoint")
    return B


@dataclass
class SolveResult:
    X: torch.Tensor
    k: torch.Tensor        # device int32 [groups]
    resid: torch.Tensor    # device float64 [groups, k_cap]
    status: torch.Tensor   # device int32 [1]


class Factor:
    """An R-tSVD (or T-tSVD) factor held by the library; solve() may be called many times."""

    def __init__(self, handle: int, dtype: torch.dtype, device, l: int, m: int, n: int, k_max: int, r: int,
                 oversample: int):
        self._h = ctypes.c_void_p(handle)
        self.dtype, self.device = dtype, device
        self.l, self.m, self.n = l, m, n
        self.k_max, self.r, self.oversample = k_max, r, oversample

    @classmethod
    def rtsvd(cls, A: torch.Tensor, k_max: int, oversample: int, power_iters: int = 0, precision: str = "fp64",
              omega: torch.Tensor | None = None, eps: float = 0.0, seed: int = 0,
              adaptive: bool = False, face_groups: int = 0, sketch_tile: int = 0) -> "Factor":
        lib = load()
        A = _dev(A, "A")
        n, m, l = A.shape
        r = min(k_max + oversample, m)
        optr = None
        if omega is not None:     # else: drawn on the device from `seed` (rtsvd_gaussian)
            omega = _dev(omega, "omega")
            if tuple(omega.shape) != (n, r, m) or omega.dtype != A.dtype or omega.device != A.device:
                raise ValueError(f"omega must have shape {(n, r, m)}, dtype {A.dtype} and A's device")
            optr = omega.data_ptr()
        opts = _Opts(k_max, oversample, power_iters, PRECISIONS[precision], int(seed) & ((1 << 64) - 1), optr, eps,
                     1 if adaptive else 0, face_groups, sketch_tile)
        h = ctypes.c_void_p()
        _check(lib.rtsvd_factor(A.data_ptr(), l, m, n, _dtype_code(A), ctypes.byref(opts), _stream(),
                                ctypes.byref(h)), "rtsvd_factor")
        f = cls(h.value, A.dtype, A.device, l, m, n, k_max, r, oversample)
        f._keep = omega  # the factor reads omega asynchronously
        if adaptive and eps > 0.0:
            f.r = f.info()[0]   # the fixed-precision factor keeps r_eps columns (the call synchronized)
        return f

    @classmethod
    def ttsvd(cls, A: torch.Tensor, k_max: int, precision: str = "fp64") -> "Factor":
        lib = load()
        A = _dev(A, "A")
        n, m, l = A.shape
        h = ctypes.c_void_p()
        _check(lib.ttsvd_factor(A.data_ptr(), l, m, n, _dtype_code(A), PRECISIONS[precision], k_max, _stream(),
                                ctypes.byref(h)), "ttsvd_factor")
        return cls(h.value, A.dtype, A.device, l, m, n, k_max, m, 0)

    @classmethod
    def ttevd(cls, A: torch.Tensor, k_max: int, precision: str = "fp64") -> "Factor":
        """T-tEVD factor of a symmetric A (Hermitian DFT faces)."""
        lib = load()
        A = _dev(A, "A")
        n, m, l = A.shape
        if l != m:
            raise ValueError("ttevd needs a square (symmetric) tensor")
        h = ctypes.c_void_p()
        _check(lib.ttevd_factor(A.data_ptr(), m, n, _dtype_code(A), PRECISIONS[precision], k_max, _stream(),
                                ctypes.byref(h)), "ttevd_factor")
        return cls(h.value, A.dtype, A.device, m, m, n, k_max, m, 0)

    def info(self, with_status: bool = False):
        """(r, faces, eta (r+1), r_eps, sigma (faces, r), flags) and, with_status, the call's status
        (OK, W_RANK_DEFICIENT or E_NOTFINITE: a non-finite A is reported, not raised); synchronizes."""
        import numpy as np
        lib = load()
        r, faces, r_eps, flags = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()
        lib.rtsvd_factor_info(self._h, ctypes.byref(r), ctypes.byref(faces), None, None, None, None)
        eta = np.zeros(r.value + 1)
        sig = np.zeros(r.value * faces.value)
        rc = lib.rtsvd_factor_info(self._h, ctypes.byref(r), ctypes.byref(faces),
                                   eta.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), ctypes.byref(r_eps),
                                   sig.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), ctypes.byref(flags))
        if rc != E_NOTFINITE:
            _check(rc, "rtsvd_factor_info")
        out = (r.value, faces.value, eta, r_eps.value, sig.reshape(faces.value, r.value), flags.value)
        return out + (rc,) if with_status else out

    def k_cap(self, k_start: int) -> int:
        return self.r if k_start == 0 else min(self.k_max, self.r)

    def check_solve_args(self, shape, dtype, device, groups: int, k_start: int, out=None) -> None:
        """Raise ValueError unless B (storage shape `shape`) and the optional output buffers fit this
        factor: the library reads l p n elements of B and writes m p n of X, sizes it takes from the
        factor, so a mismatch must be caught before the call."""
        n, p, l = shape
        if (n, l) != (self.n, self.l) or dtype != self.dtype or device != self.device:
            raise ValueError(f"B must have storage shape ({self.n}, p, {self.l}), dtype {self.dtype} and the "
                             f"factor's device; got {tuple(shape)} {dtype} {device}")
        if groups not in (1, p):
            raise ValueError(f"delta must hold 1 or p = {p} values, got {groups}")
        if not 0 <= k_start <= min(self.k_max, self.r):
            raise ValueError(f"k_start must be in [0, min(k_max, r)] = [0, {min(self.k_max, self.r)}]")
        if out is None:
            return
        kcap = self.k_cap(k_start)
        want = {"X": ((n, p, self.m), dtype), "k": ((groups,), torch.int32),
                "resid": ((groups, kcap), torch.float64), "status": ((1,), torch.int32)}
        for name, (shp, dt) in want.items():
            t = getattr(out, name)
            if tuple(t.shape) != shp or t.dtype != dt or t.device != self.device or not t.is_contiguous():
                raise ValueError(f"out.{name} must be a contiguous {dt} tensor of shape {shp} on the factor's device")

    def solve(self, B: torch.Tensor, delta, eta: float, k_start: int = 1, out: SolveResult | None = None,
              no_alloc: bool = False) -> SolveResult:
        """Truncated solution with the discrepancy principle.  no_alloc: rtsvd_solve_noalloc (the
        library's fixed scratch array instead of device allocations; pass `out` as well for a call
        that allocates nothing at all)."""
        lib = load()
        B = _dev(B, "B")
        n, p, l = B.shape
        deltas = [float(d) for d in (delta if hasattr(delta, "__len__") else [delta])]
        groups = len(deltas)
        kcap = self.k_cap(k_start)
        self.check_solve_args(tuple(B.shape), B.dtype, B.device, groups, k_start, out)
        if out is None:
            out = SolveResult(X=torch.empty((n, p, self.m), dtype=B.dtype, device=B.device),
                              k=torch.empty(groups, dtype=torch.int32, device=B.device),
                              resid=torch.empty((groups, kcap), dtype=torch.float64, device=B.device),
                              status=torch.empty(1, dtype=torch.int32, device=B.device))
        arr = (ctypes.c_double * groups)(*deltas)
        fn, name = (lib.rtsvd_solve_noalloc, "rtsvd_solve_noalloc") if no_alloc else (lib.rtsvd_solve, "rtsvd_solve")
        _check(fn(self._h, B.data_ptr(), p, _dtype_code(B), arr, groups, eta, k_start, out.X.data_ptr(),
                  out.k.data_ptr(), out.resid.data_ptr(), out.status.data_ptr(), _stream()), name)
        return out

    def close(self):
        if self._h is not None and self._h.value:
            load().rtsvd_factor_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def trim() -> None:
    """Free the library's cached device workspace (synchronizes the devices that hold it)."""
    _check(load().rtsvd_trim(), "rtsvd_trim")


def factor(A, k_max, oversample, power_iters=0, precision="fp64", omega=None, eps=0.0, adaptive=False,
           face_groups=0, sketch_tile=0, seed=0) -> Factor:
    """R-tSVD factor of A (see Factor.rtsvd); omega None: the Gaussian tensor is drawn on the device from
    `seed` (see gaussian()); adaptive=True with eps > 0: Alg. 6's fixed-precision rank;
    face_groups: 0 automatic, 1..3; sketch_tile: 0 automatic, 1, 2, 4 or 8 sixteen-column tiles per
    workgroup in the A-hat products (the result depends on neither)."""
    return Factor.rtsvd(A, k_max, oversample, power_iters, precision, omega, eps, seed=seed, adaptive=adaptive,
                        face_groups=face_groups, sketch_tile=sketch_tile)


def ttsvd_factor(A, k_max, precision="fp64") -> Factor:
    """Full facewise SVD factor of A (T-tSVD comparator)."""
    return Factor.ttsvd(A, k_max, precision)


def ttevd_factor(A, k_max, precision="fp64") -> Factor:
    """T-tEVD factor of a symmetric A (Hermitian DFT faces); solve it like any factor."""
    return Factor.ttevd(A, k_max, precision)


def tlanczos_solve(A: torch.Tensor, B: torch.Tensor, delta, eta: float, k_max: int):
    """t-Lanczos_p restoration of a symmetric A; returns (X, k (device int32 [p]), resid (device [p, k_max]), status)."""
    lib = load()
    A, B = _dev(A, "A"), _dev(B, "B")
    n, m, l = A.shape
    if l != m:
        raise ValueError("t-Lanczos needs a square (symmetric) tensor")
    _, p, _ = B.shape
    deltas = [float(d) for d in (delta if hasattr(delta, "__len__") else [delta])]
    arr = (ctypes.c_double * len(deltas))(*deltas)
    X = torch.empty((n, p, m), dtype=A.dtype, device=A.device)
    k = torch.empty(p, dtype=torch.int32, device=A.device)
    resid = torch.empty((p, k_max), dtype=torch.float64, device=A.device)
    status = torch.empty(1, dtype=torch.int32, device=A.device)
    _check(lib.tlanczos_solve(A.data_ptr(), B.data_ptr(), m, n, p, _dtype_code(A), arr, len(deltas), eta, k_max,
                              X.data_ptr(), k.data_ptr(), resid.data_ptr(), status.data_ptr(), _stream()),
           "tlanczos_solve")
    return X, k, resid, status


def tgkb_solve(A: torch.Tensor, B: torch.Tensor, delta, eta: float, k_max: int):
    """tGKB_p restoration; returns (X, k (device int32 [p]), resid (device [p, k_max]), status)."""
    lib = load()
    A, B = _dev(A, "A"), _dev(B, "B")
    n, m, l = A.shape
    _, p, _ = B.shape
    deltas = [float(d) for d in (delta if hasattr(delta, "__len__") else [delta])]
    arr = (ctypes.c_double * len(deltas))(*deltas)
    X = torch.empty((n, p, m), dtype=A.dtype, device=A.device)
    k = torch.empty(p, dtype=torch.int32, device=A.device)
    resid = torch.empty((p, k_max), dtype=torch.float64, device=A.device)
    status = torch.empty(1, dtype=torch.int32, device=A.device)
    _check(lib.tgkb_solve(A.data_ptr(), B.data_ptr(), l, m, n, p, _dtype_code(A), arr, len(deltas), eta, k_max,
                          X.data_ptr(), k.data_ptr(), resid.data_ptr(), status.data_ptr(), _stream()), "tgkb_solve")
    return X, k, resid, status


def _tikhonov(fn_name, A, B, delta, eta, k_max, mu_lo, mu_hi, square):
    lib = load()
    A, B = _dev(A, "A"), _dev(B, "B")
    n, m, l = A.shape
    if square and l != m:
        raise ValueError("t-Lanczos needs a square (symmetric) tensor")
    n2, p, l2 = B.shape
    if (n2, l2) != (n, l) or B.dtype != A.dtype or B.device != A.device:
        raise ValueError("B must have storage shape (n, p, l) of A, A's dtype and device")
    deltas = [float(d) for d in (delta if hasattr(delta, "__len__") else [delta])]
    arr = (ctypes.c_double * len(deltas))(*deltas)
    X = torch.empty((n, p, m), dtype=A.dtype, device=A.device)
    k = torch.empty(p, dtype=torch.int32, device=A.device)
    mu = torch.empty(p, dtype=torch.float64, device=A.device)
    resid = torch.empty(p, dtype=torch.float64, device=A.device)
    status = torch.empty(1, dtype=torch.int32, device=A.device)
    fn = getattr(lib, fn_name)
    dims = (m, n, p) if square else (l, m, n, p)
    _check(fn(A.data_ptr(), B.data_ptr(), *dims, _dtype_code(A), arr, len(deltas), eta, k_max, mu_lo, mu_hi,
              X.data_ptr(), k.data_ptr(), mu.data_ptr(), resid.data_ptr(), status.data_ptr(), _stream()), fn_name)
    return X, k, mu, resid, status


def tgkt_solve(A: torch.Tensor, B: torch.Tensor, delta, eta: float, k_max: int, mu_lo: float = 1e1,
               mu_hi: float = 1e7):
    """tGKT_p restoration (Tikhonov on the tGKB space, mu by bisection on [mu_lo, mu_hi]); returns
    (X, k (device int32 [p]), mu (device [p]), residual at mu (device [p]), status)."""
    return _tikhonov("tgkt_solve", A, B, delta, eta, k_max, mu_lo, mu_hi, False)


def tlanczos_tik_solve(A: torch.Tensor, B: torch.Tensor, delta, eta: float, k_max: int, mu_lo: float = 1e1,
                       mu_hi: float = 1e7):
    """t-LanczosTik_p restoration of a symmetric A; returns (X, k, mu, residual at mu, status)."""
    return _tikhonov("tlanczos_tik_solve", A, B, delta, eta, k_max, mu_lo, mu_hi, True)


def nested_tgkb_solve(A: torch.Tensor, B: torch.Tensor, delta, eta: float, k_max: int, k_init: int = 2):
    """nested_tGKB_p restoration; returns (X, k (device int32 [p]), resid (device [p, k_max]), status)."""
    lib = load()
    A, B = _dev(A, "A"), _dev(B, "B")
    n, m, l = A.shape
    _, p, _ = B.shape
    deltas = [float(d) for d in (delta if hasattr(delta, "__len__") else [delta])]
    arr = (ctypes.c_double * len(deltas))(*deltas)
    X = torch.empty((n, p, m), dtype=A.dtype, device=A.device)
    k = torch.empty(p, dtype=torch.int32, device=A.device)
    resid = torch.empty((p, k_max), dtype=torch.float64, device=A.device)
    status = torch.empty(1, dtype=torch.int32, device=A.device)
    _check(lib.nested_tgkb_solve(A.data_ptr(), B.data_ptr(), l, m, n, p, _dtype_code(A), arr, len(deltas), eta, k_max,
                                 k_init, X.data_ptr(), k.data_ptr(), resid.data_ptr(), status.data_ptr(), _stream()),
           "nested_tgkb_solve")
    return X, k, resid, status


def nested_tgkt_solve(A: torch.Tensor, B: torch.Tensor, delta, eta: float, k_max: int, k_init: int = 2,
                      mu_lo: float = 1e1, mu_hi: float = 1e7):
    """nested_tGKT_p restoration (Tikhonov on the nested space of nested_tGKB_p, mu by bisection on
    [mu_lo, mu_hi]); returns (X, k (device int32 [p]), mu (device [p]), projected residual at mu
    (device [p]), status)."""
    lib = load()
    A, B = _dev(A, "A"), _dev(B, "B")
    n, m, l = A.shape
    n2, p, l2 = B.shape
    if (n2, l2) != (n, l) or B.dtype != A.dtype or B.device != A.device:
        raise ValueError("B must have storage shape (n, p, l) of A, A's dtype and device")
    deltas = [float(d) for d in (delta if hasattr(delta, "__len__") else [delta])]
    arr = (ctypes.c_double * len(deltas))(*deltas)
    X = torch.empty((n, p, m), dtype=A.dtype, device=A.device)
    k = torch.empty(p, dtype=torch.int32, device=A.device)
    mu = torch.empty(p, dtype=torch.float64, device=A.device)
    resid = torch.empty(p, dtype=torch.float64, device=A.device)
    status = torch.empty(1, dtype=torch.int32, device=A.device)
    _check(lib.nested_tgkt_solve(A.data_ptr(), B.data_ptr(), l, m, n, p, _dtype_code(A), arr, len(deltas), eta, k_max,
                                 k_init, mu_lo, mu_hi, X.data_ptr(), k.data_ptr(), mu.data_ptr(), resid.data_ptr(),
                                 status.data_ptr(), _stream()), "nested_tgkt_solve")
    return X, k, mu, resid, status


def solve_vjp(A: torch.Tensor, dA, B: torch.Tensor, omega: torch.Tensor, gX: torch.Tensor, k: int, oversample: int):
    """(dL/dB, <dL/dX, dX/ds> or None) of the fixed-k truncated R-tSVD restoration (factor recomputed)."""
    lib = load()
    A, B, omega, gX = _dev(A, "A"), _dev(B, "B"), _dev(omega, "omega"), _dev(gX, "gX")
    n, m, l = A.shape
    _, p, _ = B.shape
    r = min(k + oversample, m)
    for name, t, shape in (("B", B, (n, p, l)), ("omega", omega, (n, r, m)), ("gX", gX, (n, p, m))):
        if tuple(t.shape) != shape or t.dtype != A.dtype or t.device != A.device:
            raise ValueError(f"{name} must have storage shape {shape}, dtype {A.dtype} and A's device; "
                             f"got {tuple(t.shape)} {t.dtype}")
    if dA is not None and (tuple(dA.shape) != tuple(A.shape) or dA.dtype != A.dtype or dA.device != A.device):
        raise ValueError("dA must match A in shape, dtype and device")
    gB = torch.empty_like(B)
    gdot = None
    dptr = None
    if dA is not None:
        dA = _dev(dA, "dA")
        gdot = torch.zeros(1, dtype=torch.float64, device=A.device)
        dptr = dA.data_ptr()
    _check(lib.rtsvd_solve_vjp(A.data_ptr(), dptr, B.data_ptr(), omega.data_ptr(), gX.data_ptr(), l, m, n, p, k,
                               oversample, _dtype_code(A), gB.data_ptr(), gdot.data_ptr() if gdot is not None else None,
                               _stream()), "rtsvd_solve_vjp")
    return gB, gdot
