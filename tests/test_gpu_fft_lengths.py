"""GPU parity of the tube transforms at tube lengths that are not powers of two (Section 2's DFT
along the tubes; Section 5 uses n = 240, 300 and 500): the mixed-radix kernels (radices 2 to 13)
and the direct DFT (lengths with a larger prime factor) against the FP64 oracle's t-product, and a
restoration of the Section 5 video shape at n = 240."""
import numpy as np
import pytest

from oracle import tproduct as tp
from oracle import solve as so
from paper_2110_02485_amd import workloads as wl
from tests.problems import blur_problem

pytestmark = pytest.mark.gpu


def _t(a, dtype="float64"):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).to(device="cuda", dtype=getattr(torch, dtype))


def _np(t):
    return t.detach().double().cpu().numpy()


def _rel(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


# (l, m, p, n): small lateral sizes for every radix and its combinations, one length with a prime
# factor above 13 (17, 34: direct DFT), enough tubes at 240 / 300 / 500 that the workgroup count
# is rounded up for the XCD spread (a ragged last group), and n = 128 (the lane-pair register
# transform in FP32) with tube counts that leave the last workgroup partly or almost wholly empty
CASES = [(13, 10, 3, n) for n in (3, 5, 6, 9, 11, 13, 17, 26, 34, 49, 210)] + \
        [(61, 37, 2, 240), (61, 37, 1, 300), (40, 33, 2, 500), (13, 10, 3, 128), (61, 37, 2, 128)]


@pytest.mark.parametrize("l,m,p,n", CASES)
@pytest.mark.parametrize("dtype,tol", [("float64", 1e-12), ("float32", 2e-5)])
def test_tprod_and_adjoint_any_tube_length(l, m, p, n, dtype, tol):
    from paper_2110_02485_amd import rtsvd as rt
    print(f"[fft_lengths] {dtype} l={l} m={m} p={p} n={n}", flush=True)
    rng = np.random.default_rng(l * 1000 + m * 10 + n)
    A = rng.standard_normal((n, m, l))
    X = rng.standard_normal((n, p, m))
    Y = rng.standard_normal((n, p, l))
    C = _np(rt.tprod(_t(A, dtype), _t(X, dtype)))
    ref = wl.to_storage(tp.tprod(wl.to_math(A), wl.to_math(X)))
    assert _rel(C, ref) <= tol
    # element-wise as well: a wrong twiddle on one face or one tube would hide in the norm
    assert np.max(np.abs(C - ref)) <= 20 * tol * np.max(np.abs(ref))
    Bt = _np(rt.tprod_adjoint(_t(A, dtype), _t(Y, dtype)))
    ref = wl.to_storage(tp.tprod(tp.ttranspose(wl.to_math(A)), wl.to_math(Y)))
    assert _rel(Bt, ref) <= tol


@pytest.mark.parametrize("n", [240, 300, 500])
def test_tprod_single_tube(n):
    # one tube pair per workgroup (l = m = p = 1): the second real tube of the packed complex
    # sequence is absent
    from paper_2110_02485_amd import rtsvd as rt
    rng = np.random.default_rng(n)
    A = rng.standard_normal((n, 1, 1))
    X = rng.standard_normal((n, 1, 1))
    C = _np(rt.tprod(_t(A), _t(X)))
    ref = wl.to_storage(tp.tprod(wl.to_math(A), wl.to_math(X)))
    assert _rel(C, ref) <= 1e-12


@pytest.mark.parametrize("dtype,tol", [("float64", 1e-11), ("float32", 1e-5)])
def test_rtsvd_video_shape_n240(dtype, tol):
    # the shape of Section 5's grey-scale video example at a reduced frame size: 6 frames as
    # lateral slices, A from eq. (za) with band 12 and sigma 2.5, tube length 240 (121 faces),
    # eta 1.2; k <= 20, rho = 10, q = 1
    import torch
    from paper_2110_02485_amd import rtsvd as rt
    A, X, B, Om, delta = blur_problem(40, 240, 2.5, 12, 6, 1e-2, 20, 10, seed=83, video=True)
    orc = so.rtsvd_restore(wl.to_math(A), wl.to_math(B), wl.to_math(Om), delta, 1.2, 20, 1, 1, False, None)
    precision = "fp64" if dtype == "float64" else "fp32"
    f = rt.factor(_t(A, dtype), 20, 10, 1, precision, _t(Om, dtype))
    res = f.solve(_t(B, dtype), delta, 1.2, 1)
    torch.cuda.synchronize()
    assert int(res.k[0]) == orc["k"] and int(res.status[0]) == orc["status"]
    Xg = _np(res.X)
    Xo = wl.to_storage(orc["X"])
    assert _rel(Xg, Xo) <= tol
    assert np.max(np.abs(Xg - Xo)) <= 20 * tol * np.max(np.abs(Xo))
    np.testing.assert_allclose(_np(res.resid)[0], orc["res"][:, 0], rtol=10 * tol)
    f.close()
