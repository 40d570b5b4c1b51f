"""GPU: the on-device Gaussian tensor against the oracle's generator, restorations that draw it on
the device, and the degenerate cases of the method -- an exactly rank-deficient sketch (Alg. 3's
breakdown), a zero Fourier face, non-finite input -- against the oracle."""
import numpy as np
import pytest

from oracle import gaussian as ga
from oracle import solve as so
from oracle import tproduct as tp
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


@pytest.mark.parametrize("seed,m,r,n", [(211002485, 64, 30, 16), (2 ** 40 + 7, 33, 5, 7), (0, 1, 1, 1)])
def test_gaussian_tensor_matches_oracle(seed, m, r, n):
    from paper_2110_02485_amd import rtsvd as rt
    import torch
    print(f"[gauss] seed={seed} m={m} r={r} n={n}", flush=True)
    ref = wl.to_storage(ga.gaussian_tensor(seed, m, r, n))
    g64 = _np(rt.gaussian(seed, m, r, n, torch.float64))
    assert np.abs(g64 - ref).max() <= 1e-13 * max(1.0, np.abs(ref).max())
    g32 = rt.gaussian(seed, m, r, n, torch.float32).cpu().numpy()
    assert np.abs(g32 - ref.astype(np.float32)).max() <= 1e-6 * max(1.0, np.abs(ref).max())


def test_gaussian_tensor_moments_and_spectrum():
    from paper_2110_02485_amd import rtsvd as rt
    import torch
    m, r, n = 1024, 120, 128                       # the 1024-wide workload's tensor: 15.7 M draws
    g = rt.gaussian(12345, m, r, n, torch.float64)
    z = g.flatten()
    nz = z.numel()
    assert abs(float(z.mean())) < 5.0 / nz ** 0.5
    assert abs(float(z.var()) - 1.0) < 5.0 * (2.0 / nz) ** 0.5
    k4 = float(((z - z.mean()) ** 4).mean() / z.var() ** 2)
    assert abs(k4 - 3.0) < 5.0 * (24.0 / nz) ** 0.5
    # sampled against the oracle element by element
    idx = np.random.default_rng(0).integers(0, nz, 4096)
    ref = ga.gaussian_tensor(12345, m, r, n).ravel(order="F")
    np.testing.assert_allclose(z.cpu().numpy()[idx], ref[idx], rtol=0, atol=1e-13)
    # its tube DFT through the library's t-product with the identity (omega * I = omega) stays
    # conjugate symmetric in the Fourier domain: real data round-trips
    small = rt.gaussian(7, 16, 4, 9, torch.float64)
    eye = torch.zeros((9, 4, 4), dtype=torch.float64, device="cuda")
    eye[0] = torch.eye(4, dtype=torch.float64, device="cuda")
    back = rt.tprod(small, eye)
    torch.testing.assert_close(back, small, rtol=0, atol=1e-14)
    oh = np.fft.fft(wl.to_math(_np(small)), axis=2)
    np.testing.assert_allclose(oh[:, :, 1:], np.conj(oh[:, :, :0:-1]), atol=1e-12)


@pytest.mark.parametrize("precision,dtype,tol", [("fp64", "float64", 1e-12), ("fp32", "float32", 1e-5)])
def test_restoration_with_device_gaussian(precision, dtype, tol):
    import torch
    from paper_2110_02485_amd import rtsvd as rt
    w = wl.WORKLOADS["blur64"]
    A, X, B, _, delta = blur_problem(w.size, w.n, w.sigma, w.band, 1, w.noise, w.k_max, w.oversample)
    seed = 0x5EED0211002485
    r = w.k_max + w.oversample
    print(f"[seeded restore] {precision} r={r}", flush=True)
    om = ga.gaussian_tensor(seed, w.size, r, w.n)
    orc = so.rtsvd_restore(wl.to_math(A), wl.to_math(B), om, delta, w.eta, w.k_max, 0)
    f = rt.factor(_t(A, dtype), w.k_max, w.oversample, 0, precision, None, seed=seed)
    res = f.solve(_t(B, dtype), delta, w.eta)
    torch.cuda.synchronize()
    assert int(res.k[0]) == orc["k"]
    assert _rel(_np(res.X), wl.to_storage(orc["X"])) <= tol
    # and the same factor as the one given the tensor explicitly (FP64: bit for bit)
    f2 = rt.factor(_t(A, dtype), w.k_max, w.oversample, 0, precision, rt.gaussian(seed, w.size, r, w.n,
                                                                                   getattr(torch, dtype)))
    res2 = f2.solve(_t(B, dtype), delta, w.eta)
    torch.cuda.synchronize()
    assert torch.equal(res.X, res2.X)


def test_rank_deficient_sketch():
    # exact tubal rank t = 6 < r = 10: A = P * R; the sketch's columns beyond t break down
    import torch
    from paper_2110_02485_amd import rtsvd as rt
    l = m = 24
    n, t_rank, rho = 8, 6, 4
    rng = np.random.default_rng(21)
    P = rng.standard_normal((l, t_rank, n))
    R = rng.standard_normal((t_rank, m, n))
    a = tp.tprod(P, R)
    x = rng.standard_normal((m, 1, n))
    b = tp.tprod(a, x) + 1e-3 * rng.standard_normal((l, 1, n))
    om = rng.standard_normal((m, t_rank + rho, n))
    print("[rank-deficient] l=m=24 n=8 t=6 r=10", flush=True)
    orc = so.rtsvd_restore(a, b, om, 1e-30, 1.01, t_rank, 0)
    f = rt.factor(_t(wl.to_storage(a)), t_rank, rho, 0, "fp64", _t(wl.to_storage(om)))
    res = f.solve(_t(wl.to_storage(b)), 1e-30, 1.01)
    torch.cuda.synchronize()
    info = f.info(with_status=True)
    assert info[5] & 1 and info[6] == rt.W_RANK_DEFICIENT
    assert int(res.k[0]) == orc["k"] == t_rank and int(res.status[0]) == rt.W_DP_NOT_MET
    assert _rel(_np(res.X), wl.to_storage(orc["X"])) <= 1e-10
    # the leading t singular values per face are those of A (the others are zero)
    sig = info[4]
    ah = tp.fft_tubes(a)
    for i in range(n // 2 + 1):
        sv = np.linalg.svd(ah[:, :, i], compute_uv=False)
        np.testing.assert_allclose(sig[i, :t_rank], sv[:t_rank], rtol=1e-10)


@pytest.mark.parametrize("precision,dtype,tol", [("fp64", "float64", 1e-11), ("fp32", "float32", 1e-5)])
def test_zero_fourier_face(precision, dtype, tol):
    # A^(t) = c_t T with sum_t c_t = 0: face 0 of A is zero (up to rounding)
    import torch
    from paper_2110_02485_amd import rtsvd as rt
    size, n, k_max, rho = 48, 16, 10, 6
    T = wl.blur_toeplitz(size, 2.0, 5)
    c = np.random.default_rng(11).random(n) + 0.5
    c -= c.mean()
    a = T[:, :, None] * c[None, None, :]
    rng = np.random.default_rng(4)
    x = rng.standard_normal((size, 2, n))
    b = tp.tprod(a, x) + 1e-3 * rng.standard_normal((size, 2, n))
    om = rng.standard_normal((size, k_max + rho, n))
    print(f"[zero face] {precision}", flush=True)
    orc = so.rtsvd_restore(a, b, om, 1e-30, 1.01, k_max, 0)
    f = rt.factor(_t(wl.to_storage(a), dtype), k_max, rho, 0, precision, _t(wl.to_storage(om), dtype))
    res = f.solve(_t(wl.to_storage(b), dtype), 1e-30, 1.01)
    torch.cuda.synchronize()
    X = _np(res.X)
    assert np.isfinite(X).all()
    assert int(res.k[0]) == orc["k"]
    assert _rel(X, wl.to_storage(orc["X"])) <= tol
    xh0 = np.fft.fft(wl.to_math(X), axis=2)[:, :, 0]
    assert np.abs(xh0).max() <= 1e-6 * np.abs(X).max()


def test_nonfinite_input_is_reported():
    import torch
    from paper_2110_02485_amd import rtsvd as rt
    w = wl.WORKLOADS["blur64"]
    A, X, B, Om, delta = blur_problem(w.size, w.n, w.sigma, w.band, 1, w.noise, w.k_max, w.oversample)
    print("[non-finite] NaN in A, then inf in B", flush=True)
    Abad = A.copy()
    Abad[3, 5, 7] = np.nan
    f = rt.factor(_t(Abad), w.k_max, w.oversample, 0, "fp64", _t(Om))
    res = f.solve(_t(B), delta, w.eta)
    torch.cuda.synchronize()
    info = f.info(with_status=True)
    assert info[6] == rt.E_NOTFINITE and info[5] & 2
    assert int(res.status[0]) == rt.E_NOTFINITE
    f.close()
    # a finite factor and a non-finite B
    f = rt.factor(_t(A), w.k_max, w.oversample, 0, "fp64", _t(Om))
    Bbad = B.copy()
    Bbad[2, 0, 1] = np.inf
    res = f.solve(_t(Bbad), delta, w.eta)
    torch.cuda.synchronize()
    assert f.info(with_status=True)[6] == rt.OK
    assert int(res.status[0]) == rt.E_NOTFINITE
    assert 1 <= int(res.k[0]) <= w.k_max
    # the same factor still solves a finite B correctly afterwards
    res = f.solve(_t(B), delta, w.eta)
    orc = so.rtsvd_restore(wl.to_math(A), wl.to_math(B), wl.to_math(Om), delta, w.eta, w.k_max, 0)
    torch.cuda.synchronize()
    assert int(res.status[0]) == orc["status"] and _rel(_np(res.X), wl.to_storage(orc["X"])) <= 1e-12


def test_r_eps_starts_at_one_and_k_start_bound():
    # eps^2 above ||A||_F^2: Alg. 6 stops after its first column, r_eps = 1 (not 0); a solve on the
    # adaptive factor (r = 1 < k_max) rejects k_start > r in the library itself
    import ctypes
    import torch
    from paper_2110_02485_amd import rtsvd as rt
    w = wl.WORKLOADS["blur64"]
    A, X, B, Om, delta = blur_problem(w.size, w.n, w.sigma, w.band, 1, w.noise, w.k_max, w.oversample)
    eps = 10.0 * float(np.linalg.norm(A))
    f = rt.factor(_t(A), w.k_max, w.oversample, 0, "fp64", _t(Om), eps=eps)
    assert f.info()[3] == 1
    fa_ = rt.factor(_t(A), w.k_max, w.oversample, 0, "fp64", _t(Om), eps=eps, adaptive=True)
    assert fa_.r == 1
    lib = rt.load()
    Bt = _t(B)
    Xo = torch.empty((w.n, 1, w.size), dtype=torch.float64, device="cuda")
    k = torch.empty(1, dtype=torch.int32, device="cuda")
    arr = (ctypes.c_double * 1)(delta)
    rc = lib.rtsvd_solve(fa_._h, Bt.data_ptr(), 1, rt.F64, arr, 1, w.eta, 2, Xo.data_ptr(), k.data_ptr(), None,
                         None, rt._stream())
    assert rc == rt.E_ARG
    rc = lib.rtsvd_solve(fa_._h, Bt.data_ptr(), 1, rt.F64, arr, 1, w.eta, 1, Xo.data_ptr(), k.data_ptr(), None,
                         None, rt._stream())
    torch.cuda.synchronize()
    assert rc in (rt.OK, rt.W_DP_NOT_MET) and int(k[0]) == 1
