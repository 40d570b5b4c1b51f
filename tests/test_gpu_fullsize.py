"""Parity at the full sizes of the benchmark configurations, in the launch configuration the
benchmark times (default face groups), on outputs the FP64 oracle can compute one face at a time
and on properties that hold at any size.

Inputs come from the seeded workload generators and B = A * X_true + E is formed by the oracle's
t-product, so no input or expected value comes from the HIP path.  Checked:
  * sigma of sampled Fourier faces against the oracle's block R-tSVD of that face (same Omega);
  * X-hat of sampled faces at the fixed truncation k = k_max (the search started at k_max) against
    the oracle's per-face truncated solution;
  * the reported residual at the chosen k against the oracle's literal ||B - A * X||_F of the
    returned X;
  * the discrepancy decision: k is the first index with a residual within eta * delta (or k_max
    with every residual above it and the status set).
Tolerances: 1e-5 (FP32) and 2e-3 (BF16 sketch with FP32 accumulation) relative to the oracle.
"""
import numpy as np
import pytest

from oracle import tproduct as tp
from oracle import factor as fa
from paper_2110_02485_amd import workloads as wl

pytestmark = pytest.mark.gpu


def _rel(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def _full_case(name, precision, tol):
    import torch
    from paper_2110_02485_amd import rtsvd as rt
    w = wl.WORKLOADS[name]
    A, X, E0, Om = wl.make_inputs(w)
    Am, Xm, Omm = wl.to_math(A), wl.to_math(X), wl.to_math(Om)
    ah = tp.fft_tubes(Am)
    Bt = tp.tprod_hat(ah, Xm)
    E = wl.scale_noise(wl.to_math(E0), Bt, w.noise)
    Bm = Bt + E
    delta = float(np.linalg.norm(E))
    B = wl.to_storage(Bm)
    dt = torch.float64 if precision == "fp64" else torch.float32
    dev = torch.device("cuda:0")
    At = torch.from_numpy(A).to(dev, dt)
    f = rt.factor(At, w.k_max, w.oversample, w.power_iters, precision, torch.from_numpy(Om).to(dev, dt))
    Bd = torch.from_numpy(B).to(dev, dt)
    res = f.solve(Bd, delta, w.eta, 1)
    fixed = f.solve(Bd, delta, w.eta, w.k_max)          # k = k_max: the search starts there
    torch.cuda.synchronize()
    sig = f.info()[4]
    Xg = wl.to_math(res.X.double().cpu().numpy())
    Xk = wl.to_math(fixed.X.double().cpu().numpy())
    k, status = int(res.k[0]), int(res.status[0])
    resid = res.resid.cpu().numpy()[0]
    f.close()
    F = w.n // 2 + 1
    faces = sorted({0, 1, F // 2, F - 1})
    s_err, x_num, x_den = 0.0, 0.0, 0.0
    for i in faces:
        A_i, O_i = ah[:, :, i], tp.dft_face(Omm, i)
        if i == (w.n - i) % w.n:
            A_i, O_i = A_i.real, O_i.real
        fc = fa.rtsvd_face(A_i, O_i, w.power_iters)
        s_err = max(s_err, float(np.max(np.abs(sig[i, :w.k_max] - fc["s"][:w.k_max]) / fc["s"][:w.k_max])))
        xo = fa.solution_face(fc, tp.dft_face(Bm, i), w.k_max)
        xg = tp.dft_face(Xk, i)
        x_num += np.linalg.norm(xg - xo) ** 2
        x_den += np.linalg.norm(xo) ** 2
    x_err = float(np.sqrt(x_num / x_den))
    lit = float(np.linalg.norm(Bm - tp.tprod_hat(ah, Xg)))
    r_err = abs(lit - resid[k - 1]) / lit
    print(f"[{name}] faces {faces}: sigma rel {s_err:.2e}, X-hat rel {x_err:.2e}, residual rel {r_err:.2e}, "
          f"k {k}, status {status}")
    assert s_err <= tol and x_err <= tol and r_err <= tol
    bound = w.eta * delta
    if status == 0:
        assert resid[k - 1] <= bound and np.all(resid[:k - 1] > bound)
    else:
        assert k == w.k_max and np.all(resid[:w.k_max] > bound)


def test_fullsize_blur256_fp32():
    # 256 x 256 x 256 (129 faces), k <= 60, rho = 10, FP32
    _full_case("blur256", "fp32", 1e-5)


def test_fullsize_video512_fp32():
    # 512 x 512 x 64 (33 faces), 64 frames as lateral slices, joint k, FP32
    _full_case("video512", "fp32", 1e-5)


def test_fullsize_blur1024_mixed():
    # the benchmark's restoration: 1024 x 1024 x 128 (65 faces), r = 100 + 20, q = 1, BF16 sketch
    _full_case("blur1024", "mixed", 2e-3)
