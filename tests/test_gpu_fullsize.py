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


def _diff_batch():
    from oracle import adjoint as ad
    w = wl.WORKLOADS["diff512"]
    A, dA, X, E0, Om, off = wl.make_clip_inputs(w)
    Am, Xm = wl.to_math(A), wl.to_math(X)
    Bt = tp.tprod(Am, Xm)
    Bm = Bt.copy()
    for j in range(len(w.problems)):
        sl = slice(off[j], off[j + 1])
        Bm[:, sl, :] += wl.scale_noise(wl.to_math(E0[j]), Bt[:, sl, :], w.noise)
    loss, gb, gs = ad.grads(Am, wl.to_math(dA), Bm, wl.to_math(Om), w.k_max, Xm)
    return w, A, dA, X, wl.to_storage(Bm), Om, off, (loss, wl.to_storage(gb), gs)


def test_fullsize_diff512_adjoint_fp32():
    # 512 x 512 x 64 (33 faces), 16 clips of 4 to 32 frames (260 lateral slices) in one batched
    # FP32 restoration at the fixed k = 80 (rho = 10); the backward pass recomputes the factor.
    # Against the FP64 oracle gradient over every element: L, dL/dB, dL/dsigma.  Then, from the
    # GPU path alone: each clip's dL/dB from a call with that clip by itself equals its part of the
    # batched one (slices are independent), and dL/dsigma matches a central difference with
    # h = 1e-3 of the GPU forward.
    import torch
    from paper_2110_02485_amd import autograd as ag
    w, A, dA, X, B, Om, off, (loss, gb, gs) = _diff_batch()
    dev = torch.device("cuda:0")
    f32 = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(dev, torch.float32)
    At, dAt, Omt, Xt = f32(A), f32(dA), f32(Om), f32(X).double()

    def run(sl, sigma=w.sigma, Aop=At, grad=True):
        Bg = f32(B[:, sl, :]).requires_grad_(grad)
        s = torch.tensor(sigma, dtype=torch.float32, device=dev, requires_grad=grad)
        Xg = ag.restore(Bg, s, Aop, dAt if grad else None, Omt, w.k_max, w.oversample)
        L = 0.5 * ((Xg.double() - Xt[:, sl, :]) ** 2).sum()
        if grad:
            L.backward()
        torch.cuda.synchronize()
        return float(L.detach()), (Bg.grad.double().cpu().numpy() if grad else None), (float(s.grad) if grad else None)

    L, gB, gS = run(slice(None))
    l_err, b_err, s_err = abs(L - loss) / loss, _rel(gB, gb), abs(gS - gs) / abs(gs)
    print(f"[diff512] {off[-1]} slices: L rel {l_err:.2e}, dL/dB rel {b_err:.2e}, dL/dsigma rel {s_err:.2e} "
          f"({gS:.6e} vs {gs:.6e})")
    c_errs = []
    for j in (0, 1):                                 # the shortest (4 frames) and longest (32) clip
        sl = slice(off[j], off[j + 1])
        _, gBj, _ = run(sl)
        c_err = _rel(gBj, gB[:, sl, :])
        print(f"[diff512] clip {j} ({off[j + 1] - off[j]} frames) alone vs batched: dL/dB rel {c_err:.2e}")
        c_errs.append(c_err)
    h = 1e-3
    Lp = run(slice(None), w.sigma + h, f32(wl.blur_operator(w.size, w.n, w.sigma + h, w.band)), False)[0]
    Lm = run(slice(None), w.sigma - h, f32(wl.blur_operator(w.size, w.n, w.sigma - h, w.band)), False)[0]
    fd = (Lp - Lm) / (2 * h)
    fd_err = abs(fd - gS) / abs(gS)
    print(f"[diff512] central difference h = {h}: {fd:.6e}, rel {fd_err:.2e}")
    assert l_err <= 1e-5 and b_err <= 1e-5 and s_err <= 1e-5
    assert max(c_errs) <= 1e-6
    assert fd_err <= 1e-3
