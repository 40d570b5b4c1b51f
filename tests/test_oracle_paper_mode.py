"""Pins of the experiments' truncation rule (eq. (kinit): start at k_init = r - rho and increase k up
to r, Section 5), of the spatial-domain R-tSVD factor (Alg. 6, final step: U-tilde = Q * U-breve),
and of the pseudo-inverse on a zero Fourier face, each against quantities computed independently of
the function under test."""
import numpy as np
import pytest

from oracle import factor as fa
from oracle import solve as so
from oracle import tproduct as tp
from paper_2110_02485_amd import workloads as wl

from problems import blur_problem


def _spatial_solutions(a, b, omega, q=0):
    """X_k for k = 1..r by spatial t-products of the spatial factor (X_k = V_k * S_k^{-1} * U_k^T * B,
    Section 4.2), and their literal residuals ||B - A * X_k||_F."""
    f = fa.rtsvd_block(a, omega, q)
    sf = fa.spatial_factor(f)
    r, n = f["s"].shape
    out = []
    for k in range(1, r + 1):
        # S_k^{-1}: the f-diagonal tensor whose DFT faces are diag(1/s_1..k) (Section 2: the inverse
        # of an f-diagonal tensor is taken face by face in the Fourier domain)
        sinv_h = np.zeros((k, k, n), dtype=complex)
        for j in range(k):
            sinv_h[j, j, :] = 1.0 / f["s"][j, :]
        sinv = tp.ifft_tubes(sinv_h)
        uk, vk = sf["U"][:, :k, :], sf["V"][:, :k, :]
        xk = tp.tprod(vk, tp.tprod(sinv, tp.tprod(tp.ttranspose(uk), b)))
        out.append((xk, tp.fro(b - tp.tprod(a, xk))))
    return out


@pytest.fixture(scope="module")
def small():
    A, X, B, Om, delta = blur_problem(24, 6, 2.0, 5, 1, 1e-2, 10, 4, seed=7)
    return wl.to_math(A), wl.to_math(B), wl.to_math(Om), delta


def _expected_paper_mode(res, tau_delta, r, rho):
    """First k >= max(1, r - rho) with res_k <= tau delta, capped at r (status 1 when none)."""
    k0 = max(1, r - rho)
    for k in range(k0, r + 1):
        if res[k - 1] <= tau_delta:
            return k, 0
    return r, 1


@pytest.mark.parametrize("rho", [4, 9, 14, 20])
def test_paper_mode_k_by_brute_force(small, rho):
    a, b, om, delta = small
    r = om.shape[1]                                # 14 columns; rho >= r clamps r - rho to 1
    sols = _spatial_solutions(a, b, om)
    res = np.array([rs for _, rs in sols])
    # bounds that exercise every branch: met inside the window above k_init, met at or below
    # k_init (so k = k_init, never lower), and never met (k = r, status 1)
    k_init = max(1, r - rho)
    inside = [k for k in range(k_init + 1, r + 1) if res[k - 1] < res[k - 2]]
    bounds = [1.0001 * res[k_init - 1] * 10.0, 0.5 * res[-1]]
    if inside:
        kk = inside[len(inside) // 2]
        bounds.append(0.5 * (res[kk - 1] + min(res[k_init - 1:kk - 1])))
    for tb in bounds:
        eta = 1.01
        dl = tb / eta
        got = so.rtsvd_restore(a, b, om, dl, eta, k_max=r, k_start=0, rho=rho)
        k_exp, st_exp = _expected_paper_mode(res, eta * dl, r, rho)
        assert got["k"] == k_exp and got["status"] == st_exp, (rho, tb, got["k"], k_exp)
        assert k_init <= got["k"] <= r
        np.testing.assert_allclose(got["X"], sols[k_exp - 1][0], atol=1e-10 * np.abs(sols[k_exp - 1][0]).max())


def test_paper_mode_window_edges(small):
    a, b, om, delta = small
    r = om.shape[1]
    sols = _spatial_solutions(a, b, om)
    res = np.array([rs for _, rs in sols])
    rho = 5
    k_init = r - rho
    # a bound met first exactly at k_init + 1 (the start is not moved by one) ...
    if res[k_init] < res[k_init - 1]:
        tb = 0.5 * (res[k_init] + res[k_init - 1])
        got = so.rtsvd_restore(a, b, om, tb / 1.01, 1.01, k_max=r, k_start=0, rho=rho)
        assert got["k"] == k_init + 1
    # ... and one met only at r (the cap is r, not r - 1 or k_max)
    if res[r - 1] < res[r - 2]:
        tb = 0.5 * (res[r - 1] + res[r - 2])
        got = so.rtsvd_restore(a, b, om, tb / 1.01, 1.01, k_max=3, k_start=0, rho=rho)
        assert got["k"] == r and got["status"] == 0


def test_spatial_factor_reconstruction_and_orthogonality(small):
    a, b, om, delta = small
    f = fa.rtsvd_block(a, om, 1)
    sf = fa.spatial_factor(f)
    eta = fa.eta_prefix(a, f["C"])
    # A - U-tilde * S-tilde * V-tilde^T = A - Q * B-tilde, whose squared norm is eta^[r] (Thm 4.2)
    approx = tp.tprod(tp.tprod(sf["U"], sf["S"]), tp.ttranspose(sf["V"]))
    assert tp.fro(a - approx) ** 2 == pytest.approx(eta[-1], rel=1e-9, abs=1e-12 * tp.fro(a) ** 2)
    np.testing.assert_allclose(tp.tprod(sf["Q"], sf["Bt"]), approx, atol=1e-12 * np.abs(a).max())
    # U-tilde^T * U-tilde = I and V-tilde^T * V-tilde = I (identity tensor of Section 2)
    r = f["s"].shape[0]
    eye = tp.identity(r, a.shape[2])
    np.testing.assert_allclose(tp.tprod(tp.ttranspose(sf["U"]), sf["U"]), eye, atol=1e-12)
    np.testing.assert_allclose(tp.tprod(tp.ttranspose(sf["V"]), sf["V"]), eye, atol=1e-12)
    # S-tilde is f-diagonal with the singular values in every Fourier face
    sh = tp.fft_tubes(sf["S"])
    for i in range(a.shape[2]):
        np.testing.assert_allclose(np.diag(sh[:, :, i]).real, f["s"][:, i], atol=1e-12)


def test_zero_fourier_face_restores_by_pseudo_inverse():
    # a tube with c-hat_0 = 0 (zero mean): face 0 of A is zero and must contribute nothing
    size, n = 16, 8
    T = wl.blur_toeplitz(size, 2.0, 5)
    c = np.random.default_rng(11).random(n) + 0.5
    c -= c.mean()                                  # every face nonzero except face 0
    assert abs(c.sum()) < 1e-12 and np.abs(np.fft.fft(c)[1:]).min() > 1e-2
    a = T[:, :, None] * c[None, None, :]
    ah = tp.fft_tubes(a)
    assert np.abs(ah[:, :, 0]).max() < 1e-12
    rng = np.random.default_rng(3)
    x = rng.standard_normal((size, 2, n))
    b = tp.tprod(a, x) + 1e-3 * rng.standard_normal((size, 2, n))
    om = rng.standard_normal((size, 10, n))
    got = so.rtsvd_restore(a, b, om, 1e-30, 1.01, k_max=6)
    assert np.isfinite(got["X"]).all()
    xh = tp.fft_tubes(got["X"])
    assert np.abs(xh[:, :, 0]).max() < 1e-12
    # the other faces are the per-face truncated solutions (face 0 of the pseudo-inverse is 0)
    for i in range(1, n):
        fc = fa.rtsvd_face(ah[:, :, i], tp.fft_tubes(om)[:, :, i])
        np.testing.assert_allclose(xh[:, :, i], fa.solution_face(fc, tp.fft_tubes(b)[:, :, i], 6,
                                                                 so.pinv_cut(got["factor"]["s"])), atol=1e-9)
    # the rule is numpy's pseudo-inverse with an absolute tolerance (rcond relative to the largest
    # singular value): exact zeros and values at or below the cutoff are dropped
    d = np.array([[1.0 + 2j], [3.0 - 1j], [5.0], [7.0]])
    s = np.array([2.0, 0.0, 4.0, 1e-9])
    cut = so.pinv_cut(s[:, None])
    assert cut == pytest.approx(np.sqrt(4 * 4 * np.finfo(float).eps) * 4.0)
    np.testing.assert_allclose(so.pinv_scale(d, s, cut), np.linalg.pinv(np.diag(s), rcond=cut / 4.0 * 1.000001) @ d)
