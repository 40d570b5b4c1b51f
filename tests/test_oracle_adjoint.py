"""Pins of the oracle's gradients: central finite differences (h = 1e-3 in sigma, directional in B)."""
import numpy as np

from oracle import adjoint as ad
from oracle import factor as fa
from oracle import solve as so
from oracle import tproduct as tp
from paper_2110_02485_amd import workloads as wl


def _setup(size=24, n=8, sigma=2.0, band=6, p=2, k=8, rho=4, seed=0):
    A = wl.to_math(wl.blur_operator(size, n, sigma, band))
    dA = wl.to_math(wl.blur_operator_dsigma(size, n, sigma, band))
    rng = np.random.default_rng(seed)
    X = rng.uniform(0, 1, (size, p, n))
    B = tp.tprod(A, X) + 1e-3 * rng.standard_normal((size, p, n))
    Om = rng.standard_normal((size, k + rho, n))
    return A, dA, B, Om, X, k


def test_fixed_k_forward_matches_rtsvd_solution():
    A, dA, B, Om, X, k = _setup()
    f = fa.rtsvd_block(A, Om)
    T = so.coefficients_rtsvd(f, B)
    np.testing.assert_allclose(ad.restore_fixed_k(A, B, Om, k), so.x_of_k(f["V"], T, k), atol=1e-9)


def test_blur_dsigma_matches_finite_difference_of_operator():
    h = 1e-6
    T0 = wl.blur_toeplitz(20, 2.5, 7)
    dT = wl.blur_toeplitz_dsigma(20, 2.5, 7)
    fd = (wl.blur_toeplitz(20, 2.5 + h, 7) - wl.blur_toeplitz(20, 2.5 - h, 7)) / (2 * h)
    np.testing.assert_allclose(dT, fd, atol=1e-8)
    assert np.abs(T0).max() > 0


def test_dsigma_gradient_vs_central_difference():
    sigma, size, n, band = 2.0, 24, 8, 6
    A, dA, B, Om, Xt, k = _setup(size, n, sigma, band)
    loss, gb, gs = ad.grads(A, dA, B, Om, k, Xt)
    h = 1e-3
    def L(s):
        As = wl.to_math(wl.blur_operator(size, n, s, band))
        x = ad.restore_fixed_k(As, B, Om, k)
        return 0.5 * float(np.sum((x - Xt) ** 2))
    fd = (L(sigma + h) - L(sigma - h)) / (2 * h)
    assert abs(fd - gs) <= 1e-4 * max(abs(fd), 1e-12) + 1e-10, (fd, gs)


def test_dB_gradient_vs_directional_difference():
    A, dA, B, Om, Xt, k = _setup(seed=3)
    loss, gb, gs = ad.grads(A, dA, B, Om, k, Xt)
    D = np.random.default_rng(4).standard_normal(B.shape)
    h = 1e-3
    def L(Bv):
        x = ad.restore_fixed_k(A, Bv, Om, k)
        return 0.5 * float(np.sum((x - Xt) ** 2))
    fd = (L(B + h * D) - L(B - h * D)) / (2 * h)
    assert abs(fd - np.sum(gb * D)) <= 1e-7 * abs(fd) + 1e-12
