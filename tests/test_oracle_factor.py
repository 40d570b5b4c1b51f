"""Pins of the oracle's factorizations and solvers (Sections 2, 4.1, 4.2; Algs. 1, 3, 6; Thms 2.1, 4.1, 4.2)."""
import numpy as np
import pytest

from oracle import tproduct as tp
from oracle import factor as fa
from oracle import solve as so
from paper_2110_02485_amd import workloads as wl


def _rand(shape, seed):
    return np.random.default_rng(seed).standard_normal(shape)


def _low_tubal_rank(l, m, n, t, seed):
    return tp.tprod(_rand((l, t, n), seed), _rand((t, m, n), seed + 1))


def test_normalize_unit_faces_and_factorization():
    x = _rand((6, 1, 8), 1)
    v, a = fa.normalize(x, 1e-12)
    vh = tp.fft_tubes(v)[:, 0, :]
    np.testing.assert_allclose(np.linalg.norm(vh, axis=0), 1.0, atol=1e-13)
    np.testing.assert_allclose(tp.tprod(v, a[None, None, :]), x, atol=1e-12)


def test_normalize_zero_face_fallback():
    # a tube with a zero Fourier face: X = [1, -1] repeated has DFT face 0 equal to zero
    x = np.zeros((4, 1, 4))
    x[:, 0, :] = np.array([1.0, -1.0, 1.0, -1.0]) * np.arange(1, 5)[:, None]
    v, a = fa.normalize(x, 1e-10, np.random.default_rng(0))
    ah = np.fft.fft(a)
    assert abs(ah[0]) == 0.0
    vh = tp.fft_tubes(v)[:, 0, :]
    np.testing.assert_allclose(np.linalg.norm(vh, axis=0), 1.0, atol=1e-13)
    np.testing.assert_allclose(tp.tprod(v, a[None, None, :]), x, atol=1e-12)


def test_tsvd_reconstruction_and_orthogonality():
    a = _rand((5, 4, 6), 2)
    f = fa.tsvd(a)
    U, S, V = tp.ifft_tubes(f["U"]), tp.ifft_tubes(f["S"]), tp.ifft_tubes(f["V"])
    np.testing.assert_allclose(tp.tprod(tp.tprod(U, S), tp.ttranspose(V)), a, atol=1e-12)
    np.testing.assert_allclose(tp.tprod(tp.ttranspose(U), U), tp.identity(4, 6), atol=1e-12)
    np.testing.assert_allclose(tp.tprod(tp.ttranspose(V), V), tp.identity(4, 6), atol=1e-12)


def test_tsvd_truncation_error_thm21():
    # Thm 2.1 (squared reading): ||A - A_k||_F^2 = (1/n) sum_i sum_{j>k} sigma_j^(i)^2
    a = _rand((6, 5, 7), 3)
    f = fa.tsvd(a)
    for k in range(1, 5):
        U = tp.ifft_tubes(f["U"][:, :k]); S = tp.ifft_tubes(f["S"][:k, :k]); V = tp.ifft_tubes(f["V"][:, :k])
        ak = tp.tprod(tp.tprod(U, S), tp.ttranspose(V))
        lhs = tp.fro(a - ak) ** 2
        rhs = np.sum(f["s"][k:] ** 2) / 7
        assert abs(lhs - rhs) <= 1e-11 * tp.fro(a) ** 2
        # optimality against a random tubal-rank-k competitor X * Y
        comp = tp.tprod(_rand((6, k, 7), 10 + k), _rand((k, 5, 7), 20 + k))
        assert tp.fro(a - ak) <= tp.fro(a - comp)


def test_literal_alg6_equals_block_form():
    a = _rand((7, 5, 6), 4)
    om = _rand((5, 4, 6), 5)
    lit = fa.rtsvd_literal(a, om, r_fixed=4)
    blk = fa.rtsvd_block(a, om)
    np.testing.assert_allclose(lit["Q"], tp.ifft_tubes(blk["Q"]), atol=1e-11)
    np.testing.assert_allclose(lit["Bt"], tp.ifft_tubes(blk["C"]), atol=1e-11)
    np.testing.assert_allclose(lit["eta"], fa.eta_prefix(a, blk["C"]), atol=1e-11 * tp.fro(a) ** 2)


def test_block_q_orthonormal_and_face_conjugation():
    a = _rand((8, 6, 7), 6)
    om = _rand((6, 3, 7), 7)
    blk = fa.rtsvd_block(a, om, power_iters=1)
    n = 7
    ah, oh = tp.fft_tubes(a), tp.fft_tubes(om)
    for i in range(n):
        np.testing.assert_allclose(blk["Q"][:, :, i].conj().T @ blk["Q"][:, :, i], np.eye(3), atol=1e-12)
        # the mirrored face n - i equals the face computed directly (the Q factor is unique)
        q, _ = fa.qr_positive(ah[:, :, i] @ oh[:, :, i])
        qz, _ = fa.qr_positive(ah[:, :, i].conj().T @ q)
        q, _ = fa.qr_positive(ah[:, :, i] @ qz)
        np.testing.assert_allclose(blk["Q"][:, :, i], q, atol=1e-12)


@pytest.mark.parametrize("power_iters", [0, 1])
def test_thm41_thm42_error_indicator(power_iters):
    a = _rand((9, 6, 5), 8)
    blk = fa.rtsvd_block(a, _rand((6, 4, 5), 9), power_iters)
    Q, Bt = tp.ifft_tubes(blk["Q"]), tp.ifft_tubes(blk["C"])
    np.testing.assert_allclose(Bt, tp.tprod(tp.ttranspose(Q), a), atol=1e-12)
    lhs = tp.fro(a - tp.tprod(Q, Bt)) ** 2
    assert abs(lhs - (tp.fro(a) ** 2 - tp.fro(Bt) ** 2)) <= 1e-11 * tp.fro(a) ** 2
    assert abs(lhs - fa.eta_prefix(a, blk["C"])[-1]) <= 1e-11 * tp.fro(a) ** 2


def test_fixed_precision_stopping():
    # Alg. 6 stops at the first r with eta^[r] < eps^2; eta decreases monotonically
    a = _low_tubal_rank(8, 6, 5, 3, 10) + 1e-3 * _rand((8, 6, 5), 12)
    lit = fa.rtsvd_literal(a, _rand((6, 6, 5), 13), eps=0.05)
    eta = lit["eta"]
    assert all(eta[i + 1] <= eta[i] + 1e-12 for i in range(len(eta) - 1))
    assert eta[-1] < 0.05 ** 2 and eta[-2] >= 0.05 ** 2


@pytest.mark.parametrize("power_iters", [0, 1])
def test_block_factor_is_nested(power_iters):
    # The fixed-precision factor keeps the first r' sketch columns of an r-column block factor.
    # QR is nested (column j of Q depends on columns <= j of its argument) and the power step
    # maps column j to column j, so those columns are the block factor built from the first r'
    # Gaussian columns; with q = 0 that is Alg. 6 stopped after r' columns.
    a = _rand((9, 7, 6), 21)
    om = _rand((7, 6, 6), 22)
    full = fa.rtsvd_block(a, om, power_iters)
    for rp in (1, 3, 5):
        part = fa.rtsvd_block(a, om[:, :rp, :], power_iters)
        np.testing.assert_allclose(full["Q"][:, :rp, :], part["Q"], atol=1e-11)
        np.testing.assert_allclose(full["C"][:rp, :, :], part["C"], atol=1e-11)
        np.testing.assert_allclose(fa.eta_prefix(a, full["C"])[:rp + 1], fa.eta_prefix(a, part["C"]),
                                   atol=1e-11 * tp.fro(a) ** 2)
    if power_iters == 0:
        eps = np.sqrt(fa.eta_prefix(a, full["C"])[3] * 1.0001)   # eta^[3] < eps^2 <= eta^[2]
        lit = fa.rtsvd_literal(a, om, eps=eps)
        assert lit["Q"].shape[1] == 3


def test_exact_low_tubal_rank_recovery():
    a = _low_tubal_rank(10, 8, 6, 3, 14)
    om = _rand((8, 5, 6), 16)
    blk = fa.rtsvd_block(a, om)
    Q, Bt = tp.ifft_tubes(blk["Q"]), tp.ifft_tubes(blk["C"])
    assert tp.fro(a - tp.tprod(Q, Bt)) <= 1e-12 * tp.fro(a)
    b = _rand((10, 2, 6), 17)
    ts = fa.tsvd(a)
    Tr = so.coefficients_rtsvd(blk, b)
    Tt = so.coefficients_tsvd(ts, b)
    for k in (1, 2, 3):
        np.testing.assert_allclose(so.x_of_k(blk["V"], Tr, k), so.x_of_k(ts["V"], Tt, k), atol=1e-10)


def test_full_sketch_equals_tsvd():
    a = _rand((7, 5, 4), 18)
    blk = fa.rtsvd_block(a, _rand((5, 5, 4), 19))
    ts = fa.tsvd(a)
    np.testing.assert_allclose(blk["s"], ts["s"], atol=1e-12)
    b = _rand((7, 1, 4), 20)
    Tr, Tt = so.coefficients_rtsvd(blk, b), so.coefficients_tsvd(ts, b)
    for k in range(1, 6):
        np.testing.assert_allclose(so.x_of_k(blk["V"], Tr, k), so.x_of_k(ts["V"], Tt, k), atol=1e-10)


def test_blur_closed_form_tsvd():
    # A^(t) = c_t T  =>  A-hat_i = c-hat_i T: singular values |c-hat_i| |lambda_j(T)| and a
    # closed-form truncated solution from one symmetric eigendecomposition of T.
    size, n, k = 16, 6, 5
    A = wl.to_math(wl.blur_operator(size, n, 2.0, 4))
    T = wl.blur_toeplitz(size, 2.0, 4)
    c = wl.tube_weights(n)
    lam, vec = np.linalg.eigh(T)
    order = np.argsort(-np.abs(lam), kind="stable")
    lam, vec = lam[order], vec[:, order]
    assert abs(abs(lam[k - 1]) - abs(lam[k])) > 1e-3  # well-separated truncation point
    ch = np.fft.fft(c)
    ts = fa.tsvd(A)
    for i in range(n):
        np.testing.assert_allclose(ts["s"][:, i], np.abs(ch[i]) * np.abs(lam), rtol=1e-11, atol=1e-14)
    b = _rand((size, 1, n), 21)
    bh = tp.fft_tubes(b)
    xh = np.empty((size, 1, n), dtype=complex)
    for i in range(n):
        xh[:, 0, i] = vec[:, :k] @ ((vec[:, :k].T @ bh[:, 0, i]) / (ch[i] * lam[:k]))
    x_closed = tp.ifft_tubes(xh)
    x_orc = so.x_of_k(ts["V"], so.coefficients_tsvd(ts, b), k)
    np.testing.assert_allclose(x_orc, x_closed, atol=1e-10 * np.abs(x_closed).max())


def test_tsvd_residual_closed_form_and_dp_index():
    # For T-tSVD, A X_k = U_k U_k^T B, so ||B - A X_k||^2 = ||B||^2 - ||U_k^T B||^2 (non-increasing)
    a = _rand((8, 6, 5), 22)
    b = _rand((8, 1, 5), 23)
    ts = fa.tsvd(a)
    T = so.coefficients_tsvd(ts, b)
    prev = np.inf
    res = []
    for k in range(1, 7):
        xk = so.x_of_k(ts["V"], T, k)
        lit = so.residual(ts["ah"], b, xk)
        Uk = tp.ifft_tubes(ts["U"][:, :k])
        closed = np.sqrt(max(tp.fro(b) ** 2 - tp.fro(tp.tprod(tp.ttranspose(Uk), b)) ** 2, 0.0))
        assert abs(lit - closed) <= 1e-10 * tp.fro(b)
        assert lit <= prev + 1e-12
        prev = lit
        res.append(lit)
    # the DP index is the first k at or below the bound
    delta, eta = res[3] / 1.05, 1.05
    k, _, _, st = so.discrepancy(ts["ah"], b, ts["V"], T, delta, eta, 1, 6)
    assert st == so.OK and k == next(i + 1 for i, r in enumerate(res) if r <= eta * delta)
    k, _, _, st = so.discrepancy(ts["ah"], b, ts["V"], T, 1e-9, eta, 1, 6)
    assert st == so.DP_NOT_MET and k == 6


def test_dp_k_start_and_per_slice():
    a = _rand((8, 6, 5), 24)
    b = _rand((8, 3, 5), 25)
    ts = fa.tsvd(a)
    T = so.coefficients_tsvd(ts, b)
    k, X, res, st = so.discrepancy(ts["ah"], b, ts["V"], T, 1e9, 1.01, 3, 6)
    assert k == 3  # never below k_start
    ks, X, res, st = so.discrepancy(ts["ah"], b, ts["V"], T, [1e9, 1e-12, 1e9], 1.01, 1, 6, per_slice=True)
    assert ks == [1, 6, 1] and st == so.DP_NOT_MET
    for j, kj in enumerate(ks):
        np.testing.assert_allclose(X[:, j:j + 1], so.x_of_k(ts["V"], T[:, j:j + 1], kj), atol=1e-13)


def test_expected_error_bound_statistical():
    # E||A - Q Q^T A||^2 <= (1 + k/(rho - 1)) (1/n) sum_i sum_{j>k} sigma_j^2 (bound of the matrix
    # case, face by face); mean over seeds must respect it.
    l, m, n, k, rho = 12, 10, 4, 3, 3
    rng = np.random.default_rng(26)
    a = _rand((l, m, n), 27)
    ts = fa.tsvd(a)
    tail = np.sum(ts["s"][k:] ** 2) / n
    errs = []
    for s in range(30):
        blk = fa.rtsvd_block(a, rng.standard_normal((m, k + rho, n)))
        errs.append(fa.eta_prefix(a, blk["C"])[-1])
    assert np.mean(errs) <= (1 + k / (rho - 1)) * tail
    # Eckart-Young (Thm 2.1): no sketch of r = k + rho columns beats the best tubal rank-r error
    tail_r = np.sum(ts["s"][k + rho:] ** 2) / n
    assert min(errs) >= tail_r * (1 - 1e-10)


@pytest.mark.parametrize("power_iters", [0, 1])
def test_per_face_factor_and_solution_match_the_block_form(power_iters):
    # rtsvd_face on a face from dft_face (the DFT by definition) reproduces rtsvd_block's face,
    # and solution_face reproduces that face of the truncated solution
    from oracle import solve as so
    rng = np.random.default_rng(81)
    a = rng.standard_normal((9, 7, 6))
    om = rng.standard_normal((7, 5, 6))
    b = rng.standard_normal((9, 2, 6))
    f = fa.rtsvd_block(a, om, power_iters)
    T = so.coefficients_rtsvd(f, b)
    for i in (0, 1, 3):
        A_i, O_i = tp.dft_face(a, i), tp.dft_face(om, i)
        np.testing.assert_allclose(A_i, tp.fft_tubes(a)[:, :, i], atol=1e-12)
        if i in (0, 3):
            A_i, O_i = A_i.real, O_i.real
        fc = fa.rtsvd_face(A_i, O_i, power_iters)
        np.testing.assert_allclose(fc["s"], f["s"][:, i], rtol=1e-12)
        np.testing.assert_allclose(np.abs(fc["Q"].conj().T @ f["Q"][:, :, i]), np.eye(5), atol=1e-10)
        for k in (1, 3, 5):
            ref = np.einsum("ij,jk->ik", f["V"][:, :k, i], T[:k, :, i])
            np.testing.assert_allclose(fa.solution_face(fc, tp.dft_face(b, i), k), ref, atol=1e-10)
