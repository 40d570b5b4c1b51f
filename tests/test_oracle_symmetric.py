"""Pins of the oracle's methods for a symmetric tensor (Section 3: Alg. 2, Alg. 4, eqs. (9t), (10))."""
import numpy as np
import pytest

from oracle import tproduct as tp
from oracle import symmetric as sy
from oracle import solve as so
from paper_2110_02485_amd import workloads as wl


def _sym(m, n, seed, shift=0.0):
    """A random t-symmetric tensor S + S^T (every DFT face Hermitian), optionally + shift * I."""
    s = np.random.default_rng(seed).standard_normal((m, m, n))
    a = s + tp.ttranspose(s)
    a[:, :, 0] += shift * np.eye(m)
    return a


def test_symmetric_tensor_has_hermitian_faces():
    a = _sym(5, 6, 1)
    np.testing.assert_allclose(tp.ttranspose(a), a)
    ah = tp.fft_tubes(a)
    for f in range(6):
        np.testing.assert_allclose(ah[:, :, f], ah[:, :, f].conj().T, atol=1e-12)


def test_tevd_reconstruction_orthogonality_and_eigen_relation():
    # A = W * D * W^T, W^T * W = I, A * W_j = W_j * d_j (eq. (3)); |d| descending per face (Alg. 2)
    a = _sym(6, 5, 2)
    f = sy.tevd(a)
    W, D = sy.spatial_tevd(f)
    assert np.abs(W.imag).max() < 1e-12 and np.abs(D.imag).max() < 1e-12
    W, D = W.real, D.real
    np.testing.assert_allclose(tp.tprod(tp.tprod(W, D), tp.ttranspose(W)), a, atol=1e-11)
    np.testing.assert_allclose(tp.tprod(tp.ttranspose(W), W), tp.identity(6, 5), atol=1e-12)
    for j in range(6):
        wj = W[:, j:j + 1, :]
        np.testing.assert_allclose(tp.tprod(a, wj), tp.tprod(wj, D[j:j + 1, j:j + 1, :]), atol=1e-11)
    assert np.all(np.diff(np.abs(f["d"]), axis=0) <= 1e-12)


def test_tevd_closed_form_for_symmetric_blur():
    # A^(t) = c_t T with a circularly symmetric tube: face i is c-hat_i T (real), so its eigenvalues
    # are c-hat_i lambda_j(T), ordered by |lambda_j(T)|
    A = wl.blur_operator(12, 8, 2.0, 4, symmetric=True)
    a = wl.to_math(A)
    T = wl.blur_toeplitz(12, 2.0, 4)
    lamT = np.linalg.eigvalsh(T)
    chat = np.fft.fft(wl.tube_weights(8, symmetric=True))
    assert np.abs(chat.imag).max() < 1e-14
    f = sy.tevd(a)
    for i in range(8):
        ref = chat.real[i] * lamT
        ref = ref[np.argsort(-np.abs(ref), kind="stable")]
        np.testing.assert_allclose(f["d"][:, i], ref, atol=1e-12)


@pytest.mark.parametrize("per_slice", [False, True])
def test_tevd_restore_equals_tsvd_restore_for_symmetric_a(per_slice):
    # on Hermitian faces the singular values are |eigenvalues| with left vectors W sign(d): the
    # truncated solutions and the discrepancy indices of T-tEVD and T-tSVD coincide
    a = _sym(7, 6, 3)
    b = np.random.default_rng(4).standard_normal((7, 2, 6))
    delta = [0.6 * np.linalg.norm(b[:, j]) for j in range(2)] if per_slice else 0.5 * np.linalg.norm(b)
    e = sy.tevd_restore(a, b, delta, 1.01, 7, per_slice=per_slice)
    s = so.tsvd_restore(a, b, delta, 1.01, 7, per_slice=per_slice)
    assert e["k"] == s["k"]
    np.testing.assert_allclose(e["X"], s["X"], atol=1e-10)
    np.testing.assert_allclose(e["res"], s["res"], rtol=1e-10, atol=1e-12 * np.linalg.norm(b))


def _singular_face_sym(m, n, seed, c0):
    """A^(t) = c_t T with T random symmetric and the symmetric tube c = (1/2, -1/4, 0, ..., 0, -1/4)
    + c0 / n: face f is c-hat_f T with c-hat_f = (1 - cos(2 pi f / n)) / 2 + c0, so face 0 is
    c0 T (exactly zero for c0 = 0) and the others are well conditioned."""
    rng = np.random.default_rng(seed)
    t = rng.standard_normal((m, m))
    t = t + t.T
    c = np.zeros(n)
    c[0], c[1], c[-1] = 0.5, -0.25, -0.25
    c = c + c0 / n
    return c[None, None, :] * t[:, :, None]


@pytest.mark.parametrize("c0", [0.0, 1e-13])
def test_tevd_singular_face_matches_tsvd_and_drops_the_face(c0):
    # a symmetric A with a zero (or numerically zero) Fourier face: T-tEVD reads diag(d)^{-1} as the
    # pseudo-inverse with the truncated SVD's tolerance, so it equals T-tSVD and the face
    # contributes nothing; without the cutoff face 0 would carry 1/c0 or 1/0
    m, n = 6, 8
    a = _singular_face_sym(m, n, 31, c0)
    assert np.abs(tp.fft_tubes(a)[:, :, 0]).max() <= max(c0, 1e-15) * 100 * np.abs(a).max() * n
    b = np.random.default_rng(32).standard_normal((m, 2, n))
    delta = 1e-3 * np.linalg.norm(b)
    e = sy.tevd_restore(a, b, delta, 1.01, m)
    s = so.tsvd_restore(a, b, delta, 1.01, m)
    assert e["k"] == s["k"]
    np.testing.assert_allclose(e["X"], s["X"], atol=1e-9 * np.abs(s["X"]).max())
    np.testing.assert_allclose(e["res"], s["res"], rtol=1e-9, atol=1e-12 * np.linalg.norm(b))
    xh = tp.fft_tubes(e["X"])
    assert np.abs(xh[:, :, 0]).max() <= 1e-13 * np.abs(xh).max()   # zero up to the DFT round trip
    # every other face: the per-face solution of the full-rank Hermitian system truncated at k
    f = sy.tevd(a)
    bh = tp.fft_tubes(b)
    k = e["k"]
    for i in range(1, n):
        W, d = f["W"][:, :k, i], f["d"][:k, i]
        np.testing.assert_allclose(xh[:, :, i], W @ ((W.conj().T @ bh[:, :, i]) / d[:, None]),
                                   atol=1e-9 * np.abs(xh).max())


def test_tlanczos_literal_equals_facewise():
    a = _sym(6, 5, 5)
    b = np.random.default_rng(6).standard_normal((6, 1, 5))
    Q, c, z = sy.tlanczos_literal(a, b, 3)
    Qh, ch, zh = sy.tlanczos_faces(tp.fft_tubes(a), tp.fft_tubes(b)[:, 0, :], 3)
    np.testing.assert_allclose(tp.fft_tubes(Q), Qh, atol=1e-11)
    np.testing.assert_allclose(np.fft.fft(c, axis=1), ch, atol=1e-11)
    np.testing.assert_allclose(np.fft.fft(z, axis=1), zh, atol=1e-11)


def test_tlanczos_decomposition():
    # A * Q_k = Q_{k+1} * T-bar_k (eq. (t-lanczos)), orthonormal columns, Q_k^T * A * Q_k = T_k
    # (eq. (slanc)), Q_{k+1}^T * B = e_1 z_0 (eq. (fra))
    a = _sym(9, 5, 7)
    b = np.random.default_rng(8).standard_normal((9, 1, 5))
    ah, bh = tp.fft_tubes(a), tp.fft_tubes(b)[:, 0, :]
    k = 4
    Q, c, z = sy.tlanczos_faces(ah, bh, k)
    for f in range(5):
        T = sy.tridiag(c, z, k, f)
        np.testing.assert_allclose(ah[:, :, f] @ Q[:, :k, f], Q[:, :, f] @ T, atol=1e-10)
        np.testing.assert_allclose(Q[:, :, f].conj().T @ Q[:, :, f], np.eye(k + 1), atol=1e-12)
        np.testing.assert_allclose(Q[:, :k, f].conj().T @ ah[:, :, f] @ Q[:, :k, f], T[:k, :], atol=1e-10)
        e1z = np.zeros(k + 1)
        e1z[0] = z[0, f]
        np.testing.assert_allclose(Q[:, :, f].conj().T @ bh[:, f], e1z, atol=1e-10)


@pytest.mark.parametrize("k", [1, 2, 4])
def test_tlanczos_solution_is_krylov_least_squares_minimizer(k):
    # per face X_k-hat minimizes ||b - A x|| over K_k(A, b) (explicit power basis + lstsq)
    a = _sym(8, 4, 9)
    b = np.random.default_rng(10).standard_normal((8, 1, 4))
    ah, bh = tp.fft_tubes(a), tp.fft_tubes(b)[:, 0, :]
    Q, c, z = sy.tlanczos_faces(ah, bh, k)
    xh = sy.tlanczos_solution(Q, c, z, k)
    for f in range(4):
        A = ah[:, :, f]
        K = [bh[:, f]]
        for _ in range(k - 1):
            K.append(A @ K[-1])
        basis, _ = np.linalg.qr(np.stack(K, axis=1))
        y, *_ = np.linalg.lstsq(A @ basis, bh[:, f], rcond=None)
        np.testing.assert_allclose(xh[:, 0, f], basis @ y, atol=1e-9 * np.linalg.norm(basis @ y))


def test_tlanczos_full_steps_and_ritz_form_give_exact_solution():
    # k = m: T_m is the whole face in the Lanczos basis; eq. (9t) and the Ritz form eq. (10) both
    # give A^{-1} B, and the Ritz values are the eigenvalues of the faces
    a = _sym(5, 4, 11, shift=8.0)
    x_true = np.random.default_rng(12).standard_normal((5, 1, 4))
    b = tp.tprod(a, x_true)
    ah, bh = tp.fft_tubes(a), tp.fft_tubes(b)[:, 0, :]
    Q, c, z = sy.tlanczos_faces(ah, bh, 5)
    np.testing.assert_allclose(tp.ifft_tubes(sy.tlanczos_solution(Q, c, z, 5)), x_true, atol=1e-9)
    np.testing.assert_allclose(tp.ifft_tubes(sy.ritz_solution(Q, c, z, 5)), x_true, atol=1e-9)
    for f in range(4):
        np.testing.assert_allclose(np.linalg.eigvalsh(sy.tridiag(c, z, 5, f)[:5, :]),
                                   np.linalg.eigvalsh(ah[:, :, f]), atol=1e-9)


def test_tlanczos_restore_dp_and_literal_residual():
    # the first k meeting the principle per slice; a bound never met takes k_max with the status
    a = _sym(10, 6, 13, shift=3.0)
    b = np.random.default_rng(14).standard_normal((10, 2, 6))
    out = sy.tlanczos_restore(a, b, [1e3, 1e-12], 1.01, 4)
    assert out["k"] == [1, 4] and out["status"] == sy.DP_NOT_MET
    # residual of the chosen solution recomputed with the spatial t-product
    x1 = out["X"][:, 1:2, :]
    assert abs(tp.fro(b[:, 1:2] - tp.tprod(a, x1)) - out["res"][3, 1]) <= 1e-10 * out["res"][3, 1]
