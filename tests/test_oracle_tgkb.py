"""Pins of the oracle's tGKB process and method (Section 4.3, Algs. 5 and 7)."""
import numpy as np
import pytest

from oracle import tproduct as tp
from oracle import tgkb as tg


def _rand(shape, seed):
    return np.random.default_rng(seed).standard_normal(shape)


def test_literal_equals_facewise():
    a, b = _rand((7, 5, 6), 1), _rand((7, 1, 6), 2)
    k = 3
    W, Q, c, z = tg.tgkb_literal(a, b, k)
    Wh, Qh, ch, zh = tg.tgkb_faces(tp.fft_tubes(a), tp.fft_tubes(b)[:, 0, :], k)
    np.testing.assert_allclose(tp.fft_tubes(W), Wh, atol=1e-11)
    np.testing.assert_allclose(tp.fft_tubes(Q), Qh, atol=1e-11)
    np.testing.assert_allclose(np.fft.fft(c, axis=1).real, ch, atol=1e-11)
    np.testing.assert_allclose(np.fft.fft(z, axis=1).real, zh, atol=1e-11)


def test_decomposition_and_orthonormality():
    # A * W_k = Q_{k+1} * P-bar_k with orthonormal tensor columns (eq. (t-gkb))
    a, b = _rand((9, 6, 5), 3), _rand((9, 1, 5), 4)
    k = 4
    ah = tp.fft_tubes(a)
    W, Q, c, z = tg.tgkb_faces(ah, tp.fft_tubes(b)[:, 0, :], k)
    for f in range(5):
        P = tg.bidiag(c, z, k, f)
        np.testing.assert_allclose(ah[:, :, f] @ W[:, :, f], Q[:, :, f] @ P, atol=1e-11)
        np.testing.assert_allclose(W[:, :, f].conj().T @ W[:, :, f], np.eye(k), atol=1e-12)
        np.testing.assert_allclose(Q[:, :, f].conj().T @ Q[:, :, f], np.eye(k + 1), atol=1e-12)


@pytest.mark.parametrize("k", [1, 2, 4])
def test_solution_is_krylov_least_squares_minimizer(k):
    # per face, X_k-hat minimizes ||b - A x|| over K_k(A^H A, A^H b): explicit Krylov basis + lstsq
    a, b = _rand((8, 6, 4), 5), _rand((8, 1, 4), 6)
    ah, bh = tp.fft_tubes(a), tp.fft_tubes(b)[:, 0, :]
    W, Q, c, z = tg.tgkb_faces(ah, bh, k)
    xh = tg.tgkb_solution(W, c, z, k)
    for f in range(4):
        A = ah[:, :, f]
        v = A.conj().T @ bh[:, f]
        K = [v]
        for _ in range(k - 1):
            K.append(A.conj().T @ (A @ K[-1]))
        basis, _ = np.linalg.qr(np.stack(K, axis=1))
        y, *_ = np.linalg.lstsq(A @ basis, bh[:, f], rcond=None)
        np.testing.assert_allclose(xh[:, 0, f], basis @ y, atol=1e-9 * np.linalg.norm(basis @ y))


def test_full_steps_give_least_squares_solution():
    # k = m steps: the Krylov space is everything, X_m solves the full least-squares problem (Alg. 5)
    a, b = _rand((7, 4, 5), 7), _rand((7, 1, 5), 8)
    ah, bh = tp.fft_tubes(a), tp.fft_tubes(b)[:, 0, :]
    W, Q, c, z = tg.tgkb_faces(ah, bh, 4)
    x = tp.ifft_tubes(tg.tgkb_solution(W, c, z, 4))
    xh_ls = np.stack([np.linalg.lstsq(ah[:, :, f], bh[:, f], rcond=None)[0] for f in range(5)], axis=1)
    np.testing.assert_allclose(x, tp.ifft_tubes(xh_ls[:, None, :]), atol=1e-10)


def test_breakdown_invariant_subspace():
    # B = A * e_1 lies in an invariant subspace: one step already solves it exactly, and further
    # steps (zero tubal scalars on every face) leave the solution unchanged.
    a = _rand((6, 4, 4), 9)
    e1 = np.zeros((4, 1, 4)); e1[0, 0, 0] = 1.0
    q, _ = np.linalg.qr(_rand((6, 6), 10))
    aq = np.zeros((6, 4, 4)); aq[:, :, 0] = q[:, :4]   # orthonormal columns on every face
    b = tp.tprod(aq, e1)
    res = tg.tgkb_restore(aq, b, 1e-14, 1.01, 3)
    assert res["k"] == [1]
    np.testing.assert_allclose(res["X"], e1, atol=1e-12)


def test_restore_dp_stops_at_first_k():
    a, b = _rand((8, 5, 4), 11), _rand((8, 2, 4), 12)
    out = tg.tgkb_restore(a, b, [1e3, 1e-12], 1.01, 3)
    assert out["k"] == [1, 3] and out["status"] == tg.DP_NOT_MET


# ---------------------------------------------------------------- nested_tGKB_p (Alg. 8)
def _krylov_lsq(A, b_start, b_rhs, k):
    """min ||A x - b_rhs|| over K_k(A^H A, A^H b_start) with an explicit power basis."""
    K = [A.conj().T @ b_start]
    for _ in range(k - 1):
        K.append(A.conj().T @ (A @ K[-1]))
    basis, _ = np.linalg.qr(np.stack(K, axis=1))
    y, *_ = np.linalg.lstsq(A @ basis, b_rhs, rcond=None)
    return basis @ y


@pytest.mark.parametrize("k", [1, 2, 3])
def test_nested_solution_is_recycled_krylov_minimizer(k):
    # slice j is solved over the space started from B_1: per face X_j-hat minimizes ||b_j - A x||
    # over K_k(A^H A, A^H b_1) (the projected problem equals it because A W_k lies in range Q_{k+1})
    a, b = _rand((8, 6, 4), 21), _rand((8, 3, 4), 22)
    ah, bh = tp.fft_tubes(a), tp.fft_tubes(b)
    W, Q, c, z = tg.tgkb_faces(ah, bh[:, 0, :], k)
    for j in range(3):
        xh, _ = tg.projected_lsq(W, Q, c, z, bh[:, j, :], k)
        for f in range(4):
            ref = _krylov_lsq(ah[:, :, f], bh[:, 0, f], bh[:, j, f], k)
            np.testing.assert_allclose(xh[:, f], ref, atol=1e-9 * max(1.0, np.linalg.norm(ref)))


def test_nested_projected_residual_identities():
    # slice 1: the projected residual is the literal one; other slices: literal^2 = projected^2 +
    # the part of B_j outside range Q_{k+1}, so the projected residual never exceeds the literal
    a, b = _rand((9, 5, 6), 23), _rand((9, 3, 6), 24)
    out = tg.nested_tgkb_restore(a, b, 1e-12, 1.01, 4, k_init=1)
    ah, bh = tp.fft_tubes(a), tp.fft_tubes(b)
    W, Q, c, z = tg.tgkb_faces(ah, bh[:, 0, :], 4)
    for k in range(1, 5):
        for j in range(3):
            xh, r = tg.projected_lsq(W, Q, c, z, bh[:, j, :], k)
            x = tp.ifft_tubes(xh[:, None, :])
            lit = tp.fro(b[:, j:j + 1, :] - tp.tprod(a, x))
            assert abs(out["res"][k - 1, j] - r) <= 1e-12 * lit
            if j == 0:
                assert abs(r - lit) <= 1e-10 * lit
            else:
                assert r <= lit * (1 + 1e-12)
                Qk = Q[:, :k + 1, :]
                outside = sum(np.linalg.norm(bh[:, j, f] - Qk[:, :, f] @ (Qk[:, :, f].conj().T @ bh[:, j, f])) ** 2
                              for f in range(6)) / 6
                assert abs(lit ** 2 - (r ** 2 + outside)) <= 1e-10 * lit ** 2


def test_nested_slice_one_matches_tgkb_from_k_init():
    # slice 1 runs Alg. 7 from B_1 exactly as tGKB does, but never stops before k_init = 2
    a, b = _rand((8, 6, 4), 25), _rand((8, 1, 4), 26)
    ref = tg.tgkb_restore(a, b, 1e-12, 1.01, 5)
    out = tg.nested_tgkb_restore(a, b, 1e-12, 1.01, 5)
    assert out["k"] == ref["k"]
    np.testing.assert_allclose(out["X"], ref["X"], atol=1e-10)
    big = tg.nested_tgkb_restore(a, b, 1e6, 1.01, 5)       # principle holds at once -> k_init
    assert big["k"] == [2] and big["status"] == tg.OK
    np.testing.assert_allclose(big["res"][:, 0], ref["res"][:, 0], rtol=1e-10)


def test_nested_k_never_decreases_and_identical_slices():
    a = _rand((10, 7, 4), 27)
    b1 = _rand((10, 1, 4), 28)
    same = tg.nested_tgkb_restore(a, np.concatenate([b1] * 3, axis=1), 0.5, 1.01, 6)
    assert len(set(same["k"])) == 1
    np.testing.assert_allclose(same["X"][:, 1], same["X"][:, 0], atol=1e-13)
    b = _rand((10, 4, 4), 29)
    d = np.array([1e3, 1e-3, 1e3, 1e-13])
    out = tg.nested_tgkb_restore(a, b, d, 1.01, 5)
    assert out["k"][0] == 2 and out["k"] == sorted(out["k"])
    assert out["k"][1] > 2 and out["k"][2] == out["k"][1]      # slice 3 keeps the larger space
    assert out["k"][3] == 5 and out["status"] == tg.DP_NOT_MET


def test_nested_full_space_gives_exact_solutions():
    # square, well-conditioned faces and k = m: every slice is solved exactly in the recycled space
    rng = np.random.default_rng(30)
    a = rng.standard_normal((5, 5, 4)) + 4.0 * np.eye(5)[:, :, None] * np.array([1, 0, 0, 0])
    x_true = rng.standard_normal((5, 3, 4))
    b = tp.tprod(a, x_true)
    out = tg.nested_tgkb_restore(a, b, 1e-9, 1.01, 5)
    np.testing.assert_allclose(out["X"], x_true, atol=1e-7)
