"""Pins of the Tikhonov variants of the oracle (tGKT_p, t-LanczosTik_p: Tikhonov on the t-Krylov
spaces of Alg. 7 / Alg. 4 with mu from bisection, Sections 4.3 and 5) against independent forms:
the normal equations and the filter factors of the projected problem, the direct Tikhonov solution
of every Fourier face when the Krylov space is the whole space, the truncated solution as mu grows,
and the discrepancy equation for the returned mu."""
import numpy as np
import pytest

from oracle import tikhonov as tk
from oracle import tgkb as tg
from oracle import symmetric as sy
from oracle import tproduct as tp
from paper_2110_02485_amd import workloads as wl


def test_projected_tikhonov_three_ways():
    rng = np.random.default_rng(2)
    k = 7
    P = np.zeros((k + 1, k))
    for i in range(k):
        P[i, i] = rng.uniform(0.5, 2.0)
        P[i + 1, i] = rng.uniform(0.1, 1.0)
    beta, lam = 1.7, 0.03
    y, res = tk.tikhonov_face(P, beta, lam)
    e1 = np.zeros(k + 1)
    e1[0] = beta
    y_ne = np.linalg.solve(P.T @ P + lam * np.eye(k), P.T @ e1)            # normal equations
    u, s, vt = np.linalg.svd(P, full_matrices=False)
    y_ff = vt.T @ ((s / (s * s + lam)) * (u.T @ e1))                        # filter factors
    np.testing.assert_allclose(y, y_ne, rtol=1e-12)
    np.testing.assert_allclose(y, y_ff, rtol=1e-12)
    assert res == pytest.approx(np.linalg.norm(P @ y - e1), rel=1e-12)


def _small(symmetric=False, seed=0):
    rng = np.random.default_rng(seed)
    m, n = 6, 4
    a = rng.standard_normal((m, m, n)) + 3.0 * np.eye(m)[:, :, None] * (np.arange(n) == 0)
    if symmetric:
        a = 0.5 * (a + tp.ttranspose(a))
    x = rng.standard_normal((m, 2, n))
    b = tp.tprod(a, x) + 0.05 * rng.standard_normal((m, 2, n))
    return a, b


@pytest.mark.parametrize("lanczos", [False, True])
def test_full_space_equals_direct_tikhonov(lanczos):
    # k = m: the t-Krylov space is the whole space on every face, so the projected Tikhonov
    # solution is the direct one, (A_f^H A_f + lam I)^{-1} A_f^H b_f face by face
    a, b = _small(symmetric=lanczos, seed=3)
    m, n = a.shape[1], a.shape[2]
    ah = tp.fft_tubes(a)
    bh = tp.fft_tubes(b[:, :1, :])[:, 0, :]
    lam = 0.02
    if lanczos:
        Bas, c, z = sy.tlanczos_faces(ah, bh, m)
        proj = lambda f: sy.tridiag(c, z, m, f)
    else:
        Bas, _, c, z = tg.tgkb_faces(ah, bh, m)
        proj = lambda f: tg.bidiag(c, z, m, f)
    for f in range(n):
        y, _ = tk.tikhonov_face(proj(f), z[0, f], lam)
        x = Bas[:, :m, f] @ y
        A = ah[:, :, f]
        direct = np.linalg.solve(A.conj().T @ A + lam * np.eye(m), A.conj().T @ bh[:, f])
        np.testing.assert_allclose(x, direct, rtol=1e-8, atol=1e-10)


def test_residual_monotone_and_limits():
    a, b = _small(seed=5)
    ah = tp.fft_tubes(a)
    bh = tp.fft_tubes(b[:, :1, :])[:, 0, :]
    k = 4
    W, Q, c, z = tg.tgkb_faces(ah, bh, k)
    n = a.shape[2]
    Ps = [tg.bidiag(c, z, k, f) for f in range(n)]
    betas = [z[0, f] for f in range(n)]
    mus = np.logspace(-3, 9, 25)
    res = [tk.projected_residual(Ps, betas, 1.0 / mu) for mu in mus]
    assert all(r1 >= r2 - 1e-14 for r1, r2 in zip(res, res[1:]))
    # mu -> infinity: the truncated (least-squares) solution of tGKB; mu -> 0: X -> 0, residual ||b||
    xt = tg.tgkb_solution(W, c, z, k)
    for f in range(n):
        y, _ = tk.tikhonov_face(Ps[f], betas[f], 1e-14)
        np.testing.assert_allclose(W[:, :k, f] @ y, xt[:, 0, f], rtol=1e-6, atol=1e-9)
    assert tk.projected_residual(Ps, betas, 1e12) == pytest.approx(np.linalg.norm(bh) / np.sqrt(n), rel=1e-9)


@pytest.mark.parametrize("lanczos", [False, True])
def test_restore_meets_the_discrepancy_equation(lanczos):
    size, n = 24, 8
    A = wl.blur_operator(size, n, 2.0, 5, symmetric=lanczos)
    rng = wl.rng_for("tik", "xtrue")
    X = wl.lateral_slices(wl.moving_blob_video(size, n, 2, rng))
    a, x = wl.to_math(A), wl.to_math(X)
    bt = tp.tprod(a, x)
    E = wl.scale_noise(wl.noise_direction(bt.shape, wl.rng_for("tik", "noise")), bt, 1e-2)
    b = bt + E
    deltas = [float(np.linalg.norm(E[:, j, :])) for j in range(2)]
    fn = tk.tlanczos_tik_restore if lanczos else tk.tgkt_restore
    out = fn(a, b, deltas, 1.1, 20, 1e-2, 1e8)
    base = (sy.tlanczos_restore if lanczos else tg.tgkb_restore)(a, b, deltas, 1.1, 20)
    assert out["k"] == base["k"]                    # the truncated method's k
    for j in range(2):
        assert 1e-2 < out["mu"][j] < 1e8
        # literal residual of the returned X equals eta delta (bisection tolerance)
        lit = tp.fro(b[:, j:j + 1, :] - tp.tprod(a, out["X"][:, j:j + 1, :]))
        assert lit == pytest.approx(out["res"][j], rel=1e-10)
        assert lit <= 1.1 * deltas[j] * (1 + 1e-12) and lit == pytest.approx(1.1 * deltas[j], rel=1e-8)
    # an interval that cannot reach the bound: mu_hi returned, status DP_NOT_MET
    out2 = fn(a, b, deltas, 1.1, 20, 1e-6, 1e-4)
    assert out2["mu"] == [1e-4, 1e-4] and out2["status"] == tk.DP_NOT_MET


# ----------------------------------------------------------------------------------------------
# nested_tGKT_p: Tikhonov on the nested t-Krylov space of Alg. 8
# ----------------------------------------------------------------------------------------------
def test_nested_tikhonov_full_space_equals_direct_for_every_slice():
    # k = m: the nested space is the whole space on every face and range(A_f) lies in the span of
    # Q_{m+1}, so for every slice (not only the one that started the basis) the projected Tikhonov
    # solution is the direct (A_f^H A_f + lam I)^{-1} A_f^H b-hat_{j,f}
    a, b = _small(seed=7)
    m, n = a.shape[1], a.shape[2]
    ah, bh = tp.fft_tubes(a), tp.fft_tubes(b)
    W, Q, c, z = tg.tgkb_faces(ah, bh[:, 0, :], m)
    lam = 0.05
    for j in range(b.shape[1]):
        xh, _ = tk.nested_tikhonov_slice(W, Q, c, z, bh[:, j, :], m, lam)
        for f in range(n):
            A = ah[:, :, f]
            direct = np.linalg.solve(A.conj().T @ A + lam * np.eye(m), A.conj().T @ bh[:, j, f])
            np.testing.assert_allclose(xh[:, f], direct, rtol=1e-8, atol=1e-10)


def test_nested_tikhonov_limits_and_monotone_residual():
    # lam -> 0: the truncated solution of nested_tGKB_p (projected least squares) with its
    # projected residual; lam -> infinity: X -> 0 and the residual -> ||Q_{k+1}^H b_j||; the
    # residual grows with lam in between
    a, b = _small(seed=9)
    ah, bh = tp.fft_tubes(a), tp.fft_tubes(b)
    k, n = 4, a.shape[2]
    W, Q, c, z = tg.tgkb_faces(ah, bh[:, 0, :], k)
    bj = bh[:, 1, :]
    xt, rt = tg.projected_lsq(W, Q, c, z, bj, k)
    x0, r0 = tk.nested_tikhonov_slice(W, Q, c, z, bj, k, 1e-14)
    np.testing.assert_allclose(x0, xt, rtol=1e-6, atol=1e-9)
    assert r0 == pytest.approx(rt, rel=1e-8)
    xi, ri = tk.nested_tikhonov_slice(W, Q, c, z, bj, k, 1e14)
    assert np.abs(xi).max() < 1e-10 * np.abs(xt).max()
    g2 = sum(float(np.sum(np.abs(Q[:, :k + 1, f].conj().T @ bj[:, f]) ** 2)) for f in range(n))
    assert ri == pytest.approx(np.sqrt(g2 / n), rel=1e-9)
    res = [tk.nested_tikhonov_slice(W, Q, c, z, bj, k, lam)[1] for lam in np.logspace(-8, 8, 17)]
    assert all(r1 <= r2 + 1e-14 for r1, r2 in zip(res, res[1:]))


def _blur_pair(seed_name, p=3, noise=1e-2):
    size, n = 24, 8
    A = wl.blur_operator(size, n, 2.0, 5)
    X = wl.lateral_slices(wl.moving_blob_video(size, n, p, wl.rng_for(seed_name, "xtrue")))
    a, x = wl.to_math(A), wl.to_math(X)
    bt = tp.tprod(a, x)
    E = wl.scale_noise(wl.noise_direction(bt.shape, wl.rng_for(seed_name, "noise")), bt, noise)
    return a, bt + E, [float(np.linalg.norm(E[:, j, :])) for j in range(p)]


def test_nested_tgkt_meets_the_projected_discrepancy_equation():
    a, b, deltas = _blur_pair("ntik")
    out = tk.nested_tgkt_restore(a, b, deltas, 1.1, 20, 1e-2, 1e8)
    base = tg.nested_tgkb_restore(a, b, deltas, 1.1, 20)
    assert out["k"] == base["k"] and out["status"] == tk.OK
    ah, bh = tp.fft_tubes(a), tp.fft_tubes(b)
    W, Q, c, z = tg.tgkb_faces(ah, bh[:, 0, :], 20)
    for j in range(3):
        bound = 1.1 * deltas[j]
        assert 1e-2 < out["mu"][j] < 1e8
        # the returned mu meets the principle, a slightly smaller one does not (bisection bracket)
        assert out["res"][j] <= bound * (1 + 1e-12) and out["res"][j] == pytest.approx(bound, rel=1e-8)
        r_below = tk.nested_tikhonov_slice(W, Q, c, z, bh[:, j, :], out["k"][j], 1.0 / (out["mu"][j] * 0.999))[1]
        assert r_below > bound
        # X is the Tikhonov solution at that mu
        xh, _ = tk.nested_tikhonov_slice(W, Q, c, z, bh[:, j, :], out["k"][j], 1.0 / out["mu"][j])
        np.testing.assert_allclose(out["X"][:, j, :], tp.ifft_tubes(xh[:, None, :])[:, 0, :], rtol=1e-12, atol=1e-14)
    out2 = tk.nested_tgkt_restore(a, b, deltas, 1.1, 20, 1e-6, 1e-4)
    assert out2["mu"] == [1e-4] * 3 and out2["status"] == tk.DP_NOT_MET


def test_nested_tgkt_first_slice_is_tgkt():
    # slice 1 started the basis (g_1 = z_1 e_1) and, with k_init = 1, takes tGKB_p's index, so it
    # is tGKT_p on B_1: same k, mu and X
    a, b, deltas = _blur_pair("ntik1")
    nt = tk.nested_tgkt_restore(a, b, deltas, 1.1, 20, 1e-2, 1e8, k_init=1)
    t1 = tk.tgkt_restore(a, b[:, :1, :], deltas[:1], 1.1, 20, 1e-2, 1e8)
    assert nt["k"][0] == t1["k"][0]
    assert nt["mu"][0] == pytest.approx(t1["mu"][0], rel=1e-9)
    np.testing.assert_allclose(nt["X"][:, 0, :], t1["X"][:, 0, :], rtol=1e-8, atol=1e-12)
