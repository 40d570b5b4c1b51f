"""Partial tGKB process (Alg. 7) and the tGKB regularization method (eqs. (9tt), (solgkb)), FP64.

TEST INFRASTRUCTURE ONLY (see the package docstring).

The process builds A * W_k = Q_{k+1} * P-bar_k with P-bar_k lower bidiagonal
(diagonal tubes c_1..c_k, sub-diagonal tubes z_2..z_{k+1}); the method takes
X_k = W_k * Y_k where Y_k solves min ||P-bar_k * Y - e_1 * z_1||_F facewise
(Alg. 5), and stops at the first k meeting the discrepancy principle.  Several
right-hand sides are handled one lateral slice at a time (tGKB_p).
"""
from __future__ import annotations

import numpy as np

from .tproduct import fft_tubes, ifft_tubes, tprod, tprod_hat, ttranspose, fro
from .factor import normalize, normalize_tol

OK = 0
DP_NOT_MET = 1


def _tube_scale(x: np.ndarray, tube: np.ndarray) -> np.ndarray:
    """t-product of a tensor column (d x 1 x n) with a tubal scalar (length-n tube)."""
    return tprod(x, tube[None, None, :])


def tgkb_literal(a: np.ndarray, b: np.ndarray, k: int, rng=None):
    """Alg. 7 written with t-products and Normalize in the spatial domain (tiny inputs).

    Re-orthogonalization (steps 5 and 8) is one classical Gram-Schmidt pass.
    Returns W (m x k x n), Q (l x (k+1) x n), c tubes (k x n), z tubes ((k+1) x n).
    """
    tol = normalize_tol(fft_tubes(a))
    at = ttranspose(a)
    q1, z1 = normalize(b, tol, rng)
    Qs, Ws, cs, zs = [q1], [], [], [z1]
    w_prev = np.zeros((a.shape[1], 1, a.shape[2]))
    for i in range(k):
        w = tprod(at, Qs[i]) - _tube_scale(w_prev, zs[i])
        proj = [tprod(wj, tprod(ttranspose(wj), w)) for wj in Ws]
        for pj in proj:
            w = w - pj
        w, c = normalize(w, tol, rng)
        q = tprod(a, w) - _tube_scale(Qs[i], c)
        proj = [tprod(qj, tprod(ttranspose(qj), q)) for qj in Qs]
        for pj in proj:
            q = q - pj
        q, z = normalize(q, tol, rng)
        Ws.append(w)
        cs.append(c)
        Qs.append(q)
        zs.append(z)
        w_prev = w
    return (np.concatenate(Ws, axis=1), np.concatenate(Qs, axis=1), np.array(cs), np.array(zs))


def tgkb_faces(ah: np.ndarray, bh: np.ndarray, k: int):
    """Alg. 7 face by face in the Fourier domain for one right-hand side.

    Every t-operation of Alg. 7 acts facewise after the tube DFT; Normalize's
    tubal scalars are, face by face, the real 2-norms.  A face whose norm is not
    above the threshold gets a zero scalar and a zero vector; the projected least
    squares problem then keeps the solution already reached on that face, the
    same solution Alg. 3's random replacement leads to.
    Returns What (m x k x n), Qhat (l x (k+1) x n), c (k x n), z ((k+1) x n) real.
    """
    l, m, n = ah.shape
    tol = normalize_tol(ah)
    W = np.zeros((m, k, n), dtype=complex)
    Q = np.zeros((l, k + 1, n), dtype=complex)
    c = np.zeros((k, n))
    z = np.zeros((k + 1, n))
    for f in range(n):
        A = ah[:, :, f]
        v = bh[:, f].astype(complex)
        nv = np.linalg.norm(v)
        if nv > tol:
            Q[:, 0, f] = v / nv
            z[0, f] = nv
        for i in range(k):
            w = A.conj().T @ Q[:, i, f]
            if i > 0:
                w = w - W[:, i - 1, f] * z[i, f]
            Wi = W[:, :i, f]
            w = w - Wi @ (Wi.conj().T @ w)
            nw = np.linalg.norm(w)
            if nw > tol:
                W[:, i, f] = w / nw
                c[i, f] = nw
            q = A @ W[:, i, f] - Q[:, i, f] * c[i, f]
            Qi = Q[:, :i + 1, f]
            q = q - Qi @ (Qi.conj().T @ q)
            nq = np.linalg.norm(q)
            if nq > tol:
                Q[:, i + 1, f] = q / nq
                z[i + 1, f] = nq
    return W, Q, c, z


def bidiag(c: np.ndarray, z: np.ndarray, k: int, f: int) -> np.ndarray:
    """P-bar_k of face f: (k+1) x k lower bidiagonal, diagonal c_1..c_k, sub-diagonal z_2..z_{k+1}."""
    P = np.zeros((k + 1, k))
    for i in range(k):
        P[i, i] = c[i, f]
        P[i + 1, i] = z[i + 1, f]
    return P


def tgkb_solution(W: np.ndarray, c: np.ndarray, z: np.ndarray, k: int) -> np.ndarray:
    """X_k-hat = W_k Y_k with Y_k = argmin ||P-bar_k y - e_1 z_1|| per face (Alg. 5, lstsq)."""
    m, _, n = W.shape
    xh = np.zeros((m, 1, n), dtype=complex)
    for f in range(n):
        P = bidiag(c, z, k, f)
        rhs = np.zeros(k + 1)
        rhs[0] = z[0, f]
        y, *_ = np.linalg.lstsq(P, rhs, rcond=None)
        xh[:, 0, f] = W[:, :k, f] @ y
    return xh


def tgkb_restore(a: np.ndarray, b: np.ndarray, delta, eta: float, k_max: int):
    """tGKB_p: for every lateral slice j, run Alg. 7 and stop at the first k with
    ||B_j - A * X_{j,k}||_F <= eta * delta_j (literal residual).  Returns ks, X, residuals, status.
    """
    l, p, n = b.shape
    deltas = np.broadcast_to(np.asarray(delta, dtype=np.float64), (p,))
    ah = fft_tubes(a)
    X = np.zeros((a.shape[1], p, n))
    ks, res = [], np.full((k_max, p), np.nan)
    status = OK
    for j in range(p):
        bj = b[:, j:j + 1, :]
        W, Q, c, z = tgkb_faces(ah, fft_tubes(bj)[:, 0, :], k_max)
        chosen = None
        for k in range(1, k_max + 1):
            xk = ifft_tubes(tgkb_solution(W, c, z, k))
            res[k - 1, j] = fro(bj - tprod_hat(ah, xk))
            if res[k - 1, j] <= eta * deltas[j]:
                chosen = k
                break
        if chosen is None:
            chosen = k_max
            status = DP_NOT_MET
        ks.append(chosen)
        X[:, j:j + 1, :] = ifft_tubes(tgkb_solution(W, c, z, chosen))
    return {"k": ks, "X": X, "res": res, "status": status}


# ----------------------------------------------------------------------------------------------
# Alg. 8 -- nested_tGKB_p: one t-Krylov space recycled over the lateral slices
# ----------------------------------------------------------------------------------------------
def projected_lsq(W: np.ndarray, Q: np.ndarray, c: np.ndarray, z: np.ndarray, bh: np.ndarray, k: int):
    """For one right-hand side b-hat (l x n): per face f, y = argmin ||P-bar_k y - Q_{k+1}^H b-hat_f||
    (the projected problem of Alg. 8, steps 3 and 9).  Returns (X_k-hat (m x n), projected residual
    ||P-bar_k Y - Q_{k+1}^T * B||_F in the spatial domain, i.e. (1/n) sum over faces, square-rooted).
    """
    m, _, n = W.shape
    xh = np.zeros((m, n), dtype=complex)
    tot = 0.0
    for f in range(n):
        P = bidiag(c, z, k, f)
        g = Q[:, :k + 1, f].conj().T @ bh[:, f]
        y, *_ = np.linalg.lstsq(P, g, rcond=None)
        xh[:, f] = W[:, :k, f] @ y
        tot += float(np.sum(np.abs(P @ y - g) ** 2))
    return xh, np.sqrt(tot / n)


def nested_tgkb_restore(a: np.ndarray, b: np.ndarray, delta, eta: float, k_max: int, k_init: int = 2):
    """nested_tGKB_p (Alg. 8): the bidiagonalization is started from B_1 only; slice j is solved in
    the present t-Krylov space, and the space grows (k <- k + 1, never restarted) while the
    projected residual of slice j is >= eta delta_j.  Slice 1 starts at k = k_init; every later
    slice at the k reached by its predecessor.  Returns ks, X, projected residuals (k_max x p, for
    every k), status (DP_NOT_MET when k_max was reached without the principle holding).
    """
    l, p, n = b.shape
    deltas = np.broadcast_to(np.asarray(delta, dtype=np.float64), (p,))
    ah = fft_tubes(a)
    bh = fft_tubes(b)
    W, Q, c, z = tgkb_faces(ah, bh[:, 0, :], k_max)
    res = np.zeros((k_max, p))
    for j in range(p):
        for k in range(1, k_max + 1):
            res[k - 1, j] = projected_lsq(W, Q, c, z, bh[:, j, :], k)[1]
    X = np.zeros((a.shape[1], p, n))
    ks, status = [], OK
    k = max(1, min(k_init, k_max))
    for j in range(p):
        while res[k - 1, j] >= eta * deltas[j]:
            if k == k_max:
                status = DP_NOT_MET
                break
            k += 1
        ks.append(k)
        X[:, j, :] = ifft_tubes(projected_lsq(W, Q, c, z, bh[:, j, :], k)[0][:, None, :])[:, 0, :]
    return {"k": ks, "X": X, "res": res, "status": status}

