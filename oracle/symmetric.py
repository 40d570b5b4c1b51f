"""Methods for a symmetric tensor A (Section 3), FP64: T-tEVD (Alg. 2, eqs. (3)-(6), (61)) and
the t-Lanczos process and method (Alg. 4, eqs. (t-lanczos), (9t), (8)-(10)), t-Lanczos_p.

TEST INFRASTRUCTURE ONLY (see the package docstring).

A in R^{m x m x n} is symmetric (A^T = A) exactly when every DFT face A-hat_i is Hermitian
(Section 3.1); the faces' lower triangles are used.  The tEVD then has real eigenvalues per face;
Alg. 2 sorts each face's eigenpairs by decreasing magnitude.  The t-Lanczos process builds
A * Q_k = Q_{k+1} * T-bar_k with T-bar_k symmetric tridiagonal on top of one extra row
(diagonal tubes c_1..c_k, off-diagonal tubes z_1..z_k); on a Hermitian face the diagonal entries
q_i^H A-hat_i q_i are real, the off-diagonal ones are norms.
"""
from __future__ import annotations

import numpy as np

from .tproduct import fft_tubes, ifft_tubes, tprod, tprod_hat, ttranspose, fro
from .factor import normalize, normalize_tol
from .solve import discrepancy, pinv_cut, pinv_scale

OK = 0
DP_NOT_MET = 1


# ----------------------------------------------------------------------------------------------
# Alg. 2 -- T-tEVD and the T-tEVD method
# ----------------------------------------------------------------------------------------------
def tevd(a: np.ndarray, k: int | None = None):
    """tEVD A = W * D * W^T (eq. (3)) by a facewise Hermitian eigendecomposition after the tube DFT,
    each face's eigenpairs sorted by decreasing |eigenvalue| (Alg. 2, step 3); the first k kept.

    Returns W (m x k x n) and d (k x n, real eigenvalues) over all n faces, and A-hat.
    """
    m, m2, n = a.shape
    assert m == m2, "the tEVD needs a square (symmetric) tensor"
    ah = fft_tubes(a)
    kk = m if k is None else k
    W = np.empty((m, kk, n), dtype=complex)
    d = np.empty((kk, n))
    for i in range(n // 2 + 1):
        A_i = ah[:, :, i].real if i == (n - i) % n else ah[:, :, i]
        lam, vec = np.linalg.eigh(A_i, UPLO="L")
        order = np.argsort(-np.abs(lam), kind="stable")[:kk]
        for face, conj in ((i, False), ((n - i) % n, True)):
            W[:, :, face] = (np.conj(vec) if conj else vec)[:, order]
            d[:, face] = lam[order]
    return {"W": W, "d": d, "ah": ah, "n": n}


def spatial_tevd(f: dict):
    """W_k and D_k = diag(d_1, ..., d_k) back in the spatial domain (Alg. 2, last step)."""
    kk, n = f["d"].shape
    D = np.zeros((kk, kk, n), dtype=complex)
    D[np.arange(kk), np.arange(kk), :] = f["d"]
    return ifft_tubes(f["W"]), ifft_tubes(D)


def coefficients_tevd(f: dict, b: np.ndarray) -> np.ndarray:
    """T_i = diag(1/d_i) W_i^H B-hat_i for every face, so that X_k = W_k * T_k is eq. (6) / (61).

    diag(d)^{-1} is read as the pseudo-inverse with the tolerance of the truncated SVD solution
    (`solve.pinv_cut` on |d|, the singular values of a Hermitian face): an eigenvalue at or below
    sqrt(4 r eps) max |d| over all faces contributes nothing, so that on a symmetric A the T-tEVD
    solution equals the T-tSVD one also when a face is (nearly) singular."""
    bh = fft_tubes(b)
    n = bh.shape[2]
    ad = np.abs(f["d"])
    cut = pinv_cut(ad)
    out = np.empty((f["d"].shape[0], b.shape[1], n), dtype=complex)
    for i in range(n):
        sgn = np.where(f["d"][:, i] < 0.0, -1.0, 1.0)
        out[:, :, i] = pinv_scale(f["W"][:, :, i].conj().T @ bh[:, :, i], ad[:, i], cut) * sgn[:, None]
    return out


def tevd_restore(a: np.ndarray, b: np.ndarray, delta, eta: float, k_max: int,
                 k_start: int = 1, per_slice: bool = False):
    """T-tEVD method: the full tEVD first, then the discrepancy principle picks the truncation."""
    f = tevd(a)
    T = coefficients_tevd(f, b)
    k, X, res, status = discrepancy(f["ah"], b, f["W"], T, delta, eta, k_start, k_max, per_slice)
    return {"k": k, "X": X, "res": res, "status": status, "factor": f, "T": T}


# ----------------------------------------------------------------------------------------------
# Alg. 4 -- the t-Lanczos process
# ----------------------------------------------------------------------------------------------
def _tube_scale(x: np.ndarray, tube: np.ndarray) -> np.ndarray:
    return tprod(x, tube[None, None, :])


def tlanczos_literal(a: np.ndarray, b: np.ndarray, k: int, rng=None):
    """Alg. 4 with t-products and Normalize in the spatial domain (tiny inputs), followed in every
    step by one classical Gram-Schmidt pass against all earlier tensor columns (the
    re-orthogonalization the experiments use).  Returns Q (m x (k+1) x n), c tubes (k x n),
    z tubes ((k+1) x n) with z[0] the tube of Normalize(B).
    """
    tol = normalize_tol(fft_tubes(a))
    q1, z0 = normalize(b, tol, rng)
    Qs, cs, zs = [q1], [], [z0]
    q_prev = np.zeros_like(q1)
    for i in range(k):
        v = tprod(a, Qs[i])
        c = tprod(ttranspose(Qs[i]), v)[0, 0, :]
        v = v - _tube_scale(q_prev, zs[i] if i > 0 else np.zeros_like(z0)) - _tube_scale(Qs[i], c)
        proj = [tprod(qj, tprod(ttranspose(qj), v)) for qj in Qs]
        for pj in proj:
            v = v - pj
        q, z = normalize(v, tol, rng)
        q_prev = Qs[i]
        Qs.append(q)
        cs.append(c)
        zs.append(z)
    return np.concatenate(Qs, axis=1), np.array(cs), np.array(zs)


def tlanczos_faces(ah: np.ndarray, bh: np.ndarray, k: int):
    """Alg. 4 face by face in the Fourier domain for one right-hand side (same re-orthogonalization).

    A face norm at or below the threshold gives a zero scalar and a zero vector (the projected
    problem then keeps the solution already reached on that face).  The diagonal entries are the
    real parts of q_i^H A-hat_i q_i (real on a Hermitian face).
    Returns Qhat (m x (k+1) x n), c (k x n), z ((k+1) x n), all real scalars.
    """
    m, _, n = ah.shape
    tol = normalize_tol(ah)
    Q = np.zeros((m, k + 1, n), dtype=complex)
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
            w = A @ Q[:, i, f]
            c[i, f] = float(np.real(np.vdot(Q[:, i, f], w)))
            w = w - Q[:, i, f] * c[i, f]
            if i > 0:
                w = w - Q[:, i - 1, f] * z[i, f]
            Qi = Q[:, :i + 1, f]
            w = w - Qi @ (Qi.conj().T @ w)
            nw = np.linalg.norm(w)
            if nw > tol:
                Q[:, i + 1, f] = w / nw
                z[i + 1, f] = nw
    return Q, c, z


def tridiag(c: np.ndarray, z: np.ndarray, k: int, f: int) -> np.ndarray:
    """T-bar_k of face f: (k+1) x k, diagonal c_1..c_k, sub- and super-diagonal z_1..z_k
    (the last sub-diagonal entry z_k closes the extra row)."""
    T = np.zeros((k + 1, k))
    for i in range(k):
        T[i, i] = c[i, f]
        T[i + 1, i] = z[i + 1, f]
        if i + 1 < k:
            T[i, i + 1] = z[i + 1, f]
    return T


def tlanczos_solution(Q: np.ndarray, c: np.ndarray, z: np.ndarray, k: int) -> np.ndarray:
    """X_k-hat = Q_k Y_k with Y_k = argmin ||T-bar_k y - e_1 z_0|| per face (eq. (9t), Alg. 5)."""
    m, _, n = Q.shape
    xh = np.zeros((m, 1, n), dtype=complex)
    for f in range(n):
        rhs = np.zeros(k + 1)
        rhs[0] = z[0, f]
        y, *_ = np.linalg.lstsq(tridiag(c, z, k, f), rhs, rcond=None)
        xh[:, 0, f] = Q[:, :k, f] @ y
    return xh


def ritz_solution(Q: np.ndarray, c: np.ndarray, z: np.ndarray, k: int) -> np.ndarray:
    """Eq. (10): X_k = (Q_k * W) * D^{-1} * (Q_k * W)^T * B with T_k = W * D * W^T (eq. (8)), the
    tEVD of the leading k x k tridiagonal; Q_k^T * B = e_1 z_0 (eq. (fra))."""
    m, _, n = Q.shape
    xh = np.zeros((m, 1, n), dtype=complex)
    for f in range(n):
        Tk = tridiag(c, z, k, f)[:k, :]
        dv, Wv = np.linalg.eigh(Tk)
        rhs = np.zeros(k)
        rhs[0] = z[0, f]
        xh[:, 0, f] = (Q[:, :k, f] @ Wv) @ ((Wv.T @ rhs) / dv)
    return xh


def tlanczos_restore(a: np.ndarray, b: np.ndarray, delta, eta: float, k_max: int):
    """t-Lanczos_p: for every lateral slice j, run Alg. 4 from B_j and stop at the first k with
    ||B_j - A * X_{j,k}||_F <= eta * delta_j (literal residual).  Returns ks, X, residuals, status.
    """
    m, p, n = b.shape
    deltas = np.broadcast_to(np.asarray(delta, dtype=np.float64), (p,))
    ah = fft_tubes(a)
    X = np.zeros((a.shape[1], p, n))
    ks, res = [], np.full((k_max, p), np.nan)
    status = OK
    for j in range(p):
        bj = b[:, j:j + 1, :]
        Q, c, z = tlanczos_faces(ah, fft_tubes(bj)[:, 0, :], k_max)
        chosen = None
        for k in range(1, k_max + 1):
            xk = ifft_tubes(tlanczos_solution(Q, c, z, k))
            res[k - 1, j] = fro(bj - tprod_hat(ah, xk))
            if res[k - 1, j] <= eta * deltas[j]:
                chosen = k
                break
        if chosen is None:
            chosen = k_max
            status = DP_NOT_MET
        ks.append(chosen)
        X[:, j:j + 1, :] = ifft_tubes(tlanczos_solution(Q, c, z, chosen))
    return {"k": ks, "X": X, "res": res, "status": status}
