"""Truncated pseudo-inverse solutions and the discrepancy principle, FP64.

TEST INFRASTRUCTURE ONLY (see the package docstring).

RT-tSVD (Section 4.2):  X_k = V_k * S_k^{-1} * U_k^T * B with U_k = Q * U-tilde(:, 1:k, :)
T-tSVD  (Section 4.1, eq. (14)):  X_s = V_s * S_s^{-1} * U_s^T * B
Discrepancy principle (eq. (disp)): the smallest k > 0 with ||B - A * X_k||_F <= eta * delta;
the experiments start at k_init = r - rho and increase k (eq. (kinit)).
"""
from __future__ import annotations

import numpy as np

from .tproduct import fft_tubes, ifft_tubes, tprod_hat, fro

OK = 0
DP_NOT_MET = 1


def pinv_cut(s: np.ndarray) -> float:
    """Numerical-rank cutoff of the truncated pseudo-inverse: sqrt(4 r eps) times the largest
    singular value over all faces (r = number of singular values per face, eps = 2^-52).  The
    inverse of S_k in X_k = V_k * S_k^{-1} * U_k^T * B is read as the Moore-Penrose inverse of the
    block-diagonal Fourier form of S_k with this tolerance: a face of A that is zero (or zero up to
    rounding) contributes nothing instead of 1/0."""
    return float(np.sqrt(4.0 * s.shape[0] * np.finfo(np.float64).eps) * s.max(initial=0.0))


def pinv_scale(d: np.ndarray, s: np.ndarray, cut: float = 0.0) -> np.ndarray:
    """diag(s)^+ d: rows divided by the singular values, rows of singular values <= cut set to zero."""
    out = np.zeros_like(d)
    nz = s > cut
    out[nz] = d[nz] / s[nz][:, None]
    return out


def coefficients_rtsvd(f: dict, b: np.ndarray) -> np.ndarray:
    """T_i = diag(1/s_i) U-breve_i^H Q_i^H B-hat_i for every face (r x p x n)."""
    bh = fft_tubes(b)
    n = bh.shape[2]
    cut = pinv_cut(f["s"])
    out = np.empty((f["s"].shape[0], b.shape[1], n), dtype=complex)
    for i in range(n):
        d = f["Ub"][:, :, i].conj().T @ (f["Q"][:, :, i].conj().T @ bh[:, :, i])
        out[:, :, i] = pinv_scale(d, f["s"][:, i], cut)
    return out


def coefficients_tsvd(f: dict, b: np.ndarray) -> np.ndarray:
    """T_i = diag(1/s_i) U_i^H B-hat_i for every face (eq. (14))."""
    bh = fft_tubes(b)
    n = bh.shape[2]
    cut = pinv_cut(f["s"])
    out = np.empty((f["s"].shape[0], b.shape[1], n), dtype=complex)
    for i in range(n):
        out[:, :, i] = pinv_scale(f["U"][:, :, i].conj().T @ bh[:, :, i], f["s"][:, i], cut)
    return out


def x_of_k(V: np.ndarray, T: np.ndarray, k: int) -> np.ndarray:
    """X_k = ifft( V_i[:, :k] T_i[:k, :] ) -- the k-term truncated solution."""
    xh = np.einsum("ijt,jkt->ikt", V[:, :k, :], T[:k, :, :])
    return ifft_tubes(xh)


def residual(ah: np.ndarray, b: np.ndarray, x: np.ndarray) -> float:
    """||B - A * X||_F with A given by its DFT (literal residual of eq. (disp))."""
    return fro(b - tprod_hat(ah, x))


def discrepancy(ah: np.ndarray, b: np.ndarray, V: np.ndarray, T: np.ndarray, delta,
                eta: float, k_start: int, k_cap: int, per_slice: bool = False):
    """Discrepancy-principle truncation index.

    Tries k = k_start, k_start + 1, ..., k_cap and returns the first k with
    ||B - A * X_k||_F <= eta * delta.  If none qualifies, k = k_cap with status
    DP_NOT_MET.  With ``per_slice`` every lateral slice j of B is its own problem
    with its own delta_j (``delta`` then is a sequence of length p) and gets its
    own k_j.  Returns (k or list of k, X, residuals (k_cap x groups), status).
    """
    p = b.shape[1]
    groups = [list(range(p))] if not per_slice else [[j] for j in range(p)]
    deltas = [float(delta)] if not per_slice else [float(d) for d in delta]
    ks, statuses = [], []
    res = np.full((k_cap, len(groups)), np.nan)
    X = np.zeros((V.shape[0], p, b.shape[2]))
    for g, cols in enumerate(groups):
        bg = b[:, cols, :]
        chosen = None
        for k in range(1, k_cap + 1):
            xk = x_of_k(V, T[:, cols, :], k)
            res[k - 1, g] = residual(ah, bg, xk)
            if chosen is None and k >= k_start and res[k - 1, g] <= eta * deltas[g]:
                chosen = k
        status = OK if chosen is not None else DP_NOT_MET
        if chosen is None:
            chosen = k_cap
        ks.append(chosen)
        statuses.append(status)
        X[:, cols, :] = x_of_k(V, T[:, cols, :], chosen)
    status = max(statuses)
    return (ks[0] if not per_slice else ks), X, res, status


def rtsvd_restore(a: np.ndarray, b: np.ndarray, omega: np.ndarray, delta, eta: float,
                  k_max: int, power_iters: int = 0, k_start: int = 1, per_slice: bool = False,
                  rho: int | None = None):
    """RT-tSVD restoration: fixed-r R-tSVD factor, coefficients, discrepancy principle.

    r = omega.shape[1] (= k_max + rho, capped at m).  ``k_start`` >= 1 starts the
    search there; ``k_start`` = 0 is the experiments' rule k_init = max(1, r - rho)
    (eq. (kinit)), in which case the search may run up to r.
    """
    from .factor import rtsvd_block
    f = rtsvd_block(a, omega, power_iters)
    r = omega.shape[1]
    k_cap = min(k_max, r)
    if k_start == 0:
        assert rho is not None
        k_start = max(1, r - rho)
        k_cap = r
    T = coefficients_rtsvd(f, b)
    k, X, res, status = discrepancy(f["ah"], b, f["V"], T, delta, eta, k_start, k_cap, per_slice)
    return {"k": k, "X": X, "res": res, "status": status, "factor": f, "T": T}


def tsvd_restore(a: np.ndarray, b: np.ndarray, delta, eta: float, k_max: int,
                 k_start: int = 1, per_slice: bool = False):
    """T-tSVD restoration (Section 4.1): full facewise SVD, then the discrepancy principle."""
    from .factor import tsvd
    f = tsvd(a)
    T = coefficients_tsvd(f, b)
    k, X, res, status = discrepancy(f["ah"], b, f["V"], T, delta, eta, k_start, k_max, per_slice)
    return {"k": k, "X": X, "res": res, "status": status, "factor": f, "T": T}


def relative_error(x: np.ndarray, x_true: np.ndarray) -> float:
    """E_method = ||X_method - X_true||_F / ||X_true||_F (Section 5)."""
    return fro(x - x_true) / fro(x_true)
