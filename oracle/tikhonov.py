"""Tikhonov regularization on the t-Krylov spaces of Alg. 7 and Alg. 4, FP64: tGKT_p and
t-LanczosTik_p (Sections 4.3 and 5).

TEST INFRASTRUCTURE ONLY (see the package docstring).

The paper compares its truncated iterations with these Tikhonov variants but defines them by
reference only; what it states is that the Tikhonov parameter mu is found by bisection over a
given interval ([1e1, 1e7] in the image examples) and that the number of Krylov steps is that of
the truncated method (the tGKT rows of the tables carry the tGKB k).  Reading used here (one
lateral slice B_j at a time, as the p-methods):

  * k: the truncated method's discrepancy index -- the first k with ||B_j - A * X_{j,k}|| <=
    eta delta_j (tGKB_p, Alg. 7 + Alg. 5; t-Lanczos_p, Alg. 4 + eq. (9t)), k_max if never;
  * X_mu = W_k * Y_mu with, face by face, Y_mu = argmin ||P-bar_k y - z_1 e_1||^2 + (1/mu) ||y||^2
    (P-bar_k the (k+1) x k bidiagonal of Alg. 7; T-bar_k, the tridiagonal, for t-Lanczos), i.e.
    min ||A * X - B_j||^2 + (1/mu) ||X||^2 over the t-Krylov space;
  * mu: bisection in log mu on [mu_lo, mu_hi] for the discrepancy principle ||B_j - A * X_mu|| =
    eta delta_j: the residual decreases as mu grows, the bracket keeps res(lo) > eta delta >=
    res(hi), and after `iters` halvings mu = hi (a mu that meets the principle).  If even mu_hi
    leaves the residual above eta delta, mu = mu_hi and the status is DP_NOT_MET; if mu_lo already
    meets it, mu = mu_lo.
The residual of the projected problem is the literal one: B_j lies in the span of the first
basis tube (Q_1 = B_j normalized), so ||B_j - A * W_k * Y|| = ||P-bar_k Y - z_1 e_1|| face by face.

nested_tGKT_p (the nested t-Krylov subspace method with Tikhonov regularization, which the paper
cites and compares): the same reading on the one t-Krylov space of nested_tGKB_p (Alg. 8), grown
from B_1.  Per slice j: k_j = nested_tGKB_p's index (the projected discrepancy principle, slices in
order, k never decreasing); Y_mu = argmin ||P-bar_k y - g_j||^2 + (1/mu) ||y||^2 face by face with
g_j = Q_{k+1}^H b-hat_j (complex), X_mu = W_k * Y_mu; mu by the same bisection for the projected
residual (the one Alg. 8 tests) = eta delta_j.  For j = 1 this is tGKT_p on B_1 (g_1 = z_1 e_1).
"""
from __future__ import annotations

import numpy as np

from .tproduct import fft_tubes, ifft_tubes, tprod_hat, fro
from .tgkb import tgkb_faces, tgkb_solution, bidiag, nested_tgkb_restore
from .symmetric import tlanczos_faces, tlanczos_solution, tridiag

OK = 0
DP_NOT_MET = 1
BISECTION_STEPS = 50


def tikhonov_face(P: np.ndarray, beta: float, lam: float):
    """argmin_y ||P y - beta e_1||^2 + lam ||y||^2 as the stacked least-squares problem
    [P; sqrt(lam) I] y ~ [beta e_1; 0]; returns (y, ||P y - beta e_1||)."""
    k1, k = P.shape
    M = np.vstack([P, np.sqrt(lam) * np.eye(k)])
    rhs = np.zeros(k1 + k)
    rhs[0] = beta
    y, *_ = np.linalg.lstsq(M, rhs, rcond=None)
    e = P @ y
    e[0] -= beta
    return y, float(np.linalg.norm(e))


def projected_residual(Ps, betas, lam: float) -> float:
    """sqrt((1/n) sum_f ||P_f y_f - beta_f e_1||^2) over all n faces (Parseval): the residual
    ||B_j - A * X|| of the Tikhonov solution with parameter lam = 1/mu."""
    n = len(Ps)
    tot = sum(tikhonov_face(P, b, lam)[1] ** 2 for P, b in zip(Ps, betas))
    return float(np.sqrt(tot / n))


def bisect_mu(res_of_mu, target: float, mu_lo: float, mu_hi: float, iters: int = BISECTION_STEPS):
    """Bisection in log mu for res(mu) = target, res decreasing in mu.  Returns (mu, status)."""
    if res_of_mu(mu_hi) > target:
        return mu_hi, DP_NOT_MET
    if res_of_mu(mu_lo) <= target:
        return mu_lo, OK
    lo, hi = np.log(mu_lo), np.log(mu_hi)
    for _ in range(iters):
        mid = 0.5 * (lo + hi)
        if res_of_mu(np.exp(mid)) > target:
            lo = mid
        else:
            hi = mid
    return float(np.exp(hi)), OK


def _restore(a, b, delta, eta, k_max, mu_lo, mu_hi, lanczos: bool):
    l, p, n = b.shape
    deltas = np.broadcast_to(np.asarray(delta, dtype=np.float64), (p,))
    ah = fft_tubes(a)
    X = np.zeros((a.shape[1], p, n))
    ks, mus, res = [], [], []
    status = OK
    for j in range(p):
        bj = b[:, j:j + 1, :]
        bhj = fft_tubes(bj)[:, 0, :]
        if lanczos:
            Bas, c, z = tlanczos_faces(ah, bhj, k_max)
            sol = lambda k: tlanczos_solution(Bas, c, z, k)
            proj = lambda k, f: tridiag(c, z, k, f)
        else:
            Bas, _, c, z = tgkb_faces(ah, bhj, k_max)
            sol = lambda k: tgkb_solution(Bas, c, z, k)
            proj = lambda k, f: bidiag(c, z, k, f)
        bound = eta * deltas[j]
        # k: the truncated method's discrepancy index (literal residual)
        k = k_max
        st = DP_NOT_MET
        for kk in range(1, k_max + 1):
            if fro(bj - tprod_hat(ah, ifft_tubes(sol(kk)))) <= bound:
                k, st = kk, OK
                break
        Ps = [proj(k, f) for f in range(n)]
        betas = [float(z[0, f]) for f in range(n)]
        mu, st_mu = bisect_mu(lambda mu: projected_residual(Ps, betas, 1.0 / mu), bound, mu_lo, mu_hi)
        xh = np.zeros((a.shape[1], 1, n), dtype=complex)
        for f in range(n):
            y, _ = tikhonov_face(Ps[f], betas[f], 1.0 / mu)
            xh[:, 0, f] = Bas[:, :k, f] @ y
        xj = ifft_tubes(xh)
        X[:, j:j + 1, :] = xj
        ks.append(k)
        mus.append(mu)
        res.append(fro(bj - tprod_hat(ah, xj)))
        status = max(status, st, st_mu)
    return {"k": ks, "mu": mus, "X": X, "res": res, "status": status}


def tgkt_restore(a: np.ndarray, b: np.ndarray, delta, eta: float, k_max: int, mu_lo: float, mu_hi: float):
    """tGKT_p: per lateral slice, k from tGKB's discrepancy principle, then Tikhonov on the
    t-Krylov space of Alg. 7 with mu from bisection (module docstring).  Returns k, mu, X, the
    literal residuals ||B_j - A * X_j|| and the status."""
    return _restore(a, b, delta, eta, k_max, mu_lo, mu_hi, lanczos=False)


def tlanczos_tik_restore(a: np.ndarray, b: np.ndarray, delta, eta: float, k_max: int, mu_lo: float,
                         mu_hi: float):
    """t-LanczosTik_p for a symmetric A: as tgkt_restore on the t-Lanczos space of Alg. 4 with the
    tridiagonal T-bar_k of eq. (9t)."""
    return _restore(a, b, delta, eta, k_max, mu_lo, mu_hi, lanczos=True)


def tikhonov_face_rhs(P: np.ndarray, g: np.ndarray, lam: float):
    """argmin_y ||P y - g||^2 + lam ||y||^2 for a general (complex) right-hand side g, as the
    stacked least-squares problem [P; sqrt(lam) I] y ~ [g; 0]; returns (y, ||P y - g||)."""
    k1, k = P.shape
    M = np.vstack([P, np.sqrt(lam) * np.eye(k)]).astype(complex)
    rhs = np.concatenate([np.asarray(g, dtype=complex), np.zeros(k, dtype=complex)])
    y, *_ = np.linalg.lstsq(M, rhs, rcond=None)
    return y, float(np.linalg.norm(P @ y - g))


def nested_tikhonov_slice(W, Q, c, z, bhj, k: int, lam: float):
    """Tikhonov solution of one slice (b-hat_j, l x n) on the first k vectors of the nested space:
    per face y = argmin ||P-bar_k y - Q_{k+1}^H b-hat_j||^2 + lam ||y||^2, x-hat = W_k y.  Returns
    (x-hat (m x n), projected residual sqrt((1/n) sum_f ||P-bar_k y - g||^2))."""
    m, _, n = W.shape
    xh = np.zeros((m, n), dtype=complex)
    tot = 0.0
    for f in range(n):
        P = bidiag(c, z, k, f)
        g = Q[:, :k + 1, f].conj().T @ bhj[:, f]
        y, r = tikhonov_face_rhs(P, g, lam)
        xh[:, f] = W[:, :k, f] @ y
        tot += r * r
    return xh, float(np.sqrt(tot / n))


def nested_tgkt_restore(a: np.ndarray, b: np.ndarray, delta, eta: float, k_max: int, mu_lo: float, mu_hi: float,
                        k_init: int = 2):
    """nested_tGKT_p: k_j from nested_tGKB_p (Alg. 8), then Tikhonov on its nested t-Krylov space
    with mu_j from bisection for the projected residual (module docstring).  Returns k, mu, X, the
    projected residuals at mu and the status."""
    l, p, n = b.shape
    deltas = np.broadcast_to(np.asarray(delta, dtype=np.float64), (p,))
    base = nested_tgkb_restore(a, b, delta, eta, k_max, k_init)
    ah = fft_tubes(a)
    bh = fft_tubes(b)
    W, Q, c, z = tgkb_faces(ah, bh[:, 0, :], k_max)
    X = np.zeros((a.shape[1], p, n))
    mus, res = [], []
    status = base["status"]
    for j in range(p):
        k = base["k"][j]
        bound = eta * deltas[j]
        mu, st_mu = bisect_mu(lambda mu: nested_tikhonov_slice(W, Q, c, z, bh[:, j, :], k, 1.0 / mu)[1], bound,
                              mu_lo, mu_hi)
        xh, r = nested_tikhonov_slice(W, Q, c, z, bh[:, j, :], k, 1.0 / mu)
        X[:, j, :] = ifft_tubes(xh[:, None, :])[:, 0, :]
        mus.append(mu)
        res.append(r)
        status = max(status, st_mu)
    return {"k": list(base["k"]), "mu": mus, "X": X, "res": res, "status": status}
