"""Facewise factorizations, FP64: Normalize (Alg. 3), R-tSVD (Alg. 6), tSVD (Alg. 1).

TEST INFRASTRUCTURE ONLY (see the package docstring).

Fourier-domain factors are dictionaries of per-face arrays over all n faces:
  Q  (l, r, n)  orthonormal columns per face       (Alg. 6, the Q of A ~ Q * B-tilde)
  C  (r, m, n)  B-tilde-hat = Q-hat^H A-hat         (Alg. 6, the rows B-tilde(j, :, :))
  Ub (r, r, n)  left singular vectors of C per face  (Alg. 6, U-breve of the tSVD of B-tilde)
  s  (r, n)     singular values, descending per face
  V  (m, r, n)  right singular vectors per face      (economy V-tilde)
"""
from __future__ import annotations

import numpy as np

from .tproduct import fft_tubes, ifft_tubes, tprod, ttranspose, fro


# ----------------------------------------------------------------------------------------------
# Alg. 3 -- Normalize
# ----------------------------------------------------------------------------------------------
def normalize(x: np.ndarray, tol: float, rng: np.random.Generator | None = None):
    """Normalize a tensor column X (d x 1 x n): X = V * a with every DFT face of V of unit 2-norm.

    Face by face in the Fourier domain: a^(j) = ||V^(j)||_2; faces whose norm is
    not above ``tol`` are replaced by a random unit vector and get a^(j) = 0
    (Alg. 3).  Returns (V, a) in the spatial domain, a as a length-n tube.
    The random replacement draws real Gaussian vectors for face j and uses the
    conjugate of that draw for face n - j, so V stays real.
    """
    d, one, n = x.shape
    assert one == 1
    vh = fft_tubes(x)[:, 0, :]
    a = np.zeros(n, dtype=complex)
    done = np.zeros(n, dtype=bool)
    for j in range(n):
        if done[j]:
            continue
        jj = (n - j) % n
        nrm = np.linalg.norm(vh[:, j])
        if nrm > tol:
            a[j] = nrm
            vh[:, j] /= nrm
            if jj != j:
                a[jj] = nrm
                vh[:, jj] = np.conj(vh[:, j])
        else:
            g = (rng or np.random.default_rng(0)).standard_normal(d) + 0j
            if jj != j:
                g = g + 1j * (rng or np.random.default_rng(1)).standard_normal(d)
            g /= np.linalg.norm(g)
            vh[:, j] = g
            a[j] = 0.0
            if jj != j:
                vh[:, jj] = np.conj(g)
                a[jj] = 0.0
        done[j] = done[jj] = True
    v = ifft_tubes(vh[:, None, :])
    tube = np.fft.ifft(a).real
    return v, tube


def normalize_tol(a_hat: np.ndarray) -> float:
    """Breakdown threshold for Normalize: 64 u max_i ||A-hat_i||_F (u = FP64 unit roundoff)."""
    return 64.0 * np.finfo(np.float64).eps / 2 * float(np.max(np.linalg.norm(a_hat, axis=(0, 1))))


# ----------------------------------------------------------------------------------------------
# Alg. 6 -- R-tSVD, the paper's incremental form (spatial domain, t-products)
# ----------------------------------------------------------------------------------------------
def rtsvd_literal(a: np.ndarray, omega: np.ndarray, eps: float | None = None,
                  r_fixed: int | None = None, rng: np.random.Generator | None = None):
    """R-tSVD built one tensor column at a time (Alg. 6, Thms 4.1-4.2).

    ``omega`` (m x R x n) supplies the Gaussian tensor columns G drawn in turn.
    Stops when the error indicator eta drops below eps^2 (fixed precision), or
    after ``r_fixed`` columns.  Step 5 subtracts the projection on all previous
    columns, Q_{1:r-1} * B-tilde(1:r-1, :, :) * G (randomized QB form), which
    equals the printed single-term expression once step 7 re-orthogonalizes.

    Returns dict(Q (l x r x n), Bt (r x m x n), eta list [eta^[0], ..., eta^[r]]).
    """
    l, m, n = a.shape
    tol = normalize_tol(fft_tubes(a))
    eta = fro(a) ** 2
    etas = [eta]
    qs: list[np.ndarray] = []
    rows: list[np.ndarray] = []
    r = 0
    while True:
        if r_fixed is not None and r >= r_fixed:
            break
        if r_fixed is None and eta < eps * eps:
            break
        if r >= omega.shape[1]:
            break
        g = omega[:, r:r + 1, :]
        z = tprod(a, g)
        if qs:
            Q = np.concatenate(qs, axis=1)
            Bt = np.concatenate(rows, axis=0)
            z = z - tprod(Q, tprod(Bt, g))
        z, _ = normalize(z, tol, rng)
        for qj in qs:
            z = z - tprod(qj, tprod(ttranspose(qj), z))
        z, _ = normalize(z, tol, rng)
        qs.append(z)
        y = tprod(ttranspose(z), a)      # 1 x m x n
        rows.append(y)
        eta = eta - fro(y) ** 2
        etas.append(eta)
        r += 1
    return {"Q": np.concatenate(qs, axis=1), "Bt": np.concatenate(rows, axis=0), "eta": etas}


# ----------------------------------------------------------------------------------------------
# block form in the Fourier domain
# ----------------------------------------------------------------------------------------------
def qr_positive(y: np.ndarray):
    """Householder QR (economy) with the diagonal of R made real and positive."""
    q, rr = np.linalg.qr(y)
    d = np.diag(rr).copy()
    ph = np.where(np.abs(d) > 0, d / np.where(np.abs(d) > 0, np.abs(d), 1.0), 1.0)
    q = q * ph[None, :]
    rr = np.conj(ph)[:, None] * rr
    return q, rr


def rtsvd_face(A_i: np.ndarray, O_i: np.ndarray, power_iters: int = 0) -> dict:
    """The block R-tSVD of one Fourier face (the per-face body of rtsvd_block): Q = orth(A_i O_i)
    refined by q power steps, C = Q^H A_i = U-breve diag(s) V^H.  Returns Q, C, Ub, s, Vh."""
    q, _ = qr_positive(A_i @ O_i)
    for _ in range(power_iters):
        qz, _ = qr_positive(A_i.conj().T @ q)
        q, _ = qr_positive(A_i @ qz)
    c = q.conj().T @ A_i
    u, sv, vh = np.linalg.svd(c, full_matrices=False)
    return {"Q": q, "C": c, "Ub": u, "s": sv, "Vh": vh}


def solution_face(fc: dict, b_i: np.ndarray, k: int, cut: float = 0.0) -> np.ndarray:
    """Face i of the truncated solution X_k = V_k * S_k^{-1} * U_k^T * B (Section 4.2) from one
    face's factor: V[:, :k] diag(1/s[:k]) U-breve[:, :k]^H Q^H b_i (b_i: l x p).  Singular values
    at or below `cut` (the all-face cutoff of solve.pinv_cut) count as zero (Moore-Penrose)."""
    d = fc["Ub"][:, :k].conj().T @ (fc["Q"].conj().T @ b_i)
    s = fc["s"][:k]
    t = np.zeros_like(d)
    t[s > cut] = d[s > cut] / s[s > cut][:, None]
    return fc["Vh"][:k, :].conj().T @ t


def rtsvd_block(a: np.ndarray, omega: np.ndarray, power_iters: int = 0):
    """Fixed-r R-tSVD, all r Gaussian columns at once, in the Fourier domain.

    For every face i: Y = A-hat_i Omega-hat_i; Q_i = Q-factor of Y with a real
    positive R diagonal -- in exact arithmetic the same Q that Alg. 6 builds by
    Gram-Schmidt with re-orthogonalization and per-face normalization; with
    ``power_iters`` = q > 0 the range is refined q times by Z = A-hat^H Q,
    Q_z = orth(Z), Y = A-hat Q_z, Q = orth(Y).  Then C_i = Q_i^H A-hat_i (the
    faces of B-tilde) and the SVD C_i = U-breve_i diag(s_i) V_i^H (Alg. 6,
    final steps).
    """
    l, m, n = a.shape
    ah = fft_tubes(a)
    oh = fft_tubes(omega)
    r = omega.shape[1]
    Q = np.empty((l, r, n), dtype=complex)
    C = np.empty((r, m, n), dtype=complex)
    Ub = np.empty((r, r, n), dtype=complex)
    s = np.empty((r, n))
    V = np.empty((m, r, n), dtype=complex)
    # Faces 0..n/2 are computed; face n - i is the complex conjugate of face i (real data).
    # Mirroring keeps the spatial-domain factors real also where a factor is not unique
    # (rank-deficient sketches, equal singular values).
    for i in range(n // 2 + 1):
        A_i, O_i = ah[:, :, i], oh[:, :, i]
        if i == (n - i) % n:  # faces 0 and n/2 of real data are real
            A_i, O_i = A_i.real, O_i.real
        fc = rtsvd_face(A_i, O_i, power_iters)
        q, c, u, sv, vh = fc["Q"], fc["C"], fc["Ub"], fc["s"], fc["Vh"]
        for face, conj in ((i, False), ((n - i) % n, True)):
            Q[:, :, face] = np.conj(q) if conj else q
            C[:, :, face] = np.conj(c) if conj else c
            Ub[:, :, face] = np.conj(u) if conj else u
            s[:, face] = sv
            V[:, :, face] = vh.T if conj else vh.conj().T
    return {"Q": Q, "C": C, "Ub": Ub, "s": s, "V": V, "ah": ah, "n": n}


def eta_prefix(a: np.ndarray, C: np.ndarray) -> np.ndarray:
    """Error indicator eta^[j] = ||A||_F^2 - sum_{j' <= j} ||B-tilde(j', :, :)||_F^2, j = 0..r.

    ||B-tilde(j', :, :)||_F^2 = (1/n) sum_i ||C_i(j', :)||^2 (Parseval); Thm 4.2.
    """
    n = C.shape[2]
    rown = np.sum(np.abs(C) ** 2, axis=(1, 2)) / n
    return fro(a) ** 2 - np.concatenate([[0.0], np.cumsum(rown)])


def spatial_factor(f) -> dict:
    """Q, B-tilde, U-tilde = Q * U-breve, S-tilde, V-tilde back in the spatial domain."""
    Q = ifft_tubes(f["Q"])
    Bt = ifft_tubes(f["C"])
    Ut = ifft_tubes(np.einsum("ijt,jkt->ikt", f["Q"], f["Ub"]))
    r, n = f["s"].shape
    Sh = np.zeros((r, r, n), dtype=complex)
    for j in range(r):
        Sh[j, j, :] = f["s"][j]
    return {"Q": Q, "Bt": Bt, "U": Ut, "S": ifft_tubes(Sh), "V": ifft_tubes(f["V"])}


# ----------------------------------------------------------------------------------------------
# Alg. 1 -- (truncated) tSVD
# ----------------------------------------------------------------------------------------------
def tsvd(a: np.ndarray, k: int | None = None):
    """tSVD A = U * S * V^T by facewise SVD after the tube DFT (Alg. 1); economy size."""
    l, m, n = a.shape
    ah = fft_tubes(a)
    kk = min(l, m) if k is None else k
    U = np.empty((l, kk, n), dtype=complex)
    S = np.zeros((kk, kk, n), dtype=complex)
    V = np.empty((m, kk, n), dtype=complex)
    s = np.empty((kk, n))
    for i in range(n // 2 + 1):
        A_i = ah[:, :, i].real if i == (n - i) % n else ah[:, :, i]
        u, sv, vh = np.linalg.svd(A_i, full_matrices=False)
        for face, conj in ((i, False), ((n - i) % n, True)):
            U[:, :, face] = (np.conj(u) if conj else u)[:, :kk]
            V[:, :, face] = (vh.T if conj else vh.conj().T)[:, :kk]
            s[:, face] = sv[:kk]
            S[np.arange(kk), np.arange(kk), face] = sv[:kk]
    return {"U": U, "S": S, "V": V, "s": s, "ah": ah, "n": n}
