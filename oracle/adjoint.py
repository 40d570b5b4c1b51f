"""Gradients of the truncated R-tSVD restoration, FP64 (extends Section 4.2; Omega and k fixed).

TEST INFRASTRUCTURE ONLY (see the package docstring).

Forward, face by face after the tube DFT (q = 0 power iterations, the form of Alg. 6):
    Y = A-hat Omega-hat,  Y = Q R  (R upper triangular with a real positive diagonal),
    C = Q^H A-hat,  G = C C^H = U diag(lambda) U^H,
    X-hat = C^H G_k^+ Q^H B-hat,   G_k^+ = sum_{j<=k} u_j u_j^H / lambda_j,
which equals V_k S_k^{-1} U_k^H B-hat of Section 4.2 (C = U diag(sqrt(lambda)) V^H).
Loss L = 1/2 ||X - X_true||_F^2 (spatial).

* dL/dB = P_k^T * (X - X_true) with P_k = V_k * S_k^{-1} * U_k^T: face by face
  Q U_k S_k^{-1} V_k^H G-hat (the adjoint t-product of Section 2).
* dL/dsigma for A = A(sigma): forward-mode derivative along dA = dA/dsigma, with
      dY = dA-hat Omega-hat,  M = Q^H dY R^{-1},
      dQ = Q (tril(M,-1) - tril(M,-1)^H + i Im diag(M)) + (I - Q Q^H) dY R^{-1},
      dC = dQ^H A-hat + Q^H dA-hat,  dG = dC C^H + C dC^H,
      d(G_k^+) = U (Phi o (U^H dG U)) U^H,
          Phi_jl = -1/(lambda_j lambda_l)              (j, l <= k)
                 = 1/(lambda_j (lambda_j - lambda_l))  (j <= k < l, and symmetrically)
                 = 0                                   (j, l > k),
      dX-hat = dC^H G_k^+ d + C^H d(G_k^+) d + C^H G_k^+ dQ^H B-hat,  d = Q^H B-hat,
  and dL/dsigma = <X - X_true, dX> (the Daleckii-Krein derivative of the spectral function
  that maps lambda_j to 1/lambda_j for j <= k and to 0 beyond).
"""
from __future__ import annotations

import numpy as np

from .tproduct import fft_tubes, ifft_tubes
from .factor import qr_positive


def _face_forward(Ai, Oi, Bi, k):
    q, R = qr_positive(Ai @ Oi)
    C = q.conj().T @ Ai
    lam, U = np.linalg.eigh(C @ C.conj().T)
    order = np.argsort(-lam, kind="stable")
    lam, U = lam[order], U[:, order]
    phi = np.zeros_like(lam)
    phi[:k] = 1.0 / lam[:k]
    Gk = (U * phi[None, :]) @ U.conj().T
    d = q.conj().T @ Bi
    X = C.conj().T @ (Gk @ d)
    return q, R, C, lam, U, Gk, d, X


def restore_fixed_k(a: np.ndarray, b: np.ndarray, omega: np.ndarray, k: int) -> np.ndarray:
    """X_k for a fixed truncation index k (math-order arrays)."""
    ah, oh, bh = fft_tubes(a), fft_tubes(omega), fft_tubes(b)
    n = ah.shape[2]
    xh = np.zeros((a.shape[1], b.shape[1], n), dtype=complex)
    for i in range(n // 2 + 1):
        Ai, Oi, Bi = ah[:, :, i], oh[:, :, i], bh[:, :, i]
        if i == (n - i) % n:
            Ai, Oi, Bi = Ai.real, Oi.real, Bi.real
        xh[:, :, i] = _face_forward(Ai, Oi, Bi, k)[7]
        xh[:, :, (n - i) % n] = np.conj(xh[:, :, i])
    return ifft_tubes(xh)


def grads(a, da, b, omega, k, x_true):
    """(L, dL/dB, dL/dsigma) for L = 1/2 ||X_k - X_true||^2 with A(sigma), dA = dA/dsigma."""
    ah, dah, oh, bh = fft_tubes(a), fft_tubes(da), fft_tubes(omega), fft_tubes(b)
    n = ah.shape[2]
    x = restore_fixed_k(a, b, omega, k)
    g = x - x_true
    gh = fft_tubes(g)
    gbh = np.zeros(bh.shape, dtype=complex)
    dxh = np.zeros((a.shape[1], b.shape[1], n), dtype=complex)
    for i in range(n // 2 + 1):
        Ai, dAi, Oi, Bi, Gi = ah[:, :, i], dah[:, :, i], oh[:, :, i], bh[:, :, i], gh[:, :, i]
        if i == (n - i) % n:
            Ai, dAi, Oi, Bi, Gi = Ai.real, dAi.real, Oi.real, Bi.real, Gi.real
        q, R, C, lam, U, Gk, d, X = _face_forward(Ai, Oi, Bi, k)
        # dL/dB: Q U_k S_k^{-1} V_k^H G = Q G_k^+ C G  (C^H G_k^+ = V_k S_k^{-1} U_k^H)
        gbh[:, :, i] = q @ (Gk @ (C @ Gi))
        # forward-mode derivative along dA
        dY = dAi @ Oi
        Rinv = np.linalg.inv(R)
        M = q.conj().T @ dY @ Rinv
        low = np.tril(M, -1)
        Xq = low - low.conj().T + 1j * np.diag(np.diag(M).imag)
        dq = q @ Xq + (dY - q @ (q.conj().T @ dY)) @ Rinv
        dC = dq.conj().T @ Ai + q.conj().T @ dAi
        dG = dC @ C.conj().T + C @ dC.conj().T
        r = lam.size
        Phi = np.zeros((r, r))
        for j in range(r):
            for l in range(r):
                if j < k and l < k:
                    Phi[j, l] = -1.0 / (lam[j] * lam[l])
                elif j < k <= l:
                    Phi[j, l] = 1.0 / (lam[j] * (lam[j] - lam[l]))
                elif l < k <= j:
                    Phi[j, l] = 1.0 / (lam[l] * (lam[l] - lam[j]))
        dGk = U @ (Phi * (U.conj().T @ dG @ U)) @ U.conj().T
        dd = dq.conj().T @ Bi
        dxh[:, :, i] = dC.conj().T @ (Gk @ d) + C.conj().T @ (dGk @ d) + C.conj().T @ (Gk @ dd)
        for face, conj in ((i, False), ((n - i) % n, True)):
            if conj:
                gbh[:, :, face] = np.conj(gbh[:, :, i])
                dxh[:, :, face] = np.conj(dxh[:, :, i])
    gb = ifft_tubes(gbh)
    dx = ifft_tubes(dxh)
    loss = 0.5 * float(np.sum(g * g))
    return loss, gb, float(np.sum(g * dx))
