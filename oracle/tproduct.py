"""t-product algebra, FP64 (Section 2: Definition 2.1 and the facts that follow it).

TEST INFRASTRUCTURE ONLY (see the package docstring).  Math-order arrays:
A[i, j, t] = A(i, j, t), shape (l, m, n).
"""
from __future__ import annotations

import numpy as np


def fft_tubes(a: np.ndarray) -> np.ndarray:
    """A-hat = fft(A, [], 3): DFT of every tube, all n faces (Section 2)."""
    return np.fft.fft(np.asarray(a, dtype=np.float64), axis=2)


def ifft_tubes(ah: np.ndarray, check_real: bool = True) -> np.ndarray:
    """Inverse DFT along the tubes; the result of a real computation must be real."""
    x = np.fft.ifft(ah, axis=2)
    if check_real:
        scale = max(1.0, float(np.abs(x).max())) if x.size else 1.0
        assert float(np.abs(x.imag).max(initial=0.0)) <= 1e-9 * scale, "inverse FFT not real"
    return np.ascontiguousarray(x.real)


def facewise(ah: np.ndarray, bh: np.ndarray) -> np.ndarray:
    """Product of corresponding frontal faces: C-hat(:,:,i) = A-hat(:,:,i) B-hat(:,:,i)."""
    return np.einsum("ijt,jkt->ikt", ah, bh)


def dft_face(a: np.ndarray, i: int) -> np.ndarray:
    """Face i of the tube DFT by its definition, A-hat_i = sum_t A(:, :, t) exp(-2 pi i i t / n)
    (Section 2), without transforming the other faces."""
    n = a.shape[2]
    w = np.exp(-2j * np.pi * i * np.arange(n) / n)
    return np.tensordot(a, w, axes=([2], [0]))


def tprod(a: np.ndarray, b: np.ndarray) -> np.ndarray:
    """t-product A * B via the DFT (Definition 2.1 computed as in Section 2)."""
    assert a.shape[1] == b.shape[0] and a.shape[2] == b.shape[2]
    return ifft_tubes(facewise(fft_tubes(a), fft_tubes(b)))


def tprod_hat(ah: np.ndarray, b: np.ndarray) -> np.ndarray:
    """A * B given A-hat already transformed (same product, A's DFT reused)."""
    return ifft_tubes(facewise(ah, fft_tubes(b)))


def tprod_conv(a: np.ndarray, b: np.ndarray) -> np.ndarray:
    """t-product from its definition: tube (i, j) is sum_k A(i,k,:) (circ-conv) B(k,j,:).

    Plain loops; meant for tiny tensors (Definition 2.1).
    """
    l, p, n = a.shape
    p2, m, n2 = b.shape
    assert p == p2 and n == n2
    out = np.zeros((l, m, n))
    for i in range(l):
        for j in range(m):
            for k in range(p):
                for t in range(n):
                    acc = 0.0
                    for s in range(n):
                        acc += a[i, k, s] * b[k, j, (t - s) % n]
                    out[i, j, t] += acc
    return out


def bcirc(a: np.ndarray) -> np.ndarray:
    """Block-circulant matrix of A: block (s, u) is the frontal slice A^((s-u) mod n)."""
    l, m, n = a.shape
    out = np.zeros((l * n, m * n))
    for s in range(n):
        for u in range(n):
            out[s * l:(s + 1) * l, u * m:(u + 1) * m] = a[:, :, (s - u) % n]
    return out


def unfold(b: np.ndarray) -> np.ndarray:
    """Stack the frontal slices of B vertically: [B^(1); B^(2); ...; B^(n)]."""
    m, p, n = b.shape
    return np.concatenate([b[:, :, t] for t in range(n)], axis=0)


def fold(mat: np.ndarray, m: int, n: int) -> np.ndarray:
    """Inverse of ``unfold``."""
    p = mat.shape[1]
    out = np.zeros((m, p, n))
    for t in range(n):
        out[:, :, t] = mat[t * m:(t + 1) * m]
    return out


def ttranspose(a: np.ndarray) -> np.ndarray:
    """Tensor transpose: transpose every frontal slice, then reverse slices 2..n (Section 2)."""
    l, m, n = a.shape
    out = np.empty((m, l, n))
    out[:, :, 0] = a[:, :, 0].T
    for t in range(1, n):
        out[:, :, t] = a[:, :, n - t].T
    return out


def identity(m: int, n: int) -> np.ndarray:
    """Identity tensor: first frontal slice I_m, all others zero (Section 2)."""
    out = np.zeros((m, m, n))
    out[:, :, 0] = np.eye(m)
    return out


def fro(a: np.ndarray) -> float:
    """Frobenius norm of a third-order tensor (Section 1)."""
    return float(np.sqrt(np.sum(np.asarray(a, dtype=np.float64) ** 2)))


def tube_inner(x: np.ndarray, y: np.ndarray) -> np.ndarray:
    """Tubal scalar X^T * Y for two tensor columns (l x 1 x n each), returned as a length-n tube."""
    return tprod(ttranspose(x), y)[0, 0, :]
