"""Seeded synthetic inputs for t-product least-squares restorations.

This module only *draws* inputs: blur operators, true images / video frames,
Gaussian noise directions and Gaussian test tensors.  It holds none of the
method's arithmetic (no FFT, no t-product, no factorization), so the FP64 oracle
and the HIP path can both be fed from it.

Storage convention (shared by every consumer): a third-order tensor
A in R^{l x m x n} is held as a C-contiguous array of shape (n, m, l) with
``arr[t, j, i] = A(i, j, t)``, i.e. column-major l x m x n with frontal slices
contiguous (MATLAB order).  ``to_math`` / ``to_storage`` switch to and from the
(l, m, n) indexing used in the paper's formulas.

Blur operator (Section 5, eq. (za)): a Gaussian Toeplitz matrix
T = toeplitz(z) / (sigma * sqrt(2 pi)) with z_j = exp(-j^2 / (2 sigma^2)) for
j < band and zero beyond; the frontal slices are A^(t) = c_t T.  The tube c is a
normalized Gaussian c_t = exp(-(t-1)^2 / (2 sigma_c^2)) / sum (the workloads'
tube, sigma_c = 2).  Noise (Section 5, eq. (e1)): E = level * E0 / ||E0||_F *
||B_true||_F with E0 standard normal, so delta = ||E||_F exactly.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

BASE_SEED = 211002485

_STREAMS = {"xtrue": 1, "noise": 2, "omega": 3, "fallback": 4, "aux": 5}


def rng_for(config: str, stream: str, extra: int = 0) -> np.random.Generator:
    """PCG64 generator for (config, stream); independent sub-streams."""
    key = [BASE_SEED, sum(ord(ch) * (31 ** i) for i, ch in enumerate(config)) % (2 ** 31),
           _STREAMS[stream], int(extra)]
    return np.random.Generator(np.random.PCG64(np.random.SeedSequence(key)))


def to_math(arr: np.ndarray) -> np.ndarray:
    """(n, m, l) storage array -> (l, m, n) view indexed like A(i, j, t)."""
    return arr.transpose(2, 1, 0)


def to_storage(a: np.ndarray) -> np.ndarray:
    """(l, m, n) math-order array -> C-contiguous (n, m, l) storage array."""
    return np.ascontiguousarray(a.transpose(2, 1, 0))


# ----------------------------------------------------------------------------------------------
# blur operator
# ----------------------------------------------------------------------------------------------
def blur_toeplitz(size: int, sigma: float, band: int) -> np.ndarray:
    """Symmetric banded Gaussian Toeplitz matrix of eq. (za), float64 (size x size)."""
    j = np.arange(size)
    z = np.where(j < band, np.exp(-(j.astype(np.float64) ** 2) / (2.0 * sigma * sigma)), 0.0)
    idx = np.abs(j[:, None] - j[None, :])
    return z[idx] / (sigma * np.sqrt(2.0 * np.pi))


def blur_toeplitz_dsigma(size: int, sigma: float, band: int) -> np.ndarray:
    """Entrywise derivative of ``blur_toeplitz`` with respect to sigma (band held fixed)."""
    j = np.arange(size).astype(np.float64)
    d = np.abs(j[:, None] - j[None, :])
    inside = d < band
    g = np.exp(-(d ** 2) / (2.0 * sigma * sigma))
    s2pi = np.sqrt(2.0 * np.pi)
    # T = g / (sigma s2pi);  dT/dsigma = g * (d^2/sigma^3) / (sigma s2pi) - g / (sigma^2 s2pi)
    val = g * (d ** 2) / (sigma ** 4 * s2pi) - g / (sigma * sigma * s2pi)
    return np.where(inside, val, 0.0)


def tube_weights(n: int, sigma_c: float | None = None, symmetric: bool = False) -> np.ndarray:
    """Normalized Gaussian tube c_t, t = 1..n (sigma_c = 2 by default).  symmetric: the circularly
    symmetric tube c_t ~ exp(-min(t-1, n-t+1)^2 / (2 sigma_c^2)), whose DFT is real (a t-symmetric
    blur); sigma_c = 0.8 by default, which keeps the DFT above 8 % of its maximum (the one-sided
    tube with sigma_c = 2 stays above 16 %), so no face of the blur is nearly singular."""
    if sigma_c is None:
        sigma_c = 0.8 if symmetric else 2.0
    t = np.arange(n, dtype=np.float64)
    if symmetric:
        t = np.minimum(t, n - t)
    c = np.exp(-(t ** 2) / (2.0 * sigma_c * sigma_c))
    return c / c.sum()


def blur_operator(size: int, n: int, sigma: float, band: int, sigma_c: float | None = None,
                  dtype=np.float64, symmetric: bool = False) -> np.ndarray:
    """Storage-order (n, m, l) blur tensor with A^(t) = c_t T (T symmetric Toeplitz); with a
    symmetric tube every DFT face c-hat_t T is real symmetric, so A^T = A."""
    T = blur_toeplitz(size, sigma, band)
    c = tube_weights(n, sigma_c, symmetric)
    # storage slice t holds A^(t) transposed; T is symmetric
    return np.ascontiguousarray((c[:, None, None] * T.T[None, :, :]).astype(dtype))


def blur_operator_dsigma(size: int, n: int, sigma: float, band: int, sigma_c: float = 2.0,
                         dtype=np.float64) -> np.ndarray:
    """Storage-order derivative dA/dsigma (the tube c does not depend on sigma)."""
    dT = blur_toeplitz_dsigma(size, sigma, band)
    c = tube_weights(n, sigma_c)
    return np.ascontiguousarray((c[:, None, None] * dT.T[None, :, :]).astype(dtype))


# ----------------------------------------------------------------------------------------------
# true solutions
# ----------------------------------------------------------------------------------------------
def _blob_field(rows: int, cols: int, centers, widths, amps) -> np.ndarray:
    """Sum of axis-aligned Gaussian blobs on a periodic rows x cols grid."""
    r = np.arange(rows, dtype=np.float64)[:, None]
    c = np.arange(cols, dtype=np.float64)[None, :]
    img = np.zeros((rows, cols))
    for (cr, cc), (wr, wc), a in zip(centers, widths, amps):
        dr = np.minimum(np.abs(r - cr), rows - np.abs(r - cr))
        dc = np.minimum(np.abs(c - cc), cols - np.abs(c - cc))
        img += a * np.exp(-0.5 * (dr / wr) ** 2 - 0.5 * (dc / wc) ** 2)
    return img


def blob_image(rows: int, cols: int, rng: np.random.Generator, nblobs: int = 5,
               squares: int = 0) -> np.ndarray:
    """rows x cols image in [0, 1]: seeded Gaussian blobs (+ optional constant squares)."""
    centers = [(rng.uniform(0, rows), rng.uniform(0, cols)) for _ in range(nblobs)]
    widths = [(rng.uniform(rows / 16, rows / 6), rng.uniform(cols / 16, cols / 6)) for _ in range(nblobs)]
    amps = rng.uniform(0.3, 1.0, size=nblobs)
    img = _blob_field(rows, cols, centers, widths, amps)
    img /= img.max()
    for _ in range(squares):
        side_r = int(rng.uniform(rows / 16, rows / 4))
        side_c = int(rng.uniform(cols / 16, cols / 4))
        r0 = int(rng.uniform(0, rows - side_r))
        c0 = int(rng.uniform(0, cols - side_c))
        img[r0:r0 + side_r, c0:c0 + side_c] += rng.uniform(0.2, 0.8)
    return np.clip(img, 0.0, 1.0)


def moving_blob_video(rows: int, cols: int, frames: int, rng: np.random.Generator,
                      nblobs: int = 5) -> np.ndarray:
    """frames x rows x cols sequence: blobs moving linearly (periodic in both image axes)."""
    centers = np.array([(rng.uniform(0, rows), rng.uniform(0, cols)) for _ in range(nblobs)])
    vel = rng.uniform(-1.0, 1.0, size=(nblobs, 2))
    widths = [(rng.uniform(rows / 16, rows / 6), rng.uniform(cols / 16, cols / 6)) for _ in range(nblobs)]
    amps = rng.uniform(0.3, 1.0, size=nblobs)
    out = np.empty((frames, rows, cols))
    for f in range(frames):
        cen = [((cr + f * vr) % rows, (cc + f * vc) % cols) for (cr, cc), (vr, vc) in zip(centers, vel)]
        out[f] = _blob_field(rows, cols, cen, widths, amps)
    out /= out.max()
    return out


def lateral_slices(frames: np.ndarray) -> np.ndarray:
    """p images of size l x n -> storage-order tensor X in R^{l x p x n}, X(:, j, :) = image j."""
    p, rows, cols = frames.shape
    return np.ascontiguousarray(frames.transpose(2, 0, 1))  # (n, p, l): arr[t, j, i] = frame_j[i, t]


# ----------------------------------------------------------------------------------------------
# noise and random test tensors
# ----------------------------------------------------------------------------------------------
def noise_direction(shape, rng: np.random.Generator) -> np.ndarray:
    """Standard normal E0 (float64)."""
    return rng.standard_normal(shape)


def scale_noise(e0: np.ndarray, b_true: np.ndarray, level: float) -> np.ndarray:
    """E = level * E0 / ||E0||_F * ||B_true||_F (eq. (e1)); delta = ||E||_F."""
    return level * e0 / np.linalg.norm(e0) * np.linalg.norm(b_true)


def gaussian_omega(m: int, r: int, n: int, rng: np.random.Generator) -> np.ndarray:
    """Storage-order real Gaussian test tensor Omega in R^{m x r x n} (shape (n, r, m))."""
    return rng.standard_normal((n, r, m))


# ----------------------------------------------------------------------------------------------
# named workloads (the benchmark configurations and the colour-image Krylov comparison)
# ----------------------------------------------------------------------------------------------
@dataclass
class Workload:
    name: str
    size: int            # l = m
    n: int               # tube length
    sigma: float         # blur width
    band: int            # blur band
    p: int               # right-hand sides (lateral slices of B)
    k_max: int           # largest truncation index considered
    oversample: int      # rho
    power_iters: int     # q
    noise: float         # relative noise level
    eta: float = 1.01    # discrepancy factor
    precision: str = "fp64"
    squares: int = 0
    video: bool = False
    problems: list = field(default_factory=list)  # per-problem frame counts (differentiable batch)
    symmetric: bool = False  # circularly symmetric blur tube (A^T = A)
    seed_name: str = ""      # draw the inputs of this workload (same X_true, noise direction, Omega)

    @property
    def r(self) -> int:
        return min(self.k_max + self.oversample, self.size)

    @property
    def faces(self) -> int:
        return self.n // 2 + 1


WORKLOADS = {
    "blur64": Workload("blur64", 64, 16, 2.0, 6, 1, 20, 10, 0, 1e-2, precision="fp64"),
    "blur256": Workload("blur256", 256, 256, 3.0, 10, 1, 60, 10, 0, 1e-3, precision="fp32", squares=3),
    # the same image and noise direction at the second noise level of the 256-wide comparison
    "blur256n2": Workload("blur256n2", 256, 256, 3.0, 10, 1, 60, 10, 0, 1e-2, precision="fp32", squares=3,
                          seed_name="blur256"),
    "video512": Workload("video512", 512, 64, 3.0, 10, 64, 80, 10, 0, 1e-2, precision="fp32", video=True),
    "blur1024": Workload("blur1024", 1024, 128, 3.0, 10, 1, 100, 20, 1, 1e-3, precision="mixed"),
    # Section 5's grey-scale video example: 240 x 240 x 240, six frames as lateral slices, band 12,
    # sigma 2.5, eta 1.2, r = 81 at relative noise 1e-3; tube length 240 = 2^4 3 5 (mixed-radix DFT)
    "video240": Workload("video240", 240, 240, 2.5, 12, 6, 71, 10, 0, 1e-3, eta=1.2, precision="fp32", video=True),
    # differentiable batch: 16 clips of uneven frame counts (4 to 32) restored in one call
    "diff512": Workload("diff512", 512, 64, 3.0, 10, 260, 80, 10, 0, 1e-2, precision="fp32", video=True,
                        problems=[4, 32, 9, 17, 6, 25, 12, 30, 5, 20, 14, 28, 8, 11, 23, 16]),
    # colour-image restoration of Section 5 (256 x 256 x 256 blur with band 12, sigma 3; three
    # channels as lateral slices): the Krylov comparison (tGKB_p, nested_tGKB_p)
    "rgb256": Workload("rgb256", 256, 256, 3.0, 12, 3, 60, 10, 0, 1e-3, precision="fp64", video=True),
    # grey-scale image restoration of Section 5 (band 9, sigma 3, eta 1.1) with a symmetric blur:
    # the comparison of the symmetric-A methods (T-tEVD, t-Lanczos) with tGKB, T-tSVD, RT-tSVD
    "sym256": Workload("sym256", 256, 256, 3.0, 9, 1, 100, 10, 0, 1e-3, eta=1.1, precision="fp64", squares=3,
                       symmetric=True),
}


def make_inputs(w: Workload, dtype=np.float64, seed_extra: int = 0):
    """Draw (A, X_true, E0, Omega) in storage order for workload ``w``.

    B is *not* formed here (that needs a t-product); callers form
    B = A * X_true + scale_noise(E0, A * X_true, w.noise) with the product of
    their choice.
    """
    A = blur_operator(w.size, w.n, w.sigma, w.band, dtype=np.float64, symmetric=w.symmetric)
    key = w.seed_name or w.name
    rx = rng_for(key, "xtrue", seed_extra)
    if w.video:
        frames = moving_blob_video(w.size, w.n, max(w.p, 1), rx)
        X = lateral_slices(frames)
    else:
        X = lateral_slices(blob_image(w.size, w.n, rx, squares=w.squares)[None])
    E0 = noise_direction((w.n, X.shape[1], w.size), rng_for(key, "noise", seed_extra))
    Om = gaussian_omega(w.size, w.r, w.n, rng_for(key, "omega", seed_extra))
    return A.astype(dtype), X.astype(dtype), E0, Om.astype(dtype)


def make_clip_inputs(w: Workload, dtype=np.float64):
    """Draw the differentiable batch of ``w``: (A, dA/dsigma, X_true, E0 per clip, Omega, offsets).

    Clip j is a moving-blob sequence of ``w.problems[j]`` frames from its own seeded stream; the
    clips sit side by side as lateral slices of X_true, clip j in slices offsets[j]:offsets[j+1].
    E0 is a list of per-clip noise directions (each clip is scaled to the relative level by the
    caller, who forms B with the t-product of their choice).
    """
    A = blur_operator(w.size, w.n, w.sigma, w.band, dtype=np.float64)
    dA = blur_operator_dsigma(w.size, w.n, w.sigma, w.band)
    clips, E0 = [], []
    for j, frames in enumerate(w.problems):
        clips.append(lateral_slices(moving_blob_video(w.size, w.n, frames, rng_for(w.name, "xtrue", j))))
        E0.append(noise_direction((w.n, frames, w.size), rng_for(w.name, "noise", j)))
    X = np.concatenate(clips, axis=1)
    offsets = np.concatenate([[0], np.cumsum(w.problems)]).astype(int)
    Om = gaussian_omega(w.size, w.r, w.n, rng_for(w.name, "omega"))
    return A.astype(dtype), dA.astype(dtype), X.astype(dtype), E0, Om.astype(dtype), offsets
