"""Seeded test problems shared by the parity tests: inputs from the workload generators, the
noise-free data B_true = A * X_true from the oracle's t-product (never from the HIP path)."""
from __future__ import annotations

import numpy as np

from oracle import tproduct as tp
from paper_2110_02485_amd import workloads as wl


def blur_problem(size, n, sigma, band, p, noise, k_max, oversample, seed=0, video=False, squares=0,
                 symmetric=False):
    """Storage-order float64 arrays A (n,m,l), X (n,p,m), B (n,p,l), Omega (n,r,m), delta.
    symmetric: the blur with a circularly symmetric tube (A^T = A)."""
    A = wl.blur_operator(size, n, sigma, band, symmetric=symmetric)
    rx = wl.rng_for("parity", "xtrue", seed)
    if video or p > 1:
        X = wl.lateral_slices(wl.moving_blob_video(size, n, p, rx))
    else:
        X = wl.lateral_slices(wl.blob_image(size, n, rx, squares=squares)[None])
    Am, Xm = wl.to_math(A), wl.to_math(X)
    Bt = tp.tprod(Am, Xm)
    E = wl.scale_noise(wl.noise_direction(Bt.shape, wl.rng_for("parity", "noise", seed)), Bt, noise)
    B = wl.to_storage(Bt + E)
    r = min(k_max + oversample, size)
    Om = wl.gaussian_omega(size, r, n, wl.rng_for("parity", "omega", seed))
    return A, X, B, Om, float(np.linalg.norm(E))


def random_problem(l, m, n, p, r, seed=0):
    rng = np.random.default_rng(seed)
    A = rng.standard_normal((n, m, l))
    B = rng.standard_normal((n, p, l))
    Om = rng.standard_normal((n, r, m))
    return A, B, Om
