"""MI355X-native randomized tSVD (R-tSVD) regularization for t-product least squares.

The hot path (tube FFT, facewise randomized SVD, discrepancy-principle truncation,
inverse FFT) runs in hand-written HIP kernels behind the C ABI declared in
``include/rtsvd.h``; ``paper_2110_02485_amd.rtsvd`` is the thin Python binding.
``paper_2110_02485_amd.workloads`` draws the seeded synthetic inputs.
"""
__all__ = ["workloads", "rtsvd"]
