"""FP64 CPU oracle for randomized-tSVD regularization of t-product least squares.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path imports, calls or links
anything in this package; only the test-suite, the smoke check and the CPU
baseline leg of the benchmark use it.  It shares no code with the HIP path.

Every function works on *math-order* float64 arrays: a tensor A in
R^{l x m x n} is an ndarray of shape (l, m, n) with ``A[i, j, t] = A(i, j, t)``.
Fourier-domain objects keep all n faces (the full spectrum of
``numpy.fft.fft`` along axis 2, the convention of Section 2), independently of
the half-spectrum storage used on the GPU.

Modules
  tproduct  -- t-product, transpose, identity, block-circulant form, norms (Section 2)
  factor    -- Normalize (Alg. 3), R-tSVD literal (Alg. 6) and block form, tSVD (Alg. 1)
  solve     -- truncated pseudo-inverse solutions, discrepancy principle, restorations
  tgkb      -- partial tGKB (Alg. 7), projected least squares (Alg. 5), tGKB method,
               nested_tGKB_p (Alg. 8)
  symmetric -- symmetric A: T-tEVD (Alg. 2), t-Lanczos process and method (Alg. 4, eq. (9t)),
               the Ritz form (eq. (10)), t-Lanczos_p
  adjoint   -- gradients of the truncated R-tSVD restoration (reverse mode in B,
               forward mode in the blur parameter)
"""
