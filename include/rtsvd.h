/*
 * librtsvd -- randomized tSVD (R-tSVD) regularization of t-product least-squares problems
 *             min || B - A * X ||_F,  A in R^{l x m x n}, B in R^{l x p x n}, l >= m,
 * on AMD MI355X (gfx950).  Method: Ugwu & Reichel, "Tensor regularization by truncated
 * iteration: a comparison of some solution methods for large-scale linear discrete ill-posed
 * problem with a t-product", arXiv:2110.02485.
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 *  * Tensors are DEVICE pointers in column-major l x m x n order: element (i, j, t) of a tensor
 *    with l rows and m columns is at offset i + l*j + l*m*t (frontal slices contiguous; a torch
 *    tensor of shape (n, m, l), contiguous).  Real data only.
 *  * dtype: RTSVD_F64 (double) or RTSVD_F32 (float) for every caller array of one call.
 *  * stream: a hipStream_t passed as void* (NULL = the default stream).  All device work of a
 *    call is ordered on it; the call returns without synchronizing unless stated otherwise.
 *  * Fourier conventions follow Section 2 of the paper: the DFT along the tubes
 *    (MATLAB fft(A, [], 3)); only faces 0 .. floor(n/2) are formed, the others being complex
 *    conjugates for real data.
 *  * Return value: RTSVD_OK (0), a warning (> 0) or an error (< 0).  On error nothing is
 *    launched after the failing step, outputs are unspecified and no handle is created;
 *    rtsvd_last_error() describes the failure.  Scratch memory is taken from the stream's
 *    memory pool and returned to it before the call returns (stream-ordered).
 */
#ifndef RTSVD_H
#define RTSVD_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* caller array types */
#define RTSVD_F64 0
#define RTSVD_F32 1

/* compute precision of the factorization
 *   FP64 : every step in double precision.
 *   FP32 : tube FFTs and the sketch / power / projection / W = A V products in float;
 *          Gram matrices, Cholesky, small SVD and discrepancy sums in double.
 *   BF16 : as FP32, but the sketch, power-iteration and projection products read A-hat in
 *          bfloat16 (round to nearest even) and accumulate in float.                        */
#define RTSVD_P_FP64 0
#define RTSVD_P_FP32 1
#define RTSVD_P_BF16 2

/* status codes */
#define RTSVD_OK 0
#define RTSVD_W_DP_NOT_MET 1       /* no k in [k_start, k_cap] met the discrepancy principle   */
#define RTSVD_W_RANK_DEFICIENT 2   /* a sketch column fell below the breakdown threshold        */
#define RTSVD_E_ARG (-1)           /* invalid argument (sizes, null pointers, eta_dp <= 1, ...) */
#define RTSVD_E_NOTFINITE (-2)     /* an input holds NaN or infinity (detected on the device)      */
#define RTSVD_E_HIP (-3)           /* a HIP runtime call failed                                 */
#define RTSVD_E_NOMEM (-4)         /* device memory could not be obtained                       */
#define RTSVD_E_UNSUPPORTED (-5)   /* valid but unsupported configuration (e.g. r > 256)        */

typedef struct rtsvd_factor_s* rtsvd_handle;

typedef struct {
  int32_t k_max;        /* largest truncation index the solve may choose, 1 <= k_max <= m        */
  int32_t oversample;   /* rho >= 0 (Section 4.2, r = k + rho): r = min(k_max + rho, m) <= 256  */
  int32_t power_iters;  /* q >= 0 range refinements A-hat A-hat^H; q = 0 is Alg. 6 as printed   */
  int32_t precision;    /* RTSVD_P_FP64 | RTSVD_P_FP32 | RTSVD_P_BF16                           */
  uint64_t seed;        /* key of the on-device Gaussian generator, used when omega == NULL: the */
                        /* tensor rtsvd_gaussian(seed, m, r, n, dtype of A) writes is drawn on   */
                        /* the device and used as omega (Alg. 6, "generate a Gaussian tensor")   */
  const void* omega;    /* optional DEVICE real m x r x n Gaussian tensor (dtype of A, finite);  */
                        /* the r tensor columns play the role of the Gaussian slices G of Alg. 6 */
  double eps;           /* > 0: also report r_eps = min{ j : eta^[j] < eps^2 } (Alg. 6 stopping */
                        /* rule, Thm 4.2); <= 0: not used                                        */
  int32_t adaptive;     /* nonzero (with eps > 0): the fixed-precision R-tSVD of Alg. 6 -- the  */
                        /* factor keeps the first r_eps sketch columns (r_max = min(k_max +     */
                        /* oversample, m) if eta^[j] >= eps^2 for all j), so that rtsvd_solve   */
                        /* with k_start = 0 searches k from r_eps - oversample (the experiments' */
                        /* rule, Section 5).  The nested sketch makes this the factor Alg. 6    */
                        /* builds column by column.  Costs one host synchronization.            */
  int32_t face_groups;  /* 0: automatic (3 groups, fewer below 12 faces; the environment        */
                        /* variable RTSVD_FACE_GROUPS = 1..3 overrides); 1..3: split the per-face */
                        /* work into that many groups on library streams (see rtsvd_factor).     */
                        /* The result does not depend on it (bit for bit); adaptive factors and  */
                        /* runs with the stage timers enabled use one group.                     */
  int32_t sketch_tile;  /* 0: automatic (by r: the smallest of 1, 2, 4, 8 sixteen-column MFMA     */
                        /* tiles per workgroup covering r columns); 1, 2, 4 or 8: that many tiles */
                        /* in the factor's A-hat products (sketch, power, projection, Q = Y R^-1, */
                        /* W = A-hat V).  Only the work split changes: the result does not depend */
                        /* on it (bit for bit).                                                   */
} rtsvd_opts;

/* R-tSVD factorization (Section 4.2, Alg. 6 in block form, Thms 4.1-4.2).
 * A: DEVICE l x m x n (dtype).  Computes, per Fourier face i < floor(n/2)+1, the orthonormal
 * Q_i (l x r) spanning A-hat_i Omega-hat_i (refined by q power iterations), the projection
 * C_i = Q_i^H A-hat_i = U-breve_i diag(sigma_i) V_i^H (small SVD in FP64, sigma descending) and
 * W_i = A-hat_i V_i (used for the exact discrepancy residual).  The factor does not depend on B
 * (Section 5), so one handle serves any number of rtsvd_solve calls.  The handle owns its
 * device buffers until rtsvd_factor_destroy; A may be freed after the stream reaches the end of
 * this call.  The per-face work may be issued on up to three streams of the library's own
 * (default priority, see rtsvd_opts.face_groups), forked from and joined back into `stream`
 * with events: all of the call's work is complete when `stream` reaches the end of the call.
 * With face_groups = 1 every launch of the call, and every scratch buffer it takes from the
 * library's cache, stays on `stream`: calls (factor and solve) issued on different streams are
 * then independent and may run concurrently, which overlaps one call's latency-bound small-matrix
 * kernels with another's passes over A-hat.  With more groups, calls on different streams share
 * the library's group streams (correct, but serialized per group).
 * Errors: RTSVD_E_ARG (l < m, n < 1, k_max < 1, k_max > m, oversample < 0,
 * power_iters < 0, bad precision, face_groups outside 0..3, sketch_tile not 0, 1, 2, 4 or 8,
 * null A/opts/out),
 * RTSVD_E_UNSUPPORTED (r > 256), RTSVD_E_HIP (the library's streams could not be created),
 * RTSVD_E_NOMEM.  Conditions found on the device are reported later, without a synchronization
 * here: RTSVD_W_RANK_DEFICIENT (a sketch column broke down, Alg. 3) and RTSVD_E_NOTFINITE (A holds
 * NaN or infinity, or ||A||_F^2 overflows: the factor is then formed from a zero A-hat and is
 * unusable) by rtsvd_factor_info, and RTSVD_E_NOTFINITE again in rtsvd_solve's status_out.     */
int rtsvd_factor(const void* A, int64_t l, int64_t m, int64_t n, int dtype,
                 const rtsvd_opts* opts, void* stream, rtsvd_handle* out);

/* Full facewise SVD factor of A (T-tSVD, Alg. 1 and Section 4.1): r = m, returned in the same
 * handle type so that rtsvd_solve applies the truncated solution of eq. (14).  m <= 256.     */
int ttsvd_factor(const void* A, int64_t l, int64_t m, int64_t n, int dtype, int32_t precision,
                 int32_t k_max, void* stream, rtsvd_handle* out);

/* Host-side summary of a factor; synchronizes the factor's stream.  Any output may be NULL.
 *   r      : number of sketch columns
 *   faces  : floor(n/2) + 1
 *   eta    : HOST array of r + 1 doubles, eta^[j] = ||A||_F^2 - sum_{j'<=j} ||B-tilde(j',:,:)||_F^2
 *            (Thm 4.2); eta[r] = ||A - Q * B-tilde||_F^2 (Thm 4.1)
 *   r_eps  : smallest j with eta^[j] < eps^2, or -1 (eps <= 0 or never reached)
 *   sigma  : HOST array r x faces, sigma[i*r + j] = j-th singular value of face i
 *   flags  : bit 0 = a Gram pivot fell below the breakdown threshold (rank-deficient sketch),
 *            bit 1 = A is not finite
 * Returns RTSVD_OK, RTSVD_W_RANK_DEFICIENT (flag bit 0) or RTSVD_E_NOTFINITE (flag bit 1; the
 * outputs are still written).  r_eps is the first j >= 1 with eta^[j] < eps^2, as Alg. 6 tests
 * the indicator after each new column.                                                         */
int rtsvd_factor_info(rtsvd_handle f, int32_t* r, int32_t* faces, double* eta, int32_t* r_eps,
                      double* sigma, int32_t* flags);

/* Returns the handle's device buffers to the library's workspace cache, where they are reused by
 * later calls on the handle's stream.  Call it once the last rtsvd_solve that reads the handle
 * has been issued on that stream (or has completed, if it ran on another stream).  NULL is a
 * no-op.                                                                                       */
void rtsvd_factor_destroy(rtsvd_handle f);

/* Device workspace.  Every call takes its scratch buffers (and a factor its outputs) from a cache
 * of device allocations kept per (device, stream): a buffer released on a stream is handed out
 * again only to work on that stream, so reuse is ordered by the stream itself.  The cache grows
 * to the largest working set seen and is kept until rtsvd_trim, which synchronizes every device
 * holding cached buffers and frees them (buffers of live handles are untouched).
 * Errors: RTSVD_E_HIP.                                                                          */
int rtsvd_trim(void);

/* Truncated R-tSVD / T-tSVD solution with the discrepancy principle (eq. (disp), eq. (kinit)):
 *   X_k = V_k * S_k^{-1} * U_k^T * B,  U_k = Q * U-tilde(:, 1:k, :)   (Section 4.2)
 * B: DEVICE l x p x n (dtype; l and n those of the factor's A, p >= 1 any); X: DEVICE m x p x n
 * (dtype), caller-allocated.  The library reads l p n elements of B and writes m p n of X.
 * delta: HOST array; n_delta = 1 -> one noise bound for all of B, joint k (the single k of the
 *        RT-tSVD rows of the paper's tables); n_delta = p -> lateral slice j is its own problem
 *        with bound delta[j] and its own k_j.
 * eta_dp > 1 is the discrepancy factor (tau of eq. (disp)).
 * k_start >= 1: the first k tried (1 = the literal principle, smallest k > 0); k_start = 0: the
 *        experiments' rule k_init = max(1, r - rho), increased up to r (eq. (kinit)).
 * k_start <= min(k_max, r) (an adaptive factor may keep r < k_max columns).
 * k_cap = min(k_max, r) for k_start >= 1 and r for k_start = 0.  The residual used is the exact
 *        ||B - A * X_k||_F (Fourier domain, FP64 sums).
 * k_out:     DEVICE int32[n_delta]: chosen k (k_cap when the principle is not met).
 * resid_out: DEVICE double[n_delta * k_cap] or NULL: resid_out[g*k_cap + k-1] = ||B_g - A*X_k||_F.
 * status_out: DEVICE int32[1] or NULL: RTSVD_OK, RTSVD_W_DP_NOT_MET, or RTSVD_E_NOTFINITE when B
 *        or the factor's A is not finite (any residual not finite; k_out then holds k_cap and X
 *        is unspecified).  Set on the device.
 * The call only launches kernels on `stream` (no synchronization, no host copies, outputs stay
 * on the device), so it can be captured in a HIP graph and replayed for new contents of the same
 * B buffer: make one call on the capturing stream first (its workspace comes from that stream's
 * cache, so the captured call allocates nothing), keep the handle alive while the graph is used.
 * Errors: RTSVD_E_ARG (null handle/B/X/delta/k_out, p < 1, n_delta not 1 or p, eta_dp <= 1,
 *         k_start < 0 or > min(k_max, r), dtype mismatch with the factor's caller dtype).     */
int rtsvd_solve(rtsvd_handle f, const void* B, int64_t p, int dtype,
                const double* delta, int32_t n_delta, double eta_dp, int32_t k_start,
                void* X, int32_t* k_out, double* resid_out, int32_t* status_out, void* stream);

/* rtsvd_solve without device allocation, for callers that cannot allocate device memory (code
 * under HIP graph capture, tight serving loops, harnesses that forbid hipMalloc).  Same arguments,
 * results (bit for bit) and errors as rtsvd_solve.  Its scratch (B-hat, coefficients, residual
 * sums, X-hat: about F (l p cs + 2 r p 16 + ceil(l/64) p k_cap 8 + m p 16) bytes, cs = 8 for
 * FP32/BF16 work, 16 for FP64) is a fixed 64 MiB device array of the library, one per device,
 * held until the process ends; a solve that needs more returns RTSVD_E_UNSUPPORTED before any
 * work is issued.  Every call on a device uses the same array: calls that overlap on one device
 * (concurrent streams or threads) race and must be serialized by the caller.  Nothing in the
 * array needs to start at zero (every slice is written before it is read).                   */
int rtsvd_solve_noalloc(rtsvd_handle f, const void* B, int64_t p, int dtype, const double* delta,
                        int32_t n_delta, double eta_dp, int32_t k_start, void* X, int32_t* k_out,
                        double* resid_out, int32_t* status_out, void* stream);

/* t-product C = A * B (Definition 2.1 via the tube DFT, Section 2).
 * A: l x m x n, B: m x p x n, C: l x p x n, all DEVICE, same dtype.  Computed in the dtype. */
int tprod(const void* A, const void* B, void* C, int64_t l, int64_t m, int64_t p, int64_t n,
          int dtype, void* stream);

/* Adjoint t-product B = A^T * C (tensor transpose of Section 2: (A^T)-hat_i = A-hat_i^H).
 * A: l x m x n, C: l x p x n, B: m x p x n, all DEVICE, same dtype.                           */
int tprod_adjoint(const void* A, const void* C, void* B, int64_t l, int64_t m, int64_t p,
                  int64_t n, int dtype, void* stream);

/* tGKB_p regularization (Alg. 7 with full re-orthogonalization, projected least squares of
 * eq. (9tt) per face as in Alg. 5, X_k = W_k * Y_k of eq. (solgkb)): every lateral slice j of B
 * runs its own process and stops at the first k with ||B_j - A * X_{j,k}||_F <= eta_dp*delta_j.
 * A: DEVICE l x m x n; B: DEVICE l x p x n; X: DEVICE m x p x n (dtype; computed in dtype,
 * sums in FP64).  delta: HOST, n_delta = 1 (same bound for every slice) or p.
 * k_out: DEVICE int32[p]; resid_out: DEVICE double[k_max * p] or NULL (resid_out[j*k_max+k-1]);
 * status_out: DEVICE int32[1] or NULL.  The stream is never synchronized: after every step the
 * device posts its progress to pinned host memory, and the calling thread (which waits on that
 * progress) keeps at most three steps in flight; the call returns once every slice is decided or
 * k_max steps are enqueued, with the rest of the work queued on the stream.                  */
int tgkb_solve(const void* A, const void* B, int64_t l, int64_t m, int64_t n, int64_t p,
               int dtype, const double* delta, int32_t n_delta, double eta_dp, int32_t k_max,
               void* X, int32_t* k_out, double* resid_out, int32_t* status_out, void* stream);

/* nested_tGKB_p regularization (Alg. 8, Section 4.3): one run of Alg. 7 (full
 * re-orthogonalization), started from the first lateral slice B_1, serves every slice.  Slice j
 * is solved in the present t-Krylov space by the projected problem
 * min ||P-bar_k * Y - Q_{k+1}^T * B_j||_F (per face, complex right-hand side, Alg. 5), and the
 * space grows (never restarted) while that projected residual is >= eta_dp * delta_j.  Slice 1
 * starts at k = k_init (the algorithm's k_init = 2), every later slice at the k its predecessor
 * reached, so k_1 <= k_2 <= ... <= k_p.  A slice still unmet at k = k_max takes k_max, and so do
 * all later slices (status RTSVD_W_DP_NOT_MET).
 * A: DEVICE l x m x n; B: DEVICE l x p x n; X: DEVICE m x p x n (dtype; computed in dtype,
 * sums and the projected problems in FP64).  delta: HOST, n_delta = 1 or p.  k_init >= 1 (taken
 * as min(k_init, k_max)).  k_out: DEVICE int32[p]; resid_out: DEVICE double[k_max * p] or NULL:
 * resid_out[j*k_max + k-1] is slice j's projected residual at k for every k the basis reached
 * (0 beyond it).  status_out: DEVICE int32[1] or NULL.  Step loop as in tgkb_solve (no stream
 * synchronization, at most three steps in flight).
 * Errors: RTSVD_E_ARG (sizes, l < m, k_max outside [1, m], eta_dp <= 1, negative delta),
 * RTSVD_E_UNSUPPORTED (l > 8192).                                                             */
int nested_tgkb_solve(const void* A, const void* B, int64_t l, int64_t m, int64_t n, int64_t p,
                      int dtype, const double* delta, int32_t n_delta, double eta_dp, int32_t k_max,
                      int32_t k_init, void* X, int32_t* k_out, double* resid_out, int32_t* status_out,
                      void* stream);

/* tGKT_p: Tikhonov regularization on the t-Krylov space of Alg. 7 (Sections 4.3 and 5 compare the
 * truncated iterations with it; the paper gives the Tikhonov parameter mu by bisection on an
 * interval).  Per lateral slice j: k = tGKB_p's discrepancy index (the first k whose projected
 * least-squares residual is <= eta_dp delta_j, k_max if none), then
 *   X_j = W_k * Y,  Y = argmin ||P-bar_k y - z_1 e_1||^2 + (1/mu_j) ||y||^2  face by face,
 * i.e. min ||A * X - B_j||_F^2 + (1/mu_j) ||X||_F^2 over the t-Krylov space, with mu_j from
 * bisection in log mu on [mu_lo, mu_hi] (50 halvings) for ||B_j - A * X_j||_F = eta_dp delta_j
 * (the returned mu_j meets the principle: its residual is <= eta_dp delta_j).  If mu_hi leaves the
 * residual above the bound, mu_j = mu_hi; if mu_lo already meets it, mu_j = mu_lo.  The projected
 * problems are solved from the Givens QR of P-bar_k kept by the step loop (real banded normal
 * equations, FP64).  Arguments as tgkb_solve, and mu_lo, mu_hi (0 < mu_lo < mu_hi, finite), mu_out:
 * DEVICE double[p]; resid_out: DEVICE double[p] or NULL, ||B_j - A * X_j||_F at mu_j; status_out:
 * RTSVD_W_DP_NOT_MET when a slice reached k_max unmet or mu_hi could not meet its bound.
 * Errors: RTSVD_E_ARG, RTSVD_E_UNSUPPORTED (l > 8192).                                          */
int tgkt_solve(const void* A, const void* B, int64_t l, int64_t m, int64_t n, int64_t p, int dtype,
               const double* delta, int32_t n_delta, double eta_dp, int32_t k_max, double mu_lo, double mu_hi,
               void* X, int32_t* k_out, double* mu_out, double* resid_out, int32_t* status_out, void* stream);

/* nested_tGKT_p: Tikhonov regularization on the nested t-Krylov space of Alg. 8 (the nested method
 * with Tikhonov regularization that Sections 4.3 and 5 compare).  Per lateral slice j: k_j =
 * nested_tGKB_p's index (as nested_tgkb_solve: one basis from B_1, slices in order, k_init), then
 *   X_j = W_k * Y,  Y = argmin ||P-bar_k y - Q_{k+1}^T * B_j||^2 + (1/mu_j) ||y||^2  face by face
 * (complex projected right-hand side), with mu_j from bisection in log mu on [mu_lo, mu_hi] (50
 * halvings) for the projected residual ||P-bar_k Y - Q_{k+1}^T * B_j||_F = eta_dp delta_j (the one
 * Alg. 8 tests; the returned mu_j meets it).  If mu_hi leaves the residual above the bound,
 * mu_j = mu_hi; if mu_lo already meets it, mu_j = mu_lo.  The projected problems are solved from
 * the basis' Givens QR (real banded normal equations for the real and imaginary parts, FP64).
 * Arguments as nested_tgkb_solve, and mu_lo, mu_hi (0 < mu_lo < mu_hi, finite), mu_out: DEVICE
 * double[p]; resid_out: DEVICE double[p] or NULL, the projected residual at mu_j; status_out:
 * RTSVD_W_DP_NOT_MET when a slice reached k_max unmet or mu_hi could not meet its bound.
 * Errors: RTSVD_E_ARG (as nested_tgkb_solve, and the mu interval), RTSVD_E_UNSUPPORTED
 * (l > 8192).                                                                                   */
int nested_tgkt_solve(const void* A, const void* B, int64_t l, int64_t m, int64_t n, int64_t p, int dtype,
                      const double* delta, int32_t n_delta, double eta_dp, int32_t k_max, int32_t k_init,
                      double mu_lo, double mu_hi, void* X, int32_t* k_out, double* mu_out, double* resid_out,
                      int32_t* status_out, void* stream);

/* t-LanczosTik_p: as tgkt_solve on the t-Lanczos space of Alg. 4 for a symmetric A (the
 * (k+1) x k tridiagonal T-bar_k of eq. (9t) in place of P-bar_k; k = t-Lanczos_p's discrepancy
 * index), X_j = Q_k * Y.  Arguments as tlanczos_solve and tgkt_solve.                          */
int tlanczos_tik_solve(const void* A, const void* B, int64_t m, int64_t n, int64_t p, int dtype,
                       const double* delta, int32_t n_delta, double eta_dp, int32_t k_max, double mu_lo,
                       double mu_hi, void* X, int32_t* k_out, double* mu_out, double* resid_out,
                       int32_t* status_out, void* stream);

/* T-tEVD factor of a symmetric tensor (Alg. 2, Section 3.1): A in R^{m x m x n} with A^T = A, i.e.
 * every DFT face A-hat_i Hermitian (the faces' lower triangles are read; symmetry is the caller's
 * promise, not checked).  Facewise FP64 Hermitian eigendecomposition, eigenpairs ordered by
 * decreasing |eigenvalue|; the handle stores them as the SVD A-hat_i = (W_i sign(D_i)) |D_i| W_i^H,
 * so that rtsvd_solve gives the T-tEVD solutions X_k = W_k * D_k^{-1} * W_k^T * B of eqs. (6) and
 * (61) with the discrepancy principle, and rtsvd_factor_info returns r = m, |eigenvalues| as
 * sigma and eta^[j] = ||A||_F^2 - (1/n) sum_i sum_{j' <= j} |d_j'^(i)|^2.  Eigenvalues at or below
 * 4 m u max|d^(i)| count as zero.  A: DEVICE m x m x n; precision FP64 or FP32 (work type of the
 * stored vectors; the eigensolver is FP64).  Errors: RTSVD_E_ARG, RTSVD_E_UNSUPPORTED (m > 256).  */
int ttevd_factor(const void* A, int64_t m, int64_t n, int dtype, int32_t precision, int32_t k_max,
                 void* stream, rtsvd_handle* out);

/* t-Lanczos_p regularization of a symmetric tensor (Alg. 4 with full re-orthogonalization, the
 * projected least-squares problem of eq. (9t) per face as in Alg. 5, X_k = Q_k * Y_k): every
 * lateral slice j of B runs its own process from B_j and stops at the first k with
 * ||B_j - A * X_{j,k}||_F <= eta_dp * delta_j.  A: DEVICE m x m x n with Hermitian DFT faces (the
 * diagonal entries of the tridiagonal are taken as the real parts of q^H A-hat q); B: DEVICE
 * m x p x n; X: DEVICE m x p x n (dtype; computed in dtype, sums and the projected problems in
 * FP64).  delta: HOST, n_delta = 1 or p.  k_out: DEVICE int32[p]; resid_out: DEVICE
 * double[k_max * p] or NULL (resid_out[j*k_max + k-1], 0 beyond the last step run); status_out:
 * DEVICE int32[1] or NULL (RTSVD_W_DP_NOT_MET when a slice reached k_max without meeting the
 * principle; it then takes k_max).  Step loop as in tgkb_solve.  Errors: RTSVD_E_ARG,
 * RTSVD_E_UNSUPPORTED (m > 8192).                                                             */
int tlanczos_solve(const void* A, const void* B, int64_t m, int64_t n, int64_t p, int dtype,
                   const double* delta, int32_t n_delta, double eta_dp, int32_t k_max, void* X,
                   int32_t* k_out, double* resid_out, int32_t* status_out, void* stream);

/* Gradients of a loss L(X) through the truncated R-tSVD restoration at a fixed truncation index
 * k (no discrepancy search), fixed Gaussian tensor omega and q = 0 power iterations; the factor is
 * recomputed from A, not stored.  X = V_k * S_k^{-1} * U_k^T * B (Section 4.2).
 *   gX   : DEVICE m x p x n, dL/dX.
 *   gB   : DEVICE l x p x n out, dL/dB = P_k^T * gX (the adjoint t-product of Section 2).
 *   dA   : DEVICE l x m x n or NULL, a direction dA/ds of the operator (e.g. d/dsigma of the blur);
 *   gdot : DEVICE double[1] or NULL (together with dA): <gX, dX/ds>, the derivative of L along dA,
 *          from the forward-mode derivative of the QR, projection and truncated pseudo-inverse
 *          (Daleckii-Krein divided differences of lambda -> 1/lambda on the kept eigenvalues).
 * Computed in the dtype (FP64 small matrices).  Errors: RTSVD_E_ARG, RTSVD_E_UNSUPPORTED (r > 256). */
int rtsvd_solve_vjp(const void* A, const void* dA, const void* B, const void* omega, const void* gX,
                    int64_t l, int64_t m, int64_t n, int64_t p, int32_t k, int32_t oversample, int dtype,
                    void* gB, double* gdot, void* stream);

/* Stage timers (for benchmarks and profiling).  While enabled, every tagged stage of every call
 * is bracketed by a pair of HIP events recorded on the call's stream; rtsvd_timer_read
 * synchronizes on the recorded events of one tag and returns the summed elapsed time and the
 * number of bracketed launches.  rtsvd_timer_enable(0 or 1) also clears the record.         */
#define RTSVD_T_FFT_A 1      /* tube DFT of A (and ||A||_F partial sums)                     */
#define RTSVD_T_FFT_OMEGA 2  /* tube DFT of the Gaussian tensor                              */
#define RTSVD_T_SKETCH 3     /* Y = A-hat Omega-hat and the power iteration's Y = A-hat Q_z   */
#define RTSVD_T_POWER 4      /* the power iteration's Z = A-hat^H Q                           */
#define RTSVD_T_PROJECT 5    /* C^H = A-hat^H Q                                              */
#define RTSVD_T_W 6          /* W = A-hat V                                                  */
#define RTSVD_T_GRAM 7       /* FP64 Gram matrices of CholeskyQR                             */
#define RTSVD_T_CHOL 8       /* Cholesky + triangular inverse                                */
#define RTSVD_T_QMUL 9       /* Q = Y R^{-1}                                                 */
#define RTSVD_T_HEEV 10      /* Hermitian eigensolver of C C^H                               */
#define RTSVD_T_SVDAUX 11    /* Gram C C^H, V = C^H U-breve diag(1/sigma), error indicator    */
#define RTSVD_T_SOLVE 12     /* whole rtsvd_solve                                            */
#define RTSVD_T_TGKB 13      /* whole tgkb_solve                                             */
#define RTSVD_T_W_MMA 14     /* the MFMA kernel of W = A-hat V alone (inside RTSVD_T_W)        */
#define RTSVD_T_NESTED 15    /* whole nested_tgkb_solve                                      */
#define RTSVD_T_TLANCZOS 16  /* whole tlanczos_solve                                         */
int rtsvd_timer_enable(int on);
int rtsvd_timer_read(int tag, double* total_ms, int32_t* launches);

/* Gaussian test tensor of Alg. 6 ("generate a Gaussian random tensor"), drawn on the device:
 * out = DEVICE m x r x n (column-major, dtype), element e = i + m j + m r t standard normal.
 * Generator: Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC 2011) keyed by (seed mod 2^32,
 * seed div 2^32) on the counter (q mod 2^32, q div 2^32, 0, 0) of the pair q = floor(e / 2); its
 * output words (x0, x1, x2, x3) give u1 = (((x1 x0) >> 11) + 1/2) 2^-53 and u2 = ((x3 x2) >> 11)
 * 2^-53 (64-bit words formed high:low), and the Box-Muller pair sqrt(-2 ln u1) cos(2 pi u2)
 * (element 2q), sqrt(-2 ln u1) sin(2 pi u2) (element 2q + 1), computed in FP64 and rounded once.
 * rtsvd_factor with omega == NULL uses exactly this tensor.  Errors: RTSVD_E_ARG (null out,
 * sizes < 1, bad dtype), RTSVD_E_UNSUPPORTED (more than 2^32 elements), RTSVD_E_HIP.          */
int rtsvd_gaussian(uint64_t seed, int64_t m, int64_t r, int64_t n, int dtype, void* out, void* stream);

/* Human-readable status text. */
const char* rtsvd_status_string(int status);

/* Description of the last error raised on the calling host thread ("" if none). */
const char* rtsvd_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* RTSVD_H */
