// tGKB_p regularization (Alg. 7, eq. (9tt), eq. (solgkb)) face by face in the Fourier domain.
//
// Every t-operation of Alg. 7 acts facewise after the tube DFT, and Normalize's tubal scalars
// are, face by face, the real 2-norms of the face vectors.  Each lateral slice c of B runs its
// own process (tGKB_p); all slices and all faces advance in lockstep:
//     w  = A-hat^H q_i - z_i w_{i-1},  re-orthogonalize (classical Gram-Schmidt, twice),
//     c_i = ||w||, w /= c_i;
//     q  = A-hat w_i - c_i q_i,        re-orthogonalize, z_{i+1} = ||q||, q /= z_{i+1}.
// A face whose norm is at or below the breakdown threshold gets a zero scalar and a zero vector
// (the projected problem then keeps the solution already reached on that face); the test is
// relative: the norm left after re-orthogonalization against the norm before it.
// The projected least-squares problem min ||P-bar_i y - e_1 z_1|| is updated with one Givens
// rotation per step (the bidiagonal is real); |phi-bar_{i+1}| is the face residual, and
//     rho_i^2 = (1/n) sum_f w_f |phi-bar_{i+1}(f)|^2
// is ||B_c - A * X_{c,i}||_F^2 exactly (A W_i = Q_{i+1} P-bar_i, Q orthonormal).  The first i with
// rho_i <= eta * delta_c fixes k_c; at the end y = R^{-1} f by back substitution and
// X-hat = W_k y.
#pragma once
#include "common.hpp"

namespace rt {

constexpr int GKB_THREADS = 1024;

// y(:, c) = A-hat x(:, c) for c < p (p <= 4), batched over faces; one thread per row.
// X column c of face f at X + f*sX + c*ldx.
template <typename T, int PMAX>
__global__ void __launch_bounds__(256)
k_gemv_n(const cplx<T>* __restrict__ A, int l, int m, int p, const cplx<T>* __restrict__ X, int64_t ldx, int64_t sX,
         cplx<T>* __restrict__ Y, int64_t ldy, int64_t sY) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  cplx<T>* xs = reinterpret_cast<cplx<T>*>(smem_raw);  // m x p
  const int f = blockIdx.y;
  const cplx<T>* Af = A + (int64_t)f * l * m;
  for (int idx = threadIdx.x; idx < m * p; idx += blockDim.x) {
    const int k = idx % m, c = idx / m;
    xs[c * m + k] = X[(int64_t)f * sX + (int64_t)c * ldx + k];
  }
  __syncthreads();
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= l) return;
  cplx<double> acc[PMAX];
#pragma unroll
  for (int c = 0; c < PMAX; ++c) acc[c] = mk(0.0, 0.0);
  for (int k = 0; k < m; ++k) {
    const cplx<T> a = Af[i + (int64_t)k * l];
#pragma unroll
    for (int c = 0; c < PMAX; ++c)
      if (c < p) {
        const cplx<T> x = xs[c * m + k];
        acc[c].re += (double)a.re * x.re - (double)a.im * x.im;
        acc[c].im += (double)a.re * x.im + (double)a.im * x.re;
      }
  }
#pragma unroll
  for (int c = 0; c < PMAX; ++c)
    if (c < p) Y[(int64_t)f * sY + (int64_t)c * ldy + i] = mk((T)acc[c].re, (T)acc[c].im);
}

// y(:, c) = A-hat^H x(:, c), one wave per output row j (a column of A-hat), p <= 4
template <typename T, int PMAX>
__global__ void __launch_bounds__(256)
k_gemv_c(const cplx<T>* __restrict__ A, int l, int m, int p, const cplx<T>* __restrict__ X, int64_t ldx, int64_t sX,
         cplx<T>* __restrict__ Y, int64_t ldy, int64_t sY) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  cplx<T>* xs = reinterpret_cast<cplx<T>*>(smem_raw);  // l x p
  const int f = blockIdx.y;
  const cplx<T>* Af = A + (int64_t)f * l * m;
  for (int idx = threadIdx.x; idx < l * p; idx += blockDim.x) {
    const int k = idx % l, c = idx / l;
    xs[c * l + k] = X[(int64_t)f * sX + (int64_t)c * ldx + k];
  }
  __syncthreads();
  const int lane = threadIdx.x & 63;
  const int j = blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
  if (j >= m) return;
  const cplx<T>* col = Af + (int64_t)j * l;
  cplx<double> acc[PMAX];
#pragma unroll
  for (int c = 0; c < PMAX; ++c) acc[c] = mk(0.0, 0.0);
  for (int i = lane; i < l; i += 64) {
    const cplx<T> a = col[i];
#pragma unroll
    for (int c = 0; c < PMAX; ++c)
      if (c < p) {
        const cplx<T> x = xs[c * l + i];
        acc[c].re += (double)a.re * x.re + (double)a.im * x.im;
        acc[c].im += (double)a.re * x.im - (double)a.im * x.re;
      }
  }
#pragma unroll
  for (int c = 0; c < PMAX; ++c) {
    double re = acc[c].re, im = acc[c].im;
    for (int o = 32; o > 0; o >>= 1) { re += __shfl_xor(re, o, 64); im += __shfl_xor(im, o, 64); }
    if (lane == 0 && c < p) Y[(int64_t)f * sY + (int64_t)c * ldy + j] = mk((T)re, (T)im);
  }
}

__device__ __forceinline__ double gkb_block_sum(double v, double* red) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  __syncthreads();
  if (lane == 0) red[w] = v;
  __syncthreads();
  double s = 0.0;
  for (int i = 0; i < (int)(blockDim.x >> 6); ++i) s += red[i];
  return s;
}

// One half-step of Alg. 7 for every (face, slice): v = raw - prevcoef * prev, CGS2 against the
// first nb basis vectors, normalize, store as basis vector nb.  Basis of (f, c): Bas + ((f*p + c)
// * ld_basis) with vectors of length len and stride len.  coef_prev / coef_out: (f, c) arrays of
// real scalars (z_i / c_i).  raw: result of the big product (face f, slice c at raw + f*sRaw + c*len).
template <typename T>
__global__ void __launch_bounds__(GKB_THREADS)
k_gkb_orth(const cplx<T>* __restrict__ raw, int64_t sRaw, cplx<T>* __restrict__ Bas, int64_t ld_basis, int len,
           int nb, const cplx<T>* __restrict__ prev, int64_t ld_prev, int prev_idx, const double* __restrict__ coef_prev,
           double* __restrict__ coef_out, int p, double tol) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  const int f = blockIdx.y, c = blockIdx.x;
  double* red = reinterpret_cast<double*>(smem_raw);              // 32 doubles
  zd* h = reinterpret_cast<zd*>(smem_raw + 32 * sizeof(double));  // nb coefficients
  cplx<T>* bas = Bas + ((int64_t)f * p + c) * ld_basis;
  const int per = (len + blockDim.x - 1) / blockDim.x;             // rows per thread (<= 8)
  zd v[8];
  const double cp = coef_prev ? coef_prev[(int64_t)f * p + c] : 0.0;
  const cplx<T>* pv = prev ? prev + ((int64_t)f * p + c) * ld_prev + (int64_t)prev_idx * len : nullptr;
#pragma unroll
  for (int t = 0; t < 8; ++t) {
    const int i = threadIdx.x + t * blockDim.x;
    zd x = mk(0.0, 0.0);
    if (t < per && i < len) {
      x = ld<double>(raw[(int64_t)f * sRaw + (int64_t)c * len + i]);
      if (pv) x = csub(x, cscale(ld<double>(pv[i]), cp));
    }
    v[t] = x;
  }
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nw = blockDim.x >> 6;
  double n0 = 0.0;
#pragma unroll
  for (int t = 0; t < 8; ++t) n0 += cabs2(v[t]);
  n0 = sqrt(gkb_block_sum(n0, red));
  for (int pass = 0; pass < 2; ++pass) {
    if (nb == 0) break;
    // h_j = b_j^H v for all j < nb: stage v in LDS (after the coefficients), one wave per j
    zd* vs = h + nb;
#pragma unroll
    for (int t = 0; t < 8; ++t) {
      const int i = threadIdx.x + t * blockDim.x;
      if (t < per && i < len) vs[i] = v[t];
    }
    __syncthreads();
    for (int j = wave; j < nb; j += nw) {
      const cplx<T>* bj = bas + (int64_t)j * len;
      double re = 0.0, im = 0.0;
      for (int i = lane; i < len; i += 64) {
        const zd b = ld<double>(bj[i]);
        const zd x = vs[i];
        re += b.re * x.re + b.im * x.im;
        im += b.re * x.im - b.im * x.re;
      }
      for (int o = 32; o > 0; o >>= 1) { re += __shfl_xor(re, o, 64); im += __shfl_xor(im, o, 64); }
      if (lane == 0) h[j] = mk(re, im);
    }
    __syncthreads();
#pragma unroll
    for (int t = 0; t < 8; ++t) {
      const int i = threadIdx.x + t * blockDim.x;
      if (t >= per || i >= len) continue;
      zd x = v[t];
      for (int j = 0; j < nb; ++j) x = csub(x, cmul(ld<double>(bas[(int64_t)j * len + i]), h[j]));
      v[t] = x;
    }
    __syncthreads();
  }
  double nn = 0.0;
#pragma unroll
  for (int t = 0; t < 8; ++t) nn += cabs2(v[t]);
  nn = sqrt(gkb_block_sum(nn, red));
  const bool ok = nn > tol * n0 && nn > 0.0;   // relative breakdown test (cancellation to rounding level)
  const double inv = ok ? 1.0 / nn : 0.0;
  cplx<T>* out = bas + (int64_t)nb * len;
#pragma unroll
  for (int t = 0; t < 8; ++t) {
    const int i = threadIdx.x + t * blockDim.x;
    if (t < per && i < len) st(out[i], cscale(v[t], inv));
  }
  if (threadIdx.x == 0) coef_out[(int64_t)f * p + c] = ok ? nn : 0.0;
}

// Givens update of the projected least-squares problem after step i (1-based), per (f, c):
// alpha = c_i, beta = z_{i+1}.  State: cprev (cosine of the previous rotation, -1 initially),
// phibar.  Records rho_i, s_i, phi_i (for the final back substitution) and the face residual.
__global__ void k_gkb_givens(const double* __restrict__ alpha, const double* __restrict__ beta, double* __restrict__ cprev,
                             double* __restrict__ phibar, double* __restrict__ rho_h, double* __restrict__ s_h,
                             double* __restrict__ phi_h, double* __restrict__ alpha_h, int kmax, int i, int count) {
  const int idx = blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= count) return;
  const double a = alpha[idx], b = beta[idx];
  const double rbar = -cprev[idx] * a;
  const double rho = sqrt(rbar * rbar + b * b);
  double c, s;
  if (rho > 0.0) { c = rbar / rho; s = b / rho; } else { c = 0.0; s = 1.0; }
  const double pb = phibar[idx];
  rho_h[(int64_t)idx * kmax + i - 1] = rho;
  s_h[(int64_t)idx * kmax + i - 1] = s;
  phi_h[(int64_t)idx * kmax + i - 1] = c * pb;
  alpha_h[(int64_t)idx * kmax + i - 1] = a;
  phibar[idx] = s * pb;
  cprev[idx] = c;
}

// discrepancy check after step i: one thread per slice c, sums over faces in a fixed order
__global__ void k_gkb_dp(const double* __restrict__ phibar, int F, int p, int n, const double* __restrict__ bound,
                         int i, int kmax, int* __restrict__ kout, double* __restrict__ resid, int* __restrict__ remaining) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= p) return;
  double tot = 0.0;
  for (int f = 0; f < F; ++f) {
    const double w = (f == 0 || 2 * f == n) ? 1.0 : 2.0;
    const double v = phibar[(int64_t)f * p + c];
    tot += w * v * v;
  }
  const double r = sqrt(tot / (double)n);
  if (resid) resid[(int64_t)c * kmax + i - 1] = r;
  if (kout[c] == 0 && r <= bound[c]) {
    kout[c] = i;
    atomicSub(remaining, 1);
  }
}

// final solution per (f, c): k = k_c (k_max if unmet), y = R^{-1} f (R upper bidiagonal:
// diag rho_j, super theta_{j+1} = s_j alpha_{j+1}), X-hat = W_k y.  One block per (c, f).
template <typename T>
__global__ void __launch_bounds__(256)
k_gkb_solution(const cplx<T>* __restrict__ Wb, int64_t ld_basis, int m, const int* __restrict__ kout, int kmax, int p,
               const double* __restrict__ rho_h, const double* __restrict__ s_h, const double* __restrict__ phi_h,
               const double* __restrict__ alpha_h, cplx<T>* __restrict__ Xh) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  double* y = reinterpret_cast<double*>(smem_raw);
  const int c = blockIdx.x, f = blockIdx.y;
  const int idx = f * p + c;
  int k = kout[c];
  if (k <= 0) k = kmax;
  if (threadIdx.x == 0) {
    const double* rh = rho_h + (int64_t)idx * kmax;
    const double* sh = s_h + (int64_t)idx * kmax;
    const double* ph = phi_h + (int64_t)idx * kmax;
    const double* ah = alpha_h + (int64_t)idx * kmax;
    double ynext = 0.0;
    for (int j = k - 1; j >= 0; --j) {      // 0-based j <-> step j+1
      const double theta = (j + 1 < k) ? sh[j] * ah[j + 1] : 0.0;
      const double yj = rh[j] > 0.0 ? (ph[j] - theta * ynext) / rh[j] : 0.0;
      y[j] = yj;
      ynext = yj;
    }
  }
  __syncthreads();
  const cplx<T>* W = Wb + (int64_t)idx * ld_basis;
  for (int i = threadIdx.x; i < m; i += blockDim.x) {
    zd acc = mk(0.0, 0.0);
    for (int j = 0; j < k; ++j) acc = cadd(acc, cscale(ld<double>(W[(int64_t)j * m + i]), y[j]));
    Xh[(int64_t)f * m * p + (int64_t)c * m + i] = mk((T)acc.re, (T)acc.im);
  }
}

// initial normalization: q_1 = b-hat / ||b-hat||, z_1 = ||b-hat|| per (f, c); phibar = z_1
template <typename T>
__global__ void __launch_bounds__(256)
k_gkb_init(const cplx<T>* __restrict__ Bh, int l, int p, cplx<T>* __restrict__ Qb, int64_t ld_basis,
           double* __restrict__ z1, double* __restrict__ phibar, double* __restrict__ cprev, double tol) {
  __shared__ double red[32];
  const int c = blockIdx.x, f = blockIdx.y;
  const cplx<T>* b = Bh + (int64_t)f * l * p + (int64_t)c * l;
  double nn = 0.0;
  for (int i = threadIdx.x; i < l; i += blockDim.x) nn += cabs2(ld<double>(b[i]));
  for (int o = 32; o > 0; o >>= 1) nn += __shfl_xor(nn, o, 64);
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  if (lane == 0) red[w] = nn;
  __syncthreads();
  double s = 0.0;
  for (int i = 0; i < (int)(blockDim.x >> 6); ++i) s += red[i];
  const double z = sqrt(s);
  const bool ok = z > tol;
  const double inv = ok ? 1.0 / z : 0.0;
  cplx<T>* q = Qb + ((int64_t)f * p + c) * ld_basis;
  for (int i = threadIdx.x; i < l; i += blockDim.x) st(q[i], cscale(ld<double>(b[i]), inv));
  if (threadIdx.x == 0) {
    z1[(int64_t)f * p + c] = ok ? z : 0.0;
    phibar[(int64_t)f * p + c] = z;   // the residual of X = 0 is ||b-hat|| even on a zero face
    cprev[(int64_t)f * p + c] = -1.0;
  }
}

// k_out = k per slice (k_max where the principle was not met), status
__global__ void k_gkb_finish(const int* __restrict__ kin, int p, int kmax, int* __restrict__ kout, int* __restrict__ status) {
  __shared__ int fail_any;
  if (threadIdx.x == 0) fail_any = 0;
  __syncthreads();
  for (int c = threadIdx.x; c < p; c += blockDim.x) {
    const int k = kin[c];
    if (k <= 0) atomicOr(&fail_any, 1);
    kout[c] = k > 0 ? k : kmax;
  }
  __syncthreads();
  if (threadIdx.x == 0 && status) *status = fail_any ? RTSVD_W_DP_NOT_MET : RTSVD_OK;
}

}  // namespace rt
