// Per-face dense kernels on r x r Hermitian matrices, FP64 (one workgroup per Fourier face).
//
//  * k_chol_inv: G = L L^H (Cholesky, right-looking) and Rinv = L^{-H}, so that for G = Y^H Y
//    the product Y Rinv has orthonormal columns with a real positive R diagonal -- the Q of the
//    QR factorization Alg. 6 builds by per-face normalization and re-orthogonalization.  A pivot
//    at or below `tol` marks a column linearly dependent on the previous ones (Alg. 3's
//    breakdown); its Q column is set to zero and the face is flagged.
//  * k_jacobi_eig: cyclic two-sided Jacobi eigensolver with the parallel round-robin ordering
//    (r/2 disjoint rotations per round), eigenvalues sorted in descending order.  Applied to
//    G = C C^H it gives C = U-breve diag(sigma) V^H with sigma = sqrt(lambda).
//
// Matrices live in global memory (column-major, ld = r, one r x r block per face); a face's
// working set stays in L2.
#pragma once
#include "common.hpp"

namespace rt {

constexpr int SMALL_THREADS = 1024;

__global__ void __launch_bounds__(256)
k_chol_inv(zd* __restrict__ G, zd* __restrict__ Rinv, int r, double tol_rel, int* __restrict__ flags) {
  const int f = blockIdx.x;
  zd* g = G + (int64_t)f * r * r;
  zd* x = Rinv + (int64_t)f * r * r;
  __shared__ double piv;
  __shared__ double tol;
  __shared__ int bad;
  if (threadIdx.x == 0) {
    double mx = 0.0;
    for (int j = 0; j < r; ++j) mx = fmax(mx, g[j + j * r].re);
    tol = tol_rel * mx;
    bad = 0;
  }
  __syncthreads();
  // right-looking Cholesky on the lower triangle
  for (int j = 0; j < r; ++j) {
    if (threadIdx.x == 0) {
      const double d = g[j + j * r].re;
      if (d > tol && d > 0.0) piv = sqrt(d); else { piv = 0.0; bad = 1; }
      g[j + j * r] = mk(piv, 0.0);
    }
    __syncthreads();
    const double p = piv;
    for (int i = j + 1 + threadIdx.x; i < r; i += blockDim.x) {
      zd v = g[i + j * r];
      g[i + j * r] = (p > 0.0) ? cscale(v, 1.0 / p) : mk(0.0, 0.0);
    }
    __syncthreads();
    const int w = r - j - 1;  // trailing size
    for (int idx = threadIdx.x; idx < w * w; idx += blockDim.x) {
      const int i = j + 1 + idx % w, c = j + 1 + idx / w;
      if (c <= i) {
        const zd li = g[i + j * r], lc = g[c + j * r];
        g[i + c * r] = csub(g[i + c * r], cmul(li, cconj(lc)));
      }
    }
    __syncthreads();
  }
  // X = L^{-1}, one thread per column, stored in the lower triangle of x
  for (int j = threadIdx.x; j < r; j += blockDim.x) {
    const double ljj = g[j + j * r].re;
    x[j + j * r] = mk(ljj > 0.0 ? 1.0 / ljj : 0.0, 0.0);
    for (int i = j + 1; i < r; ++i) {
      const double lii = g[i + i * r].re;
      zd s = mk(0.0, 0.0);
      for (int k = j; k < i; ++k) s = cadd(s, cmul(g[i + k * r], x[k + j * r]));
      x[i + j * r] = lii > 0.0 ? cscale(s, -1.0 / lii) : mk(0.0, 0.0);
    }
  }
  __syncthreads();
  // Rinv = X^H (upper triangular) in place
  for (int idx = threadIdx.x; idx < r * r; idx += blockDim.x) {
    const int i = idx % r, j = idx / r;
    if (i > j) {
      const zd lo = x[i + j * r];
      x[j + i * r] = cconj(lo);
      x[i + j * r] = mk(0.0, 0.0);
    } else if (i == j) {
      x[i + i * r].im = 0.0;
    }
  }
  if (threadIdx.x == 0 && flags && bad) atomicOr(flags, 1);
}

// Jacobi eigensolver: G (r x r Hermitian, overwritten), U (r x r, out: eigenvectors as columns,
// sorted by descending eigenvalue), lam (r, out: eigenvalues, descending).
__global__ void __launch_bounds__(SMALL_THREADS)
k_jacobi_eig(zd* __restrict__ G, zd* __restrict__ U, double* __restrict__ lam, int r, int max_sweeps) {
  const int f = blockIdx.x;
  zd* g = G + (int64_t)f * r * r;
  zd* u = U + (int64_t)f * r * r;
  double* lf = lam + (int64_t)f * r;
  __shared__ int arr[258];
  __shared__ double rc[129];
  __shared__ zd rs[129];
  __shared__ int rp[129], rq[129];
  __shared__ int nrot;
  const int P = (r + 1) / 2, R2 = 2 * P;
  for (int idx = threadIdx.x; idx < r * r; idx += blockDim.x) {
    const int i = idx % r, j = idx / r;
    u[idx] = mk(i == j ? 1.0 : 0.0, 0.0);
  }
  for (int i = threadIdx.x; i < R2; i += blockDim.x) arr[i] = i;
  __syncthreads();
  const double small = 8.67e-19;  // 2^-60: below FP64 rounding, so sweeps run to full accuracy
  for (int sweep = 0; sweep < max_sweeps; ++sweep) {
    if (threadIdx.x == 0) nrot = 0;
    __syncthreads();
    for (int round = 0; round < R2 - 1; ++round) {
      // 1. rotation parameters for the disjoint pairs of this round
      for (int k = threadIdx.x; k < P; k += blockDim.x) {
        int p = arr[k], q = arr[R2 - 1 - k];
        if (p > q) { int t = p; p = q; q = t; }
        rp[k] = p; rq[k] = q;
        rc[k] = 1.0; rs[k] = mk(0.0, 0.0);
        if (q < r) {
          const double a = g[p + p * r].re, b = g[q + q * r].re;
          const zd gpq = g[p + q * r];
          const double h = sqrt(cabs2(gpq));
          if (h > 0.0 && h > small * sqrt(fabs(a) * fabs(b))) {
            const double zeta = (b - a) / (2.0 * h);
            const double t = (zeta >= 0.0 ? 1.0 : -1.0) / (fabs(zeta) + sqrt(1.0 + zeta * zeta));
            const double c = 1.0 / sqrt(1.0 + t * t);
            const double s = t * c;
            rc[k] = c;
            rs[k] = cscale(gpq, s / h);  // sigma = s e^{i phi}
            atomicAdd(&nrot, 1);
          }
        }
      }
      __syncthreads();
      // 2. rows p, q of G:  G'[p][x] = c G[p][x] - sigma G[q][x];  G'[q][x] = conj(sigma) G[p][x] + c G[q][x]
      for (int idx = threadIdx.x; idx < P * r; idx += blockDim.x) {
        const int k = idx % P, x = idx / P;
        const int p = rp[k], q = rq[k];
        if (q >= r || (rs[k].re == 0.0 && rs[k].im == 0.0)) continue;
        const double c = rc[k]; const zd sg = rs[k];
        const zd gp = g[p + x * r], gq = g[q + x * r];
        g[p + x * r] = csub(cscale(gp, c), cmul(sg, gq));
        g[q + x * r] = cadd(cmulc(sg, gp), cscale(gq, c));
      }
      __syncthreads();
      // 3. columns p, q of G and U:  G[x][p] = c G[x][p] - conj(sigma) G[x][q];  G[x][q] = sigma G[x][p] + c G[x][q]
      for (int idx = threadIdx.x; idx < P * r; idx += blockDim.x) {
        const int k = idx % P, x = idx / P;
        const int p = rp[k], q = rq[k];
        if (q >= r || (rs[k].re == 0.0 && rs[k].im == 0.0)) continue;
        const double c = rc[k]; const zd sg = rs[k];
        zd gp = g[x + p * r], gq = g[x + q * r];
        g[x + p * r] = csub(cscale(gp, c), cmulc(sg, gq));
        g[x + q * r] = cadd(cmul(sg, gp), cscale(gq, c));
        gp = u[x + p * r]; gq = u[x + q * r];
        u[x + p * r] = csub(cscale(gp, c), cmulc(sg, gq));
        u[x + q * r] = cadd(cmul(sg, gp), cscale(gq, c));
      }
      __syncthreads();
      // 4. exact zeros in the rotated positions, real diagonal
      for (int k = threadIdx.x; k < P; k += blockDim.x) {
        const int p = rp[k], q = rq[k];
        if (q >= r || (rs[k].re == 0.0 && rs[k].im == 0.0)) continue;
        g[p + q * r] = mk(0.0, 0.0);
        g[q + p * r] = mk(0.0, 0.0);
        g[p + p * r].im = 0.0;
        g[q + q * r].im = 0.0;
      }
      // 5. next round-robin arrangement: position 0 fixed, the others rotate by one
      __syncthreads();
      if (threadIdx.x == 0) {
        const int last = arr[R2 - 1];
        for (int i = R2 - 1; i > 1; --i) arr[i] = arr[i - 1];
        arr[1] = last;
      }
      __syncthreads();
    }
    const int done = (nrot == 0);
    __syncthreads();
    if (done) break;
  }
  // sort eigenvalues in descending order (stable by index); G's storage takes a copy of U
  __shared__ double ev[256];
  __shared__ int perm[256];
  for (int i = threadIdx.x; i < r; i += blockDim.x) ev[i] = g[i + i * r].re;
  __syncthreads();
  for (int idx = threadIdx.x; idx < r * r; idx += blockDim.x) g[idx] = u[idx];
  for (int i = threadIdx.x; i < r; i += blockDim.x) {
    int rank = 0;
    for (int j = 0; j < r; ++j) rank += (ev[j] > ev[i]) || (ev[j] == ev[i] && j < i);
    perm[rank] = i;
    lf[rank] = ev[i];
  }
  __syncthreads();
  for (int idx = threadIdx.x; idx < r * r; idx += blockDim.x) {
    const int x = idx % r, c = idx / r;
    u[x + c * r] = g[x + perm[c] * r];
  }
}

}  // namespace rt
