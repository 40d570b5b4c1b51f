// Truncated pseudo-inverse coefficients and the discrepancy principle (eq. (disp), eq. (kinit)).
//
// Per face f: T_f = diag(1/sigma_f) U-breve_f^H Q_f^H B-hat_f (r x p, FP64).  The residual of
// the k-term solution is, by Parseval over the half spectrum,
//     rho_k^2 = (1/n) sum_f w_f || B-hat_f - W_f[:, :k] T_f[:k, :] ||_F^2,   W_f = A-hat_f V_f,
// with w_f = 1 for the self-conjugate faces (0 and n/2) and 2 otherwise -- the exact
// ||B - A * X_k||_F^2 (no approximation of A).  k_dp_partial forms the per-face, per-row-tile
// sums for every k in one pass (the residual is updated one rank-1 term at a time), k_dp_select
// reduces them over faces in a fixed order (deterministic) and picks the first k >= k_start
// with rho_k <= eta * delta.
#pragma once
#include "common.hpp"

namespace rt {

constexpr int DP_ROWS = 64;        // rows per block (one wave) of the residual pass
// residual orders per chunk of the residual pass (columns of W loaded at once, rows of the LDS
// transposition): two chunks of W in registers stay within 256 VGPRs, and the 16.6 KB (FP32 W) /
// 8.3 KB (FP64 W) of LDS let one round of waves cover 65 faces x 16 row tiles
template <typename TW> constexpr int dp_kch() { return sizeof(TW) <= 8 ? 32 : 16; }
constexpr int DP_SEL_THREADS = 1024;
constexpr int HEEV_RMAX_SOLVE = 256;  // largest r (the eigensolver's limit)

// T = diag(sigma)^+ E: rows divided by the singular values; a singular value at or below
// rel * sigma_max, sigma_max the largest over all faces (sigma[f * r] is face f's largest), counts
// as zero and its row is zeroed (numerical rank of the pseudo-inverse of the block-diagonal Fourier
// form of A; this also drops dependent sketch columns and faces of A that are zero up to rounding).
// Launched with 256 threads per block.
__global__ void __launch_bounds__(256) k_scale_rows(zd* __restrict__ T, const double* __restrict__ sigma, int r, int p,
                                                    int F, double rel) {
  __shared__ double red[4];
  double mx = 0.0;
  for (int f = threadIdx.x; f < F; f += blockDim.x) mx = fmax(mx, sigma[(int64_t)f * r]);
  for (int o = 32; o > 0; o >>= 1) mx = fmax(mx, __shfl_xor(mx, o, 64));
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = mx;
  __syncthreads();
  const double cut = rel * fmax(fmax(red[0], red[1]), fmax(red[2], red[3]));
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t total = (int64_t)F * r * p;
  if (idx >= total) return;
  const int j = (int)(idx % r);
  const int64_t f = idx / ((int64_t)r * p);
  const double s = sigma[f * r + j];
  T[idx] = s > cut ? cscale(T[idx], 1.0 / s) : mk(0.0, 0.0);
}

// partial[((f * tiles + tile) * pg + g) * kcap + (k-1)] = sum over the tile's rows and over the
// columns c of column group g (columns g*CPB .. g*CPB + CPB - 1 that exist; pg = ceil(p / CPB)) of
// |B-hat - W[:, :k] T[:k, c]|^2, FP64.  Block = one wave = one 64-row tile of one column group.
// The residuals are updated one rank-1 term at a time (each W entry is loaded once for the CPB
// columns); the 64 row values of each order k are summed through an LDS transposition (lane kk
// sums row kk of a KCH x 64 chunk), so there is no per-order cross-lane reduction chain.  The W
// columns of the next chunk are loaded while the current chunk is applied.  CPB = 1 keeps one
// column per partial (per-slice discrepancy principle); a joint principle sums every column and
// may take CPB = 8.
template <int CPB, typename TBh, typename TW>
__global__ void __launch_bounds__(DP_ROWS)
k_dp_partial(const TBh* __restrict__ Bh, const TW* __restrict__ W, const zd* __restrict__ T,
             int l, int p, int r, int kcap, double* __restrict__ partial) {
  constexpr int KCH = dp_kch<TW>();
  const int tile = blockIdx.x, g = blockIdx.y, f = blockIdx.z;
  const int tiles = gridDim.x, pg = gridDim.y;
  const int lane = threadIdx.x;
  const int row = tile * DP_ROWS + lane;
  const int c0 = g * CPB;
  __shared__ double sq[KCH][DP_ROWS + 1];
  const bool on = row < l;
  zd R[CPB];
#pragma unroll
  for (int j = 0; j < CPB; ++j) {
    R[j] = mk(0.0, 0.0);
    if (on && c0 + j < p) R[j] = ld<double>(Bh[(int64_t)f * l * p + (int64_t)(c0 + j) * l + row]);
  }
  const TW* __restrict__ wf = W + (int64_t)f * l * r + (on ? row : 0);
  const zd* __restrict__ tf = T + (int64_t)f * r * p;
  double* __restrict__ out = partial + (((int64_t)f * tiles + tile) * pg + g) * kcap;
  // two register chunks of W, used in turn: the next chunk's loads are issued before the current
  // chunk is applied (column indices clamp to kcap - 1: loads past the last order are re-reads
  // that are never applied)
  auto load = [&](TW (&w)[KCH], int kb) {
#pragma unroll
    for (int u = 0; u < KCH; ++u) w[u] = wf[(int64_t)min(kb + u, kcap - 1) * l];
  };
  auto apply = [&](const TW (&w)[KCH], int k0) {
    const int kn = min(KCH, kcap - k0);
#pragma unroll
    for (int u = 0; u < KCH; ++u) {
      if (u < kn) {                                // uniform
        const int k = k0 + u;                      // order k+1 uses column k
        const zd wk = ld<double>(w[u]);
        double acc = 0.0;
#pragma unroll
        for (int j = 0; j < CPB; ++j) {
          const zd t = (c0 + j < p) ? tf[(int64_t)(c0 + j) * r + k] : mk(0.0, 0.0);
          R[j] = csub(R[j], cmul(wk, t));
          acc += cabs2(R[j]);
        }
        sq[u][lane] = on ? acc : 0.0;
      }
    }
    __syncthreads();
    if (lane < kn) {
      double s = 0.0;
#pragma unroll 8
      for (int i = 0; i < DP_ROWS; ++i) s += sq[lane][i];
      out[k0 + lane] = s;
    }
    __syncthreads();
  };
  TW wa[KCH], wb[KCH];
  load(wa, 0);
  for (int k0 = 0; k0 < kcap; k0 += 2 * KCH) {
    if (k0 + KCH < kcap) load(wb, k0 + KCH);
    apply(wa, k0);
    if (k0 + KCH >= kcap) break;
    if (k0 + 2 * KCH < kcap) load(wa, k0 + 2 * KCH);
    apply(wb, k0 + KCH);
  }
}

// rho_k^2 = (1/n) sum_f w_f sum_{tiles, columns of the group} partial: one 256-thread workgroup
// per (group, k) (grid groups * kcap), summed in a fixed order (deterministic).
constexpr int DP_RHO_THREADS = 256;
__global__ void __launch_bounds__(DP_RHO_THREADS)
k_dp_rho(const double* __restrict__ partial, int F, int tiles, int p, int kcap, int n, int groups,
         double* __restrict__ resid_out, double* __restrict__ rho_tmp) {
  __shared__ double red[DP_RHO_THREADS / 64];
  const int idx = blockIdx.x;
  const int g = idx / kcap, k = idx % kcap;
  // p: partial columns per tile (column groups of the joint principle, or the slices)
  const int c0 = groups == 1 ? 0 : g, nc = groups == 1 ? p : 1;
  const int cnt = F * tiles;
  double s = 0.0;
#pragma unroll 4
  for (int e = threadIdx.x; e < cnt; e += DP_RHO_THREADS) {
    const int fi = e / tiles, t = e - fi * tiles;
    const double w = (fi == 0 || 2 * fi == n) ? 1.0 : 2.0;
    const double* pp = partial + (((int64_t)fi * tiles + t) * p + c0) * kcap + k;
    double v = 0.0;
    for (int c = 0; c < nc; ++c) v += pp[(int64_t)c * kcap];
    s += w * v;
  }
  s = wave_sum(s);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) {
    double t = 0.0;
#pragma unroll
    for (int w = 0; w < DP_RHO_THREADS / 64; ++w) t += red[w];
    const double q = t / (double)n;
    const double rho = q < 0.0 ? 0.0 : sqrt(q);     // a NaN sum stays NaN (fmax would drop it)
    rho_tmp[idx] = rho;
    if (resid_out) resid_out[idx] = rho;
  }
}

// The first k >= k_start with rho_k <= eta delta of each group (one block; k_start >= 1).  One
// wave per group: its lanes test 64 consecutive orders at once and the lowest lane that meets
// the bound gives k, so a group costs one load round per 64 orders.  bound_args holds the bounds
// when groups <= 16 (then `bound` may be null), else they are read from `bound`.
constexpr int DP_SELECT_THREADS = 256;
__global__ void __launch_bounds__(DP_SELECT_THREADS)
k_dp_select(int kcap, int groups, const double* __restrict__ bound /* eta*delta per group */, Vals16 bound_args,
            int k_start, const double* __restrict__ rho_tmp, const int* __restrict__ fflags, int* __restrict__ k_out,
            int* __restrict__ status_out) {
  __shared__ int any_fail, non_finite;
  if (threadIdx.x == 0) {
    any_fail = 0;
    non_finite = (fflags && (*fflags & 2)) ? 1 : 0;
  }
  __syncthreads();
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nw = (int)blockDim.x >> 6;
  for (int g = wave; g < groups; g += nw) {
    const double b = groups <= 16 ? bound_args.v[g] : bound[g];
    // a non-finite residual (B, or the factor, not finite) fails every test below and is reported
    bool bad = false;
    for (int k = 1 + lane; k <= kcap; k += 64) bad |= !isfinite(rho_tmp[(int64_t)g * kcap + k - 1]);
    if (__ballot(bad) && lane == 0) atomicOr(&non_finite, 1);
    int kk = -1;
    for (int k0 = k_start; k0 <= kcap && kk < 0; k0 += 64) {
      const int k = k0 + lane;
      const bool ok = k <= kcap && rho_tmp[(int64_t)g * kcap + k - 1] <= b;
      const unsigned long long hit = __ballot(ok);
      if (hit) kk = k0 + __builtin_ctzll(hit);
    }
    if (kk < 0) {
      kk = kcap;
      if (lane == 0) atomicOr(&any_fail, 1);
    }
    if (lane == 0) k_out[g] = kk;
  }
  __syncthreads();
  if (threadIdx.x == 0 && status_out)
    *status_out = non_finite ? RTSVD_E_NOTFINITE : (any_fail ? RTSVD_W_DP_NOT_MET : RTSVD_OK);
}

// T'[f][j][c] = T[f][j][c] if j < k of column c's group, else 0
__global__ void k_mask_coeffs(const zd* __restrict__ T, zd* __restrict__ Tm, const int* __restrict__ k_of,
                              int groups, int r, int p, int F) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t total = (int64_t)F * r * p;
  if (idx >= total) return;
  const int j = (int)(idx % r);
  const int c = (int)((idx / r) % p);
  const int k = k_of[groups == 1 ? 0 : c];
  Tm[idx] = j < k ? T[idx] : mk(0.0, 0.0);
}

// eta[j] = ||A||^2 - (1/n) sum_f w_f sum_{j' < j} rown[f][j'],  j = 0..r  (one block of
// DP_SEL_THREADS; fixed summation order).  rown[f][j] = rn[f * sf + j * sj] (the squared row norms
// of C_f: the real diagonal of its Gram matrix, or the eigenvalues of A-hat_f^H A-hat_f).
__global__ void __launch_bounds__(DP_SEL_THREADS)
k_eta_prefix(const double* __restrict__ sumsq, int64_t nsumsq, const double* __restrict__ rn, int64_t sf, int64_t sj,
             int F, int r, int n, double* __restrict__ eta) {
  __shared__ double red[DP_SEL_THREADS / 64];
  __shared__ double rows[HEEV_RMAX_SOLVE];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  double s = 0.0;
  // unrolled so that each lane's loads are all in flight together (same summation order)
#pragma unroll 8
  for (int64_t i = threadIdx.x; i < nsumsq; i += blockDim.x) s += sumsq[i];
  s = wave_sum(s);
  if (lane == 0) red[wave] = s;
  // row sums over the faces: 8 lanes per row j (faces f = sub, sub + 8, ...), all loads of a lane
  // independent, then a fixed-order 8-lane tree
  const int sub = threadIdx.x & 7, jl = threadIdx.x >> 3, per = (int)blockDim.x >> 3;
  for (int j0 = 0; j0 < r; j0 += per) {
    const int j = j0 + jl;
    double t = 0.0;
    if (j < r) {
#pragma unroll 9
      for (int f = sub; f < F; f += 8) t += ((f == 0 || 2 * f == n) ? 1.0 : 2.0) * rn[(int64_t)f * sf + (int64_t)j * sj];
    }
    t += dpp<DPP_XOR1>(t);
    t += dpp<DPP_XOR2>(t);
    t += __shfl_xor(t, 4, 64);
    if (sub == 0 && j < r) rows[j] = t / (double)n;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double e = 0.0;
    for (int w = 0; w < (int)(blockDim.x >> 6); ++w) e += red[w];
    eta[0] = e;
    for (int j = 0; j < r; ++j) { e -= rows[j]; eta[j + 1] = e; }
  }
}

// Out_f[:, j] = In_f[:, j] / sigma_f[j]  (zero column when sigma is zero); In and Out may alias
template <typename TI, typename TO>
__global__ void k_scale_cols(const TI* In, TO* Out, const double* __restrict__ sigma,
                             int rows, int r, int F) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t total = (int64_t)F * rows * r;
  if (idx >= total) return;
  const int j = (int)((idx / rows) % r);
  const int64_t f = idx / ((int64_t)rows * r);
  const double s = sigma[f * r + j];
  st(Out[idx], s > 0.0 ? cscale(ld<double>(In[idx]), 1.0 / s) : mk(0.0, 0.0));
}

// sigma = sqrt(max(lambda, 0)), with eigenvalues at or below tol_rel * lambda_max set to zero
__global__ void k_sqrt_eigs(const double* __restrict__ lam, double* __restrict__ sigma, int r, int F, double tol_rel) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (int64_t)F * r) return;
  const int64_t f = idx / r;
  const double lmax = lam[f * r];
  const double l = lam[idx];
  sigma[idx] = (l > tol_rel * lmax && l > 0.0) ? sqrt(l) : 0.0;
}

// Xq = tril(M, -1) - tril(M, -1)^H + i Im diag(M)   (r x r per face)
__global__ void k_skew_lower(const zd* __restrict__ M, zd* __restrict__ Xq, int r, int F) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (int64_t)F * r * r) return;
  const int i = (int)(idx % r), j = (int)((idx / r) % r);
  const int64_t base = idx - i - (int64_t)j * r;
  zd v;
  if (i > j) v = M[idx];
  else if (i < j) v = cscale(cconj(M[base + j + (int64_t)i * r]), -1.0);
  else v = mk(0.0, M[idx].im);
  Xq[idx] = v;
}

// E <- Phi o E with Phi_jl = -1/(l_j l_l) (j,l < k), 1/(l_j (l_j - l_l)) (j < k <= l),
// 1/(l_l (l_l - l_j)) (l < k <= j), 0 otherwise; lam descending per face
__global__ void k_phi_hadamard(zd* __restrict__ E, const double* __restrict__ lam, int r, int k, int F) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (int64_t)F * r * r) return;
  const int j = (int)(idx % r), l = (int)((idx / r) % r);
  const int64_t f = idx / ((int64_t)r * r);
  const double lj = lam[f * r + j], ll = lam[f * r + l];
  double ph = 0.0;
  if (j < k && l < k) ph = -1.0 / (lj * ll);
  else if (j < k && l >= k) ph = 1.0 / (lj * (lj - ll));
  else if (l < k && j >= k) ph = 1.0 / (ll * (ll - lj));
  E[idx] = cscale(E[idx], ph);
}

// Uphi = U diag(phi), phi_j = 1/lam_j for j < k, else 0
__global__ void k_scale_inv_eigs(const zd* __restrict__ U, zd* __restrict__ Uphi, const double* __restrict__ lam, int r,
                                 int k, int F) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (int64_t)F * r * r) return;
  const int j = (int)((idx / r) % r);
  const int64_t f = idx / ((int64_t)r * r);
  const double lj = lam[f * r + j];
  Uphi[idx] = (j < k && lj > 0.0) ? cscale(U[idx], 1.0 / lj) : mk(0.0, 0.0);
}

// Weighted real inner product over the half spectrum, (1/n) sum_f w_f Re <G_f, D_f> (w_f = 1 for
// faces 0 and n/2, else 2), in two fixed-order passes: k_weighted_inner_part gives every workgroup a
// contiguous run of the F x per_face elements (WI_ITEMS per thread), k_sum_partials adds the
// workgroup sums in order.
constexpr int WI_THREADS = 256;
constexpr int WI_ITEMS = 16;
template <typename TG>
__global__ void __launch_bounds__(WI_THREADS)
k_weighted_inner_part(const TG* __restrict__ G, const zd* __restrict__ D, int64_t per_face, int F, int n,
                      double* __restrict__ part) {
  __shared__ double red[WI_THREADS / 64];
  const int64_t total = (int64_t)F * per_face;
  const int64_t base = (int64_t)blockIdx.x * WI_THREADS * WI_ITEMS;
  double s = 0.0;
#pragma unroll 4
  for (int it = 0; it < WI_ITEMS; ++it) {
    const int64_t i = base + (int64_t)it * WI_THREADS + threadIdx.x;
    if (i < total) {
      const int f = (int)(i / per_face);
      const double w = (f == 0 || 2 * f == n) ? 1.0 : 2.0;
      const zd g = ld<double>(G[i]);
      const zd d = D[i];
      s += w * (g.re * d.re + g.im * d.im);
    }
  }
  s = wave_sum(s);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) {
    double t = 0.0;
    for (int w = 0; w < WI_THREADS / 64; ++w) t += red[w];
    part[blockIdx.x] = t;
  }
}

// out[0] = scale * sum of part[0 .. count) in a fixed order (one workgroup of 256 threads)
__global__ void __launch_bounds__(256) k_sum_partials(const double* __restrict__ part, int64_t count, double scale,
                                                      double* __restrict__ out) {
  __shared__ double red[4];
  double s = 0.0;
  for (int64_t i = threadIdx.x; i < count; i += blockDim.x) s += part[i];
  s = wave_sum(s);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) out[0] = scale * (((red[0] + red[1]) + red[2]) + red[3]);
}

}  // namespace rt
