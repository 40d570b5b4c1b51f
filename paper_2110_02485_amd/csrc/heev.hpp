// Hermitian eigensolver and Cholesky inverse for the r x r per-face matrices, FP64, one
// workgroup (1024 threads) per Fourier face.  The Hermitian matrix is held as a packed lower
// triangle (column-major: column j holds rows j..r-1 at offset j*r - j*(j-1)/2) in LDS when it
// fits, else in a global scratch slice; both are addressed through one generic pointer.
//
// k_heev:  G = Q_H T Q_H^H by Householder reflections (T real symmetric tridiagonal), eigenvalues
//          of T by multisection of Sturm counts (8 lanes per eigenvalue), eigenvectors of T by
//          inverse iteration with LU and partial pivoting (clusters re-orthogonalized by modified
//          Gram-Schmidt), eigenvectors of G = Q_H z.  Output sorted by descending eigenvalue.
//          Applied to G = C C^H it gives the small SVD C = U-breve diag(sigma) V^H of Alg. 6.
// k_cholinv: G = L L^H (right-looking Cholesky), in-place L^{-1}, output Rinv = L^{-H}: for
//          G = Y^H Y, Y Rinv has orthonormal columns and R = L^H has a real positive diagonal
//          (the per-face QR that Alg. 6 builds by normalization and re-orthogonalization).  A
//          pivot at or below tol_rel * max diag marks a dependent column: its row and column of
//          Rinv are zero and the face is flagged (Alg. 3's breakdown).
#pragma once
#include "common.hpp"

namespace rt {

constexpr int HEEV_THREADS = 1024;

#ifdef RTSVD_PHASE_CLOCKS
// phase timestamps of block 0 (profiling builds only)
__device__ unsigned long long rt_phase_clock[16];
#define RT_PHASE(i) do { __syncthreads(); if (blockIdx.x == 0 && threadIdx.x == 0) rt_phase_clock[i] = wall_clock64(); } while (0)
#else
#define RT_PHASE(i) do { } while (0)
#endif
constexpr int HEEV_RMAX = 256;

RT_HOST_DEVICE int64_t pk_off(int j, int r) { return (int64_t)j * r - ((int64_t)j * (j - 1)) / 2; }
RT_HOST_DEVICE int64_t packed_size(int r) { return (int64_t)r * (r + 1) / 2; }

// element (i, j) of the Hermitian matrix from its packed lower triangle
__device__ __forceinline__ zd pk_get(const zd* S, const int* cb, int i, int j) {
  if (i >= j) return S[cb[j] + (i - j)];
  return cconj(S[cb[i] + (j - i)]);
}

// reduce `v` over the 8 aligned lanes of a group
__device__ __forceinline__ double grp8_sum(double v) {
  v += __shfl_xor(v, 1, 64);
  v += __shfl_xor(v, 2, 64);
  v += __shfl_xor(v, 4, 64);
  return v;
}

// block-wide sum (all threads get the result); red has >= 17 doubles
__device__ double block_sum(double v, double* red) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  __syncthreads();
  if (lane == 0) red[w] = v;
  __syncthreads();
  if (threadIdx.x == 0) {
    double s = 0.0;
    for (int i = 0; i < (int)(blockDim.x >> 6); ++i) s += red[i];
    red[16] = s;
  }
  __syncthreads();
  return red[16];
}

// number of eigenvalues of the tridiagonal (d, e) strictly below x (Sturm sequence)
__device__ __forceinline__ int sturm_count(const double* d, const double* e2, int r, double x, double pivmin) {
  int cnt = 0;
  double q = d[0] - x;
  if (fabs(q) < pivmin) q = -pivmin;
  cnt += (q < 0.0);
  for (int i = 1; i < r; ++i) {
    q = (d[i] - x) - e2[i - 1] / q;
    if (fabs(q) < pivmin) q = -pivmin;
    cnt += (q < 0.0);
  }
  return cnt;
}

struct HeevLds {
  double d[HEEV_RMAX], e[HEEV_RMAX], e2[HEEV_RMAX], lam[HEEV_RMAX];
  zd tau[HEEV_RMAX], v[HEEV_RMAX], p[HEEV_RMAX];
  int cb[HEEV_RMAX + 1];      // packed column offsets
  int cstart[HEEV_RMAX + 1];  // cluster starts (eigenvalues closer than the cluster tolerance)
  int ncl;
  double acc[2], accre[2], accim[2];  // reduction accumulators, double-buffered by step parity
};

inline size_t heev_lds_bytes(int r, bool packed_in_lds) {
  return sizeof(HeevLds) + (packed_in_lds ? (size_t)packed_size(r) * sizeof(zd) : 0);
}

// 1/x with v_rcp_f64 refined by two Newton steps (full double precision for normal x)
__device__ __forceinline__ double inv_d(double x) {
  double y = __builtin_amdgcn_rcp(x);
  y = y * fma(-x, y, 2.0);
  y = y * fma(-x, y, 2.0);
  return y;
}

// number of eigenvalues of the tridiagonal (d, e) strictly below x (Sturm sequence)
__device__ __forceinline__ int sturm_count_fast(const double* d, const double* e2, int r, double x, double pivmin) {
  int cnt = 0;
  double q = d[0] - x;
  if (fabs(q) < pivmin) q = -pivmin;
  cnt += (q < 0.0);
  for (int i = 1; i < r; ++i) {
    q = (d[i] - x) - e2[i - 1] * inv_d(q);
    if (fabs(q) < pivmin) q = -pivmin;
    cnt += (q < 0.0);
  }
  return cnt;
}

constexpr int HEEV_UREG = 16;   // rows per lane of the register-resident back-transformation (r <= 128)

// G: F x r x r (full, column-major, only the lower triangle is read); U: F x r x r out;
// lam: F x r out (descending).  gpk: F x packed_size(r) global scratch (the reflectors; also the
// working matrix when !in_lds); zs: F x r x (r+1) doubles (eigenvectors of T when !in_lds);
// lu: F x r x 5r doubles (LU factors of T - lambda I).
__global__ void __launch_bounds__(HEEV_THREADS)
k_heev(const zd* __restrict__ Gin, int r, zd* __restrict__ Uout, double* __restrict__ lamout,
       zd* __restrict__ gpk, double* __restrict__ zs, double* __restrict__ lu, int in_lds) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  HeevLds& L = *reinterpret_cast<HeevLds*>(smem_raw);
  const int f = blockIdx.x;
  zd* S = in_lds ? reinterpret_cast<zd*>(smem_raw + sizeof(HeevLds)) : gpk + (int64_t)f * packed_size(r);
  zd* Sg = gpk + (int64_t)f * packed_size(r);
  const zd* G = Gin + (int64_t)f * r * r;
  zd* U = Uout + (int64_t)f * r * r;
  double* Z = zs + (int64_t)f * r * (r + 1);
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6, nw = blockDim.x >> 6;
  const int sub = tid & 7, grp = tid >> 3, ngrp = blockDim.x >> 3;

  RT_PHASE(0);
  for (int j = tid; j <= r; j += blockDim.x) L.cb[j] = (int)pk_off(j, r);
  if (tid < 2) { L.acc[tid] = 0.0; L.accre[tid] = 0.0; L.accim[tid] = 0.0; }
  // ---- load the lower triangle -----------------------------------------------------------
  for (int j = 0; j < r; ++j)
    for (int i = j + tid; i < r; i += blockDim.x) S[pk_off(j, r) + (i - j)] = G[i + (int64_t)j * r];
  __syncthreads();

  RT_PHASE(1);
  // ---- Householder tridiagonalization: 4 barriers per reflector ------------------------------
  for (int k = 0; k < r - 1; ++k) {
    const int par = k & 1;
    const int ck = L.cb[k];
    // (A) squared norm of the column below the sub-diagonal
    double xn = 0.0;
    for (int i = k + 2 + tid; i < r; i += blockDim.x) xn += cabs2(S[ck + (i - k)]);
    for (int o = 32; o > 0; o >>= 1) xn += __shfl_xor(xn, o, 64);
    if (lane == 0 && xn != 0.0) atomicAdd(&L.acc[par], xn);
    __syncthreads();
    // (B) reflector H = I - tau v v^H with H^H x = beta e_1 (computed redundantly by every thread)
    xn = L.acc[par];
    const zd alpha = S[ck + 1];
    zd tau = mk(0.0, 0.0), sc = mk(0.0, 0.0);
    double beta = alpha.re;
    const bool active = (xn > 0.0 || alpha.im != 0.0);
    if (active) {
      const double nrm = sqrt(alpha.re * alpha.re + alpha.im * alpha.im + xn);
      beta = alpha.re >= 0.0 ? -nrm : nrm;
      tau = mk((beta - alpha.re) / beta, -alpha.im / beta);
      const zd den = mk(alpha.re - beta, alpha.im);
      const double dd = cabs2(den);
      sc = mk(den.re / dd, -den.im / dd);
    }
    for (int i = k + 1 + tid; i < r; i += blockDim.x) {
      zd vi = (i == k + 1) ? mk(1.0, 0.0) : (active ? cmul(S[ck + (i - k)], sc) : mk(0.0, 0.0));
      S[ck + (i - k)] = vi;
      L.v[i] = vi;
    }
    if (tid == 0) {
      L.e[k] = beta;
      L.tau[k] = tau;
      L.d[k] = S[ck].re;
      L.acc[par ^ 1] = 0.0;
      L.accre[par ^ 1] = 0.0;
      L.accim[par ^ 1] = 0.0;
    }
    __syncthreads();
    if (active) {
      // (C) p = tau A22 v, 8 lanes per row, branch-free over the packed lower triangle
      for (int base = k + 1; base < r; base += ngrp) {
        const int i = base + grp;
        zd s = mk(0.0, 0.0);
        if (i < r) {
          for (int j = k + 1 + sub; j <= i; j += 8) s = cadd(s, cmul(S[L.cb[j] + (i - j)], L.v[j]));
          const int ci = L.cb[i] - i;
          for (int j = i + 1 + sub; j < r; j += 8) s = cadd(s, cmul(cconj(S[ci + j]), L.v[j]));
        }
        s.re = grp8_sum(s.re);
        s.im = grp8_sum(s.im);
        if (i < r && sub == 0) {
          const zd pi = cmul(tau, s);
          L.p[i] = pi;
          const zd c = cmulc(pi, L.v[i]);
          atomicAdd(&L.accre[par], c.re);
          atomicAdd(&L.accim[par], c.im);
        }
      }
      __syncthreads();
      // (D) A22 -= v w^H + w v^H with w = p + alpha2 v, alpha2 = -tau (p^H v) / 2
      const zd a2 = cscale(cmul(tau, mk(L.accre[par], L.accim[par])), -0.5);
      for (int c = k + 1 + wave; c < r; c += nw) {
        const zd vc = cconj(L.v[c]);
        const zd wc = cconj(cadd(L.p[c], cmul(a2, L.v[c])));
        const int cc = L.cb[c] - c;
        for (int i = c + lane; i < r; i += 64) {
          const zd vi = L.v[i];
          const zd wi = cadd(L.p[i], cmul(a2, vi));
          zd& a = S[cc + i];
          a = csub(a, cadd(cmul(vi, wc), cmul(wi, vc)));
        }
      }
    }
    __syncthreads();
  }
  if (tid == 0) {
    L.d[r - 1] = S[L.cb[r - 1]].re;
    L.e[r - 1] = 0.0;
  }
  __syncthreads();
  for (int i = tid; i < r; i += blockDim.x) L.e2[i] = L.e[i] * L.e[i];
  __syncthreads();

  RT_PHASE(2);
  // ---- eigenvalues of T: multisection, 8 lanes per eigenvalue ------------------------------
  double gl = 1e308, gu = -1e308, emax2 = 0.0;
  for (int i = 0; i < r; ++i) {
    const double off = fabs(L.e[i]) + (i > 0 ? fabs(L.e[i - 1]) : 0.0);
    gl = fmin(gl, L.d[i] - off);
    gu = fmax(gu, L.d[i] + off);
    emax2 = fmax(emax2, L.e2[i]);
  }
  const double tnorm = fmax(fabs(gl), fabs(gu));
  const double eps = 2.220446049250313e-16;
  const double pivmin = 2.2250738585072014e-308 * fmax(1.0, emax2);
  const double atol = 2.0 * eps * tnorm + 4.0 * pivmin;
  gl -= 2.0 * eps * tnorm + pivmin;
  gu += 2.0 * eps * tnorm + pivmin;
  for (int base = 0; base < r; base += ngrp) {
    const int j = base + grp;                      // j-th largest eigenvalue
    const bool on = j < r;
    const int a = r - 1 - (on ? j : 0);           // ascending index
    double lo = gl, hi = gu;
    for (int it = 0; it < 200; ++it) {
      if (hi - lo <= atol + 2.0 * eps * fmax(fabs(lo), fabs(hi))) break;
      const double x = lo + (hi - lo) * (double)(sub + 1) / 9.0;
      const int cnt = on ? sturm_count_fast(L.d, L.e2, r, x, pivmin) : 0;
      double nlo = (cnt <= a) ? x : -1e308;
      double nhi = (cnt > a) ? x : 1e308;
      for (int o = 1; o < 8; o <<= 1) {
        nlo = fmax(nlo, __shfl_xor(nlo, o, 64));
        nhi = fmin(nhi, __shfl_xor(nhi, o, 64));
      }
      if (nlo > lo) lo = nlo;
      if (nhi < hi) hi = nhi;
    }
    if (on && sub == 0) L.lam[j] = 0.5 * (lo + hi);
  }
  __syncthreads();

  RT_PHASE(3);
  // ---- the reflectors move to global memory; LDS (or the global slice) then holds Z ------------
  // Z column j (stride zst = r + 1 doubles) = eigenvector of T for lam[j]
  if (in_lds) {
    for (int64_t i = tid; i < packed_size(r); i += blockDim.x) Sg[i] = S[i];
    __syncthreads();
  }
  const int zst = r + 1;
  double* Zp = in_lds ? reinterpret_cast<double*>(smem_raw + sizeof(HeevLds)) : Z;

  // ---- eigenvectors of T: inverse iteration, one thread per eigenvalue ---------------------------
  for (int j = tid; j < r; j += blockDim.x) {
    const double lam = L.lam[j];
    double* ui = lu + ((int64_t)f * r + j) * 5 * r;   // 1 / pivot
    double* us1 = ui + r;
    double* us2 = us1 + r;
    double* ml = us2 + r;
    double* sw = ml + r;
    const double pert = eps * tnorm > 0.0 ? eps * tnorm : 1e-300;
    // LU with partial pivoting of T - lam I
    double a = L.d[0] - lam, b = r > 1 ? L.e[0] : 0.0;
    for (int k = 0; k < r - 1; ++k) {
      const double c = L.e[k];              // sub-diagonal entry of row k+1
      const double anext = L.d[k + 1] - lam;
      const double bnext = (k + 1 < r - 1) ? L.e[k + 1] : 0.0;
      if (fabs(a) >= fabs(c)) {
        const double ap = fabs(a) < pert ? (a < 0.0 ? -pert : pert) : a;
        const double ia = inv_d(ap);
        const double mlt = c * ia;
        ui[k] = ia; us1[k] = b; us2[k] = 0.0; ml[k] = mlt; sw[k] = 0.0;
        a = anext - mlt * b;
        b = bnext;
      } else {
        const double mlt = a * inv_d(c);
        ui[k] = inv_d(c); us1[k] = anext; us2[k] = bnext; ml[k] = mlt; sw[k] = 1.0;
        a = b - mlt * anext;
        b = -mlt * bnext;
      }
    }
    ui[r - 1] = inv_d(fabs(a) < pert ? (a < 0.0 ? -pert : pert) : a);
    // start vector: deterministic, not aligned with any structure
    double* z = Zp + (int64_t)j * zst;
    uint32_t st = 0x9E3779B9u ^ (uint32_t)(j * 2654435761u);
    for (int i = 0; i < r; ++i) {
      st = st * 1664525u + 1013904223u;
      z[i] = ((double)(st >> 8) / 16777216.0) - 0.5;
    }
    for (int iter = 0; iter < 2; ++iter) {
      for (int k = 0; k < r - 1; ++k) {
        if (sw[k] != 0.0) { const double t = z[k]; z[k] = z[k + 1]; z[k + 1] = t - ml[k] * z[k + 1]; }
        else z[k + 1] -= ml[k] * z[k];
      }
      double z1 = 0.0, z2 = 0.0, nn = 0.0;     // z[k+1], z[k+2] of the back substitution
      for (int k = r - 1; k >= 0; --k) {
        const double zk = (z[k] - us1[k] * z1 - us2[k] * z2) * ui[k];
        z[k] = zk;
        z2 = z1; z1 = zk;
        nn += zk * zk;
      }
      const double inv = nn > 0.0 ? 1.0 / sqrt(nn) : 0.0;
      for (int i = 0; i < r; ++i) z[i] *= inv;
    }
  }
  RT_PHASE(4);
  // clusters: maximal runs of eigenvalues with consecutive gaps <= ortol
  const double ortol = 1e-3 * tnorm;
  if (tid == 0) {
    int nc = 0;
    for (int j = 0; j < r; ++j)
      if (j == 0 || L.lam[j - 1] - L.lam[j] > ortol) L.cstart[nc++] = j;
    L.cstart[nc] = r;
    L.ncl = nc;
  }
  __syncthreads();
  // modified Gram-Schmidt inside every cluster (two passes): the pivot vector is normalized by one
  // wave, then every later vector of the cluster loses its component along it, one wave per vector
  for (int c = 0; c < L.ncl; ++c) {
    const int j0 = L.cstart[c], j1 = L.cstart[c + 1];
    if (j1 - j0 < 2) continue;
    for (int pass = 0; pass < 2; ++pass)
      for (int i = j0; i < j1; ++i) {
        double* zi = Zp + (int64_t)i * zst;
        if (wave == 0) {
          double nn = 0.0;
          for (int x = lane; x < r; x += 64) nn += zi[x] * zi[x];
          for (int o = 32; o > 0; o >>= 1) nn += __shfl_xor(nn, o, 64);
          const double inv = nn > 0.0 ? 1.0 / sqrt(nn) : 0.0;
          for (int x = lane; x < r; x += 64) zi[x] *= inv;
        }
        __syncthreads();
        for (int q = i + 1 + wave; q < j1; q += nw) {
          double* zq = Zp + (int64_t)q * zst;
          double dt = 0.0;
          for (int x = lane; x < r; x += 64) dt += zi[x] * zq[x];
          for (int o = 32; o > 0; o >>= 1) dt += __shfl_xor(dt, o, 64);
          for (int x = lane; x < r; x += 64) zq[x] -= dt * zi[x];
        }
        __syncthreads();
      }
  }
  __syncthreads();

  RT_PHASE(5);
  // ---- back-transformation U = Q_H Z, 8 lanes per column ---------------------------------------
  if (in_lds && r <= 8 * HEEV_UREG) {
    // column in registers (lane sub owns rows sub + 8 t), reflectors back in LDS
    const int c = grp;                       // one column per 8-lane group (r <= 128 = ngrp)
    const bool on = c < r;
    zd u[HEEV_UREG];
#pragma unroll
    for (int t = 0; t < HEEV_UREG; ++t) {
      const int i = sub + 8 * t;
      u[t] = mk((on && i < r) ? Zp[(int64_t)c * zst + i] : 0.0, 0.0);
    }
    __syncthreads();
    for (int64_t i = tid; i < packed_size(r); i += blockDim.x) S[i] = Sg[i];
    __syncthreads();
    for (int k = r - 2; k >= 0; --k) {
      const zd tau = L.tau[k];
      if (tau.re == 0.0 && tau.im == 0.0) continue;
      const zd* vk = S + L.cb[k] - k;        // vk[i] = v_k(i) for i > k
      zd sacc = mk(0.0, 0.0);
#pragma unroll
      for (int t = 0; t < HEEV_UREG; ++t) {
        const int i = sub + 8 * t;
        if (i > k && i < r) sacc = cadd(sacc, cmulc(vk[i], u[t]));
      }
      sacc.re = grp8_sum(sacc.re);
      sacc.im = grp8_sum(sacc.im);
      sacc = cmul(tau, sacc);
#pragma unroll
      for (int t = 0; t < HEEV_UREG; ++t) {
        const int i = sub + 8 * t;
        if (i > k && i < r) u[t] = csub(u[t], cmul(vk[i], sacc));
      }
    }
    if (on) {
#pragma unroll
      for (int t = 0; t < HEEV_UREG; ++t) {
        const int i = sub + 8 * t;
        if (i < r) U[(int64_t)c * r + i] = u[t];
      }
      if (sub == 0) lamout[(int64_t)f * r + c] = L.lam[c];
    }
  } else {
    for (int base = 0; base < r; base += ngrp) {
      const int c = base + grp;
      const bool on = c < r;
      // each lane owns the rows i = sub (mod 8) of its column for the whole loop
      zd* u = U + (int64_t)(on ? c : 0) * r;
      if (on)
        for (int i = sub; i < r; i += 8) u[i] = mk(Zp[(int64_t)c * zst + i], 0.0);
      for (int k = r - 2; k >= 0; --k) {
        const zd tau = L.tau[k];
        if (tau.re == 0.0 && tau.im == 0.0) continue;
        const zd* vk = Sg + L.cb[k] - k;
        zd sacc = mk(0.0, 0.0);
        if (on)
          for (int i = sub; i < r; i += 8)
            if (i > k) sacc = cadd(sacc, cmulc(vk[i], u[i]));
        sacc.re = grp8_sum(sacc.re);
        sacc.im = grp8_sum(sacc.im);
        sacc = cmul(tau, sacc);
        if (on)
          for (int i = sub; i < r; i += 8)
            if (i > k) u[i] = csub(u[i], cmul(vk[i], sacc));
      }
      if (on && sub == 0) lamout[(int64_t)f * r + c] = L.lam[c];
    }
  }
  RT_PHASE(6);
}

// -------------------------------------------------------------------------------------------
// Cholesky and triangular inverse: Rinv = L^{-H}
// -------------------------------------------------------------------------------------------
struct CholLds {
  zd x[HEEV_RMAX], t[HEEV_RMAX];
  int cb[HEEV_RMAX + 1];
  double piv, tol;
  int bad;
};

inline size_t chol_lds_bytes(int r, bool packed_in_lds) {
  return sizeof(CholLds) + (packed_in_lds ? (size_t)packed_size(r) * sizeof(zd) : 0);
}

__global__ void __launch_bounds__(HEEV_THREADS)
k_cholinv(const zd* __restrict__ Gin, int r, zd* __restrict__ Rinv, double tol_rel, int* __restrict__ flags,
          zd* __restrict__ gpk, int in_lds) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  CholLds& L = *reinterpret_cast<CholLds*>(smem_raw);
  const int f = blockIdx.x;
  zd* S = in_lds ? reinterpret_cast<zd*>(smem_raw + sizeof(CholLds)) : gpk + (int64_t)f * packed_size(r);
  const zd* G = Gin + (int64_t)f * r * r;
  zd* R = Rinv + (int64_t)f * r * r;
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63, nw = blockDim.x >> 6;
  for (int j = tid; j <= r; j += blockDim.x) L.cb[j] = (int)pk_off(j, r);
  for (int j = 0; j < r; ++j)
    for (int i = j + tid; i < r; i += blockDim.x) S[pk_off(j, r) + (i - j)] = G[i + (int64_t)j * r];
  if (tid == 0) { L.bad = 0; }
  __syncthreads();
  if (tid == 0) {
    double mx = 0.0;
    for (int j = 0; j < r; ++j) mx = fmax(mx, S[L.cb[j]].re);
    L.tol = tol_rel * mx;
  }
  __syncthreads();
  RT_PHASE(8);
  // right-looking Cholesky
  for (int j = 0; j < r; ++j) {
    if (tid == 0) {
      const double d = S[L.cb[j]].re;
      double pv = 0.0;
      if (d > L.tol && d > 0.0) pv = sqrt(d); else L.bad = 1;
      L.piv = pv;
      S[L.cb[j]] = mk(pv, 0.0);
    }
    __syncthreads();
    const double pv = L.piv;
    const double ipv = pv > 0.0 ? 1.0 / pv : 0.0;
    for (int i = j + 1 + tid; i < r; i += blockDim.x) {
      zd& a = S[L.cb[j] + (i - j)];
      a = cscale(a, ipv);
      L.x[i] = a;
    }
    __syncthreads();
    for (int c = j + 1 + wave; c < r; c += nw) {
      const zd lc = cconj(L.x[c]);
      for (int i = c + lane; i < r; i += 64) {
        zd& a = S[L.cb[c] + (i - c)];
        a = csub(a, cmul(L.x[i], lc));
      }
    }
    __syncthreads();
  }
  RT_PHASE(9);
  // in-place inverse of the lower triangular L (columns from the last to the first)
  for (int j = r - 1; j >= 0; --j) {
    const double ljj = S[L.cb[j]].re;
    const double ajj = ljj > 0.0 ? 1.0 / ljj : 0.0;
    for (int i = j + 1 + tid; i < r; i += blockDim.x) L.x[i] = S[L.cb[j] + (i - j)];
    __syncthreads();
    // t_i = sum_{k=j+1..i} Linv(i,k) x_k, 8 lanes per row
    for (int base = j + 1; base < r; base += (int)blockDim.x / 8) {
      const int i = base + tid / 8, sub = tid % 8;
      zd s = mk(0.0, 0.0);
      if (i < r)
        for (int k = j + 1 + sub; k <= i; k += 8) s = cadd(s, cmul(S[L.cb[k] + (i - k)], L.x[k]));
      s.re = grp8_sum(s.re);
      s.im = grp8_sum(s.im);
      if (i < r && sub == 0) L.t[i] = s;
    }
    __syncthreads();
    for (int i = j + 1 + tid; i < r; i += blockDim.x) S[L.cb[j] + (i - j)] = cscale(L.t[i], -ajj);
    if (tid == 0) S[L.cb[j]] = mk(ajj, 0.0);
    __syncthreads();
  }
  RT_PHASE(10);
  // Rinv(i, j) = conj(Linv(j, i)) for i <= j, zero below the diagonal
  for (int idx = tid; idx < r * r; idx += blockDim.x) {
    const int i = idx % r, j = idx / r;
    R[idx] = (i <= j) ? cconj(S[L.cb[i] + (j - i)]) : mk(0.0, 0.0);
  }
  if (tid == 0 && flags && L.bad) atomicOr(flags, 1);
}

}  // namespace rt
