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
#include <type_traits>
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
// lower triangle of the column-major r x r matrix G into packed storage S; every thread keeps 8
// independent loads in flight
__device__ __forceinline__ void load_lower_packed(const zd* __restrict__ G, int r, zd* S, int tid, int nt) {
  const int total = r * r;
  for (int base = 0; base < total; base += 8 * nt) {
    zd v[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int idx = base + u * nt + tid;
      v[u] = idx < total ? G[idx] : mk(0.0, 0.0);
    }
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int idx = base + u * nt + tid;
      if (idx < total) {
        const int i = idx % r, j = idx / r;
        if (i >= j) S[pk_off(j, r) + (i - j)] = v[u];
      }
    }
  }
}

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
// IN_LDS: the packed working matrix (and later Z) live in LDS; a template parameter so that LDS
// accesses compile to LDS instructions rather than generic (flat) ones.
template <bool IN_LDS>
__global__ void __launch_bounds__(HEEV_THREADS)
k_heev(const zd* __restrict__ Gin, int r, zd* __restrict__ Uout, double* __restrict__ lamout,
       zd* __restrict__ gpk, double* __restrict__ zs, double* __restrict__ lu) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  HeevLds& L = *reinterpret_cast<HeevLds*>(smem_raw);
  const int f = blockIdx.x;
  zd* S;
  if constexpr (IN_LDS) S = reinterpret_cast<zd*>(smem_raw + sizeof(HeevLds));
  else S = gpk + (int64_t)f * packed_size(r);
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
  load_lower_packed(G, r, S, tid, blockDim.x);
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
  if constexpr (IN_LDS) {
    for (int64_t i = tid; i < packed_size(r); i += blockDim.x) Sg[i] = S[i];
    __syncthreads();
  }
  const int zst = r + 1;
  double* Zp;
  if constexpr (IN_LDS) Zp = reinterpret_cast<double*>(smem_raw + sizeof(HeevLds));
  else Zp = Z;

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
  if (IN_LDS && r <= 8 * HEEV_UREG) {
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
// ---------------------------------------------------------------------------------------------
// Cholesky factor and triangular inverse of the r x r Gram matrices (one workgroup per face), FP64:
//   G = L L^H (L lower, real positive diagonal),  Rinv = L^{-H}  (upper), so Q = Y Rinv.
// Blocked by 16 columns.  Per diagonal block K, one wave factors the 16 x 16 block and inverts it
// in registers (lane (i, j) layout, column data exchanged by cross-lane shuffles); the panel below
// is G_panel D^H (D = L_KK^{-1}) and the trailing update is S -= P P^H, both on FP64 MFMA 16x16x4
// tiles spread over the waves.  The inverse runs over the diagonal blocks backwards:
//   Linv(J1:, J) = -Linv(J1:, J1:) X D_J,  X = L(J1:, J)  (MFMA tiles, three barriers per block).
// A pivot at or below tol_rel * max diag marks a dependent column: its row and column of L^{-1}
// are zero and flags gets bit 0.  The packed lower triangle lives in LDS when it fits (else in
// `gpk`, global scratch of packed_size(r) per face); `gdi` (F x ceil(r/16) x 256) keeps the block
// inverses between the two sweeps.
// ---------------------------------------------------------------------------------------------
constexpr int CH_NB = 16, CH_PS = CH_NB + 1;  // block width, padded row stride of the panel buffers
constexpr int CH_THREADS = 512;

struct CholHdr {
  double tol;
  int bad;
  int pad_;
  double ipiv[HEEV_RMAX];   // 1 / L(j, j), 0 for a dependent column
};

inline size_t chol_lds_bytes(int r, bool packed_in_lds) {
  size_t b = (sizeof(CholHdr) + 15) / 16 * 16;
  b += (size_t)r * CH_PS * sizeof(zd);       // panel buffer P
  b += (size_t)CH_NB * CH_PS * sizeof(zd);   // diagonal block inverse DI
  if (packed_in_lds) b += (size_t)packed_size(r) * sizeof(zd);
  return b;
}
RT_HOST_DEVICE int64_t chol_gdi_elems(int r) { return (int64_t)((r + CH_NB - 1) / CH_NB) * CH_NB * CH_NB; }

typedef double ch_f64x4 __attribute__((ext_vector_type(4)));
__device__ __forceinline__ ch_f64x4 ch_mma(double a, double b, ch_f64x4 c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}
// C += a b for one k-group of a complex 16 x 16 x 4 product (lane's A and B operand elements)
__device__ __forceinline__ void ch_cmma(zd a, zd b, ch_f64x4& cr, ch_f64x4& ci) {
  cr = ch_mma(a.re, b.re, cr);
  cr = ch_mma(-a.im, b.im, cr);
  ci = ch_mma(a.re, b.im, ci);
  ci = ch_mma(a.im, b.re, ci);
}
__device__ __forceinline__ zd ch_shfl(zd v, int src) { return mk(__shfl(v.re, src), __shfl(v.im, src)); }
// component-wise select (a conditional on whole structs can force them into private memory)
__device__ __forceinline__ zd zsel(bool c, zd x, zd y) { return mk(c ? x.re : y.re, c ? x.im : y.im); }
// f(integral_constant<int, I>) for I = B .. E-1, unrolled at compile time (register arrays stay
// statically indexed)
template <int B, int E, typename Fn> __device__ __forceinline__ void static_for(Fn&& fn) {
  if constexpr (B < E) {
    fn(std::integral_constant<int, B>{});
    static_for<B + 1, E>(fn);
  }
}

template <bool IN_LDS>
__global__ void __launch_bounds__(CH_THREADS)
k_cholinv(const zd* __restrict__ Gin, int r, zd* __restrict__ Rinv, double tol_rel, int* __restrict__ flags,
          zd* __restrict__ gpk, zd* __restrict__ gdi) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  CholHdr& H = *reinterpret_cast<CholHdr*>(smem_raw);
  zd* P = reinterpret_cast<zd*>(smem_raw + (sizeof(CholHdr) + 15) / 16 * 16);
  zd* DI = P + (size_t)r * CH_PS;
  const int f = blockIdx.x;
  zd* S;
  if constexpr (IN_LDS) S = DI + CH_NB * CH_PS;
  else S = gpk + (int64_t)f * packed_size(r);
  const zd* G = Gin + (int64_t)f * r * r;
  zd* R = Rinv + (int64_t)f * r * r;
  zd* GD = gdi + (int64_t)f * chol_gdi_elems(r);
  const int tid = threadIdx.x, lane = tid & 63;
  const int nw = (int)blockDim.x >> 6;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int g = lane >> 4, rho = lane & 15;   // MFMA lane coordinates
  // packed lower storage, column j at j r - j (j - 1) / 2
  auto at = [&](int i, int j) -> zd& { return S[j * r - (j * (j - 1)) / 2 + (i - j)]; };  // i >= j
  const zd zero = mk(0.0, 0.0);

  RT_PHASE(7);
  load_lower_packed(G, r, S, tid, blockDim.x);
  if (tid == 0) H.bad = 0;
  __syncthreads();
  if (wave == 0) {
    double mx = 0.0;
    for (int j = lane; j < r; j += 64) mx = fmax(mx, at(j, j).re);
    for (int o = 32; o > 0; o >>= 1) mx = fmax(mx, __shfl_xor(mx, o));
    if (lane == 0) H.tol = tol_rel * mx;
  }
  __syncthreads();
  const double tol = H.tol;

  RT_PHASE(8);
  // ---- blocked right-looking Cholesky ----
  for (int K = 0; K < r; K += CH_NB) {
    const int kb = min(CH_NB, r - K), K1 = K + kb, m = r - K1;
    // (a) wave 0: factor the diagonal block and invert it; lane holds (i, j_s), i = rho, j_s = g + 4 s.
    // A block narrower than 16 is padded with the identity (its extra pivots are 1), so the
    // unrolled column loop has no bound tests; only rows and columns < kb are written back.
    if (wave == 0) {
      zd a[4], d[4];
#pragma unroll
      for (int s2 = 0; s2 < 4; ++s2) {
        const int j = g + 4 * s2;
        const bool in = rho < kb && j < kb && rho >= j;
        const zd diag = mk(rho == j ? 1.0 : 0.0, 0.0);
        a[s2] = in ? at(K + rho, K + j) : diag;
        d[s2] = diag;
      }
      double myipv = 1.0;   // 1 / L(rho, rho) once column rho is factored
#pragma unroll
      for (int c = 0; c < CH_NB; ++c) {
        const int cs = c & 3, sl = c >> 2;
        const zd ac = a[sl];
        const double dd = __shfl(ac.re, c + 16 * cs);
        const double pv = (c >= kb) ? 1.0 : ((dd > tol && dd > 0.0) ? sqrt(dd) : 0.0);
        const double ipv = pv > 0.0 ? 1.0 / pv : 0.0;
        myipv = (rho == c) ? ipv : myipv;
        const zd acn = zsel(g != cs || rho < c, ac, zsel(rho == c, mk(pv, 0.0), cscale(ac, ipv)));
        a[sl] = acn;
        const zd lic = ch_shfl(acn, rho + 16 * cs);   // L(rho, c)
        zd ljc[4];
#pragma unroll
        for (int s2 = 0; s2 < 4; ++s2) ljc[s2] = ch_shfl(acn, g + 4 * s2 + 16 * cs);   // L(j_s, c)
#pragma unroll
        for (int s2 = 0; s2 < 4; ++s2) {
          const int j = g + 4 * s2;
          const zd upd = csub(a[s2], cmul(lic, cconj(ljc[s2])));
          a[s2] = zsel(j > c && rho >= j, upd, a[s2]);
        }
      }
      if (g == 0 && rho < kb) {
        H.ipiv[K + rho] = myipv;
        if (myipv == 0.0) H.bad = 1;
      }
      // D = L_KK^{-1}: forward substitution, row t final then eliminated from the rows below
#pragma unroll
      for (int t = 0; t < CH_NB; ++t) {
        const double sc = (rho == t) ? myipv : 1.0;   // branch-free: the arrays stay in registers
#pragma unroll
        for (int s2 = 0; s2 < 4; ++s2) d[s2] = cscale(d[s2], sc);
        const zd lit = ch_shfl(a[t >> 2], rho + 16 * (t & 3));   // L(rho, t)
        const zd lm = zsel(rho > t, lit, zero);
        zd dtj[4];
#pragma unroll
        for (int s2 = 0; s2 < 4; ++s2) dtj[s2] = ch_shfl(d[s2], t + 16 * g);   // D(t, j_s)
#pragma unroll
        for (int s2 = 0; s2 < 4; ++s2) d[s2] = csub(d[s2], cmul(lm, dtj[s2]));
      }
#pragma unroll
      for (int s2 = 0; s2 < 4; ++s2) {
        const int j = g + 4 * s2;
        if (rho < kb && j < kb && rho >= j) at(K + rho, K + j) = a[s2];
        const zd dv = zsel(rho < kb && j < kb, d[s2], zero);
        DI[rho * CH_PS + j] = dv;
        GD[(K / CH_NB) * CH_NB * CH_NB + rho * CH_NB + j] = dv;
      }
    }
    __syncthreads();
    if (K == 0) RT_PHASE(12);
    // (b) panel P(i, c) = sum_t G(i, K + t) conj(D(c, t)), rows i >= K1, 16-row MFMA tiles
    for (int ti = wave; ti * 16 < m; ti += nw) {
      const int i0 = K1 + 16 * ti;
      ch_f64x4 cr = {0, 0, 0, 0}, ci = {0, 0, 0, 0};
#pragma unroll
      for (int kg = 0; kg < 4; ++kg) {
        const int k = 4 * kg + g;
        const zd av = (i0 + rho < r && k < kb) ? at(i0 + rho, K + k) : zero;
        const zd bv = (k < kb && rho < kb) ? cconj(DI[rho * CH_PS + k]) : zero;
        ch_cmma(av, bv, cr, ci);
      }
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int i = i0 + g + 4 * v;
        if (i < r && rho < kb) {
          const zd x = mk(cr[v], ci[v]);
          at(i, K + rho) = x;
          P[(size_t)i * CH_PS + rho] = x;
        }
      }
    }
    __syncthreads();
    if (K == 0) RT_PHASE(13);
    // (c) trailing update S(i, j) -= sum_c P(i, c) conj(P(j, c)), lower 16 x 16 tiles
    const int T = (m + 15) / 16;
    for (int q = wave; q < T * (T + 1) / 2; q += nw) {
      int ti = (int)((sqrtf(8.0f * q + 1.0f) - 1.0f) * 0.5f);
      while (ti * (ti + 1) / 2 > q) --ti;
      while ((ti + 1) * (ti + 2) / 2 <= q) ++ti;
      const int tj = q - ti * (ti + 1) / 2;
      const int i0 = K1 + 16 * ti, j0 = K1 + 16 * tj;
      ch_f64x4 cr = {0, 0, 0, 0}, ci = {0, 0, 0, 0};
#pragma unroll
      for (int kg = 0; kg < 4; ++kg) {
        const int k = 4 * kg + g;
        const zd av = (i0 + rho < r && k < kb) ? P[(size_t)(i0 + rho) * CH_PS + k] : zero;
        const zd bv = (j0 + rho < r && k < kb) ? cconj(P[(size_t)(j0 + rho) * CH_PS + k]) : zero;
        ch_cmma(av, bv, cr, ci);
      }
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int i = i0 + g + 4 * v, j = j0 + rho;
        if (i < r && j < r && i >= j) at(i, j) = csub(at(i, j), mk(cr[v], ci[v]));
      }
    }
    __syncthreads();
    if (K == 0) RT_PHASE(14);
  }
  RT_PHASE(9);
  // ---- in-place inverse of L, diagonal blocks from the last to the first ----
  const int nblk = (r + CH_NB - 1) / CH_NB;
  for (int Jb = nblk - 1; Jb >= 0; --Jb) {
    const int J = Jb * CH_NB, kb = min(CH_NB, r - J), J1 = J + kb, m = r - J1;
    // (d) block inverse D_J back from global; panel X = L(J1:, J) copied into P
    for (int q = tid; q < CH_NB * CH_NB; q += blockDim.x) DI[(q / CH_NB) * CH_PS + q % CH_NB] = GD[Jb * CH_NB * CH_NB + q];
    for (int q = tid; q < m * kb; q += blockDim.x) {
      const int k = J1 + q / kb, c = q % kb;
      P[(size_t)k * CH_PS + c] = at(k, J + c);
    }
    __syncthreads();
    // (e) T = Linv(J1:, J1:) X, written over the panel slots (X is safe in P)
    for (int ti = wave; ti * 16 < m; ti += nw) {
      const int i0 = J1 + 16 * ti;
      ch_f64x4 cr = {0, 0, 0, 0}, ci = {0, 0, 0, 0};
      for (int tk = 0; tk <= ti; ++tk) {
#pragma unroll
        for (int kg = 0; kg < 4; ++kg) {
          const int kk = J1 + 16 * tk + 4 * kg + g;
          const int i = i0 + rho;
          const zd av = (i < r && kk <= i) ? at(i, kk) : zero;
          const zd bv = (kk < r && rho < kb) ? P[(size_t)kk * CH_PS + rho] : zero;
          ch_cmma(av, bv, cr, ci);
        }
      }
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int i = i0 + g + 4 * v;
        if (i < r && rho < kb) at(i, J + rho) = mk(cr[v], ci[v]);
      }
    }
    __syncthreads();
    // (f) Linv(i, J + c) = -sum_t T(i, t) D(t, c) (each wave reads back only its own row tiles);
    // the diagonal block becomes D
    for (int ti = wave; ti * 16 < m; ti += nw) {
      const int i0 = J1 + 16 * ti;
      ch_f64x4 cr = {0, 0, 0, 0}, ci = {0, 0, 0, 0};
#pragma unroll
      for (int kg = 0; kg < 4; ++kg) {
        const int t = 4 * kg + g;
        const zd av = (i0 + rho < r && t < kb) ? at(i0 + rho, J + t) : zero;
        const zd bv = (t < kb && rho < kb) ? DI[t * CH_PS + rho] : zero;
        ch_cmma(av, bv, cr, ci);
      }
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int i = i0 + g + 4 * v;
        if (i < r && rho < kb) at(i, J + rho) = mk(-cr[v], -ci[v]);
      }
    }
    for (int q = tid; q < kb * kb; q += blockDim.x) {
      const int i = q / kb, c = q % kb;
      if (i >= c) at(J + i, J + c) = DI[i * CH_PS + c];
    }
    __syncthreads();
  }
  RT_PHASE(10);
  // Rinv(i, j) = conj(Linv(j, i)) for i <= j, zero below the diagonal
  for (int idx = tid; idx < r * r; idx += blockDim.x) {
    const int i = idx % r, j = idx / r;
    R[idx] = (i <= j) ? cconj(at(j, i)) : zero;
  }
  RT_PHASE(11);
  if (tid == 0 && flags && H.bad) atomicOr(flags, 1);
}

}  // namespace rt
