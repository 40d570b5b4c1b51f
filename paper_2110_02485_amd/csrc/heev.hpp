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
__device__ unsigned long long rt_phase_clock[24];
#define RT_PHASE(i) do { __syncthreads(); if (blockIdx.x == 0 && threadIdx.x == 0) rt_phase_clock[i] = wall_clock64(); } while (0)
// timestamp of one wave's progress (its lane 0), no synchronization
#define RT_MARK(i) do { if (blockIdx.x == 0 && (threadIdx.x & 63) == 0) rt_phase_clock[i] = wall_clock64(); } while (0)
#else
#define RT_PHASE(i) do { } while (0)
#define RT_MARK(i) do { } while (0)
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

// 1/sqrt(x) for normal x > 0: v_rsq_f64 refined by two Newton steps, y <- y + y (1 - x y^2) / 2
__device__ __forceinline__ double rsqrt_d(double x) {
  double y = __builtin_amdgcn_rsq(x);
  y = fma(0.5 * y, fma(-x * y, y, 1.0), y);
  y = fma(0.5 * y, fma(-x * y, y, 1.0), y);
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

// Gershgorin interval, norm, pivot floor and absolute tolerance of the tridiagonal (d, e)
struct TriBounds { double gl, gu, tnorm, pivmin, atol; };
__device__ __forceinline__ TriBounds tri_bounds(const double* d, const double* e, const double* e2, int r) {
  double gl = 1e308, gu = -1e308, emax2 = 0.0;
  for (int i = 0; i < r; ++i) {
    const double off = fabs(e[i]) + (i > 0 ? fabs(e[i - 1]) : 0.0);
    gl = fmin(gl, d[i] - off);
    gu = fmax(gu, d[i] + off);
    emax2 = fmax(emax2, e2[i]);
  }
  TriBounds tb;
  const double eps = 2.220446049250313e-16;
  tb.tnorm = fmax(fabs(gl), fabs(gu));
  tb.pivmin = 2.2250738585072014e-308 * fmax(1.0, emax2);
  tb.atol = 2.0 * eps * tb.tnorm + 4.0 * tb.pivmin;
  tb.gl = gl - (2.0 * eps * tb.tnorm + tb.pivmin);
  tb.gu = gu + (2.0 * eps * tb.tnorm + tb.pivmin);
  return tb;
}

// j-th largest eigenvalue of the tridiagonal by multisection: the 8 aligned lanes of a group
// (sub = lane & 7) evaluate Sturm counts at 8 interior points per round.  All lanes of the group
// return the same value.
__device__ __forceinline__ double tri_eigval(const double* d, const double* e2, int r, int j, bool on, int sub,
                                             const TriBounds& tb) {
  const double eps = 2.220446049250313e-16;
  const int a = r - 1 - (on ? j : 0);           // ascending index
  double lo = tb.gl, hi = tb.gu;
  for (int it = 0; it < 200; ++it) {
    if (hi - lo <= tb.atol + 2.0 * eps * fmax(fabs(lo), fabs(hi))) break;
    const double x = lo + (hi - lo) * (double)(sub + 1) / 9.0;
    const int cnt = on ? sturm_count_fast(d, e2, r, x, tb.pivmin) : 0;
    double nlo = (cnt <= a) ? x : -1e308;
    double nhi = (cnt > a) ? x : 1e308;
    nlo = fmax(nlo, dpp<DPP_XOR1>(nlo));
    nhi = fmin(nhi, dpp<DPP_XOR1>(nhi));
    nlo = fmax(nlo, dpp<DPP_XOR2>(nlo));
    nhi = fmin(nhi, dpp<DPP_XOR2>(nhi));
    nlo = fmax(nlo, dpp<DPP_MIRROR8>(nlo));
    nhi = fmin(nhi, dpp<DPP_MIRROR8>(nhi));
    if (nlo > lo) lo = nlo;
    if (nhi < hi) hi = nhi;
  }
  return 0.5 * (lo + hi);
}

// Number of eigenvalues below x of the tridiagonal (ds, e2s), by sign changes of the leading
// principal minors p_i = det(T_i - x I):  p_i = (d_i - x) p_{i-1} - e_{i-1}^2 p_{i-2},  p_0 = 1.
// One fused multiply-add per row on the dependency chain (the ratio form needs a division).
// Expects the matrix prescaled by a power of two so that |d|, |e| <= 1; the pair (p_{i-1}, p_i)
// is rescaled by an exact power of two every 4 rows, and an exact zero takes the sign opposite
// to its predecessor (a relative perturbation of 2^-60).  Each computed p_i is the exact minor of
// a tridiagonal with d_i and e_{i-1}^2 perturbed by a few ulps, so the count is backward stable.
__device__ __forceinline__ int sturm_count_minors_safe(const double* __restrict__ ds, const double* __restrict__ e2s,
                                                       int r, double x) {
  double pm = 1.0, pmm = 0.0;
  int cnt = 0;
  for (int i = 0; i < r; ++i) {
    double p = fma(ds[i] - x, pm, -(i > 0 ? e2s[i - 1] : 0.0) * pmm);
    p = p == 0.0 ? -pm * 0x1p-60 : p;
    cnt += ((p < 0.0) != (pm < 0.0)) ? 1 : 0;
    pmm = pm;
    pm = p;
    if ((i & 3) == 3) {
      const int ex = __builtin_amdgcn_frexp_exp(fmax(fabs(pm), fabs(pmm)));
      pm = ldexp(pm, -ex);
      pmm = ldexp(pmm, -ex);
    }
  }
  return cnt;
}

// Fast path: only the fused multiply-add is on the dependency chain; signs are counted from the
// high words, and a lane that meets an exact zero minor recounts with the guarded recurrence
// (sturm_count_minors_safe: the zero takes the sign opposite to its predecessor).
__device__ __forceinline__ int sturm_count_minors(const double* __restrict__ ds, const double* __restrict__ e2s, int r,
                                                  double x) {
  double pm = 1.0, pmm = 0.0;
  int cnt = 0;
  unsigned zero = 0u;
  int i = 0;
  for (; i + 4 <= r; i += 4) {
    double dv[4], ev[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) { dv[u] = ds[i + u] - x; ev[u] = (i + u > 0) ? e2s[i + u - 1] : 0.0; }
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const double p = fma(dv[u], pm, -ev[u] * pmm);
      const unsigned hp = (unsigned)(__double_as_longlong(p) >> 32), hm = (unsigned)(__double_as_longlong(pm) >> 32);
      cnt += (int)((hp ^ hm) >> 31);
      zero |= (unsigned)(p == 0.0);
      pmm = pm;
      pm = p;
    }
    const int ex = __builtin_amdgcn_frexp_exp(fmax(fabs(pm), fabs(pmm)));
    pm = ldexp(pm, -ex);
    pmm = ldexp(pmm, -ex);
  }
  for (; i < r; ++i) {
    const double p = fma(ds[i] - x, pm, -(i > 0 ? e2s[i - 1] : 0.0) * pmm);
    const unsigned hp = (unsigned)(__double_as_longlong(p) >> 32), hm = (unsigned)(__double_as_longlong(pm) >> 32);
    cnt += (int)((hp ^ hm) >> 31);
    zero |= (unsigned)(p == 0.0);
    pmm = pm;
    pm = p;
  }
  if (zero) cnt = sturm_count_minors_safe(ds, e2s, r, x);
  return cnt;
}

// tri_eigval on the prescaled tridiagonal (ds, e2s) = (s d, s^2 e^2), s a power of two; tb holds
// the bounds of the unscaled matrix; returns the unscaled eigenvalue.
__device__ __forceinline__ double tri_eigval_minors(const double* ds, const double* e2s, double s, int r, int j,
                                                    bool on, int sub, const TriBounds& tb) {
  const double eps = 2.220446049250313e-16;
  const int a = r - 1 - (on ? j : 0);           // ascending index
  double lo = tb.gl, hi = tb.gu;
  for (int it = 0; it < 200; ++it) {
    if (hi - lo <= tb.atol + 2.0 * eps * fmax(fabs(lo), fabs(hi))) break;
    const double x = lo + (hi - lo) * (double)(sub + 1) / 9.0;
    const int cnt = on ? sturm_count_minors(ds, e2s, r, x * s) : 0;
    double nlo = (cnt <= a) ? x : -1e308;
    double nhi = (cnt > a) ? x : 1e308;
    nlo = fmax(nlo, dpp<DPP_XOR1>(nlo));
    nhi = fmin(nhi, dpp<DPP_XOR1>(nhi));
    nlo = fmax(nlo, dpp<DPP_XOR2>(nlo));
    nhi = fmin(nhi, dpp<DPP_XOR2>(nhi));
    nlo = fmax(nlo, dpp<DPP_MIRROR8>(nlo));
    nhi = fmin(nhi, dpp<DPP_MIRROR8>(nhi));
    if (nlo > lo) lo = nlo;
    if (nhi < hi) hi = nhi;
  }
  return 0.5 * (lo + hi);
}

// Eigenvector of the tridiagonal for eigenvalue lam by two steps of inverse iteration (LU of
// T - lam I with partial pivoting, tiny pivots replaced by eps ||T||), from a deterministic start
// vector; z (stride 1) gets the unit-norm result.  lu: 5 r doubles of workspace.
__device__ __forceinline__ void tri_invit(const double* d, const double* e, int r, double lam, double tnorm, int j,
                                          double* lu, double* z) {
  const double eps = 2.220446049250313e-16;
  double* ui = lu;            // 1 / pivot
  double* us1 = ui + r;
  double* us2 = us1 + r;
  double* ml = us2 + r;
  double* sw = ml + r;
  const double pert = eps * tnorm > 0.0 ? eps * tnorm : 1e-300;
  double a = d[0] - lam, b = r > 1 ? e[0] : 0.0;
  for (int k = 0; k < r - 1; ++k) {
    const double c = e[k];              // sub-diagonal entry of row k+1
    const double anext = d[k + 1] - lam;
    const double bnext = (k + 1 < r - 1) ? e[k + 1] : 0.0;
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

// tri_invit with the LU factors in LDS, branch-free (one reciprocal per elimination step), the
// pivot swaps as an int array and U's second superdiagonal recovered from e (it is e_{k+1} where
// rows k and k+1 were swapped, else 0): 3 r doubles + r ints per eigenvalue.  Same arithmetic
// as tri_invit.
__device__ __forceinline__ void tri_invit_lds(const double* __restrict__ d, const double* __restrict__ e, int r,
                                              double lam, double tnorm, int j, double* __restrict__ ui,
                                              double* __restrict__ us1, double* __restrict__ ml, int* __restrict__ sw,
                                              double* __restrict__ z) {
  const double eps = 2.220446049250313e-16;
  const double pert = eps * tnorm > 0.0 ? eps * tnorm : 1e-300;
  double a = d[0] - lam, b = r > 1 ? e[0] : 0.0;
#pragma unroll 4
  for (int k = 0; k < r - 1; ++k) {
    const double c = e[k];
    const double anext = d[k + 1] - lam;
    const double bnext = (k + 1 < r - 1) ? e[k + 1] : 0.0;
    const bool piv = fabs(a) >= fabs(c);
    const double ap = fabs(a) < pert ? (a < 0.0 ? -pert : pert) : a;
    const double ix = inv_d(piv ? ap : c);
    const double mlt = (piv ? c : a) * ix;
    ui[k] = ix;
    us1[k] = piv ? b : anext;
    ml[k] = mlt;
    sw[k] = piv ? 0 : 1;
    const double an = piv ? fma(-mlt, b, anext) : fma(-mlt, anext, b);
    b = piv ? bnext : -mlt * bnext;
    a = an;
  }
  ui[r - 1] = inv_d(fabs(a) < pert ? (a < 0.0 ? -pert : pert) : a);
  uint32_t st = 0x9E3779B9u ^ (uint32_t)(j * 2654435761u);
  for (int i = 0; i < r; ++i) {
    st = st * 1664525u + 1013904223u;
    z[i] = ((double)(st >> 8) / 16777216.0) - 0.5;
  }
  for (int iter = 0; iter < 2; ++iter) {
    // forward: apply the row operations (and swaps) of the elimination to z
    double cz = z[0];
#pragma unroll 4
    for (int k = 0; k < r - 1; ++k) {
      const double zo = z[k + 1];
      const double m = ml[k];
      const bool swp = sw[k] != 0;
      z[k] = swp ? zo : cz;
      cz = swp ? fma(-m, zo, cz) : fma(-m, cz, zo);
    }
    z[r - 1] = cz;
    // back substitution with U (diagonal 1/ui, superdiagonals us1 and us2)
    double z1 = 0.0, z2 = 0.0, nn = 0.0;
#pragma unroll 4
    for (int k = r - 1; k >= 0; --k) {
      const double u2 = (k < r - 1 && sw[k] != 0 && k + 1 < r - 1) ? e[k + 1] : 0.0;
      const double zk = (z[k] - us1[k] * z1 - u2 * z2) * ui[k];
      z[k] = zk;
      z2 = z1; z1 = zk;
      nn += zk * zk;
    }
    const double inv = nn > 0.0 ? 1.0 / sqrt(nn) : 0.0;
    for (int i = 0; i < r; ++i) z[i] *= inv;
  }
}

// acc + a b, acc - a b and acc + conj(a) b as four fused multiply-adds each
__device__ __forceinline__ zd zfma(zd a, zd b, zd acc) {
  return mk(fma(a.re, b.re, fma(-a.im, b.im, acc.re)), fma(a.re, b.im, fma(a.im, b.re, acc.im)));
}
__device__ __forceinline__ zd zfms(zd a, zd b, zd acc) {
  return mk(fma(-a.re, b.re, fma(a.im, b.im, acc.re)), fma(-a.re, b.im, fma(-a.im, b.re, acc.im)));
}
__device__ __forceinline__ zd zcfma(zd a, zd b, zd acc) {
  return mk(fma(a.re, b.re, fma(a.im, b.im, acc.re)), fma(a.re, b.im, fma(-a.im, b.re, acc.im)));
}
// acc - a conj(b)
__device__ __forceinline__ zd zfms_conj(zd a, zd b, zd acc) {
  return mk(fma(-a.re, b.re, fma(-a.im, b.im, acc.re)), fma(a.re, b.im, fma(-a.im, b.re, acc.im)));
}

constexpr int HEEV_UREG = 16;   // rows per lane of the register-resident back-transformation (r <= 128)

// G: F x r x r (full, column-major, only the lower triangle is read); U: F x r x r out;
// lam: F x r out (descending).  gpk: F x packed_size(r) global scratch (the reflectors; also the
// working matrix when !in_lds); zs: F x r x (r+1) doubles (eigenvectors of T when !in_lds);
// lu: F x r x 5r doubles (LU factors of T - lambda I).
// IN_LDS: the packed working matrix (and later Z) live in LDS; a template parameter so that LDS
// accesses compile to LDS instructions rather than generic (flat) ones.
// MODE 0: the whole solver.  MODE 1: the tridiagonal form was computed beforehand (k_hetrd_reg):
// tri holds d (r) then e (r) per face, taus the reflector scalars, gpk the reflectors; the kernel
// starts at the eigenvalues.  MODE 2: in addition the eigenvalues (lamout) and the eigenvectors of
// the tridiagonal (zs, stride r + 1) were computed by k_tri_stein; the kernel starts at the
// re-orthogonalization of clusters.  MODES 2 and 3 stop before the back-transformation, which
// k_heev_backtr does; MODE 3 runs from G (as MODE 0) and writes lamout and the reflector scalars
// (taus_out, F x r) for it.  MODE 4 only tridiagonalizes: d and e go to tri_out (as `tri` above),
// the reflector scalars to taus_out, the reflectors stay in gpk (the global working matrix).
template <bool IN_LDS, int MODE = 0>
__global__ void __launch_bounds__(HEEV_THREADS)
k_heev(const zd* __restrict__ Gin, int r, zd* __restrict__ Uout, double* __restrict__ lamout,
       zd* __restrict__ gpk, double* __restrict__ zs, double* __restrict__ lu,
       const double* __restrict__ tri, const zd* __restrict__ taus, zd* __restrict__ taus_out,
       double* __restrict__ tri_out) {
  static_assert(MODE != 4 || !IN_LDS, "the tridiagonalize-only mode keeps the reflectors in global memory");
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
  constexpr bool FROM_TRI = MODE == 1 || MODE == 2;
  if constexpr (FROM_TRI) {
    for (int j = tid; j < r; j += blockDim.x) {
      L.d[j] = tri[(int64_t)f * 2 * r + j];
      L.e[j] = tri[(int64_t)f * 2 * r + r + j];
      L.tau[j] = taus[(int64_t)f * r + j];
    }
    __syncthreads();
  } else {
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
  if constexpr (MODE == 4) {
    for (int j = tid; j < r; j += blockDim.x) {
      tri_out[(int64_t)f * 2 * r + j] = L.d[j];
      tri_out[(int64_t)f * 2 * r + r + j] = L.e[j];
      taus_out[(int64_t)f * r + j] = L.tau[j];
    }
    return;
  }
  }  // !FROM_TRI
  for (int i = tid; i < r; i += blockDim.x) L.e2[i] = L.e[i] * L.e[i];
  __syncthreads();

  RT_PHASE(2);
  // ---- eigenvalues of T: multisection, 8 lanes per eigenvalue ------------------------------
  const TriBounds tb = tri_bounds(L.d, L.e, L.e2, r);
  const double tnorm = tb.tnorm;
  if constexpr (MODE != 2) {
    for (int base = 0; base < r; base += ngrp) {
      const int j = base + grp;                      // j-th largest eigenvalue
      const bool on = j < r;
      const double lam = tri_eigval(L.d, L.e2, r, j, on, sub, tb);
      if (on && sub == 0) L.lam[j] = lam;
    }
  } else {
    for (int j = tid; j < r; j += blockDim.x) L.lam[j] = lamout[(int64_t)f * r + j];
  }
  __syncthreads();

  RT_PHASE(3);
  // ---- the reflectors move to global memory; LDS (or the global slice) then holds Z ------------
  // Z column j (stride zst = r + 1 doubles) = eigenvector of T for lam[j]
  if constexpr (IN_LDS && !FROM_TRI) {
    for (int64_t i = tid; i < packed_size(r); i += blockDim.x) Sg[i] = S[i];
    __syncthreads();
  }
  const int zst = r + 1;
  double* Zp;
  if constexpr (IN_LDS) Zp = reinterpret_cast<double*>(smem_raw + sizeof(HeevLds));
  else Zp = Z;

  // ---- eigenvectors of T: inverse iteration, one thread per eigenvalue ---------------------------
  if constexpr (MODE != 2) {
    for (int j = tid; j < r; j += blockDim.x)
      tri_invit(L.d, L.e, r, L.lam[j], tnorm, j, lu + ((int64_t)f * r + j) * 5 * r, Zp + (int64_t)j * zst);
  } else if constexpr (IN_LDS) {
    for (int64_t i = tid; i < (int64_t)r * zst; i += blockDim.x) Zp[i] = Z[i];
  }
  __syncthreads();
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
  // modified Gram-Schmidt inside every cluster (two passes).  Step i: every wave forms the pivot's
  // squared norm nn (the same arithmetic in each), and every later vector q of the cluster, one
  // wave per vector, loses (z_i . z_q / nn) z_i; the pivot itself is scaled to unit norm during
  // the next step (nobody reads it then), so one barrier per pivot suffices.
  for (int c = 0; c < L.ncl; ++c) {
    const int j0 = L.cstart[c], j1 = L.cstart[c + 1];
    if (j1 - j0 < 2) continue;
    for (int pass = 0; pass < 2; ++pass) {
      double pinv = 0.0;                     // 1/||z_{i-1}||, applied by wave (i-1) % nw
      for (int i = j0; i <= j1; ++i) {
        if (i > j0 && wave == (i - 1) % nw) {
          double* zp = Zp + (int64_t)(i - 1) * zst;
          for (int x = lane; x < r; x += 64) zp[x] *= pinv;
        }
        if (i == j1) break;
        const double* zi = Zp + (int64_t)i * zst;
        // the pivot's norm and up to 3 of this wave's dot products as independent reductions
        int q = i + 1 + wave;
        double nn = 0.0, dt[3] = {0.0, 0.0, 0.0};
        for (int x = lane; x < r; x += 64) {
          const double zx = zi[x];
          nn += zx * zx;
#pragma unroll
          for (int u = 0; u < 3; ++u)
            if (q + u * nw < j1) dt[u] += zx * Zp[(int64_t)(q + u * nw) * zst + x];
        }
        nn = wave_sum(nn);
#pragma unroll
        for (int u = 0; u < 3; ++u) dt[u] = wave_sum(dt[u]);
        const double inn = nn > 0.0 ? 1.0 / nn : 0.0;
        pinv = nn > 0.0 ? sqrt(inn) : 0.0;
#pragma unroll
        for (int u = 0; u < 3; ++u)
          if (q + u * nw < j1) {
            double* zq = Zp + (int64_t)(q + u * nw) * zst;
            const double c = dt[u] * inn;
            for (int x = lane; x < r; x += 64) zq[x] -= c * zi[x];
          }
        for (q += 3 * nw; q < j1; q += nw) {   // clusters longer than 3 nw + 1
          double* zq = Zp + (int64_t)q * zst;
          double d1 = 0.0;
          for (int x = lane; x < r; x += 64) d1 += zi[x] * zq[x];
          d1 = wave_sum(d1) * inn;
          for (int x = lane; x < r; x += 64) zq[x] -= d1 * zi[x];
        }
        __syncthreads();
      }
      __syncthreads();
    }
  }
  __syncthreads();
  if constexpr (MODE >= 2) {
    // the back-transformation runs in k_heev_backtr
    if constexpr (MODE == 3) {
      for (int j = tid; j < r; j += blockDim.x) {
        taus_out[(int64_t)f * r + j] = L.tau[j];
        lamout[(int64_t)f * r + j] = L.lam[j];
      }
    }
    if constexpr (IN_LDS) {
      for (int64_t i = tid; i < (int64_t)r * zst; i += blockDim.x) Z[i] = Zp[i];
    }
    return;
  }

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
// Eigenvalues and tridiagonal eigenvectors, STEIN_EPB eigenvalues per block (grid ceil(r/EPB) x F)
// -------------------------------------------------------------------------------------------
// Spreads the eigenvalue multisection (8 lanes per eigenvalue) and the inverse iterations (one
// lane per eigenvalue, LU factors in LDS) of every face over many workgroups; k_heev<., 2> then
// re-orthogonalizes clusters and back-transforms.  tri: d (r) then e (r) per face; lamout: F x r
// (descending); zs: F x r x (r + 1) doubles (column j = eigenvector of the tridiagonal for lam_j).
constexpr int STEIN_EPB = 8;
constexpr int STEIN_THREADS = 8 * STEIN_EPB;
// d, e, e^2; per eigenvalue: z, 1/pivots, U's first superdiagonal, multipliers (doubles), swaps (ints)
inline size_t stein_lds_bytes(int r) {
  return (size_t)(3 * r + STEIN_EPB * 4 * r) * sizeof(double) + (size_t)STEIN_EPB * r * sizeof(int);
}

__global__ void __launch_bounds__(STEIN_THREADS)
k_tri_stein(const double* __restrict__ tri, int r, double* __restrict__ lamout, double* __restrict__ zs) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  double* d = reinterpret_cast<double*>(smem_raw);
  double* e = d + r;
  double* e2 = e + r;
  double* lu = e2 + r;                    // STEIN_EPB x 3 r
  double* zl = lu + STEIN_EPB * 3 * r;    // STEIN_EPB x r
  int* swl = reinterpret_cast<int*>(zl + STEIN_EPB * r);   // STEIN_EPB x r
  double* ds = zl;                        // prescaled copies for the Sturm counts, overwritten
  double* e2s = zl + r;                   // by the eigenvectors afterwards (2 r <= STEIN_EPB r)
  __shared__ double lams[STEIN_EPB];
  const int f = blockIdx.y, j0 = blockIdx.x * STEIN_EPB;
  const int tid = threadIdx.x, sub = tid & 7, grp = tid >> 3;
  for (int i = tid; i < r; i += blockDim.x) {
    d[i] = tri[(int64_t)f * 2 * r + i];
    const double ei = tri[(int64_t)f * 2 * r + r + i];
    e[i] = ei;
    e2[i] = ei * ei;
  }
  __syncthreads();
  const TriBounds tb = tri_bounds(d, e, e2, r);
  // power-of-two scale with s ||T|| <= 1
  const double sc = tb.tnorm > 0.0 ? ldexp(1.0, -__builtin_amdgcn_frexp_exp(tb.tnorm)) : 1.0;
  for (int i = tid; i < r; i += blockDim.x) {
    ds[i] = d[i] * sc;
    e2s[i] = e2[i] * (sc * sc);
  }
  __syncthreads();
  const int j = j0 + grp;
  const bool on = j < r;
  const double lam = tri_eigval_minors(ds, e2s, sc, r, j, on, sub, tb);
  if (sub == 0) {
    lams[grp] = lam;
    if (on) lamout[(int64_t)f * r + j] = lam;
  }
  __syncthreads();
  if (tid < STEIN_EPB && j0 + tid < r) {
    double* z = zl + tid * r;
    double* l3 = lu + tid * 3 * r;
    tri_invit_lds(d, e, r, lams[tid], tb.tnorm, j0 + tid, l3, l3 + r, l3 + 2 * r, swl + tid * r, z);
  }
  __syncthreads();
  // eigenvectors out (column j0 + q, stride r + 1)
  const int nq = min(STEIN_EPB, r - j0);
  for (int idx = tid; idx < nq * r; idx += blockDim.x) {
    const int q = idx / r, i = idx % r;
    zs[((int64_t)f * r + j0 + q) * (r + 1) + i] = zl[q * r + i];
  }
}

// -------------------------------------------------------------------------------------------
// Back-transformation U = Q_H Z for r <= 8 HEEV_UREG, BT_COLS columns per block (grid ceil(r/BT_COLS) x F)
// -------------------------------------------------------------------------------------------
// Column c of U is Z(:, c) with H_{r-2}, ..., H_0 applied (H_k = I - tau_k v_k v_k^H): 8 lanes per
// column, lane s holds rows s + 8 t in registers; the reflectors pass through LDS in chunks of
// BT_CH (dense rows, zero above the sub-diagonal), last chunk first.  gpk: packed reflectors,
// taus: F x r, zs: F x r x (r + 1) (real Z), U: F x r x r out.
constexpr int BT_COLS = 32;
constexpr int BT_THREADS = 8 * BT_COLS;
constexpr int BT_CH = 32;
// UREG rows per lane (r <= 8 UREG), CH reflectors per LDS chunk: (16, 32) for r <= 128 and
// (32, 15) for r <= 256 (the chunk of dense reflector rows stays under 64 KB)
constexpr int BT_UREG_WIDE = 32, BT_CH_WIDE = 15;

template <int UREG, int CH>
__global__ void __launch_bounds__(BT_THREADS)
k_heev_backtr(const zd* __restrict__ gpk, const zd* __restrict__ taus, const double* __restrict__ zs, int r,
              zd* __restrict__ Uout) {
  constexpr int BT_RP = 8 * UREG;   // padded rows
  constexpr int BT_CH = CH;
  constexpr int HEEV_UREG = UREG;
  __shared__ zd vbuf[BT_CH][BT_RP];
  __shared__ zd tbuf[BT_CH];
  const int f = blockIdx.y;
  const int tid = threadIdx.x, sub = tid & 7, grp = tid >> 3;
  const int c = blockIdx.x * BT_COLS + grp;
  const bool on = c < r;
  const zd* __restrict__ S = gpk + (int64_t)f * packed_size(r);
  const zd* __restrict__ tf = taus + (int64_t)f * r;
  const double* __restrict__ Z = zs + (int64_t)f * r * (r + 1) + (int64_t)(on ? c : 0) * (r + 1);
  zd u[HEEV_UREG];
#pragma unroll
  for (int t = 0; t < HEEV_UREG; ++t) {
    const int i = sub + 8 * t;
    u[t] = mk((on && i < r) ? Z[i] : 0.0, 0.0);
  }
  const int nref = r - 1;
  for (int kc0 = ((nref - 1) / BT_CH) * BT_CH; kc0 >= 0; kc0 -= BT_CH) {
    const int kc1 = min(kc0 + BT_CH, nref);
    __syncthreads();
    for (int idx = tid; idx < BT_CH * BT_RP; idx += BT_THREADS) {
      const int kk = idx / BT_RP, i = idx % BT_RP, k = kc0 + kk;
      zd v = mk(0.0, 0.0);
      if (k < kc1 && i > k && i < r) v = S[pk_off(k, r) + (i - k)];
      vbuf[kk][i] = v;
    }
    if (tid < BT_CH) tbuf[tid] = kc0 + tid < kc1 ? tf[kc0 + tid] : mk(0.0, 0.0);
    __syncthreads();
    for (int k = kc1 - 1; k >= kc0; --k) {
      const zd tau = tbuf[k - kc0];
      const zd* vk = vbuf[k - kc0];
      zd part[4] = {mk(0.0, 0.0), mk(0.0, 0.0), mk(0.0, 0.0), mk(0.0, 0.0)};
#pragma unroll
      for (int t = 0; t < HEEV_UREG; ++t) part[t & 3] = zcfma(vk[sub + 8 * t], u[t], part[t & 3]);  // zeros above
      zd sacc = cadd(cadd(part[0], part[1]), cadd(part[2], part[3]));
      sacc = cadd(sacc, dpp<DPP_XOR1>(sacc));
      sacc = cadd(sacc, dpp<DPP_XOR2>(sacc));
      sacc = cadd(sacc, dpp<DPP_MIRROR8>(sacc));
      sacc = cmul(tau, sacc);
#pragma unroll
      for (int t = 0; t < HEEV_UREG; ++t) u[t] = zfms(vk[sub + 8 * t], sacc, u[t]);
    }
  }
  if (on) {
    zd* U = Uout + (int64_t)f * r * r + (int64_t)c * r;
#pragma unroll
    for (int t = 0; t < HEEV_UREG; ++t) {
      const int i = sub + 8 * t;
      if (i < r) U[i] = u[t];
    }
  }
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
// tiles spread over the waves.  L^{-1} is formed by block rows during the same sweep:
//   Linv(K, J) = -D_K sum_{J <= M < K} L(K, M) Linv(M, J)  (MFMA tiles),  Linv(K, K) = D_K,
// by waves 1.. while wave 0 factors the next diagonal block, and written over L's block row K.
// A pivot at or below tol_rel * max diag marks a dependent column: its row and column of L^{-1}
// are zero and flags gets bit 0.  The packed lower triangle lives in LDS when it fits (else in
// `gpk`, global scratch of packed_size(r) per face); `gdi` (F x ceil(r/16) x 256) keeps the block
// inverses D_K for the block rows of L^{-1}.  Guarded operand loads read a clamped in-range element and
// select zero by value: a conditional between an LDS element and a zero object would become a
// generic (flat) load, whose wait also covers the wave's outstanding global stores.
// ---------------------------------------------------------------------------------------------
constexpr int CH_NB = 16, CH_PS = CH_NB + 1;  // block width, padded row stride of the panel buffers
constexpr int CH_THREADS = 512;
constexpr int CH_LOAD_COLS = 16;
          // columns per wave and load round (all of r <= 128 at once)

struct CholHdr {
  double tol;
  int bad;
  int pad_;
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
  const int nblk = (r + CH_NB - 1) / CH_NB;
  __shared__ zd chx[2][CH_NB];                // column c of L (double-buffered)
  __shared__ zd LT[CH_NB][CH_NB];             // LT[c][t] = conj(L(t, c)) for t > c, LT[c][c] = 1 / L(c, c)
  __shared__ int tq;                          // next trailing-update tile of the step
  // packed lower storage, column j at j r - j (j - 1) / 2
  auto at = [&](int i, int j) -> zd& { return S[j * r - (j * (j - 1)) / 2 + (i - j)]; };  // i >= j

  // ---- wave 0: factor a diagonal block held in registers ----
  // Lane (rho, g) holds entries (i, j_s) = (rho, g + 4 s) of the block (identity-padded when it
  // is narrower than 16, so its extra pivots are 1).  Column c is exchanged through LDS once its
  // pivot is known; the entries right of column c then take the rank-one update, slots whose
  // columns are all done being skipped.  Entries above the diagonal are never read.  A pivot at
  // or below tol marks a dependent column: its column of L is zero and H.bad is set.  Writes LT.
  auto factor_core = [&](int Kb, zd (&a)[4], double tl, auto tiny_range) {
    constexpr bool TINY = decltype(tiny_range)::value;   // tol may be at or below 1e-280
    const int K = CH_NB * Kb, kb = min(CH_NB, r - K);
    double myipv = 1.0;    // 1 / L(rho, rho) once column rho is factored
#pragma unroll
    for (int c = 0; c < CH_NB; ++c) {
      const int cs = c & 3, sl = c >> 2;
      const zd ac = a[sl];
      const double dd = __hiloint2double(__builtin_amdgcn_readlane(__double2hiint(ac.re), c + 16 * cs),
                                         __builtin_amdgcn_readlane(__double2loint(ac.re), c + 16 * cs));
      // 1 / sqrt(dd) without branches (dd is wave-uniform): one reciprocal square root; only when
      // tol is that small can a live pivot lie near the bottom of the normal range, and then dd
      // is scaled by 2^600 first.  A dependent or padding column gets 0 or 1.
      const bool live = c < kb && dd > tl && dd > 0.0;
      double ipv0;
      if constexpr (TINY) {
        const bool tiny = dd <= 1e-280;
        const double y = rsqrt_d(tiny ? dd * 0x1p+600 : dd);
        ipv0 = tiny ? y * 0x1p+300 : y;
      } else {
        ipv0 = rsqrt_d(dd);
      }
      const double ipv = c < kb ? (live ? ipv0 : 0.0) : 1.0;
      myipv = (rho == c) ? ipv : myipv;
      // column c of L: the lanes holding it scale it (its diagonal entry and the rows above are
      // never read again)
      const zd acn = zsel(g == cs, cscale(ac, ipv), ac);
      a[sl] = acn;
      if (g == cs) chx[c & 1][rho] = acn;
      __builtin_amdgcn_wave_barrier();
      const zd lic = chx[c & 1][rho];          // L(rho, c)
#pragma unroll
      for (int s2 = 0; s2 < 4; ++s2) {
        if (s2 < sl) continue;                 // columns g + 4 s2 < c: done
        const zd ljc = chx[c & 1][g + 4 * s2];  // L(j_s, c)
        const zd upd2 = zfms_conj(lic, ljc, a[s2]);
        a[s2] = (s2 == sl) ? zsel(g + 4 * s2 > c, upd2, a[s2]) : upd2;
      }
    }
    if (rho < kb && myipv == 0.0) H.bad = 1;   // a dependent column
#pragma unroll
    for (int s2 = 0; s2 < 4; ++s2) {
      const int j = g + 4 * s2;
      if (rho > j) LT[j][rho] = cconj(a[s2]);
      if (rho == j) LT[j][j] = mk(myipv, 0.0);
    }
  };
  auto factor_block = [&](int Kb, zd (&a)[4], double tl) {
    if (tl > 1e-280) factor_core(Kb, a, tl, std::false_type{});
    else factor_core(Kb, a, tl, std::true_type{});
  };

  // ---- wave 0: D_Kb = L_KK^{-1} from the factored block in LT ----
  // Sixteen rows, the identity rows e_i', solve x L_KK^H = e_i', so x = row i' of L_KK^{-H} and
  // D(:, i') = conj(x).  Four lanes per row (lane 4 i' + h holds columns h + 4 s).  Columns left to
  // right: the owner of column c scales it, x_c = g_c / L(c, c), and passes it to its quad by DPP;
  // columns t > c subtract x_c conj(L(t, c)).  A dependent column has 1 / L(c, c) = 0 and gives a
  // zero row and column of D.  D goes to DI (for the panel) and GD (for L^{-1}), zero outside kb.
  auto diag_inverse = [&](int Kb) {
    const zd zero = mk(0.0, 0.0);
    const int K = CH_NB * Kb, kb = min(CH_NB, r - K);
    const int id = lane >> 2, gq = lane & 3;
    zd gv[4];
#pragma unroll
    for (int s = 0; s < 4; ++s) gv[s] = mk(gq + 4 * s == id ? 1.0 : 0.0, 0.0);
    static_for<0, CH_NB>([&](auto cc) {
      constexpr int c = decltype(cc)::value, cs = c & 3, sl = c >> 2;
      const zd own = cscale(gv[sl], LT[c][c].re);
      const zd p = dpp<cs * 0x55>(own);                     // quad_perm [cs, cs, cs, cs]
      {
        const zd u = zfms(p, LT[c][gq + 4 * sl], gv[sl]);
        gv[sl] = zsel(gq == cs, p, zsel(gq > cs, u, gv[sl]));
      }
      static_for<sl + 1, 4>([&](auto ss) {
        constexpr int s = decltype(ss)::value;
        gv[s] = zfms(p, LT[c][gq + 4 * s], gv[s]);
      });
    });
#pragma unroll
    for (int s = 0; s < 4; ++s) {
      const int t = gq + 4 * s;
      const zd dv = zsel(t < kb && id < kb, cconj(gv[s]), zero);   // D(t, id)
      DI[t * CH_PS + id] = dv;
      GD[Kb * CH_NB * CH_NB + t * CH_NB + id] = dv;
    }
  };

  // ---- panel of step Kb: P(i, c) = sum_t S(i, K + t) conj(D(c, t)), rows i >= K1 ----
  // 16-row MFMA tiles over the waves; the panel goes over the block column of S (it is L's) and
  // into P for the trailing update.
  auto panel = [&](int Kb) {
    const zd zero = mk(0.0, 0.0);
    const int K = CH_NB * Kb, kb = min(CH_NB, r - K), K1 = K + kb, m = r - K1;
    for (int ti = wave; ti * 16 < m; ti += nw) {
      const int i0 = K1 + 16 * ti;
      ch_f64x4 cr = {0, 0, 0, 0}, ci = {0, 0, 0, 0};
#pragma unroll
      for (int kg = 0; kg < 4; ++kg) {
        const int k = 4 * kg + g;
        const zd av = zsel(i0 + rho < r && k < kb, at(min(i0 + rho, r - 1), K + min(k, kb - 1)), zero);
        const zd bv = zsel(k < kb && rho < kb, cconj(DI[rho * CH_PS + k]), zero);
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
  };

  // ---- L^{-1} by block rows, beside the factorization ----
  // Block row Kp of L^{-1}: Linv(Kp, jt) = -D_Kp sum_{jt <= mb < Kp} L(Kp, mb) Linv(mb, jt) for
  // jt < Kp, and Linv(Kp, Kp) = D_Kp.  It needs only L's block row Kp (final once the panel of
  // step Kp - 1 is written) and block rows < Kp of L^{-1}, so waves 1.. compute it in registers
  // in the update phase of step Kp and store it in the panel phase of step Kp + 1, over L's block
  // row Kp, and its conjugate transpose into Rinv's block column Kp.  D_Kp is read back from GD.
  // An MFMA output tile (lane: rows 4 v + g of column rho) is laid out as the B operand of the
  // next product, so T = sum L Linv feeds D T directly.
  constexpr int LT_MAX = IN_LDS ? 1 : 3;   // tiles per wave: r <= 128 in LDS (<= 7), else <= 15
  ch_f64x4 lr[LT_MAX], li[LT_MAX];
  const int nlw = nw - 1;                  // waves 1 .. nw - 1 compute the block rows
  // first tile column of this wave: waves 1, 2, 3, 5, 6, 7 take 0 .. 5 (the longest rows on
  // distinct SIMDs), wave 4 the last: it shares its SIMD with wave 0, whose factorization is the
  // step's critical path, so it takes no other work
  const int ljt = wave < 4 ? wave - 1 : (wave == 4 ? nw - 2 : wave - 2);
  auto linv_tiles = [&](int Kp) {
    const zd zero = mk(0.0, 0.0);
    const int row = CH_NB * Kp + rho, rowc = min(row, r - 1);
#pragma unroll
    for (int u = 0; u < LT_MAX; ++u) {
      const int jt = ljt + nlw * u;
      lr[u] = (ch_f64x4){0, 0, 0, 0};
      li[u] = lr[u];
      if (jt >= Kp) continue;                // uniform per wave
      ch_f64x4 tr = {0, 0, 0, 0}, ti = {0, 0, 0, 0};
      const int col = CH_NB * jt + rho;
      for (int mb = jt; mb < Kp; ++mb) {
#pragma unroll
        for (int kg = 0; kg < 4; ++kg) {
          const int k = CH_NB * mb + 4 * kg + g;                  // < CH_NB Kp <= rowc
          const zd av = zsel(row < r, at(rowc, k), zero);          // L(row, k)
          const zd bv = zsel(k >= col, at(k, min(col, k)), zero);  // Linv(k, col), lower
          ch_cmma(av, bv, tr, ti);
        }
      }
      const zd* __restrict__ Dg = GD + Kp * CH_NB * CH_NB;
#pragma unroll
      for (int kg = 0; kg < 4; ++kg) ch_cmma(Dg[rho * CH_NB + 4 * kg + g], mk(tr[kg], ti[kg]), lr[u], li[u]);
    }
  };
  // block row Kp of L^{-1} over L's, Rinv(:, block Kp) = its conjugate transpose, zero below
  auto linv_store = [&](int Kp) {
    const zd zero = mk(0.0, 0.0);
    const int K = CH_NB * Kp, kb = min(CH_NB, r - K);
    if (wave > 0) {
#pragma unroll
      for (int u = 0; u < LT_MAX; ++u) {
        const int jt = ljt + nlw * u;
        if (jt >= Kp) continue;
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int i = K + 4 * v + g, c = CH_NB * jt + rho;
          if (i < r) {
            at(i, c) = mk(-lr[u][v], -li[u][v]);
            R[(int64_t)i * r + c] = mk(-lr[u][v], li[u][v]);
          }
        }
      }
    }
    for (int q = tid; q < CH_NB * CH_NB; q += blockDim.x) {
      const int i = q / CH_NB, c = q % CH_NB;
      if (i < kb && c < kb) {
        const zd dv = GD[Kp * CH_NB * CH_NB + q];
        if (i >= c) at(K + i, K + c) = dv;
        R[(int64_t)(K + i) * r + K + c] = cconj(dv);   // zero for c > i
      }
    }
    const int below = r - (K + kb);
    for (int q = tid; q < kb * below; q += blockDim.x) {
      const int c = q / below, i = K + kb + q % below;
      R[(int64_t)(K + c) * r + i] = zero;
    }
  };

  RT_PHASE(7);
  if (wave == 0) {
    // tol from the diagonal of G, and diagonal block 0 straight from G, factored while the other
    // waves load the lower triangle
    if (lane == 0) H.bad = 0;
    const int kb0 = min(CH_NB, r);
    double mx = 0.0;
    for (int j = lane; j < r; j += 64) mx = fmax(mx, G[(int64_t)j * r + j].re);
    zd a[4];
#pragma unroll
    for (int s2 = 0; s2 < 4; ++s2) {
      const int j = g + 4 * s2;
      const bool in = rho < kb0 && j < kb0 && rho >= j;
      zd v = mk(rho == j ? 1.0 : 0.0, 0.0);
      if (in) v = G[(int64_t)j * r + rho];
      a[s2] = v;
    }
    for (int o = 32; o > 0; o >>= 1) mx = fmax(mx, __shfl_xor(mx, o));
    const double tl = tol_rel * mx;
    if (lane == 0) H.tol = tl;
    factor_block(0, a, tl);
    diag_inverse(0);
  } else {
    // lower triangle, column by column (rows j.. of column j are contiguous in G and in S), all
    // loads of a round in flight together
    const int lw = wave - 1, nlw_ = nw - 1;
    for (int j0 = lw; j0 < r; j0 += CH_LOAD_COLS * nlw_) {
      zd v[CH_LOAD_COLS][2];
#pragma unroll
      for (int u = 0; u < CH_LOAD_COLS; ++u)
#pragma unroll
        for (int h = 0; h < 2; ++h) {
          const int j = j0 + nlw_ * u, i = j + lane + 64 * h;
          v[u][h] = (j < r && i < r) ? G[(int64_t)j * r + i] : mk(0.0, 0.0);
        }
#pragma unroll
      for (int u = 0; u < CH_LOAD_COLS; ++u)
#pragma unroll
        for (int h = 0; h < 2; ++h) {
          const int j = j0 + nlw_ * u, i = j + lane + 64 * h;
          if (j < r && i < r) at(i, j) = v[u][h];
        }
      for (int u = 0; u < CH_LOAD_COLS; ++u) {   // columns longer than 128 rows (r > 128 only)
        const int j = j0 + nlw_ * u;
        for (int i = j + lane + 128; j < r && i < r; i += 64) at(i, j) = G[(int64_t)j * r + i];
      }
    }
  }
  __syncthreads();
  const double tol = H.tol;
  RT_PHASE(8);
  RT_PHASE(12);

  // ---- blocked right-looking Cholesky with look-ahead ----
  for (int Kb = 0; Kb < nblk; ++Kb) {
    const int K = CH_NB * Kb, kb = min(CH_NB, r - K), K1 = K + kb, m = r - K1;
    // (b) block row Kb - 1 of L^{-1} out of the registers, the panel of block Kb and D_Kb
    if (Kb >= 1) linv_store(Kb - 1);   // rows of block Kb - 1: disjoint from the panel below
    if (tid == 0) tq = 1;              // tile 0 of the trailing update is wave 0's
    panel(Kb);
    __syncthreads();
    if (Kb == 0) RT_PHASE(13);
    if (Kb == 3) RT_PHASE(15);
    // (c) trailing update S(i, j) -= sum_c P(i, c) conj(P(j, c)), lower 16 x 16 tiles: wave 0
    // takes the first diagonal tile in registers and factors it (the next step's diagonal block);
    // waves 1.. take the other tiles, then block row Kb of L^{-1}
    if (wave == 0) {
      if (Kb + 1 < nblk) {
        // diagonal block Kb + 1 with the update of this step's panel: lane (rho, g) gets
        // T(rho, j_s) of T = P P^H as entry s of an MFMA tile with operands conj(P) and P, the
        // products and their order being those of the other tiles
        const int Kn = K1, kbn = min(CH_NB, r - Kn);
        zd a[4];
#pragma unroll
        for (int s2 = 0; s2 < 4; ++s2) {
          const int j = g + 4 * s2;
          const bool in = rho < kbn && j < kbn && rho >= j;
          const int ic = min(Kn + rho, r - 1), jc = min(Kn + j, ic);   // in range when !in
          a[s2] = zsel(in, at(ic, jc), mk(rho == j ? 1.0 : 0.0, 0.0));
        }
        ch_f64x4 cr = {0, 0, 0, 0}, ci = {0, 0, 0, 0};
        const zd* Prow = P + (size_t)min(Kn + rho, r - 1) * CH_PS;
#pragma unroll
        for (int kg = 0; kg < 4; ++kg) {
          const zd b = Prow[4 * kg + g];
          cr = ch_mma(b.re, b.re, cr);
          cr = ch_mma(b.im, b.im, cr);
          ci = ch_mma(-b.im, b.re, ci);
          ci = ch_mma(b.re, b.im, ci);
        }
#pragma unroll
        for (int s2 = 0; s2 < 4; ++s2) {
          const int j = g + 4 * s2;
          const bool in = rho < kbn && j < kbn && rho >= j;
          a[s2] = zsel(in, csub(a[s2], mk(cr[s2], ci[s2])), a[s2]);
        }
        if (Kb == 3) RT_MARK(18);
        factor_block(Kb + 1, a, tol);
        diag_inverse(Kb + 1);
        if (Kb == 3) RT_MARK(19);
      }
    } else {
      const zd zero = mk(0.0, 0.0);
      const int T = (m + 15) / 16, ntile = T * (T + 1) / 2;
      linv_tiles(Kb);
      // the trailing tiles other than the first come from a queue: waves with short or no rows
      // of L^{-1} take more of them
      for (; wave != 4;) {
        int q0 = 0;
        if (lane == 0) q0 = atomicAdd(&tq, 1);
        const int q = __builtin_amdgcn_readfirstlane(q0);
        if (q >= ntile) break;
        int ti = (int)((sqrtf(8.0f * q + 1.0f) - 1.0f) * 0.5f);
        while (ti * (ti + 1) / 2 > q) --ti;
        while ((ti + 1) * (ti + 2) / 2 <= q) ++ti;
        const int tj = q - ti * (ti + 1) / 2;
        const int i0 = K1 + 16 * ti, j0 = K1 + 16 * tj;
        ch_f64x4 cr = {0, 0, 0, 0}, ci = {0, 0, 0, 0};
#pragma unroll
        for (int kg = 0; kg < 4; ++kg) {
          const int k = 4 * kg + g;
          const zd av = zsel(i0 + rho < r && k < kb, P[(size_t)min(i0 + rho, r - 1) * CH_PS + k], zero);
          const zd bv = zsel(j0 + rho < r && k < kb, cconj(P[(size_t)min(j0 + rho, r - 1) * CH_PS + k]), zero);
          ch_cmma(av, bv, cr, ci);
        }
        static_for<0, 4>([&](auto vv) {
          constexpr int v = decltype(vv)::value;
          const int i = i0 + g + 4 * v, j = j0 + rho;
          if (i < r && j < r && i >= j) at(i, j) = csub(at(i, j), mk(cr[v], ci[v]));
        });
      }
    }
    __syncthreads();
    if (Kb == 0) RT_PHASE(14);
    if (Kb == 2) RT_PHASE(16);
    if (Kb == 3) RT_PHASE(17);
  }
  RT_PHASE(9);
  linv_store(nblk - 1);
  RT_PHASE(10);
  RT_PHASE(11);
  if (tid == 0 && flags && H.bad) atomicOr(flags, 1);
}

// -------------------------------------------------------------------------------------------
// Register-resident Householder tridiagonalization for r <= TRD_R (one 512-thread block per face)
// -------------------------------------------------------------------------------------------
// The (zero-padded) 128 x 128 Hermitian matrix lives in registers, full storage: thread
// (wave w, lane l) owns rows 4a.. 4a+3 at the eight columns b, b+16, ..., b+112, with a = 4w + l/16,
// b = l%16 (two waves per SIMD, 32 complex entries per lane).  Every lane thus holds one column of
// each 16-column block, so a block whose columns are all eliminated is skipped by a wave-uniform
// branch.  Per reflector k (x = A(k+1:, k)):
//   (1) the owners of column k put it in LDS; barrier;
//   (2) every wave forms H = I - tau v v^H with H^H x = beta e_1 from it (the same arithmetic in
//       every wave) and keeps v in a wave-private LDS row;
//   (3) p = tau A v: 4 x 8 block products, summed over the 16 lanes of a row group by a
//       reduce-scatter, p^H v summed per wave; barrier;
//   (4) w = p - (tau p^H v / 2) v, A -= v w^H + w v^H on the owned block.
// Waves whose 16 rows are all eliminated skip (3) and (4), and the others skip the column blocks
// left of column k + 1 (v and w vanish there).  FP64 throughput of the vector ALUs bounds the
// kernel (12 FMAs per stored entry and reflector).  Output: d, e (real tridiagonal,
// e_k = beta_k), tau, and v_k (rows k+1..r-1, v_k(k+1) = 1) in the packed layout of k_heev.
constexpr int TRD_R = 128;
constexpr int TRD_THREADS = 512;
constexpr int TRD_WAVES = TRD_THREADS / 64;
// LDS vectors are stored unpadded: the 16 lanes of a row group read 16 consecutive entries (one
// per column block), the four row groups of a wave read the same or neighbouring ones.
constexpr int TRD_RP = TRD_R;
__device__ __forceinline__ int trd_p(int t) { return t; }

__device__ __forceinline__ zd shfl_xor_z(zd v, int o) { return mk(__shfl_xor(v.re, o, 64), __shfl_xor(v.im, o, 64)); }


__global__ void __launch_bounds__(TRD_THREADS)
k_hetrd_reg(const zd* __restrict__ Gin, int r, double* __restrict__ tri, zd* __restrict__ taus,
            zd* __restrict__ gpk) {
  __shared__ zd xcol[2][TRD_RP];
  __shared__ zd xsh[2][TRD_RP];
  __shared__ zd xv[2][TRD_WAVES];
  __shared__ zd vpriv[TRD_WAVES][TRD_RP];
  const int f = blockIdx.x;
  const int tid = threadIdx.x, w = tid >> 6, l = tid & 63;
  const int a = 4 * w + (l >> 4), b = l & 15;
  const int r0 = 4 * a;
  const zd* __restrict__ G = Gin + (int64_t)f * r * r;
  zd* __restrict__ S = gpk + (int64_t)f * packed_size(r);
  double* __restrict__ dout = tri + (int64_t)f * 2 * r;
  double* __restrict__ eout = dout + r;
  zd* __restrict__ vp = vpriv[w];
  zd A[4][8];
#pragma unroll
  for (int ii = 0; ii < 4; ++ii)
#pragma unroll
    for (int jj = 0; jj < 8; ++jj) {
      const int i = r0 + ii, j = 16 * jj + b;
      zd v = mk(0.0, 0.0);
      if (i < r && j < r) v = i >= j ? G[i + (int64_t)j * r] : cconj(G[j + (int64_t)i * r]);
      A[ii][jj] = v;
    }
  const bool b3 = (l & 8) != 0, b2 = (l & 4) != 0;
  const int myrow = r0 + 2 * (int)b3 + (int)b2;   // row held after the reduce-scatter
  for (int k = 0; k < r - 1; ++k) {
    const int par = k & 1;
    // (1) column k into LDS (entries 0..127; the diagonal entry gives d_k).  k is uniform, so the
    // column is picked by a uniform branch, not by per-lane selects.
    if (b == (k & 15)) {
      const int jk = k >> 4;
#pragma unroll
      for (int jj = 0; jj < 8; ++jj)
        if (jk == jj) {
#pragma unroll
          for (int ii = 0; ii < 4; ++ii) xcol[par][trd_p(r0 + ii)] = A[ii][jj];
        }
    }
    __syncthreads();
    // (2) the reflector (identical in every wave)
    double xn = 0.0;
#pragma unroll
    for (int t0 = 0; t0 < TRD_R; t0 += 64) {
      const int t = t0 + l;
      const zd xt = xcol[par][trd_p(t)];
      xn += (t >= k + 2 && t < r) ? cabs2(xt) : 0.0;
    }
    xn = wave_sum(xn);
    const zd alpha = xcol[par][trd_p(k + 1)];
    const bool active = (xn > 0.0 || alpha.im != 0.0);   // uniform
    double beta = alpha.re;
    zd tau = mk(0.0, 0.0), sc = mk(0.0, 0.0);
    if (active) {
      // the norm, 1/beta and 1/|alpha - beta|^2 by Newton-refined hardware estimates (the values
      // are wave-uniform, so the branch to the IEEE operations near the bottom of the normal
      // range is uniform too)
      const double nn = alpha.re * alpha.re + alpha.im * alpha.im + xn;
      const bool normal = nn > 1e-280;
      const double nrm = normal ? nn * rsqrt_d(nn) : sqrt(nn);
      beta = alpha.re >= 0.0 ? -nrm : nrm;
      const double ib = normal ? inv_d(beta) : 1.0 / beta;
      tau = mk((beta - alpha.re) * ib, -alpha.im * ib);
      const zd den = mk(alpha.re - beta, alpha.im);
      const double dd2 = cabs2(den);
      const double idd = normal ? inv_d(dd2) : 1.0 / dd2;
      sc = mk(den.re * idd, -den.im * idd);
    }
#pragma unroll
    for (int t0 = 0; t0 < TRD_R; t0 += 64) {
      const int t = t0 + l;
      const zd sv = cmul(xcol[par][trd_p(t)], sc);
      const zd vt = zsel(t == k + 1, mk(1.0, 0.0), zsel(t > k + 1 && t < r && active, sv, mk(0.0, 0.0)));
      vp[trd_p(t)] = vt;
      if (w == 0 && t > k && t < r) S[pk_off(k, r) + (t - k)] = vt;
    }
    if (w == 0 && l == 0) {
      dout[k] = xcol[par][trd_p(k)].re;
      eout[k] = beta;
      taus[(int64_t)f * r + k] = tau;
    }
    if (!active) continue;           // uniform: H = I, nothing to update
    const bool wave_on = 16 * w + 15 > k;
    // first column block with a column right of k (uniform)
    const int jb0 = (k + 1) >> 4;
    if (wave_on) {
      // (3) p = tau A v over the owned block, reduce-scatter over the 16-lane row group
      zd sp[4];
#pragma unroll
      for (int ii = 0; ii < 4; ++ii) sp[ii] = mk(0.0, 0.0);
#pragma unroll
      for (int jj = 0; jj < 8; ++jj)
        if (jj >= jb0) {
          const zd vj = vp[trd_p(16 * jj + b)];
#pragma unroll
          for (int ii = 0; ii < 4; ++ii) sp[ii] = zfma(A[ii][jj], vj, sp[ii]);
        }
      // partners: lane ^ 8 (row rotate by 8), then lane 7 - lane within 8 (half mirror, opposite
      // bit 2), then full sums over quads
      zd k0 = zsel(b3, sp[2], sp[0]), k1 = zsel(b3, sp[3], sp[1]);
      const zd o0 = zsel(b3, sp[0], sp[2]), o1 = zsel(b3, sp[1], sp[3]);
      k0 = cadd(k0, dpp<DPP_ROR8>(o0));
      k1 = cadd(k1, dpp<DPP_ROR8>(o1));
      zd qv = zsel(b2, k1, k0);
      qv = cadd(qv, dpp<DPP_MIRROR8>(zsel(b2, k0, k1)));
      qv = cadd(qv, dpp<DPP_XOR2>(qv));
      qv = cadd(qv, dpp<DPP_XOR1>(qv));
      zd x = cmul(tau, qv);
      if (myrow <= k || myrow >= r) x = mk(0.0, 0.0);
      const bool writer = (l & 3) == 0;
      zd c = writer ? cmulc(x, vp[trd_p(myrow)]) : mk(0.0, 0.0);   // conj(x) v
      if (writer) xsh[par][trd_p(myrow)] = x;
      c = wave_sum(c);
      if (l == 0) xv[par][w] = c;
    }
    // Waves whose rows are all eliminated write nothing this step: the readers below take x as
    // zero at eliminated rows and columns (v is zero there too) and sum xv over the active waves
    // only.  They also issue no memory access that would make them wait for earlier global
    // stores before the barrier.
    __syncthreads();
    if (wave_on) {
      // (4) rank-2 update of the owned block
      zd xhv = mk(0.0, 0.0);
#pragma unroll
      for (int q = 0; q < TRD_WAVES; ++q)
        if (16 * q + 15 > k) xhv = cadd(xhv, xv[par][q]);
      const zd a2 = cscale(cmul(tau, xhv), -0.5);
      // column by column, so that only the four row values of v and w stay live beside A
      zd vi[4], wi[4];
#pragma unroll
      for (int ii = 0; ii < 4; ++ii) {
        vi[ii] = vp[trd_p(r0 + ii)];
        wi[ii] = cadd(xsh[par][trd_p(r0 + ii)], cmul(a2, vi[ii]));
      }
#pragma unroll
      for (int jj = 0; jj < 8; ++jj)
        if (jj >= jb0) {
          const int cj = 16 * jj + b;
          const zd vj = vp[trd_p(cj)];
          const zd vcc = cconj(vj);
          const zd xj = xsh[par][trd_p(cj)];
          const zd wcc = cconj(cadd(zsel(cj > k, xj, mk(0.0, 0.0)), cmul(a2, vj)));
#pragma unroll
          for (int ii = 0; ii < 4; ++ii) A[ii][jj] = zfms(wi[ii], vcc, zfms(vi[ii], wcc, A[ii][jj]));
        }
    }
  }
  // last diagonal entry
  {
    const int t = r - 1;
    if (a == (t >> 2) && b == (t & 15)) {
#pragma unroll
      for (int ii = 0; ii < 4; ++ii)
#pragma unroll
        for (int jj = 0; jj < 8; ++jj)
          if ((t & 3) == ii && (t >> 4) == jj) {
            dout[t] = A[ii][jj].re;
            eout[t] = 0.0;
          }
    }
  }
}

}  // namespace rt
