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

// The two products of every step stream all of A-hat once each (HBM-bound: about 16 l m F bytes
// in FP64), so they are written for memory-level parallelism: many blocks per face, several
// independent loads in flight per lane, the right-hand vectors staged in LDS.  Results are FP64
// partial vectors that the re-orthogonalization kernel sums in a fixed order.
constexpr int GVN_UNROLL = 8;     // columns loaded back to back per lane
constexpr int GVN_MAXCHUNK = 16;  // column chunks (partial vectors) per face at most
constexpr int GVC_COLS = 4;       // columns per wave in the conjugate product

// part[ch] (face f, slice c, row i at ch*tStride + f*sY + c*l + i) = sum over the chunk's columns
// of A-hat(i, col) x(col, c), p <= PMAX.  Grid (ceil(l/64), chunks, F); block 256 = 4 waves, each
// wave kw columns (multiple of GVN_UNROLL), lane = row; the 4 waves are summed in LDS.
template <typename T, int PMAX>
__global__ void __launch_bounds__(256)
k_gv_n(const cplx<T>* __restrict__ A, int l, int m, int p, const cplx<T>* __restrict__ X, int64_t ldx, int64_t sX,
       int kw, zd* __restrict__ part, int64_t tStride, int64_t sY, const int* __restrict__ live) {
  if (live && *live <= 0) return;   // every slice decided: a step enqueued ahead does nothing
  extern __shared__ __align__(16) unsigned char smem_raw[];
  const int KC = 4 * kw;
  zd* red = reinterpret_cast<zd*>(smem_raw);                                   // 3 x 64 x PMAX
  cplx<T>* xs = reinterpret_cast<cplx<T>*>(smem_raw + 3 * 64 * PMAX * sizeof(zd));  // p x KC
  const int f = blockIdx.z, ch = blockIdx.y;
  const int c0 = ch * KC;
  for (int idx = threadIdx.x; idx < p * KC; idx += blockDim.x) {
    const int c = idx / KC, u = idx - c * KC, col = c0 + u;
    xs[idx] = col < m ? X[(int64_t)f * sX + (int64_t)c * ldx + col] : cplx<T>{(T)0, (T)0};
  }
  __syncthreads();
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int row = blockIdx.x * 64 + lane;
  const int rr = row < l ? row : l - 1;            // clamped row: loads stay inside the face
  const cplx<T>* a = A + (int64_t)f * l * m + rr;
  const int cb = w * kw;
  zd acc[PMAX];
#pragma unroll
  for (int c = 0; c < PMAX; ++c) acc[c] = mk(0.0, 0.0);
  for (int t = 0; t < kw; t += GVN_UNROLL) {
    zd av[GVN_UNROLL];
#pragma unroll
    for (int u = 0; u < GVN_UNROLL; ++u) {
      const int col = c0 + cb + t + u;
      av[u] = col < m ? ld<double>(a[(int64_t)col * l]) : mk(0.0, 0.0);
    }
#pragma unroll
    for (int u = 0; u < GVN_UNROLL; ++u)
#pragma unroll
      for (int c = 0; c < PMAX; ++c)
        if (c < p) {
          const zd x = ld<double>(xs[c * KC + cb + t + u]);
          acc[c].re = fma(av[u].re, x.re, fma(-av[u].im, x.im, acc[c].re));
          acc[c].im = fma(av[u].re, x.im, fma(av[u].im, x.re, acc[c].im));
        }
  }
  if (w > 0) {
#pragma unroll
    for (int c = 0; c < PMAX; ++c) red[((w - 1) * 64 + lane) * PMAX + c] = acc[c];
  }
  __syncthreads();
  if (w != 0 || row >= l) return;
#pragma unroll
  for (int c = 0; c < PMAX; ++c)
    if (c < p) {
      zd v = acc[c];
      for (int q = 0; q < 3; ++q) v = cadd(v, red[(q * 64 + lane) * PMAX + c]);
      part[(int64_t)ch * tStride + (int64_t)f * sY + (int64_t)c * l + row] = v;
    }
}

// part (face f, slice c, entry j at f*sY + c*m + j) = sum_i conj(A-hat(i, j)) x(i, c), p <= PMAX.
// Grid (ceil(m / (4*GVC_COLS)), F); block 256 = 4 waves, each wave GVC_COLS columns, lanes over
// the rows; x staged in LDS (l x p).
template <typename T, int PMAX>
__global__ void __launch_bounds__(256)
k_gv_c(const cplx<T>* __restrict__ A, int l, int m, int p, const cplx<T>* __restrict__ X, int64_t ldx, int64_t sX,
       zd* __restrict__ part, int64_t sY, const int* __restrict__ live) {
  if (live && *live <= 0) return;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  cplx<T>* xs = reinterpret_cast<cplx<T>*>(smem_raw);  // p x l
  const int f = blockIdx.y;
  for (int idx = threadIdx.x; idx < l * p; idx += blockDim.x) {
    const int c = idx / l, i = idx - c * l;
    xs[idx] = X[(int64_t)f * sX + (int64_t)c * ldx + i];
  }
  __syncthreads();
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int j0 = (blockIdx.x * 4 + w) * GVC_COLS;
  if (j0 >= m) return;
  const cplx<T>* Af = A + (int64_t)f * l * m;
  zd acc[GVC_COLS][PMAX];
#pragma unroll
  for (int u = 0; u < GVC_COLS; ++u)
#pragma unroll
    for (int c = 0; c < PMAX; ++c) acc[u][c] = mk(0.0, 0.0);
  for (int i = lane; i < l; i += 64) {
    zd av[GVC_COLS];
#pragma unroll
    for (int u = 0; u < GVC_COLS; ++u) {
      const int col = j0 + u < m ? j0 + u : m - 1;  // clamped column (its sum is not stored)
      av[u] = ld<double>(Af[(int64_t)col * l + i]);
    }
#pragma unroll
    for (int c = 0; c < PMAX; ++c)
      if (c < p) {
        const zd x = ld<double>(xs[c * l + i]);
#pragma unroll
        for (int u = 0; u < GVC_COLS; ++u) {
          acc[u][c].re = fma(av[u].re, x.re, fma(av[u].im, x.im, acc[u][c].re));
          acc[u][c].im = fma(av[u].re, x.im, fma(-av[u].im, x.re, acc[u][c].im));
        }
      }
  }
#pragma unroll
  for (int c = 0; c < PMAX; ++c)
    if (c < p) {
#pragma unroll
      for (int u = 0; u < GVC_COLS; ++u) {
        const zd v = wave_sum(acc[u][c]);
        if (lane == 0 && j0 + u < m) part[(int64_t)f * sY + (int64_t)c * m + j0 + u] = v;
      }
    }
}

__device__ __forceinline__ double gkb_block_sum(double v, double* red) {
  v = wave_sum(v);
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  __syncthreads();
  if (lane == 0) red[w] = v;
  __syncthreads();
  double s = 0.0;
  for (int i = 0; i < (int)(blockDim.x >> 6); ++i) s += red[i];
  return s;
}

// Bookkeeping of step i folded into its q half-step, once z_{i+1} is known.  Givens rotation i of
// the basis (alpha = c_i, beta = z_{i+1}; cprev = cosine of rotation i-1, -1 before the first):
//     rho-bar = -cprev alpha, rho = sqrt(rho-bar^2 + beta^2), c = rho-bar / rho, s = beta / rho,
// recorded for the back substitution (rho, s, alpha) and applied to the right-hand side(s):
// MODE 1 (tGKB_p): the basis' own e_1 z_1, phi_i = c phi-bar, phi-bar <- s phi-bar (real);
// MODE 2 (nested): every slice j of B-hat, g = q_{i+1}^H b-hat_j, phi_i = c phi-bar + s g,
// phi-bar <- s phi-bar - c g (complex).
// MODE 3 (t-Lanczos, Alg. 4): the step's raw vector is A-hat q_i; the kernel forms the diagonal
// entry c_i = Re(q_i^H A-hat q_i), subtracts z_{i-1} q_{i-1} + c_i q_i, re-orthogonalizes and
// normalizes (z_i), and updates the QR factorization of the tridiagonal T-bar_i: column i holds
// z_{i-1}, c_i, z_i in rows i-1, i, i+1; rotations i-2 and i-1 (state l2, l1: cosine, sine;
// (-1, 0) before the first) give
//     eps = s2 z_{i-1}, d = -c2 z_{i-1};  delta = c1 d + s1 c_i, g = s1 d - c1 c_i;
// rotation i then zeroes z_i under g (rho = sqrt(g^2 + z_i^2)), R column i = (eps, delta, rho)
// on rows i-2, i-1, i, and phi_i = c phi-bar, phi-bar <- s phi-bar as in MODE 1.
struct GkbRot {
  const double* alpha;
  double* cprev;
  double* rho_h;
  double* s_h;
  double* alpha_h;
  double* phibar;     // MODE 1 / 3, per basis
  double* phi_h;      // MODE 1 / 3, per basis x kmax
  const void* bh;     // MODE 2: face f, slice j at bh + (f*p_rhs + j)*len (storage type of the basis)
  zd* nphibar;        // MODE 2, per (f, j)
  zd* nphi_h;         // MODE 2, per (f, j) x kmax
  int p_rhs, kmax, i;
  double* l1c;        // MODE 3: rotation i-1, per basis
  double* l1s;
  double* l2c;        // MODE 3: rotation i-2, per basis
  double* l2s;
  double* r1_h;       // MODE 3: R(i-1, i), per basis x kmax
  double* r2_h;       // MODE 3: R(i-2, i), per basis x kmax
};

// One half-step of Alg. 7 for every (face, slice): v = raw - prevcoef * prev, CGS2 against the
// first nb basis vectors, normalize, store as basis vector nb.  Basis of (f, c): Bas + ((f*p + c)
// * ld_basis) with vectors of length len and stride len.  coef_prev / coef_out: (f, c) arrays of
// real scalars (z_i / c_i).  raw = the product, as nparts FP64 partial vectors summed in order
// (partial t of face f, slice c at part + t*tStride + f*sRaw + c*len).  MODE 0: the w half-step;
// MODE 1 / 2: the q half-step with the rotation bookkeeping above.  live (or NULL): number of
// slices still undecided; at 0 the kernel returns at once (a step enqueued ahead of the host's
// knowledge that the process has ended).
template <typename T, int MODE>
__global__ void __launch_bounds__(GKB_THREADS)
k_gkb_orth(const zd* __restrict__ part, int nparts, int64_t tStride, int64_t sRaw, cplx<T>* __restrict__ Bas,
           int64_t ld_basis, int len, int nb, const cplx<T>* __restrict__ prev, int64_t ld_prev, int prev_idx,
           const double* __restrict__ coef_prev, double* __restrict__ coef_out, int p, double tol, GkbRot rot,
           const int* __restrict__ live) {
  if (live && *live <= 0) return;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  __shared__ double rcs[2];
  const int f = blockIdx.y, c = blockIdx.x;
  double* red = reinterpret_cast<double*>(smem_raw);              // 32 doubles
  zd* h = reinterpret_cast<zd*>(smem_raw + 32 * sizeof(double));  // nb coefficients
  zd* vs = h + nb;                                                 // len entries
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
      const zd* src = part + (int64_t)f * sRaw + (int64_t)c * len + i;
      x = src[0];
      for (int q = 1; q < nparts; ++q) x = cadd(x, src[(int64_t)q * tStride]);
    }
    v[t] = x;
  }
  double cdiag = 0.0;
  if (MODE == 3) {   // c_i = Re(q_i^H A-hat q_i), q_i = basis vector nb - 1
    const cplx<T>* qi = bas + (int64_t)(nb - 1) * len;
    double d = 0.0;
#pragma unroll
    for (int t = 0; t < 8; ++t) {
      const int i = threadIdx.x + t * blockDim.x;
      if (t < per && i < len) {
        const zd q = ld<double>(qi[i]);
        d = fma(q.re, v[t].re, fma(q.im, v[t].im, d));
      }
    }
    cdiag = gkb_block_sum(d, red);
#pragma unroll
    for (int t = 0; t < 8; ++t) {
      const int i = threadIdx.x + t * blockDim.x;
      if (t < per && i < len) v[t] = csub(v[t], cscale(ld<double>(qi[i]), cdiag));
    }
  }
#pragma unroll
  for (int t = 0; t < 8; ++t) {
    const int i = threadIdx.x + t * blockDim.x;
    if (pv && t < per && i < len) v[t] = csub(v[t], cscale(ld<double>(pv[i]), cp));
  }
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nw = blockDim.x >> 6;
  double n0 = 0.0;
#pragma unroll
  for (int t = 0; t < 8; ++t) n0 += cabs2(v[t]);
  n0 = sqrt(gkb_block_sum(n0, red));
  for (int pass = 0; pass < 2; ++pass) {
    if (nb == 0) break;
    // h_j = b_j^H v for all j < nb: stage v in LDS, one wave per j
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
        re = fma(b.re, x.re, fma(b.im, x.im, re));
        im = fma(b.re, x.im, fma(-b.im, x.re, im));
      }
      re = wave_sum(re);
      im = wave_sum(im);
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
    if (t < per && i < len) {
      const zd q = cscale(v[t], inv);
      st(out[i], q);
      if (MODE == 2) vs[i] = ld<double>(ld<T>(q));   // the stored (rounded) q_{i+1}
    }
  }
  const int64_t bi = (int64_t)f * p + c;
  if (threadIdx.x == 0) coef_out[bi] = ok ? nn : 0.0;
  if (MODE == 0) return;
  if (MODE == 3) {
    if (threadIdx.x == 0) {
      const double zp = cp, zn = ok ? nn : 0.0;
      const double c1 = rot.l1c[bi], s1 = rot.l1s[bi], c2 = rot.l2c[bi], s2 = rot.l2s[bi];
      const double eps = s2 * zp, d = -c2 * zp;
      const double delta = fma(c1, d, s1 * cdiag), g = fma(s1, d, -c1 * cdiag);
      const double rho = sqrt(fma(g, g, zn * zn));
      double cs, sn;
      if (rho > 0.0) { cs = g / rho; sn = zn / rho; } else { cs = 0.0; sn = 1.0; }
      const int64_t hi = bi * rot.kmax + rot.i - 1;
      rot.rho_h[hi] = rho;
      rot.r1_h[hi] = delta;
      rot.r2_h[hi] = eps;
      const double pb = rot.phibar[bi];
      rot.phi_h[hi] = cs * pb;
      rot.phibar[bi] = sn * pb;
      rot.l2c[bi] = c1;
      rot.l2s[bi] = s1;
      rot.l1c[bi] = cs;
      rot.l1s[bi] = sn;
    }
    return;
  }
  if (threadIdx.x == 0) {
    const double a = rot.alpha[bi], b = ok ? nn : 0.0;
    const double rbar = -rot.cprev[bi] * a;
    const double rho = sqrt(rbar * rbar + b * b);
    double cs, sn;
    if (rho > 0.0) { cs = rbar / rho; sn = b / rho; } else { cs = 0.0; sn = 1.0; }
    const int64_t hi = bi * rot.kmax + rot.i - 1;
    rot.rho_h[hi] = rho;
    rot.s_h[hi] = sn;
    rot.alpha_h[hi] = a;
    rot.cprev[bi] = cs;
    if (MODE == 1) {
      const double pb = rot.phibar[bi];
      rot.phi_h[hi] = cs * pb;
      rot.phibar[bi] = sn * pb;
    }
    rcs[0] = cs;
    rcs[1] = sn;
  }
  if (MODE != 2) return;
  __syncthreads();
  const double cs = rcs[0], sn = rcs[1];
  for (int j = wave; j < rot.p_rhs; j += nw) {
    const cplx<T>* bj = reinterpret_cast<const cplx<T>*>(rot.bh) + ((int64_t)f * rot.p_rhs + j) * len;
    double re = 0.0, im = 0.0;
    for (int i = lane; i < len; i += 64) {
      const zd q = vs[i], x = ld<double>(bj[i]);
      re = fma(q.re, x.re, fma(q.im, x.im, re));
      im = fma(q.re, x.im, fma(-q.im, x.re, im));
    }
    re = wave_sum(re);
    im = wave_sum(im);
    if (lane == 0) {
      const int64_t idx = (int64_t)f * rot.p_rhs + j;
      const zd pb = rot.nphibar[idx];
      rot.nphi_h[idx * rot.kmax + rot.i - 1] = mk(fma(cs, pb.re, sn * re), fma(cs, pb.im, sn * im));
      rot.nphibar[idx] = mk(fma(sn, pb.re, -cs * re), fma(sn, pb.im, -cs * im));
    }
  }
}

// Progress of the step loop for the host: after step i the discrepancy kernel stores one 64-bit
// word (call id << 48 | i << 32 | slices still undecided) into coherent pinned host memory at
// system scope, so that the host can keep a bounded number of steps in flight without
// synchronizing the stream.  i < 2^16 (k_max <= m <= 8192).
__device__ __forceinline__ void report_progress(uint64_t* prog, uint32_t pid, int i, int undecided) {
  if (!prog) return;
  const uint64_t word = ((uint64_t)(pid & 0xffffu) << 48) | ((uint64_t)(i & 0xffff) << 32) | (uint32_t)undecided;
  __hip_atomic_store(prog, word, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_SYSTEM);
}

// discrepancy check after step i (one block): one wave per slice c, lanes over the faces (a fixed
// order); remaining counts the undecided slices
__global__ void __launch_bounds__(1024)
k_gkb_dp(const double* __restrict__ phibar, int F, int p, int n, const double* __restrict__ bound, int i, int kmax,
         int* __restrict__ kout, double* __restrict__ resid, int* __restrict__ remaining, uint64_t* __restrict__ prog,
         uint32_t pid) {
  if (*remaining <= 0) return;
  __shared__ int decided;
  if (threadIdx.x == 0) decided = 0;
  __syncthreads();
  const int lane = threadIdx.x & 63, nw = blockDim.x >> 6;
  for (int c = threadIdx.x >> 6; c < p; c += nw) {
    double tot = 0.0;
    for (int f = lane; f < F; f += 64) {
      const double w = (f == 0 || 2 * f == n) ? 1.0 : 2.0;
      const double v = phibar[(int64_t)f * p + c];
      tot = fma(w * v, v, tot);
    }
    tot = wave_sum(tot);
    if (lane == 0) {
      const double r = sqrt(tot / (double)n);
      if (resid) resid[(int64_t)c * kmax + i - 1] = r;
      if (kout[c] == 0 && r <= bound[c]) {
        kout[c] = i;
        atomicAdd(&decided, 1);
      }
    }
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    const int rem = *remaining - decided;
    *remaining = rem;
    report_progress(prog, pid, i, rem);
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

// t-Lanczos solution per (f, c): k = k_c (k_max if unmet), y = R^{-1} phi with R upper triangular
// of bandwidth 3 (diagonal rho_t, R(t, t+1) = r1_{t+1}, R(t, t+2) = r2_{t+2}), X-hat = Q_k y.
// One block per (c, f).
template <typename T>
__global__ void __launch_bounds__(256)
k_tlan_solution(const cplx<T>* __restrict__ Qb, int64_t ld_basis, int m, const int* __restrict__ kout, int kmax, int p,
                const double* __restrict__ rho_h, const double* __restrict__ r1_h, const double* __restrict__ r2_h,
                const double* __restrict__ phi_h, cplx<T>* __restrict__ Xh) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  double* y = reinterpret_cast<double*>(smem_raw);
  const int c = blockIdx.x, f = blockIdx.y;
  const int idx = f * p + c;
  int k = kout[c];
  if (k <= 0) k = kmax;
  if (threadIdx.x == 0) {
    const double* rh = rho_h + (int64_t)idx * kmax;
    const double* a1 = r1_h + (int64_t)idx * kmax;
    const double* a2 = r2_h + (int64_t)idx * kmax;
    const double* ph = phi_h + (int64_t)idx * kmax;
    double y1 = 0.0, y2 = 0.0;   // y_{t+1}, y_{t+2}
    for (int t = k - 1; t >= 0; --t) {
      double num = ph[t];
      if (t + 1 < k) num = fma(-a1[t + 1], y1, num);
      if (t + 2 < k) num = fma(-a2[t + 2], y2, num);
      const double yt = rh[t] > 0.0 ? num / rh[t] : 0.0;
      y[t] = yt;
      y2 = y1;
      y1 = yt;
    }
  }
  __syncthreads();
  const cplx<T>* Q = Qb + (int64_t)idx * ld_basis;
  for (int i = threadIdx.x; i < m; i += blockDim.x) {
    zd acc = mk(0.0, 0.0);
    for (int j = 0; j < k; ++j) acc = cadd(acc, cscale(ld<double>(Q[(int64_t)j * m + i]), y[j]));
    Xh[(int64_t)f * m * p + (int64_t)c * m + i] = mk((T)acc.re, (T)acc.im);
  }
}

// initial normalization: q_1 = b-hat / ||b-hat||, z_1 = ||b-hat|| per (f, c); phibar = z_1
// (face stride of B-hat: sB)
template <typename T>
__global__ void __launch_bounds__(256)
k_gkb_init(const cplx<T>* __restrict__ Bh, int64_t sB, int l, int p, cplx<T>* __restrict__ Qb, int64_t ld_basis,
           double* __restrict__ z1, double* __restrict__ phibar, double* __restrict__ cprev, double tol) {
  __shared__ double red[32];
  const int c = blockIdx.x, f = blockIdx.y;
  const cplx<T>* b = Bh + (int64_t)f * sB + (int64_t)c * l;
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

// ---------------------------------------------------------------------------------------------
// Tikhonov on the t-Krylov space (tGKT_p on Alg. 7's space, t-LanczosTik_p on Alg. 4's)
// ---------------------------------------------------------------------------------------------
// After the step loop every (face, slice) holds the Givens QR of its projected matrix,
// Qbar^T [P-bar_k | z_1 e_1] = [R f; 0 phi-bar_{k+1}], R upper triangular with at most two
// superdiagonals (tGKB: diagonal rho_j, R(j, j+1) = s_j alpha_{j+1}; t-Lanczos: rho_j, r1_{j+1},
// r2_{j+2}).  For any y, ||P-bar_k y - z_1 e_1||^2 = ||R y - f||^2 + phi-bar_{k+1}^2 with
// phi-bar_{k+1}^2 = z_1^2 - ||f||^2, so the Tikhonov solution for lam = 1/mu solves the banded
// normal equations (R^T R + lam I) y = R^T f (Cholesky with bandwidth 2, real arithmetic).
// k_tik_mu: one workgroup per slice c; its threads take the faces in turn and keep the Cholesky
// bands and the solution in LDS (4 k_max doubles per thread).  mu by bisection in log mu on
// [mu_lo, mu_hi] for (1/n) sum_f w_f (||R_f y_f - f_f||^2 + phi-bar_f^2) = bound_c^2: the bracket
// keeps res(lo) > bound >= res(hi) and mu = hi after the last halving; mu_hi that leaves the
// residual above the bound gives mu = mu_hi and a failure flag, mu_lo that meets it gives mu_lo.
// Outputs: mu[c], the final residual, y per (face, slice) for k_basis_solution.
constexpr int TIK_MAX_THREADS = 64;
constexpr int TIK_STEPS = 50;

// R(j, j), R(j, j+1), R(j, j+2) of the face's history arrays (a, b, c: see above)
template <bool LANCZOS>
__device__ __forceinline__ void tik_band(const double* __restrict__ ha, const double* __restrict__ hb,
                                         const double* __restrict__ hc, int j, int k, double& d0, double& d1,
                                         double& d2) {
  d0 = ha[j];
  if (LANCZOS) {
    d1 = (j + 1 < k) ? hb[j + 1] : 0.0;
    d2 = (j + 2 < k) ? hc[j + 2] : 0.0;
  } else {
    d1 = (j + 1 < k) ? hb[j] * hc[j + 1] : 0.0;   // s_j alpha_{j+1}
    d2 = 0.0;
  }
}

// ||R y - f||^2 (+ nothing else) of one face at lam, y left in ys; f_i = fv[i fs].  M = R^T R + lam I:
//   M(i, i)   = d0_i^2 + d1_{i-1}^2 + d2_{i-2}^2 + lam
//   M(i+1, i) = d1_i d0_i + d2_{i-1} d1_{i-1},   M(i+2, i) = d2_i d0_i
// L L^T = M with L(i, i) = g_i, L(i+1, i) = u_i, L(i+2, i) = v_i:
//   v_i = M(i+2, i) / g_i,  u_i = (M(i+1, i) - u_{i-1} v_{i-1}) / g_i,
//   g_i = sqrt(M(i, i) - u_{i-1}^2 - v_{i-2}^2); forward then backward substitution of R^T f.
template <bool LANCZOS>
__device__ double tik_face(const double* __restrict__ ha, const double* __restrict__ hb, const double* __restrict__ hc,
                           const double* __restrict__ fv, int fs, int k, double lam, double* __restrict__ g,
                           double* __restrict__ u, double* __restrict__ v, double* __restrict__ ys) {
  double d1m1 = 0.0, d2m1 = 0.0, d2m2 = 0.0;   // d1_{i-1}, d2_{i-1}, d2_{i-2}
  double fm1 = 0.0, fm2 = 0.0;                 // f_{i-1}, f_{i-2}
  for (int i = 0; i < k; ++i) {
    double d0, d1, d2;
    tik_band<LANCZOS>(ha, hb, hc, i, k, d0, d1, d2);
    const double fi = fv[(int64_t)i * fs];
    const double um1 = i >= 1 ? u[i - 1] : 0.0, vm2 = i >= 2 ? v[i - 2] : 0.0, vm1 = i >= 1 ? v[i - 1] : 0.0;
    const double mii = fma(d0, d0, fma(d1m1, d1m1, fma(d2m2, d2m2, lam)));
    const double gi = sqrt(fmax(mii - um1 * um1 - vm2 * vm2, 0.0));
    const double ig = gi > 0.0 ? 1.0 / gi : 0.0;
    g[i] = gi;
    u[i] = (fma(d1, d0, d2m1 * d1m1) - um1 * vm1) * ig;   // L(i+1, i); u_{i-1} v_{i-1} = L(i+1,i-1) L(i,i-1)
    v[i] = d2 * d0 * ig;                                  // L(i+2, i)
    // forward: z_i = ((R^T f)_i - u_{i-1} z_{i-1} - v_{i-2} z_{i-2}) / g_i
    const double rt = fma(d0, fi, fma(d1m1, fm1, d2m2 * fm2));
    double z = rt;
    if (i >= 1) z = fma(-um1, ys[i - 1], z);
    if (i >= 2) z = fma(-vm2, ys[i - 2], z);
    ys[i] = z * ig;
    d2m2 = d2m1;
    d1m1 = d1;
    d2m1 = d2;
    fm2 = fm1;
    fm1 = fi;
  }
  // backward: y_i = (z_i - u_i y_{i+1} - v_i y_{i+2}) / g_i
  double y1 = 0.0, y2 = 0.0;
  for (int i = k - 1; i >= 0; --i) {
    const double ig = g[i] > 0.0 ? 1.0 / g[i] : 0.0;
    const double yi = (ys[i] - u[i] * y1 - v[i] * y2) * ig;
    ys[i] = yi;
    y2 = y1;
    y1 = yi;
  }
  // ||R y - f||^2
  double rr = 0.0;
  for (int i = 0; i < k; ++i) {
    double d0, d1, d2;
    tik_band<LANCZOS>(ha, hb, hc, i, k, d0, d1, d2);
    double e = d0 * ys[i] - fv[(int64_t)i * fs];
    if (i + 1 < k) e = fma(d1, ys[i + 1], e);
    if (i + 2 < k) e = fma(d2, ys[i + 2], e);
    rr = fma(e, e, rr);
  }
  return rr;
}

// ha, hb, hc: the histories (tGKB: rho, s, alpha; t-Lanczos: rho, r1, r2), phi: f, beta: z_1 per
// (face, slice) (index f * p + c, histories with stride kmax).  kin[c] <= 0: k = kmax.
template <bool LANCZOS>
__global__ void __launch_bounds__(TIK_MAX_THREADS)
k_tik_mu(const double* __restrict__ ha, const double* __restrict__ hb, const double* __restrict__ hc,
         const double* __restrict__ phi, const double* __restrict__ beta, const int* __restrict__ kin, int kmax, int p,
         int F, int n, const double* __restrict__ bound, double mu_lo, double mu_hi, double* __restrict__ mu_out,
         double* __restrict__ res_out, double* __restrict__ y_out, int* __restrict__ fail) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  __shared__ double red[TIK_MAX_THREADS];
  __shared__ double sh_res;
  const int c = blockIdx.x, tid = threadIdx.x, nt = (int)blockDim.x;
  double* base = reinterpret_cast<double*>(smem_raw) + (size_t)tid * 4 * kmax;
  double *g = base, *u = base + kmax, *v = base + 2 * kmax, *ys = base + 3 * kmax;
  const int k = kin[c] > 0 ? kin[c] : kmax;
  const double b2 = bound[c] * bound[c];
  // residual^2 of the Tikhonov solution at lam (all faces), written to y_out when `keep`
  auto residual2 = [&](double lam, bool keep) -> double {
    double acc = 0.0;
    for (int f = tid; f < F; f += nt) {
      const int64_t idx = (int64_t)f * p + c;
      const double* fa = ha + idx * kmax;
      const double* fb = hb + idx * kmax;
      const double* fc = hc + idx * kmax;
      const double* fv = phi + idx * kmax;
      double ff = 0.0;
      for (int i = 0; i < k; ++i) ff = fma(fv[i], fv[i], ff);
      const double bt = beta[idx];
      const double pb2 = fmax(bt * bt - ff, 0.0);          // phi-bar_{k+1}^2
      const double rr = tik_face<LANCZOS>(fa, fb, fc, fv, 1, k, lam, g, u, v, ys);
      const double w = (f == 0 || 2 * f == n) ? 1.0 : 2.0;
      acc = fma(w, rr + pb2, acc);
      if (keep)
        for (int i = 0; i < kmax; ++i) y_out[idx * kmax + i] = i < k ? ys[i] : 0.0;
    }
    red[tid] = acc;
    __syncthreads();
    if (tid == 0) {
      double t = 0.0;
      for (int i = 0; i < nt; ++i) t += red[i];
      sh_res = t / (double)n;
    }
    __syncthreads();
    return sh_res;
  };
  double mu;
  int failed = 0;
  if (residual2(1.0 / mu_hi, false) > b2) {
    mu = mu_hi;
    failed = 1;
  } else if (residual2(1.0 / mu_lo, false) <= b2) {
    mu = mu_lo;
  } else {
    double lo = log(mu_lo), hi = log(mu_hi);
    for (int it = 0; it < TIK_STEPS; ++it) {
      const double mid = 0.5 * (lo + hi);
      if (residual2(exp(-mid), false) > b2) lo = mid;
      else hi = mid;
    }
    mu = exp(hi);
  }
  const double r2 = residual2(1.0 / mu, true);
  if (tid == 0) {
    mu_out[c] = mu;
    if (res_out) res_out[c] = sqrt(r2);
    if (failed) atomicOr(fail, 1);
  }
}

// X-hat(:, c) of face f = basis_k y (basis vectors of length len, stride len, per (f, c) at
// basis + (f p + c) ld_basis); one workgroup per (c, f)
template <typename T>
__global__ void __launch_bounds__(256)
k_basis_solution(const cplx<T>* __restrict__ basis, int64_t ld_basis, int len, const int* __restrict__ kin, int kmax,
                 int p, const double* __restrict__ y_in, cplx<T>* __restrict__ Xh) {
  const int c = blockIdx.x, f = blockIdx.y;
  const int64_t idx = (int64_t)f * p + c;
  const int k = kin[c] > 0 ? kin[c] : kmax;
  const cplx<T>* B = basis + idx * ld_basis;
  const double* y = y_in + idx * kmax;
  for (int i = threadIdx.x; i < len; i += blockDim.x) {
    zd acc = mk(0.0, 0.0);
    for (int j = 0; j < k; ++j) acc = cadd(acc, cscale(ld<double>(B[(int64_t)j * len + i]), y[j]));
    Xh[(int64_t)f * len * p + (int64_t)c * len + i] = mk((T)acc.re, (T)acc.im);
  }
}

// k_out, status of a Tikhonov solve: not met when the truncated index reached k_max or mu_hi
// could not bring the residual down to the bound
__global__ void k_tik_finish(const int* __restrict__ kin, int p, int kmax, const int* __restrict__ fail,
                             int* __restrict__ kout, int* __restrict__ status) {
  __shared__ int fail_any;
  if (threadIdx.x == 0) fail_any = *fail;
  __syncthreads();
  for (int c = threadIdx.x; c < p; c += blockDim.x) {
    const int k = kin[c];
    if (k <= 0) atomicOr(&fail_any, 1);
    kout[c] = k > 0 ? k : kmax;
  }
  __syncthreads();
  if (threadIdx.x == 0 && status) *status = fail_any ? RTSVD_W_DP_NOT_MET : RTSVD_OK;
}

// ---------------------------------------------------------------------------------------------
// nested_tGKB_p (Alg. 8): one basis, started from B_1, shared by every lateral slice
// ---------------------------------------------------------------------------------------------
// The bidiagonal P-bar_k and its Givens rotations belong to the basis alone (one set per face);
// slice j only brings its own right-hand side g = Q_{k+1}^H b-hat_j.  With the rotation
// [c s; s -c] of step i acting on rows i, i+1 of [phi-bar_i; g_{i+1}]:
//     phi_i = c phi-bar_i + s g_{i+1},   phi-bar_{i+1} = s phi-bar_i - c g_{i+1},
// phi-bar_1 = g_1, and |phi-bar_{k+1}| is the face residual of min ||P-bar_k y - g||, so every
// slice advances in lockstep with the basis (complex right-hand sides, real rotations).

constexpr int NEST_WAVES = 4;

// phi-bar_1 = q_1^H b-hat_j for every (face f, slice j); one wave each
template <typename T>
__global__ void __launch_bounds__(64 * NEST_WAVES)
k_nest_init(const cplx<T>* __restrict__ Qb, int64_t ld_basis, const cplx<T>* __restrict__ Bh, int l, int p,
            zd* __restrict__ phibar) {
  const int lane = threadIdx.x & 63;
  const int j = blockIdx.x * NEST_WAVES + (threadIdx.x >> 6), f = blockIdx.y;
  if (j >= p) return;
  const cplx<T>* q = Qb + (int64_t)f * ld_basis;
  const cplx<T>* b = Bh + ((int64_t)f * p + j) * l;
  double re = 0.0, im = 0.0;
  for (int t = lane; t < l; t += 64) {
    const zd a = ld<double>(q[t]), x = ld<double>(b[t]);
    re = fma(a.re, x.re, fma(a.im, x.im, re));
    im = fma(a.re, x.im, fma(-a.im, x.re, im));
  }
  re = wave_sum(re);
  im = wave_sum(im);
  if (lane == 0) phibar[(int64_t)f * p + j] = mk(re, im);
}

// chain state: st[0] = slice being decided, st[1] = its smallest admissible k, st[2] = 1 once a
// slice took k_max without meeting the principle
__global__ void k_nest_reset(int* __restrict__ st, int k_init, int* __restrict__ remaining, int p) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    st[0] = 0;
    st[1] = k_init;
    st[2] = 0;
    *remaining = p;
  }
}

// After step i: residual of every slice (faces summed in a fixed order with the half-spectrum
// weights, one wave per slice), res[j*kmax + i-1]; then the slices are decided in order: slice j takes the first
// k >= k_{j-1} (k_init for j = 1), k <= i, whose residual is below eta*delta_j; at i = k_max an
// undecided slice takes k_max and the failure is recorded.  One block; nothing once every slice
// is decided.
__global__ void __launch_bounds__(256)
k_nest_dp(const zd* __restrict__ phibar, int F, int p, int n, const double* __restrict__ bound, int i, int kmax,
          double* __restrict__ res, int* __restrict__ kout, int* __restrict__ st, int* __restrict__ remaining,
          uint64_t* __restrict__ prog, uint32_t pid) {
  if (*remaining <= 0) return;
  const int lane = threadIdx.x & 63, nw = blockDim.x >> 6;
  for (int j = threadIdx.x >> 6; j < p; j += nw) {   // one wave per slice, lanes over the faces
    double tot = 0.0;
    for (int f = lane; f < F; f += 64) {
      const double w = (f == 0 || 2 * f == n) ? 1.0 : 2.0;
      tot = fma(w, cabs2(phibar[(int64_t)f * p + j]), tot);
    }
    tot = wave_sum(tot);
    if (lane == 0) res[(int64_t)j * kmax + i - 1] = sqrt(tot / (double)n);
  }
  __syncthreads();
  if (threadIdx.x != 0) return;
  int j = st[0], k = st[1], failed = st[2];
  while (j < p) {
    while (k <= i && !(res[(int64_t)j * kmax + k - 1] < bound[j])) ++k;
    if (k <= i) {
      kout[j++] = k;
    } else if (i == kmax) {
      k = kmax;
      kout[j++] = kmax;
      failed = 1;
    } else {
      break;
    }
  }
  st[0] = j;
  st[1] = k;
  st[2] = failed;
  *remaining = p - j;
  report_progress(prog, pid, i, p - j);
}

// X-hat(:, j) on face f = W_k y, y from R y = phi (R upper bidiagonal: diagonal rho_t, super-
// diagonal s_t alpha_{t+1}; complex phi of slice j), k = k_j.  One block per (j, f).
template <typename T>
__global__ void __launch_bounds__(256)
k_nest_solution(const cplx<T>* __restrict__ Wb, int64_t ld_basis, int m, const int* __restrict__ kin, int kmax, int p,
                const double* __restrict__ rho_h, const double* __restrict__ s_h, const double* __restrict__ alpha_h,
                const zd* __restrict__ phi_h, cplx<T>* __restrict__ Xh) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  zd* y = reinterpret_cast<zd*>(smem_raw);
  const int j = blockIdx.x, f = blockIdx.y;
  const int k = kin[j];
  if (threadIdx.x == 0) {
    const double* rh = rho_h + (int64_t)f * kmax;
    const double* sh = s_h + (int64_t)f * kmax;
    const double* ah = alpha_h + (int64_t)f * kmax;
    const zd* ph = phi_h + ((int64_t)f * p + j) * kmax;
    zd ynext = mk(0.0, 0.0);
    for (int t = k - 1; t >= 0; --t) {
      const double theta = (t + 1 < k) ? sh[t] * ah[t + 1] : 0.0;
      zd yt = mk(0.0, 0.0);
      if (rh[t] > 0.0) {
        const double inv = 1.0 / rh[t];
        yt = mk((ph[t].re - theta * ynext.re) * inv, (ph[t].im - theta * ynext.im) * inv);
      }
      y[t] = yt;
      ynext = yt;
    }
  }
  __syncthreads();
  const cplx<T>* W = Wb + (int64_t)f * ld_basis;
  for (int r = threadIdx.x; r < m; r += blockDim.x) {
    zd acc = mk(0.0, 0.0);
    for (int t = 0; t < k; ++t) acc = cadd(acc, cmul(ld<double>(W[(int64_t)t * m + r]), y[t]));
    Xh[(int64_t)f * m * p + (int64_t)j * m + r] = mk((T)acc.re, (T)acc.im);
  }
}

// nested_tGKT_p: Tikhonov on the nested space.  Slice j keeps, per face, the basis' Givens QR
// (R: diagonal rho_t, superdiagonal s_t alpha_{t+1}, real) and its own rotated right-hand side
// (phi_1 .. phi_k complex, phi-bar_{k+1}); for y = y_re + i y_im,
//     ||P-bar_k y - g_j||^2 = ||R y_re - Re phi||^2 + ||R y_im - Im phi||^2 + |phi-bar_{k+1}|^2,
// so the Tikhonov solution is two real banded solves with one matrix (tik_face on the real and
// the imaginary parts), and the weighted face sum of |phi-bar_{k+1}|^2 over n is the square of the
// projected residual k_nest_dp recorded at k_j.  mu by the bisection of k_tik_mu for
// (1/n) sum_f w_f (||R y - phi||^2) + res_j(k_j)^2 = bound_j^2.  One workgroup per slice, threads
// over the faces (5 k_max doubles of LDS per thread).  y_out: complex, per (face, slice).
__global__ void __launch_bounds__(TIK_MAX_THREADS)
k_nest_tik_mu(const double* __restrict__ rho_h, const double* __restrict__ s_h, const double* __restrict__ alpha_h,
              const zd* __restrict__ phi_h, const double* __restrict__ res, const int* __restrict__ kin, int kmax,
              int p, int F, int n, const double* __restrict__ bound, double mu_lo, double mu_hi,
              double* __restrict__ mu_out, double* __restrict__ res_out, zd* __restrict__ y_out,
              int* __restrict__ fail) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  __shared__ double red[TIK_MAX_THREADS];
  __shared__ double sh_res;
  const int c = blockIdx.x, tid = threadIdx.x, nt = (int)blockDim.x;
  double* base = reinterpret_cast<double*>(smem_raw) + (size_t)tid * 5 * kmax;
  double *g = base, *u = base + kmax, *v = base + 2 * kmax, *yr = base + 3 * kmax, *yi = base + 4 * kmax;
  const int k = kin[c] > 0 ? kin[c] : kmax;
  const double b2 = bound[c] * bound[c];
  const double floor2 = res[(int64_t)c * kmax + k - 1] * res[(int64_t)c * kmax + k - 1];
  auto residual2 = [&](double lam, bool keep) -> double {
    double acc = 0.0;
    for (int f = tid; f < F; f += nt) {
      const double* fa = rho_h + (int64_t)f * kmax;
      const double* fb = s_h + (int64_t)f * kmax;
      const double* fc = alpha_h + (int64_t)f * kmax;
      const double* fv = reinterpret_cast<const double*>(phi_h + ((int64_t)f * p + c) * kmax);
      const double rr = tik_face<false>(fa, fb, fc, fv, 2, k, lam, g, u, v, yr) +
                        tik_face<false>(fa, fb, fc, fv + 1, 2, k, lam, g, u, v, yi);
      const double w = (f == 0 || 2 * f == n) ? 1.0 : 2.0;
      acc = fma(w, rr, acc);
      if (keep) {
        zd* yo = y_out + ((int64_t)f * p + c) * kmax;
        for (int i = 0; i < kmax; ++i) yo[i] = i < k ? mk(yr[i], yi[i]) : mk(0.0, 0.0);
      }
    }
    red[tid] = acc;
    __syncthreads();
    if (tid == 0) {
      double t = 0.0;
      for (int i = 0; i < nt; ++i) t += red[i];
      sh_res = t / (double)n + floor2;
    }
    __syncthreads();
    return sh_res;
  };
  double mu;
  int failed = 0;
  if (residual2(1.0 / mu_hi, false) > b2) {
    mu = mu_hi;
    failed = 1;
  } else if (residual2(1.0 / mu_lo, false) <= b2) {
    mu = mu_lo;
  } else {
    double lo = log(mu_lo), hi = log(mu_hi);
    for (int it = 0; it < TIK_STEPS; ++it) {
      const double mid = 0.5 * (lo + hi);
      if (residual2(exp(-mid), false) > b2) lo = mid;
      else hi = mid;
    }
    mu = exp(hi);
  }
  const double r2 = residual2(1.0 / mu, true);
  if (tid == 0) {
    mu_out[c] = mu;
    if (res_out) res_out[c] = sqrt(r2);
    if (failed) atomicOr(fail, 1);
  }
}

// X-hat(:, j) on face f = W_k y (the nested basis, complex y of k_nest_tik_mu); one block per (j, f)
template <typename T>
__global__ void __launch_bounds__(256)
k_nest_tik_solution(const cplx<T>* __restrict__ Wb, int64_t ld_basis, int m, const int* __restrict__ kin, int kmax,
                    int p, const zd* __restrict__ y_in, cplx<T>* __restrict__ Xh) {
  const int j = blockIdx.x, f = blockIdx.y;
  const int k = kin[j] > 0 ? kin[j] : kmax;
  const cplx<T>* W = Wb + (int64_t)f * ld_basis;
  const zd* y = y_in + ((int64_t)f * p + j) * kmax;
  for (int r = threadIdx.x; r < m; r += blockDim.x) {
    zd acc = mk(0.0, 0.0);
    for (int t = 0; t < k; ++t) acc = cadd(acc, cmul(ld<double>(W[(int64_t)t * m + r]), y[t]));
    Xh[(int64_t)f * m * p + (int64_t)j * m + r] = mk((T)acc.re, (T)acc.im);
  }
}

// k_out and status of nested_tGKT_p: not met when a slice reached k_max unmet or mu_hi could not
// bring a residual down to its bound
__global__ void k_nest_tik_finish(const int* __restrict__ kin, const int* __restrict__ st, const int* __restrict__ fail,
                                  int p, int* __restrict__ kout, int* __restrict__ status) {
  for (int j = threadIdx.x; j < p; j += blockDim.x) kout[j] = kin[j];
  if (threadIdx.x == 0 && status) *status = (st[2] || *fail) ? RTSVD_W_DP_NOT_MET : RTSVD_OK;
}

__global__ void k_nest_finish(const int* __restrict__ kin, const int* __restrict__ st, int p, int* __restrict__ kout,
                              int* __restrict__ status) {
  for (int j = threadIdx.x; j < p; j += blockDim.x) kout[j] = kin[j];
  if (threadIdx.x == 0 && status) *status = st[2] ? RTSVD_W_DP_NOT_MET : RTSVD_OK;
}

}  // namespace rt
