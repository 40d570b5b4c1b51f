// FP64 Gram matrices G_f = Y_f^H Y_f of the tall panels Y_f (rows x r, column-major, leading
// dimension ldy), lower triangle only (the Cholesky factorization and the eigensolver read
// nothing else).  FP64 16x16x4 MFMA tiles (Section 2's facewise products in double precision).
//
// One workgroup per lower 16 x 16 tile (I, J), J <= I: its 4 waves split the rows into quarters,
// each accumulating the tile over its quarter, and the quarters are summed through LDS in a fixed
// order (deterministic, no atomics, no second kernel).  Operands come straight from L2: for one
// step of 16 rows, lane (i, q) (i = lane % 16, q = lane / 16) holds rows 4q .. 4q+3 of columns
// 16 I + i and 16 J + i.  The 4 MFMA k-steps use the row permutation k = 4 q + s on both sides,
// which leaves the sum unchanged and makes every lane's reads 4 consecutive elements.
// Complex: Re G += Ar Br + Ai Bi, Im G += Ar Bi - Ai Br with A = Y(:, I-tile), B = Y(:, J-tile).
#pragma once
#include "common.hpp"

namespace rt {

constexpr int GRAM_THREADS = 256;
typedef double gr_f64x4 __attribute__((ext_vector_type(4)));

template <typename TY>
__global__ void __launch_bounds__(GRAM_THREADS)
k_gram_lower(const TY* __restrict__ Y, int rows, int r, int64_t ldy, int64_t sY, zd* __restrict__ G) {
  __shared__ gr_f64x4 red[3][2][64];
  const int f = blockIdx.y;
  const int p = blockIdx.x;
  // lower tile (I, J) from its index p = I (I + 1) / 2 + J
  int I = (int)((sqrt(8.0 * (double)p + 1.0) - 1.0) * 0.5);
  while ((I + 1) * (I + 2) / 2 <= p) ++I;
  while (I * (I + 1) / 2 > p) --I;
  const int J = p - I * (I + 1) / 2;
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int i = lane & 15, q = lane >> 4;
  const int ca = 16 * I + i, cb = 16 * J + i;
  const bool oka = ca < r, okb = cb < r;
  const TY* __restrict__ ya = Y + (int64_t)f * sY + (int64_t)(oka ? ca : 0) * ldy;
  const TY* __restrict__ yb = Y + (int64_t)f * sY + (int64_t)(okb ? cb : 0) * ldy;
  const int quarter = (rows + 63) / 64 * 16;      // rows per wave, a multiple of 16
  const int k0 = w * quarter, k1 = min(rows, k0 + quarter);
  gr_f64x4 accr = {0.0, 0.0, 0.0, 0.0}, acci = {0.0, 0.0, 0.0, 0.0};
  for (int kb = k0; kb < k1; kb += 16) {
    // unconditional loads at clamped rows (in bounds), masked afterwards: no branches or waits
    // between the loads
    TY ra[4], rb[4];
#pragma unroll
    for (int s = 0; s < 4; ++s) {
      const int kc = min(kb + 4 * q + s, rows - 1);
      ra[s] = ya[kc];
      rb[s] = yb[kc];
    }
    zd a[4], bv[4];
#pragma unroll
    for (int s = 0; s < 4; ++s) {
      const bool in = kb + 4 * q + s < k1;
      const zd va = ld<double>(ra[s]), vb = ld<double>(rb[s]);
      a[s] = mk((oka && in) ? va.re : 0.0, (oka && in) ? va.im : 0.0);
      bv[s] = mk((okb && in) ? vb.re : 0.0, (okb && in) ? vb.im : 0.0);
    }
#pragma unroll
    for (int s = 0; s < 4; ++s) {
      accr = __builtin_amdgcn_mfma_f64_16x16x4f64(a[s].re, bv[s].re, accr, 0, 0, 0);
      accr = __builtin_amdgcn_mfma_f64_16x16x4f64(a[s].im, bv[s].im, accr, 0, 0, 0);
      acci = __builtin_amdgcn_mfma_f64_16x16x4f64(a[s].re, bv[s].im, acci, 0, 0, 0);
      acci = __builtin_amdgcn_mfma_f64_16x16x4f64(-a[s].im, bv[s].re, acci, 0, 0, 0);
    }
  }
  if (w > 0) {
    red[w - 1][0][lane] = accr;
    red[w - 1][1][lane] = acci;
  }
  __syncthreads();
  if (w == 0) {
#pragma unroll
    for (int u = 0; u < 3; ++u) {
      accr += red[u][0][lane];
      acci += red[u][1][lane];
    }
    // output layout of the 16x16x4 FP64 MFMA: lane holds rows 4 v + lane / 16 ... of column lane % 16
    zd* __restrict__ g = G + (int64_t)f * r * r;
    const int col = 16 * J + i;
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int row = 16 * I + q + 4 * v;
      if (row < r && col < r) g[row + (int64_t)col * r] = mk(accr[v], acci[v]);
    }
  }
}

template <typename TY>
int gram_lower(const TY* Y, int rows, int r, int64_t ldy, int64_t sY, int batch, zd* G, hipStream_t s) {
  if (r <= 0 || batch <= 0) return 0;
  const int T = (r + 15) / 16;
  hipLaunchKernelGGL((k_gram_lower<TY>), dim3((unsigned)(T * (T + 1) / 2), (unsigned)batch), dim3(GRAM_THREADS), 0, s,
                     Y, rows, r, ldy, sY, G);
  return hipGetLastError() == hipSuccess ? 0 : -1;
}

}  // namespace rt
