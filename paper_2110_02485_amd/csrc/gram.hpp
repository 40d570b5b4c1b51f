// FP64 Gram matrices G_f = Y_f^H Y_f of the tall panels Y_f (rows x r, column-major, leading
// dimension ldy), lower triangle only (the Cholesky factorization and the eigensolver read
// nothing else).  FP64 16x16x4 MFMA tiles (Section 2's facewise products in double precision).
//
// One workgroup per lower 16 x 16 tile (I, J), J <= I: its 8 waves split the rows into eighths,
// each accumulating the tile over its share, and the shares are summed through LDS in a fixed
// order (deterministic, no atomics, no second kernel).  Operands come straight from L2: for one
// step of 16 rows, lane (i, q) (i = lane % 16, q = lane / 16) holds rows 4q .. 4q+3 of columns
// 16 I + i and 16 J + i.  The 4 MFMA k-steps use the row permutation k = 4 q + s on both sides,
// which leaves the sum unchanged and makes every lane's reads 4 consecutive elements.
// Complex, with A = Y(:, I-tile), B = Y(:, J-tile): three real products per step,
//     P1 = Ar Br, P2 = Ai Bi, P3 = (Ar - Ai)(Br + Bi),  Re G = P1 + P2,  Im G = P3 - P1 + P2
// (= Ar Bi - Ai Br).  For FP32 panels every product is exact in FP64; the absolute error of the
// imaginary part stays at the level of the four-product form (a few units of u ||A|| ||B||).
#pragma once
#include "common.hpp"

namespace rt {

constexpr int GRAM_THREADS = 512;
constexpr int GRAM_WAVES = GRAM_THREADS / 64;
typedef double gr_f64x4 __attribute__((ext_vector_type(4)));

// Grid: 8 ceil(P batch / 8) blocks in one dimension (P lower tiles per face).  The hardware hands
// block b to XCD b % 8; block b takes work item (b % 8) S + b / 8 (S = ceil(P batch / 8)), item
// = face * P + tile, so each XCD works through a contiguous run of faces and reads each face's
// panels into its own L2 once instead of every XCD fetching every face.
// FP32 panels: eight waves per SIMD (64 VGPRs, four workgroups per CU; 65 faces x 36 tiles then
// take three rounds instead of four), the waves hiding one another's load latency in place of the
// one-step register prefetch, which no longer fits; FP64 panels keep the prefetch
template <typename TY> constexpr int gram_min_waves() { return sizeof(TY) == 8 ? 8 : 1; }

template <typename TY>
__global__ void __launch_bounds__(GRAM_THREADS, gram_min_waves<TY>())
k_gram_lower(const TY* __restrict__ Y, int rows, int r, int64_t ldy, int64_t sY, zd* __restrict__ G, int P,
             int batch) {
  __shared__ gr_f64x4 red[GRAM_WAVES - 1][2][64];
  const int items = P * batch, per_xcd = (items + 7) / 8;
  const int item = (int)(blockIdx.x & 7) * per_xcd + (int)(blockIdx.x >> 3);
  if (item >= items) return;   // uniform per block
  const int f = item / P;
  const int p = item - f * P;
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
  const int share = (rows + 16 * GRAM_WAVES - 1) / (16 * GRAM_WAVES) * 16;   // rows per wave, a multiple of 16
  const int k0 = w * share, k1 = min(rows, k0 + share);
  // three independent accumulators (P1, P2, P3) so that consecutive MFMAs never wait on each
  // other's results
  gr_f64x4 acc0 = {0.0, 0.0, 0.0, 0.0}, acc1 = acc0, acc2 = acc0;
  auto mfma_step = [&](const zd* a, const zd* bv) {
#pragma unroll
    for (int s = 0; s < 4; ++s) {
      acc0 = __builtin_amdgcn_mfma_f64_16x16x4f64(a[s].re, bv[s].re, acc0, 0, 0, 0);
      acc1 = __builtin_amdgcn_mfma_f64_16x16x4f64(a[s].im, bv[s].im, acc1, 0, 0, 0);
      acc2 = __builtin_amdgcn_mfma_f64_16x16x4f64(a[s].re - a[s].im, bv[s].re + bv[s].im, acc2, 0, 0, 0);
    }
  };
  int kb = k0;
  // tiles with all 16 + 16 columns inside r, whole steps of 16 rows: no clamps or masks (block-
  // and wave-uniform conditions)
  const int kfull = k0 + (k1 > k0 ? (k1 - k0) / 16 * 16 : 0);
  if (16 * I + 16 <= r && 16 * J + 16 <= r && kfull > k0) {
    const TY* __restrict__ pa = ya + k0 + 4 * q;
    const TY* __restrict__ pb = yb + k0 + 4 * q;
    if constexpr (sizeof(TY) == 8) {
      for (; kb < kfull; kb += 16) {
        zd a[4], bv[4];
#pragma unroll
        for (int s = 0; s < 4; ++s) { a[s] = ld<double>(pa[s]); bv[s] = ld<double>(pb[s]); }
        pa += 16;
        pb += 16;
        mfma_step(a, bv);
      }
    } else {
      TY na[4], nb[4];
#pragma unroll
      for (int s = 0; s < 4; ++s) { na[s] = pa[s]; nb[s] = pb[s]; }
      for (; kb < kfull; kb += 16) {
        zd a[4], bv[4];
#pragma unroll
        for (int s = 0; s < 4; ++s) { a[s] = ld<double>(na[s]); bv[s] = ld<double>(nb[s]); }
        pa += 16;
        pb += 16;
        if (kb + 16 < kfull) {
#pragma unroll
          for (int s = 0; s < 4; ++s) { na[s] = pa[s]; nb[s] = pb[s]; }
        }
        mfma_step(a, bv);
      }
    }
  }
  // edge tiles and the last partial step: loads at clamped rows (in bounds), masked afterwards;
  // the next 16 rows are loaded while the current ones are multiplied
  TY ra[4], rb[4];
  auto load = [&](int kr) {
#pragma unroll
    for (int s = 0; s < 4; ++s) {
      const int kc = min(kr + 4 * q + s, rows - 1);
      ra[s] = ya[kc];
      rb[s] = yb[kc];
    }
  };
  if (kb < k1) load(kb);
  for (; kb < k1; kb += 16) {
    zd a[4], bv[4];
#pragma unroll
    for (int s = 0; s < 4; ++s) {
      const bool in = kb + 4 * q + s < k1;
      const zd va = ld<double>(ra[s]), vb = ld<double>(rb[s]);
      a[s] = mk((oka && in) ? va.re : 0.0, (oka && in) ? va.im : 0.0);
      bv[s] = mk((okb && in) ? vb.re : 0.0, (okb && in) ? vb.im : 0.0);
    }
    load(kb + 16);
    mfma_step(a, bv);
  }
  gr_f64x4 accr = acc0 + acc1, acci = acc2 - acc0 + acc1;
  if (w > 0) {
    red[w - 1][0][lane] = accr;
    red[w - 1][1][lane] = acci;
  }
  __syncthreads();
  if (w == 0) {
#pragma unroll
    for (int u = 0; u < GRAM_WAVES - 1; ++u) {
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

// Slab variant for r <= GS_RMAX: workgroup (q, f) takes rows [q rows/GS_KS, (q+1) rows/GS_KS) of
// face f.  Per step of 16 rows the whole 16 x r slab is staged in LDS (coalesced: 4 threads per
// column, 4 consecutive rows each; double-buffered, converted to FP64), and the 8 waves share the
// lower tiles (wave w takes tiles w, w + 8, ...), so every element is fetched from memory once per
// workgroup instead of once per tile.  The GS_KS partial Gram matrices (lower tiles) go to `part`;
// k_gram_fold sums them in order and mirrors the upper triangle.
constexpr int GS_RMAX = 128;
constexpr int GS_KS = 4;
constexpr int GS_THREADS = 512;
constexpr int GS_LDR = GS_RMAX + 4;          // padded LDS row (elements): rows 4 q apart hit other banks
constexpr int GS_TMAX = (GS_RMAX / 16) * (GS_RMAX / 16 + 1) / 2;   // 36 lower tiles
constexpr int GS_TPW = (GS_TMAX + 7) / 8;                          // tiles per wave (5)

template <typename TY>
__global__ void __launch_bounds__(GS_THREADS)
k_gram_slab(const TY* __restrict__ Y, int rows, int r, int64_t ldy, int64_t sY, zd* __restrict__ part) {
  __shared__ zd slab[2][16][GS_LDR];
  const int q = blockIdx.x, f = blockIdx.y;
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int li = lane & 15, lq = lane >> 4;
  const int T = (r + 15) / 16, P = T * (T + 1) / 2;
  const int share = (rows + 16 * GS_KS - 1) / (16 * GS_KS) * 16;
  const int k0 = q * share, k1 = min(rows, k0 + share);
  const TY* __restrict__ yf = Y + (int64_t)f * sY;
  // staging: thread -> column sc = tid / 4 (< 128), rows 4 (tid % 4) .. + 3 of the slab
  const int scol = tid >> 2, srow = 4 * (tid & 3);
  const bool scol_ok = scol < r;
  const TY* __restrict__ ys = yf + (int64_t)(scol_ok ? scol : 0) * ldy;
  TY st[4];
  auto gload = [&](int kb) {
#pragma unroll
    for (int u = 0; u < 4; ++u) st[u] = ys[min(kb + srow + u, rows - 1)];
  };
  auto lstore = [&](int buf, int kb) {
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const bool ok = scol_ok && kb + srow + u < k1;
      const zd v = ld<double>(st[u]);
      slab[buf][srow + u][scol] = mk(ok ? v.re : 0.0, ok ? v.im : 0.0);
    }
  };
  // this wave's tiles
  int ti[GS_TPW], tj[GS_TPW];
#pragma unroll
  for (int u = 0; u < GS_TPW; ++u) {
    const int p = w + 8 * u;
    int I = 0;
    while ((I + 1) * (I + 2) / 2 <= p) ++I;
    ti[u] = p < P ? I : -1;
    tj[u] = p - I * (I + 1) / 2;
  }
  // per tile the three real products of k_gram_lower: P1 = Ar Br, P2 = Ai Bi, P3 = (Ar - Ai)(Br + Bi)
  gr_f64x4 ap1[GS_TPW], ap2[GS_TPW], ap3[GS_TPW];
#pragma unroll
  for (int u = 0; u < GS_TPW; ++u) { ap1[u] = (gr_f64x4){0.0, 0.0, 0.0, 0.0}; ap2[u] = ap1[u]; ap3[u] = ap1[u]; }
  int buf = 0;
  if (k0 < k1) { gload(k0); lstore(0, k0); }
  __syncthreads();
  for (int kb = k0; kb < k1; kb += 16) {
    const bool more = kb + 16 < k1;
    if (more) gload(kb + 16);
#pragma unroll
    for (int u = 0; u < GS_TPW; ++u) {
      if (ti[u] < 0) continue;                  // uniform per wave
      const int ca = 16 * ti[u] + li, cb = 16 * tj[u] + li;
      gr_f64x4 c1 = ap1[u], c2 = ap2[u], c3 = ap3[u];
#pragma unroll
      for (int s2 = 0; s2 < 4; ++s2) {
        const zd a = slab[buf][4 * lq + s2][ca];
        const zd b = slab[buf][4 * lq + s2][cb];
        c1 = __builtin_amdgcn_mfma_f64_16x16x4f64(a.re, b.re, c1, 0, 0, 0);
        c2 = __builtin_amdgcn_mfma_f64_16x16x4f64(a.im, b.im, c2, 0, 0, 0);
        c3 = __builtin_amdgcn_mfma_f64_16x16x4f64(a.re - a.im, b.re + b.im, c3, 0, 0, 0);
      }
      ap1[u] = c1;
      ap2[u] = c2;
      ap3[u] = c3;
    }
    if (more) lstore(buf ^ 1, kb + 16);
    __syncthreads();
    buf ^= 1;
  }
  zd* __restrict__ pp = part + ((int64_t)f * GS_KS + q) * r * r;
#pragma unroll
  for (int u = 0; u < GS_TPW; ++u) {
    if (ti[u] < 0) continue;
    const int col = 16 * tj[u] + li;
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int row = 16 * ti[u] + lq + 4 * v;
      if (row < r && col < r) pp[row + (int64_t)col * r] = mk(ap1[u][v] + ap2[u][v], ap3[u][v] - ap1[u][v] + ap2[u][v]);
    }
  }
}

// G = sum over the GS_KS partials (fixed order), Hermitian: lower part summed, upper mirrored,
// real diagonal
__global__ void k_gram_fold(const zd* __restrict__ part, int r, zd* __restrict__ G) {
  const int f = blockIdx.y;
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (int64_t)r * r) return;
  const int i = (int)(idx % r), j = (int)(idx / r);
  const int ii = i >= j ? i : j, jj = i >= j ? j : i;
  const zd* p = part + (int64_t)f * GS_KS * r * r + ii + (int64_t)jj * r;
  zd s = mk(0.0, 0.0);
#pragma unroll
  for (int q = 0; q < GS_KS; ++q) s = cadd(s, p[(int64_t)q * r * r]);
  if (i == j) s.im = 0.0;
  G[(int64_t)f * r * r + idx] = (i >= j) ? s : cconj(s);
}

inline int64_t gram_part_elems(int r, int batch) { return r <= GS_RMAX ? (int64_t)batch * GS_KS * r * r : 0; }

template <typename TY>
int gram_slab(const TY* Y, int rows, int r, int64_t ldy, int64_t sY, int batch, zd* part, zd* G, hipStream_t s) {
  hipLaunchKernelGGL((k_gram_slab<TY>), dim3(GS_KS, (unsigned)batch), dim3(GS_THREADS), 0, s, Y, rows, r, ldy, sY, part);
  hipLaunchKernelGGL(k_gram_fold, dim3((unsigned)(((int64_t)r * r + 255) / 256), (unsigned)batch), dim3(256), 0, s,
                     part, r, G);
  return hipGetLastError() == hipSuccess ? 0 : -1;
}

template <typename TY>
int gram_lower(const TY* Y, int rows, int r, int64_t ldy, int64_t sY, int batch, zd* G, hipStream_t s) {
  if (r <= 0 || batch <= 0) return 0;
  const int T = (r + 15) / 16, P = T * (T + 1) / 2;
  const int64_t per_xcd = ((int64_t)P * batch + 7) / 8;
  hipLaunchKernelGGL((k_gram_lower<TY>), dim3((unsigned)(8 * per_xcd)), dim3(GRAM_THREADS), 0, s,
                     Y, rows, r, ldy, sY, G, P, batch);
  return hipGetLastError() == hipSuccess ? 0 : -1;
}

}  // namespace rt
