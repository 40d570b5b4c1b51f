// Batched complex GEMM over Fourier faces: C_f = alpha * op(A_f) op(B_f) (+ C_f).
//
// op(A) is A (M x K, column-major, A[i + k*lda]) or A^H (A stored K x M: op(A)[i][k] =
// conj(A[k + i*lda])); op(B) likewise with B (K x N) or B^H (stored N x K).  Storage types of A,
// B and C are any of zd / zf / zb (double, float, bf16 complex); products accumulate in Acc.
// Every face f uses A + f*strideA etc.  Generic LDS-tiled kernel for the small and medium
// products of the path (Gram matrices, triangular factors, solve-side products); the big
// passes over A-hat use the MFMA kernels in skinny.hpp.
#pragma once
#include "common.hpp"

namespace rt {

template <int BM, int BN, int BK, typename TA, typename TB, typename TC, typename Acc, bool CA, bool CB>
__global__ void __launch_bounds__(256)
k_cgemm(int M, int N, int K, const TA* __restrict__ A, int64_t lda, int64_t sA,
        const TB* __restrict__ B, int64_t ldb, int64_t sB, TC* __restrict__ C, int64_t ldc, int64_t sC,
        Acc alpha, int accumulate) {
  constexpr int TM = BM / 16, TN = BN / 16;
  __shared__ cplx<Acc> As[BK][BM + 1];
  __shared__ cplx<Acc> Bs[BK][BN + 1];
  const int f = blockIdx.z;
  A += f * sA; B += f * sB; C += f * sC;
  const int m0 = blockIdx.x * BM, n0 = blockIdx.y * BN;
  const int tx = threadIdx.x % 16, ty = threadIdx.x / 16;
  cplx<Acc> acc[TM][TN];
#pragma unroll
  for (int a = 0; a < TM; ++a)
#pragma unroll
    for (int b = 0; b < TN; ++b) acc[a][b] = mk((Acc)0, (Acc)0);

  for (int k0 = 0; k0 < K; k0 += BK) {
    // A tile: BM x BK
    for (int idx = threadIdx.x; idx < BM * BK; idx += 256) {
      int i, k;
      if (!CA) { i = idx % BM; k = idx / BM; } else { k = idx % BK; i = idx / BK; }
      const int gi = m0 + i, gk = k0 + k;
      cplx<Acc> v = mk((Acc)0, (Acc)0);
      if (gi < M && gk < K) {
        if (!CA) v = ld<Acc>(A[gi + (int64_t)gk * lda]);
        else v = cconj(ld<Acc>(A[gk + (int64_t)gi * lda]));
      }
      As[k][i] = v;
    }
    for (int idx = threadIdx.x; idx < BN * BK; idx += 256) {
      int j, k;
      if (!CB) { k = idx % BK; j = idx / BK; } else { j = idx % BN; k = idx / BN; }
      const int gj = n0 + j, gk = k0 + k;
      cplx<Acc> v = mk((Acc)0, (Acc)0);
      if (gj < N && gk < K) {
        if (!CB) v = ld<Acc>(B[gk + (int64_t)gj * ldb]);
        else v = cconj(ld<Acc>(B[gj + (int64_t)gk * ldb]));
      }
      Bs[k][j] = v;
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < BK; ++k) {
      cplx<Acc> av[TM], bv[TN];
#pragma unroll
      for (int a = 0; a < TM; ++a) av[a] = As[k][tx + 16 * a];
#pragma unroll
      for (int b = 0; b < TN; ++b) bv[b] = Bs[k][ty + 16 * b];
#pragma unroll
      for (int a = 0; a < TM; ++a)
#pragma unroll
        for (int b = 0; b < TN; ++b) {
          acc[a][b].re += av[a].re * bv[b].re - av[a].im * bv[b].im;
          acc[a][b].im += av[a].re * bv[b].im + av[a].im * bv[b].re;
        }
    }
    __syncthreads();
  }
#pragma unroll
  for (int a = 0; a < TM; ++a)
#pragma unroll
    for (int b = 0; b < TN; ++b) {
      const int gi = m0 + tx + 16 * a, gj = n0 + ty + 16 * b;
      if (gi < M && gj < N) {
        cplx<Acc> v = cscale(acc[a][b], alpha);
        TC& dst = C[gi + (int64_t)gj * ldc];
        if (accumulate) v = cadd(v, ld<Acc>(dst));
        st(dst, v);
      }
    }
}

// Few right-hand sides (N <= GEMV_NP, op(B) = B): matrix-vector products, bound by the one pass
// over A.  A^H X: one wave per output row (a stored column of A, read contiguously by the lanes),
// reduced across the wave; with 8-byte elements (FP32 complex) on both sides and 16-byte aligned
// columns (vec, checked by the host) each lane reads two consecutive elements per 16-byte load.
// A X: one lane per output row, the K range split over the 4 waves of the block and reduced in LDS.
constexpr int GEMV_NP = 4;

template <typename TA, typename TB, typename TC, typename Acc, int NP>
__global__ void __launch_bounds__(256)
k_gemv_cn(int M, int N, int K, const TA* __restrict__ A, int64_t lda, int64_t sA,
          const TB* __restrict__ B, int64_t ldb, int64_t sB, TC* __restrict__ C, int64_t ldc, int64_t sC,
          Acc alpha, int accumulate, int vec) {
  const int f = blockIdx.y;
  const int i = blockIdx.x * 4 + (threadIdx.x >> 6), lane = threadIdx.x & 63;
  if (i >= M) return;
  const TA* __restrict__ a = A + f * sA + (int64_t)i * lda;
  const TB* __restrict__ b = B + f * sB;
  cplx<Acc> acc[NP];
#pragma unroll
  for (int c = 0; c < NP; ++c) acc[c] = mk((Acc)0, (Acc)0);
  int k = lane;
  if constexpr (sizeof(TA) == 8 && sizeof(TB) == 8) {
    if (vec) {
      // pairs (2 j, 2 j + 1), j = lane, lane + 64, ...: whole pairs below K2, the rest below
      const int K2 = K & ~1;
#pragma unroll 8
      for (int k2 = 2 * lane; k2 < K2; k2 += 128) {
        const float4 av = *reinterpret_cast<const float4*>(a + k2);
#pragma unroll
        for (int c = 0; c < NP; ++c)
          if (c < N) {
            const float4 bv = *reinterpret_cast<const float4*>(b + k2 + c * ldb);
            acc[c] = cadd(acc[c], cmulc(mk((Acc)av.x, (Acc)av.y), mk((Acc)bv.x, (Acc)bv.y)));
            acc[c] = cadd(acc[c], cmulc(mk((Acc)av.z, (Acc)av.w), mk((Acc)bv.z, (Acc)bv.w)));
          }
      }
      k = K2 + lane;
    }
  }
#pragma unroll 16
  for (; k < K; k += 64) {
    const cplx<Acc> av = ld<Acc>(a[k]);
#pragma unroll
    for (int c = 0; c < NP; ++c)
      if (c < N) acc[c] = cadd(acc[c], cmulc(av, ld<Acc>(b[k + c * ldb])));  // conj(a) b
  }
#pragma unroll
  for (int c = 0; c < NP; ++c) {
    if (c >= N) break;
    cplx<Acc> v = acc[c];
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) { v.re += __shfl_xor(v.re, o, 64); v.im += __shfl_xor(v.im, o, 64); }
    if (lane == 0) {
      v = cscale(v, alpha);
      TC& dst = C[f * sC + i + (int64_t)c * ldc];
      if (accumulate) v = cadd(v, ld<Acc>(dst));
      st(dst, v);
    }
  }
}

template <typename TA, typename TB, typename TC, typename Acc, int NP>
__global__ void __launch_bounds__(256)
k_gemv_nn(int M, int N, int K, const TA* __restrict__ A, int64_t lda, int64_t sA,
          const TB* __restrict__ B, int64_t ldb, int64_t sB, TC* __restrict__ C, int64_t ldc, int64_t sC,
          Acc alpha, int accumulate) {
  __shared__ cplx<Acc> part[3][NP][64];
  const int f = blockIdx.y;
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int i = blockIdx.x * 64 + lane;
  const bool on = i < M;
  const TA* __restrict__ a = A + f * sA + (on ? i : 0);
  const TB* __restrict__ b = B + f * sB;
  const int kq = (K + 3) / 4, k0 = w * kq, k1 = min(K, k0 + kq);
  cplx<Acc> acc[NP];
#pragma unroll
  for (int c = 0; c < NP; ++c) acc[c] = mk((Acc)0, (Acc)0);
#pragma unroll 8
  for (int k = k0; k < k1; ++k) {
    const cplx<Acc> av = ld<Acc>(a[(int64_t)k * lda]);
#pragma unroll
    for (int c = 0; c < NP; ++c)
      if (c < N) acc[c] = cadd(acc[c], cmul(av, ld<Acc>(b[k + c * ldb])));
  }
  if (w > 0) {
#pragma unroll
    for (int c = 0; c < NP; ++c) part[w - 1][c][lane] = acc[c];
  }
  __syncthreads();
  if (w == 0 && on) {
#pragma unroll
    for (int c = 0; c < NP; ++c) {
      if (c >= N) break;
      cplx<Acc> v = cadd(cadd(acc[c], part[0][c][lane]), cadd(part[1][c][lane], part[2][c][lane]));
      v = cscale(v, alpha);
      TC& dst = C[f * sC + i + (int64_t)c * ldc];
      if (accumulate) v = cadd(v, ld<Acc>(dst));
      st(dst, v);
    }
  }
}

template <typename TA, typename TB, typename TC, typename Acc>
int cgemm(bool conjA, bool conjB, int M, int N, int K, const TA* A, int64_t lda, int64_t sA,
          const TB* B, int64_t ldb, int64_t sB, TC* C, int64_t ldc, int64_t sC, int batch,
          Acc alpha, bool accumulate, hipStream_t s) {
  if (M <= 0 || N <= 0 || batch <= 0) return 0;
  if (N <= GEMV_NP && !conjB && K > 0) {
    if (conjA) {
      // 16-byte pair loads: both operands FP32 complex, every column start 16-byte aligned
      const bool vec = sizeof(TA) == 8 && sizeof(TB) == 8 && (uintptr_t)A % 16 == 0 && (uintptr_t)B % 16 == 0 &&
                       lda % 2 == 0 && sA % 2 == 0 && ldb % 2 == 0 && sB % 2 == 0;
      hipLaunchKernelGGL((k_gemv_cn<TA, TB, TC, Acc, GEMV_NP>), dim3((unsigned)ceil_div(M, 4), (unsigned)batch),
                         dim3(256), 0, s, M, N, K, A, lda, sA, B, ldb, sB, C, ldc, sC, alpha, (int)accumulate,
                         (int)vec);
    } else
      hipLaunchKernelGGL((k_gemv_nn<TA, TB, TC, Acc, GEMV_NP>), dim3((unsigned)ceil_div(M, 64), (unsigned)batch),
                         dim3(256), 0, s, M, N, K, A, lda, sA, B, ldb, sB, C, ldc, sC, alpha, (int)accumulate);
    return hipGetLastError() == hipSuccess ? 0 : -1;
  }
  constexpr int BM = 64, BN = 64, BK = 8;
  dim3 grid((unsigned)ceil_div(M, BM), (unsigned)ceil_div(N, BN), (unsigned)batch);
  if (!conjA && !conjB)
    hipLaunchKernelGGL((k_cgemm<BM, BN, BK, TA, TB, TC, Acc, false, false>), grid, dim3(256), 0, s,
                       M, N, K, A, lda, sA, B, ldb, sB, C, ldc, sC, alpha, (int)accumulate);
  else if (conjA && !conjB)
    hipLaunchKernelGGL((k_cgemm<BM, BN, BK, TA, TB, TC, Acc, true, false>), grid, dim3(256), 0, s,
                       M, N, K, A, lda, sA, B, ldb, sB, C, ldc, sC, alpha, (int)accumulate);
  else if (!conjA && conjB)
    hipLaunchKernelGGL((k_cgemm<BM, BN, BK, TA, TB, TC, Acc, false, true>), grid, dim3(256), 0, s,
                       M, N, K, A, lda, sA, B, ldb, sB, C, ldc, sC, alpha, (int)accumulate);
  else
    hipLaunchKernelGGL((k_cgemm<BM, BN, BK, TA, TB, TC, Acc, true, true>), grid, dim3(256), 0, s,
                       M, N, K, A, lda, sA, B, ldb, sB, C, ldc, sC, alpha, (int)accumulate);
  return hipGetLastError() == hipSuccess ? 0 : -1;
}

}  // namespace rt
