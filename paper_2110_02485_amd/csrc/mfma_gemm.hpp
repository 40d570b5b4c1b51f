// Batched complex GEMM on MFMA (gfx950) for the products over A-hat and the FP64 Gram matrices.
//
//   C_f = op(A_f) op(B_f),  op = identity or conjugate transpose, f = Fourier face.
//
// Complex arithmetic runs as four real MFMA products on split real/imaginary planes staged in
// LDS:  Re C += Ar Br + Ai (-Bi),  Im C += Ar Bi + Ai Br  (conjugation applied while staging).
// Precisions (operands are converted to the MFMA type while staging):
//   P64  : v_mfma_f64_16x16x4_f64,   FP64 accumulation
//   P32  : v_mfma_f32_16x16x4_f32,   FP32 accumulation
//   PB16 : v_mfma_f32_16x16x32_bf16, FP32 accumulation (bf16 operands, round to nearest even)
// MFMA lane layout (16 x 16 output tile): lane l holds A rows l%16 at k = KPER*(l/16) .. +KPER-1,
// B columns l%16 at the same k; output element v < 4 of lane l is column l%16 of row
// 4*(l/16)+v (f32, bf16) or row (l/16)+4v (f64).
//
// The skinny dimension (r <= 128 columns of the sketch) is covered by one block column, so each
// pass reads A-hat exactly once; blocks of one face are mapped onto the same XCD (block ids
// congruent mod 8) so that the skinny operand of a face is shared through that XCD's L2.
#pragma once
#include "gemm.hpp"
#include <type_traits>

namespace rt {

typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef double f64x4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));

struct P64 {
  typedef double E;
  typedef double Acc;
  typedef f64x4 V;
  static constexpr int KM = 4, KPER = 1, PAD = 1;
  static __device__ __forceinline__ E cvt(double x) { return x; }
  typedef double Frag;
  static __device__ __forceinline__ Frag frag(const E* p) { return *p; }
  static __device__ __forceinline__ Frag neg(Frag a) { return -a; }
  static __device__ __forceinline__ V mma(Frag a, Frag b, V c) { return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0); }
  // output element v of lane l sits in row (l/16) + 4 v (measured on gfx950)
  static __device__ __forceinline__ int out_row(int lane, int v) { return (lane >> 4) + 4 * v; }
};
struct P32 {
  typedef float E;
  typedef float Acc;
  typedef f32x4 V;
  static constexpr int KM = 4, KPER = 1, PAD = 1;
  static __device__ __forceinline__ E cvt(double x) { return (float)x; }
  typedef float Frag;
  static __device__ __forceinline__ Frag frag(const E* p) { return *p; }
  static __device__ __forceinline__ Frag neg(Frag a) { return -a; }
  static __device__ __forceinline__ V mma(Frag a, Frag b, V c) { return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0); }
  static __device__ __forceinline__ int out_row(int lane, int v) { return 4 * (lane >> 4) + v; }
};
struct PB16 {
  typedef uint16_t E;
  typedef float Acc;
  typedef f32x4 V;
  static constexpr int KM = 32, KPER = 8, PAD = 8;
  static __device__ __forceinline__ E cvt(double x) { return (uint16_t)f2bf((float)x); }
  typedef bf16x8 Frag;
  static __device__ __forceinline__ Frag frag(const E* p) { return *reinterpret_cast<const bf16x8*>(p); }
  static __device__ __forceinline__ Frag neg(Frag a) {
    typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
    u32x4 u = __builtin_bit_cast(u32x4, a);
    u ^= (u32x4)(0x80008000u);
    return __builtin_bit_cast(bf16x8, u);
  }
  static __device__ __forceinline__ V mma(Frag a, Frag b, V c) { return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0); }
  static __device__ __forceinline__ int out_row(int lane, int v) { return 4 * (lane >> 4) + v; }
};

// read a storage element as (re, im) in the staging type -- bf16 storage is read exactly
template <typename T> __device__ __forceinline__ void ld2(const zd& z, T& a, T& b) { a = (T)z.re; b = (T)z.im; }
template <typename T> __device__ __forceinline__ void ld2(const zf& z, T& a, T& b) { a = (T)z.re; b = (T)z.im; }
template <typename T> __device__ __forceinline__ void ld2(const zb& z, T& a, T& b) {
  a = (T)bf2f(z.bits & 0xffffu); b = (T)bf2f(z.bits >> 16);
}
// staging arithmetic type: double for the FP64 MFMA, float otherwise
template <class P> struct StageT { typedef float T; };
template <> struct StageT<P64> { typedef double T; };

// Grid: x = batch * mtiles * ntiles (XCD-aware order), y = k splits.  Block = 256 threads.
// Output: C + f*sC + split*sCsplit (split partials summed by k_gram_reduce when ksplit > 1).
// lower_only: skip tiles strictly above the diagonal (Hermitian Gram).
// Operand staging: every thread moves chunks of CH consecutive k of one row of op(A) (one column
// of B) from global memory into registers for the next k-step while the MFMAs of the current
// k-step run, then converts them and writes them to LDS after the barrier.
template <class P, bool CA, typename TA, typename TB, typename TC, int BM, int BN, int BK, int WM, int WN>
__global__ void __launch_bounds__(256)
k_mfma_cgemm(int M, int N, int K, const TA* __restrict__ A, int64_t lda, int64_t sA, const TB* __restrict__ B,
             int64_t ldb, int64_t sB, TC* __restrict__ C, int64_t ldc, int64_t sC, int batch, int mtiles, int ntiles,
             int kchunk, int64_t sCsplit, int lower_only) {
  typedef typename P::E E;
  typedef typename P::V V;
  typedef typename StageT<P>::T ST;
  constexpr int BKP = BK + P::PAD;
  constexpr int TMW = BM / WM / 16, TNW = BN / WN / 16;
  constexpr int CH = (P::KPER == 8) ? 8 : 4;               // k elements per staging chunk
  constexpr int ACH = BM * BK / CH / 256, BCH = BN * BK / CH / 256;
  static_assert(ACH >= 1 && BCH >= 1 && BM * BK % (CH * 256) == 0 && BN * BK % (CH * 256) == 0, "tile/chunk mismatch");
  __shared__ __align__(16) E As[2][BM][BKP];
  __shared__ __align__(16) E Bs[2][BN][BKP];

  // XCD-aware decode: hardware dispatches block b to XCD b % 8; the tiles of one face share b % 8
  const int tiles = mtiles * ntiles;
  const int b = blockIdx.x;
  const int nb = gridDim.x;
  int f, t;
  if (nb % 8 == 0 && batch >= 8) {
    const int xcd = b % 8, slot = b / 8;
    const int faces_per_xcd = (nb / 8) / tiles;
    const int fl = slot / tiles;
    t = slot % tiles;
    f = fl * 8 + xcd;
    if (fl >= faces_per_xcd || f >= batch) return;
  } else {
    f = b / tiles;
    t = b % tiles;
  }
  const int mt = t % mtiles, nt = t / mtiles;
  const int m0 = mt * BM, n0 = nt * BN;
  if (lower_only && n0 > m0 + BM - 1) return;
  const int split = blockIdx.y;
  const int kbeg = split * kchunk;
  const int kend = min(K, kbeg + kchunk);

  A += (int64_t)f * sA;
  B += (int64_t)f * sB;
  C += (int64_t)f * sC + (int64_t)split * sCsplit;

  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = wave % WM, wn = wave / WM;
  const int lr = lane & 15, lk = (lane >> 4) * P::KPER;

  // chunk coordinates: A chunk q -> (row ai, k offset ak); B chunk q -> (column bj, k offset bk)
  int ai[ACH], ak[ACH], bj[BCH], bk[BCH];
#pragma unroll
  for (int q = 0; q < ACH; ++q) {
    const int c = tid + 256 * q;
    if (!CA) { ai[q] = c % BM; ak[q] = (c / BM) * CH; }   // rows contiguous in global: coalesce along rows
    else { ak[q] = (c % (BK / CH)) * CH; ai[q] = c / (BK / CH); }
  }
#pragma unroll
  for (int q = 0; q < BCH; ++q) {
    const int c = tid + 256 * q;
    bk[q] = (c % (BK / CH)) * CH; bj[q] = c / (BK / CH);
  }
  ST ra[ACH][CH][2], rb[BCH][CH][2];

  auto load_tiles = [&](int k0) {
#pragma unroll
    for (int q = 0; q < ACH; ++q) {
      const int gi = m0 + ai[q];
#pragma unroll
      for (int e = 0; e < CH; ++e) {
        const int gk = k0 + ak[q] + e;
        ST re = 0, im = 0;
        if (gi < M && gk < kend) {
          if (!CA) ld2<ST>(A[gi + (int64_t)gk * lda], re, im);
          else { ld2<ST>(A[gk + (int64_t)gi * lda], re, im); im = -im; }
        }
        ra[q][e][0] = re; ra[q][e][1] = im;
      }
    }
#pragma unroll
    for (int q = 0; q < BCH; ++q) {
      const int gj = n0 + bj[q];
#pragma unroll
      for (int e = 0; e < CH; ++e) {
        const int gk = k0 + bk[q] + e;
        ST re = 0, im = 0;
        if (gj < N && gk < kend) ld2<ST>(B[gk + (int64_t)gj * ldb], re, im);
        rb[q][e][0] = re; rb[q][e][1] = im;
      }
    }
  };
  auto store_tiles = [&]() {
#pragma unroll
    for (int q = 0; q < ACH; ++q)
#pragma unroll
      for (int pl = 0; pl < 2; ++pl) {
        E tmp[CH];
#pragma unroll
        for (int e = 0; e < CH; ++e) tmp[e] = P::cvt(ra[q][e][pl]);
#pragma unroll
        for (int e = 0; e < CH; ++e) As[pl][ai[q]][ak[q] + e] = tmp[e];
      }
#pragma unroll
    for (int q = 0; q < BCH; ++q)
#pragma unroll
      for (int pl = 0; pl < 2; ++pl) {
        E tmp[CH];
#pragma unroll
        for (int e = 0; e < CH; ++e) tmp[e] = P::cvt(rb[q][e][pl]);
#pragma unroll
        for (int e = 0; e < CH; ++e) Bs[pl][bj[q]][bk[q] + e] = tmp[e];
      }
  };

  V accr[TMW][TNW], acci[TMW][TNW];
#pragma unroll
  for (int i = 0; i < TMW; ++i)
#pragma unroll
    for (int j = 0; j < TNW; ++j) {
#pragma unroll
      for (int v = 0; v < 4; ++v) { accr[i][j][v] = 0; acci[i][j][v] = 0; }
    }

  if (kbeg < kend) {
    load_tiles(kbeg);
    store_tiles();
  }
  __syncthreads();
  for (int k0 = kbeg; k0 < kend; k0 += BK) {
    const bool more = k0 + BK < kend;
    if (more) load_tiles(k0 + BK);     // global loads in flight during the MFMAs below
#pragma unroll
    for (int ks = 0; ks < BK; ks += P::KM) {
      typename P::Frag ar[TMW], aim[TMW];
#pragma unroll
      for (int i = 0; i < TMW; ++i) {
        const int row = wm * (BM / WM) + i * 16 + lr;
        ar[i] = P::frag(&As[0][row][ks + lk]);
        aim[i] = P::frag(&As[1][row][ks + lk]);
      }
#pragma unroll
      for (int j = 0; j < TNW; ++j) {
        const int col = wn * (BN / WN) + j * 16 + lr;
        const typename P::Frag br = P::frag(&Bs[0][col][ks + lk]);
        const typename P::Frag bi = P::frag(&Bs[1][col][ks + lk]);
        const typename P::Frag bn = P::neg(bi);
#pragma unroll
        for (int i = 0; i < TMW; ++i) {
          accr[i][j] = P::mma(ar[i], br, accr[i][j]);
          accr[i][j] = P::mma(aim[i], bn, accr[i][j]);
          acci[i][j] = P::mma(ar[i], bi, acci[i][j]);
          acci[i][j] = P::mma(aim[i], br, acci[i][j]);
        }
      }
    }
    __syncthreads();
    if (more) {
      store_tiles();
      __syncthreads();
    }
  }
  // ---- store ----
#pragma unroll
  for (int i = 0; i < TMW; ++i)
#pragma unroll
    for (int j = 0; j < TNW; ++j) {
      const int col = n0 + wn * (BN / WN) + j * 16 + lr;
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int row = m0 + wm * (BM / WM) + i * 16 + P::out_row(lane, v);
        if (row < M && col < N) st(C[row + (int64_t)col * ldc], mk((double)accr[i][j][v], (double)acci[i][j][v]));
      }
    }
}

// G_f = sum over splits of the partials, lower triangle; upper triangle mirrored (Hermitian).
__global__ void k_gram_reduce(const zd* __restrict__ part, int r, int ksplit, int64_t sPart, zd* __restrict__ G) {
  const int f = blockIdx.y;
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (int64_t)r * r) return;
  const int i = (int)(idx % r), j = (int)(idx / r);
  const int ii = i >= j ? i : j, jj = i >= j ? j : i;  // lower element (ii >= jj)
  const zd* p = part + (int64_t)f * ksplit * sPart;
  zd s = mk(0.0, 0.0);
  for (int q = 0; q < ksplit; ++q) s = cadd(s, p[(int64_t)q * sPart + ii + (int64_t)jj * r]);
  if (i == j) s.im = 0.0;
  G[(int64_t)f * r * r + idx] = (i >= j) ? s : cconj(s);
}

// ---------------------------------------------------------------------------------------------
// host launchers
// ---------------------------------------------------------------------------------------------
template <class P, bool CA, typename TA, typename TB, typename TC, int BM, int BN, int BK, int WM, int WN>
int launch_mfma(int M, int N, int K, const TA* A, int64_t lda, int64_t sA, const TB* B, int64_t ldb, int64_t sB,
                TC* C, int64_t ldc, int64_t sC, int batch, int ksplit, int64_t sCsplit, bool lower_only, hipStream_t s) {
  const int mtiles = (int)ceil_div(M, BM), ntiles = (int)ceil_div(N, BN);
  const int tiles = mtiles * ntiles;
  int64_t nblk = (int64_t)batch * tiles;
  if (batch >= 8) nblk = ceil_div(batch, 8) * 8 * (int64_t)tiles;  // XCD-aware decode needs a multiple of 8
  int kchunk = (int)ceil_div(ceil_div(K, ksplit), BK) * BK;
  hipLaunchKernelGGL((k_mfma_cgemm<P, CA, TA, TB, TC, BM, BN, BK, WM, WN>), dim3((unsigned)nblk, (unsigned)ksplit),
                     dim3(256), 0, s, M, N, K, A, lda, sA, B, ldb, sB, C, ldc, sC, batch, mtiles, ntiles, kchunk,
                     sCsplit, (int)lower_only);
  return hipGetLastError() == hipSuccess ? 0 : -1;
}

// Traits for the big passes by storage type of A-hat.
template <typename TA, typename Acc> struct BigP;
template <> struct BigP<zd, double> { typedef P64 P; };
template <> struct BigP<zf, float> { typedef P32 P; };
template <> struct BigP<zb, float> { typedef PB16 P; };

// Y = op(A) X with X skinny (N <= 256): one block column when N <= 128.
template <typename TA, typename TX, typename TY, typename Acc>
int big_cgemm(bool conjA, int M, int N, int K, const TA* A, int64_t lda, int64_t sA, const TX* X, int64_t ldx,
              int64_t sX, TY* Y, int64_t ldy, int64_t sY, int batch, hipStream_t s) {
  typedef typename BigP<TA, Acc>::P P;
  if constexpr (std::is_same<P, P64>::value) {
    if (!conjA) return launch_mfma<P, false, TA, TX, TY, 64, 128, 16, 1, 4>(M, N, K, A, lda, sA, X, ldx, sX, Y, ldy, sY, batch, 1, 0, false, s);
    return launch_mfma<P, true, TA, TX, TY, 64, 128, 16, 1, 4>(M, N, K, A, lda, sA, X, ldx, sX, Y, ldy, sY, batch, 1, 0, false, s);
  } else if constexpr (std::is_same<P, P32>::value) {
    if (!conjA) return launch_mfma<P, false, TA, TX, TY, 128, 128, 16, 2, 2>(M, N, K, A, lda, sA, X, ldx, sX, Y, ldy, sY, batch, 1, 0, false, s);
    return launch_mfma<P, true, TA, TX, TY, 128, 128, 16, 2, 2>(M, N, K, A, lda, sA, X, ldx, sX, Y, ldy, sY, batch, 1, 0, false, s);
  } else {
    if (!conjA) return launch_mfma<P, false, TA, TX, TY, 128, 128, 32, 2, 2>(M, N, K, A, lda, sA, X, ldx, sX, Y, ldy, sY, batch, 1, 0, false, s);
    return launch_mfma<P, true, TA, TX, TY, 128, 128, 32, 2, 2>(M, N, K, A, lda, sA, X, ldx, sX, Y, ldy, sY, batch, 1, 0, false, s);
  }
}

// Skinny-times-small products Y = X R (K = r, FP32 or FP64 MFMA by output type)
template <typename TX, typename TR, typename TY>
int small_k_cgemm(int M, int N, int K, const TX* X, int64_t ldx, int64_t sX, const TR* R, int64_t ldr, int64_t sR,
                  TY* Y, int64_t ldy, int64_t sY, int batch, hipStream_t s) {
  if constexpr (std::is_same<TY, zd>::value)
    return launch_mfma<P64, false, TX, TR, TY, 64, 128, 16, 1, 4>(M, N, K, X, ldx, sX, R, ldr, sR, Y, ldy, sY, batch, 1, 0, false, s);
  else
    return launch_mfma<P32, false, TX, TR, TY, 128, 128, 16, 2, 2>(M, N, K, X, ldx, sX, R, ldr, sR, Y, ldy, sY, batch, 1, 0, false, s);
}

// FP64 Gram G_f = Y_f^H Y_f (r x r), Y_f rows x r of any storage type; split-K partials in `part`
// (batch x ksplit x r x r doubles complex), lower tiles only, then a deterministic reduction.
template <typename TY>
int gram_fp64(const TY* Y, int64_t rows, int r, int64_t sY, int batch, zd* part, int ksplit, zd* G, hipStream_t s) {
  const int64_t sPart = (int64_t)r * r;
  int rc = launch_mfma<P64, true, TY, TY, zd, 64, 64, 16, 2, 2>(r, r, (int)rows, Y, rows, sY, Y, rows, sY, part,
                                                                       r, (int64_t)ksplit * sPart, batch, ksplit, sPart,
                                                                       true, s);
  if (rc) return rc;
  hipLaunchKernelGGL(k_gram_reduce, dim3((unsigned)ceil_div((int64_t)r * r, 256), (unsigned)batch), dim3(256), 0, s,
                     part, r, ksplit, sPart, G);
  return hipGetLastError() == hipSuccess ? 0 : -1;
}

}  // namespace rt
