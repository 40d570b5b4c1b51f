// Skinny batched complex products on MFMA (gfx950):  C_f = op(A_f) X_f,  op = identity (NN) or
// conjugate transpose (CN), f = Fourier face, X_f with few columns (the sketch width r).  These are
// the passes over A-hat of the randomized factorization (sketch, power iteration, projection,
// W = A-hat V), the FP64 Gram matrices of CholeskyQR and the right-multiplications Y R^{-1}.
//
// Design (block = 8 waves = WR row groups x WC column groups; a wave owns 16*RT rows and 16*NTW
// columns of C; the waves of a row group read the same A fragments, all but one from L1/L2):
//  * op(A) is streamed from global memory straight into MFMA operand registers, without LDS, so
//    each element of A is read from HBM once per block column.  NN (A column-major, rows contiguous): a
//    lane loads RT neighbouring rows for each of its k (16 lanes cover 128-256 contiguous bytes);
//    CN: a lane loads KL consecutive k of one column.  The MFMA k slot is a relabelling of k
//    (lane group g = lane/16 holds k = k0 + KL*g + e), applied identically to X.
//  * X is staged through LDS one macro step (KS = 4*KL values of k) at a time in a ring of three
//    buffers, one barrier per step, rows padded to 80 or 144 bytes so 16-byte fragment reads are free of
//    bank conflicts.  X arrives either pre-packed (split planes of the MFMA type, k contiguous,
//    zero padded: k_pack_planes) or raw complex (converted while staging).
//  * With RT = 2 the two row tiles of a wave interleave (row 2*rho + t), so a lane's outputs are
//    8 consecutive rows of one column and are written with 16-byte stores.
//  * Complex arithmetic is four real MFMA products on split planes:
//      Re C += Ar Xr + (-Ai) Xi,   Im C += Ar Xi + Ai Xr   (conjugation of A folded into Ai).
//  * The blocks of one face run on one XCD (block id congruent mod 8), sharing X in that L2.
// MFMA output layouts (16 x 16 tile, element v < 4 of lane l, column l % 16): f32 accumulators
// row 4*(l/16) + v; f64 accumulators row (l/16) + 4*v.
#pragma once
#include "common.hpp"
#include <type_traits>

namespace rt {
namespace sk {

typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef double f64x4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef uint32_t u32x2 __attribute__((ext_vector_type(2)));
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));

// precisions: MFMA element type E, accumulator, k per lane per macro step (every lane reads
// 16 bytes of X per plane and column tile per step), LDS row pad (16 bytes), row tiles per wave
struct B16 {  // v_mfma_f32_16x16x32_bf16
  typedef uint16_t E; typedef float Acc; typedef f32x4 V;
  static constexpr int KL = 8, PADE = 8, RT = 2;
};
struct F32 {  // v_mfma_f32_16x16x4_f32
  typedef float E; typedef float Acc; typedef f32x4 V;
  static constexpr int KL = 4, PADE = 4, RT = 2;
};
struct F64 {  // v_mfma_f64_16x16x4_f64
  typedef double E; typedef double Acc; typedef f64x4 V;
  static constexpr int KL = 2, PADE = 2, RT = 1;
};

template <typename E> __device__ __forceinline__ E cvt_e(double x);
template <> __device__ __forceinline__ uint16_t cvt_e<uint16_t>(double x) { return (uint16_t)f2bf((float)x); }
template <> __device__ __forceinline__ float cvt_e<float>(double x) { return (float)x; }
template <> __device__ __forceinline__ double cvt_e<double>(double x) { return x; }

template <int BYTES> struct VecOf;
template <> struct VecOf<4> { typedef uint32_t T; };
template <> struct VecOf<8> { typedef u32x2 T; };
template <> struct VecOf<16> { typedef u32x4 T; };

// CNT consecutive elements from an address aligned to min(16, CNT*sizeof(T)) bytes
template <typename T, int CNT>
__device__ __forceinline__ void vload(const T* p, T (&out)[CNT]) {
  constexpr int BYTES = (int)sizeof(T) * CNT;
  if constexpr (BYTES <= 16) {
    typedef typename VecOf<BYTES>::T VT;
    const VT v = *reinterpret_cast<const VT*>(p);
    __builtin_memcpy(&out[0], &v, BYTES);
  } else {
    static_assert(BYTES % 16 == 0, "vector load size");
#pragma unroll
    for (int i = 0; i < BYTES / 16; ++i) {
      const u32x4 v = reinterpret_cast<const u32x4*>(p)[i];
      __builtin_memcpy(reinterpret_cast<char*>(&out[0]) + 16 * i, &v, 16);
    }
  }
}
template <typename T, int CNT>
__device__ __forceinline__ void vstore(T* p, const T (&in)[CNT]) {
  constexpr int BYTES = (int)sizeof(T) * CNT;
  static_assert(BYTES % 16 == 0, "vector store size");
#pragma unroll
  for (int i = 0; i < BYTES / 16; ++i) {
    u32x4 v;
    __builtin_memcpy(&v, reinterpret_cast<const char*>(&in[0]) + 16 * i, 16);
    reinterpret_cast<u32x4*>(p)[i] = v;
  }
}

__device__ __forceinline__ f32x4 mma(bf16x8 a, bf16x8 b, f32x4 c) { return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0); }
__device__ __forceinline__ f32x4 mma(float a, float b, f32x4 c) { return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0); }
__device__ __forceinline__ f64x4 mma(double a, double b, f64x4 c) { return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0); }

constexpr int SK_THREADS = 512;  // 8 waves: 2 per SIMD

// Block shape for NB column tiles of 16: WC column groups of NTW tiles, WR = 8 / WC row groups.
template <int NB> struct Shape {
#ifdef SKINNY_WC
  static constexpr int WC = NB >= SKINNY_WC ? SKINNY_WC : NB;
#else
  static constexpr int WC = NB >= 4 ? 4 : NB;
#endif
  static constexpr int NTW = NB / WC, WR = 8 / WC;
};

// X staging ring: three LDS buffers of (2 planes x 16 NB rows x padded macro step)
template <class P> constexpr int lds_bytes(int NB) {
  return 3 * 2 * 16 * NB * (4 * P::KL + P::PADE) * (int)sizeof(typename P::E);
}

// Xp_f = split planes of X_f: Xp[f][plane][n][k] (plane 0 real, 1 imaginary), n < NPt, k < KP,
// zero outside K x N.  X_f is column-major K x N with leading dimension ldx.
template <typename TX, typename E>
__global__ void k_pack_planes(const TX* __restrict__ X, int64_t ldx, int64_t sX, int K, int N, E* __restrict__ Xp,
                              int KP, int NPt, int batch) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t per = (int64_t)NPt * KP;
  if (idx >= per * batch) return;
  const int64_t f = idx / per;
  const int n = (int)((idx % per) / KP), k = (int)(idx % KP);
  double re = 0.0, im = 0.0;
  if (n < N && k < K) {
    const cplx<double> v = ld<double>(X[f * sX + k + (int64_t)n * ldx]);
    re = v.re; im = v.im;
  }
  E* base = Xp + f * 2 * per + (int64_t)n * KP + k;
  base[0] = cvt_e<E>(re);
  base[per] = cvt_e<E>(im);
}

// C_f (+ split * sCsplit) = op(A_f) X_f, M x N, contraction length K.
// PACKED: X is E* planes [f][2][NPt][ldx] with face stride sX; otherwise X is TX* column-major.
// SAFE = false: the host guarantees M % (64 RT) == 0, K % (4 KL) == 0 and the alignment of the
// vector loads of A (and of raw X); SAFE = true clamps every A and X index instead (element
// loads).  Both paths are branch-free inside the k loop.  LOWER: skip column tiles strictly above
// the diagonal (Hermitian Gram).  vec_c: the host has checked the alignment of 16-byte stores.
template <class P, bool CN, bool PACKED, bool SAFE, bool LOWER, typename TA, typename TX, typename TC, int NB>
__global__ void __launch_bounds__(SK_THREADS, 2)
k_skinny(int M, int N, int K, const TA* __restrict__ A, int64_t lda, int64_t sA, const void* __restrict__ Xv,
         int64_t ldx, int64_t sX, TC* __restrict__ C, int64_t ldc, int64_t sC, int batch, int mtiles, int ntiles,
         int kchunk, int64_t sCsplit, int vec_c) {
  typedef typename P::E E;
  typedef typename P::V V;
  typedef typename P::Acc Acc;
  constexpr int KL = P::KL, RT = P::RT, KS = 4 * KL, ROWE = KS + P::PADE, NP = 16 * NB;  // NP: block columns
  constexpr int NT = Shape<NB>::NTW, WR = Shape<NB>::WR;
  constexpr int BM = WR * 16 * RT;
  constexpr int PLANE = NP * ROWE, BUF = 2 * PLANE;
  constexpr int CK = 16 / (int)sizeof(E);  // E per 16-byte chunk
  constexpr int CPR = KS / CK;             // chunks per LDS row
  static_assert(KL == CK, "one 16-byte X fragment per lane, plane and column tile");
  static_assert((RT == 2) == std::is_same<Acc, float>::value, "output layout assumes f32 accumulators iff RT = 2");
  extern __shared__ __align__(16) unsigned char sk_lds[];
  E* const Bs = reinterpret_cast<E*>(sk_lds);

  // XCD-aware decode: the hardware dispatches block b to XCD b % 8; the tiles of a face share it
  const int tiles = mtiles * ntiles;
  const int b = blockIdx.x, nb = gridDim.x;
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
  const int m0 = mt * BM, n0 = nt * NP;
  if (LOWER && n0 > m0 + BM - 1) return;
  const int split = blockIdx.y;
  const int kbeg = split * kchunk;
  const int kend = min(K, kbeg + kchunk);
  const int nsteps = kbeg < kend ? (kend - kbeg + KS - 1) / KS : 0;
  const int klast = kbeg + (nsteps - 1) * KS;   // start of the last macro step with data
  // The k loop runs a multiple of three steps (one basic block per three, so the compiler keeps the
  // prefetches where they are issued).  Steps past kend see X = 0: packed X is zero-padded up to
  // a multiple of 3 KS (host side), raw X is zeroed while staging.
  const int nsteps3 = (nsteps + 2) / 3 * 3;
  const int kxlast = PACKED ? kbeg + (nsteps3 - 1) * KS : klast;

  A += (int64_t)f * sA;
  C += (int64_t)f * sC + (int64_t)split * sCsplit;

  const int tid = threadIdx.x, lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int g = lane >> 4, rho = lane & 15;
  const int mw = m0 + (wave % WR) * 16 * RT;  // first row of op(A) owned by this wave
  const int cw = (wave / WR) * 16 * NT;       // first block column owned by this wave
  const int wmax = mw + 16 * RT - 1;
  const int r0 = (RT == 2) ? mw + 2 * rho : mw + rho;  // row of tile 0 held by this lane

  // ---- A: straight into registers (k0 clamped to the last step: prefetches past the end are
  // harmless re-reads) ----
  // Fast-path lane offsets (32-bit, loop invariant) from uniform per-step bases, so every load is
  // an SGPR base + one VGPR offset.
  uint32_t aoff[RT];
#pragma unroll
  for (int tt = 0; tt < RT; ++tt)
    aoff[tt] = CN ? (uint32_t)((r0 + tt) * lda + KL * g) : (uint32_t)(r0 + KL * g * lda);
  auto load_a = [&](TA (&ra)[RT][KL], int k0) {
    k0 = min(k0, klast);
    if constexpr (!CN) {
      if constexpr (!SAFE) {
#pragma unroll
        for (int e = 0; e < KL; ++e) {
          const TA* base = A + (int64_t)(k0 + e) * lda;
          TA tmp[RT];
          vload<TA, RT>(base + aoff[0], tmp);
#pragma unroll
          for (int tt = 0; tt < RT; ++tt) ra[tt][e] = tmp[tt];
        }
      } else {
#pragma unroll
        for (int e = 0; e < KL; ++e) {
          const int kk = min(k0 + KL * g + e, K - 1);
#pragma unroll
          for (int tt = 0; tt < RT; ++tt) ra[tt][e] = A[min(r0 + tt, M - 1) + (int64_t)kk * lda];
        }
      }
    } else {
      if constexpr (!SAFE) {
        const TA* base = A + k0;
#pragma unroll
        for (int tt = 0; tt < RT; ++tt) vload<TA, KL>(base + aoff[tt], ra[tt]);
      } else {
#pragma unroll
        for (int tt = 0; tt < RT; ++tt) {
          const int64_t col = (int64_t)min(r0 + tt, M - 1) * lda;
#pragma unroll
          for (int e = 0; e < KL; ++e) ra[tt][e] = A[min(k0 + KL * g + e, K - 1) + col];
        }
      }
    }
  };

  // ---- X: global -> registers (two steps ahead) -> LDS (one step ahead) ----
  constexpr int NCH = PACKED ? (2 * NP * CPR + SK_THREADS - 1) / SK_THREADS : (NP * CPR + SK_THREADS - 1) / SK_THREADS;
  typedef typename std::conditional<PACKED, u32x4, TX>::type RB;
  constexpr int RBN = PACKED ? 1 : CK;
  uint32_t boff[NCH];   // global offset of this thread's chunk (k0 excluded)
  int bldsoff[NCH];     // LDS offset of this thread's chunk
  int bcol[NCH];        // raw X: block column of the chunk
#pragma unroll
  for (int q = 0; q < NCH; ++q) {
    if constexpr (PACKED) {
      const int c = min(tid + SK_THREADS * q, 2 * NP * CPR - 1);
      const int pl = c / (NP * CPR), rem = c % (NP * CPR);
      const int n = rem / CPR, ch = rem % CPR;
      boff[q] = (uint32_t)(pl * (sX / 2) + (int64_t)(n0 + n) * ldx + ch * CK);
      bldsoff[q] = pl * PLANE + n * ROWE + ch * CK;
      bcol[q] = n;
    } else {
      const int c = min(tid + SK_THREADS * q, NP * CPR - 1);
      const int n = c / CPR, ch = c % CPR;
      boff[q] = (uint32_t)((int64_t)min(n0 + n, N - 1) * ldx + ch * CK);
      bldsoff[q] = n * ROWE + ch * CK;
      bcol[q] = n;
    }
  }
  auto load_b = [&](RB (&rb)[NCH][RBN], int k0) {
    k0 = min(k0, kxlast);
    if constexpr (PACKED) {
      const E* base = reinterpret_cast<const E*>(Xv) + (int64_t)f * sX + k0;
#pragma unroll
      for (int q = 0; q < NCH; ++q) rb[q][0] = *reinterpret_cast<const u32x4*>(base + boff[q]);
    } else {
      const TX* X = reinterpret_cast<const TX*>(Xv) + (int64_t)f * sX;
#pragma unroll
      for (int q = 0; q < NCH; ++q) {
        if constexpr (!SAFE) {
          vload<TX, CK>(X + k0 + boff[q], rb[q]);
        } else {
          const int ch = (int)(bldsoff[q] % ROWE) / CK;
          const int64_t col = (int64_t)min(n0 + bcol[q], N - 1) * ldx;
#pragma unroll
          for (int e = 0; e < CK; ++e) rb[q][e] = X[min(k0 + ch * CK + e, K - 1) + col];
        }
      }
    }
  };
  auto store_b = [&](const RB (&rb)[NCH][RBN], E* Bd, int k0) {
#pragma unroll
    for (int q = 0; q < NCH; ++q) {
      if constexpr (PACKED) {
        *reinterpret_cast<u32x4*>(Bd + bldsoff[q]) = rb[q][0];
      } else {
        const int ch = (bldsoff[q] % ROWE) / CK;
        const bool colok = n0 + bcol[q] < N;
        E re[CK], im[CK];
#pragma unroll
        for (int e = 0; e < CK; ++e) {
          const bool ok = colok && (k0 + ch * CK + e < kend);
          const cplx<double> v = ld<double>(rb[q][e]);
          re[e] = cvt_e<E>(ok ? v.re : 0.0);
          im[e] = cvt_e<E>(ok ? v.im : 0.0);
        }
        vstore<E, CK>(Bd + bldsoff[q], re);
        vstore<E, CK>(Bd + PLANE + bldsoff[q], im);
      }
    }
  };

  V accr[RT][NT], acci[RT][NT];
#pragma unroll
  for (int tt = 0; tt < RT; ++tt)
#pragma unroll
    for (int c = 0; c < NT; ++c)
#pragma unroll
      for (int v = 0; v < 4; ++v) { accr[tt][c][v] = 0; acci[tt][c][v] = 0; }

  auto compute = [&](const TA (&ra)[RT][KL], const E* Bc) {
    if constexpr (std::is_same<P, B16>::value) {
      static_assert(std::is_same<TA, zb>::value, "bf16 products stream bf16 A-hat");
      bf16x8 far[RT], fai[RT], fan[RT];
#pragma unroll
      for (int tt = 0; tt < RT; ++tt) {
        u32x4 re, im;
#pragma unroll
        for (int w = 0; w < 4; ++w) {
          const uint32_t a = ra[tt][2 * w].bits, bb = ra[tt][2 * w + 1].bits;
          re[w] = (a & 0xffffu) | (bb << 16);
          im[w] = (a >> 16) | (bb & 0xffff0000u);
        }
        const u32x4 imn = im ^ (u32x4)(0x80008000u);
        far[tt] = __builtin_bit_cast(bf16x8, re);
        fai[tt] = __builtin_bit_cast(bf16x8, CN ? imn : im);
        fan[tt] = __builtin_bit_cast(bf16x8, CN ? im : imn);
      }
#pragma unroll
      for (int c = 0; c < NT; ++c) {
        if (LOWER && n0 + cw + 16 * c > wmax) continue;
        const E* bp = Bc + (cw + 16 * c + rho) * ROWE + KL * g;
        const bf16x8 br = *reinterpret_cast<const bf16x8*>(bp);
        const bf16x8 bi = *reinterpret_cast<const bf16x8*>(bp + PLANE);
#pragma unroll
        for (int tt = 0; tt < RT; ++tt) {
          accr[tt][c] = mma(far[tt], br, accr[tt][c]);
          acci[tt][c] = mma(far[tt], bi, acci[tt][c]);
        }
#pragma unroll
        for (int tt = 0; tt < RT; ++tt) {
          accr[tt][c] = mma(fan[tt], bi, accr[tt][c]);
          acci[tt][c] = mma(fai[tt], br, acci[tt][c]);
        }
      }
    } else {
      Acc xr[RT][KL], xi[RT][KL], xn[RT][KL];
#pragma unroll
      for (int tt = 0; tt < RT; ++tt)
#pragma unroll
        for (int e = 0; e < KL; ++e) {
          const cplx<Acc> v = ld<Acc>(ra[tt][e]);
          xr[tt][e] = v.re;
          xi[tt][e] = CN ? -v.im : v.im;
          xn[tt][e] = -xi[tt][e];
        }
#pragma unroll
      for (int c = 0; c < NT; ++c) {
        if (LOWER && n0 + cw + 16 * c > wmax) continue;
        const E* bp = Bc + (cw + 16 * c + rho) * ROWE + KL * g;
        E br[KL], bi[KL];
        vload<E, KL>(bp, br);
        vload<E, KL>(bp + PLANE, bi);
#pragma unroll
        for (int e = 0; e < KL; ++e) {
#pragma unroll
          for (int tt = 0; tt < RT; ++tt) {
            accr[tt][c] = mma(xr[tt][e], br[e], accr[tt][c]);
            acci[tt][c] = mma(xr[tt][e], bi[e], acci[tt][c]);
          }
#pragma unroll
          for (int tt = 0; tt < RT; ++tt) {
            accr[tt][c] = mma(xn[tt][e], bi[e], accr[tt][c]);
            acci[tt][c] = mma(xi[tt][e], br[e], acci[tt][c]);
          }
        }
      }
    }
  };

  // Pipeline (step j): issue the X loads of step j+3 and the A loads of step j+2, run the MFMAs of
  // step j, write the X registers of step j+1 (loaded two steps earlier) to its LDS buffer,
  // barrier.  Rings of three register sets and three LDS buffers; the loop body holds three steps
  // so the rings need no register copies.
  if (nsteps > 0) {
    E* const B0 = Bs;
    E* const B1 = Bs + BUF;
    E* const B2 = Bs + 2 * BUF;
    TA ra0[RT][KL], ra1[RT][KL], ra2[RT][KL];
    RB rb0[NCH][RBN], rb1[NCH][RBN], rb2[NCH][RBN];
    load_b(rb0, kbeg);
    load_a(ra0, kbeg);
    load_b(rb1, kbeg + KS);
    load_a(ra1, kbeg + KS);
    load_b(rb2, kbeg + 2 * KS);
    store_b(rb0, B0, kbeg);
    __syncthreads();
    int k0 = kbeg;
    auto step = [&](const TA (&cur)[RT][KL], TA (&pre)[RT][KL], RB (&rbload)[NCH][RBN], const RB (&rbstore)[NCH][RBN],
                    const E* Bcur, E* Bnext) {
      load_b(rbload, k0 + 3 * KS);
      load_a(pre, k0 + 2 * KS);
      compute(cur, Bcur);
      store_b(rbstore, Bnext, k0 + KS);
      __syncthreads();
      __builtin_amdgcn_sched_barrier(0);  // keep each step's MFMAs between its own barriers
      k0 += KS;
    };
    for (int j = 0; j < nsteps3; j += 3) {
      step(ra0, ra2, rb0, rb1, B0, B1);
      step(ra1, ra0, rb1, rb2, B1, B2);
      step(ra2, ra1, rb2, rb0, B2, B0);
    }
  }

  // ---- store ----
#pragma unroll
  for (int c = 0; c < NT; ++c) {
    if (LOWER && n0 + cw + 16 * c > wmax) continue;
    const int col = n0 + cw + 16 * c + rho;
    if (col >= N) continue;
    TC* cp = C + (int64_t)col * ldc;
    if constexpr (RT == 2) {
      const int rb = mw + 8 * g;   // rows rb .. rb+7: element v of tile tt is row rb + 2 v + tt
      TC vals[8];
#pragma unroll
      for (int v = 0; v < 4; ++v)
#pragma unroll
        for (int tt = 0; tt < 2; ++tt) st(vals[2 * v + tt], mk((double)accr[tt][c][v], (double)acci[tt][c][v]));
      if (vec_c && rb + 8 <= M) {
        vstore<TC, 8>(cp + rb, vals);
      } else {
#pragma unroll
        for (int j = 0; j < 8; ++j)
          if (rb + j < M) cp[rb + j] = vals[j];
      }
    } else {
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int row = mw + g + 4 * v;
        if (row < M) st(cp[row], mk((double)accr[0][c][v], (double)acci[0][c][v]));
      }
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
// host side
// ---------------------------------------------------------------------------------------------
static inline bool aligned_elems(const void* p, int64_t a, int64_t b, int64_t c, int64_t elem_bytes, int64_t vec_bytes) {
  if (vec_bytes <= elem_bytes) return ((uintptr_t)p % (uintptr_t)std::min<int64_t>(elem_bytes, 16)) == 0;
  const int64_t q = vec_bytes / elem_bytes;  // offsets must be multiples of q elements
  return ((uintptr_t)p % (uintptr_t)vec_bytes) == 0 && a % q == 0 && b % q == 0 && c % q == 0;
}

// column tiles of 16 per block
template <class P> static inline int nt_for(int N) { return N <= 16 ? 1 : (N <= 32 ? 2 : (N <= 64 ? 4 : 8)); }

template <class P, bool CN, bool PACKED, bool SAFE, bool LOWER, typename TA, typename TX, typename TC, int NT>
static int sk_launch_nt(int M, int N, int K, const TA* A, int64_t lda, int64_t sA, const void* X, int64_t ldx,
                        int64_t sX, TC* C, int64_t ldc, int64_t sC, int batch, int ksplit, int64_t sCsplit,
                        hipStream_t s) {
  constexpr int BM = Shape<NT>::WR * 16 * P::RT, NP = 16 * NT, KS = 4 * P::KL;
  const int mtiles = (int)ceil_div(M, BM), ntiles = (int)ceil_div(N, NP);
  const int tiles = mtiles * ntiles;
  int64_t nblk = (int64_t)batch * tiles;
  if (batch >= 8) nblk = ceil_div(batch, 8) * 8 * (int64_t)tiles;
  const int kchunk = (int)(ceil_div(ceil_div(K, ksplit), KS) * KS);
  const int bytes = lds_bytes<P>(NT);
  static int attr_done[64] = {0};
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return -1;
  auto kern = k_skinny<P, CN, PACKED, SAFE, LOWER, TA, TX, TC, NT>;
  if (bytes > 65536 && dev >= 0 && dev < 64 && !attr_done[dev]) {
    if (hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize, bytes) != hipSuccess) return -1;
    attr_done[dev] = 1;
  }
  const bool vec_c = aligned_elems(C, ldc, sC, sCsplit, sizeof(TC), 16);
  hipLaunchKernelGGL(kern, dim3((unsigned)nblk, (unsigned)ksplit), dim3(SK_THREADS), bytes, s, M, N, K, A, lda, sA, X, ldx,
                     sX, C, ldc, sC, batch, mtiles, ntiles, kchunk, sCsplit, (int)vec_c);
  return hipGetLastError() == hipSuccess ? 0 : -1;
}

// picks the column-tile count by N and the unchecked (vector) path when shapes and alignment allow
template <class P, bool CN, bool PACKED, bool LOWER, typename TA, typename TX, typename TC>
static int sk_launch(int M, int N, int K, const TA* A, int64_t lda, int64_t sA, const void* X, int64_t ldx, int64_t sX,
                     TC* C, int64_t ldc, int64_t sC, int batch, int ksplit, int64_t sCsplit, hipStream_t s) {
  constexpr int KS = 4 * P::KL;
  constexpr int CK = 16 / (int)sizeof(typename P::E);
  // NN loads RT neighbouring rows per k, CN loads KL consecutive k (in 16-byte pieces)
  const int64_t abytes = CN ? std::min<int64_t>((int64_t)sizeof(TA) * P::KL, 16) : (int64_t)sizeof(TA) * P::RT;
  const bool vec_a = aligned_elems(A, lda, sA, 0, sizeof(TA), abytes);
  const bool vec_x = PACKED || aligned_elems(X, ldx, sX, 0, sizeof(TX), std::min<int64_t>((int64_t)sizeof(TX) * CK, 16));
  // fast path lane offsets are 32-bit: CN spans M columns of A, raw X spans N columns
  const bool small_off = (CN ? (int64_t)M * lda : (int64_t)M + 4 * P::KL * lda) < (1LL << 31) &&
                         (PACKED || (int64_t)N * ldx < (1LL << 31));
  const int nt = nt_for<P>(N);
  const int BM = (nt == 1 ? Shape<1>::WR : nt == 2 ? Shape<2>::WR : nt == 4 ? Shape<4>::WR : Shape<8>::WR) * 16 * P::RT;
  const bool fast = vec_a && vec_x && small_off && M % BM == 0 && K % KS == 0;
#define RT_SK_NT(NTV)                                                                                          \
  (fast ? sk_launch_nt<P, CN, PACKED, false, LOWER, TA, TX, TC, NTV>(M, N, K, A, lda, sA, X, ldx, sX, C, ldc, sC, \
                                                                    batch, ksplit, sCsplit, s)                 \
        : sk_launch_nt<P, CN, PACKED, true, LOWER, TA, TX, TC, NTV>(M, N, K, A, lda, sA, X, ldx, sX, C, ldc, sC,  \
                                                                   batch, ksplit, sCsplit, s))
  if (nt == 1) return RT_SK_NT(1);
  if (nt == 2) return RT_SK_NT(2);
  if (nt == 4) return RT_SK_NT(4);
  return RT_SK_NT(8);
#undef RT_SK_NT
}

// MFMA precision for a streamed operand type: bf16 A-hat -> B16, FP32 -> F32, FP64 -> F64
template <typename TA> struct PrecOf;
template <> struct PrecOf<zb> { typedef B16 P; };
template <> struct PrecOf<zf> { typedef F32 P; };
template <> struct PrecOf<zd> { typedef F64 P; };

// bytes of packed X planes for a product with contraction length K and N columns
// packed X rows are zero-padded to a multiple of three macro steps (the k loop runs in threes)
template <class P> static inline int packed_kp(int K) { return (int)(ceil_div(K, 12 * P::KL) * 12 * P::KL); }
template <class P> static inline int64_t packed_elems(int K, int N, int batch) {
  const int NP = 16 * nt_for<P>(N);
  const int64_t KP = packed_kp<P>(K);
  const int64_t NPt = ceil_div(N, NP) * NP;
  return 2 * NPt * KP * batch;
}
template <typename TA> static inline int64_t skinny_ws_bytes(int K, int N, int batch) {
  typedef typename PrecOf<TA>::P P;
  return packed_elems<P>(K, N, batch) * (int64_t)sizeof(typename P::E);
}

// C_f = op(A_f) X_f with X packed into `ws` (skinny_ws_bytes<TA>(K, N, batch) bytes) first.
template <typename TA, typename TX, typename TC>
static int skinny_cgemm(bool conjA, int M, int N, int K, const TA* A, int64_t lda, int64_t sA, const TX* X,
                        int64_t ldx, int64_t sX, TC* C, int64_t ldc, int64_t sC, int batch, void* ws, hipStream_t s) {
  typedef typename PrecOf<TA>::P P;
  typedef typename P::E E;
  if (M <= 0 || N <= 0 || batch <= 0) return 0;
  if (K <= 0) return -1;
  const int NP = 16 * nt_for<P>(N);
  const int KP = packed_kp<P>(K);
  const int NPt = (int)(ceil_div(N, NP) * NP);
  E* Xp = static_cast<E*>(ws);
  const int64_t total = (int64_t)NPt * KP * batch;
  hipLaunchKernelGGL((k_pack_planes<TX, E>), dim3((unsigned)ceil_div(total, 256)), dim3(256), 0, s, X, ldx, sX, K, N,
                     Xp, KP, NPt, batch);
  if (hipGetLastError() != hipSuccess) return -1;
  const int64_t sXp = 2 * (int64_t)NPt * KP;
  // packed X: the raw type parameter is unused, fixed to zd to share instantiations
  if (!conjA) return sk_launch<P, false, true, false, TA, zd, TC>(M, N, K, A, lda, sA, Xp, KP, sXp, C, ldc, sC, batch, 1, 0, s);
  return sk_launch<P, true, true, false, TA, zd, TC>(M, N, K, A, lda, sA, Xp, KP, sXp, C, ldc, sC, batch, 1, 0, s);
}

// FP64 Gram G_f = Y_f^H Y_f (r x r) of Y_f (rows x r, any complex storage type): split-K partials
// (batch x ksplit x r x r) in `part`, lower tiles only, then a deterministic reduction.
template <typename TY>
static int gram_fp64(const TY* Y, int64_t rows, int r, int64_t sY, int batch, zd* part, int ksplit, zd* G,
                     hipStream_t s) {
  const int64_t sPart = (int64_t)r * r;
  int rc = sk_launch<F64, true, false, true, TY, TY, zd>(r, r, (int)rows, Y, rows, sY, Y, rows, sY, part, r,
                                                         (int64_t)ksplit * sPart, batch, ksplit, sPart, s);
  if (rc) return rc;
  hipLaunchKernelGGL(k_gram_reduce, dim3((unsigned)ceil_div((int64_t)r * r, 256), (unsigned)batch), dim3(256), 0, s,
                     part, r, ksplit, sPart, G);
  return hipGetLastError() == hipSuccess ? 0 : -1;
}

}  // namespace sk
}  // namespace rt
