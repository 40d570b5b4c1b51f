// Skinny batched complex products on MFMA (gfx950):  C_f = op(A_f) X_f,  op = identity (NN) or
// conjugate transpose (CN), f = Fourier face, X_f with few columns (the sketch width r).  These are
// the passes over A-hat of the randomized factorization (sketch, power iteration, projection,
// W = A-hat V), the FP64 Gram matrices of CholeskyQR and the right-multiplications Y R^{-1}.
//
// Design (block = 8 waves = WR row groups x WC column groups over a BM x NP tile of C):
//  * Both operands move through LDS one k-group (4 KL values of k) at a time.  All 512 threads
//    load the next k-groups cooperatively with 16-byte loads (A rows or columns contiguous, X in
//    slab-major packed order), keeping SK_DEPTH k-groups in flight in a ring of register sets,
//    so the memory latency is covered without per-wave duplicate loads; the oldest set goes to
//    one of two LDS buffers each step (one barrier per k-group).
//  * A keeps its global layout in LDS; a lane reads the RT rows (NN) or the KL consecutive k (CN)
//    of its MFMA operand directly, so no transposition is needed.  The MFMA k slot is a
//    relabelling of k (lane group g = lane/16 holds k = KL*g + e), applied identically to X.
//  * With RT = 2 the two row tiles of a wave interleave (row 2*rho + t), so a lane's outputs are
//    8 consecutive rows of one column and are written with 16-byte stores.
//  * Complex arithmetic on split planes (conjugation of A folded into Ai):
//      bf16: four real MFMA products,  Re C += Ar Xr + (-Ai) Xi,  Im C += Ar Xi + Ai Xr;
//      FP32 and FP64: three (Gauss), P1 += Ar Xr, P2 += Ai Xi, P3 += (Ar + Ai)(Xr + Xi), and at the
//      end Re C = P1 - P2, Im C = (P3 - P1) - P2 -- a quarter fewer MFMAs for the MFMA-bound
//      products; the operand sums are formed in registers (in bf16 they would not be exact).
//  * The blocks of one face run on one XCD (block id congruent mod 8), sharing X in that L2.
// MFMA output layouts (16 x 16 tile, element v < 4 of lane l, column l % 16): f32 accumulators
// row 4*(l/16) + v; f64 accumulators row (l/16) + 4*v.
#pragma once
#include "common.hpp"
#include <algorithm>
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
constexpr int SK_DEPTH = 3;      // k-groups in flight in registers beyond the one being stored
constexpr int SK_RING = SK_DEPTH + 1;

// Block shape for NB column tiles of 16: WC column groups of NTW tiles, WR = 8 / WC row groups.
// Four column groups (two row groups of waves) measured fastest for the 64- and 128-column products.
template <int NB> struct Shape {
#ifdef SKINNY_WC
  static constexpr int WC = NB >= SKINNY_WC ? SKINNY_WC : NB;
#else
  static constexpr int WC = NB >= 4 ? 4 : NB;
#endif
  static constexpr int NTW = NB / WC, WR = 8 / WC;
};

// k per MFMA k-group (4 lane groups x KL); packed X is padded to whole rings of k-groups
template <class P> constexpr int kgroup() { return 4 * P::KL; }
template <class P> constexpr int kslab() { return kgroup<P>(); }

// LDS: two buffers, each an A tile (rows or columns padded by 16 bytes) and an X tile (2 planes)
template <class P, bool CN, typename TA> constexpr int a_stride_bytes(int BM) {
  return CN ? kgroup<P>() * (int)sizeof(TA) + 16 : BM * (int)sizeof(TA) + 16;
}
template <class P, bool CN, typename TA> constexpr int a_tile_bytes(int BM) {
  return (CN ? BM : kgroup<P>()) * a_stride_bytes<P, CN, TA>(BM);
}
template <class P> constexpr int x_tile_bytes(int NB) {
  return 2 * 16 * NB * (kgroup<P>() + P::PADE) * (int)sizeof(typename P::E);
}
template <class P, bool CN, typename TA> constexpr int lds_bytes(int NB, int BM) {
  return 2 * (a_tile_bytes<P, CN, TA>(BM) + x_tile_bytes<P>(NB));
}

// Packed X in slab-major order, so that one slab of one block column is a single contiguous run:
//   Xp[f][block column nt][slab s][plane][n < NP][kl < KSL],  k = s KSL + kl,  n = nt NP + n,
// plane 0 real, 1 imaginary, zero outside K x N.  X_f is column-major K x N (leading dimension ldx).
// One thread per PV = 16 / sizeof(E) consecutive kl of one column: one 16-byte store per plane
// (Xp 16-byte aligned; KSL is a multiple of PV).
template <typename E> constexpr int pack_vec() { return 16 / (int)sizeof(E); }
// Grid: x over one face's slab chunks (32-bit index, decoded without 64-bit divisions), y = face.
// vec: the host has checked that X, ldx and sX allow loads of PV consecutive elements at once.
template <typename TX, typename E, int KSL>
__global__ void k_pack_slabs(const TX* __restrict__ X, int64_t ldx, int64_t sX, int K, int N, E* __restrict__ Xp,
                             int KP, int NP, int ntiles, int vec) {
  constexpr int PV = pack_vec<E>(), KV = KSL / PV;
  static_assert(KSL % PV == 0, "a slab row holds whole 16-byte vectors");
  const int idx = (int)(blockIdx.x * blockDim.x + threadIdx.x);
  const int nsl = KP / KSL;
  if (idx >= ntiles * nsl * NP * KV) return;
  const int64_t f = blockIdx.y;
  const int kv = idx % KV;
  int t1 = idx / KV;
  const int nl = t1 % NP;
  t1 /= NP;
  const int sl = t1 % nsl;
  const int nt = t1 / nsl;
  const int k0 = sl * KSL + kv * PV, n = nt * NP + nl;
  E re[PV], im[PV];
  const TX* src = X + f * sX + k0 + (int64_t)n * ldx;
  if (vec && n < N && k0 + PV <= K) {
    TX v[PV];
    vload<TX, PV>(src, v);
#pragma unroll
    for (int e = 0; e < PV; ++e) {
      const cplx<double> z = ld<double>(v[e]);
      re[e] = cvt_e<E>(z.re);
      im[e] = cvt_e<E>(z.im);
    }
  } else {
#pragma unroll
    for (int e = 0; e < PV; ++e) {
      double vr = 0.0, vi = 0.0;
      if (n < N && k0 + e < K) {
        const cplx<double> v = ld<double>(src[e]);
        vr = v.re; vi = v.im;
      }
      re[e] = cvt_e<E>(vr);
      im[e] = cvt_e<E>(vi);
    }
  }
  E* out = Xp + (((f * ntiles + nt) * nsl + sl) * 2 * NP + nl) * KSL + kv * PV;
  vstore<E, PV>(out, re);
  vstore<E, PV>(out + (int64_t)NP * KSL, im);
}

// C_f (+ split * sCsplit) = op(A_f) X_f, M x N, contraction length K.
// PACKED: X is E* packed k-group-major ([f][nt][k-group][plane][NP][KG]) with face stride sX and
// ldx = its padded K; otherwise X is TX* column-major (raw, converted while staging).
// SAFE = false: the host guarantees M % BM == 0, K % KG == 0 and the alignment of the 16-byte
// loads of A (and of raw X); SAFE = true clamps every A and X index instead (element loads).
// Both paths are branch-free inside the k loop.  LOWER: skip column tiles strictly above the
// diagonal (Hermitian Gram).  vec_c: the host has checked the alignment of 16-byte stores.
// k-groups past kend see X = 0 (packed X is zero-padded, raw X is zeroed while staging).
// waves per SIMD the register allocation must allow: four (two workgroups per CU, so one
// workgroup's MFMAs run while the other waits at its k-group barrier) for the unchecked FP32
// products, two for the others
// Optional second output of an FP32 product: C as the packed bf16 X operand of a following bf16
// pass over A-hat (slab-major, the layout k_pack_slabs writes with 32 k per slab: k = row of C,
// n = column of C, block columns of NP = 16 NB), so that pass needs no packing kernel.  p == null:
// none.  sf: elements per face; nsl: slabs per block column (rows of C / 32, rows a multiple of 128
// so there are no padding rows).  Columns past N are written too: their values are zero.
struct PackOut {
  uint16_t* p = nullptr;
  int64_t sf = 0;
  int nsl = 0;
};

template <class P, bool SAFE> constexpr int sk_min_waves() { return (std::is_same<P, F32>::value && !SAFE) ? 4 : 2; }

template <class P, bool CN, bool PACKED, bool SAFE, bool LOWER, bool UTRI, typename TA, typename TX, typename TC, int NB>
__global__ void __launch_bounds__(SK_THREADS, (sk_min_waves<P, SAFE>()))
k_skinny(int M, int N, int K, const TA* __restrict__ A, int64_t lda, int64_t sA, const void* __restrict__ Xv,
         int64_t ldx, int64_t sX, TC* __restrict__ C, int64_t ldc, int64_t sC, int batch, int mtiles, int ntiles,
         int kchunk, int64_t sCsplit, int vec_c, PackOut cpk) {
  typedef typename P::E E;
  typedef typename P::V V;
  typedef typename P::Acc Acc;
  constexpr int KL = P::KL, RT = P::RT, KG = kgroup<P>(), ROWE = KG + P::PADE;
  constexpr int NP = 16 * NB;  // block columns
  constexpr int NT = Shape<NB>::NTW, WR = Shape<NB>::WR;
  constexpr int BM = WR * 16 * RT;
  constexpr int ASTR = a_stride_bytes<P, CN, TA>(BM);       // bytes between A rows (NN: k rows)
  constexpr int ATILE = a_tile_bytes<P, CN, TA>(BM);
  constexpr int XPLANE = NP * ROWE;                         // E per X plane
  constexpr int BUFB = ATILE + x_tile_bytes<P>(NB);         // bytes per LDS buffer
  constexpr int CK = 16 / (int)sizeof(E);                   // E per 16-byte X chunk
  constexpr int XCPR = KG / CK;                             // X chunks per LDS row
  constexpr int TAC = 16 / (int)sizeof(TA) > 0 ? 16 / (int)sizeof(TA) : 1;  // TA per 16-byte A chunk
  constexpr int ACH_PER_LINE = CN ? KG / TAC : BM / TAC;     // A chunks per column (CN) / k row (NN)
  constexpr int ACH = (CN ? BM : KG) * ACH_PER_LINE;         // A chunks per k-group
  constexpr int NAC = (ACH + SK_THREADS - 1) / SK_THREADS;   // A chunks per thread
  static_assert(KL == CK, "one 16-byte X fragment per lane, plane and column tile");
  static_assert((RT == 2) == std::is_same<Acc, float>::value, "output layout assumes f32 accumulators iff RT = 2");
  static_assert(sizeof(TA) <= 16 && 16 % sizeof(TA) == 0, "A element size");
  extern __shared__ __align__(16) unsigned char sk_lds[];

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
  const int nkg = kbeg < kend ? (kend - kbeg + KG - 1) / KG : 0;   // k-groups with data
  const int nkgr = (nkg + SK_RING - 1) / SK_RING * SK_RING;       // run in whole rings
  const int kglast = kbeg + (nkg - 1) * KG;                       // last k-group with data
  const int kxlast = PACKED ? kbeg + (nkgr - 1) * KG : kglast;    // packed X is padded to whole rings

  A += (int64_t)f * sA;
  C += (int64_t)f * sC + (int64_t)split * sCsplit;

  const int tid = threadIdx.x, lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int g = lane >> 4, rho = lane & 15;
  const int rw = (wave % WR) * 16 * RT;       // first tile row of this wave (within the block)
  const int mw = m0 + rw;
  const int cw = (wave / WR) * 16 * NT;       // first block column of this wave
  const int wmax = mw + 16 * RT - 1;

  // ---- cooperative staging: per k-group, A chunks then X chunks of 16 bytes ----
  typedef typename std::conditional<PACKED, u32x4, TX>::type XR;
  constexpr int XRN = PACKED ? 1 : CK;
  constexpr int NXC = PACKED ? (2 * NP * XCPR + SK_THREADS - 1) / SK_THREADS : (NP * XCPR + SK_THREADS - 1) / SK_THREADS;
  struct Stage { u32x4 a[NAC]; TA ae[NAC][TAC]; XR x[NXC][XRN]; };
  // chunk coordinates (loop invariant)
  int a_line[NAC], a_seg[NAC];
  uint32_t a_goff[NAC];
  int a_loff[NAC];
#pragma unroll
  for (int q = 0; q < NAC; ++q) {
    const int c = min(tid + SK_THREADS * q, ACH - 1);
    a_line[q] = c / ACH_PER_LINE;   // NN: k within the group; CN: column within the tile
    a_seg[q] = c % ACH_PER_LINE;
    // full offset of the chunk; the triangular-X products clamp the k row instead (below)
    a_goff[q] = CN ? (uint32_t)((int64_t)(m0 + a_line[q]) * lda + a_seg[q] * TAC)
                   : (uint32_t)((UTRI ? 0 : (int64_t)a_line[q] * lda) + m0 + a_seg[q] * TAC);
    a_loff[q] = a_line[q] * ASTR + a_seg[q] * 16;
  }
  int x_loff[NXC], x_col[NXC], x_k[NXC];
  uint32_t x_goff[NXC];
#pragma unroll
  for (int q = 0; q < NXC; ++q) {
    if constexpr (PACKED) {
      const int c = min(tid + SK_THREADS * q, 2 * NP * XCPR - 1);
      const int pl = c / (NP * XCPR), rem = c % (NP * XCPR);
      const int n = rem / XCPR, ch = rem % XCPR;
      x_goff[q] = (uint32_t)(c * CK);
      x_loff[q] = pl * XPLANE + n * ROWE + ch * CK;
      x_col[q] = n;
      x_k[q] = ch * CK;
    } else {
      const int c = min(tid + SK_THREADS * q, NP * XCPR - 1);
      const int n = c / XCPR, ch = c % XCPR;
      x_goff[q] = (uint32_t)((int64_t)min(n0 + n, N - 1) * ldx);
      x_loff[q] = n * ROWE + ch * CK;
      x_col[q] = n;
      x_k[q] = ch * CK;
    }
  }
  auto load_stage = [&](Stage& st, int k0) {
    // A (k-group start clamped to the last one with data: prefetches past the end are re-reads)
    const int ka = min(k0, kglast);
#pragma unroll
    for (int q = 0; q < NAC; ++q) {
      if constexpr (!SAFE) {
        if constexpr (CN) {
          st.a[q] = *reinterpret_cast<const u32x4*>(A + (int64_t)ka + a_goff[q]);
        } else if constexpr (UTRI) {
          // K need not be a multiple of the k-group here (K = r): k rows past K re-read row K - 1,
          // finite values that meet the zero padding of the packed X
          const uint32_t line = (uint32_t)min(a_line[q], K - 1 - ka);
          st.a[q] = *reinterpret_cast<const u32x4*>(A + (int64_t)ka * lda + (line * (uint32_t)lda + a_goff[q]));
        } else {
          st.a[q] = *reinterpret_cast<const u32x4*>(A + (int64_t)ka * lda + a_goff[q]);
        }
      } else {
#pragma unroll
        for (int e = 0; e < TAC; ++e) {
          int row, kk;
          if constexpr (CN) { row = m0 + a_line[q]; kk = ka + a_seg[q] * TAC + e; }
          else { row = m0 + a_seg[q] * TAC + e; kk = ka + a_line[q]; }
          st.ae[q][e] = A[min(row, M - 1) * (CN ? lda : (int64_t)1) + (int64_t)min(kk, K - 1) * (CN ? (int64_t)1 : lda)];
        }
      }
    }
    // X
    if constexpr (PACKED) {
      const int kx = min(k0, kxlast);
      const int64_t ngr = ldx / KG;
      const E* base = reinterpret_cast<const E*>(Xv) + (int64_t)f * sX + ((int64_t)nt * ngr + kx / KG) * (2 * NP * KG);
#pragma unroll
      for (int q = 0; q < NXC; ++q) st.x[q][0] = *reinterpret_cast<const u32x4*>(base + x_goff[q]);
    } else {
      const TX* X = reinterpret_cast<const TX*>(Xv) + (int64_t)f * sX;
#pragma unroll
      for (int q = 0; q < NXC; ++q) {
        if constexpr (!SAFE) {
          const int kk = min(k0 + x_k[q], K - CK);   // in bounds; k >= kend is zeroed at the store
          vload<TX, CK>(X + kk + x_goff[q], st.x[q]);
        } else {
#pragma unroll
          for (int e = 0; e < CK; ++e) st.x[q][e] = X[min(k0 + x_k[q] + e, K - 1) + (int64_t)x_goff[q]];
        }
      }
    }
  };
  auto store_stage = [&](const Stage& st, unsigned char* buf, int k0) {
    unsigned char* abuf = buf;
    E* xbuf = reinterpret_cast<E*>(buf + ATILE);
#pragma unroll
    for (int q = 0; q < NAC; ++q) {
      if (ACH % SK_THREADS == 0 || tid + SK_THREADS * q < ACH) {
        if constexpr (!SAFE) {
          *reinterpret_cast<u32x4*>(abuf + a_loff[q]) = st.a[q];
        } else {
          u32x4 v;
          __builtin_memcpy(&v, &st.ae[q][0], 16);
          *reinterpret_cast<u32x4*>(abuf + a_loff[q]) = v;
        }
      }
    }
#pragma unroll
    for (int q = 0; q < NXC; ++q) {
      if constexpr (PACKED) {
        *reinterpret_cast<u32x4*>(xbuf + x_loff[q]) = st.x[q][0];
      } else {
        const bool colok = n0 + x_col[q] < N;
        E re[CK], im[CK];
#pragma unroll
        for (int e = 0; e < CK; ++e) {
          const bool ok = colok && (k0 + x_k[q] + e < kend);
          const cplx<double> v = ld<double>(st.x[q][e]);
          re[e] = cvt_e<E>(ok ? v.re : 0.0);
          im[e] = cvt_e<E>(ok ? v.im : 0.0);
        }
        vstore<E, CK>(xbuf + x_loff[q], re);
        vstore<E, CK>(xbuf + XPLANE + x_loff[q], im);
      }
    }
  };

  // bf16: accr, acci are Re C, Im C.  FP32 / FP64: accr, acci, accs hold P1, P2, P3 (combined
  // into Re C, Im C before the store)
  constexpr bool GAUSS = !std::is_same<P, B16>::value;
  V accr[RT][NT], acci[RT][NT], accs[RT][NT];
#pragma unroll
  for (int tt = 0; tt < RT; ++tt)
#pragma unroll
    for (int c = 0; c < NT; ++c)
#pragma unroll
      for (int v = 0; v < 4; ++v) { accr[tt][c][v] = 0; acci[tt][c][v] = 0; accs[tt][c][v] = 0; }

  // one k-group from an LDS buffer
  // UTRI: X is upper triangular (X[k][n] = 0 for k > n), so column tile c skips k-groups that
  // start below its last column (NN only)
  auto skip = [&](int kc, int c) { return UTRI && kc > n0 + cw + 16 * c + 15; };
  auto compute = [&](const unsigned char* buf, int kc) {
    const unsigned char* abuf = buf;
    const E* Bc = reinterpret_cast<const E*>(buf + ATILE);
    // A fragments of this lane: ra[tt][e] = op(A) row (rw + 2 rho + tt or rw + rho), k = KL g + e
    TA ra[RT][KL];
    if constexpr (!CN) {
#pragma unroll
      for (int e = 0; e < KL; ++e) {
        TA tmp[RT];
        vload<TA, RT>(reinterpret_cast<const TA*>(abuf + (KL * g + e) * ASTR) + (RT == 2 ? rw + 2 * rho : rw + rho), tmp);
#pragma unroll
        for (int tt = 0; tt < RT; ++tt) ra[tt][e] = tmp[tt];
      }
    } else {
#pragma unroll
      for (int tt = 0; tt < RT; ++tt)
        vload<TA, KL>(reinterpret_cast<const TA*>(abuf + (RT == 2 ? rw + 2 * rho + tt : rw + rho) * ASTR) + KL * g, ra[tt]);
    }
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
      bf16x8 br[NT], bi[NT];
#pragma unroll
      for (int c = 0; c < NT; ++c) {
        const E* bp = Bc + (cw + 16 * c + rho) * ROWE + KL * g;
        br[c] = *reinterpret_cast<const bf16x8*>(bp);
        bi[c] = *reinterpret_cast<const bf16x8*>(bp + XPLANE);
      }
#pragma unroll
      for (int c = 0; c < NT; ++c) {
        if ((LOWER && n0 + cw + 16 * c > wmax) || skip(kc, c)) continue;
#pragma unroll
        for (int tt = 0; tt < RT; ++tt) {
          accr[tt][c] = mma(far[tt], br[c], accr[tt][c]);
          acci[tt][c] = mma(far[tt], bi[c], acci[tt][c]);
        }
      }
#pragma unroll
      for (int c = 0; c < NT; ++c) {
        if ((LOWER && n0 + cw + 16 * c > wmax) || skip(kc, c)) continue;
#pragma unroll
        for (int tt = 0; tt < RT; ++tt) {
          accr[tt][c] = mma(fan[tt], bi[c], accr[tt][c]);
          acci[tt][c] = mma(fai[tt], br[c], acci[tt][c]);
        }
      }
    } else {
      // three real products: P1 = Ar Xr, P2 = Ai Xi, P3 = (Ar + Ai)(Xr + Xi)
      Acc xr[RT][KL], xi[RT][KL], xs[RT][KL];
#pragma unroll
      for (int tt = 0; tt < RT; ++tt)
#pragma unroll
        for (int e = 0; e < KL; ++e) {
          const cplx<Acc> v = ld<Acc>(ra[tt][e]);
          xr[tt][e] = v.re;
          xi[tt][e] = CN ? -v.im : v.im;
          xs[tt][e] = xr[tt][e] + xi[tt][e];
        }
      E br[NT][KL], bi[NT][KL], bs[NT][KL];
#pragma unroll
      for (int c = 0; c < NT; ++c) {
        const E* bp = Bc + (cw + 16 * c + rho) * ROWE + KL * g;
        vload<E, KL>(bp, br[c]);
        vload<E, KL>(bp + XPLANE, bi[c]);
#pragma unroll
        for (int e = 0; e < KL; ++e) bs[c][e] = br[c][e] + bi[c][e];
      }
#pragma unroll
      for (int e = 0; e < KL; ++e) {
#pragma unroll
        for (int c = 0; c < NT; ++c) {
          if ((LOWER && n0 + cw + 16 * c > wmax) || skip(kc, c)) continue;
#pragma unroll
          for (int tt = 0; tt < RT; ++tt) {
            accr[tt][c] = mma(xr[tt][e], br[c][e], accr[tt][c]);
            acci[tt][c] = mma(xi[tt][e], bi[c][e], acci[tt][c]);
            accs[tt][c] = mma(xs[tt][e], bs[c][e], accs[tt][c]);
          }
        }
      }
    }
  };

  // Pipeline (step j): issue the loads of k-group j + SK_DEPTH into ring set (j + DEPTH) % RING,
  // compute k-group j from LDS buffer j % 2, store set (j + 1) % RING into buffer (j + 1) % 2,
  // barrier.  The loop body holds SK_RING = 4 steps (ring and buffer parities repeat), with no
  // branches, so the prefetches stay where they are issued.
  static_assert(SK_RING == 4, "the unrolled loop below assumes a ring of four stages");
  if (nkg > 0) {
    unsigned char* const buf0 = sk_lds;
    unsigned char* const buf1 = sk_lds + BUFB;
    Stage s0, s1, s2, s3;
    load_stage(s0, kbeg);
    load_stage(s1, kbeg + KG);
    load_stage(s2, kbeg + 2 * KG);
    store_stage(s0, buf0, kbeg);
    __syncthreads();
    // sched_barrier: keep the loads issued before the MFMAs of the step (the scheduler would
    // otherwise sink them past the LDS stores, whose waits then cover every load in flight)
#define RT_SK_STEP(LOADSET, KLOAD, BUFC, STORESET, BUFN, KSTORE) \
    load_stage(LOADSET, KLOAD);                                  \
    __builtin_amdgcn_sched_barrier(0);                           \
    compute(BUFC, (KLOAD) - SK_DEPTH * KG);                      \
    __builtin_amdgcn_sched_barrier(0);                           \
    store_stage(STORESET, BUFN, KSTORE);                         \
    __syncthreads();                                             \
    __builtin_amdgcn_sched_barrier(0);
    for (int j = 0; j < nkgr; j += SK_RING) {
      const int k0 = kbeg + j * KG;
      RT_SK_STEP(s3, k0 + 3 * KG, buf0, s1, buf1, k0 + KG)
      RT_SK_STEP(s0, k0 + 4 * KG, buf1, s2, buf0, k0 + 2 * KG)
      RT_SK_STEP(s1, k0 + 5 * KG, buf0, s3, buf1, k0 + 3 * KG)
      RT_SK_STEP(s2, k0 + 6 * KG, buf1, s0, buf0, k0 + 4 * KG)
    }
#undef RT_SK_STEP
  }

  // ---- store ----
  if constexpr (GAUSS) {
#pragma unroll
    for (int tt = 0; tt < RT; ++tt)
#pragma unroll
      for (int c = 0; c < NT; ++c)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const Acc p1 = accr[tt][c][v], p2 = acci[tt][c][v], p3 = accs[tt][c][v];
          accr[tt][c][v] = p1 - p2;
          acci[tt][c][v] = (p3 - p1) - p2;
        }
  }
#pragma unroll
  for (int c = 0; c < NT; ++c) {
    if (LOWER && n0 + cw + 16 * c > wmax) continue;
    const int col = n0 + cw + 16 * c + rho;
    if constexpr (RT == 2) {
      const int rb = mw + 8 * g;   // rows rb .. rb+7: element v of tile tt is row rb + 2 v + tt
      TC vals[8];
#pragma unroll
      for (int v = 0; v < 4; ++v)
#pragma unroll
        for (int tt = 0; tt < 2; ++tt) st(vals[2 * v + tt], mk((double)accr[tt][c][v], (double)acci[tt][c][v]));
      if (cpk.p && rb < M) {
        // the packed bf16 copy: rows rb .. rb+7 are eight consecutive k of one slab row (the same
        // rounding as k_pack_slabs applies to the stored value; M is a multiple of 128, so a tile
        // row past M starts past it by whole slabs and is skipped)
        uint16_t pre[8], pim[8];
#pragma unroll
        for (int j = 0; j < 8; ++j) {
          const cplx<double> z = ld<double>(vals[j]);
          pre[j] = cvt_e<uint16_t>(z.re);
          pim[j] = cvt_e<uint16_t>(z.im);
        }
        uint16_t* o = cpk.p + (int64_t)f * cpk.sf +
                      (((int64_t)nt * cpk.nsl + rb / 32) * 2 * NP + (cw + 16 * c + rho)) * 32 + (rb % 32);
        vstore<uint16_t, 8>(o, pre);
        vstore<uint16_t, 8>(o + NP * 32, pim);
      }
      if (col >= N) continue;
      TC* cp = C + (int64_t)col * ldc;
      if (vec_c && rb + 8 <= M) {
        vstore<TC, 8>(cp + rb, vals);
      } else {
#pragma unroll
        for (int j = 0; j < 8; ++j)
          if (rb + j < M) cp[rb + j] = vals[j];
      }
    } else {
      if (col >= N) continue;
      TC* cp = C + (int64_t)col * ldc;
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int row = mw + g + 4 * v;
        if (row < M) st(cp[row], mk((double)accr[0][c][v], (double)acci[0][c][v]));
      }
    }
  }
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
// sixteen-column tiles per workgroup: by N, unless a factor call set its sketch_tile option for
// the products it issues from this host thread (packing, workspace size and launch all read it)
inline thread_local int tile_override = 0;
struct TileOverride {
  int saved;
  explicit TileOverride(int nt) : saved(tile_override) { tile_override = nt; }
  ~TileOverride() { tile_override = saved; }
};
template <class P> static inline int nt_for(int N) {
  if (tile_override > 0) return tile_override;
  return N <= 16 ? 1 : (N <= 32 ? 2 : (N <= 64 ? 4 : 8));
}

template <class P, bool CN, bool PACKED, bool SAFE, bool LOWER, bool UTRI, typename TA, typename TX, typename TC, int NT>
static int sk_launch_nt(int M, int N, int K, const TA* A, int64_t lda, int64_t sA, const void* X, int64_t ldx,
                        int64_t sX, TC* C, int64_t ldc, int64_t sC, int batch, int ksplit, int64_t sCsplit,
                        hipStream_t s, PackOut cpk = PackOut()) {
  constexpr int BM = Shape<NT>::WR * 16 * P::RT, NP = 16 * NT, KS = kgroup<P>();
  static_assert(NP > 0 && BM > 0, "shape");
  const int mtiles = (int)ceil_div(M, BM), ntiles = (int)ceil_div(N, NP);
  const int tiles = mtiles * ntiles;
  int64_t nblk = (int64_t)batch * tiles;
  if (batch >= 8) nblk = ceil_div(batch, 8) * 8 * (int64_t)tiles;
  const int kchunk = (int)(ceil_div(ceil_div(K, ksplit), KS) * KS);
  const int bytes = lds_bytes<P, CN, TA>(NT, BM);
  static int attr_done[64] = {0};
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return -1;
  auto kern = k_skinny<P, CN, PACKED, SAFE, LOWER, UTRI, TA, TX, TC, NT>;
  if (bytes > 65536 && dev >= 0 && dev < 64 && !attr_done[dev]) {
    if (hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize, bytes) != hipSuccess) return -1;
    attr_done[dev] = 1;
  }
  const bool vec_c = aligned_elems(C, ldc, sC, sCsplit, sizeof(TC), 16);
  hipLaunchKernelGGL(kern, dim3((unsigned)nblk, (unsigned)ksplit), dim3(SK_THREADS), bytes, s, M, N, K, A, lda, sA, X, ldx,
                     sX, C, ldc, sC, batch, mtiles, ntiles, kchunk, sCsplit, (int)vec_c, cpk);
  return hipGetLastError() == hipSuccess ? 0 : -1;
}

// picks the column-tile count by N and the unchecked (vector) path when shapes and alignment allow
template <class P, bool CN, bool PACKED, bool LOWER, typename TA, typename TX, typename TC, bool UTRI = false>
static int sk_launch(int M, int N, int K, const TA* A, int64_t lda, int64_t sA, const void* X, int64_t ldx, int64_t sX,
                     TC* C, int64_t ldc, int64_t sC, int batch, int ksplit, int64_t sCsplit, hipStream_t s,
                     PackOut cpk = PackOut()) {
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
  // the triangular-X NN products clamp the k rows of a partial last k-group; the others need
  // whole k-groups on the unchecked path
  const bool fast = vec_a && vec_x && small_off && M % BM == 0 && (K % KS == 0 || (UTRI && !CN));
#define RT_SK_NT(NTV)                                                                                          \
  (fast ? sk_launch_nt<P, CN, PACKED, false, LOWER, UTRI, TA, TX, TC, NTV>(M, N, K, A, lda, sA, X, ldx, sX, C, ldc, sC, \
                                                                    batch, ksplit, sCsplit, s, cpk)            \
        : sk_launch_nt<P, CN, PACKED, true, LOWER, UTRI, TA, TX, TC, NTV>(M, N, K, A, lda, sA, X, ldx, sX, C, ldc, sC,  \
                                                                   batch, ksplit, sCsplit, s, cpk))
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
// packed X rows are zero-padded to whole rings of k-groups (the k loop runs in rings)
template <class P> static inline int packed_kp(int K) {
  return (int)(ceil_div(K, SK_RING * kgroup<P>()) * SK_RING * kgroup<P>());
}
template <class P> static inline int64_t packed_elems(int K, int N, int batch) {
  const int NP = 16 * nt_for<P>(N);
  const int64_t KP = packed_kp<P>(K);
  const int64_t NPt = ceil_div(N, NP) * NP;
  return 2 * NPt * KP * batch;
}
// P: the MFMA precision, by default the streamed operand's own (FP64 may also take an FP32 A,
// converted on its way from LDS to the MFMA operands: FP32 data with FP64 accumulation)
template <typename TA, class P = typename PrecOf<TA>::P> static inline int64_t skinny_ws_bytes(int K, int N, int batch) {
  return packed_elems<P>(K, N, batch) * (int64_t)sizeof(typename P::E);
}

// C_f = op(A_f) X_f with X packed into `ws` (skinny_ws_bytes<TA>(K, N, batch) bytes) first:
// skinny_pack, then skinny_run (split so that the caller can time the product kernel alone).
template <typename TA, typename TX, class P = typename PrecOf<TA>::P>
static int skinny_pack(int N, int K, const TX* X, int64_t ldx, int64_t sX, int batch, void* ws, hipStream_t s) {
  typedef typename P::E E;
  const int NP = 16 * nt_for<P>(N);
  const int KP = packed_kp<P>(K);
  const int NPt = (int)(ceil_div(N, NP) * NP);
  constexpr int KSL = kslab<P>();
  constexpr int PV = pack_vec<E>();
  const int64_t per_face = (int64_t)NPt * KP / PV;
  if (per_face >= (1LL << 31)) return -1;
  const int vec = aligned_elems(X, ldx, sX, 0, sizeof(TX), (int64_t)sizeof(TX) * PV) ? 1 : 0;
  // faces in chunks of at most 65535 (grid y)
  for (int f0 = 0; f0 < batch; f0 += 65535) {
    const int fb = std::min(batch - f0, 65535);
    hipLaunchKernelGGL((k_pack_slabs<TX, E, KSL>), dim3((unsigned)ceil_div(per_face, 256), (unsigned)fb), dim3(256), 0, s,
                       X + (int64_t)f0 * sX, ldx, sX, K, N, static_cast<E*>(ws) + (int64_t)f0 * 2 * NPt * KP, KP, NP,
                       NPt / NP, vec);
    if (hipGetLastError() != hipSuccess) return -1;
  }
  return 0;
}

template <typename TA, typename TC, class P = typename PrecOf<TA>::P>
static int skinny_run(bool conjA, int M, int N, int K, const TA* A, int64_t lda, int64_t sA, TC* C, int64_t ldc,
                      int64_t sC, int batch, const void* ws, hipStream_t s, int utri = 0, PackOut cpk = PackOut()) {
  typedef typename P::E E;
  const int NP = 16 * nt_for<P>(N);
  const int KP = packed_kp<P>(K);
  const int NPt = (int)(ceil_div(N, NP) * NP);
  const E* Xp = static_cast<const E*>(ws);
  const int64_t sXp = 2 * (int64_t)NPt * KP;
  // packed X: the raw type parameter is unused, fixed to zd to share instantiations
  if (conjA)
    return sk_launch<P, true, true, false, TA, zd, TC>(M, N, K, A, lda, sA, Xp, KP, sXp, C, ldc, sC, batch, 1, 0, s, cpk);
  if (utri)
    return sk_launch<P, false, true, false, TA, zd, TC, true>(M, N, K, A, lda, sA, Xp, KP, sXp, C, ldc, sC, batch, 1, 0, s,
                                                              cpk);
  return sk_launch<P, false, true, false, TA, zd, TC>(M, N, K, A, lda, sA, Xp, KP, sXp, C, ldc, sC, batch, 1, 0, s, cpk);
}

// The packed bf16 copy that an FP32 product C (rows x N per face) can write for a following bf16
// pass with X = C (K = rows): only when rows is a multiple of 128, so that the slabs have no
// padding rows (ok = false otherwise: that pass packs C itself).
struct PackPlan {
  bool ok = false;
  PackOut out;
  int64_t elems = 0;   // bf16 elements of the whole batch
};
inline PackPlan bf16_pack_plan(int N, int rows, int batch) {
  PackPlan pl;
  if (rows <= 0 || rows % 128 != 0 || packed_kp<B16>(rows) != rows) return pl;
  pl.ok = true;
  pl.out.sf = packed_elems<B16>(rows, N, 1);
  pl.out.nsl = rows / kslab<B16>();
  pl.elems = pl.out.sf * batch;
  return pl;
}

}  // namespace sk
}  // namespace rt
