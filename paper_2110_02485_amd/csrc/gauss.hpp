// Gaussian test tensor of the R-tSVD (Alg. 6 draws Gaussian tensor columns G) generated on the
// device, and the finiteness guard of the factor's input.
//
// Generator: Philox4x32-10, the counter-based generator of Salmon, Moraes, Dror and Shaw
// ("Parallel random numbers: as easy as 1, 2, 3", SC 2011): ten rounds of two 32 x 32 -> 64-bit
// multiplications (multipliers 0xD2511F53, 0xCD9E8D57) with the key bumped by the Weyl constants
// 0x9E3779B9, 0xBB67AE85 between rounds.  Element e of the column-major m x r x n tensor
// (e = i + m j + m r t) belongs to the pair q = floor(e / 2): counter (q mod 2^32, q div 2^32, 0, 0),
// key (seed mod 2^32, seed div 2^32).  The four output words give two uniforms in (0, 1) with 53
// random bits each, u1 = (((x1 << 32) | x0) >> 11 + 1/2) 2^-53 and u2 = (((x3 << 32) | x2) >> 11) 2^-53,
// and the Box-Muller transform (Box and Muller, Ann. Math. Stat. 1958) turns them into the pair
// sqrt(-2 ln u1) (cos 2 pi u2, sin 2 pi u2): element 2q takes the cosine term, 2q + 1 the sine term.
// Everything is computed in FP64 and rounded once to the output type.
#pragma once
#include "common.hpp"

namespace rt {

struct U32x4 { uint32_t v[4]; };

__device__ __forceinline__ U32x4 philox4x32_10(U32x4 c, uint32_t k0, uint32_t k1) {
#pragma unroll
  for (int round = 0; round < 10; ++round) {
    const uint64_t p0 = (uint64_t)0xD2511F53u * c.v[0];
    const uint64_t p1 = (uint64_t)0xCD9E8D57u * c.v[2];
    U32x4 o;
    o.v[0] = (uint32_t)(p1 >> 32) ^ c.v[1] ^ k0;
    o.v[1] = (uint32_t)p1;
    o.v[2] = (uint32_t)(p0 >> 32) ^ c.v[3] ^ k1;
    o.v[3] = (uint32_t)p0;
    c = o;
    k0 += 0x9E3779B9u;
    k1 += 0xBB67AE85u;
  }
  return c;
}

// the standard normal pair of pair index q (see the file comment)
__device__ __forceinline__ void gauss_pair(uint64_t seed, uint64_t q, double* z0, double* z1) {
  U32x4 c;
  c.v[0] = (uint32_t)q;
  c.v[1] = (uint32_t)(q >> 32);
  c.v[2] = 0u;
  c.v[3] = 0u;
  const U32x4 x = philox4x32_10(c, (uint32_t)seed, (uint32_t)(seed >> 32));
  const uint64_t a = (((uint64_t)x.v[1] << 32) | x.v[0]) >> 11;
  const uint64_t b = (((uint64_t)x.v[3] << 32) | x.v[2]) >> 11;
  const double u1 = ((double)a + 0.5) * 0x1p-53;
  const double u2 = (double)b * 0x1p-53;
  const double rad = sqrt(-2.0 * log(u1));
  double s, co;
  sincospi(2.0 * u2, &s, &co);
  *z0 = rad * co;
  *z1 = rad * s;
}

// out[e] = element e of the Gaussian tensor, e < count; one pair per thread
template <typename T>
__global__ void __launch_bounds__(256) k_gaussian(uint64_t seed, int64_t count, T* __restrict__ out) {
  const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t e = 2 * q;
  if (e >= count) return;
  double z0, z1;
  gauss_pair(seed, (uint64_t)q, &z0, &z1);
  out[e] = (T)z0;
  if (e + 1 < count) out[e + 1] = (T)z1;
}

// one thread per pair; the grid stays below 2^31 work-items
constexpr int64_t GAUSS_MAX_PAIRS = (int64_t)1 << 31;
template <typename T>
inline int launch_gaussian(uint64_t seed, int64_t count, T* out, hipStream_t s) {
  if (count <= 0) return 0;
  const int64_t pairs = (count + 1) / 2;
  if (pairs > GAUSS_MAX_PAIRS) return -1;
  hipLaunchKernelGGL((k_gaussian<T>), dim3((unsigned)ceil_div(pairs, 256)), dim3(256), 0, s, seed, count, out);
  return hipGetLastError() == hipSuccess ? 0 : -1;
}

// Finiteness guard after the tube DFT of A: the block partial sums of ||A||_F^2 are added in a
// fixed order; a non-finite total sets bit 1 of *flags.
constexpr int FIN_THREADS = 256;
__global__ void __launch_bounds__(FIN_THREADS)
k_finite_check(const double* __restrict__ sumsq, int64_t nblk, int* __restrict__ flags) {
  __shared__ double red[FIN_THREADS / 64];
  double s = 0.0;
  for (int64_t i = threadIdx.x; i < nblk; i += blockDim.x) s += sumsq[i];
  s = wave_sum(s);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) {
    double t = 0.0;
    for (int w = 0; w < FIN_THREADS / 64; ++w) t += red[w];
    if (!isfinite(t)) atomicOr(flags, 2);
  }
}

// p[0 .. count) = 0 when bit 1 of *flags is set (the factor then works on a zero operator, whose
// path is the zero-face path: every pivot breaks down, sigma = 0, zero solution); otherwise every
// workgroup returns at once.
template <typename T>
__global__ void __launch_bounds__(256) k_zero_if_nonfinite(T* __restrict__ p, int64_t count, const int* __restrict__ flags) {
  if ((*flags & 2) == 0) return;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count; i += stride) p[i] = T{};
}

template <typename T>
inline int launch_zero_if_nonfinite(T* p, int64_t count, const int* flags, hipStream_t s) {
  if (!p || count <= 0) return 0;
  const int64_t blocks = std::min<int64_t>(ceil_div(count, 256), 2048);
  hipLaunchKernelGGL((k_zero_if_nonfinite<T>), dim3((unsigned)blocks), dim3(256), 0, s, p, count, flags);
  return hipGetLastError() == hipSuccess ? 0 : -1;
}

}  // namespace rt
