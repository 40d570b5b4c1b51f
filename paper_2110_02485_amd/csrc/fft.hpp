// Tube DFTs (Section 2: fft(A, [], 3) and its inverse) for real tensors.
//
// A real tensor with T = (number of tubes) and tube length n is stored tube-element-major:
// element t of tube i sits at in[i + T*t] (frontal slices contiguous).  The forward kernel
// writes the half spectrum, faces f = 0 .. n/2, face-major: out[f*face_stride + i].
//
// Layout on the GPU: a workgroup takes TB consecutive tubes.  Loads of one tube element for
// TB consecutive tubes are contiguous (coalesced), the tile is staged in LDS, two real tubes
// are packed into one complex sequence (z = x + i y), a radix-2 Stockham FFT runs in LDS,
// and the two spectra are separated with X_f = (Z_f + conj Z_{n-f})/2,
// Y_f = (Z_f - conj Z_{n-f})/(2i).  Stores of one face for TB tubes are contiguous again.
#pragma once
#include "common.hpp"
#include <map>
#include <mutex>
#include <algorithm>

namespace rt {

constexpr int FFT_THREADS = 256;

// Stockham radix-2 passes over LDS buffers holding `nseq` interleaved sequences of length n:
// buf[t*nseq + s].  Returns the buffer that holds the result.  sign = -1 forward, +1 inverse.
template <typename T>
__device__ cplx<T>* stockham_lds(cplx<T>* b0, cplx<T>* b1, const cplx<T>* tw, int n, int log2n,
                                 int nseq, int sign) {
  const int half = n >> 1;
  for (int p = 0, Ns = 1; p < log2n; ++p, Ns <<= 1) {
    for (int idx = threadIdx.x; idx < half * nseq; idx += blockDim.x) {
      const int s = idx % nseq;
      const int j = idx / nseq;
      const int k = j & (Ns - 1);
      cplx<T> v0 = b0[j * nseq + s];
      cplx<T> v1 = b0[(j + half) * nseq + s];
      cplx<T> w = tw[k * (half / Ns)];
      if (sign > 0) w.im = -w.im;
      v1 = cmul(v1, w);
      const int d = (j / Ns) * 2 * Ns + k;
      b1[d * nseq + s] = cadd(v0, v1);
      b1[(d + Ns) * nseq + s] = csub(v0, v1);
    }
    __syncthreads();
    cplx<T>* tmp = b0; b0 = b1; b1 = tmp;
  }
  return b0;
}

// twiddle table in global memory: tw[k] = exp(-2 pi i k / n), k < n/2, computed in FP64
template <typename T>
__global__ void k_twiddle_table(cplx<T>* tw, int n) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k < n / 2) {
    double s, c;
    sincospi(-2.0 * (double)k / (double)n, &s, &c);
    tw[k] = mk((T)c, (T)s);
  }
}

template <typename T>
__device__ void fill_twiddles(cplx<T>* tw, const cplx<T>* __restrict__ gtw, int n) {
  for (int k = threadIdx.x; k < n / 2; k += blockDim.x) tw[k] = gtw[k];
}

// forward: real tubes (input type Tin) -> half spectrum in working precision T, optional bf16 copy.
// sumsq: per-block partial sums of the squared inputs (FP64), for ||A||_F^2.
template <typename Tin, typename T>
__global__ void __launch_bounds__(FFT_THREADS)
k_rfft_pow2(const Tin* __restrict__ in, int64_t ntubes, int n, int log2n, int TB,
            cplx<T>* __restrict__ out, int64_t face_stride, zb* __restrict__ out16,
            double* __restrict__ sumsq, const cplx<T>* __restrict__ gtw) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  const int TH = TB / 2;
  cplx<T>* tw = reinterpret_cast<cplx<T>*>(smem_raw);
  cplx<T>* b0 = tw + n / 2;
  cplx<T>* b1 = b0 + (size_t)(n + 2) * TH;
  const int64_t tube0 = (int64_t)blockIdx.x * TB;
  fill_twiddles(tw, gtw, n);
  double acc = 0.0;
  for (int idx = threadIdx.x; idx < n * TB; idx += blockDim.x) {
    const int t = idx / TB, i = idx % TB;
    const int64_t g = tube0 + i;
    T v = 0;
    if (g < ntubes) { v = (T)in[g + ntubes * (int64_t)t]; acc += (double)v * (double)v; }
    cplx<T>& z = b0[t * TH + (i % TH)];
    if (i < TH) z.re = v; else z.im = v;
  }
  __syncthreads();
  cplx<T>* res = stockham_lds(b0, b1, tw, n, log2n, TH, -1);
  const int F = n / 2 + 1;
  for (int idx = threadIdx.x; idx < F * TB; idx += blockDim.x) {
    const int f = idx / TB, i = idx % TB;
    const int s = i % TH;
    const int64_t g = tube0 + i;
    if (g >= ntubes) continue;
    const cplx<T> zf = res[f * TH + s];
    const cplx<T> zn = cconj(res[((n - f) & (n - 1)) * TH + s]);
    cplx<T> v;
    if (i < TH) v = cscale(cadd(zf, zn), (T)0.5);
    else { cplx<T> d = csub(zf, zn); v = mk((T)0.5 * d.im, (T)-0.5 * d.re); }
    if (f == 0 || 2 * f == n) v.im = 0;
    out[f * face_stride + g] = v;
    if (out16) st(out16[f * face_stride + g], v);
  }
  if (sumsq) {
    // block reduction of acc
    __shared__ double red[FFT_THREADS];
    __syncthreads();
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int s = blockDim.x / 2; s > 0; s >>= 1) {
      if ((int)threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
      __syncthreads();
    }
    if (threadIdx.x == 0) sumsq[blockIdx.x] = red[0];
  }
}

// Register-resident forward transform for short power-of-two tubes (N <= 128 in FP32, <= 64 in
// FP64): one thread per tube, so one tube element of 64 consecutive tubes is one contiguous
// 64-lane load and one face of 64 tubes one contiguous store.  The N real samples are packed
// into M = N/2 complex values z_j = x_{2j} + i x_{2j+1}, Z = DFT_M(z) by radix-2 decimation in
// frequency (output in bit-reversed order, all indices compile-time so the data stays in VGPRs),
// then X_f = E_f + w^f O_f with E_f = (Z_f + conj Z_{M-f})/2, O_f = (Z_f - conj Z_{M-f})/(2i),
// w = exp(-2 pi i / N).  gtw[k] = w^k for k < N/2 (uniform reads, served from the scalar cache).
constexpr int RFFT_REG_THREADS = 256;

template <int B> constexpr int bitrev(int k) {
  int r = 0;
  for (int i = 0; i < B; ++i) r |= ((k >> i) & 1) << (B - 1 - i);
  return r;
}
constexpr int ilog2_ce(int n) { return n <= 1 ? 0 : 1 + ilog2_ce(n / 2); }

template <int N, bool HALF, typename Tin, typename T>
// two waves per SIMD for the variant with the bf16 copy (the A-hat pass: measured faster despite
// a small spill); one for the other
__global__ void __launch_bounds__(RFFT_REG_THREADS, HALF ? 2 : 1)
k_rfft_reg(const Tin* __restrict__ in, int64_t ntubes, cplx<T>* __restrict__ out, int64_t face_stride,
           zb* __restrict__ out16, double* __restrict__ sumsq, const cplx<T>* __restrict__ gtw) {
  constexpr int M = N / 2, LM = ilog2_ce(M);
  // One uniform base and 32-bit byte offsets (the host launches this kernel only for tensors
  // below 4 GiB): per-element 64-bit row pointers would overflow the scalar register file.
  const int64_t g0 = (int64_t)blockIdx.x * RFFT_REG_THREADS;
  const bool live = g0 + (int)threadIdx.x < ntubes;
  const unsigned lt = live ? threadIdx.x : 0u;  // lane 0 of every block holds a valid tube
  const char* __restrict__ ib = reinterpret_cast<const char*>(in + g0);
  const unsigned rstride = (unsigned)(ntubes * (int64_t)sizeof(Tin));
  T re[M], im[M];
#pragma unroll
  for (int j = 0; j < M; ++j) {
    re[j] = (T)*reinterpret_cast<const Tin*>(ib + (lt * (unsigned)sizeof(Tin) + (unsigned)(2 * j) * rstride));
    im[j] = (T)*reinterpret_cast<const Tin*>(ib + (lt * (unsigned)sizeof(Tin) + (unsigned)(2 * j + 1) * rstride));
  }
  // sum of squares reduced over the wave before the transform overwrites the samples (left for
  // later, the compiler would keep a second copy of all N samples live through the butterflies)
  __shared__ double red[RFFT_REG_THREADS / 64];
  if (sumsq) {
    double acc = 0.0;
#pragma unroll
    for (int j = 0; j < M; ++j) acc += (double)re[j] * (double)re[j] + (double)im[j] * (double)im[j];
    if (!live) acc = 0.0;
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) acc += __shfl_xor(acc, o);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = acc;
  }
  __builtin_amdgcn_sched_barrier(0);
  // decimation in frequency: span M/2, M/4, ..., 1; twiddle w_M^{j * M/(2 span)} = w_N^{2 j M/(2 span)}
#pragma unroll
  for (int st_ = 0; st_ < LM; ++st_) {
    const int span = M >> (st_ + 1);
#pragma unroll
    for (int b = 0; b < M; b += 2 * span)
#pragma unroll
      for (int j = 0; j < span; ++j) {
        const int u = b + j, v = b + j + span;
        const T ar = re[u] - re[v], ai = im[u] - im[v];
        re[u] += re[v];
        im[u] += im[v];
        if (j == 0) {
          re[v] = ar; im[v] = ai;
        } else {
          const cplx<T> w = gtw[j * (N / (2 * span))];
          re[v] = ar * w.re - ai * w.im;
          im[v] = ar * w.im + ai * w.re;
        }
      }
  }
  char* __restrict__ ob = reinterpret_cast<char*>(out + g0);
  char* __restrict__ hb = reinterpret_cast<char*>(out16 + g0);
  const unsigned ostride = (unsigned)(face_stride * (int64_t)sizeof(cplx<T>));
  const unsigned hstride = (unsigned)(face_stride * 4);
  if (live) {
#pragma unroll
    for (int f = 0; f <= M; ++f) {
      const int i1 = bitrev<LM>(f % M), i2 = bitrev<LM>((M - f) % M);
      cplx<T> x;
      if (f == 0) {
        x = mk(re[0] + im[0], (T)0);
      } else if (f == M) {
        x = mk(re[0] - im[0], (T)0);
      } else {
        const T zr = re[i1], zi = im[i1], cr = re[i2], ci = -im[i2];
        const T er = (T)0.5 * (zr + cr), ei = (T)0.5 * (zi + ci);
        const T dr = zr - cr, di = zi - ci;
        const T orr = (T)0.5 * di, oi = (T)-0.5 * dr;
        const cplx<T> w = gtw[f];
        x = mk(er + (w.re * orr - w.im * oi), ei + (w.re * oi + w.im * orr));
      }
      *reinterpret_cast<cplx<T>*>(ob + (lt * (unsigned)sizeof(cplx<T>) + (unsigned)f * ostride)) = x;
      if constexpr (HALF) st(*reinterpret_cast<zb*>(hb + (lt * 4u + (unsigned)f * hstride)), x);
    }
  }
  if (sumsq) {
    __syncthreads();
    if (threadIdx.x == 0) {
      double t = 0.0;
#pragma unroll
      for (int w = 0; w < RFFT_REG_THREADS / 64; ++w) t += red[w];
      sumsq[blockIdx.x] = t;
    }
  }
}

// inverse: half spectrum (type T) -> real tubes (output type Tout), scaled by 1/n.
template <typename T, typename Tout>
__global__ void __launch_bounds__(FFT_THREADS)
k_irfft_pow2(const cplx<T>* __restrict__ in, int64_t face_stride, int64_t ntubes, int n, int log2n,
             int TB, Tout* __restrict__ out, const cplx<T>* __restrict__ gtw) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  const int TH = TB / 2;
  const int F = n / 2 + 1;
  cplx<T>* tw = reinterpret_cast<cplx<T>*>(smem_raw);
  cplx<T>* b0 = tw + n / 2;
  cplx<T>* b1 = b0 + (size_t)(n + 2) * TH;
  const int64_t tube0 = (int64_t)blockIdx.x * TB;
  fill_twiddles(tw, gtw, n);
  // stage X_f (tubes 0..TH-1) and Y_f (tubes TH..TB-1) for f < F in b1: b1[f*TB + i]
  for (int idx = threadIdx.x; idx < F * TB; idx += blockDim.x) {
    const int f = idx / TB, i = idx % TB;
    const int64_t g = tube0 + i;
    cplx<T> v = mk((T)0, (T)0);
    if (g < ntubes) v = in[f * face_stride + g];
    if (f == 0 || 2 * f == n) v.im = 0;
    b1[f * TB + i] = v;
  }
  __syncthreads();
  // Z_f = X_f + i Y_f for every f of the full spectrum (Hermitian extension of X and Y)
  for (int idx = threadIdx.x; idx < n * TH; idx += blockDim.x) {
    const int f = idx / TH, s = idx % TH;
    cplx<T> x, y;
    if (f < F) { x = b1[f * TB + s]; y = b1[f * TB + s + TH]; }
    else { x = cconj(b1[(n - f) * TB + s]); y = cconj(b1[(n - f) * TB + s + TH]); }
    b0[f * TH + s] = mk(x.re - y.im, x.im + y.re);
  }
  __syncthreads();
  cplx<T>* res = stockham_lds(b0, b1, tw, n, log2n, TH, +1);
  const T inv = (T)1 / (T)n;
  for (int idx = threadIdx.x; idx < n * TB; idx += blockDim.x) {
    const int t = idx / TB, i = idx % TB;
    const int64_t g = tube0 + i;
    if (g >= ntubes) continue;
    const cplx<T> z = res[t * TH + (i % TH)];
    out[g + ntubes * (int64_t)t] = (Tout)((i < TH ? z.re : z.im) * inv);
  }
}

// Direct DFT for tube lengths that are not powers of two (one thread per tube, twiddles in LDS).
template <typename Tin, typename T>
__global__ void k_rdft_direct(const Tin* __restrict__ in, int64_t ntubes, int n,
                              cplx<T>* __restrict__ out, int64_t face_stride, zb* __restrict__ out16,
                              double* __restrict__ sumsq) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  cplx<T>* tw = reinterpret_cast<cplx<T>*>(smem_raw);
  for (int k = threadIdx.x; k < n; k += blockDim.x) {
    double s, c;
    sincospi(-2.0 * (double)k / (double)n, &s, &c);
    tw[k] = mk((T)c, (T)s);
  }
  __syncthreads();
  const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  double acc = 0.0;
  if (g < ntubes) {
    const int F = n / 2 + 1;
    for (int f = 0; f < F; ++f) {
      cplx<T> s = mk((T)0, (T)0);
      int idx = 0;
      for (int t = 0; t < n; ++t) {
        const T v = (T)in[g + ntubes * (int64_t)t];
        s = cadd(s, cscale(tw[idx], v));
        idx += f; if (idx >= n) idx -= n;
        if (f == 0) acc += (double)v * (double)v;
      }
      if (f == 0 || 2 * f == n) s.im = 0;
      out[f * face_stride + g] = s;
      if (out16) st(out16[f * face_stride + g], s);
    }
  }
  if (sumsq) {
    __shared__ double red[FFT_THREADS];
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int s = blockDim.x / 2; s > 0; s >>= 1) {
      if ((int)threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
      __syncthreads();
    }
    if (threadIdx.x == 0) sumsq[blockIdx.x] = red[0];
  }
}

template <typename T, typename Tout>
__global__ void k_irdft_direct(const cplx<T>* __restrict__ in, int64_t face_stride, int64_t ntubes,
                               int n, Tout* __restrict__ out) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  cplx<T>* tw = reinterpret_cast<cplx<T>*>(smem_raw);
  for (int k = threadIdx.x; k < n; k += blockDim.x) {
    double s, c;
    sincospi(2.0 * (double)k / (double)n, &s, &c);
    tw[k] = mk((T)c, (T)s);
  }
  __syncthreads();
  const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= ntubes) return;
  const int F = n / 2 + 1;
  for (int t = 0; t < n; ++t) {
    T s = 0;
    for (int f = 0; f < F; ++f) {
      cplx<T> v = in[f * face_stride + g];
      if (f == 0 || 2 * f == n) v.im = 0;
      const cplx<T> w = tw[(int)(((int64_t)f * t) % n)];
      const T term = v.re * w.re - v.im * w.im;    // Re(v w)
      s += (f == 0 || 2 * f == n) ? term : (T)2 * term;
    }
    out[g + ntubes * (int64_t)t] = (Tout)(s / (T)n);
  }
}

// -------------------------------------------------------------------------------------------
// launchers
// -------------------------------------------------------------------------------------------
inline int ilog2_exact(int64_t n) {
  if (n < 1 || (n & (n - 1))) return -1;
  int l = 0; while ((1LL << l) < n) ++l; return l;
}

// per-device cache of twiddle tables (kept for the life of the process; a few KB each).  A table
// is published only once its fill kernel has completed (the calling thread waits for it), so any
// stream may read a cached table without an event.  The first use of a length n on a device must
// therefore not happen while the stream is being captured into a graph (nullptr is returned then).
// While a TwiddleLookupOnly guard lives on the calling thread, twiddles() only looks tables up
// and never creates one (callers that must not allocate device memory).
inline bool& twiddle_lookup_only() {
  static thread_local bool v = false;
  return v;
}
struct TwiddleLookupOnly {
  bool prev;
  TwiddleLookupOnly() : prev(twiddle_lookup_only()) { twiddle_lookup_only() = true; }
  ~TwiddleLookupOnly() { twiddle_lookup_only() = prev; }
};

template <typename T>
const cplx<T>* twiddles(int n, hipStream_t s) {
  static std::mutex mu;
  static std::map<std::pair<int, int>, cplx<T>*> cache;
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return nullptr;
  std::lock_guard<std::mutex> lk(mu);
  auto key = std::make_pair(dev, n);
  auto it = cache.find(key);
  if (it != cache.end()) return it->second;
  if (twiddle_lookup_only()) return nullptr;
  hipStreamCaptureStatus cap = hipStreamCaptureStatusNone;
  if (hipStreamIsCapturing(s, &cap) != hipSuccess || cap != hipStreamCaptureStatusNone) return nullptr;
  cplx<T>* tw = nullptr;
  if (hipMalloc(&tw, sizeof(cplx<T>) * (size_t)std::max(1, n / 2)) != hipSuccess) return nullptr;
  hipLaunchKernelGGL((k_twiddle_table<T>), dim3((unsigned)((n / 2 + 255) / 256 + 1)), dim3(256), 0, s, tw, n);
  if (hipGetLastError() != hipSuccess || hipStreamSynchronize(s) != hipSuccess) {
    (void)hipFree(tw);
    return nullptr;
  }
  cache[key] = tw;
  return tw;
}

// creates the tables a solve with tube length n uses (forward DFT of B in T, inverse DFT in FP64),
// so that later solves, also allocation-free ones, find them
template <typename T>
inline int ensure_solve_twiddles(int n, hipStream_t s) {
  if (ilog2_exact(n) < 0 || n < 2) return 0;   // direct DFT: no table
  return (twiddles<T>(n, s) && twiddles<double>(n, s)) ? 0 : -1;
}

template <typename T>
inline int fft_tile(int n) {
  // two ping-pong buffers of (n+2) x TB/2 complex plus n/2 twiddles within ~48 KB of LDS
  const int64_t budget = 48 * 1024;
  int tb = 256;
  while (tb > 2 && (int64_t)(2 * (n + 2) * (tb / 2) + n / 2) * (int64_t)sizeof(cplx<T>) > budget) tb >>= 1;
  return tb;
}

template <typename Tin, typename T>
int launch_rfft(const Tin* in, int64_t ntubes, int n, cplx<T>* out, int64_t face_stride, zb* out16,
                double* sumsq, int64_t* nblocks_out, hipStream_t s) {
  const int lg = ilog2_exact(n);
  const int reg_max = sizeof(T) == 4 ? 128 : 64;
  const bool small = ntubes * n * (int64_t)sizeof(Tin) < (1LL << 32) &&
                     (face_stride * (n / 2 + 1) + ntubes) * (int64_t)sizeof(cplx<T>) < (1LL << 32);
  if (lg >= 2 && n <= reg_max && small) {
    const cplx<T>* tw = twiddles<T>(n, s);
    if (!tw) return -1;
    const int64_t blocks = ceil_div(ntubes, RFFT_REG_THREADS);
    switch (n) {
#define RT_RFFT_REG(NN)                                                                                  \
  case NN:                                                                                               \
    if constexpr (NN * sizeof(T) <= 512)                                                                 \
    {                                                                                                  \
      if (out16)                                                                                         \
        hipLaunchKernelGGL((k_rfft_reg<NN, true, Tin, T>), dim3((unsigned)blocks), dim3(RFFT_REG_THREADS), \
                           0, s, in, ntubes, out, face_stride, out16, sumsq, tw);                        \
      else                                                                                               \
        hipLaunchKernelGGL((k_rfft_reg<NN, false, Tin, T>), dim3((unsigned)blocks), dim3(RFFT_REG_THREADS), \
                           0, s, in, ntubes, out, face_stride, out16, sumsq, tw);                        \
    }                                                                                                    \
    break;
      RT_RFFT_REG(4) RT_RFFT_REG(8) RT_RFFT_REG(16) RT_RFFT_REG(32) RT_RFFT_REG(64) RT_RFFT_REG(128)
#undef RT_RFFT_REG
      default: return -1;
    }
    if (nblocks_out) *nblocks_out = blocks;
  } else if (lg >= 0 && n >= 2 && (int64_t)(2 * (n + 2) + n / 2) * (int64_t)sizeof(cplx<T>) <= 48 * 1024) {
    const int TB = fft_tile<T>(n);
    const int64_t blocks = ceil_div(ntubes, TB);
    const size_t lds = (size_t)(2 * (n + 2) * (TB / 2) + n / 2) * sizeof(cplx<T>);
    const cplx<T>* tw = twiddles<T>(n, s);
    if (!tw) return -1;
    hipLaunchKernelGGL((k_rfft_pow2<Tin, T>), dim3((unsigned)blocks), dim3(FFT_THREADS), lds, s,
                       in, ntubes, n, lg, TB, out, face_stride, out16, sumsq, tw);
    if (nblocks_out) *nblocks_out = blocks;
  } else {
    const int64_t blocks = ceil_div(ntubes, FFT_THREADS);
    hipLaunchKernelGGL((k_rdft_direct<Tin, T>), dim3((unsigned)blocks), dim3(FFT_THREADS),
                       (size_t)n * sizeof(cplx<T>), s, in, ntubes, n, out, face_stride, out16, sumsq);
    if (nblocks_out) *nblocks_out = blocks;
  }
  return hipGetLastError() == hipSuccess ? 0 : -1;
}

template <typename T, typename Tout>
int launch_irfft(const cplx<T>* in, int64_t face_stride, int64_t ntubes, int n, Tout* out, hipStream_t s) {
  const int lg = ilog2_exact(n);
  if (lg >= 0 && n >= 2 && (int64_t)(2 * (n + 2) + n / 2) * (int64_t)sizeof(cplx<T>) <= 48 * 1024) {
    const int TB = fft_tile<T>(n);
    const int64_t blocks = ceil_div(ntubes, TB);
    const size_t lds = (size_t)(2 * (n + 2) * (TB / 2) + n / 2) * sizeof(cplx<T>);
    const cplx<T>* tw = twiddles<T>(n, s);
    if (!tw) return -1;
    hipLaunchKernelGGL((k_irfft_pow2<T, Tout>), dim3((unsigned)blocks), dim3(FFT_THREADS), lds, s,
                       in, face_stride, ntubes, n, lg, TB, out, tw);
  } else {
    const int64_t blocks = ceil_div(ntubes, FFT_THREADS);
    hipLaunchKernelGGL((k_irdft_direct<T, Tout>), dim3((unsigned)blocks), dim3(FFT_THREADS),
                       (size_t)n * sizeof(cplx<T>), s, in, face_stride, ntubes, n, out);
  }
  return hipGetLastError() == hipSuccess ? 0 : -1;
}

}  // namespace rt
