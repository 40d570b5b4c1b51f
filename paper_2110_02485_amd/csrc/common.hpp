// Shared device/host helpers for the R-tSVD library (gfx950).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>
#include <cmath>

#include "rtsvd.h"

#define RT_HOST_DEVICE __host__ __device__ __forceinline__

// ---------------------------------------------------------------------------------------------
// complex numbers: interleaved (re, im) pairs
// ---------------------------------------------------------------------------------------------
template <typename T> struct cplx { T re, im; };
typedef cplx<double> zd;
typedef cplx<float> zf;
// bf16 complex: two bf16 in one 32-bit word, low half = real part, high half = imaginary part
struct zb { uint32_t bits; };
// up to 16 host doubles passed by value as a kernel argument
struct Vals16 { double v[16]; };

template <typename T> RT_HOST_DEVICE cplx<T> mk(T a, T b) { cplx<T> z; z.re = a; z.im = b; return z; }
template <typename T> RT_HOST_DEVICE cplx<T> cadd(cplx<T> a, cplx<T> b) { return mk(a.re + b.re, a.im + b.im); }
template <typename T> RT_HOST_DEVICE cplx<T> csub(cplx<T> a, cplx<T> b) { return mk(a.re - b.re, a.im - b.im); }
template <typename T> RT_HOST_DEVICE cplx<T> cmul(cplx<T> a, cplx<T> b) {
  return mk(a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re);
}
// conj(a) * b
template <typename T> RT_HOST_DEVICE cplx<T> cmulc(cplx<T> a, cplx<T> b) {
  return mk(a.re * b.re + a.im * b.im, a.re * b.im - a.im * b.re);
}
template <typename T> RT_HOST_DEVICE cplx<T> cconj(cplx<T> a) { return mk(a.re, -a.im); }
template <typename T> RT_HOST_DEVICE cplx<T> cscale(cplx<T> a, T s) { return mk(a.re * s, a.im * s); }
template <typename T> RT_HOST_DEVICE T cabs2(cplx<T> a) { return a.re * a.re + a.im * a.im; }

RT_HOST_DEVICE double cadd_any(double a, double b) { return a + b; }
template <typename T> RT_HOST_DEVICE cplx<T> cadd_any(cplx<T> a, cplx<T> b) { return cadd(a, b); }

// ---------------------------------------------------------------------------------------------
// bf16 (round to nearest even) <-> float
// ---------------------------------------------------------------------------------------------
RT_HOST_DEVICE uint32_t f2bf(float f) {
#ifdef __HIP_DEVICE_COMPILE__
  // gfx950 converts with round to nearest even in one instruction (no branch for inf / nan)
  return (uint32_t)__builtin_bit_cast(unsigned short, (__bf16)f);
#endif
  union { float f; uint32_t u; } v; v.f = f;
  uint32_t u = v.u;
  if ((u & 0x7f800000u) == 0x7f800000u) return (u >> 16) | ((u & 0xffffu) ? 0x40u : 0u);  // inf / nan
  u += 0x7fffu + ((u >> 16) & 1u);
  return u >> 16;
}
RT_HOST_DEVICE float bf2f(uint32_t h) { union { uint32_t u; float f; } v; v.u = h << 16; return v.f; }

// load any storage element as a complex of the accumulation type
template <typename Acc> RT_HOST_DEVICE cplx<Acc> ld(const zd& z) { return mk((Acc)z.re, (Acc)z.im); }
template <typename Acc> RT_HOST_DEVICE cplx<Acc> ld(const zf& z) { return mk((Acc)z.re, (Acc)z.im); }
template <typename Acc> RT_HOST_DEVICE cplx<Acc> ld(const zb& z) {
  return mk((Acc)bf2f(z.bits & 0xffffu), (Acc)bf2f(z.bits >> 16));
}
template <typename Acc> RT_HOST_DEVICE void st(zd& d, cplx<Acc> v) { d.re = (double)v.re; d.im = (double)v.im; }
template <typename Acc> RT_HOST_DEVICE void st(zf& d, cplx<Acc> v) { d.re = (float)v.re; d.im = (float)v.im; }
template <typename Acc> RT_HOST_DEVICE void st(zb& d, cplx<Acc> v) {
  d.bits = f2bf((float)v.re) | (f2bf((float)v.im) << 16);
}

// ---------------------------------------------------------------------------------------------
// cross-lane moves by DPP (data-parallel primitives: VALU operand swizzles within 16-lane rows,
// no LDS round trip).  All lanes of the wave must be active.
// ---------------------------------------------------------------------------------------------
constexpr int DPP_XOR1 = 0xB1;      // quad_perm [1,0,3,2]
constexpr int DPP_XOR2 = 0x4E;      // quad_perm [2,3,0,1]
constexpr int DPP_MIRROR8 = 0x141;  // row_half_mirror: lane i <- 7 - i within 8 lanes
constexpr int DPP_MIRROR16 = 0x140; // row_mirror: lane i <- 15 - i within 16 lanes
constexpr int DPP_ROR8 = 0x128;     // row_ror:8: lane i <- i ^ 8 within 16 lanes

template <int CTRL> __device__ __forceinline__ double dpp(double v) {
  const int lo = __builtin_amdgcn_mov_dpp(__double2loint(v), CTRL, 0xf, 0xf, false);
  const int hi = __builtin_amdgcn_mov_dpp(__double2hiint(v), CTRL, 0xf, 0xf, false);
  return __hiloint2double(hi, lo);
}
template <int CTRL> __device__ __forceinline__ cplx<double> dpp(cplx<double> v) { return mk(dpp<CTRL>(v.re), dpp<CTRL>(v.im)); }
// sum over the 16 lanes of a row, every lane gets it
template <typename T> __device__ __forceinline__ T row_sum16(T v) {
  v = cadd_any(v, dpp<DPP_XOR1>(v));
  v = cadd_any(v, dpp<DPP_XOR2>(v));
  v = cadd_any(v, dpp<DPP_MIRROR8>(v));
  v = cadd_any(v, dpp<DPP_MIRROR16>(v));
  return v;
}
constexpr int DPP_ROW_BCAST15 = 0x142;  // lane 15 of each row to the next row
constexpr int DPP_ROW_BCAST31 = 0x143;  // lane 31 to rows 2 and 3
template <int CTRL, int ROWS> __device__ __forceinline__ double dpp_rows(double v) {
  const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(v), CTRL, ROWS, 0xf, false);
  const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(v), CTRL, ROWS, 0xf, false);
  return __hiloint2double(hi, lo);
}
// sum over the wave, every lane gets it: row sums, then rows combined towards lane 63 by row
// broadcasts (rows not written receive 0), then lane 63 read back as a scalar
__device__ __forceinline__ double wave_sum(double v) {
  v = row_sum16(v);
  v += dpp_rows<DPP_ROW_BCAST15, 0xa>(v);
  v += dpp_rows<DPP_ROW_BCAST31, 0xc>(v);
  const int lo = __builtin_amdgcn_readlane(__double2loint(v), 63);
  const int hi = __builtin_amdgcn_readlane(__double2hiint(v), 63);
  return __hiloint2double(hi, lo);
}
__device__ __forceinline__ cplx<double> wave_sum(cplx<double> v) { return mk(wave_sum(v.re), wave_sum(v.im)); }

// ---------------------------------------------------------------------------------------------
// error handling on the host
// ---------------------------------------------------------------------------------------------
#define RT_CHECK_HIP(expr)                                   \
  do {                                                       \
    hipError_t _e = (expr);                                  \
    if (_e != hipSuccess) { rt_set_hip_error(_e, #expr, __FILE__, __LINE__); return RTSVD_E_HIP; } \
  } while (0)

void rt_set_hip_error(hipError_t e, const char* what, const char* file, int line);

static inline int64_t ceil_div(int64_t a, int64_t b) { return (a + b - 1) / b; }
