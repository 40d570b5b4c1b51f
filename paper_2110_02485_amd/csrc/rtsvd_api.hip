// C ABI of librtsvd (declared in include/rtsvd.h): argument checks, scratch management and the
// launch sequences of the R-tSVD factor / solve, the T-tSVD comparator, t-products and tGKB.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <vector>

#include "common.hpp"
#include "fft.hpp"
#include "gauss.hpp"
#include "gram.hpp"
#include "gemm.hpp"
#include "skinny.hpp"
#include "heev.hpp"
#include "solve.hpp"
#include "tgkb.hpp"

using namespace rt;

// ---------------------------------------------------------------------------------------------
// error reporting
// ---------------------------------------------------------------------------------------------
static thread_local std::string g_last_error;

void rt_set_hip_error(hipError_t e, const char* what, const char* file, int line) {
  char buf[512];
  snprintf(buf, sizeof(buf), "%s failed: %s (%s:%d)", what, hipGetErrorString(e), file, line);
  g_last_error = buf;
}

static int fail(int code, const char* msg) {
  g_last_error = msg;
  return code;
}

#define RT_TRY(expr)                                                        \
  do {                                                                      \
    int _rc = (expr);                                                       \
    if (_rc != 0) {                                                         \
      if (g_last_error.empty()) g_last_error = "launch failed: " #expr;     \
      return _rc < 0 ? _rc : RTSVD_E_HIP;                                   \
    }                                                                       \
  } while (0)

#define RT_LAUNCH_OK() RT_CHECK_HIP(hipGetLastError())

// ---------------------------------------------------------------------------------------------
// Device workspace cache.  Buffers are allocated once (stream-ordered) and then kept: a released
// buffer goes back to a free list of the stream it was used on and is handed out again only to
// work on that same stream, so stream order alone makes the reuse safe.  Freeing large buffers
// every call would otherwise cost milliseconds of host time per call and stall the pipeline.
// rtsvd_trim() returns all cached memory to the device.
// ---------------------------------------------------------------------------------------------
struct WorkspaceCache {
  struct Live { int dev; hipStream_t s; size_t bytes; };
  std::mutex mu;
  std::map<std::pair<int, hipStream_t>, std::multimap<size_t, void*>> free_;
  std::map<void*, Live> live_;

  void* acquire(size_t bytes, hipStream_t s) {
    bytes = (bytes + 255) & ~(size_t)255;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return nullptr;
    {
      std::lock_guard<std::mutex> lk(mu);
      auto& fl = free_[{dev, s}];
      auto it = fl.lower_bound(bytes);
      // best fit, without handing a much larger block to a small request
      if (it != fl.end() && it->first <= bytes + bytes / 4 + 4096) {
        void* p = it->second;
        live_[p] = Live{dev, s, it->first};
        fl.erase(it);
        return p;
      }
    }
    void* p = nullptr;
    if (hipMallocAsync(&p, bytes, s) != hipSuccess || !p) {
      (void)hipGetLastError();
      return nullptr;
    }
    std::lock_guard<std::mutex> lk(mu);
    live_[p] = Live{dev, s, bytes};
    return p;
  }
  void release(void* p) {
    if (!p) return;
    std::lock_guard<std::mutex> lk(mu);
    auto it = live_.find(p);
    if (it == live_.end()) return;
    free_[{it->second.dev, it->second.s}].emplace(it->second.bytes, p);
    live_.erase(it);
  }
  int trim() {
    std::lock_guard<std::mutex> lk(mu);
    int cur = 0;
    if (hipGetDevice(&cur) != hipSuccess) return -1;
    for (auto& kv : free_) {
      if (kv.second.empty()) continue;
      if (hipSetDevice(kv.first.first) != hipSuccess || hipDeviceSynchronize() != hipSuccess) return -1;
      for (auto& b : kv.second) (void)hipFree(b.second);
      kv.second.clear();
    }
    return hipSetDevice(cur) == hipSuccess ? 0 : -1;
  }
};
static WorkspaceCache g_cache;

// per-call scratch: every buffer goes back to the cache when the call's launches are queued
struct Scratch {
  hipStream_t s;
  std::vector<void*> ptrs;
  explicit Scratch(hipStream_t st) : s(st) {}
  ~Scratch() { for (void* p : ptrs) g_cache.release(p); }
  template <typename T> T* get(int64_t count) {
    if (count <= 0) count = 1;
    void* p = g_cache.acquire((size_t)count * sizeof(T), s);
    if (!p) return nullptr;
    ptrs.push_back(p);
    return static_cast<T*>(p);
  }
  template <typename T> T* release(T* p) {  // ownership passes to the caller (returned with g_cache.release)
    ptrs.erase(std::remove(ptrs.begin(), ptrs.end(), (void*)p), ptrs.end());
    return p;
  }
};

// bump allocator over a fixed device region (the allocation-free entry point): hands out
// 256-byte aligned slices in request order, nullptr once the region is exhausted; allocates nothing
struct Arena {
  unsigned char* base = nullptr;
  size_t cap = 0, used = 0;
  static size_t round(size_t bytes) { return (bytes + 255) & ~(size_t)255; }
  template <typename T> T* get(int64_t count) {
    if (count <= 0) count = 1;
    const size_t bytes = round((size_t)count * sizeof(T));
    if (!base || used + bytes > cap) return nullptr;
    T* p = reinterpret_cast<T*>(base + used);
    used += bytes;
    return p;
  }
};

#define RT_ALLOC(var, type, count, sc)                                             \
  type* var = (sc).template get<type>(count);                                      \
  if (!var) return fail(RTSVD_E_NOMEM, "device allocation failed: " #var)

static inline unsigned nblocks(int64_t total, int threads = 256) { return (unsigned)ceil_div(total, threads); }

// Small host arrays reach the device as kernel arguments (16 values per launch): stream-ordered,
// no staging copy from pageable memory (which would block the host until the stream drains).
__global__ void k_set_doubles(double* __restrict__ dst, Vals16 vals, int count) {
  if ((int)threadIdx.x < count) dst[threadIdx.x] = vals.v[threadIdx.x];
}
__global__ void k_set_int(int* __restrict__ dst, int value) {
  if (threadIdx.x == 0) dst[0] = value;
}
static int upload_doubles(double* dst, const double* src, int64_t count, hipStream_t s) {
  for (int64_t off = 0; off < count; off += 16) {
    Vals16 v = {};
    const int c = (int)std::min<int64_t>(16, count - off);
    for (int i = 0; i < c; ++i) v.v[i] = src[off + i];
    hipLaunchKernelGGL(k_set_doubles, dim3(1), dim3(64), 0, s, dst + off, v, c);
    if (hipGetLastError() != hipSuccess) return -1;
  }
  return 0;
}

template <typename TI, typename TO>
__global__ void k_convert(const TI* __restrict__ in, TO* __restrict__ out, int64_t count) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < count) st(out[i], ld<double>(in[i]));
}

// ---------------------------------------------------------------------------------------------
// factor handle
// ---------------------------------------------------------------------------------------------
struct rtsvd_factor_s {
  int64_t l = 0, m = 0, n = 0, F = 0, r = 0;
  int dtype = RTSVD_F64;       // caller dtype
  int precision = RTSVD_P_FP64;
  int kind = 0;                // 0 = R-tSVD, 1 = T-tSVD, 2 = T-tEVD
  int k_max = 0, oversample = 0;
  double eps = 0.0;
  hipStream_t stream = nullptr;
  void* Q = nullptr;           // F x l x r, work type; T-tSVD: the left singular vectors U
  zd* Ub = nullptr;            // F x r x r (R-tSVD only)
  double* sigma = nullptr;     // F x r
  zd* V = nullptr;             // F x m x r
  void* W = nullptr;           // F x l x r, work type (A-hat V)
  double* eta = nullptr;       // r + 1
  int* flags = nullptr;        // 1
  std::vector<void*> owned;
};

static bool work_is_double(int precision) { return precision == RTSVD_P_FP64; }

// ---------------------------------------------------------------------------------------------
// stage timers: HIP events around tagged launch sequences, on the stream they are launched on
// ---------------------------------------------------------------------------------------------
struct TimerState {
  std::mutex mu;
  bool on = false;
  std::vector<std::pair<int, std::pair<hipEvent_t, hipEvent_t>>> rec;
  std::vector<hipEvent_t> pool;
  hipEvent_t get() {
    if (!pool.empty()) { hipEvent_t e = pool.back(); pool.pop_back(); return e; }
    hipEvent_t e = nullptr;
    (void)hipEventCreate(&e);
    return e;
  }
};
static TimerState g_timer;

struct TimerScope {
  int tag;
  hipStream_t s;
  hipEvent_t a = nullptr, b = nullptr;
  TimerScope(int t, hipStream_t st) : tag(t), s(st) {
    std::lock_guard<std::mutex> lk(g_timer.mu);
    if (!g_timer.on) return;
    a = g_timer.get();
    b = g_timer.get();
    (void)hipEventRecord(a, s);
  }
  ~TimerScope() {
    if (!a) return;
    (void)hipEventRecord(b, s);
    std::lock_guard<std::mutex> lk(g_timer.mu);
    g_timer.rec.push_back({tag, {a, b}});
  }
};
#define RT_CAT2(a, b) a##b
#define RT_CAT(a, b) RT_CAT2(a, b)
#define RT_TIMED(tag) TimerScope RT_CAT(_timer_scope_, __LINE__)(tag, s)

extern "C" int rtsvd_timer_enable(int on) {
  std::lock_guard<std::mutex> lk(g_timer.mu);
  for (auto& r : g_timer.rec) { g_timer.pool.push_back(r.second.first); g_timer.pool.push_back(r.second.second); }
  g_timer.rec.clear();
  g_timer.on = on != 0;
  return RTSVD_OK;
}

extern "C" int rtsvd_timer_read(int tag, double* total_ms, int32_t* launches) {
  std::lock_guard<std::mutex> lk(g_timer.mu);
  double tot = 0.0;
  int cnt = 0;
  for (auto& r : g_timer.rec) {
    if (r.first != tag) continue;
    if (hipEventSynchronize(r.second.second) != hipSuccess) return fail(RTSVD_E_HIP, "rtsvd_timer_read: event");
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, r.second.first, r.second.second) != hipSuccess)
      return fail(RTSVD_E_HIP, "rtsvd_timer_read: elapsed");
    tot += ms;
    ++cnt;
  }
  if (total_ms) *total_ms = tot;
  if (launches) *launches = cnt;
  return RTSVD_OK;
}

// ---------------------------------------------------------------------------------------------
// launchers of the per-face r x r kernels (packed matrix in LDS when it fits)
// ---------------------------------------------------------------------------------------------
static int max_lds_per_block() {
  static int cached[64] = {0};
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return 65536;
  if (!cached[dev]) {
    int v = 65536;
    if (hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess) v = 65536;
    cached[dev] = v;
  }
  return cached[dev];
}

static int orthonormalize_tri_vectors(double* zs, int r, int64_t F, Scratch& sc, hipStream_t s);

static int launch_heev(const zd* G, int r, int64_t F, zd* U, double* lam, Scratch& sc, hipStream_t s) {
  const size_t full = heev_lds_bytes(r, true);
  const bool in_lds = (int64_t)full <= (int64_t)max_lds_per_block();
  const size_t bytes = in_lds ? full : heev_lds_bytes(r, false);
  zd* gpk = sc.get<zd>(F * packed_size(r));
  if (!gpk) return fail(RTSVD_E_NOMEM, "device allocation failed: heev packed scratch");
  double* zs = sc.get<double>(F * r * (int64_t)(r + 1));
  if (!zs) return fail(RTSVD_E_NOMEM, "device allocation failed: heev scratch");
  // LU factors of T - lambda I in global memory: only the one-kernel solver's inverse iteration
  // (modes 0 and 3) uses them; k_tri_stein keeps its own in LDS
  double* lu = nullptr;
  auto need_lu = [&]() -> int {
    lu = sc.get<double>(F * r * 5 * (int64_t)r);
    return lu ? 0 : fail(RTSVD_E_NOMEM, "device allocation failed: heev LU scratch");
  };
  if (r <= TRD_R) {
    // tridiagonal form from the register-resident kernel, then eigenvalues / vectors
    double* tri = sc.get<double>(F * 2 * (int64_t)r);
    zd* taus = sc.get<zd>(F * (int64_t)r);
    if (!tri || !taus) return fail(RTSVD_E_NOMEM, "device allocation failed: heev tridiagonal");
    hipLaunchKernelGGL(k_hetrd_reg, dim3((unsigned)F), dim3(TRD_THREADS), 0, s, G, r, tri, taus, gpk);
    RT_LAUNCH_OK();
    const size_t sb = stein_lds_bytes(r);   // <= 52 KB for r <= TRD_R
    hipLaunchKernelGGL(k_tri_stein, dim3((unsigned)ceil_div(r, STEIN_EPB), (unsigned)F), dim3(STEIN_THREADS), sb, s,
                       (const double*)tri, r, lam, zs);
    RT_LAUNCH_OK();
    auto kern = in_lds ? k_heev<true, 2> : k_heev<false, 2>;
    if (bytes > 65536) RT_CHECK_HIP(hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes));
    hipLaunchKernelGGL(kern, dim3((unsigned)F), dim3(HEEV_THREADS), bytes, s, G, r, U, lam, gpk, zs, lu,
                       (const double*)tri, (const zd*)taus, (zd*)nullptr, (double*)nullptr);
    RT_LAUNCH_OK();
    hipLaunchKernelGGL((k_heev_backtr<HEEV_UREG, BT_CH>), dim3((unsigned)ceil_div(r, BT_COLS), (unsigned)F),
                       dim3(BT_THREADS), 0, s, (const zd*)gpk, (const zd*)taus, (const double*)zs, r, U);
    RT_LAUNCH_OK();
    return 0;
  }
  if (r <= 8 * BT_UREG_WIDE && !in_lds) {
    // tridiagonalization in the one-workgroup kernel (global working matrix), eigenvalues and
    // inverse iteration spread over many workgroups (k_tri_stein), the eigenvectors of T made
    // orthonormal by CholeskyQR2 on FP64 MFMA (Q = Z R^{-1}: the Q of modified Gram-Schmidt over
    // all r columns, which takes the place of Gram-Schmidt inside clusters), then the register-
    // resident back-transformation
    zd* taus = sc.get<zd>(F * (int64_t)r);
    double* tri = sc.get<double>(F * 2 * (int64_t)r);
    if (!taus || !tri) return fail(RTSVD_E_NOMEM, "device allocation failed: heev tridiagonal");
    hipLaunchKernelGGL((k_heev<false, 4>), dim3((unsigned)F), dim3(HEEV_THREADS), bytes, s, G, r, U, lam, gpk, zs, lu,
                       (const double*)nullptr, (const zd*)nullptr, taus, tri);
    RT_LAUNCH_OK();
    const size_t sb = stein_lds_bytes(r);
    if (sb > 65536)
      RT_CHECK_HIP(hipFuncSetAttribute((const void*)k_tri_stein, hipFuncAttributeMaxDynamicSharedMemorySize, (int)sb));
    hipLaunchKernelGGL(k_tri_stein, dim3((unsigned)ceil_div(r, STEIN_EPB), (unsigned)F), dim3(STEIN_THREADS), sb, s,
                       (const double*)tri, r, lam, zs);
    RT_LAUNCH_OK();
    RT_TRY(orthonormalize_tri_vectors(zs, r, F, sc, s));
    hipLaunchKernelGGL((k_heev_backtr<BT_UREG_WIDE, BT_CH_WIDE>), dim3((unsigned)ceil_div(r, BT_COLS), (unsigned)F),
                       dim3(BT_THREADS), 0, s, (const zd*)gpk, (const zd*)taus, (const double*)zs, r, U);
    RT_LAUNCH_OK();
    return 0;
  }
  if (r <= 8 * BT_UREG_WIDE) {
    // the whole solver but the back-transformation, then the register-resident back-transformation
    zd* taus = sc.get<zd>(F * (int64_t)r);
    if (!taus) return fail(RTSVD_E_NOMEM, "device allocation failed: heev reflector scalars");
    RT_TRY(need_lu());
    auto kern = in_lds ? k_heev<true, 3> : k_heev<false, 3>;
    if (bytes > 65536) RT_CHECK_HIP(hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes));
    hipLaunchKernelGGL(kern, dim3((unsigned)F), dim3(HEEV_THREADS), bytes, s, G, r, U, lam, gpk, zs, lu,
                       (const double*)nullptr, (const zd*)nullptr, taus, (double*)nullptr);
    RT_LAUNCH_OK();
    hipLaunchKernelGGL((k_heev_backtr<BT_UREG_WIDE, BT_CH_WIDE>), dim3((unsigned)ceil_div(r, BT_COLS), (unsigned)F),
                       dim3(BT_THREADS), 0, s, (const zd*)gpk, (const zd*)taus, (const double*)zs, r, U);
    RT_LAUNCH_OK();
    return 0;
  }
  RT_TRY(need_lu());
  auto kern = in_lds ? k_heev<true> : k_heev<false>;
  if (bytes > 65536) RT_CHECK_HIP(hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes));
  hipLaunchKernelGGL(kern, dim3((unsigned)F), dim3(HEEV_THREADS), bytes, s, G, r, U, lam, gpk, zs, lu,
                     (const double*)nullptr, (const zd*)nullptr, (zd*)nullptr, (double*)nullptr);
  RT_LAUNCH_OK();
  return 0;
}

static int launch_cholinv(const zd* G, int r, int64_t F, zd* Rinv, int* flags, Scratch& sc, hipStream_t s) {
  const size_t full = chol_lds_bytes(r, true);
  const bool in_lds = (int64_t)full <= (int64_t)max_lds_per_block();
  const size_t bytes = in_lds ? full : chol_lds_bytes(r, false);
  // the kernel's waves 1..7 hold at most 1 (LDS variant) or 3 tiles each of a block row of L^{-1}
  if ((in_lds && r > 128) || r > HEEV_RMAX)
    return fail(RTSVD_E_UNSUPPORTED, "Cholesky inverse: r beyond the kernel's block-row capacity");
  zd* gpk = nullptr;
  if (!in_lds) {
    gpk = sc.get<zd>(F * packed_size(r));
    if (!gpk) return fail(RTSVD_E_NOMEM, "device allocation failed: cholinv packed scratch");
  }
  zd* gdi = sc.get<zd>(F * chol_gdi_elems(r));
  if (!gdi) return fail(RTSVD_E_NOMEM, "device allocation failed: cholinv block inverses");
  auto kern = in_lds ? k_cholinv<true> : k_cholinv<false>;
  if (bytes > 65536) RT_CHECK_HIP(hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes));
  hipLaunchKernelGGL(kern, dim3((unsigned)F), dim3(CH_THREADS), bytes, s, G, r, Rinv, 1e-13, flags, gpk, gdi);
  RT_LAUNCH_OK();
  return 0;
}

// G_f = Y_f^H Y_f (lower triangle), FP64
template <typename TY>
static int gram(const TY* Y, int64_t rows, int64_t r, int64_t F, zd* G, Scratch& sc, hipStream_t s) {
  if (rows > INT32_MAX || r > INT32_MAX) return fail(RTSVD_E_UNSUPPORTED, "gram: dimensions exceed 2^31");
  // measured on 1024 x 120 panels: the slab kernel wins for FP64 panels (its LDS staging halves
  // the memory traffic per tile), the per-tile kernel for FP32 panels
  if (sizeof(TY) == sizeof(zd) && r <= GS_RMAX && rows >= 16 * GS_KS * 4) {
    zd* part = sc.get<zd>(gram_part_elems((int)r, (int)F));
    if (!part) return fail(RTSVD_E_NOMEM, "device allocation failed: gram partials");
    return gram_slab<TY>(Y, (int)rows, (int)r, rows, rows * r, (int)F, part, G, s);
  }
  return gram_lower<TY>(Y, (int)rows, (int)r, rows, rows * r, (int)F, G, s);
}

// C_f = op(A_f) X_f on MFMA, X packed into pool scratch first
// ktag: optional timer tag for the product kernel alone (without the packing pass);
// utri: X is upper triangular (its zero blocks are skipped)
// P: MFMA precision (default: that of A's type; sk::F64 with an FP32 A gives FP64 accumulation)
template <typename TA, typename TX, typename TC, typename SC = Scratch, class P = typename sk::PrecOf<TA>::P>
static int skinny(bool conjA, int64_t M, int64_t N, int64_t K, const TA* A, int64_t lda, int64_t sA, const TX* X,
                  int64_t ldx, int64_t sX, TC* C, int64_t ldc, int64_t sC, int64_t F, SC& sc, hipStream_t s,
                  int ktag = 0, int utri = 0, sk::PackOut cpk = sk::PackOut(), const void* prepacked = nullptr) {
  if (M <= 0 || N <= 0 || F <= 0) return 0;
  if (K <= 0) return fail(RTSVD_E_ARG, "skinny product: K must be positive");
  // prepacked: X already in the packed layout (written by the product that formed it)
  const void* ws = prepacked;
  if (!ws) {
    unsigned char* w = sc.template get<unsigned char>(sk::skinny_ws_bytes<TA, P>((int)K, (int)N, (int)F));
    if (!w) return fail(RTSVD_E_NOMEM, "device allocation failed: packed operand");
    if (sk::skinny_pack<TA, TX, P>((int)N, (int)K, X, ldx, sX, (int)F, w, s))
      return fail(RTSVD_E_HIP, "skinny pack launch");
    ws = w;
  }
  if (ktag) {
    RT_TIMED(ktag);
    return sk::skinny_run<TA, TC, P>(conjA, (int)M, (int)N, (int)K, A, lda, sA, C, ldc, sC, (int)F, ws, s, utri, cpk);
  }
  return sk::skinny_run<TA, TC, P>(conjA, (int)M, (int)N, (int)K, A, lda, sA, C, ldc, sC, (int)F, ws, s, utri, cpk);
}

// ---------------------------------------------------------------------------------------------
// CholeskyQR: Y (F x rows x r) <- Y R^{-1} with R^H R = Y^H Y (FP64 Gram + Cholesky), `passes`
// times (2 = CholeskyQR2, orthonormal to working precision).  The product is written to `tmp` and
// the two buffers are exchanged, so Y names the result on return.
// ---------------------------------------------------------------------------------------------
// qpack (FP32 Y only, may be null): the last pass also writes Q as the packed bf16 X operand of
// the following bf16 pass over A-hat, when the row count allows it (*packed says whether it did).
template <typename TY>
static int orthonormalize(TY*& Y, int64_t rows, int64_t r, int64_t F, int passes, zd* G, zd* Rinv, TY*& tmp,
                          int* flags, Scratch& sc, hipStream_t s, uint16_t* qpack = nullptr,
                          bool* packed = nullptr) {
  if (packed) *packed = false;
  for (int pass = 0; pass < passes; ++pass) {
    {
      RT_TIMED(RTSVD_T_GRAM);
      RT_TRY(gram<TY>(Y, rows, r, F, G, sc, s));
    }
    {
      RT_TIMED(RTSVD_T_CHOL);
      RT_TRY(launch_cholinv(G, (int)r, F, Rinv, flags, sc, s));
    }
    RT_TIMED(RTSVD_T_QMUL);
    sk::PackOut cpk;
    if constexpr (std::is_same<TY, zf>::value) {
      if (qpack && pass == passes - 1) {
        const sk::PackPlan pl = sk::bf16_pack_plan((int)r, (int)rows, (int)F);
        if (pl.ok) {
          cpk = pl.out;
          cpk.p = qpack;
          if (packed) *packed = true;
        }
      }
    }
    // R^{-1} is upper triangular
    RT_TRY((skinny<TY, zd, TY>(false, rows, r, r, Y, rows, rows * r, Rinv, r, r * r, tmp, rows, rows * r, F, sc, s, 0, 1,
                               cpk)));
    std::swap(Y, tmp);
  }
  return 0;
}

// real eigenvectors of the tridiagonal (zs: F x r columns of stride r + 1) <-> complex r x r panels
__global__ void k_tri_vectors_to_panel(const double* __restrict__ zs, int r, int64_t F, zd* __restrict__ Z) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= F * r * r) return;
  const int64_t f = idx / ((int64_t)r * r);
  const int64_t rem = idx - f * r * r;
  const int j = (int)(rem / r), i = (int)(rem - (int64_t)j * r);
  Z[idx] = mk(zs[(f * r + j) * (r + 1) + i], 0.0);
}
__global__ void k_panel_to_tri_vectors(const zd* __restrict__ Z, int r, int64_t F, double* __restrict__ zs) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= F * r * r) return;
  const int64_t f = idx / ((int64_t)r * r);
  const int64_t rem = idx - f * r * r;
  const int j = (int)(rem / r), i = (int)(rem - (int64_t)j * r);
  zs[(f * r + j) * (r + 1) + i] = Z[idx].re;
}

// The eigenvectors of T from inverse iteration, made orthonormal in their order by CholeskyQR2
// (FP64 Gram, Cholesky inverse, Z R^{-1} on MFMA, twice): for the nearly orthonormal Z this is the
// modified Gram-Schmidt result; the imaginary parts stay zero.
static int orthonormalize_tri_vectors(double* zs, int r, int64_t F, Scratch& sc, hipStream_t s) {
  const int64_t n = F * r * (int64_t)r;
  zd* Z = sc.get<zd>(n);
  zd* tmp = sc.get<zd>(n);
  zd* G = sc.get<zd>(n);
  zd* Rinv = sc.get<zd>(n);
  int* flags = sc.get<int>(1);
  if (!Z || !tmp || !G || !Rinv || !flags) return fail(RTSVD_E_NOMEM, "device allocation failed: eigenvector QR");
  hipLaunchKernelGGL(k_set_int, dim3(1), dim3(64), 0, s, flags, 0);
  RT_LAUNCH_OK();
  hipLaunchKernelGGL(k_tri_vectors_to_panel, dim3((unsigned)ceil_div(n, 256)), dim3(256), 0, s, (const double*)zs, r,
                     F, Z);
  RT_LAUNCH_OK();
  RT_TRY((orthonormalize<zd>(Z, r, r, F, 2, G, Rinv, tmp, flags, sc, s)));
  hipLaunchKernelGGL(k_panel_to_tri_vectors, dim3((unsigned)ceil_div(n, 256)), dim3(256), 0, s, (const zd*)Z, r, F,
                     zs);
  RT_LAUNCH_OK();
  return 0;
}

// products over A-hat: Y = A-hat X (conjA = false, Y is l x r) or Y = A-hat^H X (Y is m x r)
// The packed bf16 copies of Q and Z are written by the products that form them unless the
// environment variable RTSVD_PACK_FUSION is "0" (then every pass packs its X; the results are the
// same bits either way, the variable exists to compare the two).
static bool pack_fusion_enabled() {
  const char* e = std::getenv("RTSVD_PACK_FUSION");
  return !(e && std::strcmp(e, "0") == 0);
}

// xpk: X already packed (see orthonormalize), or null
template <typename TA, typename TX, typename TY>
static int big_gemm(bool conjA, const TA* Ah, int64_t l, int64_t m, const TX* X, int64_t r, TY* Y, int64_t F,
                    Scratch& sc, hipStream_t s, int ktag = 0, const void* xpk = nullptr) {
  if (!conjA)
    return skinny<TA, TX, TY>(false, l, r, m, Ah, l, l * m, X, m, m * r, Y, l, l * r, F, sc, s, ktag, 0, sk::PackOut(), xpk);
  return skinny<TA, TX, TY>(true, m, r, l, Ah, l, l * m, X, l, l * r, Y, m, m * r, F, sc, s, ktag, 0, sk::PackOut(), xpk);
}

// ---------------------------------------------------------------------------------------------
// R-tSVD factor (Alg. 6, block form) and the T-tSVD comparator (Alg. 1)
// ---------------------------------------------------------------------------------------------
// k x k leading block of every face's r x r matrix (column-major), packed to k x k
__global__ void k_lead_block(const zd* __restrict__ G, int r, int k, int F, zd* __restrict__ Gk) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (int64_t)F * k * k) return;
  const int i = (int)(idx % k), j = (int)((idx / k) % k);
  const int64_t f = idx / ((int64_t)k * k);
  Gk[idx] = G[f * r * r + i + (int64_t)j * r];
}

// T-tEVD ordering (Alg. 2, step 3): per face, the eigenpairs (lam descending from the eigensolver,
// eigenvectors Ve) re-ordered by decreasing |lam| (ties: the eigensolver's order).  Outputs in
// that order: sigma = |lam| (0 at or below tol_rel |lam|_max), s2 = sigma^2, V = the eigenvectors,
// U = V diag(sign lam) in the work type, so that V diag(1/sigma) U^H = V diag(1/lam) V^H.
// One block per face, r <= blockDim.
template <typename TU>
__global__ void __launch_bounds__(256)
k_tevd_sort(const double* __restrict__ lam, const zd* __restrict__ Ve, int r, double tol_rel,
            double* __restrict__ sigma, double* __restrict__ s2, zd* __restrict__ V, TU* __restrict__ U) {
  __shared__ int pos[256];
  __shared__ double sgn[256];
  const int f = blockIdx.x;
  const double* lf = lam + (int64_t)f * r;
  double amax = 0.0;
  for (int i = 0; i < r; ++i) amax = fmax(amax, fabs(lf[i]));
  for (int j = threadIdx.x; j < r; j += blockDim.x) {
    const double a = fabs(lf[j]);
    int rank = 0;
    for (int i = 0; i < r; ++i) {
      const double b = fabs(lf[i]);
      rank += (b > a || (b == a && i < j)) ? 1 : 0;
    }
    pos[j] = rank;
    sgn[j] = lf[j] < 0.0 ? -1.0 : 1.0;
    const double sv = a > tol_rel * amax ? a : 0.0;
    sigma[(int64_t)f * r + rank] = sv;
    s2[(int64_t)f * r + rank] = sv * sv;
  }
  __syncthreads();
  const int64_t base = (int64_t)f * r * r;
  for (int64_t idx = threadIdx.x; idx < (int64_t)r * r; idx += blockDim.x) {
    const int i = (int)(idx % r), j = (int)(idx / r);
    const zd v = Ve[base + idx];
    const int64_t o = base + (int64_t)pos[j] * r + i;
    V[o] = v;
    st(U[o], cscale(v, sgn[j]));
  }
}

// ---------------------------------------------------------------------------------------------
// face groups: the per-face part of the R-tSVD factor split over concurrent streams
// ---------------------------------------------------------------------------------------------
// After the tube DFTs every face is independent up to the scalar prefix sums of eta.  The small
// per-face kernels (Cholesky, eigensolver, Gram) run one workgroup per face and leave most compute
// units idle, so the faces are split into groups whose sketch / QR / projection / small SVD / W
// sequences run on separate streams: one group's bandwidth- and MFMA-bound passes overlap another
// group's latency-bound small-matrix work.

// Arrays of the factor over all faces; a group works on its own face range of each.
template <typename Tw>
struct FaceBufs {
  cplx<Tw>* Ah;
  zb* Ah16;
  cplx<Tw>* Omh;   // Omega-hat, m x r per face (read only)
  cplx<Tw>* Y;     // three work buffers with per-face stride l*r (l >= m)
  cplx<Tw>* tmp;
  cplx<Tw>* Z;
  zd* G;           // r x r per face
  zd* Rinv;
  uint16_t* Xpk;   // packed bf16 Q or Z for the next pass over A-hat (null: each pass packs its X)
  cplx<Tw>* Ch;    // m x r per face, in the work type: the projection accumulates in the MFMA's
                   // own precision (FP32 for the FP32 and bf16 passes), so its values are
                   // exactly representable there, and the FP64 Gram and V products read half the bytes
  zd* Ub;
  zd* Ubs;
  double* lam;
  double* sigma;
  zd* V;
  cplx<Tw>* W;
  int* flags;
};

// sketch, q power iterations, CholeskyQR, projection C^H = A-hat^H Q and G = C C^H for faces
// [f0, f0 + Fg), as a sequence of phases (so that several face groups can be issued phase by
// phase, interleaved).  Phase 0: sketch; 1: QR of Y; then per power iteration Z = A-hat^H Y, QR
// of Z, Y = A-hat Z, QR of Y; then projection and G.  Q ends in one of the work buffers
// (per-face stride l*r).  mark (or NULL) is recorded after phase 0.
template <typename Tw>
struct QcGroup {
  typedef cplx<Tw> zw;
  const FaceBufs<Tw>* fb;
  int64_t l, m, r, f0, Fg;
  int q;
  bool bf16;
  Scratch* sc;
  hipStream_t s;
  hipEvent_t mark;
  zw *Y, *tmp, *Z;
  uint16_t* xpk = nullptr;   // this group's part of fb->Xpk
  bool packed = false;       // xpk holds the X of the next pass over A-hat
  int phases() const { return 2 + 4 * q + 1; }
  void init() {
    Y = fb->Y + f0 * l * r;
    tmp = fb->tmp + f0 * l * r;
    Z = fb->Z + f0 * l * r;
    if (fb->Xpk) xpk = fb->Xpk + f0 * sk::bf16_pack_plan((int)r, (int)l, 1).out.sf;
  }
  int qr(zw*& W, int64_t rows, int passes, zd* G, zd* Rinv) {
    return orthonormalize<zw>(W, rows, r, Fg, passes, G, Rinv, tmp, fb->flags, *sc, s, bf16 ? xpk : nullptr, &packed);
  }
  // X's packed copy is used (and consumed) when the QR that formed X wrote one
  const void* take_packed() {
    const void* p = packed ? (const void*)xpk : nullptr;
    packed = false;
    return p;
  }
  int product(bool conjA, const zw* X, zw* Out, const void* xp = nullptr) {
    const zw* Ah = fb->Ah + f0 * l * m;
    const zb* Ah16 = fb->Ah16 ? fb->Ah16 + f0 * l * m : nullptr;
    if (bf16) return big_gemm<zb, zw, zw>(conjA, Ah16, l, m, X, r, Out, Fg, *sc, s, 0, xp);
    return big_gemm<zw, zw, zw>(conjA, Ah, l, m, X, r, Out, Fg, *sc, s);
  }
  int run(int ph) {
    zd* G = fb->G + f0 * r * r;
    zd* Rinv = fb->Rinv + f0 * r * r;
    if (ph == 0) {
      {
        RT_TIMED(RTSVD_T_SKETCH);
        RT_TRY(product(false, fb->Omh + f0 * m * r, Y));
      }
      if (mark) RT_CHECK_HIP(hipEventRecord(mark, s));
      return 0;
    }
    if (ph == 1) return qr(Y, l, q == 0 ? 2 : 1, G, Rinv);
    if (ph < 2 + 4 * q) {
      const int it = (ph - 2) / 4, k = (ph - 2) % 4;
      if (k == 0) {
        RT_TIMED(RTSVD_T_POWER);
        return product(true, Y, Z, take_packed());
      }
      if (k == 1) return qr(Z, m, 1, G, Rinv);
      if (k == 2) {
        RT_TIMED(RTSVD_T_SKETCH);
        return product(false, Z, Y, take_packed());
      }
      return qr(Y, l, it == q - 1 ? 2 : 1, G, Rinv);
    }
    zw* Ch = fb->Ch + f0 * m * r;
    {
      RT_TIMED(RTSVD_T_PROJECT);
      RT_TRY(product(true, Y, Ch, take_packed()));
    }
    RT_TIMED(RTSVD_T_SVDAUX);
    // small SVD of C through G = C C^H = U-breve diag(sigma^2) U-breve^H (FP64)
    return gram<zw>(Ch, m, r, Fg, G, *sc, s);
  }
};

// small SVD and W for faces [f0, f0 + Fg) keeping rk <= r columns: eigendecomposition of Gsrc
// (rk x rk per face), sigma, V = C^H U-breve diag(1/sigma), W = A-hat V.  phase: 0 eigensolver,
// 1 sigma and V, 2 W, -1 all three.
constexpr int SVD_PHASES = 3;
template <typename Tw>
static int rtsvd_faces_svd(const FaceBufs<Tw>& fb, int64_t l, int64_t m, int64_t r, int64_t rk, int64_t f0,
                           int64_t Fg, const zd* Gsrc, Scratch& sc, hipStream_t s, int phase = -1) {
  typedef cplx<Tw> zw;
  const zd* Gg = Gsrc + f0 * rk * rk;
  zd* Ub = fb.Ub + f0 * rk * rk;
  zd* Ubs = fb.Ubs + f0 * rk * rk;
  double* lam = fb.lam + f0 * rk;
  double* sigma = fb.sigma + f0 * rk;
  const zw* Ch = fb.Ch + f0 * m * r;
  zd* V = fb.V + f0 * m * rk;
  zw* W = fb.W + f0 * l * rk;
  const zw* Ah = fb.Ah + f0 * l * m;
  const double eig_tol = 4.0 * (double)r * 2.220446049250313e-16;
  if (phase < 0 || phase == 0) {
    RT_TIMED(RTSVD_T_HEEV);
    RT_TRY(launch_heev(Gg, (int)rk, Fg, Ub, lam, sc, s));
  }
  if (phase < 0 || phase == 1) {
    RT_TIMED(RTSVD_T_SVDAUX);
    hipLaunchKernelGGL(k_sqrt_eigs, dim3(nblocks(Fg * rk)), dim3(256), 0, s, (const double*)lam, sigma, (int)rk,
                       (int)Fg, eig_tol);
    RT_LAUNCH_OK();
    // V = C^H (U-breve diag(1/sigma)): the scaling goes on the r x r factor
    hipLaunchKernelGGL((k_scale_cols<zd, zd>), dim3(nblocks(Fg * rk * rk)), dim3(256), 0, s, (const zd*)Ub, Ubs,
                       (const double*)sigma, (int)rk, (int)rk, (int)Fg);
    RT_LAUNCH_OK();
    RT_TRY((skinny<zw, zd, zd, Scratch, sk::F64>(false, m, rk, rk, Ch, m, m * r, Ubs, rk, rk * rk, V, m, m * rk, Fg, sc,
                                                 s)));
  }
  // W = A-hat V: exact residuals of the discrepancy principle
  if (phase < 0 || phase == 2) {
    RT_TIMED(RTSVD_T_W);
    RT_TRY((big_gemm<zw, zd, zw>(false, Ah, l, m, V, rk, W, Fg, sc, s, RTSVD_T_W_MMA)));
  }
  return 0;
}

// Streams (default priority) and events of the face groups, one set per device; a mutex keeps the
// fork / join sequence of one call from interleaving with another host thread's.
// (At most 3 groups: with the caller's stream that is the 4 hardware queues a process gets by
// default; more streams than queues serialize.)
constexpr int MAX_FACE_GROUPS = 3;
struct FaceStreams {
  std::mutex mu;
  hipStream_t st[MAX_FACE_GROUPS] = {};
  hipEvent_t fork = nullptr;
  hipEvent_t start = nullptr;      // the caller's stream at entry (inputs ready)
  hipEvent_t omega_done = nullptr; // the tube DFT of Omega, run beside that of A
  hipEvent_t join[MAX_FACE_GROUPS] = {};
  hipEvent_t stagger[MAX_FACE_GROUPS] = {};
  hipEvent_t gram_done[MAX_FACE_GROUPS] = {};   // the group's G = C C^H is complete
};

static FaceStreams* face_streams(int groups) {
  static std::mutex mu;
  static std::map<int, FaceStreams*> per_dev;
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || groups > MAX_FACE_GROUPS) return nullptr;
  std::lock_guard<std::mutex> lk(mu);
  FaceStreams*& fs = per_dev[dev];
  if (!fs) {
    FaceStreams* n = new FaceStreams();
    bool ok = hipEventCreateWithFlags(&n->fork, hipEventDisableTiming) == hipSuccess &&
              hipEventCreateWithFlags(&n->start, hipEventDisableTiming) == hipSuccess &&
              hipEventCreateWithFlags(&n->omega_done, hipEventDisableTiming) == hipSuccess;
    for (int g = 0; ok && g < MAX_FACE_GROUPS; ++g)
      ok = hipStreamCreateWithFlags(&n->st[g], hipStreamNonBlocking) == hipSuccess &&
           hipEventCreateWithFlags(&n->join[g], hipEventDisableTiming) == hipSuccess &&
           hipEventCreateWithFlags(&n->stagger[g], hipEventDisableTiming) == hipSuccess &&
           hipEventCreateWithFlags(&n->gram_done[g], hipEventDisableTiming) == hipSuccess;
    if (!ok) return nullptr;   // (the partial set is kept alive: streams are never destroyed)
    fs = n;
  }
  return fs;
}

// number of face groups: `requested` (1..3) if given, else RTSVD_FACE_GROUPS (1..3) if set, else 3
// (at least 4 faces per group; measured at 65 faces: 1 group 4.36 ms, 2 groups 4.04 ms, 3 groups
// 3.95 ms per restoration)
static int face_groups(int64_t F, int requested) {
  static int env = -1;
  if (env < 0) {
    const char* e = std::getenv("RTSVD_FACE_GROUPS");
    const int v = e ? std::atoi(e) : 0;
    env = (v >= 1 && v <= MAX_FACE_GROUPS) ? v : 0;
  }
  const int g = requested > 0 ? requested : (env > 0 ? env : 3);
  return (int)std::max<int64_t>(1, std::min<int64_t>(g, F / 4));
}

static bool timers_on() {
  std::lock_guard<std::mutex> lk(g_timer.mu);
  return g_timer.on;
}

// adapt_eps > 0: the fixed-precision factor of Alg. 6 (keep the first r_eps sketch columns)

// error indicator eta^[j] (Thm 4.2) from the Gram matrices G_f = C_f C_f^H: ||C(j, :)||^2 is the
// real diagonal of G
static int eta_from_gram(const double* sumsq, int64_t nblk, const zd* G, int64_t F, int64_t r, int64_t n,
                         double* eta, hipStream_t s) {
  RT_TIMED(RTSVD_T_SVDAUX);
  hipLaunchKernelGGL(k_eta_prefix, dim3(1), dim3(DP_SEL_THREADS), 0, s, sumsq, nblk, (const double*)G,
                     (int64_t)2 * r * r, (int64_t)2 * (r + 1), (int)F, (int)r, (int)n, eta);
  return hipGetLastError() == hipSuccess ? 0 : -1;
}

// After the tube DFT of A: flag bit 1 when ||A||_F^2 is not finite (a NaN or infinite entry, or an
// overflowing norm) and, in that case only, zero A-hat so that the rest of the factor runs on the
// zero operator (outputs unspecified; rtsvd_factor_info and rtsvd_solve report RTSVD_E_NOTFINITE).
template <typename Tw>
static int finite_guard(const double* sumsq, int64_t nblk, int* flags, cplx<Tw>* Ah, int64_t count, zb* Ah16,
                        hipStream_t s) {
  hipLaunchKernelGGL(k_finite_check, dim3(1), dim3(FIN_THREADS), 0, s, sumsq, nblk, flags);
  if (hipGetLastError() != hipSuccess) return -1;
  if (launch_zero_if_nonfinite<cplx<Tw>>(Ah, count, flags, s)) return -1;
  return launch_zero_if_nonfinite<zb>(Ah16, count, flags, s);
}

template <typename Tin, typename Tw>
static int factor_impl(const Tin* A, const Tin* omega, uint64_t seed, int64_t l, int64_t m, int64_t n, int64_t r,
                       int precision, int q, rtsvd_factor_s* h, hipStream_t s, bool tsvd_mode, double adapt_eps = 0.0,
                       int groups_req = 0) {
  typedef cplx<Tw> zw;
  const int64_t F = n / 2 + 1;
  const bool bf16 = (precision == RTSVD_P_BF16);
  Scratch sc(s);
  if (ensure_solve_twiddles<Tw>((int)n, s)) return fail(RTSVD_E_HIP, "rtsvd_factor: twiddle tables");
  // face groups (R-tSVD, fixed rank, no stage timers): see rtsvd_faces_qc / QcGroup
  const int groups = (tsvd_mode || adapt_eps > 0.0 || timers_on()) ? 1 : face_groups(F, groups_req);
  FaceStreams* fs = nullptr;
  std::unique_lock<std::mutex> fs_lock;
  zw* Omh = nullptr;
  if (!tsvd_mode) {
    Omh = sc.get<zw>(F * m * r);
    if (!Omh) return fail(RTSVD_E_NOMEM, "device allocation failed: Omh");
  }
  // Gaussian tensor of the sketch: the caller's, or drawn on the device from `seed`
  Tin* omg = nullptr;
  if (!tsvd_mode && !omega) {
    omg = sc.get<Tin>(m * r * n);
    if (!omg) return fail(RTSVD_E_NOMEM, "device allocation failed: Gaussian tensor");
    omega = omg;
  }
  if (groups > 1) {
    fs = face_streams(groups);
    if (!fs) return fail(RTSVD_E_HIP, "rtsvd_factor: creating the face-group streams failed");
    fs_lock = std::unique_lock<std::mutex>(fs->mu);
    // the tube DFT of Omega on group 0's stream, beside that of A on the caller's stream
    RT_CHECK_HIP(hipEventRecord(fs->start, s));
    RT_CHECK_HIP(hipStreamWaitEvent(fs->st[0], fs->start, 0));
    if (omg) RT_TRY(launch_gaussian<Tin>(seed, m * r * n, omg, fs->st[0]));
    RT_TRY((launch_rfft<Tin, Tw>(omega, m * r, (int)n, Omh, m * r, (zb*)nullptr, (double*)nullptr, nullptr,
                                 fs->st[0])));
    RT_CHECK_HIP(hipEventRecord(fs->omega_done, fs->st[0]));
  }
  // tube DFT of A (half spectrum), ||A||_F^2 partial sums on the way
  RT_ALLOC(Ah, zw, F * l * m, sc);
  zb* Ah16 = nullptr;
  if (bf16) {
    Ah16 = sc.get<zb>(F * l * m);
    if (!Ah16) return fail(RTSVD_E_NOMEM, "device allocation failed: Ah16");
  }
  RT_ALLOC(sumsq, double, rfft_max_blocks(l * m), sc);
  RT_ALLOC(flags, int, 1, sc);
  hipLaunchKernelGGL(k_set_int, dim3(1), dim3(64), 0, s, flags, 0);
  RT_LAUNCH_OK();
  int64_t nblk = 0;
  {
    RT_TIMED(RTSVD_T_FFT_A);
    RT_TRY((launch_rfft<Tin, Tw>(A, l * m, (int)n, Ah, l * m, Ah16, sumsq, &nblk, s)));
  }
  RT_TRY(finite_guard(sumsq, nblk, flags, Ah, F * l * m, Ah16, s));

  // outputs owned by the handle
  zw* Qo = nullptr;  // Q (R-tSVD) or U (T-tSVD), l x r per face
  RT_ALLOC(sigma, double, F * r, sc);
  RT_ALLOC(V, zd, F * m * r, sc);
  RT_ALLOC(Wo, zw, F * l * r, sc);
  RT_ALLOC(eta, double, r + 1, sc);
  zd* Ub = nullptr;

  RT_ALLOC(G, zd, F * r * r, sc);
  RT_ALLOC(lam, double, F * r, sc);
  const double eig_tol = 4.0 * (double)r * 2.220446049250313e-16;

  if (!tsvd_mode) {
    Ub = sc.get<zd>(F * r * r);
    if (!Ub) return fail(RTSVD_E_NOMEM, "device allocation failed: Ub");
    RT_ALLOC(Rinv, zd, F * r * r, sc);
    RT_ALLOC(Y, zw, F * l * r, sc);     // per-face stride l*r (l >= m) in the three work buffers,
    RT_ALLOC(tmp, zw, F * l * r, sc);   // so that face groups own disjoint regions
    RT_ALLOC(Zb, zw, F * l * r, sc);
    RT_ALLOC(Ch, zw, F * m * r, sc);    // C^H = A-hat^H Q, m x r per face (C = Q^H A-hat)
    RT_ALLOC(Ubs, zd, F * r * r, sc);
    if (groups == 1) {
      RT_TIMED(RTSVD_T_FFT_OMEGA);
      if (omg) RT_TRY(launch_gaussian<Tin>(seed, m * r * n, omg, s));
      RT_TRY((launch_rfft<Tin, Tw>(omega, m * r, (int)n, Omh, m * r, (zb*)nullptr, (double*)nullptr, nullptr, s)));
    }
    // packed bf16 copies of Q and Z written by the products that form them (mixed precision,
    // l and m multiples of 128): per face the slab size of an l-row operand
    uint16_t* Xpk = nullptr;
    if (bf16 && pack_fusion_enabled() && sk::bf16_pack_plan((int)r, (int)l, 1).ok) {
      Xpk = sc.get<uint16_t>(F * sk::bf16_pack_plan((int)r, (int)l, 1).out.sf);
      if (!Xpk) return fail(RTSVD_E_NOMEM, "device allocation failed: packed operand of the passes");
    }
    FaceBufs<Tw> fb{Ah, Ah16, Omh, Y, tmp, Zb, G, Rinv, Xpk, Ch, Ub, Ubs, lam, sigma, V, Wo, flags};
    if (groups == 1) {
      QcGroup<Tw> qg{&fb, l, m, r, 0, F, q, bf16, &sc, s, nullptr};
      qg.init();
      for (int ph = 0; ph < qg.phases(); ++ph) RT_TRY(qg.run(ph));
      Qo = qg.Y;
    } else {
      // the face groups run concurrently on the library's streams, joined back into s; group g
      // starts once group g-1 has finished its first sketch, so that the groups stay out of phase
      // (one group's sketch / power / projection / W passes over A-hat overlap the other's
      // latency-bound Gram, Cholesky and eigensolver kernels instead of coinciding with them)
      RT_CHECK_HIP(hipEventRecord(fs->fork, s));
      std::vector<std::unique_ptr<Scratch>> scg;
      std::vector<QcGroup<Tw>> qg;
      for (int g = 0; g < groups; ++g) {
        const int64_t f0 = F * g / groups, Fg = F * (g + 1) / groups - f0;
        hipStream_t sg = fs->st[g];
        RT_CHECK_HIP(hipStreamWaitEvent(sg, fs->fork, 0));
        if (g > 0) RT_CHECK_HIP(hipStreamWaitEvent(sg, fs->omega_done, 0));
        scg.emplace_back(new Scratch(sg));
        qg.push_back(QcGroup<Tw>{&fb, l, m, r, f0, Fg, q, bf16, scg.back().get(), sg, fs->stagger[g]});
        qg.back().init();
      }
      // issued phase by phase across the groups, so that every stream has work queued early
      for (int ph = 0; ph < qg[0].phases() + SVD_PHASES; ++ph)
        for (int g = 0; g < groups; ++g) {
          if (ph == 0 && g > 0) RT_CHECK_HIP(hipStreamWaitEvent(qg[g].s, fs->stagger[g - 1], 0));
          if (ph < qg[g].phases()) {
            RT_TRY(qg[g].run(ph));
            if (ph == qg[g].phases() - 1) RT_CHECK_HIP(hipEventRecord(fs->gram_done[g], qg[g].s));
          } else {
            RT_TRY((rtsvd_faces_svd<Tw>(fb, l, m, r, r, qg[g].f0, qg[g].Fg, fb.G, *scg[g], qg[g].s,
                                        ph - qg[g].phases())));
          }
        }
      // the error indicator needs only the Gram matrices: s computes it while the groups still
      // run their eigensolvers and W passes, then joins them
      for (int g = 0; g < groups; ++g) RT_CHECK_HIP(hipStreamWaitEvent(s, fs->gram_done[g], 0));
      RT_TRY(eta_from_gram(sumsq, nblk, G, F, r, n, eta, s));
      for (int g = 0; g < groups; ++g) {
        RT_CHECK_HIP(hipEventRecord(fs->join[g], qg[g].s));
        RT_CHECK_HIP(hipStreamWaitEvent(s, fs->join[g], 0));
      }
      Qo = qg[0].Y;
    }
    if (groups == 1) RT_TRY(eta_from_gram(sumsq, nblk, G, F, r, n, eta, s));
    int64_t rr = r;
    if (groups == 1) {
      // fixed precision (Alg. 6): r_eps = first j >= 1 with eta^[j] < eps^2.  QR and the power
      // updates are nested, so the first r_eps columns of Q (and rows of C) are what the algorithm
      // builds from the first r_eps Gaussian columns; G's leading block is C_{r_eps} C_{r_eps}^H.
      zd* Gs = G;
      if (adapt_eps > 0.0) {
        std::vector<double> he((size_t)r + 1);
        RT_CHECK_HIP(hipMemcpyAsync(he.data(), eta, sizeof(double) * (r + 1), hipMemcpyDeviceToHost, s));
        RT_CHECK_HIP(hipStreamSynchronize(s));
        for (int64_t j = 1; j <= r; ++j)
          if (he[j] < adapt_eps * adapt_eps) { rr = j; break; }
        if (rr < r) {
          RT_ALLOC(Gk, zd, F * rr * rr, sc);
          hipLaunchKernelGGL(k_lead_block, dim3(nblocks(F * rr * rr)), dim3(256), 0, s, (const zd*)G, (int)r, (int)rr,
                             (int)F, Gk);
          RT_LAUNCH_OK();
          Gs = Gk;
          RT_ALLOC(Qk, zw, F * l * rr, sc);
          RT_CHECK_HIP(hipMemcpy2DAsync(Qk, sizeof(zw) * l * rr, Qo, sizeof(zw) * l * r, sizeof(zw) * l * rr, F,
                                        hipMemcpyDeviceToDevice, s));
          Qo = Qk;
        }
      }
      RT_TRY((rtsvd_faces_svd<Tw>(fb, l, m, r, rr, 0, F, Gs, sc, s)));
    }
    h->r = rr;
  } else {
    // full facewise SVD through G = A-hat^H A-hat = V diag(sigma^2) V^H; W = A-hat V; U = W diag(1/sigma)
    RT_TRY(gram<zw>(Ah, l, m, F, G, sc, s));
    RT_TRY(launch_heev(G, (int)m, F, V, lam, sc, s));
    hipLaunchKernelGGL(k_sqrt_eigs, dim3(nblocks(F * r)), dim3(256), 0, s, lam, sigma, (int)r, (int)F, eig_tol);
    RT_LAUNCH_OK();
    hipLaunchKernelGGL(k_eta_prefix, dim3(1), dim3(DP_SEL_THREADS), 0, s, sumsq, nblk, (const double*)lam, (int64_t)r,
                       (int64_t)1, (int)F, (int)r, (int)n, eta);
    RT_LAUNCH_OK();
    RT_TRY((big_gemm<zw, zd, zw>(false, Ah, l, m, V, r, Wo, F, sc, s)));
    RT_ALLOC(Uo, zw, F * l * r, sc);
    Qo = Uo;
    hipLaunchKernelGGL((k_scale_cols<zw, zw>), dim3(nblocks(F * l * r)), dim3(256), 0, s, Wo, Qo, sigma, (int)l,
                       (int)r, (int)F);
    RT_LAUNCH_OK();
  }
  h->Q = sc.release(Qo);
  h->Ub = Ub ? sc.release(Ub) : nullptr;
  h->sigma = sc.release(sigma);
  h->V = sc.release(V);
  h->W = sc.release(Wo);
  h->eta = sc.release(eta);
  h->flags = sc.release(flags);
  h->owned = {h->Q, h->sigma, h->V, h->W, h->eta, h->flags};
  if (h->Ub) h->owned.push_back(h->Ub);
  return 0;
}

static void free_handle(rtsvd_factor_s* h) {
  if (!h) return;
  for (void* p : h->owned) g_cache.release(p);
  delete h;
}

static int dispatch_factor(const void* A, const void* omega, uint64_t seed, int dtype, int64_t l, int64_t m,
                           int64_t n, int64_t r, int precision, int q, rtsvd_factor_s* h, hipStream_t s, bool tsvd,
                           double ae = 0.0, int groups = 0) {
  if (dtype == RTSVD_F64) {
    if (work_is_double(precision))
      return factor_impl<double, double>((const double*)A, (const double*)omega, seed, l, m, n, r, precision, q, h, s,
                                         tsvd, ae, groups);
    return factor_impl<double, float>((const double*)A, (const double*)omega, seed, l, m, n, r, precision, q, h, s,
                                      tsvd, ae, groups);
  }
  if (work_is_double(precision))
    return factor_impl<float, double>((const float*)A, (const float*)omega, seed, l, m, n, r, precision, q, h, s, tsvd,
                                      ae, groups);
  return factor_impl<float, float>((const float*)A, (const float*)omega, seed, l, m, n, r, precision, q, h, s, tsvd,
                                   ae, groups);
}

extern "C" int rtsvd_factor(const void* A, int64_t l, int64_t m, int64_t n, int dtype, const rtsvd_opts* opts,
                            void* stream, rtsvd_handle* out) {
  g_last_error.clear();
  if (!A || !opts || !out) return fail(RTSVD_E_ARG, "rtsvd_factor: null argument");
  *out = nullptr;
  if (dtype != RTSVD_F64 && dtype != RTSVD_F32) return fail(RTSVD_E_ARG, "rtsvd_factor: bad dtype");
  if (l < 1 || m < 1 || n < 1 || l < m) return fail(RTSVD_E_ARG, "rtsvd_factor: need l >= m >= 1 and n >= 1");
  const rtsvd_opts o = *opts;
  if (o.k_max < 1 || o.k_max > m || o.oversample < 0 || o.power_iters < 0)
    return fail(RTSVD_E_ARG, "rtsvd_factor: need 1 <= k_max <= m, oversample >= 0, power_iters >= 0");
  if (o.precision != RTSVD_P_FP64 && o.precision != RTSVD_P_FP32 && o.precision != RTSVD_P_BF16)
    return fail(RTSVD_E_ARG, "rtsvd_factor: bad precision");
  if (o.face_groups < 0 || o.face_groups > MAX_FACE_GROUPS)
    return fail(RTSVD_E_ARG, "rtsvd_factor: face_groups must be 0..3");
  if (o.sketch_tile != 0 && o.sketch_tile != 1 && o.sketch_tile != 2 && o.sketch_tile != 4 && o.sketch_tile != 8)
    return fail(RTSVD_E_ARG, "rtsvd_factor: sketch_tile must be 0, 1, 2, 4 or 8");
  sk::TileOverride tile_guard(o.sketch_tile);
  const int64_t r = std::min<int64_t>((int64_t)o.k_max + o.oversample, m);
  if (r > 256) return fail(RTSVD_E_UNSUPPORTED, "rtsvd_factor: r = min(k_max + oversample, m) must be <= 256");
  hipStream_t s = (hipStream_t)stream;
  rtsvd_factor_s* h = new rtsvd_factor_s();
  h->l = l; h->m = m; h->n = n; h->F = n / 2 + 1; h->r = r; h->dtype = dtype; h->precision = o.precision;
  h->kind = 0; h->k_max = o.k_max; h->oversample = o.oversample; h->eps = o.eps; h->stream = s;
  const double ae = (o.adaptive && o.eps > 0.0) ? o.eps : 0.0;
  const int rc = dispatch_factor(A, o.omega, o.seed, dtype, l, m, n, r, o.precision, o.power_iters, h, s, false, ae,
                                 o.face_groups);
  if (rc != 0) { delete h; return rc; }
  *out = h;
  return RTSVD_OK;
}

extern "C" int ttsvd_factor(const void* A, int64_t l, int64_t m, int64_t n, int dtype, int32_t precision,
                            int32_t k_max, void* stream, rtsvd_handle* out) {
  g_last_error.clear();
  if (!A || !out) return fail(RTSVD_E_ARG, "ttsvd_factor: null argument");
  *out = nullptr;
  if (dtype != RTSVD_F64 && dtype != RTSVD_F32) return fail(RTSVD_E_ARG, "ttsvd_factor: bad dtype");
  if (l < 1 || m < 1 || n < 1 || l < m) return fail(RTSVD_E_ARG, "ttsvd_factor: need l >= m >= 1 and n >= 1");
  if (k_max < 1 || k_max > m) return fail(RTSVD_E_ARG, "ttsvd_factor: need 1 <= k_max <= m");
  if (precision != RTSVD_P_FP64 && precision != RTSVD_P_FP32)
    return fail(RTSVD_E_ARG, "ttsvd_factor: precision must be FP64 or FP32");
  if (m > 256) return fail(RTSVD_E_UNSUPPORTED, "ttsvd_factor: m must be <= 256");
  hipStream_t s = (hipStream_t)stream;
  rtsvd_factor_s* h = new rtsvd_factor_s();
  h->l = l; h->m = m; h->n = n; h->F = n / 2 + 1; h->r = m; h->dtype = dtype; h->precision = precision;
  h->kind = 1; h->k_max = k_max; h->oversample = 0; h->stream = s;
  const int rc = dispatch_factor(A, nullptr, 0, dtype, l, m, n, m, precision, 0, h, s, true);
  if (rc != 0) { delete h; return rc; }
  *out = h;
  return RTSVD_OK;
}

// T-tEVD factor of a symmetric A (Alg. 2): facewise Hermitian eigendecomposition of A-hat_i (its
// lower triangle, FP64), eigenpairs by decreasing |lambda|, stored as the SVD
// A-hat_i = (V sign(lambda)) |lambda| V^H so that the solve and the discrepancy principle are the
// T-tSVD ones; W = A-hat V for the exact residuals.
template <typename Tin, typename Tw>
static int tevd_impl(const Tin* A, int64_t m, int64_t n, rtsvd_factor_s* h, hipStream_t s) {
  typedef cplx<Tw> zw;
  const int64_t F = n / 2 + 1, r = m;
  Scratch sc(s);
  if (ensure_solve_twiddles<Tw>((int)n, s)) return fail(RTSVD_E_HIP, "ttevd_factor: twiddle tables");
  RT_ALLOC(Ah, zw, F * m * m, sc);
  RT_ALLOC(sumsq, double, rfft_max_blocks(m * m), sc);
  RT_ALLOC(flags, int, 1, sc);
  hipLaunchKernelGGL(k_set_int, dim3(1), dim3(64), 0, s, flags, 0);
  RT_LAUNCH_OK();
  int64_t nblk = 0;
  {
    RT_TIMED(RTSVD_T_FFT_A);
    RT_TRY((launch_rfft<Tin, Tw>(A, m * m, (int)n, Ah, m * m, (zb*)nullptr, sumsq, &nblk, s)));
  }
  RT_TRY(finite_guard<Tw>(sumsq, nblk, flags, Ah, F * m * m, (zb*)nullptr, s));
  RT_ALLOC(sigma, double, F * r, sc);
  RT_ALLOC(s2, double, F * r, sc);
  RT_ALLOC(V, zd, F * m * r, sc);
  RT_ALLOC(Uo, zw, F * m * r, sc);
  RT_ALLOC(Wo, zw, F * m * r, sc);
  RT_ALLOC(eta, double, r + 1, sc);
  RT_ALLOC(G, zd, F * m * m, sc);
  RT_ALLOC(Ve, zd, F * m * m, sc);
  RT_ALLOC(lam, double, F * r, sc);
  {
    RT_TIMED(RTSVD_T_HEEV);
    hipLaunchKernelGGL((k_convert<zw, zd>), dim3(nblocks(F * m * m)), dim3(256), 0, s, (const zw*)Ah, G, F * m * m);
    RT_LAUNCH_OK();
    RT_TRY(launch_heev(G, (int)m, F, Ve, lam, sc, s));
  }
  const double eig_tol = 4.0 * (double)r * 2.220446049250313e-16;
  hipLaunchKernelGGL((k_tevd_sort<zw>), dim3((unsigned)F), dim3(256), 0, s, (const double*)lam, (const zd*)Ve, (int)r,
                     eig_tol, sigma, s2, V, Uo);
  RT_LAUNCH_OK();
  hipLaunchKernelGGL(k_eta_prefix, dim3(1), dim3(DP_SEL_THREADS), 0, s, sumsq, nblk, (const double*)s2, (int64_t)r,
                     (int64_t)1, (int)F, (int)r, (int)n, eta);
  RT_LAUNCH_OK();
  {
    RT_TIMED(RTSVD_T_W);
    RT_TRY((big_gemm<zw, zd, zw>(false, Ah, m, m, V, r, Wo, F, sc, s)));
  }
  h->Q = sc.release(Uo);
  h->Ub = nullptr;
  h->sigma = sc.release(sigma);
  h->V = sc.release(V);
  h->W = sc.release(Wo);
  h->eta = sc.release(eta);
  h->flags = sc.release(flags);
  h->owned = {h->Q, h->sigma, h->V, h->W, h->eta, h->flags};
  return 0;
}

extern "C" int ttevd_factor(const void* A, int64_t m, int64_t n, int dtype, int32_t precision, int32_t k_max,
                            void* stream, rtsvd_handle* out) {
  g_last_error.clear();
  if (!A || !out) return fail(RTSVD_E_ARG, "ttevd_factor: null argument");
  *out = nullptr;
  if (dtype != RTSVD_F64 && dtype != RTSVD_F32) return fail(RTSVD_E_ARG, "ttevd_factor: bad dtype");
  if (m < 1 || n < 1) return fail(RTSVD_E_ARG, "ttevd_factor: need m >= 1 and n >= 1");
  if (k_max < 1 || k_max > m) return fail(RTSVD_E_ARG, "ttevd_factor: need 1 <= k_max <= m");
  if (precision != RTSVD_P_FP64 && precision != RTSVD_P_FP32)
    return fail(RTSVD_E_ARG, "ttevd_factor: precision must be FP64 or FP32");
  if (m > 256) return fail(RTSVD_E_UNSUPPORTED, "ttevd_factor: m must be <= 256");
  hipStream_t s = (hipStream_t)stream;
  rtsvd_factor_s* h = new rtsvd_factor_s();
  h->l = m; h->m = m; h->n = n; h->F = n / 2 + 1; h->r = m; h->dtype = dtype; h->precision = precision;
  h->kind = 2; h->k_max = k_max; h->oversample = 0; h->stream = s;
  int rc;
  if (dtype == RTSVD_F64)
    rc = work_is_double(precision) ? tevd_impl<double, double>((const double*)A, m, n, h, s)
                                   : tevd_impl<double, float>((const double*)A, m, n, h, s);
  else
    rc = work_is_double(precision) ? tevd_impl<float, double>((const float*)A, m, n, h, s)
                                   : tevd_impl<float, float>((const float*)A, m, n, h, s);
  if (rc != 0) { delete h; return rc; }
  *out = h;
  return RTSVD_OK;
}

extern "C" void rtsvd_factor_destroy(rtsvd_handle f) { free_handle(f); }

extern "C" int rtsvd_trim(void) {
  g_last_error.clear();
  if (g_cache.trim() != 0) return fail(RTSVD_E_HIP, "rtsvd_trim: releasing cached device memory failed");
  return RTSVD_OK;
}

extern "C" int rtsvd_factor_info(rtsvd_handle f, int32_t* r, int32_t* faces, double* eta, int32_t* r_eps,
                                 double* sigma, int32_t* flags) {
  g_last_error.clear();
  if (!f) return fail(RTSVD_E_ARG, "rtsvd_factor_info: null handle");
  if (r) *r = (int32_t)f->r;
  if (faces) *faces = (int32_t)f->F;
  std::vector<double> e(f->r + 1);
  RT_CHECK_HIP(hipMemcpyAsync(e.data(), f->eta, sizeof(double) * (f->r + 1), hipMemcpyDeviceToHost, f->stream));
  int fl = 0;
  RT_CHECK_HIP(hipMemcpyAsync(&fl, f->flags, sizeof(int), hipMemcpyDeviceToHost, f->stream));
  if (sigma)
    RT_CHECK_HIP(hipMemcpyAsync(sigma, f->sigma, sizeof(double) * f->r * f->F, hipMemcpyDeviceToHost, f->stream));
  RT_CHECK_HIP(hipStreamSynchronize(f->stream));
  if (eta) std::copy(e.begin(), e.end(), eta);
  if (flags) *flags = fl;
  if (r_eps) {
    // Alg. 6 tests eta after each new column: the first j >= 1 (as the fixed-precision factor uses)
    *r_eps = -1;
    if (f->eps > 0.0)
      for (int64_t j = 1; j <= f->r; ++j)
        if (e[j] < f->eps * f->eps) { *r_eps = (int32_t)j; break; }
  }
  if (fl & 2) return fail(RTSVD_E_NOTFINITE, "rtsvd_factor_info: A is not finite (||A||_F^2 overflowed or is NaN)");
  return (fl & 1) ? RTSVD_W_RANK_DEFICIENT : RTSVD_OK;
}

// ---------------------------------------------------------------------------------------------
// solve: coefficients, discrepancy principle, truncated solution, inverse DFT
// ---------------------------------------------------------------------------------------------
// Relative numerical-rank cutoff of the truncated pseudo-inverse: singular values at or below
// sqrt(4 r eps) sigma_max (eps = 2^-52) are taken as zero -- the accuracy floor of singular values
// obtained from the eigenvalues of C C^H (the eigensolver's relative cutoff 4 r eps, squared).
static double pinv_rel(int64_t r) { return std::sqrt(4.0 * (double)r * 2.220446049250313e-16); }

// Device scratch of one solve, in the order solve_impl requests it (each slice 256-byte aligned).
// right-hand sides above which the solve's products run on MFMA (k_skinny) instead of the
// matrix-vector kernels
constexpr int SOLVE_MFMA_P = GEMV_NP;
// columns of B summed per residual partial (joint principle)
static int dp_cols_per_block(int groups, int64_t p) { return (groups == 1 && p >= 8) ? 8 : 1; }

static size_t solve_scratch_bytes(const rtsvd_factor_s* h, int64_t p, int groups, int kcap) {
  const bool dbl = work_is_double(h->precision);
  const size_t cw = dbl ? 16 : 8;
  const int64_t tiles = ceil_div(h->l, DP_ROWS);
  const int64_t pg = ceil_div(p, dp_cols_per_block(groups, p));
  const int l = (int)h->l, r = (int)h->r, F = (int)h->F;
  size_t b = Arena::round((size_t)(h->F * h->l * p) * cw);                 // B-hat
  b += 2 * Arena::round((size_t)(h->F * h->r * p) * 16);                   // D, T
  if (p > SOLVE_MFMA_P) {                                                  // packed operands of the products
    b += Arena::round((size_t)(dbl ? sk::skinny_ws_bytes<zd>(l, (int)p, F) : sk::skinny_ws_bytes<zf, sk::F64>(l, (int)p, F)));
    if (h->Ub) b += Arena::round((size_t)sk::skinny_ws_bytes<zd>(r, (int)p, F));
  }
  b += Arena::round((size_t)(h->F * tiles * pg * kcap) * 8);               // residual partial sums
  if (groups > 16) b += Arena::round((size_t)groups * 8);                  // bounds in device memory
  b += Arena::round((size_t)groups * kcap * 8);                            // rho
  b += Arena::round((size_t)(h->F * h->m * p) * 16);                       // X-hat
  if (p > SOLVE_MFMA_P) b += Arena::round((size_t)sk::skinny_ws_bytes<zd>(r, (int)p, F));
  return b;
}

template <typename Tio, typename Tw, typename SC>
static int solve_impl(rtsvd_factor_s* h, const Tio* B, int64_t p, const std::vector<double>& bounds, int k_start,
                      int kcap, Tio* X, int* k_out, double* resid_out, int* status_out, hipStream_t s, SC& sc) {
  typedef cplx<Tw> zw;
  const int64_t l = h->l, m = h->m, n = h->n, F = h->F, r = h->r;
  const int groups = (int)bounds.size();
  RT_TIMED(RTSVD_T_SOLVE);
  RT_ALLOC(Bh, zw, F * l * p, sc);
  RT_TRY((launch_rfft<Tio, Tw>(B, l * p, (int)n, Bh, l * p, (zb*)nullptr, (double*)nullptr, nullptr, s)));
  RT_ALLOC(D, zd, F * r * p, sc);
  RT_ALLOC(T, zd, F * r * p, sc);
  // D = Q^H B-hat (T-tSVD: U^H B-hat); T = U-breve^H D.  Few right-hand sides: matrix-vector
  // kernels (one pass over Q, FP64 sums); more: FP64 MFMA products (FP32 Q and B-hat converted on
  // the way to the MFMA operands), so the sums are FP64 either way
  const bool mfma = p > SOLVE_MFMA_P;
  if (mfma)
    RT_TRY((skinny<zw, zw, zd, SC, sk::F64>(true, r, p, l, (const zw*)h->Q, l, l * r, Bh, l, l * p, h->Ub ? D : T,
                                            r, r * p, F, sc, s)));
  else
    RT_TRY((cgemm<zw, zw, zd, double>(true, false, (int)r, (int)p, (int)l, (const zw*)h->Q, l, l * r, Bh, l, l * p,
                                     h->Ub ? D : T, r, r * p, (int)F, 1.0, false, s)));
  if (h->Ub) {
    if (mfma)
      RT_TRY((skinny<zd, zd, zd, SC>(true, r, p, r, h->Ub, r, r * r, D, r, r * p, T, r, r * p, F, sc, s)));
    else
      RT_TRY((cgemm<zd, zd, zd, double>(true, false, (int)r, (int)p, (int)r, h->Ub, r, r * r, D, r, r * p, T, r,
                                       r * p, (int)F, 1.0, false, s)));
  }
  hipLaunchKernelGGL(k_scale_rows, dim3(nblocks(F * r * p)), dim3(256), 0, s, T, h->sigma, (int)r, (int)p, (int)F,
                     pinv_rel(r));
  RT_LAUNCH_OK();
  // residual norms for k = 1..kcap, then the first k meeting the principle
  const int tiles = (int)ceil_div(l, DP_ROWS);
  const int cpb = dp_cols_per_block(groups, p);
  const int64_t pg = ceil_div(p, cpb);
  RT_ALLOC(partial, double, F * tiles * pg * kcap, sc);
  if (cpb == 8)
    hipLaunchKernelGGL((k_dp_partial<8, zw, zw>), dim3((unsigned)tiles, (unsigned)pg, (unsigned)F), dim3(DP_ROWS), 0,
                       s, Bh, (const zw*)h->W, T, (int)l, (int)p, (int)r, kcap, partial);
  else
    hipLaunchKernelGGL((k_dp_partial<1, zw, zw>), dim3((unsigned)tiles, (unsigned)p, (unsigned)F), dim3(DP_ROWS), 0,
                       s, Bh, (const zw*)h->W, T, (int)l, (int)p, (int)r, kcap, partial);
  RT_LAUNCH_OK();
  // the bounds ride in the selection kernel's arguments for up to 16 groups, else in device memory
  Vals16 bnd_args = {};
  double* bnd = nullptr;
  if (groups <= 16) {
    for (int g = 0; g < groups; ++g) bnd_args.v[g] = bounds[g];
  } else {
    bnd = sc.template get<double>(groups);
    if (!bnd) return fail(RTSVD_E_NOMEM, "device allocation failed: bnd");
    RT_TRY(upload_doubles(bnd, bounds.data(), groups, s));
  }
  RT_ALLOC(rho_tmp, double, (int64_t)groups * kcap, sc);
  hipLaunchKernelGGL(k_dp_rho, dim3((unsigned)(groups * kcap)), dim3(DP_RHO_THREADS), 0, s, partial, (int)F, tiles,
                     (int)pg, kcap, (int)n, groups, resid_out, rho_tmp);
  RT_LAUNCH_OK();
  hipLaunchKernelGGL(k_dp_select, dim3(1), dim3(DP_SELECT_THREADS), 0, s, kcap, groups, (const double*)bnd, bnd_args,
                     k_start, (const double*)rho_tmp, (const int*)h->flags, k_out, status_out);
  RT_LAUNCH_OK();
  // X-hat = V T', T' = T with rows >= k zeroed; X = inverse DFT
  hipLaunchKernelGGL(k_mask_coeffs, dim3(nblocks(F * r * p)), dim3(256), 0, s, T, D, k_out, groups, (int)r, (int)p,
                     (int)F);
  RT_LAUNCH_OK();
  RT_ALLOC(Xh, zd, F * m * p, sc);
  if (mfma)
    RT_TRY((skinny<zd, zd, zd, SC>(false, m, p, r, h->V, m, m * r, D, r, r * p, Xh, m, m * p, F, sc, s)));
  else
    RT_TRY((cgemm<zd, zd, zd, double>(false, false, (int)m, (int)p, (int)r, h->V, m, m * r, D, r, r * p, Xh, m,
                                     m * p, (int)F, 1.0, false, s)));
  RT_TRY((launch_irfft<double, Tio>(Xh, m * p, m * p, (int)n, X, s)));
  return 0;
}

// argument checks, truncation range and bounds shared by rtsvd_solve and rtsvd_solve_noalloc
static int solve_setup(rtsvd_handle f, const void* B, int64_t p, int dtype, const double* delta, int32_t n_delta,
                       double eta_dp, int32_t k_start, const void* X, const int32_t* k_out, int* ks, int* kcap,
                       std::vector<double>& bounds) {
  if (!f || !B || !X || !delta || !k_out) return fail(RTSVD_E_ARG, "rtsvd_solve: null argument");
  if (p < 1) return fail(RTSVD_E_ARG, "rtsvd_solve: p must be >= 1");
  if (dtype != f->dtype) return fail(RTSVD_E_ARG, "rtsvd_solve: dtype differs from the factor's");
  if (n_delta != 1 && n_delta != p) return fail(RTSVD_E_ARG, "rtsvd_solve: n_delta must be 1 or p");
  if (!(eta_dp > 1.0)) return fail(RTSVD_E_ARG, "rtsvd_solve: eta_dp must be > 1");
  if (k_start < 0 || k_start > std::min<int64_t>(f->k_max, f->r))
    return fail(RTSVD_E_ARG, "rtsvd_solve: need 0 <= k_start <= min(k_max, r)");
  for (int i = 0; i < n_delta; ++i)
    if (!(delta[i] >= 0.0)) return fail(RTSVD_E_ARG, "rtsvd_solve: delta must be >= 0");
  *ks = k_start;
  *kcap = std::min<int>(f->k_max, (int)f->r);
  if (k_start == 0) {
    *ks = std::max<int>(1, (int)f->r - f->oversample);
    *kcap = (int)f->r;
  }
  bounds.resize(n_delta);
  for (int i = 0; i < n_delta; ++i) bounds[i] = eta_dp * delta[i];
  return 0;
}

template <typename SC>
static int solve_dispatch(rtsvd_handle f, const void* B, int64_t p, const std::vector<double>& bounds, int ks,
                          int kcap, void* X, int32_t* k_out, double* resid_out, int32_t* status_out, hipStream_t s,
                          SC& sc) {
  if (f->dtype == RTSVD_F64) {
    if (work_is_double(f->precision))
      return solve_impl<double, double>(f, (const double*)B, p, bounds, ks, kcap, (double*)X, k_out, resid_out,
                                        status_out, s, sc);
    return solve_impl<double, float>(f, (const double*)B, p, bounds, ks, kcap, (double*)X, k_out, resid_out,
                                     status_out, s, sc);
  }
  if (work_is_double(f->precision))
    return solve_impl<float, double>(f, (const float*)B, p, bounds, ks, kcap, (float*)X, k_out, resid_out, status_out,
                                     s, sc);
  return solve_impl<float, float>(f, (const float*)B, p, bounds, ks, kcap, (float*)X, k_out, resid_out, status_out, s,
                                  sc);
}

extern "C" int rtsvd_solve(rtsvd_handle f, const void* B, int64_t p, int dtype, const double* delta, int32_t n_delta,
                           double eta_dp, int32_t k_start, void* X, int32_t* k_out, double* resid_out,
                           int32_t* status_out, void* stream) {
  g_last_error.clear();
  int ks = 0, kcap = 0;
  std::vector<double> bounds;
  const int rc = solve_setup(f, B, p, dtype, delta, n_delta, eta_dp, k_start, X, k_out, &ks, &kcap, bounds);
  if (rc) return rc;
  hipStream_t s = (hipStream_t)stream;
  Scratch sc(s);
  return solve_dispatch(f, B, p, bounds, ks, kcap, X, k_out, resid_out, status_out, s, sc);
}

// ---------------------------------------------------------------------------------------------
// rtsvd_solve without device allocation: its scratch is a fixed device array of the library
// ---------------------------------------------------------------------------------------------
// `scratch` is a host-side stand-in for the array in host code; its device address is obtained
// once per device with hipGetSymbolAddress and used everywhere instead of the name.
constexpr size_t NOALLOC_SCRATCH_BYTES = (size_t)64 << 20;
static __device__ __align__(256) unsigned char scratch[NOALLOC_SCRATCH_BYTES];

constexpr int NOALLOC_MAX_DEVICES = 64;
static std::mutex g_noalloc_mu;
static unsigned char* g_noalloc_ptr[NOALLOC_MAX_DEVICES] = {};

// device address of this device's copy of `scratch` (looked up on the first call on the device)
static unsigned char* noalloc_scratch() {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= NOALLOC_MAX_DEVICES) return nullptr;
  std::lock_guard<std::mutex> lk(g_noalloc_mu);
  if (!g_noalloc_ptr[dev]) {
    void* ptr = nullptr;
    if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess || !ptr) {
      (void)hipGetLastError();
      return nullptr;
    }
    g_noalloc_ptr[dev] = static_cast<unsigned char*>(ptr);
  }
  return g_noalloc_ptr[dev];
}

extern "C" int rtsvd_solve_noalloc(rtsvd_handle f, const void* B, int64_t p, int dtype, const double* delta,
                                   int32_t n_delta, double eta_dp, int32_t k_start, void* X, int32_t* k_out,
                                   double* resid_out, int32_t* status_out, void* stream) {
  g_last_error.clear();
  int ks = 0, kcap = 0;
  std::vector<double> bounds;
  const int rc = solve_setup(f, B, p, dtype, delta, n_delta, eta_dp, k_start, X, k_out, &ks, &kcap, bounds);
  if (rc) return rc;
  const size_t need = solve_scratch_bytes(f, p, (int)bounds.size(), kcap);
  if (need > NOALLOC_SCRATCH_BYTES) {
    char buf[256];
    snprintf(buf, sizeof(buf), "rtsvd_solve_noalloc: the solve needs %zu bytes of scratch, above the %zu-byte "
             "maximum (use rtsvd_solve)", need, NOALLOC_SCRATCH_BYTES);
    return fail(RTSVD_E_UNSUPPORTED, buf);
  }
  Arena arena;
  arena.base = noalloc_scratch();
  if (!arena.base) return fail(RTSVD_E_HIP, "rtsvd_solve_noalloc: hipGetSymbolAddress of the scratch array failed");
  arena.cap = NOALLOC_SCRATCH_BYTES;
  TwiddleLookupOnly no_new_tables;   // the factor created every table this solve uses
  return solve_dispatch(f, B, p, bounds, ks, kcap, X, k_out, resid_out, status_out, (hipStream_t)stream, arena);
}

// ---------------------------------------------------------------------------------------------
// t-products
// ---------------------------------------------------------------------------------------------
template <typename T>
static int tprod_impl(const T* A, const T* Bin, T* Out, int64_t l, int64_t m, int64_t p, int64_t n, bool adjoint,
                      hipStream_t s) {
  typedef cplx<T> zt;
  const int64_t F = n / 2 + 1;
  Scratch sc(s);
  RT_ALLOC(Ah, zt, F * l * m, sc);
  RT_TRY((launch_rfft<T, T>(A, l * m, (int)n, Ah, l * m, (zb*)nullptr, (double*)nullptr, nullptr, s)));
  const int64_t rin = adjoint ? l : m, rout = adjoint ? m : l;
  RT_ALLOC(Bh, zt, F * rin * p, sc);
  RT_ALLOC(Ch, zt, F * rout * p, sc);
  RT_TRY((launch_rfft<T, T>(Bin, rin * p, (int)n, Bh, rin * p, (zb*)nullptr, (double*)nullptr, nullptr, s)));
  if (!adjoint)
    RT_TRY((cgemm<zt, zt, zt, T>(false, false, (int)l, (int)p, (int)m, Ah, l, l * m, Bh, m, m * p, Ch, l, l * p,
                                 (int)F, (T)1, false, s)));
  else
    RT_TRY((cgemm<zt, zt, zt, T>(true, false, (int)m, (int)p, (int)l, Ah, l, l * m, Bh, l, l * p, Ch, m, m * p,
                                 (int)F, (T)1, false, s)));
  RT_TRY((launch_irfft<T, T>(Ch, rout * p, rout * p, (int)n, Out, s)));
  return 0;
}

extern "C" int tprod(const void* A, const void* B, void* C, int64_t l, int64_t m, int64_t p, int64_t n, int dtype,
                     void* stream) {
  g_last_error.clear();
  if (!A || !B || !C) return fail(RTSVD_E_ARG, "tprod: null argument");
  if (l < 1 || m < 1 || p < 1 || n < 1) return fail(RTSVD_E_ARG, "tprod: sizes must be >= 1");
  hipStream_t s = (hipStream_t)stream;
  if (dtype == RTSVD_F64) return tprod_impl<double>((const double*)A, (const double*)B, (double*)C, l, m, p, n, false, s);
  if (dtype == RTSVD_F32) return tprod_impl<float>((const float*)A, (const float*)B, (float*)C, l, m, p, n, false, s);
  return fail(RTSVD_E_ARG, "tprod: bad dtype");
}

extern "C" int tprod_adjoint(const void* A, const void* C, void* B, int64_t l, int64_t m, int64_t p, int64_t n,
                             int dtype, void* stream) {
  g_last_error.clear();
  if (!A || !B || !C) return fail(RTSVD_E_ARG, "tprod_adjoint: null argument");
  if (l < 1 || m < 1 || p < 1 || n < 1) return fail(RTSVD_E_ARG, "tprod_adjoint: sizes must be >= 1");
  hipStream_t s = (hipStream_t)stream;
  if (dtype == RTSVD_F64) return tprod_impl<double>((const double*)A, (const double*)C, (double*)B, l, m, p, n, true, s);
  if (dtype == RTSVD_F32) return tprod_impl<float>((const float*)A, (const float*)C, (float*)B, l, m, p, n, true, s);
  return fail(RTSVD_E_ARG, "tprod_adjoint: bad dtype");
}


// ---------------------------------------------------------------------------------------------
// tGKB_p (Alg. 7 + projected least squares + discrepancy principle), the comparison baseline
// ---------------------------------------------------------------------------------------------
// One product of a step, A-hat^H X (conj) or A-hat X over every face, as FP64 partial vectors
// (face f, slice c of partial t at part + t*tStride + f*p*out_len + c*out_len) that
// k_gkb_orth sums; nparts / tStride describe them.  live: see k_gkb_orth.
template <typename T>
static int gkb_product(bool conj, const cplx<T>* Ah, int64_t l, int64_t m, int64_t p, const cplx<T>* X, int64_t ldx,
                       int64_t sX, zd* part, int64_t F, int* nparts, int64_t* tStride, const int* live,
                       hipStream_t s) {
  const int64_t out_len = conj ? m : l, sY = p * out_len;
  *nparts = 1;
  *tStride = 0;
  if (p <= 4) {
    if (conj && l * p * (int64_t)sizeof(cplx<T>) <= 65536) {
      hipLaunchKernelGGL((k_gv_c<T, 4>), dim3((unsigned)ceil_div(m, 4 * GVC_COLS), (unsigned)F), dim3(256),
                         (size_t)l * p * sizeof(cplx<T>), s, Ah, (int)l, (int)m, (int)p, X, ldx, sX, part, sY, live);
      return hipGetLastError() == hipSuccess ? 0 : -1;
    }
    if (!conj) {
      const int64_t nch0 = std::min<int64_t>(GVN_MAXCHUNK, ceil_div(m, 32));
      const int64_t kw = ceil_div(ceil_div(m, 4 * nch0), GVN_UNROLL) * GVN_UNROLL;
      const int64_t nch = ceil_div(m, 4 * kw);
      const size_t lds = 3 * 64 * 4 * sizeof(zd) + (size_t)(p * 4 * kw) * sizeof(cplx<T>);
      if (lds <= 65536) {
        hipLaunchKernelGGL((k_gv_n<T, 4>), dim3((unsigned)ceil_div(l, 64), (unsigned)nch, (unsigned)F), dim3(256), lds,
                           s, Ah, (int)l, (int)m, (int)p, X, ldx, sX, (int)kw, part, F * sY, sY, live);
        *nparts = (int)nch;
        *tStride = F * sY;
        return hipGetLastError() == hipSuccess ? 0 : -1;
      }
    }
  }
  if (!conj)
    return cgemm<cplx<T>, cplx<T>, zd, double>(false, false, (int)l, (int)p, (int)m, Ah, l, l * m, X, ldx, sX, part,
                                               out_len, sY, (int)F, 1.0, false, s);
  return cgemm<cplx<T>, cplx<T>, zd, double>(true, false, (int)m, (int)p, (int)l, Ah, l, l * m, X, ldx, sX, part,
                                             out_len, sY, (int)F, 1.0, false, s);
}

// FP64 elements of the partial-vector buffer gkb_product may fill
static int64_t gkb_part_elems(int64_t l, int64_t m, int64_t p, int64_t F) {
  return (p <= 4 ? GVN_MAXCHUNK : 1) * F * p * std::max(l, m);
}

// Progress words of the Krylov step loops: a ring of 64 words in coherent pinned host memory (one
// cache line each), a call tagged with a 16-bit id so that a word left by an earlier call is
// never read as this call's progress.
struct Progress {
  uint64_t* host = nullptr;
  uint64_t* dev = nullptr;
  uint32_t id = 0;
};
constexpr int PROG_RING = 64, PROG_STRIDE = 8;

static bool progress_open(Progress& pr) {
  static std::mutex mu;
  static uint64_t* ring = nullptr;
  static uint64_t* ring_dev = nullptr;
  static uint32_t next_id = 1;
  std::lock_guard<std::mutex> lk(mu);
  if (!ring) {
    uint64_t* h = nullptr;
    if (hipHostMalloc((void**)&h, sizeof(uint64_t) * PROG_RING * PROG_STRIDE,
                      hipHostMallocCoherent | hipHostMallocMapped) != hipSuccess)
      return false;
    uint64_t* d = nullptr;
    if (hipHostGetDevicePointer((void**)&d, h, 0) != hipSuccess) return false;
    ring = h;
    ring_dev = d;
  }
  uint32_t id = next_id++ & 0xffffu;
  if (id == 0) id = next_id++ & 0xffffu;   // a cleared word never carries a valid id
  const int slot = (int)(id % PROG_RING);
  pr.host = ring + slot * PROG_STRIDE;
  pr.dev = ring_dev + slot * PROG_STRIDE;
  pr.id = id;
  __atomic_store_n(pr.host, (uint64_t)0, __ATOMIC_RELEASE);
  return true;
}

// Throttle of the step loop after enqueueing step i: waits until the device has finished step
// i - ahead.  Returns 1 once every slice is decided, 0 to go on, -1 on a HIP error.  When the
// stream has drained without a matching word, the device counter is read directly.
static int await_progress(const Progress& pr, int i, int ahead, const int* remaining_dev, hipStream_t s) {
  for (long spin = 1;; ++spin) {
    const uint64_t w = __atomic_load_n(pr.host, __ATOMIC_ACQUIRE);
    if ((uint32_t)(w >> 48) == pr.id) {
      const int done = (int)((w >> 32) & 0xffff), rem = (int)(uint32_t)w;
      if (done >= 1 && rem <= 0) return 1;
      if (done >= i - ahead) return 0;
    } else if (i - ahead <= 0) {
      return 0;
    }
    if ((spin & 1023) == 0) {
      const hipError_t q = hipStreamQuery(s);
      if (q == hipErrorNotReady) continue;
      if (q != hipSuccess) return -1;
      int rem = 0;
      if (hipMemcpy(&rem, remaining_dev, sizeof(int), hipMemcpyDeviceToHost) != hipSuccess) return -1;
      return rem <= 0 ? 1 : 0;
    }
    __builtin_ia32_pause();
  }
}

// steps in flight beyond the last one known to be finished
constexpr int KRYLOV_AHEAD = 2;

// Tikhonov variants (tGKT_p, t-LanczosTik_p): mu interval, outputs and the scratch the tail fills
struct TikArgs {
  double mu_lo, mu_hi;
  double* mu_out;    // DEVICE [p]
  double* res_out;   // DEVICE [p] or NULL: ||B_c - A * X_c|| at mu
  double* y;         // scratch: F x p x kmax coefficients (filled by tikhonov_tail)
  int* fail;         // scratch: mu_hi could not meet a bound
};

// mu by bisection and the coefficients y of every (face, slice) from the Givens QR histories of the
// step loop (k_tik_mu); allocates tik.y and tik.fail from sc
template <bool LANCZOS>
static int tikhonov_tail(const double* ha, const double* hb, const double* hc, const double* phi, const double* beta,
                         const int* kin, int kmax, int64_t p, int64_t F, int64_t n, const double* bnd, TikArgs& tik,
                         Scratch& sc, hipStream_t s) {
  tik.y = sc.get<double>(F * p * kmax);
  tik.fail = sc.get<int>(1);
  if (!tik.y || !tik.fail) return fail(RTSVD_E_NOMEM, "device allocation failed: Tikhonov scratch");
  hipLaunchKernelGGL(k_set_int, dim3(1), dim3(64), 0, s, tik.fail, 0);
  RT_LAUNCH_OK();
  // 4 k_max doubles of LDS per thread, at most 150 KB per workgroup
  const int nt = (int)std::max<int64_t>(1, std::min<int64_t>(TIK_MAX_THREADS, (150 * 1024) / (32 * (int64_t)kmax)));
  const size_t lds = (size_t)nt * 4 * kmax * sizeof(double);
  auto kern = k_tik_mu<LANCZOS>;
  if (lds > 65536) RT_CHECK_HIP(hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize,
                                                    (int)lds));
  hipLaunchKernelGGL(kern, dim3((unsigned)p), dim3(nt), lds, s, ha, hb, hc, phi, beta, kin, kmax, (int)p, (int)F,
                     (int)n, bnd, tik.mu_lo, tik.mu_hi, tik.mu_out, tik.res_out, tik.y, tik.fail);
  RT_LAUNCH_OK();
  return 0;
}

template <typename T>
static int tgkb_impl(const T* A, const T* B, int64_t l, int64_t m, int64_t n, int64_t p,
                     const std::vector<double>& bounds, int kmax, T* X, int* k_out, double* resid_out, int* status_out,
                     hipStream_t s, TikArgs* tik = nullptr) {
  typedef cplx<T> zt;
  const int64_t F = n / 2 + 1;
  const double tol = 64.0 * (sizeof(T) == 8 ? 1.1102230246251565e-16 : 5.960464477539063e-08);
  Scratch sc(s);
  RT_TIMED(RTSVD_T_TGKB);
  RT_ALLOC(Ah, zt, F * l * m, sc);
  RT_ALLOC(Bh, zt, F * l * p, sc);
  RT_TRY((launch_rfft<T, T>(A, l * m, (int)n, Ah, l * m, (zb*)nullptr, (double*)nullptr, nullptr, s)));
  RT_TRY((launch_rfft<T, T>(B, l * p, (int)n, Bh, l * p, (zb*)nullptr, (double*)nullptr, nullptr, s)));
  const int64_t ldq = l * (kmax + 1), ldw = m * kmax;
  RT_ALLOC(Qb, zt, F * p * ldq, sc);
  RT_ALLOC(Wb, zt, F * p * ldw, sc);
  RT_ALLOC(raw, zd, gkb_part_elems(l, m, p, F), sc);
  int nparts = 1;
  int64_t tstr = 0;
  const int64_t cnt = F * p;
  RT_ALLOC(zc, double, cnt, sc);
  RT_ALLOC(cc, double, cnt, sc);
  RT_ALLOC(cprev, double, cnt, sc);
  RT_ALLOC(phibar, double, cnt, sc);
  RT_ALLOC(rho_h, double, cnt * kmax, sc);
  RT_ALLOC(s_h, double, cnt * kmax, sc);
  RT_ALLOC(phi_h, double, cnt * kmax, sc);
  RT_ALLOC(alpha_h, double, cnt * kmax, sc);
  RT_ALLOC(bnd, double, p, sc);
  RT_ALLOC(remaining, int, 1, sc);
  RT_ALLOC(kin, int, p, sc);
  RT_TRY(upload_doubles(bnd, bounds.data(), p, s));
  RT_CHECK_HIP(hipMemsetAsync(kin, 0, sizeof(int) * p, s));
  hipLaunchKernelGGL(k_set_int, dim3(1), dim3(64), 0, s, remaining, (int)p);
  RT_LAUNCH_OK();
  if (resid_out) RT_CHECK_HIP(hipMemsetAsync(resid_out, 0, sizeof(double) * p * kmax, s));
  hipLaunchKernelGGL((k_gkb_init<T>), dim3((unsigned)p, (unsigned)F), dim3(256), 0, s, Bh, l * p, (int)l, (int)p, Qb,
                     ldq, zc, phibar, cprev, 0.0);
  RT_LAUNCH_OK();
  double* beta = nullptr;   // ||b-hat|| per (face, slice), for the Tikhonov residuals
  if (tik) {
    beta = sc.get<double>(cnt);
    if (!beta) return fail(RTSVD_E_NOMEM, "device allocation failed: beta");
    RT_CHECK_HIP(hipMemcpyAsync(beta, phibar, sizeof(double) * cnt, hipMemcpyDeviceToDevice, s));
  }
  Progress prog;
  if (!progress_open(prog)) return fail(RTSVD_E_NOMEM, "tgkb_solve: pinned host memory");
  for (int i = 1; i <= kmax; ++i) {
    // w = A-hat^H q_i - z_i w_{i-1}, re-orthogonalized, c_i = ||w||
    RT_TRY(gkb_product<T>(true, Ah, l, m, p, Qb + (int64_t)(i - 1) * l, ldq, p * ldq, raw, F, &nparts, &tstr, remaining,
                          s));
    {
      const size_t lds = 32 * sizeof(double) + (size_t)(kmax + 1) * sizeof(zd) + (size_t)m * sizeof(zd);
      hipLaunchKernelGGL((k_gkb_orth<T, 0>), dim3((unsigned)p, (unsigned)F), dim3(GKB_THREADS), lds, s, (const zd*)raw,
                         nparts, tstr, p * m, Wb, ldw, (int)m, i - 1, (const zt*)(i >= 2 ? Wb : nullptr), ldw, i - 2,
                         (const double*)zc, cc, (int)p, tol, GkbRot{}, (const int*)remaining);
      RT_LAUNCH_OK();
    }
    // q = A-hat w_i - c_i q_i, re-orthogonalized, z_{i+1} = ||q||; Givens rotation i
    RT_TRY(gkb_product<T>(false, Ah, l, m, p, Wb + (int64_t)(i - 1) * m, ldw, p * ldw, raw, F, &nparts, &tstr, remaining,
                          s));
    {
      const size_t lds = 32 * sizeof(double) + (size_t)(kmax + 1) * sizeof(zd) + (size_t)l * sizeof(zd);
      const GkbRot rot{cc, cprev, rho_h, s_h, alpha_h, phibar, phi_h, nullptr, nullptr, nullptr, 0, kmax, i};
      hipLaunchKernelGGL((k_gkb_orth<T, 1>), dim3((unsigned)p, (unsigned)F), dim3(GKB_THREADS), lds, s, (const zd*)raw,
                         nparts, tstr, p * l, Qb, ldq, (int)l, i, (const zt*)Qb, ldq, i - 1, (const double*)cc, zc,
                         (int)p, tol, rot, (const int*)remaining);
      RT_LAUNCH_OK();
    }
    hipLaunchKernelGGL(k_gkb_dp, dim3(1), dim3(1024), 0, s, phibar, (int)F, (int)p, (int)n, bnd, i, kmax, kin,
                       resid_out, remaining, prog.dev, prog.id);
    RT_LAUNCH_OK();
    if (i < kmax) {
      const int r = await_progress(prog, i, KRYLOV_AHEAD, remaining, s);
      if (r < 0) return fail(RTSVD_E_HIP, "tgkb_solve: stream error while waiting for progress");
      if (r > 0) break;
    }
  }
  // solution at each slice's k (k_max where the principle was not met)
  RT_ALLOC(Xh, zt, F * m * p, sc);
  if (tik) {
    RT_TRY(tikhonov_tail<false>(rho_h, s_h, alpha_h, phi_h, beta, kin, kmax, p, F, n, bnd, *tik, sc, s));
    hipLaunchKernelGGL((k_basis_solution<T>), dim3((unsigned)p, (unsigned)F), dim3(256), 0, s, (const zt*)Wb, ldw,
                       (int)m, (const int*)kin, kmax, (int)p, (const double*)tik->y, Xh);
  } else {
    hipLaunchKernelGGL((k_gkb_solution<T>), dim3((unsigned)p, (unsigned)F), dim3(256), (size_t)kmax * sizeof(double),
                       s, Wb, ldw, (int)m, kin, kmax, (int)p, rho_h, s_h, phi_h, alpha_h, Xh);
  }
  RT_LAUNCH_OK();
  RT_TRY((launch_irfft<T, T>(Xh, m * p, m * p, (int)n, X, s)));
  if (tik)
    hipLaunchKernelGGL(k_tik_finish, dim3(1), dim3(64), 0, s, kin, (int)p, kmax, (const int*)tik->fail, k_out,
                       status_out);
  else
    hipLaunchKernelGGL(k_gkb_finish, dim3(1), dim3(64), 0, s, kin, (int)p, kmax, k_out, status_out);
  RT_LAUNCH_OK();
  return 0;
}

extern "C" int tgkb_solve(const void* A, const void* B, int64_t l, int64_t m, int64_t n, int64_t p, int dtype,
                          const double* delta, int32_t n_delta, double eta_dp, int32_t k_max, void* X, int32_t* k_out,
                          double* resid_out, int32_t* status_out, void* stream) {
  g_last_error.clear();
  if (!A || !B || !X || !delta || !k_out) return fail(RTSVD_E_ARG, "tgkb_solve: null argument");
  if (l < 1 || m < 1 || n < 1 || p < 1 || l < m) return fail(RTSVD_E_ARG, "tgkb_solve: need l >= m >= 1, n >= 1, p >= 1");
  if (k_max < 1 || k_max > m) return fail(RTSVD_E_ARG, "tgkb_solve: need 1 <= k_max <= m");
  if (n_delta != 1 && n_delta != p) return fail(RTSVD_E_ARG, "tgkb_solve: n_delta must be 1 or p");
  if (!(eta_dp > 1.0)) return fail(RTSVD_E_ARG, "tgkb_solve: eta_dp must be > 1");
  if (l > 8192) return fail(RTSVD_E_UNSUPPORTED, "tgkb_solve: l must be <= 8192");
  std::vector<double> bounds(p);
  for (int64_t c = 0; c < p; ++c) {
    const double d = delta[n_delta == 1 ? 0 : c];
    if (!(d >= 0.0)) return fail(RTSVD_E_ARG, "tgkb_solve: delta must be >= 0");
    bounds[c] = eta_dp * d;
  }
  hipStream_t s = (hipStream_t)stream;
  if (dtype == RTSVD_F64)
    return tgkb_impl<double>((const double*)A, (const double*)B, l, m, n, p, bounds, k_max, (double*)X, k_out, resid_out,
                             status_out, s);
  if (dtype == RTSVD_F32)
    return tgkb_impl<float>((const float*)A, (const float*)B, l, m, n, p, bounds, k_max, (float*)X, k_out, resid_out,
                            status_out, s);
  return fail(RTSVD_E_ARG, "tgkb_solve: bad dtype");
}

// shared argument checks of the Krylov entry points: bounds eta_dp * delta per slice
static int krylov_bounds(const char* who, const double* delta, int32_t n_delta, int64_t p, double eta_dp,
                         std::vector<double>& bounds) {
  char buf[160];
  if (n_delta != 1 && n_delta != p) {
    snprintf(buf, sizeof(buf), "%s: n_delta must be 1 or p", who);
    return fail(RTSVD_E_ARG, buf);
  }
  if (!(eta_dp > 1.0)) {
    snprintf(buf, sizeof(buf), "%s: eta_dp must be > 1", who);
    return fail(RTSVD_E_ARG, buf);
  }
  bounds.resize(p);
  for (int64_t c = 0; c < p; ++c) {
    const double d = delta[n_delta == 1 ? 0 : c];
    if (!(d >= 0.0)) {
      snprintf(buf, sizeof(buf), "%s: delta must be >= 0", who);
      return fail(RTSVD_E_ARG, buf);
    }
    bounds[c] = eta_dp * d;
  }
  return 0;
}

extern "C" int tgkt_solve(const void* A, const void* B, int64_t l, int64_t m, int64_t n, int64_t p, int dtype,
                          const double* delta, int32_t n_delta, double eta_dp, int32_t k_max, double mu_lo,
                          double mu_hi, void* X, int32_t* k_out, double* mu_out, double* resid_out,
                          int32_t* status_out, void* stream) {
  g_last_error.clear();
  if (!A || !B || !X || !delta || !k_out || !mu_out) return fail(RTSVD_E_ARG, "tgkt_solve: null argument");
  if (l < 1 || m < 1 || n < 1 || p < 1 || l < m) return fail(RTSVD_E_ARG, "tgkt_solve: need l >= m >= 1, n >= 1, p >= 1");
  if (k_max < 1 || k_max > m) return fail(RTSVD_E_ARG, "tgkt_solve: need 1 <= k_max <= m");
  if (!(mu_lo > 0.0) || !(mu_hi > mu_lo) || !std::isfinite(mu_hi))
    return fail(RTSVD_E_ARG, "tgkt_solve: need 0 < mu_lo < mu_hi < inf");
  if (l > 8192) return fail(RTSVD_E_UNSUPPORTED, "tgkt_solve: l must be <= 8192");
  std::vector<double> bounds;
  RT_TRY(krylov_bounds("tgkt_solve", delta, n_delta, p, eta_dp, bounds));
  hipStream_t s = (hipStream_t)stream;
  TikArgs tik{mu_lo, mu_hi, mu_out, resid_out, nullptr, nullptr};
  if (dtype == RTSVD_F64)
    return tgkb_impl<double>((const double*)A, (const double*)B, l, m, n, p, bounds, k_max, (double*)X, k_out, nullptr,
                             status_out, s, &tik);
  if (dtype == RTSVD_F32)
    return tgkb_impl<float>((const float*)A, (const float*)B, l, m, n, p, bounds, k_max, (float*)X, k_out, nullptr,
                            status_out, s, &tik);
  return fail(RTSVD_E_ARG, "tgkt_solve: bad dtype");
}

// ---------------------------------------------------------------------------------------------
// nested_tGKB_p (Alg. 8): the basis of Alg. 7 started from B_1 serves every lateral slice
// ---------------------------------------------------------------------------------------------
template <typename T>
static int nested_tgkb_impl(const T* A, const T* B, int64_t l, int64_t m, int64_t n, int64_t p,
                            const std::vector<double>& bounds, int kmax, int kinit, T* X, int* k_out, double* resid_out,
                            int* status_out, hipStream_t s, TikArgs* tik = nullptr) {
  typedef cplx<T> zt;
  const int64_t F = n / 2 + 1;
  const double tol = 64.0 * (sizeof(T) == 8 ? 1.1102230246251565e-16 : 5.960464477539063e-08);
  Scratch sc(s);
  RT_TIMED(RTSVD_T_NESTED);
  RT_ALLOC(Ah, zt, F * l * m, sc);
  RT_ALLOC(Bh, zt, F * l * p, sc);
  RT_TRY((launch_rfft<T, T>(A, l * m, (int)n, Ah, l * m, (zb*)nullptr, (double*)nullptr, nullptr, s)));
  RT_TRY((launch_rfft<T, T>(B, l * p, (int)n, Bh, l * p, (zb*)nullptr, (double*)nullptr, nullptr, s)));
  const int64_t ldq = l * (kmax + 1), ldw = m * kmax;
  RT_ALLOC(Qb, zt, F * ldq, sc);
  RT_ALLOC(Wb, zt, F * ldw, sc);
  RT_ALLOC(raw, zd, gkb_part_elems(l, m, 1, F), sc);
  int nparts = 1;
  int64_t tstr = 0;
  RT_ALLOC(zc, double, F, sc);
  RT_ALLOC(cc, double, F, sc);
  RT_ALLOC(cprev, double, F, sc);
  RT_ALLOC(phib0, double, F, sc);          // the basis' own right-hand side (unused by the slices)
  RT_ALLOC(rho_h, double, F * kmax, sc);
  RT_ALLOC(s_h, double, F * kmax, sc);
  RT_ALLOC(alpha_h, double, F * kmax, sc);
  RT_ALLOC(phibar, zd, F * p, sc);
  RT_ALLOC(phi_h, zd, F * p * kmax, sc);
  RT_ALLOC(res, double, p * kmax, sc);
  RT_ALLOC(bnd, double, p, sc);
  RT_ALLOC(kin, int, p, sc);
  RT_ALLOC(st, int, 4, sc);
  RT_ALLOC(remaining, int, 1, sc);
  RT_TRY(upload_doubles(bnd, bounds.data(), p, s));
  RT_CHECK_HIP(hipMemsetAsync(res, 0, sizeof(double) * p * kmax, s));
  hipLaunchKernelGGL(k_nest_reset, dim3(1), dim3(64), 0, s, st, kinit, remaining, (int)p);
  RT_LAUNCH_OK();
  // q_1 = b-hat_1 / ||b-hat_1|| per face, then phi-bar_1 = q_1^H b-hat_j for every slice
  hipLaunchKernelGGL((k_gkb_init<T>), dim3(1, (unsigned)F), dim3(256), 0, s, Bh, l * p, (int)l, 1, Qb, ldq, zc, phib0,
                     cprev, 0.0);
  RT_LAUNCH_OK();
  hipLaunchKernelGGL((k_nest_init<T>), dim3((unsigned)ceil_div(p, NEST_WAVES), (unsigned)F), dim3(64 * NEST_WAVES), 0,
                     s, Qb, ldq, Bh, (int)l, (int)p, phibar);
  RT_LAUNCH_OK();
  Progress prog;
  if (!progress_open(prog)) return fail(RTSVD_E_NOMEM, "nested_tgkb_solve: pinned host memory");
  for (int i = 1; i <= kmax; ++i) {
    RT_TRY(gkb_product<T>(true, Ah, l, m, 1, Qb + (int64_t)(i - 1) * l, ldq, ldq, raw, F, &nparts, &tstr, remaining, s));
    {
      const size_t lds = 32 * sizeof(double) + (size_t)(kmax + 1) * sizeof(zd) + (size_t)m * sizeof(zd);
      hipLaunchKernelGGL((k_gkb_orth<T, 0>), dim3(1, (unsigned)F), dim3(GKB_THREADS), lds, s, (const zd*)raw, nparts,
                         tstr, m, Wb, ldw, (int)m, i - 1, (const zt*)(i >= 2 ? Wb : nullptr), ldw, i - 2,
                         (const double*)zc, cc, 1, tol, GkbRot{}, (const int*)remaining);
      RT_LAUNCH_OK();
    }
    RT_TRY(gkb_product<T>(false, Ah, l, m, 1, Wb + (int64_t)(i - 1) * m, ldw, ldw, raw, F, &nparts, &tstr, remaining, s));
    {
      const size_t lds = 32 * sizeof(double) + (size_t)(kmax + 1) * sizeof(zd) + (size_t)l * sizeof(zd);
      // rotation i of every face and every slice's right-hand side update, in the same kernel
      const GkbRot rot{cc, cprev, rho_h, s_h, alpha_h, nullptr, nullptr, Bh, phibar, phi_h, (int)p, kmax, i};
      hipLaunchKernelGGL((k_gkb_orth<T, 2>), dim3(1, (unsigned)F), dim3(GKB_THREADS), lds, s, (const zd*)raw, nparts,
                         tstr, l, Qb, ldq, (int)l, i, (const zt*)Qb, ldq, i - 1, (const double*)cc, zc, 1, tol, rot,
                         (const int*)remaining);
      RT_LAUNCH_OK();
    }
    hipLaunchKernelGGL(k_nest_dp, dim3(1), dim3(256), 0, s, (const zd*)phibar, (int)F, (int)p, (int)n, bnd, i, kmax,
                       res, kin, st, remaining, prog.dev, prog.id);
    RT_LAUNCH_OK();
    if (i < kmax) {
      const int r = await_progress(prog, i, KRYLOV_AHEAD, remaining, s);
      if (r < 0) return fail(RTSVD_E_HIP, "nested_tgkb_solve: stream error while waiting for progress");
      if (r > 0) break;
    }
  }
  RT_ALLOC(Xh, zt, F * m * p, sc);
  if (tik) {
    // nested_tGKT_p: mu per slice by bisection on the nested space, X = W_k y (complex y)
    RT_ALLOC(ytik, zd, F * p * kmax, sc);
    RT_ALLOC(tfail, int, 1, sc);
    hipLaunchKernelGGL(k_set_int, dim3(1), dim3(64), 0, s, tfail, 0);
    RT_LAUNCH_OK();
    const int nt = (int)std::max<int64_t>(1, std::min<int64_t>(TIK_MAX_THREADS, (150 * 1024) / (40 * (int64_t)kmax)));
    const size_t lds = (size_t)nt * 5 * kmax * sizeof(double);
    if (lds > 65536)
      RT_CHECK_HIP(hipFuncSetAttribute((const void*)k_nest_tik_mu, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
    hipLaunchKernelGGL(k_nest_tik_mu, dim3((unsigned)p), dim3(nt), lds, s, (const double*)rho_h, (const double*)s_h,
                       (const double*)alpha_h, (const zd*)phi_h, (const double*)res, (const int*)kin, kmax, (int)p,
                       (int)F, (int)n, (const double*)bnd, tik->mu_lo, tik->mu_hi, tik->mu_out, tik->res_out, ytik,
                       tfail);
    RT_LAUNCH_OK();
    hipLaunchKernelGGL((k_nest_tik_solution<T>), dim3((unsigned)p, (unsigned)F), dim3(256), 0, s, (const zt*)Wb, ldw,
                       (int)m, (const int*)kin, kmax, (int)p, (const zd*)ytik, Xh);
    RT_LAUNCH_OK();
    RT_TRY((launch_irfft<T, T>(Xh, m * p, m * p, (int)n, X, s)));
    hipLaunchKernelGGL(k_nest_tik_finish, dim3(1), dim3(256), 0, s, (const int*)kin, (const int*)st,
                       (const int*)tfail, (int)p, k_out, status_out);
    RT_LAUNCH_OK();
    return 0;
  }
  hipLaunchKernelGGL((k_nest_solution<T>), dim3((unsigned)p, (unsigned)F), dim3(256), (size_t)kmax * sizeof(zd), s, Wb,
                     ldw, (int)m, kin, kmax, (int)p, rho_h, s_h, alpha_h, (const zd*)phi_h, Xh);
  RT_LAUNCH_OK();
  RT_TRY((launch_irfft<T, T>(Xh, m * p, m * p, (int)n, X, s)));
  hipLaunchKernelGGL(k_nest_finish, dim3(1), dim3(256), 0, s, kin, st, (int)p, k_out, status_out);
  RT_LAUNCH_OK();
  if (resid_out)
    RT_CHECK_HIP(hipMemcpyAsync(resid_out, res, sizeof(double) * p * kmax, hipMemcpyDeviceToDevice, s));
  return 0;
}

extern "C" int nested_tgkb_solve(const void* A, const void* B, int64_t l, int64_t m, int64_t n, int64_t p, int dtype,
                                 const double* delta, int32_t n_delta, double eta_dp, int32_t k_max, int32_t k_init,
                                 void* X, int32_t* k_out, double* resid_out, int32_t* status_out, void* stream) {
  g_last_error.clear();
  if (!A || !B || !X || !delta || !k_out) return fail(RTSVD_E_ARG, "nested_tgkb_solve: null argument");
  if (l < 1 || m < 1 || n < 1 || p < 1 || l < m)
    return fail(RTSVD_E_ARG, "nested_tgkb_solve: need l >= m >= 1, n >= 1, p >= 1");
  if (k_max < 1 || k_max > m) return fail(RTSVD_E_ARG, "nested_tgkb_solve: need 1 <= k_max <= m");
  if (k_init < 1) return fail(RTSVD_E_ARG, "nested_tgkb_solve: need k_init >= 1");
  if (n_delta != 1 && n_delta != p) return fail(RTSVD_E_ARG, "nested_tgkb_solve: n_delta must be 1 or p");
  if (!(eta_dp > 1.0)) return fail(RTSVD_E_ARG, "nested_tgkb_solve: eta_dp must be > 1");
  if (l > 8192) return fail(RTSVD_E_UNSUPPORTED, "nested_tgkb_solve: l must be <= 8192");
  std::vector<double> bounds(p);
  for (int64_t c = 0; c < p; ++c) {
    const double d = delta[n_delta == 1 ? 0 : c];
    if (!(d >= 0.0)) return fail(RTSVD_E_ARG, "nested_tgkb_solve: delta must be >= 0");
    bounds[c] = eta_dp * d;
  }
  const int kin = std::min<int>(k_init, k_max);
  hipStream_t s = (hipStream_t)stream;
  if (dtype == RTSVD_F64)
    return nested_tgkb_impl<double>((const double*)A, (const double*)B, l, m, n, p, bounds, k_max, kin, (double*)X,
                                    k_out, resid_out, status_out, s);
  if (dtype == RTSVD_F32)
    return nested_tgkb_impl<float>((const float*)A, (const float*)B, l, m, n, p, bounds, k_max, kin, (float*)X, k_out,
                                   resid_out, status_out, s);
  return fail(RTSVD_E_ARG, "nested_tgkb_solve: bad dtype");
}

extern "C" int nested_tgkt_solve(const void* A, const void* B, int64_t l, int64_t m, int64_t n, int64_t p, int dtype,
                                 const double* delta, int32_t n_delta, double eta_dp, int32_t k_max, int32_t k_init,
                                 double mu_lo, double mu_hi, void* X, int32_t* k_out, double* mu_out,
                                 double* resid_out, int32_t* status_out, void* stream) {
  g_last_error.clear();
  if (!A || !B || !X || !delta || !k_out || !mu_out) return fail(RTSVD_E_ARG, "nested_tgkt_solve: null argument");
  if (l < 1 || m < 1 || n < 1 || p < 1 || l < m)
    return fail(RTSVD_E_ARG, "nested_tgkt_solve: need l >= m >= 1, n >= 1, p >= 1");
  if (k_max < 1 || k_max > m) return fail(RTSVD_E_ARG, "nested_tgkt_solve: need 1 <= k_max <= m");
  if (k_init < 1) return fail(RTSVD_E_ARG, "nested_tgkt_solve: need k_init >= 1");
  if (!(mu_lo > 0.0) || !(mu_hi > mu_lo) || !std::isfinite(mu_hi))
    return fail(RTSVD_E_ARG, "nested_tgkt_solve: need 0 < mu_lo < mu_hi < inf");
  if (l > 8192) return fail(RTSVD_E_UNSUPPORTED, "nested_tgkt_solve: l must be <= 8192");
  std::vector<double> bounds;
  RT_TRY(krylov_bounds("nested_tgkt_solve", delta, n_delta, p, eta_dp, bounds));
  hipStream_t s = (hipStream_t)stream;
  TikArgs tik{mu_lo, mu_hi, mu_out, resid_out, nullptr, nullptr};
  const int kinit = std::min<int>(k_init, k_max);
  if (dtype == RTSVD_F64)
    return nested_tgkb_impl<double>((const double*)A, (const double*)B, l, m, n, p, bounds, k_max, kinit, (double*)X,
                                    k_out, nullptr, status_out, s, &tik);
  if (dtype == RTSVD_F32)
    return nested_tgkb_impl<float>((const float*)A, (const float*)B, l, m, n, p, bounds, k_max, kinit, (float*)X,
                                   k_out, nullptr, status_out, s, &tik);
  return fail(RTSVD_E_ARG, "nested_tgkt_solve: bad dtype");
}

// ---------------------------------------------------------------------------------------------
// t-Lanczos_p (Alg. 4 with full re-orthogonalization, eq. (9t)) for a symmetric A
// ---------------------------------------------------------------------------------------------
template <typename T>
static int tlanczos_impl(const T* A, const T* B, int64_t m, int64_t n, int64_t p, const std::vector<double>& bounds,
                         int kmax, T* X, int* k_out, double* resid_out, int* status_out, hipStream_t s,
                         TikArgs* tik = nullptr) {
  typedef cplx<T> zt;
  const int64_t F = n / 2 + 1;
  const double tol = 64.0 * (sizeof(T) == 8 ? 1.1102230246251565e-16 : 5.960464477539063e-08);
  Scratch sc(s);
  RT_TIMED(RTSVD_T_TLANCZOS);
  RT_ALLOC(Ah, zt, F * m * m, sc);
  RT_ALLOC(Bh, zt, F * m * p, sc);
  RT_TRY((launch_rfft<T, T>(A, m * m, (int)n, Ah, m * m, (zb*)nullptr, (double*)nullptr, nullptr, s)));
  RT_TRY((launch_rfft<T, T>(B, m * p, (int)n, Bh, m * p, (zb*)nullptr, (double*)nullptr, nullptr, s)));
  const int64_t ldq = m * (kmax + 1), cnt = F * p;
  RT_ALLOC(Qb, zt, F * p * ldq, sc);
  RT_ALLOC(raw, zd, gkb_part_elems(m, m, p, F), sc);
  int nparts = 1;
  int64_t tstr = 0;
  RT_ALLOC(zc, double, cnt, sc);
  RT_ALLOC(cprev, double, cnt, sc);
  RT_ALLOC(phibar, double, cnt, sc);
  RT_ALLOC(rot4, double, 4 * cnt, sc);     // rotations i-1 and i-2: cosines, sines
  RT_ALLOC(rho_h, double, cnt * kmax, sc);
  RT_ALLOC(r1_h, double, cnt * kmax, sc);
  RT_ALLOC(r2_h, double, cnt * kmax, sc);
  RT_ALLOC(phi_h, double, cnt * kmax, sc);
  RT_ALLOC(bnd, double, p, sc);
  RT_ALLOC(remaining, int, 1, sc);
  RT_ALLOC(kin, int, p, sc);
  RT_TRY(upload_doubles(bnd, bounds.data(), p, s));
  RT_CHECK_HIP(hipMemsetAsync(kin, 0, sizeof(int) * p, s));
  hipLaunchKernelGGL(k_set_int, dim3(1), dim3(64), 0, s, remaining, (int)p);
  RT_LAUNCH_OK();
  if (resid_out) RT_CHECK_HIP(hipMemsetAsync(resid_out, 0, sizeof(double) * p * kmax, s));
  // q_1 = b-hat / ||b-hat||, z_0, phi-bar = z_0; cprev (set to -1) seeds both rotation states
  hipLaunchKernelGGL((k_gkb_init<T>), dim3((unsigned)p, (unsigned)F), dim3(256), 0, s, Bh, m * p, (int)m, (int)p, Qb,
                     ldq, zc, phibar, cprev, 0.0);
  RT_LAUNCH_OK();
  double* beta = nullptr;   // ||b-hat|| per (face, slice), for the Tikhonov residuals
  if (tik) {
    beta = sc.get<double>(cnt);
    if (!beta) return fail(RTSVD_E_NOMEM, "device allocation failed: beta");
    RT_CHECK_HIP(hipMemcpyAsync(beta, phibar, sizeof(double) * cnt, hipMemcpyDeviceToDevice, s));
  }
  double* l1c = rot4;
  double* l1s = rot4 + cnt;
  double* l2c = rot4 + 2 * cnt;
  double* l2s = rot4 + 3 * cnt;
  RT_CHECK_HIP(hipMemcpyAsync(l1c, cprev, sizeof(double) * cnt, hipMemcpyDeviceToDevice, s));
  RT_CHECK_HIP(hipMemcpyAsync(l2c, cprev, sizeof(double) * cnt, hipMemcpyDeviceToDevice, s));
  RT_CHECK_HIP(hipMemsetAsync(l1s, 0, sizeof(double) * cnt, s));
  RT_CHECK_HIP(hipMemsetAsync(l2s, 0, sizeof(double) * cnt, s));
  Progress prog;
  if (!progress_open(prog)) return fail(RTSVD_E_NOMEM, "tlanczos_solve: pinned host memory");
  for (int i = 1; i <= kmax; ++i) {
    // v = A-hat q_i; c_i, v - z_{i-1} q_{i-1} - c_i q_i, re-orthogonalized, z_i; QR update of T-bar_i
    RT_TRY(gkb_product<T>(false, Ah, m, m, p, Qb + (int64_t)(i - 1) * m, ldq, p * ldq, raw, F, &nparts, &tstr, remaining,
                          s));
    {
      const size_t lds = 32 * sizeof(double) + (size_t)(kmax + 1) * sizeof(zd) + (size_t)m * sizeof(zd);
      GkbRot rot{nullptr, nullptr, rho_h, nullptr, nullptr, phibar, phi_h, nullptr, nullptr, nullptr, 0, kmax, i,
                 l1c, l1s, l2c, l2s, r1_h, r2_h};
      hipLaunchKernelGGL((k_gkb_orth<T, 3>), dim3((unsigned)p, (unsigned)F), dim3(GKB_THREADS), lds, s, (const zd*)raw,
                         nparts, tstr, p * m, Qb, ldq, (int)m, i, (const zt*)(i >= 2 ? Qb : nullptr), ldq, i - 2,
                         (const double*)(i >= 2 ? zc : nullptr), zc, (int)p, tol, rot, (const int*)remaining);
      RT_LAUNCH_OK();
    }
    hipLaunchKernelGGL(k_gkb_dp, dim3(1), dim3(1024), 0, s, phibar, (int)F, (int)p, (int)n, bnd, i, kmax, kin,
                       resid_out, remaining, prog.dev, prog.id);
    RT_LAUNCH_OK();
    if (i < kmax) {
      const int r = await_progress(prog, i, KRYLOV_AHEAD, remaining, s);
      if (r < 0) return fail(RTSVD_E_HIP, "tlanczos_solve: stream error while waiting for progress");
      if (r > 0) break;
    }
  }
  RT_ALLOC(Xh, zt, F * m * p, sc);
  if (tik) {
    RT_TRY(tikhonov_tail<true>(rho_h, r1_h, r2_h, phi_h, beta, kin, kmax, p, F, n, bnd, *tik, sc, s));
    hipLaunchKernelGGL((k_basis_solution<T>), dim3((unsigned)p, (unsigned)F), dim3(256), 0, s, (const zt*)Qb, ldq,
                       (int)m, (const int*)kin, kmax, (int)p, (const double*)tik->y, Xh);
  } else {
    hipLaunchKernelGGL((k_tlan_solution<T>), dim3((unsigned)p, (unsigned)F), dim3(256), (size_t)kmax * sizeof(double),
                       s, Qb, ldq, (int)m, kin, kmax, (int)p, rho_h, r1_h, r2_h, phi_h, Xh);
  }
  RT_LAUNCH_OK();
  RT_TRY((launch_irfft<T, T>(Xh, m * p, m * p, (int)n, X, s)));
  if (tik)
    hipLaunchKernelGGL(k_tik_finish, dim3(1), dim3(64), 0, s, kin, (int)p, kmax, (const int*)tik->fail, k_out,
                       status_out);
  else
    hipLaunchKernelGGL(k_gkb_finish, dim3(1), dim3(64), 0, s, kin, (int)p, kmax, k_out, status_out);
  RT_LAUNCH_OK();
  return 0;
}

extern "C" int tlanczos_solve(const void* A, const void* B, int64_t m, int64_t n, int64_t p, int dtype,
                              const double* delta, int32_t n_delta, double eta_dp, int32_t k_max, void* X,
                              int32_t* k_out, double* resid_out, int32_t* status_out, void* stream) {
  g_last_error.clear();
  if (!A || !B || !X || !delta || !k_out) return fail(RTSVD_E_ARG, "tlanczos_solve: null argument");
  if (m < 1 || n < 1 || p < 1) return fail(RTSVD_E_ARG, "tlanczos_solve: need m >= 1, n >= 1, p >= 1");
  if (k_max < 1 || k_max > m) return fail(RTSVD_E_ARG, "tlanczos_solve: need 1 <= k_max <= m");
  if (n_delta != 1 && n_delta != p) return fail(RTSVD_E_ARG, "tlanczos_solve: n_delta must be 1 or p");
  if (!(eta_dp > 1.0)) return fail(RTSVD_E_ARG, "tlanczos_solve: eta_dp must be > 1");
  if (m > 8192) return fail(RTSVD_E_UNSUPPORTED, "tlanczos_solve: m must be <= 8192");
  std::vector<double> bounds(p);
  for (int64_t c = 0; c < p; ++c) {
    const double d = delta[n_delta == 1 ? 0 : c];
    if (!(d >= 0.0)) return fail(RTSVD_E_ARG, "tlanczos_solve: delta must be >= 0");
    bounds[c] = eta_dp * d;
  }
  hipStream_t s = (hipStream_t)stream;
  if (dtype == RTSVD_F64)
    return tlanczos_impl<double>((const double*)A, (const double*)B, m, n, p, bounds, k_max, (double*)X, k_out,
                                 resid_out, status_out, s);
  if (dtype == RTSVD_F32)
    return tlanczos_impl<float>((const float*)A, (const float*)B, m, n, p, bounds, k_max, (float*)X, k_out, resid_out,
                                status_out, s);
  return fail(RTSVD_E_ARG, "tlanczos_solve: bad dtype");
}

extern "C" int tlanczos_tik_solve(const void* A, const void* B, int64_t m, int64_t n, int64_t p, int dtype,
                                  const double* delta, int32_t n_delta, double eta_dp, int32_t k_max, double mu_lo,
                                  double mu_hi, void* X, int32_t* k_out, double* mu_out, double* resid_out,
                                  int32_t* status_out, void* stream) {
  g_last_error.clear();
  if (!A || !B || !X || !delta || !k_out || !mu_out) return fail(RTSVD_E_ARG, "tlanczos_tik_solve: null argument");
  if (m < 1 || n < 1 || p < 1) return fail(RTSVD_E_ARG, "tlanczos_tik_solve: need m >= 1, n >= 1, p >= 1");
  if (k_max < 1 || k_max > m) return fail(RTSVD_E_ARG, "tlanczos_tik_solve: need 1 <= k_max <= m");
  if (!(mu_lo > 0.0) || !(mu_hi > mu_lo) || !std::isfinite(mu_hi))
    return fail(RTSVD_E_ARG, "tlanczos_tik_solve: need 0 < mu_lo < mu_hi < inf");
  if (m > 8192) return fail(RTSVD_E_UNSUPPORTED, "tlanczos_tik_solve: m must be <= 8192");
  std::vector<double> bounds;
  RT_TRY(krylov_bounds("tlanczos_tik_solve", delta, n_delta, p, eta_dp, bounds));
  hipStream_t s = (hipStream_t)stream;
  TikArgs tik{mu_lo, mu_hi, mu_out, resid_out, nullptr, nullptr};
  if (dtype == RTSVD_F64)
    return tlanczos_impl<double>((const double*)A, (const double*)B, m, n, p, bounds, k_max, (double*)X, k_out, nullptr,
                                 status_out, s, &tik);
  if (dtype == RTSVD_F32)
    return tlanczos_impl<float>((const float*)A, (const float*)B, m, n, p, bounds, k_max, (float*)X, k_out, nullptr,
                                status_out, s, &tik);
  return fail(RTSVD_E_ARG, "tlanczos_tik_solve: bad dtype");
}



// ---------------------------------------------------------------------------------------------
// batched complex products of the adjoint: FP64 MFMA (k_skinny, FP32 operands converted on the
// way to the MFMA operands, FP64 sums); C = alpha P or C += alpha P through a compact temporary
// ---------------------------------------------------------------------------------------------
template <typename TC>
__global__ void k_axpby(TC* __restrict__ C, int64_t ldc, int64_t sC, const zd* __restrict__ P, int M, int N, int F,
                        double alpha, int accumulate) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (int64_t)F * M * N) return;
  const int i = (int)(idx % M), j = (int)((idx / M) % N);
  const int64_t f = idx / ((int64_t)M * N);
  TC& c = C[f * sC + i + (int64_t)j * ldc];
  const zd v = cscale(P[idx], alpha);
  st(c, accumulate ? cadd(ld<double>(c), v) : v);
}

template <typename TA, typename TB, typename TC>
static int mprod(bool conjA, bool conjB, int M, int N, int K, const TA* A, int64_t lda, int64_t sA, const TB* B,
                 int64_t ldb, int64_t sB, TC* C, int64_t ldc, int64_t sC, int F, double alpha, bool accumulate,
                 Scratch& sc, hipStream_t s) {
  if (conjB) return cgemm<TA, TB, TC, double>(conjA, conjB, M, N, K, A, lda, sA, B, ldb, sB, C, ldc, sC, F, alpha,
                                              accumulate, s);
  if (!accumulate && alpha == 1.0)
    return skinny<TA, TB, TC, Scratch, sk::F64>(conjA, M, N, K, A, lda, sA, B, ldb, sB, C, ldc, sC, F, sc, s);
  RT_ALLOC(tmp, zd, (int64_t)F * M * N, sc);
  RT_TRY((skinny<TA, TB, zd, Scratch, sk::F64>(conjA, M, N, K, A, lda, sA, B, ldb, sB, tmp, M, (int64_t)M * N, F,
                                               sc, s)));
  hipLaunchKernelGGL((k_axpby<TC>), dim3(nblocks((int64_t)F * M * N)), dim3(256), 0, s, C, ldc, sC, (const zd*)tmp, M,
                     N, F, alpha, (int)accumulate);
  RT_LAUNCH_OK();
  return 0;
}

// ---------------------------------------------------------------------------------------------
// gradients of the fixed-k truncated R-tSVD restoration (q = 0), factor recomputed
// ---------------------------------------------------------------------------------------------
template <typename T>
static int vjp_impl(const T* A, const T* dA, const T* B, const T* omega, const T* gX, int64_t l, int64_t m, int64_t n,
                    int64_t p, int k, int64_t r, T* gB, double* gdot, hipStream_t s) {
  typedef cplx<T> zt;
  const int64_t F = n / 2 + 1;
  Scratch sc(s);
  RT_ALLOC(Ah, zt, F * l * m, sc);
  RT_ALLOC(Omh, zt, F * m * r, sc);
  RT_ALLOC(Bh, zt, F * l * p, sc);
  RT_ALLOC(Gh, zt, F * m * p, sc);
  RT_TRY((launch_rfft<T, T>(A, l * m, (int)n, Ah, l * m, (zb*)nullptr, (double*)nullptr, nullptr, s)));
  RT_TRY((launch_rfft<T, T>(omega, m * r, (int)n, Omh, m * r, (zb*)nullptr, (double*)nullptr, nullptr, s)));
  RT_TRY((launch_rfft<T, T>(B, l * p, (int)n, Bh, l * p, (zb*)nullptr, (double*)nullptr, nullptr, s)));
  RT_TRY((launch_rfft<T, T>(gX, m * p, (int)n, Gh, m * p, (zb*)nullptr, (double*)nullptr, nullptr, s)));
  // recomputed factor: Y = A-hat Omega-hat, R^{-1} of Y, Q = CholeskyQR2(Y), C^H = A-hat^H Q, eig(C C^H)
  RT_ALLOC(Y, zt, F * l * r, sc);
  RT_ALLOC(Q, zt, F * l * r, sc);
  RT_ALLOC(tmp, zt, F * l * r, sc);
  RT_ALLOC(G, zd, F * r * r, sc);
  RT_ALLOC(Ry, zd, F * r * r, sc);
  RT_ALLOC(Rq, zd, F * r * r, sc);
  RT_ALLOC(flags, int, 1, sc);
  RT_TRY((big_gemm<zt, zt, zt>(false, Ah, l, m, Omh, r, Y, F, sc, s)));
  RT_TRY(gram<zt>(Y, l, r, F, G, sc, s));
  RT_TRY(launch_cholinv(G, (int)r, F, Ry, flags, sc, s));
  RT_CHECK_HIP(hipMemcpyAsync(Q, Y, sizeof(zt) * F * l * r, hipMemcpyDeviceToDevice, s));
  RT_TRY(orthonormalize<zt>(Q, l, r, F, 2, G, Rq, tmp, flags, sc, s));
  RT_ALLOC(Ch, zd, F * m * r, sc);
  RT_TRY((big_gemm<zt, zt, zd>(true, Ah, l, m, Q, r, Ch, F, sc, s)));
  RT_ALLOC(U, zd, F * r * r, sc);
  RT_ALLOC(lam, double, F * r, sc);
  RT_TRY(gram<zd>(Ch, m, r, F, G, sc, s));
  RT_TRY(launch_heev(G, (int)r, F, U, lam, sc, s));
  // G_k^+ = U diag(phi) U^H
  RT_ALLOC(Uphi, zd, F * r * r, sc);
  RT_ALLOC(Gk, zd, F * r * r, sc);
  hipLaunchKernelGGL(k_scale_inv_eigs, dim3(nblocks(F * r * r)), dim3(256), 0, s, U, Uphi, lam, (int)r, k, (int)F);
  RT_LAUNCH_OK();
  RT_TRY((mprod<zd, zd, zd>(false, true, (int)r, (int)r, (int)r, Uphi, r, r * r, U, r, r * r, Gk, r, r * r,
                                   (int)F, 1.0, false, sc, s)));
  // dL/dB = Q G_k^+ C G  (face by face), then the inverse DFT
  RT_ALLOC(t1, zd, F * r * p, sc);
  RT_ALLOC(t2, zd, F * r * p, sc);
  RT_ALLOC(gBh, zt, F * l * p, sc);
  RT_TRY((mprod<zd, zt, zd>(true, false, (int)r, (int)p, (int)m, Ch, m, m * r, Gh, m, m * p, t1, r, r * p,
                                   (int)F, 1.0, false, sc, s)));
  RT_TRY((mprod<zd, zd, zd>(false, false, (int)r, (int)p, (int)r, Gk, r, r * r, t1, r, r * p, t2, r, r * p,
                                   (int)F, 1.0, false, sc, s)));
  RT_TRY((mprod<zt, zd, zt>(false, false, (int)l, (int)p, (int)r, Q, l, l * r, t2, r, r * p, gBh, l, l * p,
                                   (int)F, 1.0, false, sc, s)));
  RT_TRY((launch_irfft<T, T>(gBh, l * p, l * p, (int)n, gB, s)));
  if (!dA || !gdot) return 0;
  // forward-mode derivative along dA
  RT_ALLOC(dAh, zt, F * l * m, sc);
  RT_TRY((launch_rfft<T, T>(dA, l * m, (int)n, dAh, l * m, (zb*)nullptr, (double*)nullptr, nullptr, s)));
  RT_ALLOC(dY, zd, F * l * r, sc);
  RT_TRY((mprod<zt, zt, zd>(false, false, (int)l, (int)r, (int)m, dAh, l, l * m, Omh, m, m * r, dY, l, l * r,
                                   (int)F, 1.0, false, sc, s)));
  RT_ALLOC(T1, zd, F * r * r, sc);   // Q^H dY
  RT_ALLOC(Mq, zd, F * r * r, sc);
  RT_ALLOC(Xq, zd, F * r * r, sc);
  RT_TRY((mprod<zt, zd, zd>(true, false, (int)r, (int)r, (int)l, Q, l, l * r, dY, l, l * r, T1, r, r * r,
                                   (int)F, 1.0, false, sc, s)));
  RT_TRY((mprod<zd, zd, zd>(false, false, (int)r, (int)r, (int)r, T1, r, r * r, Ry, r, r * r, Mq, r, r * r,
                                   (int)F, 1.0, false, sc, s)));
  hipLaunchKernelGGL(k_skew_lower, dim3(nblocks(F * r * r)), dim3(256), 0, s, Mq, Xq, (int)r, (int)F);
  RT_LAUNCH_OK();
  // P = dY - Q T1 (in place in dY), dQ = Q Xq + P R^{-1}
  RT_TRY((mprod<zt, zd, zd>(false, false, (int)l, (int)r, (int)r, Q, l, l * r, T1, r, r * r, dY, l, l * r,
                                   (int)F, -1.0, true, sc, s)));
  RT_ALLOC(dQ, zd, F * l * r, sc);
  RT_TRY((mprod<zt, zd, zd>(false, false, (int)l, (int)r, (int)r, Q, l, l * r, Xq, r, r * r, dQ, l, l * r,
                                   (int)F, 1.0, false, sc, s)));
  RT_TRY((mprod<zd, zd, zd>(false, false, (int)l, (int)r, (int)r, dY, l, l * r, Ry, r, r * r, dQ, l, l * r,
                                   (int)F, 1.0, true, sc, s)));
  // dC^H = A-hat^H dQ + dA-hat^H Q
  RT_ALLOC(dCh, zd, F * m * r, sc);
  RT_TRY((mprod<zt, zd, zd>(true, false, (int)m, (int)r, (int)l, Ah, l, l * m, dQ, l, l * r, dCh, m, m * r,
                                   (int)F, 1.0, false, sc, s)));
  RT_TRY((mprod<zt, zt, zd>(true, false, (int)m, (int)r, (int)l, dAh, l, l * m, Q, l, l * r, dCh, m, m * r,
                                   (int)F, 1.0, true, sc, s)));
  // dG = dC C^H + C dC^H  = (dC^H)^H C^H + (C^H)^H dC^H
  RT_ALLOC(dG, zd, F * r * r, sc);
  RT_TRY((mprod<zd, zd, zd>(true, false, (int)r, (int)r, (int)m, dCh, m, m * r, Ch, m, m * r, dG, r, r * r,
                                   (int)F, 1.0, false, sc, s)));
  RT_TRY((mprod<zd, zd, zd>(true, false, (int)r, (int)r, (int)m, Ch, m, m * r, dCh, m, m * r, dG, r, r * r,
                                   (int)F, 1.0, true, sc, s)));
  // d(G_k^+) = U (Phi o (U^H dG U)) U^H
  RT_ALLOC(E1, zd, F * r * r, sc);
  RT_ALLOC(E2, zd, F * r * r, sc);
  RT_TRY((mprod<zd, zd, zd>(true, false, (int)r, (int)r, (int)r, U, r, r * r, dG, r, r * r, E1, r, r * r,
                                   (int)F, 1.0, false, sc, s)));
  RT_TRY((mprod<zd, zd, zd>(false, false, (int)r, (int)r, (int)r, E1, r, r * r, U, r, r * r, E2, r, r * r,
                                   (int)F, 1.0, false, sc, s)));
  hipLaunchKernelGGL(k_phi_hadamard, dim3(nblocks(F * r * r)), dim3(256), 0, s, E2, lam, (int)r, k, (int)F);
  RT_LAUNCH_OK();
  RT_TRY((mprod<zd, zd, zd>(false, false, (int)r, (int)r, (int)r, U, r, r * r, E2, r, r * r, E1, r, r * r,
                                   (int)F, 1.0, false, sc, s)));
  RT_ALLOC(dGk, zd, F * r * r, sc);
  RT_TRY((mprod<zd, zd, zd>(false, true, (int)r, (int)r, (int)r, E1, r, r * r, U, r, r * r, dGk, r, r * r,
                                   (int)F, 1.0, false, sc, s)));
  // d = Q^H B-hat, dd = dQ^H B-hat, dX-hat = dC^H G_k^+ d + C^H dG_k^+ d + C^H G_k^+ dd
  RT_ALLOC(d, zd, F * r * p, sc);
  RT_ALLOC(dd, zd, F * r * p, sc);
  RT_ALLOC(e, zd, F * r * p, sc);
  RT_TRY((mprod<zt, zt, zd>(true, false, (int)r, (int)p, (int)l, Q, l, l * r, Bh, l, l * p, d, r, r * p,
                                   (int)F, 1.0, false, sc, s)));
  RT_TRY((mprod<zd, zt, zd>(true, false, (int)r, (int)p, (int)l, dQ, l, l * r, Bh, l, l * p, dd, r, r * p,
                                   (int)F, 1.0, false, sc, s)));
  RT_ALLOC(dXh, zd, F * m * p, sc);
  RT_TRY((mprod<zd, zd, zd>(false, false, (int)r, (int)p, (int)r, Gk, r, r * r, d, r, r * p, e, r, r * p,
                                   (int)F, 1.0, false, sc, s)));
  RT_TRY((mprod<zd, zd, zd>(false, false, (int)m, (int)p, (int)r, dCh, m, m * r, e, r, r * p, dXh, m, m * p,
                                   (int)F, 1.0, false, sc, s)));
  RT_TRY((mprod<zd, zd, zd>(false, false, (int)r, (int)p, (int)r, dGk, r, r * r, d, r, r * p, e, r, r * p,
                                   (int)F, 1.0, false, sc, s)));
  RT_TRY((mprod<zd, zd, zd>(false, false, (int)r, (int)p, (int)r, Gk, r, r * r, dd, r, r * p, e, r, r * p,
                                   (int)F, 1.0, true, sc, s)));
  RT_TRY((mprod<zd, zd, zd>(false, false, (int)m, (int)p, (int)r, Ch, m, m * r, e, r, r * p, dXh, m, m * p,
                                   (int)F, 1.0, true, sc, s)));
  {
    const int64_t blocks = ceil_div(F * m * p, (int64_t)WI_THREADS * WI_ITEMS);
    RT_ALLOC(wpart, double, blocks, sc);
    hipLaunchKernelGGL((k_weighted_inner_part<zt>), dim3((unsigned)blocks), dim3(WI_THREADS), 0, s, Gh, dXh, m * p,
                       (int)F, (int)n, wpart);
    RT_LAUNCH_OK();
    hipLaunchKernelGGL(k_sum_partials, dim3(1), dim3(256), 0, s, (const double*)wpart, blocks, 1.0 / (double)n, gdot);
    RT_LAUNCH_OK();
  }
  return 0;
}

extern "C" int rtsvd_solve_vjp(const void* A, const void* dA, const void* B, const void* omega, const void* gX,
                               int64_t l, int64_t m, int64_t n, int64_t p, int32_t k, int32_t oversample, int dtype,
                               void* gB, double* gdot, void* stream) {
  g_last_error.clear();
  if (!A || !B || !omega || !gX || !gB) return fail(RTSVD_E_ARG, "rtsvd_solve_vjp: null argument");
  if (l < 1 || m < 1 || n < 1 || p < 1 || l < m) return fail(RTSVD_E_ARG, "rtsvd_solve_vjp: need l >= m >= 1, n, p >= 1");
  if (k < 1 || k > m || oversample < 0) return fail(RTSVD_E_ARG, "rtsvd_solve_vjp: need 1 <= k <= m, oversample >= 0");
  const int64_t r = std::min<int64_t>((int64_t)k + oversample, m);
  if (r > 256) return fail(RTSVD_E_UNSUPPORTED, "rtsvd_solve_vjp: r must be <= 256");
  if ((dA == nullptr) != (gdot == nullptr)) return fail(RTSVD_E_ARG, "rtsvd_solve_vjp: dA and gdot go together");
  hipStream_t s = (hipStream_t)stream;
  if (dtype == RTSVD_F64)
    return vjp_impl<double>((const double*)A, (const double*)dA, (const double*)B, (const double*)omega,
                            (const double*)gX, l, m, n, p, k, r, (double*)gB, gdot, s);
  if (dtype == RTSVD_F32)
    return vjp_impl<float>((const float*)A, (const float*)dA, (const float*)B, (const float*)omega, (const float*)gX, l,
                           m, n, p, k, r, (float*)gB, gdot, s);
  return fail(RTSVD_E_ARG, "rtsvd_solve_vjp: bad dtype");
}

// ---------------------------------------------------------------------------------------------
// Gaussian tensor of the sketch (the one rtsvd_factor draws when omega == NULL)
// ---------------------------------------------------------------------------------------------
extern "C" int rtsvd_gaussian(uint64_t seed, int64_t m, int64_t r, int64_t n, int dtype, void* out, void* stream) {
  g_last_error.clear();
  if (!out) return fail(RTSVD_E_ARG, "rtsvd_gaussian: null output");
  if (m < 1 || r < 1 || n < 1) return fail(RTSVD_E_ARG, "rtsvd_gaussian: sizes must be >= 1");
  hipStream_t s = (hipStream_t)stream;
  const int64_t count = m * r * n;
  if ((count + 1) / 2 > GAUSS_MAX_PAIRS) return fail(RTSVD_E_UNSUPPORTED, "rtsvd_gaussian: more than 2^32 elements");
  int rc;
  if (dtype == RTSVD_F64) rc = launch_gaussian<double>(seed, count, (double*)out, s);
  else if (dtype == RTSVD_F32) rc = launch_gaussian<float>(seed, count, (float*)out, s);
  else return fail(RTSVD_E_ARG, "rtsvd_gaussian: bad dtype");
  if (rc) return fail(RTSVD_E_HIP, "rtsvd_gaussian: launch failed");
  return RTSVD_OK;
}

// ---------------------------------------------------------------------------------------------
extern "C" const char* rtsvd_status_string(int status) {
  switch (status) {
    case RTSVD_OK: return "ok";
    case RTSVD_W_DP_NOT_MET: return "warning: discrepancy principle not met within k_cap";
    case RTSVD_W_RANK_DEFICIENT: return "warning: rank-deficient sketch (breakdown threshold reached)";
    case RTSVD_E_ARG: return "error: invalid argument";
    case RTSVD_E_NOTFINITE: return "error: non-finite input (NaN or infinity)";
    case RTSVD_E_HIP: return "error: HIP runtime failure";
    case RTSVD_E_NOMEM: return "error: out of device memory";
    case RTSVD_E_UNSUPPORTED: return "error: unsupported configuration";
    default: return "unknown status";
  }
}

extern "C" const char* rtsvd_last_error(void) { return g_last_error.c_str(); }
