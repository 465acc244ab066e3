// Internal runtime pieces shared by the library's translation units:
// complex arithmetic, error reporting, device buffers, reductions.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <string>

#include "../../include/hdcg.h"

namespace hdk {

// ---------------------------------------------------------------- errors ---
void set_error(const std::string& msg);

struct Status {
  int code = DWF_OK;
  Status() = default;
  Status(int c) : code(c) {}
  bool ok() const { return code == DWF_OK; }
};

#define HDCG_HIP(...)                                                            \
  do {                                                                           \
    hipError_t e_ = (__VA_ARGS__);                                               \
    if (e_ != hipSuccess) {                                                      \
      ::hdk::set_error(std::string(#__VA_ARGS__) + ": " + hipGetErrorString(e_)); \
      return DWF_ERR_HIP;                                                        \
    }                                                                            \
  } while (0)

#define HDCG_TRY(...)                  \
  do {                                 \
    int s_ = (__VA_ARGS__);            \
    if (s_ < 0) return s_;             \
  } while (0)

inline int fail(int code, const std::string& msg) {
  set_error(msg);
  return code;
}

// --------------------------------------------------------------- complex ---
template <typename R>
struct alignas(2 * sizeof(R)) cplx {
  R re, im;
};
using c128 = cplx<double>;
using c64 = cplx<float>;

template <typename R>
__host__ __device__ __forceinline__ cplx<R> cmk(R a, R b) {
  cplx<R> c;
  c.re = a;
  c.im = b;
  return c;
}
template <typename R>
__host__ __device__ __forceinline__ cplx<R> operator+(cplx<R> a, cplx<R> b) {
  return cmk(a.re + b.re, a.im + b.im);
}
template <typename R>
__host__ __device__ __forceinline__ cplx<R> operator-(cplx<R> a, cplx<R> b) {
  return cmk(a.re - b.re, a.im - b.im);
}
template <typename R>
__host__ __device__ __forceinline__ cplx<R> operator*(cplx<R> a, cplx<R> b) {
  return cmk(a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re);
}
template <typename R>
__host__ __device__ __forceinline__ cplx<R> operator*(R s, cplx<R> a) {
  return cmk(s * a.re, s * a.im);
}
template <typename R>
__host__ __device__ __forceinline__ cplx<R> conj(cplx<R> a) {
  return cmk(a.re, -a.im);
}
// i*a and -i*a
template <typename R>
__host__ __device__ __forceinline__ cplx<R> timesI(cplx<R> a) {
  return cmk(-a.im, a.re);
}
template <typename R>
__host__ __device__ __forceinline__ cplx<R> timesMinusI(cplx<R> a) {
  return cmk(a.im, -a.re);
}
// a += b*c ; a += conj(b)*c, as four chained fused multiply-adds each
template <typename R>
__host__ __device__ __forceinline__ void cmac(cplx<R>& a, cplx<R> b, cplx<R> c) {
  a.re = fma(b.re, c.re, a.re);
  a.re = fma(-b.im, c.im, a.re);
  a.im = fma(b.re, c.im, a.im);
  a.im = fma(b.im, c.re, a.im);
}
template <typename R>
__host__ __device__ __forceinline__ void cjmac(cplx<R>& a, cplx<R> b, cplx<R> c) {
  a.re = fma(b.re, c.re, a.re);
  a.re = fma(b.im, c.im, a.re);
  a.im = fma(b.re, c.im, a.im);
  a.im = fma(-b.im, c.re, a.im);
}

// ------------------------------------------------------ field storage ---
// A complex number stored as two bfloat16 values (re, im): 4 bytes, for
// fields whose arithmetic runs in FP32 but whose storage may be 16-bit.
struct alignas(4) bf16c {
  unsigned short re, im;
};

__host__ __device__ __forceinline__ float bf16_to_f32(unsigned short h) {
  unsigned u = (unsigned)h << 16;
  float f;
  __builtin_memcpy(&f, &u, 4);
  return f;
}
// round to nearest even: on the device gfx950's conversion instruction
// (v_cvt_pk_bf16_f32); on the host the same rounding in integer arithmetic
// (a NaN may come out as an infinity there, still non-finite)
__host__ __device__ __forceinline__ unsigned short f32_to_bf16(float f) {
#if defined(__HIP_DEVICE_COMPILE__)
  return __builtin_bit_cast(unsigned short, (__bf16)f);
#else
  unsigned u;
  __builtin_memcpy(&u, &f, 4);
  u += 0x7fffu + ((u >> 16) & 1u);
  return (unsigned short)(u >> 16);
#endif
}
typedef __bf16 bf16x2_t __attribute__((ext_vector_type(2)));
typedef float f32x2_t __attribute__((ext_vector_type(2)));
// (re, im) rounded to nearest even and packed re | im << 16: one
// v_cvt_pk_bf16_f32
__device__ __forceinline__ unsigned f32x2_to_bf16x2(float re, float im) {
  const f32x2_t v = {re, im};
  return __builtin_bit_cast(unsigned, __builtin_convertvector(v, bf16x2_t));
}

// Storage traits: St<T>::R is the arithmetic type of a field stored as T;
// ld / st convert between the two.
template <typename T>
struct St;
template <>
struct St<cplx<double>> {
  using R = double;
  __device__ __forceinline__ static cplx<double> ld(const cplx<double>* p) { return *p; }
  __device__ __forceinline__ static void st(cplx<double>* p, cplx<double> v) { *p = v; }
};
template <>
struct St<cplx<float>> {
  using R = float;
  __device__ __forceinline__ static cplx<float> ld(const cplx<float>* p) { return *p; }
  __device__ __forceinline__ static void st(cplx<float>* p, cplx<float> v) { *p = v; }
};
template <>
struct St<bf16c> {
  using R = float;
  __device__ __forceinline__ static cplx<float> ld(const bf16c* p) {
    const bf16c v = *p;
    return cmk(bf16_to_f32(v.re), bf16_to_f32(v.im));
  }
  __device__ __forceinline__ static void st(bf16c* p, cplx<float> v) {
    *reinterpret_cast<unsigned*>(p) = f32x2_to_bf16x2(v.re, v.im);
  }
};

template <typename R>
inline int prec_of();
template <>
inline int prec_of<double>() {
  return DWF_C128;
}
template <>
inline int prec_of<float>() {
  return DWF_C64;
}
// bytes per complex of a fine field in precision prec (DWF_BF16: 16-bit storage)
inline size_t cbytes(int prec) { return prec == DWF_C128 ? 16 : (prec == DWF_BF16 ? 4 : 8); }

// --------------------------------------------------------------- buffers ---
// Grow-only device buffer owned by a handle.
struct DevBuf {
  void* ptr = nullptr;
  size_t bytes = 0;
  int ensure(size_t want) {
    if (want <= bytes) return DWF_OK;
    if (ptr) (void)hipFree(ptr);
    ptr = nullptr;
    bytes = 0;
    hipError_t e = hipMalloc(&ptr, want);
    if (e != hipSuccess) {
      ptr = nullptr;
      return fail(DWF_ERR_OOM, "hipMalloc of " + std::to_string(want) + " bytes failed");
    }
    bytes = want;
    return DWF_OK;
  }
  template <typename T>
  T* as() const {
    return static_cast<T*>(ptr);
  }
  void release() {
    if (ptr) (void)hipFree(ptr);
    ptr = nullptr;
    bytes = 0;
  }
};

// ------------------------------------------------------------ reductions ---
// Deterministic two-stage reductions: every workgroup writes one partial per
// output, the last workgroup to finish (ticket counter) sums the partials in
// a fixed order and resets the counter.
constexpr int kMaxPartials = 1 << 16;  // partial slots per reduced quantity
constexpr int kPinnedDoubles = 1024;   // host pinned scalars of an operator handle
constexpr int kRedThreads = 256;

struct Reducer {
  DevBuf partials;  // double [nq][kMaxPartials]
  DevBuf counters;  // unsigned [64]
  DevBuf results;   // double [nq]
  int ensure(int nq);
};

// Sum of a double across the workgroup; valid in thread 0.  blockDim.x must
// be a multiple of 64 and at most 1024.
__device__ __forceinline__ double wave_sum(double v) {
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

template <int NQ>
__device__ __forceinline__ void block_sum(double (&v)[NQ], double* lds /* NQ*16 */) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int nw = (blockDim.x + 63) >> 6;
#pragma unroll
  for (int q = 0; q < NQ; ++q) v[q] = wave_sum(v[q]);
  if (lane == 0) {
#pragma unroll
    for (int q = 0; q < NQ; ++q) lds[q * 16 + wave] = v[q];
  }
  __syncthreads();
  if (threadIdx.x == 0) {
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
      double s = 0.0;
      for (int w = 0; w < nw; ++w) s += lds[q * 16 + w];
      v[q] = s;
    }
  }
}

// Thread 0 of every workgroup stores its partial sums: partials[q * nslots +
// slot].  A separate finalize launch (launch_finalize) then sums the
// partials of each right-hand side in a fixed order, so results are
// deterministic and no workgroup waits on a fence or an atomic.
template <int NQ>
__device__ __forceinline__ void store_partial(const double (&v)[NQ], double* partials, int nslots,
                                              int slot) {
  if (threadIdx.x == 0) {
#pragma unroll
    for (int q = 0; q < NQ; ++q) partials[q * nslots + slot] = v[q];
  }
}

// res[nq * rhs + q] = sum_{i < nblocks} partials[rhs * rstride + q * nslots + i]
int launch_finalize(int nq, const double* partials, int nslots, int nblocks, int nrhs, double* res,
                    hipStream_t st, size_t rstride = kMaxPartials);

// Map blockIdx.x so that each of the 8 XCDs (workgroups are dispatched to
// XCDs round-robin) receives one contiguous range of tiles: neighbouring
// tiles then share that XCD's L2.  A bijection on [0, n).
__device__ __forceinline__ int xcd_remap(int bid, int n) {
  const int q = n >> 3, r = n & 7;
  const int x = bid & 7, k = bid >> 3;
  const int base = x < r ? x * (q + 1) : r * (q + 1) + (x - r) * q;
  return base + k;
}

}  // namespace hdk
