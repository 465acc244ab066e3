// BLAS-1 kernels with device-resident coefficients and FP64 reductions.
#include "blas.h"

namespace hdk {

namespace {

constexpr int kT = 256;

inline int nblocks(size_t n) {
  size_t b = (n + kT * 8 - 1) / (kT * 8);
  if (b < 1) b = 1;
  if (b > 1024) b = 1024;
  return (int)b;
}

template <typename R>
__device__ __forceinline__ double nrm(cplx<R> a) {
  return (double)a.re * a.re + (double)a.im * a.im;
}

__device__ __forceinline__ void coef(const double* num, bool cnum, const double* den,
                                     const double* den2, double lam, int rhs, double& re,
                                     double& im, int dstr) {
  double d = den[rhs * dstr];
  if (den2) d += lam * den2[rhs];
  if (d == 0.0) {
    re = im = 0.0;
    return;
  }
  if (cnum) {
    re = num[2 * rhs] / d;
    im = num[2 * rhs + 1] / d;
  } else {
    re = num[rhs] / d;
    im = 0.0;
  }
}

// Workgroup sums of one right-hand side's NQ quantities, reduced over the
// grid inside the producing kernel: each workgroup stores its partials with
// coherent device-scope stores, waits for them to complete and takes a
// ticket; the workgroup that takes the last ticket sums every partial in a
// fixed order (the result does not depend on which one it is), writes
// res[NQ * rhs + q] and resets the ticket counter.  No workgroup waits for
// another, and no cache maintenance is needed.
template <int NQ>
__device__ __forceinline__ void reduce_out(double (&v)[NQ], Red red, int rhs, double* res) {
  __shared__ double lds[NQ * 16];
  __shared__ int last;
  constexpr int nslots = kMaxPartials / NQ;
  double* part = red.partials + (size_t)rhs * kMaxPartials;
  block_sum<NQ>(v, lds);
  if (threadIdx.x == 0) {
#pragma unroll
    for (int q = 0; q < NQ; ++q)
      __hip_atomic_store(part + q * nslots + blockIdx.x, v[q], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    __builtin_amdgcn_s_waitcnt(0);
    const unsigned t = __hip_atomic_fetch_add(red.counters + rhs, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    last = t == gridDim.x - 1;
  }
  __syncthreads();
  if (!last) return;
  double s[NQ];
  const int G = (int)gridDim.x, B = (int)blockDim.x;
#pragma unroll
  for (int q = 0; q < NQ; ++q) {
    s[q] = 0.0;
    // four partials per trip, loads first (the last workgroup's sum is on
    // the kernel's critical path)
    for (int i0 = threadIdx.x; i0 < G; i0 += 4 * B) {
      double a[4];
#pragma unroll
      for (int u = 0; u < 4; ++u)
        a[u] = i0 + u * B < G ? __hip_atomic_load(part + q * nslots + i0 + u * B, __ATOMIC_RELAXED,
                                                  __HIP_MEMORY_SCOPE_AGENT)
                              : 0.0;
#pragma unroll
      for (int u = 0; u < 4; ++u) s[q] += a[u];
    }
  }
  block_sum<NQ>(s, lds);
  if (threadIdx.x == 0) {
#pragma unroll
    for (int q = 0; q < NQ; ++q) res[NQ * rhs + q] = s[q];
    __hip_atomic_store(red.counters + rhs, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
}

// Sum of the per-workgroup partials of a kernel that does not finish its own
// reduction (the hop kernel's fused norm: one partial per workgroup, up to
// ~10^5).  One 1024-thread workgroup per right-hand side; each lane keeps
// eight independent accumulators so eight loads are in flight per trip
// (fixed order: deterministic).
constexpr int kFinT = 1024;
template <int NQ>
__global__ void __launch_bounds__(kFinT) k_finalize(const double* __restrict__ partials, int nslots,
                                                    int nblocks, size_t rstride, double* __restrict__ res) {
  const int rhs = blockIdx.x;
  const double* p = partials + (size_t)rhs * rstride;
  __shared__ double lds[kFinT / 64];
  for (int q = 0; q < NQ; ++q) {
    const double* pq = p + (size_t)q * nslots;
    double s[8] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
    int i = threadIdx.x;
    for (; i + 7 * kFinT < nblocks; i += 8 * kFinT) {
#pragma unroll
      for (int u = 0; u < 8; ++u) s[u] += pq[i + u * kFinT];
    }
    for (; i < nblocks; i += kFinT) s[0] += pq[i];
    double t = ((s[0] + s[1]) + (s[2] + s[3])) + ((s[4] + s[5]) + (s[6] + s[7]));
    t = wave_sum(t);
    if ((threadIdx.x & 63) == 0) lds[threadIdx.x >> 6] = t;
    __syncthreads();
    if (threadIdx.x == 0) {
      double r = 0.0;
      for (int w = 0; w < kFinT / 64; ++w) r += lds[w];
      res[NQ * rhs + q] = r;
    }
    __syncthreads();
  }
}

// Fields are stored as T (cplx<R>, or bf16c with FP32 arithmetic).  The
// streaming kernels move Vec<T>::V consecutive values per lane and operand
// with one load or store: one complex for cplx<R>, four bf16c (16 bytes) for
// the 16-bit storage, so a lane keeps as many bytes in flight as in complex64
// or wider.  n must be a multiple of V (the launchers check).
template <typename T>
struct Vec {
  static constexpr int V = 1;
  using R = typename St<T>::R;
  __device__ __forceinline__ static void ld(const T* p, size_t g, cplx<R> (&o)[1]) { o[0] = St<T>::ld(p + g); }
  __device__ __forceinline__ static void st(T* p, size_t g, const cplx<R> (&v)[1]) { St<T>::st(p + g, v[0]); }
};
struct alignas(16) bf16c4 {
  bf16c v[4];
};
template <>
struct Vec<bf16c> {
  static constexpr int V = 4;
  __device__ __forceinline__ static void ld(const bf16c* p, size_t g, cplx<float> (&o)[4]) {
    const bf16c4 q = reinterpret_cast<const bf16c4*>(p)[g];
#pragma unroll
    for (int k = 0; k < 4; ++k) o[k] = St<bf16c>::ld(&q.v[k]);
  }
  __device__ __forceinline__ static void st(bf16c* p, size_t g, const cplx<float> (&v)[4]) {
    bf16c4 q;
#pragma unroll
    for (int k = 0; k < 4; ++k) St<bf16c>::st(&q.v[k], v[k]);
    reinterpret_cast<bf16c4*>(p)[g] = q;
  }
};
template <typename T>
__global__ void __launch_bounds__(kT) k_norm2(const T* __restrict__ x, size_t n, Red red,
                                              double* res) {
  using R = typename St<T>::R;
  const int rhs = blockIdx.y;
  x += rhs * n;
  constexpr int V = Vec<T>::V;
  double acc = 0.0;
  for (size_t g = (size_t)blockIdx.x * kT + threadIdx.x; g < n / V; g += (size_t)gridDim.x * kT) {
    cplx<R> v[V];
    Vec<T>::ld(x, g, v);
#pragma unroll
    for (int k = 0; k < V; ++k) acc += nrm(v[k]);
  }
  double v[1] = {acc};
  reduce_out<1>(v, red, rhs, res);
}

template <typename T>
__global__ void __launch_bounds__(kT) k_dot(const T* __restrict__ a, const T* __restrict__ b,
                                            size_t n, Red red, double* res) {
  const int rhs = blockIdx.y;
  a += rhs * n;
  b += rhs * n;
  double re = 0.0, im = 0.0;
  for (size_t i = (size_t)blockIdx.x * kT + threadIdx.x; i < n; i += (size_t)gridDim.x * kT) {
    const auto x = St<T>::ld(a + i), y = St<T>::ld(b + i);
    re += (double)x.re * y.re + (double)x.im * y.im;
    im += (double)x.re * y.im - (double)x.im * y.re;
  }
  double v[2] = {re, im};
  reduce_out<2>(v, red, rhs, res);
}

template <typename T, int MODE>
__global__ void __launch_bounds__(kT)
k_update(T* __restrict__ x, T* __restrict__ r, const T* __restrict__ p, const T* __restrict__ w,
         size_t n, const double* num, bool cnum, const double* den, const double* den2, double lam,
         Red red, double* rr, int dstr) {
  constexpr bool X0 = MODE & kUpdX0, XONLY = MODE & kUpdXOnly;
  using R = typename St<T>::R;
  const int rhs = blockIdx.y;
  const size_t off = rhs * n;
  double are, aim;
  coef(num, cnum, den, den2, lam, rhs, are, aim, dstr);
  const cplx<R> a = cmk((R)are, (R)aim);
  const R l = (R)lam;
  constexpr int V = Vec<T>::V;
  x += off;
  r += off;
  p += off;
  w += off;
  double acc = 0.0;
  for (size_t g = (size_t)blockIdx.x * kT + threadIdx.x; g < n / V; g += (size_t)gridDim.x * kT) {
    cplx<R> pv[V], wv[V], xv[V], rv[V];
    Vec<T>::ld(p, g, pv);
    if constexpr (!XONLY) {
      Vec<T>::ld(w, g, wv);
      Vec<T>::ld(r, g, rv);
    }
    if constexpr (X0) {
#pragma unroll
      for (int k = 0; k < V; ++k) xv[k] = cmk((R)0, (R)0);
    } else {
      Vec<T>::ld(x, g, xv);
    }
#pragma unroll
    for (int k = 0; k < V; ++k) {
      xv[k] = xv[k] + a * pv[k];
      if constexpr (!XONLY) {
        if (den2) wv[k] = wv[k] + l * pv[k];
        rv[k] = rv[k] - a * wv[k];
        acc += nrm(rv[k]);
      }
    }
    Vec<T>::st(x, g, xv);
    if constexpr (!XONLY) Vec<T>::st(r, g, rv);
  }
  if (!XONLY && rr) {
    double v[1] = {acc};
    reduce_out<1>(v, red, rhs, rr);
  }
}

template <typename T>
__global__ void __launch_bounds__(kT)
k_xpay(T* __restrict__ p, const T* __restrict__ y, size_t n, const double* num, bool cnum,
       const double* den, double sign, Red red, double* pp, int dstr) {
  using R = typename St<T>::R;
  const int rhs = blockIdx.y;
  const size_t off = rhs * n;
  double bre, bim;
  coef(num, cnum, den, nullptr, 0.0, rhs, bre, bim, dstr);
  const cplx<R> b = cmk((R)(sign * bre), (R)(sign * bim));
  constexpr int V = Vec<T>::V;
  p += off;
  y += off;
  double acc = 0.0;
  for (size_t g = (size_t)blockIdx.x * kT + threadIdx.x; g < n / V; g += (size_t)gridDim.x * kT) {
    cplx<R> yv[V], pv[V];
    Vec<T>::ld(y, g, yv);
    Vec<T>::ld(p, g, pv);
#pragma unroll
    for (int k = 0; k < V; ++k) {
      pv[k] = yv[k] + b * pv[k];
      acc += nrm(pv[k]);
    }
    Vec<T>::st(p, g, pv);
  }
  if (pp) {
    double v[1] = {acc};
    reduce_out<1>(v, red, rhs, pp);
  }
}

// Fixed-count CG on 16-bit fields (M_IRS), first step: r = p = bf16(b) for
// b complex64 [site][12][Ls] and r, p 16-bit [site][Ls][12] (rounded to
// nearest even as every 16-bit store), and rr[rhs] = |r|^2 of the rounded
// values.  One (site, s) row of 12 values per thread; rows per RHS.
__global__ void __launch_bounds__(kT)
k_mirs16_init(bf16c* __restrict__ r, bf16c* __restrict__ p, const c64* __restrict__ b, size_t rows, int Ls,
              Red red, double* rr) {
  const int rhs = blockIdx.y;
  const size_t off = (size_t)rhs * rows * 12;
  double acc = 0.0;
  for (size_t row = (size_t)blockIdx.x * kT + threadIdx.x; row < rows; row += (size_t)gridDim.x * kT) {
    const size_t site = row / Ls;
    const int s = (int)(row - site * Ls);
    const c64* f = b + off + site * 12 * Ls + s;
    bf16c4 q[3];
#pragma unroll
    for (int c = 0; c < 12; ++c) {
      St<bf16c>::st(&q[c >> 2].v[c & 3], f[c * Ls]);
      acc += nrm(St<bf16c>::ld(&q[c >> 2].v[c & 3]));
    }
    const size_t o = (off + site * 12 * Ls + (size_t)s * 12) / 4;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      reinterpret_cast<bf16c4*>(r)[o + k] = q[k];
      reinterpret_cast<bf16c4*>(p)[o + k] = q[k];
    }
  }
  double v[1] = {acc};
  reduce_out<1>(v, red, rhs, rr);
}

// Its last step: only x is still needed, x_out = x + alpha p rounded to 16
// bits as the stored x would be, written in complex64 [site][12][Ls]
// (x == nullptr: x = 0); alpha as in k_update.
__global__ void __launch_bounds__(kT)
k_mirs16_last(c64* __restrict__ xo, const bf16c* __restrict__ x, const bf16c* __restrict__ p, size_t rows,
              int Ls, const double* num, const double* den, const double* den2, double lam) {
  const int rhs = blockIdx.y;
  const size_t off = (size_t)rhs * rows * 12;
  double are, aim;
  coef(num, false, den, den2, lam, rhs, are, aim, 1);
  const cplx<float> a = cmk((float)are, (float)aim);
  for (size_t row = (size_t)blockIdx.x * kT + threadIdx.x; row < rows; row += (size_t)gridDim.x * kT) {
    const size_t site = row / Ls;
    const int s = (int)(row - site * Ls);
    const size_t o = (off + site * 12 * Ls + (size_t)s * 12) / 4;
    c64* f = xo + off + site * 12 * Ls + s;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      const bf16c4 pq = reinterpret_cast<const bf16c4*>(p)[o + k];
      bf16c4 xq;
      if (x) xq = reinterpret_cast<const bf16c4*>(x)[o + k];
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const cplx<float> xv = x ? St<bf16c>::ld(&xq.v[e]) : cmk(0.f, 0.f);
        bf16c t;
        St<bf16c>::st(&t, xv + a * St<bf16c>::ld(&pq.v[e]));
        f[(4 * k + e) * Ls] = St<bf16c>::ld(&t);
      }
    }
  }
}

template <typename R>
__global__ void k_axpby(cplx<R>* __restrict__ y, const cplx<R>* __restrict__ x, R a, R b,
                        size_t total) {
  for (size_t i = (size_t)blockIdx.x * kT + threadIdx.x; i < total; i += (size_t)gridDim.x * kT)
    y[i] = a * x[i] + b * y[i];
}

template <typename Ry, typename Rx>
__global__ void k_axpy_mixed(cplx<Ry>* __restrict__ y, const cplx<Rx>* __restrict__ x,
                             const double* s, size_t n, bool sqrt_s) {
  const int rhs = blockIdx.y;
  const size_t off = rhs * n;
  const Ry f = s ? (Ry)(sqrt_s ? sqrt(s[rhs]) : s[rhs]) : (Ry)1;
  for (size_t i = (size_t)blockIdx.x * kT + threadIdx.x; i < n; i += (size_t)gridDim.x * kT) {
    const cplx<Rx> v = x[off + i];
    y[off + i] = y[off + i] + f * cmk((Ry)v.re, (Ry)v.im);
  }
}

template <typename Ry, typename Rx>
__global__ void k_scale_copy(cplx<Ry>* __restrict__ y, const cplx<Rx>* __restrict__ x,
                             const double* v, bool invsqrt, size_t n) {
  const int rhs = blockIdx.y;
  const size_t off = rhs * n;
  double s = v ? v[rhs] : 1.0;
  if (invsqrt) s = s > 0.0 ? 1.0 / sqrt(s) : 0.0;
  for (size_t i = (size_t)blockIdx.x * kT + threadIdx.x; i < n; i += (size_t)gridDim.x * kT) {
    const cplx<Rx> a = x[off + i];
    y[off + i] = cmk((Ry)(s * a.re), (Ry)(s * a.im));
  }
}

template <typename T>
__global__ void k_zero(T* __restrict__ y, size_t total) {
  using R = typename St<T>::R;
  constexpr int V = Vec<T>::V;
  cplx<R> z[V];
#pragma unroll
  for (int k = 0; k < V; ++k) z[k] = cmk((R)0, (R)0);
  for (size_t g = (size_t)blockIdx.x * kT + threadIdx.x; g < total / V; g += (size_t)gridDim.x * kT)
    Vec<T>::st(y, g, z);
}

}  // namespace

#define LAUNCH_CHECK() HDCG_HIP(hipGetLastError())

int launch_finalize(int nq, const double* partials, int nslots, int nblocks, int nrhs, double* res,
                    hipStream_t st, size_t rstride) {
  if (nblocks > nslots || (size_t)nq * nslots > rstride) return fail(DWF_ERR_ARG, "too many partial sums");
  if (nq == 1)
    hipLaunchKernelGGL((k_finalize<1>), dim3(nrhs), dim3(kFinT), 0, st, partials, nslots, nblocks, rstride, res);
  else
    hipLaunchKernelGGL((k_finalize<2>), dim3(nrhs), dim3(kFinT), 0, st, partials, nslots, nblocks, rstride, res);
  LAUNCH_CHECK();
  return DWF_OK;
}

template <typename T>
int norm2_t(Red red, const T* x, size_t n, int nrhs, double* res, hipStream_t st) {
  if (n % Vec<T>::V) return fail(DWF_ERR_ARG, "16-bit fields need a multiple of 4 complex values");
  if (nrhs > 64) return fail(DWF_ERR_ARG, "nrhs > 64");
  hipLaunchKernelGGL((k_norm2<T>), dim3(nblocks(n), nrhs), dim3(kT), 0, st, x, n, red, res);
  LAUNCH_CHECK();
  return DWF_OK;
}
template <typename T>
int dot_t(Red red, const T* a, const T* b, size_t n, int nrhs, double* res, hipStream_t st) {
  if (nrhs > 64) return fail(DWF_ERR_ARG, "nrhs > 64");
  hipLaunchKernelGGL((k_dot<T>), dim3(nblocks(n), nrhs), dim3(kT), 0, st, a, b, n, red, res);
  LAUNCH_CHECK();
  return DWF_OK;
}
template <typename T>
int update_t(Red red, T* x, T* r, const T* p, const T* w, size_t n, int nrhs, const double* num,
             bool cnum, const double* den, const double* den2, double lam, double* rr,
             hipStream_t st, int dstr, int mode) {
  if (n % Vec<T>::V) return fail(DWF_ERR_ARG, "16-bit fields need a multiple of 4 complex values");
  if (nrhs > 64) return fail(DWF_ERR_ARG, "nrhs > 64");
  if (mode < 0 || mode > (kUpdX0 | kUpdXOnly)) return fail(DWF_ERR_ARG, "update: bad mode");
  const dim3 grid(nblocks(n), nrhs);
#define HDCG_UPDATE(M)                                                                                      \
  hipLaunchKernelGGL((k_update<T, M>), grid, dim3(kT), 0, st, x, r, p, w, n, num, cnum, den, den2, lam, red, \
                     rr, dstr)
  switch (mode) {
    case 0: HDCG_UPDATE(0); break;
    case kUpdX0: HDCG_UPDATE(kUpdX0); break;
    case kUpdXOnly: HDCG_UPDATE(kUpdXOnly); break;
    default: HDCG_UPDATE(kUpdX0 | kUpdXOnly); break;
  }
#undef HDCG_UPDATE
  LAUNCH_CHECK();
  return DWF_OK;
}
template <typename T>
int xpay_t(Red red, T* p, const T* y, size_t n, int nrhs, const double* num, bool cnum,
           const double* den, double sign, double* pp, hipStream_t st, int dstr) {
  if (n % Vec<T>::V) return fail(DWF_ERR_ARG, "16-bit fields need a multiple of 4 complex values");
  if (nrhs > 64) return fail(DWF_ERR_ARG, "nrhs > 64");
  hipLaunchKernelGGL((k_xpay<T>), dim3(nblocks(n), nrhs), dim3(kT), 0, st, p, y, n, num, cnum, den,
                     sign, red, pp, dstr);
  LAUNCH_CHECK();
  return DWF_OK;
}
template <typename T>
int zero_t(T* y, size_t total, hipStream_t st) {
  if (total % Vec<T>::V) return fail(DWF_ERR_ARG, "16-bit fields need a multiple of 4 complex values");
  hipLaunchKernelGGL((k_zero<T>), dim3(nblocks(total)), dim3(kT), 0, st, y, total);
  LAUNCH_CHECK();
  return DWF_OK;
}

template <typename R>
int b_norm2(Red red, const cplx<R>* x, size_t n, int nrhs, double* res, hipStream_t st) {
  return norm2_t(red, x, n, nrhs, res, st);
}
template <typename R>
int b_dot(Red red, const cplx<R>* a, const cplx<R>* b, size_t n, int nrhs, double* res,
          hipStream_t st) {
  return dot_t(red, a, b, n, nrhs, res, st);
}
template <typename R>
int b_update(Red red, cplx<R>* x, cplx<R>* r, const cplx<R>* p, const cplx<R>* w, size_t n,
             int nrhs, const double* num, bool cnum, const double* den, const double* den2,
             double lam, double* rr, hipStream_t st, int dstr, int mode) {
  return update_t(red, x, r, p, w, n, nrhs, num, cnum, den, den2, lam, rr, st, dstr, mode);
}
template <typename R>
int b_xpay(Red red, cplx<R>* p, const cplx<R>* y, size_t n, int nrhs, const double* num, bool cnum,
           const double* den, double sign, double* pp, hipStream_t st, int dstr) {
  return xpay_t(red, p, y, n, nrhs, num, cnum, den, sign, pp, st, dstr);
}
int b_norm2(Red red, const bf16c* x, size_t n, int nrhs, double* res, hipStream_t st) {
  return norm2_t(red, x, n, nrhs, res, st);
}
int b_update(Red red, bf16c* x, bf16c* r, const bf16c* p, const bf16c* w, size_t n, int nrhs,
             const double* num, const double* den, const double* den2, double lam, double* rr,
             hipStream_t st, int mode) {
  return update_t(red, x, r, p, w, n, nrhs, num, false, den, den2, lam, rr, st, 1, mode);
}
int b_mirs16_init(Red red, bf16c* r, bf16c* p, const c64* b, size_t n, int nrhs, int Ls, double* rr,
                  hipStream_t st) {
  if (n % 12 || (n / 12) % Ls) return fail(DWF_ERR_ARG, "M_IRS: field size not a whole number of site rows");
  if (nrhs > 64) return fail(DWF_ERR_ARG, "nrhs > 64");
  hipLaunchKernelGGL(k_mirs16_init, dim3(nblocks(n), nrhs), dim3(kT), 0, st, r, p, b, n / 12, Ls, red, rr);
  LAUNCH_CHECK();
  return DWF_OK;
}
int b_mirs16_last(c64* x_out, const bf16c* x, const bf16c* p, size_t n, int nrhs, int Ls, const double* num,
                  const double* den, const double* den2, double lam, hipStream_t st) {
  if (n % 12 || (n / 12) % Ls) return fail(DWF_ERR_ARG, "M_IRS: field size not a whole number of site rows");
  hipLaunchKernelGGL(k_mirs16_last, dim3(nblocks(n), nrhs), dim3(kT), 0, st, x_out, x, p, n / 12, Ls, num, den,
                     den2, lam);
  LAUNCH_CHECK();
  return DWF_OK;
}
int b_xpay(Red red, bf16c* p, const bf16c* y, size_t n, int nrhs, const double* num,
           const double* den, double* pp, hipStream_t st) {
  return xpay_t(red, p, y, n, nrhs, num, false, den, 1.0, pp, st, 1);
}
int b_zero(bf16c* y, size_t total, hipStream_t st) { return zero_t(y, total, st); }
template <typename R>
int b_axpby(cplx<R>* y, const cplx<R>* x, double a, double b, size_t total, hipStream_t st) {
  hipLaunchKernelGGL((k_axpby<R>), dim3(nblocks(total)), dim3(kT), 0, st, y, x, (R)a, (R)b, total);
  LAUNCH_CHECK();
  return DWF_OK;
}
template <typename Ry, typename Rx>
int b_axpy_mixed(cplx<Ry>* y, const cplx<Rx>* x, const double* s, size_t n, int nrhs,
                 hipStream_t st, bool sqrt_s) {
  hipLaunchKernelGGL((k_axpy_mixed<Ry, Rx>), dim3(nblocks(n), nrhs), dim3(kT), 0, st, y, x, s, n, sqrt_s);
  LAUNCH_CHECK();
  return DWF_OK;
}
template <typename Ry, typename Rx>
int b_scale_copy(cplx<Ry>* y, const cplx<Rx>* x, const double* v, bool invsqrt, size_t n, int nrhs,
                 hipStream_t st) {
  hipLaunchKernelGGL((k_scale_copy<Ry, Rx>), dim3(nblocks(n), nrhs), dim3(kT), 0, st, y, x, v,
                     invsqrt, n);
  LAUNCH_CHECK();
  return DWF_OK;
}
template <typename R>
int b_zero(cplx<R>* y, size_t total, hipStream_t st) {
  return zero_t(y, total, st);
}

#define INST(R)                                                                                   \
  template int b_norm2<R>(Red, const cplx<R>*, size_t, int, double*, hipStream_t);               \
  template int b_dot<R>(Red, const cplx<R>*, const cplx<R>*, size_t, int, double*, hipStream_t); \
  template int b_update<R>(Red, cplx<R>*, cplx<R>*, const cplx<R>*, const cplx<R>*, size_t, int, \
                           const double*, bool, const double*, const double*, double, double*,   \
                           hipStream_t, int, int);                                                \
  template int b_xpay<R>(Red, cplx<R>*, const cplx<R>*, size_t, int, const double*, bool,        \
                         const double*, double, double*, hipStream_t, int);                       \
  template int b_axpby<R>(cplx<R>*, const cplx<R>*, double, double, size_t, hipStream_t);        \
  template int b_zero<R>(cplx<R>*, size_t, hipStream_t);
INST(double)
INST(float)
template int b_axpy_mixed<double, float>(cplx<double>*, const cplx<float>*, const double*, size_t, int, hipStream_t, bool);
template int b_axpy_mixed<double, double>(cplx<double>*, const cplx<double>*, const double*, size_t, int, hipStream_t, bool);
template int b_axpy_mixed<float, float>(cplx<float>*, const cplx<float>*, const double*, size_t, int, hipStream_t, bool);
template int b_scale_copy<float, double>(cplx<float>*, const cplx<double>*, const double*, bool, size_t, int, hipStream_t);
template int b_scale_copy<double, float>(cplx<double>*, const cplx<float>*, const double*, bool, size_t, int, hipStream_t);
template int b_scale_copy<double, double>(cplx<double>*, const cplx<double>*, const double*, bool, size_t, int, hipStream_t);
template int b_scale_copy<float, float>(cplx<float>*, const cplx<float>*, const double*, bool, size_t, int, hipStream_t);

}  // namespace hdk
