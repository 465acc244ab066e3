// BLAS-1 kernels over complex vectors of n elements per right-hand side,
// nrhs right-hand sides stored one after another, FP64 accumulation for
// every reduction (deterministic two-stage sums).  Scalars produced by one
// kernel and consumed by the next stay in device memory, so a solver
// iteration needs no host round trip.
#pragma once

#include "common.h"

namespace hdk {

struct Red {
  double* partials;   // [64][kMaxPartials]
  unsigned* counters; // [64]
};

// res[rhs] = |x_rhs|^2
template <typename R>
int b_norm2(Red red, const cplx<R>* x, size_t n, int nrhs, double* res, hipStream_t st);
// res[2 rhs], res[2 rhs + 1] = <a_rhs, b_rhs> = sum conj(a) b
template <typename R>
int b_dot(Red red, const cplx<R>* a, const cplx<R>* b, size_t n, int nrhs, double* res,
          hipStream_t st);
// alpha = num / (den + lam * den2)   (num complex when cnum, den2 optional;
// den read with stride dstr, e.g. 2 for the real parts of dot results; a zero
// denominator gives a zero coefficient)
// x += alpha p ; r -= alpha (w + lam p) ; rr[rhs] = |r|^2 (if rr)
// mode bits: kUpdX0, x is zero (not read: x = alpha p); kUpdXOnly, only x
// is updated (r, w, rr untouched: the last step of a fixed-count CG)
constexpr int kUpdX0 = 1, kUpdXOnly = 2;
template <typename R>
int b_update(Red red, cplx<R>* x, cplx<R>* r, const cplx<R>* p, const cplx<R>* w, size_t n,
             int nrhs, const double* num, bool cnum, const double* den, const double* den2,
             double lam, double* rr, hipStream_t st, int dstr = 1, int mode = 0);
// beta = sign * num / den (num complex when cnum) ; p = y + beta p ;
// pp[rhs] = |p|^2 (if pp)
template <typename R>
int b_xpay(Red red, cplx<R>* p, const cplx<R>* y, size_t n, int nrhs, const double* num, bool cnum,
           const double* den, double sign, double* pp, hipStream_t st, int dstr = 1);
// y = a x + b y over `total` elements (host coefficients)
template <typename R>
int b_axpby(cplx<R>* y, const cplx<R>* x, double a, double b, size_t total, hipStream_t st);
// y (Ry) += f[rhs] * x (Rx): f = s[rhs] (or sqrt(s[rhs]) when sqrt_s; 1 when s == nullptr)
template <typename Ry, typename Rx>
int b_axpy_mixed(cplx<Ry>* y, const cplx<Rx>* x, const double* s, size_t n, int nrhs,
                 hipStream_t st, bool sqrt_s = false);
// y (Ry) = s[rhs] * x (Rx); s = 1/sqrt(v[rhs]) when invsqrt, else s = v[rhs]
template <typename Ry, typename Rx>
int b_scale_copy(cplx<Ry>* y, const cplx<Rx>* x, const double* v, bool invsqrt, size_t n, int nrhs,
                 hipStream_t st);
// y = 0
template <typename R>
int b_zero(cplx<R>* y, size_t total, hipStream_t st);

// The real-coefficient forms of the above on fields stored in 16 bits
// (bf16c): FP32 arithmetic on each loaded value, results rounded to nearest
// even on store, FP64 accumulation of the norms.
int b_norm2(Red red, const bf16c* x, size_t n, int nrhs, double* res, hipStream_t st);
int b_update(Red red, bf16c* x, bf16c* r, const bf16c* p, const bf16c* w, size_t n, int nrhs,
             const double* num, const double* den, const double* den2, double lam, double* rr,
             hipStream_t st, int mode = 0);
// fixed-count CG on 16-bit fields: r = p = 16-bit b (complex64 [site][12][Ls]
// to the 16-bit [site][Ls][12] layout), rr = |r|^2 of the stored values; and
// its last step x_out (complex64 layout) = 16-bit(x + alpha p), x == nullptr
// meaning zero, alpha = num / (den + lam den2)
int b_mirs16_init(Red red, bf16c* r, bf16c* p, const c64* b, size_t n, int nrhs, int Ls, double* rr,
                  hipStream_t st);
int b_mirs16_last(c64* x_out, const bf16c* x, const bf16c* p, size_t n, int nrhs, int Ls, const double* num,
                  const double* den, const double* den2, double lam, hipStream_t st);
int b_xpay(Red red, bf16c* p, const bf16c* y, size_t n, int nrhs, const double* num,
           const double* den, double* pp, hipStream_t st);
int b_zero(bf16c* y, size_t total, hipStream_t st);

}  // namespace hdk
