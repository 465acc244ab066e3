// The truncated little Dirac operator and the ADEF1 preconditioner of the
// coarse solve (Sec. V.B, "Truncated little Dirac operator as
// preconditioner"; the optimised parameters of Table "optimised": Chebyshev
// bounds 0.5 and 45, order 16).
//
// Q_trunc keeps of the 81-point little Dirac operator only the zero- and
// one-hop terms (the site itself and its eight axis neighbours; the Table
// "frobnorm" coupling norms fall by two orders of magnitude per hop), plus an
// optional infra-red shift on the diagonal: nine matrices per site, a ninth
// of the bytes of A.  It is stored like AT64 / AT128, transposed per stencil
// point, TT[a][m][k][j] = A[a][l_m][j][k] (+ shift delta_jk at m = 0).
//
// The high-mode preconditioner M is the Chebyshev iteration for
// (Q_trunc + shift) y = u from y = 0 with the spectrum taken in [lo, hi]:
// the residual is R_n(x) u, R_n(x) = T_n((d - x)/c) / T_n(d/c),
// d = (hi + lo)/2, c = (hi - lo)/2.  With sigma = d/c and
// omega_1 = 2, omega_{k+1} = 1 / (1 - omega_k / (4 sigma^2)):
//     delta_1 = u / d,   y = delta_1,   res = u
//     res -= Q_trunc delta_k;  delta_{k+1} = (omega_{k+1}/d) res + (omega_{k+1} - 1) delta_k;  y += delta_{k+1}
// for k = 1 .. n-1.  One kernel per step: the truncated mat-vec of delta_k
// for a site and the three site-local updates (delta ping-pongs between two
// buffers because neighbours read delta_k).
//
// or, the paper's alternative, M_IRS(Q_trunc): a fixed number of CG
// iterations on (Q_trunc + shift) y = u from y = 0.
//
// ADEF1 (the second level, Z orthonormal with Z^+ A Z = diag(D), A Z stored):
//     M_1 r = M (r - A Z D^-1 Z^+ r) + Z D^-1 Z^+ r
// needs no application of the untruncated A.
#include <algorithm>
#include <cmath>
#include <vector>

#include "coarse_dev.h"

namespace hdk {

namespace {

constexpr int kTS = kOneHop;

template <typename R>
__global__ void k_trunc_build(cplx<R>* __restrict__ TT, const c128* __restrict__ A, int Nc, int nvec, double shift) {
  const size_t total = (size_t)Nc * kTS * nvec * nvec;
  for (size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x; idx < total; idx += (size_t)gridDim.x * blockDim.x) {
    const int j = (int)(idx % nvec);
    const int k = (int)((idx / nvec) % nvec);
    const size_t am = idx / ((size_t)nvec * nvec);
    const int m = (int)(am % kTS);
    const size_t a = am / kTS;
    c128 v = A[((a * kStencil + one_hop_l(m)) * nvec + j) * nvec + k];
    if (m == 0 && j == k) v.re += shift;
    TT[idx] = cmk((R)v.re, (R)v.im);
  }
}

__global__ void k_nbr9(int* __restrict__ nbr9, const int* __restrict__ nbr, int Nc) {
  const int idx = blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= Nc * kTS) return;
  const int a = idx / kTS, m = idx - a * kTS;
  nbr9[idx] = nbr[(size_t)a * kStencil + one_hop_l(m)];
}

template <typename R, int NR, int U>
__global__ void __launch_bounds__(kCT)
k_trunc_apply(const cplx<R>* __restrict__ TT, const int* __restrict__ nbr9, const cplx<R>* __restrict__ in,
              cplx<R>* __restrict__ out, int Nc, int nvec, int nr) {
  __shared__ cplx<R> red[kCT * NR];
  capply_site<R, NR, U, false, kTS>(TT, nbr9, in, out, blockIdx.x, Nc, nvec, nr, blockIdx.y * NR, red);
}

// One Chebyshev step at the sites of this workgroup: tw = Q_trunc dcur, then
// res -= tw, dnext = ca res + cb dcur, y += dnext.  A thread updates the
// entries of tw it stored itself.
template <typename R, int NR, int U>
__global__ void __launch_bounds__(kCT)
k_cheb_step(const cplx<R>* __restrict__ TT, const int* __restrict__ nbr9, const cplx<R>* __restrict__ dcur,
            cplx<R>* __restrict__ dnext, cplx<R>* __restrict__ res, cplx<R>* __restrict__ y, cplx<R>* __restrict__ tw,
            int Nc, int nvec, int nr, double ca, double cb) {
  __shared__ cplx<R> red[kCT * NR];
  const int a = blockIdx.x, r0 = blockIdx.y * NR;
  capply_site<R, NR, U, false, kTS>(TT, nbr9, dcur, tw, a, Nc, nvec, nr, r0, red);
  if (threadIdx.x >= nvec) return;
#pragma unroll
  for (int r = 0; r < NR; ++r) {
    if (r0 + r >= nr) break;
    const size_t idx = ((size_t)(r0 + r) * Nc + a) * nvec + threadIdx.x;
    const cplx<R> t = tw[idx], rv = res[idx], dv = dcur[idx], yv = y[idx];
    const double rre = (double)rv.re - t.re, rim = (double)rv.im - t.im;
    const double dre = ca * rre + cb * dv.re, dim = ca * rim + cb * dv.im;
    res[idx] = cmk((R)rre, (R)rim);
    dnext[idx] = cmk((R)dre, (R)dim);
    y[idx] = cmk((R)(yv.re + dre), (R)(yv.im + dim));
  }
}

// The same with the nine-point operand of the workgroup's NR right-hand
// sides first gathered into LDS (one coalesced pass), so the column loop
// streams only the operator.
constexpr int kStageNvec = 64;
template <typename R, int NR, int U>
__global__ void __launch_bounds__(kCT)
k_cheb_step_staged(const cplx<R>* __restrict__ TT, const int* __restrict__ nbr9, const cplx<R>* __restrict__ dcur,
                   cplx<R>* __restrict__ dnext, cplx<R>* __restrict__ res, cplx<R>* __restrict__ y,
                   cplx<R>* __restrict__ tw, int Nc, int nvec, int nr, double ca, double cb) {
  __shared__ cplx<R> red[kCT * NR];
  __shared__ cplx<R> s_in[NR * kTS * kStageNvec];
  const int a = blockIdx.x, r0 = blockIdx.y * NR;
  const int K = kTS * nvec;
  const int* nb = nbr9 + (size_t)a * kTS;
  for (int e = threadIdx.x; e < NR * K; e += kCT) {
    const int r = e / K, rem = e - r * K, m = rem / nvec;
    s_in[e] = r0 + r < nr ? dcur[((size_t)(r0 + r) * Nc + nb[m]) * nvec + (rem - m * nvec)] : cmk((R)0, (R)0);
  }
  __syncthreads();
  capply_site<R, NR, U, true, kTS>(TT, nbr9, s_in, tw, a, Nc, nvec, nr, r0, red);
  if (threadIdx.x >= nvec) return;
#pragma unroll
  for (int r = 0; r < NR; ++r) {
    if (r0 + r >= nr) break;
    const size_t idx = ((size_t)(r0 + r) * Nc + a) * nvec + threadIdx.x;
    // point 0 of the staged operand is the site itself
    const cplx<R> t = tw[idx], rv = res[idx], dv = s_in[r * K + threadIdx.x], yv = y[idx];
    const double rre = (double)rv.re - t.re, rim = (double)rv.im - t.im;
    const double dre = ca * rre + cb * dv.re, dim = ca * rim + cb * dv.im;
    res[idx] = cmk((R)rre, (R)rim);
    dnext[idx] = cmk((R)dre, (R)dim);
    y[idx] = cmk((R)(yv.re + dre), (R)(yv.im + dim));
  }
}

template <typename R, int U>
__global__ void __launch_bounds__(kCT)
k_trunc_apply1(const cplx<R>* __restrict__ TT, const int* __restrict__ nbr9, const cplx<R>* __restrict__ in,
               cplx<R>* __restrict__ out, int Nc, int nvec) {
  __shared__ cplx<R> red[kCT];
  __shared__ cplx<R> s_in[kTS * kStageNvec];
  const int a = blockIdx.x;
  const int* nb = nbr9 + (size_t)a * kTS;
  for (int e = threadIdx.x; e < kTS * nvec; e += kCT) {
    const int m = e / nvec;
    s_in[e] = in[(size_t)nb[m] * nvec + (e - m * nvec)];
  }
  __syncthreads();
  capply_site<R, 1, U, true, kTS>(TT, nbr9, s_in, out, a, Nc, nvec, 1, 0, red);
}

// d1 = u / d; y = d1 (acc = 0) or y += d1 (acc = 1)
template <typename R>
__global__ void k_cheb_first(cplx<R>* __restrict__ d1, cplx<R>* __restrict__ y, const cplx<R>* __restrict__ u,
                             size_t total, double inv_d, int acc) {
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= total) return;
  const cplx<R> v = u[i];
  const cplx<R> dv = cmk((R)(inv_d * v.re), (R)(inv_d * v.im));
  d1[i] = dv;
  if (acc) {
    const cplx<R> yv = y[i];
    y[i] = cmk((R)(yv.re + dv.re), (R)(yv.im + dv.im));
  } else {
    y[i] = dv;
  }
}

// res -= tw, dnext = ca res + cb dcur, y += dnext (the updates of
// k_cheb_step after a separate mat-vec tw = Q_trunc dcur)
template <typename R>
__global__ void k_cheb_update(const cplx<R>* __restrict__ tw, cplx<R>* __restrict__ res,
                              const cplx<R>* __restrict__ dcur, cplx<R>* __restrict__ dnext, cplx<R>* __restrict__ y,
                              size_t total, double ca, double cb) {
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= total) return;
  const cplx<R> t = tw[i], rv = res[i], dv = dcur[i], yv = y[i];
  const double rre = (double)rv.re - t.re, rim = (double)rv.im - t.im;
  const double dre = ca * rre + cb * dv.re, dim = ca * rim + cb * dv.im;
  res[i] = cmk((R)rre, (R)rim);
  dnext[i] = cmk((R)dre, (R)dim);
  y[i] = cmk((R)(yv.re + dre), (R)(yv.im + dim));
}

template <typename R>
DevBuf& tt_buf(hdcg* h) {
  return sizeof(R) == 8 ? h->TT128 : h->TT64;
}
template <typename R>
double& tt_shift(hdcg* h) {
  return sizeof(R) == 8 ? h->tt_shift128 : h->tt_shift64;
}

// TT (in R) and the neighbour table for the current shift
// the 16-bit storage of Q_trunc in use for complex64 vectors (0: complex64)
template <typename R>
int trunc16_prec(hdcg* h) {
  return sizeof(R) == 4 && (h->prm.m1_prec == DWF_BF16 || h->prm.m1_prec == DWF_F16) ? h->prm.m1_prec : 0;
}

template <typename R>
int trunc_ensure(hdcg* h, hipStream_t st) {
  const double shift = h->prm.m1_shift;
  if (h->A128.bytes == 0) return fail(DWF_ERR_ARG, "the truncated operator needs the little Dirac operator");
  if (h->nbr9.bytes == 0) {
    HDCG_TRY(h->nbr9.ensure(sizeof(int) * (size_t)h->Nc * kTS));
    const int n = h->Nc * kTS;
    hipLaunchKernelGGL(k_nbr9, dim3((n + 255) / 256), dim3(256), 0, st, h->nbr9.as<int>(), h->nbr.as<int>(), h->Nc);
    HDCG_HIP(hipGetLastError());
  }
  if (const int p16 = trunc16_prec<R>(h)) {
    if ((p16 == DWF_BF16 ? h->tq_shift_bf16 : h->tq_shift_f16) == shift) return DWF_OK;
    return trunc16_build(h, p16, shift, st);
  }
  DevBuf& TT = tt_buf<R>(h);
  if (TT.bytes != 0 && tt_shift<R>(h) == shift) return DWF_OK;
  const size_t total = (size_t)h->Nc * kTS * h->nvec * h->nvec;
  HDCG_TRY(TT.ensure(sizeof(cplx<R>) * total));
  const unsigned grid = (unsigned)std::min<size_t>((total + 255) / 256, 65536);
  hipLaunchKernelGGL((k_trunc_build<R>), dim3(grid), dim3(256), 0, st, TT.as<cplx<R>>(), h->A128.as<c128>(), h->Nc,
                     h->nvec, shift);
  HDCG_HIP(hipGetLastError());
  tt_shift<R>(h) = shift;
  return DWF_OK;
}

constexpr int kMaxOrder = 256;

template <typename R>
int trunc_launch(hdcg* h, const cplx<R>* in, cplx<R>* out, int nr, hipStream_t st) {
  if constexpr (sizeof(R) == 4) {
    if (const int p16 = trunc16_prec<R>(h)) return trunc16_apply(h, p16, in, out, nr, st);
  }
  if (nr == 1 && h->nvec <= kStageNvec) {
    hipLaunchKernelGGL((k_trunc_apply1<R, 16>), dim3(h->Nc), dim3(kCT), 0, st, tt_buf<R>(h).template as<cplx<R>>(),
                       h->nbr9.as<int>(), in, out, h->Nc, h->nvec);
    HDCG_HIP(hipGetLastError());
    return DWF_OK;
  }
  constexpr int NR = sizeof(R) == 8 ? 2 : 4;
  hipLaunchKernelGGL((k_trunc_apply<R, NR, 8>), dim3(h->Nc, (nr + NR - 1) / NR), dim3(kCT), 0, st,
                     tt_buf<R>(h).template as<cplx<R>>(), h->nbr9.as<int>(), in, out, h->Nc, h->nvec, nr);
  HDCG_HIP(hipGetLastError());
  return DWF_OK;
}

// y = (acc ? y : 0) + p(Q_trunc + shift) u; u is overwritten (it ends as the
// Chebyshev residual)
template <typename R>
int cheb_run(hdcg* h, cplx<R>* y, cplx<R>* u, int nr, bool acc, double lo, double hi, hipStream_t st) {
  const size_t n = (size_t)h->Nc * h->nvec * nr;
  for (int i = 6; i < 9; ++i) HDCG_TRY(h->cw[i].ensure(n * sizeof(c128)));
  cplx<R>* dl[2] = {h->cw[6].as<cplx<R>>(), h->cw[7].as<cplx<R>>()};
  cplx<R>* tw = h->cw[8].as<cplx<R>>();
  const double d = 0.5 * (hi + lo), c = 0.5 * (hi - lo), sigma = d / c;
  hipLaunchKernelGGL((k_cheb_first<R>), dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, dl[0], y, u, n, 1.0 / d,
                     acc ? 1 : 0);
  HDCG_HIP(hipGetLastError());
  constexpr int NR = sizeof(R) == 8 ? 2 : 4;
  double omega = 2.0;
  for (int k = 1; k < h->prm.m1_order; ++k) {
    omega = 1.0 / (1.0 - omega / (4.0 * sigma * sigma));
    if (trunc16_prec<R>(h)) {  // the 16-bit mat-vec, then the site-local updates
      HDCG_TRY(trunc_launch<R>(h, dl[(k - 1) & 1], tw, nr, st));
      hipLaunchKernelGGL((k_cheb_update<R>), dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, tw, u, dl[(k - 1) & 1],
                         dl[k & 1], y, n, omega / d, omega - 1.0);
      HDCG_HIP(hipGetLastError());
      continue;
    }
    if (h->nvec <= kStageNvec) {
      const cplx<R>* TTp = tt_buf<R>(h).template as<cplx<R>>();
      if (nr == 1)
        hipLaunchKernelGGL((k_cheb_step_staged<R, 1, 16>), dim3(h->Nc, 1), dim3(kCT), 0, st, TTp, h->nbr9.as<int>(),
                           dl[(k - 1) & 1], dl[k & 1], u, y, tw, h->Nc, h->nvec, nr, omega / d, omega - 1.0);
      else
        hipLaunchKernelGGL((k_cheb_step_staged<R, NR, 16 / NR>), dim3(h->Nc, (nr + NR - 1) / NR), dim3(kCT), 0, st,
                           TTp, h->nbr9.as<int>(), dl[(k - 1) & 1], dl[k & 1], u, y, tw, h->Nc, h->nvec, nr,
                           omega / d, omega - 1.0);
      HDCG_HIP(hipGetLastError());
      continue;
    }
    hipLaunchKernelGGL((k_cheb_step<R, NR, 8>), dim3(h->Nc, (nr + NR - 1) / NR), dim3(kCT), 0, st,
                       tt_buf<R>(h).template as<cplx<R>>(), h->nbr9.as<int>(), dl[(k - 1) & 1], dl[k & 1], u, y, tw,
                       h->Nc, h->nvec, nr, omega / d, omega - 1.0);
    HDCG_HIP(hipGetLastError());
  }
  return DWF_OK;
}

// y = (acc ? y : 0) + x_n, x_n the n-th iterate (n = m1_order) of CG on
// (Q_trunc + shift) x = u from x = 0: the infra-red shifted preconditioner
// M_IRS(Q_trunc, n, shift) of Sec. IV.C on the truncated operator (the
// paper's alternative to the Chebyshev polynomial).  Every step runs for
// every right-hand side with its own alpha and beta in device memory (a zero
// residual gives zero coefficients), so nothing waits for the host.  u is
// overwritten (it ends as the CG residual).
template <typename R>
int mirs_run(hdcg* h, cplx<R>* y, cplx<R>* u, int nr, bool acc, hipStream_t st) {
  const size_t n = (size_t)h->Nc * h->nvec;
  for (int i = 6; i < 8; ++i) HDCG_TRY(h->cw[i].ensure(n * nr * sizeof(c128)));
  HDCG_TRY(h->cw[8].ensure(std::max<size_t>(n * nr * sizeof(c128), 4 * 64 * sizeof(double))));
  cplx<R>* p = h->cw[6].as<cplx<R>>();
  cplx<R>* w = h->cw[7].as<cplx<R>>();
  double* sc = h->cw[8].as<double>();
  double* rr[2] = {sc, sc + 64};
  double* pw = sc + 128;  // complex (p, w) per right-hand side
  const Red red{h->op->red.partials.as<double>(), h->op->red.counters.as<unsigned>()};
  if (!acc) HDCG_TRY(b_zero<R>(y, n * nr, st));
  HDCG_TRY(b_norm2<R>(red, u, n, nr, rr[0], st));
  HDCG_HIP(hipMemcpyAsync(p, u, n * nr * sizeof(cplx<R>), hipMemcpyDeviceToDevice, st));
  for (int k = 0; k < h->prm.m1_order; ++k) {
    HDCG_TRY(trunc_launch<R>(h, p, w, nr, st));
    HDCG_TRY(b_dot<R>(red, p, w, n, nr, pw, st));
    // y += alpha p, u -= alpha w, alpha = |u|^2 / (p, w); then p = u + beta p
    HDCG_TRY(b_update<R>(red, y, u, p, w, n, nr, rr[k & 1], false, pw, nullptr, 0.0, rr[(k + 1) & 1], st, 2));
    if (k + 1 < h->prm.m1_order)
      HDCG_TRY(b_xpay<R>(red, p, u, n, nr, rr[(k + 1) & 1], false, rr[k & 1], 1.0, nullptr, st));
  }
  return DWF_OK;
}

}  // namespace

void trunc_invalidate(hdcg* h) {
  h->tt_shift64 = h->tt_shift128 = std::nan("");
  h->tq_shift_bf16 = h->tq_shift_f16 = std::nan("");
  h->m1_hi_est = 0.0;
}

template <typename R>
int trunc_apply(hdcg* h, const cplx<R>* in, cplx<R>* out, int nr, hipStream_t st) {
  if (h->nvec > kCT) return fail(DWF_ERR_ARG, "nvec too large for the coarse mat-vec");
  HDCG_TRY(trunc_ensure<R>(h, st));
  return trunc_launch<R>(h, in, out, nr, st);
}

// The Chebyshev interval: lo = m1_lo, hi = m1_hi, or when m1_hi <= 0 1.05
// times |Q_trunc v| for the unit v that 30 steps of the power method (from a
// fixed pseudo-random start) leave, an estimate of the largest eigenvalue
// from below; a slight underestimate only leaves the few modes above hi
// damped a little less (R_n stays far below 1 just above hi).
int m1_bounds(hdcg* h, double* lo, double* hi, hipStream_t st) {
  *lo = h->prm.m1_lo;
  if (h->prm.m1_hi > 0.0) {
    *hi = h->prm.m1_hi;
    return DWF_OK;  // m1_hi > m1_lo is checked with the parameters
  }
  if (h->m1_hi_est > 0.0) {
    *hi = h->m1_hi_est;
    if (!(*hi > *lo)) return fail(DWF_ERR_NUMERIC, "Chebyshev upper bound estimate not above m1_lo");
    return DWF_OK;
  }
  HDCG_TRY(trunc_ensure<float>(h, st));
  const size_t n = (size_t)h->Nc * h->nvec;
  for (int i = 6; i < 9; ++i) HDCG_TRY(h->cw[i].ensure(n * sizeof(c128)));
  c64* v = h->cw[6].as<c64>();
  c64* w = h->cw[7].as<c64>();
  double* sn = h->cw[8].as<double>();  // |Q_trunc v|^2
  std::vector<c64> hv(n);
  unsigned long long s = 0x9E3779B97F4A7C15ull;
  double nrm = 0.0;
  for (size_t i = 0; i < n; ++i) {
    float p[2];
    for (float& q : p) {
      s = s * 6364136223846793005ull + 1442695040888963407ull;
      q = (float)((double)(s >> 11) * (1.0 / 9007199254740992.0) - 0.5);
    }
    hv[i] = cmk(p[0], p[1]);
    nrm += (double)p[0] * p[0] + (double)p[1] * p[1];
  }
  const float inv = (float)(1.0 / std::sqrt(nrm));
  for (auto& x : hv) x = cmk(x.re * inv, x.im * inv);
  HDCG_HIP(hipMemcpyAsync(v, hv.data(), n * sizeof(c64), hipMemcpyHostToDevice, st));
  const Red red{h->op->red.partials.as<double>(), h->op->red.counters.as<unsigned>()};
  for (int it = 0; it < 30; ++it) {
    HDCG_TRY(trunc_launch<float>(h, v, w, 1, st));
    HDCG_TRY(b_norm2<float>(red, w, n, 1, sn, st));
    if (it < 29) HDCG_TRY((b_scale_copy<float, float>(v, w, sn, true, n, 1, st)));
  }
  HDCG_HIP(hipMemcpyAsync(h->pinned + 64 * 15, sn, sizeof(double), hipMemcpyDeviceToHost, st));
  HDCG_HIP(hipStreamSynchronize(st));
  const double lam = std::sqrt(h->pinned[64 * 15]);
  if (!std::isfinite(lam) || !(lam > 0.0)) return fail(DWF_ERR_NUMERIC, "Chebyshev upper bound estimate not positive");
  h->m1_hi_est = 1.05 * lam;
  *hi = h->m1_hi_est;
  if (!(*hi > *lo)) return fail(DWF_ERR_NUMERIC, "Chebyshev upper bound estimate not above m1_lo");
  return DWF_OK;
}

template <typename R>
int m1_chebyshev(hdcg* h, cplx<R>* y, const cplx<R>* r, int nr, hipStream_t st) {
  double lo = 0, hi = 0;
  HDCG_TRY(m1_bounds(h, &lo, &hi, st));
  HDCG_TRY(trunc_ensure<R>(h, st));
  const size_t n = (size_t)h->Nc * h->nvec * nr;
  HDCG_TRY(h->cw[9].ensure(n * sizeof(c128)));
  cplx<R>* u = h->cw[9].as<cplx<R>>();
  HDCG_HIP(hipMemcpyAsync(u, r, n * sizeof(cplx<R>), hipMemcpyDeviceToDevice, st));
  return cheb_run<R>(h, y, u, nr, false, lo, hi, st);
}

template <typename R>
int m1_trunc_cg(hdcg* h, cplx<R>* y, const cplx<R>* r, int nr, hipStream_t st) {
  HDCG_TRY(trunc_ensure<R>(h, st));
  const size_t n = (size_t)h->Nc * h->nvec * nr;
  HDCG_TRY(h->cw[9].ensure(n * sizeof(c128)));
  cplx<R>* u = h->cw[9].as<cplx<R>>();
  HDCG_HIP(hipMemcpyAsync(u, r, n * sizeof(cplx<R>), hipMemcpyDeviceToDevice, st));
  return mirs_run<R>(h, y, u, nr, false, st);
}

// M is the Chebyshev polynomial (ldop_m1 = 1) or M_IRS(Q_trunc) (ldop_m1 = 2)
template <typename R>
int m1_adef1(hdcg* h, cplx<R>* y, const cplx<R>* r, int nr, hipStream_t st) {
  if (h->ng == 0) return fail(DWF_ERR_ARG, "ADEF1 needs the second deflation level (hdcg_ldop_setup)");
  const bool cg = h->prm.ldop_m1 == 2;
  double lo = 0, hi = 0;
  if (!cg) HDCG_TRY(m1_bounds(h, &lo, &hi, st));
  HDCG_TRY(trunc_ensure<R>(h, st));
  const size_t n = (size_t)h->Nc * h->nvec * nr;
  HDCG_TRY(h->cw[9].ensure(n * sizeof(c128)));
  cplx<R>* u = h->cw[9].as<cplx<R>>();
  const cplx<R>* Z = reinterpret_cast<const cplx<R>*>(sizeof(R) == 8 ? h->ldZ128.ptr : h->ldZ64.ptr);
  const cplx<R>* AZ = reinterpret_cast<const cplx<R>*>(sizeof(R) == 8 ? h->ldAZ128.ptr : h->ldAZ64.ptr);
  // c = D^-1 Z^+ r ; u = r - A Z c ; y = Z c ; y += p(Q_trunc) u
  HDCG_TRY(ldop_coef<R>(h, Z, r, nr, st));
  HDCG_TRY(ldop_apply<R>(h, u, r, nullptr, nullptr, AZ, nr, -1.0, true, st));
  HDCG_TRY(ldop_apply<R>(h, y, nullptr, nullptr, nullptr, Z, nr, 1.0, false, st));
  return cg ? mirs_run<R>(h, y, u, nr, true, st) : cheb_run<R>(h, y, u, nr, true, lo, hi, st);
}

int m1_check_params(int ldop_m1, double lo, double hi, int order, double shift) {
  if (ldop_m1 < 0 || ldop_m1 > 2) return fail(DWF_ERR_ARG, "ldop_m1 must be 0, 1 or 2");
  if (!(lo > 0.0) || !(hi == 0.0 || hi > lo) || order < 1 || order > kMaxOrder || !(shift >= 0.0))
    return fail(DWF_ERR_ARG, "truncated-operator preconditioner: need m1_lo > 0, m1_hi = 0 or > m1_lo, "
                             "1 <= m1_order <= 256, m1_shift >= 0");
  return DWF_OK;
}

template int trunc_apply<float>(hdcg*, const c64*, c64*, int, hipStream_t);
template int trunc_apply<double>(hdcg*, const c128*, c128*, int, hipStream_t);
template int m1_chebyshev<float>(hdcg*, c64*, const c64*, int, hipStream_t);
template int m1_chebyshev<double>(hdcg*, c128*, const c128*, int, hipStream_t);
template int m1_trunc_cg<float>(hdcg*, c64*, const c64*, int, hipStream_t);
template int m1_trunc_cg<double>(hdcg*, c128*, const c128*, int, hipStream_t);
template int m1_adef1<float>(hdcg*, c64*, const c64*, int, hipStream_t);
template int m1_adef1<double>(hdcg*, c128*, const c128*, int, hipStream_t);

}  // namespace hdk
