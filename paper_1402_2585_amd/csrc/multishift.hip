// Multi-shift CG on complex128 fields: (H + s_j) x_j = b for j < ns from one
// Krylov space, the one of the smallest shift s_0 (Sec. IV.B: the rational
// filter of the subspace generation is one multi-shift solve).  The other
// shifts' residuals are zeta_j r, and their CG coefficients follow from the
// base system's by the three-term recurrence of zeta.  Every scalar stays on
// the device; the host reads |r|^2 through a pinned ring two iterations
// late.  Also: the rational-filter combination sum_j c_j x_j and the wall
// mask of the subspace noise.
#include <cmath>
#include <cstring>
#include <vector>

#include "fine_op.h"

namespace hdk {

namespace {

constexpr int kT = 256;
constexpr int kMaxShift = 8;

inline int nblocks(size_t n) {
  size_t b = (n + kT * 8 - 1) / (kT * 8);
  if (b < 1) b = 1;
  if (b > 1024) b = 1024;
  return (int)b;
}

// device scalars: per right-hand side (64 slots each), then per
// (right-hand side, shift)
struct MsScal {
  double* rr;         // |r|^2
  double* rrn;        // |r_new|^2
  double* pap;        // |M_pc p_0|^2 (fused into H)
  double* pp;         // |p_0|^2
  double* alpha;      // base CG alpha
  double* alpha_old;  // previous alpha
  double* beta_old;   // previous beta
  double* zeta;       // [rhs][kMaxShift]
  double* zeta_old;
  double* zeta_new;
  double* as;         // alpha_j
  double* bs;         // beta_j
};

MsScal ms_scal(double* base) {
  MsScal s;
  s.rr = base;
  s.rrn = base + 64;
  s.pap = base + 128;
  s.pp = base + 192;
  s.alpha = base + 256;
  s.alpha_old = base + 320;
  s.beta_old = base + 384;
  s.zeta = base + 448;
  s.zeta_old = s.zeta + 64 * kMaxShift;
  s.zeta_new = s.zeta_old + 64 * kMaxShift;
  s.as = s.zeta_new + 64 * kMaxShift;
  s.bs = s.as + 64 * kMaxShift;
  return s;
}
constexpr size_t kMsScalDoubles = 448 + 5 * 64 * kMaxShift;

struct Shifts {
  double s[kMaxShift];
  int ns;
};

__global__ void k_ms_init(MsScal S, int nrhs) {
  const int rhs = threadIdx.x;
  if (rhs >= nrhs) return;
  S.alpha_old[rhs] = 1.0;
  S.beta_old[rhs] = 0.0;
  S.pp[rhs] = S.rr[rhs];
  for (int j = 0; j < kMaxShift; ++j) {
    S.zeta[rhs * kMaxShift + j] = 1.0;
    S.zeta_old[rhs * kMaxShift + j] = 1.0;
  }
}

// alpha = rr / (pap + s_0 pp); zeta_new_j and alpha_j = alpha zeta_new_j / zeta_j
__global__ void k_ms_alpha(MsScal S, Shifts sh, int nrhs) {
  const int rhs = threadIdx.x;
  if (rhs >= nrhs) return;
  const double den = S.pap[rhs] + sh.s[0] * S.pp[rhs];
  const double a = den != 0.0 ? S.rr[rhs] / den : 0.0;
  S.alpha[rhs] = a;
  const double ao = S.alpha_old[rhs], bo = S.beta_old[rhs];
  double* z = S.zeta + rhs * kMaxShift;
  double* zo = S.zeta_old + rhs * kMaxShift;
  double* zn = S.zeta_new + rhs * kMaxShift;
  double* as = S.as + rhs * kMaxShift;
  zn[0] = 1.0;
  as[0] = a;
  for (int j = 1; j < sh.ns; ++j) {
    const double d = sh.s[j] - sh.s[0];
    const double q = a * bo * (zo[j] - z[j]) + zo[j] * ao * (1.0 + d * a);
    // a shift whose residual factor has vanished is converged: freeze it
    const bool live = z[j] != 0.0 && q != 0.0;
    zn[j] = live ? z[j] * zo[j] * ao / q : 0.0;
    as[j] = live ? a * zn[j] / z[j] : 0.0;
  }
}

// beta = rrn / rr, beta_j = beta (zeta_new_j / zeta_j)^2; then the recurrences
// move one step on
__global__ void k_ms_beta(MsScal S, Shifts sh, int nrhs) {
  const int rhs = threadIdx.x;
  if (rhs >= nrhs) return;
  const double b = S.rr[rhs] != 0.0 ? S.rrn[rhs] / S.rr[rhs] : 0.0;
  double* z = S.zeta + rhs * kMaxShift;
  double* zo = S.zeta_old + rhs * kMaxShift;
  double* zn = S.zeta_new + rhs * kMaxShift;
  double* bs = S.bs + rhs * kMaxShift;
  bs[0] = b;
  for (int j = 1; j < sh.ns; ++j) {
    const double f = z[j] != 0.0 ? zn[j] / z[j] : 0.0;
    bs[j] = b * f * f;
  }
  for (int j = 0; j < sh.ns; ++j) {
    zo[j] = z[j];
    z[j] = zn[j];
  }
  S.alpha_old[rhs] = S.alpha[rhs];
  S.beta_old[rhs] = b;
  S.rr[rhs] = S.rrn[rhs];
}

__device__ __forceinline__ double nrm2(c128 a) { return a.re * a.re + a.im * a.im; }

// x_j += alpha_j p_j (all j); r -= alpha (w + s_0 p_0); partial |r|^2
__global__ void __launch_bounds__(kT) k_ms_xr(c128* __restrict__ x, const c128* __restrict__ p, c128* __restrict__ r,
                                              const c128* __restrict__ w, size_t n, int nrhs, MsScal S, Shifts sh,
                                              double* partials) {
  const int rhs = blockIdx.y;
  double as[kMaxShift];
#pragma unroll
  for (int j = 0; j < kMaxShift; ++j) as[j] = j < sh.ns ? S.as[rhs * kMaxShift + j] : 0.0;
  const double a = S.alpha[rhs], s0 = sh.s[0];
  const size_t off = (size_t)rhs * n, fs = (size_t)nrhs * n;
  double acc = 0.0;
  for (size_t i = (size_t)blockIdx.x * kT + threadIdx.x; i < n; i += (size_t)gridDim.x * kT) {
    const size_t e = off + i;
    c128 p0 = p[e];
#pragma unroll
    for (int j = 0; j < kMaxShift; ++j) {
      if (j < sh.ns) {
        const c128 pj = j == 0 ? p0 : p[j * fs + e];
        c128 xj = x[j * fs + e];
        xj.re = fma(as[j], pj.re, xj.re);
        xj.im = fma(as[j], pj.im, xj.im);
        x[j * fs + e] = xj;
      }
    }
    const c128 wv = w[e];
    c128 rv = r[e];
    rv.re -= a * fma(s0, p0.re, wv.re);
    rv.im -= a * fma(s0, p0.im, wv.im);
    r[e] = rv;
    acc += nrm2(rv);
  }
  double v[1] = {acc};
  __shared__ double lds[16];
  block_sum<1>(v, lds);
  store_partial<1>(v, partials + (size_t)rhs * kMaxPartials, 0, blockIdx.x);
}

// p_0 = r + beta p_0 (partial |p_0|^2), p_j = zeta_j r + beta_j p_j
__global__ void __launch_bounds__(kT) k_ms_p(c128* __restrict__ p, const c128* __restrict__ r, size_t n, int nrhs,
                                             MsScal S, Shifts sh, double* partials) {
  const int rhs = blockIdx.y;
  double bs[kMaxShift], z[kMaxShift];
#pragma unroll
  for (int j = 0; j < kMaxShift; ++j) {
    bs[j] = j < sh.ns ? S.bs[rhs * kMaxShift + j] : 0.0;
    z[j] = j < sh.ns ? S.zeta[rhs * kMaxShift + j] : 0.0;
  }
  const size_t off = (size_t)rhs * n, fs = (size_t)nrhs * n;
  double acc = 0.0;
  for (size_t i = (size_t)blockIdx.x * kT + threadIdx.x; i < n; i += (size_t)gridDim.x * kT) {
    const size_t e = off + i;
    const c128 rv = r[e];
#pragma unroll
    for (int j = 0; j < kMaxShift; ++j) {
      if (j < sh.ns) {
        c128 pj = p[j * fs + e];
        const double zj = j == 0 ? 1.0 : z[j];
        pj.re = fma(bs[j], pj.re, zj * rv.re);
        pj.im = fma(bs[j], pj.im, zj * rv.im);
        p[j * fs + e] = pj;
        if (j == 0) acc += nrm2(pj);
      }
    }
  }
  double v[1] = {acc};
  __shared__ double lds[16];
  block_sum<1>(v, lds);
  store_partial<1>(v, partials + (size_t)rhs * kMaxPartials, 0, blockIdx.x);
}

// out[rhs] = sum_j c_j x_j[rhs]
__global__ void k_ms_combine(c128* __restrict__ out, const c128* __restrict__ x, size_t total, Shifts c) {
  for (size_t i = (size_t)blockIdx.x * kT + threadIdx.x; i < total; i += (size_t)gridDim.x * kT) {
    double re = 0.0, im = 0.0;
    for (int j = 0; j < c.ns; ++j) {
      const c128 v = x[j * total + i];
      re = fma(c.s[j], v.re, re);
      im = fma(c.s[j], v.im, im);
    }
    out[i] = cmk(re, im);
  }
}

// keep P- (spin 2, 3 in the chiral basis) at s = 0 and P+ (spin 0, 1) at
// s = Ls - 1; native layout [rhs][cb][spin * 3 + colour][s]
template <typename R>
__global__ void k_wall_mask(cplx<R>* __restrict__ f, size_t total, int Ls) {
  for (size_t i = (size_t)blockIdx.x * kT + threadIdx.x; i < total; i += (size_t)gridDim.x * kT) {
    const int s = (int)(i % Ls);
    const int spin = (int)((i / Ls) % 12) / 3;
    const bool keep = (s == 0 && spin >= 2) || (s == Ls - 1 && spin < 2);
    if (!keep) f[i] = cmk((R)0, (R)0);
  }
}

}  // namespace

int wall_mask(dwf_op* op, c128* f, int nrhs, hipStream_t st) {
  const size_t total = op->field_elems(nrhs);
  hipLaunchKernelGGL((k_wall_mask<double>), dim3(nblocks(total)), dim3(kT), 0, st, f, total, op->g.Ls);
  HDCG_HIP(hipGetLastError());
  return DWF_OK;
}

int multishift_combine(dwf_op* op, c128* out, const c128* x, int nrhs, const double* coef, int ns, hipStream_t st) {
  if (ns < 1 || ns > kMaxShift) return fail(DWF_ERR_ARG, "1 to 8 shifts");
  Shifts c;
  c.ns = ns;
  for (int j = 0; j < kMaxShift; ++j) c.s[j] = j < ns ? coef[j] : 0.0;
  const size_t total = op->field_elems(nrhs);
  hipLaunchKernelGGL(k_ms_combine, dim3(nblocks(total)), dim3(kT), 0, st, out, x, total, c);
  HDCG_HIP(hipGetLastError());
  return DWF_OK;
}

int multishift_cg(dwf_op* op, c128* x, const c128* b, int nrhs, const double* shifts, int ns, double tol,
                  int maxiter, int* iters, double* resid, hipStream_t st) {
  if (ns < 1 || ns > kMaxShift) return fail(DWF_ERR_ARG, "multishift_cg takes 1 to 8 shifts");
  if (nrhs < 1 || nrhs > 64) return fail(DWF_ERR_ARG, "nrhs must be in 1..64");
  for (int j = 1; j < ns; ++j)
    if (!(shifts[j] >= shifts[0])) return fail(DWF_ERR_ARG, "shifts[0] must be the smallest shift");
  if (!(tol > 0.0) || maxiter < 0) return fail(DWF_ERR_ARG, "tol must be positive, maxiter >= 0");
  const size_t n = op->field_elems(1), fs = op->field_elems(nrhs);
  HDCG_TRY(ensure_reducer(op));
  HDCG_TRY(op->msw[0].ensure(fs * ns * sizeof(c128)));  // p_j
  HDCG_TRY(op->msw[1].ensure(fs * sizeof(c128)));       // r
  HDCG_TRY(op->msw[2].ensure(fs * sizeof(c128)));       // w
  HDCG_TRY(op->msw[3].ensure(kMsScalDoubles * sizeof(double)));
  c128* p = op->msw[0].as<c128>();
  c128* r = op->msw[1].as<c128>();
  c128* w = op->msw[2].as<c128>();
  const MsScal S = ms_scal(op->msw[3].as<double>());
  Shifts sh;
  sh.ns = ns;
  for (int j = 0; j < kMaxShift; ++j) sh.s[j] = j < ns ? shifts[j] : 0.0;
  double* partials = op->red.partials.as<double>();
  const int nb = nblocks(n);

  HDCG_HIP(hipMemsetAsync(x, 0, fs * ns * sizeof(c128), st));
  HDCG_HIP(hipMemcpyAsync(r, b, fs * sizeof(c128), hipMemcpyDeviceToDevice, st));
  for (int j = 0; j < ns; ++j) HDCG_HIP(hipMemcpyAsync(p + j * fs, b, fs * sizeof(c128), hipMemcpyDeviceToDevice, st));
  HDCG_TRY(launch_norm2<double>(op, r, nrhs, S.rr, st));
  hipLaunchKernelGGL(k_ms_init, dim3(1), dim3(64), 0, st, S, nrhs);
  HDCG_HIP(hipGetLastError());
  double* hp = op->pinned;  // [0, 64): |b|^2; ring of 8 x 64 from 64
  HDCG_HIP(hipMemcpyAsync(hp, S.rr, nrhs * sizeof(double), hipMemcpyDeviceToHost, st));
  HDCG_HIP(hipStreamSynchronize(st));
  std::vector<double> bb(hp, hp + nrhs);
  for (double v : bb)
    if (!std::isfinite(v)) return fail(DWF_ERR_NUMERIC, "multishift_cg: source norm not finite");

  constexpr int kRing = 8, kLag = 2;
  hipEvent_t ev[kRing];
  for (int i = 0; i < kRing; ++i)
    if (hipEventCreateWithFlags(&ev[i], hipEventDisableTiming) != hipSuccess) {
      for (int k = 0; k < i; ++k) (void)hipEventDestroy(ev[k]);
      return fail(DWF_ERR_HIP, "event creation failed");
    }
  int rc = DWF_OK, k = 0, checked = 0;
  bool done = true;
  for (double v : bb) done = done && v == 0.0;
  std::vector<double> last(bb);
  auto step = [&]() -> int {
    HDCG_TRY(launch_mpcdagmpc<double>(op, w, p, nrhs, st, S.pap));
    hipLaunchKernelGGL(k_ms_alpha, dim3(1), dim3(64), 0, st, S, sh, nrhs);
    HDCG_HIP(hipGetLastError());
    hipLaunchKernelGGL(k_ms_xr, dim3(nb, nrhs), dim3(kT), 0, st, x, p, r, w, n, nrhs, S, sh, partials);
    HDCG_HIP(hipGetLastError());
    HDCG_TRY(launch_finalize(1, partials, kMaxPartials, nb, nrhs, S.rrn, st));
    hipLaunchKernelGGL(k_ms_beta, dim3(1), dim3(64), 0, st, S, sh, nrhs);
    HDCG_HIP(hipGetLastError());
    hipLaunchKernelGGL(k_ms_p, dim3(nb, nrhs), dim3(kT), 0, st, p, r, n, nrhs, S, sh, partials);
    HDCG_HIP(hipGetLastError());
    HDCG_TRY(launch_finalize(1, partials, kMaxPartials, nb, nrhs, S.pp, st));
    const int slot = k % kRing;
    HDCG_HIP(hipMemcpyAsync(hp + 64 + 64 * slot, S.rr, nrhs * sizeof(double), hipMemcpyDeviceToHost, st));
    HDCG_HIP(hipEventRecord(ev[slot], st));
    return DWF_OK;
  };
  while (!done && k < maxiter) {
    rc = step();
    if (rc < 0) break;
    ++k;
    while (checked < k && (k - checked > kLag || k >= maxiter)) {
      const int slot = checked % kRing;
      if (hipEventSynchronize(ev[slot]) != hipSuccess) {
        rc = fail(DWF_ERR_HIP, "event synchronisation failed");
        break;
      }
      ++checked;
      bool conv = true;
      for (int i = 0; i < nrhs; ++i) {
        const double v = hp[64 + 64 * slot + i];
        last[i] = v;
        if (!std::isfinite(v)) {
          rc = fail(DWF_ERR_NUMERIC, "multishift_cg: residual not finite");
          break;
        }
        if (v > tol * tol * bb[i]) conv = false;
      }
      if (rc < 0 || conv) {
        done = conv;
        break;
      }
    }
    if (rc < 0) break;
  }
  if (rc >= 0 && hipStreamSynchronize(st) != hipSuccess) rc = fail(DWF_ERR_HIP, "stream synchronisation failed");
  for (int i = 0; i < kRing; ++i) (void)hipEventDestroy(ev[i]);
  if (rc < 0) return rc;
  if (iters) *iters = k;
  double worst = 0.0;
  if (!done) {
    // the residual of the last queued iteration
    HDCG_HIP(hipMemcpy(hp, S.rr, nrhs * sizeof(double), hipMemcpyDeviceToHost));
    for (int i = 0; i < nrhs; ++i) last[i] = hp[i];
  }
  for (int i = 0; i < nrhs; ++i)
    if (bb[i] > 0.0) worst = std::max(worst, std::sqrt(last[i] / bb[i]));
  if (resid) *resid = worst;
  return worst <= tol ? DWF_OK : DWF_NOT_CONVERGED;
}

}  // namespace hdk
