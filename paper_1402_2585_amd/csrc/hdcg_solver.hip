// HDCG setup and solve: subspace (inverse iteration + block Cholesky-QR),
// little Dirac operator by the Fourier trick, coarse CG, Q, M_IRS, the
// flexible A-DEF2 inner solver (complex64) and the FP64 defect-correction
// outer loop; plus the C ABI of these steps.
#include <chrono>
#include <cmath>
#include <complex>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <new>
#include <vector>

#include "hdcg_impl.h"

using hdk::c128;
using hdk::c64;
using hdk::cplx;

namespace hdk {

namespace {

constexpr double kPi = 3.14159265358979323846;

Red red_of(dwf_op* op) { return Red{op->red.partials.as<double>(), op->red.counters.as<unsigned>()}; }

// m1_prec: complex64, or 16-bit MFMA storage where nvec allows it
int check_m1_prec(int prec, int nvec) {
  if (prec == DWF_C64) return DWF_OK;
  if (prec != DWF_BF16 && prec != DWF_F16) return fail(DWF_ERR_ARG, "m1_prec must be DWF_C64, DWF_BF16 or DWF_F16");
  if (nvec % 4 != 0 || nvec > 64)
    return fail(DWF_ERR_ARG, "a 16-bit truncated operator needs nvec a multiple of 4 and at most 64");
  return DWF_OK;
}

// device scalar slots, 128 doubles each (room for 64 right-hand sides x 2)
enum {
  S_RR0, S_RR1, S_PAP, S_PP,                       // fine CG
  S_CRR0, S_CRR1, S_CPAP, S_CPP, S_CPR, S_CWY,      // coarse CG, coarse ADEF1
  S_ARR, S_APR, S_AWY, S_ARY0, S_ARY1, S_AINIT, S_APW,  // A-DEF2 (own slots: M_IRS runs inside)
  S_ORR, S_OBB,                                     // outer loop
  S_NSLOT
};
inline double* slot(hdcg* h, int s) { return h->scal.as<double>() + 128 * s; }

inline size_t fine_elems(hdcg* h) { return h->op->field_elems(1); }

// RAII section of one phase category (no-op when phase timing is off)
struct Phase {
  hdcg* h;
  hipStream_t st;
  int idx;
  Phase(hdcg* hh, int cat, hipStream_t s) : h(hh), st(s), idx(hh->timer.begin(cat, s)) {}
  ~Phase() { h->timer.end(idx, st); }
};

// Host reads of device residual norms through a pinned ring: iteration k is
// inspected once `lag` later iterations are queued, so the GPU never idles.
struct LagRing {
  static constexpr int kRing = 8;
  hipEvent_t ev[kRing];
  double* host = nullptr;  // [kRing][64]
  int nr = 1, queued = 0, checked = 0;
  bool ok = false;
  int init(double* pinned, int n) {
    host = pinned;
    nr = n;
    for (int i = 0; i < kRing; ++i)
      if (hipEventCreateWithFlags(&ev[i], hipEventDisableTiming) != hipSuccess)
        return fail(DWF_ERR_HIP, "event creation failed");
    ok = true;
    return DWF_OK;
  }
  ~LagRing() {
    if (ok)
      for (int i = 0; i < kRing; ++i) (void)hipEventDestroy(ev[i]);
  }
  int push(const double* dev, hipStream_t st) {
    const int s = queued % kRing;
    HDCG_HIP(hipMemcpyAsync(host + 64 * s, dev, nr * sizeof(double), hipMemcpyDeviceToHost, st));
    HDCG_HIP(hipEventRecord(ev[s], st));
    ++queued;
    return DWF_OK;
  }
  // wait for the oldest unchecked iteration; *vals points at its nr values
  int pop(const double** vals) {
    const int s = checked % kRing;
    HDCG_HIP(hipEventSynchronize(ev[s]));
    *vals = host + 64 * s;
    ++checked;
    return DWF_OK;
  }
};

// Per right-hand side, the first checked iteration whose recursive
// residual met the tolerance (0 for a zero right-hand side).
struct ConvAt {
  int at[64];
  void init(const std::vector<double>& bb, int nr) {
    for (int i = 0; i < nr; ++i) at[i] = bb[i] > 0.0 ? -1 : 0;
  }
  void note(const double* v, const std::vector<double>& bb, double tol, int nr, int iteration) {
    for (int i = 0; i < nr; ++i)
      if (at[i] < 0 && v[i] <= tol * tol * bb[i]) at[i] = iteration;
  }
  void out(int* iters_rhs, int nr, int k) const {
    if (iters_rhs)
      for (int i = 0; i < nr; ++i) iters_rhs[i] = at[i] >= 0 ? at[i] : k;
  }
};

__global__ void k_probe(c128* __restrict__ c, const c128* __restrict__ z, int k0, int nbt, int Nc,
                        int nvec) {
  const size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  const size_t total = (size_t)nbt * Nc * nvec;
  if (e >= total) return;
  const int k = (int)(e % nvec);
  const size_t ra = e / nvec;
  const int a = (int)(ra % Nc);
  const int r = (int)(ra / Nc);
  c[e] = (k == k0 + r) ? z[a] : cmk(0.0, 0.0);
}

// Philox4x32-10 (Salmon, Moraes, Dror and Shaw, SC 2011) from its published
// definition: ten rounds of two 32x32 -> 64-bit products with the Weyl key
// schedule.  Complex number i of the starting vectors takes the block with
// counter (i lo, i hi, 0, 0) and key (seed lo, seed hi): two 53-bit uniforms
// from the word pairs (0, 1) and (2, 3), then Box-Muller.
__global__ void k_philox_gaussian(c128* __restrict__ out, size_t n, unsigned long long seed) {
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  unsigned c0 = (unsigned)i, c1 = (unsigned)((unsigned long long)i >> 32), c2 = 0u, c3 = 0u;
  unsigned k0 = (unsigned)seed, k1 = (unsigned)(seed >> 32);
  for (int r = 0; r < 10; ++r) {
    if (r > 0) {
      k0 += 0x9E3779B9u;
      k1 += 0xBB67AE85u;
    }
    const unsigned long long p0 = (unsigned long long)0xD2511F53u * c0;
    const unsigned long long p1 = (unsigned long long)0xCD9E8D57u * c2;
    const unsigned n0 = (unsigned)(p1 >> 32) ^ c1 ^ k0, n1 = (unsigned)p1;
    const unsigned n2 = (unsigned)(p0 >> 32) ^ c3 ^ k1, n3 = (unsigned)p0;
    c0 = n0;
    c1 = n1;
    c2 = n2;
    c3 = n3;
  }
  const double scale = 1.0 / 9007199254740992.0;  // 2^-53
  const double u = (double)((((unsigned long long)c1 << 32) | c0) >> 11) * scale;
  const double v = (double)((((unsigned long long)c3 << 32) | c2) >> 11) * scale;
  const double rad = sqrt(-2.0 * log1p(-u));
  double sv, cv;
  sincos(2.0 * kPi * v, &sv, &cv);
  out[i] = cmk(rad * cv, rad * sv);
}

int ensure_fine64(hdcg* h, int idx, int nr) {
  return h->fw64[idx].ensure(fine_elems(h) * nr * sizeof(c64));
}

}  // namespace

// ---------------------------------------------------------------- fine CG --
// CG on (H + lam) in complex64 from x = 0.  fixed > 0: exactly `fixed`
// iterations with no host interaction (M_IRS); otherwise until
// |r| <= tol |b| for every right-hand side or maxiter.
int fine_cg(hdcg* h, c64* x, const c64* b, int nr, double lam, int fixed, double tol, int maxiter,
            int* iters, hipStream_t st) {
  dwf_op* op = h->op;
  const size_t n = fine_elems(h);
  for (int i = 8; i <= 10; ++i) HDCG_TRY(ensure_fine64(h, i, nr));
  c64* r = h->fw64[8].as<c64>();
  c64* p = h->fw64[9].as<c64>();
  c64* w = h->fw64[10].as<c64>();
  const Red red = red_of(op);
  double* rr[2] = {slot(h, S_RR0), slot(h, S_RR1)};
  double* pap = slot(h, S_PAP);
  double* pp = slot(h, S_PP);
  // a fixed count writes x in its first step (x = alpha p) and skips the r,
  // p and norm work of its last one, whose results nothing reads
  if (fixed <= 0) HDCG_TRY(b_zero<float>(x, n * nr, st));
  HDCG_HIP(hipMemcpyAsync(r, b, n * nr * sizeof(c64), hipMemcpyDeviceToDevice, st));
  HDCG_HIP(hipMemcpyAsync(p, b, n * nr * sizeof(c64), hipMemcpyDeviceToDevice, st));
  HDCG_TRY(b_norm2<float>(red, r, n, nr, rr[0], st));
  if (lam != 0.0) HDCG_HIP(hipMemcpyAsync(pp, rr[0], nr * sizeof(double), hipMemcpyDeviceToDevice, st));
  std::vector<double> bb(nr, 0.0);
  LagRing ring;
  if (fixed <= 0) {
    HDCG_TRY(ring.init(h->pinned, nr));
    HDCG_HIP(hipMemcpyAsync(h->pinned + 64 * 8, rr[0], nr * sizeof(double), hipMemcpyDeviceToHost, st));
    HDCG_HIP(hipStreamSynchronize(st));
    for (int i = 0; i < nr; ++i) bb[i] = h->pinned[64 * 8 + i];
  }
  const int limit = fixed > 0 ? fixed : maxiter;
  int k = 0;
  bool done = false;
  while (!done && k < limit) {
    double* cur = rr[k & 1];
    double* nxt = rr[(k + 1) & 1];
    {
      Phase ph(h, PH_FINE_SP, st);
      HDCG_TRY(launch_mpcdagmpc<float>(op, w, p, nr, st, pap));
    }
    {
      Phase ph(h, PH_LINALG, st);
      const bool last = fixed > 0 && k == fixed - 1;
      const int mode = (fixed > 0 && k == 0 ? kUpdX0 : 0) | (last ? kUpdXOnly : 0);
      HDCG_TRY(b_update<float>(red, x, r, p, w, n, nr, cur, false, pap, lam != 0.0 ? pp : nullptr, lam,
                               last ? nullptr : nxt, st, 1, mode));
      if (!last) HDCG_TRY(b_xpay<float>(red, p, r, n, nr, nxt, false, cur, 1.0, lam != 0.0 ? pp : nullptr, st));
    }
    ++k;
    if (fixed > 0) continue;
    HDCG_TRY(ring.push(nxt, st));
    while (ring.checked < ring.queued && (ring.queued - ring.checked > 2 || k >= limit)) {
      const double* v;
      HDCG_TRY(ring.pop(&v));
      bool conv = true;
      for (int i = 0; i < nr; ++i) {
        if (!std::isfinite(v[i])) return fail(DWF_ERR_NUMERIC, "fine CG residual not finite");
        if (v[i] > tol * tol * bb[i]) conv = false;
      }
      if (conv) {
        done = true;
        break;
      }
    }
  }
  if (iters) *iters = k;
  return DWF_OK;
}

// M_IRS with 16-bit fields: exactly `fixed` CG iterations on (H + lam) from
// x = 0 with x, r, p, w stored as bf16c (FP32 arithmetic inside every kernel,
// FP64 norms, H itself on 16-bit fields); b and x_out are complex64.
int fine_cg_bf16(hdcg* h, c64* x_out, const c64* b, int nr, double lam, int fixed, hipStream_t st) {
  dwf_op* op = h->op;
  const size_t n = fine_elems(h);
  if (fixed <= 0) return b_zero<float>(x_out, n * nr, st);
  for (int i = 0; i < 4; ++i) HDCG_TRY(h->fw16[i].ensure(n * nr * sizeof(bf16c)));
  bf16c* x = h->fw16[0].as<bf16c>();
  bf16c* r = h->fw16[1].as<bf16c>();
  bf16c* p = h->fw16[2].as<bf16c>();
  bf16c* w = h->fw16[3].as<bf16c>();
  const Red red = red_of(op);
  double* rr[2] = {slot(h, S_RR0), slot(h, S_RR1)};
  double* pap = slot(h, S_PAP);
  double* pp = lam != 0.0 ? slot(h, S_PP) : nullptr;
  {
    // r = p = b in 16 bits, |r|^2; x is first written by the first step
    Phase ph(h, PH_CONVERT, st);
    HDCG_TRY(b_mirs16_init(red, r, p, b, n, nr, op->g.Ls, rr[0], st));
  }
  if (pp) HDCG_HIP(hipMemcpyAsync(pp, rr[0], nr * sizeof(double), hipMemcpyDeviceToDevice, st));
  for (int k = 0; k < fixed; ++k) {
    double* cur = rr[k & 1];
    double* nxt = rr[(k + 1) & 1];
    {
      Phase ph(h, PH_FINE_SP, st);
      HDCG_TRY((launch_mpcdagmpc<float, bf16c>(op, w, p, nr, st, pap)));
    }
    Phase ph(h, PH_LINALG, st);
    if (k == fixed - 1) {
      // the last step: x_out = x + alpha p, rounded as the stored x would be
      HDCG_TRY(b_mirs16_last(x_out, k == 0 ? nullptr : x, p, n, nr, op->g.Ls, cur, pap, pp, lam, st));
    } else {
      HDCG_TRY(b_update(red, x, r, p, w, n, nr, cur, pap, pp, lam, nxt, st, k == 0 ? kUpdX0 : 0));
      HDCG_TRY(b_xpay(red, p, r, n, nr, nxt, cur, pp, st));
    }
  }
  return DWF_OK;
}

// M_IRS in the storage precision the parameters select
static int apply_mirs(hdcg* h, c64* z, const c64* r, int nr, int* it, hipStream_t st) {
  if (h->prm.irs_prec == DWF_BF16) {
    *it = h->prm.n_irs;
    return fine_cg_bf16(h, z, r, nr, h->prm.lambda_irs, h->prm.n_irs, st);
  }
  return fine_cg(h, z, r, nr, h->prm.lambda_irs, h->prm.n_irs, 0.0, 0, it, st);
}

// ---------------------------------------------------------- coarse ADEF1 --
// Flexible CG on A x = b preconditioned by ADEF1 with the Chebyshev
// approximate inverse of the truncated operator (Sec. V.B, "Truncated little
// Dirac operator as preconditioner"): x0 = Z D^-1 Z^+ b, y = M_1 r, p = y;
// alpha = (p, r) / (p, A p); beta = -(A p, y) / (p, A p) (the new direction
// A-orthogonal to the last; M_1 is not symmetric).  Stops at |r| <= tol |b|.
template <typename R>
int coarse_adef1(hdcg* h, const cplx<R>* AT, cplx<R>* x, const cplx<R>* b, int nr, double tol, int maxiter,
                 int* iters, hipStream_t st, int mprec, int* iters_rhs = nullptr) {
  const size_t n = (size_t)h->Nc * h->nvec;
  for (int i = 0; i < 3; ++i) HDCG_TRY(h->cw[i].ensure(n * nr * sizeof(c128)));
  HDCG_TRY(h->ycw.ensure(n * nr * sizeof(c128)));
  cplx<R>* r = h->cw[0].as<cplx<R>>();
  cplx<R>* p = h->cw[1].as<cplx<R>>();
  cplx<R>* w = h->cw[2].as<cplx<R>>();
  cplx<R>* y = h->ycw.as<cplx<R>>();
  const Red red = red_of(h->op);
  double* rr[2] = {slot(h, S_CRR0), slot(h, S_CRR1)};
  double* pw = slot(h, S_CPAP);
  double* pr = slot(h, S_CPR);
  double* wy = slot(h, S_CWY);
  const cplx<R>* Z = reinterpret_cast<const cplx<R>*>(sizeof(R) == 8 ? h->ldZ128.ptr : h->ldZ64.ptr);
  auto matvec = [&](const cplx<R>* in, cplx<R>* out) -> int {
    if constexpr (sizeof(R) == 4) {
      if (mprec == DWF_BF16 || mprec == DWF_F16) return crs_apply_mfma(h, mprec, in, out, nr, st);
    }
    return crs_apply<R>(h, AT, in, out, nr, st);
  };
  HDCG_TRY(b_norm2<R>(red, b, n, nr, rr[0], st));
  HDCG_HIP(hipMemcpyAsync(h->pinned + 64 * 9, rr[0], nr * sizeof(double), hipMemcpyDeviceToHost, st));
  HDCG_HIP(hipMemcpyAsync(r, b, n * nr * sizeof(cplx<R>), hipMemcpyDeviceToDevice, st));
  // x0 = Z D^-1 Z^+ b ; r0 = b - A x0 ; p0 = y0 = M_1 r0
  HDCG_TRY(ldop_coef<R>(h, Z, b, nr, st));
  HDCG_TRY(ldop_apply<R>(h, x, nullptr, nullptr, nullptr, Z, nr, 1.0, false, st));
  HDCG_TRY(matvec(x, w));
  HDCG_TRY(b_axpby<R>(r, w, -1.0, 1.0, n * nr, st));
  HDCG_TRY(m1_adef1<R>(h, y, r, nr, st));
  HDCG_HIP(hipMemcpyAsync(p, y, n * nr * sizeof(cplx<R>), hipMemcpyDeviceToDevice, st));
  HDCG_HIP(hipStreamSynchronize(st));
  std::vector<double> bb(h->pinned + 64 * 9, h->pinned + 64 * 9 + nr);
  bool any = false;
  for (double v : bb) any = any || v > 0.0;
  int k = 0;
  ConvAt ca;
  ca.init(bb, nr);
  if (any) {
    LagRing ring;
    HDCG_TRY(ring.init(h->pinned, nr));
    bool done = false;
    while (!done && k < maxiter) {
      double* nxt = rr[(k + 1) & 1];
      HDCG_TRY(matvec(p, w));
      HDCG_TRY(b_dot<R>(red, p, w, n, nr, pw, st));
      HDCG_TRY(b_dot<R>(red, p, r, n, nr, pr, st));
      HDCG_TRY(b_update<R>(red, x, r, p, w, n, nr, pr, true, pw, nullptr, 0.0, nxt, st, 2));
      HDCG_TRY(m1_adef1<R>(h, y, r, nr, st));
      HDCG_TRY(b_dot<R>(red, w, y, n, nr, wy, st));
      HDCG_TRY(b_xpay<R>(red, p, y, n, nr, wy, true, pw, -1.0, nullptr, st, 2));
      ++k;
      HDCG_TRY(ring.push(nxt, st));
      while (ring.checked < ring.queued && (ring.queued - ring.checked > 2 || k >= maxiter)) {
        const double* v;
        HDCG_TRY(ring.pop(&v));
        bool conv = true;
        for (int i = 0; i < nr; ++i) {
          if (!std::isfinite(v[i])) return fail(DWF_ERR_NUMERIC, "coarse ADEF1 residual not finite");
          if (v[i] > tol * tol * bb[i]) conv = false;
        }
        ca.note(v, bb, tol, nr, ring.checked);
        if (conv) {
          done = true;
          break;
        }
      }
    }
  } else {
    HDCG_TRY(b_zero<R>(x, n * nr, st));
  }
  if (iters) *iters = k;
  ca.out(iters_rhs, nr, k);
  return DWF_OK;
}

// -------------------------------------------------------------- coarse CG --
// CG on (A + shift) x = b from x = 0 (shift >= 0; the coarse operator in the
// storage mprec selects for complex64).  With the second deflation level
// built (and enabled, shift 0) it is deflated CG (Sec. V.B): x0 = Z D^-1 Z^+ b
// and p = r + beta p - Z D^-1 (AZ)^+ r.  Stops at |r| <= tol |b|.
template <typename R>
int coarse_cg(hdcg* h, const cplx<R>* AT, cplx<R>* x, const cplx<R>* b, int nr, double tol,
              int maxiter, int* iters, hipStream_t st, int mprec = -1, double shift = 0.0, int* iters_rhs = nullptr) {
  const bool defl = h->ng > 0 && h->prm.ldop_defl != 0 && shift == 0.0;
  if (defl && h->prm.ldop_m1 >= 1)
    return coarse_adef1<R>(h, AT, x, b, nr, tol, maxiter, iters, st, mprec, iters_rhs);
  if constexpr (sizeof(R) == 4) {
    if (h->persistent_coarse && !defl && shift == 0.0) {
      int done = 0;
      HDCG_TRY(coarse_cg_persistent(h, mprec == DWF_BF16 || mprec == DWF_F16 ? mprec : DWF_C64, x, b, nr, tol,
                                    maxiter, iters, iters_rhs, &done, st));
      if (done) return DWF_OK;
    }
  }
  const size_t n = (size_t)h->Nc * h->nvec;
  for (int i = 0; i < 3; ++i) HDCG_TRY(h->cw[i].ensure(n * nr * sizeof(c128)));
  cplx<R>* r = h->cw[0].as<cplx<R>>();
  cplx<R>* p = h->cw[1].as<cplx<R>>();
  cplx<R>* w = h->cw[2].as<cplx<R>>();
  const Red red = red_of(h->op);
  double* rr[2] = {slot(h, S_CRR0), slot(h, S_CRR1)};
  double* pap = slot(h, S_CPAP);
  double* pp = shift != 0.0 ? slot(h, S_CPP) : nullptr;
  const cplx<R>* Z = nullptr;
  const cplx<R>* AZ = nullptr;
  if (defl) {
    Z = reinterpret_cast<const cplx<R>*>(sizeof(R) == 8 ? h->ldZ128.ptr : h->ldZ64.ptr);
    AZ = reinterpret_cast<const cplx<R>*>(sizeof(R) == 8 ? h->ldAZ128.ptr : h->ldAZ64.ptr);
  }
  auto matvec = [&](const cplx<R>* in, cplx<R>* out) -> int {
    if constexpr (sizeof(R) == 4) {
      if (mprec == DWF_BF16 || mprec == DWF_F16) return crs_apply_mfma(h, mprec, in, out, nr, st);
    }
    return crs_apply<R>(h, AT, in, out, nr, st);
  };
  HDCG_TRY(b_norm2<R>(red, b, n, nr, rr[0], st));
  HDCG_HIP(hipMemcpyAsync(h->pinned + 64 * 9, rr[0], nr * sizeof(double), hipMemcpyDeviceToHost, st));
  HDCG_HIP(hipMemcpyAsync(r, b, n * nr * sizeof(cplx<R>), hipMemcpyDeviceToDevice, st));
  if (defl) {
    // x0 = Z D^-1 Z^+ b ; r0 = b - A x0 ; p0 = r0 - Z D^-1 (AZ)^+ r0
    HDCG_TRY(ldop_coef<R>(h, Z, b, nr, st));
    HDCG_TRY(ldop_apply<R>(h, x, nullptr, nullptr, nullptr, Z, nr, 1.0, false, st));
    HDCG_TRY(matvec(x, w));
    HDCG_TRY(b_axpby<R>(r, w, -1.0, 1.0, n * nr, st));
    HDCG_TRY(b_norm2<R>(red, r, n, nr, rr[0], st));
    HDCG_TRY(ldop_coef<R>(h, AZ, r, nr, st));
    HDCG_TRY(ldop_apply<R>(h, p, r, nullptr, nullptr, Z, nr, -1.0, true, st));
  } else {
    HDCG_TRY(b_zero<R>(x, n * nr, st));
    HDCG_HIP(hipMemcpyAsync(p, b, n * nr * sizeof(cplx<R>), hipMemcpyDeviceToDevice, st));
    if (pp) HDCG_HIP(hipMemcpyAsync(pp, rr[0], nr * sizeof(double), hipMemcpyDeviceToDevice, st));
  }
  HDCG_HIP(hipStreamSynchronize(st));
  std::vector<double> bb(h->pinned + 64 * 9, h->pinned + 64 * 9 + nr);
  bool any = false;
  for (double v : bb) any = any || v > 0.0;
  int k = 0;
  ConvAt ca;
  ca.init(bb, nr);
  if (any) {
    LagRing ring;
    HDCG_TRY(ring.init(h->pinned, nr));
    bool done = false;
    while (!done && k < maxiter) {
      double* cur = rr[k & 1];
      double* nxt = rr[(k + 1) & 1];
      HDCG_TRY(matvec(p, w));
      HDCG_TRY(b_dot<R>(red, p, w, n, nr, pap, st));
      HDCG_TRY(b_update<R>(red, x, r, p, w, n, nr, cur, false, pap, pp, shift, nxt, st, 2));
      if (defl) {
        HDCG_TRY(ldop_coef<R>(h, AZ, r, nr, st));
        HDCG_TRY(ldop_apply<R>(h, p, r, nxt, cur, Z, nr, -1.0, true, st));
      } else {
        HDCG_TRY(b_xpay<R>(red, p, r, n, nr, nxt, false, cur, 1.0, pp, st));
      }
      ++k;
      HDCG_TRY(ring.push(nxt, st));
      while (ring.checked < ring.queued && (ring.queued - ring.checked > 2 || k >= maxiter)) {
        const double* v;
        HDCG_TRY(ring.pop(&v));
        bool conv = true;
        for (int i = 0; i < nr; ++i) {
          if (!std::isfinite(v[i])) return fail(DWF_ERR_NUMERIC, "coarse CG residual not finite");
          if (v[i] > tol * tol * bb[i]) conv = false;
        }
        ca.note(v, bb, tol, nr, ring.checked);
        if (conv) {
          done = true;
          break;
        }
      }
    }
  }
  if (iters) *iters = k;
  ca.out(iters_rhs, nr, k);
  return DWF_OK;
}

int coarse_cg_shifted(hdcg* h, c128* x, const c128* b, int nr, double shift, double tol, int maxiter, int* iters,
                      hipStream_t st) {
  HDCG_TRY(ensure_at128_impl(h, st));
  return coarse_cg<double>(h, h->AT128.as<c128>(), x, b, nr, tol, maxiter, iters, st, -1, shift);
}

int ensure_at128_impl(hdcg* h, hipStream_t st) {
  if (h->AT128.bytes == 0) HDCG_TRY(crs_transpose(h, true, st));
  return DWF_OK;
}

struct InnerStats {
  int iterations = 0, coarse_solves = 0, coarse_iterations = 0, graph_replays = 0;
  double matmuls32 = 0, matmuls16 = 0;
  long long coarse_it_rhs[64] = {};
};

// Q v = P A^-1 P^+ v (complex64): out = base + sign * Q in.  deferred: the
// coarse solve is the persistent kernel enqueued without reading its result
// back (its counts go to the device totals), so that the whole application
// can be captured into a graph.
static int apply_Q(hdcg* h, c64* out, const c64* in, int nr, const c64* base, double sign, InnerStats* is,
                   hipStream_t st, bool deferred = false) {
  const size_t n = (size_t)h->Nc * h->nvec;
  HDCG_TRY(h->cw[3].ensure(n * nr * sizeof(c128)));
  HDCG_TRY(h->cw[4].ensure(n * nr * sizeof(c128)));
  c64* cb = h->cw[3].as<c64>();
  c64* cx = h->cw[4].as<c64>();
  const bool p16 = h->prm.phi_prec == DWF_BF16;
  {
    Phase ph(h, PH_PROJ, st);
    HDCG_TRY(solve_project(h, p16, in, fine_elems(h), nr, cb, n, h->nvec, 1, st));
  }
  {
    Phase ph(h, PH_COARSE, st);
    const int cp = h->prm.coarse_prec;
    if (deferred) {
      int done = 0;
      HDCG_TRY(coarse_cg_persistent_deferred(h, cp == DWF_BF16 || cp == DWF_F16 ? cp : DWF_C64, cx, cb, nr,
                                             h->prm.coarse_tol, h->prm.coarse_maxiter, &done, st));
      if (!done) return fail(DWF_ERR_STATE, "deferred coarse solve not available");
    } else {
      int it = 0, itr[64];
      HDCG_TRY(coarse_cg<float>(h, h->AT64.as<c64>(), cx, cb, nr, h->prm.coarse_tol, h->prm.coarse_maxiter, &it, st,
                                cp, 0.0, itr));
      is->coarse_iterations += it;
      for (int i = 0; i < nr; ++i) is->coarse_it_rhs[i] += itr[i];
    }
  }
  Phase ph(h, PH_PROJ, st);
  HDCG_TRY(solve_promote(h, p16, cx, nr, out, base, sign, fine_elems(h), st));
  return DWF_OK;
}

// y = M_1 r = P_R M_IRS r + Q r = z - Q (H z - r), z = M_IRS r.  z is
// computed in y's storage and the correction subtracted in place.  No host
// step when deferred (see apply_Q).
static int precondition_body(hdcg* h, c64* y, const c64* r, int nr, InnerStats* is, hipStream_t st, bool deferred) {
  const size_t n = fine_elems(h);
  c64* z = y;
  c64* t = h->fw64[6].as<c64>();
  int it = 0;
  HDCG_TRY(apply_mirs(h, z, r, nr, &it, st));
  {
    Phase ph(h, PH_FINE_SP, st);
    HDCG_TRY(launch_mpcdagmpc<float>(h->op, t, z, nr, st, nullptr));
  }
  {
    Phase ph(h, PH_LINALG, st);
    HDCG_TRY(b_axpby<float>(t, r, -1.0, 1.0, n * nr, st));  // t = H z - r
  }
  HDCG_TRY(apply_Q(h, y, t, nr, z, -1.0, is, st, deferred));
  return DWF_OK;
}

static void count_precondition(hdcg* h, int nr, InnerStats* is) {
  if (h->prm.irs_prec == DWF_BF16)
    is->matmuls16 += (double)h->prm.n_irs * nr;
  else
    is->matmuls32 += (double)h->prm.n_irs * nr;
  is->matmuls32 += nr;
  is->coarse_solves += 1;
}

// The preconditioner of one inner solve as a graph: every call after the
// first (which runs eagerly and sizes every buffer) replays one capture of
// the whole application, taken on a stream of the handle that never runs
// work itself.  Applies when the coarse solve is the persistent kernel.
struct PrecGraph {
  hipGraphExec_t exec = nullptr;
  bool warm = false, failed = false;
  ~PrecGraph() {
    if (exec) (void)hipGraphExecDestroy(exec);
  }
};

static bool graph_applies(hdcg* h, int nr) {
  if (!h->use_graph || h->timer.on || !h->persistent_coarse) return false;
  if (h->ng > 0 && h->prm.ldop_defl != 0) return false;
  const int cp = h->prm.coarse_prec;
  return coarse_cg_work_bytes(h, cp == DWF_BF16 || cp == DWF_F16 ? cp : DWF_C64, nr) > 0;
}

static int precondition(hdcg* h, c64* y, const c64* r, int nr, InnerStats* is, hipStream_t st, PrecGraph* g) {
  count_precondition(h, nr, is);
  if (!g || g->failed || !g->warm) {
    if (g) g->warm = true;
    return precondition_body(h, y, r, nr, is, st, false);
  }
  if (!g->exec) {
    if (!h->cap_stream) HDCG_HIP(hipStreamCreateWithFlags(&h->cap_stream, hipStreamNonBlocking));
    HDCG_HIP(hipStreamBeginCapture(h->cap_stream, hipStreamCaptureModeThreadLocal));
    const int rc = precondition_body(h, y, r, nr, is, h->cap_stream, true);
    hipGraph_t graph = nullptr;
    const hipError_t ec = hipStreamEndCapture(h->cap_stream, &graph);
    hipError_t ei = hipErrorUnknown;
    if (rc == DWF_OK && ec == hipSuccess && graph) ei = hipGraphInstantiate(&g->exec, graph, nullptr, nullptr, 0);
    if (graph) (void)hipGraphDestroy(graph);
    if (rc != DWF_OK || ec != hipSuccess || ei != hipSuccess) {
      // the capture did not work out: this inner solve runs eagerly
      (void)hipGetLastError();
      g->failed = true;
      g->exec = nullptr;
      return precondition_body(h, y, r, nr, is, st, false);
    }
  }
  HDCG_HIP(hipGraphLaunch(g->exec, st));
  is->graph_replays += 1;
  return DWF_OK;
}

// Inner solve H e = rin in complex64 by the generalised PCG with the A-DEF2
// choices (V_start = Q rin, M_1 = P_R M_IRS + Q), flexible or standard
// search-direction update, to |r| <= tol |rin| or maxiter.
static int adef2(hdcg* h, c64* x, const c64* rin, int nr, double tol, int maxiter, InnerStats* is,
                 hipStream_t st) {
  dwf_op* op = h->op;
  const size_t n = fine_elems(h);
  for (int i : {1, 2, 3, 5, 6}) HDCG_TRY(ensure_fine64(h, i, nr));
  c64* r = h->fw64[1].as<c64>();
  c64* p = h->fw64[2].as<c64>();
  c64* w = h->fw64[3].as<c64>();
  c64* y = h->fw64[5].as<c64>();
  const Red red = red_of(op);
  double* rr = slot(h, S_ARR);
  double* pr = slot(h, S_APR);
  double* wy = slot(h, S_AWY);
  double* ry[2] = {slot(h, S_ARY0), slot(h, S_ARY1)};
  double* pw = slot(h, S_APW);
  double* init = slot(h, S_AINIT);
  const bool flex = h->prm.flexible != 0;
  PrecGraph graph;
  PrecGraph* g = graph_applies(h, nr) ? &graph : nullptr;
  if (g) HDCG_TRY(coarse_cg_clear_totals(h, st));
  HDCG_TRY(b_norm2<float>(red, rin, n, nr, init, st));
  HDCG_HIP(hipMemcpyAsync(h->pinned + 64 * 10, init, nr * sizeof(double), hipMemcpyDeviceToHost, st));
  // x0 = Q rin ; r0 = rin - H x0
  HDCG_TRY(apply_Q(h, x, rin, nr, nullptr, 1.0, is, st));
  is->coarse_solves += 1;
  {
    Phase ph(h, PH_FINE_SP, st);
    HDCG_TRY(launch_mpcdagmpc<float>(op, w, x, nr, st, nullptr));
  }
  is->matmuls32 += nr;
  {
    Phase ph(h, PH_LINALG, st);
    HDCG_HIP(hipMemcpyAsync(r, rin, n * nr * sizeof(c64), hipMemcpyDeviceToDevice, st));
    HDCG_TRY(b_axpby<float>(r, w, -1.0, 1.0, n * nr, st));
  }
  HDCG_TRY(precondition(h, y, r, nr, is, st, g));
  {
    Phase ph(h, PH_LINALG, st);
    HDCG_HIP(hipMemcpyAsync(p, y, n * nr * sizeof(c64), hipMemcpyDeviceToDevice, st));
    if (!flex) HDCG_TRY(b_dot<float>(red, r, y, n, nr, ry[0], st));
  }
  HDCG_HIP(hipStreamSynchronize(st));
  std::vector<double> r0(h->pinned + 64 * 10, h->pinned + 64 * 10 + nr);
  int k = 0;
  while (k < maxiter) {
    // w = H p, (p, w) = |M_pc p|^2 fused into the operator
    {
      Phase ph(h, PH_FINE_SP, st);
      HDCG_TRY(launch_mpcdagmpc<float>(op, w, p, nr, st, pw));
    }
    is->matmuls32 += nr;
    {
      Phase ph(h, PH_LINALG, st);
      if (flex) {
        HDCG_TRY(b_dot<float>(red, p, r, n, nr, pr, st));  // alpha = (p, r) / (p, w)
        HDCG_TRY(b_update<float>(red, x, r, p, w, n, nr, pr, true, pw, nullptr, 0.0, rr, st));
      } else {
        HDCG_TRY(b_update<float>(red, x, r, p, w, n, nr, ry[k & 1], true, pw, nullptr, 0.0, rr, st));
      }
    }
    ++k;
    HDCG_HIP(hipMemcpyAsync(h->pinned + 64 * 11, rr, nr * sizeof(double), hipMemcpyDeviceToHost, st));
    HDCG_HIP(hipStreamSynchronize(st));
    bool conv = true;
    for (int i = 0; i < nr; ++i) {
      const double v = h->pinned[64 * 11 + i];
      if (!std::isfinite(v)) return fail(DWF_ERR_NUMERIC, "A-DEF2 residual not finite");
      if (v > tol * tol * r0[i]) conv = false;
    }
    if (conv) break;
    HDCG_TRY(precondition(h, y, r, nr, is, st, g));
    Phase ph(h, PH_LINALG, st);
    if (flex) {
      HDCG_TRY(b_dot<float>(red, w, y, n, nr, wy, st));  // beta = -(w, y) / (p, w)
      HDCG_TRY(b_xpay<float>(red, p, y, n, nr, wy, true, pw, -1.0, nullptr, st));
    } else {
      // beta = (r', y') / (r, y)
      HDCG_TRY(b_dot<float>(red, r, y, n, nr, ry[(k) & 1], st));
      HDCG_TRY(b_xpay<float>(red, p, y, n, nr, ry[k & 1], true, ry[(k + 1) & 1], 1.0, nullptr, st, 2));
    }
  }
  is->iterations += k;
  if (g && graph.exec) {
    // the replays' coarse solves left their counts on the device
    long long its = 0;
    HDCG_TRY(coarse_cg_totals(h, nr, nullptr, &its, is->coarse_it_rhs, st));
    is->coarse_iterations += (int)its;
  }
  if (h->timer.on) {
    HDCG_HIP(hipStreamSynchronize(st));
    HDCG_TRY(h->timer.collect());
  }
  return DWF_OK;
}

}  // namespace hdk

using namespace hdk;

static int check_solve_params(int coarse_prec, int irs_prec, int phi_prec) {
  if (coarse_prec != DWF_C64 && coarse_prec != DWF_BF16 && coarse_prec != DWF_F16)
    return fail(DWF_ERR_ARG, "coarse_prec must be DWF_C64, DWF_BF16 or DWF_F16");
  if (irs_prec != DWF_C64 && irs_prec != DWF_BF16)
    return fail(DWF_ERR_ARG, "irs_prec must be DWF_C64 or DWF_BF16");
  if (phi_prec != DWF_C64 && phi_prec != DWF_BF16)
    return fail(DWF_ERR_ARG, "phi_prec must be DWF_C64 or DWF_BF16");
  return DWF_OK;
}

// ====================================================================== ABI
extern "C" {

void hdcg_default_params(struct hdcg_params* p) {
  if (!p) return;
  p->n_ii = 0;
  p->lambda_ii = 0.0;
  p->tol_ii = 1e-4;
  p->maxiter_ii = 500;
  p->n_irs = 7;
  p->lambda_irs = 1.0;
  p->coarse_tol = 0.04;
  p->coarse_maxiter = 2000;
  p->flexible = 1;
  p->inner_tol = 1e-5;
  p->inner_maxiter = 500;
  p->outer_maxiter = 50;
  p->build_batch = 16;
  p->coarse_prec = DWF_C64;
  p->verbose = 0;
  p->irs_prec = DWF_C64;
  p->subspace_gen = 0;
  p->rat_lo = 3e-4;
  p->rat_eps = 1e-4;
  p->rat_tol = 1e-6;
  p->rat_maxiter = 10000;
  p->wall_noise = 0;
  p->ldop_defl = 1;
  p->phi_prec = DWF_C64;
  p->ldop_m1 = 0;
  p->m1_lo = 0.5;
  p->m1_hi = 0.0;
  p->m1_order = 16;
  p->m1_shift = 0.0;
  p->surface_depth = 0;
  p->coarse_persistent = 1;
  p->graph = 1;
  p->phase_timing = 0;
  p->mfma_tile = -1;
  p->seed = 1;
  p->keep_subspace_fp64 = 1;
  p->m1_prec = DWF_C64;
}

int hdcg_destroy(hdcg_t h) {
  if (!h) return DWF_OK;
  (void)hipDeviceSynchronize();
  h->site_of.release();
  h->nbr.release();
  h->phi128.release();
  h->phi64.release();
  h->phi16.release();
  h->A128.release();
  h->AT64.release();
  h->AT128.release();
  h->gram.release();
  h->rinv.release();
  h->flag.release();
  for (auto& b : h->cw) b.release();
  for (auto& b : h->fw64) b.release();
  for (auto& b : h->fw128) b.release();
  for (auto& b : h->fw16) b.release();
  h->scal.release();
  h->probe_c.release();
  h->mf_rho.release();
  h->mf_smax.release();
  h->mf_bf16.release();
  h->mf_f16.release();
  h->pcg_part.release();
  h->pcg_state.release();
  h->ldZ128.release();
  h->ldAZ128.release();
  h->ldZ64.release();
  h->ldAZ64.release();
  h->ldD.release();
  h->ldc.release();
  h->ldpart.release();
  h->TT64.release();
  h->phis64.release();
  h->phis16.release();
  h->TT128.release();
  h->nbr9.release();
  h->ycw.release();
  if (h->pinned) (void)hipHostFree(h->pinned);
  if (h->cap_stream) (void)hipStreamDestroy(h->cap_stream);
  delete h;
  return DWF_OK;
}

static int setup_impl(hdcg* h, const void* vectors, hipStream_t st) {
  dwf_op* op = h->op;
  const Geom& g = op->g;
  const size_t fe = op->field_elems(1);
  const int nv = h->nvec;
  HDCG_TRY(ensure_reducer(op));
  HDCG_TRY(h->scal.ensure(sizeof(double) * 128 * S_NSLOT));
  HDCG_TRY(h->flag.ensure(sizeof(int) * 4));
  HDCG_HIP(hipMemsetAsync(h->flag.ptr, 0, sizeof(int) * 4, st));
  HDCG_TRY(blk_build_maps(h, st));

  // ---- subspace: inverse iteration on the given starting vectors ---------
  DevBuf work;  // canonical c128 copy of the vectors
  HDCG_TRY(work.ensure(fe * nv * sizeof(c128)));
  if (vectors) {
    HDCG_HIP(hipMemcpyAsync(work.ptr, vectors, fe * nv * sizeof(c128), hipMemcpyDeviceToDevice, st));
  } else {
    // no vectors given: seeded Gaussian starting vectors drawn on the device
    const size_t n = fe * nv;
    hipLaunchKernelGGL(k_philox_gaussian, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, work.as<c128>(), n,
                       h->seed);
    HDCG_HIP(hipGetLastError());
  }
  if (h->prm.subspace_gen == 1) {
    // rational filter, Sec. IV.B: prod_j (H + lo + j eps)^-1 eta as
    // sum_j c_j (H + s_j)^-1 eta, c_j = prod_{i != j} 1 / (s_i - s_j), the
    // shifted solutions from one multi-shift CG (groups of up to 8 vectors)
    const int G = std::min(nv, 8);
    double sh[4], cf[4];
    for (int j = 0; j < 4; ++j) sh[j] = h->prm.rat_lo + j * h->prm.rat_eps;
    for (int j = 0; j < 4; ++j) {
      double d = 1.0;
      for (int i = 0; i < 4; ++i)
        if (i != j) d *= sh[i] - sh[j];
      cf[j] = 1.0 / d;
    }
    DevBuf xs;
    HDCG_TRY(xs.ensure(fe * 4 * G * sizeof(c128)));
    HDCG_TRY(h->fw128[0].ensure(fe * G * sizeof(c128)));
    HDCG_TRY(h->fw128[1].ensure(fe * G * sizeof(c128)));
    c128* v128 = h->fw128[0].as<c128>();
    c128* f128 = h->fw128[1].as<c128>();
    double* nrm = slot(h, S_ORR);
    for (int k0 = 0; k0 < nv; k0 += G) {
      const int g = std::min(G, nv - k0);
      c128* can = work.as<c128>() + (size_t)k0 * fe;
      HDCG_TRY(dwf_import(op, v128, can, DWF_C128, g, st));
      if (h->prm.wall_noise) HDCG_TRY(wall_mask(op, v128, g, st));
      int it = 0;
      double res = 0.0;
      HDCG_TRY(multishift_cg(op, xs.as<c128>(), v128, g, sh, 4, h->prm.rat_tol, h->prm.rat_maxiter, &it, &res, st));
      h->setup_matmuls += (long long)it * g;
      HDCG_TRY(multishift_combine(op, f128, xs.as<c128>(), g, cf, 4, st));
      HDCG_TRY(b_norm2<double>(red_of(op), f128, fe, g, nrm, st));
      HDCG_TRY(b_scale_copy<double, double>(v128, f128, nrm, true, fe, g, st));  // normalise
      HDCG_TRY(dwf_export(op, can, v128, DWF_C128, g, st));
      if (h->prm.verbose) {
        HDCG_HIP(hipStreamSynchronize(st));
        std::fprintf(stderr, "[hdcg_setup] rational filter: vectors %d-%d done, %d multi-shift iterations (residual %.1e)\n",
                     k0, k0 + g - 1, it, res);
        std::fflush(stderr);
      }
    }
  }
  if (h->prm.n_ii > 0) {
    const int G = std::min(nv, 8);
    HDCG_TRY(h->fw128[0].ensure(fe * G * sizeof(c128)));
    HDCG_TRY(ensure_fine64(h, 0, G));
    HDCG_TRY(ensure_fine64(h, 1, G));
    c128* v128 = h->fw128[0].as<c128>();
    c64* v = h->fw64[0].as<c64>();
    c64* xv = h->fw64[1].as<c64>();
    double* nrm = slot(h, S_ORR);
    // groups of vectors share one multi-RHS CG (all of a group iterate until
    // every member reaches tol_ii)
    for (int k0 = 0; k0 < nv; k0 += G) {
      const int g = std::min(G, nv - k0);
      c128* can = work.as<c128>() + (size_t)k0 * fe;
      HDCG_TRY(dwf_import(op, v128, can, DWF_C128, g, st));
      HDCG_TRY(launch_convert(v, v128, fe * g, st));
      int its = 0;
      for (int s = 0; s < h->prm.n_ii; ++s) {
        int it = 0;
        HDCG_TRY(fine_cg(h, xv, v, g, h->prm.lambda_ii, 0, h->prm.tol_ii, h->prm.maxiter_ii, &it, st));
        h->setup_matmuls += (long long)it * g;
        its += it;
        HDCG_TRY(b_norm2<float>(red_of(op), xv, fe, g, nrm, st));
        HDCG_TRY(b_scale_copy<float, float>(v, xv, nrm, true, fe, g, st));  // normalise
      }
      HDCG_TRY(launch_convert(v128, v, fe * g, st));
      HDCG_TRY(dwf_export(op, can, v128, DWF_C128, g, st));
      if (h->prm.verbose) {
        HDCG_HIP(hipStreamSynchronize(st));
        std::fprintf(stderr, "[hdcg_setup] inverse iteration: vectors %d-%d done, %d CG iterations\n", k0,
                     k0 + g - 1, its);
        std::fflush(stderr);
      }
    }
  }
  HDCG_TRY(h->phi128.ensure(fe * nv * sizeof(c128)));
  HDCG_TRY(blk_phi_layout<double>(h, h->phi128.as<c128>(), work.as<c128>(), true, nv, st));
  // surface-depth truncation (Sec. IV.B): the fifth-dimension interior removed
  if (h->sd > 0) HDCG_TRY(blk_surface_zero(h, st));
  work.release();

  // ---- block orthonormalisation: Cholesky-QR, twice (FP64) -------------
  HDCG_TRY(blk_cholqr_step(h, st));
  HDCG_TRY(blk_cholqr_step(h, st));
  int flag = 0;
  HDCG_HIP(hipMemcpyAsync(&flag, h->flag.ptr, sizeof(int), hipMemcpyDeviceToHost, st));
  HDCG_HIP(hipStreamSynchronize(st));
  if (flag) return fail(DWF_ERR_NUMERIC, "block Gram matrix not positive definite (subspace vectors dependent on a block)");
  HDCG_TRY(h->phi64.ensure(fe * nv * sizeof(c64)));
  HDCG_TRY(launch_convert(h->phi64.as<c64>(), h->phi128.as<c128>(), fe * nv, st));
  if (h->prm.phi_prec == DWF_BF16 && h->sd == 0) HDCG_TRY(blk_phi16(h, st));

  // ---- little Dirac operator by the Fourier trick (Sec. V.A.1) ---------
  const size_t n2 = (size_t)nv * nv;
  HDCG_TRY(h->A128.ensure((size_t)h->Nc * kStencil * n2 * sizeof(c128)));
  const int NB = std::max(1, std::min(h->prm.build_batch, std::min(nv, 16)));
  HDCG_TRY(h->fw128[1].ensure(fe * NB * sizeof(c128)));
  HDCG_TRY(h->fw128[2].ensure(fe * NB * sizeof(c128)));
  HDCG_TRY(h->probe_c.ensure((size_t)NB * h->Nc * nv * sizeof(c128)));
  DevBuf zbuf;
  HDCG_TRY(zbuf.ensure(sizeof(c128) * 2 * h->Nc));
  double m[4];
  for (int mu = 0; mu < 4; ++mu) m[mu] = std::max(1.0, std::round(h->C[mu] / 3.0));
  std::vector<c128> z(2 * h->Nc);
  for (int s = 0; s < kStencil; ++s) {
    double p[4];
    (void)kPi;
    int q = s;
    for (int mu = 0; mu < 4; ++mu) {
      p[mu] = 2.0 * kPi * (q % 3 - 1) * m[mu] / h->C[mu];
      q /= 3;
    }
    for (int a = 0; a < h->Nc; ++a) {
      int r = a;
      double ph = 0.0;
      for (int mu = 0; mu < 4; ++mu) {
        ph += p[mu] * (r % h->C[mu]);
        r /= h->C[mu];
      }
      z[a] = cmk(std::cos(ph), std::sin(ph));            // z^s_a = exp(i p.x^a)
      z[h->Nc + a] = cmk(std::cos(ph), -std::sin(ph));   // its conjugate
    }
    HDCG_HIP(hipMemcpyAsync(zbuf.ptr, z.data(), sizeof(c128) * 2 * h->Nc, hipMemcpyHostToDevice, st));
    for (int k0 = 0; k0 < nv; k0 += NB) {
      const int nbt = std::min(NB, nv - k0);
      const size_t tot = (size_t)nbt * h->Nc * nv;
      hipLaunchKernelGGL(k_probe, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, st,
                         h->probe_c.as<c128>(), zbuf.as<c128>(), k0, nbt, h->Nc, nv);
      HDCG_HIP(hipGetLastError());
      // phi~_k(p^s) = sum_b z^s_b phi^b_k, then H, then <phi^b_k'| . > e^{-ip.x^b}
      HDCG_TRY(blk_promote<double>(h, h->phi128.as<c128>(), h->probe_c.as<c128>(), nbt,
                                   h->fw128[1].as<c128>(), nullptr, 1.0, fe, st));
      HDCG_TRY(launch_mpcdagmpc<double>(op, h->fw128[2].as<c128>(), h->fw128[1].as<c128>(), nbt, st, nullptr));
      h->setup_matmuls += nbt;
      HDCG_TRY(blk_dot<double>(h, h->phi128.as<c128>(), h->fw128[2].as<c128>(), fe, nullptr, nbt,
                               h->A128.as<c128>() + (size_t)s * n2 + k0, 1, (size_t)kStencil * n2, nv,
                               zbuf.as<c128>() + h->Nc, st));
    }
    HDCG_HIP(hipStreamSynchronize(st));  // z is rewritten next
    if (h->prm.verbose && (s % 9 == 8)) {
      std::fprintf(stderr, "[hdcg_setup] coarse operator: %d of 81 momenta done\n", s + 1);
      std::fflush(stderr);
    }
  }
  // invert M_sl = prod_mu exp(i p^s_mu delta^l_mu) one dimension at a time
  c128 finv[4][9];
  for (int mu = 0; mu < 4; ++mu) {
    std::complex<double> F[3][3], I[3][3];
    for (int a = 0; a < 3; ++a)
      for (int b = 0; b < 3; ++b) F[a][b] = std::polar(1.0, 2.0 * kPi * m[mu] / h->C[mu] * (a - 1) * (b - 1));
    const std::complex<double> det = F[0][0] * (F[1][1] * F[2][2] - F[1][2] * F[2][1]) -
                                     F[0][1] * (F[1][0] * F[2][2] - F[1][2] * F[2][0]) +
                                     F[0][2] * (F[1][0] * F[2][1] - F[1][1] * F[2][0]);
    if (std::abs(det) < 1e-10) return fail(DWF_ERR_GEOMETRY, "phase matrix singular (coarse extent < 3?)");
    for (int a = 0; a < 3; ++a)
      for (int b = 0; b < 3; ++b) {
        const int a1 = (b + 1) % 3, a2 = (b + 2) % 3, b1 = (a + 1) % 3, b2 = (a + 2) % 3;
        I[a][b] = (F[a1][b1] * F[a2][b2] - F[a1][b2] * F[a2][b1]) / det;  // adjugate / det
      }
    for (int a = 0; a < 3; ++a)
      for (int b = 0; b < 3; ++b) finv[mu][a * 3 + b] = cmk(I[a][b].real(), I[a][b].imag());
  }
  HDCG_TRY(crs_idft(h, h->A128.as<c128>(), finv, st));
  HDCG_TRY(crs_transpose(h, false, st));
  if (h->prm.coarse_prec == DWF_BF16 || h->prm.coarse_prec == DWF_F16)
    HDCG_TRY(crs_build_mfma(h, h->prm.coarse_prec, st));
  HDCG_HIP(hipStreamSynchronize(st));
  // without keep_subspace_fp64 the FP64 subspace goes too, once the solve's
  // copies (complex64, and 16-bit or surface-only as the parameters ask) exist
  if (!h->keep_phi128) {
    HDCG_TRY(blk_surface_copies(h, h->prm.phi_prec == DWF_BF16, st));
    HDCG_HIP(hipStreamSynchronize(st));
    h->phi128.release();
  }
  // setup-only work memory goes back before the solve allocates its own
  for (int i = 0; i < 3; ++i) h->fw128[i].release();
  for (int i : {0, 1, 8, 9, 10}) h->fw64[i].release();
  h->probe_c.release();
  release_tmp(op);
  return DWF_OK;
}

int hdcg_setup(hdcg_t* out, dwf_op_t op, const int block[4], int nvec, const void* vectors_c128,
               const struct hdcg_params* p, void* stream) {
  if (!out || !op || !block) return fail(DWF_ERR_ARG, "null argument to hdcg_setup");
  *out = nullptr;
  if (nvec < 1 || nvec > 64) return fail(DWF_ERR_ARG, "nvec must be in 1..64");
  const int L[4] = {op->g.X, op->g.Y, op->g.Z, op->g.T};
  for (int mu = 0; mu < 4; ++mu) {
    if (block[mu] < 4 || (block[mu] & 1) || L[mu] % block[mu])
      return fail(DWF_ERR_GEOMETRY, "blocks must be even, >= 4 and divide the lattice");
    if (L[mu] / block[mu] < 3) return fail(DWF_ERR_GEOMETRY, "coarse extent must be >= 3 in every direction");
  }
  hdcg* h = new (std::nothrow) hdcg();
  if (!h) return fail(DWF_ERR_OOM, "host allocation failed");
  h->op = op;
  h->Nc = 1;
  int bvol = 1;
  for (int mu = 0; mu < 4; ++mu) {
    h->B[mu] = block[mu];
    h->C[mu] = L[mu] / block[mu];
    h->Nc *= h->C[mu];
    bvol *= block[mu];
  }
  h->nsb = bvol / 2;
  h->nvec = nvec;
  h->nb = (size_t)h->nsb * 12 * op->g.Ls;
  if (p) {
    h->prm.n_ii = p->n_ii;
    h->prm.lambda_ii = p->lambda_ii;
    h->prm.tol_ii = p->tol_ii;
    h->prm.maxiter_ii = p->maxiter_ii;
    h->prm.n_irs = p->n_irs;
    h->prm.lambda_irs = p->lambda_irs;
    h->prm.coarse_tol = p->coarse_tol;
    h->prm.coarse_maxiter = p->coarse_maxiter;
    h->prm.flexible = p->flexible;
    h->prm.inner_tol = p->inner_tol;
    h->prm.inner_maxiter = p->inner_maxiter;
    h->prm.outer_maxiter = p->outer_maxiter;
    h->prm.build_batch = p->build_batch;
    h->prm.coarse_prec = p->coarse_prec;
    h->prm.verbose = p->verbose;
    h->prm.irs_prec = p->irs_prec;
    h->prm.subspace_gen = p->subspace_gen;
    h->prm.rat_lo = p->rat_lo;
    h->prm.rat_eps = p->rat_eps;
    h->prm.rat_tol = p->rat_tol;
    h->prm.rat_maxiter = p->rat_maxiter;
    h->prm.wall_noise = p->wall_noise;
    h->prm.ldop_defl = p->ldop_defl;
    h->prm.phi_prec = p->phi_prec;
    h->prm.ldop_m1 = p->ldop_m1;
    h->prm.m1_lo = p->m1_lo;
    h->prm.m1_hi = p->m1_hi;
    h->prm.m1_order = p->m1_order;
    h->prm.m1_shift = p->m1_shift;
    h->prm.m1_prec = p->m1_prec;
    h->prm.surface_depth = p->surface_depth;
    h->seed = p->seed;
    h->keep_phi128 = p->keep_subspace_fp64 != 0;
    h->persistent_coarse = p->coarse_persistent != 0;
    h->use_graph = p->graph != 0;
    h->timer.on = p->phase_timing != 0;
    h->mfma_tile = p->mfma_tile;
  }
  if (const int rc = check_solve_params(h->prm.coarse_prec, h->prm.irs_prec, h->prm.phi_prec); rc < 0) {
    delete h;
    return rc;
  }
  if (const int rc = m1_check_params(h->prm.ldop_m1, h->prm.m1_lo, h->prm.m1_hi, h->prm.m1_order, h->prm.m1_shift);
      rc < 0) {
    delete h;
    return rc;
  }
  if (const int rc = check_m1_prec(h->prm.m1_prec, h->nvec); rc < 0) {
    delete h;
    return rc;
  }
  {
    const int d = h->prm.surface_depth, Ls = op->g.Ls;
    if (d < 0 || (d > 0 && 2 * d < Ls && d % 4 != 0)) {
      delete h;
      return fail(DWF_ERR_ARG, "surface_depth must be 0, a multiple of 4 below Ls / 2, or at least Ls / 2");
    }
    h->sd = d > 0 && 2 * d < Ls ? d : 0;
  }
  if ((h->prm.subspace_gen != 0 && h->prm.subspace_gen != 1) ||
      (h->prm.subspace_gen == 1 &&
       !(h->prm.rat_lo > 0.0 && h->prm.rat_eps > 0.0 && h->prm.rat_tol > 0.0 && h->prm.rat_maxiter >= 1))) {
    delete h;
    return fail(DWF_ERR_ARG, "subspace_gen must be 0 or 1; the rational filter needs rat_lo, rat_eps, rat_tol > 0 "
                             "and rat_maxiter >= 1");
  }
  if (hipHostMalloc((void**)&h->pinned, 64 * 16 * sizeof(double), hipHostMallocDefault) != hipSuccess) {
    h->pinned = nullptr;
    hdcg_destroy(h);
    return fail(DWF_ERR_HIP, "pinned allocation failed");
  }
  const auto t0 = std::chrono::steady_clock::now();
  const int rc = setup_impl(h, vectors_c128, static_cast<hipStream_t>(stream));
  if (rc < 0) {
    hdcg_destroy(h);
    return rc;
  }
  h->setup_seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  *out = h;
  return DWF_OK;
}

int hdcg_dims(hdcg_t h, int coarse_dims[4], int* ncoarse, int* nvec) {
  if (!h) return fail(DWF_ERR_ARG, "null handle");
  if (coarse_dims)
    for (int mu = 0; mu < 4; ++mu) coarse_dims[mu] = h->C[mu];
  if (ncoarse) *ncoarse = h->Nc;
  if (nvec) *nvec = h->nvec;
  return DWF_OK;
}

int hdcg_export_block_map(hdcg_t h, int* block_of_site, int* index_in_block) {
  if (!h || !block_of_site || !index_in_block) return fail(DWF_ERR_ARG, "null argument");
  std::vector<int> so((size_t)h->Nc * h->nsb);
  HDCG_HIP(hipMemcpy(so.data(), h->site_of.ptr, so.size() * sizeof(int), hipMemcpyDeviceToHost));
  for (int a = 0; a < h->Nc; ++a)
    for (int j = 0; j < h->nsb; ++j) {
      const int cb = so[(size_t)a * h->nsb + j];
      if (cb < 0 || cb >= h->op->g.Vh) return fail(DWF_ERR_STATE, "block map out of range");
      block_of_site[cb] = a;
      index_in_block[cb] = j;
    }
  return DWF_OK;
}

int hdcg_export_subspace(hdcg_t h, void* phi_c128, void* stream) {
  if (!h || !phi_c128) return fail(DWF_ERR_ARG, "null argument");
  if (h->phi128.bytes == 0) return fail(DWF_ERR_STATE, "the FP64 subspace was released after setup");
  return blk_phi_layout<double>(h, h->phi128.as<c128>(), static_cast<const c128*>(phi_c128), false, h->nvec,
                                static_cast<hipStream_t>(stream));
}

int hdcg_export_coarse(hdcg_t h, void* A_c128, void* stream) {
  if (!h || !A_c128) return fail(DWF_ERR_ARG, "null argument");
  HDCG_HIP(hipMemcpyAsync(A_c128, h->A128.ptr, (size_t)h->Nc * kStencil * h->nvec * h->nvec * sizeof(c128),
                          hipMemcpyDeviceToDevice, static_cast<hipStream_t>(stream)));
  return DWF_OK;
}

int hdcg_import_coarse(hdcg_t h, const void* A_c128, void* stream) {
  if (!h || !A_c128) return fail(DWF_ERR_ARG, "null argument");
  auto st = static_cast<hipStream_t>(stream);
  HDCG_HIP(hipMemcpyAsync(h->A128.ptr, A_c128, (size_t)h->Nc * kStencil * h->nvec * h->nvec * sizeof(c128),
                          hipMemcpyDeviceToDevice, st));
  // every copy derived from A is rebuilt now or on its next use
  HDCG_TRY(crs_transpose(h, false, st));
  if (h->AT128.bytes) HDCG_TRY(crs_transpose(h, true, st));
  h->mf_smax.release();
  h->mf_rho.release();
  const int had_bf16 = h->mf_have_bf16, had_f16 = h->mf_have_f16;
  h->mf_have_bf16 = h->mf_have_f16 = 0;
  if (had_bf16) HDCG_TRY(crs_build_mfma(h, DWF_BF16, st));
  if (had_f16) HDCG_TRY(crs_build_mfma(h, DWF_F16, st));
  trunc_invalidate(h);
  h->ng = 0;  // the second level was built on the old operator
  HDCG_HIP(hipStreamSynchronize(st));
  return DWF_OK;
}

static int check_h(hdcg* h, int prec, int nrhs, bool allow16 = false) {
  if (!h) return fail(DWF_ERR_ARG, "null hdcg handle");
  if (prec != DWF_C128 && prec != DWF_C64 && !(allow16 && prec == DWF_BF16))
    return fail(DWF_ERR_ARG, allow16 ? "precision must be DWF_C128, DWF_C64 or DWF_BF16"
                                     : "precision must be DWF_C128 or DWF_C64");
  if (nrhs < 1 || nrhs > 64) return fail(DWF_ERR_ARG, "nrhs must be in 1..64");
  return DWF_OK;
}

static int ensure_phi16(hdcg* h, hipStream_t st) {
  if (h->phi16.bytes == 0) HDCG_TRY(blk_phi16(h, st));
  return DWF_OK;
}

int hdcg_project(hdcg_t h, void* coarse_out, const void* fine_in, int prec, int nrhs, void* stream) {
  HDCG_TRY(check_h(h, prec, nrhs, true));
  if (!coarse_out || !fine_in) return fail(DWF_ERR_ARG, "null argument");
  auto st = static_cast<hipStream_t>(stream);
  const size_t n = (size_t)h->Nc * h->nvec, fe = h->op->field_elems(1);
  if (prec == DWF_C128 && h->phi128.bytes == 0)
    return fail(DWF_ERR_STATE, "the FP64 subspace was released after setup");
  if (prec == DWF_C128)
    return blk_dot<double>(h, h->phi128.as<c128>(), static_cast<const c128*>(fine_in), fe, nullptr, nrhs,
                           static_cast<c128*>(coarse_out), n, h->nvec, 1, nullptr, st);
  return solve_project(h, prec == DWF_BF16, static_cast<const c64*>(fine_in), fe, nrhs,
                       static_cast<c64*>(coarse_out), n, h->nvec, 1, st);
}

int hdcg_promote(hdcg_t h, void* fine_out, const void* coarse_in, int prec, int nrhs, void* stream) {
  HDCG_TRY(check_h(h, prec, nrhs, true));
  if (!coarse_in || !fine_out) return fail(DWF_ERR_ARG, "null argument");
  auto st = static_cast<hipStream_t>(stream);
  const size_t fe = h->op->field_elems(1);
  if (prec == DWF_C128 && h->phi128.bytes == 0)
    return fail(DWF_ERR_STATE, "the FP64 subspace was released after setup");
  if (prec == DWF_C128)
    return blk_promote<double>(h, h->phi128.as<c128>(), static_cast<const c128*>(coarse_in), nrhs,
                               static_cast<c128*>(fine_out), nullptr, 1.0, fe, st);
  return solve_promote(h, prec == DWF_BF16, static_cast<const c64*>(coarse_in), nrhs, static_cast<c64*>(fine_out),
                       nullptr, 1.0, fe, st);
}

static int ensure_at128(hdcg* h, hipStream_t st) { return ensure_at128_impl(h, st); }

int coarse_apply(hdcg_t h, void* out, const void* in, int prec, int nrhs, void* stream) {
  const bool m16 = prec == DWF_BF16 || prec == DWF_F16;
  HDCG_TRY(check_h(h, m16 ? DWF_C64 : prec, nrhs));
  if (!out || !in || out == in) return fail(DWF_ERR_ARG, "coarse_apply needs distinct in/out buffers");
  auto st = static_cast<hipStream_t>(stream);
  if (m16) return crs_apply_mfma(h, prec, static_cast<const c64*>(in), static_cast<c64*>(out), nrhs, st);
  if (prec == DWF_C128) {
    HDCG_TRY(ensure_at128(h, st));
    return crs_apply<double>(h, h->AT128.as<c128>(), static_cast<const c128*>(in), static_cast<c128*>(out), nrhs, st);
  }
  return crs_apply<float>(h, h->AT64.as<c64>(), static_cast<const c64*>(in), static_cast<c64*>(out), nrhs, st);
}

int hdcg_coarse_solve(hdcg_t h, void* x, const void* b, int prec, int nrhs, double tol, int maxiter,
                      int* iters, void* stream) {
  const bool m16 = prec == DWF_BF16 || prec == DWF_F16;
  HDCG_TRY(check_h(h, m16 ? DWF_C64 : prec, nrhs));
  if (!x || !b || !(tol > 0)) return fail(DWF_ERR_ARG, "bad arguments to hdcg_coarse_solve");
  auto st = static_cast<hipStream_t>(stream);
  int it = 0;
  if (prec == DWF_C128)
  {
    HDCG_TRY(ensure_at128(h, st));
    HDCG_TRY(coarse_cg<double>(h, h->AT128.as<c128>(), static_cast<c128*>(x), static_cast<const c128*>(b), nrhs,
                               tol, maxiter, &it, st, -1, 0.0, h->last_coarse_iters));
  } else
    HDCG_TRY(coarse_cg<float>(h, h->AT64.as<c64>(), static_cast<c64*>(x), static_cast<const c64*>(b), nrhs, tol,
                              maxiter, &it, st, m16 ? prec : -1, 0.0, h->last_coarse_iters));
  h->last_coarse_nrhs = nrhs;
  HDCG_HIP(hipStreamSynchronize(st));
  if (iters) *iters = it;
  return it >= maxiter ? DWF_NOT_CONVERGED : DWF_OK;
}

int hdcg_mfma_tile(hdcg_t h, int prec, int nrhs_per_launch, int tile[3], float* ms, int* ntiles, void* stream) {
  if (!h || !tile) return fail(DWF_ERR_ARG, "null argument");
  if (prec != DWF_BF16 && prec != DWF_F16) return fail(DWF_ERR_ARG, "prec must be DWF_BF16 or DWF_F16");
  if (nrhs_per_launch < 1 || nrhs_per_launch > 16) return fail(DWF_ERR_ARG, "nrhs_per_launch must be in 1..16");
  return crs_mfma_tile(h, prec, nrhs_per_launch, tile, ms, ntiles, static_cast<hipStream_t>(stream));
}

int hdcg_coarse_iterations(hdcg_t h, int* iters_rhs, int nrhs) {
  if (!h || !iters_rhs) return fail(DWF_ERR_ARG, "null argument");
  if (nrhs != h->last_coarse_nrhs) return fail(DWF_ERR_ARG, "nrhs differs from the last hdcg_coarse_solve");
  for (int i = 0; i < nrhs; ++i) iters_rhs[i] = h->last_coarse_iters[i];
  return DWF_OK;
}

int hdcg_mirs(hdcg_t h, void* out, const void* in, int nrhs, void* stream) {
  HDCG_TRY(check_h(h, DWF_C64, nrhs));
  if (!out || !in || out == in) return fail(DWF_ERR_ARG, "hdcg_mirs needs distinct in/out buffers");
  int it = 0;
  return apply_mirs(h, static_cast<c64*>(out), static_cast<const c64*>(in), nrhs, &it,
                    static_cast<hipStream_t>(stream));
}

int hdcg_set_params(hdcg_t h, const struct hdcg_params* p, void* stream) {
  if (!h || !p) return fail(DWF_ERR_ARG, "null argument to hdcg_set_params");
  HDCG_TRY(check_solve_params(p->coarse_prec, p->irs_prec, p->phi_prec));
  HDCG_TRY(m1_check_params(p->ldop_m1, p->m1_lo, p->m1_hi, p->m1_order, p->m1_shift));
  HDCG_TRY(check_m1_prec(p->m1_prec, h->nvec));
  if (p->n_irs < 0 || p->coarse_maxiter < 1 || p->inner_maxiter < 1 || p->outer_maxiter < 1 ||
      !(p->coarse_tol > 0.0) || !(p->inner_tol > 0.0 && p->inner_tol < 1.0))
    return fail(DWF_ERR_ARG, "hdcg_set_params: iteration caps must be positive, tolerances in (0, 1)");
  auto st = static_cast<hipStream_t>(stream);
  if (p->coarse_prec == DWF_BF16 && !h->mf_have_bf16) HDCG_TRY(crs_build_mfma(h, DWF_BF16, st));
  if (p->coarse_prec == DWF_F16 && !h->mf_have_f16) HDCG_TRY(crs_build_mfma(h, DWF_F16, st));
  if (p->phi_prec == DWF_BF16 && h->sd == 0) HDCG_TRY(ensure_phi16(h, st));
  HDCG_HIP(hipStreamSynchronize(st));
  const auto old = h->prm;
  h->prm.n_irs = p->n_irs;
  h->prm.lambda_irs = p->lambda_irs;
  h->prm.coarse_tol = p->coarse_tol;
  h->prm.coarse_maxiter = p->coarse_maxiter;
  h->prm.flexible = p->flexible;
  h->prm.inner_tol = p->inner_tol;
  h->prm.inner_maxiter = p->inner_maxiter;
  h->prm.outer_maxiter = p->outer_maxiter;
  h->prm.coarse_prec = p->coarse_prec;
  h->prm.irs_prec = p->irs_prec;
  h->prm.ldop_defl = p->ldop_defl;
  h->prm.phi_prec = p->phi_prec;
  if (p->m1_shift != h->prm.m1_shift) trunc_invalidate(h);
  if (p->m1_prec != h->prm.m1_prec) h->m1_hi_est = 0.0;  // estimated on the other storage
  h->prm.m1_prec = p->m1_prec;
  h->prm.ldop_m1 = p->ldop_m1;
  h->prm.m1_lo = p->m1_lo;
  h->prm.m1_hi = p->m1_hi;
  h->prm.m1_order = p->m1_order;
  h->prm.m1_shift = p->m1_shift;
  h->persistent_coarse = p->coarse_persistent != 0;
  h->use_graph = p->graph != 0;
  h->timer.on = p->phase_timing != 0;
  h->mfma_tile = p->mfma_tile;
  // the estimated Chebyshev bound (m1_hi <= 0) is taken now, not inside a
  // solve; if it fails the previous parameters are restored
  if (h->prm.ldop_m1 == 1 && h->prm.m1_hi <= 0.0) {
    double lo = 0, hi = 0;
    if (const int rc = m1_bounds(h, &lo, &hi, st); rc < 0) {
      if (h->prm.m1_shift != old.m1_shift) trunc_invalidate(h);
      h->prm = old;
      return rc;
    }
  }
  return DWF_OK;
}

int hdcg_trunc_apply(hdcg_t h, void* out, const void* in, int prec, int nrhs, void* stream) {
  HDCG_TRY(check_h(h, prec, nrhs));
  if (!out || !in || out == in) return fail(DWF_ERR_ARG, "hdcg_trunc_apply needs distinct in/out buffers");
  auto st = static_cast<hipStream_t>(stream);
  if (prec == DWF_C128) return trunc_apply<double>(h, static_cast<const c128*>(in), static_cast<c128*>(out), nrhs, st);
  return trunc_apply<float>(h, static_cast<const c64*>(in), static_cast<c64*>(out), nrhs, st);
}

int hdcg_m1_interval(hdcg_t h, double* lo, double* hi, void* stream) {
  if (!h || !lo || !hi) return fail(DWF_ERR_ARG, "null argument to hdcg_m1_interval");
  return m1_bounds(h, lo, hi, static_cast<hipStream_t>(stream));
}

int hdcg_chebyshev(hdcg_t h, void* y, const void* r, int prec, int nrhs, void* stream) {
  HDCG_TRY(check_h(h, prec, nrhs));
  if (!y || !r || y == r) return fail(DWF_ERR_ARG, "hdcg_chebyshev needs distinct in/out buffers");
  auto st = static_cast<hipStream_t>(stream);
  if (prec == DWF_C128) return m1_chebyshev<double>(h, static_cast<c128*>(y), static_cast<const c128*>(r), nrhs, st);
  return m1_chebyshev<float>(h, static_cast<c64*>(y), static_cast<const c64*>(r), nrhs, st);
}

int hdcg_trunc_cg(hdcg_t h, void* y, const void* r, int prec, int nrhs, void* stream) {
  HDCG_TRY(check_h(h, prec, nrhs));
  if (!y || !r || y == r) return fail(DWF_ERR_ARG, "hdcg_trunc_cg needs distinct in/out buffers");
  auto st = static_cast<hipStream_t>(stream);
  if (prec == DWF_C128) return m1_trunc_cg<double>(h, static_cast<c128*>(y), static_cast<const c128*>(r), nrhs, st);
  return m1_trunc_cg<float>(h, static_cast<c64*>(y), static_cast<const c64*>(r), nrhs, st);
}

int hdcg_adef1_precondition(hdcg_t h, void* y, const void* r, int prec, int nrhs, void* stream) {
  HDCG_TRY(check_h(h, prec, nrhs));
  if (!y || !r || y == r) return fail(DWF_ERR_ARG, "hdcg_adef1_precondition needs distinct in/out buffers");
  auto st = static_cast<hipStream_t>(stream);
  if (prec == DWF_C128) return m1_adef1<double>(h, static_cast<c128*>(y), static_cast<const c128*>(r), nrhs, st);
  return m1_adef1<float>(h, static_cast<c64*>(y), static_cast<const c64*>(r), nrhs, st);
}

int hdcg_ldop_setup(hdcg_t h, int n_extra, const void* noise_c128, double shift, int n_steps, double tol,
                    void* stream) {
  if (!h) return fail(DWF_ERR_ARG, "null handle");
  return ldop_build(h, n_extra, static_cast<const c128*>(noise_c128), shift, n_steps, tol, 100000,
                    static_cast<hipStream_t>(stream));
}

int hdcg_export_ldop(hdcg_t h, int* n_global, void* Z_c128, double* D_host, void* stream) {
  if (!h) return fail(DWF_ERR_ARG, "null handle");
  if (n_global) *n_global = h->ng;
  if (h->ng == 0) return DWF_OK;
  auto st = static_cast<hipStream_t>(stream);
  if (Z_c128) {
    HDCG_HIP(hipMemcpyAsync(Z_c128, h->ldZ128.ptr, sizeof(c128) * h->ng * h->Nc * h->nvec,
                            hipMemcpyDeviceToDevice, st));
    HDCG_HIP(hipStreamSynchronize(st));
  }
  if (D_host)
    for (int i = 0; i < h->ng; ++i) D_host[i] = h->ldDh[i];
  return DWF_OK;
}

// FP64 defect correction for one group of right-hand sides solved together.
static int solve_group(hdcg* h, c128* x, const c128* b, int nrhs, double tol, InnerStats* is,
                       int* outer_out, double* mm64_out, double* rel_rhs, hipStream_t st) {
  dwf_op* op = h->op;
  const size_t fe = op->field_elems(1);
  constexpr int kOuterChunk = 4;  // FP64 residual computed a few right-hand sides at a time
  HDCG_TRY(h->fw128[0].ensure(fe * nrhs * sizeof(c128)));
  HDCG_TRY(h->fw128[1].ensure(fe * std::min(nrhs, kOuterChunk) * sizeof(c128)));
  HDCG_TRY(ensure_fine64(h, 0, nrhs));
  HDCG_TRY(ensure_fine64(h, 7, nrhs));
  c128* r = h->fw128[0].as<c128>();
  c128* w = h->fw128[1].as<c128>();
  c64* r64 = h->fw64[7].as<c64>();
  c64* e64 = h->fw64[0].as<c64>();
  const Red red = red_of(op);
  double* orr = slot(h, S_ORR);
  double* obb = slot(h, S_OBB);
  HDCG_TRY(b_norm2<double>(red, b, fe, nrhs, obb, st));
  HDCG_HIP(hipMemcpyAsync(h->pinned + 64 * 12, obb, nrhs * sizeof(double), hipMemcpyDeviceToHost, st));
  HDCG_TRY(b_zero<double>(x, fe * nrhs, st));
  HDCG_HIP(hipStreamSynchronize(st));
  std::vector<double> bb(h->pinned + 64 * 12, h->pinned + 64 * 12 + nrhs);
  int outer = 0;
  double mm64 = 0;
  int status = DWF_OK;
  for (;;) {
    // r = b - H x in FP64
    HDCG_HIP(hipMemcpyAsync(r, b, fe * nrhs * sizeof(c128), hipMemcpyDeviceToDevice, st));
    if (outer > 0) {
      for (int r0 = 0; r0 < nrhs; r0 += kOuterChunk) {
        const int nc = std::min(kOuterChunk, nrhs - r0);
        {
          Phase ph(h, PH_FINE_DP, st);
          HDCG_TRY(launch_mpcdagmpc<double>(op, w, x + (size_t)r0 * fe, nc, st, nullptr));
        }
        Phase ph(h, PH_LINALG, st);
        HDCG_TRY(b_axpby<double>(r + (size_t)r0 * fe, w, -1.0, 1.0, fe * nc, st));
      }
      mm64 += nrhs;
    }
    {
      Phase ph(h, PH_LINALG, st);
      HDCG_TRY(b_norm2<double>(red, r, fe, nrhs, orr, st));
    }
    HDCG_HIP(hipMemcpyAsync(h->pinned + 64 * 13, orr, nrhs * sizeof(double), hipMemcpyDeviceToHost, st));
    HDCG_HIP(hipStreamSynchronize(st));
    double rel = 0;
    for (int i = 0; i < nrhs; ++i) {
      const double v = h->pinned[64 * 13 + i];
      if (!std::isfinite(v)) return fail(DWF_ERR_NUMERIC, "outer residual not finite");
      rel_rhs[i] = bb[i] > 0 ? std::sqrt(v / bb[i]) : 0.0;
      rel = std::max(rel, rel_rhs[i]);
    }
    if (rel <= tol) break;
    if (outer >= h->prm.outer_maxiter) {
      status = DWF_NOT_CONVERGED;
      break;
    }
    // inner complex64 solve on the normalised residual, x += |r| e; the inner
    // target is only as tight as the remaining reduction needs (never below
    // the complex64 floor inner_tol)
    {
      Phase ph(h, PH_CONVERT, st);
      HDCG_TRY(b_scale_copy<float, double>(r64, r, orr, true, fe, nrhs, st));
    }
    const double itol = std::max(h->prm.inner_tol, 0.5 * tol / rel);
    HDCG_TRY(adef2(h, e64, r64, nrhs, itol, h->prm.inner_maxiter, is, st));
    {
      Phase ph(h, PH_CONVERT, st);
      HDCG_TRY(b_axpy_mixed<double, float>(x, e64, orr, fe, nrhs, st, true));
    }
    ++outer;
  }
  if (h->timer.on) {
    HDCG_HIP(hipStreamSynchronize(st));
    HDCG_TRY(h->timer.collect());
  }
  *outer_out = outer;
  *mm64_out += mm64;
  return status;
}

// Right-hand sides solved together: up to 16 (one batch shares every pass
// over the operators, and the coarse solve of all of them is one persistent
// kernel), fewer when the work fields of that many would not fit the free
// device memory (about 13 complex64, 7 16-bit and 2 complex128 fine fields
// per right-hand side, counting those already held for reuse).
static int group_size(hdcg* h, int nrhs) {
  const size_t fe = fine_elems(h);
  const size_t per = fe * (13 * sizeof(c64) + 7 * sizeof(bf16c) + 2 * sizeof(c128));
  size_t held = 0;
  for (auto& b : h->fw64) held += b.bytes;
  for (auto& b : h->fw16) held += b.bytes;
  for (auto& b : h->fw128) held += b.bytes;
  for (auto& a : h->op->tmp)
    for (auto& b : a) held += b.bytes;
  size_t free_b = 0, total_b = 0;
  if (hipMemGetInfo(&free_b, &total_b) != hipSuccess) free_b = 0;
  const size_t avail = free_b + held;
  int g = std::min(16, nrhs);
  while (g > 1 && per * (size_t)g + ((size_t)1 << 30) > avail) --g;
  return g;
}

// ---------------------------------------------------------- phase timer --
int PhaseTimer::begin(int c, hipStream_t st) {
  if (!on) return -1;
  if (2 * used + 2 > pool.size()) {
    for (int i = 0; i < 2; ++i) {
      hipEvent_t e;
      if (hipEventCreate(&e) != hipSuccess) return -1;
      pool.push_back(e);
    }
  }
  if (cat.size() <= used) cat.resize(used + 1);
  const int idx = (int)used++;
  cat[idx] = c;
  if (hipEventRecord(pool[2 * idx], st) != hipSuccess) return -1;
  return idx;
}

void PhaseTimer::end(int idx, hipStream_t st) {
  if (idx >= 0) (void)hipEventRecord(pool[2 * idx + 1], st);
}

int PhaseTimer::collect() {
  for (size_t i = 0; i < used; ++i) {
    float ms = 0.f;
    if (hipEventSynchronize(pool[2 * i + 1]) != hipSuccess ||
        hipEventElapsedTime(&ms, pool[2 * i], pool[2 * i + 1]) != hipSuccess)
      return fail(DWF_ERR_HIP, "phase timing event failed");
    sec[cat[i]] += ms * 1e-3;
  }
  used = 0;
  return DWF_OK;
}

PhaseTimer::~PhaseTimer() {
  for (hipEvent_t e : pool) (void)hipEventDestroy(e);
}

int hdcg_solve(hdcg_t h, void* x_c128, const void* b_c128, int nrhs, double tol, struct hdcg_stats* stats,
               void* stream) {
  HDCG_TRY(check_h(h, DWF_C128, nrhs));
  if (!x_c128 || !b_c128 || !(tol > 0)) return fail(DWF_ERR_ARG, "bad arguments to hdcg_solve");
  auto st = static_cast<hipStream_t>(stream);
  const auto t0 = std::chrono::steady_clock::now();
  const size_t fe = h->op->field_elems(1);
  const int kGroup = group_size(h, nrhs);
  h->timer.reset();
  InnerStats is;
  int outer = 0, status = DWF_OK;
  double mm64 = 0, rel = 0;
  double rel_rhs[64] = {};
  for (int g0 = 0; g0 < nrhs; g0 += kGroup) {
    const int ng = std::min(kGroup, nrhs - g0);
    int o = 0;
    InnerStats gs;
    const int rc = solve_group(h, static_cast<c128*>(x_c128) + (size_t)g0 * fe,
                               static_cast<const c128*>(b_c128) + (size_t)g0 * fe, ng, tol, &gs, &o, &mm64,
                               rel_rhs + g0, st);
    if (rc < 0) return rc;
    if (rc == DWF_NOT_CONVERGED) status = DWF_NOT_CONVERGED;
    outer = std::max(outer, o);
    is.iterations += gs.iterations;
    is.coarse_solves += gs.coarse_solves;
    is.coarse_iterations += gs.coarse_iterations;
    is.graph_replays += gs.graph_replays;
    is.matmuls32 += gs.matmuls32;
    is.matmuls16 += gs.matmuls16;
    for (int i = 0; i < ng; ++i) is.coarse_it_rhs[g0 + i] = gs.coarse_it_rhs[i];
  }
  for (int i = 0; i < nrhs; ++i) rel = std::max(rel, rel_rhs[i]);
  if (stats) {
    std::memset(stats, 0, sizeof(*stats));
    stats->outer_iterations = outer;
    stats->inner_iterations = is.iterations;
    stats->coarse_solves = is.coarse_solves;
    stats->coarse_iterations = is.coarse_iterations;
    stats->converged = status == DWF_OK;
    stats->nrhs = nrhs;
    stats->true_residual = rel;
    stats->seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    stats->setup_seconds = h->setup_seconds;
    stats->matmuls_fp64 = mm64;
    stats->matmuls_fp32 = is.matmuls32;
    stats->matmuls_bf16 = is.matmuls16;
    stats->group_size = kGroup;
    stats->graph_replays = is.graph_replays;
    stats->t_fine_dp = h->timer.sec[PH_FINE_DP];
    stats->t_fine_sp = h->timer.sec[PH_FINE_SP];
    stats->t_coarse = h->timer.sec[PH_COARSE];
    stats->t_project_promote = h->timer.sec[PH_PROJ];
    stats->t_linalg = h->timer.sec[PH_LINALG];
    stats->t_convert = h->timer.sec[PH_CONVERT];
    for (int i = 0; i < nrhs; ++i) {
      stats->coarse_iterations_rhs[i] = is.coarse_it_rhs[i];
      stats->true_residual_rhs[i] = rel_rhs[i];
    }
  }
  if (status == DWF_NOT_CONVERGED) set_error("hdcg_solve: outer iteration limit reached");
  return status;
}

}  // extern "C"
