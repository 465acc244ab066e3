// C ABI: fine operator, BLAS-1 and the plain FP64 CG comparator.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <new>
#include <vector>

#include "fine_op.h"

namespace hdk {

static thread_local std::string g_last_error;
void set_error(const std::string& msg) { g_last_error = msg; }

int import_gauge(dwf_op* op, const void* gauge_c128, hipStream_t stream);
template <typename R>
int launch_layout(dwf_op* op, void* dst, const void* src, int nrhs, bool to_native,
                  hipStream_t stream);

static int check_op(dwf_op* op) {
  if (!op) return fail(DWF_ERR_ARG, "null operator handle");
  return DWF_OK;
}
static int check_prec(int prec) {
  if (prec != DWF_C128 && prec != DWF_C64)
    return fail(DWF_ERR_ARG, "precision must be DWF_C128 or DWF_C64 for fine fields");
  return DWF_OK;
}
// the calls that also take 16-bit (bfloat16 pair) fields
static int check_prec16(int prec) {
  if (prec != DWF_C128 && prec != DWF_C64 && prec != DWF_BF16)
    return fail(DWF_ERR_ARG, "precision must be DWF_C128, DWF_C64 or DWF_BF16 for fine fields");
  return DWF_OK;
}
static int check_nrhs(int nrhs) {
  if (nrhs < 1 || nrhs > 64) return fail(DWF_ERR_ARG, "nrhs must be in 1..64");
  return DWF_OK;
}

// ------------------------------------------------------------- CG solver ---
// Plain CG on H x = b in FP64 with device-resident scalars.  The host reads
// |r|^2 through a pinned ring with a lag of kLag iterations, so the GPU queue
// never drains while the host checks convergence; the few iterations queued
// past convergence only reduce the residual further.
static int cg_one(dwf_op* op, c128* x, const c128* b, double tol, int maxiter, int* iters,
                  int* restarts, double* true_res, double* matmuls, hipStream_t stream) {
  constexpr int kLag = 2, kRing = 8;
  const size_t n = op->field_elems(1);
  HDCG_TRY(ensure_reducer(op));
  for (int i = 0; i < 3; ++i) HDCG_TRY(op->cgw[i].ensure(n * sizeof(c128)));
  c128* r = op->cgw[0].as<c128>();
  c128* p = op->cgw[1].as<c128>();
  c128* w = op->cgw[2].as<c128>();
  // device scalar slots (in the reducer's result buffer, after slot 128)
  double* sc = op->red.results.as<double>() + 128;
  double* rr_slot[2] = {sc + 0, sc + 1};
  double* pap = sc + 2;
  double* bb = sc + 3;
  double* hp = op->pinned;  // [kRing + 4]
  hipEvent_t ev[kRing];
  for (int i = 0; i < kRing; ++i) HDCG_HIP(hipEventCreateWithFlags(&ev[i], hipEventDisableTiming));
  int status = DWF_OK;
  int it = 0, rs = 0;
  double mm = 0.0;
  double bnorm2 = 0.0, tr = 0.0;
  auto cleanup = [&]() {
    for (int i = 0; i < kRing; ++i) (void)hipEventDestroy(ev[i]);
  };
#define CG_TRY(expr)          \
  do {                        \
    int s_ = (expr);          \
    if (s_ < 0) {             \
      cleanup();              \
      return s_;              \
    }                         \
  } while (0)
#define CG_HIP(expr)                                                             \
  do {                                                                           \
    hipError_t e_ = (expr);                                                      \
    if (e_ != hipSuccess) {                                                      \
      cleanup();                                                                 \
      return fail(DWF_ERR_HIP, std::string(#expr) + ": " + hipGetErrorString(e_)); \
    }                                                                            \
  } while (0)

  CG_TRY(launch_norm2<double>(op, b, 1, bb, stream));
  CG_HIP(hipMemcpyAsync(hp + kRing, bb, sizeof(double), hipMemcpyDeviceToHost, stream));
  CG_HIP(hipStreamSynchronize(stream));
  bnorm2 = hp[kRing];
  if (!std::isfinite(bnorm2)) {
    cleanup();
    return fail(DWF_ERR_NUMERIC, "source norm is not finite");
  }
  if (bnorm2 == 0.0) {
    CG_HIP(hipMemsetAsync(x, 0, n * sizeof(c128), stream));
    CG_HIP(hipStreamSynchronize(stream));
    *iters = 0;
    *restarts = 0;
    *true_res = 0.0;
    *matmuls = 0.0;
    cleanup();
    return DWF_OK;
  }
  const double stop = tol * tol * bnorm2;
  for (;;) {
    // r = b - H x (FP64 true residual), p = r
    CG_TRY(launch_mpcdagmpc<double>(op, w, x, 1, stream, nullptr));
    mm += 1;
    CG_HIP(hipMemcpyAsync(r, b, n * sizeof(c128), hipMemcpyDeviceToDevice, stream));
    CG_TRY(launch_axpby<double>(op, r, w, -1.0, 1.0, n, stream));
    CG_TRY(launch_norm2<double>(op, r, 1, rr_slot[0], stream));
    CG_HIP(hipMemcpyAsync(hp + kRing, rr_slot[0], sizeof(double), hipMemcpyDeviceToHost, stream));
    CG_HIP(hipStreamSynchronize(stream));
    const double rr0 = hp[kRing];
    if (!std::isfinite(rr0)) {
      cleanup();
      return fail(DWF_ERR_NUMERIC, "residual is not finite");
    }
    tr = std::sqrt(rr0 / bnorm2);
    if (rr0 <= stop || it >= maxiter) break;
    if (it > 0) ++rs;
    CG_HIP(hipMemcpyAsync(p, r, n * sizeof(c128), hipMemcpyDeviceToDevice, stream));
    int k = 0;  // iterations in this cycle
    int checked = 0;
    bool done = false;
    while (!done) {
      if (it + k < maxiter) {
        double* cur = rr_slot[k & 1];
        double* nxt = rr_slot[(k + 1) & 1];
        // w = H p with pap = <p, H p> = |M_pc p|^2 fused into stage 2
        CG_TRY(launch_mpcdagmpc<double>(op, w, p, 1, stream, pap));
        CG_TRY(launch_cg_update<double>(op, x, r, p, w, cur, pap, nullptr, nxt, 1, stream));
        CG_TRY(launch_xpay<double>(op, p, r, nxt, cur, nullptr, 1, stream));
        CG_HIP(hipMemcpyAsync(hp + (k % kRing), nxt, sizeof(double), hipMemcpyDeviceToHost, stream));
        CG_HIP(hipEventRecord(ev[k % kRing], stream));
        ++k;
      }
      // check iteration `checked` once it is kLag behind (or everything queued)
      const bool drain = (it + k >= maxiter);
      while (checked < k && (k - checked > kLag || drain)) {
        CG_HIP(hipEventSynchronize(ev[checked % kRing]));
        const double rrv = hp[checked % kRing];
        ++checked;
        if (!std::isfinite(rrv)) {
          cleanup();
          return fail(DWF_ERR_NUMERIC, "CG residual became non-finite");
        }
        if (rrv <= stop) {
          done = true;
          break;
        }
      }
      if (drain && checked == k) done = true;
    }
    // iterations queued past the converged one have run too
    CG_HIP(hipStreamSynchronize(stream));
    it += k;
    mm += k;
  }
  *iters = it;
  *restarts = rs;
  *true_res = tr;
  *matmuls = mm;
  cleanup();
  return (tr <= tol) ? DWF_OK : DWF_NOT_CONVERGED;
#undef CG_TRY
#undef CG_HIP
}

// ------------------------------------------------ mixed-precision CG ---
// complex64 CG from e = 0 on H e = f until the recursive residual has
// |r| <= rtol |f| (lag-2 host checks through the pinned ring, as cg_one) or
// maxiter iterations have run.
static int cg_inner64(dwf_op* op, c64* e, const c64* f, double rtol, int maxiter, int* iters,
                      hipStream_t stream) {
  constexpr int kLag = 2, kRing = 8;
  const size_t n = op->field_elems(1);
  for (int i = 0; i < 3; ++i) HDCG_TRY(op->mgw[i].ensure(n * sizeof(c64)));
  c64* r = op->mgw[0].as<c64>();
  c64* p = op->mgw[1].as<c64>();
  c64* w = op->mgw[2].as<c64>();
  double* sc = op->red.results.as<double>() + 128;
  double* rr_slot[2] = {sc + 8, sc + 9};
  double* pap = sc + 10;
  double* hp = op->pinned;
  HDCG_HIP(hipMemsetAsync(e, 0, n * sizeof(c64), stream));
  HDCG_HIP(hipMemcpyAsync(r, f, n * sizeof(c64), hipMemcpyDeviceToDevice, stream));
  HDCG_HIP(hipMemcpyAsync(p, f, n * sizeof(c64), hipMemcpyDeviceToDevice, stream));
  HDCG_TRY(launch_norm2<float>(op, r, 1, rr_slot[0], stream));
  HDCG_HIP(hipMemcpyAsync(hp + kRing, rr_slot[0], sizeof(double), hipMemcpyDeviceToHost, stream));
  HDCG_HIP(hipStreamSynchronize(stream));
  const double ff = hp[kRing];
  *iters = 0;
  if (!(ff > 0.0)) return std::isfinite(ff) ? DWF_OK : fail(DWF_ERR_NUMERIC, "inner source not finite");
  const double stop = rtol * rtol * ff;
  hipEvent_t ev[kRing];
  for (int i = 0; i < kRing; ++i) HDCG_HIP(hipEventCreateWithFlags(&ev[i], hipEventDisableTiming));
  int k = 0, checked = 0, rc = DWF_OK;
  bool done = false;
  while (!done && rc == DWF_OK) {
    if (k < maxiter) {
      double* cur = rr_slot[k & 1];
      double* nxt = rr_slot[(k + 1) & 1];
      rc = launch_mpcdagmpc<float>(op, w, p, 1, stream, pap);
      if (rc == DWF_OK) rc = launch_cg_update<float>(op, e, r, p, w, cur, pap, nullptr, nxt, 1, stream);
      if (rc == DWF_OK) rc = launch_xpay<float>(op, p, r, nxt, cur, nullptr, 1, stream);
      if (rc == DWF_OK && hipMemcpyAsync(hp + (k % kRing), nxt, sizeof(double), hipMemcpyDeviceToHost, stream) != hipSuccess)
        rc = fail(DWF_ERR_HIP, "copy of the residual norm failed");
      if (rc == DWF_OK && hipEventRecord(ev[k % kRing], stream) != hipSuccess) rc = fail(DWF_ERR_HIP, "event record failed");
      ++k;
    }
    const bool drain = k >= maxiter;
    while (rc == DWF_OK && checked < k && (k - checked > kLag || drain)) {
      if (hipEventSynchronize(ev[checked % kRing]) != hipSuccess) {
        rc = fail(DWF_ERR_HIP, "event synchronisation failed");
        break;
      }
      const double rrv = hp[checked % kRing];
      ++checked;
      if (!std::isfinite(rrv)) {
        rc = fail(DWF_ERR_NUMERIC, "inner CG residual became non-finite");
        break;
      }
      if (rrv <= stop) {
        done = true;
        break;
      }
    }
    if (drain && checked == k) done = true;
  }
  if (rc == DWF_OK && hipStreamSynchronize(stream) != hipSuccess) rc = fail(DWF_ERR_HIP, "stream synchronisation failed");
  for (int i = 0; i < kRing; ++i) (void)hipEventDestroy(ev[i]);
  *iters = k;
  return rc;
}

// Mixed-precision CG: FP64 defect correction (true residual r = b - H x in
// complex128) around the complex64 CG of cg_inner64, whose relative target
// is max(inner_tol, tol / (2 rel)) for the current FP64 residual rel.
static int cg_mixed_one(dwf_op* op, c128* x, const c128* b, double tol, double inner_tol, int maxiter,
                        int* iters, int* restarts, double* true_res, double* matmuls, hipStream_t stream) {
  const size_t n = op->field_elems(1);
  HDCG_TRY(ensure_reducer(op));
  for (int i = 0; i < 2; ++i) HDCG_TRY(op->cgw[i].ensure(n * sizeof(c128)));
  HDCG_TRY(op->mgw[3].ensure(n * sizeof(c64)));
  HDCG_TRY(op->mgw[4].ensure(n * sizeof(c64)));
  c128* r = op->cgw[0].as<c128>();
  c128* t = op->cgw[1].as<c128>();
  c64* f = op->mgw[3].as<c64>();
  c64* e = op->mgw[4].as<c64>();
  double* sc = op->red.results.as<double>() + 128;
  double* hp = op->pinned;
  HDCG_TRY(launch_norm2<double>(op, b, 1, sc + 12, stream));
  HDCG_HIP(hipMemcpyAsync(hp + 8, sc + 12, sizeof(double), hipMemcpyDeviceToHost, stream));
  HDCG_HIP(hipStreamSynchronize(stream));
  const double bb = hp[8];
  *iters = 0;
  *restarts = 0;
  *true_res = 0.0;
  *matmuls = 0.0;
  if (!std::isfinite(bb)) return fail(DWF_ERR_NUMERIC, "source norm is not finite");
  if (bb == 0.0) {
    HDCG_HIP(hipMemsetAsync(x, 0, n * sizeof(c128), stream));
    HDCG_HIP(hipStreamSynchronize(stream));
    return DWF_OK;
  }
  int it = 0;
  for (;;) {
    // r = b - H x in FP64
    HDCG_TRY(launch_mpcdagmpc<double>(op, t, x, 1, stream, nullptr));
    *matmuls += 1;
    HDCG_HIP(hipMemcpyAsync(r, b, n * sizeof(c128), hipMemcpyDeviceToDevice, stream));
    HDCG_TRY(launch_axpby<double>(op, r, t, -1.0, 1.0, n, stream));
    HDCG_TRY(launch_norm2<double>(op, r, 1, sc + 12, stream));
    HDCG_HIP(hipMemcpyAsync(hp + 8, sc + 12, sizeof(double), hipMemcpyDeviceToHost, stream));
    HDCG_HIP(hipStreamSynchronize(stream));
    if (!std::isfinite(hp[8])) return fail(DWF_ERR_NUMERIC, "residual is not finite");
    const double rel = std::sqrt(hp[8] / bb);
    *true_res = rel;
    if (rel <= tol || it >= maxiter) break;
    // H e = r in complex64, then x += e in FP64
    HDCG_TRY(launch_convert(f, r, n, stream));
    int k = 0;
    HDCG_TRY(cg_inner64(op, e, f, std::max(inner_tol, 0.5 * tol / rel), maxiter - it, &k, stream));
    it += k;
    *matmuls += k;
    ++*restarts;
    HDCG_TRY(launch_convert(t, e, n, stream));
    HDCG_TRY(launch_axpby<double>(op, x, t, 1.0, 1.0, n, stream));
  }
  *iters = it;
  return *true_res <= tol ? DWF_OK : DWF_NOT_CONVERGED;
}

}  // namespace hdk

using namespace hdk;

extern "C" {

const char* dwf_last_error(void) { return g_last_error.c_str(); }

int dwf_create(dwf_op_t* out, const int dims[4], int Ls, double M5, double mass,
               const void* gauge_c128, const double bc_phase[8], void* stream) {
  return dwf_create_mobius(out, dims, Ls, M5, mass, 1.0, 0.0, gauge_c128, bc_phase, stream);
}

int dwf_create_mobius(dwf_op_t* out, const int dims[4], int Ls, double M5, double mass, double b5, double c5,
                      const void* gauge_c128, const double bc_phase[8], void* stream) {
  if (!out || !dims || !gauge_c128) return fail(DWF_ERR_ARG, "null argument to dwf_create");
  *out = nullptr;
  for (int mu = 0; mu < 4; ++mu)
    if (dims[mu] < 2 || (dims[mu] & 1)) return fail(DWF_ERR_GEOMETRY, "lattice extents must be even and >= 2");
  if (Ls < 1 || Ls > 64) return fail(DWF_ERR_GEOMETRY, "Ls must be in 1..64");
  // M_5 = alpha + beta K; the M_5^-1 recurrence needs |beta / alpha| < 1
  // (Shamir: |5 - M5| > 1)
  const double alpha = b5 * (4.0 - M5) + 1.0, beta = c5 * (4.0 - M5) - 1.0;
  if (!std::isfinite(alpha) || !std::isfinite(beta) || !(std::fabs(beta) < std::fabs(alpha)))
    return fail(DWF_ERR_ARG, "need |c5 (4 - M5) - 1| < |b5 (4 - M5) + 1| for the M_5^-1 recurrence");
  dwf_op* op = new (std::nothrow) dwf_op();
  if (!op) return fail(DWF_ERR_OOM, "host allocation failed");
  op->g.X = dims[0];
  op->g.Y = dims[1];
  op->g.Z = dims[2];
  op->g.T = dims[3];
  op->g.Xh = dims[0] / 2;
  op->g.Ls = Ls;
  const size_t V = (size_t)dims[0] * dims[1] * dims[2] * dims[3];
  if (V / 2 > (size_t)0x7fffffff / 12) {
    delete op;
    return fail(DWF_ERR_GEOMETRY, "lattice too large");
  }
  op->g.Vh = (int)(V / 2);
  op->M5 = M5;
  op->mass = mass;
  const double defbc[8] = {1, 0, 1, 0, 1, 0, -1, 0};
  std::memcpy(op->bc, bc_phase ? bc_phase : defbc, sizeof(op->bc));
  op->f5.alpha = alpha;
  op->f5.beta = beta;
  op->f5.ia = 1.0 / alpha;
  op->f5.kap = -beta / alpha;
  op->f5.b5 = b5;
  op->f5.c5 = c5;
  op->f5.mobius = !(b5 == 1.0 && c5 == 0.0);
  op->f5.mass = mass;
  // closed form of M_5^-1: (M+^-1)_{ss'} = pw[(s-s') mod Ls] * (s >= s' ? 1 : -m)
  const double kap = op->f5.kap;
  const double den = alpha * (1.0 + mass * std::pow(kap, Ls));
  for (int n = 0; n < 64; ++n) op->f5.pw[n] = n < Ls ? std::pow(kap, n) / den : 0.0;
  (void)hipGetDevice(&op->device);
  hipStream_t st = static_cast<hipStream_t>(stream);
  int rc = DWF_OK;
  do {
    rc = op->pw128.ensure(64 * sizeof(double));
    if (rc) break;
    rc = op->pw64.ensure(64 * sizeof(float));
    if (rc) break;
    float pwf[64];
    for (int n = 0; n < 64; ++n) pwf[n] = (float)op->f5.pw[n];
    if (hipMemcpy(op->pw128.ptr, op->f5.pw, 64 * sizeof(double), hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(op->pw64.ptr, pwf, 64 * sizeof(float), hipMemcpyHostToDevice) != hipSuccess) {
      rc = fail(DWF_ERR_HIP, "copy of the M_5^-1 table failed");
      break;
    }
    if (hipHostMalloc((void**)&op->pinned, kPinnedDoubles * sizeof(double), hipHostMallocDefault) != hipSuccess) {
      op->pinned = nullptr;
      rc = fail(DWF_ERR_HIP, "pinned host allocation failed");
      break;
    }
    rc = ensure_reducer(op);
    if (rc) break;
    rc = import_gauge(op, gauge_c128, st);
    if (rc) break;
    if (hipStreamSynchronize(st) != hipSuccess) {
      rc = fail(DWF_ERR_HIP, "gauge import failed");
      break;
    }
  } while (0);
  if (rc != DWF_OK) {
    dwf_destroy(op);
    return rc;
  }
  *out = op;
  return DWF_OK;
}

int dwf_set_hop_shape(dwf_op_t op, const int shape[10]) {
  if (!op || !shape) return fail(DWF_ERR_ARG, "null argument to dwf_set_hop_shape");
  if (shape[0] == -1) {  // back to the autotuned shapes
    op->hop_autotune = 1;
    return DWF_OK;
  }
  auto pow2 = [](int n) { return n > 0 && (n & (n - 1)) == 0; };
  const int* b = shape;
  const bool linear = b[0] == 0 && b[1] == 0 && b[2] == 0 && b[3] == 0;
  if (!linear && !(pow2(b[0]) && pow2(b[1]) && pow2(b[2]) && pow2(b[3])))
    return fail(DWF_ERR_ARG, "dwf_set_hop_shape: block extents must be powers of two (or all 0)");
  if (b[5] < 0 || b[5] > 150 || (b[8] != 0 && b[8] != 2 && b[8] != 4) || b[7] < 0 || b[7] > 4 || b[9] < 1 || b[9] > 64)
    return fail(DWF_ERR_ARG, "dwf_set_hop_shape: lds_kb must be in 0..150, order 0..4, phases 0, 2 or 4 and "
                             "rhs per workgroup 1..64");
  for (int i = 0; i < 4; ++i) op->tune.block[i] = b[i];
  op->tune.remap = b[4] != 0;
  op->tune.lds_kb = b[5];
  op->tune.nt = b[6] & 1;
  op->tune.morton = b[7];
  op->tune.phases = b[8];
  op->tune.rg = b[9];
  op->hop_autotune = 0;
  return DWF_OK;
}

int dwf_get_hop_shape(dwf_op_t op, int prec, int nrhs, int shape[10], float* ms, int* ncand) {
  if (!op || !shape || nrhs < 1) return fail(DWF_ERR_ARG, "bad arguments to dwf_get_hop_shape");
  if (prec != DWF_C128 && prec != DWF_C64 && prec != DWF_BF16) return fail(DWF_ERR_ARG, "bad precision");
  const int pi = prec == DWF_C128 ? 0 : (prec == DWF_BF16 ? 2 : 1), ri = nrhs > 1;
  const int c = op->hop_choice[pi][ri];
  const int n = hop_shape_candidates();
  if (ncand) *ncand = n;
  if (ms)
    for (int i = 0; i < n; ++i) ms[i] = c >= 0 ? op->hop_ms[pi][ri][i] : -1.f;
  int cand[7];
  const bool tuned = op->hop_autotune && c >= 0;
  if (tuned) hop_shape_of(c, cand);
  for (int i = 0; i < 4; ++i) shape[i] = tuned ? cand[i] : op->tune.block[i];
  shape[4] = tuned ? cand[4] : op->tune.remap;
  shape[5] = op->tune.lds_kb;
  shape[6] = op->tune.nt;
  shape[7] = tuned ? cand[5] : op->tune.morton;
  shape[8] = op->tune.phases;
  shape[9] = tuned ? cand[6] : op->tune.rg;
  return op->hop_autotune && c < 0 ? 1 : DWF_OK;
}

int dwf_destroy(dwf_op_t op) {
  if (!op) return DWF_OK;
  (void)hipDeviceSynchronize();
  op->gauge128.release();
  op->gauge64.release();
  op->pw128.release();
  op->pw64.release();
  for (auto& a : op->tmp)
    for (auto& b : a) b.release();
  for (auto& b : op->cgw) b.release();
  op->red.partials.release();
  op->hop_part.release();
  for (auto& kv : op->hop_tables) kv.second.dev.release();
  for (auto& m : op->mgw) m.release();
  for (auto& m : op->msw) m.release();
  op->red.counters.release();
  op->red.results.release();
  if (op->pinned) (void)hipHostFree(op->pinned);
  delete op;
  return DWF_OK;
}

int dwf_release_workspace(dwf_op_t op) {
  HDCG_TRY(check_op(op));
  HDCG_HIP(hipDeviceSynchronize());
  for (auto& a : op->tmp)
    for (auto& b : a) b.release();
  for (auto& b : op->cgw) b.release();
  for (auto& m : op->mgw) m.release();
  for (auto& m : op->msw) m.release();
  return DWF_OK;
}

int dwf_field_bytes(dwf_op_t op, int prec, int nrhs, size_t* bytes) {
  HDCG_TRY(check_op(op));
  HDCG_TRY(check_prec16(prec));
  if (!bytes || nrhs < 1) return fail(DWF_ERR_ARG, "bad arguments to dwf_field_bytes");
  *bytes = op->field_elems(nrhs) * cbytes(prec);
  return DWF_OK;
}

int dwf_import(dwf_op_t op, void* native, const void* canonical, int prec, int nrhs, void* stream) {
  HDCG_TRY(check_op(op));
  HDCG_TRY(check_prec(prec));
  if (!native || !canonical || nrhs < 1) return fail(DWF_ERR_ARG, "bad arguments to dwf_import");
  auto st = static_cast<hipStream_t>(stream);
  return prec == DWF_C128 ? launch_layout<double>(op, native, canonical, nrhs, true, st)
                          : launch_layout<float>(op, native, canonical, nrhs, true, st);
}

int dwf_export(dwf_op_t op, void* canonical, const void* native, int prec, int nrhs, void* stream) {
  HDCG_TRY(check_op(op));
  HDCG_TRY(check_prec(prec));
  if (!native || !canonical || nrhs < 1) return fail(DWF_ERR_ARG, "bad arguments to dwf_export");
  auto st = static_cast<hipStream_t>(stream);
  return prec == DWF_C128 ? launch_layout<double>(op, canonical, native, nrhs, false, st)
                          : launch_layout<float>(op, canonical, native, nrhs, false, st);
}

int dwf_convert(dwf_op_t op, void* dst, int dst_prec, const void* src, int src_prec, int nrhs,
                void* stream) {
  HDCG_TRY(check_op(op));
  HDCG_TRY(check_prec16(dst_prec));
  HDCG_TRY(check_prec16(src_prec));
  if (!dst || !src || nrhs < 1) return fail(DWF_ERR_ARG, "bad arguments to dwf_convert");
  if ((dst_prec == DWF_BF16 && src_prec == DWF_C128) || (dst_prec == DWF_C128 && src_prec == DWF_BF16))
    return fail(DWF_ERR_ARG, "DWF_BF16 fields convert to and from DWF_C64 only");
  auto st = static_cast<hipStream_t>(stream);
  const size_t n = op->field_elems(nrhs);
  if (dst_prec == src_prec) {
    HDCG_HIP(hipMemcpyAsync(dst, src, n * cbytes(src_prec), hipMemcpyDeviceToDevice, st));
    return DWF_OK;
  }
  if (dst_prec == DWF_BF16)
    return launch_convert16(op, static_cast<bf16c*>(dst), static_cast<const c64*>(src), nrhs, st);
  if (src_prec == DWF_BF16)
    return launch_convert16(op, static_cast<c64*>(dst), static_cast<const bf16c*>(src), nrhs, st);
  if (dst_prec == DWF_C64)
    return launch_convert(static_cast<c64*>(dst), static_cast<const c128*>(src), n, st);
  return launch_convert(static_cast<c128*>(dst), static_cast<const c64*>(src), n, st);
}

int dwf_multishift_cg(dwf_op_t op, void* x, const void* b, int nrhs, const double* shifts, int nshift, double tol,
                      int maxiter, struct dwf_solve_stats* st, void* stream) {
  HDCG_TRY(check_op(op));
  HDCG_TRY(check_nrhs(nrhs));
  if (!x || !b || !shifts || x == b) return fail(DWF_ERR_ARG, "dwf_multishift_cg needs x, b (distinct) and shifts");
  auto s = static_cast<hipStream_t>(stream);
  const auto t0 = std::chrono::steady_clock::now();
  int it = 0;
  double res = 0.0;
  const int rc = multishift_cg(op, static_cast<c128*>(x), static_cast<const c128*>(b), nrhs, shifts, nshift, tol,
                               maxiter, &it, &res, s);
  if (rc < 0) return rc;
  if (st) {
    st->iterations = it;
    st->restarts = 0;
    st->converged = rc == DWF_OK;
    st->true_residual = res;
    st->seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    st->matmuls = (double)it * nrhs;
  }
  return rc;
}

int mpc_apply(dwf_op_t op, void* out, const void* in, int prec, int dagger, int nrhs, void* stream) {
  HDCG_TRY(check_op(op));
  HDCG_TRY(check_prec16(prec));
  HDCG_TRY(check_nrhs(nrhs));
  if (!out || !in || out == in) return fail(DWF_ERR_ARG, "mpc_apply needs distinct in/out buffers");
  auto st = static_cast<hipStream_t>(stream);
  if (prec == DWF_C128)
    return launch_mpc<double>(op, static_cast<c128*>(out), static_cast<const c128*>(in), dagger != 0, nrhs, st, nullptr);
  if (prec == DWF_BF16)
    return launch_mpc<float, bf16c>(op, static_cast<bf16c*>(out), static_cast<const bf16c*>(in), dagger != 0, nrhs,
                                    st, nullptr);
  return launch_mpc<float>(op, static_cast<c64*>(out), static_cast<const c64*>(in), dagger != 0, nrhs, st, nullptr);
}

int mpc_dag_mpc_apply(dwf_op_t op, void* out, const void* in, int prec, int nrhs, void* stream) {
  HDCG_TRY(check_op(op));
  HDCG_TRY(check_prec16(prec));
  HDCG_TRY(check_nrhs(nrhs));
  if (!out || !in || out == in) return fail(DWF_ERR_ARG, "mpc_dag_mpc_apply needs distinct in/out buffers");
  auto st = static_cast<hipStream_t>(stream);
  if (prec == DWF_C128)
    return launch_mpcdagmpc<double>(op, static_cast<c128*>(out), static_cast<const c128*>(in), nrhs, st, nullptr);
  if (prec == DWF_BF16)
    return launch_mpcdagmpc<float, bf16c>(op, static_cast<bf16c*>(out), static_cast<const bf16c*>(in), nrhs, st,
                                          nullptr);
  return launch_mpcdagmpc<float>(op, static_cast<c64*>(out), static_cast<const c64*>(in), nrhs, st, nullptr);
}

int dwf_tune_hop(dwf_op_t op, int prec, int nrhs, void* stream) {
  HDCG_TRY(check_op(op));
  HDCG_TRY(check_prec16(prec));
  HDCG_TRY(check_nrhs(nrhs));
  auto st = static_cast<hipStream_t>(stream);
  const int pi = prec == DWF_C128 ? 0 : (prec == DWF_BF16 ? 2 : 1);
  if (!op->hop_autotune || op->hop_choice[pi][nrhs > 1] >= 0) return DWF_OK;
  const size_t bytes = op->field_elems(nrhs) * cbytes(prec);
  DevBuf a, b;
  HDCG_TRY(a.ensure(bytes));
  HDCG_TRY(b.ensure(bytes));
  int rc = hipMemsetAsync(a.ptr, 0, bytes, st) == hipSuccess ? DWF_OK : fail(DWF_ERR_HIP, "dwf_tune_hop: memset failed");
  if (rc == DWF_OK) rc = mpc_dag_mpc_apply(op, b.ptr, a.ptr, prec, nrhs, stream);
  if (rc == DWF_OK && hipStreamSynchronize(st) != hipSuccess) rc = fail(DWF_ERR_HIP, "dwf_tune_hop: sync failed");
  a.release();
  b.release();
  return rc;
}

static int fetch(dwf_op* op, double* host, const double* dev, int n, hipStream_t st) {
  HDCG_HIP(hipMemcpyAsync(op->pinned, dev, n * sizeof(double), hipMemcpyDeviceToHost, st));
  HDCG_HIP(hipStreamSynchronize(st));
  std::memcpy(host, op->pinned, n * sizeof(double));
  return DWF_OK;
}

int dwf_norm2(dwf_op_t op, double* out_host, const void* x, int prec, int nrhs, void* stream) {
  HDCG_TRY(check_op(op));
  HDCG_TRY(check_prec16(prec));
  HDCG_TRY(check_nrhs(nrhs));
  if (!out_host || !x) return fail(DWF_ERR_ARG, "null argument");
  auto st = static_cast<hipStream_t>(stream);
  double* res = op->red.results.as<double>();
  if (prec == DWF_C128)
    HDCG_TRY(launch_norm2<double>(op, static_cast<const c128*>(x), nrhs, res, st));
  else if (prec == DWF_BF16)
    HDCG_TRY((launch_norm2<float, bf16c>(op, static_cast<const bf16c*>(x), nrhs, res, st)));
  else
    HDCG_TRY(launch_norm2<float>(op, static_cast<const c64*>(x), nrhs, res, st));
  return fetch(op, out_host, res, nrhs, st);
}

int dwf_dot(dwf_op_t op, double* out_host, const void* a, const void* b, int prec, int nrhs,
            void* stream) {
  HDCG_TRY(check_op(op));
  HDCG_TRY(check_prec(prec));
  HDCG_TRY(check_nrhs(nrhs));
  if (!out_host || !a || !b) return fail(DWF_ERR_ARG, "null argument");
  auto st = static_cast<hipStream_t>(stream);
  double* res = op->red.results.as<double>();
  if (prec == DWF_C128)
    HDCG_TRY(launch_dot<double>(op, static_cast<const c128*>(a), static_cast<const c128*>(b), nrhs, res, st));
  else
    HDCG_TRY(launch_dot<float>(op, static_cast<const c64*>(a), static_cast<const c64*>(b), nrhs, res, st));
  return fetch(op, out_host, res, 2 * nrhs, st);
}

int dwf_cg_update(dwf_op_t op, void* x, void* r, const void* p, const void* w,
                  const double* alpha_host, double* rr_host, int prec, int nrhs, void* stream) {
  HDCG_TRY(check_op(op));
  HDCG_TRY(check_prec(prec));
  HDCG_TRY(check_nrhs(nrhs));
  if (!x || !r || !p || !w || !alpha_host || !rr_host) return fail(DWF_ERR_ARG, "null argument");
  auto st = static_cast<hipStream_t>(stream);
  double* res = op->red.results.as<double>();
  double* dal = res + 192;
  HDCG_HIP(hipMemcpyAsync(dal, alpha_host, nrhs * sizeof(double), hipMemcpyHostToDevice, st));
  if (prec == DWF_C128)
    HDCG_TRY(launch_cg_update<double>(op, static_cast<c128*>(x), static_cast<c128*>(r),
                                      static_cast<const c128*>(p), static_cast<const c128*>(w),
                                      nullptr, nullptr, dal, res, nrhs, st));
  else
    HDCG_TRY(launch_cg_update<float>(op, static_cast<c64*>(x), static_cast<c64*>(r),
                                     static_cast<const c64*>(p), static_cast<const c64*>(w),
                                     nullptr, nullptr, dal, res, nrhs, st));
  return fetch(op, rr_host, res, nrhs, st);
}

int dwf_xpay(dwf_op_t op, void* p, const void* r, const double* beta_host, int prec, int nrhs,
             void* stream) {
  HDCG_TRY(check_op(op));
  HDCG_TRY(check_prec(prec));
  HDCG_TRY(check_nrhs(nrhs));
  if (!p || !r || !beta_host) return fail(DWF_ERR_ARG, "null argument");
  auto st = static_cast<hipStream_t>(stream);
  double* dbeta = op->red.results.as<double>() + 192;
  HDCG_HIP(hipMemcpyAsync(dbeta, beta_host, nrhs * sizeof(double), hipMemcpyHostToDevice, st));
  if (prec == DWF_C128)
    return launch_xpay<double>(op, static_cast<c128*>(p), static_cast<const c128*>(r), nullptr, nullptr, dbeta, nrhs, st);
  return launch_xpay<float>(op, static_cast<c64*>(p), static_cast<const c64*>(r), nullptr, nullptr, dbeta, nrhs, st);
}

int cg_solve(dwf_op_t op, void* x, const void* b, int nrhs, double tol, int maxiter,
             struct dwf_solve_stats* st, void* stream) {
  HDCG_TRY(check_op(op));
  HDCG_TRY(check_nrhs(nrhs));
  if (!x || !b || !(tol > 0) || maxiter < 0) return fail(DWF_ERR_ARG, "bad arguments to cg_solve");
  auto s = static_cast<hipStream_t>(stream);
  const auto t0 = std::chrono::steady_clock::now();
  dwf_solve_stats acc{};
  acc.converged = 1;
  int worst = DWF_OK;
  const size_t n = op->field_elems(1);
  for (int i = 0; i < nrhs; ++i) {
    int it = 0, rs = 0;
    double tr = 0, mm = 0;
    int rc = cg_one(op, static_cast<c128*>(x) + i * n, static_cast<const c128*>(b) + i * n, tol,
                    maxiter, &it, &rs, &tr, &mm, s);
    if (rc < 0) return rc;
    if (rc == DWF_NOT_CONVERGED) {
      worst = DWF_NOT_CONVERGED;
      acc.converged = 0;
    }
    acc.iterations += it;
    acc.restarts += rs;
    acc.matmuls += mm;
    if (tr > acc.true_residual) acc.true_residual = tr;
  }
  acc.seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  if (st) *st = acc;
  if (worst == DWF_NOT_CONVERGED) set_error("cg_solve: maxiter reached before tol");
  return worst;
}

int cg_solve_mixed(dwf_op_t op, void* x, const void* b, int nrhs, double tol, double inner_tol, int maxiter,
                   struct dwf_solve_stats* st, void* stream) {
  HDCG_TRY(check_op(op));
  HDCG_TRY(check_nrhs(nrhs));
  if (!x || !b || !(tol > 0) || !(inner_tol > 0) || !(inner_tol < 1) || maxiter < 0)
    return fail(DWF_ERR_ARG, "bad arguments to cg_solve_mixed");
  auto s = static_cast<hipStream_t>(stream);
  const auto t0 = std::chrono::steady_clock::now();
  dwf_solve_stats acc{};
  acc.converged = 1;
  int worst = DWF_OK;
  const size_t n = op->field_elems(1);
  for (int i = 0; i < nrhs; ++i) {
    int it = 0, rs = 0;
    double tr = 0, mm = 0;
    int rc = cg_mixed_one(op, static_cast<c128*>(x) + i * n, static_cast<const c128*>(b) + i * n, tol, inner_tol,
                          maxiter, &it, &rs, &tr, &mm, s);
    if (rc < 0) return rc;
    if (rc == DWF_NOT_CONVERGED) {
      worst = DWF_NOT_CONVERGED;
      acc.converged = 0;
    }
    acc.iterations += it;
    acc.restarts += rs;
    acc.matmuls += mm;
    if (tr > acc.true_residual) acc.true_residual = tr;
  }
  acc.seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  if (st) *st = acc;
  if (worst == DWF_NOT_CONVERGED) set_error("cg_solve_mixed: maxiter reached before tol");
  return worst;
}

}  // extern "C"
