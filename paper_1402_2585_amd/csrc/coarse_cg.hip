// The coarse solve inside Q (A-DEF2, Sec. IV.E): conjugate gradient on the
// little Dirac operator A (Sec. V.A) as ONE persistent kernel, for one
// right-hand side or for up to 16 at once with per-right-hand-side
// convergence masks (the solves of a batch need uneven iteration counts).
//
// A coarse CG iteration is a mat-vec over Nc sites plus a few reductions
// over Nc * Nvec numbers; launched kernel by kernel it is dominated by
// launch and reduction latency.  Here every workgroup owns the coarse sites
// a = wg, wg + G, ... for the whole solve.
//
// One right-hand side (two grid barriers per iteration):
//   phase A   p_k = r_k + beta_{k-1} p_{k-1} on own sites (p double
//             buffered); w = A p_k with p_k at neighbour sites formed from
//             r_k and p_{k-1} as they are staged into LDS; partial <p_k, w>
//   barrier   alpha_k = |r_k|^2 / <p_k, A p_k>
//   phase B   x += alpha_k p_k, r -= alpha_k w on own sites; partial |r|^2
//   barrier   beta_k = |r_{k+1}|^2 / |r_k|^2; stop when |r|^2 <= tol^2 |b|^2
//             or at maxiter
//
// Several right-hand sides (three grid barriers per iteration): the
// neighbour operands of all of them no longer fit LDS, so p_{k+1} is formed
// on the owner's sites after beta_k is known and the mat-vec reads it at the
// neighbours directly:
//   phase A   w = A p_k (all right-hand sides, one GEMM per site); partial <p, w>
//   barrier   alpha_k[r] = |r_k[r]|^2 / <p_k, w>[r], 0 once r has converged
//   phase B   x += alpha p_k, r -= alpha w; partial |r|^2
//   barrier   beta_k[r]; right-hand side r is masked off at the first k with
//             |r_k[r]|^2 <= tol^2 |b[r]|^2 (its x and r no longer change);
//             the solve ends when every one is masked, or at maxiter
//   phase P   p_{k+1} = r_{k+1} + beta_k p_k on own sites
//   barrier
//
// Reductions are deterministic: each workgroup stores one partial per
// right-hand side, and every workgroup sums all partials in the same fixed
// order, so every workgroup takes the same branch.  Partials alternate
// between two buffers (a buffer is rewritten only after the barrier that
// follows its last read).  The barrier uses per-workgroup arrival flags that
// workgroup 0 polls and a release flag the others poll, with bounded waits:
// a wait that exceeds its spin limit sets an error flag and every workgroup
// leaves.
//
// Coherence without cache maintenance: every value one workgroup writes and
// another reads (r in the single form, p, the partial sums) is stored and
// loaded with relaxed device-scope atomics, which are coherent across the
// XCDs' L2 caches; before arriving at a barrier every wave waits for its
// stores to complete.  Values a workgroup only reads and writes for its own
// sites (x, w, r in the batched form) and the operator itself use ordinary
// accesses.
//
// The kernel leaves its results on the device (PcgState): per solve, and
// summed over solves until the host clears the totals, so a sequence of
// solves can run without the host in between (inside a captured graph).
#include <algorithm>

#include "coarse_dev.h"

namespace hdk {

namespace {

constexpr int kMaxR = 16;  // right-hand sides per persistent solve

// Grid barrier state.  Barrier number e (e = 1, 2, ...): every workgroup
// stores e into its own arrival slot; workgroup 0 polls all slots (one per
// thread) until every one holds e, then stores e into the release flag,
// which the other workgroups poll.  Plain coherent stores and loads, no
// read-modify-write on a shared address; the values only grow, so nothing
// is reset between barriers of one solve.
constexpr int kMaxGrid = 4096;
struct PcgState {
  unsigned arrive[kMaxGrid];  // last barrier each workgroup reached
  alignas(128) unsigned release;
  alignas(128) struct Result {
    unsigned err;              // 1: barrier wait exceeded, 2: non-finite residual
    unsigned iters;            // iterations run
    unsigned iters_rhs[kMaxR]; // iterations each right-hand side ran before its mask
    double rr[kMaxR];          // final |r|^2
  } res;
  alignas(128) struct Totals { // deferred solves, summed until cleared by k_pcg_clear
    unsigned err;
    unsigned solves;
    unsigned iters;              // sum over solves of the iterations each ran
    unsigned iters_rhs[kMaxR];
  } tot;
};

struct PcgArgs {
  int Nc, nvec, nr, maxiter, ksteps, gmax;
  int accumulate;             // 1: add this solve's counts to the totals (deferred solves)
  double tol2;
  unsigned spin_limit;
  const c64* AT;              // complex64 operator, AT[a][l][k][j]
  const unsigned short* F;    // 16-bit fragment storage
  const float* rho;
  const float* smax;
  const int* nbr;
  const c64* b;
  c64 *x, *r, *p0, *p1, *w;  // p0, p1 (and r in the single form): coherent accesses only
  double* part;               // [2][kMaxR][gmax]
  PcgState* st;
};

// Per-solve state (barrier flags, results); G workgroups.
__global__ void k_pcg_reset(PcgState* st, int G) {
  for (int g = threadIdx.x; g < G; g += blockDim.x) st->arrive[g] = 0;
  if (threadIdx.x == 0) {
    st->release = 0;
    st->res.err = 0;
    st->res.iters = 0;
  }
  if (threadIdx.x < kMaxR) {
    st->res.iters_rhs[threadIdx.x] = 0;
    st->res.rr[threadIdx.x] = 0.0;
  }
}

// The totals (a kernel, not a memset, so that it can sit in a captured graph).
__global__ void k_pcg_clear(PcgState* st) {
  if (threadIdx.x == 0) {
    st->tot.err = 0;
    st->tot.solves = 0;
    st->tot.iters = 0;
  }
  if (threadIdx.x < kMaxR) st->tot.iters_rhs[threadIdx.x] = 0;
}

__device__ __forceinline__ unsigned ld_flag(const unsigned* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void st_flag(unsigned* p, unsigned v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Grid-wide barrier number `epoch`; false if a wait exceeded its limit (then
// st->res.err is set) or another workgroup reported an error.
__device__ __forceinline__ bool grid_barrier(PcgState* st, unsigned nblocks, unsigned epoch, unsigned spin_limit) {
  __shared__ int ok;
  __builtin_amdgcn_s_waitcnt(0);  // this wave's stores have completed
  __syncthreads();
  int good = 1;
  if (blockIdx.x == 0) {
    // master: wait until every workgroup has arrived, then release
    unsigned it = 0;
    for (;;) {
      int mine = 1;
      for (unsigned g = 1 + threadIdx.x; g < nblocks; g += kCT) mine &= ld_flag(&st->arrive[g]) >= epoch;
      if (__syncthreads_and(mine)) break;
      __builtin_amdgcn_s_sleep(1);
      if (++it > spin_limit) {
        good = 0;
        break;
      }
    }
    if (threadIdx.x == 0) {
      __builtin_amdgcn_s_waitcnt(0);
      st_flag(&st->release, epoch);
    }
  } else if (threadIdx.x == 0) {
    st_flag(&st->arrive[blockIdx.x], epoch);
    unsigned it = 0;
    while (ld_flag(&st->release) < epoch) {
      __builtin_amdgcn_s_sleep(1);
      if (++it > spin_limit) {
        good = 0;
        break;
      }
    }
  }
  if (threadIdx.x == 0) {
    if (!good) st_flag(&st->res.err, 1u);
    ok = good && ld_flag(&st->res.err) == 0;
  }
  __syncthreads();
  return ok != 0;
}

// This workgroup's partial of right-hand side r (r < nr) into buffer `buf`.
// v[q] is the thread's sum for right-hand side q (single form: kMaxR
// registers), or, in the batched form, acc0 / acc1 are the thread's sums for
// its two element slots e = tid and tid + kCT of every site (right-hand
// sides e / nvec), summed through LDS in a fixed order.
__device__ __forceinline__ void store_partials_slots(double acc0, double acc1, int nr, int nvec, double* part, int buf,
                                                     int gmax, double* lds /* 2 kCT */) {
  lds[threadIdx.x] = acc0;
  lds[kCT + threadIdx.x] = acc1;
  __syncthreads();
  if (threadIdx.x < nr) {
    double s = 0.0;
    const int e0 = threadIdx.x * nvec;
    for (int e = e0; e < e0 + nvec; ++e) s += lds[e];
    __hip_atomic_store(part + ((size_t)buf * kMaxR + threadIdx.x) * gmax + blockIdx.x, s, __ATOMIC_RELAXED,
                       __HIP_MEMORY_SCOPE_AGENT);
  }
  __syncthreads();
}

__device__ __forceinline__ void store_partials_one(double v, double* part, int buf, int gmax, double* lds /* 8 */) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const double s = wave_sum(v);
  if (lane == 0) lds[wave] = s;
  __syncthreads();
  if (threadIdx.x == 0) {
    double t = 0.0;
    for (int w = 0; w < kCT / 64; ++w) t += lds[w];
    __hip_atomic_store(part + (size_t)buf * kMaxR * gmax + blockIdx.x, t, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
  __syncthreads();
}

// out[r] = sum over all workgroups' partials of buffer `buf` (the same
// fixed order in every workgroup), r < nr.
__device__ __forceinline__ void sum_partials(double* part, int buf, int nr, int gmax, double* out,
                                             double* lds /* kMaxR * 8 */) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  for (int r = 0; r < nr; ++r) {
    double s = 0.0;
    for (int g = threadIdx.x; g < (int)gridDim.x; g += kCT)
      s += __hip_atomic_load(part + ((size_t)buf * kMaxR + r) * gmax + g, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    s = wave_sum(s);
    if (lane == 0) lds[r * 8 + wave] = s;
  }
  __syncthreads();
  if (threadIdx.x < nr) {
    double s = 0.0;
    for (int w = 0; w < kCT / 64; ++w) s += lds[threadIdx.x * 8 + w];
    out[threadIdx.x] = s;
  }
  __syncthreads();
}

// Results of one solve, written by workgroup 0, thread 0 (after the last
// barrier every workgroup holds the same values).
__device__ __forceinline__ void finish(PcgState* st, int k, int nr, const double* rr, const unsigned* it_rhs,
                                       int accumulate) {
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    st->res.iters = (unsigned)k;
    for (int r = 0; r < nr; ++r) {
      st->res.rr[r] = rr[r];
      st->res.iters_rhs[r] = it_rhs[r];
      if (accumulate) st->tot.iters_rhs[r] += it_rhs[r];
    }
    if (accumulate) {
      st->tot.solves += 1;
      st->tot.iters += (unsigned)k;
    }
  }
}

// A solve that ended early on an error still flags it in the totals (every
// workgroup leaves through here or through finish).
__device__ __forceinline__ void flag_error(PcgState* st, int accumulate) {
  if (accumulate && blockIdx.x == 0 && threadIdx.x == 0) st->tot.err |= ld_flag(&st->res.err) | 1u;
}

// One right-hand side.  MODE 0: complex64 VALU operator; 1: bf16 MFMA;
// 2: fp16 MFMA (MT M tiles).
constexpr int kMaxNvec = 64;
// K32: the 16x16x32 MFMA form (nvec % 8 == 0), else 16x16x16.
template <int MODE, int MT, bool K32>
__global__ void __launch_bounds__(kCT) __attribute__((amdgpu_waves_per_eu(4))) k_coarse_cg(PcgArgs A) {
  constexpr int kRedBytes = MODE == 0 ? kCT * (int)sizeof(c64) : 8 * MT * 64 * (int)sizeof(f32x4);
  __shared__ __align__(16) unsigned char red_raw[kRedBytes];
  __shared__ c64 s_in[kStencil * kMaxNvec];  // the site's operand at its neighbours
  __shared__ double s_tmp[8];
  __shared__ double s_rr[kMaxR], s_bb[kMaxR], s_pap[kMaxR];
  __shared__ unsigned s_it[kMaxR];
  __shared__ float s_beta;
  __shared__ double s_alpha;
  const int G = gridDim.x, wg = blockIdx.x, tid = threadIdx.x;
  const int Nc = A.Nc, nvec = A.nvec;

  // ---- x = 0, r = b, p_{-1} = 0; |b|^2
  double acc = 0.0;
  for (int a = wg; a < Nc; a += G)
    for (int e = tid; e < nvec; e += kCT) {
      const size_t idx = (size_t)a * nvec + e;
      const c64 bv = A.b[idx];
      A.x[idx] = cmk(0.f, 0.f);
      st_coherent(A.r + idx, bv);
      st_coherent(A.p1 + idx, cmk(0.f, 0.f));
      acc += (double)bv.re * bv.re + (double)bv.im * bv.im;
    }
  int buf = 0;
  unsigned epoch = 0;
  store_partials_one(acc, A.part, buf, A.gmax, s_tmp);
  if (!grid_barrier(A.st, G, ++epoch, A.spin_limit)) return flag_error(A.st, A.accumulate);
  sum_partials(A.part, buf, 1, A.gmax, s_rr, s_tmp);
  buf ^= 1;
  if (tid == 0) {
    s_bb[0] = s_rr[0];
    s_beta = 0.f;
    s_it[0] = 0;
  }
  __syncthreads();

  int k = 0;
  for (;; ++k) {
    // uniform stopping test (every workgroup holds the same sums)
    if (!isfinite(s_rr[0])) {
      if (tid == 0) __hip_atomic_store(&A.st->res.err, 2u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      break;
    }
    if (s_rr[0] <= A.tol2 * s_bb[0] || k >= A.maxiter) break;
    c64* pk = (k & 1) ? A.p1 : A.p0;
    const c64* pprev = (k & 1) ? A.p0 : A.p1;

    // ---- phase A: p_k on own sites, w = A p_k, partial <p_k, w>
    acc = 0.0;
    const float be = s_beta;
    for (int a = wg; a < Nc; a += G) {
      for (int e = tid; e < nvec; e += kCT) {
        const size_t idx = (size_t)a * nvec + e;
        const c64 rv = ld_coherent(A.r + idx), qv = ld_coherent(pprev + idx);
        st_coherent(pk + idx, cmk(fmaf(be, qv.re, rv.re), fmaf(be, qv.im, rv.im)));
      }
      // the site's operand p_k at its 81 neighbours, formed from r_k and
      // p_{k-1} (coherent loads) into LDS in one coalesced pass
      {
        const int* nb = A.nbr + (size_t)a * kStencil;
        for (int e = tid; e < kStencil * nvec; e += kCT) {
          const int l = e / nvec;
          const size_t idx = (size_t)nb[l] * nvec + (e - l * nvec);
          const c64 rv = ld_coherent(A.r + idx), qv = ld_coherent(pprev + idx);
          s_in[e] = cmk(fmaf(be, qv.re, rv.re), fmaf(be, qv.im, rv.im));
        }
        __syncthreads();
      }
      if constexpr (MODE == 0) {
        capply_site<float, 1, 12, true>(A.AT, A.nbr, s_in, A.w, a, Nc, nvec, 1, 0, reinterpret_cast<c64*>(red_raw));
      } else {
        capply_site_mfma<MODE == 1, MT, 1, 8, (K32 ? 2 : (MT >= 3 ? 3 : 4)), true, false, K32>(
            A.F, A.rho, A.smax, A.nbr, s_in, A.w, a, Nc, nvec, 1, A.ksteps, reinterpret_cast<f32x4*>(red_raw));
      }
      for (int e = tid; e < nvec; e += kCT) {
        const size_t idx = (size_t)a * nvec + e;
        const c64 pv = ld_coherent(pk + idx), wv = A.w[idx];
        acc += (double)pv.re * wv.re + (double)pv.im * wv.im;
      }
    }
    store_partials_one(acc, A.part, buf, A.gmax, s_tmp);
    if (!grid_barrier(A.st, G, ++epoch, A.spin_limit)) return flag_error(A.st, A.accumulate);
    sum_partials(A.part, buf, 1, A.gmax, s_pap, s_tmp);
    buf ^= 1;
    if (tid == 0) s_alpha = s_pap[0] != 0.0 ? s_rr[0] / s_pap[0] : 0.0;
    __syncthreads();

    // ---- phase B: x += alpha p_k, r -= alpha w; partial |r|^2
    acc = 0.0;
    const float al = (float)s_alpha;
    for (int a = wg; a < Nc; a += G)
      for (int e = tid; e < nvec; e += kCT) {
        const size_t idx = (size_t)a * nvec + e;
        const c64 pv = ld_coherent(pk + idx), wv = A.w[idx];
        c64 xv = A.x[idx], rv = ld_coherent(A.r + idx);
        xv = cmk(fmaf(al, pv.re, xv.re), fmaf(al, pv.im, xv.im));
        rv = cmk(fmaf(-al, wv.re, rv.re), fmaf(-al, wv.im, rv.im));
        A.x[idx] = xv;
        st_coherent(A.r + idx, rv);
        acc += (double)rv.re * rv.re + (double)rv.im * rv.im;
      }
    store_partials_one(acc, A.part, buf, A.gmax, s_tmp);
    if (!grid_barrier(A.st, G, ++epoch, A.spin_limit)) return flag_error(A.st, A.accumulate);
    sum_partials(A.part, buf, 1, A.gmax, s_pap, s_tmp);  // s_pap reused for |r_{k+1}|^2
    buf ^= 1;
    if (tid == 0) {
      const double old = s_rr[0], nw = s_pap[0];
      s_beta = old > 0.0 ? (float)(nw / old) : 0.f;
      s_rr[0] = nw;
      s_it[0] = (unsigned)(k + 1);
    }
    __syncthreads();
  }
  if (wg == 0 && tid == 0 && A.accumulate) A.st->tot.err |= ld_flag(&A.st->res.err);
  finish(A.st, k, 1, s_rr, s_it, A.accumulate);
}

// Several right-hand sides (2 <= nr <= 16; NT = 1 for nr <= 8, 2 above).
// Complex64 on the FP32 MFMA (MODE 3, nvec % 4 == 0): NT and MT as for the
// 16-bit modes.  Complex64 on the VALU (MODE 0, any other nvec): NT = 1, 2,
// 4 for nr <= 4, 8, 16, and the mat-vec takes 4 NT right-hand sides per
// pass over the operator (one pass).
// Element slots: thread tid owns the elements e = tid and e = tid + kCT of
// every site (e = rhs * nvec + j < nr * nvec <= 2 kCT), so each thread's
// partial sums belong to two fixed right-hand sides.
template <int MODE, int MT, int NT, bool K32>
__global__ void __launch_bounds__(kCT) __attribute__((amdgpu_waves_per_eu(2))) k_coarse_cg_mrhs(PcgArgs A) {
  constexpr int NR0 = 4 * NT;                        // MODE 0: right-hand sides per pass
  constexpr int U0 = NR0 >= 16 ? 2 : (NR0 >= 8 ? 4 : 8);  // and columns in flight
  constexpr int kRedBytes = MODE == 0 ? kCT * NR0 * (int)sizeof(c64) : 8 * MT * NT * 64 * (int)sizeof(f32x4);
  __shared__ __align__(16) unsigned char red_raw[kRedBytes];
  __shared__ double s_tmp[2 * kCT];
  __shared__ double s_rr[kMaxR], s_bb[kMaxR], s_sum[kMaxR], s_alpha[kMaxR];
  __shared__ float s_beta[kMaxR];
  __shared__ unsigned s_it[kMaxR];
  __shared__ int s_act[kMaxR];
  __shared__ int s_any;
  const int G = gridDim.x, wg = blockIdx.x, tid = threadIdx.x;
  const int Nc = A.Nc, nvec = A.nvec, nr = A.nr;
  const int ne = nr * nvec;
  const int e0 = tid, e1 = tid + kCT;
  const bool has0 = e0 < ne, has1 = e1 < ne;
  const int q0 = has0 ? e0 / nvec : 0, q1 = has1 ? e1 / nvec : 0;  // their right-hand sides
  const size_t o0 = has0 ? (size_t)q0 * Nc * nvec + (e0 - q0 * nvec) : 0;
  const size_t o1 = has1 ? (size_t)q1 * Nc * nvec + (e1 - q1 * nvec) : 0;

  // ---- x = 0, r = b, p_0 = b; |b|^2
  double acc0 = 0.0, acc1 = 0.0;
  for (int a = wg; a < Nc; a += G) {
    const size_t so = (size_t)a * nvec;
    if (has0) {
      const c64 bv = A.b[o0 + so];
      A.x[o0 + so] = cmk(0.f, 0.f);
      A.r[o0 + so] = bv;
      st_coherent(A.p0 + o0 + so, bv);
      acc0 += (double)bv.re * bv.re + (double)bv.im * bv.im;
    }
    if (has1) {
      const c64 bv = A.b[o1 + so];
      A.x[o1 + so] = cmk(0.f, 0.f);
      A.r[o1 + so] = bv;
      st_coherent(A.p0 + o1 + so, bv);
      acc1 += (double)bv.re * bv.re + (double)bv.im * bv.im;
    }
  }
  int buf = 0;
  unsigned epoch = 0;
  store_partials_slots(acc0, acc1, nr, nvec, A.part, buf, A.gmax, s_tmp);
  if (!grid_barrier(A.st, G, ++epoch, A.spin_limit)) return flag_error(A.st, A.accumulate);
  sum_partials(A.part, buf, nr, A.gmax, s_rr, s_tmp);
  buf ^= 1;
  if (tid < nr) {
    s_bb[tid] = s_rr[tid];
    s_act[tid] = 1;
    s_it[tid] = 0;
  }
  __syncthreads();

  int k = 0;
  for (;; ++k) {
    // uniform per-right-hand-side masks (every workgroup holds the same sums)
    if (tid == 0) {
      int any = 0, bad = 0;
      for (int r = 0; r < nr; ++r) {
        if (!isfinite(s_rr[r])) bad = 1;
        if (s_act[r] && s_rr[r] <= A.tol2 * s_bb[r]) {
          s_act[r] = 0;  // converged after k iterations: x and r frozen from here
          s_it[r] = (unsigned)k;
        }
        any |= s_act[r];
      }
      if (bad) __hip_atomic_store(&A.st->res.err, 2u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      s_any = bad ? 0 : any;
    }
    __syncthreads();
    if (!s_any || k >= A.maxiter) break;
    const c64* pk = (k & 1) ? A.p1 : A.p0;
    c64* pn = (k & 1) ? A.p0 : A.p1;

    // ---- phase A: w = A p_k for all right-hand sides, partial <p_k, w>
    // (p_k, published by coherent stores before the barrier, is gathered
    // through the caches after an agent-scope acquire, which drops this
    // XCD's stale lines, so that its 81-fold reuse across the sites hits L2)
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    acc0 = acc1 = 0.0;
    for (int a = wg; a < Nc; a += G) {
      if constexpr (MODE == 0) {
        for (int r0 = 0; r0 < nr; r0 += NR0)
          capply_site<float, NR0, U0, false, kStencil, false>(A.AT, A.nbr, pk, A.w, a, Nc, nvec, nr, r0,
                                                              reinterpret_cast<c64*>(red_raw));
      } else if constexpr (MODE == 3) {
        capply_site_cmfma<float, MT, NT, 8, 2>(A.AT, A.nbr, pk, A.w, a, Nc, nvec, nr,
                                                reinterpret_cast<f32x4*>(red_raw));
      } else {
        capply_site_mfma<MODE == 1, MT, NT, 8, (K32 ? 2 : (MT >= 3 ? 3 : 4)), false, false, K32>(
            A.F, A.rho, A.smax, A.nbr, pk, A.w, a, Nc, nvec, nr, A.ksteps, reinterpret_cast<f32x4*>(red_raw));
      }
      const size_t so = (size_t)a * nvec;
      if (has0) {
        const c64 pv = ld_coherent(pk + o0 + so), wv = A.w[o0 + so];
        acc0 += (double)pv.re * wv.re + (double)pv.im * wv.im;
      }
      if (has1) {
        const c64 pv = ld_coherent(pk + o1 + so), wv = A.w[o1 + so];
        acc1 += (double)pv.re * wv.re + (double)pv.im * wv.im;
      }
    }
    store_partials_slots(acc0, acc1, nr, nvec, A.part, buf, A.gmax, s_tmp);
    if (!grid_barrier(A.st, G, ++epoch, A.spin_limit)) return flag_error(A.st, A.accumulate);
    sum_partials(A.part, buf, nr, A.gmax, s_sum, s_tmp);
    buf ^= 1;
    if (tid < nr) s_alpha[tid] = (s_act[tid] && s_sum[tid] != 0.0) ? s_rr[tid] / s_sum[tid] : 0.0;
    __syncthreads();

    // ---- phase B: x += alpha p_k, r -= alpha w; partial |r|^2
    acc0 = acc1 = 0.0;
    {
      const float al0 = (float)s_alpha[q0], al1 = (float)s_alpha[q1];
      for (int a = wg; a < Nc; a += G) {
        const size_t so = (size_t)a * nvec;
        if (has0) {
          const size_t i = o0 + so;
          const c64 pv = ld_coherent(pk + i), wv = A.w[i];
          c64 xv = A.x[i], rv = A.r[i];
          xv = cmk(fmaf(al0, pv.re, xv.re), fmaf(al0, pv.im, xv.im));
          rv = cmk(fmaf(-al0, wv.re, rv.re), fmaf(-al0, wv.im, rv.im));
          A.x[i] = xv;
          A.r[i] = rv;
          acc0 += (double)rv.re * rv.re + (double)rv.im * rv.im;
        }
        if (has1) {
          const size_t i = o1 + so;
          const c64 pv = ld_coherent(pk + i), wv = A.w[i];
          c64 xv = A.x[i], rv = A.r[i];
          xv = cmk(fmaf(al1, pv.re, xv.re), fmaf(al1, pv.im, xv.im));
          rv = cmk(fmaf(-al1, wv.re, rv.re), fmaf(-al1, wv.im, rv.im));
          A.x[i] = xv;
          A.r[i] = rv;
          acc1 += (double)rv.re * rv.re + (double)rv.im * rv.im;
        }
      }
    }
    store_partials_slots(acc0, acc1, nr, nvec, A.part, buf, A.gmax, s_tmp);
    if (!grid_barrier(A.st, G, ++epoch, A.spin_limit)) return flag_error(A.st, A.accumulate);
    sum_partials(A.part, buf, nr, A.gmax, s_sum, s_tmp);
    buf ^= 1;
    if (tid < nr) {
      const double old = s_rr[tid], nw = s_sum[tid];
      s_beta[tid] = (s_act[tid] && old > 0.0) ? (float)(nw / old) : 0.f;
      s_rr[tid] = nw;
    }
    __syncthreads();

    // ---- phase P: p_{k+1} = r_{k+1} + beta_k p_k on own sites
    {
      const float be0 = s_beta[q0], be1 = s_beta[q1];
      for (int a = wg; a < Nc; a += G) {
        const size_t so = (size_t)a * nvec;
        if (has0) {
          const size_t i = o0 + so;
          const c64 rv = A.r[i], qv = ld_coherent(pk + i);
          st_coherent(pn + i, cmk(fmaf(be0, qv.re, rv.re), fmaf(be0, qv.im, rv.im)));
        }
        if (has1) {
          const size_t i = o1 + so;
          const c64 rv = A.r[i], qv = ld_coherent(pk + i);
          st_coherent(pn + i, cmk(fmaf(be1, qv.re, rv.re), fmaf(be1, qv.im, rv.im)));
        }
      }
    }
    if (!grid_barrier(A.st, G, ++epoch, A.spin_limit)) return flag_error(A.st, A.accumulate);
  }
  if (tid < nr && s_act[tid]) s_it[tid] = (unsigned)k;  // still unconverged at maxiter
  __syncthreads();
  if (wg == 0 && tid == 0 && A.accumulate) A.st->tot.err |= ld_flag(&A.st->res.err);
  finish(A.st, k, nr, s_rr, s_it, A.accumulate);
}

// kernel of (single or batched, mode, M tiles, N tiles, MFMA form)
template <int MODE, int MT, int NT, bool BATCH, bool K32>
const void* kernel_of() {
  if constexpr (BATCH)
    return reinterpret_cast<const void*>(&k_coarse_cg_mrhs<MODE, MT, NT, K32>);
  else
    return reinterpret_cast<const void*>(&k_coarse_cg<MODE, MT, K32>);
}

// Workgroups of the kernel that can be resident at once, cached per kernel.
template <int MODE, int MT, int NT, bool BATCH, bool K32>
int max_grid(int* out) {
  static int cached = 0;
  if (!cached) {
    int dev = 0, cus = 0, per = 0;
    HDCG_HIP(hipGetDevice(&dev));
    HDCG_HIP(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
    HDCG_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, kernel_of<MODE, MT, NT, BATCH, K32>(), kCT, 0));
    cached = per * cus;
  }
  *out = cached;
  return DWF_OK;
}

// The instantiation for the runtime (batch, mode, M tiles, N tiles, form):
// its resident-grid size (query) or its launch.  The launch is an ordinary
// one (it may then sit in a captured graph) with a grid no larger than what
// can be resident at once; every workgroup then runs concurrently, and a
// barrier that still waited past its spin limit ends the solve with an
// error instead of hanging.
template <int MODE, int MT, int NT, bool BATCH, bool K32>
int pcg_call(bool query, const PcgArgs* a, int G, int* gmax, hipStream_t st) {
  if (query) return max_grid<MODE, MT, NT, BATCH, K32>(gmax);
  if constexpr (BATCH)
    hipLaunchKernelGGL((k_coarse_cg_mrhs<MODE, MT, NT, K32>), dim3(G), dim3(kCT), 0, st, *a);
  else
    hipLaunchKernelGGL((k_coarse_cg<MODE, MT, K32>), dim3(G), dim3(kCT), 0, st, *a);
  HDCG_HIP(hipGetLastError());
  return DWF_OK;
}

template <int MODE, bool BATCH, int NT, bool K32>
int pcg_mt(int mt, bool query, const PcgArgs* a, int G, int* gmax, hipStream_t st) {
  switch (mt) {
    case 1: return pcg_call<MODE, 1, NT, BATCH, K32>(query, a, G, gmax, st);
    case 2: return pcg_call<MODE, 2, NT, BATCH, K32>(query, a, G, gmax, st);
    case 3: return pcg_call<MODE, 3, NT, BATCH, K32>(query, a, G, gmax, st);
    default: return pcg_call<MODE, 4, (NT > 1 && MODE != 0 ? 1 : NT), BATCH, K32>(query, a, G, gmax, st);
  }
}

template <int MODE, bool BATCH, int NT>
int pcg_form(bool k32, int mt, bool query, const PcgArgs* a, int G, int* gmax, hipStream_t st) {
  return k32 ? pcg_mt<MODE, BATCH, NT, true>(mt, query, a, G, gmax, st)
             : pcg_mt<MODE, BATCH, NT, false>(mt, query, a, G, gmax, st);
}

// k32: the 16x16x32 MFMA form (16-bit modes with nvec % 8 == 0)
int pcg_dispatch(int mode, int mt, bool k32, int nr, bool query, const PcgArgs* a, int G, int* gmax, hipStream_t st) {
  if (nr == 1) {
    if (mode == 0) return pcg_call<0, 1, 1, false, false>(query, a, G, gmax, st);
    return mode == 1 ? pcg_form<1, false, 1>(k32, mt, query, a, G, gmax, st)
                     : pcg_form<2, false, 1>(k32, mt, query, a, G, gmax, st);
  }
  if (mode == 3) return nr <= 8 ? pcg_mt<3, true, 1, false>(mt, query, a, G, gmax, st)
                                 : pcg_mt<3, true, 2, false>(mt, query, a, G, gmax, st);
  if (mode == 0) {
    if (nr <= 4) return pcg_call<0, 1, 1, true, false>(query, a, G, gmax, st);
    if (nr <= 8) return pcg_call<0, 1, 2, true, false>(query, a, G, gmax, st);
    return pcg_call<0, 1, 4, true, false>(query, a, G, gmax, st);
  }
  if (nr <= 8)
    return mode == 1 ? pcg_form<1, true, 1>(k32, mt, query, a, G, gmax, st)
                     : pcg_form<2, true, 1>(k32, mt, query, a, G, gmax, st);
  return mode == 1 ? pcg_form<1, true, 2>(k32, mt, query, a, G, gmax, st)
                   : pcg_form<2, true, 2>(k32, mt, query, a, G, gmax, st);
}

// ---------------------------------------------------------- workspace --
// Device memory of one persistent solve: r, p0, p1, w (n = Nc nvec nr
// complex64 each), the partial sums and the barrier / result state.
struct PcgWork {
  c64 *r, *p0, *p1, *w;
  double* part;
  PcgState* st;
};

constexpr size_t align256(size_t n) { return (n + 255) & ~(size_t)255; }

size_t work_bytes(size_t n, int G) {
  return 4 * align256(n * sizeof(c64)) + align256(sizeof(double) * 2 * kMaxR * (size_t)G) + align256(sizeof(PcgState));
}

PcgWork carve(unsigned char* base, size_t n, int G) {
  PcgWork w;
  const size_t v = align256(n * sizeof(c64));
  w.r = reinterpret_cast<c64*>(base);
  w.p0 = reinterpret_cast<c64*>(base + v);
  w.p1 = reinterpret_cast<c64*>(base + 2 * v);
  w.w = reinterpret_cast<c64*>(base + 3 * v);
  w.part = reinterpret_cast<double*>(base + 4 * v);
  w.st = reinterpret_cast<PcgState*>(base + 4 * v + align256(sizeof(double) * 2 * kMaxR * (size_t)G));
  return w;
}

// The 16x16x32 MFMA form for the 16-bit modes when nvec allows it (8 K
// values of one stencil point per lane); the autotuner of the standalone
// mat-vec picks this form on every workload shape measured.
bool use_k32(int mode, int nvec) { return (mode == 1 || mode == 2) && nvec % 8 == 0; }

// Shape of the launch for (mprec, nr): mode, M tiles and the grid; false
// when the persistent form does not apply.
bool plan(hdcg* h, int mprec, int nr, int* mode, int* mt, int* G) {
  const int nv = h->nvec;
  const bool m16 = mprec == DWF_BF16 || mprec == DWF_F16;
  if (nr < 1 || nr > kMaxR || nv > kMaxNvec || nr * nv > 2 * kCT) return false;
  if (m16 && (nv % 4 != 0 || nv > 64)) return false;
  *mt = (nv + 15) / 16;
  if (m16 && nr > 8 && *mt > 3) return false;  // the 2-tile-wide reduction of 4 M tiles exceeds LDS
  *mode = !m16 ? 0 : (mprec == DWF_BF16 ? 1 : 2);
  // complex64 with several right-hand sides: the FP32 MFMA form where its
  // column runs and LDS reduction fit
  if (!m16 && nr > 1 && nv % 4 == 0 && nv <= 64 && (nr <= 8 || *mt <= 3)) *mode = 3;
  int gmax = 0;
  if (pcg_dispatch(*mode, *mt, use_k32(*mode, nv), nr, true, nullptr, 0, &gmax, nullptr) < 0 || gmax < 1) return false;
  *G = std::min(std::min(h->Nc, gmax), kMaxGrid);
  return true;
}

// Enqueue one persistent solve on `st` (no host synchronisation).
int launch_solve(hdcg* h, const PcgWork& wk, int mode, int mt, int G, int mprec, c64* x, const c64* b, int nr,
                 double tol, int maxiter, hipStream_t st, int accumulate = 0) {
  const int nv = h->nvec;
  const bool m16 = mode == 1 || mode == 2;
  PcgArgs a;
  a.Nc = h->Nc;
  a.nvec = nv;
  a.nr = nr;
  a.maxiter = maxiter;
  a.accumulate = accumulate;
  a.ksteps = (2 * kStencil * nv + 15) / 16;
  a.gmax = G;
  a.tol2 = tol * tol;
  a.spin_limit = 1u << 21;  // >= 50 ms of waiting at 64+ cycles per poll
  a.AT = h->AT64.as<c64>();
  a.F = m16 ? (mprec == DWF_BF16 ? h->mf_bf16 : h->mf_f16).as<unsigned short>() : nullptr;
  a.rho = h->mf_rho.as<float>();
  a.smax = h->mf_smax.as<float>();
  a.nbr = h->nbr.as<int>();
  a.b = b;
  a.x = x;
  a.r = wk.r;
  a.p0 = wk.p0;
  a.p1 = wk.p1;
  a.w = wk.w;
  a.part = wk.part;
  a.st = wk.st;
  hipLaunchKernelGGL(k_pcg_reset, dim3(1), dim3(256), 0, st, a.st, G);
  HDCG_HIP(hipGetLastError());
  return pcg_dispatch(mode, mt, use_k32(mode, nv), nr, false, &a, G, nullptr, st);
}

// Read one solve's results back (synchronises).
int read_result(hdcg* h, const PcgWork& wk, int nr, int* iters, int* iters_rhs, hipStream_t st) {
  auto* hs = reinterpret_cast<PcgState::Result*>(h->pinned + 64 * 14);
  HDCG_HIP(hipMemcpyAsync(hs, &wk.st->res, sizeof(PcgState::Result), hipMemcpyDeviceToHost, st));
  HDCG_HIP(hipStreamSynchronize(st));
  if (hs->err == 1) return fail(DWF_ERR_HIP, "persistent coarse CG: grid barrier wait exceeded its limit");
  if (hs->err == 2) return fail(DWF_ERR_NUMERIC, "coarse CG residual not finite");
  if (iters) *iters = (int)hs->iters;
  if (iters_rhs)
    for (int r = 0; r < nr; ++r) iters_rhs[r] = (int)hs->iters_rhs[r];
  return DWF_OK;
}

bool mfma_ready(hdcg* h, int mprec) {
  return (mprec == DWF_BF16 && h->mf_have_bf16) || (mprec == DWF_F16 && h->mf_have_f16);
}

PcgWork handle_work(hdcg* h) {
  PcgWork w;
  w.r = h->cw[0].as<c64>();
  w.p0 = h->cw[1].as<c64>();
  w.p1 = h->cw[2].as<c64>();
  w.w = h->cw[5].as<c64>();
  w.part = h->pcg_part.as<double>();
  w.st = h->pcg_state.as<PcgState>();
  return w;
}

int ensure_handle_work(hdcg* h, int nr, int G) {
  const size_t n = (size_t)h->Nc * h->nvec * nr;
  for (int i : {0, 1, 2, 5}) HDCG_TRY(h->cw[i].ensure(n * sizeof(c128)));
  HDCG_TRY(h->pcg_part.ensure(sizeof(double) * 2 * kMaxR * (size_t)G));
  HDCG_TRY(h->pcg_state.ensure(sizeof(PcgState)));
  return DWF_OK;
}

}  // namespace

// Returns DWF_OK with *done = 0 when the persistent form does not apply
// (more than 16 right-hand sides, unsuited nvec); the caller then runs the
// launch-per-step coarse CG.  iters_rhs (nullable): per right-hand side, the
// iterations it ran before its residual reached tol.
int coarse_cg_persistent(hdcg* h, int mprec, c64* x, const c64* b, int nr, double tol, int maxiter, int* iters,
                         int* iters_rhs, int* done, hipStream_t st) {
  *done = 0;
  int mode = 0, mt = 1, G = 0;
  if (!plan(h, mprec, nr, &mode, &mt, &G)) return DWF_OK;
  if ((mprec == DWF_BF16 || mprec == DWF_F16) && !mfma_ready(h, mprec)) HDCG_TRY(crs_build_mfma(h, mprec, st));
  HDCG_TRY(ensure_handle_work(h, nr, G));
  const PcgWork wk = handle_work(h);
  HDCG_TRY(launch_solve(h, wk, mode, mt, G, mprec, x, b, nr, tol, maxiter, st));
  HDCG_TRY(read_result(h, wk, nr, iters, iters_rhs, st));
  *done = 1;
  return DWF_OK;
}

// The same without reading the result: the solve only enqueues work on st
// (it may be captured into a graph), and its iteration counts and error
// flag are added to the device totals that coarse_cg_totals reads.  The
// work memory must already be sized (a solve with coarse_cg_persistent of
// the same shape ran before); *done = 0 otherwise.
int coarse_cg_persistent_deferred(hdcg* h, int mprec, c64* x, const c64* b, int nr, double tol, int maxiter,
                                  int* done, hipStream_t st) {
  *done = 0;
  int mode = 0, mt = 1, G = 0;
  if (!plan(h, mprec, nr, &mode, &mt, &G)) return DWF_OK;
  if ((mprec == DWF_BF16 || mprec == DWF_F16) && !mfma_ready(h, mprec)) return DWF_OK;
  const size_t n = (size_t)h->Nc * h->nvec * nr;
  if (h->cw[5].bytes < n * sizeof(c128) || h->pcg_part.bytes < sizeof(double) * 2 * kMaxR * (size_t)G ||
      h->pcg_state.bytes < sizeof(PcgState))
    return DWF_OK;
  HDCG_TRY(launch_solve(h, handle_work(h), mode, mt, G, mprec, x, b, nr, tol, maxiter, st, 1));
  *done = 1;
  return DWF_OK;
}

// Clear the device totals of the handle's persistent solves (a kernel, so
// it may precede captured solves).
int coarse_cg_clear_totals(hdcg* h, hipStream_t st) {
  HDCG_TRY(h->pcg_state.ensure(sizeof(PcgState)));
  hipLaunchKernelGGL(k_pcg_clear, dim3(1), dim3(64), 0, st, h->pcg_state.as<PcgState>());
  HDCG_HIP(hipGetLastError());
  return DWF_OK;
}

// Read the totals of the deferred solves (synchronises): their number, and
// (added to *iters and iters_rhs[0..nr)) the iterations summed over them,
// overall and per right-hand side; an error flag raised by any of them
// becomes the return code.
int coarse_cg_totals(hdcg* h, int nr, int* solves, long long* iters, long long* iters_rhs, hipStream_t st) {
  if (h->pcg_state.bytes < sizeof(PcgState)) return fail(DWF_ERR_STATE, "no persistent coarse solve has run");
  auto* hs = reinterpret_cast<PcgState::Totals*>(h->pinned + 64 * 15);
  HDCG_HIP(hipMemcpyAsync(hs, &h->pcg_state.as<PcgState>()->tot, sizeof(PcgState::Totals), hipMemcpyDeviceToHost,
                          st));
  HDCG_HIP(hipStreamSynchronize(st));
  if (hs->err & 1u) return fail(DWF_ERR_HIP, "persistent coarse CG: grid barrier wait exceeded its limit");
  if (hs->err & 2u) return fail(DWF_ERR_NUMERIC, "coarse CG residual not finite");
  if (solves) *solves = (int)hs->solves;
  if (iters) *iters += hs->iters;
  if (iters_rhs)
    for (int r = 0; r < nr && r < kMaxR; ++r) iters_rhs[r] += hs->iters_rhs[r];
  return DWF_OK;
}

// Bytes of work memory a persistent solve of nr right-hand sides needs on
// this handle (0 when the persistent form does not apply).
size_t coarse_cg_work_bytes(hdcg* h, int mprec, int nr) {
  int mode = 0, mt = 1, G = 0;
  if (!plan(h, mprec, nr, &mode, &mt, &G)) return 0;
  return work_bytes((size_t)h->Nc * h->nvec * nr, G);
}

// The persistent solve with its work memory at `work` (device,
// coarse_cg_work_bytes bytes, 256-byte aligned) instead of the handle's
// buffers; allocates nothing.  The 16-bit storage must exist.  Synchronises.
int coarse_cg_persistent_in(hdcg* h, void* work, int mprec, c64* x, const c64* b, int nr, double tol, int maxiter,
                            int* iters, hipStream_t st) {
  int mode = 0, mt = 1, G = 0;
  if (!plan(h, mprec, nr, &mode, &mt, &G)) return fail(DWF_ERR_ARG, "shape not covered by the persistent coarse solve");
  if ((mprec == DWF_BF16 || mprec == DWF_F16) && !mfma_ready(h, mprec))
    return fail(DWF_ERR_STATE, "the 16-bit coarse storage is not built");
  const PcgWork wk = carve(static_cast<unsigned char*>(work), (size_t)h->Nc * h->nvec * nr, G);
  HDCG_TRY(launch_solve(h, wk, mode, mt, G, mprec, x, b, nr, tol, maxiter, st));
  return read_result(h, wk, nr, iters, nullptr, st);
}

}  // namespace hdk

