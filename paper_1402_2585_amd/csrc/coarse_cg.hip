// The coarse solve inside Q (A-DEF2, Sec. IV.E): conjugate gradient on the
// little Dirac operator A (Sec. V.A) as ONE persistent cooperative kernel.
//
// A coarse CG iteration is a mat-vec over Nc sites plus a few reductions
// over Nc * Nvec numbers; launched kernel by kernel it is dominated by
// launch and reduction latency.  Here every workgroup owns the coarse sites
// a = wg, wg + G, ... for the whole solve and the iteration needs two
// grid-wide barriers:
//
//   phase A   p_k = r_k + beta_{k-1} p_{k-1} on own sites (p double
//             buffered); w = A p_k with p_k at neighbour sites formed from
//             r_k and p_{k-1} as they are read; partial <p_k, w>
//   barrier   alpha_k = |r_k|^2 / <p_k, A p_k>
//   phase B   x += alpha_k p_k, r -= alpha_k w on own sites; partial |r|^2
//   barrier   beta_k = |r_{k+1}|^2 / |r_k|^2; stop when every right-hand
//             side has |r|^2 <= tol^2 |b|^2, or at maxiter
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
// another reads (r and p at a site, the partial sums) is stored and loaded
// with relaxed device-scope atomics, which are coherent across the XCDs'
// L2 caches; before arriving at a barrier every wave waits for its stores
// to complete.  Values a workgroup only reads and writes for its own sites
// (x, w) and the operator itself use ordinary accesses.
#include <algorithm>

#include "coarse_dev.h"

namespace hdk {

namespace {

constexpr int kMaxR = 8;  // right-hand sides per persistent solve

// Grid barrier state.  Barrier number e (e = 1, 2, ...): every workgroup
// stores e into its own arrival slot; workgroup 0 polls all slots (one per
// thread) until every one holds e, then stores e into the release flag,
// which the other workgroups poll.  Plain coherent stores and loads, no
// read-modify-write on a shared address; the values only grow, so nothing
// is reset between barriers.
constexpr int kMaxGrid = 4096;
struct PcgState {
  unsigned arrive[kMaxGrid];  // last barrier each workgroup reached
  alignas(128) unsigned release;
  alignas(128) struct Result {
    unsigned err;             // 1: barrier wait exceeded, 2: non-finite residual
    unsigned iters;
    double rr[kMaxR];         // final |r|^2
  } res;
};

struct PcgArgs {
  int Nc, nvec, nr, maxiter, ksteps, gmax;
  double tol2;
  unsigned spin_limit;
  const c64* AT;              // complex64 operator, AT[a][l][k][j]
  const unsigned short* F;    // 16-bit fragment storage
  const float* rho;
  const float* smax;
  const int* nbr;
  const c64* b;
  c64 *x, *r, *p0, *p1, *w;  // r, p0, p1: coherent accesses only
  double* part;               // [2][kMaxR][gmax]
  PcgState* st;
};

__global__ void k_pcg_reset(PcgState* st, int G) {
  for (int g = threadIdx.x; g < G; g += blockDim.x) st->arrive[g] = 0;
  if (threadIdx.x == 0) {
    st->release = 0;
    st->res.err = 0;
    st->res.iters = 0;
  }
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

// Sum v[r] over the workgroup; thread 0 stores it as this workgroup's
// partial in buffer `buf`.
__device__ __forceinline__ void store_partials(double (&v)[kMaxR], int nr, double* part, int buf, int gmax,
                                               double* lds /* kMaxR * 8 */) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  for (int r = 0; r < nr; ++r) {
    const double s = wave_sum(v[r]);
    if (lane == 0) lds[r * 8 + wave] = s;
  }
  __syncthreads();
  if (threadIdx.x < nr) {
    double s = 0.0;
    for (int w = 0; w < kCT / 64; ++w) s += lds[threadIdx.x * 8 + w];
    __hip_atomic_store(part + ((size_t)buf * kMaxR + threadIdx.x) * gmax + blockIdx.x, s, __ATOMIC_RELAXED,
                       __HIP_MEMORY_SCOPE_AGENT);
  }
  __syncthreads();
}

// out[r] = sum over all workgroups' partials of buffer `buf` (the same
// fixed order in every workgroup).
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

// One right-hand side.  MODE 0: complex64 VALU operator; 1: bf16 MFMA;
// 2: fp16 MFMA (MT M tiles).
constexpr int kMaxNvec = 64;
template <int MODE, int MT>
__global__ void __launch_bounds__(kCT) __attribute__((amdgpu_waves_per_eu(4))) k_coarse_cg(PcgArgs A) {
  constexpr int kRedBytes = MODE == 0 ? kCT * (int)sizeof(c64) : 8 * MT * 64 * (int)sizeof(f32x4);
  __shared__ __align__(16) unsigned char red_raw[kRedBytes];
  __shared__ c64 s_in[kStencil * kMaxNvec];  // the site's operand at its neighbours
  __shared__ double s_tmp[kMaxR * 8];
  __shared__ double s_rr[kMaxR], s_bb[kMaxR], s_pap[kMaxR], s_alpha[kMaxR];
  __shared__ float s_beta[kMaxR];
  const int G = gridDim.x, wg = blockIdx.x, tid = threadIdx.x;
  const int Nc = A.Nc, nvec = A.nvec, nr = A.nr;
  const int ne = nr * nvec;  // elements per site over all right-hand sides

  // ---- x = 0, r = b, p_{-1} = 0; |b|^2
  double acc[kMaxR];
#pragma unroll
  for (int r = 0; r < kMaxR; ++r) acc[r] = 0.0;
  for (int a = wg; a < Nc; a += G)
    for (int e = tid; e < ne; e += kCT) {
      const int rr = e / nvec, j = e - rr * nvec;
      const size_t idx = ((size_t)rr * Nc + a) * nvec + j;
      const c64 bv = A.b[idx];
      A.x[idx] = cmk(0.f, 0.f);
      st_coherent(A.r + idx, bv);
      st_coherent(A.p1 + idx, cmk(0.f, 0.f));
#pragma unroll
      for (int r = 0; r < kMaxR; ++r)
        if (r == rr) acc[r] += (double)bv.re * bv.re + (double)bv.im * bv.im;
    }
  int buf = 0;
  unsigned epoch = 0;
  store_partials(acc, nr, A.part, buf, A.gmax, s_tmp);
  if (!grid_barrier(A.st, G, ++epoch, A.spin_limit)) return;
  sum_partials(A.part, buf, nr, A.gmax, s_rr, s_tmp);
  buf ^= 1;
  if (tid < nr) {
    s_bb[tid] = s_rr[tid];
    s_beta[tid] = 0.f;
  }
  __syncthreads();

  int k = 0;
  for (;; ++k) {
    // uniform stopping test (every workgroup holds the same sums)
    bool conv = true, bad = false;
    for (int r = 0; r < nr; ++r) {
      if (!isfinite(s_rr[r])) bad = true;
      if (!(s_rr[r] <= A.tol2 * s_bb[r])) conv = false;
    }
    if (bad) {
      if (tid == 0) __hip_atomic_store(&A.st->res.err, 2u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      break;
    }
    if (conv || k >= A.maxiter) break;
    c64* pk = (k & 1) ? A.p1 : A.p0;
    const c64* pprev = (k & 1) ? A.p0 : A.p1;

    // ---- phase A: p_k on own sites, w = A p_k, partial <p_k, w>
#pragma unroll
    for (int r = 0; r < kMaxR; ++r) acc[r] = 0.0;
    for (int a = wg; a < Nc; a += G) {
      for (int e = tid; e < ne; e += kCT) {
        const int rr = e / nvec;
        const size_t idx = ((size_t)rr * Nc + a) * nvec + (e - rr * nvec);
        const c64 rv = ld_coherent(A.r + idx), qv = ld_coherent(pprev + idx);
        st_coherent(pk + idx, cmk(fmaf(s_beta[rr], qv.re, rv.re), fmaf(s_beta[rr], qv.im, rv.im)));
      }
      // the site's operand p_k at its 81 neighbours, formed from r_k and
      // p_{k-1} (coherent loads) into LDS in one coalesced pass
      {
        const int* nb = A.nbr + (size_t)a * kStencil;
        const float be = s_beta[0];
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
        capply_site_mfma<MODE == 1, MT, 1, 8, (MT >= 3 ? 3 : 4), true>(A.F, A.rho, A.smax, A.nbr, s_in, A.w, a, Nc, nvec, 1,
                                                       A.ksteps, reinterpret_cast<f32x4*>(red_raw));
      }
      for (int e = tid; e < ne; e += kCT) {
        const int rr = e / nvec;
        const size_t idx = ((size_t)rr * Nc + a) * nvec + (e - rr * nvec);
        const c64 pv = ld_coherent(pk + idx), wv = A.w[idx];
        const double d = (double)pv.re * wv.re + (double)pv.im * wv.im;
#pragma unroll
        for (int r = 0; r < kMaxR; ++r)
          if (r == rr) acc[r] += d;
      }
    }
    store_partials(acc, nr, A.part, buf, A.gmax, s_tmp);
    if (!grid_barrier(A.st, G, ++epoch, A.spin_limit)) return;
    sum_partials(A.part, buf, nr, A.gmax, s_pap, s_tmp);
    buf ^= 1;
    if (tid < nr) s_alpha[tid] = s_pap[tid] != 0.0 ? s_rr[tid] / s_pap[tid] : 0.0;
    __syncthreads();

    // ---- phase B: x += alpha p_k, r -= alpha w; partial |r|^2
#pragma unroll
    for (int r = 0; r < kMaxR; ++r) acc[r] = 0.0;
    for (int a = wg; a < Nc; a += G)
      for (int e = tid; e < ne; e += kCT) {
        const int rr = e / nvec;
        const size_t idx = ((size_t)rr * Nc + a) * nvec + (e - rr * nvec);
        const float al = (float)s_alpha[rr];
        const c64 pv = ld_coherent(pk + idx), wv = A.w[idx];
        c64 xv = A.x[idx], rv = ld_coherent(A.r + idx);
        xv = cmk(fmaf(al, pv.re, xv.re), fmaf(al, pv.im, xv.im));
        rv = cmk(fmaf(-al, wv.re, rv.re), fmaf(-al, wv.im, rv.im));
        A.x[idx] = xv;
        st_coherent(A.r + idx, rv);
        const double d = (double)rv.re * rv.re + (double)rv.im * rv.im;
#pragma unroll
        for (int r = 0; r < kMaxR; ++r)
          if (r == rr) acc[r] += d;
      }
    store_partials(acc, nr, A.part, buf, A.gmax, s_tmp);
    if (!grid_barrier(A.st, G, ++epoch, A.spin_limit)) return;
    sum_partials(A.part, buf, nr, A.gmax, s_pap, s_tmp);  // s_pap reused for |r_{k+1}|^2
    buf ^= 1;
    if (tid < nr) {
      const double old = s_rr[tid], nw = s_pap[tid];
      s_beta[tid] = old > 0.0 ? (float)(nw / old) : 0.f;
      s_rr[tid] = nw;
    }
    __syncthreads();
  }
  if (wg == 0 && tid == 0) {
    A.st->res.iters = (unsigned)k;
    for (int r = 0; r < nr; ++r) A.st->res.rr[r] = s_rr[r];
  }
}

template <int MODE, int MT>
int launch_pcg(const PcgArgs& args, int G, hipStream_t st) {
  void* params[] = {const_cast<PcgArgs*>(&args)};
  HDCG_HIP(hipLaunchCooperativeKernel(reinterpret_cast<const void*>(&k_coarse_cg<MODE, MT>), dim3(G), dim3(kCT),
                                      params, 0, st));
  return DWF_OK;
}

// workgroups of k_coarse_cg<MODE, MT> that can be resident at once
template <int MODE, int MT>
int max_grid(int* out) {
  static int cached = 0;
  if (!cached) {
    int dev = 0, cus = 0, per = 0;
    HDCG_HIP(hipGetDevice(&dev));
    HDCG_HIP(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
    HDCG_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(
        &per, reinterpret_cast<const void*>(&k_coarse_cg<MODE, MT>), kCT, 0));
    cached = per * cus;
  }
  *out = cached;
  return DWF_OK;
}

// The instantiation for the runtime (mode, M tiles): its resident-grid size
// (query) or its launch.
template <int MODE, int MT>
int pcg_call(bool query, const PcgArgs* a, int G, int* gmax, hipStream_t st) {
  return query ? max_grid<MODE, MT>(gmax) : launch_pcg<MODE, MT>(*a, G, st);
}
int pcg_dispatch(int mode, int mt, bool query, const PcgArgs* a, int G, int* gmax, hipStream_t st) {
  if (mode == 0) return pcg_call<0, 1>(query, a, G, gmax, st);
  switch (mode * 8 + mt) {
    case 9: return pcg_call<1, 1>(query, a, G, gmax, st);
    case 10: return pcg_call<1, 2>(query, a, G, gmax, st);
    case 11: return pcg_call<1, 3>(query, a, G, gmax, st);
    case 12: return pcg_call<1, 4>(query, a, G, gmax, st);
    case 17: return pcg_call<2, 1>(query, a, G, gmax, st);
    case 18: return pcg_call<2, 2>(query, a, G, gmax, st);
    case 19: return pcg_call<2, 3>(query, a, G, gmax, st);
    default: return pcg_call<2, 4>(query, a, G, gmax, st);
  }
}

}  // namespace

// Returns DWF_OK with *done = 0 when the persistent form does not apply
// (too many right-hand sides, nvec not suited); the caller then runs the
// launch-per-step coarse CG.
int coarse_cg_persistent(hdcg* h, int mprec, c64* x, const c64* b, int nr, double tol, int maxiter,
                         int* iters, int* done, hipStream_t st) {
  *done = 0;
  const int nv = h->nvec;
  const bool m16 = mprec == DWF_BF16 || mprec == DWF_F16;
  // one right-hand side: with several, the operands a workgroup reads from
  // neighbour sites (coherent loads, not cached in L2) cost more than the
  // launches the persistent form saves
  if (nr != 1 || nv > kMaxNvec) return DWF_OK;
  if (m16 && (nv % 4 != 0 || nv > 64)) return DWF_OK;
  const int mt = (nv + 15) / 16;
  int gmax = 0;
  const int mode = !m16 ? 0 : (mprec == DWF_BF16 ? 1 : 2);
  HDCG_TRY(pcg_dispatch(mode, mt, true, nullptr, 0, &gmax, st));
  if (gmax < 1) return DWF_OK;
  const int G = std::min(std::min(h->Nc, gmax), kMaxGrid);
  if (m16 && !((mprec == DWF_BF16 && h->mf_have_bf16) || (mprec == DWF_F16 && h->mf_have_f16)))
    HDCG_TRY(crs_build_mfma(h, mprec, st));

  const size_t n = (size_t)h->Nc * nv * nr;
  for (int i = 0; i < 3; ++i) HDCG_TRY(h->cw[i].ensure(n * sizeof(c128)));
  HDCG_TRY(h->pcg_part.ensure(sizeof(double) * 2 * kMaxR * (size_t)G));
  HDCG_TRY(h->pcg_state.ensure(sizeof(PcgState)));
  PcgArgs a;
  a.Nc = h->Nc;
  a.nvec = nv;
  a.nr = nr;
  a.maxiter = maxiter;
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
  a.r = h->cw[0].as<c64>();
  a.p0 = h->cw[1].as<c64>();
  a.p1 = h->cw[1].as<c64>() + n;  // cw[1] holds 2n complex64 (sized for complex128)
  a.w = h->cw[2].as<c64>();
  a.part = h->pcg_part.as<double>();
  a.st = h->pcg_state.as<PcgState>();
  hipLaunchKernelGGL(k_pcg_reset, dim3(1), dim3(256), 0, st, a.st, G);
  HDCG_HIP(hipGetLastError());
  HDCG_TRY(pcg_dispatch(mode, mt, false, &a, G, nullptr, st));
  auto* hs = reinterpret_cast<PcgState::Result*>(h->pinned + 64 * 14);
  HDCG_HIP(hipMemcpyAsync(hs, &a.st->res, sizeof(PcgState::Result), hipMemcpyDeviceToHost, st));
  HDCG_HIP(hipStreamSynchronize(st));
  if (hs->err == 1) return fail(DWF_ERR_HIP, "persistent coarse CG: grid barrier wait exceeded its limit");
  if (hs->err == 2) return fail(DWF_ERR_NUMERIC, "coarse CG residual not finite");
  if (iters) *iters = (int)hs->iters;
  *done = 1;
  return DWF_OK;
}

}  // namespace hdk
