// Device code of the little Dirac operator mat-vec, shared by the
// standalone mat-vec kernels and the persistent coarse CG kernel.
//
// (A c)[r][a][j] = sum_l sum_k A[a][l][j][k] c[r][nbr(a,l)][k]   (Sec. V.A)
//
// Every form takes one coarse site a per workgroup: 512 threads for the VALU
// form, NW waves for the MFMA forms.
#pragma once

#include <type_traits>

#include "hdcg_impl.h"

namespace hdk {

constexpr int kCT = 512;  // threads per coarse-site workgroup

// The one-hop truncation of the stencil (Sec. V.B): kOneHop points, point m
// at stencil index l = sum_mu (d_mu + 1) 3^mu; m = 0 the site, m = 2 mu + 1
// and 2 mu + 2 the neighbours at -1 and +1 in direction mu.
constexpr int kOneHop = 9;
__host__ __device__ inline int one_hop_l(int m) {
  if (m == 0) return 40;
  const int mu = (m - 1) >> 1;
  const int p3 = mu == 0 ? 1 : mu == 1 ? 3 : mu == 2 ? 9 : 27;
  return (m & 1) ? 40 - p3 : 40 + p3;
}

// Loads and stores of complex64 values that other workgroups of a running
// persistent kernel write or read: relaxed device-scope atomics, coherent
// across the XCDs' L2 caches without whole-cache write-back or invalidation.
__device__ __forceinline__ c64 ld_coherent(const c64* p) {
  const unsigned long long v =
      __hip_atomic_load(reinterpret_cast<const unsigned long long*>(p), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  return __builtin_bit_cast(c64, v);
}
__device__ __forceinline__ void st_coherent(c64* p, c64 v) {
  __hip_atomic_store(reinterpret_cast<unsigned long long*>(p), __builtin_bit_cast(unsigned long long, v),
                     __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
// KL consecutive complex64 values at byte offset `off` of the buffer `rs`,
// two per 16-byte load, with the same agent-scope coherence as ld_coherent
// (the loads carry the sc1 cache-policy bit that a relaxed agent-scope
// atomic load carries on gfx950: cache policy 16); half the load
// instructions of KL 8-byte atomic loads.
typedef unsigned u32x4_coh __attribute__((ext_vector_type(4)));
template <int KL>
__device__ __forceinline__ void ld_coherent_run(__amdgpu_buffer_rsrc_t rs, unsigned off, c64 (&x)[KL]) {
#pragma unroll
  for (int q = 0; q < KL / 2; ++q) {
    const u32x4_coh v = __builtin_amdgcn_raw_buffer_load_b128(rs, (int)(off + 16u * q), 0, 16);
    x[2 * q] = cmk(__uint_as_float(v.x), __uint_as_float(v.y));
    x[2 * q + 1] = cmk(__uint_as_float(v.z), __uint_as_float(v.w));
  }
}
// a raw buffer resource over `bytes` bytes at p (word 3 as for every gfx9 buffer)
__device__ __forceinline__ __amdgpu_buffer_rsrc_t coherent_rsrc(const void* p, unsigned bytes) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(p), 0, (int)bytes, 0x00020000);
}

// ---------------------------------------------------- complex64/128 VALU --
// AT[a][l][k][j] (transposed per stencil point).  Thread (part, j) sums the
// columns q = (l, k) = part, part + parts, ... of row j, U columns at a time
// with all their loads issued before the multiply-adds (the operator is read
// once per mat-vec, so many loads must be in flight per wave).  Writes
// out[r][a][j] for r0 <= r < min(r0 + NR, nr).  `red` is kCT * NR complex
// of LDS.  With STAGED `in` is instead the site's operand already gathered
// into LDS for the NR right-hand sides r0 .. r0 + NR - 1:
// in[r * NS * nvec + l * nvec + k] = c[r0 + r][nbr(a,l)][k].
// Every thread of the workgroup must call it.  NS is the number of stencil
// points (the 81 of A, or the 9 of the one-hop truncation): AT holds NS
// matrices per site and nbr NS neighbours per site.  COH (complex64 only):
// the operand is read with coherent loads (written by other workgroups of a
// running persistent kernel).
template <typename R, int NR, int U, bool STAGED = false, int NS = kStencil, bool COH = false>
__device__ __forceinline__ void capply_site(const cplx<R>* __restrict__ AT, const int* __restrict__ nbr,
                                            const cplx<R>* __restrict__ in, cplx<R>* __restrict__ out,
                                            int a, int Nc, int nvec, int nr, int r0, cplx<R>* red) {
  const int parts = kCT / nvec;
  const int j = threadIdx.x % nvec, part = threadIdx.x / nvec;
  const int K = NS * nvec;
  cplx<R> acc[NR];
#pragma unroll
  for (int r = 0; r < NR; ++r) acc[r] = cmk((R)0, (R)0);
  if (part < parts) {
    const cplx<R>* Aa = AT + (size_t)a * K * nvec + j;
    const int* nb = nbr + (size_t)a * NS;
    for (int q0 = part; q0 < K; q0 += parts * U) {
      cplx<R> Av[U], xv[U][NR];
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int q = q0 + u * parts;
        Av[u] = cmk((R)0, (R)0);
#pragma unroll
        for (int r = 0; r < NR; ++r) xv[u][r] = cmk((R)0, (R)0);
        if (q < K) {
          Av[u] = Aa[(size_t)q * nvec];
          if constexpr (STAGED) {
#pragma unroll
            for (int r = 0; r < NR; ++r)
              if (r0 + r < nr) xv[u][r] = in[r * K + q];
          } else {
            const int l = q / nvec, k = q - l * nvec;
            const size_t vo = (size_t)nb[l] * nvec + k;
#pragma unroll
            for (int r = 0; r < NR; ++r)
              if (r0 + r < nr) {
                if constexpr (COH)
                  xv[u][r] = ld_coherent(in + (size_t)(r0 + r) * Nc * nvec + vo);
                else
                  xv[u][r] = in[(size_t)(r0 + r) * Nc * nvec + vo];
              }
          }
        }
      }
#pragma unroll
      for (int u = 0; u < U; ++u)
#pragma unroll
        for (int r = 0; r < NR; ++r) cmac(acc[r], Av[u], xv[u][r]);
    }
  }
#pragma unroll
  for (int r = 0; r < NR; ++r) red[r * kCT + threadIdx.x] = acc[r];
  __syncthreads();
  if (threadIdx.x < nvec) {
#pragma unroll
    for (int r = 0; r < NR; ++r) {
      if (r0 + r >= nr) continue;
      cplx<R> s = cmk((R)0, (R)0);
      for (int p = 0; p < parts; ++p) s = s + red[r * kCT + p * nvec + threadIdx.x];
      out[((size_t)(r0 + r) * Nc + a) * nvec + threadIdx.x] = s;
    }
  }
  __syncthreads();  // `red` may be reused by the caller
}

// ------------------------------------------------------ 16-bit MFMA form --
// For one coarse site the 81-point stencil is one real GEMM
//   out[j][n] = sum_kappa Ahat[j][kappa] B[kappa][n]
// with kappa = (part, l, k) over K = 2 * 81 * Nvec:
//   Ahat[j][(0,l,k)] = Re A[a][l][j][k] / s_al,  Ahat[j][(1,l,k)] = Im A[a][l][j][k] / s_al
//   B[(0,l,k)][r]          = rho_al Re c_r[a+dl][k],   B[(1,l,k)][r]          = -rho_al Im c_r[a+dl][k]
//   B[(0,l,k)][nrhs + r]   = rho_al Im c_r[a+dl][k],   B[(1,l,k)][nrhs + r]   =  rho_al Re c_r[a+dl][k]
// so that columns r and nrhs + r give Re and Im of (A c_r)[a][j] / smax_a.
// s_al is the largest |Re|, |Im| entry of the matrix A[a][l] (per-matrix
// scale), smax_a = max_l s_al and rho_al = s_al / smax_a <= 1, which keeps
// both operands within the fp16 range.
//
// Ahat is stored per coarse site and K step as [row m < nvec][kgroup 0..3][4]
// (the 16 K values of one step and row are contiguous), so the A fragment of
// an M tile is one contiguous run that a wave reads with 8-byte lanes, and no
// bytes are stored or read for the rows that pad nvec to a multiple of 16.
// The NW waves take U consecutive K steps at a time, with all their loads
// issued before the MFMAs, and reduce through LDS.
typedef short s16x4 __attribute__((ext_vector_type(4)));
typedef _Float16 h16x4 __attribute__((ext_vector_type(4)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ unsigned short f2bf(float f) {
  return __builtin_bit_cast(unsigned short, (__bf16)f);  // round to nearest even (v_cvt_pk_bf16_f32)
}
__device__ __forceinline__ unsigned short f2h(float f) {
  _Float16 h = (_Float16)f;
  return __builtin_bit_cast(unsigned short, h);
}
template <bool BF16>
__device__ __forceinline__ unsigned short to16(float f) {
  return BF16 ? f2bf(f) : f2h(f);
}

// `red` is NW * MT * NT * 64 f32x4 of LDS.  Writes out[r][a][:] for the
// nrhs right-hand sides of `in` (at most 16 when NT = 2, 8 when NT = 1).
// With STAGED (one right-hand side) `in` is the site's operand gathered
// into LDS: in[l * nvec + k] = c[nbr(a,l)][k].  COH: the operand is read
// with coherent loads (persistent kernels).  K32: gfx950's 16x16x32 MFMA
// (8 K values per lane; the A fragment of one 32-wide step is two
// consecutive 16-wide storage steps, one 16-byte load per lane; needs
// nvec % 8 == 0), else the 16x16x16 form.  NS: stencil points (the 81 of A,
// or the 9 of the one-hop truncation; F, rho and nbr then hold NS per site).
// Every thread of the workgroup (NW * 64 threads) must call it.
typedef short s16x8 __attribute__((ext_vector_type(8)));
typedef _Float16 h16x8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));

template <bool BF16, int MT, int NT, int NW, int U, bool STAGED = false, bool COH = false, bool K32 = false,
          int NS = kStencil>
__device__ __forceinline__ void capply_site_mfma(const unsigned short* __restrict__ F,
                                                 const float* __restrict__ rho,
                                                 const float* __restrict__ smax, const int* __restrict__ nbr,
                                                 const c64* __restrict__ in, c64* __restrict__ out, int a,
                                                 int Nc, int nvec, int nrhs, int ksteps, f32x4* red) {
  using frag = std::conditional_t<K32, s16x8, s16x4>;
  static_assert(!STAGED || NT == 1, "the LDS-staged operand serves one right-hand side");
  constexpr int KL = K32 ? 8 : 4;  // K values per lane and step
  constexpr int KS = 4 * KL;       // K values per step
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int ktot = 2 * NS * nvec;
  const int kn = NS * nvec;
  const int r16 = lane & 15, kg = lane >> 4;
  const int nsteps = K32 ? (ksteps + 1) / 2 : ksteps;
  f32x4 acc[MT][NT];
#pragma unroll
  for (int i = 0; i < MT; ++i)
#pragma unroll
    for (int j = 0; j < NT; ++j) acc[i][j] = f32x4{0.f, 0.f, 0.f, 0.f};
  const unsigned short* Fa = F + (size_t)a * ksteps * nvec * 16;
  const int* nb = nbr + (size_t)a * NS;
  const float* rh = rho + (size_t)a * NS;
  // COH: the operand of all nrhs right-hand sides as one buffer resource
  // (offsets stay below 2 GiB: nrhs <= 16 columns of Nc * nvec values)
  const __amdgpu_buffer_rsrc_t rs = coherent_rsrc(in, COH ? (unsigned)((size_t)nrhs * Nc * nvec * sizeof(c64)) : 0u);
  // storage step and k group of this lane's A fragment at step S
  const int sub = K32 ? (kg >> 1) : 0, kgs = K32 ? 2 * (kg & 1) : kg;
  // the right-hand side of this lane's B columns: with NT = 2 (9-16 RHS)
  // lane r16 takes RHS r16, its Re column in tile 0 and its Im column in
  // tile 1; with NT = 1 (1-8 RHS) columns 0 .. nrhs-1 are the Re columns and
  // nrhs .. 2 nrhs-1 the Im columns
  const int rr = NT == 2 ? r16 : (r16 < nrhs ? r16 : r16 - nrhs);
  const bool cok = NT == 2 ? r16 < nrhs : r16 < 2 * nrhs;
  const bool im1 = NT == 1 && r16 >= nrhs;
  for (int s0 = wave * U; s0 < nsteps; s0 += NW * U) {
    frag af[U][MT];
    frag bf[U][NT];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int s = (K32 ? 2 * (s0 + u) : s0 + u) + sub;
#pragma unroll
      for (int mt = 0; mt < MT; ++mt) {
        const int m = mt * 16 + r16;
        af[u][mt] = (s < ksteps && m < nvec)
                        ? *reinterpret_cast<const frag*>(Fa + (((size_t)s * nvec + m) * 4 + kgs) * 4)
                        : frag{};
      }
    }
    if constexpr (STAGED) {
      // one right-hand side, operand in LDS: each step's run converted as read
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int k0 = KS * (s0 + u) + KL * kg;
        bf[u][0] = frag{};
        if (cok && s0 + u < nsteps && k0 < ktot) {
          const int part = k0 / kn;
          const int rem = k0 - part * kn;
          const float r = rh[rem / nvec];
          frag b;
#pragma unroll
          for (int i = 0; i < KL; ++i) {
            const c64 x = in[rem + i];
            b[i] = (short)to16<BF16>(r * (im1 ? (part == 0 ? x.im : x.re) : (part == 0 ? x.re : -x.im)));
          }
          bf[u][0] = b;
        }
      }
    } else {
      // the operand runs of all U steps are loaded before any is converted
      // (addresses clamped to valid ones, invalid lanes zeroed afterwards), one
      // run per lane and step: its right-hand side feeds both of its columns
      c64 xs[U][KL];
      float rsc[U];
      int prt[U];
      bool okv[U];
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int k0 = KS * (s0 + u) + KL * kg;
        const bool ok = cok && s0 + u < nsteps && k0 < ktot;
        const int kk = ok ? k0 : 0;
        const int part = kk / kn;
        const int rem = kk - part * kn;
        const int l = rem / nvec, k = rem - l * nvec;
        okv[u] = ok;
        prt[u] = part;
        rsc[u] = rh[l];
        const size_t co = (size_t)(ok ? rr : 0) * Nc * nvec + (size_t)nb[l] * nvec + k;
        if constexpr (COH) {
          ld_coherent_run<KL>(rs, (unsigned)(co * sizeof(c64)), xs[u]);
        } else {
#pragma unroll
          for (int i = 0; i < KL; ++i) xs[u][i] = in[co + i];
        }
      }
#pragma unroll
      for (int u = 0; u < U; ++u)
#pragma unroll
        for (int nt = 0; nt < NT; ++nt) {
          const bool imcol = NT == 2 ? nt == 1 : im1;
          frag b;
#pragma unroll
          for (int i = 0; i < KL; ++i) {
            const c64 x = xs[u][i];
            // Re columns: part 0 -> Re c, part 1 -> -Im c
            // Im columns: part 0 -> Im c, part 1 ->  Re c
            const float v = rsc[u] * (imcol ? (prt[u] == 0 ? x.im : x.re) : (prt[u] == 0 ? x.re : -x.im));
            b[i] = okv[u] ? (short)to16<BF16>(v) : (short)0;
          }
          bf[u][nt] = b;
        }
    }
#pragma unroll
    for (int u = 0; u < U; ++u)
#pragma unroll
      for (int mt = 0; mt < MT; ++mt)
#pragma unroll
        for (int nt = 0; nt < NT; ++nt) {
          if constexpr (K32) {
            if constexpr (BF16)
              acc[mt][nt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8, af[u][mt]),
                                                                    __builtin_bit_cast(bf16x8, bf[u][nt]),
                                                                    acc[mt][nt], 0, 0, 0);
            else
              acc[mt][nt] = __builtin_amdgcn_mfma_f32_16x16x32_f16(__builtin_bit_cast(h16x8, af[u][mt]),
                                                                   __builtin_bit_cast(h16x8, bf[u][nt]),
                                                                   acc[mt][nt], 0, 0, 0);
          } else {
            if constexpr (BF16)
              acc[mt][nt] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(af[u][mt], bf[u][nt], acc[mt][nt], 0, 0, 0);
            else
              acc[mt][nt] = __builtin_amdgcn_mfma_f32_16x16x16f16(__builtin_bit_cast(h16x4, af[u][mt]),
                                                                  __builtin_bit_cast(h16x4, bf[u][nt]),
                                                                  acc[mt][nt], 0, 0, 0);
          }
        }
  }
#pragma unroll
  for (int mt = 0; mt < MT; ++mt)
#pragma unroll
    for (int nt = 0; nt < NT; ++nt) red[(wave * MT * NT + mt * NT + nt) * 64 + lane] = acc[mt][nt];
  __syncthreads();
  const float sm = smax[a];
  for (int q = threadIdx.x; q < MT * NT * 64; q += NW * 64) {
    const int tile = q >> 6, ln = q & 63;
    const int mt = tile / NT, nt = tile - mt * NT;
    f32x4 v = red[tile * 64 + ln];
#pragma unroll
    for (int w = 1; w < NW; ++w) v += red[(w * MT * NT + tile) * 64 + ln];
    // lane ln holds D[m = 4 (ln / 16) + i][n = ln % 16]; columns as loaded
    const int n = ln & 15;
    if (NT == 2 ? n >= nrhs : n >= 2 * nrhs) continue;
    const bool imcol = NT == 2 ? nt == 1 : n >= nrhs;
    const int rr = NT == 2 ? n : (imcol ? n - nrhs : n);
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int m = mt * 16 + 4 * (ln >> 4) + i;
      if (m >= nvec) continue;
      float* o = reinterpret_cast<float*>(out + ((size_t)rr * Nc + a) * nvec + m);
      o[imcol ? 1 : 0] = sm * v[i];
    }
  }
  __syncthreads();  // `red` may be reused by the caller
}

// ------------------------------- complex64 / complex128 on the MFMA --
// The real GEMM of the 16-bit form (Re and Im columns per right-hand side,
// K = (part, l, k)), on the complex operator in the VALU form's storage
// AT[a][l][k][j] and gfx950's FP32 16x16x4 MFMA (complex64) or FP64 16x16x4
// MFMA (complex128): no scales and no rounding of either operand,
// accumulation in the storage precision as in the VALU form.  The complex
// columns q = (l, k) of the site go in groups of 16: MFMA step i of a group
// takes column q = q0 + 4 kg + i in lane group kg, where lane (m, kg)
// supplies A[a][l][mt * 16 + m][k] (Re for part 0, Im for part 1) and lane
// (kg, n) its right-hand side's operand value c[nbr(a,l)][k]; a lane's four
// operand values are then one contiguous run (nvec % 4 == 0, so a run never
// crosses a stencil point), and its A values four rows of AT.  Columns of
// the N tiles as in capply_site_mfma (NT = 1: nrhs <= 8; NT = 2: nrhs <=
// 16).  The FP32 form holds D[4 (lane / 16) + i][lane % 16] in its i-th
// accumulator value, the FP64 form D[lane / 16 + 4 i][lane % 16].  `red` is
// NW * MT * NT * 64 accumulators of LDS.  The operand is read through the
// caches (a persistent caller acquires first).  Every thread of the
// workgroup (NW * 64 threads) must call it.
typedef double f64x4 __attribute__((ext_vector_type(4)));
template <typename R>
using macc_t = std::conditional_t<sizeof(R) == 4, f32x4, f64x4>;

template <typename R>
__device__ __forceinline__ macc_t<R> mfma_4(R a, R b, macc_t<R> c) {
  if constexpr (sizeof(R) == 4)
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  else
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

template <typename R, int MT, int NT, int NW, int U, int NS = kStencil>
__device__ __forceinline__ void capply_site_cmfma(const cplx<R>* __restrict__ AT, const int* __restrict__ nbr,
                                                  const cplx<R>* __restrict__ in, cplx<R>* __restrict__ out, int a,
                                                  int Nc, int nvec, int nrhs, macc_t<R>* red) {
  using acc_t = macc_t<R>;
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int r16 = lane & 15, kg = lane >> 4;
  const int K = NS * nvec;
  const int ngroups = (K + 15) / 16;
  acc_t acc[MT][NT];
#pragma unroll
  for (int i = 0; i < MT; ++i)
#pragma unroll
    for (int j = 0; j < NT; ++j) acc[i][j] = acc_t{0, 0, 0, 0};
  const cplx<R>* Aa = AT + (size_t)a * K * nvec;
  const int* nb = nbr + (size_t)a * NS;
  const int rr = NT == 2 ? r16 : (r16 < nrhs ? r16 : r16 - nrhs);
  const bool cok = NT == 2 ? r16 < nrhs : r16 < 2 * nrhs;
  const bool im1 = NT == 1 && r16 >= nrhs;
  const size_t rbase = (size_t)(cok ? rr : 0) * Nc * nvec;
  for (int g0 = wave * U; g0 < ngroups; g0 += NW * U) {
    cplx<R> av[U][4][MT];
    cplx<R> xv[U][4];
    bool okv[U];
    // all loads of the U groups before any MFMA (addresses clamped to valid
    // ones; lanes past the end of K contribute zeros)
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int q = 16 * (g0 + u) + 4 * kg;
      const bool okq = g0 + u < ngroups && q < K;
      const int qc = okq ? q : 0;
      okv[u] = okq;
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int mt = 0; mt < MT; ++mt) {
          const int m = mt * 16 + r16;
          av[u][i][mt] = Aa[(size_t)(qc + i) * nvec + (m < nvec ? m : 0)];
        }
      const int l = qc / nvec, k = qc - l * nvec;
      const cplx<R>* xp = in + rbase + (size_t)nb[l] * nvec + k;
#pragma unroll
      for (int i = 0; i < 4; ++i) xv[u][i] = xp[i];
    }
#pragma unroll
    for (int u = 0; u < U; ++u)
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        // Re columns: part 0 -> Re c, part 1 -> -Im c; Im columns: part 0 ->
        // Im c, part 1 -> Re c (invalid lanes: zero operand)
        const cplx<R> x = okv[u] && cok ? xv[u][i] : cmk((R)0, (R)0);
        R b0[NT], b1[NT];
#pragma unroll
        for (int nt = 0; nt < NT; ++nt) {
          const bool imcol = NT == 2 ? nt == 1 : im1;
          b0[nt] = imcol ? x.im : x.re;
          b1[nt] = imcol ? x.re : -x.im;
        }
#pragma unroll
        for (int mt = 0; mt < MT; ++mt) {
          const cplx<R> A = av[u][i][mt];
#pragma unroll
          for (int nt = 0; nt < NT; ++nt) acc[mt][nt] = mfma_4<R>(A.re, b0[nt], acc[mt][nt]);
#pragma unroll
          for (int nt = 0; nt < NT; ++nt) acc[mt][nt] = mfma_4<R>(A.im, b1[nt], acc[mt][nt]);
        }
      }
  }
#pragma unroll
  for (int mt = 0; mt < MT; ++mt)
#pragma unroll
    for (int nt = 0; nt < NT; ++nt) red[(wave * MT * NT + mt * NT + nt) * 64 + lane] = acc[mt][nt];
  __syncthreads();
  for (int q = threadIdx.x; q < MT * NT * 64; q += NW * 64) {
    const int tile = q >> 6, ln = q & 63;
    const int mt = tile / NT, nt = tile - mt * NT;
    acc_t v = red[tile * 64 + ln];
#pragma unroll
    for (int w = 1; w < NW; ++w) v += red[(w * MT * NT + tile) * 64 + ln];
    const int n = ln & 15;
    if (NT == 2 ? n >= nrhs : n >= 2 * nrhs) continue;
    const bool imcol = NT == 2 ? nt == 1 : n >= nrhs;
    const int rn = NT == 2 ? n : (imcol ? n - nrhs : n);
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int m = mt * 16 + (sizeof(R) == 4 ? 4 * (ln >> 4) + i : (ln >> 4) + 4 * i);
      if (m >= nvec) continue;
      R* o = reinterpret_cast<R*>(out + ((size_t)rn * Nc + a) * nvec + m);
      o[imcol ? 1 : 0] = v[i];
    }
  }
  __syncthreads();  // `red` may be reused by the caller
}

}  // namespace hdk
