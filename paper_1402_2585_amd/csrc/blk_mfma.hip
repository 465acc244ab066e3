// Block project and promote (Sec. V.A: the restriction P^+ and prolongation
// P between the fine grid and the coarse grid) for several right-hand sides
// with the subspace stored in 16 bits.  Per block a both are dense complex
// contractions, Nvec x nb times nb x nrhs (project) and nb x Nvec times
// Nvec x nrhs (promote): with 16 right-hand sides a block holds about 20
// FLOP per byte, more than the FP32 vector units sustain per byte of HBM, so
// they run on gfx950's 16x16x32 bf16 MFMA with FP32 accumulation.
//
// The subspace values are bf16 already.  The complex64 operand of each (the
// fine field, or the coarse vector) enters as three bf16 terms
// x = hi + mid + lo with |x - hi - mid - lo| <= 2^-24 |x|: every product is
// exact in FP32 and equal to the one the FP32 kernels form with x, so the
// results differ from theirs only in the order of the sums.
#include "coarse_dev.h"

namespace hdk {

namespace {

typedef unsigned w32x4 __attribute__((ext_vector_type(4)));

// (re, im) as three packed bf16 pairs: hi = bf16(x), mid = bf16(x - hi),
// lo = bf16(x - hi - mid).  Each difference is exact in FP32 (the operands
// lie within a factor of two of each other), so x = hi + mid + r2 exactly
// and |r2 - lo| <= 2^-8 |r2| <= 2^-24 |x|.
struct Split3 {
  unsigned w[3];  // hi, mid, lo
};
__device__ __forceinline__ Split3 split3(float re, float im) {
  Split3 o;
  o.w[0] = f32x2_to_bf16x2(re, im);
  const float r1re = re - __uint_as_float(o.w[0] << 16), r1im = im - __uint_as_float(o.w[0] & 0xffff0000u);
  o.w[1] = f32x2_to_bf16x2(r1re, r1im);
  const float r2re = r1re - __uint_as_float(o.w[1] << 16), r2im = r1im - __uint_as_float(o.w[1] & 0xffff0000u);
  o.w[2] = f32x2_to_bf16x2(r2re, r2im);
  return o;
}

// one bf16 pair (a, b) -> (-b, a): the row of Im(conj(p) q) against (Re q, Im q)
__device__ __forceinline__ unsigned rot_neg(unsigned w) {
  return ((w >> 16) ^ 0x8000u) | (w << 16);
}

__device__ __forceinline__ f32x4 mfma(w32x4 a, w32x4 b, f32x4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8, a), __builtin_bit_cast(bf16x8, b), c, 0,
                                                 0, 0);
}

// out[r*sr + a*sa + k*sk] = sum_i conj(P[a][k][i]) Q_r(site(a, i)) for the
// right-hand sides r0 .. r0 + 15 (r < nr) of this workgroup (blockIdx.y).
// One workgroup per block a (blockIdx.x); its NW waves split the nb entries
// in K steps of 16 (U consecutive steps per wave at a time, their loads
// issued before the MFMAs) and reduce through LDS (`red`, dynamic:
// NW * MT * 2 * 64 f32x4).  Real GEMM: rows (k, Re) carry the K pairs
// (Re P, Im P), rows (k, Im) (-Im P, Re P), columns r (Re Q, Im Q) per
// entry i.  Lane layout of the 16x16x32 form: A row lane % 16 and B column
// lane % 16, each with K values 8 (lane / 16) .. + 7 (the entries
// i0 + 4 (lane / 16) .. + 3); D rows 4 (lane / 16) .. + 3, column lane % 16.
// Needs nb % 4 == 0 and 12 Ls % 4 == 0 (four entries of a lane stay in one
// site column), 16-byte aligned rows of P and Q; MT = ceil(nvec / 16).
template <int NW, int U, int MT>
__global__ void __launch_bounds__(NW * 64)
k_project_mfma(const unsigned* __restrict__ P, const c64* __restrict__ Q, size_t fstride,
               const int* __restrict__ site_of, int nsb, int col, int nb, int nvec, int nr,
               c64* __restrict__ out, size_t sr, size_t sa, size_t sk) {
  extern __shared__ f32x4 red[];
  const int a = blockIdx.x, r0 = blockIdx.y * 16;
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int r16 = lane & 15, kg = lane >> 4;
  const int rr = r0 + r16;
  const bool rok = rr < nr;
  const unsigned* Pa = P + (size_t)a * nvec * nb;
  const c64* Qr = Q + (size_t)(rok ? rr : 0) * fstride;
  const int* so = site_of + (size_t)a * nsb;
  f32x4 acc[MT][2];
#pragma unroll
  for (int m = 0; m < MT; ++m) acc[m][0] = acc[m][1] = f32x4{0.f, 0.f, 0.f, 0.f};
  const int nsteps = (nb + 15) / 16;
  for (int s0 = wave * U; s0 < nsteps; s0 += NW * U) {
    w32x4 pa[U][MT];
    f32x4 qa[U][2];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int i = (s0 + u) * 16 + 4 * kg;
      const bool iok = s0 + u < nsteps && i < nb;
#pragma unroll
      for (int m = 0; m < MT; ++m) {
        const int k = m * 16 + r16;
        pa[u][m] = (iok && k < nvec) ? *reinterpret_cast<const w32x4*>(Pa + (size_t)k * nb + i) : w32x4{0u, 0u, 0u, 0u};
      }
      if (iok && rok) {
        const int j = i / col, q = i - j * col;
        const f32x4* src = reinterpret_cast<const f32x4*>(Qr + (size_t)so[j] * col + q);
        qa[u][0] = src[0];
        qa[u][1] = src[1];
      } else {
        qa[u][0] = qa[u][1] = f32x4{0.f, 0.f, 0.f, 0.f};
      }
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const Split3 e0 = split3(qa[u][0][0], qa[u][0][1]), e1 = split3(qa[u][0][2], qa[u][0][3]);
      const Split3 e2 = split3(qa[u][1][0], qa[u][1][1]), e3 = split3(qa[u][1][2], qa[u][1][3]);
      w32x4 b[3];
#pragma unroll
      for (int t = 0; t < 3; ++t) b[t] = w32x4{e0.w[t], e1.w[t], e2.w[t], e3.w[t]};
#pragma unroll
      for (int m = 0; m < MT; ++m) {
        const w32x4 are = pa[u][m];
        const w32x4 aim = {rot_neg(are[0]), rot_neg(are[1]), rot_neg(are[2]), rot_neg(are[3])};
#pragma unroll
        for (int t = 0; t < 3; ++t) {
          acc[m][0] = mfma(are, b[t], acc[m][0]);
          acc[m][1] = mfma(aim, b[t], acc[m][1]);
        }
      }
    }
  }
#pragma unroll
  for (int m = 0; m < MT; ++m) {
    red[((wave * MT + m) * 2 + 0) * 64 + lane] = acc[m][0];
    red[((wave * MT + m) * 2 + 1) * 64 + lane] = acc[m][1];
  }
  __syncthreads();
  for (int q = threadIdx.x; q < MT * 64; q += NW * 64) {
    const int m = q >> 6, ln = q & 63;
    f32x4 vre = red[(m * 2 + 0) * 64 + ln], vim = red[(m * 2 + 1) * 64 + ln];
    for (int w = 1; w < NW; ++w) {
      vre += red[((w * MT + m) * 2 + 0) * 64 + ln];
      vim += red[((w * MT + m) * 2 + 1) * 64 + ln];
    }
    const int r = r0 + (ln & 15);
    if (r >= nr) continue;
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const int k = m * 16 + 4 * (ln >> 4) + e;
      if (k < nvec) out[r * sr + a * sa + k * sk] = cmk(vre[e], vim[e]);
    }
  }
}

// fine_out[r][site(a, i)] = base + sign * sum_k P[a][k][i] c[r][a][k] for
// the right-hand sides r0 .. r0 + 8 NT - 1 (r < nr) of this workgroup
// (blockIdx.z), block a = blockIdx.y.  Real GEMM: rows i carry the K pairs
// (Re P[k][i], Im P[k][i]); column (r, Re) takes (Re c, -Im c) and column
// (r, Im) (Im c, Re c) for each k.  The B fragments (KS = ceil(nvec / 16)
// K steps, three bf16 terms of c) are built once per wave; each wave then
// takes MPW row tiles of 16 entries, U adjacent tiles at a time.  The two
// lanes of a column pair swap halves so that each stores whole complex
// values (two consecutive entries of one site column, 16 bytes).
template <int NW, int U, int MPW, int KS, int NT>
__global__ void __launch_bounds__(NW * 64)
k_promote_mfma(const unsigned* __restrict__ P, const c64* __restrict__ c, int Nc, int nvec, int nb, int nsb, int col,
               const int* __restrict__ site_of, c64* out, const c64* base, float sign, size_t fstride, int nr) {
  const int a = blockIdx.y, r0 = blockIdx.z * 8 * NT;
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int r16 = lane & 15, kg = lane >> 4;
  w32x4 bfr[NT][KS][3];
#pragma unroll
  for (int nt = 0; nt < NT; ++nt) {
    const int r = r0 + nt * 8 + (r16 >> 1);
    const bool imcol = r16 & 1;
#pragma unroll
    for (int ks = 0; ks < KS; ++ks) {
      Split3 sp[4];
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int k = ks * 16 + 4 * kg + j;
        c64 v = cmk(0.f, 0.f);
        if (r < nr && k < nvec) v = c[((size_t)r * Nc + a) * nvec + k];
        sp[j] = split3(imcol ? v.im : v.re, imcol ? v.re : -v.im);
      }
#pragma unroll
      for (int t = 0; t < 3; ++t) bfr[nt][ks][t] = w32x4{sp[0].w[t], sp[1].w[t], sp[2].w[t], sp[3].w[t]};
    }
  }
  const unsigned* Pa = P + (size_t)a * nvec * nb;
  const int* so = site_of + (size_t)a * nsb;
  const int tile0 = (blockIdx.x * NW + wave) * MPW;
  for (int u0 = 0; u0 < MPW; u0 += U) {
    if ((tile0 + u0) * 16 >= nb) break;  // wave-uniform
    w32x4 afr[U][KS];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int i = (tile0 + u0 + u) * 16 + r16;
#pragma unroll
      for (int ks = 0; ks < KS; ++ks) {
        unsigned wv[4];
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          const int k = ks * 16 + 4 * kg + j;
          wv[j] = (u0 + u < MPW && i < nb && k < nvec) ? Pa[(size_t)k * nb + i] : 0u;
        }
        afr[u][ks] = w32x4{wv[0], wv[1], wv[2], wv[3]};
      }
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      f32x4 acc[NT];
#pragma unroll
      for (int nt = 0; nt < NT; ++nt) {
        acc[nt] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int ks = 0; ks < KS; ++ks)
#pragma unroll
          for (int t = 0; t < 3; ++t) acc[nt] = mfma(afr[u][ks], bfr[nt][ks][t], acc[nt]);
      }
      // lane holds entries i0 + 4 kg + 0..3 of column r16 = (r, Re | Im)
      const int i4 = (tile0 + u0 + u) * 16 + 4 * kg;
      const bool imcol = r16 & 1;
#pragma unroll
      for (int nt = 0; nt < NT; ++nt) {
        f32x4 oth;
#pragma unroll
        for (int e = 0; e < 4; ++e) oth[e] = __shfl_xor(acc[nt][e], 1);
        const int r = r0 + nt * 8 + (r16 >> 1);
        if (u0 + u >= MPW || i4 >= nb || r >= nr) continue;
        // the Re lane stores entries 0, 1 of its four, the Im lane 2, 3
        const int e0 = imcol ? 2 : 0;
        const float re0 = imcol ? oth[2] : acc[nt][0], im0 = imcol ? acc[nt][2] : oth[0];
        const float re1 = imcol ? oth[3] : acc[nt][1], im1 = imcol ? acc[nt][3] : oth[1];
        const int i = i4 + e0;
        const int jj = i / col, q = i - jj * col;
        const size_t addr = (size_t)r * fstride + (size_t)so[jj] * col + q;
        f32x4 o = {sign * re0, sign * im0, sign * re1, sign * im1};
        if (base) o += *reinterpret_cast<const f32x4*>(base + addr);
        *reinterpret_cast<f32x4*>(out + addr) = o;
      }
    }
  }
}

bool aligned16(const void* p) { return (reinterpret_cast<uintptr_t>(p) & 15u) == 0; }

}  // namespace

bool blk_mfma_applies(hdcg* h, const void* P, const void* f, size_t fstride, int sd) {
  const int col = 12 * h->op->g.Ls;
  const size_t nb = (size_t)h->nsb * col;
  return sd == 0 && h->nvec <= 64 && col % 4 == 0 && nb % 4 == 0 && nb < (1u << 30) && aligned16(P) &&
         aligned16(f) && (fstride * sizeof(c64)) % 16 == 0;
}

int blk_project_mfma(hdcg* h, const bf16c* P, const c64* fine, size_t fstride, int nr, c64* out, size_t sr,
                     size_t sa, size_t sk, hipStream_t st) {
  if (!blk_mfma_applies(h, P, fine, fstride, 0)) return fail(DWF_ERR_ARG, "project (MFMA): layout not supported");
  constexpr int NW = 4, U = 2;
  const int col = 12 * h->op->g.Ls;
  const int nb = h->nsb * col;
  const int mt = (h->nvec + 15) / 16;
  const dim3 grid(h->Nc, (nr + 15) / 16);
  const size_t lds = (size_t)NW * mt * 2 * 64 * sizeof(f32x4);
  const unsigned* Pw = reinterpret_cast<const unsigned*>(P);
#define HDCG_PROJ_MFMA(M)                                                                                      \
  hipLaunchKernelGGL((k_project_mfma<NW, U, M>), grid, dim3(NW * 64), lds, st, Pw, fine, fstride,              \
                     h->site_of.as<int>(), h->nsb, col, nb, h->nvec, nr, out, sr, sa, sk)
  switch (mt) {
    case 1: HDCG_PROJ_MFMA(1); break;
    case 2: HDCG_PROJ_MFMA(2); break;
    case 3: HDCG_PROJ_MFMA(3); break;
    default: HDCG_PROJ_MFMA(4); break;
  }
#undef HDCG_PROJ_MFMA
  HDCG_HIP(hipGetLastError());
  return DWF_OK;
}

int blk_promote_mfma(hdcg* h, const bf16c* P, const c64* c, int nr, c64* out, const c64* base, double sign,
                     size_t fstride, hipStream_t st) {
  if (!blk_mfma_applies(h, P, out, fstride, 0) || (base && !aligned16(base)))
    return fail(DWF_ERR_ARG, "promote (MFMA): layout not supported");
  constexpr int NW = 4, U = 2, MPW = 8;
  const int col = 12 * h->op->g.Ls;
  const int nb = h->nsb * col;
  const int ks = (h->nvec + 15) / 16;
  const int tiles = (nb + 15) / 16;
  const int per_wg = NW * MPW;
  const unsigned* Pw = reinterpret_cast<const unsigned*>(P);
  const float sg = (float)sign;
  // eight right-hand sides per N tile, two N tiles per launch when more than 8
  const int nt = nr > 8 ? 2 : 1;
  const dim3 grid((tiles + per_wg - 1) / per_wg, h->Nc, (nr + 8 * nt - 1) / (8 * nt));
#define HDCG_PROM_MFMA(K, N)                                                                                   \
  hipLaunchKernelGGL((k_promote_mfma<NW, U, MPW, K, N>), grid, dim3(NW * 64), 0, st, Pw, c, h->Nc, h->nvec, nb, \
                     h->nsb, col, h->site_of.as<int>(), out, base, sg, fstride, nr)
  if (nt == 2) {
    switch (ks) {
      case 1: HDCG_PROM_MFMA(1, 2); break;
      case 2: HDCG_PROM_MFMA(2, 2); break;
      case 3: HDCG_PROM_MFMA(3, 2); break;
      default: HDCG_PROM_MFMA(4, 2); break;
    }
  } else {
    switch (ks) {
      case 1: HDCG_PROM_MFMA(1, 1); break;
      case 2: HDCG_PROM_MFMA(2, 1); break;
      case 3: HDCG_PROM_MFMA(3, 1); break;
      default: HDCG_PROM_MFMA(4, 1); break;
    }
  }
#undef HDCG_PROM_MFMA
  HDCG_HIP(hipGetLastError());
  return DWF_OK;
}

}  // namespace hdk
