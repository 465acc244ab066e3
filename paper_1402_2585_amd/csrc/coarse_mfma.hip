// Little Dirac operator mat-vec on MFMA with 16-bit matrix storage (bf16
// or fp16) and FP32 accumulation: per-matrix scales, fragment-ordered
// storage and the standalone mat-vec launch.  The per-site GEMM itself
// (operand layout, scaling) is capply_site_mfma in coarse_dev.h.
#include "coarse_dev.h"

namespace hdk {

namespace {

// per-matrix scales: s[a][l] = max |Re|, |Im| over A[a][l]
__global__ void k_scales(const c128* __restrict__ A, float* __restrict__ s, int nvec2) {
  const int al = blockIdx.x;
  const c128* M = A + (size_t)al * nvec2;
  float m = 0.f;
  for (int e = threadIdx.x; e < nvec2; e += blockDim.x) {
    const c128 v = M[e];
    m = fmaxf(m, fmaxf(fabsf((float)v.re), fabsf((float)v.im)));
  }
  __shared__ float red[256];
  red[threadIdx.x] = m;
  __syncthreads();
  for (int w = blockDim.x / 2; w > 0; w >>= 1) {
    if (threadIdx.x < w) red[threadIdx.x] = fmaxf(red[threadIdx.x], red[threadIdx.x + w]);
    __syncthreads();
  }
  if (threadIdx.x == 0) s[al] = red[0];
}

// rho[a][l] = s_al / smax_a (in place), smax[a]
__global__ void k_rho(float* __restrict__ s, float* __restrict__ smax, int Nc) {
  const int a = blockIdx.x * blockDim.x + threadIdx.x;
  if (a >= Nc) return;
  float m = 0.f;
  for (int l = 0; l < kStencil; ++l) m = fmaxf(m, s[a * kStencil + l]);
  smax[a] = m;
  for (int l = 0; l < kStencil; ++l) {
    const float v = s[a * kStencil + l];
    s[a * kStencil + l] = m > 0.f ? v / m : 0.f;
  }
}

template <bool BF16>
__global__ void k_frag(const c128* __restrict__ A, const float* __restrict__ rho,
                       const float* __restrict__ smax, unsigned short* __restrict__ F, int Nc,
                       int nvec, int ksteps) {
  const size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x;  // one (a, s, m, kg)
  const size_t total = (size_t)Nc * ksteps * nvec * 4;
  if (e >= total) return;
  const int kg = (int)(e % 4);
  const int m = (int)((e / 4) % nvec);
  const size_t as = e / (4 * (size_t)nvec);
  const int s = (int)(as % ksteps);
  const int a = (int)(as / ksteps);
  const int ktot = 2 * kStencil * nvec;
  unsigned short v4[4];
  for (int i = 0; i < 4; ++i) {
    const int kap = 16 * s + 4 * kg + i;
    float v = 0.f;
    if (kap < ktot) {
      const int part = kap / (kStencil * nvec);
      const int rem = kap - part * kStencil * nvec;
      const int l = rem / nvec, k = rem - (rem / nvec) * nvec;
      const float sal = rho[a * kStencil + l] * smax[a];
      const c128 x = A[(((size_t)a * kStencil + l) * nvec + m) * nvec + k];
      v = sal > 0.f ? (float)((part == 0 ? x.re : x.im) / sal) : 0.f;
    }
    v4[i] = to16<BF16>(v);
  }
  unsigned short* o = F + e * 4;
  for (int i = 0; i < 4; ++i) o[i] = v4[i];
}

template <bool BF16, int MT, int NT, int NW, int U>
__global__ void __launch_bounds__(NW * 64)
k_capply_mfma(const unsigned short* __restrict__ F, const float* __restrict__ rho,
              const float* __restrict__ smax, const int* __restrict__ nbr, const c64* __restrict__ in,
              c64* __restrict__ out, int Nc, int nvec, int nrhs, int ksteps) {
  __shared__ f32x4 red[NW * MT * NT * 64];
  capply_site_mfma<BF16, MT, NT, NW, U>(F, rho, smax, nbr, in, out, blockIdx.x, Nc, nvec, nrhs, ksteps, red);
}

// One right-hand side: the site's operand at its 81 neighbours is gathered
// into LDS first (one coalesced pass).
template <bool BF16, int MT>
__global__ void __launch_bounds__(8 * 64)
k_capply_mfma_staged(const unsigned short* __restrict__ F, const float* __restrict__ rho,
                     const float* __restrict__ smax, const int* __restrict__ nbr, const c64* __restrict__ in,
                     c64* __restrict__ out, int Nc, int nvec, int ksteps) {
  __shared__ f32x4 red[8 * MT * 64];
  __shared__ c64 xin[kStencil * 64];
  const int a = blockIdx.x;
  const int* nb = nbr + (size_t)a * kStencil;
  for (int e = threadIdx.x; e < kStencil * nvec; e += 8 * 64) {
    const int l = e / nvec;
    xin[e] = in[(size_t)nb[l] * nvec + (e - l * nvec)];
  }
  __syncthreads();
  capply_site_mfma<BF16, MT, 1, 8, 4, true>(F, rho, smax, nbr, xin, out, a, Nc, nvec, 1, ksteps, red);
}

// 8 waves per workgroup while their LDS reduction buffers fit in 48 KiB
template <bool BF16, int MT, int NT>
void launch_tile(const unsigned short* F, const float* rho, const float* smax, const int* nbr,
                 const c64* in, c64* out, int Nc, int nvec, int n, int ksteps, hipStream_t st) {
  constexpr int U = 4;
  if constexpr (MT * NT <= 6)
    hipLaunchKernelGGL((k_capply_mfma<BF16, MT, NT, 8, U>), dim3(Nc), dim3(8 * 64), 0, st, F, rho, smax,
                       nbr, in, out, Nc, nvec, n, ksteps);
  else
    hipLaunchKernelGGL((k_capply_mfma<BF16, MT, NT, 4, U>), dim3(Nc), dim3(4 * 64), 0, st, F, rho, smax,
                       nbr, in, out, Nc, nvec, n, ksteps);
}

template <bool BF16, int MT>
int launch_mt(hdcg* h, const unsigned short* F, const c64* in, c64* out, int nr, int ksteps,
              hipStream_t st) {
  const float* rho = h->mf_rho.as<float>();
  const float* smax = h->mf_smax.as<float>();
  for (int r0 = 0; r0 < nr; r0 += 16) {
    const int n = nr - r0 < 16 ? nr - r0 : 16;
    const c64* i0 = in + (size_t)r0 * h->Nc * h->nvec;
    c64* o0 = out + (size_t)r0 * h->Nc * h->nvec;
    if (n == 1)
      hipLaunchKernelGGL((k_capply_mfma_staged<BF16, MT>), dim3(h->Nc), dim3(8 * 64), 0, st, F, rho, smax,
                         h->nbr.as<int>(), i0, o0, h->Nc, h->nvec, ksteps);
    else if (2 * n <= 16)
      launch_tile<BF16, MT, 1>(F, rho, smax, h->nbr.as<int>(), i0, o0, h->Nc, h->nvec, n, ksteps, st);
    else
      launch_tile<BF16, MT, 2>(F, rho, smax, h->nbr.as<int>(), i0, o0, h->Nc, h->nvec, n, ksteps, st);
    HDCG_HIP(hipGetLastError());
  }
  return DWF_OK;
}

}  // namespace

int crs_build_mfma(hdcg* h, int prec, hipStream_t st) {
  const int nv = h->nvec;
  if (nv % 4 != 0 || nv > 64)
    return fail(DWF_ERR_ARG, "16-bit coarse storage needs nvec a multiple of 4 and <= 64");
  const int ksteps = (2 * kStencil * nv + 15) / 16;
  if (h->mf_smax.bytes == 0) {
    HDCG_TRY(h->mf_rho.ensure(sizeof(float) * h->Nc * kStencil));
    HDCG_TRY(h->mf_smax.ensure(sizeof(float) * h->Nc));
    hipLaunchKernelGGL(k_scales, dim3(h->Nc * kStencil), dim3(256), 0, st, h->A128.as<c128>(),
                       h->mf_rho.as<float>(), nv * nv);
    HDCG_HIP(hipGetLastError());
    hipLaunchKernelGGL(k_rho, dim3((h->Nc + 127) / 128), dim3(128), 0, st, h->mf_rho.as<float>(),
                       h->mf_smax.as<float>(), h->Nc);
    HDCG_HIP(hipGetLastError());
  }
  DevBuf& F = prec == DWF_BF16 ? h->mf_bf16 : h->mf_f16;
  const size_t total = (size_t)h->Nc * ksteps * nv * 4;  // (a, s, m, kg), 4 values each
  HDCG_TRY(F.ensure(total * 4 * sizeof(unsigned short)));
  if (prec == DWF_BF16)
    hipLaunchKernelGGL((k_frag<true>), dim3((unsigned)((total + 255) / 256)), dim3(256), 0, st,
                       h->A128.as<c128>(), h->mf_rho.as<float>(), h->mf_smax.as<float>(),
                       F.as<unsigned short>(), h->Nc, nv, ksteps);
  else
    hipLaunchKernelGGL((k_frag<false>), dim3((unsigned)((total + 255) / 256)), dim3(256), 0, st,
                       h->A128.as<c128>(), h->mf_rho.as<float>(), h->mf_smax.as<float>(),
                       F.as<unsigned short>(), h->Nc, nv, ksteps);
  HDCG_HIP(hipGetLastError());
  if (prec == DWF_BF16)
    h->mf_have_bf16 = 1;
  else
    h->mf_have_f16 = 1;
  return DWF_OK;
}

int crs_apply_mfma(hdcg* h, int prec, const c64* in, c64* out, int nr, hipStream_t st) {
  if ((prec == DWF_BF16 && !h->mf_have_bf16) || (prec == DWF_F16 && !h->mf_have_f16))
    HDCG_TRY(crs_build_mfma(h, prec, st));
  const int mtiles = (h->nvec + 15) / 16;
  const int ksteps = (2 * kStencil * h->nvec + 15) / 16;
  const unsigned short* F = (prec == DWF_BF16 ? h->mf_bf16 : h->mf_f16).as<unsigned short>();
  const bool bf = prec == DWF_BF16;
  switch (mtiles) {
    case 1: return bf ? launch_mt<true, 1>(h, F, in, out, nr, ksteps, st) : launch_mt<false, 1>(h, F, in, out, nr, ksteps, st);
    case 2: return bf ? launch_mt<true, 2>(h, F, in, out, nr, ksteps, st) : launch_mt<false, 2>(h, F, in, out, nr, ksteps, st);
    case 3: return bf ? launch_mt<true, 3>(h, F, in, out, nr, ksteps, st) : launch_mt<false, 3>(h, F, in, out, nr, ksteps, st);
    default: return bf ? launch_mt<true, 4>(h, F, in, out, nr, ksteps, st) : launch_mt<false, 4>(h, F, in, out, nr, ksteps, st);
  }
}

}  // namespace hdk
