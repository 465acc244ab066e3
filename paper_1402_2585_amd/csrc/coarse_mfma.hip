// Little Dirac operator mat-vec on MFMA with 16-bit matrix storage (bf16
// or fp16) and FP32 accumulation: per-matrix scales, fragment-ordered
// storage and the standalone mat-vec launch.  The per-site GEMM itself
// (operand layout, scaling) is capply_site_mfma in coarse_dev.h.
#include <algorithm>
#include <cmath>
#include <map>
#include <mutex>
#include <tuple>
#include <vector>

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

// rho[a][l] = s_al / smax_a (in place), smax[a]; NS matrices per site
template <int NS>
__global__ void k_rho(float* __restrict__ s, float* __restrict__ smax, int Nc) {
  const int a = blockIdx.x * blockDim.x + threadIdx.x;
  if (a >= Nc) return;
  float m = 0.f;
  for (int l = 0; l < NS; ++l) m = fmaxf(m, s[a * NS + l]);
  smax[a] = m;
  for (int l = 0; l < NS; ++l) {
    const float v = s[a * NS + l];
    s[a * NS + l] = m > 0.f ? v / m : 0.f;
  }
}

// A: [Nc][NS][nvec][nvec] row-major matrices (NS = 81: the little Dirac
// operator; NS = 9: its one-hop truncation)
template <bool BF16, int NS>
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
  const int ktot = 2 * NS * nvec;
  unsigned short v4[4];
  for (int i = 0; i < 4; ++i) {
    const int kap = 16 * s + 4 * kg + i;
    float v = 0.f;
    if (kap < ktot) {
      const int part = kap / (NS * nvec);
      const int rem = kap - part * NS * nvec;
      const int l = rem / nvec, k = rem - (rem / nvec) * nvec;
      const float sal = rho[a * NS + l] * smax[a];
      const c128 x = A[(((size_t)a * NS + l) * nvec + m) * nvec + k];
      v = sal > 0.f ? (float)((part == 0 ? x.re : x.im) / sal) : 0.f;
    }
    v4[i] = to16<BF16>(v);
  }
  unsigned short* o = F + e * 4;
  for (int i = 0; i < 4; ++i) o[i] = v4[i];
}

template <bool BF16, int MT, int NT, int NW, int U, bool K32, int NS = kStencil>
__global__ void __launch_bounds__(NW * 64)
k_capply_mfma(const unsigned short* __restrict__ F, const float* __restrict__ rho,
              const float* __restrict__ smax, const int* __restrict__ nbr, const c64* __restrict__ in,
              c64* __restrict__ out, int Nc, int nvec, int nrhs, int ksteps) {
  __shared__ f32x4 red[NW * MT * NT * 64];
  capply_site_mfma<BF16, MT, NT, NW, U, false, false, K32, NS>(F, rho, smax, nbr, in, out, blockIdx.x, Nc, nvec,
                                                               nrhs, ksteps, red);
}

// One right-hand side: the site's operand at its NS neighbours is gathered
// into LDS first (one coalesced pass).
template <bool BF16, int MT, int U, bool K32, int NS = kStencil>
__global__ void __launch_bounds__(8 * 64)
k_capply_mfma_staged(const unsigned short* __restrict__ F, const float* __restrict__ rho,
                     const float* __restrict__ smax, const int* __restrict__ nbr, const c64* __restrict__ in,
                     c64* __restrict__ out, int Nc, int nvec, int ksteps) {
  __shared__ f32x4 red[8 * MT * 64];
  __shared__ c64 xin[NS * 64];
  const int a = blockIdx.x;
  const int* nb = nbr + (size_t)a * NS;
  for (int e = threadIdx.x; e < NS * nvec; e += 8 * 64) {
    const int l = e / nvec;
    xin[e] = in[(size_t)nb[l] * nvec + (e - l * nvec)];
  }
  __syncthreads();
  capply_site_mfma<BF16, MT, 1, 8, U, true, false, K32, NS>(F, rho, smax, nbr, xin, out, a, Nc, nvec, 1, ksteps,
                                                            red);
}

// ---------------------------------------------------------- tile shapes --
// The variants the autotuner chooses from: MFMA form (16x16x16, or gfx950's
// 16x16x32 with 8 K values per lane), waves per workgroup (the K range is
// split over them and reduced through LDS) and K steps per wave in flight.
// The N tiles follow the right-hand sides (one 16-column tile for up to 8,
// two for up to 16 per launch) and the M tiles nvec.
struct Tile {
  int k32, nw, u;
};
constexpr Tile kTiles[] = {{0, 8, 4}, {0, 4, 4}, {0, 8, 2}, {1, 8, 2}, {1, 4, 2}, {1, 8, 4}};
constexpr int kNumTiles = sizeof(kTiles) / sizeof(kTiles[0]);
constexpr int kDefaultTile = 0;  // the 16x16x16 form, 8 waves, 4 steps

bool tile_allowed(int t, int nvec, int mt, int nt, bool staged) {
  const Tile& T = kTiles[t];
  if (T.k32 && nvec % 8 != 0) return false;
  if (staged) return T.nw == 8 && (T.k32 ? T.u == 2 : T.u == 4);
  return (size_t)T.nw * mt * nt * 64 * sizeof(f32x4) <= 48 * 1024;
}

// the untuned choice: 8 waves while their LDS reduction buffers fit 48 KiB, else 4
int default_tile(int nvec, int n) {
  const int mt = (nvec + 15) / 16, nt = 2 * n <= 16 ? 1 : 2;
  return tile_allowed(kDefaultTile, nvec, mt, nt, n == 1) ? kDefaultTile : 1;
}

template <bool BF16, int MT, int NT, int NW, int U, bool K32>
void launch_plain(const unsigned short* F, const float* rho, const float* smax, const int* nbr, const c64* in, c64* out,
                  int Nc, int nvec, int n, int ksteps, hipStream_t st) {
  if constexpr ((size_t)NW * MT * NT * 64 * sizeof(f32x4) <= 48 * 1024)
    hipLaunchKernelGGL((k_capply_mfma<BF16, MT, NT, NW, U, K32>), dim3(Nc), dim3(NW * 64), 0, st, F, rho, smax, nbr,
                       in, out, Nc, nvec, n, ksteps);
}

template <bool BF16, int MT, int NT>
void launch_tile(int t, const unsigned short* F, const float* rho, const float* smax, const int* nbr, const c64* in,
                 c64* out, int Nc, int nvec, int n, int ksteps, hipStream_t st) {
  switch (t) {
    case 0: return launch_plain<BF16, MT, NT, 8, 4, false>(F, rho, smax, nbr, in, out, Nc, nvec, n, ksteps, st);
    case 1: return launch_plain<BF16, MT, NT, 4, 4, false>(F, rho, smax, nbr, in, out, Nc, nvec, n, ksteps, st);
    case 2: return launch_plain<BF16, MT, NT, 8, 2, false>(F, rho, smax, nbr, in, out, Nc, nvec, n, ksteps, st);
    case 3: return launch_plain<BF16, MT, NT, 8, 2, true>(F, rho, smax, nbr, in, out, Nc, nvec, n, ksteps, st);
    case 4: return launch_plain<BF16, MT, NT, 4, 2, true>(F, rho, smax, nbr, in, out, Nc, nvec, n, ksteps, st);
    default: return launch_plain<BF16, MT, NT, 8, 4, true>(F, rho, smax, nbr, in, out, Nc, nvec, n, ksteps, st);
  }
}

// One launch of tile t for right-hand sides [r0, r0 + n) (n <= 16).
template <bool BF16, int MT>
int launch_chunk(hdcg* h, int t, const unsigned short* F, const c64* in, c64* out, int n, int ksteps, hipStream_t st) {
  const float* rho = h->mf_rho.as<float>();
  const float* smax = h->mf_smax.as<float>();
  const int* nbr = h->nbr.as<int>();
  if (n == 1) {
    if (kTiles[t].k32)
      hipLaunchKernelGGL((k_capply_mfma_staged<BF16, MT, 2, true>), dim3(h->Nc), dim3(8 * 64), 0, st, F, rho, smax,
                         nbr, in, out, h->Nc, h->nvec, ksteps);
    else
      hipLaunchKernelGGL((k_capply_mfma_staged<BF16, MT, 4, false>), dim3(h->Nc), dim3(8 * 64), 0, st, F, rho, smax,
                         nbr, in, out, h->Nc, h->nvec, ksteps);
  } else if (2 * n <= 16) {
    launch_tile<BF16, MT, 1>(t, F, rho, smax, nbr, in, out, h->Nc, h->nvec, n, ksteps, st);
  } else {
    launch_tile<BF16, MT, 2>(t, F, rho, smax, nbr, in, out, h->Nc, h->nvec, n, ksteps, st);
  }
  HDCG_HIP(hipGetLastError());
  return DWF_OK;
}

template <bool BF16>
int launch_all(hdcg* h, int t, const unsigned short* F, const c64* in, c64* out, int nr, int ksteps, hipStream_t st) {
  const int mt = (h->nvec + 15) / 16;
  for (int r0 = 0; r0 < nr; r0 += 16) {
    const int n = nr - r0 < 16 ? nr - r0 : 16;
    const c64* i0 = in + (size_t)r0 * h->Nc * h->nvec;
    c64* o0 = out + (size_t)r0 * h->Nc * h->nvec;
    switch (mt) {
      case 1: HDCG_TRY((launch_chunk<BF16, 1>(h, t, F, i0, o0, n, ksteps, st))); break;
      case 2: HDCG_TRY((launch_chunk<BF16, 2>(h, t, F, i0, o0, n, ksteps, st))); break;
      case 3: HDCG_TRY((launch_chunk<BF16, 3>(h, t, F, i0, o0, n, ksteps, st))); break;
      default: HDCG_TRY((launch_chunk<BF16, 4>(h, t, F, i0, o0, n, ksteps, st))); break;
    }
  }
  return DWF_OK;
}

// --------------------------------------------------------- the autotuner --
// The tile of a shape (storage precision, Nc, nvec, right-hand sides per
// launch) is chosen once per process by timing every allowed variant on the
// caller's own operands (one warm-up launch, then the best of three timed
// with HIP events) and kept in a cache shared by all handles.  Tuning needs
// a host synchronisation, so a call made while its stream is being captured
// into a graph uses the cached tile, or the default one if there is none.
struct TuneKey {
  int prec, Nc, nvec, n;
  bool operator<(const TuneKey& o) const {
    return std::tie(prec, Nc, nvec, n) < std::tie(o.prec, o.Nc, o.nvec, o.n);
  }
};
std::mutex g_tune_mu;
std::map<TuneKey, int> g_tune;
std::map<TuneKey, std::vector<float>> g_tune_ms;  // measured ms per tile (negative: not allowed)

int tune(hdcg* h, int prec, const unsigned short* F, const c64* in, c64* out, int n, int ksteps, hipStream_t st,
         int* best) {
  const int mt = (h->nvec + 15) / 16, nt = 2 * n <= 16 ? 1 : 2;
  std::vector<float> ms(kNumTiles, -1.f);
  hipEvent_t e0, e1;
  HDCG_HIP(hipEventCreate(&e0));
  HDCG_HIP(hipEventCreate(&e1));
  int rc = DWF_OK, bt = default_tile(h->nvec, n);
  float bms = 0.f;
  for (int t = 0; t < kNumTiles && rc == DWF_OK; ++t) {
    if (!tile_allowed(t, h->nvec, mt, nt, n == 1)) continue;
    if (n == 1) {  // the staged kernel has one variant per MFMA form
      bool dup = false;
      for (int q = 0; q < t; ++q)
        if (ms[q] >= 0.f && kTiles[q].k32 == kTiles[t].k32) dup = true;
      if (dup) continue;
    }
    auto run = [&]() {
      return prec == DWF_BF16 ? launch_all<true>(h, t, F, in, out, n, ksteps, st)
                              : launch_all<false>(h, t, F, in, out, n, ksteps, st);
    };
    rc = run();
    float m = 1e30f;
    for (int rep = 0; rep < 3 && rc == DWF_OK; ++rep) {
      if (hipEventRecord(e0, st) != hipSuccess) rc = fail(DWF_ERR_HIP, "autotuner event failed");
      if (rc == DWF_OK) rc = run();
      if (rc == DWF_OK && (hipEventRecord(e1, st) != hipSuccess || hipEventSynchronize(e1) != hipSuccess))
        rc = fail(DWF_ERR_HIP, "autotuner event failed");
      float x = 0.f;
      if (rc == DWF_OK && hipEventElapsedTime(&x, e0, e1) == hipSuccess) m = std::min(m, x);
    }
    ms[t] = m;
    if (rc == DWF_OK && (bms == 0.f || m < bms)) {
      bms = m;
      bt = t;
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  HDCG_TRY(rc);
  *best = bt;
  std::lock_guard<std::mutex> lk(g_tune_mu);
  g_tune_ms[TuneKey{prec, h->Nc, h->nvec, n}] = ms;
  return DWF_OK;
}

int tile_for(hdcg* h, int prec, const unsigned short* F, const c64* in, c64* out, int n, int ksteps, hipStream_t st,
             int* t) {
  if (h->mfma_tile >= 0) {  // a fixed candidate (when allowed on the shape)
    const int mt = (h->nvec + 15) / 16, nt = 2 * n <= 16 ? 1 : 2;
    *t = h->mfma_tile < kNumTiles && tile_allowed(h->mfma_tile, h->nvec, mt, nt, n == 1) ? h->mfma_tile
                                                                                         : default_tile(h->nvec, n);
    return DWF_OK;
  }
  const TuneKey key{prec, h->Nc, h->nvec, n};
  {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    auto it = g_tune.find(key);
    if (it != g_tune.end()) {
      *t = it->second;
      return DWF_OK;
    }
  }
  *t = default_tile(h->nvec, n);
  hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
  if (hipStreamIsCapturing(st, &cs) != hipSuccess || cs != hipStreamCaptureStatusNone) return DWF_OK;
  HDCG_TRY(tune(h, prec, F, in, out, n, ksteps, st, t));
  std::lock_guard<std::mutex> lk(g_tune_mu);
  g_tune[key] = *t;
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
    hipLaunchKernelGGL(k_rho<kStencil>, dim3((h->Nc + 127) / 128), dim3(128), 0, st, h->mf_rho.as<float>(),
                       h->mf_smax.as<float>(), h->Nc);
    HDCG_HIP(hipGetLastError());
  }
  DevBuf& F = prec == DWF_BF16 ? h->mf_bf16 : h->mf_f16;
  const size_t total = (size_t)h->Nc * ksteps * nv * 4;  // (a, s, m, kg), 4 values each
  HDCG_TRY(F.ensure(total * 4 * sizeof(unsigned short)));
  if (prec == DWF_BF16)
    hipLaunchKernelGGL((k_frag<true, kStencil>), dim3((unsigned)((total + 255) / 256)), dim3(256), 0, st,
                       h->A128.as<c128>(), h->mf_rho.as<float>(), h->mf_smax.as<float>(),
                       F.as<unsigned short>(), h->Nc, nv, ksteps);
  else
    hipLaunchKernelGGL((k_frag<false, kStencil>), dim3((unsigned)((total + 255) / 256)), dim3(256), 0, st,
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
  const int ksteps = (2 * kStencil * h->nvec + 15) / 16;
  const unsigned short* F = (prec == DWF_BF16 ? h->mf_bf16 : h->mf_f16).as<unsigned short>();
  // one tile for the full 16-column launches, one for the last, smaller one
  const int nfull = nr / 16, rest = nr % 16;
  if (nfull > 0) {
    int t = 0;
    HDCG_TRY(tile_for(h, prec, F, in, out, 16, ksteps, st, &t));
    for (int c = 0; c < nfull; ++c) {
      const size_t off = (size_t)c * 16 * h->Nc * h->nvec;
      HDCG_TRY(prec == DWF_BF16 ? launch_all<true>(h, t, F, in + off, out + off, 16, ksteps, st)
                                : launch_all<false>(h, t, F, in + off, out + off, 16, ksteps, st));
    }
  }
  if (rest > 0) {
    const size_t off = (size_t)nfull * 16 * h->Nc * h->nvec;
    int t = 0;
    HDCG_TRY(tile_for(h, prec, F, in + off, out + off, rest, ksteps, st, &t));
    HDCG_TRY(prec == DWF_BF16 ? launch_all<true>(h, t, F, in + off, out + off, rest, ksteps, st)
                              : launch_all<false>(h, t, F, in + off, out + off, rest, ksteps, st));
  }
  return DWF_OK;
}

// ------------------------------------------- 16-bit truncated operator --
// Q_trunc + shift (the zero- and one-hop matrices of A, Sec. V.B) in the same
// 16-bit fragment storage as A, with its own per-matrix scales: nine matrices
// per site instead of 81.  Built from A128 through a temporary complex128
// copy of the nine matrices; applied with a fixed tile (the gfx950 16x16x32
// form when nvec % 8 == 0, eight waves; one right-hand side through the
// LDS-staged kernel).

namespace {

constexpr int kTS9 = kOneHop;

__global__ void k_q9(c128* __restrict__ Q, const c128* __restrict__ A, int Nc, int nvec, double shift) {
  const size_t total = (size_t)Nc * kTS9 * nvec * nvec;
  for (size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x; idx < total; idx += (size_t)gridDim.x * blockDim.x) {
    const int k = (int)(idx % nvec);
    const int j = (int)((idx / nvec) % nvec);
    const size_t am = idx / ((size_t)nvec * nvec);
    const int m = (int)(am % kTS9);
    const size_t a = am / kTS9;
    c128 v = A[((a * kStencil + one_hop_l(m)) * nvec + j) * nvec + k];
    if (m == 0 && j == k) v.re += shift;
    Q[idx] = v;
  }
}

template <bool BF16, int MT>
int trunc16_chunk(hdcg* h, const unsigned short* F, const c64* in, c64* out, int n, int ksteps, hipStream_t st) {
  const float* rho = h->tq_rho.as<float>();
  const float* smax = h->tq_smax.as<float>();
  const int* nbr = h->nbr9.as<int>();
  const bool k32 = h->nvec % 8 == 0;
  if (n == 1) {
    if (k32)
      hipLaunchKernelGGL((k_capply_mfma_staged<BF16, MT, 2, true, kTS9>), dim3(h->Nc), dim3(8 * 64), 0, st, F, rho,
                         smax, nbr, in, out, h->Nc, h->nvec, ksteps);
    else
      hipLaunchKernelGGL((k_capply_mfma_staged<BF16, MT, 4, false, kTS9>), dim3(h->Nc), dim3(8 * 64), 0, st, F, rho,
                         smax, nbr, in, out, h->Nc, h->nvec, ksteps);
  } else if (2 * n <= 16) {
    if (k32)
      hipLaunchKernelGGL((k_capply_mfma<BF16, MT, 1, 8, 2, true, kTS9>), dim3(h->Nc), dim3(8 * 64), 0, st, F, rho,
                         smax, nbr, in, out, h->Nc, h->nvec, n, ksteps);
    else
      hipLaunchKernelGGL((k_capply_mfma<BF16, MT, 1, 8, 4, false, kTS9>), dim3(h->Nc), dim3(8 * 64), 0, st, F, rho,
                         smax, nbr, in, out, h->Nc, h->nvec, n, ksteps);
  } else {
    // two 16-column tiles: the LDS reduction buffer of 8 waves is 8 * MT * 2
    // * 1 KiB, within 48 KiB for MT <= 3; 4 waves for MT = 4
    if constexpr (MT <= 3) {
      if (k32)
        hipLaunchKernelGGL((k_capply_mfma<BF16, MT, 2, 8, 2, true, kTS9>), dim3(h->Nc), dim3(8 * 64), 0, st, F, rho,
                           smax, nbr, in, out, h->Nc, h->nvec, n, ksteps);
      else
        hipLaunchKernelGGL((k_capply_mfma<BF16, MT, 2, 8, 4, false, kTS9>), dim3(h->Nc), dim3(8 * 64), 0, st, F,
                           rho, smax, nbr, in, out, h->Nc, h->nvec, n, ksteps);
    } else {
      if (k32)
        hipLaunchKernelGGL((k_capply_mfma<BF16, MT, 2, 4, 2, true, kTS9>), dim3(h->Nc), dim3(4 * 64), 0, st, F, rho,
                           smax, nbr, in, out, h->Nc, h->nvec, n, ksteps);
      else
        hipLaunchKernelGGL((k_capply_mfma<BF16, MT, 2, 4, 4, false, kTS9>), dim3(h->Nc), dim3(4 * 64), 0, st, F,
                           rho, smax, nbr, in, out, h->Nc, h->nvec, n, ksteps);
    }
  }
  HDCG_HIP(hipGetLastError());
  return DWF_OK;
}

template <bool BF16>
int trunc16_all(hdcg* h, const unsigned short* F, const c64* in, c64* out, int nr, hipStream_t st) {
  const int ksteps = (2 * kTS9 * h->nvec + 15) / 16;
  const int mt = (h->nvec + 15) / 16;
  for (int r0 = 0; r0 < nr; r0 += 16) {
    const int n = nr - r0 < 16 ? nr - r0 : 16;
    const size_t off = (size_t)r0 * h->Nc * h->nvec;
    switch (mt) {
      case 1: HDCG_TRY((trunc16_chunk<BF16, 1>(h, F, in + off, out + off, n, ksteps, st))); break;
      case 2: HDCG_TRY((trunc16_chunk<BF16, 2>(h, F, in + off, out + off, n, ksteps, st))); break;
      case 3: HDCG_TRY((trunc16_chunk<BF16, 3>(h, F, in + off, out + off, n, ksteps, st))); break;
      default: HDCG_TRY((trunc16_chunk<BF16, 4>(h, F, in + off, out + off, n, ksteps, st))); break;
    }
  }
  return DWF_OK;
}

}  // namespace

int trunc16_build(hdcg* h, int prec, double shift, hipStream_t st) {
  const int nv = h->nvec;
  if (nv % 4 != 0 || nv > 64)
    return fail(DWF_ERR_ARG, "16-bit truncated operator needs nvec a multiple of 4 and <= 64");
  if (h->A128.bytes == 0) return fail(DWF_ERR_ARG, "the truncated operator needs the little Dirac operator");
  if (h->nbr9.bytes == 0) return fail(DWF_ERR_STATE, "one-hop neighbour table not built");
  const size_t nmat = (size_t)h->Nc * kTS9;
  DevBuf q;
  HDCG_TRY(q.ensure(sizeof(c128) * nmat * nv * nv));
  const size_t tot = nmat * nv * nv;
  hipLaunchKernelGGL(k_q9, dim3((unsigned)std::min<size_t>((tot + 255) / 256, 65536)), dim3(256), 0, st, q.as<c128>(),
                     h->A128.as<c128>(), h->Nc, nv, shift);
  HDCG_HIP(hipGetLastError());
  HDCG_TRY(h->tq_rho.ensure(sizeof(float) * nmat));
  HDCG_TRY(h->tq_smax.ensure(sizeof(float) * h->Nc));
  hipLaunchKernelGGL(k_scales, dim3((unsigned)nmat), dim3(256), 0, st, q.as<c128>(), h->tq_rho.as<float>(), nv * nv);
  HDCG_HIP(hipGetLastError());
  hipLaunchKernelGGL(k_rho<kTS9>, dim3((h->Nc + 127) / 128), dim3(128), 0, st, h->tq_rho.as<float>(),
                     h->tq_smax.as<float>(), h->Nc);
  HDCG_HIP(hipGetLastError());
  const int ksteps = (2 * kTS9 * nv + 15) / 16;
  const size_t total = (size_t)h->Nc * ksteps * nv * 4;
  DevBuf& F = prec == DWF_BF16 ? h->tq_bf16 : h->tq_f16;
  HDCG_TRY(F.ensure(total * 4 * sizeof(unsigned short)));
  if (prec == DWF_BF16)
    hipLaunchKernelGGL((k_frag<true, kTS9>), dim3((unsigned)((total + 255) / 256)), dim3(256), 0, st, q.as<c128>(),
                       h->tq_rho.as<float>(), h->tq_smax.as<float>(), F.as<unsigned short>(), h->Nc, nv, ksteps);
  else
    hipLaunchKernelGGL((k_frag<false, kTS9>), dim3((unsigned)((total + 255) / 256)), dim3(256), 0, st, q.as<c128>(),
                       h->tq_rho.as<float>(), h->tq_smax.as<float>(), F.as<unsigned short>(), h->Nc, nv, ksteps);
  HDCG_HIP(hipGetLastError());
  HDCG_HIP(hipStreamSynchronize(st));  // before the temporary copy is freed
  q.release();
  (prec == DWF_BF16 ? h->tq_shift_bf16 : h->tq_shift_f16) = shift;
  // the scales are shared by the two 16-bit forms: the other one is stale now
  (prec == DWF_BF16 ? h->tq_shift_f16 : h->tq_shift_bf16) = std::nan("");
  return DWF_OK;
}

int trunc16_apply(hdcg* h, int prec, const c64* in, c64* out, int nr, hipStream_t st) {
  const unsigned short* F = (prec == DWF_BF16 ? h->tq_bf16 : h->tq_f16).as<unsigned short>();
  return prec == DWF_BF16 ? trunc16_all<true>(h, F, in, out, nr, st) : trunc16_all<false>(h, F, in, out, nr, st);
}

// The tile the autotuner chose for (prec, n right-hand sides per launch) on
// this handle's shape, tuning now on scratch operands if it has not run:
// out[0..2] = {MFMA form (16 or 32 K per instruction), waves, K steps per
// wave}; ms (nullable, kNumTiles entries) the measured times, -1 for tiles
// not allowed on the shape.
int crs_mfma_tile(hdcg* h, int prec, int n, int out[3], float* ms, int* ntiles, hipStream_t st) {
  if (ntiles) *ntiles = kNumTiles;
  if ((prec == DWF_BF16 && !h->mf_have_bf16) || (prec == DWF_F16 && !h->mf_have_f16))
    HDCG_TRY(crs_build_mfma(h, prec, st));
  const TuneKey key{prec, h->Nc, h->nvec, n};
  bool have = false;
  {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    have = g_tune.count(key) > 0;
  }
  if (!have) {
    DevBuf a, b;
    const size_t bytes = (size_t)n * h->Nc * h->nvec * sizeof(c64);
    HDCG_TRY(a.ensure(bytes));
    HDCG_TRY(b.ensure(bytes));
    HDCG_HIP(hipMemsetAsync(a.ptr, 0, bytes, st));
    int t = 0;
    const int rc = tile_for(h, prec, (prec == DWF_BF16 ? h->mf_bf16 : h->mf_f16).as<unsigned short>(), a.as<c64>(),
                            b.as<c64>(), n, (2 * kStencil * h->nvec + 15) / 16, st, &t);
    HDCG_HIP(hipStreamSynchronize(st));
    a.release();
    b.release();
    HDCG_TRY(rc);
  }
  std::lock_guard<std::mutex> lk(g_tune_mu);
  auto it = g_tune.find(key);
  const int t = it != g_tune.end() ? it->second : default_tile(h->nvec, n);
  out[0] = kTiles[t].k32 ? 32 : 16;
  out[1] = kTiles[t].nw;
  out[2] = kTiles[t].u;
  if (ms) {
    auto m = g_tune_ms.find(key);
    for (int i = 0; i < kNumTiles; ++i) ms[i] = m != g_tune_ms.end() ? m->second[i] : -1.f;
  }
  return DWF_OK;
}

}  // namespace hdk
