// Kernels of the blocked subspace and the little Dirac operator:
//   block map (integer index tables), subspace layout, batched block inner
//   products (project, Gram matrices), promote, Cholesky-QR
//   orthonormalisation, the per-dimension inverse of the 81-point phase
//   matrix, and the complex64/complex128 coarse block-stencil mat-vec.
#include "coarse_dev.h"

namespace hdk {

namespace {

constexpr int kT = 256;
// right-hand-side counts from which the 16-bit-subspace project / promote
// run on MFMA
constexpr int kProjectMfmaRhs = 2;
constexpr int kPromoteMfmaRhs = 2;

__global__ void k_blockmap(int* __restrict__ site_of, Geom g, int4 B, int4 C, int nsb, int total) {
  const int idx = blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= total) return;
  const int a = idx / nsb, j = idx - (idx / nsb) * nsb;
  int r = a;
  const int cx = r % C.x;
  r /= C.x;
  const int cy = r % C.y;
  r /= C.y;
  const int cz = r % C.z;
  const int ct = r / C.z;
  // odd site j of the block: one of the local lexicographic pair (2j, 2j+1)
  int L = 2 * j;
  const int lx0 = L % B.x;
  L /= B.x;
  const int ly = L % B.y;
  L /= B.y;
  const int lz = L % B.z;
  const int lt = L / B.z;
  const int x0 = cx * B.x + lx0, y = cy * B.y + ly, z = cz * B.z + lz, t = ct * B.w + lt;
  const int x = x0 + ((x0 + y + z + t + 1) & 1);
  const long lex = x + (long)g.X * (y + (long)g.Y * (z + (long)g.Z * t));
  site_of[idx] = (int)(lex >> 1);
}

__global__ void k_nbr(int* __restrict__ nbr, int4 C, int Nc) {
  const int idx = blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= Nc * kStencil) return;
  const int a = idx / kStencil, l = idx % kStencil;
  const int Cd[4] = {C.x, C.y, C.z, C.w};
  int c[4];
  int r = a;
  for (int mu = 0; mu < 4; ++mu) {
    c[mu] = r % Cd[mu];
    r /= Cd[mu];
  }
  int q = l;
  for (int mu = 0; mu < 4; ++mu) {
    const int d = q % 3 - 1;
    q /= 3;
    c[mu] = (c[mu] + d + Cd[mu]) % Cd[mu];
  }
  nbr[idx] = c[0] + C.x * (c[1] + C.y * (c[2] + C.z * c[3]));
}

template <typename R>
__global__ void k_phi_layout(cplx<R>* __restrict__ phi, const cplx<double>* __restrict__ can,
                             const int* __restrict__ site_of, int nsb, int Ls, int Vh, int nvec,
                             size_t nb, size_t total, bool to_native) {
  const size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= total) return;
  const size_t panel = (size_t)nvec * nb;
  const size_t a = e / panel, rem = e - a * panel;
  const size_t k = rem / nb, i = rem - k * nb;
  const int col = 12 * Ls;
  const int j = (int)(i / col), q = (int)(i - (size_t)j * col);
  const int c = q / Ls, s = q - (q / Ls) * Ls;
  const size_t cb = (size_t)site_of[a * nsb + j];
  const size_t ci = ((k * Ls + s) * (size_t)Vh + cb) * 12 + c;
  if (to_native) {
    const cplx<double> v = can[ci];
    phi[e] = cmk((R)v.re, (R)v.im);
  } else {
    const cplx<R> v = phi[e];
    const_cast<cplx<double>*>(can)[ci] = cmk((double)v.re, (double)v.im);
  }
}

// Position in a fine site column (12 Ls: [spin-colour][s]) of entry q of a
// subspace column that keeps only the surface slices (12 x 2 sd: s < sd, then
// s >= Ls - sd); sd = 0: the full column, q itself.
__device__ __forceinline__ int surf_q(int q, int Ls, int sd) {
  if (sd == 0) return q;
  const int w = 2 * sd, c = q / w, sp = q - c * w;
  return c * Ls + (sp < sd ? sp : Ls - w + sp);
}

// out[r*sr + a*sa + k*sk] = ph[a] * sum_i conj(P[a][k][i]) Q(r, a, i)
// P is stored as TP (cplx<R>, or bf16c with R = float); arithmetic in R.
// P's site column has colP entries (col, or the surface-only 24 sd).
template <typename TP, bool FINE, typename R = typename St<TP>::R>
__global__ void __launch_bounds__(kT)
k_blkdot(const TP* __restrict__ P, const cplx<R>* __restrict__ Q, size_t fstride,
         const int* __restrict__ site_of, int nsb, int col, int colP, int Ls, int sd, size_t nb, int nvec, int nr,
         cplx<R>* __restrict__ out, size_t sr, size_t sa, size_t sk,
         const cplx<double>* __restrict__ phase) {
  __shared__ cplx<R> Ps[16][33];
  __shared__ cplx<R> Qs[32][17];
  const int a = blockIdx.x, k0 = blockIdx.y * 16, r0 = blockIdx.z * 16;
  const int t = threadIdx.x, tk = t >> 4, tr = t & 15;
  cplx<R> acc = cmk((R)0, (R)0);
  const TP* Pa = P + (size_t)a * nvec * nb;
  for (size_t i0 = 0; i0 < nb; i0 += 32) {
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const int e = t + h * kT;
      const int kk = e >> 5, ii = e & 31;
      const int k = k0 + kk;
      cplx<R> v = cmk((R)0, (R)0);
      if (k < nvec) v = conj(St<TP>::ld(Pa + (size_t)k * nb + i0 + ii));
      Ps[kk][ii] = v;
      const int rr = e >> 5;  // 0..15
      const int r = r0 + rr;
      cplx<R> q = cmk((R)0, (R)0);
      if (r < nr) {
        const size_t i = i0 + ii;
        if (FINE) {
          const int j = (int)(i / colP), qq = (int)(i - (size_t)j * colP);
          q = Q[r * fstride + (size_t)site_of[(size_t)a * nsb + j] * col + surf_q(qq, Ls, sd)];
        } else {
          q = Q[((size_t)a * nr + r) * nb + i];
        }
      }
      Qs[ii][rr] = q;
    }
    __syncthreads();
#pragma unroll 8
    for (int ii = 0; ii < 32; ++ii) cmac(acc, Ps[tk][ii], Qs[ii][tr]);
    __syncthreads();
  }
  const int k = k0 + tk, r = r0 + tr;
  if (k < nvec && r < nr) {
    if (phase) {
      const cplx<double> ph = phase[a];
      acc = cmk((R)(ph.re * acc.re - ph.im * acc.im), (R)(ph.re * acc.im + ph.im * acc.re));
    }
    out[r * sr + a * sa + k * sk] = acc;
  }
}

// V consecutive subspace values (V = 4: one 16-byte load of bf16 pairs)
template <typename TP, int V, typename R = typename St<TP>::R>
__device__ __forceinline__ void ld_phi(const TP* p, cplx<R> (&o)[V]) {
  if constexpr (V == 4 && sizeof(TP) == 4) {
    const uint4 w = *reinterpret_cast<const uint4*>(p);
    const unsigned u[4] = {w.x, w.y, w.z, w.w};
#pragma unroll
    for (int e = 0; e < 4; ++e) o[e] = cmk(__uint_as_float(u[e] << 16), __uint_as_float(u[e] & 0xffff0000u));
  } else {
#pragma unroll
    for (int e = 0; e < V; ++e) o[e] = St<TP>::ld(p + e);
  }
}

// Few right-hand sides: one 128-thread workgroup per (block a, group of KG
// subspace vectors k0 .. k0 + KG - 1) streams the KG rows P[a][k][:] once,
// lanes striding over the entries V at a time; each fine value loaded serves
// all KG rows, so the block's fine data is read Nvec / KG times from L2
// instead of Nvec times.  out[r*sr + a*sa + k*sk] =
// sum_i conj(P[a][k][i]) Q_r(site(a, i)).  The workgroups of one block are
// consecutive after the XCD remap, so its fine data stays in one L2.
template <typename TP, int NR, int V, int KG, typename R = typename St<TP>::R>
__global__ void __launch_bounds__(128)
k_project_small(const TP* __restrict__ P, const cplx<R>* __restrict__ Q, size_t fstride,
                const int* __restrict__ site_of, int nsb, int col, int colP, int Ls, int sd, size_t nb, int nvec,
                int nr, cplx<R>* __restrict__ out, size_t sr, size_t sa, size_t sk) {
  const int wg = xcd_remap(blockIdx.x, gridDim.x);
  const int ngrp = (nvec + KG - 1) / KG;
  const int k0 = (wg % ngrp) * KG, a = wg / ngrp;
  const TP* Pk = P + ((size_t)a * nvec + k0) * nb;
  const int* so = site_of + (size_t)a * nsb;
  cplx<R> acc[KG][NR];
#pragma unroll
  for (int g = 0; g < KG; ++g)
#pragma unroll
    for (int r = 0; r < NR; ++r) acc[g][r] = cmk((R)0, (R)0);
  // each row P[a][k][:] is one contiguous run of nsb colP entries; V
  // consecutive entries stay in one site column and one surface run
  // (colP % V == 0, sd % V == 0); U strides' loads are issued before the
  // multiply-adds
  constexpr int U = V == 4 ? 1 : 4;
  const int total = nsb * colP;
  const int step = blockDim.x * V;
  for (int e0 = threadIdx.x * V; e0 < total; e0 += step * U) {
    cplx<R> pv[U][KG][V], qv[U][NR][V];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int e = e0 + u * step;
#pragma unroll
      for (int x = 0; x < V; ++x) {
#pragma unroll
        for (int g = 0; g < KG; ++g) pv[u][g][x] = cmk((R)0, (R)0);
#pragma unroll
        for (int r = 0; r < NR; ++r) qv[u][r][x] = cmk((R)0, (R)0);
      }
      if (e < total) {
        const int j = e / colP, q = e - j * colP;
#pragma unroll
        for (int g = 0; g < KG; ++g)
          if (k0 + g < nvec) ld_phi<TP, V>(Pk + (size_t)g * nb + e, pv[u][g]);
        const size_t base = (size_t)so[j] * col + surf_q(q, Ls, sd);
#pragma unroll
        for (int r = 0; r < NR; ++r)
          if (r < nr)
#pragma unroll
            for (int x = 0; x < V; ++x) qv[u][r][x] = Q[r * fstride + base + x];
      }
    }
#pragma unroll
    for (int u = 0; u < U; ++u)
#pragma unroll
      for (int g = 0; g < KG; ++g)
#pragma unroll
        for (int r = 0; r < NR; ++r)
#pragma unroll
          for (int x = 0; x < V; ++x) cjmac(acc[g][r], pv[u][g][x], qv[u][r][x]);
  }
  __shared__ double red[KG * NR][2][2];  // [(g, r)][re / im][wave]
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
  for (int g = 0; g < KG; ++g)
#pragma unroll
    for (int r = 0; r < NR; ++r) {
      const double re = wave_sum((double)acc[g][r].re), im = wave_sum((double)acc[g][r].im);
      if (lane == 0) {
        red[g * NR + r][0][wave] = re;
        red[g * NR + r][1][wave] = im;
      }
    }
  __syncthreads();
  if (threadIdx.x < KG * NR) {
    const int g = threadIdx.x / NR, r = threadIdx.x - g * NR;
    if (r < nr && k0 + g < nvec) {
      const double re = red[threadIdx.x][0][0] + red[threadIdx.x][0][1];
      const double im = red[threadIdx.x][1][0] + red[threadIdx.x][1][1];
      out[r * sr + a * sa + (k0 + g) * sk] = cmk((R)re, (R)im);
    }
  }
}

// fine_out[r][site(a, i)] = base + sign * sum_k P[a][k][i] c[r][a][k], V
// consecutive i per thread (they lie in one site column: 12 Ls % V == 0)
template <typename TP, int NR, int V, typename R = typename St<TP>::R>
__global__ void __launch_bounds__(kT)
k_promote(const TP* __restrict__ P, const cplx<R>* __restrict__ c, int nr, int Nc, int nvec,
          size_t nb, int nsb, int col, int colP, int Ls, int sd, const int* __restrict__ site_of, cplx<R>* out,
          const cplx<R>* base, R sign, size_t fstride) {  // out may alias base (in place)
  __shared__ cplx<R> cs[NR * 64];
  const int a = blockIdx.y;
  const size_t i = ((size_t)blockIdx.x * kT + threadIdx.x) * V;
  for (int e = threadIdx.x; e < nr * nvec; e += kT)
    cs[e] = c[((size_t)(e / nvec) * Nc + a) * nvec + e % nvec];
  __syncthreads();
  if (i >= nb) return;
  cplx<R> acc[NR][V];
#pragma unroll
  for (int r = 0; r < NR; ++r)
#pragma unroll
    for (int e = 0; e < V; ++e) acc[r][e] = cmk((R)0, (R)0);
  const TP* Pa = P + (size_t)a * nvec * nb + i;
  // U subspace vectors at a time, their loads issued before the multiply-adds
  constexpr int U = 8;
  for (int k0 = 0; k0 < nvec; k0 += U) {
    cplx<R> pv[U][V];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      if (k0 + u < nvec) {
        ld_phi<TP, V>(Pa + (size_t)(k0 + u) * nb, pv[u]);
      } else {
#pragma unroll
        for (int e = 0; e < V; ++e) pv[u][e] = cmk((R)0, (R)0);
      }
    }
#pragma unroll
    for (int u = 0; u < U; ++u)
#pragma unroll
      for (int r = 0; r < NR; ++r)
        if (r < nr && k0 + u < nvec)
#pragma unroll
          for (int e = 0; e < V; ++e) cmac(acc[r][e], pv[u][e], cs[r * nvec + k0 + u]);
  }
  const int j = (int)(i / colP), q = (int)(i - (size_t)j * colP);
  const size_t addr = (size_t)site_of[(size_t)a * nsb + j] * col + surf_q(q, Ls, sd);
#pragma unroll
  for (int r = 0; r < NR; ++r) {
    if (r < nr) {
#pragma unroll
      for (int e = 0; e < V; ++e) {
        cplx<R> o = sign * acc[r][e];
        if (base) o = base[r * fstride + addr + e] + o;
        out[r * fstride + addr + e] = o;
      }
    }
  }
}

// Cholesky G = R^+ R (R upper, positive diagonal) of one block's Gram
// matrix, then X = R^-1; one workgroup per block, thread m owns column m.
__global__ void __launch_bounds__(64)
k_chol_inv(const c128* __restrict__ G, c128* __restrict__ X, int nvec, int* flag) {
  extern __shared__ __align__(16) unsigned char smem[];
  c128* S = reinterpret_cast<c128*>(smem);  // [nvec][nvec], upper triangle used
  const int a = blockIdx.x, m = threadIdx.x;
  const size_t off = (size_t)a * nvec * nvec;
  for (int e = m; e < nvec * nvec; e += blockDim.x) S[e] = G[off + e];
  __syncthreads();
  for (int k = 0; k < nvec; ++k) {
    if (m == 0) {
      const double d = S[k * nvec + k].re;
      if (!(d > 0.0)) {
        atomicExch(flag, 1);
        S[k * nvec + k] = cmk(1.0, 0.0);
      } else {
        S[k * nvec + k] = cmk(sqrt(d), 0.0);
      }
    }
    __syncthreads();
    const double rkk = S[k * nvec + k].re;
    if (m > k && m < nvec) S[k * nvec + m] = (1.0 / rkk) * S[k * nvec + m];
    __syncthreads();
    if (m > k && m < nvec) {
      const c128 rkm = S[k * nvec + m];
      for (int i = k + 1; i <= m; ++i) {
        const c128 rki = S[k * nvec + i];
        c128 v = S[i * nvec + m];
        v.re -= rki.re * rkm.re + rki.im * rkm.im;  // conj(R[k][i]) R[k][m]
        v.im -= rki.re * rkm.im - rki.im * rkm.re;
        S[i * nvec + m] = v;
      }
    }
    __syncthreads();
  }
  // column m of X = R^-1 by back substitution
  if (m < nvec) {
    c128* Xa = X + off;
    for (int i = m + 1; i < nvec; ++i) Xa[i * nvec + m] = cmk(0.0, 0.0);
    c128 xm = cmk(1.0 / S[m * nvec + m].re, 0.0);
    Xa[m * nvec + m] = xm;
    for (int i = m - 1; i >= 0; --i) {
      c128 s = cmk(0.0, 0.0);
      for (int j = i + 1; j <= m; ++j) cmac(s, S[i * nvec + j], Xa[j * nvec + m]);
      Xa[i * nvec + m] = (-1.0 / S[i * nvec + i].re) * s;
    }
  }
}

// phi[a][k][i] <- sum_{j <= k} phi[a][j][i] X[j][k]
__global__ void __launch_bounds__(kT)
k_gs_apply(c128* __restrict__ phi, const c128* __restrict__ X, int nvec, size_t nb) {
  extern __shared__ __align__(16) unsigned char smem[];
  c128* S = reinterpret_cast<c128*>(smem);  // [nvec][32]
  const int a = blockIdx.y;
  const size_t i0 = (size_t)blockIdx.x * 32;
  const int ii = threadIdx.x & 31, kg = threadIdx.x >> 5;
  c128* Pa = phi + (size_t)a * nvec * nb;
  const c128* Xa = X + (size_t)a * nvec * nvec;
  for (int e = threadIdx.x; e < nvec * 32; e += kT) {
    const int j = e >> 5, q = e & 31;
    S[j * 32 + q] = (i0 + q < nb) ? Pa[(size_t)j * nb + i0 + q] : cmk(0.0, 0.0);
  }
  __syncthreads();
  c128 res[8];
#pragma unroll
  for (int u = 0; u < 8; ++u) {
    const int k = kg + 8 * u;
    c128 acc = cmk(0.0, 0.0);
    if (k < nvec)
      for (int j = 0; j <= k; ++j) cmac(acc, S[j * 32 + ii], Xa[j * nvec + k]);
    res[u] = acc;
  }
#pragma unroll
  for (int u = 0; u < 8; ++u) {
    const int k = kg + 8 * u;
    if (k < nvec && i0 + ii < nb) Pa[(size_t)k * nb + i0 + ii] = res[u];
  }
}

__global__ void k_idft_dim(c128* __restrict__ Y, int nvec2, int Nc, int mu, c128 f00, c128 f01,
                           c128 f02, c128 f10, c128 f11, c128 f12, c128 f20, c128 f21, c128 f22) {
  const size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  const size_t total = (size_t)Nc * 27 * nvec2;
  if (idx >= total) return;
  const int jk = (int)(idx % nvec2);
  const int o = (int)((idx / nvec2) % 27);
  const size_t a = idx / ((size_t)nvec2 * 27);
  int d[4];
  int q = o;
  for (int nu = 0; nu < 4; ++nu) {
    if (nu == mu) {
      d[nu] = 0;
      continue;
    }
    d[nu] = q % 3;
    q /= 3;
  }
  int stride = 1;
  for (int nu = 0; nu < mu; ++nu) stride *= 3;
  const int l0 = d[0] + 3 * (d[1] + 3 * (d[2] + 3 * d[3]));
  c128* base = Y + (a * kStencil) * nvec2 + jk;
  const c128 y0 = base[(size_t)(l0)*nvec2];
  const c128 y1 = base[(size_t)(l0 + stride) * nvec2];
  const c128 y2 = base[(size_t)(l0 + 2 * stride) * nvec2];
  c128 r0 = f00 * y0, r1 = f10 * y0, r2 = f20 * y0;
  cmac(r0, f01, y1);
  cmac(r0, f02, y2);
  cmac(r1, f11, y1);
  cmac(r1, f12, y2);
  cmac(r2, f21, y1);
  cmac(r2, f22, y2);
  base[(size_t)(l0)*nvec2] = r0;
  base[(size_t)(l0 + stride) * nvec2] = r1;
  base[(size_t)(l0 + 2 * stride) * nvec2] = r2;
}

__global__ void k_transpose(const c128* __restrict__ A, c128* __restrict__ AT128,
                            c64* __restrict__ AT64, int nvec, size_t total) {
  const size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= total) return;
  const size_t n2 = (size_t)nvec * nvec;
  const size_t al = e / n2;
  const int jk = (int)(e - al * n2);
  const int j = jk / nvec, k = jk - j * nvec;
  const c128 v = A[e];
  const size_t o = al * n2 + (size_t)k * nvec + j;
  if (AT128) AT128[o] = v;
  if (AT64) AT64[o] = cmk((float)v.re, (float)v.im);
}

// (A c)[r][a][j] = sum_l sum_k A[a][l][j][k] c[r][nbr(a,l)][k], with AT[a][l][k][j].
template <typename R, int NR, int U>
__global__ void __launch_bounds__(kCT)
k_capply(const cplx<R>* __restrict__ AT, const int* __restrict__ nbr, const cplx<R>* __restrict__ in,
         cplx<R>* __restrict__ out, int Nc, int nvec, int nr) {
  __shared__ cplx<R> red[kCT * NR];
  capply_site<R, NR, U>(AT, nbr, in, out, blockIdx.x, Nc, nvec, nr, blockIdx.y * NR, red);
}

// One right-hand side in complex64: the site's operand at its 81 neighbours
// is first gathered into LDS (one coalesced pass), so the column loop reads
// only the operator from memory.
constexpr int kStageNvec = 64;
template <int U>
__global__ void __launch_bounds__(kCT)
k_capply_staged(const c64* __restrict__ AT, const int* __restrict__ nbr, const c64* __restrict__ in,
                c64* __restrict__ out, int Nc, int nvec) {
  __shared__ c64 red[kCT];
  __shared__ c64 xin[kStencil * kStageNvec];
  const int a = blockIdx.x;
  const int* nb = nbr + (size_t)a * kStencil;
  for (int e = threadIdx.x; e < kStencil * nvec; e += kCT) {
    const int l = e / nvec;
    xin[e] = in[(size_t)nb[l] * nvec + (e - l * nvec)];
  }
  __syncthreads();
  capply_site<float, 1, U, true>(AT, nbr, xin, out, a, Nc, nvec, 1, 0, red);
}

// Complex64 / complex128 with several right-hand sides on the FP32 / FP64
// MFMA: up to 16 per launch row (blockIdx.y takes the right-hand sides
// 16 y .. 16 y + 15).
template <typename R, int MT, int NT, int NW, int U>
__global__ void __launch_bounds__(NW * 64)
k_capply_cmfma(const cplx<R>* __restrict__ AT, const int* __restrict__ nbr, const cplx<R>* __restrict__ in,
               cplx<R>* __restrict__ out, int Nc, int nvec, int nr) {
  __shared__ macc_t<R> red[NW * MT * NT * 64];
  const int r0 = 16 * blockIdx.y;
  const size_t off = (size_t)r0 * Nc * nvec;
  capply_site_cmfma<R, MT, NT, NW, U>(AT, nbr, in + off, out + off, blockIdx.x, Nc, nvec, min(16, nr - r0), red);
}

template <typename R, int MT, int NT>
void launch_cmfma(const cplx<R>* AT, const int* nbr, const cplx<R>* in, cplx<R>* out, int Nc, int nvec, int nr,
                  hipStream_t st) {
  // eight waves while their LDS reduction buffers fit 48 KiB, else four or two
  constexpr size_t kTile = 64 * sizeof(macc_t<R>);
  constexpr int NW = 8 * MT * NT * kTile <= 48 * 1024 ? 8 : (4 * MT * NT * kTile <= 48 * 1024 ? 4 : 2);
  hipLaunchKernelGGL((k_capply_cmfma<R, MT, NT, NW, 2>), dim3(Nc, (nr + 15) / 16), dim3(NW * 64), 0, st, AT, nbr, in,
                     out, Nc, nvec, nr);
}

template <typename R, int MT>
void launch_cmfma_nt(const cplx<R>* AT, const int* nbr, const cplx<R>* in, cplx<R>* out, int Nc, int nvec, int nr,
                     hipStream_t st) {
  if (nr > 8)
    launch_cmfma<R, MT, 2>(AT, nbr, in, out, Nc, nvec, nr, st);
  else
    launch_cmfma<R, MT, 1>(AT, nbr, in, out, Nc, nvec, nr, st);
}

}  // namespace

// ================================================================= host ===
int blk_build_maps(hdcg* h, hipStream_t st) {
  const Geom& g = h->op->g;
  HDCG_TRY(h->site_of.ensure(sizeof(int) * (size_t)h->Nc * h->nsb));
  HDCG_TRY(h->nbr.ensure(sizeof(int) * (size_t)h->Nc * kStencil));
  const int total = h->Nc * h->nsb;
  hipLaunchKernelGGL(k_blockmap, dim3((total + 255) / 256), dim3(256), 0, st, h->site_of.as<int>(), g,
                     make_int4(h->B[0], h->B[1], h->B[2], h->B[3]),
                     make_int4(h->C[0], h->C[1], h->C[2], h->C[3]), h->nsb, total);
  HDCG_HIP(hipGetLastError());
  const int tn = h->Nc * kStencil;
  hipLaunchKernelGGL(k_nbr, dim3((tn + 255) / 256), dim3(256), 0, st, h->nbr.as<int>(),
                     make_int4(h->C[0], h->C[1], h->C[2], h->C[3]), h->Nc);
  HDCG_HIP(hipGetLastError());
  return DWF_OK;
}

template <typename R>
int blk_phi_layout(hdcg* h, cplx<R>* phi, const cplx<double>* can, bool to_native, int,
                   hipStream_t st) {
  const size_t total = (size_t)h->Nc * h->nvec * h->nb;
  hipLaunchKernelGGL((k_phi_layout<R>), dim3((unsigned)((total + 255) / 256)), dim3(256), 0, st, phi,
                     can, h->site_of.as<int>(), h->nsb, h->op->g.Ls, h->op->g.Vh, h->nvec, h->nb,
                     total, to_native);
  HDCG_HIP(hipGetLastError());
  return DWF_OK;
}

// sd > 0: P holds only the surface slices (columns of 24 sd entries)
template <typename TP, typename R = typename St<TP>::R>
int blk_dot_t(hdcg* h, const TP* P, const cplx<R>* fine, size_t fstride, const cplx<R>* blockq,
              int nr, cplx<R>* out, size_t sr, size_t sa, size_t sk, const cplx<double>* phase,
              hipStream_t st, int sd = 0) {
  const int Ls = h->op->g.Ls;
  const int col = 12 * Ls;
  const int colP = sd > 0 ? 24 * sd : col;
  const size_t nbP = (size_t)h->nsb * colP;
  if (sd > 0 && (!fine || phase)) return fail(DWF_ERR_ARG, "surface subspace: fine-field projection only");
  if constexpr (std::is_same_v<TP, bf16c>) {
    if (fine && !phase && nr >= kProjectMfmaRhs && blk_mfma_applies(h, P, fine, fstride, sd))
      return blk_project_mfma(h, P, fine, fstride, nr, out, sr, sa, sk, st);
  }
  if (fine && !phase && nr <= 4) {
    // streaming kernel: P read once, few accumulators per lane
    constexpr int V = sizeof(TP) == 4 ? 4 : 1;  // 16-byte loads of the 16-bit subspace
    if (col % V || sd % V) return fail(DWF_ERR_ARG, "project: 12 Ls and the surface depth must be multiples of 4");
    // two waves per workgroup (the kernel's reduction assumes 128 threads)
    if (nr == 1) {
      constexpr int KG = 8;
      dim3 g2(h->Nc * ((h->nvec + KG - 1) / KG));
      hipLaunchKernelGGL((k_project_small<TP, 1, V, KG>), g2, dim3(128), 0, st, P, fine, fstride,
                         h->site_of.as<int>(), h->nsb, col, colP, Ls, sd, nbP, h->nvec, nr, out, sr, sa, sk);
    } else {
      constexpr int KG = 2;
      dim3 g2(h->Nc * ((h->nvec + KG - 1) / KG));
      hipLaunchKernelGGL((k_project_small<TP, 4, V, KG>), g2, dim3(128), 0, st, P, fine, fstride,
                         h->site_of.as<int>(), h->nsb, col, colP, Ls, sd, nbP, h->nvec, nr, out, sr, sa, sk);
    }
    HDCG_HIP(hipGetLastError());
    return DWF_OK;
  }
  dim3 grid(h->Nc, (h->nvec + 15) / 16, (nr + 15) / 16);
  if (fine)
    hipLaunchKernelGGL((k_blkdot<TP, true>), grid, dim3(kT), 0, st, P, fine, fstride,
                       h->site_of.as<int>(), h->nsb, col, colP, Ls, sd, nbP, h->nvec, nr, out, sr, sa, sk, phase);
  else
    hipLaunchKernelGGL((k_blkdot<TP, false>), grid, dim3(kT), 0, st, P, blockq, (size_t)0,
                       h->site_of.as<int>(), h->nsb, col, colP, Ls, sd, nbP, h->nvec, nr, out, sr, sa, sk, phase);
  HDCG_HIP(hipGetLastError());
  return DWF_OK;
}

// fine_out = base + sign P c on the interior slices too when sd > 0: there
// P is zero, so out = base (or 0 without base)
template <typename R>
__global__ void k_surface_rest(cplx<R>* out, const cplx<R>* base, size_t fe, size_t fstride, int nr, int Ls,
                               int sd) {
  const size_t total = fe * nr;
  for (size_t idx = (size_t)blockIdx.x * kT + threadIdx.x; idx < total; idx += (size_t)gridDim.x * kT) {
    const size_t r = idx / fe, i = idx - r * fe;
    const int s = (int)(i % Ls);
    if (s < sd || s >= Ls - sd) continue;
    out[r * fstride + i] = base ? base[r * fstride + i] : cmk((R)0, (R)0);
  }
}

template <typename TP, typename R = typename St<TP>::R>
int blk_promote_t(hdcg* h, const TP* P, const cplx<R>* c, int nr, cplx<R>* out,
                  const cplx<R>* base, double sign, size_t fstride, hipStream_t st, int sd = 0) {
  if (nr < 1 || h->nvec > 64) return fail(DWF_ERR_ARG, "promote: bad nr / nvec");
  const int Ls = h->op->g.Ls;
  const int col = 12 * Ls;
  const int colP = sd > 0 ? 24 * sd : col;
  const size_t nbP = (size_t)h->nsb * colP;
  constexpr int V = sizeof(TP) == 4 ? 4 : 1;  // 16-byte loads of the 16-bit subspace
  if (col % V || sd % V) return fail(DWF_ERR_ARG, "promote: 12 Ls and the surface depth must be multiples of 4");
  if constexpr (std::is_same_v<TP, bf16c>) {
    if (nr >= kPromoteMfmaRhs && blk_mfma_applies(h, P, out, fstride, sd) &&
        (!base || (reinterpret_cast<uintptr_t>(base) & 15u) == 0))
      return blk_promote_mfma(h, P, c, nr, out, base, sign, fstride, st);
  }
  if (sd > 0 && out != base) {
    const size_t fe = h->op->field_elems(1);
    size_t nbk = (fe * nr + kT - 1) / kT;
    if (nbk > 65536) nbk = 65536;
    hipLaunchKernelGGL((k_surface_rest<R>), dim3((unsigned)nbk), dim3(kT), 0, st, out, base, fe, fstride, nr, Ls, sd);
    HDCG_HIP(hipGetLastError());
  }
  for (int r0 = 0; r0 < nr; r0 += 16) {
    const int n = nr - r0 < 16 ? nr - r0 : 16;
    dim3 grid((unsigned)((nbP + kT - 1) / kT), h->Nc);
    dim3 gridv((unsigned)((nbP / V + kT - 1) / kT), h->Nc);
    const cplx<R>* cc = c + (size_t)r0 * h->Nc * h->nvec;
    cplx<R>* o = out + (size_t)r0 * fstride;
    const cplx<R>* b = base ? base + (size_t)r0 * fstride : nullptr;
    if (n <= 1)
      hipLaunchKernelGGL((k_promote<TP, 1, V>), gridv, dim3(kT), 0, st, P, cc, n, h->Nc, h->nvec, nbP, h->nsb,
                         col, colP, Ls, sd, h->site_of.as<int>(), o, b, (R)sign, fstride);
    else if (n <= 4)
      hipLaunchKernelGGL((k_promote<TP, 4, V>), gridv, dim3(kT), 0, st, P, cc, n, h->Nc, h->nvec, nbP, h->nsb,
                         col, colP, Ls, sd, h->site_of.as<int>(), o, b, (R)sign, fstride);
    else
      hipLaunchKernelGGL((k_promote<TP, 16, 1>), grid, dim3(kT), 0, st, P, cc, n, h->Nc, h->nvec, nbP, h->nsb,
                         col, colP, Ls, sd, h->site_of.as<int>(), o, b, (R)sign, fstride);
    HDCG_HIP(hipGetLastError());
  }
  return DWF_OK;
}

template <typename R>
int blk_dot(hdcg* h, const cplx<R>* P, const cplx<R>* fine, size_t fstride, const cplx<R>* blockq,
            int nr, cplx<R>* out, size_t sr, size_t sa, size_t sk, const cplx<double>* phase,
            hipStream_t st) {
  return blk_dot_t(h, P, fine, fstride, blockq, nr, out, sr, sa, sk, phase, st);
}
template <typename R>
int blk_promote(hdcg* h, const cplx<R>* P, const cplx<R>* c, int nr, cplx<R>* out,
                const cplx<R>* base, double sign, size_t fstride, hipStream_t st) {
  return blk_promote_t(h, P, c, nr, out, base, sign, fstride, st);
}
int blk_dot(hdcg* h, const bf16c* P, const c64* fine, size_t fstride, int nr, c64* out, size_t sr, size_t sa,
            size_t sk, hipStream_t st) {
  return blk_dot_t<bf16c, float>(h, P, fine, fstride, nullptr, nr, out, sr, sa, sk, nullptr, st);
}
int blk_promote(hdcg* h, const bf16c* P, const c64* c, int nr, c64* out, const c64* base, double sign,
                size_t fstride, hipStream_t st) {
  return blk_promote_t(h, P, c, nr, out, base, sign, fstride, st);
}

// The subspace in 16 bits: phi16 = phi128 rounded to the nearest bfloat16
// pair (ties to even), directly from FP64 (no intermediate float rounding)
__device__ __forceinline__ unsigned short f64_to_bf16(double d) {
  const unsigned long long u = __double_as_longlong(d);
  const unsigned sign = (unsigned)(u >> 63);
  const int e = (int)((u >> 52) & 0x7ff) - 1023 + 127;
  const unsigned long long m = u & ((1ull << 52) - 1);
  if (e <= 0) return (unsigned short)(sign << 15);              // below the normal range: signed zero
  if (e >= 255) return (unsigned short)((sign << 15) | 0x7f80u);  // above it: infinity
  unsigned v = ((unsigned)e << 7) | (unsigned)(m >> 45);
  const unsigned long long rem = m & ((1ull << 45) - 1), half = 1ull << 44;
  if (rem > half || (rem == half && (v & 1u))) ++v;  // a carry moves into the exponent
  return (unsigned short)((sign << 15) | v);
}
__global__ void k_phi_bf16(bf16c* __restrict__ out, const c128* __restrict__ in, size_t total) {
  for (size_t i = (size_t)blockIdx.x * kT + threadIdx.x; i < total; i += (size_t)gridDim.x * kT) {
    const c128 v = in[i];
    bf16c o;
    o.re = f64_to_bf16(v.re);
    o.im = f64_to_bf16(v.im);
    out[i] = o;
  }
}
int blk_phi16(hdcg* h, hipStream_t st) {
  if (h->phi128.bytes == 0) return fail(DWF_ERR_STATE, "the FP64 subspace was released after setup");
  const size_t total = (size_t)h->Nc * h->nvec * h->nb;
  HDCG_TRY(h->phi16.ensure(total * sizeof(bf16c)));
  size_t nbk = (total + kT - 1) / kT;
  if (nbk > 65536) nbk = 65536;
  hipLaunchKernelGGL(k_phi_bf16, dim3((unsigned)nbk), dim3(kT), 0, st, h->phi16.as<bf16c>(), h->phi128.as<c128>(),
                     total);
  HDCG_HIP(hipGetLastError());
  return DWF_OK;
}

// Surface-depth truncation of the subspace (Sec. IV.B, closing paragraph of
// the subspace-generation subsection): the interior slices sd <= s < Ls - sd
// of phi128 are zeroed before the block orthonormalisation, and the solve's
// complex64 / 16-bit copies keep only the 2 sd surface slices of each site
// column ([a][k][j][spin-colour][s'], s' < sd: s = s', else s = Ls - 2 sd + s'),
// so project and promote read Ls / (2 sd) times fewer subspace bytes.
__global__ void k_surface_zero(c128* __restrict__ phi, size_t total, int Ls, int sd) {
  for (size_t i = (size_t)blockIdx.x * kT + threadIdx.x; i < total; i += (size_t)gridDim.x * kT) {
    const int s = (int)(i % Ls);
    if (s >= sd && s < Ls - sd) phi[i] = cmk(0.0, 0.0);
  }
}
__global__ void k_phi_surface(c64* __restrict__ o64, bf16c* __restrict__ o16, const c128* __restrict__ in,
                              size_t total, int Ls, int sd) {
  const int w = 2 * sd;
  for (size_t i = (size_t)blockIdx.x * kT + threadIdx.x; i < total; i += (size_t)gridDim.x * kT) {
    const size_t row = i / w;
    const int sp = (int)(i - row * w);
    const c128 v = in[row * Ls + (sp < sd ? sp : Ls - w + sp)];
    if (o64) o64[i] = cmk((float)v.re, (float)v.im);
    if (o16) {
      bf16c b;
      b.re = f64_to_bf16(v.re);
      b.im = f64_to_bf16(v.im);
      o16[i] = b;
    }
  }
}
static unsigned grid_of(size_t total) {
  const size_t nbk = (total + kT - 1) / kT;
  return (unsigned)(nbk > 65536 ? 65536 : nbk);
}
int blk_surface_zero(hdcg* h, hipStream_t st) {
  const size_t total = (size_t)h->Nc * h->nvec * h->nb;
  hipLaunchKernelGGL(k_surface_zero, dim3(grid_of(total)), dim3(kT), 0, st, h->phi128.as<c128>(), total,
                     h->op->g.Ls, h->sd);
  HDCG_HIP(hipGetLastError());
  return DWF_OK;
}
static int surface_copy(hdcg* h, bool sixteen, hipStream_t st) {
  if (h->phi128.bytes == 0) return fail(DWF_ERR_STATE, "the FP64 subspace was released after setup");
  const size_t total = (size_t)h->Nc * h->nvec * h->nsb * 24 * h->sd;
  DevBuf& b = sixteen ? h->phis16 : h->phis64;
  HDCG_TRY(b.ensure(total * (sixteen ? sizeof(bf16c) : sizeof(c64))));
  hipLaunchKernelGGL(k_phi_surface, dim3(grid_of(total)), dim3(kT), 0, st, sixteen ? nullptr : b.as<c64>(),
                     sixteen ? b.as<bf16c>() : nullptr, h->phi128.as<c128>(), total, h->op->g.Ls, h->sd);
  HDCG_HIP(hipGetLastError());
  return DWF_OK;
}

// The solve's surface-only subspace copy (sd > 0), built now if missing.
int blk_surface_copies(hdcg* h, bool p16, hipStream_t st) {
  if (h->sd == 0) return DWF_OK;
  if ((p16 ? h->phis16 : h->phis64).bytes == 0) HDCG_TRY(surface_copy(h, p16, st));
  return DWF_OK;
}

// The subspace copy the solve reads: 16-bit or complex64, surface-only when
// sd > 0 (built on first use)
int solve_project(hdcg* h, bool p16, const c64* fine, size_t fstride, int nr, c64* out, size_t sr, size_t sa,
                  size_t sk, hipStream_t st) {
  if (h->sd > 0) {
    if (p16) {
      if (h->phis16.bytes == 0) HDCG_TRY(surface_copy(h, true, st));
      return blk_dot_t<bf16c, float>(h, h->phis16.as<bf16c>(), fine, fstride, nullptr, nr, out, sr, sa, sk, nullptr,
                                     st, h->sd);
    }
    if (h->phis64.bytes == 0) HDCG_TRY(surface_copy(h, false, st));
    return blk_dot_t<c64, float>(h, h->phis64.as<c64>(), fine, fstride, nullptr, nr, out, sr, sa, sk, nullptr, st,
                                 h->sd);
  }
  if (p16) {
    if (h->phi16.bytes == 0) HDCG_TRY(blk_phi16(h, st));
    return blk_dot_t<bf16c, float>(h, h->phi16.as<bf16c>(), fine, fstride, nullptr, nr, out, sr, sa, sk, nullptr, st);
  }
  return blk_dot_t<c64, float>(h, h->phi64.as<c64>(), fine, fstride, nullptr, nr, out, sr, sa, sk, nullptr, st);
}
int solve_promote(hdcg* h, bool p16, const c64* c, int nr, c64* out, const c64* base, double sign, size_t fstride,
                  hipStream_t st) {
  if (h->sd > 0) {
    if (p16) {
      if (h->phis16.bytes == 0) HDCG_TRY(surface_copy(h, true, st));
      return blk_promote_t(h, h->phis16.as<bf16c>(), c, nr, out, base, sign, fstride, st, h->sd);
    }
    if (h->phis64.bytes == 0) HDCG_TRY(surface_copy(h, false, st));
    return blk_promote_t(h, h->phis64.as<c64>(), c, nr, out, base, sign, fstride, st, h->sd);
  }
  if (p16) {
    if (h->phi16.bytes == 0) HDCG_TRY(blk_phi16(h, st));
    return blk_promote_t(h, h->phi16.as<bf16c>(), c, nr, out, base, sign, fstride, st);
  }
  return blk_promote_t(h, h->phi64.as<c64>(), c, nr, out, base, sign, fstride, st);
}

int blk_cholqr_step(hdcg* h, hipStream_t st) {
  const int n = h->nvec;
  const size_t n2 = (size_t)n * n;
  HDCG_TRY(h->gram.ensure(sizeof(c128) * h->Nc * n2));
  HDCG_TRY(h->rinv.ensure(sizeof(c128) * h->Nc * n2));
  c128* phi = h->phi128.as<c128>();
  // G[a][k'][k] = <phi_k', phi_k> on block a
  HDCG_TRY(blk_dot<double>(h, phi, nullptr, 0, phi, n, h->gram.as<c128>(), 1, n2, n, nullptr, st));
  hipLaunchKernelGGL(k_chol_inv, dim3(h->Nc), dim3(64), n2 * sizeof(c128), st, h->gram.as<c128>(),
                     h->rinv.as<c128>(), n, h->flag.as<int>());
  HDCG_HIP(hipGetLastError());
  dim3 grid((unsigned)((h->nb + 31) / 32), h->Nc);
  hipLaunchKernelGGL(k_gs_apply, grid, dim3(kT), (size_t)n * 32 * sizeof(c128), st, phi,
                     h->rinv.as<c128>(), n, h->nb);
  HDCG_HIP(hipGetLastError());
  return DWF_OK;
}

template <typename R>
int crs_apply(hdcg* h, const cplx<R>* AT, const cplx<R>* in, cplx<R>* out, int nr, hipStream_t st) {
  if (h->nvec > kCT) return fail(DWF_ERR_ARG, "nvec too large for the coarse mat-vec");
  if (nr == 1) {
    if constexpr (sizeof(R) == 4) {
      if (h->nvec <= kStageNvec) {
        hipLaunchKernelGGL((k_capply_staged<16>), dim3(h->Nc), dim3(kCT), 0, st, AT, h->nbr.as<int>(), in, out,
                           h->Nc, h->nvec);
        HDCG_HIP(hipGetLastError());
        return DWF_OK;
      }
    }
    hipLaunchKernelGGL((k_capply<R, 1, 16>), dim3(h->Nc, 1), dim3(kCT), 0, st, AT, h->nbr.as<int>(), in, out,
                       h->Nc, h->nvec, nr);
  } else if (h->nvec % 4 == 0 && h->nvec <= 64) {
    // several right-hand sides: the FP32 (complex64) or FP64 (complex128)
    // MFMA form, all of up to 16 per pass over A
    const int* nbr = h->nbr.as<int>();
    switch ((h->nvec + 15) / 16) {
      case 1: launch_cmfma_nt<R, 1>(AT, nbr, in, out, h->Nc, h->nvec, nr, st); break;
      case 2: launch_cmfma_nt<R, 2>(AT, nbr, in, out, h->Nc, h->nvec, nr, st); break;
      case 3: launch_cmfma_nt<R, 3>(AT, nbr, in, out, h->Nc, h->nvec, nr, st); break;
      default: launch_cmfma_nt<R, 4>(AT, nbr, in, out, h->Nc, h->nvec, nr, st); break;
    }
  } else if (sizeof(R) == 8 && nr > 2) {
    // complex128 with many right-hand sides (the second deflation level's
    // setup): eight per pass over A, so A is read nr / 8 times
    hipLaunchKernelGGL((k_capply<R, 8, 2>), dim3(h->Nc, (nr + 7) / 8), dim3(kCT), 0, st, AT, h->nbr.as<int>(), in,
                       out, h->Nc, h->nvec, nr);
  } else if (sizeof(R) == 4 && nr > 8) {
    // complex64, 9-16 right-hand sides: all of them per pass over A
    hipLaunchKernelGGL((k_capply<R, 16, 2>), dim3(h->Nc, (nr + 15) / 16), dim3(kCT), 0, st, AT, h->nbr.as<int>(),
                       in, out, h->Nc, h->nvec, nr);
  } else if (sizeof(R) == 4 && nr > 4) {
    hipLaunchKernelGGL((k_capply<R, 8, 4>), dim3(h->Nc, (nr + 7) / 8), dim3(kCT), 0, st, AT, h->nbr.as<int>(), in,
                       out, h->Nc, h->nvec, nr);
  } else {
    constexpr int NR = sizeof(R) == 8 ? 2 : 4;
    hipLaunchKernelGGL((k_capply<R, NR, 8>), dim3(h->Nc, (nr + NR - 1) / NR), dim3(kCT), 0, st, AT,
                       h->nbr.as<int>(), in, out, h->Nc, h->nvec, nr);
  }
  HDCG_HIP(hipGetLastError());
  return DWF_OK;
}

int crs_idft(hdcg* h, c128* Y, const c128 finv[4][9], hipStream_t st) {
  const size_t total = (size_t)h->Nc * 27 * h->nvec * h->nvec;
  for (int mu = 0; mu < 4; ++mu) {
    const c128* f = finv[mu];
    hipLaunchKernelGGL(k_idft_dim, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, st, Y,
                       h->nvec * h->nvec, h->Nc, mu, f[0], f[1], f[2], f[3], f[4], f[5], f[6], f[7],
                       f[8]);
    HDCG_HIP(hipGetLastError());
  }
  return DWF_OK;
}

int crs_transpose(hdcg* h, bool fp64, hipStream_t st) {
  const size_t total = (size_t)h->Nc * kStencil * h->nvec * h->nvec;
  if (fp64)
    HDCG_TRY(h->AT128.ensure(total * sizeof(c128)));
  else
    HDCG_TRY(h->AT64.ensure(total * sizeof(c64)));
  hipLaunchKernelGGL(k_transpose, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, st,
                     h->A128.as<c128>(), fp64 ? h->AT128.as<c128>() : nullptr,
                     fp64 ? nullptr : h->AT64.as<c64>(), h->nvec, total);
  HDCG_HIP(hipGetLastError());
  return DWF_OK;
}

#define INST(R)                                                                                    \
  template int blk_phi_layout<R>(hdcg*, cplx<R>*, const cplx<double>*, bool, int, hipStream_t);   \
  template int blk_dot<R>(hdcg*, const cplx<R>*, const cplx<R>*, size_t, const cplx<R>*, int,     \
                          cplx<R>*, size_t, size_t, size_t, const cplx<double>*, hipStream_t);     \
  template int blk_promote<R>(hdcg*, const cplx<R>*, const cplx<R>*, int, cplx<R>*,              \
                              const cplx<R>*, double, size_t, hipStream_t);                       \
  template int crs_apply<R>(hdcg*, const cplx<R>*, const cplx<R>*, cplx<R>*, int, hipStream_t);
INST(double)
INST(float)

}  // namespace hdk
