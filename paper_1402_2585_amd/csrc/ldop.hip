// Second deflation level of the little Dirac operator (Sec. V.B, "Little
// Dirac operator deflation") and the pre-diagonalised third level.
//
// Global coarse vectors (no further blocking): the Nvec that come free with
// the blocked subspace, w_k[a][j] = delta_jk / sqrt(Nc), and n_extra more
// from shifted inverse iteration on A started from caller-drawn coarse
// noise.  They are orthonormalised (Cholesky-QR twice, FP64), E = W^+ A W is
// diagonalised on the host (cyclic Jacobi, E = U D U^+), and Z = W U, A Z
// kept in complex128 and complex64.  The coarse solve then runs deflated CG:
// x0 = Z D^-1 Z^+ b and search directions p = r + beta p - Z D^-1 (AZ)^+ r.
#include <algorithm>
#include <cmath>
#include <complex>
#include <cstdio>
#include <vector>

#include "hdcg_impl.h"

namespace hdk {

namespace {

constexpr int kT = 256;

// G[i][j] = sum_n conj(X_i[n]) Y_j[n] in FP64; one workgroup per (i, j); with
// herm set only j >= i is summed and G[j][i] = conj(G[i][j]) (X == Y)
template <typename R>
__global__ void __launch_bounds__(kT) k_gram(const cplx<R>* __restrict__ X, const cplx<R>* __restrict__ Y, int ny,
                                             size_t N, c128* __restrict__ G, int herm) {
  const int i = blockIdx.x, j = blockIdx.y;
  if (herm && j < i) return;
  const cplx<R>* x = X + (size_t)i * N;
  const cplx<R>* y = Y + (size_t)j * N;
  double re = 0.0, im = 0.0;
  for (size_t n = threadIdx.x; n < N; n += kT) {
    const cplx<R> a = x[n], b = y[n];
    re += (double)a.re * b.re + (double)a.im * b.im;
    im += (double)a.re * b.im - (double)a.im * b.re;
  }
  double v[2] = {re, im};
  __shared__ double lds[32];
  block_sum<2>(v, lds);
  if (threadIdx.x == 0) {
    G[(size_t)i * ny + j] = cmk(v[0], v[1]);
    if (herm && j != i) G[(size_t)j * ny + i] = cmk(v[0], -v[1]);
  }
}

// out_j[n] = sum_i X_i[n] M[i][j], j < ny, i < nx
template <typename Rin, typename Rout>
__global__ void __launch_bounds__(kT) k_expand(const cplx<Rin>* __restrict__ X, const c128* __restrict__ M, int nx,
                                               int ny, size_t N, cplx<Rout>* __restrict__ out) {
  const size_t n = (size_t)blockIdx.x * kT + threadIdx.x;
  const int j = blockIdx.y;
  if (n >= N) return;
  double re = 0.0, im = 0.0;
  for (int i = 0; i < nx; ++i) {
    const cplx<Rin> a = X[(size_t)i * N + n];
    const c128 m = M[(size_t)i * ny + j];
    re += (double)a.re * m.re - (double)a.im * m.im;
    im += (double)a.re * m.im + (double)a.im * m.re;
  }
  out[(size_t)j * N + n] = cmk((Rout)re, (Rout)im);
}

// W[k] = e_k / sqrt(Nc) on every block: w_k[a][j] = delta_jk / sqrt(Nc)
__global__ void k_free_vectors(c128* __restrict__ W, int Nc, int nvec) {
  const size_t N = (size_t)Nc * nvec;
  const size_t e = (size_t)blockIdx.x * kT + threadIdx.x;
  if (e >= N * nvec) return;
  const int k = (int)(e / N);
  const int j = (int)(e % nvec);
  W[e] = cmk(j == k ? 1.0 / std::sqrt((double)Nc) : 0.0, 0.0);
}

// c[rhs][k] = (V_k, r_rhs) / D[k]; one workgroup per (k, slice, rhs).  With
// one slice the workgroup writes c; with S slices (long vectors: a single
// workgroup per k would leave most CUs idle) it writes its partial sum to
// part[rhs][k][slice] and k_defl_coef_sum adds the S partials in order.
template <typename R>
__global__ void __launch_bounds__(kT) k_defl_coef(const cplx<R>* __restrict__ V, const cplx<R>* __restrict__ r,
                                                  const double* __restrict__ D, int ng, size_t N,
                                                  c128* __restrict__ c, c128* __restrict__ part) {
  const int k = blockIdx.x, sl = blockIdx.y, S = gridDim.y, rhs = blockIdx.z;
  const size_t chunk = (N + S - 1) / S;
  const size_t n0 = (size_t)sl * chunk, n1 = n0 + chunk < N ? n0 + chunk : N;
  const cplx<R>* v = V + (size_t)k * N;
  const cplx<R>* x = r + (size_t)rhs * N;
  double re = 0.0, im = 0.0;
  // four strided elements per trip, loads first
  size_t n = n0 + threadIdx.x;
  for (; n + 3 * kT < n1; n += 4 * kT) {
    cplx<R> a[4], b[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      a[u] = v[n + u * kT];
      b[u] = x[n + u * kT];
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      re += (double)a[u].re * b[u].re + (double)a[u].im * b[u].im;
      im += (double)a[u].re * b[u].im - (double)a[u].im * b[u].re;
    }
  }
  for (; n < n1; n += kT) {
    const cplx<R> a = v[n], b = x[n];
    re += (double)a.re * b.re + (double)a.im * b.im;
    im += (double)a.re * b.im - (double)a.im * b.re;
  }
  double s[2] = {re, im};
  __shared__ double lds[32];
  block_sum<2>(s, lds);
  if (threadIdx.x != 0) return;
  if (S == 1)
    c[(size_t)rhs * ng + k] = cmk(s[0] / D[k], s[1] / D[k]);
  else
    part[((size_t)rhs * ng + k) * S + sl] = cmk(s[0], s[1]);
}

__global__ void k_defl_coef_sum(const c128* __restrict__ part, const double* __restrict__ D, int ng, int S,
                                c128* __restrict__ c) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x, rhs = blockIdx.y;
  if (k >= ng) return;
  const c128* p = part + ((size_t)rhs * ng + k) * S;
  double re = 0.0, im = 0.0;
  for (int sl = 0; sl < S; ++sl) {
    re += p[sl].re;
    im += p[sl].im;
  }
  c[(size_t)rhs * ng + k] = cmk(re / D[k], im / D[k]);
}

// out = (use_r ? r : 0) + (num ? num/den * out : 0) + sign * sum_k Z_k c[rhs][k].
// A workgroup takes 64 elements; its four waves split the sum over k and
// meet in LDS (more workgroups in flight and four times shorter load chains).
constexpr int kMaxGlobal = 1024;
constexpr int kDefE = 64;
template <typename R>
__global__ void __launch_bounds__(kT) k_defl_apply(cplx<R>* __restrict__ out, const cplx<R>* __restrict__ r,
                                                   const double* __restrict__ num, const double* __restrict__ den,
                                                   const cplx<R>* __restrict__ Z, const c128* __restrict__ c, int ng,
                                                   size_t N, double sign, int use_r) {
  __shared__ c128 cs[kMaxGlobal];
  __shared__ double part[kT / kDefE][kDefE][2];
  const int rhs = blockIdx.y;
  for (int k = threadIdx.x; k < ng; k += kT) cs[k] = c[(size_t)rhs * ng + k];
  __syncthreads();
  const int el = threadIdx.x % kDefE, slice = threadIdx.x / kDefE;
  constexpr int kSlices = kT / kDefE;
  const size_t n = (size_t)blockIdx.x * kDefE + el;
  double zr = 0.0, zi = 0.0;
  if (n < N) {
    for (int k = slice; k < ng; k += kSlices) {
      const cplx<R> z = Z[(size_t)k * N + n];
      zr += (double)z.re * cs[k].re - (double)z.im * cs[k].im;
      zi += (double)z.re * cs[k].im + (double)z.im * cs[k].re;
    }
  }
  part[slice][el][0] = zr;
  part[slice][el][1] = zi;
  __syncthreads();
  if (slice != 0 || n >= N) return;
  for (int q = 1; q < kSlices; ++q) {
    zr += part[q][el][0];
    zi += part[q][el][1];
  }
  const size_t e = (size_t)rhs * N + n;
  double re = 0.0, im = 0.0;
  if (use_r) {
    re = r[e].re;
    im = r[e].im;
  }
  if (num) {
    const double d = den[rhs];
    const double beta = d != 0.0 ? num[rhs] / d : 0.0;
    re += beta * out[e].re;
    im += beta * out[e].im;
  }
  out[e] = cmk((R)(re + sign * zr), (R)(im + sign * zi));
}

using cd = std::complex<double>;

// Cholesky G = R^+ R (upper R) of an n x n Hermitian matrix, in place into R;
// false when G is not positive definite
bool cholesky_upper(const std::vector<cd>& G, int n, std::vector<cd>& R) {
  R.assign((size_t)n * n, cd(0.0));
  for (int i = 0; i < n; ++i) {
    cd s = G[(size_t)i * n + i];
    for (int k = 0; k < i; ++k) s -= std::conj(R[(size_t)k * n + i]) * R[(size_t)k * n + i];
    if (!(s.real() > 0.0) || !std::isfinite(s.real())) return false;
    const double d = std::sqrt(s.real());
    R[(size_t)i * n + i] = d;
    for (int j = i + 1; j < n; ++j) {
      cd t = G[(size_t)i * n + j];
      for (int k = 0; k < i; ++k) t -= std::conj(R[(size_t)k * n + i]) * R[(size_t)k * n + j];
      R[(size_t)i * n + j] = t / d;
    }
  }
  return true;
}

// inverse of an upper-triangular matrix
std::vector<cd> upper_inverse(const std::vector<cd>& R, int n) {
  std::vector<cd> X((size_t)n * n, cd(0.0));
  for (int j = 0; j < n; ++j) {
    X[(size_t)j * n + j] = 1.0 / R[(size_t)j * n + j];
    for (int i = j - 1; i >= 0; --i) {
      cd s = 0.0;
      for (int k = i + 1; k <= j; ++k) s += R[(size_t)i * n + k] * X[(size_t)k * n + j];
      X[(size_t)i * n + j] = -s / R[(size_t)i * n + i];
    }
  }
  return X;
}

// Hermitian eigen-decomposition by cyclic Jacobi rotations: E = U diag(d) U^+,
// eigenvalues ascending, U column-major in the sense U[i * n + k] = U_ik.
void jacobi_eigh(std::vector<cd> A, int n, std::vector<double>& d, std::vector<cd>& U) {
  U.assign((size_t)n * n, cd(0.0));
  for (int i = 0; i < n; ++i) U[(size_t)i * n + i] = 1.0;
  auto a = [&](int i, int j) -> cd& { return A[(size_t)i * n + j]; };
  for (int sweep = 0; sweep < 100; ++sweep) {
    double off = 0.0, tot = 0.0;
    for (int i = 0; i < n; ++i)
      for (int j = 0; j < n; ++j) {
        const double v = std::norm(a(i, j));
        tot += v;
        if (i != j) off += v;
      }
    if (off <= 1e-30 * tot) break;
    for (int p = 0; p < n - 1; ++p)
      for (int q = p + 1; q < n; ++q) {
        const cd apq = a(p, q);
        const double mag = std::abs(apq);
        if (mag == 0.0) continue;
        // rotate the 2x2 block [[a_pp, a_pq], [conj(a_pq), a_qq]] to diagonal
        const cd ph = apq / mag;  // a_pq = mag e^{i phi}
        const double app = a(p, p).real(), aqq = a(q, q).real();
        const double theta = 0.5 * std::atan2(2.0 * mag, aqq - app);
        const double c = std::cos(theta), s = std::sin(theta);
        // columns p, q of the rotation: J = [[c, s ph], [-s conj(ph), c]]
        for (int k = 0; k < n; ++k) {  // A <- A J
          const cd akp = a(k, p), akq = a(k, q);
          a(k, p) = c * akp - s * std::conj(ph) * akq;
          a(k, q) = s * ph * akp + c * akq;
        }
        for (int k = 0; k < n; ++k) {  // A <- J^+ A
          const cd apk = a(p, k), aqk = a(q, k);
          a(p, k) = c * apk - s * ph * aqk;
          a(q, k) = s * std::conj(ph) * apk + c * aqk;
        }
        for (int k = 0; k < n; ++k) {  // U <- U J
          const cd ukp = U[(size_t)k * n + p], ukq = U[(size_t)k * n + q];
          U[(size_t)k * n + p] = c * ukp - s * std::conj(ph) * ukq;
          U[(size_t)k * n + q] = s * ph * ukp + c * ukq;
        }
      }
  }
  d.resize(n);
  for (int i = 0; i < n; ++i) d[i] = a(i, i).real();
  // ascending order
  std::vector<int> idx(n);
  for (int i = 0; i < n; ++i) idx[i] = i;
  std::sort(idx.begin(), idx.end(), [&](int x, int y) { return d[x] < d[y]; });
  std::vector<double> d2(n);
  std::vector<cd> U2((size_t)n * n);
  for (int k = 0; k < n; ++k) {
    d2[k] = d[idx[k]];
    for (int i = 0; i < n; ++i) U2[(size_t)i * n + k] = U[(size_t)i * n + idx[k]];
  }
  d.swap(d2);
  U.swap(U2);
}

int gram(const c128* X, const c128* Y, int nx, int ny, size_t N, bool herm, DevBuf& Gd, std::vector<cd>& G,
         hipStream_t st) {
  HDCG_TRY(Gd.ensure(sizeof(c128) * nx * ny));
  hipLaunchKernelGGL((k_gram<double>), dim3(nx, ny), dim3(kT), 0, st, X, Y, ny, N, Gd.as<c128>(), herm ? 1 : 0);
  HDCG_HIP(hipGetLastError());
  G.resize((size_t)nx * ny);
  HDCG_HIP(hipMemcpyAsync(G.data(), Gd.ptr, sizeof(c128) * nx * ny, hipMemcpyDeviceToHost, st));
  HDCG_HIP(hipStreamSynchronize(st));
  return DWF_OK;
}

template <typename Rout>
int expand(const c128* X, const std::vector<cd>& M, int nx, int ny, size_t N, DevBuf& Md, cplx<Rout>* out,
           hipStream_t st) {
  HDCG_TRY(Md.ensure(sizeof(c128) * nx * ny));
  HDCG_HIP(hipMemcpyAsync(Md.ptr, M.data(), sizeof(c128) * nx * ny, hipMemcpyHostToDevice, st));
  hipLaunchKernelGGL((k_expand<double, Rout>), dim3((unsigned)((N + kT - 1) / kT), ny), dim3(kT), 0, st, X,
                     Md.as<c128>(), nx, ny, N, out);
  HDCG_HIP(hipGetLastError());
  HDCG_HIP(hipStreamSynchronize(st));  // M is host memory reused by the caller
  return DWF_OK;
}

}  // namespace

template <typename R>
int ldop_coef(hdcg* h, const cplx<R>* V, const cplx<R>* r, int nr, hipStream_t st) {
  const size_t N = (size_t)h->Nc * h->nvec;
  // up to 16 slices per vector, each of at least 128 elements
  const int S = (int)std::max<size_t>(1, std::min<size_t>(16, N / 128));
  c128* part = nullptr;
  if (S > 1) {
    HDCG_TRY(h->ldpart.ensure(sizeof(c128) * (size_t)nr * h->ng * S));
    part = h->ldpart.as<c128>();
  }
  hipLaunchKernelGGL((k_defl_coef<R>), dim3(h->ng, S, nr), dim3(kT), 0, st, V, r, h->ldD.as<double>(), h->ng, N,
                     h->ldc.as<c128>(), part);
  HDCG_HIP(hipGetLastError());
  if (S > 1) {
    hipLaunchKernelGGL(k_defl_coef_sum, dim3((h->ng + 255) / 256, nr), dim3(256), 0, st, part, h->ldD.as<double>(),
                       h->ng, S, h->ldc.as<c128>());
    HDCG_HIP(hipGetLastError());
  }
  return DWF_OK;
}

template <typename R>
int ldop_apply(hdcg* h, cplx<R>* out, const cplx<R>* r, const double* num, const double* den, const cplx<R>* Z,
               int nr, double sign, bool use_r, hipStream_t st) {
  const size_t N = (size_t)h->Nc * h->nvec;
  hipLaunchKernelGGL((k_defl_apply<R>), dim3((unsigned)((N + kDefE - 1) / kDefE), nr), dim3(kT), 0, st, out, r, num, den, Z,
                     h->ldc.as<c128>(), h->ng, N, sign, use_r ? 1 : 0);
  HDCG_HIP(hipGetLastError());
  return DWF_OK;
}
template int ldop_coef<float>(hdcg*, const c64*, const c64*, int, hipStream_t);
template int ldop_coef<double>(hdcg*, const c128*, const c128*, int, hipStream_t);
template int ldop_apply<float>(hdcg*, c64*, const c64*, const double*, const double*, const c64*, int, double, bool,
                               hipStream_t);
template int ldop_apply<double>(hdcg*, c128*, const c128*, const double*, const double*, const c128*, int, double,
                                bool, hipStream_t);

int ldop_build(hdcg* h, int n_extra, const c128* noise, double shift, int n_steps, double tol, int maxiter,
               hipStream_t st) {
  const int nv = h->nvec;
  const int ng = nv + n_extra;
  if (n_extra < 0 || ng > kMaxGlobal) return fail(DWF_ERR_ARG, "n_extra must be in 0 .. 1024 - Nvec");
  if (n_extra > 0 && !noise) return fail(DWF_ERR_ARG, "n_extra > 0 needs the coarse noise vectors");
  if (!(tol > 0.0) || n_steps < 0 || shift < 0.0) return fail(DWF_ERR_ARG, "tol > 0, n_steps >= 0, shift >= 0");
  const size_t N = (size_t)h->Nc * nv;
  if ((size_t)ng > N) return fail(DWF_ERR_ARG, "more global vectors than coarse unknowns");
  h->ng = 0;
  DevBuf W, AW, tmp, Gd, Md;
  HDCG_TRY(W.ensure(sizeof(c128) * N * ng));
  HDCG_TRY(AW.ensure(sizeof(c128) * N * ng));
  c128* Wp = W.as<c128>();
  hipLaunchKernelGGL(k_free_vectors, dim3((unsigned)((N * nv + kT - 1) / kT)), dim3(kT), 0, st, Wp, h->Nc, nv);
  HDCG_HIP(hipGetLastError());
  if (n_extra > 0) {
    c128* X = Wp + N * nv;
    HDCG_HIP(hipMemcpyAsync(X, noise, sizeof(c128) * N * n_extra, hipMemcpyDeviceToDevice, st));
    // shifted inverse iteration, groups of up to 16 share one coarse CG
    // (its mat-vec reads A once per 16 right-hand sides)
    const int G = 16;
    HDCG_TRY(tmp.ensure(sizeof(c128) * N * G));
    double* nrm = nullptr;
    HDCG_TRY(h->ldc.ensure(sizeof(c128) * 64 * kMaxGlobal));
    nrm = reinterpret_cast<double*>(h->ldc.ptr);  // scratch for the norms
    for (int k0 = 0; k0 < n_extra; k0 += G) {
      const int g = std::min(G, n_extra - k0);
      c128* v = X + N * k0;
      for (int s = 0; s < n_steps; ++s) {
        int it = 0;
        HDCG_TRY(coarse_cg_shifted(h, tmp.as<c128>(), v, g, shift, tol, maxiter, &it, st));
        HDCG_TRY(b_norm2<double>(Red{h->op->red.partials.as<double>(), h->op->red.counters.as<unsigned>()},
                                 tmp.as<c128>(), N, g, nrm, st));
        HDCG_TRY(b_scale_copy<double, double>(v, tmp.as<c128>(), nrm, true, N, g, st));
      }
    }
  }
  // orthonormalise: Cholesky-QR twice in FP64 (W <- W R^-1)
  std::vector<cd> Gh, R;
  for (int pass = 0; pass < 2; ++pass) {
    HDCG_TRY(gram(Wp, Wp, ng, ng, N, true, Gd, Gh, st));
    if (!cholesky_upper(Gh, ng, R))
      return fail(DWF_ERR_NUMERIC, "global coarse vectors are linearly dependent");
    const std::vector<cd> Ri = upper_inverse(R, ng);
    HDCG_TRY(expand<double>(Wp, Ri, ng, ng, N, Md, AW.as<c128>(), st));
    HDCG_HIP(hipMemcpyAsync(Wp, AW.ptr, sizeof(c128) * N * ng, hipMemcpyDeviceToDevice, st));
  }
  // third level: E = W^+ A W, diagonalised
  HDCG_TRY(ensure_at128_impl(h, st));
  HDCG_TRY(crs_apply<double>(h, h->AT128.as<c128>(), Wp, AW.as<c128>(), ng, st));
  std::vector<cd> E;
  HDCG_TRY(gram(Wp, AW.as<c128>(), ng, ng, N, false, Gd, E, st));
  for (int i = 0; i < ng; ++i)
    for (int j = i; j < ng; ++j) {
      const cd m = 0.5 * (E[(size_t)i * ng + j] + std::conj(E[(size_t)j * ng + i]));
      E[(size_t)i * ng + j] = m;
      E[(size_t)j * ng + i] = std::conj(m);
    }
  std::vector<double> d;
  std::vector<cd> U;
  jacobi_eigh(E, ng, d, U);
  if (!(d[0] > 0.0)) return fail(DWF_ERR_NUMERIC, "coarse operator not positive on the global vectors");
  HDCG_TRY(h->ldZ128.ensure(sizeof(c128) * N * ng));
  HDCG_TRY(h->ldAZ128.ensure(sizeof(c128) * N * ng));
  HDCG_TRY(h->ldZ64.ensure(sizeof(c64) * N * ng));
  HDCG_TRY(h->ldAZ64.ensure(sizeof(c64) * N * ng));
  HDCG_TRY(expand<double>(Wp, U, ng, ng, N, Md, h->ldZ128.as<c128>(), st));
  HDCG_TRY(expand<double>(AW.as<c128>(), U, ng, ng, N, Md, h->ldAZ128.as<c128>(), st));
  HDCG_TRY(expand<float>(Wp, U, ng, ng, N, Md, h->ldZ64.as<c64>(), st));
  HDCG_TRY(expand<float>(AW.as<c128>(), U, ng, ng, N, Md, h->ldAZ64.as<c64>(), st));
  HDCG_TRY(h->ldD.ensure(sizeof(double) * ng));
  HDCG_HIP(hipMemcpyAsync(h->ldD.ptr, d.data(), sizeof(double) * ng, hipMemcpyHostToDevice, st));
  HDCG_TRY(h->ldc.ensure(sizeof(c128) * 64 * kMaxGlobal));
  HDCG_HIP(hipStreamSynchronize(st));
  h->ldDh = d;
  h->ng = ng;
  return DWF_OK;
}

}  // namespace hdk
