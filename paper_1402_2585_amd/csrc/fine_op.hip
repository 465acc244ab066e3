// Fine domain-wall operator kernels for gfx950.
//
// One hop stage = one launch.  A workgroup owns `spw` output sites of one
// checkerboard (a small 4D block of sites, or consecutive sites) and all Ls
// slices of each (thread = (site, s)).  The Ls threads of a site copy its
// eight links into LDS once, the neighbour spinors of a site column are
// contiguous runs of Ls complex numbers per component, and each thread
// issues the loads of several neighbour spinors before any arithmetic, so
// many bytes are in flight per wave and few sites need to be resident per
// CU: the neighbour columns a CU touches then stay in its XCD's L2 between
// their consumers.
//
// Epilogues (the fifth-dimension factors of M_pc, Sec. IV):
//   EPI_INV  out = M_5^-1 (Dh in)          or M_5^-+ (Dh^+ in)   [dense in s]
//   EPI_SUB  out = M_5 c - 1/4 (Dh in)      or M_5^+ c - 1/4 (Dh^+ in)
// EPI_INV stages the hop result in LDS and solves the Ls x Ls system per
// (site, component) with the O(Ls) recurrence of the closed-form inverse.
#include <algorithm>
#include <type_traits>

#include "fine_op.h"

namespace hdk {

enum { EPI_INV = 0, EPI_SUB = 1 };

// ------------------------------------------------------------ coordinates --
struct Site {
  int x, y, z, t, xh;
  int rest;  // y + Y (z + Z t)
  int zt;    // z + Z t
};

__device__ __forceinline__ Site site_coords(int v, int parity, const Geom& g) {
  Site c;
  c.xh = v % g.Xh;
  c.rest = v / g.Xh;
  c.y = c.rest % g.Y;
  c.zt = c.rest / g.Y;
  c.z = c.zt % g.Z;
  c.t = c.zt / g.Z;
  c.x = 2 * c.xh + ((c.y + c.z + c.t + parity) & 1);
  return c;
}

// ------------------------------------------------------------ gauge import -
__global__ void gauge_import_kernel(const c128* __restrict__ U, c128* __restrict__ G128,
                                    c64* __restrict__ G64, Geom g, double4 bcxy, double4 bczt) {
  const int idx = blockIdx.x * blockDim.x + threadIdx.x;  // (parity, cb)
  if (idx >= 2 * g.Vh) return;
  const int p = idx / g.Vh, v = idx % g.Vh;
  const Site c = site_coords(v, p, g);
  const int L[4] = {g.X, g.Y, g.Z, g.T};
  const int xc[4] = {c.x, c.y, c.z, c.t};
  const double zr[4] = {bcxy.x, bcxy.z, bczt.x, bczt.z};
  const double zi[4] = {bcxy.y, bcxy.w, bczt.y, bczt.w};
  const size_t lex = c.x + (size_t)g.X * (c.y + (size_t)g.Y * (c.z + (size_t)g.Z * c.t));
  c128* out128 = G128 + (size_t)idx * 72;
  c64* out64 = G64 + (size_t)idx * 72;
  for (int mu = 0; mu < 4; ++mu) {
    // forward link U_mu(x), phase when the hop x -> x+mu wraps
    const c128 zf = (xc[mu] == L[mu] - 1) ? cmk(zr[mu], zi[mu]) : cmk(1.0, 0.0);
    const c128* u = U + (lex * 4 + mu) * 9;
    for (int e = 0; e < 9; ++e) {
      c128 w = zf * u[e];
      out128[mu * 9 + e] = w;
      out64[mu * 9 + e] = cmk((float)w.re, (float)w.im);
    }
    // backward link U_mu(x-mu)^+, conj phase when the hop x -> x-mu wraps
    int xm[4] = {c.x, c.y, c.z, c.t};
    xm[mu] = (xm[mu] == 0) ? L[mu] - 1 : xm[mu] - 1;
    const size_t lexm = xm[0] + (size_t)g.X * (xm[1] + (size_t)g.Y * (xm[2] + (size_t)g.Z * xm[3]));
    const c128 zb = (xc[mu] == 0) ? cmk(zr[mu], -zi[mu]) : cmk(1.0, 0.0);
    const c128* ub = U + (lexm * 4 + mu) * 9;
    for (int a = 0; a < 3; ++a)
      for (int b = 0; b < 3; ++b) {
        c128 w = zb * conj(ub[b * 3 + a]);
        out128[(4 + mu) * 9 + a * 3 + b] = w;
        out64[(4 + mu) * 9 + a * 3 + b] = cmk((float)w.re, (float)w.im);
      }
  }
}

// ----------------------------------------------------------- field layout --
// canonical [rhs][s][cb][c]  <->  native [rhs][cb][c][s]
template <typename R, bool TO_NATIVE>
__global__ void field_layout_kernel(cplx<R>* __restrict__ dst, const cplx<R>* __restrict__ src,
                                    int Ls, int Vh, size_t total) {
  const size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= total) return;
  // idx enumerates the native layout
  const int s = idx % Ls;
  const int c = (idx / Ls) % 12;
  const size_t cb = (idx / ((size_t)Ls * 12)) % Vh;
  const size_t rhs = idx / ((size_t)Ls * 12 * Vh);
  const size_t can = ((rhs * Ls + s) * Vh + cb) * 12 + c;
  if (TO_NATIVE)
    dst[idx] = src[can];
  else
    dst[can] = src[idx];
}

// dst (stored as Td) = src (stored as Ts), rounded to nearest (even)
template <typename Td, typename Ts>
__global__ void convert_kernel(Td* __restrict__ dst, const Ts* __restrict__ src, size_t n) {
  using Rd = typename St<Td>::R;
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (size_t)gridDim.x * blockDim.x) {
    const auto v = St<Ts>::ld(src + i);
    St<Td>::st(dst + i, cmk((Rd)v.re, (Rd)v.im));
  }
}

// ------------------------------------------------------------- hop stage --
// Spin structure in the chiral basis: gamma_mu = [[0, A_mu], [A_mu^+, 0]]
// with A_x = -i sigma_x, A_y = -i sigma_y, A_z = -i sigma_z, A_t = 1.
// (1 + sg*gamma_mu) psi = (h ; sg A^+ h) with h = u + sg A l, where u, l are
// the upper and lower spin pairs of psi: the hop moves 6 complex numbers
// through the SU(3) link instead of 12.
template <typename R, int MU>
__device__ __forceinline__ void apply_A(const cplx<R> l0, const cplx<R> l1, cplx<R>& a0,
                                        cplx<R>& a1) {
  if (MU == 0) {  // A_x l = (-i l1, -i l0)
    a0 = timesMinusI(l1);
    a1 = timesMinusI(l0);
  } else if (MU == 1) {  // A_y l = (-l1, l0)
    a0 = cmk(-l1.re, -l1.im);
    a1 = l0;
  } else if (MU == 2) {  // A_z l = (-i l0, i l1)
    a0 = timesMinusI(l0);
    a1 = timesI(l1);
  } else {  // A_t l = l
    a0 = l0;
    a1 = l1;
  }
}
template <typename R, int MU>
__device__ __forceinline__ void apply_Adag(const cplx<R> h0, const cplx<R> h1, cplx<R>& a0,
                                           cplx<R>& a1) {
  if (MU == 0) {  // A_x^+ h = (i h1, i h0)
    a0 = timesI(h1);
    a1 = timesI(h0);
  } else if (MU == 1) {  // A_y^+ h = (h1, -h0)
    a0 = h1;
    a1 = cmk(-h0.re, -h0.im);
  } else if (MU == 2) {  // A_z^+ h = (i h0, -i h1)
    a0 = timesI(h0);
    a1 = timesMinusI(h1);
  } else {
    a0 = h0;
    a1 = h1;
  }
}

template <typename R>
__device__ __forceinline__ void store_field(cplx<R>* p, cplx<R> v, bool nt) {
  if (nt) {
    __builtin_nontemporal_store(v.re, &p->re);
    __builtin_nontemporal_store(v.im, &p->im);
  } else {
    *p = v;
  }
}
// 16-bit fields keep each site s-major, [s][spin*colour] (48 bytes per
// (site, s)), where the wider types keep [spin*colour][s]: a lane, which owns
// one s of one site, then moves its twelve values with three 16-byte
// accesses instead of twelve 4-byte ones.
template <typename T>
constexpr bool kSMajor = std::is_same<T, bf16c>::value;
typedef unsigned u32x4 __attribute__((ext_vector_type(4)));
typedef unsigned u32x2 __attribute__((ext_vector_type(2)));

__device__ __forceinline__ cplx<float> bf16_word(unsigned w) {
  return cmk(__uint_as_float(w << 16), __uint_as_float(w & 0xffff0000u));
}
__device__ __forceinline__ unsigned bf16_pack(cplx<float> v) {
  return f32x2_to_bf16x2(v.re, v.im);
}
// the twelve values of one (site, s) row; p 16-byte aligned
__device__ __forceinline__ void ld_row12(const bf16c* p, cplx<float> (&v)[12]) {
  const u32x4* q = reinterpret_cast<const u32x4*>(p);
  const u32x4 a = q[0], b = q[1], c = q[2];
  v[0] = bf16_word(a.x), v[1] = bf16_word(a.y), v[2] = bf16_word(a.z), v[3] = bf16_word(a.w);
  v[4] = bf16_word(b.x), v[5] = bf16_word(b.y), v[6] = bf16_word(b.z), v[7] = bf16_word(b.w);
  v[8] = bf16_word(c.x), v[9] = bf16_word(c.y), v[10] = bf16_word(c.z), v[11] = bf16_word(c.w);
}
// six values (one chirality half of a row); p 8-byte aligned
__device__ __forceinline__ void ld_half6(const bf16c* p, cplx<float>* v) {
  const u32x2* q = reinterpret_cast<const u32x2*>(p);
  const u32x2 a = q[0], b = q[1], c = q[2];
  v[0] = bf16_word(a.x), v[1] = bf16_word(a.y), v[2] = bf16_word(b.x);
  v[3] = bf16_word(b.y), v[4] = bf16_word(c.x), v[5] = bf16_word(c.y);
}
__device__ __forceinline__ void st_row12(bf16c* p, const cplx<float> (&v)[12], bool nt) {
  u32x4* q = reinterpret_cast<u32x4*>(p);
  u32x4 w[3];
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    w[k].x = bf16_pack(v[4 * k]);
    w[k].y = bf16_pack(v[4 * k + 1]);
    w[k].z = bf16_pack(v[4 * k + 2]);
    w[k].w = bf16_pack(v[4 * k + 3]);
  }
  if (nt) {
#pragma unroll
    for (int k = 0; k < 3; ++k) __builtin_nontemporal_store(w[k], q + k);
  } else {
#pragma unroll
    for (int k = 0; k < 3; ++k) q[k] = w[k];
  }
}

// complex64 [site][12][Ls] <-> 16-bit [site][Ls][12], one (site, s) row per
// thread; rows = nrhs * Vh * Ls
__global__ void to_bf16_kernel(bf16c* __restrict__ dst, const cplx<float>* __restrict__ src, size_t rows,
                               int Ls) {
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < rows; i += (size_t)gridDim.x * blockDim.x) {
    const size_t site = i / Ls;
    const int s = (int)(i - site * Ls);
    const cplx<float>* f = src + site * 12 * Ls + s;
    cplx<float> v[12];
#pragma unroll
    for (int c = 0; c < 12; ++c) v[c] = f[c * Ls];
    st_row12(dst + site * 12 * Ls + s * 12, v, false);
  }
}
__global__ void from_bf16_kernel(cplx<float>* __restrict__ dst, const bf16c* __restrict__ src, size_t rows,
                                 int Ls) {
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < rows; i += (size_t)gridDim.x * blockDim.x) {
    const size_t site = i / Ls;
    const int s = (int)(i - site * Ls);
    cplx<float> v[12];
    ld_row12(src + site * 12 * Ls + s * 12, v);
    cplx<float>* f = dst + site * 12 * Ls + s;
#pragma unroll
    for (int c = 0; c < 12; ++c) f[c * Ls] = v[c];
  }
}

// acc += (1 + SG*gamma_mu) W psi from the projected half-spinor
// h = u + SG A l (two spin pairs of 3 colours), W = 3x3 link at `w`.
template <typename R, int MU, int SG>
__device__ __forceinline__ void link_mul_add(cplx<R> (&acc)[12], const cplx<R> (&h)[2][3],
                                             const cplx<R>* __restrict__ w) {
  cplx<R> Wh[2][3];
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    const cplx<R> w0 = w[a * 3 + 0], w1 = w[a * 3 + 1], w2 = w[a * 3 + 2];
#pragma unroll
    for (int sp = 0; sp < 2; ++sp) {
      cplx<R> t = w0 * h[sp][0];
      cmac(t, w1, h[sp][1]);
      cmac(t, w2, h[sp][2]);
      Wh[sp][a] = t;
    }
  }
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    acc[0 * 3 + a] = acc[0 * 3 + a] + Wh[0][a];
    acc[1 * 3 + a] = acc[1 * 3 + a] + Wh[1][a];
    cplx<R> b0, b1;
    apply_Adag<R, MU>(Wh[0][a], Wh[1][a], b0, b1);
    if (SG > 0) {
      acc[2 * 3 + a] = acc[2 * 3 + a] + b0;
      acc[3 * 3 + a] = acc[3 * 3 + a] + b1;
    } else {
      acc[2 * 3 + a] = acc[2 * 3 + a] - b0;
      acc[3 * 3 + a] = acc[3 * 3 + a] - b1;
    }
  }
}

// Spin projection h = u + SG A_mu l of the components c0 (u0 u1 l0 l1 for
// colour c).
template <typename R, int MU, int SG>
__device__ __forceinline__ void project(cplx<R> (&h)[2][3], int c, cplx<R> u0, cplx<R> u1,
                                        cplx<R> l0, cplx<R> l1) {
  cplx<R> a0, a1;
  apply_A<R, MU>(l0, l1, a0, a1);
  if (SG > 0) {
    h[0][c] = u0 + a0;
    h[1][c] = u1 + a1;
  } else {
    h[0][c] = u0 - a0;
    h[1][c] = u1 - a1;
  }
}

// acc += (1 + SG*gamma_mu) W psi for a spinor psi already in registers.
template <typename R, int MU, int SG>
__device__ __forceinline__ void hop_term_vals(cplx<R> (&acc)[12], const cplx<R> (&psi)[12],
                                              const cplx<R>* __restrict__ w) {
  cplx<R> h[2][3];
#pragma unroll
  for (int c = 0; c < 3; ++c) project<R, MU, SG>(h, c, psi[c], psi[3 + c], psi[6 + c], psi[9 + c]);
  link_mul_add<R, MU, SG>(acc, h, w);
}

struct HopArgs {
  Geom g;
  int out_parity;
  int spw;            // sites per workgroup
  int bx, by, bz, bt; // 4D site block per workgroup in (x/2, y, z, t), powers of two; bx = 0: linear cb order
  int lbx, lby, lbz;  // log2 of bx, by, bz
  int nbx, nby, nbz;  // block-grid extents
  int remap;          // XCD-contiguous workgroup order
  int nt;             // non-temporal output stores
  int morton;         // Morton (bit-interleaved) order of the block grid (power-of-two grids)
  int nbt;            // block-grid extent in t
  const int* order;   // nullable: block of workgroup blockIdx.x, packed gx | gy << 8 | gz << 16 | gt << 24
  int rg;             // right-hand sides per workgroup (blockIdx.y takes rg of the nrhs)
  int nrhs;
  int epi_off;        // byte offset of the epilogue's LDS buffer (0: it reuses the link rows)
  size_t field;       // complex elements per rhs
  // fifth dimension: M_5 = alpha + beta K, recurrence of M_5^-1 y_s = ia x_s + kap y_{s-1},
  // Mobius C_5 = b5 + c5 K (K: P+ from s-1, P- from s+1, -mass at the wrap)
  double alpha, beta, ia, kap, b5, c5, mass;
  double* partials;   // EPI_SUB norm: [rhs][pstride] per-workgroup partials (nullable)
  size_t pstride;     // = number of workgroups
  unsigned* counters; // [rhs]
  double* result;     // [rhs]
};

// Block coordinates of workgroup wg in the block grid (lexicographic or
// Morton order); uniform across the workgroup.
__device__ __forceinline__ void hop_block(const HopArgs& A, int wg, int& gx, int& gy, int& gz, int& gt) {
  if (A.order) {
    const int q = A.order[wg];
    gx = q & 255;
    gy = (q >> 8) & 255;
    gz = (q >> 16) & 255;
    gt = (q >> 24) & 255;
  } else if (A.morton) {
    // de-interleave the bits of wg over the four block-grid dimensions
    gx = gy = gz = gt = 0;
    int bit = 0, px = 0, py = 0, pz = 0, pt = 0;
    while ((1 << px) < A.nbx || (1 << py) < A.nby || (1 << pz) < A.nbz || (1 << pt) < A.nbt) {
      if ((1 << px) < A.nbx) gx |= ((wg >> bit++) & 1) << px++;
      if ((1 << py) < A.nby) gy |= ((wg >> bit++) & 1) << py++;
      if ((1 << pz) < A.nbz) gz |= ((wg >> bit++) & 1) << pz++;
      if ((1 << pt) < A.nbt) gt |= ((wg >> bit++) & 1) << pt++;
    }
  } else {
    int q = wg;
    gx = q % A.nbx; q /= A.nbx;
    gy = q % A.nby; q /= A.nby;
    gz = q % A.nbz;
    gt = q / A.nbz;
  }
}

// Coordinates and checkerboard index of the vloc-th output site of
// workgroup wg: either `spw` consecutive sites, or one bx*by*bz*bt block of
// the (x/2, y, z, t) grid, the blocks taken in lexicographic or Morton
// (bit-interleaved) order.  The index may exceed Vh - 1 only in the linear
// order's last workgroup (then the coordinates are not meaningful).
__device__ __forceinline__ int hop_site(const HopArgs& A, int wg, int vloc, Site& c) {
  const Geom& g = A.g;
  if (A.bx <= 0) {
    const int v = wg * A.spw + vloc;
    c = site_coords(v, A.out_parity, g);
    return v;
  }
  int gx, gy, gz, gt;
  hop_block(A, wg, gx, gy, gz, gt);
  c.xh = gx * A.bx + (vloc & (A.bx - 1));
  c.y = gy * A.by + ((vloc >> A.lbx) & (A.by - 1));
  c.z = gz * A.bz + ((vloc >> (A.lbx + A.lby)) & (A.bz - 1));
  c.t = gt * A.bt + (vloc >> (A.lbx + A.lby + A.lbz));
  c.zt = c.z + g.Z * c.t;
  c.rest = c.y + g.Y * c.zt;
  c.x = 2 * c.xh + ((c.y + c.z + c.t + A.out_parity) & 1);
  return c.xh + g.Xh * c.rest;
}

// row <- (b + c S) row in place along s, S taking s+1 (up) or s-1 (down),
// with -m times the wrapped entry at the wall.
template <typename R>
__device__ __forceinline__ void bcs_row(cplx<R>* row, int Ls, R b, R c, R m, bool up) {
  if (up) {
    const cplx<R> first = row[0];
    for (int t = 0; t < Ls - 1; ++t) row[t] = b * row[t] + c * row[t + 1];
    row[Ls - 1] = b * row[Ls - 1] + (-m * c) * first;
  } else {
    const cplx<R> last = row[Ls - 1];
    for (int t = Ls - 1; t > 0; --t) row[t] = b * row[t] + c * row[t - 1];
    row[0] = b * row[0] + (-m * c) * last;
  }
}

// Fifth-dimension epilogue of a hop stage: acc holds (Dh in) or (Dh^+ in)
// at (site v, slice s).  EPI_INV stages acc in LDS (`smem_raw`, spw*12*(Ls+1)
// complex) and applies M_5^-1 (or M_5^-+); EPI_SUB forms M_5 c - acc/4 (or
// M_5^+ c - acc/4) and, when A.partials is set, stores this workgroup's part
// of its squared norm.  Every thread of the workgroup must call it.
template <typename R, bool DAG, int EPI, int LS = 0, bool MOB = false, typename T = cplx<R>>
__device__ __forceinline__ void hop_epilogue(const cplx<R> (&acc)[12], bool active, int vloc, int s,
                                             int v, int wg, int rhs, T* __restrict__ out,
                                             const T* __restrict__ center,
                                             const R* __restrict__ pw, const HopArgs& A,
                                             unsigned char* smem_raw) {
  const Geom& g = A.g;
  const int Ls = LS > 0 ? LS : g.Ls;
  const int tid = threadIdx.x;
  if (EPI == EPI_INV) {
    // ---- M_5^-1 (or its adjoint) across s, through LDS --------------------
    cplx<R>* buf = reinterpret_cast<cplx<R>*>(smem_raw);  // [spw][12][Ls+1]
    const int ld = Ls + 1;
    if (active) {
#pragma unroll
      for (int c = 0; c < 12; ++c) buf[(vloc * 12 + c) * ld + s] = acc[c];
    }
    __syncthreads();
    const R ia = (R)A.ia, kap = (R)A.kap;
    const R m = (R)A.mass;
    for (int q = tid; q < A.spw * 12; q += blockDim.x) {
      const int vl = q / 12, c = q - vl * 12;
      if (A.bx == 0 && wg * A.spw + vl >= g.Vh) continue;
      cplx<R>* row = buf + (vl * 12 + c) * ld;
      // Mobius, adjoint chain: C_5^+ = b5 + c5 K^+ on the hop result first
      // (K^+ takes P+ from s+1 and P- from s-1)
      if (MOB && DAG) bcs_row(row, Ls, (R)A.b5, (R)A.c5, m, c < 6);
      // P+ (c < 6) takes M+^-1 (lower-triangular recurrence), P- takes M-^-1;
      // the adjoint swaps the two.
      const bool lower = ((c < 6) != DAG);
      if (lower) {
        cplx<R> tsum = cmk((R)0, (R)0);
        for (int sp = 1; sp < Ls; ++sp) tsum = tsum + pw[Ls - sp] * row[sp];
        cplx<R> y = pw[0] * row[0] - m * tsum;
        row[0] = y;
        for (int sp = 1; sp < Ls; ++sp) {
          y = ia * row[sp] + kap * y;
          row[sp] = y;
        }
      } else {
        cplx<R> tsum = cmk((R)0, (R)0);
        for (int t = 1; t < Ls; ++t) tsum = tsum + pw[Ls - t] * row[Ls - 1 - t];
        cplx<R> y = pw[0] * row[Ls - 1] - m * tsum;
        row[Ls - 1] = y;
        for (int sp = Ls - 2; sp >= 0; --sp) {
          y = ia * row[sp] + kap * y;
          row[sp] = y;
        }
      }
      // Mobius: C_5 = b5 + c5 K after M_5^-1 (K takes P+ from s-1, P- from s+1)
      if (MOB && !DAG) bcs_row(row, Ls, (R)A.b5, (R)A.c5, m, c >= 6);
    }
    __syncthreads();
    if (active) {
      if constexpr (kSMajor<T>) {
        cplx<R> row[12];
#pragma unroll
        for (int c = 0; c < 12; ++c) row[c] = buf[(vloc * 12 + c) * ld + s];
        st_row12(out + (size_t)v * 12 * Ls + s * 12, row, A.nt & 1);
      } else {
        T* o = out + (size_t)v * 12 * Ls + s;
#pragma unroll
        for (int c = 0; c < 12; ++c) store_field(o + c * Ls, buf[(vloc * 12 + c) * ld + s], A.nt & 1);
      }
    }
  } else {
    // ---- M_5 c - 1/4 hop (or M_5^+ c - 1/4 hop^+) --------------------------
    cplx<R> hop[12];
#pragma unroll
    for (int c = 0; c < 12; ++c) hop[c] = acc[c];
    if (MOB && DAG) {
      // adjoint chain: C_5^+ = b5 + c5 K^+ on the hop result, through LDS
      // (K^+ takes P+ from s+1 and P- from s-1, -mass at the wrap)
      cplx<R>* buf = reinterpret_cast<cplx<R>*>(smem_raw);  // [spw][12][Ls+1]
      const int ld = Ls + 1;
      if (active) {
#pragma unroll
        for (int c = 0; c < 12; ++c) buf[(vloc * 12 + c) * ld + s] = acc[c];
      }
      __syncthreads();
      if (active) {
        const R b5 = (R)A.b5, c5 = (R)A.c5, m = (R)A.mass;
        const int s_up = (s < Ls - 1) ? s + 1 : 0, s_dn = (s > 0) ? s - 1 : Ls - 1;
        const R w_up = (s < Ls - 1) ? c5 : -m * c5, w_dn = (s > 0) ? c5 : -m * c5;
#pragma unroll
        for (int c = 0; c < 12; ++c) {
          const cplx<R>* row = buf + (vloc * 12 + c) * ld;
          hop[c] = b5 * row[s] + (c < 6 ? w_up * row[s_up] : w_dn * row[s_dn]);
        }
      }
    }
    double nrm = 0.0;
    if constexpr (kSMajor<T>) {
      if (active) {
        const T* cen = center + rhs * A.field + (size_t)v * 12 * Ls;
        const R al = (R)A.alpha, be = (R)A.beta, m = (R)A.mass, q = (R)0.25;
        const int s_dn = (s > 0) ? s - 1 : Ls - 1, s_up = (s < Ls - 1) ? s + 1 : 0;
        const R f_dn = (s > 0) ? be : -m * be, f_up = (s < Ls - 1) ? be : -m * be;
        // the P+ half (c < 6) couples to s-1 and the P- half to s+1 (swapped
        // in the adjoint), as in the branch below
        const int sa = DAG ? s_up : s_dn, sb = DAG ? s_dn : s_up;
        const R fa = DAG ? f_up : f_dn, fb = DAG ? f_dn : f_up;
        cplx<R> x[12], y[12], r[12];
        ld_row12(cen + s * 12, x);
        ld_half6(cen + sa * 12, y);
        ld_half6(cen + sb * 12 + 6, y + 6);
#pragma unroll
        for (int c = 0; c < 12; ++c) {
          r[c] = al * x[c] + (c < 6 ? fa : fb) * y[c] - q * hop[c];
          nrm += (double)r[c].re * (double)r[c].re + (double)r[c].im * (double)r[c].im;
        }
        st_row12(out + (size_t)v * 12 * Ls + s * 12, r, A.nt & 1);
      }
    } else if (active) {
      const T* cen = center + rhs * A.field + (size_t)v * 12 * Ls;
      T* o = out + (size_t)v * 12 * Ls + s;
      const R al = (R)A.alpha, be = (R)A.beta, m = (R)A.mass, q = (R)0.25;
      // M_5 = alpha + beta K: P+ couples to s-1 (-mass times Ls-1 at s = 0),
      // P- to s+1 (-mass times 0 at s = Ls-1); the adjoint swaps the directions.
      const int s_dn = (s > 0) ? s - 1 : Ls - 1;
      const R f_dn = (s > 0) ? be : -m * be;
      const int s_up = (s < Ls - 1) ? s + 1 : 0;
      const R f_up = (s < Ls - 1) ? be : -m * be;
#pragma unroll
      for (int c = 0; c < 12; ++c) {
        const T* cc = cen + c * Ls;
        const bool from_below = ((c < 6) != DAG);
        const int sn = from_below ? s_dn : s_up;
        const R fn = from_below ? f_dn : f_up;
        const cplx<R> r = al * St<T>::ld(cc + s) + fn * St<T>::ld(cc + sn) - q * hop[c];
        store_field(o + c * Ls, r, A.nt & 1);
        nrm += (double)r.re * (double)r.re + (double)r.im * (double)r.im;
      }
    }
    if (A.partials) {
      double vv[1] = {nrm};
      __shared__ double red[16];
      block_sum<1>(vv, red);
      store_partial<1>(vv, A.partials + (size_t)rhs * A.pstride, 0, wg);
    }
  }
}

// ---------------------------------------------------------- hop kernel --
constexpr int kLinkLd = 73;  // LDS row of one site's 72 link entries (odd: no bank aliasing)

// Checkerboard indices of the eight neighbours of site c, in the order
// x+, x-, y+, y-, z+, z-, t+, t-.
__device__ __forceinline__ void hop_neighbours(const Geom& g, const Site& c, int (&nb)[8]) {
  const int rowyzt = c.rest * g.Xh;
  const int xp = (c.x + 1 == g.X) ? 0 : c.x + 1;
  const int xm = (c.x == 0) ? g.X - 1 : c.x - 1;
  nb[0] = (xp >> 1) + rowyzt;
  nb[1] = (xm >> 1) + rowyzt;
  const int yp = (c.y + 1 == g.Y) ? 0 : c.y + 1;
  const int ym = (c.y == 0) ? g.Y - 1 : c.y - 1;
  nb[2] = c.xh + g.Xh * (yp + g.Y * c.zt);
  nb[3] = c.xh + g.Xh * (ym + g.Y * c.zt);
  const int zp = (c.z + 1 == g.Z) ? 0 : c.z + 1;
  const int zm = (c.z == 0) ? g.Z - 1 : c.z - 1;
  const int bz = c.xh + g.Xh * c.y, sy = g.Xh * g.Y;
  nb[4] = bz + sy * (zp + g.Z * c.t);
  nb[5] = bz + sy * (zm + g.Z * c.t);
  const int tp = (c.t + 1 == g.T) ? 0 : c.t + 1;
  const int tm = (c.t == 0) ? g.T - 1 : c.t - 1;
  const int bt = c.xh + g.Xh * (c.y + g.Y * c.z), sz = g.Xh * g.Y * g.Z;
  nb[6] = bt + sz * tp;
  nb[7] = bt + sz * tm;
}

// Direction D of hop_neighbours: mu = D/2, forward (even D, link mu) or
// backward (odd D, link 4 + mu); SF is the sign of gamma_mu on forward hops.
template <typename R, int D, int SF>
__device__ __forceinline__ void dir_term(cplx<R> (&acc)[12], const cplx<R> (&psi)[12],
                                         const cplx<R>* links) {
  constexpr int MU = D / 2;
  constexpr int SG = (D & 1) ? -SF : SF;
  hop_term_vals<R, MU, SG>(acc, psi, links + ((D & 1) ? 4 + MU : MU) * 9);
}

template <typename T, int D0, int N>
__device__ __forceinline__ void load_dirs(cplx<typename St<T>::R> (&psi)[N][12], const T* __restrict__ in,
                                          const int (&nb)[8], size_t col, int s, int Ls) {
#pragma unroll
  for (int k = 0; k < N; ++k) {
    if constexpr (kSMajor<T>) {
      ld_row12(in + (size_t)nb[D0 + k] * col + s * 12, psi[k]);
    } else {
      const T* p = in + (size_t)nb[D0 + k] * col + s;
#pragma unroll
      for (int c = 0; c < 12; ++c) psi[k][c] = St<T>::ld(p + c * Ls);
    }
  }
}

// load_dirs for the Mobius first stage: each neighbour spinor is read as
// C_5 psi = b5 psi_s + c5 (K psi)_s (K: P+ from s-1, P- from s+1, -mass at the
// wrap), the s +- 1 entries read from the same contiguous column.
template <typename T, int D0, int N, typename R = typename St<T>::R>
__device__ __forceinline__ void load_dirs_c5(cplx<R> (&psi)[N][12], const T* __restrict__ in,
                                             const int (&nb)[8], size_t col, int s, int Ls, R b5, R c5,
                                             R m) {
  const int s_dn = (s > 0) ? s - 1 : Ls - 1, s_up = (s < Ls - 1) ? s + 1 : 0;
  const R w_dn = (s > 0) ? c5 : -m * c5, w_up = (s < Ls - 1) ? c5 : -m * c5;
#pragma unroll
  for (int k = 0; k < N; ++k) {
    const T* p = in + (size_t)nb[D0 + k] * col;
    if constexpr (kSMajor<T>) {
      cplx<R> x[12], y[12];
      ld_row12(p + s * 12, x);
      ld_half6(p + s_dn * 12, y);
      ld_half6(p + s_up * 12 + 6, y + 6);
#pragma unroll
      for (int c = 0; c < 12; ++c) psi[k][c] = b5 * x[c] + (c < 6 ? w_dn : w_up) * y[c];
    } else {
#pragma unroll
      for (int c = 0; c < 12; ++c) {
        const cplx<R> x = St<T>::ld(p + c * Ls + s);
        const cplx<R> y = St<T>::ld(c < 6 ? p + c * Ls + s_dn : p + c * Ls + s_up);
        psi[k][c] = b5 * x + (c < 6 ? w_dn : w_up) * y;
      }
    }
  }
}

template <typename R, int D0, int N, int SF>
__device__ __forceinline__ void apply_dirs(cplx<R> (&acc)[12], const cplx<R> (&psi)[N][12],
                                           const cplx<R>* links) {
  dir_term<R, D0 + 0, SF>(acc, psi[0], links);
  if (N > 1) dir_term<R, D0 + 1, SF>(acc, psi[N > 1 ? 1 : 0], links);
  if (N > 2) dir_term<R, D0 + 2, SF>(acc, psi[N > 2 ? 2 : 0], links);
  if (N > 3) dir_term<R, D0 + 3, SF>(acc, psi[N > 3 ? 3 : 0], links);
  if (N > 4) dir_term<R, (D0 + 4) & 7, SF>(acc, psi[N > 4 ? 4 : 0], links);
  if (N > 5) dir_term<R, (D0 + 5) & 7, SF>(acc, psi[N > 5 ? 5 : 0], links);
  if (N > 6) dir_term<R, (D0 + 6) & 7, SF>(acc, psi[N > 6 ? 6 : 0], links);
  if (N > 7) dir_term<R, (D0 + 7) & 7, SF>(acc, psi[N > 7 ? 7 : 0], links);
}

// NPH = number of load phases (2: four directions in flight at a time; 4:
// two).  LS > 0 fixes Ls at compile time.  Dynamic LDS:
// max(spw * kLinkLd, spw * 12 * (Ls + 1)) complex.
template <typename R, bool DAG, int EPI, int NPH, int LS, bool MOB, typename T, bool MR>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(1, 2)))
hop_kernel(T* __restrict__ out, const T* __restrict__ in, const T* __restrict__ center,
           const cplx<R>* __restrict__ gauge, const R* __restrict__ pw, HopArgs A) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  const Geom& g = A.g;
  const int Ls = LS > 0 ? LS : g.Ls;  // compile-time when LS > 0: immediate load offsets
  // a table order already places each workgroup on its XCD's region
  const int wg = (A.remap && !A.order) ? xcd_remap(blockIdx.x, gridDim.x) : (int)blockIdx.x;
  const int rhs0 = blockIdx.y * A.rg;
  // MR: several right-hand sides per workgroup (a separate instantiation,
  // so that the one-RHS kernel keeps the register footprint of straight-line
  // code)
  const int nr = MR ? min(A.rg, A.nrhs - rhs0) : 1;
  const int tid = threadIdx.x;
  const int vloc = tid / Ls, s = tid - vloc * Ls;
  Site c;
  const int v = hop_site(A, wg, vloc, c);
  const bool active = (vloc < A.spw) && (v < g.Vh);

  cplx<R>* links = reinterpret_cast<cplx<R>*>(smem_raw);  // [spw][kLinkLd]
  constexpr int ND = 8 / NPH;
  constexpr int SF = DAG ? 1 : -1;
  constexpr int NL = LS > 0 ? (72 + LS - 1) / LS : 1;
  const size_t col = (size_t)12 * Ls;
  // Mobius: the first stage of M_pc hops C_5 in (C_5 on the neighbours' columns)
  constexpr bool C5IN = MOB && !DAG && EPI == EPI_INV;
  int nb[8];
  cplx<R> psi[ND][12];
  // The site's 72 link entries, entry e by thread s = e mod Ls.  With Ls
  // fixed at compile time they are loaded before the first right-hand
  // side's first-phase neighbour loads are issued and written to LDS after
  // them, so the wave waits for memory once instead of once per entry.
  if (active) {
    const cplx<R>* G = gauge + (size_t)v * 72;
    cplx<R> lk[NL];
    if constexpr (LS > 0) {
      // (the last entries of the short threads re-read entry 71: no branch)
#pragma unroll
      for (int k = 0; k < NL; ++k) lk[k] = G[min(s + k * LS, 71)];
    } else {
      for (int e = s; e < 72; e += Ls) links[vloc * kLinkLd + e] = G[e];
    }
    hop_neighbours(g, c, nb);
    if (C5IN)
      load_dirs_c5<T, 0, ND>(psi, in + rhs0 * A.field, nb, col, s, Ls, (R)A.b5, (R)A.c5, (R)A.mass);
    else
      load_dirs<T, 0, ND>(psi, in + rhs0 * A.field, nb, col, s, Ls);
    if constexpr (LS > 0) {
#pragma unroll
      for (int k = 0; k < NL; ++k)
        if (s + k * LS < 72) links[vloc * kLinkLd + s + k * LS] = lk[k];
    }
  }
  // The workgroup's right-hand sides one after another, all on the links
  // staged once (with several, the epilogue has an LDS buffer of its own).
  for (int rr = 0; rr < nr; ++rr) {
    const int rhs = rhs0 + rr;
    const T* __restrict__ inr = in + rhs * A.field;
    T* __restrict__ outr = out + rhs * A.field;
    if (rr > 0 && active) {
      if (C5IN)
        load_dirs_c5<T, 0, ND>(psi, inr, nb, col, s, Ls, (R)A.b5, (R)A.c5, (R)A.mass);
      else
        load_dirs<T, 0, ND>(psi, inr, nb, col, s, Ls);
    }
    __syncthreads();  // links in LDS

    cplx<R> acc[12];
  #pragma unroll
    for (int c = 0; c < 12; ++c) acc[c] = cmk((R)0, (R)0);
    if (active) {
      const cplx<R>* L = links + vloc * kLinkLd;
      apply_dirs<R, 0, ND, SF>(acc, psi, L);
      const R b5 = (R)A.b5, c5 = (R)A.c5, mm = (R)A.mass;
      if (NPH >= 2) {
        if (C5IN)
          load_dirs_c5<T, ND % 8, ND>(psi, inr, nb, col, s, Ls, b5, c5, mm);
        else
          load_dirs<T, ND % 8, ND>(psi, inr, nb, col, s, Ls);
        apply_dirs<R, ND % 8, ND, SF>(acc, psi, L);
      }
      if (NPH == 4) {
        if (C5IN)
          load_dirs_c5<T, 4, ND>(psi, inr, nb, col, s, Ls, b5, c5, mm);
        else
          load_dirs<T, 4, ND>(psi, inr, nb, col, s, Ls);
        apply_dirs<R, 4, ND, SF>(acc, psi, L);
        if (C5IN)
          load_dirs_c5<T, 6, ND>(psi, inr, nb, col, s, Ls, b5, c5, mm);
        else
          load_dirs<T, 6, ND>(psi, inr, nb, col, s, Ls);
        apply_dirs<R, 6, ND, SF>(acc, psi, L);
      }
    }
    // the epilogue's LDS buffer reuses the link rows (one right-hand side per
    // workgroup) or the previous right-hand side's buffer
    if (EPI == EPI_INV || (MOB && DAG)) __syncthreads();
    hop_epilogue<R, DAG, EPI, LS, MOB, T>(acc, active, vloc, s, v, wg, rhs, outr, center, pw, A,
                                          smem_raw + A.epi_off);
  }
}

// ------------------------------------------------------------------ BLAS ---
template <typename R>
__device__ __forceinline__ double cnorm(cplx<R> a) {
  return (double)a.re * a.re + (double)a.im * a.im;
}

struct RedArgs {
  size_t n;  // complex elements per rhs
  double* partials;
  unsigned* counters;
  double* result;
};

template <typename T>
__global__ void __launch_bounds__(256) norm2_kernel(const T* __restrict__ x, RedArgs A) {
  const int rhs = blockIdx.y;
  x += rhs * A.n;
  double acc = 0.0;
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < A.n;
       i += (size_t)gridDim.x * blockDim.x)
    acc += cnorm(St<T>::ld(x + i));
  double v[1] = {acc};
  __shared__ double red[16];
  block_sum<1>(v, red);
  store_partial<1>(v, A.partials + (size_t)rhs * kMaxPartials, 0, blockIdx.x);
}

template <typename R>
__global__ void __launch_bounds__(256)
dot_kernel(const cplx<R>* __restrict__ a, const cplx<R>* __restrict__ b, RedArgs A) {
  const int rhs = blockIdx.y;
  a += rhs * A.n;
  b += rhs * A.n;
  double re = 0.0, im = 0.0;
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < A.n;
       i += (size_t)gridDim.x * blockDim.x) {
    const cplx<R> x = a[i], y = b[i];
    re += (double)x.re * y.re + (double)x.im * y.im;  // conj(a) b
    im += (double)x.re * y.im - (double)x.im * y.re;
  }
  double v[2] = {re, im};
  __shared__ double red[32];
  block_sum<2>(v, red);
  // partial layout [rhs][2][kMaxPartials/2]
  store_partial<2>(v, A.partials + (size_t)rhs * kMaxPartials, kMaxPartials / 2, blockIdx.x);
}

template <typename R>
__global__ void __launch_bounds__(256)
cg_update_kernel(cplx<R>* __restrict__ x, cplx<R>* __restrict__ r, const cplx<R>* __restrict__ p,
                 const cplx<R>* __restrict__ w, const double* num, const double* den,
                 const double* alpha_host, RedArgs A) {
  const int rhs = blockIdx.y;
  const size_t off = rhs * A.n;
  const double al = num ? num[rhs] / den[rhs] : alpha_host[rhs];
  const R a = (R)al;
  double acc = 0.0;
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < A.n;
       i += (size_t)gridDim.x * blockDim.x) {
    const cplx<R> pi = p[off + i], wi = w[off + i];
    cplx<R> xi = x[off + i], ri = r[off + i];
    xi = xi + a * pi;
    ri = ri - a * wi;
    x[off + i] = xi;
    r[off + i] = ri;
    acc += cnorm(ri);
  }
  double v[1] = {acc};
  __shared__ double red[16];
  block_sum<1>(v, red);
  store_partial<1>(v, A.partials + (size_t)rhs * kMaxPartials, 0, blockIdx.x);
}

template <typename R>
__global__ void __launch_bounds__(256)
xpay_kernel(cplx<R>* __restrict__ p, const cplx<R>* __restrict__ r, const double* num,
            const double* den, const double* beta_host, size_t n) {
  const int rhs = blockIdx.y;
  const size_t off = rhs * n;
  const R b = (R)(num ? num[rhs] / den[rhs] : beta_host[rhs]);
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (size_t)gridDim.x * blockDim.x)
    p[off + i] = r[off + i] + b * p[off + i];
}

template <typename R>
__global__ void axpby_kernel(cplx<R>* __restrict__ y, const cplx<R>* __restrict__ x, R a, R b,
                             size_t n) {
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (size_t)gridDim.x * blockDim.x)
    y[i] = a * x[i] + b * y[i];
}

// ============================================================= launchers ===
static inline int red_blocks(size_t n) {
  size_t b = (n + 256 * 8 - 1) / (256 * 8);
  if (b < 1) b = 1;
  if (b > 1024) b = 1024;
  return (int)b;
}

int ensure_reducer(dwf_op* op) {
  HDCG_TRY(op->red.partials.ensure(sizeof(double) * (size_t)kMaxPartials * 64));
  if (op->red.counters.bytes == 0) {
    HDCG_TRY(op->red.counters.ensure(sizeof(unsigned) * 64));
    HDCG_HIP(hipMemset(op->red.counters.ptr, 0, sizeof(unsigned) * 64));
  }
  HDCG_TRY(op->red.results.ensure(sizeof(double) * 256));
  return DWF_OK;
}

void release_tmp(dwf_op* op) {
  for (auto& a : op->tmp)
    for (auto& b : a) b.release();
}

static int tmp_index(int prec) { return prec == DWF_C128 ? 0 : (prec == DWF_BF16 ? 2 : 1); }

int ensure_tmp(dwf_op* op, int prec, int nrhs) {
  const size_t bytes = op->field_elems(nrhs) * cbytes(prec);
  const int pi = tmp_index(prec);
  for (int i = 0; i < 3; ++i) HDCG_TRY(op->tmp[pi][i].ensure(bytes));
  return DWF_OK;
}

template <typename R, int NPH, int LS, bool MOB, typename T, bool MR>
static void launch_hop_mr(bool dagger, int epi, dim3 grid, dim3 block, size_t lds, hipStream_t stream,
                          T* out, const T* in, const T* center, const cplx<R>* G, const R* pw, const HopArgs& A) {
  if (epi == EPI_INV) {
    if (dagger)
      hipLaunchKernelGGL((hop_kernel<R, true, EPI_INV, NPH, LS, MOB, T, MR>), grid, block, lds, stream, out, in, center,
                         G, pw, A);
    else
      hipLaunchKernelGGL((hop_kernel<R, false, EPI_INV, NPH, LS, MOB, T, MR>), grid, block, lds, stream, out, in,
                         center, G, pw, A);
  } else {
    if (dagger)
      hipLaunchKernelGGL((hop_kernel<R, true, EPI_SUB, NPH, LS, MOB, T, MR>), grid, block, lds, stream, out, in, center,
                         G, pw, A);
    else
      hipLaunchKernelGGL((hop_kernel<R, false, EPI_SUB, NPH, LS, MOB, T, MR>), grid, block, lds, stream, out, in,
                         center, G, pw, A);
  }
}

// several right-hand sides per workgroup are built for the compile-time Ls
// = 16 kernels only (the launch keeps A.rg = 1 otherwise)
template <typename R, int NPH, int LS, bool MOB, typename T>
static void launch_hop(bool dagger, int epi, dim3 grid, dim3 block, size_t lds, hipStream_t stream,
                       T* out, const T* in, const T* center, const cplx<R>* G, const R* pw, const HopArgs& A) {
  if constexpr (LS == 16) {
    if (A.rg > 1)
      return launch_hop_mr<R, NPH, LS, MOB, T, true>(dagger, epi, grid, block, lds, stream, out, in, center, G, pw, A);
  }
  launch_hop_mr<R, NPH, LS, MOB, T, false>(dagger, epi, grid, block, lds, stream, out, in, center, G, pw, A);
}

// ------------------------------------------------- region block orders --
// Orders 2-4 place the site blocks with a table instead of an index
// formula, so that they work on block grids of any extents (Morton's bit
// interleaving needs powers of two).  The block grid is bisected three times
// into eight compact regions, one per XCD (each cut halves the region's
// longest extent in lattice sites), so each XCD's L2 serves one region and
// its halo; within a region the blocks run in Morton order of the region's
// power-of-two bounding grid with the blocks outside skipped (order 2), or
// t-plane by t-plane with Morton order inside each plane (order 3).  Order 4
// cuts only x, y and z, so every region spans all of t and the eight XCDs
// march through t together, plane by plane: a plane's t +- 1 neighbours are
// the planes the same XCD has just read or reads next.
// Workgroup b runs on XCD b mod 8 as the (b / 8)-th of that XCD's, so it
// takes the entry of the concatenated region list that the XCD-contiguous
// remap gives it.
static void morton_box(const int lo[4], const int len[4], int dims, std::vector<int>& out) {
  int bits[4] = {0, 0, 0, 0}, total = 0;
  for (int d = 0; d < dims; ++d) {
    while ((1 << bits[d]) < len[d]) ++bits[d];
    total += bits[d];
  }
  for (long long code = 0; code < (1LL << total); ++code) {
    int c[4] = {0, 0, 0, 0}, used[4] = {0, 0, 0, 0}, bit = 0;
    while (bit < total)
      for (int d = 0; d < dims && bit < total; ++d)
        if (used[d] < bits[d]) c[d] |= (int)((code >> bit++) & 1) << used[d]++;
    bool inside = true;
    for (int d = 0; d < dims; ++d) inside = inside && c[d] < len[d];
    if (!inside) continue;
    int q = 0;
    for (int d = 0; d < dims; ++d) q |= (lo[d] + c[d]) << (8 * d);
    out.push_back(q);
  }
}

static void region_blocks(int lo[4], int len[4], const int site_ext[4], int parts, int kind, std::vector<int>& out) {
  if (parts > 1) {
    int d = -1;
    long best = 0;
    for (int k = kind == 4 ? 2 : 3; k >= 0; --k)
      if (len[k] >= 2 && (long)len[k] * site_ext[k] > best) {
        best = (long)len[k] * site_ext[k];
        d = k;
      }
    if (d >= 0) {
      int lo2[4], len2[4];
      for (int k = 0; k < 4; ++k) lo2[k] = lo[k], len2[k] = len[k];
      len2[d] = len[d] / 2;
      region_blocks(lo2, len2, site_ext, parts / 2, kind, out);
      lo2[d] = lo[d] + len[d] / 2;
      len2[d] = len[d] - len[d] / 2;
      region_blocks(lo2, len2, site_ext, parts / 2, kind, out);
      return;
    }
  }
  if (kind == 2) {
    morton_box(lo, len, 4, out);
  } else {
    for (int t = 0; t < len[3]; ++t) {
      const size_t at = out.size();
      morton_box(lo, len, 3, out);
      for (size_t i = at; i < out.size(); ++i) out[i] |= (lo[3] + t) << 24;
    }
  }
}

// The table for the current block shape and order (2, 3 or 4) on `stream`,
// built on first use; nullptr when the stream is being captured and the
// table does not exist yet (the launch then uses the index-formula order).
static const int* hop_order_table(dwf_op* op, const HopArgs& A, int kind, hipStream_t stream, int* rc) {
  *rc = DWF_OK;
  const std::array<int, 5> key = {A.bx, A.by, A.bz, A.bt, kind};
  auto it = op->hop_tables.find(key);
  if (it != op->hop_tables.end()) return it->second.dev.as<int>();
  hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
  if (hipStreamIsCapturing(stream, &cs) != hipSuccess || cs != hipStreamCaptureStatusNone) return nullptr;
  dwf_op::OrderTable& t = op->hop_tables[key];
  const int nb[4] = {A.nbx, A.nby, A.nbz, A.nbt};
  const int site_ext[4] = {2 * A.bx, A.by, A.bz, A.bt};
  int lo[4] = {0, 0, 0, 0}, len[4] = {nb[0], nb[1], nb[2], nb[3]};
  std::vector<int> list;
  list.reserve((size_t)nb[0] * nb[1] * nb[2] * nb[3]);
  region_blocks(lo, len, site_ext, 8, kind, list);
  const int n = (int)list.size();
  t.host.resize(n);
  const int q = n >> 3, r = n & 7;
  for (int b = 0; b < n; ++b) {  // the device's xcd_remap, on the host
    const int x = b & 7, k = b >> 3;
    t.host[b] = list[(x < r ? x * (q + 1) : r * (q + 1) + (x - r) * q) + k];
  }
  *rc = t.dev.ensure(sizeof(int) * (size_t)n);
  if (*rc == DWF_OK && hipMemcpyAsync(t.dev.ptr, t.host.data(), sizeof(int) * (size_t)n, hipMemcpyHostToDevice,
                                      stream) != hipSuccess)
    *rc = fail(DWF_ERR_HIP, "hop order table upload failed");
  if (*rc != DWF_OK) {
    op->hop_tables.erase(key);
    return nullptr;
  }
  return t.dev.as<int>();
}

template <typename R, typename T = cplx<R>>
static int hop_launch(dwf_op* op, T* out, const T* in, const T* center,
                      bool dagger, int epi, int out_parity, int nrhs, hipStream_t stream,
                      double* norm_result) {
  const Geom& g = op->g;
  HopArgs A;
  A.g = g;
  A.out_parity = out_parity;
  // linear order: one wave's worth of threads per workgroup (at least one site)
  A.spw = g.Ls >= 64 ? 1 : 64 / g.Ls;
  A.bx = A.by = A.bz = A.bt = 0;
  A.lbx = A.lby = A.lbz = 0;
  A.nbx = A.nby = A.nbz = 1;
  A.remap = op->tune.remap;
  A.nt = op->tune.nt;
  A.morton = 0;
  A.nbt = 1;
  A.order = nullptr;
  A.nrhs = nrhs;
  A.rg = g.Ls == 16 ? std::max(1, std::min(op->tune.rg, nrhs)) : 1;
  {
    const int* b = op->tune.block;
    auto pow2 = [](int n) { return n > 0 && (n & (n - 1)) == 0; };
    if (b[0] > 0 && pow2(b[0]) && pow2(b[1]) && pow2(b[2]) && pow2(b[3]) && b[0] * b[1] * b[2] * b[3] * g.Ls <= 256 &&
        (size_t)b[0] * b[1] * b[2] * b[3] * 12 * (g.Ls + 1) * sizeof(c128) <= 65536 && g.Xh % b[0] == 0 && g.Y % b[1] == 0 &&
        g.Z % b[2] == 0 && g.T % b[3] == 0) {
      A.bx = b[0];
      A.by = b[1];
      A.bz = b[2];
      A.bt = b[3];
      A.spw = b[0] * b[1] * b[2] * b[3];
      A.nbx = g.Xh / b[0];
      A.nby = g.Y / b[1];
      A.nbz = g.Z / b[2];
      A.nbt = g.T / b[3];
      A.lbx = __builtin_ctz(b[0]);
      A.lby = __builtin_ctz(b[1]);
      A.lbz = __builtin_ctz(b[2]);
      const bool p2 = pow2(A.nbx) && pow2(A.nby) && pow2(A.nbz) && pow2(A.nbt);
      A.morton = op->tune.morton != 0 && p2;
      if (op->tune.morton >= 2 && A.nbx <= 256 && A.nby <= 256 && A.nbz <= 256 && A.nbt <= 128) {
        int rc = DWF_OK;
        A.order = hop_order_table(op, A, op->tune.morton, stream, &rc);
        HDCG_TRY(rc);
      }
    }
  }
  A.field = (size_t)g.Vh * 12 * g.Ls;
  A.alpha = op->f5.alpha;
  A.beta = op->f5.beta;
  A.ia = op->f5.ia;
  A.kap = op->f5.kap;
  A.b5 = op->f5.b5;
  A.c5 = op->f5.c5;
  A.mass = op->f5.mass;
  const bool mob = op->f5.mobius;
  A.partials = nullptr;
  A.counters = nullptr;
  A.result = nullptr;
  const int threads = ((A.spw * g.Ls + 63) / 64) * 64;
  const int nwg = (g.Vh + A.spw - 1) / A.spw;
  A.pstride = (size_t)nwg;
  if (norm_result) {
    if (nrhs > 64) return fail(DWF_ERR_ARG, "nrhs > 64");
    HDCG_TRY(op->hop_part.ensure(sizeof(double) * (size_t)nwg * nrhs));
    A.partials = op->hop_part.as<double>();
    A.counters = op->red.counters.as<unsigned>();
    A.result = norm_result;
  }
  const bool dbl = sizeof(R) == 8;
  const cplx<R>* G = reinterpret_cast<const cplx<R>*>(dbl ? op->gauge128.ptr : op->gauge64.ptr) +
                     (size_t)out_parity * g.Vh * 72;
  const R* pw = reinterpret_cast<const R*>(dbl ? op->pw128.ptr : op->pw64.ptr);
  dim3 grid(nwg, (nrhs + A.rg - 1) / A.rg), block(threads);
  const size_t epi_lds = (epi == EPI_INV || (mob && dagger)) ? (size_t)A.spw * 12 * (g.Ls + 1) * sizeof(cplx<R>) : 0;
  const size_t link_lds = (size_t)A.spw * kLinkLd * sizeof(cplx<R>);
  size_t lds;
  if (A.rg > 1 && epi_lds > 0) {  // separate regions: the links stay for the next right-hand side
    A.epi_off = (int)((link_lds + 15) / 16 * 16);
    lds = A.epi_off + epi_lds;
  } else {
    A.epi_off = 0;
    lds = std::max(epi_lds, link_lds);
  }
  // optional LDS request that caps the resident workgroups per CU
  if ((size_t)op->tune.lds_kb * 1024 > lds) lds = (size_t)op->tune.lds_kb * 1024;
  // directions whose neighbour loads are in flight together: 8 / phases
  // (the Mobius kernels are built for four phases only)
  const int phases = op->tune.phases > 0 ? op->tune.phases : (sizeof(R) == 8 ? 4 : 2);
  const bool two = phases == 4 || mob;
  if (mob) {
    if (g.Ls == 16)
      launch_hop<R, 4, 16, true, T>(dagger, epi, grid, block, lds, stream, out, in, center, G, pw, A);
    else
      launch_hop<R, 4, 0, true, T>(dagger, epi, grid, block, lds, stream, out, in, center, G, pw, A);
  } else if (g.Ls == 16) {
    if (two)
      launch_hop<R, 4, 16, false, T>(dagger, epi, grid, block, lds, stream, out, in, center, G, pw, A);
    else
      launch_hop<R, 2, 16, false, T>(dagger, epi, grid, block, lds, stream, out, in, center, G, pw, A);
  } else {
    if (two)
      launch_hop<R, 4, 0, false, T>(dagger, epi, grid, block, lds, stream, out, in, center, G, pw, A);
    else
      launch_hop<R, 2, 0, false, T>(dagger, epi, grid, block, lds, stream, out, in, center, G, pw, A);
  }
  HDCG_HIP(hipGetLastError());
  if (norm_result) return launch_finalize(1, A.partials, nwg, nwg, nrhs, norm_result, stream, A.pstride);
  return DWF_OK;
}

template <typename R, typename T>
int launch_mpc(dwf_op* op, T* out, const T* in, bool dagger, int nrhs, hipStream_t stream,
               double* norm_result) {
  const int prec = std::is_same<T, bf16c>::value ? DWF_BF16 : prec_of<R>();
  if (kSMajor<T> && (!aligned16(out) || !aligned16(in)))
    return fail(DWF_ERR_ARG, "16-bit fields must be 16-byte aligned");
  HDCG_TRY(ensure_tmp(op, prec, nrhs));
  T* te = op->tmp[tmp_index(prec)][0].as<T>();
  // stage 1: t_e = M_5^-1 Dh_eo in    (adjoint: M_5^-+ Dh^+_eo in)
  HDCG_TRY((hop_launch<R, T>(op, te, in, nullptr, dagger, EPI_INV, 0, nrhs, stream, nullptr)));
  // stage 2: out = M_5 in - 1/4 Dh_oe t_e  (adjoint: M_5^+ in - 1/4 Dh^+_oe t_e)
  HDCG_TRY((hop_launch<R, T>(op, out, te, in, dagger, EPI_SUB, 1, nrhs, stream, norm_result)));
  return DWF_OK;
}

// ------------------------------------------------ launch-shape autotuner --
// Candidate launch shapes of the hop stages: the workgroup's site block in
// (x/2, y, z, t) and whether workgroups are reordered XCD-contiguously.  Which
// is fastest depends on the lattice (how the block grid divides over the 8
// XCDs and their L2 caches) and on the bytes per site; on 16^4 x 16 the
// 2x2x1x1 XCD-contiguous Morton order wins, on 24^3 x 48 x 16 (a block grid
// that is not a power of two) other shapes do.
struct HopShape {
  int block[4];
  int remap;
  int order;  // 1 Morton (index formula), 2-4 region tables
  int rg;     // right-hand sides per workgroup (candidates with rg > 1 are tried only for several)
};
constexpr HopShape kHopShapes[] = {
    {{2, 2, 1, 1}, 1, 1, 1},  {{2, 2, 1, 1}, 0, 1, 1},  {{2, 2, 2, 2}, 1, 1, 1}, {{2, 2, 2, 2}, 0, 1, 1},
    {{4, 2, 1, 1}, 1, 1, 1},  {{1, 2, 2, 1}, 1, 1, 1},  {{2, 2, 1, 1}, 1, 2, 1}, {{1, 2, 2, 1}, 1, 2, 1},
    {{2, 2, 1, 1}, 1, 3, 1},  {{2, 2, 2, 2}, 1, 2, 1},  {{2, 2, 1, 1}, 1, 4, 1}, {{1, 2, 2, 1}, 1, 4, 1},
    {{2, 2, 2, 2}, 1, 4, 1},  {{2, 2, 1, 1}, 1, 4, 16}, {{2, 2, 1, 1}, 1, 1, 16}, {{1, 2, 2, 1}, 1, 4, 16},
    {{2, 2, 1, 1}, 0, 0, 16}, {{2, 2, 1, 1}, 1, 4, 4}};
constexpr int kNumHopShapes = sizeof(kHopShapes) / sizeof(kHopShapes[0]);
static_assert(kNumHopShapes <= 24, "hop_ms holds 24 candidates");

int hop_shape_candidates() { return kNumHopShapes; }
void hop_shape_of(int c, int shape[7]) {
  for (int i = 0; i < 4; ++i) shape[i] = kHopShapes[c].block[i];
  shape[4] = kHopShapes[c].remap;
  shape[5] = kHopShapes[c].order;
  shape[6] = kHopShapes[c].rg;
}

static void apply_shape(dwf_op* op, int c) {
  for (int i = 0; i < 4; ++i) op->tune.block[i] = kHopShapes[c].block[i];
  op->tune.remap = kHopShapes[c].remap;
  op->tune.morton = kHopShapes[c].order;
  op->tune.rg = kHopShapes[c].rg;
}

template <typename R, typename T>
static int apply_mpcdagmpc(dwf_op* op, T* out, const T* in, int nrhs, hipStream_t stream, double* pap_result) {
  const int prec = std::is_same<T, bf16c>::value ? DWF_BF16 : prec_of<R>();
  HDCG_TRY(ensure_tmp(op, prec, nrhs));
  T* chi = op->tmp[tmp_index(prec)][1].as<T>();
  HDCG_TRY((launch_mpc<R, T>(op, chi, in, false, nrhs, stream, pap_result)));
  HDCG_TRY((launch_mpc<R, T>(op, out, chi, true, nrhs, stream, nullptr)));
  return DWF_OK;
}

// The shape for (storage, right-hand sides): tuned on this call's own
// operands the first time (one warm-up and the best of three applications of
// H per candidate, timed with HIP events on the stream), unless the stream is
// being captured into a graph (then the default until a later call tunes).
template <typename R, typename T>
static int select_shape(dwf_op* op, T* out, const T* in, int nrhs, hipStream_t st) {
  if (!op->hop_autotune) return DWF_OK;
  const int pi = tmp_index(std::is_same<T, bf16c>::value ? DWF_BF16 : prec_of<R>()), ri = nrhs > 1;
  int& choice = op->hop_choice[pi][ri];
  if (choice < 0) {
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    if (hipStreamIsCapturing(st, &cs) != hipSuccess || cs != hipStreamCaptureStatusNone) {
      apply_shape(op, 0);
      return DWF_OK;
    }
    hipEvent_t e0, e1;
    HDCG_HIP(hipEventCreate(&e0));
    HDCG_HIP(hipEventCreate(&e1));
    int rc = DWF_OK, best = 0;
    float bms = 0.f;
    for (int c = 0; c < kNumHopShapes && rc == DWF_OK; ++c) {
      op->hop_ms[pi][ri][c] = -1.f;
      if (kHopShapes[c].rg > 1 && nrhs == 1) continue;  // the same as its one-RHS form
      apply_shape(op, c);
      rc = apply_mpcdagmpc<R, T>(op, out, in, nrhs, st, nullptr);
      float m = 1e30f;
      for (int rep = 0; rep < 3 && rc == DWF_OK; ++rep) {
        float x = 0.f;
        if (hipEventRecord(e0, st) != hipSuccess) rc = fail(DWF_ERR_HIP, "hop autotuner event failed");
        if (rc == DWF_OK) rc = apply_mpcdagmpc<R, T>(op, out, in, nrhs, st, nullptr);
        if (rc == DWF_OK && (hipEventRecord(e1, st) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
                             hipEventElapsedTime(&x, e0, e1) != hipSuccess))
          rc = fail(DWF_ERR_HIP, "hop autotuner event failed");
        m = std::min(m, x);
      }
      op->hop_ms[pi][ri][c] = m;
      if (rc == DWF_OK && (c == 0 || m < bms)) {
        bms = m;
        best = c;
      }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    HDCG_TRY(rc);
    choice = best;
  }
  apply_shape(op, choice);
  return DWF_OK;
}

template <typename R, typename T>
int launch_mpcdagmpc(dwf_op* op, T* out, const T* in, int nrhs, hipStream_t stream, double* pap_result) {
  HDCG_TRY((select_shape<R, T>(op, out, in, nrhs, stream)));
  return apply_mpcdagmpc<R, T>(op, out, in, nrhs, stream, pap_result);
}

template <typename R, typename T>
int launch_norm2(dwf_op* op, const T* x, int nrhs, double* result, hipStream_t stream) {
  RedArgs A{op->field_elems(1), op->red.partials.as<double>(), op->red.counters.as<unsigned>(),
            result};
  if (nrhs > 64) return fail(DWF_ERR_ARG, "nrhs > 64");
  dim3 grid(red_blocks(A.n), nrhs);
  hipLaunchKernelGGL((norm2_kernel<T>), grid, dim3(256), 0, stream, x, A);
  HDCG_HIP(hipGetLastError());
  return launch_finalize(1, A.partials, kMaxPartials, grid.x, nrhs, result, stream);
}

template <typename R>
int launch_dot(dwf_op* op, const cplx<R>* a, const cplx<R>* b, int nrhs, double* result,
               hipStream_t stream) {
  RedArgs A{op->field_elems(1), op->red.partials.as<double>(), op->red.counters.as<unsigned>(),
            result};
  if (nrhs > 64) return fail(DWF_ERR_ARG, "nrhs > 64");
  dim3 grid(red_blocks(A.n), nrhs);
  hipLaunchKernelGGL((dot_kernel<R>), grid, dim3(256), 0, stream, a, b, A);
  HDCG_HIP(hipGetLastError());
  return launch_finalize(2, A.partials, kMaxPartials / 2, grid.x, nrhs, result, stream);
}

template <typename R>
int launch_cg_update(dwf_op* op, cplx<R>* x, cplx<R>* r, const cplx<R>* p, const cplx<R>* w,
                     const double* num, const double* den, const double* alpha_host, double* rr,
                     int nrhs, hipStream_t stream) {
  RedArgs A{op->field_elems(1), op->red.partials.as<double>(), op->red.counters.as<unsigned>(), rr};
  if (nrhs > 64) return fail(DWF_ERR_ARG, "nrhs > 64");
  dim3 grid(red_blocks(A.n), nrhs);
  hipLaunchKernelGGL((cg_update_kernel<R>), grid, dim3(256), 0, stream, x, r, p, w, num, den,
                     alpha_host, A);
  HDCG_HIP(hipGetLastError());
  return launch_finalize(1, A.partials, kMaxPartials, grid.x, nrhs, rr, stream);
}

template <typename R>
int launch_xpay(dwf_op* op, cplx<R>* p, const cplx<R>* r, const double* num, const double* den,
                const double* beta_host, int nrhs, hipStream_t stream) {
  const size_t n = op->field_elems(1);
  dim3 grid(red_blocks(n), nrhs);
  hipLaunchKernelGGL((xpay_kernel<R>), grid, dim3(256), 0, stream, p, r, num, den, beta_host, n);
  HDCG_HIP(hipGetLastError());
  return DWF_OK;
}

template <typename R>
int launch_axpby(dwf_op*, cplx<R>* y, const cplx<R>* x, double a, double b, size_t n,
                 hipStream_t stream) {
  hipLaunchKernelGGL((axpby_kernel<R>), dim3(red_blocks(n)), dim3(256), 0, stream, y, x, (R)a,
                     (R)b, n);
  HDCG_HIP(hipGetLastError());
  return DWF_OK;
}

static bool aligned16(const void* p) { return (reinterpret_cast<uintptr_t>(p) & 15) == 0; }

int launch_convert16(dwf_op* op, bf16c* dst, const c64* src, int nrhs, hipStream_t stream) {
  if (!aligned16(dst)) return fail(DWF_ERR_ARG, "16-bit fields must be 16-byte aligned");
  const size_t rows = (size_t)nrhs * op->g.Vh * op->g.Ls;
  hipLaunchKernelGGL(to_bf16_kernel, dim3(red_blocks(rows * 12)), dim3(256), 0, stream, dst, src, rows, op->g.Ls);
  HDCG_HIP(hipGetLastError());
  return DWF_OK;
}
int launch_convert16(dwf_op* op, c64* dst, const bf16c* src, int nrhs, hipStream_t stream) {
  if (!aligned16(src)) return fail(DWF_ERR_ARG, "16-bit fields must be 16-byte aligned");
  const size_t rows = (size_t)nrhs * op->g.Vh * op->g.Ls;
  hipLaunchKernelGGL(from_bf16_kernel, dim3(red_blocks(rows * 12)), dim3(256), 0, stream, dst, src, rows,
                     op->g.Ls);
  HDCG_HIP(hipGetLastError());
  return DWF_OK;
}

template <typename Td, typename Ts>
int launch_convert(Td* dst, const Ts* src, size_t n, hipStream_t stream) {
  hipLaunchKernelGGL((convert_kernel<Td, Ts>), dim3(red_blocks(n)), dim3(256), 0, stream, dst, src, n);
  HDCG_HIP(hipGetLastError());
  return DWF_OK;
}

#define INST(R)                                                                                 \
  template int launch_mpc<R, cplx<R>>(dwf_op*, cplx<R>*, const cplx<R>*, bool, int, hipStream_t, double*); \
  template int launch_mpcdagmpc<R, cplx<R>>(dwf_op*, cplx<R>*, const cplx<R>*, int, hipStream_t, double*); \
  template int launch_norm2<R, cplx<R>>(dwf_op*, const cplx<R>*, int, double*, hipStream_t);    \
  template int launch_dot<R>(dwf_op*, const cplx<R>*, const cplx<R>*, int, double*, hipStream_t); \
  template int launch_cg_update<R>(dwf_op*, cplx<R>*, cplx<R>*, const cplx<R>*, const cplx<R>*, \
                                   const double*, const double*, const double*, double*, int,  \
                                   hipStream_t);                                                \
  template int launch_xpay<R>(dwf_op*, cplx<R>*, const cplx<R>*, const double*, const double*,  \
                              const double*, int, hipStream_t);                                 \
  template int launch_axpby<R>(dwf_op*, cplx<R>*, const cplx<R>*, double, double, size_t,      \
                               hipStream_t);
INST(double)
INST(float)
template int launch_mpc<float, bf16c>(dwf_op*, bf16c*, const bf16c*, bool, int, hipStream_t, double*);
template int launch_mpcdagmpc<float, bf16c>(dwf_op*, bf16c*, const bf16c*, int, hipStream_t, double*);
template int launch_norm2<float, bf16c>(dwf_op*, const bf16c*, int, double*, hipStream_t);
template int launch_convert<c128, c64>(c128*, const c64*, size_t, hipStream_t);
template int launch_convert<c64, c128>(c64*, const c128*, size_t, hipStream_t);


// ------------------------------------------------------------ host setup ---
int import_gauge(dwf_op* op, const void* gauge_c128, hipStream_t stream) {
  const Geom& g = op->g;
  HDCG_TRY(op->gauge128.ensure(sizeof(c128) * 2 * (size_t)g.Vh * 72));
  HDCG_TRY(op->gauge64.ensure(sizeof(c64) * 2 * (size_t)g.Vh * 72));
  double4 bcxy = make_double4(op->bc[0], op->bc[1], op->bc[2], op->bc[3]);
  double4 bczt = make_double4(op->bc[4], op->bc[5], op->bc[6], op->bc[7]);
  const int n = 2 * g.Vh;
  hipLaunchKernelGGL(gauge_import_kernel, dim3((n + 127) / 128), dim3(128), 0, stream,
                     static_cast<const c128*>(gauge_c128), op->gauge128.as<c128>(),
                     op->gauge64.as<c64>(), g, bcxy, bczt);
  HDCG_HIP(hipGetLastError());
  return DWF_OK;
}

template <typename R>
int launch_layout(dwf_op* op, void* dst, const void* src, int nrhs, bool to_native,
                  hipStream_t stream) {
  const size_t total = op->field_elems(nrhs);
  const int blocks = (int)((total + 255) / 256);
  if (to_native)
    hipLaunchKernelGGL((field_layout_kernel<R, true>), dim3(blocks), dim3(256), 0, stream,
                       static_cast<cplx<R>*>(dst), static_cast<const cplx<R>*>(src), op->g.Ls,
                       op->g.Vh, total);
  else
    hipLaunchKernelGGL((field_layout_kernel<R, false>), dim3(blocks), dim3(256), 0, stream,
                       static_cast<cplx<R>*>(dst), static_cast<const cplx<R>*>(src), op->g.Ls,
                       op->g.Vh, total);
  HDCG_HIP(hipGetLastError());
  return DWF_OK;
}
template int launch_layout<double>(dwf_op*, void*, const void*, int, bool, hipStream_t);
template int launch_layout<float>(dwf_op*, void*, const void*, int, bool, hipStream_t);

}  // namespace hdk
