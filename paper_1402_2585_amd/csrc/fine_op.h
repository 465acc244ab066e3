// The fine domain-wall operator: handle state and host-side launchers.
//
// Native half-field layout (private): field[rhs][cb][c][s] with
// c = spin*3 + colour (12 components) and s innermost, complex.  One 4D
// site's whole fifth-dimension column is contiguous (12*Ls complex), so a
// workgroup owning a few sites and all their s reads and writes long
// contiguous runs, reuses each gauge link Ls times, and can apply the dense-
// in-s inverse M_5^-1 from LDS.
//
// Native gauge layout (private): gauge[parity][cb][dir][3][3] for the sites
// of each parity; dir 0..3 = U_mu(x) (times zeta_mu when x_mu = L_mu - 1),
// dir 4..7 = U_mu(x - mu)^+ (times conj(zeta_mu) when x_mu = 0).  Each hop
// stage reads the eight links of its output site contiguously.
#pragma once

#include <array>
#include <map>
#include <vector>

#include "common.h"

namespace hdk {

struct Geom {
  int X, Y, Z, T;  // 4D extents
  int Xh;          // X / 2
  int Ls;
  int Vh;          // sites per checkerboard
};

// Fifth dimension of the domain-wall kernel.  Mobius (Cayley form) with
// C_5 = b5 + c5 K and M_5 = alpha + beta K, K the chiral shift (P+ from s-1,
// P- from s+1, -mass at the wrap); Shamir is b5 = 1, c5 = 0 (alpha = 5 - M5,
// beta = -1).  M_5^-1 on P+: pw[(s - s') mod Ls] (s >= s' ? 1 : -mass) with
// pw[n] = kap^n / (alpha (1 + mass kap^Ls)), kap = -beta / alpha, and the
// recurrence y_s = ia x_s + kap y_{s-1}, ia = 1 / alpha.
struct FifthDim {
  double alpha, beta, ia, kap;
  double b5, c5;
  bool mobius;
  double mass;
  double pw[64];
};

struct dwf_op_impl;

}  // namespace hdk

struct dwf_op {
  hdk::Geom g;
  double M5, mass;
  double bc[8];
  hdk::FifthDim f5;
  hdk::DevBuf gauge128, gauge64;  // [2][Vh][8][9]
  hdk::DevBuf pw128, pw64;        // closed-form table on the device
  hdk::DevBuf tmp[3][3];          // [c128, c64, bf16][t_e, chi, s_e] work fields
  hdk::DevBuf cgw[4];             // CG work fields (c128): r, p, w, spare
  hdk::DevBuf mgw[5];             // mixed-precision CG work fields (c64): r, p, w, source, correction
  hdk::DevBuf msw[4];             // multi-shift CG: p_j (c128), r, w, device scalars
  hdk::Reducer red;
  hdk::DevBuf hop_part;           // fused-norm partials of the hop stage: [rhs][workgroups]
  struct {
    // hop launch shape (measured best on MI355X at 16^4 and 24^3x48, Ls = 16;
    // block, remap and order are the autotuner's)
    int block[4] = {2, 2, 1, 1};  // workgroup site block in (x/2, y, z, t), powers of two; 0 = linear
    int remap = 1;                // XCD-contiguous workgroup order
    int lds_kb = 0;               // minimum LDS per workgroup (caps occupancy)
    int nt = 0;                   // non-temporal output stores
    int morton = 1;               // block order: 0 lexicographic, 1 Morton (power-of-two block
                                  // grids), 2-4 per-XCD regions from a table
    int phases = 0;               // neighbour-load phases per stage (2 or 4; 0: 4 for complex128,
                                  // 2 for the FP32 kernels, whose spinors take half the registers)
    int rg = 1;                   // right-hand sides per workgroup (sharing the links staged in LDS)
  } tune;
  // launch-shape autotuner: the candidate chosen per (field storage c128 /
  // c64 / 16-bit, one / several right-hand sides), -1 before it has run;
  // off after dwf_set_hop_shape fixes a shape
  int hop_autotune = 1;
  int hop_choice[3][2] = {{-1, -1}, {-1, -1}, {-1, -1}};
  float hop_ms[3][2][24] = {};  // measured ms per H of each candidate (-1: not tried)
  // workgroup -> site-block tables of the region orders, one per
  // (bx, by, bz, bt, order); built on first use outside graph capture, kept
  // until the operator is destroyed (a launch in flight may still read one)
  struct OrderTable {
    std::vector<int> host;
    hdk::DevBuf dev;
  };
  std::map<std::array<int, 5>, OrderTable> hop_tables;
  hdk::DevBuf host_pinned_dummy;
  double* pinned = nullptr;        // host pinned scalars [kPinnedDoubles]
  int device = 0;
  size_t site_elems() const { return (size_t)12 * g.Ls; }
  size_t field_elems(int nrhs) const { return (size_t)nrhs * g.Vh * 12 * g.Ls; }
};

namespace hdk {

// Launch helpers (all asynchronous on `stream`).
// Fields stored as T (cplx<R>, or bf16c with R = float), arithmetic in R.
template <typename R, typename T = cplx<R>>
int launch_mpc(dwf_op* op, T* out, const T* in, bool dagger, int nrhs, hipStream_t stream,
               double* norm_result /*nullable: |M_pc in|^2 per rhs*/);
template <typename R, typename T = cplx<R>>
int launch_mpcdagmpc(dwf_op* op, T* out, const T* in, int nrhs, hipStream_t stream,
                     double* pap_result /*nullable: <in, H in> = |M_pc in|^2 per rhs*/);

// BLAS-1 (FP64 accumulation); results are device doubles, one per rhs.
template <typename R, typename T = cplx<R>>
int launch_norm2(dwf_op* op, const T* x, int nrhs, double* result, hipStream_t stream);
template <typename R>
int launch_dot(dwf_op* op, const cplx<R>* a, const cplx<R>* b, int nrhs, double* result /*2*nrhs*/,
               hipStream_t stream);
// x += alpha p ; r -= alpha w ; |r|^2 -> rr.  alpha = num[i]/den[i] (device)
// or alpha_host if num == nullptr.
template <typename R>
int launch_cg_update(dwf_op* op, cplx<R>* x, cplx<R>* r, const cplx<R>* p, const cplx<R>* w,
                     const double* num, const double* den, const double* alpha_host, double* rr,
                     int nrhs, hipStream_t stream);
// p = r + beta p, beta = num/den (device) or beta_host.
template <typename R>
int launch_xpay(dwf_op* op, cplx<R>* p, const cplx<R>* r, const double* num, const double* den,
                const double* beta_host, int nrhs, hipStream_t stream);
// y = a*x + b*y (generic real coefficients on host)
template <typename R>
int launch_axpby(dwf_op* op, cplx<R>* y, const cplx<R>* x, double a, double b, size_t n,
                 hipStream_t stream);
// Multi-shift CG (complex128): (H + shifts[j]) x_j = b for j < ns (<= 8),
// shifts[0] the smallest; x: [ns][nrhs] fields, overwritten (starts from 0).
// Stops when |r| <= tol |b| for the base system of every right-hand side;
// *iters = iterations run, *resid = max relative base residual (the value
// checked last).  Synchronises; DWF_NOT_CONVERGED at maxiter.
int multishift_cg(dwf_op* op, c128* x, const c128* b, int nrhs, const double* shifts, int ns, double tol,
                  int maxiter, int* iters, double* resid, hipStream_t stream);
// out = sum_j coef[j] x_j over nrhs fields (x: [ns][nrhs] fields)
int multishift_combine(dwf_op* op, c128* out, const c128* x, int nrhs, const double* coef, int ns,
                       hipStream_t stream);
// keep only P- at s = 0 and P+ at s = Ls - 1 (the physical wall components)
int wall_mask(dwf_op* op, c128* f, int nrhs, hipStream_t stream);

// dst = src between c128 and c64 (n complex values), rounded to nearest even
template <typename Td, typename Ts>
int launch_convert(Td* dst, const Ts* src, size_t n, hipStream_t stream);
// complex64 <-> 16-bit native fields (nrhs of them; the 16-bit native layout
// keeps each site s-major), rounded to nearest even
int launch_convert16(dwf_op* op, bf16c* dst, const c64* src, int nrhs, hipStream_t stream);
int launch_convert16(dwf_op* op, c64* dst, const bf16c* src, int nrhs, hipStream_t stream);

// the hop launch-shape candidates of the autotuner: their number, and
// candidate c as {bx, by, bz, bt, remap, order, rhs per workgroup}
int hop_shape_candidates();
void hop_shape_of(int c, int shape[7]);

int ensure_tmp(dwf_op* op, int prec, int nrhs);
void release_tmp(dwf_op* op);  // drop the operator's work fields (regrown on demand)
int ensure_reducer(dwf_op* op);

}  // namespace hdk
