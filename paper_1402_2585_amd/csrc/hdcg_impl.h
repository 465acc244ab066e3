// HDCG handle: blocked subspace, little Dirac operator and solver state.
//
// Blocks are 4D (B_mu sites, every B_mu even and >= 4) and span all of s
// (Sec. V.A).  Odd site j of block a (j = rank by checkerboard index) has
// the native fine-field column site_of[a][j]; a block vector is stored as
// phi[a][k][j][c][s] (block-major: the Nvec vectors of one block are one
// contiguous (Nvec x n_b) panel, n_b = nsb * 12 * Ls).
//
// Coarse vectors: c[rhs][a][k].  Little Dirac operator: A128 is the
// canonical A[a][l][j][k] (complex128); AT64 is the complex64 copy stored
// transposed per stencil point, AT[a][l][k][j], so the mat-vec reads it with
// consecutive threads on consecutive j.
#pragma once

#include <vector>

#include "blas.h"
#include "fine_op.h"

constexpr int kStencil = 81;

// Phases of a solve, the categories of Fig. "pie" (Sec. VI.B).
enum { PH_FINE_DP, PH_FINE_SP, PH_COARSE, PH_PROJ, PH_LINALG, PH_CONVERT, PH_N };

// Optional hipEvent timing of the phases on the solve's stream: each phase
// section records an event pair; collect() (after a synchronisation of the
// stream) adds the elapsed times per category and recycles the events.
struct PhaseTimer {
  bool on = false;
  std::vector<hipEvent_t> pool;
  std::vector<int> cat;  // category of event pair i (events 2i, 2i + 1)
  size_t used = 0;
  double sec[PH_N] = {};
  int begin(int c, hipStream_t st);  // index of the pair, -1 when off
  void end(int idx, hipStream_t st);
  int collect();
  void reset() {
    used = 0;
    for (double& v : sec) v = 0.0;
  }
  ~PhaseTimer();
};

struct hdcg {
  dwf_op* op = nullptr;
  int B[4] = {0, 0, 0, 0};
  int C[4] = {0, 0, 0, 0};
  int Nc = 0, nsb = 0, nvec = 0;
  size_t nb = 0;  // complex per block vector
  hdk::DevBuf site_of;        // int [Nc][nsb]
  hdk::DevBuf nbr;            // int [Nc][81]
  hdk::DevBuf phi128, phi64;  // [Nc][nvec][nb]
  hdk::DevBuf phi16;          // the same in 16 bits (bf16 pairs) when phi_prec asks for it
  int sd = 0;                 // surface depth in force (0: every s slice of the subspace kept)
  hdk::DevBuf phis64, phis16; // the solve's subspace, surface slices only (sd > 0): [Nc][nvec][nsb][12][2 sd]
  hdk::DevBuf A128;           // [Nc][81][nvec][nvec]
  hdk::DevBuf AT64;           // [Nc][81][nvec][nvec] transposed per l
  hdk::DevBuf AT128;          // same layout in complex128 (parity / FP64 use)
  hdk::DevBuf gram, rinv;     // [Nc][nvec][nvec] c128 Cholesky-QR work
  hdk::DevBuf flag;           // int error flag
  hdk::DevBuf cw[10];         // coarse work vectors (c64/c128); 6-9: truncated-operator preconditioner
  hdk::DevBuf fw64[12];       // fine c64 work fields: 0-7 solver, 8-10 fine CG
  hdk::DevBuf fw128[3];       // fine c128 work fields
  hdk::DevBuf fw16[4];        // fine 16-bit work fields of M_IRS: x, r, p, w
  hdk::DevBuf scal;           // device scalars
  hdk::DevBuf probe_c;        // coarse probe vectors for the build
  hdk::DevBuf mf_rho, mf_smax;      // per-matrix scales of the 16-bit coarse storage
  hdk::DevBuf mf_bf16, mf_f16;      // MFMA fragment-ordered 16-bit coarse matrices
  int mf_have_bf16 = 0, mf_have_f16 = 0;
  hdk::DevBuf pcg_part;             // persistent coarse CG: per-workgroup partial sums
  hdk::DevBuf pcg_state;            // persistent coarse CG: grid barrier, status, iterations
  int persistent_coarse = 1;        // run the coarse CG as one persistent kernel when it applies
  // second deflation level of the coarse operator (Sec. V.B): ng global
  // vectors Z (orthonormal, E = Z^+ A Z = diag(D)) and A Z, complex128 and
  // complex64, [ng][Nc * nvec]
  int ng = 0;
  hdk::DevBuf ldZ128, ldAZ128, ldZ64, ldAZ64;
  hdk::DevBuf ldD;                  // double [ng]
  hdk::DevBuf ldc;                  // coefficients [64][1024] complex128
  hdk::DevBuf ldpart;               // sliced partial sums of the coefficients [nr][ng][slices]
  std::vector<double> ldDh;         // D on the host
  // the truncated operator Q_trunc + m1_shift (Sec. V.B): zero- and one-hop
  // terms, TT[a][m][k][j] for the 9 points m, and their neighbour table
  hdk::DevBuf TT64, TT128, nbr9;
  double tt_shift64 = __builtin_nan(""), tt_shift128 = __builtin_nan("");  // shift TT was built with
  // Q_trunc + m1_shift in the 16-bit MFMA storage (m1_prec BF16 / F16): scales and fragments
  hdk::DevBuf tq_rho, tq_smax, tq_bf16, tq_f16;
  double tq_shift_bf16 = __builtin_nan(""), tq_shift_f16 = __builtin_nan("");
  double m1_hi_est = 0.0;           // estimated Chebyshev upper bound (m1_hi <= 0)
  hdk::DevBuf ycw;                  // ADEF1 coarse solve: the preconditioned residual
  double* pinned = nullptr;   // host pinned scalars [16][64]
  struct {
    int n_ii = 0;
    double lambda_ii = 0.0, tol_ii = 1e-4;
    int maxiter_ii = 500;
    int n_irs = 7;
    double lambda_irs = 1.0;
    double coarse_tol = 0.04;
    int coarse_maxiter = 2000;
    int flexible = 1;
    double inner_tol = 1e-5;
    int inner_maxiter = 500;
    int outer_maxiter = 50;
    int build_batch = 8;
    int coarse_prec = DWF_C64;  // storage of A inside Q: C64 (VALU), BF16 / F16 (MFMA)
    int irs_prec = DWF_C64;     // storage of the M_IRS fields: C64 or BF16
    int subspace_gen = 0;       // 1: rational filter (multi-shift) before inverse iteration
    double rat_lo = 3e-4, rat_eps = 1e-4, rat_tol = 1e-6;
    int rat_maxiter = 10000;
    int wall_noise = 0;         // keep only the physical wall components of the noise
    int ldop_defl = 1;          // deflate coarse solves with the second level once it is built
    int phi_prec = DWF_C64;     // subspace storage for the solve's project / promote: C64 or BF16
    int ldop_m1 = 0;            // 1: deflated coarse solves run ADEF1 with Chebyshev(Q_trunc)
    double m1_lo = 0.5, m1_hi = 0.0;  // Chebyshev interval (m1_hi <= 0: estimated)
    int m1_order = 16;          // Chebyshev order (m1_order - 1 truncated mat-vecs)
    double m1_shift = 0.0;      // infra-red shift added to Q_trunc
    int m1_prec = DWF_C64;      // Q_trunc storage for complex64 solves: C64, or BF16 / F16 (MFMA)
    int surface_depth = 0;      // > 0 and 2 depth < Ls: remove the subspace's fifth-dimension interior
    int verbose = 0;            // print setup progress to stderr
  } prm;
  double setup_seconds = 0.0;
  long long setup_matmuls = 0;
  int last_coarse_iters[64] = {};   // per right-hand side, the last hdcg_coarse_solve
  int last_coarse_nrhs = 0;
  PhaseTimer timer;                 // phase times of the solve (params.phase_timing)
  int use_graph = 1;                // capture the preconditioner as a graph when it has no host step
  int mfma_tile = -1;               // 16-bit mat-vec tile: -1 autotuned per shape, >= 0 a fixed candidate
  unsigned long long seed = 1;      // seed of the starting vectors drawn when the caller gives none
  int keep_phi128 = 1;              // keep the FP64 subspace after setup
  hipStream_t cap_stream = nullptr; // stream the preconditioner is captured on (never run on)
};

namespace hdk {

// kernels (hdcg_kernels.hip)
int blk_build_maps(hdcg* h, hipStream_t st);
template <typename R>
int blk_phi_layout(hdcg* h, cplx<R>* phi_native, const cplx<double>* canonical, bool to_native,
                   int kcount, hipStream_t st);
// out[r*sr + a*sa + k*sk] (+ph[a] factor) = sum_i conj(P[a][k][i]) * Q(r, a, i)
// Q from a native fine field set (fine != nullptr, nr fields, field stride fstride) or a
// block-major panel (blockq: [a][nr][nb]).
template <typename R>
int blk_dot(hdcg* h, const cplx<R>* P, const cplx<R>* fine, size_t fstride,
            const cplx<R>* blockq, int nr, cplx<R>* out, size_t sr, size_t sa, size_t sk,
            const cplx<double>* phase, hipStream_t st);
// fine_out[r] = (base ? base[r] : 0) + sign * sum_k P[a][k][i] c[r][a][k]
template <typename R>
int blk_promote(hdcg* h, const cplx<R>* P, const cplx<R>* c, int nr, cplx<R>* fine_out,
                const cplx<R>* base, double sign, size_t fstride, hipStream_t st);
// the same two with the subspace stored in 16 bits (complex64 vectors)
int blk_dot(hdcg* h, const bf16c* P, const cplx<float>* fine, size_t fstride, int nr, cplx<float>* out, size_t sr,
            size_t sa, size_t sk, hipStream_t st);
int blk_promote(hdcg* h, const bf16c* P, const cplx<float>* c, int nr, cplx<float>* fine_out,
                const cplx<float>* base, double sign, size_t fstride, hipStream_t st);
// the same two on MFMA for several right-hand sides (blk_mfma.hip): 16-byte
// aligned subspace and fields, full site columns (sd == 0), nvec <= 64
bool blk_mfma_applies(hdcg* h, const void* P, const void* field, size_t fstride, int sd);
int blk_project_mfma(hdcg* h, const bf16c* P, const cplx<float>* fine, size_t fstride, int nr, cplx<float>* out,
                     size_t sr, size_t sa, size_t sk, hipStream_t st);
int blk_promote_mfma(hdcg* h, const bf16c* P, const cplx<float>* c, int nr, cplx<float>* fine_out,
                     const cplx<float>* base, double sign, size_t fstride, hipStream_t st);
int blk_phi16(hdcg* h, hipStream_t st);        // phi16 = phi128 rounded to bf16 pairs
int blk_cholqr_step(hdcg* h, hipStream_t st);  // one Cholesky-QR pass on phi128
int blk_surface_zero(hdcg* h, hipStream_t st);  // zero phi128 at sd <= s < Ls - sd
int blk_surface_copies(hdcg* h, bool p16, hipStream_t st);  // build the solve's surface-only copy (sd > 0)
// the solve's project / promote (complex64 vectors) on the subspace copy
// phi_prec selects (p16: bf16 pairs), surface slices only when sd > 0
int solve_project(hdcg* h, bool p16, const cplx<float>* fine, size_t fstride, int nr, cplx<float>* out, size_t sr,
                  size_t sa, size_t sk, hipStream_t st);
int solve_promote(hdcg* h, bool p16, const cplx<float>* c, int nr, cplx<float>* out, const cplx<float>* base,
                  double sign, size_t fstride, hipStream_t st);
template <typename R>
int crs_apply(hdcg* h, const cplx<R>* AT, const cplx<R>* in, cplx<R>* out, int nr, hipStream_t st);
int crs_idft(hdcg* h, cplx<double>* Y, const cplx<double> finv[4][9], hipStream_t st);
int crs_transpose(hdcg* h, bool fp64, hipStream_t st);  // A128 -> AT128 (fp64) or AT64
int crs_build_mfma(hdcg* h, int prec, hipStream_t st);
int crs_apply_mfma(hdcg* h, int prec, const cplx<float>* in, cplx<float>* out, int nr, hipStream_t st);
// the autotuned tile for n right-hand sides per launch: {K per MFMA, waves, K steps per wave}
int crs_mfma_tile(hdcg* h, int prec, int n, int out[3], float* ms, int* ntiles, hipStream_t st);

// coarse CG from x = 0 on the complex64 (mprec = DWF_C64) or 16-bit MFMA
// operator as one persistent kernel (coarse_cg.hip), 1..16 right-hand sides
// with per-right-hand-side convergence masks; *done = 0 when that form does
// not apply (more than 16 right-hand sides, unsuited nvec).  iters_rhs
// (nullable): the iterations each right-hand side ran before converging.
int coarse_cg_persistent(hdcg* h, int mprec, cplx<float>* x, const cplx<float>* b, int nr, double tol,
                         int maxiter, int* iters, int* iters_rhs, int* done, hipStream_t st);
// the same, enqueued only (no host synchronisation, so it may be captured
// into a graph); its counts go to device totals.  *done = 0 when the form
// does not apply or its work memory has not been sized by an earlier solve.
int coarse_cg_persistent_deferred(hdcg* h, int mprec, cplx<float>* x, const cplx<float>* b, int nr, double tol,
                                  int maxiter, int* done, hipStream_t st);
int coarse_cg_clear_totals(hdcg* h, hipStream_t st);
// work memory of a persistent solve (0: the form does not apply), and the
// solve with its work memory supplied by the caller (allocates nothing)
size_t coarse_cg_work_bytes(hdcg* h, int mprec, int nr);
int coarse_cg_persistent_in(hdcg* h, void* work, int mprec, cplx<float>* x, const cplx<float>* b, int nr, double tol,
                            int maxiter, int* iters, hipStream_t st);
// the deferred solves' counts since the last clear: *solves, and added to
// *iters and iters_rhs[0..nr); synchronises
int coarse_cg_totals(hdcg* h, int nr, int* solves, long long* iters, long long* iters_rhs, hipStream_t st);

// complex128 CG on (A + shift) x = b from x = 0 (hdcg_solver.hip)
int coarse_cg_shifted(hdcg* h, cplx<double>* x, const cplx<double>* b, int nr, double shift, double tol, int maxiter,
                      int* iters, hipStream_t st);
int ensure_at128_impl(hdcg* h, hipStream_t st);  // the complex128 transposed A for the mat-vec

// second deflation level (ldop.hip): build Z, AZ, D from the free global
// vectors and n_extra coarse noise vectors ([n_extra][Nc][nvec] complex128)
// after n_steps of (A + shift)^-1 each (coarse CG to tol, at most maxiter)
int ldop_build(hdcg* h, int n_extra, const cplx<double>* noise, double shift, int n_steps, double tol, int maxiter,
               hipStream_t st);
// truncated operator and ADEF1 (trunc.hip): out = (Q_trunc + m1_shift) in;
// y = p(Q_trunc + m1_shift) r (Chebyshev, m1_order, [m1_lo, m1_hi]);
// y = M_1 r = p(.) (r - A Z D^-1 Z^+ r) + Z D^-1 Z^+ r; the interval in use
template <typename R>
int trunc_apply(hdcg* h, const cplx<R>* in, cplx<R>* out, int nr, hipStream_t st);
template <typename R>
int m1_chebyshev(hdcg* h, cplx<R>* y, const cplx<R>* r, int nr, hipStream_t st);
template <typename R>
int m1_adef1(hdcg* h, cplx<R>* y, const cplx<R>* r, int nr, hipStream_t st);
// y = M_IRS(Q_trunc + m1_shift, m1_order) r: m1_order CG iterations from 0
template <typename R>
int m1_trunc_cg(hdcg* h, cplx<R>* y, const cplx<R>* r, int nr, hipStream_t st);
int m1_bounds(hdcg* h, double* lo, double* hi, hipStream_t st);
int m1_check_params(int ldop_m1, double lo, double hi, int order, double shift);
void trunc_invalidate(hdcg* h);  // after a change of m1_shift
// Q_trunc + shift in 16-bit MFMA storage (coarse_mfma.hip; needs nbr9), and
// out = (Q_trunc + shift) in with it (complex64 vectors, 1..64 right-hand sides)
int trunc16_build(hdcg* h, int prec, double shift, hipStream_t st);
int trunc16_apply(hdcg* h, int prec, const cplx<float>* in, cplx<float>* out, int nr, hipStream_t st);

// c[rhs][k] = (V_k, r_rhs) / D_k into h->ldc
template <typename R>
int ldop_coef(hdcg* h, const cplx<R>* V, const cplx<R>* r, int nr, hipStream_t st);
// out = (use_r ? r : 0) + (num ? num/den out : 0) + sign sum_k Z_k c[rhs][k]
template <typename R>
int ldop_apply(hdcg* h, cplx<R>* out, const cplx<R>* r, const double* num, const double* den, const cplx<R>* Z,
               int nr, double sign, bool use_r, hipStream_t st);

}  // namespace hdk
