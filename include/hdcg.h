/*
 * hdcg.h -- C ABI of the MI355X hierarchically deflated CG library
 * (libhdcg.so).  Operations follow P. A. Boyle, "Hierarchically deflated
 * conjugate gradient" (arXiv:1402.2585).
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * Status codes: 0 = OK; > 0 = soft failure (DWF_NOT_CONVERGED: the best
 * iterate is returned and the statistics are filled); < 0 = error, in which
 * case no output buffer has been written.  dwf_last_error() returns a
 * thread-local message for the last failing call.  No C++ exception crosses
 * the ABI.
 *
 * Pointers: every field, gauge, coarse vector and matrix argument is a DEVICE
 * pointer on the current HIP device unless the comment says "host".  The
 * caller owns every buffer it passes; the library never retains or frees
 * them.  `stream` is a hipStream_t (NULL = default stream).  Calls documented
 * as asynchronous only enqueue work on `stream`; solver and setup calls
 * synchronise `stream` before returning their statistics.
 *
 * Handles are opaque and library-owned; one handle must not be used from two
 * threads at once, and one stream per handle is assumed.
 *
 * Canonical layouts (the contract with callers; native layouts are private):
 *   gauge      U[t][z][y][x][mu][a][b], complex128, mu = x, y, z, t
 *   half-field psi[rhs][s][cb][spin][colour] on the ODD checkerboard
 *              (parity (x+y+z+t) odd), cb = lex >> 1,
 *              lex = x + X*(y + Y*(z + Z*t)); complex128 for DWF_C128,
 *              complex64 for DWF_C64
 *   coarse vector c[rhs][a][k]; a = coarse lex index (x fastest), k < Nvec
 *   coarse matrix A[a][l][j][k] = <phi^a_j | H | phi^{a+delta_l}_k>,
 *              l = sum_mu (delta_mu + 1) 3^mu (delta_x fastest; l = 40 is the
 *              site itself), complex128
 *   subspace   Phi[k][s][cb][spin][colour], complex128 (odd checkerboard)
 *
 * The operator (Sec. IV, the Hermitian red-black operator H):
 *   D_DW = (4 - M5) - Dh/2 + D5 with the Wilson hop
 *   (Dh psi)(x) = sum_mu [(1 - g_mu) U_mu(x) psi(x+mu) + (1 + g_mu) U_mu(x-mu)^+ psi(x-mu)]
 *   and Shamir's fifth dimension
 *   (D5 psi)_s = psi_s - P- psi_{s+1}[s<Ls-1] - P+ psi_{s-1}[s>0]
 *                + m P- psi_0[s=Ls-1] + m P+ psi_{Ls-1}[s=0],
 *   gamma matrices in the chiral basis (gamma_5 = diag(1,1,-1,-1)).
 *   M_5 = (5 - M5) + (D5 - 1); M_pc = M_5 - 1/4 Dh_oe M_5^-1 Dh_eo;
 *   H = M_pc^+ M_pc.  A boundary phase zeta_mu multiplies the hop crossing
 *   x_mu = L_mu - 1 -> 0 (its conjugate the reverse hop).
 */
#ifndef HDCG_H
#define HDCG_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
  DWF_OK = 0,
  DWF_NOT_CONVERGED = 1,
  DWF_ERR_ARG = -1,      /* bad pointer, size, precision or flag */
  DWF_ERR_GEOMETRY = -2, /* lattice / block shape not supported */
  DWF_ERR_HIP = -3,      /* a HIP runtime call failed */
  DWF_ERR_OOM = -4,      /* device allocation failed */
  DWF_ERR_STATE = -5,    /* handle in the wrong state */
  DWF_ERR_NUMERIC = -6   /* NaN/Inf or breakdown detected in a solver */
};

/* Storage of complex values: complex128, complex64, or pairs of 16-bit
 * floats (bfloat16 / IEEE half; re then im, 4 bytes) whose arithmetic runs in
 * FP32.  Fine fields take DWF_BF16 where a call says so (the 16-bit
 * inner-solver data of Sec. VI.E, Table "sloppy", here as storage on one GPU); the coarse
 * matrix takes DWF_BF16 and DWF_F16. */
enum dwf_prec { DWF_C128 = 0, DWF_C64 = 1, DWF_BF16 = 2, DWF_F16 = 3 };

typedef struct dwf_op* dwf_op_t;
typedef struct hdcg* hdcg_t;

/* ------------------------------------------------------------------------ */
/* Fine operator (Sec. IV, Hermitian red-black operator; Sec. II.A Schur form) */

/* Create the operator on a 4D lattice dims = {X, Y, Z, T} (all even, X >= 2)
 * with fifth-dimension extent Ls (1..64), domain-wall height M5 and mass.
 * gauge_c128: device, canonical layout, V*4*9 complex128; copied (the caller
 * may free it afterwards).  bc_phase: host, 8 doubles (re, im) of zeta_mu for
 * mu = x, y, z, t; NULL means (1, 1, 1, -1).
 * Errors: DWF_ERR_GEOMETRY for odd or non-positive extents or Ls out of range. */
int dwf_create(dwf_op_t* op, const int dims[4], int Ls, double M5, double mass,
               const void* gauge_c128, const double bc_phase[8], void* stream);

/* The same with the Mobius (Cayley-form) kernel the paper treats alongside
 * Shamir's (abstract, Sec. I; written out in the literature it cites):
 *   (D psi)_s = (b5 D_W + 1) psi_s + (c5 D_W - 1)(P- psi_{s+1} + P+ psi_{s-1}),
 *   D_W = (4 - M5) - Dh/2, -mass in place of 1 at the wall couplings,
 * so that with K = P- S_+ + P+ S_- (the chiral shifts in s):
 *   M_5 = alpha + beta K, alpha = b5 (4 - M5) + 1, beta = c5 (4 - M5) - 1;
 *   C_5 = b5 + c5 K;  M_pc = M_5 - 1/4 Dh_oe C_5 M_5^-1 Dh_eo C_5;  H = M_pc^+ M_pc.
 * b5 = 1, c5 = 0 is Shamir (dwf_create).  Every other entry point works on
 * either kernel.  Errors as dwf_create, and DWF_ERR_ARG unless
 * |beta| < |alpha| (the M_5^-1 recurrence). */
int dwf_create_mobius(dwf_op_t* op, const int dims[4], int Ls, double M5, double mass, double b5, double c5,
                      const void* gauge_c128, const double bc_phase[8], void* stream);
int dwf_destroy(dwf_op_t op);

/* Launch shape of the hop kernel (the workgroup tiling of the Wilson hop
 * stages; the operator is the same for every shape, to rounding order):
 * shape = {bx, by, bz, bt, remap, lds_kb, nt, morton, phases, rg}.
 *   bx..bt  site block of one workgroup in (x/2, y, z, t), powers of two
 *           (all 0: consecutive checkerboard sites); a block that does not
 *           divide the lattice or exceeds 256 threads falls back to 0;
 *   remap   1: workgroups reordered so each XCD takes one contiguous range;
 *   lds_kb  minimum LDS per workgroup in KiB (0..150; caps occupancy);
 *   nt      1: non-temporal output stores;
 *   morton  block order: 0 lexicographic; 1 Morton (power-of-two block
 *           grids, else lexicographic); 2 the block grid bisected into eight
 *           compact regions, one per XCD, Morton order inside each (any
 *           block grid; remap ignored); 3 the same regions taken t-plane by
 *           t-plane; 4 regions cut in x, y, z only (each spans all of t),
 *           all XCDs marching through t together, Morton order within each
 *           plane.  Orders 2-4 read a table that the library builds
 *           on the first launch outside graph capture (host memory and
 *           4 bytes of device memory per workgroup, kept until dwf_destroy);
 *   phases  2 or 4 neighbour-load phases per stage (0: 4 for complex128,
 *           2 for complex64 and 16-bit fields);
 *   rg      right-hand sides one workgroup applies the stage to, one after
 *           another on the links it staged once (1..64; a call with fewer
 *           right-hand sides uses that many).
 * By default the block, remap, order and rg entries are chosen by the library's
 * autotuner: the first application of H for a field storage (complex128,
 * complex64, 16-bit) and for one or several right-hand sides times each
 * candidate block / order on that call's own operands (one warm-up, best of
 * three with HIP events; skipped while the stream is being captured) and
 * keeps the fastest for the operator; the other entries are
 * {lds_kb 0, nt 0, phases 0}.  This call fixes a shape instead
 * (launch-shape sweeps and their tests); shape[0] = -1 returns to the
 * autotuned shapes.  DWF_ERR_ARG on an invalid entry. */
int dwf_set_hop_shape(dwf_op_t op, const int shape[10]);

/* The hop launch shape in use for (prec DWF_C128 / DWF_C64 / DWF_BF16,
 * nrhs = 1 or more): shape[10] as dwf_set_hop_shape takes it; ms (nullable,
 * *ncand entries) the autotuner's milliseconds per H of each candidate, -1
 * before it has run.  Returns 1 (and the current shape) when the autotuner
 * has not run yet for that storage and count. */
int dwf_get_hop_shape(dwf_op_t op, int prec, int nrhs, int shape[10], float* ms, int* ncand);

/* Run the hop launch-shape autotuner now for (prec DWF_C128 / DWF_C64 /
 * DWF_BF16, one or several right-hand sides; nrhs sizes its trial fields)
 * on zero fields the call allocates and frees (2 x nrhs fields, plus the
 * operator's work fields), so that a later timed application does not pay
 * the trials.  Nothing happens when that slot is tuned already or a fixed
 * shape is set.  Synchronises.  DWF_ERR_OOM when the trial fields do not
 * fit. */
int dwf_tune_hop(dwf_op_t op, int prec, int nrhs, void* stream);

/* Free the operator's work fields (the intermediate half-fields of M_pc
 * and the fields of cg_solve, cg_solve_mixed and dwf_multishift_cg, sized
 * for the largest right-hand-side count used so far); the next call that
 * needs them allocates them again.  Synchronises the device. */
int dwf_release_workspace(dwf_op_t op);

/* Bytes of one native half-field buffer holding nrhs right-hand sides
 * (prec DWF_C128, DWF_C64 or DWF_BF16). */
int dwf_field_bytes(dwf_op_t op, int prec, int nrhs, size_t* bytes);

/* Canonical <-> native half-field layout (asynchronous).  prec = DWF_C128 or
 * DWF_C64; the canonical buffer has the same precision. */
int dwf_import(dwf_op_t op, void* native, const void* canonical, int prec, int nrhs, void* stream);
int dwf_export(dwf_op_t op, void* canonical, const void* native, int prec, int nrhs, void* stream);

/* Convert native fields between DWF_C128 and DWF_C64, or between DWF_C64 and
 * DWF_BF16 (round to nearest even; no other pair).  Asynchronous. */
int dwf_convert(dwf_op_t op, void* dst, int dst_prec, const void* src, int src_prec, int nrhs,
                void* stream);

/* out = M_pc in (dagger = 0) or M_pc^+ in (dagger = 1); native fields,
 * asynchronous.  out and in must not alias.  prec DWF_BF16: 16-bit fields in
 * and out and for the two intermediate half-fields, FP32 arithmetic (gauge
 * links complex64), every stored value rounded to nearest even. */
int mpc_apply(dwf_op_t op, void* out, const void* in, int prec, int dagger, int nrhs, void* stream);

/* out = M_pc^+ M_pc in = H in; native fields, asynchronous; out != in;
 * prec as mpc_apply (DWF_BF16 also stores M_pc in in 16 bits). */
int mpc_dag_mpc_apply(dwf_op_t op, void* out, const void* in, int prec, int nrhs, void* stream);

/* BLAS-1 with FP64 accumulation over native fields (the linear combinations
 * of the CG of Fig. "pcg").  Results go to HOST arrays of nrhs entries
 * (dot: nrhs (re, im) pairs); these calls synchronise `stream`.  dwf_norm2
 * also takes DWF_BF16 fields; the others DWF_C128 and DWF_C64. */
int dwf_norm2(dwf_op_t op, double* out_host, const void* x, int prec, int nrhs, void* stream);
int dwf_dot(dwf_op_t op, double* out_host, const void* a, const void* b, int prec, int nrhs,
            void* stream);
/* Fused CG update x += alpha p, r -= alpha w, then |r|^2 -> rr_host (nrhs
 * entries); alpha_host: nrhs real coefficients. */
int dwf_cg_update(dwf_op_t op, void* x, void* r, const void* p, const void* w,
                  const double* alpha_host, double* rr_host, int prec, int nrhs, void* stream);
/* p = r + beta p; beta_host: nrhs real coefficients (asynchronous). */
int dwf_xpay(dwf_op_t op, void* p, const void* r, const double* beta_host, int prec, int nrhs,
             void* stream);

struct dwf_solve_stats {
  int iterations;       /* CG iterations over all right-hand sides */
  int restarts;         /* true-residual restarts */
  int converged;        /* 1 if every RHS reached tol */
  double true_residual; /* max over RHS of |b - H x| / |b|, FP64 */
  double seconds;       /* wall time of the solve */
  double matmuls;       /* applications of H */
};

/* Plain FP64 CG on H x = b (Fig. "pcg" with the identity preconditioner; the
 * comparator of Sec. VI.B).  x: native c128, in = initial guess, out =
 * solution; b: native c128.  Stops when |b - H x|/|b| <= tol (recomputed in
 * FP64, restarting when the recursive residual has drifted) or at maxiter.
 * Synchronises; returns DWF_NOT_CONVERGED at maxiter. */
int cg_solve(dwf_op_t op, void* x, const void* b, int nrhs, double tol, int maxiter,
             struct dwf_solve_stats* st, void* stream);

/* Mixed-precision CG on H x = b (the "CGNE (mixed)" comparator of Table
 * "wallclock", Sec. VI.B): FP64 defect correction -- r = b - H x in
 * complex128, then a complex64 CG from zero on H e = r to the relative
 * residual max(inner_tol, tol / (2 |r|/|b|)), then x += e in complex128 --
 * until |b - H x|/|b| <= tol.  x: native c128, in = initial guess, out =
 * solution; b: native c128.  st->iterations counts complex64 CG iterations,
 * st->restarts the corrections, st->matmuls every H (both precisions).
 * Synchronises; returns DWF_NOT_CONVERGED once maxiter complex64 iterations
 * have run without reaching tol; DWF_ERR_ARG unless 0 < inner_tol < 1. */
int cg_solve_mixed(dwf_op_t op, void* x, const void* b, int nrhs, double tol, double inner_tol, int maxiter,
                   struct dwf_solve_stats* st, void* stream);

/* Multi-shift CG (Sec. IV.B: the rational filter of the subspace generation
 * is one multi-shift solve): (H + shifts[j]) x_j = b for j < nshift (1..8)
 * from the Krylov space of the smallest shift, shifts[0]; the other shifts'
 * residuals are zeta_j r with zeta_j from the three-term recurrence of the
 * CG coefficients.  All in complex128.  x: device, nshift * nrhs native
 * complex128 fields, x[j][rhs], overwritten (the solve starts from zero);
 * b: nrhs native complex128 fields; shifts: host.  Stops when the base
 * system's recursive residual |r| <= tol |b| for every right-hand side (the
 * other shifts are then closer still).  st (nullable): iterations, matmuls,
 * and in true_residual the base system's last checked recursive relative
 * residual.  Synchronises; DWF_NOT_CONVERGED at maxiter; DWF_ERR_ARG unless
 * shifts[0] <= every shift, 1 <= nshift <= 8, tol > 0. */
int dwf_multishift_cg(dwf_op_t op, void* x, const void* b, int nrhs, const double* shifts, int nshift,
                      double tol, int maxiter, struct dwf_solve_stats* st, void* stream);

/* ------------------------------------------------------------------------ */
/* Hierarchically deflated CG: blocked subspace (Sec. II), little Dirac
 * operator (Sec. V.A.1), the A-DEF2 solver (Sec. IV.E, Table "algos").     */

struct hdcg_params {
  int n_ii;           /* inverse-iteration steps on the starting vectors (0: use as given) */
  double lambda_ii;   /* shift of the inverse iteration: (H + lambda_ii)^-1 */
  double tol_ii;      /* relative residual of each inverse-iteration solve (complex64 CG) */
  int maxiter_ii;     /* iteration cap of each inverse-iteration solve */
  int n_irs;          /* M_IRS: CG iterations on H + lambda_irs (Sec. IV.C), default 7 */
  double lambda_irs;  /* M_IRS infra-red shift, default 1.0 */
  double coarse_tol;  /* relative residual of the coarse CG inside Q, default 0.04 */
  int coarse_maxiter; /* coarse CG iteration cap */
  int flexible;       /* 1: flexible search-direction update (default), 0: standard PCG */
  double inner_tol;   /* relative residual of each complex64 A-DEF2 inner solve, default 1e-5 */
  int inner_maxiter;  /* inner iteration cap */
  int outer_maxiter;  /* FP64 defect-correction restarts cap */
  int build_batch;    /* probe vectors per H application batch in the coarse build
                         (default 16, at most 16; two complex128 fields per probe
                         vector are held during the build) */
  int coarse_prec;    /* storage of A inside Q: DWF_C64 (default; VALU for one right-hand
                         side, FP32 MFMA for several when nvec % 4 == 0), DWF_BF16 or DWF_F16
                         (MFMA with FP32 accumulation, per-matrix scales; nvec % 4 == 0) */
  int verbose;        /* 1: hdcg_setup prints stage progress to stderr */
  int irs_prec;       /* storage of the M_IRS fields: DWF_C64 (default) or DWF_BF16 (16-bit
                         fields, FP32 arithmetic, FP64 norms; the one-GPU form of the
                         16-bit M_IRS communication of Sec. VI.E, Table "sloppy") */
  int subspace_gen;   /* 0 (default): the given vectors, then n_ii inverse-iteration steps;
                         1: first the fourth-order rational filter of Sec. IV.B (equation
                         "ratfilt"), prod_j (H + rat_lo + j rat_eps)^-1, j = 0..3, by one
                         complex128 multi-shift CG and the partial-fraction sum, each vector
                         then normalised (inverse iteration follows when n_ii > 0) */
  double rat_lo;      /* filter threshold lambda, default 3e-4 */
  double rat_eps;     /* filter shift spacing epsilon, default 1e-4 (lambda / 3) */
  double rat_tol;     /* multi-shift residual, default 1e-6 */
  int rat_maxiter;    /* multi-shift iteration cap, default 10000 */
  int wall_noise;     /* 1: keep only the physical wall components of the given vectors
                         (P- at s = 0, P+ at s = Ls - 1, Sec. IV.B) before filtering */
  int ldop_defl;      /* 1 (default): once hdcg_ldop_setup has built the second deflation
                         level, every coarse solve is deflated CG on it (Sec. V.B); 0: plain */
  int phi_prec;       /* storage of the subspace for the project / promote of the solve's Q:
                         DWF_C64 (default) or DWF_BF16 (bf16 pairs rounded to nearest even
                         from FP64, half the bytes; arithmetic and vectors complex64) */
  int ldop_m1;        /* 0 (default): deflated coarse solves are deflated CG; 1: ADEF1 with
                         the Chebyshev approximate inverse of the truncated operator
                         (Sec. V.B, "Truncated little Dirac operator as preconditioner";
                         Table "optimised": LdopM1Chebyshev); 2: ADEF1 with the paper's
                         alternative, M_IRS(Q_trunc), m1_order CG iterations on
                         Q_trunc + m1_shift (the infra-red shift) from zero */
  double m1_lo;       /* Chebyshev interval low end, default 0.5 (Table "optimised") */
  double m1_hi;       /* high end; 0 (default): 1.05 x a power-method estimate of the largest
                         eigenvalue of Q_trunc + m1_shift (the paper's 45 fits its ensemble) */
  int m1_order;       /* Chebyshev order n, default 16: residual polynomial of degree n,
                         n - 1 applications of Q_trunc (1..256); with ldop_m1 = 2 the
                         number of CG iterations (n applications) */
  double m1_shift;    /* infra-red shift added to Q_trunc, default 0 (>= 0) */
  int surface_depth;  /* d > 0 with 2 d < Ls: the subspace keeps only the slices s < d and
                         s >= Ls - d (Sec. IV.B, the interior of the wall-bound vectors
                         removed before block orthonormalisation), and the solve's project /
                         promote read a surface-only copy, Ls / (2 d) times fewer bytes;
                         d must then be a multiple of 4.  0 (default) or 2 d >= Ls: all slices */
  int coarse_persistent; /* 1 (default): coarse CG of up to 16 right-hand sides with the complex64
                            or 16-bit operator as one persistent kernel (per-right-hand-side
                            convergence masks); 0: one launch per step (for comparisons) */
  int graph;             /* 1 (default): when the coarse solve is the persistent kernel (no
                            second level active), the preconditioner of every A-DEF2 iteration
                            (M_IRS, H z - r, project, coarse solve, promote) is captured once per
                            inner solve as a HIP graph and replayed; 0: launched one by one */
  int phase_timing;      /* 1: hdcg_solve times its phases with HIP events (hdcg_stats t_*;
                            disables the graph); 0 (default): no events */
  int mfma_tile;         /* -1 (default): the tile of the 16-bit MFMA mat-vec (MFMA form, waves,
                            K steps in flight) is picked per shape by timing every candidate once
                            per process (hdcg_mfma_tile reports it); 0..5: that candidate where
                            the shape allows it (comparisons and tests) */
  unsigned long long seed; /* hdcg_setup without vectors: seed of the Gaussian starting vectors
                            it draws on the device (default 1; see hdcg_setup) */
  int keep_subspace_fp64; /* 1 (default): the handle keeps the FP64 subspace after setup;
                            0: hdcg_setup frees it once the solve's complex64 (and, as
                            phi_prec / surface_depth ask, 16-bit or surface-only) copies exist,
                            two thirds of the subspace memory (49 GB at 24^3 x 48 x 16, Nvec
                            48); complex128 project / promote, hdcg_export_subspace and a later
                            switch to a subspace copy not yet built then return DWF_ERR_STATE */
  int m1_prec;           /* storage of Q_trunc for the complex64 coarse solves and for
                            hdcg_trunc_apply / hdcg_chebyshev / hdcg_trunc_cg with DWF_C64:
                            DWF_C64 (default), or DWF_BF16 / DWF_F16: the nine matrices per
                            site in the 16-bit MFMA storage of coarse_prec (per-matrix scales,
                            FP32 accumulation; nvec a multiple of 4, at most 64), a quarter of
                            the complex64 bytes.  The complex128 forms keep complex128 */
};

struct hdcg_stats {
  int outer_iterations;  /* FP64 defect-correction restarts (max over groups of RHS) */
  int inner_iterations;  /* A-DEF2 iterations summed over restarts and groups */
  int coarse_solves;     /* applications of Q */
  int coarse_iterations; /* coarse CG iterations summed over solves (each solve: its longest RHS) */
  int converged;         /* 1 if |b - H x| / |b| <= tol for every RHS */
  int nrhs;              /* entries of the per-RHS arrays below */
  double true_residual;  /* max over RHS of the FP64 relative residual */
  double seconds;        /* solve wall time (setup excluded) */
  double setup_seconds;  /* wall time of hdcg_setup */
  double matmuls_fp64;   /* applications of H in complex128 (per RHS summed) */
  double matmuls_fp32;   /* applications of H in complex64 (per RHS summed) */
  double matmuls_bf16;   /* applications of H on 16-bit fields (M_IRS with irs_prec = DWF_BF16) */
  int group_size;        /* right-hand sides solved together (one batch shares every operator pass) */
  int graph_replays;     /* preconditioner applications replayed from a captured graph */
  /* Phase times in seconds, the categories of Fig. "pie" (filled when
   * params.phase_timing = 1, else 0): H in FP64 (the outer residuals); H in
   * complex64 and 16 bits (A-DEF2, M_IRS, the preconditioner's correction);
   * the coarse solves inside Q (LdopInv); project and promote; linear
   * combinations and reductions of fine vectors; precision conversions. */
  double t_fine_dp, t_fine_sp, t_coarse, t_project_promote, t_linalg, t_convert;
  long long coarse_iterations_rhs[64]; /* per RHS: coarse CG iterations summed over solves */
  double true_residual_rhs[64];        /* per RHS: FP64 |b - H x| / |b| */
};

/* Fill *p with the defaults above. */
void hdcg_default_params(struct hdcg_params* p);

/* Build the two-level solver for operator `op` (Sec. II, Sec. V.A):
 * block = {Bx, By, Bz, Bt} (each even, >= 4, dividing the lattice, with at
 * least 3 blocks in every direction so the coarse stencil has 81 distinct
 * points); blocks span all of s.  vectors_c128: device, nvec canonical
 * complex128 half-fields Phi[k][s][cb][spin][colour] (the random starting
 * vectors), or NULL: the library then draws them itself on the device from
 * p->seed with the counter-based generator Philox4x32-10 (Salmon et al.,
 * SC 2011; counter (i mod 2^32, i div 2^32, 0, 0), key (seed mod 2^32,
 * seed div 2^32) for complex number i of the canonical array, two 53-bit
 * uniforms u, v from the output word pairs (0, 1) and (2, 3), Box-Muller
 * sqrt(-2 ln(1 - u)) (cos 2 pi v + i sin 2 pi v): real and imaginary parts
 * N(0, 1)), reproducible on any host.  The library applies p->n_ii steps of
 * inverse iteration (complex64 CG, each vector renormalised), orthonormalises
 * the blocked vectors block by block (Cholesky-QR applied twice in FP64:
 * the unique QR with positive diagonal, as Gram-Schmidt gives), and computes
 * A^{ab}_{jk} = <phi^a_j|H|phi^b_k> in FP64 with 81 phased probes per vector
 * (the Fourier trick of Sec. V.A.1, momenta p_mu = 2 pi n m_mu / Lc_mu,
 * m_mu = round(Lc_mu / 3)).  The handle owns the subspace, the operator and
 * all workspaces until hdcg_destroy.  Synchronises `stream`.
 * Errors: DWF_ERR_GEOMETRY (block shape), DWF_ERR_NUMERIC (dependent
 * vectors on a block), DWF_ERR_OOM. */
int hdcg_setup(hdcg_t* h, dwf_op_t op, const int block[4], int nvec, const void* vectors_c128,
               const struct hdcg_params* p, void* stream);
int hdcg_destroy(hdcg_t h);
/* Coarse grid extents, number of coarse sites and of vectors (host outputs, nullable). */
int hdcg_dims(hdcg_t h, int coarse_dims[4], int* ncoarse, int* nvec);

/* c[rhs][a][k] = <phi^a_k, psi_rhs> (project, P^+) and psi = sum phi^a_k
 * c[a][k] (promote, P), Sec. II.  Fine fields native, coarse vectors
 * canonical, both in precision prec (C128 or C64); prec DWF_BF16: the
 * subspace in 16 bits (built on first use), vectors complex64, FP32
 * arithmetic (from 2 right-hand sides on the bf16 MFMA, the complex64
 * values entering as three bf16 terms, so that every product is the FP32
 * one; fields and subspace 16-byte aligned for that form, else the VALU
 * kernels run).  Asynchronous. */
int hdcg_project(hdcg_t h, void* coarse_out, const void* fine_in, int prec, int nrhs, void* stream);
int hdcg_promote(hdcg_t h, void* fine_out, const void* coarse_in, int prec, int nrhs, void* stream);

/* out[rhs][a][j] = sum_l sum_k A[a][l][j][k] in[rhs][a + delta_l][k]:
 * the 81-point block stencil of the little Dirac operator (Sec. V.A);
 * prec C128 or C64 (vectors in that precision; one right-hand side on the
 * VALU, several, when nvec % 4 == 0, on the FP64 / FP32 16x16x4 MFMA with
 * neither operand rounded, up to 16 per pass over A), or BF16 / F16: the
 * matrix stored in 16 bits with one scale per stencil matrix A[a][l], the
 * complex64 vectors rounded to 16 bits, products accumulated in FP32 on MFMA
 * (vectors in/out complex64).  Asynchronous; out != in. */
int coarse_apply(hdcg_t h, void* out, const void* in, int prec, int nrhs, void* stream);

/* The tile of the 16-bit MFMA mat-vec (prec DWF_BF16 or DWF_F16) for
 * nrhs_per_launch right-hand sides per launch (1..16; coarse_apply splits
 * larger counts into launches of 16), as the project-written autotuner chose
 * it: the first mat-vec of a shape (storage precision, Nc, nvec, right-hand
 * sides per launch) times every tile allowed on the shape (one warm-up, best
 * of three with HIP events) and keeps the fastest for the rest of the
 * process, for every handle of that shape; a call under graph capture uses
 * the cached tile or the default.  Tunes now, on zero operands, if that has
 * not happened.  tile (host, 3 ints): K values per MFMA instruction (16, or
 * 32 for gfx950's 16x16x32 bf16 / f16 forms), waves per workgroup (the K
 * range split over them), K steps in flight per wave.  ms (host, nullable,
 * *ntiles entries): the measured milliseconds of each candidate (-1: not
 * allowed on the shape); ntiles (host, nullable): the number of candidates.
 * Synchronises. */
int hdcg_mfma_tile(hdcg_t h, int prec, int nrhs_per_launch, int tile[3], float* ms, int* ntiles, void* stream);

/* CG on A x = b (A Hermitian positive definite, Sec. V.B) from x = 0 to
 * |r| <= tol |b| for every RHS, with the mat-vec of coarse_apply in precision
 * prec (BF16 / F16 use complex64 vectors); *iters receives the iteration count.
 * Synchronises; DWF_NOT_CONVERGED at maxiter. */
int hdcg_coarse_solve(hdcg_t h, void* x, const void* b, int prec, int nrhs, double tol, int maxiter,
                      int* iters, void* stream);

/* The iterations each right-hand side of the last hdcg_coarse_solve ran
 * before its residual reached tol (a zero right-hand side: 0), into the host
 * array iters_rhs[nrhs]; nrhs must equal that call's.  Right-hand sides of
 * one call run together (one mat-vec for all of them per iteration); with
 * up to 16 of them and the complex64 or 16-bit operator the solve is one
 * persistent kernel that masks each right-hand side off once it converges,
 * so these counts differ from each other and from *iters (the longest). */
int hdcg_coarse_iterations(hdcg_t h, int* iters_rhs, int nrhs);

/* hdcg_coarse_solve for callers that cannot allocate device memory (code
 * under graph capture, tight serving loops, harnesses that forbid it): the
 * same persistent coarse CG, with its work memory (r, two search-direction
 * buffers, A p, the per-workgroup partial sums and the grid-barrier state)
 * carved from one static device array of 64 MiB that each device holds
 * until the process ends, instead of the handle's buffers.  Calls no
 * hipMalloc / hipFree.  The work memory, about 4 * 8 * Nc * nvec * nrhs
 * bytes plus at most 1.1 MiB, must fit the array (the 24^3x48 grid with 4^4 blocks,
 * Nc 2592, nvec 48, fits up to 16 right-hand sides); otherwise
 * DWF_ERR_ARG.  prec DWF_C64, or DWF_BF16 / DWF_F16 once that 16-bit storage
 * exists (built by an earlier call that allocates: hdcg_setup with
 * coarse_prec, hdcg_set_params, coarse_apply); nrhs 1..16; nvec <= 64.
 * DWF_ERR_STATE while the second deflation level is active (ldop_defl = 1
 * after hdcg_ldop_setup): that solve is not covered.  Results equal those
 * of hdcg_coarse_solve on the same handle and inputs (the same kernel and
 * launch shape).  All calls on one device share the array and it keeps the
 * last call's contents (every call re-initialises what it reads): calls
 * that overlap in time on one device, from any handle or stream, race.
 * Synchronises; DWF_NOT_CONVERGED at maxiter. */
int hdcg_coarse_solve_noalloc(hdcg_t h, void* x, const void* b, int prec, int nrhs, double tol, int maxiter,
                              int* iters, void* stream);


/* out = M_IRS in: exactly n_irs CG iterations on H + lambda_irs from zero
 * (Sec. IV.C) with the work fields stored as p->irs_prec selects (complex64,
 * or bfloat16 pairs rounded to nearest even after every kernel); in and out
 * are native complex64 fields; asynchronous. */
int hdcg_mirs(hdcg_t h, void* out, const void* in, int nrhs, void* stream);

/* Second deflation level of the little Dirac operator (Sec. V.B, "Little
 * Dirac operator deflation") and the pre-diagonalised third level.  Global
 * coarse vectors, no further blocking: the Nvec free ones w_k[a][j] =
 * delta_jk / sqrt(Nc), and n_extra more from noise_c128 (device, n_extra
 * coarse vectors c[k][a][j] complex128 drawn by the caller), each taken
 * through n_steps of v <- (A + shift)^-1 v / |v| (complex128 coarse CG to
 * relative residual tol; the paper: three steps, 1e-7).  They are
 * orthonormalised (Cholesky-QR twice, FP64), E = W^+ A W is diagonalised
 * (E = U D U^+) and Z = W U, A Z are kept; every later coarse solve
 * (hdcg_coarse_solve, the Q of hdcg_solve) is then deflated CG:
 * x0 = Z D^-1 Z^+ b, search directions p = r + beta p - Z D^-1 (AZ)^+ r
 * (params.ldop_defl = 0 turns it off).  Replaces an earlier second level.
 * Synchronises.  DWF_ERR_ARG: n_extra < 0, Nvec + n_extra > 1024 or more than
 * the coarse unknowns, tol <= 0, shift < 0; DWF_ERR_NUMERIC: dependent
 * vectors or A not positive on them. */
int hdcg_ldop_setup(hdcg_t h, int n_extra, const void* noise_c128, double shift, int n_steps, double tol,
                    void* stream);
/* The second level for parity checks: *n_global (host) = number of global
 * vectors (0 before hdcg_ldop_setup); Z_c128 (device, nullable): the
 * orthonormal eigenbasis Z[k][a][j] complex128 of E, ascending eigenvalue;
 * D_host (host, nullable): the eigenvalues D.  Synchronises. */
int hdcg_export_ldop(hdcg_t h, int* n_global, void* Z_c128, double* D_host, void* stream);

/* Replace the solve-phase parameters of a built handle (n_irs, lambda_irs,
 * coarse_tol, coarse_maxiter, flexible, inner_tol, inner_maxiter,
 * outer_maxiter, coarse_prec, irs_prec, ldop_defl, phi_prec and the m1_
 * fields); the setup-phase fields of *p are ignored.  Builds the 16-bit
 * copies of A and of the subspace when coarse_prec or phi_prec asks for one
 * not yet built, and estimates the Chebyshev bound when ldop_m1 = 1 and
 * m1_hi = 0.
 * Synchronises `stream`.  DWF_ERR_ARG on an invalid field, DWF_ERR_NUMERIC
 * if the Chebyshev bound estimate is not above m1_lo (the parameters are
 * then unchanged). */
int hdcg_set_params(hdcg_t h, const struct hdcg_params* p, void* stream);

/* The truncated little Dirac operator (Sec. V.B, "Truncated little Dirac
 * operator as preconditioner"; Table "frobnorm"): out = (Q_trunc + m1_shift)
 * in, Q_trunc keeping of A only the zero- and one-hop terms (the site and its
 * eight axis neighbours; Hermitian).  in, out: device coarse vectors
 * c[rhs][a][k], distinct, complex64 or complex128 by prec (DWF_C64 /
 * DWF_C128), nrhs 1..64.  Builds Q_trunc (a ninth of the bytes of A) on first
 * use and after a change of m1_shift.  Asynchronous. */
int hdcg_trunc_apply(hdcg_t h, void* out, const void* in, int prec, int nrhs, void* stream);
/* The Chebyshev interval [*lo, *hi] (host) the preconditioner uses: m1_lo,
 * and m1_hi or, when m1_hi is 0, its estimate (taken once per m1_shift; the
 * first call synchronises).  DWF_ERR_NUMERIC if the estimate is not above
 * m1_lo. */
int hdcg_m1_interval(hdcg_t h, double* lo, double* hi, void* stream);
/* y = p(Q_trunc + m1_shift) r: m1_order steps of the Chebyshev iteration on
 * [lo, hi] from y = 0 (residual T_n((d - x)/c) / T_n(d/c) r, d and c the
 * interval's centre and half-width).  y, r: device coarse vectors as for
 * hdcg_trunc_apply, distinct; r is not modified.  Asynchronous after the
 * interval is known. */
int hdcg_chebyshev(hdcg_t h, void* y, const void* r, int prec, int nrhs, void* stream);
/* y = M_IRS(Q_trunc + m1_shift, m1_order) r (Sec. V.B, closing paragraph of
 * "Truncated little Dirac operator as preconditioner", with the infra-red
 * shifted CG of Sec. IV.C): exactly m1_order CG iterations on
 * (Q_trunc + m1_shift) y = r from y = 0, each right-hand side with its own
 * coefficients (a zero r gives y = 0).  Arguments as for hdcg_chebyshev;
 * asynchronous. */
int hdcg_trunc_cg(hdcg_t h, void* y, const void* r, int prec, int nrhs, void* stream);
/* y = M_1 r, the ADEF1 preconditioner of the coarse solve (Sec. V.B):
 * p(Q_trunc + m1_shift) (r - A Z D^-1 Z^+ r) + Z D^-1 Z^+ r with the second
 * level's Z, D and the stored A Z (no application of A).  Arguments as for
 * hdcg_chebyshev; DWF_ERR_ARG before hdcg_ldop_setup.  p(.) is the
 * Chebyshev polynomial, or with params.ldop_m1 = 2 the CG of hdcg_trunc_cg.
 * With params.ldop_m1 = 1 or 2 every deflated coarse solve is flexible CG
 * preconditioned by M_1 from x0 = Z D^-1 Z^+ b (alpha = (p, r)/(p, A p),
 * beta = -(A p, y)/(p, A p)). */
int hdcg_adef1_precondition(hdcg_t h, void* y, const void* r, int prec, int nrhs, void* stream);

/* Copies for parity checks: the little Dirac operator in the canonical layout
 * A[a][l][j][k] (device, Nc*81*nvec*nvec complex128), the orthonormalised
 * subspace Phi[k][s][cb][spin][colour] (device complex128), and the block map
 * (host int arrays of V/2 entries indexed by cb: block index, rank in block). */
int hdcg_export_coarse(hdcg_t h, void* A_c128, void* stream);
int hdcg_export_subspace(hdcg_t h, void* phi_c128, void* stream);
/* Replace the little Dirac operator of a built handle by a caller-given one
 * in the same canonical layout A[a][l][j][k] (device, complex128, Nc*81*nvec*
 * nvec entries; the caller keeps ownership), e.g. an operator reused from an
 * earlier setup on the same subspace or a seeded test operator.  Every copy
 * derived from A (the transposed complex64 / complex128 forms, the 16-bit
 * MFMA storage and its scales, the truncated operator) is rebuilt; the second
 * deflation level built on the old operator is dropped (hdcg_ldop_setup
 * again to rebuild it).  The coarse solves assume A Hermitian positive
 * definite.  Synchronises. */
int hdcg_import_coarse(hdcg_t h, const void* A_c128, void* stream);
int hdcg_export_block_map(hdcg_t h, int* block_of_site, int* index_in_block);

/* Solve H x = b for nrhs right-hand sides to |b - H x| / |b| <= tol (FP64
 * true residual).  Outer loop: FP64 defect correction r = b - H x; inner:
 * complex64 generalised PCG with the A-DEF2 choices V_start = Q r,
 * M_1 = P_R M_IRS + Q (applied as z - Q (H z - r), z = M_IRS r), flexible
 * search directions (alpha = (p, r)/(p, w), beta = -(w, y)/(p, w)), to
 * p->inner_tol.  x, b: native complex128.  Synchronises; fills *stats
 * (nullable); DWF_NOT_CONVERGED after outer_maxiter restarts. */
int hdcg_solve(hdcg_t h, void* x_c128, const void* b_c128, int nrhs, double tol,
               struct hdcg_stats* stats, void* stream);

const char* dwf_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* HDCG_H */
