/*
 * dcgs2.h -- C ABI of libdcgs2.so: the one-reduction DCGS2 Arnoldi-QR expansion
 * on AMD Instinct MI355X (gfx950), and the GMRES and Krylov-Schur drivers on top.
 *
 * Method: Bielich, Langou, Thomas, Swirydowicz, Yamazaki, Boman, "Low-Synch
 * Gram-Schmidt with Delayed Reorthogonalization for Krylov Solvers"
 * (arXiv 2104.01253).  Section/equation/algorithm labels below are the paper's.
 *
 * Conventions for every entry point
 *   - Matrices are column-major (FP64).  "device" pointers are HIP device
 *     memory on the context's device; "host" pointers are ordinary host memory.
 *   - The caller owns every array passed in; the library never frees caller
 *     memory and keeps no pointer to it after the call returns.
 *   - Work is enqueued on the context's stream; every call returns after that
 *     stream has synchronised.  Use one context per host thread.
 *   - Arguments are validated before any device work is enqueued: a violation
 *     returns DCGS2_EINVAL and leaves every output untouched.
 *   - Negative return codes are errors; positive codes are numerical outcomes
 *     whose valid prefix stays usable (see dcgs2_stats.breakdown_step).
 */
#ifndef DCGS2_H
#define DCGS2_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Status codes. */
enum {
  DCGS2_OK = 0,
  DCGS2_EINVAL = -1,        /* invalid argument (nothing was done)               */
  DCGS2_EDEVICE = -2,       /* a HIP runtime call failed                          */
  DCGS2_ENOMEM = -3,        /* device workspace allocation failed                 */
  DCGS2_BREAKDOWN = 1,      /* alpha_{j} <= eta * rho_j: invariant subspace/rank
                               deficiency; the first k columns are valid          */
  DCGS2_NOT_CONVERGED = 2,  /* iteration budget exhausted; best result returned   */
  DCGS2_NONFINITE = 3       /* NaN/Inf in a reduced scalar; valid prefix returned  */
};

/* Largest basis size (columns) accepted by the expansion entry points. */
#define DCGS2_MAX_N 1024

/* Opaque context: binds a device and a HIP stream, owns the device workspace
 * (reduction partials, coefficient buffers, the control block, the Hessenberg
 * matrix, internal Krylov bases).  The workspace grows on demand and is freed
 * by dcgs2_destroy. */
typedef struct dcgs2_ctx_s* dcgs2_ctx;

/* Sparse operator A (m x m).  All array pointers are DEVICE pointers.
 *  CSR:      rowptr[m+1], colind[nnz] (int32, column indices in [0, m)), val[nnz].
 *  STENCIL5: 2-D grid nx*ny (m = nx*ny), lexicographic with x fastest; row of
 *            point (ix,iy): c0*u + cxm*u(ix-1) + cxp*u(ix+1) + cym*u(iy-1) + cyp*u(iy+1),
 *            neighbours outside the grid are zero (homogeneous Dirichlet).
 *  STENCIL7: 3-D grid nx*ny*nz likewise, plus czm*u(iz-1) + czp*u(iz+1).
 * This is the central-difference convection-diffusion operator of Sec. 6.1
 * (Manteuffel's matrix) and of the workloads. */
typedef enum { DCGS2_OP_CSR = 0, DCGS2_OP_STENCIL5 = 1, DCGS2_OP_STENCIL7 = 2 } dcgs2_op_kind;

typedef struct {
  int32_t kind;                 /* dcgs2_op_kind                                   */
  int64_t m;                    /* rows = columns                                  */
  const int32_t* rowptr;        /* CSR only (device)                               */
  const int32_t* colind;        /* CSR only (device)                               */
  const double* val;            /* CSR only (device)                               */
  int64_t nnz;                  /* CSR only                                        */
  int32_t nx, ny, nz;           /* stencils: grid extents (nz = 1 for STENCIL5)    */
  double c0, cxm, cxp, cym, cyp, czm, czp;   /* stencil coefficients               */
} dcgs2_op;

/* Per-call statistics. */
typedef struct {
  int32_t reductions;       /* global reductions performed (one per step, Tab. full) */
  int32_t pyth_fallbacks;   /* steps whose Pythagorean norm was replaced by an
                               explicit norm (one extra reduction each)              */
  int32_t breakdown_step;   /* number k of valid columns when status != OK, else -1  */
  int32_t kernels;          /* kernel launches enqueued                             */
} dcgs2_stats;

typedef struct {
  int32_t iters;            /* Arnoldi steps (matvecs) over all cycles              */
  int32_t cycles;           /* restart cycles                                       */
  int32_t status;           /* same as the return value                              */
  int32_t pad;
  double relres_true;       /* ||b - A x|| / ||b|| at return                          */
  double relres_est;        /* least-squares residual estimate of the last cycle    */
  dcgs2_stats st;
} dcgs2_gmres_info;

typedef struct {
  int32_t restarts;         /* Krylov-Schur truncations performed                   */
  int32_t nconv;            /* size of the converged leading Schur block (>= nev)   */
  int32_t matvecs;
  int32_t status;
  double resid;             /* ||b_{1:nconv}|| / min |theta| of the last test        */
  dcgs2_stats st;
} dcgs2_ks_info;

/* Create a context on `device` (HIP ordinal).  `hip_stream` is the hipStream_t to
 * enqueue on; NULL selects the device's null (legacy default) stream, which is
 * ordered with the other blocking streams of the process.  No device call is
 * made here: the device is bound and the workspace allocated on first use.
 * Returns DCGS2_OK, DCGS2_EINVAL (out == NULL or bad device), DCGS2_EDEVICE. */
int dcgs2_create(dcgs2_ctx* out, int device, void* hip_stream);

/* Free the workspace.  NULL is accepted. */
int dcgs2_destroy(dcgs2_ctx ctx);

/* Tolerances of the two readings where the paper is silent (defaults 1e-8, 1e-12):
 *  tau -- Pythagorean guard: the delayed norm alpha^2 = beta - C^T C (Sec. 3) is
 *         used only when beta - C^T C > tau * beta; otherwise alpha is recomputed
 *         explicitly as ||w - Q C|| with one extra reduction (tau >= 1 forces it).
 *  eta -- breakdown: alpha_j <= eta * rho_j, rho_j the norm of the vector that w_j
 *         was projected from.
 * Returns DCGS2_EINVAL unless 0 <= tau and 0 <= eta < 1. */
int dcgs2_set_tolerances(dcgs2_ctx ctx, double tau, double eta);

/* Pass schedule of dcgs2_qr.  one_pass = 1 (default): the update of step j and the
 * reduction of step j+1 share one read of Q (the next column a_{j+1} is already
 * known in QR, so both use the same Q rows); the arithmetic and the one reduction
 * per column are those of Alg. qr.  one_pass = 0: separate reduction and update
 * passes, as for Arnoldi.  The one-pass schedule is used when n <= 127 and
 * m < 2^28 (an FP64 column of fewer than 2^31 bytes; otherwise two passes).
 * Returns DCGS2_EINVAL unless one_pass is 0 or 1. */
int dcgs2_set_qr_schedule(dcgs2_ctx ctx, int one_pass);

/* Kernel shape knobs (chosen by the autotuner in paper_2104_01253_amd/autotune.py,
 * or left at their defaults).  They change launch shapes only, never the
 * arithmetic or the summation order within a workgroup.
 *  DCGS2_TUNE_FUSED_WAVES : wavefronts per workgroup of the one-pass QR kernel,
 *                           8 or 16 (default 8).
 *  DCGS2_TUNE_REDUCE_GRID : upper bound on the workgroups of a reduction pass,
 *                           1..1024, or 0 for automatic (default: one per CU with
 *                           an FP64 basis, two with FP32).
 *  DCGS2_TUNE_FUSED_MIN_J : one-pass QR schedule: steps whose basis has fewer
 *                           than this many columns run as a separate update and
 *                           reduction pass (same arithmetic per pass, another
 *                           summation order), 0..DCGS2_MAX_N (default 0).
 *  DCGS2_TUNE_BATCH_REDUCE_ROWS : krylov_schur_batched: rows per workgroup of an
 *                           instance's reduction passes (up to 32 workgroups per
 *                           instance), a power of two in 512..65536 (default 2048).
 *  DCGS2_TUNE_FUSED_PAIR_SLOTS : one-pass QR kernel: two rows per lane (16-byte
 *                           loads) while the basis needs at most this many column
 *                           slots per wavefront, one row per lane (deeper
 *                           prefetch) beyond, 0..16 (default 16).
 *  DCGS2_TUNE_BATCH_DENSE : krylov_schur_batched: where the dense restart work
 *                           (Schur form, reordering, residual test, truncated H)
 *                           runs: 0 on the GPU, one wavefront per instance (used
 *                           while ncv <= 96), 1 on host threads (default: faster,
 *                           as the host work of one group of instances overlaps
 *                           the other group's expansion on the GPU).  Both follow
 *                           the same algorithms; results agree to rounding.
 *  DCGS2_TUNE_MATVEC_FOLD : Arnoldi, GMRES and Krylov-Schur with a stencil operator:
 *                           1 computes w = A q inside the step's reduction pass
 *                           (x read once; needs m < 2^29, m even when the basis
 *                           takes 16-byte row pairs, and LDS for a workgroup's
 *                           slab of rows, else the separate matvec runs), 0 runs
 *                           the matvec kernel first (default 1).  Bitwise the
 *                           same results.
 *  DCGS2_TUNE_UPDATE_GRID : upper bound on the workgroups of an update pass, each
 *                           over a contiguous slab of rows, 1..65536, or 0 for
 *                           automatic (default: one per CU with an FP64 basis,
 *                           two with FP32).  Bitwise the same results.
 * Returns DCGS2_EINVAL for an unknown key or value. */
enum { DCGS2_TUNE_FUSED_WAVES = 0, DCGS2_TUNE_REDUCE_GRID = 1, DCGS2_TUNE_FUSED_MIN_J = 2,
       DCGS2_TUNE_BATCH_REDUCE_ROWS = 3, DCGS2_TUNE_FUSED_PAIR_SLOTS = 4,
       DCGS2_TUNE_BATCH_DENSE = 5, DCGS2_TUNE_MATVEC_FOLD = 6, DCGS2_TUNE_UPDATE_GRID = 7 };
int dcgs2_set_tuning(dcgs2_ctx ctx, int32_t key, int32_t value);
int dcgs2_get_tuning(dcgs2_ctx ctx, int32_t key, int32_t* value);

/* Left-looking DCGS2 QR, Alg. qr (Sec. 3): B = Q R with one global reduction per
 * column, the last column finished by CGS2 (two reductions; end of Sec. 3).
 *  m, n    : 1 <= n <= min(m, DCGS2_MAX_N).
 *  B       : device, m x n, leading dimension ldb >= m; read only.
 *  Q       : device, m x n output, ldq >= m; must not overlap B.
 *  R_host  : host, n x n output (upper triangular, R_jj > 0), ldr >= n.
 *  st      : host, optional (NULL allowed).
 * Returns DCGS2_OK, DCGS2_BREAKDOWN (first st->breakdown_step columns of Q and R
 * valid), DCGS2_NONFINITE, or an error. */
int dcgs2_qr(dcgs2_ctx ctx, int64_t m, int32_t n, const double* B, int64_t ldb,
             double* Q, int64_t ldq, double* R_host, int32_t ldr, dcgs2_stats* st);

/* DCGS2 Arnoldi-QR expansion, Alg. arnoldi (Sec. 4): n steps from r0, giving
 * A Q_{1:n} = Q_{1:n+1} H_{1:n+1,1:n} (eq. eq:arnoldi) with q_1 = r0/||r0||.
 * Each step is one matvec A w_{j-1} on the unnormalised vector and one global
 * reduction; H column j-2 is completed at step j through the buffer K
 * (eqs. (41)-(52)); column n is finished by CGS2 (two reductions).
 *  A       : host struct describing a device operator.
 *  r0      : device, m; read only.
 *  Q       : device, m x (n+1) output, ldq >= m.
 *  H_host  : host, (n+1) x n output, ldh >= n+1.
 * 1 <= n <= min(m-1, DCGS2_MAX_N).  Returns as dcgs2_qr; on DCGS2_BREAKDOWN the
 * first k = st->breakdown_step columns of Q and H_{1:k+1,1:k} are valid. */
int dcgs2_arnoldi(dcgs2_ctx ctx, const dcgs2_op* A, const double* r0, int32_t n,
                  double* Q, int64_t ldq, double* H_host, int32_t ldh, dcgs2_stats* st);

/* FP32-stored basis.  Same algorithms and arguments as dcgs2_qr / dcgs2_arnoldi,
 * but Q is a float array: each basis column is rounded once to FP32 when it is
 * written, and every product with Q, every reduction (accumulated in FP64), the
 * Pythagorean norm, R, H and K stay FP64; the projections use the stored
 * columns.  Halves the bytes of the dominant basis streams.  Q (device, float)
 * must be 8-byte aligned with an even ldq for the two-row loads (otherwise
 * one-row loads are used). */
int dcgs2_qr_q32(dcgs2_ctx ctx, int64_t m, int32_t n, const double* B, int64_t ldb,
                 float* Q, int64_t ldq, double* R_host, int32_t ldr, dcgs2_stats* st);
int dcgs2_arnoldi_q32(dcgs2_ctx ctx, const dcgs2_op* A, const double* r0, int32_t n,
                      float* Q, int64_t ldq, double* H_host, int32_t ldh, dcgs2_stats* st);

/* dcgs2_qr for callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * factorisation, kernels and results as dcgs2_qr, with every device buffer beyond
 * B, Q and the outputs (the working vectors, reduction partials, coefficient and
 * control blocks, R) in one fixed array of the library (about 36 MB, held by each
 * GPU the library runs on until the process ends).  No hipMalloc, hipFree or other
 * allocating routine is called, also not on a context's first use; kernel timing
 * (dcgs2_profile_enable) is not recorded.  The array is shared by every call on the
 * same GPU and keeps the last call's contents: calls that overlap on one GPU (from
 * several threads or contexts) race and must be serialised by the caller.
 * Limits: m <= 2,097,152 and n <= 128 (DCGS2_EINVAL beyond), otherwise the
 * arguments, layouts, status codes and stats of dcgs2_qr. */
int dcgs2_qr_noalloc(dcgs2_ctx ctx, int64_t m, int32_t n, const double* B, int64_t ldb,
                     double* Q, int64_t ldq, double* R_host, int32_t ldr, dcgs2_stats* st);

/* Steps j0..j1 of Alg. arnoldi (Sec. 4) from a caller-given state, for checking
 * the expansion one step at a time and for resuming it.  Step j is the matvec
 * v = A w_{j-1}, the one global reduction [Q_{1:j-2}, w_{j-1}]^T [w_{j-1}, v], the
 * scalar finalisation (Pythagorean alpha_{j-1}, T, the Hessenberg column j-2
 * completed from K, then the new K column j-1) and the update that writes q_{j-1}
 * and w_j, with the explicit-norm fallback of dcgs2_set_tolerances.  The
 * last-column finish of dcgs2_arnoldi is not run.
 *  j0, j1  : 2 <= j0 <= j1 <= min(m, DCGS2_MAX_N + 1).
 *  Q       : device, m x (j1-1), ldq >= m; columns 1..j0-2 (1-based) are the
 *            state's basis and are read; columns j0-1..j1-1 are written.
 *  w       : device, m; in: w_{j0-1}, out: w_{j1} (valid when the return is OK).
 *  H_host, K_host : host, ldh x (j1-1) each, ldh >= j1; in: H columns 1..j0-3
 *            final and K column j0-2 partial (as dcgs2_arnoldi holds them after
 *            step j0-1); out: H columns through j1-2 and K column j1-1.  Entries
 *            outside the rows and columns a step writes come back unchanged.
 *  rho     : breakdown scale of w_{j0-1} (sqrt(gamma_{j0-1}) / alpha_{j0-2}); not
 *            used when j0 = 2 (the scale is then ||w_1||); finite, >= 0.
 *  rec_host: host, optional (NULL), (j1-j0+1) records of 3 j1 + 1 doubles, record
 *            r for step j = j0 + r: the 2j reduced values [Q^T w, w^T w, v^T w,
 *            Q^T v, w^T v, v^T v], then T_{1:j-1}, alpha_{j-1} and the breakdown
 *            scale of w_j; the rest of a record, and the records of steps that
 *            did not run, are NaN.
 * Returns as dcgs2_arnoldi (st->breakdown_step is the number of final H columns). */
int dcgs2_arnoldi_steps(dcgs2_ctx ctx, const dcgs2_op* A, int32_t j0, int32_t j1, double* Q,
                        int64_t ldq, double* w, double* H_host, double* K_host, int32_t ldh,
                        double rho, double* rec_host, dcgs2_stats* st);

/* Steps j0..j1 of Alg. qr (Sec. 3) from a caller-given state, under the context's
 * pass schedule (dcgs2_set_qr_schedule: with the one-pass schedule the update of
 * step j and the reduction of step j+1 share one pass for j0 <= j < j1).  Step j is
 * the reduction [Q_{1:j-2}, w_{j-1}]^T [w_{j-1}, a_j], alpha_{j-1}, Stephen's trick
 * for S_{j-1,j}, R column j-1, and the update that writes q_{j-1} and
 * w_j = a_j - Q_{1:j-1} S_{1:j-1,j}.  The last-column finish is not run.
 *  m, j0, j1 : 2 <= j0 <= j1 <= min(m, DCGS2_MAX_N).
 *  B       : device, m x j1, ldb >= m; columns a_{j0}..a_{j1} are read.
 *  Q       : device, m x (j1-1), ldq >= m; columns 1..j0-2 read, j0-1..j1-1 written.
 *  w       : device, m; in: w_{j0-1}, out: w_{j1} (valid when the return is OK).
 *  R_host  : host, ldr x (j1-1), ldr >= j1-1; columns j0-1..j1-1 (1-based) are
 *            written, the others are left alone.
 *  S_host  : host, j1-1 doubles; in: S_{1:j0-2, j0-1} (the first j0-2 entries),
 *            out: S_{1:j1-1, j1}.
 *  rho     : ||a_{j0-1}||, the breakdown scale of step j0 (not used when j0 = 2).
 *  rec_host: optional, records as dcgs2_arnoldi_steps with the S column of step j
 *            (S_{1:j-1,j}) in place of T and ||a_j|| as the next scale.
 * Returns as dcgs2_qr. */
int dcgs2_qr_steps(dcgs2_ctx ctx, int64_t m, int32_t j0, int32_t j1, const double* B, int64_t ldb,
                   double* Q, int64_t ldq, double* w, double* R_host, int32_t ldr,
                   double* S_host, double rho, double* rec_host, dcgs2_stats* st);

/* Comparator: classical Gram-Schmidt with reorthogonalisation, Alg. cgs2 (Sec. 3):
 * per column S = Q^T a_j, w = a_j - Q S, C = Q^T w, u = w - Q C, alpha = ||u||,
 * q_j = u/alpha, R_{1:j-1,j} = S + C -- three global reductions and four passes
 * over Q per column (the method DCGS2 is measured against).  Same arguments,
 * layout, ownership and status codes as dcgs2_qr (FP64 basis only). */
int cgs2_qr(dcgs2_ctx ctx, int64_t m, int32_t n, const double* B, int64_t ldb, double* Q,
            int64_t ldq, double* R_host, int32_t ldr, dcgs2_stats* st);

/* Comparator: modified Gram-Schmidt, column by column (the classical sequential
 * form the paper takes as its baseline, Sec. 2): for column j, w = a_j; for each
 * k < j, r_kj = q_k^T w (one global reduction) and w -= r_kj q_k; alpha = ||w||
 * (one reduction); q_j = w / alpha -- n(n+1)/2 reductions.  Same arguments,
 * layout, ownership and status codes as dcgs2_qr (FP64 basis only); breakdown
 * when alpha <= eta ||a_j||. */
int mgs_qr(dcgs2_ctx ctx, int64_t m, int32_t n, const double* B, int64_t ldb, double* Q,
           int64_t ldq, double* R_host, int32_t ldr, dcgs2_stats* st);

/* Storage precision (64 = FP64, default; 32 = FP32) of the internal Krylov bases
 * of gmres_solve and krylov_schur_eigs; x, r, H, the Givens and Schur work and
 * all reductions stay FP64.  Returns DCGS2_EINVAL for other values. */
int dcgs2_set_basis_precision(dcgs2_ctx ctx, int bits);

/* Restarted GMRES(restart) (Sec. 1, Saad & Schultz) on the DCGS2 basis.
 *  b       : device, m; read only.
 *  x       : device, m; in: initial guess x0, out: solution.
 * Stops when ||b - A x|| / ||b|| <= rtol (true residual) or after max_iters
 * Arnoldi steps.  Givens rotations are applied on the device as each Hessenberg
 * column completes; a cycle ends early once the least-squares residual estimate
 * reaches rtol*||b||.  b = 0 gives x = 0 and DCGS2_OK.
 * 1 <= restart <= min(m-1, DCGS2_MAX_N), rtol > 0, max_iters >= 0.
 * Returns DCGS2_OK, DCGS2_NOT_CONVERGED, DCGS2_NONFINITE or an error. */
int gmres_solve(dcgs2_ctx ctx, const dcgs2_op* A, const double* b, double* x,
                int32_t restart, double rtol, int32_t max_iters, dcgs2_gmres_info* info);

/* Krylov-Schur (Sec. 6.1, Stewart) for the nev largest-magnitude eigenvalues.
 * Expands to ncv columns with DCGS2, computes a real Schur form of H on the host
 * with the largest-magnitude Ritz values leading, accepts when
 * ||b_{1:nev}|| <= tol * min|theta| (b = h_{p+1,p} times the last row of the
 * Schur vectors), else keeps `keep` Schur vectors (a cut never splits Ritz values
 * of equal magnitude) and resumes the expansion.
 *  v0      : device, m start vector; read only.
 *  eig_re_host, eig_im_host : host, nev outputs, by decreasing magnitude.
 * 1 <= nev < keep < ncv <= min(m-1, DCGS2_MAX_N), tol > 0, max_restarts >= 0.
 * Returns DCGS2_OK, DCGS2_NOT_CONVERGED (current Ritz values returned),
 * DCGS2_BREAKDOWN, DCGS2_NONFINITE or an error. */
int krylov_schur_eigs(dcgs2_ctx ctx, const dcgs2_op* A, int32_t nev, int32_t ncv, int32_t keep,
                      double tol, int32_t max_restarts, const double* v0,
                      double* eig_re_host, double* eig_im_host, dcgs2_ks_info* info);

/* Kernel timing.  While enabled, every kernel launch of the context is
 * bracketed by two HIP events on the context stream; the device duration of
 * each launch and its algorithmic HBM bytes (the bytes the method must move:
 * basis columns read once, vectors read/written once) accumulate per kernel
 * class ("spmv", "reduce", "update", "project_norm", "scale", "tsgemm",
 * "fused_qr", "aux").  Two further records are wall-clock phases of
 * krylov_schur_batched, not kernels (bytes 0): "phase_batched_cycle" (from a
 * cycle's launch to its completion) and "phase_host_dense" (the host Schur work
 * between cycles).
 * dcgs2_profile_read synchronises the stream, writes up to max_entries records
 * and returns the number of classes (>= 0), or DCGS2_EINVAL; reset != 0 clears
 * the accumulators afterwards. */
typedef struct {
  char name[24];
  int64_t launches;
  double total_ms;          /* summed device time of the launches               */
  double bytes;             /* summed algorithmic HBM bytes of the launches     */
} dcgs2_kernel_stat;

int dcgs2_profile_enable(dcgs2_ctx ctx, int enable);
int dcgs2_profile_read(dcgs2_ctx ctx, dcgs2_kernel_stat* out, int32_t max_entries, int32_t reset);

/* Batched Krylov-Schur over `count` independent 2-D convection-diffusion operators
 * (5-point stencils with constant coefficients, grids of different sizes).  Every
 * DCGS2 expansion step is ONE launch of each step kernel covering all instances
 * (workgroups mapped to instances by prefix sums; a per-instance grid reduction
 * and finaliser); converged instances drop out.  A restart cycle's launches are
 * captured into a HIP graph (use_graph != 0) and replayed.  The per-instance
 * Schur work runs on host threads between cycles.  Algorithm and readings as
 * krylov_schur_eigs, with shared nev, ncv, keep, tol, max_restarts.
 *  ops         : host, count descriptors (m_b = nx*ny > ncv).
 *  v0          : device, the count start vectors concatenated in instance order.
 *  eig_re_host, eig_im_host : host, count x nev (instance-major).
 *  info_host   : host, count records (status per instance).
 * When an instance's Pythagorean guard fails at a step, that step's explicit-norm
 * fallback and the rest of the instance's cycle run through the single-instance
 * schedule, as in krylov_schur_eigs (st.pyth_fallbacks counts them).  Returns
 * DCGS2_OK when every instance converged, DCGS2_NOT_CONVERGED otherwise, or an error. */
typedef struct {
  int32_t nx, ny;
  double c0, cxm, cxp, cym, cyp;
} dcgs2_stencil2d;

int krylov_schur_batched(dcgs2_ctx ctx, int32_t count, const dcgs2_stencil2d* ops,
                         int32_t nev, int32_t ncv, int32_t keep, double tol,
                         int32_t max_restarts, const double* v0, double* eig_re_host,
                         double* eig_im_host, dcgs2_ks_info* info_host, int32_t use_graph);

/* Batched DCGS2 Arnoldi (Alg. arnoldi, Sec. 4) over `count` independent 2-D
 * convection-diffusion operators (5-point stencils, grids of different sizes), each
 * with its own number of steps n_b: every expansion step is ONE launch of each step
 * kernel covering all instances (workgroups mapped to instances by prefix sums, a
 * per-instance grid reduction and finaliser), an instance is idle after its own n_b
 * steps, and each instance's last column is finished by CGS2 (two reductions) in
 * launches shared by all.  The kernels and readings are those of
 * krylov_schur_batched's expansion cycles; a failed Pythagorean guard runs the
 * explicit-norm fallback as dcgs2_arnoldi does.
 *  ops        : host, count descriptors (m_b = nx*ny >= 2).
 *  n          : host, count step counts, 1 <= n_b <= min(m_b - 1, DCGS2_MAX_N).
 *  r0         : device, the count start vectors concatenated (instance b at element
 *               offset sum_{i<b} m_i); read only.
 *  Q          : device output, 16-byte aligned: instance b's basis is m_b x (n_b+1),
 *               column-major with leading dimension ld_b = m_b rounded up to a
 *               multiple of 64, at element offset sum_{i<b} ld_i (n_i + 1).
 *  H_host     : host output, the count (n_b+1) x n_b Hessenberg matrices, each
 *               column-major with leading dimension n_b+1, concatenated (instance b
 *               at offset sum_{i<b} (n_i+1) n_i).
 *  status_host: host, count statuses (optional): DCGS2_OK, DCGS2_BREAKDOWN (the
 *               first st.breakdown_step columns valid) or DCGS2_NONFINITE.
 *  st_host    : host, count statistics records (optional).
 * Returns DCGS2_NONFINITE if any instance saw a non-finite value, else
 * DCGS2_BREAKDOWN if any broke down, else DCGS2_OK; or an error. */
int dcgs2_arnoldi_batched(dcgs2_ctx ctx, int32_t count, const dcgs2_stencil2d* ops,
                          const int32_t* n, const double* r0, double* Q, double* H_host,
                          int32_t* status_host, dcgs2_stats* st_host);

/* Batched restarted GMRES (Sec. 1) on the DCGS2 basis over `count` independent 2-D
 * convection-diffusion systems A_b x_b = b_b (5-point stencils, grids of different
 * sizes), each with its own restart length.  Every DCGS2 step of a restart cycle is
 * ONE launch of each step kernel covering all instances (the batched expansion of
 * dcgs2_arnoldi_batched, with each instance's Givens rotations and least-squares
 * estimate in its finaliser); a cycle's launches are captured once into a HIP graph
 * and replayed.  Between cycles one launch forms every residual b - A x, one grid
 * reduction per instance its norm, and one launch adds Q_k y to every iterate (y from
 * a back substitution on the host).  Each instance follows gmres_solve's readings:
 * it stops when ||b - A x|| / ||b|| <= rtol (true residual) or after max_iters steps,
 * a cycle ends early once its least-squares residual reaches rtol ||b||, b_b = 0 gives
 * x_b = 0.
 *  ops       : host, count descriptors (m_b = nx*ny >= 2).
 *  restart   : host, count restart lengths, 1 <= restart_b <= min(m_b-1, DCGS2_MAX_N).
 *  b         : device, the right-hand sides concatenated (instance b at element offset
 *              sum_{i<b} m_i); read only.
 *  x         : device, same layout; in: x0, out: the solutions.
 *  info_host : host, count records (iterations, cycles, status, residuals).
 * rtol > 0, max_iters >= 0.  Returns DCGS2_OK when every instance converged, else
 * DCGS2_NONFINITE if any instance saw a non-finite value, else the first other
 * status in instance order (DCGS2_NOT_CONVERGED, DCGS2_BREAKDOWN); or an error. */
int gmres_batched(dcgs2_ctx ctx, int32_t count, const dcgs2_stencil2d* ops,
                  const int32_t* restart, const double* b, double* x, double rtol,
                  int32_t max_iters, dcgs2_gmres_info* info_host);

/* ------------------------------------------------------------------------------------
 * Learned initial guess for GMRES (x0 of the minimisation over x0 + K_k, Sec. 1).
 * Not part of the paper's method: a data-driven start vector for families of
 * 2-D problems on an n x n interior grid (x fastest, h = 1/(n+1)).  A coarse
 * nc x nc grid (n divisible by nc, r = n/nc) carries the learned part:
 *   restriction   R : mean of each r x r block of fine values;
 *   prolongation  P : tensor-product linear interpolation of the values at the
 *                     coarse block centres, zero at the Dirichlet boundary;
 *   features        : [R(b)/s, operator parameters, zero padding], s = RMS of R(b);
 *   guess           : x0 = (s / gain) * P(MLP(features)).
 * The perceptron (FP32; Z_l = X_l W_l + b_l, ReLU on hidden layers, linear
 * output) is trained with the mean squared error on targets gain * R(x)/s of
 * solved instances and Adam (Kingma & Ba, 2015); gain > 0 brings the targets to
 * order one.  Its products run on the matrix cores.
 * Arrays marked device are caller-owned device memory; samples are rows
 * (row-major, sample-major).  All calls synchronise the context's stream.
 * ---------------------------------------------------------------------------------- */
typedef struct dcgs2_mlp_s* dcgs2_mlp;

/* Perceptron with nlayers layers of widths[0] -> ... -> widths[nlayers] (each
 * 1..16384, 1 <= nlayers <= 16) for batches of up to max_batch (<= 65536) rows.
 * Parameters start at zero; they are packed layer by layer as W_l (row-major,
 * widths[l] x widths[l+1]) followed by b_l. */
int dcgs2_mlp_create(dcgs2_ctx ctx, int32_t nlayers, const int32_t* widths, int32_t max_batch,
                     dcgs2_mlp* out);
int dcgs2_mlp_destroy(dcgs2_mlp mlp);
int dcgs2_mlp_num_params(dcgs2_mlp mlp, int64_t* count);
/* Host copy in (resets the Adam moments and step count) / out. */
int dcgs2_mlp_set_params(dcgs2_mlp mlp, const float* params_host);
int dcgs2_mlp_get_params(dcgs2_mlp mlp, float* params_host);
/* Gradients of the last dcgs2_mlp_loss_grad, packed like the parameters. */
int dcgs2_mlp_get_grads(dcgs2_mlp mlp, float* grads_host);
/* Y (device, batch x widths[nlayers]) = MLP(X) (device, batch x widths[0]). */
int dcgs2_mlp_forward(dcgs2_mlp mlp, int32_t batch, const float* X, float* Y);
/* Forward pass, loss = mean((Y - T)^2) over all batch x widths[nlayers] entries
 * (host, may be NULL) and its gradients into the gradient buffer. */
int dcgs2_mlp_loss_grad(dcgs2_mlp mlp, int32_t batch, const float* X, const float* T,
                        double* loss_host);
/* One Adam step with the stored gradients (0 <= beta < 1, lr > 0, eps > 0). */
int dcgs2_mlp_adam(dcgs2_mlp mlp, float lr, float beta1, float beta2, float eps);

/* Features of `count` instances: b (device, count x n*n doubles), prm (device,
 * count x np floats) -> feat (device, count x fdim floats, fdim >= nc*nc + np)
 * and scale (device, count doubles).  nc <= 64. */
int dcgs2_guess_features(dcgs2_ctx ctx, int32_t count, int32_t n, int32_t nc, const double* b,
                         const float* prm, int32_t np, int32_t fdim, float* feat, double* scale);
/* Training targets t = gain R(x)/scale (device, count x nc*nc floats; zero where
 * scale = 0; gain finite and > 0). */
int dcgs2_guess_targets(dcgs2_ctx ctx, int32_t count, int32_t n, int32_t nc, const double* x,
                        const double* scale, double gain, float* t);
/* x0 = (scale / gain) P(y): y device count x nc*nc floats, x0 device count x n*n
 * doubles. */
int dcgs2_guess_prolong(dcgs2_ctx ctx, int32_t count, int32_t n, int32_t nc, const float* y,
                        const double* scale, double gain, double* x0);
/* Zero-guess fallback: ratio = ||b - A x0|| / ||b|| (host, may be NULL); keeps x0
 * (kept = 1) when the ratio is finite and below max_ratio (> 0), otherwise sets
 * x0 = 0 (kept = 0).  A coarse guess leaves interpolation kinks whose residual
 * can exceed ||b|| while its error is small, so max_ratio is taken well above 1
 * (the training driver uses 10).  b, x0: device vectors of length A->m. */
int dcgs2_guess_guard(dcgs2_ctx ctx, const dcgs2_op* A, const double* b, double* x0,
                      double max_ratio, int32_t* kept, double* ratio_host);

/* y = A x (device vectors of length A->m).  The matvec of each expansion step;
 * exported so the operator can be checked on its own. */
int dcgs2_apply(dcgs2_ctx ctx, const dcgs2_op* A, const double* x, double* y);

/* Static description of a status code. */
const char* dcgs2_status_str(int status);

#ifdef __cplusplus
}
#endif
#endif /* DCGS2_H */
