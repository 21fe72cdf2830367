// Internal declarations shared by the host driver (api.cpp) and the kernels
// (kernels.hip).  Not part of the public ABI.
#pragma once

#include <hip/hip_runtime_api.h>
#include <stdint.h>

#include "dcgs2.h"
#include "schur.h"

namespace dcgs2 {

// Device-resident control block, one per context.  Written by the finalising
// workgroup of each reduction, read by every later kernel of the same call.
enum : int {
  ST_RUNNING = 0,
  ST_BREAKDOWN = 1,
  ST_FALLBACK = 2,     // stopped: the host must run the explicit-norm fallback
  ST_NONFINITE = 3,
  ST_DONE = 4,         // GMRES: least-squares residual reached the threshold
};

struct Ctrl {
  int state;
  int stop_step;       // paper's step j at which the state left RUNNING
  int k;               // number of final Hessenberg (or R) columns
  int reductions;
  int fallbacks;
  int pad0;
  double rho_next;     // breakdown scale of the vector currently held in w
  double tau, eta;
  double gmres_thresh; // rtol * ||b||
  double resid_est;    // |g_{k+1}|, least-squares residual estimate
  double norm2;        // result of a plain squared-norm reduction
};

// What the finalising workgroup does with the reduced scalars.
enum FinKind : int {
  FIN_STEP = 0,        // DCGS2 step: Pythagorean alpha, T, H/K (or R) updates
  FIN_FALLBACK = 1,    // same step after the explicit norm ||w - Q C||
  FIN_RESTART = 2,     // first step after a Krylov-Schur truncation (C = 0, alpha = 1)
  FIN_LAST1 = 3,       // last column, reduction 1: c = Q^T w
  FIN_LAST2 = 4,       // last column, reduction 2: alpha = ||w - Q c||
  FIN_NORM = 5,        // plain squared norm into ctrl->norm2
  FIN_NONE = 6,        // no scalar work (a projection whose norm is not needed)
  FIN_CGS2_S = 7,      // CGS2 first projection: S = Q^T a into coef and Sprev, rho = ||a||
  FIN_MGS_DOT = 8,     // MGS: r = q_k^T w into R(k, j) and coef[0] (J = k, j = column)
  FIN_MGS_NORM = 9,    // MGS: alpha = ||w|| into R(j, j) and the coefficient block
};

struct FinArgs {
  int kind;            // FinKind
  int qr;              // 1: QR (Alg. qr), 0: Arnoldi (Alg. arnoldi)
  int j;               // paper's step index (1-based)
  int J;               // number of basis columns dotted (j-2 for a step)
  int gmres;           // apply Givens rotations to each completed H column
  int ldc;             // stride between the C and T blocks of coef
  Ctrl* ctrl;
  double* coef;        // [0,ldc): C ; [ldc, 2ldc): T ; [2ldc]: alpha
  double* pend;        // fallback hand-over: C, S, sigma, gamma
  double* H; double* K; int ldh;           // Arnoldi (device, column-major)
  double* R; int ldr; double* Sprev;       // QR     (device, column-major)
  double* Rg; double* cs; double* sn; double* g;   // GMRES Givens state
  // Optional step record (nullptr: none).  A DCGS2 step (FIN_STEP, and its
  // FIN_FALLBACK completion) writes its 2(J+2) reduced values, then T (or the S
  // column in QR, J+1 values), alpha and the next breakdown scale.
  double* rec;
};

// Deterministic grid reduction: each of the G workgroups of a streaming kernel
// stores its partials in row bid of P1; a one-workgroup finishing kernel sums them
// in a fixed order and finalises the step.
struct GridRed {
  double* P1;          // [G][ldp] per-workgroup partials
  int G, ldp;
};

// Unsigned 32-bit division by an invariant divisor d >= 1 as a multiply-high, two
// shifts and two adds (Granlund and Montgomery, "Division by invariant integers using
// multiplication", PLDI 1994, unsigned case): with l = ceil(log2 d),
// mul = floor(2^32 (2^l - d) / d) + 1, sh1 = min(l, 1), sh2 = max(l - 1, 0),
// t = mulhi(mul, n) and n / d = (t + ((n - t) >> sh1)) >> sh2 for every n < 2^32.
struct DivMagic {
  uint32_t mul;
  int sh1, sh2;
};
DivMagic div_magic(uint32_t d);

struct OpDev {
  int kind;
  int64_t m;
  const int32_t* rowptr; const int32_t* colind; const double* val;
  int64_t nnz;
  int nx, ny, nz;
  double c0, cxm, cxp, cym, cyp, czm, czp;
  DivMagic dx, dy;              // stencils: division by nx and by ny
};

// ---- launchers (kernels.hip) -------------------------------------------------------
// Every launcher returns the hipError_t of its launch.
// rho: initial breakdown scale (rho_next) of the vector held in w.
hipError_t launch_init_ctrl(Ctrl* ctrl, double tau, double eta, double thresh, hipStream_t s,
                            double rho = 0.0);
hipError_t launch_fill(double* p, int64_t n, double val, hipStream_t s);
hipError_t launch_set_state(Ctrl* ctrl, int state, hipStream_t s);
hipError_t launch_copy(double* dst, const double* src, int64_t n, hipStream_t s);
hipError_t launch_copy_cols(double* dst, int64_t ldd, const double* src, int64_t lds,
                            int64_t m, int ncols, hipStream_t s);
// y = A x, or y = b - A x when b != nullptr; skipped unless ctrl->state == RUNNING
// (ctrl may be nullptr: always runs).
hipError_t launch_spmv(const OpDev& op, const double* x, const double* b, double* y,
                       const Ctrl* ctrl, hipStream_t s);
// Basis pointers are `const void*` / `void*` with q32 selecting float (FP32
// storage, FP64 arithmetic) or double elements.
// One DCGS2 reduction: [Q_{0..J-1}, x, (y)]^T [x, (y)] over m rows into per-workgroup
// partials, then a finishing kernel sums them and finalises according to fin.
// The reducing launchers enqueue both kernels; `mid`, when given, is recorded
// between them (so that HIP events can time the streaming kernel alone).
hipError_t launch_reduce(const void* Q, int q32, int64_t ldq, int J, const double* x,
                         const double* y, int64_t m, const GridRed& gr, const FinArgs& fin,
                         hipStream_t s, hipEvent_t mid = nullptr);
// The reduction of an Arnoldi step with the stencil matvec y = A x folded in: y is
// written (as by launch_spmv with ctrl, b = nullptr) and the pass then reduces as
// launch_reduce(.., x, y, ..), bitwise alike.  reduce_mv_fits tells whether the
// operator (a stencil), the sizes (m < 2^29, no odd last row past 16-byte units) and
// the LDS for the workgroup's slab allow it; launch_reduce_mv returns
// hipErrorInvalidValue (nothing launched) when they do not.
bool reduce_mv_fits(const void* Q, int q32, int64_t ldq, const double* x, const double* y,
                    int64_t m, const OpDev& op, const GridRed& gr);
hipError_t launch_reduce_mv(const void* Q, int q32, int64_t ldq, int J, const double* x,
                            double* y, int64_t m, const OpDev& op, const GridRed& gr,
                            const FinArgs& fin, hipStream_t s, hipEvent_t mid);
// u = x - Q_{0..J-1} C written to ubuf; ||u||^2 grid-reduced and finalised.
hipError_t launch_project_norm(const void* Q, int q32, int64_t ldq, int J, const double* x,
                               double* ubuf, int64_t m, const GridRed& gr, const FinArgs& fin,
                               hipStream_t s, hipEvent_t mid = nullptr);
// q_{j-1} = (x - Q C)/alpha (or ubuf/alpha when qcol) into Q[:, J] (rounded to the
// basis type), x <- yscale(y) - Q_{0..J-1} T - q T_J with the stored q,
// yscale(y) = y/alpha (Arnoldi) or y (QR).  At most `slabs` workgroups, each over a
// contiguous slab of rows (0: automatic).
hipError_t launch_update(void* Q, int q32, int64_t ldq, int J, double* x, const double* y,
                         const double* ubuf, int64_t m, const double* coef, int ldc, int arnoldi,
                         int qcol, const Ctrl* ctrl, hipStream_t s, int slabs = 0);
// One-pass QR step: update of step j (q into Q[:, J], w <- w_j) fused with the
// reduction of step j+1 over [Q_{0..J}, w_j, a_next]; last != 0 reduces only
// [Q_{0..J}, w_j]^T w_j (a_next unused).  The launcher sizes the grid itself (one
// workgroup per CU, capped by gmax > 0 and the tile count); gr supplies the
// partial buffer and ldp.
hipError_t launch_fused_qr(void* Q, int q32, int64_t ldq, int J, double* w, const double* a_cur,
                           const double* a_next, int64_t m, const double* coef, int ldc, int last,
                           int fw, int gmax, int pair_max_ns, const GridRed& gr,
                           const FinArgs& fin, hipStream_t s, hipEvent_t mid = nullptr);
// fw: wavefronts per workgroup (8 or 16); two-row slots are used (when the data
// allow them) only while the slot count NS <= pair_max_ns.
int device_cus();                         // multiprocessors of the current device
constexpr int FUSED_QR_MAX_J = 125;       // one-pass QR for n <= 127 (J <= 125 basis columns)
// Q[:, J] = ubuf / alpha (coef[2 ldc]) when ctrl->state == RUNNING.
hipError_t launch_scale_col(void* Q, int q32, int64_t ldq, int J, const double* ubuf, int64_t m,
                            const double* coef, int ldc, const Ctrl* ctrl, hipStream_t s);
// Out[:, 0..k) = (acc ? Out : 0) + Q[:, 0..p) Z[0..p, 0..k)   (Z device, ldz)
hipError_t launch_tsgemm(const void* Q, int q32, int64_t ldq, int p, const double* Z, int ldz,
                         int k, void* Out, int o32, int64_t ldo, int64_t m, int acc,
                         hipStream_t s);
// dst[0..m) = src[0..m) with element-type conversion.
hipError_t launch_convert(void* dst, int d32, const void* src, int s32, int64_t m,
                          hipStream_t s);

// ---- batched Krylov-Schur (batched.hip) ----------------------------------------------
// One record per instance in a device table; see batched.hip.
struct BInst {
  int64_t m, ldq;
  double* Q;           // basis of the current cycle, m x (p+1), leading dimension ldq
  double* Qn;          // truncation target (swapped with Q after a truncation)
  double *w, *v, *r;   // working vectors (length m)
  double *coef, *pend; // per-instance coefficient and fallback hand-over blocks
  double *H, *K;       // (p+1) x (p+1), leading dimension p+1
  double* Z;           // p x p Schur vectors of the last truncation (leading dimension p)
  Ctrl* ctrl;
  double* P1;          // reduction partials (G x ldp)
  int G;               // workgroups of the instance's reduction passes
  int nx, ny;
  double c0, cxm, cxp, cym, cyp;
  int first_j;         // first step of the current cycle (2 for a fresh start)
  int restart;         // the first step is the Krylov-Schur continuation step
  int k;               // Schur vectors kept by the last truncation
  int active;          // 0: converged or stopped -- every batched kernel skips it
  int truncate;        // 1: btruncate acts on this instance
  int n;               // steps of a cycle: steps first_j..n+1, then the last-column
                       // finish over n columns (Krylov-Schur: n = p for every instance)
  // batched GMRES (gmres != 0): right-hand side, iterate, Givens state and the
  // least-squares solution of the last cycle (ksol entries of y)
  int gmres;
  int ksol;
  const double* bvec;
  double* x;
  double *Rg, *cs, *sn, *g, *y;
  double thresh;       // rtol ||b||: a cycle ends once the least-squares residual is below
};
hipError_t launch_bstencil(const BInst* tab, const int* pre_rows, int count, int nblocks, int j,
                           hipStream_t s);
hipError_t launch_breduce(const BInst* tab, const int* pre_red, int count, int nblocks, int j,
                          int last, int ldp, int ldc, int ldh, hipStream_t s);
hipError_t launch_bupdate(const BInst* tab, const int* pre_rows, int count, int nblocks, int j,
                          int ldc, hipStream_t s);
// The last-column launches work on each instance's own n columns; j = (largest n) + 2
// sizes the finishing kernel's LDS.
hipError_t launch_bproject_norm(const BInst* tab, const int* pre_red, int count, int nblocks,
                                int j, int ldp, int ldc, int ldh, hipStream_t s);
hipError_t launch_bscale(const BInst* tab, const int* pre_rows, int count, int nblocks, int j,
                         int ldc, hipStream_t s);
hipError_t launch_btruncate(const BInst* tab, const int* pre_rows, int count, int nblocks, int p,
                            hipStream_t s);
hipError_t launch_breset(const BInst* tab, int count, double tau, double eta, hipStream_t s);
// Batched GMRES: w = b - A x (or w = b when copy_b) for every active instance; the
// squared norm of w into each instance's ctrl->norm2 (one grid reduction per
// instance); x += Q_{:,0..ksol) y.
hipError_t launch_bresidual(const BInst* tab, const int* pre_rows, int count, int nblocks,
                            int copy_b, hipStream_t s);
hipError_t launch_bnorm(const BInst* tab, const int* pre_red, int count, int nblocks, int ldp,
                        int ldc, int ldh, hipStream_t s);
hipError_t launch_bxupdate(const BInst* tab, const int* pre_rows, int count, int nblocks,
                           hipStream_t s);
// Dense restart work of every active, running instance on the GPU (one wavefront per
// instance, T and Z in LDS): real Schur form of the p x p H, reordering by magnitude
// for nev (Ritz values into ere/eim, residual estimate into resid) and then for keep
// (Schur vectors into Z, p x p per instance; the truncated H written back in place).
// ires[4 b] = state (0 skipped, 1 done, -1 Schur form or first reordering failed,
// -2 reordering for keep failed), ires[4 b + 1] = leading block for nev,
// ires[4 b + 2] = kept block size.  p <= BSCHUR_MAX_P.
constexpr int BSCHUR_MAX_P = 96;
hipError_t launch_bschur(const BInst* tab, int count, int p, int ld, int nev, int keep,
                         double cut_gap, double* H, double* Z, int* ires, double* resid,
                         double* ere, double* eim, hipStream_t s);
constexpr int BATCH_ROWS_PER_BLOCK = 512;  // rows per workgroup of the row-parallel kernels

// Learned initial guess (guess.hip): FP32 MFMA products, loss, Adam, grid transfers.
enum GemmEpilogue : int { GEMM_PLAIN = 0, GEMM_BIAS = 1, GEMM_BIAS_RELU = 2, GEMM_MASK = 3 };
hipError_t launch_gemm_f32(int ta, int tb, int epi, int M, int N, int K, const float* A, int lda,
                           const float* B, int ldb, float* C, int ldc, const float* bias,
                           const float* mask, hipStream_t s);
hipError_t launch_colsum(int rows, int cols, const float* dZ, int ld, float* out, hipStream_t s);
int mse_parts(int64_t count);
hipError_t launch_mse(int64_t count, const float* Y, const float* T, float* dY, double* part,
                      double* loss, hipStream_t s);
hipError_t launch_adam(int64_t n, float* theta, const float* g, float* m, float* v, float lr,
                       float b1, float b2, float eps, float c1, float c2, hipStream_t s);
hipError_t launch_features(int count, int n, int nc, const double* b, const float* prm, int np,
                           int fdim, float* feat, double* scale, hipStream_t s);
hipError_t launch_targets(int count, int n, int nc, const double* x, const double* scale,
                          double gain, float* t, hipStream_t s);
hipError_t launch_prolong(int count, int n, int nc, const float* y, const double* scale,
                          double gain, double* x0, hipStream_t s);

// Fixed device scratch of dcgs2_qr_noalloc (kernels.hip): one array per device, sized
// for m <= NOALLOC_MAX_M rows and n <= NOALLOC_MAX_N columns.  Layout in doubles, each
// region starting on a 512-byte boundary: w and r (NOALLOC_MAX_M each), the reduction
// partials (REDUCE_GMAX x NOALLOC_LDP), coef and pend (NOALLOC_LDCOEF each), R
// (NOALLOC_MAX_N^2), S_prev (NOALLOC_MAX_N + 2) and the control block.
constexpr int64_t NOALLOC_MAX_M = int64_t(1) << 21;
constexpr int NOALLOC_MAX_N = 128;
constexpr int NOALLOC_LDP = 2 * (NOALLOC_MAX_N + 2) + 8;
constexpr int NOALLOC_LDCOEF = 2 * (DCGS2_MAX_N + 2) + 8;
// Address of the current device's copy of the scratch array, looked up with
// hipGetSymbolAddress on the first call for each device and cached (device < 64).
hipError_t noalloc_scratch(int device, double** out, size_t* doubles);

// Context access for the other host sources of the library: makes the context's
// device current (allocating its workspace on first use) and returns its stream.
int ctx_prepare(dcgs2_ctx c, hipStream_t* stream);

// Grid sizing for the reductions (number of workgroups for m rows).
void reduce_grid(int64_t m, int gmax, int q32, int* G);
constexpr int REDUCE_GMAX = 1024;
constexpr int BATCH_GMAX = 32;            // reduction workgroups per batched instance

}  // namespace dcgs2
