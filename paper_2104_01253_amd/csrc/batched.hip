// Batched Krylov-Schur kernels: one launch per DCGS2 step covers every instance.
//
// Each instance b (a 2-D convection-diffusion operator on an nx x ny grid, its own
// basis, vectors, Hessenberg matrix and control block) is described by a BInst
// record in a device table.  A launch's workgroups are mapped to (instance,
// slab) pairs through prefix sums of the per-instance workgroup counts, so small
// and large instances share one grid without idle workgroups.  Each instance's
// reduction partials are summed and finalised by a finishing kernel with one
// workgroup per instance, with exactly the arithmetic of the single-instance
// kernels (device_common.h and the *_body functions are shared).
//
// All instances advance the same step index j.  After a Krylov-Schur truncation
// instance b keeps k_b Schur vectors and starts at j = k_b + 2 with the
// continuation step (C = 0, alpha = 1); for smaller j it is idle.  Every
// instance therefore reaches the last column at the same launch.
#include <hip/hip_runtime.h>
#include <math.h>

#include "internal.h"
#include "std2x2.h"

namespace dcgs2 {
namespace {

#include "device_common.h"

// Device memory that no kernel writes while a reader of this view runs (the
// instance table, the prefix sums, Z during the truncation), seen through the
// constant address space: loads from it at a wavefront-uniform address become
// scalar loads.
template <class T>
using ConstPtr = const __attribute__((address_space(4))) T*;
template <class T>
__device__ __forceinline__ ConstPtr<T> as_const(const T* p) {
  return (ConstPtr<T>)p;
}

// Record b of the instance table, read through the constant view (the table is
// written only by host copies).  Only the device pass compiles the copy out of
// the constant address space; the host pass never runs this body.
__device__ __forceinline__ BInst load_inst(const BInst* tab, int b) {
#if defined(__HIP_DEVICE_COMPILE__)
  return as_const(tab)[b];
#else
  return tab[b];
#endif
}

// Instance owning workgroup `blk` given the prefix sums pre[0..count] (pre[0] = 0);
// returns the workgroup index within the instance in *local.
__device__ __forceinline__ int find_instance(const int* __restrict__ pre_, int count, int blk,
                                             int* local) {
  const ConstPtr<int> pre = as_const(pre_);
  int lo = 0, hi = count;                  // invariant: pre[lo] <= blk < pre[hi]
  while (hi - lo > 1) {
    const int mid = (lo + hi) >> 1;
    if (pre[mid] <= blk) lo = mid; else hi = mid;
  }
  *local = blk - pre[lo];
  return __builtin_amdgcn_readfirstlane(lo);
}

__device__ __forceinline__ GridRed inst_grid(const BInst& I, int ldp) {
  GridRed g;
  g.P1 = I.P1;
  g.G = I.G;
  g.ldp = ldp;
  return g;
}

__device__ __forceinline__ FinArgs inst_fin(const BInst& I, int kind, int j, int J, int ldc,
                                            int ldh) {
  FinArgs f{};
  f.kind = kind; f.qr = 0; f.j = j; f.J = J; f.ldc = ldc;
  f.ctrl = I.ctrl; f.coef = I.coef; f.pend = I.pend;
  f.H = I.H; f.K = I.K; f.ldh = ldh;
  f.R = nullptr; f.ldr = 0; f.Sprev = nullptr;
  f.gmres = I.gmres;
  f.Rg = I.Rg; f.cs = I.cs; f.sn = I.sn; f.g = I.g;
  return f;
}

// Does instance I take part in step j (its steps are first_j..n+1)?
__device__ __forceinline__ bool inst_active(const BInst& I, int j) {
  return I.active && j >= I.first_j && j <= I.n + 1 && I.ctrl->state == ST_RUNNING;
}

// Does instance I take part in the last-column finish (over its own n columns)?
__device__ __forceinline__ bool inst_running(const BInst& I) {
  return I.active && I.ctrl->state == ST_RUNNING;
}

// v = A w (5-point stencil), 512 rows per workgroup (two per thread).
__global__ __launch_bounds__(BS) void bstencil_kernel(const BInst* __restrict__ tab,
                                                      const int* __restrict__ pre, int count,
                                                      int j) {
  int local;
  const int b = find_instance(pre, count, blockIdx.x, &local);
  const BInst I = load_inst(tab, b);
  if (!inst_active(I, j)) return;
  const uint32_t nx = I.nx, ny = I.ny;
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    const int64_t i = (int64_t)local * 2 * BS + h * BS + threadIdx.x;
    if (i >= I.m) continue;
    const uint32_t ii = (uint32_t)i;
    const uint32_t ix = ii % nx, iy = ii / nx;
    const double* x = I.w;
    const bool ym = iy > 0, yp = iy + 1 < ny, xm = ix > 0, xp = ix + 1 < nx;
    // unconditional loads (an absent neighbour reads the row itself); an absent
    // term adds an exact zero
    const double vym = x[ym ? i - nx : i], vxm = x[xm ? i - 1 : i], vc = x[i];
    const double vxp = x[xp ? i + 1 : i], vyp = x[yp ? i + nx : i];
    double s = 0.0;
    s = fma(ym ? I.cym : 0.0, vym, s);
    s = fma(xm ? I.cxm : 0.0, vxm, s);
    s = fma(I.c0, vc, s);
    s = fma(xp ? I.cxp : 0.0, vxp, s);
    s = fma(yp ? I.cyp : 0.0, vyp, s);
    I.v[i] = s;
  }
}

// The DCGS2 reduction of step j for every active instance (or, when last != 0,
// the first reduction c = Q^T w of the last-column finish).
__global__ __launch_bounds__(BS) void breduce_kernel(const BInst* __restrict__ tab,
                                                     const int* __restrict__ pre, int count,
                                                     int j, int last, int ldp, int ldc, int ldh) {
  int local;
  const int b = find_instance(pre, count, blockIdx.x, &local);
  const BInst I = load_inst(tab, b);
  if (last ? !inst_running(I) : !inst_active(I, j)) return;
  const GridRed g = inst_grid(I, ldp);
  if (last == 2) {                        // plain squared norm of w (batched GMRES)
    reduce_body<2, false, double>(I.Q, I.ldq, 0, I.w, nullptr, I.m, g,
                                  inst_fin(I, FIN_NORM, 0, 0, ldc, ldh), local);
  } else if (last) {                      // over the instance's own n columns
    reduce_body<2, false, double>(I.Q, I.ldq, I.n, I.w, nullptr, I.m, g,
                                  inst_fin(I, FIN_LAST1, I.n + 2, I.n, ldc, ldh), local);
  } else {
    const int J = j - 2;
    const int kind = (I.restart && j == I.first_j) ? FIN_RESTART : FIN_STEP;
    reduce_body<2, true, double>(I.Q, I.ldq, J, I.w, I.v, I.m, g,
                                 inst_fin(I, kind, j, J, ldc, ldh), local);
  }
}

// q_{j-1} and w_j for every active instance.
__global__ __launch_bounds__(BS) void bupdate_kernel(const BInst* __restrict__ tab,
                                                     const int* __restrict__ pre, int count,
                                                     int j, int ldc) {
  int local;
  const int b = find_instance(pre, count, blockIdx.x, &local);
  const BInst I = load_inst(tab, b);
  if (!inst_active(I, j)) return;
  update_body<2, true, false, double>(I.Q, I.ldq, j - 2, I.w, I.v, nullptr, I.m, I.coef, ldc,
                                      I.ctrl, local);
}

// Last column, reduction 2: u = w - Q c into r, alpha = ||u||, H column closed.
__global__ __launch_bounds__(BS) void bproject_norm_kernel(const BInst* __restrict__ tab,
                                                           const int* __restrict__ pre,
                                                           int count, int ldp, int ldc,
                                                           int ldh) {
  int local;
  const int b = find_instance(pre, count, blockIdx.x, &local);
  const BInst I = load_inst(tab, b);
  if (!inst_running(I)) return;
  const int J = I.n;
  project_norm_body<2, double>(I.Q, I.ldq, J, I.w, I.r, I.m, inst_grid(I, ldp),
                               inst_fin(I, FIN_LAST2, J + 2, J, ldc, ldh), local);
}

// q_{n+1} = u / alpha into column n of every active instance's basis.
__global__ __launch_bounds__(BS) void bscale_kernel(const BInst* __restrict__ tab,
                                                    const int* __restrict__ pre, int count,
                                                    int ldc) {
  int local;
  const int b = find_instance(pre, count, blockIdx.x, &local);
  const BInst I = load_inst(tab, b);
  if (!inst_running(I)) return;
  const double alpha = I.coef[2 * ldc];
  const int J = I.n;
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    const int64_t i = (int64_t)local * 2 * BS + h * BS + threadIdx.x;
    if (i < I.m) I.Q[(int64_t)J * I.ldq + i] = I.r[i] / alpha;
  }
}

// Krylov-Schur truncation for the instances with truncate != 0:
//   Qn[:, 0..k) = Q[:, 0..p) Z[0..p, 0..k),  Qn[:, k] = Q[:, p],  w = Q[:, p].
// One row per thread, NO output columns per pass over Q: with NO >= k (the kept
// block, keep or keep + 1 when a complex pair is not split) Q is read once.
template <int NO>
__global__ __launch_bounds__(BS) void btruncate_kernel(const BInst* __restrict__ tab,
                                                       const int* __restrict__ pre, int count,
                                                       int p) {
  int local;
  const int b = find_instance(pre, count, blockIdx.x, &local);
  const BInst I = load_inst(tab, b);
  if (!I.active || !I.truncate) return;
  const int k = I.k;
  const ConstPtr<double> Z = as_const(I.Z);
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    const int64_t i = (int64_t)local * 2 * BS + h * BS + threadIdx.x;
    if (i >= I.m) continue;
    for (int o0 = 0; o0 < k; o0 += NO) {
      // Columns past k read column k-1 of Z (always in bounds) and are not stored:
      // no branch in the loop, so the loads of several c overlap.
      ConstPtr<double> zc[NO];
#pragma unroll
      for (int o = 0; o < NO; ++o) zc[o] = Z + (int64_t)min(o0 + o, k - 1) * p;
      double acc[NO];
#pragma unroll
      for (int o = 0; o < NO; ++o) acc[o] = 0.0;
#pragma unroll 4
      for (int c = 0; c < p; ++c) {
        const double q = I.Q[(int64_t)c * I.ldq + i];
#pragma unroll
        for (int o = 0; o < NO; ++o) acc[o] = fma(q, zc[o][c], acc[o]);
      }
#pragma unroll
      for (int o = 0; o < NO; ++o)
        if (o0 + o < k) I.Qn[(int64_t)(o0 + o) * I.ldq + i] = acc[o];
    }
    const double qp = I.Q[(int64_t)p * I.ldq + i];
    I.Qn[(int64_t)k * I.ldq + i] = qp;
    I.w[i] = qp;
  }
}

// Second half of the reductions, one workgroup per instance (see finish_body):
// mode 0 the reduction of step j, 1 and 2 the two reductions of the last-column
// finish over the instance's own n columns.
__global__ __launch_bounds__(FINISH_BS) void bfinish_kernel(const BInst* __restrict__ tab, int j,
                                                            int mode, int ldp, int ldc, int ldh) {
  const BInst I = load_inst(tab, blockIdx.x);
  if (mode == 0 ? !inst_active(I, j) : !inst_running(I)) return;
  const int J = mode == 0 ? j - 2 : mode == 3 ? 0 : I.n;
  const int jj = mode == 0 ? j : mode == 3 ? 0 : I.n + 2;
  const int kind = mode == 1 ? FIN_LAST1
                 : mode == 2 ? FIN_LAST2
                 : mode == 3 ? FIN_NORM
                 : (I.restart && j == I.first_j) ? FIN_RESTART : FIN_STEP;
  const int V = mode == 1 ? J + 1 : (mode == 2 || mode == 3) ? 1 : 2 * (J + 2);
  finish_body(inst_grid(I, ldp), V, inst_fin(I, kind, jj, J, ldc, ldh), J);
}

// LDS of bfinish_kernel for the largest J of the launch (j - 2 at step j; the largest
// instance n, passed as j - 2, for the last-column modes).
inline size_t bfinish_smem(int j, int mode) {
  const int J = j - 2;
  return finish_smem(mode == 1 ? J + 1 : mode == 2 ? 1 : 2 * (J + 2), J);
}

// Per-instance control reset at the start of a cycle (one thread per instance).
__global__ void breset_kernel(const BInst* __restrict__ tab, int count, double tau, double eta) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= count) return;
  const BInst I = tab[b];
  if (!I.active) return;
  Ctrl* c = I.ctrl;
  c->state = ST_RUNNING;
  c->stop_step = -1;
  c->k = 0;
  c->reductions = 0;
  c->fallbacks = 0;
  c->rho_next = 0.0;
  c->tau = tau;
  c->eta = eta;
  c->gmres_thresh = I.thresh;
  c->resid_est = 0.0;
  c->norm2 = 0.0;
}

// Batched GMRES residual: w = b - A x (copy_b: w = b), 512 rows per workgroup.
__global__ __launch_bounds__(BS) void bresidual_kernel(const BInst* __restrict__ tab,
                                                       const int* __restrict__ pre, int count,
                                                       int copy_b) {
  int local;
  const int b = find_instance(pre, count, blockIdx.x, &local);
  const BInst I = load_inst(tab, b);
  if (!I.active) return;
  const uint32_t nx = I.nx, ny = I.ny;
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    const int64_t i = (int64_t)local * 2 * BS + h * BS + threadIdx.x;
    if (i >= I.m) continue;
    if (copy_b) {
      I.w[i] = I.bvec[i];
      continue;
    }
    const uint32_t ii = (uint32_t)i;
    const uint32_t ix = ii % nx, iy = ii / nx;
    const double* x = I.x;
    const bool ym = iy > 0, yp = iy + 1 < ny, xm = ix > 0, xp = ix + 1 < nx;
    const double vym = x[ym ? i - nx : i], vxm = x[xm ? i - 1 : i], vc = x[i];
    const double vxp = x[xp ? i + 1 : i], vyp = x[yp ? i + nx : i];
    double s = 0.0;
    s = fma(ym ? I.cym : 0.0, vym, s);
    s = fma(xm ? I.cxm : 0.0, vxm, s);
    s = fma(I.c0, vc, s);
    s = fma(xp ? I.cxp : 0.0, vxp, s);
    s = fma(yp ? I.cyp : 0.0, vyp, s);
    I.w[i] = I.bvec[i] - s;
  }
}

// x += Q_{:,0..ksol) y for every active instance with a solution (y read through the
// constant view: written by a host copy before the launch).
__global__ __launch_bounds__(BS) void bxupdate_kernel(const BInst* __restrict__ tab,
                                                      const int* __restrict__ pre, int count) {
  int local;
  const int b = find_instance(pre, count, blockIdx.x, &local);
  const BInst I = load_inst(tab, b);
  if (!I.active || I.ksol <= 0) return;
  const ConstPtr<double> y = as_const(I.y);
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    const int64_t i = (int64_t)local * 2 * BS + h * BS + threadIdx.x;
    if (i >= I.m) continue;
    double acc = 0.0;
#pragma unroll 8
    for (int c = 0; c < I.ksol; ++c) acc = fma(I.Q[(int64_t)c * I.ldq + i], y[c], acc);
    I.x[i] += acc;
  }
}

inline unsigned bnb(int n) { return (unsigned)((n + BS - 1) / BS); }

// ---------------------------------------------------------------------------------
// Dense work of the Krylov-Schur restart on the GPU, one wavefront per instance:
// real Schur form of the p x p projected matrix, reordering by eigenvalue magnitude,
// the residual test, and the truncated Hessenberg matrix of the next cycle.
//
// The algorithms are those of the host implementation (schur.cpp): Householder
// reduction to Hessenberg form, the implicit Francis double-shift QR step (Golub &
// Van Loan, Alg. 7.5.1) with EISPACK's exceptional shifts, the standard form of 2x2
// blocks by a double-angle rotation, and adjacent block swaps through the Sylvester
// equation (Bai & Demmel).  T and Z live in LDS.  Scalar decisions (deflation, shifts, reflectors,
// rotations) are taken identically by every lane; each update of rows or columns
// gives one row or column to a lane, with the per-element arithmetic of the host
// code, so both paths agree up to the rounding of hypot.
constexpr int SCHUR_THREADS = 64;
constexpr double SEPS = 2.220446049250313e-16;

struct LMat {
  double* a;
  int ld;
  __device__ double& operator()(int i, int j) const { return a[j * ld + i]; }
};

__device__ __forceinline__ void wsync() { __syncthreads(); }

// Householder vector of x[0..n) (x, v: LDS or thread-private); every lane computes
// the same tau; lane-parallel writes when v is shared.
__device__ double s_make_house(const double* x, int n, double* v, bool shared_v) {
  double sigma = 0.0;
  for (int i = 1; i < n; ++i) sigma += x[i] * x[i];
  const double x0 = x[0];
  double v0 = 1.0, tau = 0.0;
  if (sigma != 0.0) {
    const double mu = sqrt(x0 * x0 + sigma);
    v0 = (x0 <= 0.0) ? x0 - mu : -sigma / (x0 + mu);
    tau = 2.0 * v0 * v0 / (sigma + v0 * v0);
  }
  if (shared_v) {
    wsync();                              // every lane has read x before v is written
    for (int i = threadIdx.x; i < n; i += SCHUR_THREADS)
      v[i] = i == 0 ? 1.0 : (sigma == 0.0 ? x[i] : x[i] / v0);
    wsync();
  } else {
    v[0] = 1.0;
    for (int i = 1; i < n; ++i) v[i] = sigma == 0.0 ? x[i] : x[i] / v0;
  }
  return tau;
}

// rows r0..r0+n-1, columns c0..c1: A <- (I - tau v v^T) A   (a column per lane)
__device__ void s_house_left(const LMat& A, const double* v, int n, double tau, int r0, int c0,
                             int c1) {
  for (int j = c0 + threadIdx.x; j <= c1; j += SCHUR_THREADS) {
    double s = 0.0;
    for (int i = 0; i < n; ++i) s += v[i] * A(r0 + i, j);
    s *= tau;
    for (int i = 0; i < n; ++i) A(r0 + i, j) -= s * v[i];
  }
  wsync();
}

// columns c0..c0+n-1, rows r0..r1: A <- A (I - tau v v^T)   (a row per lane)
__device__ void s_house_right(const LMat& A, const double* v, int n, double tau, int c0, int r0,
                              int r1) {
  for (int i = r0 + threadIdx.x; i <= r1; i += SCHUR_THREADS) {
    double s = 0.0;
    for (int k = 0; k < n; ++k) s += A(i, c0 + k) * v[k];
    s *= tau;
    for (int k = 0; k < n; ++k) A(i, c0 + k) -= s * v[k];
  }
  wsync();
}

__device__ void s_rot_rows(const LMat& A, int i, int c0, int c1, double cs, double sn) {
  for (int j = c0 + threadIdx.x; j <= c1; j += SCHUR_THREADS) {
    const double x = A(i, j), y = A(i + 1, j);
    A(i, j) = cs * x + sn * y;
    A(i + 1, j) = -sn * x + cs * y;
  }
  wsync();
}

__device__ void s_rot_cols(const LMat& A, int i, int r0, int r1, double cs, double sn) {
  for (int r = r0 + threadIdx.x; r <= r1; r += SCHUR_THREADS) {
    const double x = A(r, i), y = A(r, i + 1);
    A(r, i) = cs * x + sn * y;
    A(r, i + 1) = -sn * x + cs * y;
  }
  wsync();
}

__device__ __forceinline__ void dswap(double& a, double& b) { const double t = a; a = b; b = t; }

__device__ void s_standardize(int p, const LMat& T, const LMat& Z, int i) {
  double a = T(i, i), b = T(i, i + 1), c = T(i + 1, i), d = T(i + 1, i + 1), cs, sn;
  std2x2(a, b, c, d, cs, sn);
  wsync();
  if (i + 2 <= p - 1) s_rot_rows(T, i, i + 2, p - 1, cs, sn);
  if (i >= 1) s_rot_cols(T, i, 0, i - 1, cs, sn);
  s_rot_cols(Z, i, 0, p - 1, cs, sn);
  if (threadIdx.x == 0) { T(i, i) = a; T(i, i + 1) = b; T(i + 1, i) = c; T(i + 1, i + 1) = d; }
  wsync();
}

__device__ __forceinline__ int s_block_size(const LMat& T, int p, int i) {
  return (i + 1 < p && T(i + 1, i) != 0.0) ? 2 : 1;
}

__device__ __forceinline__ double s_block_mag(const LMat& T, int i, int sz) {
  if (sz == 1) return fabs(T(i, i));
  return sqrt(T(i, i) * T(i, i) + fabs(T(i, i + 1) * T(i + 1, i)));
}

// Gaussian elimination with partial pivoting, N <= 4 (scalar)
__device__ bool s_small_solve(int N, double* M, double* rhs) {
  for (int k = 0; k < N; ++k) {
    int piv = k;
    for (int i = k + 1; i < N; ++i)
      if (fabs(M[k * N + i]) > fabs(M[k * N + piv])) piv = i;
    if (M[k * N + piv] == 0.0) return false;
    if (piv != k) {
      for (int j = 0; j < N; ++j) dswap(M[j * N + k], M[j * N + piv]);
      dswap(rhs[k], rhs[piv]);
    }
    for (int i = k + 1; i < N; ++i) {
      const double f = M[k * N + i] / M[k * N + k];
      for (int j = k; j < N; ++j) M[j * N + i] -= f * M[j * N + k];
      rhs[i] -= f * rhs[k];
    }
  }
  for (int i = N - 1; i >= 0; --i) {
    double s = rhs[i];
    for (int j = i + 1; j < N; ++j) s -= M[j * N + i] * rhs[j];
    rhs[i] = s / M[i * N + i];
  }
  return true;
}

// Swap the adjacent diagonal blocks at j (sizes n1, n2); returns 0 on success.
__device__ int s_swap_blocks(int p, const LMat& T, const LMat& Z, int j, int n1, int n2) {
  if (n1 == 1 && n2 == 1) {
    const double t11 = T(j, j), t22 = T(j + 1, j + 1), t12 = T(j, j + 1);
    const double r = hypot(t12, t22 - t11);
    if (r == 0.0) return 0;
    const double cs = t12 / r, sn = (t22 - t11) / r;
    wsync();
    s_rot_rows(T, j, j, p - 1, cs, sn);
    s_rot_cols(T, j, 0, j + 1, cs, sn);
    s_rot_cols(Z, j, 0, p - 1, cs, sn);
    if (threadIdx.x == 0) { T(j, j) = t22; T(j + 1, j + 1) = t11; T(j + 1, j) = 0.0; }
    wsync();
    return 0;
  }
  const int n = n1 + n2;
  const int N = n1 * n2;
  double M[16], x[4];
  for (int i = 0; i < 16; ++i) M[i] = 0.0;
  for (int jj = 0; jj < n2; ++jj)
    for (int ii = 0; ii < n1; ++ii) {
      const int row = ii + jj * n1;
      for (int k = 0; k < n1; ++k) M[(k + jj * n1) * N + row] += T(j + ii, j + k);
      for (int k = 0; k < n2; ++k) M[(ii + k * n1) * N + row] -= T(j + n1 + k, j + n1 + jj);
      x[row] = T(j + ii, j + n1 + jj);
    }
  if (!s_small_solve(N, M, x)) return 1;
  double W[16], Qh[16];
  for (int i = 0; i < 16; ++i) { W[i] = 0.0; Qh[i] = 0.0; }
  for (int jj = 0; jj < n2; ++jj) {
    for (int ii = 0; ii < n1; ++ii) W[jj * n + ii] = -x[ii + jj * n1];
    W[jj * n + n1 + jj] = 1.0;
  }
  for (int i = 0; i < n; ++i) Qh[i * n + i] = 1.0;
  for (int c = 0; c < n2; ++c) {          // thread-private 4 x 4 Householder QR
    double v[4], col[4];
    const int len = n - c;
    for (int i = 0; i < len; ++i) col[i] = W[c * n + c + i];
    const double tau = s_make_house(col, len, v, false);
    if (tau == 0.0) continue;
    for (int jc = c; jc <= n2 - 1; ++jc) {
      double s = 0.0;
      for (int i = 0; i < len; ++i) s += v[i] * W[jc * n + c + i];
      s *= tau;
      for (int i = 0; i < len; ++i) W[jc * n + c + i] -= s * v[i];
    }
    for (int r = 0; r <= n - 1; ++r) {
      double s = 0.0;
      for (int k = 0; k < len; ++k) s += Qh[(c + k) * n + r] * v[k];
      s *= tau;
      for (int k = 0; k < len; ++k) Qh[(c + k) * n + r] -= s * v[k];
    }
  }
  wsync();
  // T <- Qh^T T Qh on the affected rows and columns, Z <- Z Qh
  for (int col = j + threadIdx.x; col < p; col += SCHUR_THREADS) {   // rows j..j+n-1
    double tmp[4];
    for (int i = 0; i < n; ++i) {
      double s = 0.0;
      for (int k = 0; k < n; ++k) s += Qh[i * n + k] * T(j + k, col);
      tmp[i] = s;
    }
    for (int i = 0; i < n; ++i) T(j + i, col) = tmp[i];
  }
  wsync();
  for (int r = threadIdx.x; r <= j + n - 1; r += SCHUR_THREADS) {
    double tmp[4];
    for (int i = 0; i < n; ++i) {
      double s = 0.0;
      for (int k = 0; k < n; ++k) s += T(r, j + k) * Qh[i * n + k];
      tmp[i] = s;
    }
    for (int i = 0; i < n; ++i) T(r, j + i) = tmp[i];
  }
  for (int r = threadIdx.x; r <= p - 1; r += SCHUR_THREADS) {
    double tmp[4];
    for (int i = 0; i < n; ++i) {
      double s = 0.0;
      for (int k = 0; k < n; ++k) s += Z(r, j + k) * Qh[i * n + k];
      tmp[i] = s;
    }
    for (int i = 0; i < n; ++i) Z(r, j + i) = tmp[i];
  }
  wsync();
  if (threadIdx.x == 0) {
    for (int cc = 0; cc < n2; ++cc)
      for (int rr = n2; rr < n; ++rr) T(j + rr, j + cc) = 0.0;
    if (n2 != 2) T(j + 1, j) = 0.0;
  }
  wsync();
  if (n2 == 2) s_standardize(p, T, Z, j);
  if (n1 == 2) s_standardize(p, T, Z, j + n2);
  return 0;
}

// Real Schur form of A (p x p, LDS) in place, Z accumulated; 0 on success.
__device__ int s_real_schur(int p, const LMat& A, const LMat& Z, double* vbuf) {
  for (int t = threadIdx.x; t < p * p; t += SCHUR_THREADS)
    Z(t % p, t / p) = (t % p == t / p) ? 1.0 : 0.0;
  wsync();
  if (p <= 1) return 0;
  for (int k = 0; k + 2 < p; ++k) {        // Hessenberg reduction
    const int n = p - k - 1;
    for (int i = threadIdx.x; i < n; i += SCHUR_THREADS) vbuf[p + i] = A(k + 1 + i, k);
    wsync();
    const double tau = s_make_house(vbuf + p, n, vbuf, true);
    if (tau != 0.0) {
      s_house_left(A, vbuf, n, tau, k + 1, k, p - 1);
      s_house_right(A, vbuf, n, tau, k + 1, 0, p - 1);
      s_house_right(Z, vbuf, n, tau, k + 1, 0, p - 1);
    }
    for (int i = k + 2 + threadIdx.x; i < p; i += SCHUR_THREADS) A(i, k) = 0.0;
    wsync();
  }
  double anorm = 0.0;
  for (int j = 0; j < p; ++j)
    for (int i = 0; i <= min(j + 1, p - 1); ++i) anorm = fmax(anorm, fabs(A(i, j)));
  int hi = p - 1, its = 0, total = 0;
  const int max_total = 60 * p + 100;
  while (hi >= 0) {
    int l = hi;
    for (; l > 0; --l) {
      double s = fabs(A(l - 1, l - 1)) + fabs(A(l, l));
      if (s == 0.0) s = anorm;
      if (fabs(A(l, l - 1)) <= SEPS * s) break;
    }
    wsync();
    if (l > 0) {
      if (threadIdx.x == 0) A(l, l - 1) = 0.0;
      wsync();
    }
    if (l == hi) { hi -= 1; its = 0; continue; }
    if (l == hi - 1) { s_standardize(p, A, Z, hi - 1); hi -= 2; its = 0; continue; }
    if (++total > max_total) return 1;
    ++its;
    double s, t;
    if (its == 10 || its == 20) {
      const double ex = fabs(A(hi, hi - 1)) + fabs(A(hi - 1, hi - 2));
      s = 1.5 * ex;
      t = ex * ex;
    } else {
      s = A(hi - 1, hi - 1) + A(hi, hi);
      t = A(hi - 1, hi - 1) * A(hi, hi) - A(hi - 1, hi) * A(hi, hi - 1);
    }
    double xx = A(l, l) * A(l, l) + A(l, l + 1) * A(l + 1, l) - s * A(l, l) + t;
    double yy = A(l + 1, l) * (A(l, l) + A(l + 1, l + 1) - s);
    double zz = A(l + 1, l) * A(l + 2, l + 1);
    for (int k = l; k <= hi - 2; ++k) {
      const double xv[3] = {xx, yy, zz};
      double hv[3];
      const double tau = s_make_house(xv, 3, hv, false);
      wsync();
      if (tau != 0.0) {
        s_house_left(A, hv, 3, tau, k, max(l, k - 1), p - 1);
        s_house_right(A, hv, 3, tau, k, 0, min(k + 3, hi));
        s_house_right(Z, hv, 3, tau, k, 0, p - 1);
      }
      if (k > l && threadIdx.x == 0) { A(k + 1, k - 1) = 0.0; A(k + 2, k - 1) = 0.0; }
      wsync();
      xx = A(k + 1, k);
      yy = A(k + 2, k);
      if (k < hi - 2) zz = A(k + 3, k);
    }
    const double xv[2] = {xx, yy};
    double hv[2];
    const double tau = s_make_house(xv, 2, hv, false);
    wsync();
    if (tau != 0.0) {
      s_house_left(A, hv, 2, tau, hi - 1, hi - 2, p - 1);
      s_house_right(A, hv, 2, tau, hi - 1, 0, hi);
      s_house_right(Z, hv, 2, tau, hi - 1, 0, p - 1);
    }
    if (threadIdx.x == 0) A(hi, hi - 2) = 0.0;
    wsync();
  }
  return 0;
}

// Eigenvalues of the standardised quasi-triangular T (every lane, same values).
__device__ void s_eigen(int p, const LMat& T, double* re, double* im) {
  wsync();
  if (threadIdx.x == 0) {
    for (int i = 0; i < p;) {
      if (s_block_size(T, p, i) == 2) {
        const double a = 0.5 * (T(i, i) + T(i + 1, i + 1));
        const double w = sqrt(fabs(T(i, i + 1))) * sqrt(fabs(T(i + 1, i)));
        re[i] = a; im[i] = w; re[i + 1] = a; im[i + 1] = -w;
        i += 2;
      } else {
        re[i] = T(i, i); im[i] = 0.0;
        i += 1;
      }
    }
  }
  wsync();
}

// Leading `count` eigenvalues by magnitude (see schur.cpp); -1 on failure.
__device__ int s_reorder(int p, const LMat& T, const LMat& Z, int count, double cut_gap,
                         double* re, double* im, double* mags) {
  if (count >= p) count = p;
  s_eigen(p, T, re, im);
  if (threadIdx.x == 0) {                  // magnitudes, sorted descending (insertion)
    for (int i = 0; i < p; ++i) {
      const double v = hypot(re[i], im[i]);
      int k = i;
      while (k > 0 && mags[k - 1] < v) { mags[k] = mags[k - 1]; --k; }
      mags[k] = v;
    }
  }
  wsync();
  int cnt = count > 1 ? count : 1;
  while (cnt < p && mags[cnt - 1] - mags[cnt] <= cut_gap * mags[0]) ++cnt;
  int filled = 0, guard = 0;
  while (filled < cnt) {
    if (++guard > 4 * p + 4) return -1;
    int best = -1;
    double bmag = -1.0;
    for (int i = filled; i < p;) {
      const int sz = s_block_size(T, p, i);
      const double mg = s_block_mag(T, i, sz);
      if (mg > bmag) { bmag = mg; best = i; }
      i += sz;
    }
    int pos = best;
    while (pos > filled) {
      int i = filled, prev = filled;
      while (i < pos) { prev = i; i += s_block_size(T, p, i); }
      if (i != pos) return -1;
      const int above = pos - prev;
      const int cur = s_block_size(T, p, pos);
      wsync();
      if (s_swap_blocks(p, T, Z, prev, above, cur) != 0) return -1;
      pos = prev;
    }
    filled += s_block_size(T, p, filled);
    wsync();
  }
  return filled;
}

// Restart work of every active, running instance: Schur form and reordering of its
// p x p projected matrix H (ld x ld in B.H), the Ritz values (the first nev after
// reordering) and residual estimate, then reordering for `keep` and the truncated
// Hessenberg matrix and Schur vectors of the next cycle, written in place (H) and to
// Zout (p x p per instance).  ires[b] = {state, kn, k, 0}: state 0 skipped (inactive
// or stopped), 1 done, -1 the Schur form or the first reordering failed (no Ritz
// values), -2 the reordering for keep failed (Ritz values and residual valid).
__global__ __launch_bounds__(SCHUR_THREADS) void bschur_kernel(
    const BInst* __restrict__ tab, int p, int ld, int nev, int keep, double cut_gap,
    double* __restrict__ Hall, double* __restrict__ Zall, int* __restrict__ ires,
    double* __restrict__ resid, double* __restrict__ ere, double* __restrict__ eim) {
  extern __shared__ double sm[];
  const int b = blockIdx.x;
  const BInst I = load_inst(tab, b);
  int* out = ires + 4 * b;
  if (!I.active || I.ctrl->state != ST_RUNNING) {
    if (threadIdx.x == 0) { out[0] = 0; out[1] = 0; out[2] = 0; out[3] = 0; }
    return;
  }
  double* Hb = Hall + (size_t)b * ld * ld;
  double* Zb = Zall + (size_t)b * p * p;
  const LMat T{sm, p}, Z{sm + p * p, p};
  double* vbuf = sm + 2 * p * p;          // 2p
  double* re = vbuf + 2 * p;
  double* im = re + p;
  double* mags = im + p;
  const double h = Hb[(size_t)(p - 1) * ld + p];
  for (int t = threadIdx.x; t < p * p; t += SCHUR_THREADS) T(t % p, t / p) = Hb[(t / p) * ld + t % p];
  wsync();
  int fail = s_real_schur(p, T, Z, vbuf);
  int kn = fail ? -1 : s_reorder(p, T, Z, nev, cut_gap, re, im, mags);
  if (kn < 0) {
    if (threadIdx.x == 0) { out[0] = -1; out[1] = 0; out[2] = 0; out[3] = 0; }
    return;
  }
  s_eigen(p, T, re, im);
  if (threadIdx.x == 0) {
    double bn = 0.0, tmin = INFINITY;
    for (int i = 0; i < kn; ++i) {
      const double bi = h * Z(p - 1, i);
      bn += bi * bi;
      tmin = fmin(tmin, hypot(re[i], im[i]));
    }
    resid[b] = sqrt(bn) / tmin;
    for (int i = 0; i < nev; ++i) {
      ere[(size_t)b * nev + i] = re[i];
      eim[(size_t)b * nev + i] = im[i];
    }
  }
  wsync();
  const int k = s_reorder(p, T, Z, keep, cut_gap, re, im, mags);
  if (threadIdx.x == 0) { out[0] = (k < 0 || k >= p) ? -2 : 1; out[1] = kn; out[2] = k; out[3] = 0; }
  if (k < 0 || k >= p) return;
  // next cycle: H = [T_k; h Z(p-1, 0:k)] in the leading (k+1) x k block, zero elsewhere
  for (int t = threadIdx.x; t < ld * ld; t += SCHUR_THREADS) {
    const int i = t % ld, jj = t / ld;
    double v = 0.0;
    if (jj < k && i < k) v = T(i, jj);
    else if (jj < k && i == k) v = h * Z(p - 1, jj);
    Hb[t] = v;
  }
  for (int t = threadIdx.x; t < p * p; t += SCHUR_THREADS) Zb[t] = Z(t % p, t / p);
}

}  // namespace


hipError_t launch_bstencil(const BInst* tab, const int* pre_rows, int count, int nblocks, int j,
                           hipStream_t s) {
  bstencil_kernel<<<nblocks, BS, 0, s>>>(tab, pre_rows, count, j);
  return hipGetLastError();
}

hipError_t launch_breduce(const BInst* tab, const int* pre_red, int count, int nblocks, int j,
                          int last, int ldp, int ldc, int ldh, hipStream_t s) {
  breduce_kernel<<<nblocks, BS, sizeof(double) * NW * 2 * NT, s>>>(tab, pre_red, count, j, last,
                                                                  ldp, ldc, ldh);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  const int mode = last ? 1 : 0;
  bfinish_kernel<<<count, FINISH_BS, bfinish_smem(j, mode), s>>>(tab, j, mode, ldp, ldc, ldh);
  return hipGetLastError();
}

hipError_t launch_bupdate(const BInst* tab, const int* pre_rows, int count, int nblocks, int j,
                          int ldc, hipStream_t s) {
  bupdate_kernel<<<nblocks, BS, 0, s>>>(tab, pre_rows, count, j, ldc);
  return hipGetLastError();
}

hipError_t launch_bproject_norm(const BInst* tab, const int* pre_red, int count, int nblocks,
                                int j, int ldp, int ldc, int ldh, hipStream_t s) {
  bproject_norm_kernel<<<nblocks, BS, sizeof(double) * NW, s>>>(tab, pre_red, count, ldp, ldc,
                                                               ldh);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  bfinish_kernel<<<count, FINISH_BS, bfinish_smem(j, 2), s>>>(tab, j, 2, ldp, ldc, ldh);
  return hipGetLastError();
}

hipError_t launch_bscale(const BInst* tab, const int* pre_rows, int count, int nblocks, int j,
                         int ldc, hipStream_t s) {
  (void)j;
  bscale_kernel<<<nblocks, BS, 0, s>>>(tab, pre_rows, count, ldc);
  return hipGetLastError();
}

hipError_t launch_btruncate(const BInst* tab, const int* pre_rows, int count, int nblocks, int p,
                            hipStream_t s) {
  btruncate_kernel<24><<<nblocks, BS, 0, s>>>(tab, pre_rows, count, p);
  return hipGetLastError();
}

size_t bschur_smem(int p) { return sizeof(double) * (size_t)(2 * p * p + 5 * p); }

hipError_t launch_bschur(const BInst* tab, int count, int p, int ld, int nev, int keep,
                         double cut_gap, double* H, double* Z, int* ires, double* resid,
                         double* ere, double* eim, hipStream_t s) {
  if (count <= 0) return hipSuccess;
  if (p < 2 || p > BSCHUR_MAX_P || nev < 1 || keep < 1) return hipErrorInvalidValue;
  bschur_kernel<<<count, SCHUR_THREADS, bschur_smem(p), s>>>(tab, p, ld, nev, keep, cut_gap, H, Z,
                                                             ires, resid, ere, eim);
  return hipGetLastError();
}

hipError_t launch_bresidual(const BInst* tab, const int* pre_rows, int count, int nblocks,
                            int copy_b, hipStream_t s) {
  bresidual_kernel<<<nblocks, BS, 0, s>>>(tab, pre_rows, count, copy_b);
  return hipGetLastError();
}

hipError_t launch_bnorm(const BInst* tab, const int* pre_red, int count, int nblocks, int ldp,
                        int ldc, int ldh, hipStream_t s) {
  breduce_kernel<<<nblocks, BS, sizeof(double) * NW * 2 * NT, s>>>(tab, pre_red, count, 0, 2,
                                                                  ldp, ldc, ldh);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  bfinish_kernel<<<count, FINISH_BS, finish_smem(1, 0), s>>>(tab, 0, 3, ldp, ldc, ldh);
  return hipGetLastError();
}

hipError_t launch_bxupdate(const BInst* tab, const int* pre_rows, int count, int nblocks,
                           hipStream_t s) {
  bxupdate_kernel<<<nblocks, BS, 0, s>>>(tab, pre_rows, count);
  return hipGetLastError();
}

hipError_t launch_breset(const BInst* tab, int count, double tau, double eta, hipStream_t s) {
  breset_kernel<<<bnb(count), BS, 0, s>>>(tab, count, tau, eta);
  return hipGetLastError();
}

}  // namespace dcgs2
