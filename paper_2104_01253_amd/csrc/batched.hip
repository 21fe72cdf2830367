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

namespace dcgs2 {
namespace {

#include "device_common.h"

// Instance owning workgroup `blk` given the prefix sums pre[0..count] (pre[0] = 0);
// returns the workgroup index within the instance in *local.
__device__ __forceinline__ int find_instance(const int* __restrict__ pre, int count, int blk,
                                             int* local) {
  int lo = 0, hi = count;                  // invariant: pre[lo] <= blk < pre[hi]
  while (hi - lo > 1) {
    const int mid = (lo + hi) >> 1;
    if (pre[mid] <= blk) lo = mid; else hi = mid;
  }
  *local = blk - pre[lo];
  return lo;
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
  f.kind = kind; f.qr = 0; f.j = j; f.J = J; f.gmres = 0; f.ldc = ldc;
  f.ctrl = I.ctrl; f.coef = I.coef; f.pend = I.pend;
  f.H = I.H; f.K = I.K; f.ldh = ldh;
  f.R = nullptr; f.ldr = 0; f.Sprev = nullptr;
  f.Rg = nullptr; f.cs = nullptr; f.sn = nullptr; f.g = nullptr;
  return f;
}

// Does instance I take part in step j?
__device__ __forceinline__ bool inst_active(const BInst& I, int j) {
  return I.active && j >= I.first_j && I.ctrl->state == ST_RUNNING;
}

// v = A w (5-point stencil), 512 rows per workgroup (two per thread).
__global__ __launch_bounds__(BS) void bstencil_kernel(const BInst* __restrict__ tab,
                                                      const int* __restrict__ pre, int count,
                                                      int j) {
  int local;
  const int b = find_instance(pre, count, blockIdx.x, &local);
  const BInst I = tab[b];
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
  const BInst I = tab[b];
  if (!inst_active(I, j)) return;
  const int J = j - 2;
  const GridRed g = inst_grid(I, ldp);
  if (last) {
    reduce_body<2, false, double>(I.Q, I.ldq, J, I.w, nullptr, I.m, g,
                                  inst_fin(I, FIN_LAST1, j, J, ldc, ldh), local);
  } else {
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
  const BInst I = tab[b];
  if (!inst_active(I, j)) return;
  update_body<2, true, false, double>(I.Q, I.ldq, j - 2, I.w, I.v, nullptr, I.m, I.coef, ldc,
                                      I.ctrl, local);
}

// Last column, reduction 2: u = w - Q c into r, alpha = ||u||, H column closed.
__global__ __launch_bounds__(BS) void bproject_norm_kernel(const BInst* __restrict__ tab,
                                                           const int* __restrict__ pre,
                                                           int count, int j, int ldp, int ldc,
                                                           int ldh) {
  int local;
  const int b = find_instance(pre, count, blockIdx.x, &local);
  const BInst I = tab[b];
  if (!inst_active(I, j)) return;
  const int J = j - 2;
  project_norm_body<2, double>(I.Q, I.ldq, J, I.w, I.r, I.m, inst_grid(I, ldp),
                               inst_fin(I, FIN_LAST2, j, J, ldc, ldh), local);
}

// q_{p+1} = u / alpha into column J of every active instance's basis.
__global__ __launch_bounds__(BS) void bscale_kernel(const BInst* __restrict__ tab,
                                                    const int* __restrict__ pre, int count,
                                                    int j, int ldc) {
  int local;
  const int b = find_instance(pre, count, blockIdx.x, &local);
  const BInst I = tab[b];
  if (!inst_active(I, j)) return;
  const double alpha = I.coef[2 * ldc];
  const int J = j - 2;
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    const int64_t i = (int64_t)local * 2 * BS + h * BS + threadIdx.x;
    if (i < I.m) I.Q[(int64_t)J * I.ldq + i] = I.r[i] / alpha;
  }
}

// Krylov-Schur truncation for the instances with truncate != 0:
//   Qn[:, 0..k) = Q[:, 0..p) Z[0..p, 0..k),  Qn[:, k] = Q[:, p],  w = Q[:, p].
// One row per thread, NO output columns per pass.
template <int NO>
__global__ __launch_bounds__(BS) void btruncate_kernel(const BInst* __restrict__ tab,
                                                       const int* __restrict__ pre, int count,
                                                       int p) {
  int local;
  const int b = find_instance(pre, count, blockIdx.x, &local);
  const BInst I = tab[b];
  if (!I.active || !I.truncate) return;
  const int k = I.k;
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    const int64_t i = (int64_t)local * 2 * BS + h * BS + threadIdx.x;
    if (i >= I.m) continue;
    for (int o0 = 0; o0 < k; o0 += NO) {
      double acc[NO];
#pragma unroll
      for (int o = 0; o < NO; ++o) acc[o] = 0.0;
      for (int c = 0; c < p; ++c) {
        const double q = I.Q[(int64_t)c * I.ldq + i];
#pragma unroll
        for (int o = 0; o < NO; ++o)
          if (o0 + o < k) acc[o] = fma(q, I.Z[(int64_t)(o0 + o) * p + c], acc[o]);
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

// Second half of the reductions of step j, one workgroup per instance (see
// finish_body): mode 0 the step's reduction, 1 and 2 the two reductions of the
// last-column finish.
__global__ __launch_bounds__(FINISH_BS) void bfinish_kernel(const BInst* __restrict__ tab, int j,
                                                            int mode, int ldp, int ldc, int ldh) {
  const BInst I = tab[blockIdx.x];
  if (!inst_active(I, j)) return;
  const int J = j - 2;
  const int kind = mode == 1 ? FIN_LAST1
                 : mode == 2 ? FIN_LAST2
                 : (I.restart && j == I.first_j) ? FIN_RESTART : FIN_STEP;
  const int V = mode == 1 ? J + 1 : mode == 2 ? 1 : 2 * (J + 2);
  finish_body(inst_grid(I, ldp), V, inst_fin(I, kind, j, J, ldc, ldh), J);
}

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
  c->gmres_thresh = 0.0;
  c->resid_est = 0.0;
  c->norm2 = 0.0;
}

inline unsigned bnb(int n) { return (unsigned)((n + BS - 1) / BS); }

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
  bproject_norm_kernel<<<nblocks, BS, sizeof(double) * NW, s>>>(tab, pre_red, count, j, ldp, ldc,
                                                               ldh);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  bfinish_kernel<<<count, FINISH_BS, bfinish_smem(j, 2), s>>>(tab, j, 2, ldp, ldc, ldh);
  return hipGetLastError();
}

hipError_t launch_bscale(const BInst* tab, const int* pre_rows, int count, int nblocks, int j,
                         int ldc, hipStream_t s) {
  bscale_kernel<<<nblocks, BS, 0, s>>>(tab, pre_rows, count, j, ldc);
  return hipGetLastError();
}

hipError_t launch_btruncate(const BInst* tab, const int* pre_rows, int count, int nblocks, int p,
                            hipStream_t s) {
  btruncate_kernel<8><<<nblocks, BS, 0, s>>>(tab, pre_rows, count, p);
  return hipGetLastError();
}

hipError_t launch_breset(const BInst* tab, int count, double tau, double eta, hipStream_t s) {
  breset_kernel<<<bnb(count), BS, 0, s>>>(tab, count, tau, eta);
  return hipGetLastError();
}

}  // namespace dcgs2
