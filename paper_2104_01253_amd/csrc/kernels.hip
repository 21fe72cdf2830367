// HIP kernels for the DCGS2 Arnoldi-QR expansion on gfx950 (MI355X).
//
// Method: Bielich et al., "Low-Synch Gram-Schmidt with Delayed
// Reorthogonalization for Krylov Solvers" (arXiv 2104.01253), Sec. 3 (Alg. qr),
// Sec. 4 (Alg. arnoldi and eqs. (08)-(52)).
//
// One DCGS2 step j is two streaming passes over the tall-skinny basis Q plus a
// scalar tail that a single workgroup runs:
//   reduce   [Q_{1:j-2}, w_{j-1}, y]^T [w_{j-1}, y]   (y = A w_{j-1} or a_j)
//            -> per-workgroup partials; a one-workgroup finishing kernel sums
//            them in a fixed order and finalises the step (alpha by the
//            Pythagorean trick, Stephen's trick, T, and the H/K or R updates).
//   update   q_{j-1} = (w - Q C)/alpha into Q[:, j-1] and
//            w_j = y/alpha - Q_{1:j-1} T (Arnoldi) or a_j - Q_{1:j-1} S (QR).
// Both passes are bound by HBM bandwidth (about 0.5 flop per byte, far below
// the fp64 ridge of the chip), so they are written as coalesced 16-byte
// streams over rows with the per-column coefficients held uniform (scalar
// registers), not as matrix-core tiles.  The grid sum is deterministic: the
// partials are added in a fixed order, so repeated runs are bitwise identical.
#include <hip/hip_runtime.h>
#include <math.h>

#include <algorithm>
#include <mutex>
#include <type_traits>
#include <utility>

#include "internal.h"

// Fixed scratch of the allocation-free QR entry point (dcgs2_qr_noalloc): every GPU the
// library runs on holds its own copy until the process ends.  Host code never passes
// this name to a kernel (on the host it is only a stand-in for the symbol): it takes
// the device address from dcgs2::noalloc_scratch.
namespace {
constexpr size_t noalloc_region(size_t doubles) { return (doubles + 63) / 64 * 64; }
constexpr size_t NOALLOC_DOUBLES =
    2 * noalloc_region(dcgs2::NOALLOC_MAX_M) +
    noalloc_region((size_t)dcgs2::REDUCE_GMAX * dcgs2::NOALLOC_LDP) +
    2 * noalloc_region(dcgs2::NOALLOC_LDCOEF) +
    noalloc_region((size_t)dcgs2::NOALLOC_MAX_N * dcgs2::NOALLOC_MAX_N) +
    noalloc_region(dcgs2::NOALLOC_MAX_N + 2) + noalloc_region(sizeof(dcgs2::Ctrl) / 8 + 1);
}  // namespace
static __device__ __align__(256) double scratch[NOALLOC_DOUBLES];

namespace dcgs2 {
namespace {

#include "device_common.h"

template <int VW, bool HASY, typename TQ, bool STAGED>
__global__ __launch_bounds__(BS) void reduce_kernel(const TQ* __restrict__ Q, int64_t ldq,
                                                    int J, const double* __restrict__ x,
                                                    const double* __restrict__ y, int64_t m,
                                                    GridRed gr, FinArgs fin) {
  reduce_body<VW, HASY, TQ, STAGED ? 1 : 0>(Q, ldq, J, x, y, m, gr, fin, blockIdx.x);
}

// ---------------------------------------------------------------------------------
// Stencil rows (lexicographic grid, x fastest; out-of-grid neighbours are zero, as
// for Dirichlet boundaries), shared by the matvec kernel and the reduction pass that
// computes its own y = A x.

__device__ __forceinline__ uint32_t div_by(uint32_t n, DivMagic g) {
  const uint32_t t = __umulhi(g.mul, n);
  return (t + ((n - t) >> g.sh1)) >> g.sh2;
}

// Loads the seven values of x that row i reads, in the order (z-, y-, x-, centre,
// x+, y+, z+); an absent neighbour reads row i and is flagged false.  Grid
// coordinates come from two divisions by the invariant nx and ny done as
// multiplications.  OFF32: every byte offset into x fits 32 bits (m < 2^29), so the
// loads take a 32-bit offset from one base register.
template <bool OFF32>
__device__ __forceinline__ void stencil_gather(const OpDev& op, const double* __restrict__ x,
                                               uint32_t i, double (&v)[7], bool (&in)[7]) {
  const uint32_t nx = op.nx, ny = op.ny, nz = op.nz;
  const uint32_t sxy = nx * ny;
  const uint32_t r = div_by(i, op.dx);            // i / nx
  const uint32_t ix = i - r * nx;
  const uint32_t iz = div_by(r, op.dy);           // i / (nx ny)
  const uint32_t iy = r - iz * ny;
  in[0] = nz > 1 && iz > 0;
  in[1] = iy > 0;
  in[2] = ix > 0;
  in[3] = true;
  in[4] = ix + 1 < nx;
  in[5] = iy + 1 < ny;
  in[6] = nz > 1 && iz + 1 < nz;
  const uint32_t nb[7] = {i - sxy, i - nx, i - 1, i, i + 1, i + nx, i + sxy};
#pragma unroll
  for (int t = 0; t < 7; ++t) {
    const uint32_t k = in[t] ? nb[t] : i;
    if constexpr (OFF32)
      v[t] = *reinterpret_cast<const double*>(reinterpret_cast<const char*>(x) +
                                              k * (uint32_t)sizeof(double));
    else
      v[t] = x[k];
  }
}

// (A x)_i from the gathered values: terms in neighbour order, an absent term adds an
// exact zero.
__device__ __forceinline__ double stencil_sum(const OpDev& op, const double (&v)[7],
                                              const bool (&in)[7]) {
  const double c[7] = {op.czm, op.cym, op.cxm, op.c0, op.cxp, op.cyp, op.czp};
  double s = 0.0;
#pragma unroll
  for (int t = 0; t < 7; ++t) s = fma(in[t] ? c[t] : 0.0, v[t], s);
  return s;
}

// Reduction pass of an Arnoldi step with the matvec folded in: [Q_{0..J-1}, x, y]^T
// [x, y] as reduce_kernel, where y = A x is computed for the workgroup's slab (stored to
// y for the update pass and kept with x in LDS for the sweeps) by the first column-group
// sweep (FP64 basis) or before the sweeps (FP32 basis).
// Needs a stencil operator, m < 2^29, no odd last row outside the units, and LDS for
// the slab (checked by the launcher).  Bitwise the same y and partial sums as the
// matvec kernel followed by reduce_kernel.
template <int VW, typename TQ>
__global__ __launch_bounds__(BS) void reduce_mv_kernel(const TQ* __restrict__ Q, int64_t ldq,
                                                       int J, const double* __restrict__ x,
                                                       double* __restrict__ y, int64_t m,
                                                       OpDev op, GridRed gr, FinArgs fin) {
  auto yf = [&](int64_t u, RowVec<VW>& xv, RowVec<VW>& yv) __attribute__((always_inline)) {
    double v[VW][7];
    bool in[VW][7];
#pragma unroll
    for (int e = 0; e < VW; ++e) stencil_gather<true>(op, x, (uint32_t)(u * VW + e), v[e], in[e]);
#pragma unroll
    for (int e = 0; e < VW; ++e) {
      xv.e[e] = v[e][3];
      yv.e[e] = stencil_sum(op, v[e], in[e]);
    }
    yv.store(y, u);
  };
  if constexpr (sizeof(TQ) == 8) {
    reduce_body<VW, true, TQ, 3>(Q, ldq, J, x, y, m, gr, fin, blockIdx.x, yf);
  } else {
    // FP32 basis: the matvec as a pass of its own over the slab before the sweeps
    // (measured faster than inside the first sweep, unlike an FP64 basis)
    extern __shared__ double smem[];
    if (fin.ctrl->state != ST_RUNNING) return;
    int64_t per, u0, u1;
    reduce_slab<VW>(m, gr.G, blockIdx.x, &per, &u0, &u1);
    double* sx = smem + REDUCE_SCRATCH;
    double* sy = sx + per * VW;
    for (int64_t u = u0 + threadIdx.x; u < u1; u += BS) {
      RowVec<VW> xv, yv;
      yf(u, xv, yv);
      xv.store(sx, u - u0);
      yv.store(sy, u - u0);
    }
    reduce_body<VW, true, TQ, 2>(Q, ldq, J, x, y, m, gr, fin, blockIdx.x);
  }
}

template <int VW, typename TQ>
__global__ __launch_bounds__(BS) void project_norm_kernel(const TQ* __restrict__ Q, int64_t ldq,
                                                          int J, const double* __restrict__ x,
                                                          double* __restrict__ ubuf, int64_t m,
                                                          GridRed gr, FinArgs fin) {
  project_norm_body<VW, TQ>(Q, ldq, J, x, ubuf, m, gr, fin, blockIdx.x);
}

template <int VW, bool ARN, bool QCOL, typename TQ>
__global__ __launch_bounds__(BS) void update_slab_kernel(TQ* __restrict__ Q, int64_t ldq, int J,
                                                         double* __restrict__ x,
                                                         const double* __restrict__ y,
                                                         const double* __restrict__ ubuf,
                                                         int64_t m,
                                                         const double* __restrict__ coef,
                                                         int ldc, const Ctrl* __restrict__ ctrl) {
  update_slab_body<VW, ARN, QCOL, TQ>(Q, ldq, J, x, y, ubuf, m, coef, ldc, ctrl, blockIdx.x,
                                      gridDim.x);
}

// One-pass QR step (Alg. qr): the update of step j and the reduction of step j+1
// share a single read of Q.  The next column a_{j+1} is known in advance, so the
// rows of q_{j-1} and w_j produced by the update can be dotted at once:
//   q = (w - Q C)/alpha,  w' = a_j - Q T_{1:J} - q T_J          (update, step j)
//   [Q_{0..J-1}, q, w', a_{j+1}]^T [w', a_{j+1}]                 (reduction, step j+1)
// A workgroup of FW wavefronts walks tiles of 64 rows (lane = row).  Basis column k
// belongs to wavefront k mod FW, slot k / FW; NS = ceil(J / FW) slots (at least one)
// is a template parameter, so the tile's loads of a wavefront are unconditional and
// all in flight together.  Every slot but the last of a wavefront holds a basis
// column; the last one does when wv + FW (NS - 1) < J, and otherwise reads one
// cache line and contributes zero.  The wavefronts form partial Q C and Q T from
// their slots, wavefronts 0..VR-1 combine them in a fixed order and publish q, w',
// a_{j+1} of the tile through LDS, and every lane then accumulates its rows'
// products for its slots in registers across all tiles; wavefronts 0, 1 and 2 also
// accumulate those of q, w' and a_{j+1} (one vector each).  One transposed butterfly
// per wavefront (a plain wavefront sum for the vectors) at the end yields the
// workgroup partials.
// LAST: a_{j+1} does not exist (the CGS2 finish of the last column); only
// [Q_{0..J-1}, q, w']^T w' is reduced.
constexpr int FMAXCOL = 128;             // basis columns per workgroup: FW x (FMAXCOL / FW) slots

// Workgroup barrier for LDS hand-offs only: waits for this wavefront's LDS
// traffic, not for its outstanding global loads, so the next tile's prefetch
// stays in flight across the barrier.  (The generic barrier also waits for every
// global access, which would expose the full memory latency once per tile.)
__device__ __forceinline__ void lds_barrier() {
  asm volatile("s_waitcnt lgkmcnt(0)\n\ts_barrier" ::: "memory");
}

// Calls f(std::integral_constant<int, I>) for I = 0, 1, ... in order, so that
// every index f derives from I is a compile-time constant.
template <int... I, class F>
__device__ __forceinline__ void static_for(std::integer_sequence<int, I...>, F&& f) {
  (f(std::integral_constant<int, I>{}), ...);
}

// VR consecutive basis elements as loaded (converted to double where used).
template <int VR, typename T>
struct RawVec {
  T e[VR];
};

template <int VR, typename T>
__device__ __forceinline__ RawVec<VR, T> load_raw(const T* p, uint32_t off) {
  const char* b = reinterpret_cast<const char*>(p) + off;
  RawVec<VR, T> r;
  static_assert(VR != 4 || sizeof(T) == 4, "four-row slots hold floats");
  if constexpr (VR == 4) {
    const float4 t = *reinterpret_cast<const float4*>(b);
    r.e[0] = t.x;
    r.e[1] = t.y;
    r.e[2] = t.z;
    r.e[3] = t.w;
  } else if constexpr (VR == 2 && sizeof(T) == 8) {
    const double2 t = *reinterpret_cast<const double2*>(b);
    r.e[0] = t.x;
    r.e[1] = t.y;
  } else if constexpr (VR == 2) {
    const float2 t = *reinterpret_cast<const float2*>(b);
    r.e[0] = t.x;
    r.e[1] = t.y;
  } else {
    r.e[0] = *reinterpret_cast<const T*>(b);
  }
  return r;
}

template <typename TQ, bool LAST, int FW, int NS, int VR, int PD>
__global__ __launch_bounds__(FW * 64) void fused_qr_kernel(TQ* __restrict__ Q, int64_t ldq,
                                                           int J, double* __restrict__ w,
                                                           const double* __restrict__ a_cur,
                                                           const double* __restrict__ a_next,
                                                           int64_t m,
                                                           const double* __restrict__ coef,
                                                           int ldc, GridRed gr, FinArgs fin) {
  // VR rows per lane (1; 2 with paired 16-byte loads; 4 with 16-byte float4 loads of
  // an FP32 basis; VR > 1 needs m divisible by VR and every column aligned to the load
  // width), TR = 64 VR rows per tile.
  constexpr int FS = FMAXCOL / FW;        // slot capacity per wavefront (power of two)
  constexpr int NV = LAST ? FS : 2 * FS;  // products reduced per wavefront
  constexpr int TR = 64 * VR;
  constexpr int NVEC = LAST ? 2 : 3;      // q, w' (, a_{j+1}): one per wavefront 0..NVEC-1
  static_assert(NS >= 1 && NS <= FS, "slot count");
  static_assert(PD >= 1, "prefetch depth");
  static_assert(FW >= NVEC && FW >= VR, "wavefronts");
  using RV = RowVec<VR>;
  extern __shared__ double smem[];
  const int Jt = J + (LAST ? 2 : 3);
  // LDS is laid out value-major, so that neighbouring lanes touch neighbouring
  // doubles (no bank conflicts): part[((e 2 + c) FW + wavefront) 64 + lane] holds
  // the partial (Q C for c = 0, Q T for c = 1) of row element e of the lane
  double* part = smem;                    // FW * TR * 2 partials
  double* vq = part + FW * TR * 2;        // q, w', a_{j+1} of the tile rows: [e 64 + lane]
  double* vw = vq + TR;                   // (consecutive: vector i starts at vq + i TR)
  double* va = vw + TR;
  // With more than 11 two-row slots per wavefront (not the last column) the per-slot
  // coefficients are kept in LDS as (c_k, t_k) pairs and read per tile (one broadcast
  // address per wavefront), which leaves the scalar and vector registers to the ring.
  constexpr bool CL = VR == 2 && NS > 11 && !LAST;
  double* cts = va + TR;                  // 2 FMAXCOL: (c_k, t_k), zero for k >= J
  const int lane = threadIdx.x & 63;
  const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  // the wavefront's last slot holds a basis column (uniform)
  const bool lastlive = wv + FW * (NS - 1) < J;
  // per-slot column pointers and coefficients (uniform per wavefront; the
  // coefficients are read once the first tiles' loads are in flight)
  const TQ* colp[NS];
  double alpha = 0.0, tJ = 0.0, cs[CL ? 1 : NS], ts[CL ? 1 : NS];
#pragma unroll
  for (int sl = 0; sl < NS; ++sl) {
    const int k = wv + FW * sl;
    const int kl = k < J ? k : (J > 0 ? J - 1 : 0);
    colp[sl] = Q + (int64_t)kl * ldq;
  }
  const int64_t units = m / VR;           // row units of VR rows (m % VR == 0)
  const int64_t ntiles = (units + 63) / 64;
  double ax[NS], ay[NS];
#pragma unroll
  for (int sl = 0; sl < NS; ++sl) { ax[sl] = 0.0; ay[sl] = 0.0; }
  double bx = 0.0, by = 0.0;              // vector wv's products (wavefronts < NVEC)

  // Prefetch ring: PD + 1 register stages, tile t + PD G is loaded while tile t is
  // processed.  The ring is walked by a loop unrolled PD + 1 times, so each stage
  // keeps fixed registers: no register copies between iterations, which would make
  // the compiler wait for every outstanding load (the whole prefetch) once per tile.
  struct Stage {
    RawVec<VR, TQ> q[NS];
    double x0, x1, x2;                    // element wv of the lane's rows of w, a_j and
                                          // a_{j+1} (used by wavefronts 0..VR-1)
  };
  Stage ring[PD + 1];
  auto issue = [&](int64_t t, Stage& S) __attribute__((always_inline)) {
    const int64_t ul = min(t * 64 + lane, units - 1);
    // columns hold fewer than 2^31 bytes, also in FP64 (checked by the launcher):
    // one 32-bit offset register serves every slot's column base
    const uint32_t off = (uint32_t)ul * (uint32_t)(VR * sizeof(TQ));
    // Every wavefront issues the same loads, so that all of them have the same
    // number in flight and the waits for a stage are exact.  Loads whose values are
    // not used (a last slot past the basis, the vectors outside wavefronts 0..VR-1)
    // read the first element of their array in every lane: one cache line, not a tile.
#pragma unroll
    for (int sl = 0; sl < NS; ++sl)
      S.q[sl] = load_raw<VR>(colp[sl], (sl + 1 < NS || lastlive) ? off : 0u);
    // wavefront e < VR combines row element e of the lanes' units: it loads only that
    // element of each vector (the VR wavefronts together read whole cache lines)
    const uint32_t offv =
        wv < VR ? ((uint32_t)ul * (uint32_t)VR + (uint32_t)wv) * (uint32_t)sizeof(double) : 0u;
    S.x0 = *reinterpret_cast<const double*>(reinterpret_cast<const char*>(w) + offv);
    S.x1 = *reinterpret_cast<const double*>(reinterpret_cast<const char*>(a_cur) + offv);
    if (!LAST) S.x2 = *reinterpret_cast<const double*>(reinterpret_cast<const char*>(a_next) + offv);
  };
  auto process = [&](int64_t tix, const Stage& S) __attribute__((always_inline)) {
    const int64_t u = tix * 64 + lane;
    const bool live = u < units;
    double sc[VR], st[VR];
#pragma unroll
    for (int e = 0; e < VR; ++e) { sc[e] = 0.0; st[e] = 0.0; }
#pragma unroll
    for (int sl = 0; sl < NS; ++sl) {
      double c, t;                        // zero past the basis
      if constexpr (CL) {
        c = cts[2 * (wv + FW * sl)];
        t = cts[2 * (wv + FW * sl) + 1];
      } else {
        c = cs[sl];
        t = ts[sl];
      }
#pragma unroll
      for (int e = 0; e < VR; ++e) {
        double qx = (double)S.q[sl].e[e];
        // a last slot past the basis holds whatever Q[0, .] holds: an exact zero instead
        if (sl + 1 == NS) qx = lastlive ? qx : 0.0;
        sc[e] = fma(qx, c, sc[e]);
        st[e] = fma(qx, t, st[e]);
      }
    }
#pragma unroll
    for (int e = 0; e < VR; ++e) {
      part[((e * 2) * FW + wv) * 64 + lane] = sc[e];
      part[((e * 2 + 1) * FW + wv) * 64 + lane] = st[e];
    }
    lds_barrier();
    if (wv < VR) {
      // wavefront e combines row element e of every lane's VR rows (for VR = 2 the
      // two halves of the tile at the same time), summing the wavefronts' partials
      // in wavefront order
      const int e = wv;
      const int r = e * 64 + lane;
      double SC = part[((e * 2) * FW) * 64 + lane], ST = part[((e * 2 + 1) * FW) * 64 + lane];
#pragma unroll
      for (int v = 1; v < FW; ++v) {
        SC += part[((e * 2) * FW + v) * 64 + lane];
        ST += part[((e * 2 + 1) * FW + v) * 64 + lane];
      }
      const double x0 = S.x0, x1 = S.x1, x2 = S.x2;
      double qo = 0.0, wo = 0.0, ao = 0.0;
      if (live) {
        qo = stored<TQ>((x0 - SC) / alpha);
        wo = x1 - fma(qo, tJ, ST);
        ao = x2;
        Q[(int64_t)J * ldq + u * VR + e] = (TQ)qo;
        w[u * VR + e] = wo;
      }
      vq[r] = qo;
      vw[r] = wo;
      va[r] = ao;
    }
    lds_barrier();
    RV ww, aa;
#pragma unroll
    for (int e = 0; e < VR; ++e) {
      ww.e[e] = vw[e * 64 + lane];
      aa.e[e] = LAST ? 0.0 : va[e * 64 + lane];
    }

#pragma unroll
    for (int sl = 0; sl < NS; ++sl) {
#pragma unroll
      for (int e = 0; e < VR; ++e) {
        // four-row slots: the basis element is widened to FP64 again here rather than
        // kept widened across the tile's barriers (which would hold eight more registers
        // per slot); the empty asm only hides the earlier conversion from the compiler.
        // (The products of a last slot past the basis are never stored.)
        TQ qraw = S.q[sl].e[e];
        if constexpr (VR == 4) asm volatile("" : "+v"(qraw));
        const double val = (double)qraw;
        ax[sl] = fma(val, ww.e[e], ax[sl]);
        if constexpr (!LAST) ay[sl] = fma(val, aa.e[e], ay[sl]);
      }
    }
    if (wv < NVEC) {                      // uniform
#pragma unroll
      for (int e = 0; e < VR; ++e) {
        const double val = vq[wv * TR + e * 64 + lane];
        bx = fma(val, ww.e[e], bx);
        if constexpr (!LAST) by = fma(val, aa.e[e], by);
      }
    }
    // (the next tile's part writes follow the second barrier, and its vq writes
    // its first one, so two barriers per tile suffice)
    // Keep the stage's last uses above the next issue into the same stage: were the
    // products sunk below it (towards their next use), the stage's old and new values
    // would both be live there, the loads would land in other registers, and the
    // copies back at the loop's back edge would wait for those loads (one tile in
    // flight, not two).  The empty asm needs the products here, and its memory
    // clobber keeps the next loads after it.
#pragma unroll
    for (int sl = 0; sl < NS; ++sl) {
      if constexpr (LAST) asm volatile("" : "+v"(ax[sl]) : : "memory");
      else asm volatile("" : "+v"(ax[sl]), "+v"(ay[sl]) : : "memory");
    }
  };
  // Stage s holds tile tix + s G (s < PD) at the top of every round.  A round of
  // PD + 1 tiles runs only when all of them exist, so the loop body has no exits
  // and the waits at its back edge are those of the steady state; the last (at
  // most PD) tiles, already in the ring, are processed after the loop.
  int64_t tix = blockIdx.x;
  if (tix < ntiles) {
    static_for(std::make_integer_sequence<int, PD>{}, [&](auto R) __attribute__((always_inline)) {
      constexpr int r = decltype(R)::value;
      issue(min(tix + (int64_t)r * gr.G, ntiles - 1), ring[r]);
    });
  }
  // The control block and the coefficients are read while the first tiles load
  // (their latencies overlap); a stopped expansion still exits before any store.
  if (fin.ctrl->state != ST_RUNNING) return;
  alpha = coef[2 * ldc];
  tJ = coef[ldc + J];
  if constexpr (CL) {
    for (int k = threadIdx.x; k < FW * NS; k += FW * 64) {
      const int kc = k < J ? k : 0;
      const double c = coef[kc], t = coef[ldc + kc];
      cts[2 * k] = k < J ? c : 0.0;
      cts[2 * k + 1] = k < J ? t : 0.0;
    }
    lds_barrier();
  } else {
#pragma unroll
    for (int sl = 0; sl < NS; ++sl) {     // unconditional loads (clamped index): one wait
      const int k = wv + FW * sl;
      const int kc = k < J ? k : 0;
      const double c = coef[kc], t = coef[ldc + kc];
      cs[sl] = k < J ? c : 0.0;
      ts[sl] = k < J ? t : 0.0;
    }
  }
  while (tix + (int64_t)PD * gr.G < ntiles) {
    static_for(std::make_integer_sequence<int, PD + 1>{}, [&](auto R) __attribute__((always_inline)) {
      constexpr int r = decltype(R)::value;
      // tile tix + PD G goes to the stage of the tile processed last
      issue(min(tix + (int64_t)PD * gr.G, ntiles - 1), ring[(r + PD) % (PD + 1)]);
      process(tix, ring[r]);
      tix += gr.G;
    });
  }
  static_for(std::make_integer_sequence<int, PD>{}, [&](auto R) __attribute__((always_inline)) {
    constexpr int r = decltype(R)::value;
    if (tix < ntiles) {
      process(tix, ring[r]);
      tix += gr.G;
    }
  });
  // dead rows contribute 0: q = w' = a = 0 there, and basis values only meet them
  double pv[NV];
#pragma unroll
  for (int sl = 0; sl < FS; ++sl) {
    pv[sl] = sl < NS ? ax[sl] : 0.0;
    if constexpr (!LAST) pv[FS + sl] = sl < NS ? ay[sl] : 0.0;
  }
  wave_transpose_sum(pv, lane);
  {
    const int idx = transpose_index<NV>(lane);
    const int k = wv + FW * (idx % FS);
    const int rhs = idx / FS;
    if (k < J) gr.P1[(int64_t)blockIdx.x * gr.ldp + rhs * Jt + k] = pv[0];
  }
  if (wv < NVEC) {
    const double sx = wave_sum(bx);
    const double sy = LAST ? 0.0 : wave_sum(by);
    if (lane == 0) {
      gr.P1[(int64_t)blockIdx.x * gr.ldp + J + wv] = sx;
      if (!LAST) gr.P1[(int64_t)blockIdx.x * gr.ldp + Jt + J + wv] = sy;
    }
  }
}

// q = u / alpha into Q[:, J] (rounded once to the basis type).
template <typename TQ>
__global__ void scale_col_kernel(TQ* Q, int64_t ldq, int J, const double* ubuf, int64_t m,
                                 const double* coef, int ldc, const Ctrl* ctrl) {
  if (ctrl->state != ST_RUNNING) return;
  const double alpha = coef[2 * ldc];
  const int64_t i = (int64_t)blockIdx.x * BS + threadIdx.x;
  if (i < m) Q[(int64_t)J * ldq + i] = (TQ)(ubuf[i] / alpha);
}

// ---------------------------------------------------------------------------------
// Matvec of each Arnoldi step.  Stencils: one row per thread, neighbours summed in column
// order; out-of-grid neighbours are zero (Dirichlet).
// Block index for rows with XCD-local neighbours.  Workgroup b of a launch runs on
// XCD b mod 8 (the chip's round-robin dispatch over its 8 XCDs, each with its own
// L2).  Mapping the blocks of XCD x to one contiguous range of rows (the k-th of
// them to range start + k) keeps a row's far stencil neighbours (a plane away) in
// the L2 that has just read them.  The map is a bijection of [0, gridDim.x).
__device__ __forceinline__ unsigned xcd_local_block() {
  const unsigned nb = gridDim.x, b = blockIdx.x;
  const unsigned q = nb / 8, r = nb % 8, x = b % 8, k = b / 8;
  return x * q + (x < r ? x : r) + k;
}

// Rows per thread of the stencil matvec: two, a block width apart (coalesced), so
// that fourteen loads are in flight per thread.
constexpr int STENCIL_ROWS = 2;

template <bool OFF32>
__global__ __launch_bounds__(BS) void stencil_kernel(OpDev op, const double* __restrict__ x,
                                                     const double* __restrict__ b,
                                                     double* __restrict__ y,
                                                     const Ctrl* __restrict__ ctrl) {
  const uint32_t m = (uint32_t)op.m;
  const uint32_t base = xcd_local_block() * (BS * STENCIL_ROWS) + threadIdx.x;
  double v[STENCIL_ROWS][7];
  bool in[STENCIL_ROWS][7];
  // all loads first: an absent neighbour (or a row past m) reads a valid row
#pragma unroll
  for (int h = 0; h < STENCIL_ROWS; ++h) {
    const uint32_t i0 = base + h * BS;
    stencil_gather<OFF32>(op, x, i0 < m ? i0 : m - 1, v[h], in[h]);
  }
  // the control block is read while the loads are in flight; a stopped expansion
  // still exits before any store
  if (ctrl && ctrl->state != ST_RUNNING) return;
#pragma unroll
  for (int h = 0; h < STENCIL_ROWS; ++h) {
    const uint32_t i = base + h * BS;
    if (i >= m) continue;
    const double s = stencil_sum(op, v[h], in[h]);
    y[i] = b ? b[i] - s : s;
  }
}

__global__ __launch_bounds__(BS) void csr_kernel(OpDev op, const double* __restrict__ x,
                                                 const double* __restrict__ b,
                                                 double* __restrict__ y,
                                                 const Ctrl* __restrict__ ctrl) {
  if (ctrl && ctrl->state != ST_RUNNING) return;
  const int64_t i = (int64_t)blockIdx.x * BS + threadIdx.x;
  if (i >= op.m) return;
  double s = 0.0;
  for (int32_t p = op.rowptr[i]; p < op.rowptr[i + 1]; ++p) s += op.val[p] * x[op.colind[p]];
  y[i] = b ? b[i] - s : s;
}

// Out[:, k0+o] = (acc ? Out : 0) + sum_c Q[:, c] Z[c, k0+o]   for o < NO (one row per thread)
template <int NO, typename TQ, typename TO>
__global__ __launch_bounds__(BS) void tsgemm_kernel(const TQ* __restrict__ Q, int64_t ldq,
                                                    int p, const double* __restrict__ Z, int ldz,
                                                    int k, TO* __restrict__ Out, int64_t ldo,
                                                    int64_t m, int accum) {
  const int64_t i = (int64_t)blockIdx.x * BS + threadIdx.x;
  const int k0 = blockIdx.y * NO;
  if (i >= m) return;
  double acc[NO];
  const double* zc[NO];                   // output columns past k repeat column k-1 (not stored)
#pragma unroll
  for (int o = 0; o < NO; ++o) {
    acc[o] = 0.0;
    zc[o] = Z + (int64_t)(k0 + o < k ? k0 + o : k - 1) * ldz;
  }
#pragma unroll 8
  for (int c = 0; c < p; ++c) {
    const double q = (double)Q[(int64_t)c * ldq + i];
#pragma unroll
    for (int o = 0; o < NO; ++o) acc[o] = fma(q, zc[o][c], acc[o]);
  }
#pragma unroll
  for (int o = 0; o < NO; ++o) {
    if (k0 + o < k) {
      TO* out = Out + (int64_t)(k0 + o) * ldo + i;
      *out = (TO)(accum ? (double)*out + acc[o] : acc[o]);
    }
  }
}

__global__ void init_ctrl_kernel(Ctrl* c, double tau, double eta, double thresh, double rho) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    c->state = ST_RUNNING;
    c->stop_step = -1;
    c->k = 0;
    c->reductions = 0;
    c->fallbacks = 0;
    c->pad0 = 0;
    c->rho_next = rho;
    c->tau = tau;
    c->eta = eta;
    c->gmres_thresh = thresh;
    c->resid_est = 0.0;
    c->norm2 = 0.0;
  }
}

__global__ void set_state_kernel(Ctrl* c, int state) {
  if (threadIdx.x == 0 && blockIdx.x == 0) c->state = state;
}

__global__ void fill_kernel(double* p, int64_t n, double val) {
  const int64_t i = (int64_t)blockIdx.x * BS + threadIdx.x;
  if (i < n) p[i] = val;
}

template <typename TD, typename TS>
__global__ void convert_col_kernel(TD* dst, const TS* src, int64_t m) {
  const int64_t i = (int64_t)blockIdx.x * BS + threadIdx.x;
  if (i < m) dst[i] = (TD)src[i];
}

__global__ void copy_cols_kernel(double* dst, int64_t ldd, const double* src, int64_t lds,
                                 int64_t m) {
  const int64_t i = (int64_t)blockIdx.x * BS + threadIdx.x;
  const int c = blockIdx.y;
  if (i < m) dst[(int64_t)c * ldd + i] = src[(int64_t)c * lds + i];
}

inline unsigned nblocks(int64_t n) { return (unsigned)((n + BS - 1) / BS); }

template <typename P>
inline bool aligned16(P p) { return (reinterpret_cast<uintptr_t>(p) & 15u) == 0; }
inline bool aligned_to(const void* p, unsigned a) {
  return (reinterpret_cast<uintptr_t>(p) & (uintptr_t)(a - 1)) == 0;
}

size_t reduce_smem() { return sizeof(double) * (size_t)REDUCE_SCRATCH; }

// LDS a reduction workgroup may use with its staged slab: the device's limit per
// workgroup (queried once; 160 KiB on gfx950).
size_t reduce_lds_cap() {
  static size_t cap = 0;
  if (cap == 0) {
    int dev = 0, v = 0;
    size_t c = 64 * 1024;
    if (hipGetDevice(&dev) == hipSuccess &&
        hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) == hipSuccess &&
        v > 0)
      c = (size_t)v;
    cap = c;
  }
  return cap;
}

}  // namespace

// ---------------------------------------------------------------------------------
void reduce_grid(int64_t m, int gmax, int q32, int* G) {
  // one two-row unit per thread and sweep until the cap: short slabs keep the
  // latency chain of a sweep short when m is small
  const int64_t units = (m + 1) / 2;
  int64_t g = (units + (int64_t)BS - 1) / (int64_t)BS;
  if (g < 1) g = 1;
  // default: at most one workgroup per CU with an FP64 basis, two with an FP32 basis
  // (half the bytes per load, so twice the wavefronts keep as many bytes in flight);
  // measured best for the 16-column sweeps at m = 2^21 (the tuning knob overrides it)
  const int cap = gmax > 0 ? gmax : device_cus() * (q32 ? 2 : 1);
  if (g > cap) g = cap;
  if (g > REDUCE_GMAX) g = REDUCE_GMAX;
  *G = (int)g;
}

hipError_t noalloc_scratch(int device, double** out, size_t* doubles) {
  constexpr int MAXDEV = 64;
  static std::mutex mu;
  static double* addr[MAXDEV] = {};
  if (device < 0 || device >= MAXDEV) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(mu);
  if (!addr[device]) {
    int cur = -1;
    hipError_t e = hipGetDevice(&cur);
    if (e != hipSuccess) return e;
    if (cur != device) return hipErrorInvalidDevice;   // the caller makes it current
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    if (!p) return hipErrorInvalidSymbol;
    addr[device] = static_cast<double*>(p);
  }
  *out = addr[device];
  *doubles = NOALLOC_DOUBLES;
  return hipSuccess;
}

hipError_t launch_init_ctrl(Ctrl* ctrl, double tau, double eta, double thresh, hipStream_t s,
                            double rho) {
  init_ctrl_kernel<<<1, 64, 0, s>>>(ctrl, tau, eta, thresh, rho);
  return hipGetLastError();
}

hipError_t launch_set_state(Ctrl* ctrl, int state, hipStream_t s) {
  set_state_kernel<<<1, 64, 0, s>>>(ctrl, state);
  return hipGetLastError();
}

hipError_t launch_fill(double* p, int64_t n, double val, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  fill_kernel<<<nblocks(n), BS, 0, s>>>(p, n, val);
  return hipGetLastError();
}

hipError_t launch_copy(double* dst, const double* src, int64_t n, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  copy_cols_kernel<<<dim3(nblocks(n), 1), BS, 0, s>>>(dst, n, src, n, n);
  return hipGetLastError();
}

hipError_t launch_copy_cols(double* dst, int64_t ldd, const double* src, int64_t lds, int64_t m,
                            int ncols, hipStream_t s) {
  if (m <= 0 || ncols <= 0) return hipSuccess;
  copy_cols_kernel<<<dim3(nblocks(m), ncols), BS, 0, s>>>(dst, ldd, src, lds, m);
  return hipGetLastError();
}

hipError_t launch_spmv(const OpDev& op, const double* x, const double* b, double* y,
                       const Ctrl* ctrl, hipStream_t s) {
  if (op.kind == DCGS2_OP_CSR)
    csr_kernel<<<nblocks(op.m), BS, 0, s>>>(op, x, b, y, ctrl);
  else {
    // row indices are 32-bit (m < 2^31, also past the last row of the grid), and the
    // division constants must be set (mul >= 1 for every divisor)
    const int64_t rows = BS * STENCIL_ROWS;
    const int64_t nb = (op.m + rows - 1) / rows;
    if (op.m < 1 || nb * rows >= ((int64_t)1 << 32) || op.dx.mul == 0 || op.dy.mul == 0)
      return hipErrorInvalidValue;
    if (op.m < ((int64_t)1 << 29))
      stencil_kernel<true><<<(unsigned)nb, BS, 0, s>>>(op, x, b, y, ctrl);
    else
      stencil_kernel<false><<<(unsigned)nb, BS, 0, s>>>(op, x, b, y, ctrl);
  }
  return hipGetLastError();
}

namespace {
__global__ __launch_bounds__(FINISH_BS) void finish_kernel(GridRed gr, int V, int J,
                                                           FinArgs fin) {
  finish_body(gr, V, fin, J);
}

// Enqueues the finishing kernel of a reduction over J basis columns with V values
// per workgroup; records `mid` (when given) between the streaming kernel and it.
hipError_t launch_finish(const GridRed& gr, int V, int J, const FinArgs& fin, hipEvent_t mid,
                         hipStream_t s) {
  hipError_t e = hipGetLastError();      // the streaming kernel's launch status
  if (e != hipSuccess) return e;
  if (mid && (e = hipEventRecord(mid, s)) != hipSuccess) return e;
  const int Jf = J > fin.J ? J : fin.J;
  // long bases need more than the default dynamic LDS limit (about 90 KB at
  // J = DCGS2_MAX_N); a refusal is cleared here and shows as that launch's error
  static std::once_flag once;
  std::call_once(once, [] {
    const int most = (int)finish_smem(2 * (DCGS2_MAX_N + 3), DCGS2_MAX_N + 1);
    if (hipFuncSetAttribute(reinterpret_cast<const void*>(&finish_kernel),
                            hipFuncAttributeMaxDynamicSharedMemorySize, most) != hipSuccess)
      (void)hipGetLastError();
  });
  finish_kernel<<<1, FINISH_BS, finish_smem(V, Jf), s>>>(gr, V, Jf, fin);
  return hipGetLastError();
}
}  // namespace

namespace {
// Vector width of a reduction pass over these operands (2: 16-byte row units).
int reduce_vw(const void* Q, int q32, int64_t ldq, const double* x, const double* y) {
  return aligned_to(Q, q32 ? 8 : 16) && (ldq % 2 == 0) && aligned16(x) && (!y || aligned16(y))
             ? 2 : 1;
}

size_t reduce_mv_smem(int vw, int64_t m, int G) {
  const int64_t per = (m / vw + G - 1) / G;
  return reduce_smem() + sizeof(double) * (size_t)per * vw * 2;
}

template <int VW, typename T>
void allow_mv_lds() {
  static std::once_flag once;
  std::call_once(once, [] {
    if (hipFuncSetAttribute(reinterpret_cast<const void*>(&reduce_mv_kernel<VW, T>),
                            hipFuncAttributeMaxDynamicSharedMemorySize, (int)reduce_lds_cap()) !=
        hipSuccess)
      (void)hipGetLastError();            // shows as the launch's error instead
  });
}
}  // namespace

// A staged reduction may take more dynamic LDS than the default launch limit: raise the
// limit of each staged instantiation to the cap once.
template <int VW, bool HY, typename T>
void allow_staged_lds() {
  static std::once_flag once;
  std::call_once(once, [] {
    if (hipFuncSetAttribute(reinterpret_cast<const void*>(&reduce_kernel<VW, HY, T, true>),
                            hipFuncAttributeMaxDynamicSharedMemorySize, (int)reduce_lds_cap()) !=
        hipSuccess)
      (void)hipGetLastError();            // shows as the launch's error instead
  });
}

hipError_t launch_reduce(const void* Q, int q32, int64_t ldq, int J, const double* x,
                         const double* y, int64_t m, const GridRed& gr, const FinArgs& fin,
                         hipStream_t s, hipEvent_t mid) {
  const bool vec = reduce_vw(Q, q32, ldq, x, y) == 2;
  // stage the workgroup's slab of x (and y) in LDS when it fits: every sweep over a
  // column group (and the final x^T x, x^T y, y^T y) then reads them there
  const int64_t units = vec ? m / 2 : m;
  const int64_t per = (units + gr.G - 1) / gr.G;
  const size_t stage = sizeof(double) * (size_t)per * (vec ? 2 : 1) * (y ? 2 : 1);
  const bool staged = J >= 1 && reduce_smem() + stage <= reduce_lds_cap();
  const size_t sm = reduce_smem() + (staged ? stage : 0);
  const dim3 grid(gr.G), block(BS);
#define DCGS2_RED(VW, HY, T)                                                                  \
  do {                                                                                        \
    if (staged) {                                                                             \
      allow_staged_lds<VW, HY, T>();                                                          \
      reduce_kernel<VW, HY, T, true><<<grid, block, sm, s>>>((const T*)Q, ldq, J, x, y, m, gr, \
                                                             fin);                            \
    } else                                                                                    \
      reduce_kernel<VW, HY, T, false><<<grid, block, sm, s>>>((const T*)Q, ldq, J, x, y, m,    \
                                                              gr, fin);                       \
  } while (0)
  if (q32) {
    if (y) { if (vec) DCGS2_RED(2, true, float); else DCGS2_RED(1, true, float); }
    else { if (vec) DCGS2_RED(2, false, float); else DCGS2_RED(1, false, float); }
  } else {
    if (y) { if (vec) DCGS2_RED(2, true, double); else DCGS2_RED(1, true, double); }
    else { if (vec) DCGS2_RED(2, false, double); else DCGS2_RED(1, false, double); }
  }
#undef DCGS2_RED
  const int Jt = J + (y ? 2 : 1);
  return launch_finish(gr, y ? 2 * Jt : Jt, J, fin, mid, s);
}


bool reduce_mv_fits(const void* Q, int q32, int64_t ldq, const double* x, const double* y,
                    int64_t m, const OpDev& op, const GridRed& gr) {
  if (op.kind == DCGS2_OP_CSR || op.m != m || m < 1 || m >= ((int64_t)1 << 29) ||
      op.dx.mul == 0 || op.dy.mul == 0 || gr.G < 1)
    return false;
  const int vw = reduce_vw(Q, q32, ldq, x, y);
  if (vw == 2 && (m & 1)) return false;       // no odd last row outside the units
  return reduce_mv_smem(vw, m, gr.G) <= reduce_lds_cap();
}

hipError_t launch_reduce_mv(const void* Q, int q32, int64_t ldq, int J, const double* x,
                            double* y, int64_t m, const OpDev& op, const GridRed& gr,
                            const FinArgs& fin, hipStream_t s, hipEvent_t mid) {
  if (!reduce_mv_fits(Q, q32, ldq, x, y, m, op, gr)) return hipErrorInvalidValue;
  const int vw = reduce_vw(Q, q32, ldq, x, y);
  const size_t sm = reduce_mv_smem(vw, m, gr.G);
#define DCGS2_RMV(VW, T)                                                                     \
  do {                                                                                       \
    allow_mv_lds<VW, T>();                                                                   \
    reduce_mv_kernel<VW, T><<<gr.G, BS, sm, s>>>((const T*)Q, ldq, J, x, y, m, op, gr, fin); \
  } while (0)
  if (q32) { if (vw == 2) DCGS2_RMV(2, float); else DCGS2_RMV(1, float); }
  else { if (vw == 2) DCGS2_RMV(2, double); else DCGS2_RMV(1, double); }
#undef DCGS2_RMV
  const int Jt = J + 2;
  return launch_finish(gr, 2 * Jt, J, fin, mid, s);
}

hipError_t launch_project_norm(const void* Q, int q32, int64_t ldq, int J, const double* x,
                               double* ubuf, int64_t m, const GridRed& gr, const FinArgs& fin,
                               hipStream_t s, hipEvent_t mid) {
  const bool vec = aligned_to(Q, q32 ? 8 : 16) && (ldq % 2 == 0) && aligned16(x) &&
                   aligned16(ubuf);
  const size_t sm = sizeof(double) * (size_t)NW;
#define DCGS2_PN(VW, T) \
  project_norm_kernel<VW, T><<<gr.G, BS, sm, s>>>((const T*)Q, ldq, J, x, ubuf, m, gr, fin)
  if (q32) { if (vec) DCGS2_PN(2, float); else DCGS2_PN(1, float); }
  else { if (vec) DCGS2_PN(2, double); else DCGS2_PN(1, double); }
#undef DCGS2_PN
  return launch_finish(gr, 1, J, fin, mid, s);
}

hipError_t launch_update(void* Q, int q32, int64_t ldq, int J, double* x, const double* y,
                         const double* ubuf, int64_t m, const double* coef, int ldc, int arnoldi,
                         int qcol, const Ctrl* ctrl, hipStream_t s, int slabs) {
  const bool vec = aligned_to(Q, q32 ? 8 : 16) && (ldq % 2 == 0) && aligned16(x) &&
                   aligned16(y) && (!ubuf || aligned16(ubuf));
  const int64_t units = vec ? m / 2 : m;
  // automatic: one slab per CU with an FP64 basis, two with an FP32 basis (half the
  // bytes per load: more wavefronts keep as many bytes in flight); measured best at
  // m = 2^21 among 256, 384, 512, 768, 1024, 2048 slabs and one row unit per thread
  if (slabs == 0) slabs = device_cus() * (q32 ? 2 : 1);
  const unsigned nb =
      (unsigned)std::max<int64_t>(1, std::min<int64_t>(slabs, (units + BS - 1) / BS));
#define DCGS2_UPD(VW, A, QC, T)                                                              \
  update_slab_kernel<VW, A, QC, T><<<nb, BS, 0, s>>>((T*)Q, ldq, J, x, y, ubuf, m, coef, ldc, \
                                                     ctrl)
#define DCGS2_UPD_T(VW, T)                                                   \
  do {                                                                       \
    if (arnoldi) { if (qcol) DCGS2_UPD(VW, true, true, T); else DCGS2_UPD(VW, true, false, T); } \
    else { if (qcol) DCGS2_UPD(VW, false, true, T); else DCGS2_UPD(VW, false, false, T); }       \
  } while (0)
  if (q32) { if (vec) DCGS2_UPD_T(2, float); else DCGS2_UPD_T(1, float); }
  else { if (vec) DCGS2_UPD_T(2, double); else DCGS2_UPD_T(1, double); }
#undef DCGS2_UPD_T
#undef DCGS2_UPD
  return hipGetLastError();
}

size_t fused_qr_smem(int fw, int vr) {
  return sizeof(double) * ((size_t)fw * 128 * vr + 3 * 64 * vr + 2 * FMAXCOL);
}

// Multiprocessors of the current device (cached).
int device_cus() {
  static int ncu = 0;
  if (ncu == 0) {
    int dev = 0, v = 0;
    if (hipGetDevice(&dev) == hipSuccess &&
        hipDeviceGetAttribute(&v, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess &&
        v > 0)
      ncu = v;
    else
      return 256;
  }
  return ncu;
}

namespace {
// Prefetch depth of the one-pass kernel: the deepest ring (PD <= 4) whose PD + 1
// register stages of NS slots fit, with the accumulators, in the registers of a
// wavefront (256 with 8 wavefronts per workgroup, 128 with 16) without spilling.
// The limits are the largest NS per depth found free of scratch use by compiling
// every instantiation for gfx950 (pd1: the largest NS that fits at all), except for
// the two-row FP64 and four-row FP32 slots of a non-last column: these use the
// shallower rings measured fastest (the deepest ones that fit, up to PD 4 at seven
// slots, were slower; shallower still was no faster).
struct RingLimits {
  int pd4, pd3, pd2, pd1;
};
template <typename T, bool L, int F, int VR>
constexpr RingLimits ring_limits() {
  if constexpr (F == 16) return RingLimits{0, 0, 0, 8};
  if constexpr (VR == 4) return L ? RingLimits{3, 5, 8, 16} : RingLimits{2, 4, 6, 16};
  if constexpr (sizeof(T) == 8 && VR == 2) return L ? RingLimits{4, 6, 8, 16} : RingLimits{2, 3, 5, 16};
  if constexpr (sizeof(T) == 8) return L ? RingLimits{15, 16, 16, 16} : RingLimits{12, 15, 16, 16};
  if constexpr (VR == 2) return L ? RingLimits{13, 16, 16, 16} : RingLimits{10, 12, 14, 16};
  return RingLimits{16, 16, 16, 16};
}
template <typename T, bool L, int F, int VR, int NS>
constexpr int ring_depth() {
  constexpr RingLimits r = ring_limits<T, L, F, VR>();
  return NS <= r.pd4 ? 4 : NS <= r.pd3 ? 3 : NS <= r.pd2 ? 2 : 1;
}

// Dispatch on the slot count NS = max(1, ceil(J / FW)) (compile-time in the kernel).
// One workgroup per CU: measured faster at m = 2e6 than filling each CU to the
// occupancy of the instantiation (several workgroups per CU for short bases).
template <typename T, bool L, int F, int VR, int NS>
hipError_t fused_qr_ns(int ns, T* Q, int64_t ldq, int J, double* w, const double* a_cur,
                       const double* a_next, int64_t m, const double* coef, int ldc, size_t sm,
                       GridRed gr, int gmax, const FinArgs& fin, hipStream_t s, hipEvent_t mid) {
  if constexpr (NS > FMAXCOL / F || NS > ring_limits<T, L, F, VR>().pd1) {
    return hipErrorInvalidValue;          // not dispatched (the launcher checks the fit)
  } else {
    if (ns == NS) {
      const int64_t ntiles = (m / VR + 63) / 64;
      int64_t g = device_cus();
      if (gmax > 0 && g > gmax) g = gmax;
      if (g > REDUCE_GMAX) g = REDUCE_GMAX;
      if (g > ntiles) g = ntiles;
      gr.G = (int)(g < 1 ? 1 : g);
      constexpr int PD = ring_depth<T, L, F, VR, NS>();
      fused_qr_kernel<T, L, F, NS, VR, PD><<<gr.G, F * 64, sm, s>>>(Q, ldq, J, w, a_cur, a_next,
                                                                    m, coef, ldc, gr, fin);
      const int Jt = J + (L ? 2 : 3);
      return launch_finish(gr, L ? Jt : 2 * Jt, J, fin, mid, s);
    }
    return fused_qr_ns<T, L, F, VR, NS + 1>(ns, Q, ldq, J, w, a_cur, a_next, m, coef, ldc, sm, gr,
                                            gmax, fin, s, mid);
  }
}
}  // namespace

hipError_t launch_fused_qr(void* Q, int q32, int64_t ldq, int J, double* w, const double* a_cur,
                           const double* a_next, int64_t m, const double* coef, int ldc, int last,
                           int fw, int gmax, int pair_max_ns, const GridRed& gr,
                           const FinArgs& fin, hipStream_t s, hipEvent_t mid) {
  // 16-wavefront workgroups (one-row slots, 128 registers) when the slots fit
  const int F = (fw == 16 && (J + 15) / 16 <= ring_limits<double, false, 16, 1>().pd1) ? 16 : 8;
  const int ns = J > 0 ? (J + F - 1) / F : 1;
  if (ns < 1 || ns > FMAXCOL / F) return hipErrorInvalidValue;
  if ((double)m * 8.0 >= 2147483648.0) return hipErrorInvalidValue;  // 32-bit offsets
  // paired rows: m even, every column start 16-byte aligned (8 for an FP32 basis);
  // 8-wavefront workgroups only, and only up to the slot count whose two register
  // stages of two-row slots fit without spilling
  const int pair_fit = q32 ? (last ? ring_limits<float, true, 8, 2>().pd1
                                   : ring_limits<float, false, 8, 2>().pd1)
                           : (last ? ring_limits<double, true, 8, 2>().pd1
                                   : ring_limits<double, false, 8, 2>().pd1);
  const bool rows2 = (m % 2 == 0) && aligned_to(Q, q32 ? 8 : 16) && (ldq % 2 == 0) &&
                     aligned16(w) && aligned16(a_cur) && (last || aligned16(a_next));
  const bool pair = F == 8 && ns <= pair_max_ns && ns <= pair_fit && rows2;
  // FP32 basis: four rows per lane (one 16-byte load per column) when m and ldq are
  // multiples of four, up to the slot count whose two register stages fit
  const int quad_fit = last ? ring_limits<float, true, 8, 4>().pd1
                            : ring_limits<float, false, 8, 4>().pd1;
  const bool quad = q32 && pair && ns <= quad_fit && (m % 4 == 0) && (ldq % 4 == 0) &&
                    aligned16(Q);
  const size_t sm = fused_qr_smem(F, quad ? 4 : pair ? 2 : 1);
#define DCGS2_FQ(T, L, FF, VR)                                                                 \
  return fused_qr_ns<T, L, FF, VR, 1>(ns, (T*)Q, ldq, J, w, a_cur, a_next, m, coef, ldc, sm, gr, \
                                      gmax, fin, s, mid)
#define DCGS2_FQ_V(FF, VR)                                                                    \
  do {                                                                                        \
    if (q32) { if (last) DCGS2_FQ(float, true, FF, VR); DCGS2_FQ(float, false, FF, VR); }     \
    if (last) DCGS2_FQ(double, true, FF, VR);                                                 \
    DCGS2_FQ(double, false, FF, VR);                                                          \
  } while (0)
  if (F == 8) {
    if (quad) {
      if (last) DCGS2_FQ(float, true, 8, 4);
      DCGS2_FQ(float, false, 8, 4);
    }
    if (pair) DCGS2_FQ_V(8, 2);
    DCGS2_FQ_V(8, 1);
  }
  DCGS2_FQ_V(16, 1);
#undef DCGS2_FQ_V
#undef DCGS2_FQ
}

hipError_t launch_scale_col(void* Q, int q32, int64_t ldq, int J, const double* ubuf, int64_t m,
                            const double* coef, int ldc, const Ctrl* ctrl, hipStream_t s) {
  if (q32)
    scale_col_kernel<float><<<nblocks(m), BS, 0, s>>>((float*)Q, ldq, J, ubuf, m, coef, ldc, ctrl);
  else
    scale_col_kernel<double><<<nblocks(m), BS, 0, s>>>((double*)Q, ldq, J, ubuf, m, coef, ldc,
                                                       ctrl);
  return hipGetLastError();
}

hipError_t launch_tsgemm(const void* Q, int q32, int64_t ldq, int p, const double* Z, int ldz,
                         int k, void* Out, int o32, int64_t ldo, int64_t m, int acc,
                         hipStream_t s) {
  if (m <= 0 || k <= 0) return hipSuccess;
  constexpr int NO = 8;
  const dim3 grid(nblocks(m), (unsigned)((k + NO - 1) / NO));
#define DCGS2_TS(TQ, TO) \
  tsgemm_kernel<NO, TQ, TO><<<grid, BS, 0, s>>>((const TQ*)Q, ldq, p, Z, ldz, k, (TO*)Out, ldo, m, acc)
  if (q32) { if (o32) DCGS2_TS(float, float); else DCGS2_TS(float, double); }
  else { if (o32) DCGS2_TS(double, float); else DCGS2_TS(double, double); }
#undef DCGS2_TS
  return hipGetLastError();
}

hipError_t launch_convert(void* dst, int d32, const void* src, int s32, int64_t m,
                          hipStream_t s) {
  if (m <= 0) return hipSuccess;
  if (d32 && s32) convert_col_kernel<float, float><<<nblocks(m), BS, 0, s>>>((float*)dst, (const float*)src, m);
  else if (d32) convert_col_kernel<float, double><<<nblocks(m), BS, 0, s>>>((float*)dst, (const double*)src, m);
  else if (s32) convert_col_kernel<double, float><<<nblocks(m), BS, 0, s>>>((double*)dst, (const float*)src, m);
  else convert_col_kernel<double, double><<<nblocks(m), BS, 0, s>>>((double*)dst, (const double*)src, m);
  return hipGetLastError();
}

}  // namespace dcgs2
