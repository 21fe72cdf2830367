// Device code shared by the single-instance kernels (kernels.hip) and the
// batched kernels (batched.hip): row vectors, wavefront and workgroup reductions,
// the fixed-order sum of the per-workgroup partials and the scalar finaliser of a
// DCGS2 step.  Included inside namespace dcgs2 { namespace { ... } } of each file.
#pragma once

constexpr int BS = 256;          // threads per workgroup (4 wavefronts of 64)
constexpr int NW = BS / 64;
constexpr int NT = 16;           // basis columns per reduction tile

// ---------------------------------------------------------------------------------
// Row vectors: a "unit" is VW consecutive rows; VW = 2 uses 16-byte loads and
// requires every column start to be 16-byte aligned (checked by the host).
template <int VW>
struct RowVec {
  double e[VW];
  // Loads VW consecutive elements (unit u) of a double or float array, widened
  // to double; stores round to the array's element type.
  template <typename T>
  __device__ static RowVec load(const T* p, int64_t u) {
    RowVec r;
    if constexpr (VW == 2 && sizeof(T) == 8) {
      const double2 t = reinterpret_cast<const double2*>(p)[u];
      r.e[0] = t.x;
      r.e[1] = t.y;
    } else if constexpr (VW == 2) {
      const float2 t = reinterpret_cast<const float2*>(p)[u];
      r.e[0] = (double)t.x;
      r.e[1] = (double)t.y;
    } else {
      r.e[0] = (double)p[u];
    }
    return r;
  }
  // Same as load(p, u) with the byte offset of unit u given as a 32-bit value, so
  // that the address is a uniform base plus a 32-bit lane offset (one offset
  // register can serve many columns).
  template <typename T>
  __device__ static RowVec load_off32(const T* p, uint32_t off) {
    const char* b = reinterpret_cast<const char*>(p) + off;
    RowVec r;
    if constexpr (VW == 2 && sizeof(T) == 8) {
      const double2 t = *reinterpret_cast<const double2*>(b);
      r.e[0] = t.x;
      r.e[1] = t.y;
    } else if constexpr (VW == 2) {
      const float2 t = *reinterpret_cast<const float2*>(b);
      r.e[0] = (double)t.x;
      r.e[1] = (double)t.y;
    } else {
      r.e[0] = (double)*reinterpret_cast<const T*>(b);
    }
    return r;
  }
  template <typename T>
  __device__ void store(T* p, int64_t u) const {
    if constexpr (VW == 2 && sizeof(T) == 8) {
      reinterpret_cast<double2*>(p)[u] = make_double2(e[0], e[1]);
    } else if constexpr (VW == 2) {
      reinterpret_cast<float2*>(p)[u] = make_float2((float)e[0], (float)e[1]);
    } else {
      p[u] = (T)e[0];
    }
  }
  __device__ static RowVec zero() {
    RowVec r;
#pragma unroll
    for (int i = 0; i < VW; ++i) r.e[i] = 0.0;
    return r;
  }
  __device__ double dot(const RowVec& o) const {
    double s = e[0] * o.e[0];
#pragma unroll
    for (int i = 1; i < VW; ++i) s = fma(e[i], o.e[i], s);
    return s;
  }
};

// Value of x as stored in an array of T (rounded once when T is float).
template <typename T>
__device__ __forceinline__ double stored(double x) { return (double)(T)x; }

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// Transposed butterfly: reduce NV (a power of two <= 32) per-lane values over the
// 64 lanes of a wavefront with NV + log2(64/NV) - 1 exchanges instead of
// 6 NV.  At each of the first log2(NV) steps a lane keeps half of its values
// (the half selected by its lane bit), swaps the other half with the partner lane
// and adds; the remaining steps are plain butterflies.  Afterwards v[0] of lane l
// holds the wavefront total of value index transpose_index<NV>(l).  The order of
// additions is fixed, so the result is deterministic.
template <int CNT, int OFF>
struct TransposeStep {
  template <int NV>
  __device__ static void run(double (&v)[NV], int lane) {
    if constexpr (OFF >= 1) {
      if constexpr (CNT > 1) {
        constexpr int H = CNT / 2;
        const bool up = (lane & OFF) != 0;
#pragma unroll
        for (int i = 0; i < H; ++i) {
          const double keep = up ? v[H + i] : v[i];
          const double give = up ? v[i] : v[H + i];
          v[i] = keep + __shfl_xor(give, OFF, 64);
        }
        TransposeStep<H, OFF / 2>::run(v, lane);
      } else {
        v[0] += __shfl_xor(v[0], OFF, 64);
        TransposeStep<1, OFF / 2>::run(v, lane);
      }
    }
  }
};

template <int NV>
__device__ __forceinline__ int transpose_index(int lane) {
  int idx = 0, cnt = NV;
#pragma unroll
  for (int off = 32; off >= 1 && cnt > 1; off >>= 1) {
    cnt >>= 1;
    if (lane & off) idx += cnt;
  }
  return idx;
}

template <int NV>
__device__ __forceinline__ void wave_transpose_sum(double (&v)[NV], int lane) {
  TransposeStep<NV, 32>::run(v, lane);
}

// Deterministic workgroup sum of NV (power of two <= 32) per-thread values by the
// transposed butterfly; value c lands in out_lo[c] for c < NLO, else out_hi[c - NLO],
// for c < nvalid_lo / nvalid_hi.  sh: NW*NV doubles of LDS.
template <int NV, int NLO>
__device__ void block_sum_t(double (&acc)[NV], double* sh, double* out_lo, int nvalid_lo,
                            double* out_hi, int nvalid_hi) {
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  wave_transpose_sum(acc, lane);
  sh[wid * NV + transpose_index<NV>(lane)] = acc[0];   // lanes sharing an index agree
  __syncthreads();
  const int c = threadIdx.x;
  if (c < NV) {
    double s = sh[c];
#pragma unroll
    for (int w = 1; w < NW; ++w) s += sh[w * NV + c];
    if (c < NLO) { if (c < nvalid_lo) out_lo[c] = s; }
    else if (c - NLO < nvalid_hi) out_hi[c - NLO] = s;
  }
  __syncthreads();
}

// Deterministic workgroup sum of NV per-thread values; results land in out[0..NV)
// (global or shared), written by threads 0..NV-1.  sh: NW*NV doubles of LDS.
template <int NV>
__device__ void block_sum(const double (&acc)[NV], double* sh, double* out, int nvalid) {
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
#pragma unroll
  for (int c = 0; c < NV; ++c) {
    const double v = wave_sum(acc[c]);
    if (lane == 0) sh[wid * NV + c] = v;
  }
  __syncthreads();
  if (threadIdx.x < NV && (int)threadIdx.x < nvalid) {
    double s = sh[threadIdx.x];
#pragma unroll
    for (int w = 1; w < NW; ++w) s += sh[w * NV + threadIdx.x];
    out[threadIdx.x] = s;
  }
  __syncthreads();
}

// red[v] = sum over g < G of P[g ldp + v] for v < V, by the whole workgroup, in a
// fixed order: the G partials of each value are split into C chunks of consecutive
// workgroups (C depends on V and the block size only), each chunk is summed in
// workgroup order by one thread with 16 loads in flight, then the chunk sums are
// added in chunk order.  sp: LDS scratch of max(V, blockDim.x) doubles.
__device__ void partial_sum(const double* __restrict__ P, int64_t ldp, int G, int V,
                            double* red, double* sp) {
  const int nt = (int)blockDim.x;
  int C = V >= nt ? 1 : nt / V;
  if (C > 32) C = 32;
  if (C > G) C = G;
  const int L = (G + C - 1) / C;
  for (int t = threadIdx.x; t < V * C; t += nt) {
    const int v = t % V, c = t / V;     // neighbouring threads read neighbouring values
    const int lo = c * L, hi = min(G, lo + L);
    double s = 0.0;
    for (int g0 = lo; g0 < hi; g0 += 16) {
      double x[16];
#pragma unroll
      for (int i = 0; i < 16; ++i) x[i] = P[(int64_t)min(g0 + i, hi - 1) * ldp + v];
#pragma unroll
      for (int i = 0; i < 16; ++i) s += (g0 + i < hi) ? x[i] : 0.0;
    }
    sp[t] = s;                          // t = c V + v
  }
  __syncthreads();
  for (int v = threadIdx.x; v < V; v += nt) {
    double s = 0.0;
    for (int c = 0; c < C; ++c) s += sp[c * V + v];
    red[v] = s;
  }
  __syncthreads();
}

__device__ __forceinline__ bool finite(double v) { return isfinite(v); }

// Control-block fields that a finishing kernel reads before it writes any, loaded at
// its start so that their latency overlaps that of the partial sums.
struct CtrlSnap {
  int state;
  double rho_next, tau, eta;
};

// Deterministic dot product of two LDS/global vectors of length n by wavefront 0;
// the result is broadcast through *out (LDS).  Call from all threads.
__device__ void small_dot(const double* a, const double* b, int n, double* out) {
  if (threadIdx.x < 64) {
    double s = 0.0;
    for (int i = threadIdx.x; i < n; i += 64) s = fma(a[i], b[i], s);
    s = wave_sum(s);
    if (threadIdx.x == 0) *out = s;
  }
  __syncthreads();
}

// The scalars of a DCGS2 step, by wavefront 0 in one pass: C^T C and C^T S (each
// summed as small_dot sums it) and whether any of v[0..nv) is non-finite; broadcast
// through out[0], out[1] and *flag (LDS).  Call from all threads.
__device__ void step_scalars(const double* C, const double* S, int n, const double* v, int nv,
                             double* out, int* flag) {
  if (threadIdx.x < 64) {
    double cc = 0.0, cs = 0.0;
    for (int i = threadIdx.x; i < n; i += 64) {
      cc = fma(C[i], C[i], cc);
      cs = fma(C[i], S[i], cs);
    }
    int bad = 0;
    for (int i = threadIdx.x; i < nv; i += 64) bad |= !finite(v[i]);
    cc = wave_sum(cc);
    cs = wave_sum(cs);
    const bool any = __any(bad);
    if (threadIdx.x == 0) {
      out[0] = cc;
      out[1] = cs;
      *flag = any ? 1 : 0;
    }
  }
  __syncthreads();
}

// Any non-finite value among v[0..n)?  Result broadcast through *flag (LDS).
__device__ void any_nonfinite(const double* v, int n, int* flag) {
  if (threadIdx.x == 0) *flag = 0;
  __syncthreads();
  int bad = 0;
  for (int i = threadIdx.x; i < n; i += (int)blockDim.x) bad |= !finite(v[i]);
  if (bad) atomicOr(flag, 1);
  __syncthreads();
}

// GMRES: apply the stored Givens rotations to the just-completed Hessenberg column
// c (rows 0..c+1), form rotation c, update g and test the least-squares residual
// |g_{c+1}| against ctrl->gmres_thresh.  Thread 0 runs the recurrence; sh holds
// at least 3(c+2) doubles of LDS scratch.
__device__ void gmres_givens(const FinArgs& f, int c, int j, double* sh) {
  double* h = sh;
  double* cs = sh + (c + 2);
  double* sn = cs + (c + 1);
  for (int i = threadIdx.x; i <= c + 1; i += (int)blockDim.x) h[i] = f.H[(int64_t)c * f.ldh + i];
  for (int i = threadIdx.x; i < c; i += (int)blockDim.x) { cs[i] = f.cs[i]; sn[i] = f.sn[i]; }
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int i = 0; i < c; ++i) {
      const double a = h[i], b = h[i + 1];
      h[i] = cs[i] * a + sn[i] * b;
      h[i + 1] = -sn[i] * a + cs[i] * b;
    }
    const double a = h[c], b = h[c + 1];
    const double r = hypot(a, b);
    const double cc = r > 0.0 ? a / r : 1.0;
    const double ss = r > 0.0 ? b / r : 0.0;
    f.cs[c] = cc;
    f.sn[c] = ss;
    h[c] = r;
    const double gc = f.g[c];
    f.g[c] = cc * gc;
    f.g[c + 1] = -ss * gc;
    const double est = fabs(ss * gc);
    f.ctrl->resid_est = est;
    if (est <= f.ctrl->gmres_thresh && f.ctrl->state == ST_RUNNING) {
      f.ctrl->state = ST_DONE;
      f.ctrl->stop_step = j;
      f.ctrl->k = c + 1;
    }
  }
  __syncthreads();
  for (int i = threadIdx.x; i <= c; i += (int)blockDim.x) f.Rg[(int64_t)c * f.ldh + i] = h[i];
  __syncthreads();
}

// Complete the Hessenberg column J-1 with the reorthogonalisation coefficients:
// H_{1:J, J-1} = K_{1:J, J-1} + C,  H_{J+1, J-1} = alpha  (Alg. arnoldi, columns
// completed one step late).  Then GMRES rotations when enabled.
__device__ void complete_h_column(const FinArgs& f, const double* C, int J, double alpha,
                                  double* scratch) {
  const int col = J - 1;
  for (int i = threadIdx.x; i < J; i += (int)blockDim.x)
    f.H[(int64_t)col * f.ldh + i] = f.K[(int64_t)col * f.ldh + i] + C[i];
  if (threadIdx.x == 0) f.H[(int64_t)col * f.ldh + J] = alpha;
  __syncthreads();
  if (threadIdx.x == 0 && f.ctrl->state == ST_RUNNING) f.ctrl->k = J;
  if (f.gmres) gmres_givens(f, col, f.j, scratch);
}

// Scalar tail of a DCGS2 step once alpha_{j-1} is known (Alg. arnoldi: T, then the
// Hessenberg column H_{:,j-2} = K + C with H_{j-1,j-2} = alpha, then the new K column
// -- H is completed before K is formed, as the derivation after eq. (52) requires;
// or Alg. qr: R column and Stephen's trick).
//   C, S : LDS vectors of length J; sigma, gamma, cs = C^T S; rho = breakdown scale.
//   sprev: S_prev (QR; an LDS copy in the finishing kernel)
__device__ void step_tail(const FinArgs& f, const CtrlSnap& snap, const double* C, const double* S,
                          double sigma, double gamma, double csum, double alpha, double rho,
                          double* T, double* scratch, const double* sprev) {
  Ctrl* ctrl = f.ctrl;
  const int J = f.J, j = f.j;
  if (!finite(alpha)) {
    if (threadIdx.x == 0) { ctrl->state = ST_NONFINITE; ctrl->stop_step = j; }
    return;
  }
  if (alpha <= snap.eta * rho) {                  // breakdown: close column j-2 and stop
    if (f.qr) {
      for (int i = threadIdx.x; i < J; i += (int)blockDim.x) f.R[(int64_t)J * f.ldr + i] = sprev[i] + C[i];
      if (threadIdx.x == 0) f.R[(int64_t)J * f.ldr + J] = alpha;
      __syncthreads();
      if (threadIdx.x == 0) ctrl->k = J;
    } else if (j >= 3) {
      complete_h_column(f, C, J, alpha, scratch);
    }
    __syncthreads();
    if (threadIdx.x == 0 && (ctrl->state == ST_RUNNING || ctrl->state == ST_DONE)) {
      if (ctrl->state == ST_RUNNING) { ctrl->state = ST_BREAKDOWN; ctrl->stop_step = j; }
    }
    return;
  }
  // T_{1:j-2} = S/alpha, T_{j-1} = (sigma - C^T S)/alpha^2 (Arnoldi);
  // S_{j-1,j} = (sigma - C^T S)/alpha (QR, Stephen's trick)
  for (int i = threadIdx.x; i < J; i += (int)blockDim.x) T[i] = f.qr ? S[i] : S[i] / alpha;
  if (threadIdx.x == 0) T[J] = f.qr ? (sigma - csum) / alpha : (sigma - csum) / (alpha * alpha);
  __syncthreads();
  if (f.rec) {                                    // step record: T, alpha, next rho
    double* r = f.rec + 2 * (J + 2);
    for (int i = threadIdx.x; i <= J; i += (int)blockDim.x) r[i] = T[i];
    if (threadIdx.x == 0) {
      r[J + 1] = alpha;
      r[J + 2] = f.qr ? sqrt(gamma) : sqrt(gamma) / alpha;
    }
  }
  for (int i = threadIdx.x; i < J; i += (int)blockDim.x) f.coef[i] = C[i];
  for (int i = threadIdx.x; i <= J; i += (int)blockDim.x) f.coef[f.ldc + i] = T[i];
  if (threadIdx.x == 0) f.coef[2 * f.ldc] = alpha;
  if (f.qr) {
    // R_{1:j-2, j-1} = S_{1:j-2, j-1} + C ; R_{j-1,j-1} = alpha ; keep S_{1:j-1, j}
    for (int i = threadIdx.x; i < J; i += (int)blockDim.x) f.R[(int64_t)J * f.ldr + i] = sprev[i] + C[i];
    if (threadIdx.x == 0) f.R[(int64_t)J * f.ldr + J] = alpha;
    for (int i = threadIdx.x; i <= J; i += (int)blockDim.x) f.Sprev[i] = T[i];
    if (threadIdx.x == 0) { ctrl->k = J + 1; ctrl->rho_next = sqrt(gamma); }
  } else {
    if (f.gmres && j == 2 && threadIdx.x == 0) f.g[0] = alpha;   // beta e_1 of the cycle
    if (j >= 3) complete_h_column(f, C, J, alpha, scratch);      // H_{:,j-2}, H_{j-1,j-2}
    __syncthreads();
    // K_{1:j-1, j-1} = T - (1/alpha) H_{1:j-1, 1:j-2} C   (dense product).  Each row's
    // dot product is split over CH threads (column chunks, then the chunk partials
    // in order), so the chain of dependent global loads per thread stays short.
    // (Chunks over every thread of the workgroup, with 16 loads in flight, measured
    // slower.)
    {
      const int R = J + 1;
      const int cap = 3 * (J + 2) + 64;         // doubles of scratch
      int CH = (int)blockDim.x / R;
      if (CH > cap / R) CH = cap / R;
      if (CH < 1) CH = 1;
      const int L = (J + CH - 1) / CH;          // columns per chunk
      for (int t = threadIdx.x; t < R * CH; t += (int)blockDim.x) {
        const int i = t / CH, part = t % CH;
        const int c_lo = part * L, c_hi = min(J, c_lo + L);
        double hc = 0.0;
        for (int c0 = c_lo; c0 < c_hi; c0 += 8) {   // eight loads in flight, FMAs in order
          double h[8];
#pragma unroll
          for (int u = 0; u < 8; ++u) h[u] = f.H[(int64_t)min(c0 + u, c_hi - 1) * f.ldh + i];
#pragma unroll
          for (int u = 0; u < 8; ++u)
            if (c0 + u < c_hi) hc = fma(h[u], C[c0 + u], hc);
        }
        scratch[t] = hc;
      }
      __syncthreads();
      for (int i = threadIdx.x; i < R; i += (int)blockDim.x) {
        double hc = 0.0;
        for (int part = 0; part < CH; ++part) hc += scratch[i * CH + part];
        f.K[(int64_t)J * f.ldh + i] = T[i] - hc / alpha;
      }
    }
    if (threadIdx.x == 0) ctrl->rho_next = sqrt(gamma) / alpha;
  }
  __syncthreads();
}

// The finalising workgroup: red[] holds the grid-reduced values of this kernel; snap
// the control block as it was at the kernel's start; sprev: S_prev (QR steps and their
// fallback completion; an LDS copy).
__device__ void finalize(const FinArgs& f, const CtrlSnap& snap, double* red, double* T,
                         double* scratch, const double* sprev) {
  Ctrl* ctrl = f.ctrl;
  const int J = f.J, j = f.j;
  __shared__ double s_dot[2];
  __shared__ int s_flag;
  switch (f.kind) {
    case FIN_NORM:
      if (threadIdx.x == 0) { ctrl->norm2 = red[0]; ctrl->reductions += 1; }
      return;
    case FIN_NONE:
      return;
    case FIN_CGS2_S: {                     // S = Q^T a (and a^T a): first CGS2 projection
      any_nonfinite(red, J + 1, &s_flag);
      if (threadIdx.x == 0) {
        ctrl->reductions += 1;
        if (s_flag) { ctrl->state = ST_NONFINITE; ctrl->stop_step = j; }
        ctrl->rho_next = sqrt(red[J]);
      }
      for (int i = threadIdx.x; i < J; i += (int)blockDim.x) {
        f.coef[i] = red[i];
        f.Sprev[i] = red[i];
      }
      return;
    }
    case FIN_MGS_DOT: {                    // r = q_k^T w, w^T w (k = J, column j)
      if (threadIdx.x == 0) {
        ctrl->reductions += 1;
        const double r = red[0];
        if (!finite(r) || !finite(red[1])) {
          ctrl->state = ST_NONFINITE;
          ctrl->stop_step = j;
        } else {
          f.R[(int64_t)j * f.ldr + J] = r;
          f.coef[0] = r;
          if (J == 0) ctrl->rho_next = sqrt(red[1]);    // ||a_j|| before any projection
        }
      }
      return;
    }
    case FIN_MGS_NORM: {                   // alpha = ||w|| closes column j
      if (threadIdx.x == 0) {
        ctrl->reductions += 1;
        const double alpha = sqrt(red[0]);
        const double rho = j == 0 ? alpha : snap.rho_next;
        if (!finite(alpha)) {
          ctrl->state = ST_NONFINITE;
          ctrl->stop_step = j;
        } else {
          f.R[(int64_t)j * f.ldr + j] = alpha;
          f.coef[2 * f.ldc] = alpha;
          if (alpha <= snap.eta * rho || alpha == 0.0) {
            ctrl->state = ST_BREAKDOWN;
            ctrl->stop_step = j;
            ctrl->k = j;
          } else {
            ctrl->k = j + 1;
          }
        }
      }
      return;
    }
    case FIN_LAST1: {                      // c = Q^T w (and w^T w)
      any_nonfinite(red, J + 1, &s_flag);
      if (threadIdx.x == 0) {
        ctrl->reductions += 1;
        if (s_flag) { ctrl->state = ST_NONFINITE; ctrl->stop_step = j; }
        if (J == 0) ctrl->rho_next = sqrt(red[0]);   // single-column QR: rho = ||a_1||
      }
      for (int i = threadIdx.x; i < J; i += (int)blockDim.x) f.coef[i] = red[i];
      return;
    }
    case FIN_LAST2: {                      // alpha = ||w - Q c||, close the last column
      const double alpha = sqrt(red[0]);
      const double* c = f.coef;
      if (threadIdx.x == 0) ctrl->reductions += 1;
      if (!finite(alpha)) {
        if (threadIdx.x == 0) { ctrl->state = ST_NONFINITE; ctrl->stop_step = j; }
        return;
      }
      for (int i = threadIdx.x; i < J; i += (int)blockDim.x) T[i] = c[i];   // c into LDS
      __syncthreads();
      const bool brk = alpha <= snap.eta * snap.rho_next;
      if (f.qr) {
        for (int i = threadIdx.x; i < J; i += (int)blockDim.x) f.R[(int64_t)J * f.ldr + i] = f.Sprev[i] + T[i];
        if (threadIdx.x == 0) {
          f.R[(int64_t)J * f.ldr + J] = alpha;
          ctrl->k = brk ? J : J + 1;
        }
      } else {
        complete_h_column(f, T, J, alpha, scratch);
      }
      __syncthreads();
      if (threadIdx.x == 0) {
        f.coef[2 * f.ldc] = alpha;
        if (brk && ctrl->state == ST_RUNNING) { ctrl->state = ST_BREAKDOWN; ctrl->stop_step = j; }
      }
      return;
    }
    case FIN_RESTART: {                    // C = 0, alpha = 1: T = Q_{1:k+1}^T v
      const int Jt = J + 2;
      const double* S = red + Jt;
      any_nonfinite(red, 2 * Jt, &s_flag);
      if (s_flag) {
        if (threadIdx.x == 0) { ctrl->state = ST_NONFINITE; ctrl->stop_step = j; ctrl->reductions += 1; }
        return;
      }
      for (int i = threadIdx.x; i < J; i += (int)blockDim.x) { T[i] = S[i]; f.coef[i] = 0.0; }
      if (threadIdx.x == 0) T[J] = S[J];   // sigma = q_{k+1}^T v
      __syncthreads();
      for (int i = threadIdx.x; i <= J; i += (int)blockDim.x) {
        f.coef[f.ldc + i] = T[i];
        f.K[(int64_t)J * f.ldh + i] = T[i];
      }
      if (threadIdx.x == 0) {
        f.coef[2 * f.ldc] = 1.0;
        ctrl->rho_next = sqrt(S[J + 1]);
        ctrl->reductions += 1;
      }
      __syncthreads();
      return;
    }
    case FIN_STEP: {
      const int Jt = J + 2;
      const double* C = red;
      const double beta = red[J];
      const double* S = red + Jt;
      const double sigma = red[Jt + J];
      const double gamma = red[Jt + J + 1];
      step_scalars(C, S, J, red, 2 * Jt, s_dot, &s_flag);
      if (s_flag) {
        if (threadIdx.x == 0) { ctrl->state = ST_NONFINITE; ctrl->stop_step = j; ctrl->reductions += 1; }
        return;
      }
      const double rho = (j == 2) ? sqrt(beta) : snap.rho_next;
      const double d = beta - s_dot[0];
      if (threadIdx.x == 0) ctrl->reductions += 1;
      if (!(finite(d) && d > snap.tau * beta)) {
        // hand the reduced step over to the explicit-norm fallback (run by the host)
        for (int i = threadIdx.x; i < J; i += (int)blockDim.x) {
          f.pend[i] = C[i];
          f.pend[J + i] = S[i];
          f.coef[i] = C[i];
        }
        if (threadIdx.x == 0) {
          f.pend[2 * J] = sigma;
          f.pend[2 * J + 1] = gamma;
          f.pend[2 * J + 2] = beta;
          ctrl->state = ST_FALLBACK;
          ctrl->stop_step = j;
        }
        return;
      }
      step_tail(f, snap, C, S, sigma, gamma, s_dot[1], sqrt(d), rho, T, scratch, sprev);
      return;
    }
    case FIN_FALLBACK: {
      const double alpha = sqrt(red[0]);
      double* C = scratch;                 // pend -> LDS
      double* S = scratch + J;
      for (int i = threadIdx.x; i < J; i += (int)blockDim.x) { C[i] = f.pend[i]; S[i] = f.pend[J + i]; }
      __syncthreads();
      const double sigma = f.pend[2 * J], gamma = f.pend[2 * J + 1], beta = f.pend[2 * J + 2];
      small_dot(C, S, J, &s_dot[1]);
      const double rho = (j == 2) ? sqrt(beta) : snap.rho_next;
      if (threadIdx.x == 0) { ctrl->reductions += 1; ctrl->fallbacks += 1; }
      step_tail(f, snap, C, S, sigma, gamma, s_dot[1], alpha, rho, T, scratch + 2 * J, sprev);
      return;
    }
  }
}

// Threads of the finishing workgroup (one per reduction).
constexpr int FINISH_BS = 1024;

// LDS of finish_body for V reduced values and J basis columns: the sums (V), the
// finaliser's T (J + 3) and scratch (5 (J + 3) + 64), and the chunk sums of
// partial_sum (max(V, FINISH_BS)).
__host__ __device__ inline size_t finish_smem(int V, int J) {
  const int Jp = J + 3;
  return sizeof(double) * (size_t)(V + Jp + 5 * Jp + 64 + (V > FINISH_BS ? V : FINISH_BS) + Jp);
}

// Second half of every DCGS2 reduction, run by a single workgroup after the
// streaming kernel has stored its per-workgroup partials: the G partials of each
// of the V values are summed in a fixed order and the step is finalised.  Running
// it as a kernel of its own (instead of letting the last workgroup to arrive do
// it) needs no device-scope fence in the streaming kernel: on this chip such a
// fence writes back the L2 of the workgroup's XCD, which measured tens of
// microseconds per launch; the kernel boundary makes the partials visible.
__device__ void finish_body(const GridRed& gr, int V, const FinArgs& fin, int J) {
  extern __shared__ double smem[];
  double* red = smem;                     // V
  double* T = red + V;                    // J + 3
  double* scratch = T + (J + 3);          // 5 (J + 3) + 64
  double* sp = scratch + 5 * (J + 3) + 64;        // max(V, FINISH_BS)
  double* sprev = sp + (V > FINISH_BS ? V : FINISH_BS);   // J + 3
  // the control block and (QR) S_prev are read before the partials are summed, so
  // that their memory latencies overlap (a stopped expansion still returns here)
  CtrlSnap snap;
  snap.state = fin.ctrl->state;
  snap.rho_next = fin.ctrl->rho_next;
  snap.tau = fin.ctrl->tau;
  snap.eta = fin.ctrl->eta;
  const bool qstep = fin.qr && (fin.kind == FIN_STEP || fin.kind == FIN_FALLBACK);
  if (qstep)
    for (int i = threadIdx.x; i < J; i += (int)blockDim.x) sprev[i] = fin.Sprev[i];
  partial_sum(gr.P1, gr.ldp, gr.G, V, red, sp);   // ends with a barrier
  if (snap.state != ST_RUNNING) return;
  if (fin.rec && fin.kind == FIN_STEP)
    for (int v = threadIdx.x; v < V; v += (int)blockDim.x) fin.rec[v] = red[v];
  finalize(fin, snap, red, T, scratch, qstep ? sprev : fin.Sprev);
}


// ---------------------------------------------------------------------------------
// Reduction pass: per-workgroup partial dot products of [Q_{0..J-1}, x, (y)] with
// [x, (y)] over a contiguous slab of rows.
//
// The basis columns are taken in column groups of exactly NC = 16, 8, 4, 2 or 1
// (J = 16 q + binary digits of the remainder), each group one sweep over the
// slab, so no load in a sweep is conditional: every load of an unrolled
// iteration is issued before the first one is waited for.  (A per-column bound
// test inside the sweep would make each load wait for the previous one.)  A last
// sweep forms x^T x, x^T y and y^T y.  Partial layout (V values per workgroup):
//   [0, Jt)   = [Q, x, y]^T x,   [Jt, 2 Jt) = [Q, x, y]^T y   (HASY, Jt = J + 2)
//   [0, Jt)   = [Q, x]^T x                                      (Jt = J + 1)
//
// XS: where x and y come from -- 0 the vectors, 1 the vectors, also copied into the
// workgroup's LDS slab sx, sy (unit u at index u - u0), 2 that LDS copy, 3 yf (x and
// y = A x of the unit, y stored by yf), also copied into the slab.  Each thread copies
// and later reads back the same units, so the copy needs no barrier.  x, y themselves
// serve the odd last row.
// A reduction without its own y (never called).
struct NoY {
  template <int VW>
  __device__ void operator()(int64_t, RowVec<VW>&, RowVec<VW>&) const {}
};

template <int VW, bool HASY, int NC, typename TQ, int XS, class YF = NoY>
__device__ __forceinline__ void reduce_sweep(const TQ* __restrict__ Q, int64_t ldq, int k0,
                                             const double* __restrict__ x,
                                             const double* __restrict__ y, double* sx,
                                             double* sy, int64_t u0, int64_t u1, bool tail,
                                             int64_t m, double* shb, double* P, int Jt,
                                             const YF& yf = YF{}) {
  constexpr int NA = HASY ? 2 * NC : NC;
  using RV = RowVec<VW>;
  double acc[NA];
#pragma unroll
  for (int c = 0; c < NA; ++c) acc[c] = 0.0;
  const TQ* __restrict__ qb = Q + (int64_t)k0 * ldq;
  // (two units a block width apart per iteration measured slower here, with either basis)
  for (int64_t u = u0 + threadIdx.x; u < u1; u += BS) {
    RV xv, yv;
    if constexpr (XS == 3) {
      yf(u, xv, yv);                       // x and y = A x of the unit (y stored by yf)
    } else {
      xv = XS == 2 ? RV::load(sx, u - u0) : RV::load(x, u);
      yv = !HASY ? RV::zero() : XS == 2 ? RV::load(sy, u - u0) : RV::load(y, u);
    }
    if (XS == 1 || XS == 3) {
      xv.store(sx, u - u0);
      if (HASY) yv.store(sy, u - u0);
    }
    RV q[NC];
#pragma unroll
    for (int c = 0; c < NC; ++c) q[c] = RV::load(qb + (int64_t)c * ldq, u);
#pragma unroll
    for (int c = 0; c < NC; ++c) {
      acc[c] += q[c].dot(xv);
      if (HASY) acc[NC + c] += q[c].dot(yv);
    }
  }
  if (tail) {                              // odd m with 2-row units: last row
    const int64_t r = m - 1;
    const double xr = x[r], yr = HASY ? y[r] : 0.0;
#pragma unroll
    for (int c = 0; c < NC; ++c) {
      const double q = (double)qb[(int64_t)c * ldq + r];
      acc[c] += q * xr;
      if (HASY) acc[NC + c] += q * yr;
    }
  }
  block_sum_t<NA, NC>(acc, shb, P + k0, NC, P + Jt + k0, HASY ? NC : 0);
}

template <int VW, bool HASY, bool LDSX>
__device__ __forceinline__ void reduce_self(const double* __restrict__ x,
                                            const double* __restrict__ y, const double* sx,
                                            const double* sy, int64_t u0, int64_t u1,
                                            bool tail, int64_t m, double* shb, double* P, int J,
                                            int Jt) {
  using RV = RowVec<VW>;
  double acc[4] = {0.0, 0.0, 0.0, 0.0};   // x.x, x.y, y.y, unused
#pragma unroll 4
  for (int64_t u = u0 + threadIdx.x; u < u1; u += BS) {
    const RV xv = LDSX ? RV::load(sx, u - u0) : RV::load(x, u);
    acc[0] += xv.dot(xv);
    if (HASY) {
      const RV yv = LDSX ? RV::load(sy, u - u0) : RV::load(y, u);
      acc[1] += xv.dot(yv);
      acc[2] += yv.dot(yv);
    }
  }
  if (tail) {
    const int64_t r = m - 1;
    const double xr = x[r], yr = HASY ? y[r] : 0.0;
    acc[0] += xr * xr;
    if (HASY) { acc[1] += xr * yr; acc[2] += yr * yr; }
  }
  double* out = shb + NW * 4;
  block_sum_t<4, 4>(acc, shb, out, 3, nullptr, 0);
  if (threadIdx.x == 0) {
    P[J] = out[0];
    if (HASY) {
      P[J + 1] = out[1];                     // y^T x
      P[Jt + J] = out[1];                    // x^T y
      P[Jt + J + 1] = out[2];
    }
  }
}

// STAGE 1: the first column-group sweep also copies the workgroup's slab of x and y
// into LDS (after the block-sum scratch), and the later sweeps and the final
// x^T x, x^T y, y^T y read them there.  Read from HBM by every sweep, x and y are
// fetched again each time: a slab is far larger than what stays in L2 while a sweep
// streams its basis columns.  STAGE 2: the slab is in LDS already (written there by
// the same threads that read it back).  STAGE 3: as STAGE 1, with x and y of each unit
// given by yf (which computes y = A x and stores it), so that the matvec's loads
// overlap the first sweep's.  STAGE 0: every sweep reads x and y.
constexpr int REDUCE_SCRATCH = NW * 2 * NT;   // doubles of block-sum scratch

// Rows [u0 VW, u1 VW) of workgroup bid of a reduction grid of G over m rows.
template <int VW>
__device__ __forceinline__ void reduce_slab(int64_t m, int G, int bid, int64_t* per,
                                            int64_t* u0, int64_t* u1) {
  const int64_t units = m / VW;
  *per = (units + G - 1) / G;
  *u0 = (int64_t)bid * *per;
  *u1 = min(units, *u0 + *per);
}

template <int VW, bool HASY, typename TQ, int STAGE = 0, class YF = NoY>
__device__ __forceinline__ void reduce_body(const TQ* __restrict__ Q, int64_t ldq,
                                                    int J, const double* __restrict__ x,
                                                    const double* __restrict__ y, int64_t m,
                                                    const GridRed& gr, const FinArgs& fin, int bid,
                                                    const YF& yf = YF{}) {
  extern __shared__ double smem[];
  if (fin.ctrl->state != ST_RUNNING) return;
  const int Jt = J + (HASY ? 2 : 1);
  double* shb = smem;                       // REDUCE_SCRATCH
  int64_t per, u0, u1;
  reduce_slab<VW>(m, gr.G, bid, &per, &u0, &u1);
  const bool tail = (VW == 2) && (m & 1) && bid == gr.G - 1 && threadIdx.x == 0;
  double* P = gr.P1 + (int64_t)bid * gr.ldp;
  double* sx = smem + REDUCE_SCRATCH;       // STAGE > 0: per VW doubles of each vector
  double* sy = sx + per * VW;
  constexpr int XF = STAGE;                 // the first sweep
  constexpr int XN = STAGE > 0 ? 2 : 0;     // the later ones
  // the groups in order 16 ... 16, 8, 4, 2, 1; the first one present copies the slab
  int k0 = 0;
  bool first = true;
#define DCGS2_SWEEP(NC)                                                                  \
  do {                                                                                   \
    if (first)                                                                           \
      reduce_sweep<VW, HASY, NC, TQ, XF>(Q, ldq, k0, x, y, sx, sy, u0, u1, tail, m, shb,  \
                                         P, Jt, yf);                                     \
    else                                                                                 \
      reduce_sweep<VW, HASY, NC, TQ, XN>(Q, ldq, k0, x, y, sx, sy, u0, u1, tail, m, shb,  \
                                         P, Jt, yf);                                     \
    first = false;                                                                       \
    k0 += NC;                                                                            \
  } while (0)
  if (STAGE == 3 && J == 0) {               // no sweep: the slab is staged on its own
    for (int64_t u = u0 + threadIdx.x; u < u1; u += BS) {
      RowVec<VW> xv, yv;
      yf(u, xv, yv);
      xv.store(sx, u - u0);
      yv.store(sy, u - u0);
    }
  }
  while (k0 + 16 <= J) DCGS2_SWEEP(16);
  if (k0 + 8 <= J) DCGS2_SWEEP(8);
  if (k0 + 4 <= J) DCGS2_SWEEP(4);
  if (k0 + 2 <= J) DCGS2_SWEEP(2);
  if (k0 + 1 <= J) DCGS2_SWEEP(1);
#undef DCGS2_SWEEP
  if (STAGE >= 2 || (STAGE == 1 && J > 0))
    reduce_self<VW, HASY, true>(x, y, sx, sy, u0, u1, tail, m, shb, P, J, Jt);
  else
    reduce_self<VW, HASY, false>(x, y, sx, sy, u0, u1, tail, m, shb, P, J, Jt);
}

// u = x - Q_{0..J-1} C written to ubuf; ||u||^2 grid-reduced and finalised.
template <int VW, typename TQ>
__device__ __forceinline__ void project_norm_body(const TQ* __restrict__ Q, int64_t ldq,
                                                          int J, const double* __restrict__ x,
                                                          double* __restrict__ ubuf, int64_t m,
                                                          const GridRed& gr, const FinArgs& fin, int bid) {
  extern __shared__ double smem[];
  if (fin.ctrl->state != ST_RUNNING) return;
  double* shb = smem;                       // NW
  const double* __restrict__ C = fin.coef;
  const int64_t units = m / VW;
  const int64_t per = (units + gr.G - 1) / gr.G;
  const int64_t u0 = (int64_t)bid * per;
  const int64_t u1 = min(units, u0 + per);
  using RV = RowVec<VW>;
  double acc[1] = {0.0};
  for (int64_t u = u0 + threadIdx.x; u < u1; u += BS) {
    RV sc = RV::zero();
#pragma unroll 8
    for (int k = 0; k < J; ++k) {
      const RV q = RV::load(Q + (int64_t)k * ldq, u);
      const double ck = C[k];
#pragma unroll
      for (int e = 0; e < VW; ++e) sc.e[e] = fma(q.e[e], ck, sc.e[e]);
    }
    const RV xv = RV::load(x, u);
    RV uu;
#pragma unroll
    for (int e = 0; e < VW; ++e) uu.e[e] = xv.e[e] - sc.e[e];
    uu.store(ubuf, u);
    acc[0] += uu.dot(uu);
  }
  if ((VW == 2) && (m & 1) && bid == gr.G - 1 && threadIdx.x == 0) {
    const int64_t r = m - 1;
    double s = 0.0;
    for (int k = 0; k < J; ++k) s = fma((double)Q[(int64_t)k * ldq + r], C[k], s);
    const double uval = x[r] - s;
    ubuf[r] = uval;
    acc[0] += uval * uval;
  }
  block_sum<1>(acc, shb, gr.P1 + (int64_t)bid * gr.ldp, 1);
}

// NC basis columns of one row unit into the update's two products: all NC loads are
// issued before the first one is used (the coefficients are wavefront-uniform).
template <int NC, int VW, typename TQ>
__device__ __forceinline__ void update_group(const TQ* __restrict__ Q, int64_t ldq, int k0,
                                             int64_t u, const double* __restrict__ C,
                                             const double* __restrict__ T, RowVec<VW>& sc,
                                             RowVec<VW>& st) {
  RowVec<VW> q[NC];
#pragma unroll
  for (int c = 0; c < NC; ++c) q[c] = RowVec<VW>::load(Q + (int64_t)(k0 + c) * ldq, u);
#pragma unroll
  for (int c = 0; c < NC; ++c) {
    const double ck = C[k0 + c], tk = T[k0 + c];
#pragma unroll
    for (int e = 0; e < VW; ++e) {
      sc.e[e] = fma(q[c].e[e], ck, sc.e[e]);
      st.e[e] = fma(q[c].e[e], tk, st.e[e]);
    }
  }
}

// q_{j-1} and w_j of row unit u from its products sc = (Q C)_u and st = (Q T)_u.
template <int VW, bool ARN, bool QCOL, typename TQ>
__device__ __forceinline__ void update_finish_unit(double* __restrict__ x,
                                                   const double* __restrict__ y,
                                                   const double* __restrict__ ubuf, double alpha,
                                                   double tJ, TQ* __restrict__ qout, int64_t u,
                                                   const RowVec<VW>& sc, const RowVec<VW>& st) {
  const RowVec<VW> xv = RowVec<VW>::load(x, u);
  const RowVec<VW> yv = RowVec<VW>::load(y, u);
  RowVec<VW> qc = RowVec<VW>::zero();
  if (QCOL) qc = RowVec<VW>::load(ubuf, u);
  RowVec<VW> qn, wn;
#pragma unroll
  for (int e = 0; e < VW; ++e) {
    const double q = stored<TQ>(QCOL ? qc.e[e] / alpha : (xv.e[e] - sc.e[e]) / alpha);
    const double yt = ARN ? yv.e[e] / alpha : yv.e[e];
    qn.e[e] = q;
    wn.e[e] = yt - fma(q, tJ, st.e[e]);
  }
  qn.store(qout, u);
  wn.store(x, u);
}

// Update of one row unit u: q_{j-1} and w_j.  The basis columns are taken in exact
// groups of 16, 8, 4, 2 and 1 (J = 16 q + the binary digits of the rest), so that every
// load of a group is in flight together, as in the reduction sweeps.
template <int VW, bool ARN, bool QCOL, typename TQ>
__device__ __forceinline__ void update_unit(const TQ* __restrict__ Q, int64_t ldq, int J,
                                            double* __restrict__ x,
                                            const double* __restrict__ y,
                                            const double* __restrict__ ubuf,
                                            const double* __restrict__ C,
                                            const double* __restrict__ T, double alpha,
                                            double tJ, TQ* __restrict__ qout, int64_t u) {
  RowVec<VW> sc = RowVec<VW>::zero(), st = RowVec<VW>::zero();
  int k0 = 0;
  for (; k0 + 16 <= J; k0 += 16) update_group<16, VW, TQ>(Q, ldq, k0, u, C, T, sc, st);
  if (k0 + 8 <= J) { update_group<8, VW, TQ>(Q, ldq, k0, u, C, T, sc, st); k0 += 8; }
  if (k0 + 4 <= J) { update_group<4, VW, TQ>(Q, ldq, k0, u, C, T, sc, st); k0 += 4; }
  if (k0 + 2 <= J) { update_group<2, VW, TQ>(Q, ldq, k0, u, C, T, sc, st); k0 += 2; }
  if (k0 + 1 <= J) update_group<1, VW, TQ>(Q, ldq, k0, u, C, T, sc, st);
  update_finish_unit<VW, ARN, QCOL, TQ>(x, y, ubuf, alpha, tJ, qout, u, sc, st);
}

// update_group for two row units at once (all 2 NC loads issued before the first use).
template <int NC, int VW, typename TQ>
__device__ __forceinline__ void update_group2(const TQ* __restrict__ Q, int64_t ldq, int k0,
                                              int64_t u, int64_t u2, const double* __restrict__ C,
                                              const double* __restrict__ T, RowVec<VW>& sc,
                                              RowVec<VW>& st, RowVec<VW>& sc2, RowVec<VW>& st2) {
  RowVec<VW> q[NC], q2[NC];
#pragma unroll
  for (int c = 0; c < NC; ++c) {
    q[c] = RowVec<VW>::load(Q + (int64_t)(k0 + c) * ldq, u);
    q2[c] = RowVec<VW>::load(Q + (int64_t)(k0 + c) * ldq, u2);
  }
#pragma unroll
  for (int c = 0; c < NC; ++c) {
    const double ck = C[k0 + c], tk = T[k0 + c];
#pragma unroll
    for (int e = 0; e < VW; ++e) {
      sc.e[e] = fma(q[c].e[e], ck, sc.e[e]);
      st.e[e] = fma(q[c].e[e], tk, st.e[e]);
      sc2.e[e] = fma(q2[c].e[e], ck, sc2.e[e]);
      st2.e[e] = fma(q2[c].e[e], tk, st2.e[e]);
    }
  }
}

template <int VW, bool ARN, bool QCOL, typename TQ>
__device__ __forceinline__ void update_unit2(const TQ* __restrict__ Q, int64_t ldq, int J,
                                             double* __restrict__ x,
                                             const double* __restrict__ y,
                                             const double* __restrict__ ubuf,
                                             const double* __restrict__ C,
                                             const double* __restrict__ T, double alpha,
                                             double tJ, TQ* __restrict__ qout, int64_t u,
                                             int64_t u2) {
  RowVec<VW> sc = RowVec<VW>::zero(), st = RowVec<VW>::zero();
  RowVec<VW> sc2 = RowVec<VW>::zero(), st2 = RowVec<VW>::zero();
  int k0 = 0;
  for (; k0 + 16 <= J; k0 += 16) update_group2<16, VW, TQ>(Q, ldq, k0, u, u2, C, T, sc, st, sc2, st2);
  if (k0 + 8 <= J) { update_group2<8, VW, TQ>(Q, ldq, k0, u, u2, C, T, sc, st, sc2, st2); k0 += 8; }
  if (k0 + 4 <= J) { update_group2<4, VW, TQ>(Q, ldq, k0, u, u2, C, T, sc, st, sc2, st2); k0 += 4; }
  if (k0 + 2 <= J) { update_group2<2, VW, TQ>(Q, ldq, k0, u, u2, C, T, sc, st, sc2, st2); k0 += 2; }
  if (k0 + 1 <= J) update_group2<1, VW, TQ>(Q, ldq, k0, u, u2, C, T, sc, st, sc2, st2);
  update_finish_unit<VW, ARN, QCOL, TQ>(x, y, ubuf, alpha, tJ, qout, u, sc, st);
  update_finish_unit<VW, ARN, QCOL, TQ>(x, y, ubuf, alpha, tJ, qout, u2, sc2, st2);
}

// The odd last row of an update with two-row units.
template <bool ARN, bool QCOL, typename TQ>
__device__ __forceinline__ void update_last_row(const TQ* __restrict__ Q, int64_t ldq, int J,
                                                double* __restrict__ x,
                                                const double* __restrict__ y,
                                                const double* __restrict__ ubuf, int64_t m,
                                                const double* __restrict__ C,
                                                const double* __restrict__ T, double alpha,
                                                double tJ, TQ* __restrict__ qout) {
  const int64_t r = m - 1;
  double sc = 0.0, st = 0.0;
  for (int k = 0; k < J; ++k) {
    const double q = (double)Q[(int64_t)k * ldq + r];
    sc = fma(q, C[k], sc);
    st = fma(q, T[k], st);
  }
  const double q = stored<TQ>(QCOL ? ubuf[r] / alpha : (x[r] - sc) / alpha);
  const double yt = ARN ? y[r] / alpha : y[r];
  qout[r] = (TQ)q;
  x[r] = yt - fma(q, tJ, st);
}

// Update pass: q_{j-1} and w_j, one row unit per thread of workgroup bid (the odd last
// row with two-row units by the thread after the last unit).
template <int VW, bool ARN, bool QCOL, typename TQ>
__device__ __forceinline__ void update_body(TQ* __restrict__ Q, int64_t ldq, int J,
                                                    double* __restrict__ x,
                                                    const double* __restrict__ y,
                                                    const double* __restrict__ ubuf, int64_t m,
                                                    const double* __restrict__ coef, int ldc,
                                                    const Ctrl* __restrict__ ctrl, int bid) {
  if (ctrl->state != ST_RUNNING) return;
  const double* __restrict__ C = coef;
  const double* __restrict__ T = coef + ldc;
  const double alpha = coef[2 * ldc];
  const double tJ = T[J];
  const int64_t units = m / VW;
  const int64_t u = (int64_t)bid * BS + threadIdx.x;
  TQ* qout = Q + (int64_t)J * ldq;
  if (u < units)
    update_unit<VW, ARN, QCOL, TQ>(Q, ldq, J, x, y, ubuf, C, T, alpha, tJ, qout, u);
  else if (VW == 2 && (m & 1) && u == units)
    update_last_row<ARN, QCOL, TQ>(Q, ldq, J, x, y, ubuf, m, C, T, alpha, tJ, qout);
}

// Update pass over slabs: workgroup bid of nb takes a contiguous slab of row units,
// BS at a time (the odd last row by thread 0 of the last workgroup).
template <int VW, bool ARN, bool QCOL, typename TQ>
__device__ __forceinline__ void update_slab_body(TQ* __restrict__ Q, int64_t ldq, int J,
                                                 double* __restrict__ x,
                                                 const double* __restrict__ y,
                                                 const double* __restrict__ ubuf, int64_t m,
                                                 const double* __restrict__ coef, int ldc,
                                                 const Ctrl* __restrict__ ctrl, int bid,
                                                 int nb) {
  if (ctrl->state != ST_RUNNING) return;
  const double* __restrict__ C = coef;
  const double* __restrict__ T = coef + ldc;
  const double alpha = coef[2 * ldc];
  const double tJ = T[J];
  const int64_t units = m / VW;
  const int64_t per = (units + nb - 1) / nb;
  const int64_t u0 = (int64_t)bid * per;
  const int64_t u1 = min(units, u0 + per);
  TQ* qout = Q + (int64_t)J * ldq;
  if constexpr (sizeof(TQ) == 4) {
    // FP32 basis: two row units per iteration, a block width apart, so that a
    // wavefront has as many bytes in flight as with an FP64 basis (measured faster
    // there, slower with FP64)
    for (int64_t u = u0 + threadIdx.x; u < u1; u += 2 * BS) {
      if (u + BS < u1)
        update_unit2<VW, ARN, QCOL, TQ>(Q, ldq, J, x, y, ubuf, C, T, alpha, tJ, qout, u, u + BS);
      else
        update_unit<VW, ARN, QCOL, TQ>(Q, ldq, J, x, y, ubuf, C, T, alpha, tJ, qout, u);
    }
  } else {
    for (int64_t u = u0 + threadIdx.x; u < u1; u += BS)
      update_unit<VW, ARN, QCOL, TQ>(Q, ldq, J, x, y, ubuf, C, T, alpha, tJ, qout, u);
  }
  if (VW == 2 && (m & 1) && bid == nb - 1 && threadIdx.x == 0)
    update_last_row<ARN, QCOL, TQ>(Q, ldq, J, x, y, ubuf, m, C, T, alpha, tJ, qout);
}

