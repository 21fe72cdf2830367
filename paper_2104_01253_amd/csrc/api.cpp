// Host driver of libdcgs2.so: argument validation, device workspace, the step
// schedule of the DCGS2 expansion (Alg. qr / Alg. arnoldi of arXiv 2104.01253),
// and the GMRES and Krylov-Schur drivers built on it.
//
// Schedule of one expansion (all launches are asynchronous on the context
// stream; the host synchronises once at the end, or once per restart cycle):
//   step j = 2..n+1 : [A w_{j-1} -> v]  reduce(j) + finalise  update(j)
//   last column     : reduce(c = Q^T w)  project + norm  scale    (CGS2 finish)
// Every kernel first reads the device control block and returns at once unless
// the expansion is still RUNNING, so a breakdown, a non-finite value, GMRES
// convergence or a Pythagorean-guard failure stops the remaining launches
// without a host round trip.  The guard failure is then resolved here: the
// explicit-norm fallback of that step is enqueued and the schedule resumes.
#include <hip/hip_runtime_api.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <atomic>
#include <new>
#include <thread>
#include <vector>

#include "internal.h"

using namespace dcgs2;

namespace {

constexpr int LDC = DCGS2_MAX_N + 2;              // coef block stride
constexpr int LDP = 2 * (DCGS2_MAX_N + 2) + 8;    // partials stride
constexpr int LDH_MAX = DCGS2_MAX_N + 1;          // square small-matrix buffers

}  // namespace

struct dcgs2_ctx_s {
  int device = 0;
  hipStream_t stream = nullptr;
  bool own_stream = false;
  bool ready = false;
  double tau = 1e-8, eta = 1e-12;
  bool qr_one_pass = true;
  int tune_fused_waves = 8;      // DCGS2_TUNE_FUSED_WAVES
  int tune_reduce_gmax = 0;      // DCGS2_TUNE_REDUCE_GRID (0: automatic)
  int tune_fused_min_j = 0;      // DCGS2_TUNE_FUSED_MIN_J
  int tune_batch_units = 1024;   // DCGS2_TUNE_BATCH_REDUCE_ROWS / 2
  int tune_pair_max_ns = 16;     // DCGS2_TUNE_FUSED_PAIR_SLOTS
  int tune_batch_host_dense = 1; // DCGS2_TUNE_BATCH_DENSE
  int tune_matvec_fold = 1;      // DCGS2_TUNE_MATVEC_FOLD
  int tune_update_grid = 0;      // DCGS2_TUNE_UPDATE_GRID (0: automatic)
  int64_t cap_m = 0;
  int64_t cap_qa = 0, cap_qb = 0;
  double *w = nullptr, *v = nullptr, *r = nullptr;
  double* P1 = nullptr;
  double *coef = nullptr, *pend = nullptr;
  double *H = nullptr, *K = nullptr, *Rg = nullptr, *R = nullptr, *Z = nullptr;
  double *Sprev = nullptr, *cs = nullptr, *sn = nullptr, *g = nullptr;
  double *Qa = nullptr, *Qb = nullptr;    // internal bases (GMRES, Krylov-Schur)
  double* rec = nullptr;                  // step records of the steps entry points
  int64_t cap_rec = 0;
  int basis_q32 = 0;                         // internal bases stored in FP32
  Ctrl* ctrl = nullptr;
  Ctrl* ctrl_host = nullptr;       // pinned
  int kernels = 0;
  // kernel timing (dcgs2_profile_enable): HIP events bracket each launch
  struct ProfRec { int cls; hipEvent_t a, b; double bytes; };
  struct ProfAcc { int64_t launches = 0; double ms = 0.0, bytes = 0.0; };
  bool prof = false;
  std::vector<hipEvent_t> evpool;
  std::vector<ProfRec> pending;
  ProfAcc acc[16];
};

namespace {

#define CK(call)                                   \
  do {                                             \
    hipError_t e_ = (call);                        \
    if (e_ != hipSuccess) return DCGS2_EDEVICE;    \
  } while (0)

#define CKL(call)                                  \
  do {                                             \
    hipError_t e_ = (call);                        \
    if (e_ != hipSuccess) return DCGS2_EDEVICE;    \
    ++c->kernels;                                  \
  } while (0)

// Kernel classes reported by dcgs2_profile_read.
// The last two are wall-clock phases of the batched solver, not kernels: device
// time of an expansion cycle (launch to completion) and the host dense work.
enum KClass { K_SPMV = 0, K_REDUCE, K_UPDATE, K_PROJNORM, K_SCALE, K_TSGEMM, K_FUSED, K_AUX,
              K_BATCH_CYCLE, K_HOST_DENSE, K_NCLASS };
const char* const kClassName[K_NCLASS] = {"spmv", "reduce", "update", "project_norm",
                                          "scale", "tsgemm", "fused_qr", "aux",
                                          "phase_batched_cycle", "phase_host_dense"};

hipEvent_t prof_event(dcgs2_ctx c) {
  if (!c->evpool.empty()) {
    hipEvent_t e = c->evpool.back();
    c->evpool.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  if (hipEventCreate(&e) != hipSuccess) return nullptr;
  return e;
}

// Fold completed launch timings into the accumulators (call after a stream sync).
void prof_resolve(dcgs2_ctx c) {
  for (auto& r : c->pending) {
    float ms = 0.0f;
    if (hipEventElapsedTime(&ms, r.a, r.b) == hipSuccess) {
      c->acc[r.cls].launches += 1;
      c->acc[r.cls].ms += ms;
      c->acc[r.cls].bytes += r.bytes;
    }
    c->evpool.push_back(r.a);
    c->evpool.push_back(r.b);
  }
  c->pending.clear();
}

// Reducing launchers enqueue a streaming kernel and its one-workgroup finishing
// kernel; they take the event `mid_` (recorded between the two) as last argument.
constexpr bool reducing(int cls) { return cls == K_REDUCE || cls == K_PROJNORM || cls == K_FUSED; }

// Launch with optional timing: KL(class, algorithmic HBM bytes, launcher call).  The
// timed interval is the streaming kernel (for a reducing class, up to `mid_`).
#define KL(cls, nbytes, call)                                            \
  do {                                                                   \
    hipEvent_t ea_ = nullptr, eb_ = nullptr;                             \
    if (c->prof) {                                                       \
      ea_ = prof_event(c);                                               \
      eb_ = prof_event(c);                                               \
      if (ea_) (void)hipEventRecord(ea_, c->stream);                     \
    }                                                                    \
    hipEvent_t mid_ = (ea_ && eb_) ? eb_ : nullptr;                      \
    (void)mid_;                                                          \
    hipError_t e_ = (call);                                              \
    if (e_ != hipSuccess) return DCGS2_EDEVICE;                          \
    c->kernels += reducing(cls) ? 2 : 1;                                 \
    if (c->prof && ea_ && eb_) {                                         \
      if (!reducing(cls)) (void)hipEventRecord(eb_, c->stream);          \
      c->pending.push_back({(int)(cls), ea_, eb_, (double)(nbytes)});    \
    }                                                                    \
  } while (0)

// A reducing launch without timing (two kernels).
#define CKR(call)                                  \
  do {                                             \
    hipError_t e_ = (call);                        \
    if (e_ != hipSuccess) return DCGS2_EDEVICE;    \
    c->kernels += 2;                               \
  } while (0)

int dalloc(void** p, size_t bytes) {
  if (hipMalloc(p, bytes) != hipSuccess) { *p = nullptr; return DCGS2_ENOMEM; }
  return DCGS2_OK;
}

void dfree(void* p) { if (p) (void)hipFree(p); }

// First device use of a context: bind the device, create the stream, allocate
// the size-independent workspace.
int ctx_ready(dcgs2_ctx c) {
  if (c->ready) {
    CK(hipSetDevice(c->device));
    return DCGS2_OK;
  }
  int count = 0;
  if (hipGetDeviceCount(&count) != hipSuccess || c->device < 0 || c->device >= count)
    return DCGS2_EDEVICE;
  CK(hipSetDevice(c->device));
  int rc;
  if ((rc = dalloc((void**)&c->P1, sizeof(double) * (size_t)REDUCE_GMAX * LDP))) return rc;
  if ((rc = dalloc((void**)&c->coef, sizeof(double) * (2 * LDC + 8)))) return rc;
  if ((rc = dalloc((void**)&c->pend, sizeof(double) * (2 * LDC + 8)))) return rc;
  const size_t sq = sizeof(double) * (size_t)LDH_MAX * (LDH_MAX + 1);
  if ((rc = dalloc((void**)&c->H, sq))) return rc;
  if ((rc = dalloc((void**)&c->K, sq))) return rc;
  if ((rc = dalloc((void**)&c->Rg, sq))) return rc;
  if ((rc = dalloc((void**)&c->R, sq))) return rc;
  if ((rc = dalloc((void**)&c->Z, sq))) return rc;
  if ((rc = dalloc((void**)&c->Sprev, sizeof(double) * (LDH_MAX + 2)))) return rc;
  if ((rc = dalloc((void**)&c->cs, sizeof(double) * (LDH_MAX + 2)))) return rc;
  if ((rc = dalloc((void**)&c->sn, sizeof(double) * (LDH_MAX + 2)))) return rc;
  if ((rc = dalloc((void**)&c->g, sizeof(double) * (LDH_MAX + 2)))) return rc;
  if ((rc = dalloc((void**)&c->ctrl, sizeof(Ctrl)))) return rc;
  if (hipHostMalloc((void**)&c->ctrl_host, sizeof(Ctrl), hipHostMallocDefault) != hipSuccess)
    return DCGS2_ENOMEM;
  c->ready = true;
  return DCGS2_OK;
}

// Length-m work vectors (w, v, r), grown on demand.
int ensure_vectors(dcgs2_ctx c, int64_t m) {
  if (m <= c->cap_m) return DCGS2_OK;
  CK(hipStreamSynchronize(c->stream));
  dfree(c->w); dfree(c->v); dfree(c->r);
  c->w = c->v = c->r = nullptr;
  c->cap_m = 0;
  const int64_t mm = (m + 63) / 64 * 64;
  int rc;
  if ((rc = dalloc((void**)&c->w, sizeof(double) * mm))) return rc;
  if ((rc = dalloc((void**)&c->v, sizeof(double) * mm))) return rc;
  if ((rc = dalloc((void**)&c->r, sizeof(double) * mm))) return rc;
  c->cap_m = mm;
  return DCGS2_OK;
}

int ensure_basis(dcgs2_ctx c, double** buf, int64_t* cap, int64_t elems) {
  if (elems <= *cap) return DCGS2_OK;
  CK(hipStreamSynchronize(c->stream));
  dfree(*buf);
  *buf = nullptr;
  *cap = 0;
  int rc = dalloc((void**)buf, sizeof(double) * (size_t)elems);
  if (rc) return rc;
  *cap = elems;
  return DCGS2_OK;
}

int64_t pad_ld(int64_t m) { return (m + 63) / 64 * 64; }

int read_ctrl(dcgs2_ctx c, Ctrl* out) {
  CK(hipMemcpyAsync(c->ctrl_host, c->ctrl, sizeof(Ctrl), hipMemcpyDeviceToHost, c->stream));
  CK(hipStreamSynchronize(c->stream));
  *out = *c->ctrl_host;
  if (c->prof) prof_resolve(c);
  return DCGS2_OK;
}

int status_of(const Ctrl& s) {
  switch (s.state) {
    case ST_BREAKDOWN: return DCGS2_BREAKDOWN;
    case ST_NONFINITE: return DCGS2_NONFINITE;
    default: return DCGS2_OK;
  }
}

bool valid_op(const dcgs2_op* A) {
  if (!A || A->m < 2) return false;
  switch (A->kind) {
    case DCGS2_OP_CSR:
      return A->rowptr && A->colind && A->val && A->nnz >= 0 && A->m < INT32_MAX;
    case DCGS2_OP_STENCIL5:
      return A->nx >= 1 && A->ny >= 1 && (int64_t)A->nx * A->ny == A->m && A->m < INT32_MAX;
    case DCGS2_OP_STENCIL7:
      return A->nx >= 1 && A->ny >= 1 && A->nz >= 1 &&
             (int64_t)A->nx * A->ny * A->nz == A->m && A->m < INT32_MAX;
    default:
      return false;
  }
}

DivMagic div_magic(uint32_t d) {
  int l = 0;
  while (l < 32 && ((uint64_t)1 << l) < d) ++l;
  DivMagic g;
  g.mul = (uint32_t)((((uint64_t)1 << 32) * (((uint64_t)1 << l) - d)) / d + 1);
  g.sh1 = l < 1 ? l : 1;
  g.sh2 = l > 1 ? l - 1 : 0;
  return g;
}

OpDev to_dev(const dcgs2_op* A) {
  OpDev o;
  o.kind = A->kind;
  o.m = A->m;
  o.rowptr = A->rowptr; o.colind = A->colind; o.val = A->val; o.nnz = A->nnz;
  o.nx = A->nx; o.ny = A->ny; o.nz = A->kind == DCGS2_OP_STENCIL7 ? A->nz : 1;
  o.c0 = A->c0; o.cxm = A->cxm; o.cxp = A->cxp; o.cym = A->cym; o.cyp = A->cyp;
  o.czm = A->czm; o.czp = A->czp;
  if (A->kind != DCGS2_OP_CSR) {
    o.dx = div_magic((uint32_t)o.nx);
    o.dy = div_magic((uint32_t)o.ny);
  }
  return o;
}

// Algorithmic HBM bytes of one matvec: a stencil reads x once (neighbours come
// from cache) and writes y; CSR also streams its arrays.
double op_bytes(const OpDev& op) {
  const double m = (double)op.m;
  if (op.kind == DCGS2_OP_CSR) return 16.0 * m + 4.0 * (m + 1) + 12.0 * (double)op.nnz;
  return 16.0 * m;
}

// Device workspace of one expansion: the context's buffers, or views into the
// library's fixed scratch array (dcgs2_qr_noalloc).
struct Work {
  double *w = nullptr, *v = nullptr, *r = nullptr;     // length-m vectors
  double* P1 = nullptr;                                 // reduction partials
  int ldp = 0;
  int G = 0;                                            // reduction workgroups (0: sized by m)
  int ldc = 0;                                          // stride of the coefficient block
  double *coef = nullptr, *pend = nullptr;
  double *H = nullptr, *K = nullptr, *Rg = nullptr, *R = nullptr;
  double *Sprev = nullptr, *cs = nullptr, *sn = nullptr, *g = nullptr;
  Ctrl* ctrl = nullptr;
  Ctrl* ctrl_host = nullptr;                            // pinned read-back, or nullptr
};

Work ctx_work(dcgs2_ctx c) {
  Work k;
  k.w = c->w; k.v = c->v; k.r = c->r;
  k.P1 = c->P1; k.ldp = LDP; k.ldc = LDC;
  k.coef = c->coef; k.pend = c->pend;
  k.H = c->H; k.K = c->K; k.Rg = c->Rg; k.R = c->R;
  k.Sprev = c->Sprev; k.cs = c->cs; k.sn = c->sn; k.g = c->g;
  k.ctrl = c->ctrl; k.ctrl_host = c->ctrl_host;
  return k;
}

// Control block into *out: through the pinned buffer when there is one, else
// straight into *out (pageable; the copy completes before the synchronisation).
int read_ctrl(dcgs2_ctx c, const Work& k, Ctrl* out) {
  if (!k.ctrl_host) {
    CK(hipMemcpyAsync(out, k.ctrl, sizeof(Ctrl), hipMemcpyDeviceToHost, c->stream));
    CK(hipStreamSynchronize(c->stream));
    if (c->prof) prof_resolve(c);
    return DCGS2_OK;
  }
  CK(hipMemcpyAsync(k.ctrl_host, k.ctrl, sizeof(Ctrl), hipMemcpyDeviceToHost, c->stream));
  CK(hipStreamSynchronize(c->stream));
  *out = *k.ctrl_host;
  if (c->prof) prof_resolve(c);
  return DCGS2_OK;
}

// One expansion (QR or Arnoldi) over a basis Q.
struct Expansion {
  dcgs2_ctx c;
  bool qr = false;
  bool gmres = false;
  int64_t m = 0;
  void* Q = nullptr;            // basis (double, or float when q32)
  int q32 = 0;
  int64_t ldq = 0;
  const double* B = nullptr;    // QR input columns
  int64_t ldb = 0;
  OpDev op{};                   // Arnoldi operator
  bool one_pass = false;        // QR: fuse update(j) with the reduction of step j+1
  int ldh = 0;                  // leading dimension of H/K/Rg (Arnoldi) or R (QR)
  GridRed gr{};
  Work wk{};                    // device workspace (set by setup_expansion)
  // step records (the steps entry points): step j writes rec + (j - rec_j0) rec_ld
  double* rec = nullptr;
  int rec_j0 = 0, rec_ld = 0;

  FinArgs fin(int kind, int j, int J) const {
    FinArgs f{};
    f.kind = kind; f.qr = qr; f.j = j; f.J = J; f.gmres = gmres; f.ldc = wk.ldc;
    f.ctrl = wk.ctrl; f.coef = wk.coef; f.pend = wk.pend;
    f.H = wk.H; f.K = wk.K; f.ldh = ldh;
    f.R = wk.R; f.ldr = ldh; f.Sprev = wk.Sprev;
    f.Rg = wk.Rg; f.cs = wk.cs; f.sn = wk.sn; f.g = wk.g;
    if (rec && (kind == FIN_STEP || kind == FIN_FALLBACK) && j >= rec_j0)
      f.rec = rec + (int64_t)(j - rec_j0) * rec_ld;
    return f;
  }
  const double* ycol(int j) const { return qr ? B + (int64_t)(j - 1) * ldb : wk.v; }
  double spmv_bytes() const { return op_bytes(op); }

  int enqueue_step(int j, int kind) {
    const int J = j - 2;
    hipStream_t s = c->stream;
    const double vm = 8.0 * (double)m;
    const double qb = q32 ? 4.0 * (double)m : vm;      // bytes of one basis column
    if (!qr && c->tune_matvec_fold && reduce_mv_fits(Q, q32, ldq, wk.w, wk.v, m, op, gr)) {
      // the matvec inside the reduction pass: x read once, y written (not read back)
      KL(K_REDUCE, qb * J + 2 * vm,
         launch_reduce_mv(Q, q32, ldq, J, wk.w, wk.v, m, op, gr, fin(kind, j, J), s, mid_));
    } else {
      if (!qr) KL(K_SPMV, spmv_bytes(), launch_spmv(op, wk.w, nullptr, wk.v, wk.ctrl, s));
      KL(K_REDUCE, qb * J + 2 * vm,
         launch_reduce(Q, q32, ldq, J, wk.w, ycol(j), m, gr, fin(kind, j, J), s, mid_));
    }
    KL(K_UPDATE, qb * (J + 1) + 3 * vm,
       launch_update(Q, q32, ldq, J, wk.w, ycol(j), nullptr, m, wk.coef, wk.ldc, !qr, 0, wk.ctrl, s,
                     c->tune_update_grid));
    return DCGS2_OK;
  }
  int enqueue_fallback(int j) {
    const int J = j - 2;
    hipStream_t s = c->stream;
    const double vm = 8.0 * (double)m;
    const double qb = q32 ? 4.0 * (double)m : vm;
    KL(K_PROJNORM, qb * J + 2 * vm,
       launch_project_norm(Q, q32, ldq, J, wk.w, wk.r, m, gr, fin(FIN_FALLBACK, j, J), s, mid_));
    KL(K_UPDATE, qb * (J + 1) + 4 * vm,
       launch_update(Q, q32, ldq, J, wk.w, ycol(j), wk.r, m, wk.coef, wk.ldc, !qr, 1, wk.ctrl, s,
                     c->tune_update_grid));
    return DCGS2_OK;
  }
  // CGS2 finish of the last column: J final columns already in Q.
  int enqueue_last(int J, int jvirt) {
    hipStream_t s = c->stream;
    const double vm = 8.0 * (double)m;
    const double qb = q32 ? 4.0 * (double)m : vm;
    // with no earlier columns (single-column QR) c is empty: only the norm is reduced,
    // and the breakdown test alpha <= eta * ||a_1|| = eta * alpha reduces to alpha == 0
    // (rho_next keeps its initial 0)
    if (J > 0)
      KL(K_REDUCE, qb * J + vm,
         launch_reduce(Q, q32, ldq, J, wk.w, nullptr, m, gr, fin(FIN_LAST1, jvirt, J), s, mid_));
    KL(K_PROJNORM, qb * J + 2 * vm,
       launch_project_norm(Q, q32, ldq, J, wk.w, wk.r, m, gr, fin(FIN_LAST2, jvirt, J), s, mid_));
    KL(K_SCALE, vm + qb,
       launch_scale_col(Q, q32, ldq, J, wk.r, m, wk.coef, wk.ldc, wk.ctrl, s));
    return DCGS2_OK;
  }
  // One-pass QR schedule for steps j0..j_to: reduce(j0), then fused(j) =
  // update(j) + reduction(j+1) for j < j_to, then update(j_to) fused with the
  // first reduction of the last-column finish.
  int enqueue_one_pass(int j0, int kind0, int j_to, int J_last) {
    hipStream_t s = c->stream;
    const double vm = 8.0 * (double)m;
    if (j0 > j_to) return J_last >= 0 ? enqueue_last(J_last, j_to + 1) : DCGS2_OK;
    const double qb = q32 ? 4.0 * (double)m : vm;
    KL(K_REDUCE, qb * (j0 - 2) + 2 * vm,
       launch_reduce(Q, q32, ldq, j0 - 2, wk.w, ycol(j0), m, gr, fin(kind0, j0, j0 - 2), s, mid_));
    for (int j = j0; j <= j_to; ++j) {
      const int J = j - 2;
      const bool last = (j == j_to);
      if (last && J_last < 0) {
        KL(K_UPDATE, qb * (J + 1) + 3 * vm,
           launch_update(Q, q32, ldq, J, wk.w, ycol(j), nullptr, m, wk.coef, wk.ldc, 0, 0, wk.ctrl,
                         s, c->tune_update_grid));
        break;
      }
      const FinArgs f = last ? fin(FIN_LAST1, j + 1, J + 1) : fin(FIN_STEP, j + 1, J + 1);
      if (J < c->tune_fused_min_j) {
        // a short basis: the separate passes stream better than the tiled fused pass
        KL(K_UPDATE, qb * (J + 1) + 3 * vm,
           launch_update(Q, q32, ldq, J, wk.w, ycol(j), nullptr, m, wk.coef, wk.ldc, 0, 0, wk.ctrl,
                         s, c->tune_update_grid));
        KL(K_REDUCE, qb * (J + 1) + (last ? 1 : 2) * vm,
           launch_reduce(Q, q32, ldq, J + 1, wk.w, last ? nullptr : ycol(j + 1), m, gr, f, s, mid_));
        continue;
      }
      // bytes: Q_{0..J-1}, w, a_j, a_{j+1} read; q, w written (grid sized inside)
      KL(K_FUSED, qb * (J + 1) + vm * (last ? 3 : 4),
         launch_fused_qr(Q, q32, ldq, J, wk.w, ycol(j), last ? nullptr : ycol(j + 1), m,
                         wk.coef, wk.ldc, last ? 1 : 0, c->tune_fused_waves,
                         c->tune_reduce_gmax, c->tune_pair_max_ns, gr, f, s, mid_));
    }
    if (J_last >= 0) {
      KL(K_PROJNORM, qb * J_last + 2 * vm,
         launch_project_norm(Q, q32, ldq, J_last, wk.w, wk.r, m, gr,
                             fin(FIN_LAST2, j_to + 1, J_last), s, mid_));
      KL(K_SCALE, vm + qb,
         launch_scale_col(Q, q32, ldq, J_last, wk.r, m, wk.coef, wk.ldc, wk.ctrl, s));
    }
    return DCGS2_OK;
  }
  // Steps j_from..j_to (the first one of kind first_kind), then the last-column
  // finish with J_last columns when J_last >= 0.  Resolves guard fallbacks.
  // fallback_first: step j_from stopped at its Pythagorean guard (the control block
  // says so); its explicit-norm fallback is enqueued first.
  int run(int j_from, int j_to, int first_kind, int J_last, Ctrl* out,
          bool fallback_first = false) {
    int rc;
    int j0 = j_from;
    int kind0 = first_kind;
    bool pending_fallback = fallback_first;
    for (;;) {
      if (pending_fallback) {
        CKL(launch_set_state(wk.ctrl, ST_RUNNING, c->stream));
        if ((rc = enqueue_fallback(j0))) return rc;
        ++j0;
        kind0 = FIN_STEP;
      }
      if (one_pass) {
        if ((rc = enqueue_one_pass(j0, kind0, j_to, J_last))) return rc;
      } else {
        for (int j = j0; j <= j_to; ++j) {
          if ((rc = enqueue_step(j, j == j0 ? kind0 : FIN_STEP))) return rc;
        }
        if (J_last >= 0 && (rc = enqueue_last(J_last, j_to + 1))) return rc;
      }
      if ((rc = read_ctrl(c, wk, out))) return rc;
      if (out->state != ST_FALLBACK) return DCGS2_OK;
      j0 = out->stop_step;
      pending_fallback = true;
    }
  }
};

int setup_expansion(dcgs2_ctx c, Expansion& e, double thresh, double rho = 0.0) {
  e.c = c;
  if (!e.wk.ctrl) e.wk = ctx_work(c);
  if (e.wk.G > 0)
    e.gr.G = e.wk.G;
  else
    reduce_grid(e.m, c->tune_reduce_gmax, e.q32, &e.gr.G);
  e.gr.P1 = e.wk.P1;
  e.gr.ldp = e.wk.ldp;
  CK(launch_init_ctrl(e.wk.ctrl, c->tau, c->eta, thresh, c->stream, rho));
  c->kernels += 1;
  return DCGS2_OK;
}

void fill_stats(dcgs2_stats* st, const Ctrl& s, int kernels, int status) {
  if (!st) return;
  st->reductions = s.reductions;
  st->pyth_fallbacks = s.fallbacks;
  st->breakdown_step = status == DCGS2_OK ? -1 : s.k;
  st->kernels = kernels;
}

// Copy a device (rows x cols, ld ldd) block to host (ld ldh).
int copy_to_host(dcgs2_ctx c, const double* dev, int ldd, int rows, int cols, double* host,
                 int ldhost) {
  std::vector<double> tmp((size_t)ldd * cols);
  CK(hipMemcpyAsync(tmp.data(), dev, sizeof(double) * tmp.size(), hipMemcpyDeviceToHost,
                    c->stream));
  CK(hipStreamSynchronize(c->stream));
  for (int jj = 0; jj < cols; ++jj)
    for (int i = 0; i < rows; ++i) host[(size_t)jj * ldhost + i] = tmp[(size_t)jj * ldd + i];
  return DCGS2_OK;
}

}  // namespace

int dcgs2::ctx_prepare(dcgs2_ctx c, hipStream_t* stream) {
  if (!c) return DCGS2_EINVAL;
  const int rc = ctx_ready(c);
  if (rc) return rc;
  *stream = c->stream;
  return DCGS2_OK;
}

// =====================================================================================
extern "C" {

const char* dcgs2_status_str(int status) {
  switch (status) {
    case DCGS2_OK: return "ok";
    case DCGS2_EINVAL: return "invalid argument";
    case DCGS2_EDEVICE: return "HIP runtime error";
    case DCGS2_ENOMEM: return "device allocation failed";
    case DCGS2_BREAKDOWN: return "breakdown (invariant subspace or rank deficiency)";
    case DCGS2_NOT_CONVERGED: return "not converged";
    case DCGS2_NONFINITE: return "non-finite value in a reduction";
    default: return "unknown status";
  }
}

int dcgs2_create(dcgs2_ctx* out, int device, void* hip_stream) {
  if (!out || device < 0) return DCGS2_EINVAL;
  dcgs2_ctx c = new (std::nothrow) dcgs2_ctx_s();
  if (!c) return DCGS2_ENOMEM;
  c->device = device;
  c->stream = static_cast<hipStream_t>(hip_stream);
  *out = c;
  return DCGS2_OK;
}

int dcgs2_destroy(dcgs2_ctx c) {
  if (!c) return DCGS2_OK;
  if (c->ready) {
    (void)hipSetDevice(c->device);
    if (c->stream) (void)hipStreamSynchronize(c->stream);
    double* bufs[] = {c->w, c->v, c->r, c->P1, c->coef, c->pend, c->H, c->K, c->Rg,
                      c->R, c->Z, c->Sprev, c->cs, c->sn, c->g, c->Qa, c->Qb, c->rec};
    for (double* b : bufs) dfree(b);
    dfree(c->ctrl);
    prof_resolve(c);
    for (hipEvent_t ev : c->evpool) (void)hipEventDestroy(ev);
    if (c->ctrl_host) (void)hipHostFree(c->ctrl_host);
    if (c->own_stream && c->stream) (void)hipStreamDestroy(c->stream);
  }
  delete c;
  return DCGS2_OK;
}

int dcgs2_set_tolerances(dcgs2_ctx c, double tau, double eta) {
  if (!c || !(tau >= 0.0) || !(eta >= 0.0) || !(eta < 1.0)) return DCGS2_EINVAL;
  c->tau = tau;
  c->eta = eta;
  return DCGS2_OK;
}

int dcgs2_set_tuning(dcgs2_ctx c, int32_t key, int32_t value) {
  if (!c) return DCGS2_EINVAL;
  switch (key) {
    case DCGS2_TUNE_FUSED_WAVES:
      if (value != 8 && value != 16) return DCGS2_EINVAL;
      c->tune_fused_waves = value;
      return DCGS2_OK;
    case DCGS2_TUNE_REDUCE_GRID:
      if (value != 0 && (value < 1 || value > REDUCE_GMAX)) return DCGS2_EINVAL;
      c->tune_reduce_gmax = value;
      return DCGS2_OK;
    case DCGS2_TUNE_FUSED_MIN_J:
      if (value < 0 || value > DCGS2_MAX_N) return DCGS2_EINVAL;
      c->tune_fused_min_j = value;
      return DCGS2_OK;
    case DCGS2_TUNE_BATCH_REDUCE_ROWS:
      if (value < 512 || value > 65536 || (value & (value - 1)) != 0) return DCGS2_EINVAL;
      c->tune_batch_units = value / 2;
      return DCGS2_OK;
    case DCGS2_TUNE_FUSED_PAIR_SLOTS:
      if (value < 0 || value > 16) return DCGS2_EINVAL;
      c->tune_pair_max_ns = value;
      return DCGS2_OK;
    case DCGS2_TUNE_BATCH_DENSE:
      if (value != 0 && value != 1) return DCGS2_EINVAL;
      c->tune_batch_host_dense = value;
      return DCGS2_OK;
    case DCGS2_TUNE_MATVEC_FOLD:
      if (value != 0 && value != 1) return DCGS2_EINVAL;
      c->tune_matvec_fold = value;
      return DCGS2_OK;
    case DCGS2_TUNE_UPDATE_GRID:
      if (value < 0 || value > 65536) return DCGS2_EINVAL;
      c->tune_update_grid = value;
      return DCGS2_OK;
    default:
      return DCGS2_EINVAL;
  }
}

int dcgs2_get_tuning(dcgs2_ctx c, int32_t key, int32_t* value) {
  if (!c || !value) return DCGS2_EINVAL;
  switch (key) {
    case DCGS2_TUNE_FUSED_WAVES: *value = c->tune_fused_waves; return DCGS2_OK;
    case DCGS2_TUNE_REDUCE_GRID: *value = c->tune_reduce_gmax; return DCGS2_OK;
    case DCGS2_TUNE_FUSED_MIN_J: *value = c->tune_fused_min_j; return DCGS2_OK;
    case DCGS2_TUNE_BATCH_REDUCE_ROWS: *value = 2 * c->tune_batch_units; return DCGS2_OK;
    case DCGS2_TUNE_FUSED_PAIR_SLOTS: *value = c->tune_pair_max_ns; return DCGS2_OK;
    case DCGS2_TUNE_BATCH_DENSE: *value = c->tune_batch_host_dense; return DCGS2_OK;
    case DCGS2_TUNE_MATVEC_FOLD: *value = c->tune_matvec_fold; return DCGS2_OK;
    case DCGS2_TUNE_UPDATE_GRID: *value = c->tune_update_grid; return DCGS2_OK;
    default: return DCGS2_EINVAL;
  }
}

int dcgs2_set_qr_schedule(dcgs2_ctx c, int one_pass) {
  if (!c || (one_pass != 0 && one_pass != 1)) return DCGS2_EINVAL;
  c->qr_one_pass = one_pass == 1;
  return DCGS2_OK;
}

int dcgs2_profile_enable(dcgs2_ctx c, int enable) {
  if (!c) return DCGS2_EINVAL;
  c->prof = enable != 0;
  return DCGS2_OK;
}

int dcgs2_profile_read(dcgs2_ctx c, dcgs2_kernel_stat* out, int32_t max_entries, int32_t reset) {
  if (!c || (max_entries > 0 && !out) || max_entries < 0) return DCGS2_EINVAL;
  if (c->ready) {
    CK(hipSetDevice(c->device));
    CK(hipStreamSynchronize(c->stream));
    prof_resolve(c);
  }
  const int n = std::min<int>(max_entries, K_NCLASS);
  for (int i = 0; i < n; ++i) {
    std::memset(&out[i], 0, sizeof(out[i]));
    std::snprintf(out[i].name, sizeof(out[i].name), "%s", kClassName[i]);
    out[i].launches = c->acc[i].launches;
    out[i].total_ms = c->acc[i].ms;
    out[i].bytes = c->acc[i].bytes;
  }
  if (reset)
    for (auto& a : c->acc) a = dcgs2_ctx_s::ProfAcc();
  return K_NCLASS;
}

int dcgs2_apply(dcgs2_ctx c, const dcgs2_op* A, const double* x, double* y) {
  if (!c || !valid_op(A) || !x || !y) return DCGS2_EINVAL;
  int rc;
  if ((rc = ctx_ready(c))) return rc;
  CK(launch_spmv(to_dev(A), x, nullptr, y, nullptr, c->stream));
  CK(hipStreamSynchronize(c->stream));
  return DCGS2_OK;
}

static int qr_impl(dcgs2_ctx c, int64_t m, int32_t n, const double* B, int64_t ldb, void* Q,
                   int q32, int64_t ldq, double* R_host, int32_t ldr, dcgs2_stats* st) {
  if (!c || m < 1 || n < 1 || n > DCGS2_MAX_N || (int64_t)n > m || !B || !Q || !R_host ||
      ldb < m || ldq < m || ldr < n)
    return DCGS2_EINVAL;
  int rc;
  if ((rc = ctx_ready(c))) return rc;
  if ((rc = ensure_vectors(c, m))) return rc;
  c->kernels = 0;
  Expansion e;
  e.qr = true;
  e.m = m;
  e.Q = Q; e.q32 = q32; e.ldq = ldq; e.B = B; e.ldb = ldb;
  e.ldh = n;
  // the one-pass kernel addresses a column with 32-bit byte offsets
  e.one_pass = c->qr_one_pass && n - 2 <= FUSED_QR_MAX_J &&
               (double)m * 8.0 < 2147483648.0;
  if ((rc = setup_expansion(c, e, 0.0))) return rc;
  CKL(launch_fill(c->R, (int64_t)n * n, 0.0, c->stream));
  CKL(launch_copy(c->w, B, m, c->stream));               // w_1 = a_1
  Ctrl s{};
  if ((rc = e.run(2, n, FIN_STEP, n - 1, &s))) return rc;
  const int status = status_of(s);
  if ((rc = copy_to_host(c, c->R, n, n, n, R_host, ldr))) return rc;
  fill_stats(st, s, c->kernels, status);
  return status;
}

static int arnoldi_impl(dcgs2_ctx c, const dcgs2_op* A, const double* r0, int32_t n, void* Q,
                        int q32, int64_t ldq, double* H_host, int32_t ldh, dcgs2_stats* st) {
  if (!c || !valid_op(A) || !r0 || !Q || !H_host || n < 1 || n > DCGS2_MAX_N ||
      (int64_t)n >= A->m || ldq < A->m || ldh < n + 1)
    return DCGS2_EINVAL;
  int rc;
  if ((rc = ctx_ready(c))) return rc;
  const int64_t m = A->m;
  if ((rc = ensure_vectors(c, m))) return rc;
  c->kernels = 0;
  Expansion e;
  e.qr = false;
  e.m = m;
  e.Q = Q; e.q32 = q32; e.ldq = ldq;
  e.op = to_dev(A);
  e.ldh = n + 1;
  if ((rc = setup_expansion(c, e, 0.0))) return rc;
  CKL(launch_fill(c->H, (int64_t)(n + 1) * (n + 1), 0.0, c->stream));
  CKL(launch_fill(c->K, (int64_t)(n + 1) * (n + 1), 0.0, c->stream));
  CKL(launch_copy(c->w, r0, m, c->stream));              // w_1 = r0 (unnormalised)
  Ctrl s{};
  if ((rc = e.run(2, n + 1, FIN_STEP, n, &s))) return rc;
  const int status = status_of(s);
  if ((rc = copy_to_host(c, c->H, n + 1, n + 1, n, H_host, ldh))) return rc;
  fill_stats(st, s, c->kernels, status);
  return status;
}

int dcgs2_qr(dcgs2_ctx c, int64_t m, int32_t n, const double* B, int64_t ldb, double* Q,
             int64_t ldq, double* R_host, int32_t ldr, dcgs2_stats* st) {
  return qr_impl(c, m, n, B, ldb, Q, 0, ldq, R_host, ldr, st);
}

int dcgs2_qr_q32(dcgs2_ctx c, int64_t m, int32_t n, const double* B, int64_t ldb, float* Q,
                 int64_t ldq, double* R_host, int32_t ldr, dcgs2_stats* st) {
  return qr_impl(c, m, n, B, ldb, Q, 1, ldq, R_host, ldr, st);
}

int dcgs2_arnoldi(dcgs2_ctx c, const dcgs2_op* A, const double* r0, int32_t n, double* Q,
                  int64_t ldq, double* H_host, int32_t ldh, dcgs2_stats* st) {
  return arnoldi_impl(c, A, r0, n, Q, 0, ldq, H_host, ldh, st);
}

int dcgs2_arnoldi_q32(dcgs2_ctx c, const dcgs2_op* A, const double* r0, int32_t n, float* Q,
                      int64_t ldq, double* H_host, int32_t ldh, dcgs2_stats* st) {
  return arnoldi_impl(c, A, r0, n, Q, 1, ldq, H_host, ldh, st);
}

}  // extern "C"

namespace {

// Host block (rows x cols, leading dimension ldhost) into a zero-padded device block of
// leading dimension ld.
int put_small(dcgs2_ctx c, double* dev, int ld, int rows, int cols, const double* host,
              int ldhost) {
  std::vector<double> tmp((size_t)ld * cols, 0.0);
  for (int jj = 0; jj < cols; ++jj)
    for (int i = 0; i < rows; ++i) tmp[(size_t)jj * ld + i] = host[(size_t)jj * ldhost + i];
  CK(hipMemcpyAsync(dev, tmp.data(), sizeof(double) * tmp.size(), hipMemcpyHostToDevice,
                    c->stream));
  CK(hipStreamSynchronize(c->stream));
  return DCGS2_OK;
}

// Step records of steps j0..j1: one record of 3 j1 + 1 doubles per step (the largest,
// step j1, has 2 j1 reduced values, j1 - 1 coefficients, alpha and rho), NaN-filled
// so that a step that did not run is visible.
int steps_records(dcgs2_ctx c, Expansion& e, int j0, int j1) {
  const int ld = 3 * j1 + 1;
  const int64_t need = (int64_t)(j1 - j0 + 1) * ld;
  if (need > c->cap_rec) {
    CK(hipStreamSynchronize(c->stream));
    dfree(c->rec);
    c->rec = nullptr;
    c->cap_rec = 0;
    const int rc = dalloc((void**)&c->rec, sizeof(double) * (size_t)need);
    if (rc) return rc;
    c->cap_rec = need;
  }
  CKL(launch_fill(c->rec, need, NAN, c->stream));
  e.rec = c->rec;
  e.rec_j0 = j0;
  e.rec_ld = ld;
  return DCGS2_OK;
}

int read_records(dcgs2_ctx c, int j0, int j1, double* rec_host) {
  const size_t n = (size_t)(j1 - j0 + 1) * (3 * j1 + 1);
  CK(hipMemcpyAsync(rec_host, c->rec, sizeof(double) * n, hipMemcpyDeviceToHost, c->stream));
  CK(hipStreamSynchronize(c->stream));
  return DCGS2_OK;
}

}  // namespace

extern "C" {

int dcgs2_arnoldi_steps(dcgs2_ctx c, const dcgs2_op* A, int32_t j0, int32_t j1, double* Q,
                        int64_t ldq, double* w, double* H_host, double* K_host, int32_t ldh,
                        double rho, double* rec_host, dcgs2_stats* st) {
  if (!c || !valid_op(A) || !Q || !w || !H_host || !K_host || j0 < 2 || j1 < j0 ||
      j1 > DCGS2_MAX_N + 1 || (int64_t)j1 > A->m || ldq < A->m || ldh < j1 ||
      !(rho >= 0.0) || !std::isfinite(rho))
    return DCGS2_EINVAL;
  int rc;
  if ((rc = ctx_ready(c))) return rc;
  const int64_t m = A->m;
  if ((rc = ensure_vectors(c, m))) return rc;
  c->kernels = 0;
  Expansion e;
  e.qr = false;
  e.m = m;
  e.Q = Q; e.q32 = 0; e.ldq = ldq;
  e.op = to_dev(A);
  e.ldh = j1;                                  // H, K rows 0..j1-2 and columns 0..j1-2
  if (rec_host && (rc = steps_records(c, e, j0, j1))) return rc;
  if ((rc = setup_expansion(c, e, 0.0, rho))) return rc;
  if ((rc = put_small(c, c->H, j1, j1, j1 - 1, H_host, ldh))) return rc;
  if ((rc = put_small(c, c->K, j1, j1, j1 - 1, K_host, ldh))) return rc;
  CKL(launch_copy(c->w, w, m, c->stream));
  Ctrl s{};
  if ((rc = e.run(j0, j1, FIN_STEP, -1, &s))) return rc;
  const int status = status_of(s);
  if ((rc = copy_to_host(c, c->H, j1, j1, j1 - 1, H_host, ldh))) return rc;
  if ((rc = copy_to_host(c, c->K, j1, j1, j1 - 1, K_host, ldh))) return rc;
  CKL(launch_copy(w, c->w, m, c->stream));
  CK(hipStreamSynchronize(c->stream));
  if (rec_host && (rc = read_records(c, j0, j1, rec_host))) return rc;
  fill_stats(st, s, c->kernels, status);
  return status;
}

int dcgs2_qr_steps(dcgs2_ctx c, int64_t m, int32_t j0, int32_t j1, const double* B, int64_t ldb,
                   double* Q, int64_t ldq, double* w, double* R_host, int32_t ldr,
                   double* S_host, double rho, double* rec_host, dcgs2_stats* st) {
  if (!c || m < 2 || j0 < 2 || j1 < j0 || j1 > DCGS2_MAX_N || (int64_t)j1 > m || !B || !Q ||
      !w || !R_host || !S_host || ldb < m || ldq < m || ldr < j1 - 1 || !(rho >= 0.0) ||
      !std::isfinite(rho))
    return DCGS2_EINVAL;
  int rc;
  if ((rc = ctx_ready(c))) return rc;
  if ((rc = ensure_vectors(c, m))) return rc;
  c->kernels = 0;
  Expansion e;
  e.qr = true;
  e.m = m;
  e.Q = Q; e.q32 = 0; e.ldq = ldq; e.B = B; e.ldb = ldb;
  e.ldh = j1;                                  // R rows 0..j1-2 and columns 0..j1-2
  e.one_pass = c->qr_one_pass && j1 - 2 <= FUSED_QR_MAX_J && (double)m * 8.0 < 2147483648.0;
  if (rec_host && (rc = steps_records(c, e, j0, j1))) return rc;
  if ((rc = setup_expansion(c, e, 0.0, rho))) return rc;
  CKL(launch_fill(c->R, (int64_t)j1 * j1, 0.0, c->stream));
  if (j0 > 2) {
    CK(hipMemcpyAsync(c->Sprev, S_host, sizeof(double) * (j0 - 2), hipMemcpyHostToDevice,
                      c->stream));
  }
  CKL(launch_copy(c->w, w, m, c->stream));
  Ctrl s{};
  if ((rc = e.run(j0, j1, FIN_STEP, -1, &s))) return rc;
  const int status = status_of(s);
  std::vector<double> Rd((size_t)j1 * (j1 - 1));
  if ((rc = copy_to_host(c, c->R, j1, j1, j1 - 1, Rd.data(), j1))) return rc;
  for (int jj = j0 - 2; jj <= j1 - 2; ++jj)
    for (int i = 0; i <= jj; ++i) R_host[(size_t)jj * ldr + i] = Rd[(size_t)jj * j1 + i];
  CK(hipMemcpyAsync(S_host, c->Sprev, sizeof(double) * (j1 - 1), hipMemcpyDeviceToHost,
                    c->stream));
  CKL(launch_copy(w, c->w, m, c->stream));
  CK(hipStreamSynchronize(c->stream));
  if (rec_host && (rc = read_records(c, j0, j1, rec_host))) return rc;
  fill_stats(st, s, c->kernels, status);
  return status;
}

int dcgs2_qr_noalloc(dcgs2_ctx c, int64_t m, int32_t n, const double* B, int64_t ldb,
                     double* Q, int64_t ldq, double* R_host, int32_t ldr, dcgs2_stats* st) {
  if (!c || m < 1 || n < 1 || n > DCGS2_MAX_N || (int64_t)n > m || !B || !Q || !R_host ||
      ldb < m || ldq < m || ldr < n)
    return DCGS2_EINVAL;
  if (m > NOALLOC_MAX_M || n > NOALLOC_MAX_N) return DCGS2_EINVAL;   // beyond the scratch
  CK(hipSetDevice(c->device));
  double* base = nullptr;
  size_t cap = 0;
  CK(noalloc_scratch(c->device, &base, &cap));
  // views into the fixed scratch (the layout noalloc_scratch documents)
  auto region = [](size_t d) { return (d + 63) / 64 * 64; };
  Work k;
  double* p = base;
  k.w = p; p += region(NOALLOC_MAX_M);
  k.r = p; p += region(NOALLOC_MAX_M);
  k.P1 = p; p += region((size_t)REDUCE_GMAX * NOALLOC_LDP);
  k.ldp = NOALLOC_LDP;
  k.ldc = LDC;
  k.coef = p; p += region(NOALLOC_LDCOEF);
  k.pend = p; p += region(NOALLOC_LDCOEF);
  k.R = p; p += region((size_t)NOALLOC_MAX_N * NOALLOC_MAX_N);
  k.Sprev = p; p += region(NOALLOC_MAX_N + 2);
  k.ctrl = reinterpret_cast<Ctrl*>(p); p += region(sizeof(Ctrl) / 8 + 1);
  if ((size_t)(p - base) > cap) return DCGS2_EDEVICE;      // layout and array disagree
  // kernel timing records host events and is not used here
  struct ProfOff {
    dcgs2_ctx c; bool was;
    ~ProfOff() { c->prof = was; }
  } prof_off{c, c->prof};
  c->prof = false;
  c->kernels = 0;
  Expansion e;
  e.qr = true;
  e.m = m;
  e.Q = Q; e.q32 = 0; e.ldq = ldq; e.B = B; e.ldb = ldb;
  e.ldh = n;
  e.wk = k;
  e.one_pass = c->qr_one_pass && n - 2 <= FUSED_QR_MAX_J && (double)m * 8.0 < 2147483648.0;
  int rc;
  if ((rc = setup_expansion(c, e, 0.0))) return rc;
  CKL(launch_fill(k.R, (int64_t)n * n, 0.0, c->stream));
  CKL(launch_copy(k.w, B, m, c->stream));                 // w_1 = a_1
  Ctrl s{};
  if ((rc = e.run(2, n, FIN_STEP, n - 1, &s))) return rc;
  const int status = status_of(s);
  CK(hipMemcpy2DAsync(R_host, sizeof(double) * (size_t)ldr, k.R, sizeof(double) * (size_t)n,
                      sizeof(double) * (size_t)n, (size_t)n, hipMemcpyDeviceToHost, c->stream));
  CK(hipStreamSynchronize(c->stream));
  fill_stats(st, s, c->kernels, status);
  return status;
}

int cgs2_qr(dcgs2_ctx c, int64_t m, int32_t n, const double* B, int64_t ldb, double* Q,
            int64_t ldq, double* R_host, int32_t ldr, dcgs2_stats* st) {
  if (!c || m < 1 || n < 1 || n > DCGS2_MAX_N || (int64_t)n > m || !B || !Q || !R_host ||
      ldb < m || ldq < m || ldr < n)
    return DCGS2_EINVAL;
  int rc;
  if ((rc = ctx_ready(c))) return rc;
  if ((rc = ensure_vectors(c, m))) return rc;
  c->kernels = 0;
  Expansion e;
  e.qr = true;
  e.m = m;
  e.Q = Q; e.q32 = 0; e.ldq = ldq; e.B = B; e.ldb = ldb;
  e.ldh = n;
  if ((rc = setup_expansion(c, e, 0.0))) return rc;
  CKL(launch_fill(c->R, (int64_t)n * n, 0.0, c->stream));
  hipStream_t s = c->stream;
  const double vm = 8.0 * (double)m;
  // Alg. cgs2, column j (0-based): S = Q^T a; w = a - Q S; C = Q^T w; u = w - Q C;
  // alpha = ||u||; q = u/alpha; R_{:,j} = [S + C; alpha] -- three reductions.
  for (int j = 0; j < n; ++j) {
    const double* a = B + (int64_t)j * ldb;
    const double* x = a;
    if (j > 0) {
      KL(K_REDUCE, vm * (j + 1),
         launch_reduce(Q, 0, ldq, j, a, nullptr, m, e.gr, e.fin(FIN_CGS2_S, j + 2, j), s, mid_));
      KL(K_PROJNORM, vm * (j + 2),
         launch_project_norm(Q, 0, ldq, j, a, c->w, m, e.gr, e.fin(FIN_NONE, j + 2, j), s, mid_));
      KL(K_REDUCE, vm * (j + 1),
         launch_reduce(Q, 0, ldq, j, c->w, nullptr, m, e.gr, e.fin(FIN_LAST1, j + 2, j), s, mid_));
      x = c->w;
    }
    KL(K_PROJNORM, vm * (j + 2),
       launch_project_norm(Q, 0, ldq, j, x, c->r, m, e.gr, e.fin(FIN_LAST2, j + 2, j), s, mid_));
    KL(K_SCALE, vm * 2, launch_scale_col(Q, 0, ldq, j, c->r, m, c->coef, LDC, c->ctrl, s));
  }
  Ctrl sc{};
  if ((rc = read_ctrl(c, &sc))) return rc;
  const int status = status_of(sc);
  if ((rc = copy_to_host(c, c->R, n, n, n, R_host, ldr))) return rc;
  fill_stats(st, sc, c->kernels, status);
  return status;
}

int mgs_qr(dcgs2_ctx c, int64_t m, int32_t n, const double* B, int64_t ldb, double* Q,
           int64_t ldq, double* R_host, int32_t ldr, dcgs2_stats* st) {
  if (!c || m < 1 || n < 1 || n > DCGS2_MAX_N || (int64_t)n > m || !B || !Q || !R_host ||
      ldb < m || ldq < m || ldr < n)
    return DCGS2_EINVAL;
  int rc;
  if ((rc = ctx_ready(c))) return rc;
  if ((rc = ensure_vectors(c, m))) return rc;
  c->kernels = 0;
  Expansion e;
  e.qr = true;
  e.m = m;
  e.Q = Q; e.q32 = 0; e.ldq = ldq; e.B = B; e.ldb = ldb;
  e.ldh = n;
  if ((rc = setup_expansion(c, e, 0.0))) return rc;
  CKL(launch_fill(c->R, (int64_t)n * n, 0.0, c->stream));
  hipStream_t s = c->stream;
  const double vm = 8.0 * (double)m;
  // classical column-by-column MGS (the paper's Sec. 2 baseline): for column j,
  // w = a_j; for k < j: r = q_k^T w (one reduction), w -= r q_k; alpha = ||w||
  // (one reduction); q_j = w / alpha -- n(n+1)/2 reductions in all.
  for (int j = 0; j < n; ++j) {
    CKL(launch_copy(c->w, B + (int64_t)j * ldb, m, s));
    for (int k = 0; k < j; ++k) {
      const double* qk = Q + (int64_t)k * ldq;
      KL(K_REDUCE, vm * 2,
         launch_reduce(qk, 0, ldq, 1, c->w, nullptr, m, e.gr, e.fin(FIN_MGS_DOT, j, k), s, mid_));
      // w -= r q_k in place (the pass also forms ||w||^2 partials, unused)
      KL(K_PROJNORM, vm * 3,
         launch_project_norm(qk, 0, ldq, 1, c->w, c->w, m, e.gr, e.fin(FIN_NONE, j, 1), s, mid_));
    }
    KL(K_REDUCE, vm,
       launch_reduce(Q, 0, ldq, 0, c->w, nullptr, m, e.gr, e.fin(FIN_MGS_NORM, j, 0), s, mid_));
    KL(K_SCALE, vm * 2, launch_scale_col(Q, 0, ldq, j, c->w, m, c->coef, LDC, c->ctrl, s));
  }
  Ctrl sc{};
  if ((rc = read_ctrl(c, &sc))) return rc;
  const int status = status_of(sc);
  if ((rc = copy_to_host(c, c->R, n, n, n, R_host, ldr))) return rc;
  fill_stats(st, sc, c->kernels, status);
  return status;
}

int dcgs2_set_basis_precision(dcgs2_ctx c, int bits) {
  if (!c || (bits != 32 && bits != 64)) return DCGS2_EINVAL;
  c->basis_q32 = bits == 32;
  return DCGS2_OK;
}

int gmres_solve(dcgs2_ctx c, const dcgs2_op* A, const double* b, double* x, int32_t restart,
                double rtol, int32_t max_iters, dcgs2_gmres_info* info) {
  if (!c || !valid_op(A) || !b || !x || restart < 1 || restart > DCGS2_MAX_N ||
      (int64_t)restart >= A->m || !(rtol > 0.0) || max_iters < 0)
    return DCGS2_EINVAL;
  int rc;
  if ((rc = ctx_ready(c))) return rc;
  const int64_t m = A->m;
  if ((rc = ensure_vectors(c, m))) return rc;
  const int64_t ldq = pad_ld(m);
  if ((rc = ensure_basis(c, &c->Qa, &c->cap_qa, ldq * (restart + 1)))) return rc;
  c->kernels = 0;
  dcgs2_gmres_info inf{};
  Expansion e;
  e.qr = false;
  e.gmres = true;
  e.m = m;
  e.Q = c->Qa; e.q32 = c->basis_q32; e.ldq = ldq;
  e.op = to_dev(A);
  e.ldh = restart + 1;
  // ||b||
  if ((rc = setup_expansion(c, e, 0.0))) return rc;
  Ctrl s{};
  CKR(launch_reduce(nullptr, 0, ldq, 0, b, nullptr, m, e.gr, e.fin(FIN_NORM, 0, 0), c->stream));
  if ((rc = read_ctrl(c, &s))) return rc;
  const double bnorm = std::sqrt(s.norm2);
  int status = DCGS2_OK;
  if (!std::isfinite(bnorm)) {
    status = DCGS2_NONFINITE;
  } else if (bnorm == 0.0) {
    CKL(launch_fill(x, m, 0.0, c->stream));
    CK(hipStreamSynchronize(c->stream));
  } else {
    std::vector<double> Rh, gh, y;
    for (;;) {
      // r = b - A x into w (w_1 of the cycle), then ||r||
      if ((rc = setup_expansion(c, e, rtol * bnorm))) return rc;
      KL(K_SPMV, op_bytes(e.op) + 8.0 * m, launch_spmv(e.op, x, b, c->w, nullptr, c->stream));
      CKR(launch_reduce(nullptr, 0, ldq, 0, c->w, nullptr, m, e.gr, e.fin(FIN_NORM, 0, 0),
                        c->stream));
      if ((rc = read_ctrl(c, &s))) return rc;
      inf.relres_true = std::sqrt(s.norm2) / bnorm;
      if (!std::isfinite(inf.relres_true)) { status = DCGS2_NONFINITE; break; }
      if (inf.relres_true <= rtol) { status = DCGS2_OK; break; }
      if (inf.iters >= max_iters) { status = DCGS2_NOT_CONVERGED; break; }
      const int nc = std::min(restart, max_iters - inf.iters);
      inf.cycles += 1;
      if ((rc = setup_expansion(c, e, rtol * bnorm))) return rc;
      e.ldh = nc + 1;
      CKL(launch_fill(c->H, (int64_t)(nc + 1) * (nc + 1), 0.0, c->stream));
      CKL(launch_fill(c->K, (int64_t)(nc + 1) * (nc + 1), 0.0, c->stream));
      CKL(launch_fill(c->g, nc + 2, 0.0, c->stream));
      if ((rc = e.run(2, nc + 1, FIN_STEP, nc, &s))) return rc;
      inf.st.reductions += s.reductions;
      inf.st.pyth_fallbacks += s.fallbacks;
      if (s.state == ST_NONFINITE) { status = DCGS2_NONFINITE; break; }
      const int steps = (s.state == ST_RUNNING) ? nc : std::min(s.stop_step - 1, nc);
      inf.iters += steps;
      const int k = s.k;
      inf.relres_est = s.resid_est / bnorm;
      if (k <= 0) { status = DCGS2_BREAKDOWN; break; }
      // y = R_k^{-1} g_{1:k} (back substitution on the rotated Hessenberg matrix)
      const int ld = nc + 1;
      Rh.assign((size_t)ld * k, 0.0);
      gh.assign(k, 0.0);
      CK(hipMemcpyAsync(Rh.data(), c->Rg, sizeof(double) * Rh.size(), hipMemcpyDeviceToHost,
                        c->stream));
      CK(hipMemcpyAsync(gh.data(), c->g, sizeof(double) * k, hipMemcpyDeviceToHost, c->stream));
      CK(hipStreamSynchronize(c->stream));
      y.assign(k, 0.0);
      for (int i = k - 1; i >= 0; --i) {
        double sum = gh[i];
        for (int jj = i + 1; jj < k; ++jj) sum -= Rh[(size_t)jj * ld + i] * y[jj];
        y[i] = sum / Rh[(size_t)i * ld + i];
      }
      CK(hipMemcpyAsync(c->Z, y.data(), sizeof(double) * k, hipMemcpyHostToDevice, c->stream));
      KL(K_TSGEMM, (e.q32 ? 4.0 : 8.0) * m * k + 16.0 * m,
         launch_tsgemm(c->Qa, e.q32, ldq, k, c->Z, k, 1, x, 0, m, m, 1, c->stream));
    }
  }
  inf.status = status;
  inf.st.kernels = c->kernels;
  inf.st.breakdown_step = -1;
  if (info) *info = inf;
  return status;
}

int krylov_schur_eigs(dcgs2_ctx c, const dcgs2_op* A, int32_t nev, int32_t ncv, int32_t keep,
                      double tol, int32_t max_restarts, const double* v0, double* eig_re,
                      double* eig_im, dcgs2_ks_info* info) {
  if (!c || !valid_op(A) || !v0 || !eig_re || !eig_im || nev < 1 || keep <= nev ||
      ncv <= keep || ncv > DCGS2_MAX_N || (int64_t)ncv >= A->m || !(tol > 0.0) ||
      max_restarts < 0)
    return DCGS2_EINVAL;
  int rc;
  if ((rc = ctx_ready(c))) return rc;
  const int64_t m = A->m;
  if ((rc = ensure_vectors(c, m))) return rc;
  const int64_t ldq = pad_ld(m);
  const int p = ncv;
  if ((rc = ensure_basis(c, &c->Qa, &c->cap_qa, ldq * (p + 1)))) return rc;
  if ((rc = ensure_basis(c, &c->Qb, &c->cap_qb, ldq * (p + 1)))) return rc;
  c->kernels = 0;
  dcgs2_ks_info inf{};
  Expansion e;
  e.qr = false;
  e.m = m;
  e.Q = c->Qa; e.q32 = c->basis_q32; e.ldq = ldq;
  e.op = to_dev(A);
  e.ldh = p + 1;
  const int ld = p + 1;
  if ((rc = setup_expansion(c, e, 0.0))) return rc;
  CKL(launch_fill(c->H, (int64_t)ld * ld, 0.0, c->stream));
  CKL(launch_fill(c->K, (int64_t)ld * ld, 0.0, c->stream));
  CKL(launch_copy(c->w, v0, m, c->stream));
  Ctrl s{};
  if ((rc = e.run(2, p + 1, FIN_STEP, p, &s))) return rc;
  inf.matvecs = p;
  inf.st.reductions = s.reductions;
  inf.st.pyth_fallbacks = s.fallbacks;
  int status = status_of(s);
  std::vector<double> Hh((size_t)ld * p), T((size_t)p * p), Zm((size_t)p * p), Hn((size_t)ld * p);
  std::vector<double> ere(p), eim(p);
  const double CUT_GAP = 1e-8;
  while (status == DCGS2_OK) {
    if ((rc = copy_to_host(c, c->H, ld, ld, p, Hh.data(), ld))) return rc;
    const double h = Hh[(size_t)(p - 1) * ld + p];
    for (int jj = 0; jj < p; ++jj)
      for (int i = 0; i < p; ++i) T[(size_t)jj * p + i] = Hh[(size_t)jj * ld + i];
    if (real_schur(p, T.data(), p, Zm.data(), p) != 0) { status = DCGS2_NOT_CONVERGED; break; }
    // convergence test on the leading nev (cut-adjusted) Schur vectors
    const int kn = reorder_schur_by_magnitude(p, T.data(), p, Zm.data(), p, nev, CUT_GAP);
    if (kn < 0) { status = DCGS2_NOT_CONVERGED; break; }
    schur_eigenvalues(p, T.data(), p, ere.data(), eim.data());
    double bn = 0.0, tmin = INFINITY;
    for (int i = 0; i < kn; ++i) {
      const double bi = h * Zm[(size_t)i * p + (p - 1)];
      bn += bi * bi;
      tmin = std::min(tmin, std::hypot(ere[i], eim[i]));
    }
    inf.resid = std::sqrt(bn) / tmin;
    for (int i = 0; i < nev; ++i) { eig_re[i] = ere[i]; eig_im[i] = eim[i]; }
    if (inf.resid <= tol) { inf.nconv = kn; break; }
    if (inf.restarts >= max_restarts) { status = DCGS2_NOT_CONVERGED; break; }
    // truncate to the leading `keep` Schur vectors
    const int k = reorder_schur_by_magnitude(p, T.data(), p, Zm.data(), p, keep, CUT_GAP);
    if (k < 0 || k >= p) { status = DCGS2_NOT_CONVERGED; break; }
    CK(hipMemcpyAsync(c->Z, Zm.data(), sizeof(double) * (size_t)p * k, hipMemcpyHostToDevice,
                      c->stream));
    const int64_t es = e.q32 ? 4 : 8;                                         // element bytes
    char* qa = reinterpret_cast<char*>(c->Qa);
    char* qbuf = reinterpret_cast<char*>(c->Qb);
    KL(K_TSGEMM, (double)es * m * (p + k),
       launch_tsgemm(c->Qa, e.q32, ldq, p, c->Z, p, k, c->Qb, e.q32, ldq, m, 0, c->stream));
    CKL(launch_convert(qbuf + es * k * ldq, e.q32, qa + es * p * ldq, e.q32, m, c->stream));
    CKL(launch_convert(c->w, 0, qa + es * p * ldq, e.q32, m, c->stream));    // w = q_{k+1}
    std::fill(Hn.begin(), Hn.end(), 0.0);
    for (int jj = 0; jj < k; ++jj) {
      for (int i = 0; i < k; ++i) Hn[(size_t)jj * ld + i] = T[(size_t)jj * p + i];
      Hn[(size_t)jj * ld + k] = h * Zm[(size_t)jj * p + (p - 1)];
    }
    CKL(launch_fill(c->K, (int64_t)ld * ld, 0.0, c->stream));
    CK(hipMemcpyAsync(c->H, Hn.data(), sizeof(double) * Hn.size(), hipMemcpyHostToDevice,
                      c->stream));
    std::swap(c->Qa, c->Qb);
    std::swap(c->cap_qa, c->cap_qb);
    e.Q = c->Qa;
    inf.restarts += 1;
    if ((rc = setup_expansion(c, e, 0.0))) return rc;
    if ((rc = e.run(k + 2, p + 1, FIN_RESTART, p, &s))) return rc;
    inf.matvecs += p - k;
    inf.st.reductions += s.reductions;
    inf.st.pyth_fallbacks += s.fallbacks;
    status = status_of(s);
  }
  inf.status = status;
  inf.st.kernels = c->kernels;
  inf.st.breakdown_step = status == DCGS2_OK ? -1 : s.k;
  if (info) *info = inf;
  return status;
}

}  // extern "C"

extern "C" int dcgs2_guess_guard(dcgs2_ctx c, const dcgs2_op* A, const double* b, double* x0,
                                 double max_ratio, int32_t* kept, double* ratio) {
  if (!c || !valid_op(A) || !b || !x0 || !kept || !(max_ratio > 0.0)) return DCGS2_EINVAL;
  int rc;
  if ((rc = ctx_ready(c))) return rc;
  const int64_t m = A->m;
  if ((rc = ensure_vectors(c, m))) return rc;
  Expansion e;
  e.qr = false;
  e.m = m;
  e.op = to_dev(A);
  Ctrl s{};
  // ||b||^2, then ||b - A x0||^2 (r into w)
  if ((rc = setup_expansion(c, e, 0.0))) return rc;
  CKR(launch_reduce(nullptr, 0, m, 0, b, nullptr, m, e.gr, e.fin(FIN_NORM, 0, 0), c->stream));
  if ((rc = read_ctrl(c, &s))) return rc;
  const double bn2 = s.norm2;
  if ((rc = setup_expansion(c, e, 0.0))) return rc;
  CKL(launch_spmv(e.op, x0, b, c->w, nullptr, c->stream));
  CKR(launch_reduce(nullptr, 0, m, 0, c->w, nullptr, m, e.gr, e.fin(FIN_NORM, 0, 0), c->stream));
  if ((rc = read_ctrl(c, &s))) return rc;
  const double rn2 = s.norm2;
  const double q = bn2 > 0.0 ? std::sqrt(rn2 / bn2) : INFINITY;
  if (ratio) *ratio = q;
  *kept = (std::isfinite(q) && q < max_ratio) ? 1 : 0;
  if (!*kept) {
    CKL(launch_fill(x0, m, 0.0, c->stream));
    CK(hipStreamSynchronize(c->stream));
  }
  return DCGS2_OK;
}

// =====================================================================================
// Batched Krylov-Schur: every expansion step is one launch of each batched kernel
// over all instances (batched.hip); the per-instance dense work (real Schur form,
// reordering, convergence test, truncation matrices) runs on host threads between
// cycles.  A cycle's launch sequence depends only on its first step index, so it is
// captured once per first index into a HIP graph and replayed.
namespace {

struct BatchedState {
  int count = 0, p = 0, ld = 0, ldc = 0, ldp = 0;
  std::vector<dcgs2::BInst> tab;
  std::vector<int> pre_rows, pre_red;
  int nb_rows = 0, nb_red = 0;
  dcgs2::BInst* d_tab = nullptr;
  int* d_pre_rows = nullptr;
  int* d_pre_red = nullptr;
  double *Qa = nullptr, *Qb = nullptr, *vec = nullptr, *coef = nullptr, *pend = nullptr;
  double *H = nullptr, *K = nullptr, *Z = nullptr, *P1 = nullptr;
  double *resid = nullptr, *ere = nullptr, *eim = nullptr;   // dense results on the GPU
  int* ires = nullptr;
  double* gm = nullptr;          // batched GMRES: Rg, cs, sn, g and y of every instance
  Ctrl* ctrl = nullptr;
  hipStream_t s = nullptr;
  std::vector<std::pair<int, hipGraphExec_t>> graphs;
  std::vector<hipGraph_t> graph_defs;
  ~BatchedState() {
    for (auto& g : graphs) (void)hipGraphExecDestroy(g.second);
    for (auto& g : graph_defs) (void)hipGraphDestroy(g);
    void* bufs[] = {d_tab, d_pre_rows, d_pre_red, Qa, Qb, vec, coef, pend, H, K, Z, P1, ctrl,
                    resid, ere, eim, ires, gm};
    for (void* b : bufs) if (b) (void)hipFree(b);
    if (s) (void)hipStreamDestroy(s);
  }
};

int batched_cycle(BatchedState& B, int jmin, double tau, double eta, int* kernels) {
  hipStream_t s = B.s;
  const int p = B.p;
  CK(launch_breset(B.d_tab, B.count, tau, eta, s));
  for (int j = jmin; j <= p + 1; ++j) {
    CK(launch_bstencil(B.d_tab, B.d_pre_rows, B.count, B.nb_rows, j, s));
    CK(launch_breduce(B.d_tab, B.d_pre_red, B.count, B.nb_red, j, 0, B.ldp, B.ldc, B.ld, s));
    CK(launch_bupdate(B.d_tab, B.d_pre_rows, B.count, B.nb_rows, j, B.ldc, s));
    *kernels += 4;
  }
  const int jl = p + 2;                     // last column: J = p
  CK(launch_breduce(B.d_tab, B.d_pre_red, B.count, B.nb_red, jl, 1, B.ldp, B.ldc, B.ld, s));
  CK(launch_bproject_norm(B.d_tab, B.d_pre_red, B.count, B.nb_red, jl, B.ldp, B.ldc, B.ld, s));
  CK(launch_bscale(B.d_tab, B.d_pre_rows, B.count, B.nb_rows, jl, B.ldc, s));
  *kernels += 6;
  return DCGS2_OK;
}

int batched_run_cycle(BatchedState& B, int jmin, double tau, double eta, bool use_graph,
                      int* kernels) {
  if (!use_graph) return batched_cycle(B, jmin, tau, eta, kernels);
  for (auto& g : B.graphs) {
    if (g.first == jmin) {
      CK(hipGraphLaunch(g.second, B.s));
      *kernels += 4 * (B.p + 2 - jmin) + 6;
      return DCGS2_OK;
    }
  }
  hipGraph_t graph = nullptr;
  CK(hipStreamBeginCapture(B.s, hipStreamCaptureModeThreadLocal));
  int k0 = 0;
  const int rc = batched_cycle(B, jmin, tau, eta, &k0);
  hipGraph_t captured = nullptr;
  const hipError_t ec = hipStreamEndCapture(B.s, &captured);
  if (rc != DCGS2_OK) return rc;
  if (ec != hipSuccess) return DCGS2_EDEVICE;
  graph = captured;
  hipGraphExec_t exec = nullptr;
  CK(hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0));
  B.graph_defs.push_back(graph);
  B.graphs.push_back({jmin, exec});
  CK(hipGraphLaunch(exec, B.s));
  *kernels += k0;
  return DCGS2_OK;
}

}  // namespace

namespace {

// Explicit-norm fallback of instance b of a batched cycle whose Pythagorean guard
// failed at step ctrl->stop_step (the reading of Sec. 3 that the single-instance
// solver and the oracle follow): that step's fallback, the instance's remaining steps
// and its last-column finish run through the single-instance schedule on the
// instance's own buffers (on the context's stream), and *out receives its control
// block.  The batched launches of the cycle skipped the instance from that step on.
int batched_fallback(dcgs2_ctx c, const BatchedState& B, int b, Ctrl* out) {
  const dcgs2::BInst& I = B.tab[b];
  Expansion e;
  e.c = c;
  e.qr = false;
  e.m = I.m;
  e.Q = I.Q; e.q32 = 0; e.ldq = I.ldq;
  OpDev op{};
  op.kind = DCGS2_OP_STENCIL5;
  op.m = I.m;
  op.nx = I.nx; op.ny = I.ny; op.nz = 1;
  op.c0 = I.c0; op.cxm = I.cxm; op.cxp = I.cxp; op.cym = I.cym; op.cyp = I.cyp;
  op.dx = div_magic((uint32_t)I.nx);
  op.dy = div_magic((uint32_t)I.ny);
  e.op = op;
  e.ldh = B.ld;
  Work k;
  k.w = I.w; k.v = I.v; k.r = I.r;
  k.P1 = I.P1; k.ldp = B.ldp; k.G = I.G; k.ldc = B.ldc;
  k.coef = I.coef; k.pend = I.pend; k.H = I.H; k.K = I.K;
  k.ctrl = I.ctrl;
  if (I.gmres) {
    k.Rg = I.Rg; k.cs = I.cs; k.sn = I.sn; k.g = I.g;
    e.gmres = true;
  }
  e.wk = k;
  e.gr.P1 = k.P1; e.gr.ldp = k.ldp; e.gr.G = k.G;
  return e.run(out->stop_step, I.n + 1, FIN_STEP, I.n, out, true);
}

// One group of instances of the batched solver: its own stream, buffers, table
// and graphs.  Two groups alternate so that the host dense work of one overlaps
// the device cycle of the other.
struct BatchedGroup {
  BatchedState B;
  std::vector<int> gid;                 // global index of each local instance
  std::vector<Ctrl> hctrl;
  std::vector<double> Hh, Zh;
  // dense restart work on the GPU (device_dense): its parameters and host copies of
  // its per-instance results
  bool device_dense = false;
  int nev = 0, keep = 0;
  std::vector<int> hres;
  std::vector<double> hresid, here, heim;
  std::vector<dcgs2::BInst> tab_trunc;
  int kernels = 0;
  bool done = false;
  std::chrono::steady_clock::time_point t_cycle;
};

// nsteps (indexed like ops; nullptr: ncv for every instance) gives each instance's
// step count n_b <= ncv.  Qext, when given, holds the bases (instance b at element
// offset sum of pad_ld(m_i) (n_i + 1) over the instances before it, leading dimension
// pad_ld(m_b)); otherwise the group allocates two bases of ncv + 1 columns (the
// Krylov-Schur truncation target).
int group_setup(dcgs2_ctx c, BatchedGroup& g, const dcgs2_stencil2d* ops, const double* v0,
                const std::vector<int64_t>& v0off, int ncv, const int32_t* nsteps = nullptr,
                double* Qext = nullptr, bool two_bases = true) {
  BatchedState& B = g.B;
  const int count = (int)g.gid.size();
  B.count = count;
  B.p = ncv;
  B.ld = ncv + 1;
  B.ldc = ncv + 2;
  B.ldp = 2 * (ncv + 2) + 8;
  const int p = B.p, ld = B.ld;
  CK(hipStreamCreateWithFlags(&B.s, hipStreamNonBlocking));   // default priority
  std::vector<int64_t> ldq(count), qoff(count), voff(count);
  int64_t qtot = 0, vtot = 0, gtot = 0;
  B.pre_rows.assign(count + 1, 0);
  B.pre_red.assign(count + 1, 0);
  std::vector<int> G(count);
  for (int b = 0; b < count; ++b) {
    const dcgs2_stencil2d& o = ops[g.gid[b]];
    const int64_t mb = (int64_t)o.nx * o.ny;
    ldq[b] = pad_ld(mb);
    qoff[b] = qtot;
    qtot += ldq[b] * ((nsteps ? nsteps[g.gid[b]] : p) + 1);
    voff[b] = vtot;
    vtot += 3 * ldq[b];
    const int64_t gg = ((mb + 1) / 2 + c->tune_batch_units - 1) / c->tune_batch_units;
    G[b] = (int)std::max<int64_t>(1, std::min<int64_t>(gg, BATCH_GMAX));
    gtot += G[b];
    B.pre_rows[b + 1] =
        B.pre_rows[b] + (int)((mb + BATCH_ROWS_PER_BLOCK - 1) / BATCH_ROWS_PER_BLOCK);
    B.pre_red[b + 1] = B.pre_red[b] + G[b];
  }
  B.nb_rows = B.pre_rows[count];
  B.nb_red = B.pre_red[count];
  int rc;
  if (!Qext) {
    if ((rc = dalloc((void**)&B.Qa, sizeof(double) * qtot))) return rc;
    if (two_bases && (rc = dalloc((void**)&B.Qb, sizeof(double) * qtot))) return rc;
  }
  if ((rc = dalloc((void**)&B.vec, sizeof(double) * vtot))) return rc;
  if ((rc = dalloc((void**)&B.coef, sizeof(double) * (size_t)count * (2 * B.ldc + 8)))) return rc;
  if ((rc = dalloc((void**)&B.pend, sizeof(double) * (size_t)count * (2 * B.ldc + 8)))) return rc;
  if ((rc = dalloc((void**)&B.H, sizeof(double) * (size_t)count * ld * ld))) return rc;
  if ((rc = dalloc((void**)&B.K, sizeof(double) * (size_t)count * ld * ld))) return rc;
  if ((rc = dalloc((void**)&B.Z, sizeof(double) * (size_t)count * p * p))) return rc;
  if ((rc = dalloc((void**)&B.P1, sizeof(double) * (size_t)gtot * B.ldp))) return rc;
  if ((rc = dalloc((void**)&B.ctrl, sizeof(Ctrl) * (size_t)count))) return rc;
  if ((rc = dalloc((void**)&B.d_tab, sizeof(dcgs2::BInst) * (size_t)count))) return rc;
  if ((rc = dalloc((void**)&B.d_pre_rows, sizeof(int) * (size_t)(count + 1)))) return rc;
  if ((rc = dalloc((void**)&B.d_pre_red, sizeof(int) * (size_t)(count + 1)))) return rc;
  B.tab.resize(count);
  int64_t goff = 0;
  for (int b = 0; b < count; ++b) {
    const dcgs2_stencil2d& o = ops[g.gid[b]];
    dcgs2::BInst& I = B.tab[b];
    std::memset(&I, 0, sizeof(I));
    I.m = (int64_t)o.nx * o.ny;
    I.ldq = ldq[b];
    I.Q = (Qext ? Qext : B.Qa) + qoff[b];
    I.Qn = B.Qb ? B.Qb + qoff[b] : nullptr;
    I.w = B.vec + voff[b];
    I.v = I.w + ldq[b];
    I.r = I.v + ldq[b];
    I.coef = B.coef + (size_t)b * (2 * B.ldc + 8);
    I.pend = B.pend + (size_t)b * (2 * B.ldc + 8);
    I.H = B.H + (size_t)b * ld * ld;
    I.K = B.K + (size_t)b * ld * ld;
    I.Z = B.Z + (size_t)b * p * p;
    I.ctrl = B.ctrl + b;
    I.P1 = B.P1 + goff * B.ldp;
    I.G = G[b];
    goff += G[b];
    I.nx = o.nx; I.ny = o.ny;
    I.c0 = o.c0; I.cxm = o.cxm; I.cxp = o.cxp; I.cym = o.cym; I.cyp = o.cyp;
    I.first_j = 2;
    I.restart = 0;
    I.active = 1;
    I.n = nsteps ? nsteps[g.gid[b]] : p;
    CK(hipMemcpyAsync(I.w, v0 + v0off[g.gid[b]], sizeof(double) * I.m, hipMemcpyDeviceToDevice,
                      B.s));
  }
  CK(hipMemcpyAsync(B.d_pre_rows, B.pre_rows.data(), sizeof(int) * (count + 1),
                    hipMemcpyHostToDevice, B.s));
  CK(hipMemcpyAsync(B.d_pre_red, B.pre_red.data(), sizeof(int) * (count + 1),
                    hipMemcpyHostToDevice, B.s));
  CK(hipMemcpyAsync(B.d_tab, B.tab.data(), sizeof(dcgs2::BInst) * count, hipMemcpyHostToDevice,
                    B.s));
  CK(launch_fill(B.H, (int64_t)count * ld * ld, 0.0, B.s));
  CK(launch_fill(B.K, (int64_t)count * ld * ld, 0.0, B.s));
  g.hctrl.resize(count);
  if (g.device_dense) {
    if ((rc = dalloc((void**)&B.ires, sizeof(int) * (size_t)count * 4))) return rc;
    if ((rc = dalloc((void**)&B.resid, sizeof(double) * (size_t)count))) return rc;
    if ((rc = dalloc((void**)&B.ere, sizeof(double) * (size_t)count * g.nev))) return rc;
    if ((rc = dalloc((void**)&B.eim, sizeof(double) * (size_t)count * g.nev))) return rc;
    g.hres.resize((size_t)count * 4);
    g.hresid.resize(count);
    g.here.resize((size_t)count * g.nev);
    g.heim.resize((size_t)count * g.nev);
  } else {
    g.Hh.resize((size_t)count * ld * ld);
    g.Zh.resize((size_t)count * p * p);
  }
  return DCGS2_OK;
}

// Enqueue the read-back of a finished cycle's control blocks and H.
constexpr double BATCH_CUT_GAP = 1e-8;   // a complex pair is never split by the cut

// Enqueued behind a cycle: the control blocks, and either the projected matrices (dense
// work on the host) or the dense work on the GPU and its per-instance results.
int group_readback(BatchedGroup& g) {
  BatchedState& B = g.B;
  CK(hipMemcpyAsync(g.hctrl.data(), B.ctrl, sizeof(Ctrl) * B.count, hipMemcpyDeviceToHost, B.s));
  if (!g.device_dense) {
    CK(hipMemcpyAsync(g.Hh.data(), B.H, sizeof(double) * g.Hh.size(), hipMemcpyDeviceToHost,
                      B.s));
    return DCGS2_OK;
  }
  CK(launch_bschur(B.d_tab, B.count, B.p, B.ld, g.nev, g.keep, BATCH_CUT_GAP, B.H, B.Z, B.ires,
                   B.resid, B.ere, B.eim, B.s));
  g.kernels += 1;
  CK(hipMemcpyAsync(g.hres.data(), B.ires, sizeof(int) * g.hres.size(), hipMemcpyDeviceToHost,
                    B.s));
  CK(hipMemcpyAsync(g.hresid.data(), B.resid, sizeof(double) * g.hresid.size(),
                    hipMemcpyDeviceToHost, B.s));
  CK(hipMemcpyAsync(g.here.data(), B.ere, sizeof(double) * g.here.size(), hipMemcpyDeviceToHost,
                    B.s));
  CK(hipMemcpyAsync(g.heim.data(), B.eim, sizeof(double) * g.heim.size(), hipMemcpyDeviceToHost,
                    B.s));
  return DCGS2_OK;
}

// Host dense work of one finished cycle (threads), then the truncation and the
// next cycle's launch for the instances still active.
int group_step(dcgs2_ctx c, BatchedGroup& g, int nev, int keep, double tol, int max_restarts,
               double* eig_re, double* eig_im, dcgs2_ks_info* infos, bool use_graph,
               int nthreads) {
  using clk = std::chrono::steady_clock;
  BatchedState& B = g.B;
  const int p = B.p, ld = B.ld, count = B.count;
  CK(hipStreamSynchronize(B.s));
  if (c->prof) {
    c->acc[K_BATCH_CYCLE].launches += 1;
    c->acc[K_BATCH_CYCLE].ms +=
        std::chrono::duration<double, std::milli>(clk::now() - g.t_cycle).count();
  }
  // Pythagorean-guard failures of this cycle: resolved instance by instance, after
  // which their projected matrices are read again and their dense work runs on host
  // threads (also in a group whose dense work otherwise runs on the GPU)
  std::vector<char> repaired(count, 0);
  for (int b = 0; b < count; ++b) {
    if (!B.tab[b].active || g.hctrl[b].state != ST_FALLBACK) continue;
    int rc = batched_fallback(c, B, b, &g.hctrl[b]);
    if (rc) return rc;
    repaired[b] = 1;
    if (g.Hh.size() < (size_t)count * ld * ld) g.Hh.resize((size_t)count * ld * ld);
    if (g.Zh.size() < (size_t)count * p * p) g.Zh.resize((size_t)count * p * p);
    CK(hipMemcpy(g.Hh.data() + (size_t)b * ld * ld, B.tab[b].H, sizeof(double) * ld * ld,
                 hipMemcpyDeviceToHost));
  }
  const clk::time_point t_host = clk::now();
  const double CUT_GAP = BATCH_CUT_GAP;
  std::vector<std::thread> pool;
  std::atomic<int> next{0};
  auto worker = [&]() {
    std::vector<double> T((size_t)p * p), Zm((size_t)p * p), ere(p), eim(p);
    for (int b = next++; b < count; b = next++) {
      dcgs2::BInst& I = B.tab[b];
      if (!I.active || (g.device_dense && !repaired[b])) continue;
      const int gb = g.gid[b];
      dcgs2_ks_info& inf = infos[gb];
      const Ctrl& hc = g.hctrl[b];
      inf.st.reductions += hc.reductions;
      I.truncate = 0;
      if (hc.state != ST_RUNNING) {
        inf.status = hc.state == ST_BREAKDOWN ? DCGS2_BREAKDOWN
                     : hc.state == ST_NONFINITE ? DCGS2_NONFINITE : DCGS2_NOT_CONVERGED;
        inf.st.pyth_fallbacks += hc.fallbacks;
        inf.st.breakdown_step = hc.k;
        I.active = 0;
        continue;
      }
      inf.st.pyth_fallbacks += hc.fallbacks;
      const double* Hb = g.Hh.data() + (size_t)b * ld * ld;
      const double h = Hb[(size_t)(p - 1) * ld + p];
      for (int jj = 0; jj < p; ++jj)
        for (int i = 0; i < p; ++i) T[(size_t)jj * p + i] = Hb[(size_t)jj * ld + i];
      if (real_schur(p, T.data(), p, Zm.data(), p) != 0) { I.active = 0; continue; }
      const int kn = reorder_schur_by_magnitude(p, T.data(), p, Zm.data(), p, nev, CUT_GAP);
      if (kn < 0) { I.active = 0; continue; }
      schur_eigenvalues(p, T.data(), p, ere.data(), eim.data());
      double bn = 0.0, tmin = INFINITY;
      for (int i = 0; i < kn; ++i) {
        const double bi = h * Zm[(size_t)i * p + (p - 1)];
        bn += bi * bi;
        tmin = std::min(tmin, std::hypot(ere[i], eim[i]));
      }
      inf.resid = std::sqrt(bn) / tmin;
      for (int i = 0; i < nev; ++i) {
        eig_re[(size_t)gb * nev + i] = ere[i];
        eig_im[(size_t)gb * nev + i] = eim[i];
      }
      if (inf.resid <= tol) { inf.nconv = kn; inf.status = DCGS2_OK; I.active = 0; continue; }
      if (inf.restarts >= max_restarts) {
        inf.status = DCGS2_NOT_CONVERGED;
        I.active = 0;
        continue;
      }
      const int k = reorder_schur_by_magnitude(p, T.data(), p, Zm.data(), p, keep, CUT_GAP);
      if (k < 0 || k >= p) { I.active = 0; continue; }
      std::copy(Zm.begin(), Zm.end(), g.Zh.begin() + (size_t)b * p * p);
      double* Hn = g.Hh.data() + (size_t)b * ld * ld;
      std::fill(Hn, Hn + (size_t)ld * ld, 0.0);
      for (int jj = 0; jj < k; ++jj) {
        for (int i = 0; i < k; ++i) Hn[(size_t)jj * ld + i] = T[(size_t)jj * p + i];
        Hn[(size_t)jj * ld + k] = h * Zm[(size_t)jj * p + (p - 1)];
      }
      I.k = k;
      I.first_j = k + 2;
      I.restart = 1;
      I.truncate = 1;
      inf.restarts += 1;
      inf.matvecs += p - k;
    }
  };
  // dense work done on the GPU: the same decisions from its per-instance results
  auto settle = [&]() {
    for (int b = 0; b < count; ++b) {
      dcgs2::BInst& I = B.tab[b];
      if (!I.active || repaired[b]) continue;
      const int gb = g.gid[b];
      dcgs2_ks_info& inf = infos[gb];
      const Ctrl& hc = g.hctrl[b];
      inf.st.reductions += hc.reductions;
      I.truncate = 0;
      if (hc.state != ST_RUNNING) {
        inf.status = hc.state == ST_BREAKDOWN ? DCGS2_BREAKDOWN
                     : hc.state == ST_NONFINITE ? DCGS2_NONFINITE : DCGS2_NOT_CONVERGED;
        inf.st.pyth_fallbacks += hc.fallbacks;
        inf.st.breakdown_step = hc.k;
        I.active = 0;
        continue;
      }
      const int* r = &g.hres[(size_t)4 * b];
      if (r[0] != 1 && r[0] != -2) { I.active = 0; continue; }   // no Ritz values
      inf.resid = g.hresid[b];
      for (int i = 0; i < nev; ++i) {
        eig_re[(size_t)gb * nev + i] = g.here[(size_t)b * nev + i];
        eig_im[(size_t)gb * nev + i] = g.heim[(size_t)b * nev + i];
      }
      if (inf.resid <= tol) { inf.nconv = r[1]; inf.status = DCGS2_OK; I.active = 0; continue; }
      if (inf.restarts >= max_restarts) {
        inf.status = DCGS2_NOT_CONVERGED;
        I.active = 0;
        continue;
      }
      if (r[0] != 1) { I.active = 0; continue; }
      const int k = r[2];
      I.k = k;
      I.first_j = k + 2;
      I.restart = 1;
      I.truncate = 1;
      inf.restarts += 1;
      inf.matvecs += p - k;
    }
  };
  bool any_repaired = false;
  for (int b = 0; b < count; ++b) any_repaired = any_repaired || repaired[b];
  if (g.device_dense) settle();
  if (!g.device_dense || any_repaired) {
    for (int t = 0; t < nthreads; ++t) pool.emplace_back(worker);
    for (auto& t : pool) t.join();
  }
  if (c->prof) {
    c->acc[K_HOST_DENSE].launches += 1;
    c->acc[K_HOST_DENSE].ms +=
        std::chrono::duration<double, std::milli>(clk::now() - t_host).count();
  }
  int jmin = INT32_MAX;
  for (int b = 0; b < count; ++b)
    if (B.tab[b].active) jmin = std::min(jmin, B.tab[b].first_j);
  if (jmin == INT32_MAX) {
    g.done = true;
    return DCGS2_OK;
  }
  // truncation: Qn = Q Z_k, q_{k+1} and w; then swap the bases of truncated instances.
  // The truncation reads g.tab_trunc and the next cycle the swapped g.B.tab: two host
  // buffers, neither changed before this group's next synchronisation.
  if (!g.device_dense) {                 // on the GPU, Z and H are already in place
    CK(hipMemcpyAsync(B.Z, g.Zh.data(), sizeof(double) * g.Zh.size(), hipMemcpyHostToDevice,
                      B.s));
    CK(hipMemcpyAsync(B.H, g.Hh.data(), sizeof(double) * g.Hh.size(), hipMemcpyHostToDevice,
                      B.s));
  } else {                                // except for instances repaired on the host
    for (int b = 0; b < count; ++b) {
      if (!repaired[b] || !B.tab[b].active || !B.tab[b].truncate) continue;
      CK(hipMemcpyAsync(B.tab[b].Z, g.Zh.data() + (size_t)b * p * p, sizeof(double) * p * p,
                        hipMemcpyHostToDevice, B.s));
      CK(hipMemcpyAsync(B.tab[b].H, g.Hh.data() + (size_t)b * ld * ld, sizeof(double) * ld * ld,
                        hipMemcpyHostToDevice, B.s));
    }
  }
  CK(launch_fill(B.K, (int64_t)count * ld * ld, 0.0, B.s));
  g.tab_trunc = B.tab;
  CK(hipMemcpyAsync(B.d_tab, g.tab_trunc.data(), sizeof(dcgs2::BInst) * count,
                    hipMemcpyHostToDevice, B.s));
  CK(launch_btruncate(B.d_tab, B.d_pre_rows, count, B.nb_rows, p, B.s));
  g.kernels += 2;
  for (int b = 0; b < count; ++b) {
    dcgs2::BInst& I = B.tab[b];
    if (I.active && I.truncate) { std::swap(I.Q, I.Qn); I.truncate = 0; }
  }
  CK(hipMemcpyAsync(B.d_tab, B.tab.data(), sizeof(dcgs2::BInst) * count, hipMemcpyHostToDevice,
                    B.s));
  g.t_cycle = clk::now();
  int rc;
  if ((rc = batched_run_cycle(B, jmin, c->tau, c->eta, use_graph, &g.kernels))) return rc;
  return group_readback(g);
}

}  // namespace

extern "C" int krylov_schur_batched(dcgs2_ctx c, int32_t count, const dcgs2_stencil2d* ops,
                                    int32_t nev, int32_t ncv, int32_t keep, double tol,
                                    int32_t max_restarts, const double* v0, double* eig_re,
                                    double* eig_im, dcgs2_ks_info* infos, int32_t use_graph) {
  if (!c || count < 1 || count > 65536 || !ops || !v0 || !eig_re || !eig_im || !infos ||
      nev < 1 || keep <= nev || ncv <= keep || ncv > DCGS2_MAX_N || !(tol > 0.0) ||
      max_restarts < 0)
    return DCGS2_EINVAL;
  for (int b = 0; b < count; ++b) {
    const int64_t mb = (int64_t)ops[b].nx * ops[b].ny;
    if (ops[b].nx < 1 || ops[b].ny < 1 || mb <= ncv || mb >= INT32_MAX) return DCGS2_EINVAL;
  }
  int rc;
  if ((rc = ctx_ready(c))) return rc;
  CK(hipStreamSynchronize(c->stream));      // inputs produced on the caller's stream
  std::vector<int64_t> v0off(count);
  int64_t v0tot = 0;
  for (int b = 0; b < count; ++b) {
    v0off[b] = v0tot;
    v0tot += (int64_t)ops[b].nx * ops[b].ny;
    std::memset(&infos[b], 0, sizeof(infos[b]));
    infos[b].matvecs = ncv;
    infos[b].status = DCGS2_NOT_CONVERGED;
  }
  // two groups of similar total size: instances by decreasing m, dealt alternately
  const int ngroups = count >= 2 ? 2 : 1;
  std::vector<int> order(count);
  for (int b = 0; b < count; ++b) order[b] = b;
  std::stable_sort(order.begin(), order.end(), [&](int x, int y) {
    return (int64_t)ops[x].nx * ops[x].ny > (int64_t)ops[y].nx * ops[y].ny;
  });
  std::vector<BatchedGroup> groups(ngroups);
  for (int i = 0; i < count; ++i) groups[i % ngroups].gid.push_back(order[i]);
  for (auto& g : groups) std::sort(g.gid.begin(), g.gid.end());
  for (auto& g : groups) {
    g.device_dense = c->tune_batch_host_dense == 0 && ncv <= BSCHUR_MAX_P;
    g.nev = nev;
    g.keep = keep;
    if ((rc = group_setup(c, g, ops, v0, v0off, ncv))) return rc;
    g.t_cycle = std::chrono::steady_clock::now();
    if ((rc = batched_run_cycle(g.B, 2, c->tau, c->eta, use_graph != 0, &g.kernels))) return rc;
    if ((rc = group_readback(g))) return rc;
  }
  const int nthreads = (int)std::max(1u, std::min(16u, std::thread::hardware_concurrency()));
  for (;;) {
    bool any = false;
    for (auto& g : groups) {
      if (g.done) continue;
      any = true;
      if ((rc = group_step(c, g, nev, keep, tol, max_restarts, eig_re, eig_im, infos,
                           use_graph != 0, nthreads)))
        return rc;
    }
    if (!any) break;
  }
  int overall = DCGS2_OK;
  int kernels = 0;
  for (auto& g : groups) {
    CK(hipStreamSynchronize(g.B.s));
    kernels += g.kernels;
  }
  for (int b = 0; b < count; ++b) {
    infos[b].st.kernels = kernels;
    if (infos[b].status != DCGS2_OK) overall = DCGS2_NOT_CONVERGED;
    if (infos[b].status == DCGS2_OK) infos[b].st.breakdown_step = -1;
  }
  return overall;
}

extern "C" int dcgs2_arnoldi_batched(dcgs2_ctx c, int32_t count, const dcgs2_stencil2d* ops,
                                     const int32_t* n, const double* r0, double* Q,
                                     double* H_host, int32_t* status_host,
                                     dcgs2_stats* st_host) {
  if (!c || count < 1 || count > 65536 || !ops || !n || !r0 || !Q || !H_host ||
      (reinterpret_cast<uintptr_t>(Q) & 15u) != 0)
    return DCGS2_EINVAL;
  int nmax = 0;
  for (int b = 0; b < count; ++b) {
    const int64_t mb = (int64_t)ops[b].nx * ops[b].ny;
    if (ops[b].nx < 1 || ops[b].ny < 1 || mb < 2 || mb >= INT32_MAX || n[b] < 1 ||
        n[b] > DCGS2_MAX_N || (int64_t)n[b] >= mb)
      return DCGS2_EINVAL;
    nmax = std::max(nmax, (int)n[b]);
  }
  int rc;
  if ((rc = ctx_ready(c))) return rc;
  CK(hipStreamSynchronize(c->stream));      // inputs produced on the caller's stream
  std::vector<int64_t> v0off(count);
  int64_t v0tot = 0;
  for (int b = 0; b < count; ++b) {
    v0off[b] = v0tot;
    v0tot += (int64_t)ops[b].nx * ops[b].ny;
  }
  BatchedGroup g;
  g.gid.resize(count);
  for (int b = 0; b < count; ++b) g.gid[b] = b;
  if ((rc = group_setup(c, g, ops, r0, v0off, nmax, n, Q))) return rc;
  BatchedState& B = g.B;
  int kernels = 0;
  if ((rc = batched_run_cycle(B, 2, c->tau, c->eta, false, &kernels))) return rc;
  const int ld = B.ld;
  g.Hh.resize((size_t)count * ld * ld);
  CK(hipMemcpyAsync(g.hctrl.data(), B.ctrl, sizeof(Ctrl) * count, hipMemcpyDeviceToHost, B.s));
  CK(hipMemcpyAsync(g.Hh.data(), B.H, sizeof(double) * g.Hh.size(), hipMemcpyDeviceToHost, B.s));
  CK(hipStreamSynchronize(B.s));
  // Pythagorean-guard failures: the explicit-norm fallback and the rest of the
  // instance's expansion through the single-instance schedule
  for (int b = 0; b < count; ++b) {
    if (g.hctrl[b].state != ST_FALLBACK) continue;
    if ((rc = batched_fallback(c, B, b, &g.hctrl[b]))) return rc;
    CK(hipMemcpy(g.Hh.data() + (size_t)b * ld * ld, B.tab[b].H, sizeof(double) * ld * ld,
                 hipMemcpyDeviceToHost));
  }
  int overall = DCGS2_OK;
  int64_t hoff = 0;
  for (int b = 0; b < count; ++b) {
    const Ctrl& hc = g.hctrl[b];
    const int nb = n[b];
    const int st = status_of(hc);
    if (st == DCGS2_NONFINITE || (st == DCGS2_BREAKDOWN && overall == DCGS2_OK)) overall = st;
    for (int jj = 0; jj < nb; ++jj)
      for (int i = 0; i <= nb; ++i)
        H_host[hoff + (int64_t)jj * (nb + 1) + i] = g.Hh[(size_t)b * ld * ld + (size_t)jj * ld + i];
    hoff += (int64_t)(nb + 1) * nb;
    if (status_host) status_host[b] = st;
    if (st_host) fill_stats(&st_host[b], hc, kernels, st);
  }
  return overall;
}

extern "C" int gmres_batched(dcgs2_ctx c, int32_t count, const dcgs2_stencil2d* ops,
                             const int32_t* restart, const double* b, double* x, double rtol,
                             int32_t max_iters, dcgs2_gmres_info* info_host) {
  if (!c || count < 1 || count > 65536 || !ops || !restart || !b || !x || !info_host ||
      !(rtol > 0.0) || max_iters < 0)
    return DCGS2_EINVAL;
  int pmax = 0;
  for (int i = 0; i < count; ++i) {
    const int64_t mb = (int64_t)ops[i].nx * ops[i].ny;
    if (ops[i].nx < 1 || ops[i].ny < 1 || mb < 2 || mb >= INT32_MAX || restart[i] < 1 ||
        restart[i] > DCGS2_MAX_N || (int64_t)restart[i] >= mb)
      return DCGS2_EINVAL;
    pmax = std::max(pmax, (int)restart[i]);
  }
  int rc;
  if ((rc = ctx_ready(c))) return rc;
  CK(hipStreamSynchronize(c->stream));      // b and x0 produced on the caller's stream
  std::vector<int64_t> off(count);
  int64_t tot = 0;
  for (int i = 0; i < count; ++i) {
    off[i] = tot;
    tot += (int64_t)ops[i].nx * ops[i].ny;
  }
  BatchedGroup g;
  g.gid.resize(count);
  for (int i = 0; i < count; ++i) g.gid[i] = i;
  if ((rc = group_setup(c, g, ops, b, off, pmax, restart, nullptr, false))) return rc;
  BatchedState& B = g.B;
  const int p = B.p, ld = B.ld;
  // Givens state and least-squares solution of every instance
  const size_t per = (size_t)ld * ld + 3 * (size_t)(p + 2) + (size_t)(p + 1);
  if ((rc = dalloc((void**)&B.gm, sizeof(double) * per * count))) return rc;
  for (int i = 0; i < count; ++i) {
    dcgs2::BInst& I = B.tab[i];
    double* q = B.gm + per * i;
    I.gmres = 1;
    I.Rg = q; q += (size_t)ld * ld;
    I.cs = q; q += p + 2;
    I.sn = q; q += p + 2;
    I.g = q; q += p + 2;
    I.y = q;
    I.bvec = b + off[i];
    I.x = x + off[i];
    I.ksol = 0;
    I.thresh = 0.0;
    std::memset(&info_host[i], 0, sizeof(info_host[i]));
    info_host[i].st.breakdown_step = -1;
  }
  hipStream_t s = B.s;
  auto upload_tab = [&]() -> int {
    CK(hipMemcpyAsync(B.d_tab, B.tab.data(), sizeof(dcgs2::BInst) * count, hipMemcpyHostToDevice,
                      s));
    return DCGS2_OK;
  };
  auto read_ctrls = [&]() -> int {
    CK(hipMemcpyAsync(g.hctrl.data(), B.ctrl, sizeof(Ctrl) * count, hipMemcpyDeviceToHost, s));
    CK(hipStreamSynchronize(s));
    return DCGS2_OK;
  };
  int kernels = 0;
  // ||b|| of every instance
  if ((rc = upload_tab())) return rc;
  CK(launch_breset(B.d_tab, count, c->tau, c->eta, s));
  CK(launch_bresidual(B.d_tab, B.d_pre_rows, count, B.nb_rows, 1, s));
  CK(launch_bnorm(B.d_tab, B.d_pre_red, count, B.nb_red, B.ldp, B.ldc, ld, s));
  kernels += 4;
  if ((rc = read_ctrls())) return rc;
  std::vector<double> bnorm(count), yh((size_t)count * (p + 1)), Rh((size_t)count * ld * ld),
      gh((size_t)count * (p + 2));
  for (int i = 0; i < count; ++i) {
    dcgs2::BInst& I = B.tab[i];
    bnorm[i] = std::sqrt(g.hctrl[i].norm2);
    info_host[i].st.reductions += g.hctrl[i].reductions;
    if (!std::isfinite(bnorm[i])) {
      info_host[i].status = DCGS2_NONFINITE;
      I.active = 0;
    } else if (bnorm[i] == 0.0) {               // b = 0: x = 0
      CK(launch_fill(I.x, I.m, 0.0, s));
      info_host[i].status = DCGS2_OK;
      I.active = 0;
    }
  }
  for (;;) {
    // r = b - A x and ||r|| for every active instance; decide who runs a cycle
    if ((rc = upload_tab())) return rc;
    CK(launch_breset(B.d_tab, count, c->tau, c->eta, s));
    CK(launch_bresidual(B.d_tab, B.d_pre_rows, count, B.nb_rows, 0, s));
    CK(launch_bnorm(B.d_tab, B.d_pre_red, count, B.nb_red, B.ldp, B.ldc, ld, s));
    kernels += 4;
    if ((rc = read_ctrls())) return rc;
    int running = 0;
    for (int i = 0; i < count; ++i) {
      dcgs2::BInst& I = B.tab[i];
      I.ksol = 0;
      if (!I.active) continue;
      dcgs2_gmres_info& inf = info_host[i];
      inf.st.reductions += g.hctrl[i].reductions;
      inf.relres_true = std::sqrt(g.hctrl[i].norm2) / bnorm[i];
      if (!std::isfinite(inf.relres_true)) { inf.status = DCGS2_NONFINITE; I.active = 0; continue; }
      if (inf.relres_true <= rtol) { inf.status = DCGS2_OK; I.active = 0; continue; }
      if (inf.iters >= max_iters) { inf.status = DCGS2_NOT_CONVERGED; I.active = 0; continue; }
      I.n = std::min((int)restart[i], max_iters - inf.iters);
      I.thresh = rtol * bnorm[i];
      inf.cycles += 1;
      ++running;
    }
    if (running == 0) break;
    if ((rc = upload_tab())) return rc;
    CK(launch_fill(B.H, (int64_t)count * ld * ld, 0.0, s));
    CK(launch_fill(B.K, (int64_t)count * ld * ld, 0.0, s));
    CK(launch_fill(B.gm, (int64_t)(per * count), 0.0, s));
    kernels += 3;
    if ((rc = batched_run_cycle(B, 2, c->tau, c->eta, true, &kernels))) return rc;
    CK(hipMemcpyAsync(g.hctrl.data(), B.ctrl, sizeof(Ctrl) * count, hipMemcpyDeviceToHost, s));
    CK(hipStreamSynchronize(s));
    for (int i = 0; i < count; ++i) {         // explicit-norm fallbacks, one instance at a time
      if (!B.tab[i].active || g.hctrl[i].state != ST_FALLBACK) continue;
      if ((rc = batched_fallback(c, B, i, &g.hctrl[i]))) return rc;
    }
    for (int i = 0; i < count; ++i) {
      dcgs2::BInst& I = B.tab[i];
      if (!I.active) continue;
      CK(hipMemcpyAsync(Rh.data() + (size_t)i * ld * ld, I.Rg, sizeof(double) * ld * ld,
                        hipMemcpyDeviceToHost, s));
      CK(hipMemcpyAsync(gh.data() + (size_t)i * (p + 2), I.g, sizeof(double) * (p + 2),
                        hipMemcpyDeviceToHost, s));
    }
    CK(hipStreamSynchronize(s));
    for (int i = 0; i < count; ++i) {
      dcgs2::BInst& I = B.tab[i];
      if (!I.active) continue;
      dcgs2_gmres_info& inf = info_host[i];
      const Ctrl& hc = g.hctrl[i];
      inf.st.reductions += hc.reductions;
      inf.st.pyth_fallbacks += hc.fallbacks;
      if (hc.state == ST_NONFINITE) { inf.status = DCGS2_NONFINITE; I.active = 0; continue; }
      const int nc = I.n;
      inf.iters += (hc.state == ST_RUNNING) ? nc : std::min(hc.stop_step - 1, nc);
      inf.relres_est = hc.resid_est / bnorm[i];
      const int k = hc.k;
      if (k <= 0) { inf.status = DCGS2_BREAKDOWN; I.active = 0; continue; }
      // y = R_k^{-1} g_{1:k} (back substitution on the rotated Hessenberg matrix)
      const double* R = Rh.data() + (size_t)i * ld * ld;
      const double* gg = gh.data() + (size_t)i * (p + 2);
      double* y = yh.data() + (size_t)i * (p + 1);
      for (int r = k - 1; r >= 0; --r) {
        double sum = gg[r];
        for (int jj = r + 1; jj < k; ++jj) sum -= R[(size_t)jj * ld + r] * y[jj];
        y[r] = sum / R[(size_t)r * ld + r];
      }
      I.ksol = k;
      CK(hipMemcpyAsync(I.y, y, sizeof(double) * k, hipMemcpyHostToDevice, s));
    }
    if ((rc = upload_tab())) return rc;
    CK(launch_bxupdate(B.d_tab, B.d_pre_rows, count, B.nb_rows, s));
    kernels += 1;
  }
  CK(hipStreamSynchronize(s));
  int overall = DCGS2_OK;
  for (int i = 0; i < count; ++i) {
    info_host[i].st.kernels = kernels;
    const int st = info_host[i].status;
    if (st == DCGS2_NONFINITE) overall = DCGS2_NONFINITE;
    else if (st != DCGS2_OK && overall == DCGS2_OK) overall = st;
  }
  return overall;
}

