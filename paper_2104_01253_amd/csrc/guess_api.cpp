// Host side of the learned initial guess: the perceptron object (parameters,
// gradients, Adam moments and activations in device memory) and the transfer
// entry points.  All work is enqueued on the context's stream; every entry point
// returns after that stream has synchronised.
#include <hip/hip_runtime_api.h>

#include <cmath>
#include <cstring>
#include <new>
#include <vector>

#include "internal.h"

using namespace dcgs2;

struct dcgs2_mlp_s {
  dcgs2_ctx ctx = nullptr;
  hipStream_t s = nullptr;
  int L = 0;                         // layers
  std::vector<int> w;                // widths, L + 1
  std::vector<int64_t> offW, offb;   // offsets of W_l and b_l in the packed parameters
  int64_t P = 0;                     // parameter count
  int max_batch = 0;
  int64_t t = 0;                     // Adam steps taken
  float *theta = nullptr, *grad = nullptr, *m1 = nullptr, *m2 = nullptr;
  std::vector<float*> act;           // hidden activations ReLU(Z_l), l < L-1 (max_batch x w[l+1])
  float *out = nullptr;              // output of the last forward (max_batch x w[L])
  float *dA = nullptr, *dB = nullptr;  // backward ping-pong (max_batch x max width)
  double *part = nullptr, *loss = nullptr;
};

namespace {

#define CK(call)                                   \
  do {                                             \
    hipError_t e_ = (call);                        \
    if (e_ != hipSuccess) return DCGS2_EDEVICE;    \
  } while (0)

int alloc_f(float** p, int64_t n) {
  if (hipMalloc((void**)p, sizeof(float) * (size_t)(n > 0 ? n : 1)) != hipSuccess) {
    *p = nullptr;
    return DCGS2_ENOMEM;
  }
  return DCGS2_OK;
}

void release(dcgs2_mlp_s* q) {
  void* bufs[] = {q->theta, q->grad, q->m1, q->m2, q->out, q->dA, q->dB, q->part, q->loss};
  for (void* b : bufs) if (b) (void)hipFree(b);
  for (float* a : q->act) if (a) (void)hipFree(a);
  delete q;
}

// forward pass of `batch` rows of X; leaves activations and the output in q
int forward(dcgs2_mlp_s* q, int batch, const float* X) {
  const float* in = X;
  for (int l = 0; l < q->L; ++l) {
    const bool last = (l == q->L - 1);
    float* o = last ? q->out : q->act[l];
    CK(launch_gemm_f32(0, 0, last ? GEMM_BIAS : GEMM_BIAS_RELU, batch, q->w[l + 1], q->w[l], in,
                       q->w[l], q->theta + q->offW[l], q->w[l + 1], o, q->w[l + 1],
                       q->theta + q->offb[l], nullptr, q->s));
    in = o;
  }
  return DCGS2_OK;
}

}  // namespace

extern "C" {

int dcgs2_mlp_create(dcgs2_ctx ctx, int32_t nlayers, const int32_t* widths, int32_t max_batch,
                     dcgs2_mlp* out) {
  if (!ctx || !out || !widths || nlayers < 1 || nlayers > 16 || max_batch < 1 ||
      max_batch > 65536)
    return DCGS2_EINVAL;
  for (int l = 0; l <= nlayers; ++l)
    if (widths[l] < 1 || widths[l] > 16384) return DCGS2_EINVAL;
  hipStream_t s;
  int rc = ctx_prepare(ctx, &s);
  if (rc) return rc;
  dcgs2_mlp_s* q = new (std::nothrow) dcgs2_mlp_s();
  if (!q) return DCGS2_ENOMEM;
  q->ctx = ctx;
  q->s = s;
  q->L = nlayers;
  q->w.assign(widths, widths + nlayers + 1);
  q->max_batch = max_batch;
  int wmax = 0;
  for (int l = 0; l < nlayers; ++l) {
    q->offW.push_back(q->P);
    q->P += (int64_t)widths[l] * widths[l + 1];
    q->offb.push_back(q->P);
    q->P += widths[l + 1];
  }
  for (int l = 0; l <= nlayers; ++l) wmax = widths[l] > wmax ? widths[l] : wmax;
  if ((rc = alloc_f(&q->theta, q->P)) || (rc = alloc_f(&q->grad, q->P)) ||
      (rc = alloc_f(&q->m1, q->P)) || (rc = alloc_f(&q->m2, q->P)) ||
      (rc = alloc_f(&q->out, (int64_t)max_batch * widths[nlayers])) ||
      (rc = alloc_f(&q->dA, (int64_t)max_batch * wmax)) ||
      (rc = alloc_f(&q->dB, (int64_t)max_batch * wmax))) {
    release(q);
    return rc;
  }
  q->act.assign(nlayers > 1 ? nlayers - 1 : 0, nullptr);
  for (int l = 0; l + 1 < nlayers; ++l)
    if ((rc = alloc_f(&q->act[l], (int64_t)max_batch * widths[l + 1]))) { release(q); return rc; }
  if (hipMalloc((void**)&q->part, sizeof(double) * 256) != hipSuccess ||
      hipMalloc((void**)&q->loss, sizeof(double)) != hipSuccess) {
    release(q);
    return DCGS2_ENOMEM;
  }
  if (hipMemsetAsync(q->theta, 0, sizeof(float) * q->P, s) != hipSuccess ||
      hipMemsetAsync(q->m1, 0, sizeof(float) * q->P, s) != hipSuccess ||
      hipMemsetAsync(q->m2, 0, sizeof(float) * q->P, s) != hipSuccess ||
      hipMemsetAsync(q->grad, 0, sizeof(float) * q->P, s) != hipSuccess ||
      hipStreamSynchronize(s) != hipSuccess) {
    release(q);
    return DCGS2_EDEVICE;
  }
  *out = q;
  return DCGS2_OK;
}

int dcgs2_mlp_destroy(dcgs2_mlp q) {
  if (!q) return DCGS2_OK;
  (void)hipStreamSynchronize(q->s);
  release(q);
  return DCGS2_OK;
}

int dcgs2_mlp_num_params(dcgs2_mlp q, int64_t* n) {
  if (!q || !n) return DCGS2_EINVAL;
  *n = q->P;
  return DCGS2_OK;
}

int dcgs2_mlp_set_params(dcgs2_mlp q, const float* host) {
  if (!q || !host) return DCGS2_EINVAL;
  CK(hipMemcpyAsync(q->theta, host, sizeof(float) * q->P, hipMemcpyHostToDevice, q->s));
  CK(hipMemsetAsync(q->m1, 0, sizeof(float) * q->P, q->s));
  CK(hipMemsetAsync(q->m2, 0, sizeof(float) * q->P, q->s));
  CK(hipStreamSynchronize(q->s));
  q->t = 0;
  return DCGS2_OK;
}

int dcgs2_mlp_get_params(dcgs2_mlp q, float* host) {
  if (!q || !host) return DCGS2_EINVAL;
  CK(hipMemcpyAsync(host, q->theta, sizeof(float) * q->P, hipMemcpyDeviceToHost, q->s));
  CK(hipStreamSynchronize(q->s));
  return DCGS2_OK;
}

int dcgs2_mlp_get_grads(dcgs2_mlp q, float* host) {
  if (!q || !host) return DCGS2_EINVAL;
  CK(hipMemcpyAsync(host, q->grad, sizeof(float) * q->P, hipMemcpyDeviceToHost, q->s));
  CK(hipStreamSynchronize(q->s));
  return DCGS2_OK;
}

int dcgs2_mlp_forward(dcgs2_mlp q, int32_t batch, const float* X, float* Y) {
  if (!q || !X || !Y || batch < 1 || batch > q->max_batch) return DCGS2_EINVAL;
  int rc = forward(q, batch, X);
  if (rc) return rc;
  CK(hipMemcpyAsync(Y, q->out, sizeof(float) * (size_t)batch * q->w[q->L],
                    hipMemcpyDeviceToDevice, q->s));
  CK(hipStreamSynchronize(q->s));
  return DCGS2_OK;
}

int dcgs2_mlp_loss_grad(dcgs2_mlp q, int32_t batch, const float* X, const float* T,
                        double* loss_host) {
  if (!q || !X || !T || batch < 1 || batch > q->max_batch) return DCGS2_EINVAL;
  int rc = forward(q, batch, X);
  if (rc) return rc;
  const int L = q->L;
  const int64_t count = (int64_t)batch * q->w[L];
  float* dZ = q->dA;
  float* other = q->dB;
  CK(launch_mse(count, q->out, T, dZ, q->part, q->loss, q->s));
  for (int l = L - 1; l >= 0; --l) {
    const int K = q->w[l], N = q->w[l + 1];
    const float* Ain = l == 0 ? X : q->act[l - 1];
    // dW_l = A_in^T dZ_l (K x N), db_l = column sums of dZ_l
    CK(launch_gemm_f32(1, 0, GEMM_PLAIN, K, N, batch, Ain, K, dZ, N, q->grad + q->offW[l], N,
                       nullptr, nullptr, q->s));
    CK(launch_colsum(batch, N, dZ, N, q->grad + q->offb[l], q->s));
    if (l > 0) {
      // dZ_{l-1} = (dZ_l W_l^T) masked by ReLU'(Z_{l-1}) (A_in > 0 exactly where Z > 0)
      CK(launch_gemm_f32(0, 1, GEMM_MASK, batch, K, N, dZ, N, q->theta + q->offW[l], N, other, K,
                         nullptr, Ain, q->s));
      float* tmp = dZ;
      dZ = other;
      other = tmp;
    }
  }
  if (loss_host)
    CK(hipMemcpyAsync(loss_host, q->loss, sizeof(double), hipMemcpyDeviceToHost, q->s));
  CK(hipStreamSynchronize(q->s));
  return DCGS2_OK;
}

int dcgs2_mlp_adam(dcgs2_mlp q, float lr, float beta1, float beta2, float eps) {
  if (!q || !(lr > 0.f) || !(beta1 >= 0.f && beta1 < 1.f) || !(beta2 >= 0.f && beta2 < 1.f) ||
      !(eps > 0.f))
    return DCGS2_EINVAL;
  q->t += 1;
  const double c1 = 1.0 / (1.0 - std::pow((double)beta1, (double)q->t));
  const double c2 = 1.0 / (1.0 - std::pow((double)beta2, (double)q->t));
  CK(launch_adam(q->P, q->theta, q->grad, q->m1, q->m2, lr, beta1, beta2, eps, (float)c1,
                 (float)c2, q->s));
  CK(hipStreamSynchronize(q->s));
  return DCGS2_OK;
}

int dcgs2_guess_features(dcgs2_ctx ctx, int32_t count, int32_t n, int32_t nc, const double* b,
                         const float* prm, int32_t np, int32_t fdim, float* feat, double* scale) {
  if (!ctx || !b || !feat || !scale || count < 1 || nc < 1 || n < nc || n % nc != 0 ||
      nc > 64 || np < 0 || (np > 0 && !prm) || fdim < nc * nc + np)
    return DCGS2_EINVAL;
  hipStream_t s;
  int rc = ctx_prepare(ctx, &s);
  if (rc) return rc;
  CK(launch_features(count, n, nc, b, prm, np, fdim, feat, scale, s));
  CK(hipStreamSynchronize(s));
  return DCGS2_OK;
}

int dcgs2_guess_targets(dcgs2_ctx ctx, int32_t count, int32_t n, int32_t nc, const double* x,
                        const double* scale, double gain, float* t) {
  if (!ctx || !x || !scale || !t || count < 1 || nc < 1 || n < nc || n % nc != 0 ||
      !(gain > 0.0) || !std::isfinite(gain))
    return DCGS2_EINVAL;
  hipStream_t s;
  int rc = ctx_prepare(ctx, &s);
  if (rc) return rc;
  CK(launch_targets(count, n, nc, x, scale, gain, t, s));
  CK(hipStreamSynchronize(s));
  return DCGS2_OK;
}

int dcgs2_guess_prolong(dcgs2_ctx ctx, int32_t count, int32_t n, int32_t nc, const float* y,
                        const double* scale, double gain, double* x0) {
  if (!ctx || !y || !scale || !x0 || count < 1 || nc < 2 || n < nc || n % nc != 0 ||
      !(gain > 0.0) || !std::isfinite(gain))
    return DCGS2_EINVAL;
  hipStream_t s;
  int rc = ctx_prepare(ctx, &s);
  if (rc) return rc;
  CK(launch_prolong(count, n, nc, y, scale, gain, x0, s));
  CK(hipStreamSynchronize(s));
  return DCGS2_OK;
}

}  // extern "C"
