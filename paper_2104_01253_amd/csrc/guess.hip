// Learned initial guess for GMRES: grid transfers, feature assembly and the
// multilayer perceptron's forward pass, backward pass and Adam update, in FP32.
//
// The perceptron's products are dense contractions, so they run on the matrix
// cores: gemm_f32_kernel tiles C = op(A) op(B) into 64 x 64 blocks per
// workgroup (four wavefronts of 32 x 32, each 2 x 2 MFMA 16x16x4 FP32 tiles),
// staging 16-deep K slices of both operands through LDS.  Transposed operands
// are read transposed while staging, so the forward product X W, the input
// gradient dZ W^T and the weight gradient X^T dZ share one kernel.  Epilogues:
// bias, bias + ReLU, or the ReLU derivative mask.
//
// Grid transfers (fine n x n interior grid, x fastest, h = 1/(n+1); coarse
// nc x nc, r = n / nc):
//   restriction   -- mean of each r x r block;
//   prolongation  -- tensor-product linear interpolation of the values at the
//                    coarse block centres, zero at the Dirichlet boundary.
#include <hip/hip_runtime.h>
#include <math.h>

#include "internal.h"

namespace dcgs2 {
namespace {

constexpr int GBM = 64, GBN = 64, GBK = 16, GPAD = 4, GTHREADS = 256;
typedef float floatx4 __attribute__((ext_vector_type(4)));

template <bool TA, bool TB, int EPI>
__global__ __launch_bounds__(GTHREADS) void gemm_f32_kernel(
    int M, int N, int K, const float* __restrict__ A, int lda, const float* __restrict__ B,
    int ldb, float* __restrict__ C, int ldc, const float* __restrict__ bias,
    const float* __restrict__ mask) {
  __shared__ float As[GBK][GBM + GPAD];
  __shared__ float Bs[GBK][GBN + GPAD];
  const int t = threadIdx.x;
  const int lane = t & 63, wave = t >> 6;
  const int i0 = blockIdx.y * GBM, j0 = blockIdx.x * GBN;
  const int wr = (wave >> 1) * 32, wc = (wave & 1) * 32;
  floatx4 acc[2][2];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b) acc[a][b] = floatx4{0.f, 0.f, 0.f, 0.f};
  for (int k0 = 0; k0 < K; k0 += GBK) {
    // stage op(A)[i0..i0+64, k0..k0+16] as As[k][i]
    if (!TA) {
      const int i = t >> 2, kq = (t & 3) * 4;
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int gi = i0 + i, gk = k0 + kq + e;
        As[kq + e][i] = (gi < M && gk < K) ? A[(int64_t)gi * lda + gk] : 0.f;
      }
    } else {
      const int k = t >> 4, iq = (t & 15) * 4;
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int gi = i0 + iq + e, gk = k0 + k;
        As[k][iq + e] = (gi < M && gk < K) ? A[(int64_t)gk * lda + gi] : 0.f;
      }
    }
    // stage op(B)[k0..k0+16, j0..j0+64] as Bs[k][j]
    if (!TB) {
      const int k = t >> 4, jq = (t & 15) * 4;
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int gj = j0 + jq + e, gk = k0 + k;
        Bs[k][jq + e] = (gj < N && gk < K) ? B[(int64_t)gk * ldb + gj] : 0.f;
      }
    } else {
      const int j = t >> 2, kq = (t & 3) * 4;
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int gj = j0 + j, gk = k0 + kq + e;
        Bs[kq + e][j] = (gj < N && gk < K) ? B[(int64_t)gj * ldb + gk] : 0.f;
      }
    }
    __syncthreads();
    // 16x16x4 MFMA: lane holds A[row = lane % 16][k = lane / 16] and
    // B[k = lane / 16][col = lane % 16]
    const int lr = lane & 15, lk = lane >> 4;
#pragma unroll
    for (int kk = 0; kk < GBK; kk += 4) {
      float av[2], bv[2];
#pragma unroll
      for (int a = 0; a < 2; ++a) av[a] = As[kk + lk][wr + a * 16 + lr];
#pragma unroll
      for (int b = 0; b < 2; ++b) bv[b] = Bs[kk + lk][wc + b * 16 + lr];
#pragma unroll
      for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b)
          acc[a][b] = __builtin_amdgcn_mfma_f32_16x16x4f32(av[a], bv[b], acc[a][b], 0, 0, 0);
    }
    __syncthreads();
  }
  // result element (row 4 * (lane / 16) + e, column lane % 16) of each 16 x 16 tile
  const int lc = lane & 15, lrow = (lane >> 4) * 4;
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int gi = i0 + wr + a * 16 + lrow + e, gj = j0 + wc + b * 16 + lc;
        if (gi < M && gj < N) {
          float v = acc[a][b][e];
          if (EPI == GEMM_BIAS || EPI == GEMM_BIAS_RELU) v += bias[gj];
          if (EPI == GEMM_BIAS_RELU) v = fmaxf(v, 0.f);
          if (EPI == GEMM_MASK) v = mask[(int64_t)gi * ldc + gj] > 0.f ? v : 0.f;
          C[(int64_t)gi * ldc + gj] = v;
        }
      }
}

// db[j] = sum_i dZ[i, j], rows summed in order.
__global__ void colsum_kernel(int rows, int cols, const float* __restrict__ dZ, int ld,
                              float* __restrict__ out) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= cols) return;
  float s = 0.f;
  for (int i = 0; i < rows; ++i) s += dZ[(int64_t)i * ld + j];
  out[j] = s;
}

// dY = 2 (Y - T) / count and per-workgroup partial sums of (Y - T)^2 (in double).
__global__ __launch_bounds__(256) void mse_grad_kernel(int64_t count, const float* __restrict__ Y,
                                                       const float* __restrict__ T,
                                                       float* __restrict__ dY,
                                                       double* __restrict__ part) {
  __shared__ double sh[256];
  double s = 0.0;
  const float sc = (float)(2.0 / (double)count);
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < count;
       i += (int64_t)gridDim.x * 256) {
    const float d = Y[i] - T[i];
    dY[i] = sc * d;
    s += (double)d * (double)d;
  }
  sh[threadIdx.x] = s;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) sh[threadIdx.x] += sh[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = sh[0];
}

// loss = sum(part) / count, one workgroup, partials summed in order.
__global__ void mse_finish_kernel(int nparts, int64_t count, const double* __restrict__ part,
                                  double* __restrict__ loss) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    double s = 0.0;
    for (int i = 0; i < nparts; ++i) s += part[i];
    *loss = s / (double)count;
  }
}

// Adam (Kingma & Ba, Algorithm 1); c1 = 1/(1 - beta1^t), c2 = 1/(1 - beta2^t).
__global__ void adam_kernel(int64_t n, float* __restrict__ theta, const float* __restrict__ g,
                            float* __restrict__ m, float* __restrict__ v, float lr, float b1,
                            float b2, float eps, float c1, float c2) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const float gi = g[i];
  const float mi = b1 * m[i] + (1.f - b1) * gi;
  const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
  m[i] = mi;
  v[i] = vi;
  theta[i] -= lr * (mi * c1) / (sqrtf(vi * c2) + eps);
}

// One workgroup per instance: coarse means of b (double, in LDS), their RMS s,
// then feat = [R(b)/s, params, 0...] and scale = s.
__global__ __launch_bounds__(256) void features_kernel(int n, int nc, const double* __restrict__ b,
                                                       const float* __restrict__ prm, int np,
                                                       int fdim, float* __restrict__ feat,
                                                       double* __restrict__ scale) {
  extern __shared__ double bc[];          // nc * nc coarse means, then 256 partials
  double* red = bc + nc * nc;
  const int inst = blockIdx.x;
  const int r = n / nc;
  const double* bi = b + (int64_t)inst * n * n;
  const double inv = 1.0 / (double)(r * r);
  double ss = 0.0;
  for (int c = threadIdx.x; c < nc * nc; c += blockDim.x) {
    const int I = c % nc, J = c / nc;     // x and y block indices
    double s = 0.0;
    for (int y = 0; y < r; ++y)
      for (int x = 0; x < r; ++x) s += bi[(int64_t)(J * r + y) * n + I * r + x];
    s *= inv;
    bc[c] = s;
    ss += s * s;
  }
  red[threadIdx.x] = ss;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  const double s = sqrt(red[0] / (double)(nc * nc));
  float* f = feat + (int64_t)inst * fdim;
  for (int c = threadIdx.x; c < fdim; c += blockDim.x) {
    float v = 0.f;
    if (c < nc * nc) v = s > 0.0 ? (float)(bc[c] / s) : 0.f;
    else if (c < nc * nc + np) v = prm[(int64_t)inst * np + (c - nc * nc)];
    f[c] = v;
  }
  if (threadIdx.x == 0) scale[inst] = s;
}

// Training targets: t = gain R(x) / s (zero when s = 0); one thread per coarse point.
__global__ void targets_kernel(int count, int n, int nc, const double* __restrict__ x,
                               const double* __restrict__ scale, double gain,
                               float* __restrict__ t) {
  const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= (int64_t)count * nc * nc) return;
  const int inst = (int)(g / (nc * nc));
  const int c = (int)(g % (nc * nc));
  const int I = c % nc, J = c / nc;
  const int r = n / nc;
  const double* xi = x + (int64_t)inst * n * n;
  double s = 0.0;
  for (int y = 0; y < r; ++y)
    for (int xx = 0; xx < r; ++xx) s += xi[(int64_t)(J * r + y) * n + I * r + xx];
  s /= (double)(r * r);
  const double sc = scale[inst];
  t[g] = sc > 0.0 ? (float)(gain * s / sc) : 0.f;
}

// 1-D interpolation weights of fine point i: value = wl * c[kl] + wr * c[kl + 1],
// kl = -1 and kl + 1 = nc denote the zero boundary values.
__device__ __forceinline__ void interp_1d(int i, int n, int nc, int* kl, double* wl,
                                          double* wr) {
  const int r = n / nc;
  const double h = 1.0 / (double)(n + 1);
  const double x = (double)(i + 1) * h;
  const double half = 0.5 * (double)(r - 1);
  const double c0 = (half + 1.0) * h;                                 // first centre
  const double cl = ((double)(nc - 1) * r + half + 1.0) * h;          // last centre
  if (x < c0) {
    *kl = -1;
    *wr = x / c0;
    *wl = 1.0 - *wr;
  } else if (x >= cl) {
    *kl = nc - 1;
    *wl = (1.0 - x) / (1.0 - cl);
    *wr = 1.0 - *wl;
  } else {
    int k = (int)floor(((double)i - half) / (double)r);
    if (k > nc - 2) k = nc - 2;
    const double xa = ((double)k * r + half + 1.0) * h;
    const double xb = ((double)(k + 1) * r + half + 1.0) * h;
    *kl = k;
    *wr = (x - xa) / (xb - xa);
    *wl = 1.0 - *wr;
  }
}

// x0 = (s / gain) P(y): one thread per fine point.
__global__ void prolong_kernel(int count, int n, int nc, const float* __restrict__ y,
                               const double* __restrict__ scale, double gain,
                               double* __restrict__ x0) {
  const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= (int64_t)count * n * n) return;
  const int inst = (int)(g / ((int64_t)n * n));
  const int p = (int)(g % ((int64_t)n * n));
  const int ix = p % n, iy = p / n;
  int kx, ky;
  double wxl, wxr, wyl, wyr;
  interp_1d(ix, n, nc, &kx, &wxl, &wxr);
  interp_1d(iy, n, nc, &ky, &wyl, &wyr);
  const float* yi = y + (int64_t)inst * nc * nc;
  auto at = [&](int I, int J) -> double {
    return (I < 0 || I >= nc || J < 0 || J >= nc) ? 0.0 : (double)yi[J * nc + I];
  };
  const double v = wyl * (wxl * at(kx, ky) + wxr * at(kx + 1, ky)) +
                   wyr * (wxl * at(kx, ky + 1) + wxr * at(kx + 1, ky + 1));
  x0[g] = (scale[inst] / gain) * v;
}

inline unsigned blocks_for(int64_t n, int bs) { return (unsigned)((n + bs - 1) / bs); }

}  // namespace

hipError_t launch_gemm_f32(int ta, int tb, int epi, int M, int N, int K, const float* A, int lda,
                           const float* B, int ldb, float* C, int ldc, const float* bias,
                           const float* mask, hipStream_t s) {
  if (M <= 0 || N <= 0) return hipSuccess;
  const dim3 grid(blocks_for(N, GBN), blocks_for(M, GBM));
#define DCGS2_G(TA, TB, E)                                                          \
  gemm_f32_kernel<TA, TB, E><<<grid, GTHREADS, 0, s>>>(M, N, K, A, lda, B, ldb, C, ldc, bias, mask)
  if (!ta && !tb) {
    if (epi == GEMM_BIAS) DCGS2_G(false, false, GEMM_BIAS);
    else if (epi == GEMM_BIAS_RELU) DCGS2_G(false, false, GEMM_BIAS_RELU);
    else DCGS2_G(false, false, GEMM_PLAIN);
  } else if (ta && !tb) {
    DCGS2_G(true, false, GEMM_PLAIN);
  } else if (!ta && tb) {
    if (epi == GEMM_MASK) DCGS2_G(false, true, GEMM_MASK);
    else DCGS2_G(false, true, GEMM_PLAIN);
  } else {
    DCGS2_G(true, true, GEMM_PLAIN);
  }
#undef DCGS2_G
  return hipGetLastError();
}

hipError_t launch_colsum(int rows, int cols, const float* dZ, int ld, float* out, hipStream_t s) {
  colsum_kernel<<<blocks_for(cols, 256), 256, 0, s>>>(rows, cols, dZ, ld, out);
  return hipGetLastError();
}

int mse_parts(int64_t count) {
  const int64_t b = (count + 255) / 256;
  return (int)(b < 256 ? (b < 1 ? 1 : b) : 256);
}

hipError_t launch_mse(int64_t count, const float* Y, const float* T, float* dY, double* part,
                      double* loss, hipStream_t s) {
  const int np = mse_parts(count);
  mse_grad_kernel<<<np, 256, 0, s>>>(count, Y, T, dY, part);
  mse_finish_kernel<<<1, 64, 0, s>>>(np, count, part, loss);
  return hipGetLastError();
}

hipError_t launch_adam(int64_t n, float* theta, const float* g, float* m, float* v, float lr,
                       float b1, float b2, float eps, float c1, float c2, hipStream_t s) {
  adam_kernel<<<blocks_for(n, 256), 256, 0, s>>>(n, theta, g, m, v, lr, b1, b2, eps, c1, c2);
  return hipGetLastError();
}

hipError_t launch_features(int count, int n, int nc, const double* b, const float* prm, int np,
                           int fdim, float* feat, double* scale, hipStream_t s) {
  const size_t sm = sizeof(double) * ((size_t)nc * nc + 256);
  features_kernel<<<count, 256, sm, s>>>(n, nc, b, prm, np, fdim, feat, scale);
  return hipGetLastError();
}

hipError_t launch_targets(int count, int n, int nc, const double* x, const double* scale,
                          double gain, float* t, hipStream_t s) {
  targets_kernel<<<blocks_for((int64_t)count * nc * nc, 256), 256, 0, s>>>(count, n, nc, x, scale,
                                                                          gain, t);
  return hipGetLastError();
}

hipError_t launch_prolong(int count, int n, int nc, const float* y, const double* scale,
                          double gain, double* x0, hipStream_t s) {
  prolong_kernel<<<blocks_for((int64_t)count * n * n, 256), 256, 0, s>>>(count, n, nc, y, scale,
                                                                         gain, x0);
  return hipGetLastError();
}

}  // namespace dcgs2
