// mlp.hip -- the autotuner's cost model: a small fp32 multilayer perceptron
// (F inputs -> H -> H -> 1, ReLU after the two hidden layers) with forward,
// backward, mean-squared-error gradient and Adam kernels.
//
// Parameter layout (one float array): W1[F][H], b1[H], W2[H][H], b2[H],
// W3[H], b3.  Activations act = [h1 (B x H), h2 (B x H)] post-ReLU.
// Reductions over the batch are plain loops (no atomics), so every result is
// deterministic.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/ks.h"

namespace ks {

struct MlpView {
  const float *W1, *b1, *W2, *b2, *W3, *b3;
};
__host__ __device__ inline MlpView mlp_view(const float *p, uint32_t F, uint32_t H) {
  MlpView v;
  v.W1 = p;
  v.b1 = v.W1 + (size_t)F * H;
  v.W2 = v.b1 + H;
  v.b2 = v.W2 + (size_t)H * H;
  v.W3 = v.b2 + H;
  v.b3 = v.W3 + H;
  return v;
}

// out[b][j] = relu?(sum_i in[b][i] W[i][j] + bias[j]); one thread per (b, j).
__global__ __launch_bounds__(256) void k_dense(const float *in, const float *W, const float *bias, float *out,
                                               uint32_t B, uint32_t I, uint32_t J, int relu) {
  const size_t idx = (size_t)blockIdx.x * 256 + threadIdx.x;
  if (idx >= (size_t)B * J) return;
  const uint32_t b = (uint32_t)(idx / J), j = (uint32_t)(idx % J);
  float s = bias[j];
  for (uint32_t i = 0; i < I; i++) s = fmaf(in[(size_t)b * I + i], W[(size_t)i * J + j], s);
  out[idx] = relu ? fmaxf(s, 0.f) : s;
}

// dY = 2 (Y - T) / B, loss = mean((Y - T)^2) (one block).
__global__ __launch_bounds__(256) void k_mse(const float *Y, const float *T, float *dY, float *loss, uint32_t B) {
  __shared__ float red[256];
  float s = 0.f;
  for (uint32_t b = threadIdx.x; b < B; b += 256) {
    const float d = Y[b] - T[b];
    dY[b] = 2.f * d / (float)B;
    s = fmaf(d, d, s);
  }
  red[threadIdx.x] = s;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) *loss = red[0] / (float)B;
}

// Backward of out = relu(in W + bias) given dOut (masked by the ReLU of the
// stored post-activation `out` when relu != 0):
//   g[b][j]  = dOut[b][j] * [out[b][j] > 0]        (written to gmask)
//   dW[i][j] = sum_b in[b][i] g[b][j];  db[j] = sum_b g[b][j]
//   dIn[b][i] = sum_j g[b][j] W[i][j]              (if dIn != null)
__global__ __launch_bounds__(256) void k_mask(const float *dOut, const float *out, float *g, uint32_t n, int relu) {
  const size_t i = (size_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= n) return;
  g[i] = (!relu || out[i] > 0.f) ? dOut[i] : 0.f;
}
__global__ __launch_bounds__(256) void k_dense_wgrad(const float *in, const float *g, float *dW, float *db, uint32_t B,
                                                     uint32_t I, uint32_t J) {
  const size_t idx = (size_t)blockIdx.x * 256 + threadIdx.x;
  if (idx < (size_t)I * J) {
    const uint32_t i = (uint32_t)(idx / J), j = (uint32_t)(idx % J);
    float s = 0.f;
    for (uint32_t b = 0; b < B; b++) s = fmaf(in[(size_t)b * I + i], g[(size_t)b * J + j], s);
    dW[idx] = s;
  } else if (idx < (size_t)I * J + J) {
    const uint32_t j = (uint32_t)(idx - (size_t)I * J);
    float s = 0.f;
    for (uint32_t b = 0; b < B; b++) s += g[(size_t)b * J + j];
    db[j] = s;
  }
}
__global__ __launch_bounds__(256) void k_dense_xgrad(const float *g, const float *W, float *dIn, uint32_t B, uint32_t I,
                                                     uint32_t J) {
  const size_t idx = (size_t)blockIdx.x * 256 + threadIdx.x;
  if (idx >= (size_t)B * I) return;
  const uint32_t b = (uint32_t)(idx / I), i = (uint32_t)(idx % I);
  float s = 0.f;
  for (uint32_t j = 0; j < J; j++) s = fmaf(g[(size_t)b * J + j], W[(size_t)i * J + j], s);
  dIn[idx] = s;
}

__global__ __launch_bounds__(256) void k_adam(float *p, const float *g, float *m, float *v, uint32_t n, float lr,
                                              float b1, float b2, float eps, float c1, float c2) {
  const size_t i = (size_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= n) return;
  const float gi = g[i];
  const float mi = b1 * m[i] + (1.f - b1) * gi;
  const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
  m[i] = mi;
  v[i] = vi;
  p[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
}

inline dim3 grid_for(size_t n) { return dim3((unsigned)((n + 255) / 256)); }

}  // namespace ks

using namespace ks;

extern "C" {

uint32_t ks_mlp_param_count(uint32_t F, uint32_t H) { return F * H + H + H * H + H + H + 1; }

ks_status_t ks_mlp_forward(uint32_t F, uint32_t H, uint32_t B, const float *params, const float *X, float *Y,
                           float *act, void *stream) {
  if (!F || !H || !B || !params || !X || !Y || !act || F > 256 || H > 1024) return KS_ERR_INVALID_ARG;
  hipStream_t st = (hipStream_t)stream;
  const MlpView v = mlp_view(params, F, H);
  float *h1 = act, *h2 = act + (size_t)B * H;
  hipLaunchKernelGGL(k_dense, grid_for((size_t)B * H), dim3(256), 0, st, X, v.W1, v.b1, h1, B, F, H, 1);
  hipLaunchKernelGGL(k_dense, grid_for((size_t)B * H), dim3(256), 0, st, h1, v.W2, v.b2, h2, B, H, H, 1);
  hipLaunchKernelGGL(k_dense, grid_for(B), dim3(256), 0, st, h2, v.W3, v.b3, Y, B, H, 1u, 0);
  return hipGetLastError() == hipSuccess ? KS_OK : KS_ERR_DEVICE;
}

ks_status_t ks_mlp_mse_grad(uint32_t B, const float *Y, const float *T, float *dY, float *loss, void *stream) {
  if (!B || !Y || !T || !dY || !loss) return KS_ERR_INVALID_ARG;
  hipLaunchKernelGGL(k_mse, dim3(1), dim3(256), 0, (hipStream_t)stream, Y, T, dY, loss, B);
  return hipGetLastError() == hipSuccess ? KS_OK : KS_ERR_DEVICE;
}

ks_status_t ks_mlp_backward(uint32_t F, uint32_t H, uint32_t B, const float *params, const float *X, const float *act,
                            const float *dY, float *grads, float *scratch, void *stream) {
  if (!F || !H || !B || !params || !X || !act || !dY || !grads || !scratch || F > 256 || H > 1024)
    return KS_ERR_INVALID_ARG;
  hipStream_t st = (hipStream_t)stream;
  const MlpView v = mlp_view(params, F, H);
  float *gW1 = grads, *gb1 = gW1 + (size_t)F * H, *gW2 = gb1 + H, *gb2 = gW2 + (size_t)H * H, *gW3 = gb2 + H,
        *gb3 = gW3 + H;
  const float *h1 = act, *h2 = act + (size_t)B * H;
  float *d2 = scratch, *d1 = scratch + (size_t)B * H;
  // layer 3 (linear): dW3 = h2^T dY, db3 = sum dY, d(h2) = dY W3^T
  hipLaunchKernelGGL(k_dense_wgrad, grid_for((size_t)H + 1), dim3(256), 0, st, h2, dY, gW3, gb3, B, H, 1u);
  hipLaunchKernelGGL(k_dense_xgrad, grid_for((size_t)B * H), dim3(256), 0, st, dY, v.W3, d2, B, H, 1u);
  // layer 2: mask by relu(h2), dW2 = h1^T g2, d(h1) = g2 W2^T
  hipLaunchKernelGGL(k_mask, grid_for((size_t)B * H), dim3(256), 0, st, d2, h2, d2, (uint32_t)(B * H), 1);
  hipLaunchKernelGGL(k_dense_wgrad, grid_for((size_t)H * H + H), dim3(256), 0, st, h1, d2, gW2, gb2, B, H, H);
  hipLaunchKernelGGL(k_dense_xgrad, grid_for((size_t)B * H), dim3(256), 0, st, d2, v.W2, d1, B, H, H);
  // layer 1: mask by relu(h1), dW1 = X^T g1
  hipLaunchKernelGGL(k_mask, grid_for((size_t)B * H), dim3(256), 0, st, d1, h1, d1, (uint32_t)(B * H), 1);
  hipLaunchKernelGGL(k_dense_wgrad, grid_for((size_t)F * H + H), dim3(256), 0, st, X, d1, gW1, gb1, B, F, H);
  return hipGetLastError() == hipSuccess ? KS_OK : KS_ERR_DEVICE;
}

ks_status_t ks_mlp_adam(uint32_t n, float *params, const float *grads, float *m, float *v, float lr, float beta1,
                        float beta2, float eps, uint32_t step, void *stream) {
  if (!n || !params || !grads || !m || !v || !step) return KS_ERR_INVALID_ARG;
  float c1 = 1.f - powf(beta1, (float)step), c2 = 1.f - powf(beta2, (float)step);
  hipLaunchKernelGGL(k_adam, grid_for(n), dim3(256), 0, (hipStream_t)stream, params, grads, m, v, n, lr, beta1, beta2,
                     eps, c1, c2);
  return hipGetLastError() == hipSuccess ? KS_OK : KS_ERR_DEVICE;
}

}  // extern "C"
