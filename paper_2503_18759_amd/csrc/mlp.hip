// Two-layer MLP for the learned extrapolation weight (a feature of this
// library, not part of the paper): features (F) -> 64 tanh units -> 1 linear
// output, float32, mean-squared-error loss, Adam.
//
// Parameter layout (w, float32, MLP_PARAMS entries):
//   W1[j * F + f] (64 x F, row-major), b1[64], w2[64], b2[1].
//
//  * mlp_forward:  one thread per sample.
//  * mlp_grad_partial: one wave per chunk of samples; lane j owns hidden unit
//    j.  For each sample the output is a wave sum, then lane j accumulates
//    its own gradient terms (F + 3 values).  Partial sums go to
//    partial[chunk][param] and are added in chunk order by mlp_grad_reduce,
//    so the gradient is deterministic.
//  * mlp_adam: elementwise Adam step with bias correction.
#include "common.h"
#include "mlp.h"

namespace cpqr {

static_assert(MLP_HIDDEN == 64, "one wave lane per hidden unit");

__device__ __forceinline__ float mlp_unit(const float* __restrict__ w, const float* x, int j, float* hj) {
  float z = w[MLP_OFF_B1 + j];
#pragma unroll
  for (int f = 0; f < MLP_FEATURES; ++f) z = fmaf(w[MLP_OFF_W1 + j * MLP_FEATURES + f], x[f], z);
  const float h = tanhf(z);
  *hj = h;
  return w[MLP_OFF_W2 + j] * h;
}

__global__ __launch_bounds__(256) void mlp_forward_kernel(const float* __restrict__ w,
                                                          const float* __restrict__ X, int n,
                                                          float* __restrict__ y) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  float x[MLP_FEATURES];
#pragma unroll
  for (int f = 0; f < MLP_FEATURES; ++f) x[f] = X[(int64_t)i * MLP_FEATURES + f];
  float out = w[MLP_OFF_B2];
  for (int j = 0; j < MLP_HIDDEN; ++j) {
    float h;
    out += mlp_unit(w, x, j, &h);
  }
  y[i] = out;
}

// Block = one wave (64 lanes).  Samples idx[chunk * per .. +per) (or rows
// chunk * per .. when idx is null).
__global__ __launch_bounds__(64) void mlp_grad_partial(const float* __restrict__ w,
                                                       const float* __restrict__ X,
                                                       const float* __restrict__ Y,
                                                       const int* __restrict__ idx, int n, int per,
                                                       float inv_n, float* __restrict__ partial,
                                                       float* __restrict__ loss_part) {
  const int j = threadIdx.x;
  const int i0 = blockIdx.x * per;
  int i1 = i0 + per;
  if (i1 > n) i1 = n;
  float gW1[MLP_FEATURES];
#pragma unroll
  for (int f = 0; f < MLP_FEATURES; ++f) gW1[f] = 0.f;
  float gb1 = 0.f, gw2 = 0.f, gb2 = 0.f, loss = 0.f;
  const float w2j = w[MLP_OFF_W2 + j];
  for (int i = i0; i < i1; ++i) {
    const int r = idx ? idx[i] : i;
    float x[MLP_FEATURES];
#pragma unroll
    for (int f = 0; f < MLP_FEATURES; ++f) x[f] = X[(int64_t)r * MLP_FEATURES + f];
    float h;
    const float contrib = mlp_unit(w, x, j, &h);
    const float yhat = wave_sum_f(contrib) + w[MLP_OFF_B2];
    const float e = yhat - Y[r];
    const float dy = e * inv_n;
    loss += 0.5f * e * e * inv_n;
    gw2 = fmaf(dy, h, gw2);
    gb2 += dy;
    const float dz = dy * w2j * (1.f - h * h);
    gb1 += dz;
#pragma unroll
    for (int f = 0; f < MLP_FEATURES; ++f) gW1[f] = fmaf(dz, x[f], gW1[f]);
  }
  float* out = partial + (int64_t)blockIdx.x * MLP_PARAMS;
#pragma unroll
  for (int f = 0; f < MLP_FEATURES; ++f) out[MLP_OFF_W1 + j * MLP_FEATURES + f] = gW1[f];
  out[MLP_OFF_B1 + j] = gb1;
  out[MLP_OFF_W2 + j] = gw2;
  if (j == 0) {
    out[MLP_OFF_B2] = gb2;
    loss_part[blockIdx.x] = loss;
  }
}

__global__ __launch_bounds__(256) void mlp_grad_reduce(const float* __restrict__ partial, int chunks,
                                                       const float* __restrict__ loss_part,
                                                       float* __restrict__ grad, float* __restrict__ loss) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p < MLP_PARAMS) {
    float s = 0.f;
    for (int c = 0; c < chunks; ++c) s += partial[(int64_t)c * MLP_PARAMS + p];
    grad[p] = s;
  }
  if (p == 0) {
    float s = 0.f;
    for (int c = 0; c < chunks; ++c) s += loss_part[c];
    *loss = s;
  }
}

__global__ __launch_bounds__(256) void mlp_adam_kernel(float* __restrict__ w, const float* __restrict__ g,
                                                       float* __restrict__ m, float* __restrict__ v,
                                                       float lr, float b1, float b2, float eps,
                                                       float c1, float c2) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= MLP_PARAMS) return;
  const float gp = g[p];
  const float mp = b1 * m[p] + (1.f - b1) * gp;
  const float vp = b2 * v[p] + (1.f - b2) * gp * gp;
  m[p] = mp;
  v[p] = vp;
  const float mh = mp / c1, vh = vp / c2;
  w[p] -= lr * mh / (sqrtf(vh) + eps);
}

int mlp_grad_chunks(int n, int per) { return n <= 0 ? 0 : (n + per - 1) / per; }

hipError_t launch_mlp_forward(const float* w, const float* X, int n, float* y, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(mlp_forward_kernel, dim3((n + 255) / 256), dim3(256), 0, st, w, X, n, y);
  return hipGetLastError();
}

hipError_t launch_mlp_grad(const float* w, const float* X, const float* Y, const int* idx, int n,
                           float* partial, float* loss_part, float* grad, float* loss, hipStream_t st) {
  if (n <= 0) return hipErrorInvalidValue;
  const int chunks = mlp_grad_chunks(n, MLP_GRAD_PER_WAVE);
  hipLaunchKernelGGL(mlp_grad_partial, dim3(chunks), dim3(64), 0, st, w, X, Y, idx, n, MLP_GRAD_PER_WAVE,
                     1.f / (float)n, partial, loss_part);
  hipLaunchKernelGGL(mlp_grad_reduce, dim3((MLP_PARAMS + 255) / 256), dim3(256), 0, st, partial, chunks,
                     loss_part, grad, loss);
  return hipGetLastError();
}

hipError_t launch_mlp_adam(float* w, const float* g, float* m, float* v, int t, float lr, float b1,
                           float b2, float eps, hipStream_t st) {
  const float c1 = 1.f - powf(b1, (float)t), c2 = 1.f - powf(b2, (float)t);
  hipLaunchKernelGGL(mlp_adam_kernel, dim3((MLP_PARAMS + 255) / 256), dim3(256), 0, st, w, g, m, v, lr, b1,
                     b2, eps, c1, c2);
  return hipGetLastError();
}

}  // namespace cpqr
