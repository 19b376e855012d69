// Internal interface of the learned-extrapolation MLP kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/cpqr.h"

namespace cpqr {

constexpr int MLP_FEATURES = CPQR_MLP_FEATURES;
constexpr int MLP_HIDDEN = CPQR_MLP_HIDDEN;
constexpr int MLP_PARAMS = CPQR_MLP_PARAMS;
constexpr int MLP_OFF_W1 = 0;
constexpr int MLP_OFF_B1 = MLP_HIDDEN * MLP_FEATURES;
constexpr int MLP_OFF_W2 = MLP_OFF_B1 + MLP_HIDDEN;
constexpr int MLP_OFF_B2 = MLP_OFF_W2 + MLP_HIDDEN;
static_assert(MLP_OFF_B2 + 1 == MLP_PARAMS, "parameter layout");
constexpr int MLP_GRAD_PER_WAVE = 16;   // samples per wave in the gradient kernel

int mlp_grad_chunks(int n, int per);
hipError_t launch_mlp_forward(const float* w, const float* X, int n, float* y, hipStream_t st);
// Mean-squared-error gradient over n samples (rows idx[0..n) of X/Y, or the
// first n rows when idx is null); partial holds mlp_grad_chunks(n) x
// MLP_PARAMS floats, loss_part that many floats.
hipError_t launch_mlp_grad(const float* w, const float* X, const float* Y, const int* idx, int n,
                           float* partial, float* loss_part, float* grad, float* loss, hipStream_t st);
hipError_t launch_mlp_adam(float* w, const float* g, float* m, float* v, int t, float lr, float b1,
                           float b2, float eps, hipStream_t st);

}  // namespace cpqr
