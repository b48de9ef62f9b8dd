// gz_select.h -- launchers of the selector training kernels (gz_select.hip).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace gzs {

constexpr uint32_t MLP_PARAMS = 643;    // W1[32][16], b1[32], W2[3][32], b2[3]
constexpr uint32_t MLP_ROW = 68;        // per-sample backward terms
constexpr uint32_t MLP_MAX_BATCH = 65536;

// bytes of the training workspace (per-sample rows and per-group sums)
size_t mlp_workspace_bytes();
hipError_t launch_mlp_grad(const float* w, const int8_t* feat, const uint8_t* label,
                           uint32_t nsamp, float* ws, float* grad, float* loss, hipStream_t st);
hipError_t launch_mlp_adam(float* w, const float* g, float* m, float* v, float lr, float bc1,
                           float bc2, hipStream_t st);

}  // namespace gzs
