// gz_select.hip -- training kernels of the learned predictor selector.
//
// The selector is an int8 network 16 -> 32 (ReLU) -> 3 that picks each
// tile's predictor (NONE, L1D, L2D).  It is trained as an fp32 "shadow"
// network with softmax cross-entropy on labels from exhaustive trial, then
// exported to int8.  Gradients are made deterministic: a per-sample kernel
// writes each sample's backward terms, and two reduction kernels sum them in
// a fixed order in fp64 (per group of 64 samples, then over the groups).
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include "gz_select.h"

namespace gzs {

constexpr int NIN = 16, NH = 32, NOUT = 3;
constexpr int NW1 = NH * NIN, NB1 = NH, NW2 = NOUT * NH, NB2 = NOUT;
constexpr int NPARAM = NW1 + NB1 + NW2 + NB2;  // 643
constexpr int ROW = NH + NH + NOUT + 1;         // dz1, h, dz2, loss

__global__ __launch_bounds__(256) void k_mlp_fwdbwd(const float* __restrict__ w,
                                                   const int8_t* __restrict__ feat,
                                                   const uint8_t* __restrict__ label,
                                                   uint32_t nsamp, float* __restrict__ ws) {
  __shared__ float sw[NPARAM];
  for (int k = threadIdx.x; k < NPARAM; k += blockDim.x) sw[k] = w[k];
  __syncthreads();
  const float* W1 = sw;
  const float* b1 = sw + NW1;
  const float* W2 = sw + NW1 + NB1;
  const float* b2 = sw + NW1 + NB1 + NW2;
  const uint32_t s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= nsamp) return;
  float* out = ws + (uint64_t)s * ROW;
  const uint32_t lab = label[s];
  if (lab >= NOUT) {  // RAW/ZERO tiles carry no label
    for (int k = 0; k < ROW; ++k) out[k] = 0.0f;
    return;
  }
  float f[NIN];
  for (int i = 0; i < NIN; ++i) f[i] = (float)feat[(uint64_t)s * NIN + i];
  float z1[NH], h[NH];
  for (int k = 0; k < NH; ++k) {
    float a = b1[k];
    for (int i = 0; i < NIN; ++i) a = a + W1[k * NIN + i] * f[i];
    z1[k] = a;
    h[k] = a > 0.0f ? a : 0.0f;
  }
  float z2[NOUT];
  for (int o = 0; o < NOUT; ++o) {
    float a = b2[o];
    for (int k = 0; k < NH; ++k) a = a + W2[o * NH + k] * h[k];
    z2[o] = a;
  }
  const float m = fmaxf(z2[0], fmaxf(z2[1], z2[2]));
  float e[NOUT], S = 0.0f;
  for (int o = 0; o < NOUT; ++o) {
    e[o] = expf(z2[o] - m);
    S = S + e[o];
  }
  float dz2[NOUT];
  for (int o = 0; o < NOUT; ++o) dz2[o] = e[o] / S - (o == (int)lab ? 1.0f : 0.0f);
  for (int k = 0; k < NH; ++k) {
    float d = 0.0f;
    for (int o = 0; o < NOUT; ++o) d = d + W2[o * NH + k] * dz2[o];
    out[k] = z1[k] > 0.0f ? d : 0.0f;  // dz1
    out[NH + k] = h[k];
  }
  for (int o = 0; o < NOUT; ++o) out[2 * NH + o] = dz2[o];
  out[2 * NH + NOUT] = logf(S) + m - z2[lab];
}

// Gradient sums in a fixed order, in two levels: block g sums every
// parameter over its GROUP consecutive samples (staged in LDS) into
// part[g][p]; then one thread per parameter adds the groups in group order.
// Slot NPARAM of a group holds the loss sum, slot NPARAM + 1 the number of
// labelled samples.
constexpr int GROUP = 64;
constexpr int PSTRIDE = NPARAM + 2;

__global__ __launch_bounds__(704) void k_mlp_partial(const int8_t* __restrict__ feat,
                                                    const uint8_t* __restrict__ label,
                                                    uint32_t nsamp, const float* __restrict__ ws,
                                                    double* __restrict__ part) {
  __shared__ float srow[GROUP * ROW];
  __shared__ float sfeat[GROUP * NIN];
  __shared__ uint32_t slab[GROUP];
  const uint32_t s0 = blockIdx.x * GROUP;
  const uint32_t m = min((uint32_t)GROUP, nsamp - s0);
  for (uint32_t k = threadIdx.x; k < m * ROW; k += blockDim.x)
    srow[k] = ws[(uint64_t)s0 * ROW + k];
  for (uint32_t k = threadIdx.x; k < m * NIN; k += blockDim.x)
    sfeat[k] = (float)feat[(uint64_t)s0 * NIN + k];
  for (uint32_t k = threadIdx.x; k < m; k += blockDim.x) slab[k] = label[s0 + k];
  __syncthreads();
  const int p = threadIdx.x;
  if (p > NPARAM + 1) return;
  double acc = 0.0;
  if (p < NW1) {
    const int k = p / NIN, i = p % NIN;
    for (uint32_t s = 0; s < m; ++s) acc += (double)srow[s * ROW + k] * (double)sfeat[s * NIN + i];
  } else if (p < NW1 + NB1) {
    const int k = p - NW1;
    for (uint32_t s = 0; s < m; ++s) acc += (double)srow[s * ROW + k];
  } else if (p < NW1 + NB1 + NW2) {
    const int o = (p - NW1 - NB1) / NH, k = (p - NW1 - NB1) % NH;
    for (uint32_t s = 0; s < m; ++s)
      acc += (double)srow[s * ROW + 2 * NH + o] * (double)srow[s * ROW + NH + k];
  } else if (p < NPARAM) {
    const int o = p - NW1 - NB1 - NW2;
    for (uint32_t s = 0; s < m; ++s) acc += (double)srow[s * ROW + 2 * NH + o];
  } else if (p == NPARAM) {
    for (uint32_t s = 0; s < m; ++s) acc += (double)srow[s * ROW + 2 * NH + NOUT];
  } else {
    for (uint32_t s = 0; s < m; ++s) acc += slab[s] < NOUT ? 1.0 : 0.0;
  }
  part[(uint64_t)blockIdx.x * PSTRIDE + p] = acc;
}

__global__ __launch_bounds__(704) void k_mlp_reduce(uint32_t ngroups,
                                                   const double* __restrict__ part,
                                                   float* __restrict__ grad,
                                                   float* __restrict__ loss) {
  __shared__ double cnt;
  const int p = threadIdx.x;
  if (p == 0) {
    double c = 0.0;
    for (uint32_t g = 0; g < ngroups; ++g) c += part[(uint64_t)g * PSTRIDE + NPARAM + 1];
    cnt = c;
  }
  __syncthreads();
  if (p > NPARAM) return;
  double acc = 0.0;
  for (uint32_t g = 0; g < ngroups; ++g) acc += part[(uint64_t)g * PSTRIDE + p];
  const double inv = cnt > 0.0 ? 1.0 / cnt : 0.0;
  if (p < NPARAM) grad[p] = (float)(acc * inv);
  else *loss = (float)(acc * inv);
}

__global__ void k_mlp_adam(float* __restrict__ w, const float* __restrict__ g,
                           float* __restrict__ m, float* __restrict__ v, float lr, float bc1,
                           float bc2) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= NPARAM) return;
  const float gi = g[p];
  const float mi = 0.9f * m[p] + 0.1f * gi;
  const float vi = 0.999f * v[p] + 0.001f * gi * gi;
  m[p] = mi;
  v[p] = vi;
  w[p] = w[p] - lr * (mi / bc1) / (sqrtf(vi / bc2) + 1e-8f);
}

size_t mlp_workspace_bytes() {
  return (size_t)MLP_MAX_BATCH * MLP_ROW * sizeof(float) +
         (size_t)(MLP_MAX_BATCH / GROUP) * PSTRIDE * sizeof(double);
}

hipError_t launch_mlp_grad(const float* w, const int8_t* feat, const uint8_t* label,
                           uint32_t nsamp, float* ws, float* grad, float* loss, hipStream_t st) {
  // ws: per-sample rows, then the per-group partial sums (8-byte aligned)
  double* part = (double*)(ws + (size_t)MLP_MAX_BATCH * MLP_ROW);
  const uint32_t ngroups = (nsamp + GROUP - 1) / GROUP;
  if (nsamp) {
    hipLaunchKernelGGL(k_mlp_fwdbwd, dim3((nsamp + 255) / 256), dim3(256), 0, st, w, feat, label,
                       nsamp, ws);
    hipLaunchKernelGGL(k_mlp_partial, dim3(ngroups), dim3(704), 0, st, feat, label, nsamp, ws,
                       part);
  }
  hipLaunchKernelGGL(k_mlp_reduce, dim3(1), dim3(704), 0, st, ngroups, part, grad, loss);
  return hipGetLastError();
}

hipError_t launch_mlp_adam(float* w, const float* g, float* m, float* v, float lr, float bc1,
                           float bc2, hipStream_t st) {
  hipLaunchKernelGGL(k_mlp_adam, dim3((NPARAM + 255) / 256), dim3(256), 0, st, w, g, m, v, lr,
                     bc1, bc2);
  return hipGetLastError();
}

}  // namespace gzs
