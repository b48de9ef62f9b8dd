// gz_select.hip -- training kernels of the learned predictor selector.
//
// The selector is an int8 network 16 -> 32 (ReLU) -> 3 that picks each
// tile's predictor (NONE, L1D, L2D).  It is trained as an fp32 "shadow"
// network with softmax cross-entropy on labels from exhaustive trial, then
// exported to int8.  Gradients are made deterministic: a per-sample kernel
// writes each sample's backward terms, and a reduction kernel sums them in
// sample order in fp64, one thread per parameter.
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

// One block; thread p sums parameter p's gradient over the samples in order.
__global__ __launch_bounds__(1024) void k_mlp_reduce(const int8_t* __restrict__ feat,
                                                    const uint8_t* __restrict__ label,
                                                    uint32_t nsamp, const float* __restrict__ ws,
                                                    float* __restrict__ grad,
                                                    float* __restrict__ loss) {
  __shared__ uint32_t cnt_part[1024];
  uint32_t cnt = 0;
  for (uint32_t s = threadIdx.x; s < nsamp; s += blockDim.x) cnt += label[s] < NOUT ? 1u : 0u;
  cnt_part[threadIdx.x] = cnt;
  __syncthreads();
  for (uint32_t st = blockDim.x / 2; st > 0; st >>= 1) {
    if (threadIdx.x < st) cnt_part[threadIdx.x] += cnt_part[threadIdx.x + st];
    __syncthreads();
  }
  const double inv = cnt_part[0] ? 1.0 / (double)cnt_part[0] : 0.0;
  const int p = threadIdx.x;
  if (p > NPARAM) return;
  double acc = 0.0;
  if (p < NW1) {
    const int k = p / NIN, i = p % NIN;
    for (uint32_t s = 0; s < nsamp; ++s)
      acc += (double)ws[(uint64_t)s * ROW + k] * (double)feat[(uint64_t)s * NIN + i];
  } else if (p < NW1 + NB1) {
    const int k = p - NW1;
    for (uint32_t s = 0; s < nsamp; ++s) acc += (double)ws[(uint64_t)s * ROW + k];
  } else if (p < NW1 + NB1 + NW2) {
    const int o = (p - NW1 - NB1) / NH, k = (p - NW1 - NB1) % NH;
    for (uint32_t s = 0; s < nsamp; ++s)
      acc += (double)ws[(uint64_t)s * ROW + 2 * NH + o] * (double)ws[(uint64_t)s * ROW + NH + k];
  } else if (p < NPARAM) {
    const int o = p - NW1 - NB1 - NW2;
    for (uint32_t s = 0; s < nsamp; ++s) acc += (double)ws[(uint64_t)s * ROW + 2 * NH + o];
  } else {
    for (uint32_t s = 0; s < nsamp; ++s) acc += (double)ws[(uint64_t)s * ROW + 2 * NH + NOUT];
  }
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

hipError_t launch_mlp_grad(const float* w, const int8_t* feat, const uint8_t* label,
                           uint32_t nsamp, float* ws, float* grad, float* loss, hipStream_t st) {
  if (nsamp) {
    hipLaunchKernelGGL(k_mlp_fwdbwd, dim3((nsamp + 255) / 256), dim3(256), 0, st, w, feat, label,
                       nsamp, ws);
  }
  hipLaunchKernelGGL(k_mlp_reduce, dim3(1), dim3(1024), 0, st, feat, label, nsamp, ws, grad, loss);
  return hipGetLastError();
}

hipError_t launch_mlp_adam(float* w, const float* g, float* m, float* v, float lr, float bc1,
                           float bc2, hipStream_t st) {
  hipLaunchKernelGGL(k_mlp_adam, dim3((NPARAM + 255) / 256), dim3(256), 0, st, w, g, m, v, lr,
                     bc1, bc2);
  return hipGetLastError();
}

}  // namespace gzs
