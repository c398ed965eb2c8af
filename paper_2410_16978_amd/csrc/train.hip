// The optimiser step of layered training and the per-Gaussian statistics
// it produces.
//
// Inactive-pruning activity from the optimiser's update (Sec. 3.2.2: the
// optimisation of each Gaussian's position, colour and scale is tracked and
// Gaussians whose activity over a window stays at or below a threshold are
// removed).  Per trainable Gaussian and optimiser step,
//   activity += 2 |d mean| + 0.1 |d sh| + 0.1 |d log scale|,
// d the change the step made and |.| the Euclidean norm over the Gaussian's
// 3, 3 (D+1)^2 and 3 values.  One thread per Gaussian; every parameter plane
// is read with consecutive threads on consecutive Gaussians, so each load of
// a wave is one contiguous 256-byte line.  HBM-bound: 8 (6 + 3 (D+1)^2) + 8
// bytes per Gaussian.
#include <algorithm>

#include "common.hpp"

namespace gsr {

namespace {

__device__ __forceinline__ float plane_sq(const float* __restrict__ a, const float* __restrict__ b, int planes,
                                          size_t n, size_t i) {
  float s = 0.f;
  for (int p = 0; p < planes; ++p) {
    const float d = b[(size_t)p * n + i] - a[(size_t)p * n + i];
    s += d * d;
  }
  return s;
}

}  // namespace

__global__ void __launch_bounds__(256)
k_update_activity(int n, int n_sh_planes, uint32_t trainable, const float* __restrict__ mean0,
                  const float* __restrict__ mean1, const float* __restrict__ ls0, const float* __restrict__ ls1,
                  const float* __restrict__ sh0, const float* __restrict__ sh1, const uint8_t* __restrict__ layer,
                  float* __restrict__ activity) {
  const size_t nn = (size_t)n;
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < nn; i += (size_t)gridDim.x * blockDim.x) {
    const uint32_t l = layer[i];
    if (l >= 32u || !((trainable >> l) & 1u)) continue;
    const float dm = plane_sq(mean0, mean1, 3, nn, i);
    const float ds = plane_sq(ls0, ls1, 3, nn, i);
    const float dc = plane_sq(sh0, sh1, n_sh_planes, nn, i);
    activity[i] += (2.f * sqrtf(dm) + 0.1f * sqrtf(dc)) + 0.1f * sqrtf(ds);
  }
}

hipError_t launch_update_activity(int n, int sh_degree, uint32_t trainable, const float* mean0, const float* mean1,
                                  const float* ls0, const float* ls1, const float* sh0, const float* sh1,
                                  const uint8_t* layer, float* activity, hipStream_t s) {
  if (n == 0) return hipSuccess;
  const int planes = 3 * (sh_degree + 1) * (sh_degree + 1);
  const uint32_t blocks = (uint32_t)std::min<size_t>(((size_t)n + 255) / 256, 8192);
  hipLaunchKernelGGL(k_update_activity, dim3(blocks), dim3(256), 0, s, n, planes, trainable, mean0, mean1, ls0, ls1,
                     sh0, sh1, layer, activity);
  return hipGetLastError();
}

// Adam on the Gaussians of the trainable layers (Sec. 3.2: the other layers
// are frozen; their gradients are zero and their moments stay zero, so Adam
// would leave them unchanged: they are skipped, parameters, gradients and
// moments untouched).  Per value, with the bias corrections of the step:
//   m <- m + (1 - beta1) (g - m),  v <- beta2 v + (1 - beta2) g^2,
//   p <- p - (lr / bc1) m / (sqrt(v) / sqrt(bc2) + eps).
// With activity, the Gaussian's update-norm activity of the step (the
// change p_new - p_old of its mean, SH and log-scale values, weights 2, 0.1,
// 0.1) is added, as k_update_activity computes it.  One thread per Gaussian,
// planes read with consecutive threads on consecutive Gaussians.
__global__ void __launch_bounds__(256)
k_adam(int n, AdamArgs a, const uint8_t* __restrict__ layer, uint32_t trainable, float* __restrict__ activity) {
  const size_t nn = (size_t)n;
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < nn; i += (size_t)gridDim.x * blockDim.x) {
    const uint32_t l = layer[i];
    if (l >= 32u || !((trainable >> l) & 1u)) continue;
    float sq[kAdamGroups];
#pragma unroll
    for (int gi = 0; gi < kAdamGroups; ++gi) {
      const AdamGroupD& G = a.g[gi];
      float acc = 0.f;
      for (int q = 0; q < G.planes; ++q) {
        const size_t k = (size_t)q * nn + i;
        const float g = G.grad[k];
        float m = G.m[k], v = G.v[k];
        m = m + a.one_minus_b1 * (g - m);
        v = a.b2 * v + a.one_minus_b2 * (g * g);
        const float p = G.p[k];
        const float pn = p - G.step_size * (m / (sqrtf(v) / a.bc2_sqrt + a.eps));
        G.m[k] = m;
        G.v[k] = v;
        G.p[k] = pn;
        const float d = pn - p;
        acc += d * d;
      }
      sq[gi] = acc;
    }
    if (activity) activity[i] += (2.f * sqrtf(sq[0]) + 0.1f * sqrtf(sq[4])) + 0.1f * sqrtf(sq[1]);
  }
}

hipError_t launch_adam(int n, const AdamArgs& a, const uint8_t* layer, uint32_t trainable, float* activity,
                       hipStream_t s) {
  if (n == 0) return hipSuccess;
  const uint32_t blocks = (uint32_t)std::min<size_t>(((size_t)n + 255) / 256, 8192);
  hipLaunchKernelGGL(k_adam, dim3(blocks), dim3(256), 0, s, n, a, layer, trainable, activity);
  return hipGetLastError();
}

}  // namespace gsr
