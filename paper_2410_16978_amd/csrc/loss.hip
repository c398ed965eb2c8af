// L1 loss of the alpha-channel training (Sec. 3.2.1) and its gradient.
//
// Per view v with background colour bg_v, the target colour is the target's
// premultiplied colour composited over that background,
//   target = t_rgb + (1 - t_alpha) bg_v,
// and L = mean |rgb - target| + mean |alpha - t_alpha| (the means over all
// V x 3 x H x W colour values and V x H x W alpha values).  The loss is
// reduced per block (grid-stride) and the block sums are added in a fixed
// order by one block (deterministic); the gradient is sign(d) g / N per
// value, g the incoming gradient of L.
#include "common.hpp"

namespace gsr {

struct LossBg {
  float bg[kMaxJobViews][3];
};

__device__ __forceinline__ float l1_block_sum(float v, float* lds) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  if (lane == 0) lds[wave] = v;
  __syncthreads();
  float s = 0.f;
  if (threadIdx.x == 0)
    for (int w = 0; w < (int)(blockDim.x >> 6); ++w) s += lds[w];
  return s;  // valid in thread 0
}

constexpr uint32_t kLossBlocks = 1024;  // partial sums (grid-stride)

// Block partial sums of the loss; with dL_drgb / dL_dalpha (both or
// neither) also the gradient, in the same pass (it does not depend on L).
__global__ void __launch_bounds__(256)
k_l1_loss(int n_views, int hw, const float* __restrict__ rgb, const float* __restrict__ alpha,
          const float* __restrict__ t_rgb, const float* __restrict__ t_alpha, LossBg bg,
          float* __restrict__ partials, const float* __restrict__ g_loss, float* __restrict__ dL_drgb,
          float* __restrict__ dL_dalpha) {
  __shared__ float lds[8];
  const uint32_t total = (uint32_t)n_views * (uint32_t)hw;
  const bool grad = dL_drgb != nullptr;
  const float g = grad && g_loss ? g_loss[0] : 1.f;
  const float kc = g / (float)(3 * (size_t)total), ka = g / (float)total;
  float sc = 0.f, sa = 0.f;
  for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < total; i += gridDim.x * blockDim.x) {
    const uint32_t v = i / (uint32_t)hw, q = i - v * (uint32_t)hw;
    const size_t b3 = (size_t)v * 3 * hw + q;
    const float ta = t_alpha[i];
    const float om = 1.f - ta;
#pragma unroll
    for (int ch = 0; ch < 3; ++ch) {
      const float target = t_rgb[b3 + (size_t)ch * hw] + om * bg.bg[v][ch];
      const float d = rgb[b3 + (size_t)ch * hw] - target;
      sc += fabsf(d);
      if (grad) dL_drgb[b3 + (size_t)ch * hw] = d > 0.f ? kc : (d < 0.f ? -kc : 0.f);
    }
    const float d = alpha[i] - ta;
    sa += fabsf(d);
    if (grad) dL_dalpha[i] = d > 0.f ? ka : (d < 0.f ? -ka : 0.f);
  }
  const float bc = l1_block_sum(sc, lds);
  __syncthreads();
  const float ba = l1_block_sum(sa, lds);
  if (threadIdx.x == 0) {
    partials[2 * blockIdx.x] = bc;
    partials[2 * blockIdx.x + 1] = ba;
  }
}

// The same with four consecutive pixels per thread and step (hw a multiple
// of 4 and every array 16-byte aligned): eight 16-byte loads in flight per
// step instead of one pixel's eight 4-byte loads.
__global__ void __launch_bounds__(256)
k_l1_loss4(int n_views, int hw, const float4* __restrict__ rgb, const float4* __restrict__ alpha,
           const float4* __restrict__ t_rgb, const float4* __restrict__ t_alpha, LossBg bg,
           float* __restrict__ partials, const float* __restrict__ g_loss, float4* __restrict__ dL_drgb,
           float4* __restrict__ dL_dalpha) {
  __shared__ float lds[8];
  const uint32_t total = (uint32_t)n_views * (uint32_t)hw;
  const uint32_t hw4 = (uint32_t)hw / 4u, total4 = total / 4u;
  const bool grad = dL_drgb != nullptr;
  const float g = grad && g_loss ? g_loss[0] : 1.f;
  const float kc = g / (float)(3 * (size_t)total), ka = g / (float)total;
  float sc = 0.f, sa = 0.f;
  for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < total4; i += gridDim.x * blockDim.x) {
    const uint32_t v = i / hw4, q = i - v * hw4;
    const size_t b3 = (size_t)v * 3 * hw4 + q;
    const float4 ta = t_alpha[i], al = alpha[i];
    float4 tc[3], c[3];
#pragma unroll
    for (int ch = 0; ch < 3; ++ch) {
      tc[ch] = t_rgb[b3 + (size_t)ch * hw4];
      c[ch] = rgb[b3 + (size_t)ch * hw4];
    }
    auto sgn = [](float d, float k) { return d > 0.f ? k : (d < 0.f ? -k : 0.f); };
#pragma unroll
    for (int ch = 0; ch < 3; ++ch) {
      const float bgc = bg.bg[v][ch];
      const float dx = c[ch].x - (tc[ch].x + (1.f - ta.x) * bgc), dy = c[ch].y - (tc[ch].y + (1.f - ta.y) * bgc);
      const float dz = c[ch].z - (tc[ch].z + (1.f - ta.z) * bgc), dw = c[ch].w - (tc[ch].w + (1.f - ta.w) * bgc);
      sc += fabsf(dx) + fabsf(dy) + fabsf(dz) + fabsf(dw);
      if (grad) dL_drgb[b3 + (size_t)ch * hw4] = make_float4(sgn(dx, kc), sgn(dy, kc), sgn(dz, kc), sgn(dw, kc));
    }
    const float dx = al.x - ta.x, dy = al.y - ta.y, dz = al.z - ta.z, dw = al.w - ta.w;
    sa += fabsf(dx) + fabsf(dy) + fabsf(dz) + fabsf(dw);
    if (grad) dL_dalpha[i] = make_float4(sgn(dx, ka), sgn(dy, ka), sgn(dz, ka), sgn(dw, ka));
  }
  const float bc = l1_block_sum(sc, lds);
  __syncthreads();
  const float ba = l1_block_sum(sa, lds);
  if (threadIdx.x == 0) {
    partials[2 * blockIdx.x] = bc;
    partials[2 * blockIdx.x + 1] = ba;
  }
}

// One block of 1024 threads: the partial sums in a fixed order (one pair of
// partials per thread - there are at most kLossBlocks - then wave sums, then
// the sixteen wave sums in order): one load round trip and one barrier.
static_assert(kLossBlocks <= 1024, "one pair of partials per thread");
__global__ void __launch_bounds__(1024)
k_l1_loss_final(uint32_t n_part, uint32_t total, const float* __restrict__ partials, float* __restrict__ loss) {
  __shared__ float lds[2][16];
  float c = 0.f, a = 0.f;
  for (uint32_t b = threadIdx.x; b < n_part; b += blockDim.x) {
    c += partials[2 * b];
    a += partials[2 * b + 1];
  }
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    c += __shfl_xor(c, off, 64);
    a += __shfl_xor(a, off, 64);
  }
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  if (lane == 0) {
    lds[0][wave] = c;
    lds[1][wave] = a;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    float tc = 0.f, ta = 0.f;
    for (int w = 0; w < (int)(blockDim.x >> 6); ++w) {
      tc += lds[0][w];
      ta += lds[1][w];
    }
    loss[0] = tc / (float)(3 * (size_t)total) + ta / (float)total;
  }
}

__global__ void __launch_bounds__(256)
k_l1_loss_grad(int n_views, int hw, const float* __restrict__ rgb, const float* __restrict__ alpha,
               const float* __restrict__ t_rgb, const float* __restrict__ t_alpha, LossBg bg,
               const float* __restrict__ g_loss, float* __restrict__ dL_drgb, float* __restrict__ dL_dalpha) {
  const uint32_t total = (uint32_t)n_views * (uint32_t)hw;
  const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= total) return;
  const float g = g_loss ? g_loss[0] : 1.f;
  const float kc = g / (float)(3 * (size_t)total), ka = g / (float)total;
  const uint32_t v = i / (uint32_t)hw, q = i - v * (uint32_t)hw;
  const size_t b3 = (size_t)v * 3 * hw + q;
  const float ta = t_alpha[i];
  const float om = 1.f - ta;
#pragma unroll
  for (int ch = 0; ch < 3; ++ch) {
    const size_t o = b3 + (size_t)ch * hw;
    const float d = rgb[o] - (t_rgb[o] + om * bg.bg[v][ch]);
    dL_drgb[o] = d > 0.f ? kc : (d < 0.f ? -kc : 0.f);
  }
  const float d = alpha[i] - ta;
  dL_dalpha[i] = d > 0.f ? ka : (d < 0.f ? -ka : 0.f);
}

uint32_t l1_loss_blocks(int n_views, int hw) { return div_up((uint32_t)n_views * (uint32_t)hw, 256u); }

hipError_t launch_l1_loss(int n_views, int hw, const float* rgb, const float* alpha, const float* t_rgb,
                          const float* t_alpha, const float* bg_host, float* partials, float* loss,
                          const float* g_loss, float* dL_drgb, float* dL_dalpha, hipStream_t s) {
  LossBg bg;
  for (int v = 0; v < kMaxJobViews; ++v)
    for (int ch = 0; ch < 3; ++ch) bg.bg[v][ch] = v < n_views ? bg_host[3 * v + ch] : 0.f;
  const uint32_t blocks = l1_loss_blocks(n_views, hw);
  if (blocks == 0) return hipSuccess;
  const bool grads = dL_drgb && dL_dalpha;
  auto a16 = [](const void* p) { return (reinterpret_cast<uintptr_t>(p) & 15u) == 0; };
  const uint32_t blocks4 = min(div_up((uint32_t)n_views * (uint32_t)hw / 4u, 256u), kLossBlocks);
  const bool vec = hw % 4 == 0 && a16(rgb) && a16(alpha) && a16(t_rgb) && a16(t_alpha) &&
                   (!grads || (a16(dL_drgb) && a16(dL_dalpha)));
  if (loss && vec) {
    hipLaunchKernelGGL(k_l1_loss4, dim3(blocks4), dim3(256), 0, s, n_views, hw,
                       reinterpret_cast<const float4*>(rgb), reinterpret_cast<const float4*>(alpha),
                       reinterpret_cast<const float4*>(t_rgb), reinterpret_cast<const float4*>(t_alpha), bg, partials,
                       g_loss, grads ? reinterpret_cast<float4*>(dL_drgb) : nullptr,
                       grads ? reinterpret_cast<float4*>(dL_dalpha) : nullptr);
    hipLaunchKernelGGL(k_l1_loss_final, dim3(1), dim3(1024), 0, s, blocks4, (uint32_t)n_views * (uint32_t)hw,
                       partials, loss);
  } else if (loss) {  // with the gradient in the same pass when both are asked for
    const uint32_t n_part = min(blocks, kLossBlocks);
    hipLaunchKernelGGL(k_l1_loss, dim3(n_part), dim3(256), 0, s, n_views, hw, rgb, alpha, t_rgb, t_alpha, bg,
                       partials, g_loss, grads ? dL_drgb : nullptr, grads ? dL_dalpha : nullptr);
    hipLaunchKernelGGL(k_l1_loss_final, dim3(1), dim3(1024), 0, s, n_part, (uint32_t)n_views * (uint32_t)hw,
                       partials, loss);
  } else if (grads)
    hipLaunchKernelGGL(k_l1_loss_grad, dim3(blocks), dim3(256), 0, s, n_views, hw, rgb, alpha, t_rgb, t_alpha, bg,
                       g_loss, dL_drgb, dL_dalpha);
  return hipGetLastError();
}

}  // namespace gsr
