// Per-tile front-to-back compositing and its backward.
//
// One 256-thread block (4 waves) per 16 x 16 tile, one pixel per thread; each
// wave covers an 8 x 8 quadrant so that a small splat touches few waves.  The
// tile's depth-sorted pairs are staged through LDS in batches of 256 records
// (every lane then reads the same LDS address, a broadcast); a block stops
// loading as soon as every pixel has reached the transmittance stop.
//
// Per pixel, front to back: alpha = min(0.99, o exp(-q/2)) with
// q = d^T conic d; pairs with q < 0 (rounding) or alpha < 1/255 are skipped;
// a pair that would bring T below 1e-4 ends the pixel without being blended.
// The backward walks each tile's list back to front from the last blended
// pair, rebuilds T by division by (1 - alpha) (alpha <= 0.99) and sums the
// per-pixel gradients of each pair over the wave before one atomic per
// wave, pair and component.
#include "common.hpp"

namespace gsr {

struct BatchLds {
  float4 a[256];  // u, v, conic a, conic b
  float4 b[256];  // conic c, opacity, r, g
  float c[256];   // b
  uint32_t rec[256];
};

__device__ __forceinline__ int find_view(const ViewD* __restrict__ views, int n_views, uint32_t tile) {
  int lo = 0, hi = n_views - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (views[mid].tile_off <= tile) lo = mid; else hi = mid - 1;
  }
  return lo;
}

__device__ __forceinline__ void pixel_of(int tid, int tx, int ty, int& px, int& py) {
  const int wave = tid >> 6, lane = tid & 63;
  px = tx * kTile + (wave & 1) * 8 + (lane & 7);
  py = ty * kTile + (wave >> 1) * 8 + (lane >> 3);
}

__device__ __forceinline__ void stage(BatchLds& L, const float* __restrict__ records, uint32_t n_rec,
                                      const uint32_t* __restrict__ vals, uint32_t k, bool ok, int tid) {
  if (ok) {
    uint32_t r = vals[k];
    if (r >= n_rec) r = 0;  // never read out of range (a sort fault shows up as wrong pixels)
    const float4* rec = reinterpret_cast<const float4*>(records + (size_t)r * kRecordFloats);
    const float4 r0 = rec[0], r1 = rec[1];
    const float r2 = records[(size_t)r * kRecordFloats + 8];
    L.a[tid] = r0;
    L.b[tid] = r1;
    L.c[tid] = r2;
    L.rec[tid] = r;
  }
}

// Exponent -q/2 of one pair at a pixel offset (dx, dy) = centre - pixel,
// q = a dx^2 + 2 b dx dy + c dy^2.  This file is compiled without implicit
// FMA contraction, so the forward and the backward evaluate this (and alpha)
// with the same instructions and take the same skip decisions.
__device__ __forceinline__ float pair_power(const float4 A, const float4 B, float dx, float dy) {
  const float q = fmaf(A.z * dx, dx, fmaf(B.x * dy, dy, (2.f * A.w) * (dx * dy)));
  return -0.5f * q;
}

__device__ void blend_tile(const ViewD& V, uint32_t tile, const float* __restrict__ records, uint32_t n_rec,
                           const uint32_t* __restrict__ vals, uint32_t cap, const uint32_t* __restrict__ ranges,
                           BatchLds& L) {
  const int tid = threadIdx.x;
  const uint32_t local = tile - V.tile_off;
  const int tx = (int)(local % (uint32_t)V.tiles_x), ty = (int)(local / (uint32_t)V.tiles_x);
  int px, py;
  pixel_of(tid, tx, ty, px, py);
  const bool inside = px < V.W && py < V.H;
  const float fx = (float)px + 0.5f, fy = (float)py + 0.5f;
  const uint32_t end = min(ranges[2 * tile + 1], cap);
  const uint32_t start = min(ranges[2 * tile], end);
  float T = 1.f, C0 = 0.f, C1 = 0.f, C2 = 0.f;
  uint32_t last = 0;
  bool done = !inside;
  for (uint32_t b = start; b < end; b += 256) {
    if (__syncthreads_and(done)) break;
    const uint32_t k = b + tid;
    stage(L, records, n_rec, vals, k, k < end, tid);
    __syncthreads();
    const int n = (int)min(256u, end - b);
    if (!done) {
      for (int j = 0; j < n; ++j) {
        const float4 A = L.a[j], B = L.b[j];
        const float dx = A.x - fx, dy = A.y - fy;
        const float power = pair_power(A, B, dx, dy);
        if (power > 0.f) continue;
        const float alpha = fminf(kAlphaMax, B.y * __expf(power));
        if (alpha < kAlphaMin) continue;
        const float Tn = T * (1.f - alpha);
        if (Tn < kTStop) { done = true; break; }
        const float w = alpha * T;
        C0 = fmaf(B.z, w, C0);
        C1 = fmaf(B.w, w, C1);
        C2 = fmaf(L.c[j], w, C2);
        T = Tn;
        last = b + (uint32_t)j + 1;
      }
    }
  }
  if (inside) {
    const size_t pix = (size_t)py * V.W + px;
    const size_t plane = (size_t)V.W * V.H;
    V.rgb[pix] = fmaf(T, V.bg[0], C0);
    V.rgb[plane + pix] = fmaf(T, V.bg[1], C1);
    V.rgb[2 * plane + pix] = fmaf(T, V.bg[2], C2);
    V.alpha[pix] = 1.f - T;
    V.final_T[pix] = T;
    V.last[pix] = last;
  }
}

template <bool PERSISTENT>
__global__ void __launch_bounds__(256)
k_blend_fwd(const ViewD* __restrict__ views, int n_views, uint32_t total_tiles, const float* __restrict__ records,
            uint32_t n_rec, const uint32_t* __restrict__ pair_vals, const uint32_t* __restrict__ sel, uint32_t cap,
            const uint32_t* __restrict__ ranges, uint32_t* __restrict__ tile_ctr,
            const int32_t* __restrict__ req_status) {
  __shared__ BatchLds L;
  __shared__ uint32_t s_tile;
  const uint32_t* vals = pair_vals + (*sel ? cap : 0u);
  if (!PERSISTENT) {
    const uint32_t tile = blockIdx.x;
    if (tile >= total_tiles) return;
    const ViewD& V = views[find_view(views, n_views, tile)];
    if (req_status && req_status[V.request] != 0) return;
    blend_tile(V, tile, records, n_rec, vals, cap, ranges, L);
    return;
  }
  for (;;) {
    __syncthreads();
    if (threadIdx.x == 0) s_tile = atomicAdd(tile_ctr, 1u);
    __syncthreads();
    const uint32_t tile = s_tile;
    if (tile >= total_tiles) return;
    const ViewD& V = views[find_view(views, n_views, tile)];
    if (req_status && req_status[V.request] != 0) continue;
    blend_tile(V, tile, records, n_rec, vals, cap, ranges, L);
  }
}

hipError_t launch_blend_fwd(const ViewD* views_dev, int n_views, uint32_t total_tiles, const float* records,
                            uint32_t n_rec, const uint32_t* pair_vals, const uint32_t* sel, uint32_t cap,
                            const uint32_t* ranges, uint32_t* tile_ctr, const int32_t* req_status,
                            bool persistent, hipStream_t s) {
  if (total_tiles == 0) return hipSuccess;
  if (persistent) {
    const uint32_t grid = min(total_tiles, 256u * 8u);
    hipLaunchKernelGGL(k_blend_fwd<true>, dim3(grid), dim3(256), 0, s, views_dev, n_views, total_tiles, records,
                       n_rec, pair_vals, sel, cap, ranges, tile_ctr, req_status);
  } else {
    hipLaunchKernelGGL(k_blend_fwd<false>, dim3(total_tiles), dim3(256), 0, s, views_dev, n_views, total_tiles,
                       records, n_rec, pair_vals, sel, cap, ranges, tile_ctr, req_status);
  }
  return hipGetLastError();
}

// ---------------------------------------------------------------- backward
__device__ __forceinline__ float wave_sum(float v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

__device__ __forceinline__ float wave_max(float v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v = fmaxf(v, __shfl_xor(v, off, 64));
  return v;
}

// g2d: [9][R] planes u, v, conic a, b, c, opacity, r, g, b.
__global__ void __launch_bounds__(256)
k_blend_bwd(const ViewD* __restrict__ views, int n_views, uint32_t total_tiles, const float* __restrict__ records,
            const uint32_t* __restrict__ pair_vals, const uint32_t* __restrict__ sel, uint32_t cap,
            const uint32_t* __restrict__ ranges, const float* __restrict__ dL_drgb,
            const float* __restrict__ dL_dalpha, float* __restrict__ g2d, uint32_t n_rec,
            float* __restrict__ max_contrib) {
  __shared__ BatchLds L;
  __shared__ uint32_t s_max_last;
  const uint32_t tile = blockIdx.x;
  if (tile >= total_tiles) return;
  const int vi = find_view(views, n_views, tile);
  const ViewD& V = views[vi];
  const uint32_t* vals = pair_vals + (*sel ? cap : 0u);
  const int tid = threadIdx.x, lane = tid & 63;
  const uint32_t local = tile - V.tile_off;
  const int tx = (int)(local % (uint32_t)V.tiles_x), ty = (int)(local / (uint32_t)V.tiles_x);
  int px, py;
  pixel_of(tid, tx, ty, px, py);
  const bool inside = px < V.W && py < V.H;
  const float fx = (float)px + 0.5f, fy = (float)py + 0.5f;
  const size_t plane = (size_t)V.W * V.H;
  const size_t pix = inside ? (size_t)py * V.W + px : 0;
  // per-view gradient planes follow the view's pixel offset in the call
  const size_t vpix = (size_t)vi * plane;
  float T = 1.f, Tfin = 1.f, G0 = 0.f, G1 = 0.f, G2 = 0.f, GA = 0.f;
  uint32_t plast = 0;
  if (inside) {
    Tfin = V.final_T[pix];
    T = Tfin;
    plast = V.last[pix];
    if (dL_drgb) {
      G0 = dL_drgb[3 * vpix + pix];
      G1 = dL_drgb[3 * vpix + plane + pix];
      G2 = dL_drgb[3 * vpix + 2 * plane + pix];
    }
    if (dL_dalpha) GA = dL_dalpha[vpix + pix];
  }
  if (tid == 0) s_max_last = 0;
  __syncthreads();
  if (plast) atomicMax(&s_max_last, plast);
  __syncthreads();
  const uint32_t stop = min(s_max_last, cap);  // one past the last pair any pixel blended
  const uint32_t start = min(ranges[2 * tile], stop);
  float S0 = Tfin * V.bg[0], S1 = Tfin * V.bg[1], S2 = Tfin * V.bg[2];
  const uint32_t gaussian_base = V.rec_off;
  for (uint32_t e = stop; e > start;) {
    const uint32_t b = (e - start > 256u) ? e - 256u : start;
    const uint32_t k = b + tid;
    stage(L, records, n_rec, vals, k, k < e, tid);
    __syncthreads();
    for (int j = (int)(e - b) - 1; j >= 0; --j) {
      const uint32_t kk = b + (uint32_t)j;
      const float4 A = L.a[j], B = L.b[j];
      const float cb = L.c[j];
      float gu = 0.f, gv = 0.f, ga = 0.f, gb = 0.f, gc = 0.f, go = 0.f, gr = 0.f, gg = 0.f, gbl = 0.f, w = 0.f;
      bool contrib = false;
      if (kk < plast) {
        const float dx = A.x - fx, dy = A.y - fy;
        const float power = pair_power(A, B, dx, dy);
        if (power <= 0.f) {
          const float G = __expf(power);
          const float oG = B.y * G;
          const float alpha = fminf(kAlphaMax, oG);
          if (alpha >= kAlphaMin) {
            contrib = true;
            const float inv1m = 1.f / (1.f - alpha);
            const float Tb = T * inv1m;
            w = alpha * Tb;
            gr = G0 * w;
            gg = G1 * w;
            gbl = G2 * w;
            const float dalpha = G0 * (B.z * Tb - S0 * inv1m) + G1 * (B.w * Tb - S1 * inv1m) +
                                 G2 * (cb * Tb - S2 * inv1m) + GA * Tfin * inv1m;
            S0 += B.z * w;
            S1 += B.w * w;
            S2 += cb * w;
            T = Tb;
            if (!(oG > kAlphaMax)) {
              go = dalpha * G;
              const float dq = dalpha * (-0.5f * oG);
              gu = dq * 2.f * (A.z * dx + A.w * dy);
              gv = dq * 2.f * (A.w * dx + B.x * dy);
              ga = dq * dx * dx;
              gb = dq * 2.f * dx * dy;
              gc = dq * dy * dy;
            }
          }
        }
      }
      if (__ballot(contrib) == 0ull) continue;
      gu = wave_sum(gu);
      gv = wave_sum(gv);
      ga = wave_sum(ga);
      gb = wave_sum(gb);
      gc = wave_sum(gc);
      go = wave_sum(go);
      gr = wave_sum(gr);
      gg = wave_sum(gg);
      gbl = wave_sum(gbl);
      w = wave_max(w);
      if (lane == 0) {
        const uint32_t r = L.rec[j];
        atomicAdd(&g2d[0 * (size_t)n_rec + r], gu);
        atomicAdd(&g2d[1 * (size_t)n_rec + r], gv);
        atomicAdd(&g2d[2 * (size_t)n_rec + r], ga);
        atomicAdd(&g2d[3 * (size_t)n_rec + r], gb);
        atomicAdd(&g2d[4 * (size_t)n_rec + r], gc);
        atomicAdd(&g2d[5 * (size_t)n_rec + r], go);
        atomicAdd(&g2d[6 * (size_t)n_rec + r], gr);
        atomicAdd(&g2d[7 * (size_t)n_rec + r], gg);
        atomicAdd(&g2d[8 * (size_t)n_rec + r], gbl);
        if (max_contrib) atomicMax(reinterpret_cast<uint32_t*>(&max_contrib[r - gaussian_base]), __float_as_uint(w));
      }
    }
    __syncthreads();
    e = b;
  }
}

hipError_t launch_blend_bwd(const ViewD* views_dev, int n_views, uint32_t total_tiles, const float* records,
                            const uint32_t* pair_vals, const uint32_t* sel, uint32_t cap, const uint32_t* ranges,
                            const float* dL_drgb, const float* dL_dalpha, float* g2d, uint32_t n_rec,
                            float* max_contrib, hipStream_t s) {
  if (total_tiles == 0) return hipSuccess;
  hipLaunchKernelGGL(k_blend_bwd, dim3(total_tiles), dim3(256), 0, s, views_dev, n_views, total_tiles, records,
                     pair_vals, sel, cap, ranges, dL_drgb, dL_dalpha, g2d, n_rec, max_contrib);
  return hipGetLastError();
}

}  // namespace gsr
