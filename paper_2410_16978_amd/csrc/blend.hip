// Per-tile front-to-back compositing and its backward.
//
// Forward: one 256-thread block (4 waves) per 16 x 16 tile, one pixel per
// thread; each wave covers an 8 x 8 quadrant so that a small splat touches
// few waves.  The tile's depth-sorted pairs are staged through LDS in batches
// of 256 records (every lane then reads the same LDS address, a broadcast);
// the block stops loading once every pixel has reached the transmittance
// stop.  For each batch the block stores every pixel's transmittance before
// the batch and the colour the batch adds (a checkpoint), so that the
// backward can start at any batch.
//
// Per pixel, front to back: alpha = min(0.99, o exp(-q/2)) with
// q = d^T conic d; pairs with q < 0 (rounding) or alpha < 1/255 are skipped;
// a pair that would bring T below 1e-4 ends the pixel without being blended.
//
// Backward: one block per (tile, batch) - the heavy tiles' lists are walked
// by many blocks at once.  Each block starts at the end of its batch: the
// transmittance there is the next batch's checkpoint (or the final one), the
// colour behind it is the background term plus the later batches' colours,
// summed from the back.  It walks the batch back to front, rebuilding T by
// division by (1 - alpha) (alpha <= 0.99) and accumulating the colour behind
// each pair from the back, which keeps that colour relatively accurate deep
// in a pixel's list.  The per-pixel gradients of each pair are summed over
// the wave with DPP (lane 63 holds the sum), the four wave sums in a fixed
// order through LDS, and written as the pair's partial gradient: no atomics,
// bitwise reproducible.
#include "common.hpp"

namespace gsr {

struct BatchLds {
  float4 a[kBatch];  // u, v, conic a, conic b
  float4 b[kBatch];  // conic c, opacity, r, g
  float c[kBatch];   // b
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

__device__ __forceinline__ float pair_alpha(const float4 B, float power) {
  return fminf(kAlphaMax, B.y * __expf(power));
}

__device__ void blend_tile(const ViewD& V, uint32_t tile, const float* __restrict__ records, uint32_t n_rec,
                           const uint32_t* __restrict__ vals, uint32_t cap, const uint32_t* __restrict__ ranges,
                           float4* __restrict__ ckpt, BatchLds& L) {
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
  uint32_t batch = 0;
  for (uint32_t b = start; b < end; b += kBatch, ++batch) {
    if (__syncthreads_and(done)) break;
    const float T0 = T;
    float D0 = 0.f, D1 = 0.f, D2 = 0.f;  // colour added by this batch
    const uint32_t k = b + tid;
    stage(L, records, n_rec, vals, k, k < end, tid);
    __syncthreads();
    const int n = (int)min((uint32_t)kBatch, end - b);
    if (!done) {
      for (int j = 0; j < n; ++j) {
        const float4 A = L.a[j], B = L.b[j];
        const float dx = A.x - fx, dy = A.y - fy;
        const float power = pair_power(A, B, dx, dy);
        if (power > 0.f) continue;
        const float alpha = pair_alpha(B, power);
        if (alpha < kAlphaMin) continue;
        const float Tn = T * (1.f - alpha);
        if (Tn < kTStop) { done = true; break; }
        const float w = alpha * T;
        D0 = fmaf(B.z, w, D0);
        D1 = fmaf(B.w, w, D1);
        D2 = fmaf(L.c[j], w, D2);
        T = Tn;
        last = b + (uint32_t)j + 1;
      }
    }
    if (ckpt) ckpt[(size_t)batch * kBatch + tid] = make_float4(T0, D0, D1, D2);
    C0 += D0;
    C1 += D1;
    C2 += D2;
  }
  if (inside) {
    const size_t pix = (size_t)py * V.W + px;
    const size_t plane = (size_t)V.W * V.H;
    V.rgb[pix] = fmaf(T, V.bg[0], C0);
    V.rgb[plane + pix] = fmaf(T, V.bg[1], C1);
    V.rgb[2 * plane + pix] = fmaf(T, V.bg[2], C2);
    V.alpha[pix] = 1.f - T;
    reinterpret_cast<float4*>(V.pix)[pix] = make_float4(T, C0, C1, C2);
    V.last[pix] = last;
  }
}

template <bool PERSISTENT>
__global__ void __launch_bounds__(256)
k_blend_fwd(const ViewD* __restrict__ views, int n_views, uint32_t total_tiles, const float* __restrict__ records,
            uint32_t n_rec, const uint32_t* __restrict__ pair_vals, const uint32_t* __restrict__ sel, uint32_t cap,
            const uint32_t* __restrict__ ranges, uint32_t* __restrict__ tile_ctr,
            const int32_t* __restrict__ req_status, float4* __restrict__ ckpt,
            const uint32_t* __restrict__ batch_off, uint32_t batch_cap) {
  __shared__ BatchLds L;
  __shared__ uint32_t s_tile;
  const uint32_t* vals = pair_vals + (*sel ? cap : 0u);
  for (;;) {
    uint32_t tile;
    if (PERSISTENT) {
      __syncthreads();
      if (threadIdx.x == 0) s_tile = atomicAdd(tile_ctr, 1u);
      __syncthreads();
      tile = s_tile;
    } else {
      tile = blockIdx.x;
    }
    if (tile >= total_tiles) return;
    const ViewD& V = views[find_view(views, n_views, tile)];
    if (!(req_status && req_status[V.request] != 0)) {
      float4* tck = nullptr;
      if (ckpt) {
        const uint32_t b0 = batch_off[tile], b1 = batch_off[tile + 1];
        if (b1 <= batch_cap && b0 <= b1) tck = ckpt + (size_t)b0 * kBatch;
      }
      blend_tile(V, tile, records, n_rec, vals, cap, ranges, tck, L);
    }
    if (!PERSISTENT) return;
  }
}

hipError_t launch_blend_fwd(const ViewD* views_dev, int n_views, uint32_t total_tiles, const float* records,
                            uint32_t n_rec, const uint32_t* pair_vals, const uint32_t* sel, uint32_t cap,
                            const uint32_t* ranges, uint32_t* tile_ctr, const int32_t* req_status,
                            float4* ckpt, const uint32_t* batch_off, uint32_t batch_cap, bool persistent,
                            hipStream_t s) {
  if (total_tiles == 0) return hipSuccess;
  if (persistent) {
    const uint32_t grid = min(total_tiles, 256u * 8u);
    hipLaunchKernelGGL(k_blend_fwd<true>, dim3(grid), dim3(256), 0, s, views_dev, n_views, total_tiles, records,
                       n_rec, pair_vals, sel, cap, ranges, tile_ctr, req_status, ckpt, batch_off, batch_cap);
  } else {
    hipLaunchKernelGGL(k_blend_fwd<false>, dim3(total_tiles), dim3(256), 0, s, views_dev, n_views, total_tiles,
                       records, n_rec, pair_vals, sel, cap, ranges, tile_ctr, req_status, ckpt, batch_off,
                       batch_cap);
  }
  return hipGetLastError();
}

// ---------------------------------------------------------------- backward
// Wave64 reductions with DPP: quad swaps, half-row and row mirrors, then the
// row broadcasts 15 and 31; lane 63 ends with the result.
template <unsigned CTRL, unsigned ROW_MASK>
__device__ __forceinline__ float dpp(float v) {
  return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, ROW_MASK, 0xF, false));
}

__device__ __forceinline__ float wave_sum63(float v) {
  v += dpp<0xB1, 0xF>(v);   // quad_perm [1,0,3,2]
  v += dpp<0x4E, 0xF>(v);   // quad_perm [2,3,0,1]
  v += dpp<0x141, 0xF>(v);  // row_half_mirror
  v += dpp<0x140, 0xF>(v);  // row_mirror
  v += dpp<0x142, 0xA>(v);  // row_bcast15 into rows 1 and 3
  v += dpp<0x143, 0xC>(v);  // row_bcast31 into rows 2 and 3
  return v;
}

__device__ __forceinline__ float wave_max63(float v) {  // v >= 0
  v = fmaxf(v, dpp<0xB1, 0xF>(v));
  v = fmaxf(v, dpp<0x4E, 0xF>(v));
  v = fmaxf(v, dpp<0x141, 0xF>(v));
  v = fmaxf(v, dpp<0x140, 0xF>(v));
  v = fmaxf(v, dpp<0x142, 0xA>(v));
  v = fmaxf(v, dpp<0x143, 0xC>(v));
  return v;
}

constexpr int kGradSlots = 10;  // u, v, conic a, b, c, opacity, r, g, b, max alpha*T

// g_pair: [P][12] per sorted pair: the 10 slots above, 2 unused.
__global__ void __launch_bounds__(256)
k_blend_bwd(const ViewD* __restrict__ views, int n_views, const float* __restrict__ records, uint32_t n_rec,
            const uint32_t* __restrict__ pair_vals, const uint32_t* __restrict__ sel, uint32_t cap,
            const uint32_t* __restrict__ ranges, const float4* __restrict__ ckpt,
            const uint32_t* __restrict__ batch_off, const uint32_t* __restrict__ batch_tile,
            const uint32_t* __restrict__ counters, const float* __restrict__ dL_drgb,
            const float* __restrict__ dL_dalpha, float* __restrict__ g_pair) {
  __shared__ BatchLds L;
  __shared__ float part[4][kGradSlots][kBatch];
  const uint32_t bi = blockIdx.x;
  if (bi >= counters[kCntBatches]) return;
  const uint32_t tile = batch_tile[bi];
  const uint32_t c = bi - batch_off[tile];
  const int vi = find_view(views, n_views, tile);
  const ViewD& V = views[vi];
  const uint32_t* vals = pair_vals + (*sel ? cap : 0u);
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const uint32_t t_end = min(ranges[2 * tile + 1], cap);
  const uint32_t start = min(ranges[2 * tile] + c * kBatch, t_end);
  const uint32_t end = min(start + kBatch, t_end);
  const int n = (int)(end - start);

  const uint32_t local = tile - V.tile_off;
  const int tx = (int)(local % (uint32_t)V.tiles_x), ty = (int)(local / (uint32_t)V.tiles_x);
  int px, py;
  pixel_of(tid, tx, ty, px, py);
  const bool inside = px < V.W && py < V.H;
  const float fx = (float)px + 0.5f, fy = (float)py + 0.5f;
  const size_t plane = (size_t)V.W * V.H;
  const size_t pix = inside ? (size_t)py * V.W + px : 0;
  const size_t vpix = (size_t)vi * plane;  // views of one call share a resolution
  uint32_t plast = 0;
  float T = 1.f, Tfin = 1.f, S0 = 0.f, S1 = 0.f, S2 = 0.f, G0 = 0.f, G1 = 0.f, G2 = 0.f, GA = 0.f;
  if (inside) {
    plast = V.last[pix];
    if (plast > start) {
      const float4 ps = reinterpret_cast<const float4*>(V.pix)[pix];
      Tfin = ps.x;
      // batch of the pixel's last blended pair (>= c)
      const uint32_t tile_start = ranges[2 * tile];
      const uint32_t c_last = (plast - 1 - tile_start) / kBatch;
      const float4* tck = ckpt + (size_t)(bi - c) * kBatch + tid;
      // transmittance at the end of this batch, colour behind it
      T = (c_last == c) ? Tfin : tck[(size_t)(c + 1) * kBatch].x;
      S0 = Tfin * V.bg[0];
      S1 = Tfin * V.bg[1];
      S2 = Tfin * V.bg[2];
      for (uint32_t cc = c_last; cc > c; --cc) {
        const float4 d = tck[(size_t)cc * kBatch];
        S0 += d.y;
        S1 += d.z;
        S2 += d.w;
      }
      if (dL_drgb) {
        G0 = dL_drgb[3 * vpix + pix];
        G1 = dL_drgb[3 * vpix + plane + pix];
        G2 = dL_drgb[3 * vpix + 2 * plane + pix];
      }
      if (dL_dalpha) GA = dL_dalpha[vpix + pix];
    } else {
      plast = 0;
    }
  }
  stage(L, records, n_rec, vals, start + tid, tid < n, tid);
  for (int i = tid; i < 4 * kGradSlots * kBatch; i += 256) (&part[0][0][0])[i] = 0.f;
  __syncthreads();

  for (int j = n - 1; j >= 0; --j) {
    const uint32_t kk = start + (uint32_t)j;
    float gu = 0.f, gv = 0.f, ga = 0.f, gb = 0.f, gc = 0.f, go = 0.f, gr = 0.f, gg = 0.f, gbl = 0.f, w = 0.f;
    bool contrib = false;
    if (kk < plast) {
      const float4 A = L.a[j], B = L.b[j];
      const float cbl = L.c[j];
      const float dx = A.x - fx, dy = A.y - fy;
      const float power = pair_power(A, B, dx, dy);
      if (power <= 0.f) {
        const float G = __expf(power);
        const float oG = B.y * G;
        const float alpha = fminf(kAlphaMax, oG);
        if (alpha >= kAlphaMin) {
          contrib = true;
          const float inv1m = 1.f / (1.f - alpha);
          const float Tb = T * inv1m;  // transmittance in front of this pair
          w = alpha * Tb;
          const float dalpha = G0 * (B.z * Tb - S0 * inv1m) + G1 * (B.w * Tb - S1 * inv1m) +
                               G2 * (cbl * Tb - S2 * inv1m) + GA * Tfin * inv1m;
          S0 = fmaf(B.z, w, S0);
          S1 = fmaf(B.w, w, S1);
          S2 = fmaf(cbl, w, S2);
          T = Tb;
          gr = G0 * w;
          gg = G1 * w;
          gbl = G2 * w;
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
    gu = wave_sum63(gu);
    gv = wave_sum63(gv);
    ga = wave_sum63(ga);
    gb = wave_sum63(gb);
    gc = wave_sum63(gc);
    go = wave_sum63(go);
    gr = wave_sum63(gr);
    gg = wave_sum63(gg);
    gbl = wave_sum63(gbl);
    w = wave_max63(w);
    if (lane == 63) {
      part[wave][0][j] = gu;
      part[wave][1][j] = gv;
      part[wave][2][j] = ga;
      part[wave][3][j] = gb;
      part[wave][4][j] = gc;
      part[wave][5][j] = go;
      part[wave][6][j] = gr;
      part[wave][7][j] = gg;
      part[wave][8][j] = gbl;
      part[wave][9][j] = w;
    }
  }
  __syncthreads();
  if (tid < n) {
    float o[12];
#pragma unroll
    for (int s = 0; s < 9; ++s) o[s] = ((part[0][s][tid] + part[1][s][tid]) + part[2][s][tid]) + part[3][s][tid];
    o[9] = fmaxf(fmaxf(part[0][9][tid], part[1][9][tid]), fmaxf(part[2][9][tid], part[3][9][tid]));
    o[10] = 0.f;
    o[11] = 0.f;
    float4* dst = reinterpret_cast<float4*>(g_pair + (size_t)(start + tid) * 12);
    dst[0] = make_float4(o[0], o[1], o[2], o[3]);
    dst[1] = make_float4(o[4], o[5], o[6], o[7]);
    dst[2] = make_float4(o[8], o[9], o[10], o[11]);
  }
}

hipError_t launch_blend_bwd(const ViewD* views_dev, int n_views, const float* records, uint32_t n_rec,
                            const uint32_t* pair_vals, const uint32_t* sel, uint32_t cap, const uint32_t* ranges,
                            const float4* ckpt, const uint32_t* batch_off, const uint32_t* batch_tile,
                            uint32_t batch_cap, const uint32_t* counters, const float* dL_drgb,
                            const float* dL_dalpha, float* g_pair, hipStream_t s) {
  if (batch_cap == 0) return hipSuccess;
  hipLaunchKernelGGL(k_blend_bwd, dim3(batch_cap), dim3(256), 0, s, views_dev, n_views, records, n_rec, pair_vals,
                     sel, cap, ranges, ckpt, batch_off, batch_tile, counters, dL_drgb, dL_dalpha, g_pair);
  return hipGetLastError();
}

}  // namespace gsr
