// Projection of Gaussians into splat records (gates, EWA covariance, SH
// colour, tile box).  Compiled with -ffp-contract=off: every expression is
// evaluated as written, each + - * / sqrt correctly rounded, so the records,
// tile boxes and depth keys are reproducible bit for bit.
#include <algorithm>
#include <cstring>

#include "common.hpp"

#include <cstddef>
#include "sh.hpp"

namespace gsr {

// Correctly rounded square root.  The hardware square root is within one ulp;
// the exactly rounded residuals x - s' s of its two neighbours s' decide
// whether the round-to-nearest root is a neighbour.  (x - dn*s <= 0 means
// sqrt(x) lies below the geometric, hence below the arithmetic, mean of dn
// and s; a float x cannot fall between dn*s and the squared midpoint, which
// differ by a quarter of a squared ulp, less than one unit of the exact
// product.  Symmetrically for the upper neighbour.)  Tiny inputs are scaled
// by 2^32 so the estimate stays accurate.
__device__ __forceinline__ float sqrt_rn(float x) {
  if (!(x > 0.f) || isinf(x)) return __builtin_sqrtf(x);
  const bool tiny = x < 0x1p-96f;
  const float xs = tiny ? x * 0x1p+32f : x;
  float s = __builtin_amdgcn_sqrtf(xs);
  const float dn = __uint_as_float(__float_as_uint(s) - 1u);
  const float up = __uint_as_float(__float_as_uint(s) + 1u);
  if (fmaf(-dn, s, xs) <= 0.f) {
    s = dn;
  } else if (fmaf(-up, s, xs) > 0.f) {
    s = up;
  }
  return tiny ? s * 0x1p-16f : s;
}

__global__ void __launch_bounds__(256) k_clear_u32(uint32_t* __restrict__ p, size_t n) {
  size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  const size_t stride = (size_t)gridDim.x * blockDim.x;
  for (; i < n; i += stride) p[i] = 0u;
}

hipError_t launch_clear_u32(uint32_t* p, size_t n, hipStream_t s) {
  if (n == 0) return hipSuccess;
  const size_t blocks = n / 256 + 1;
  const unsigned grid = (unsigned)(blocks < 4096 ? blocks : 4096);
  hipLaunchKernelGGL(k_clear_u32, dim3(grid), dim3(256), 0, s, p, n);
  return hipGetLastError();
}

// Several ranges in one launch (the per-call control words), and an
// optional upload of words carried in the arguments (block 0).  The upload's
// words are read from the argument segment, where it follows the ClearSet.
static_assert(sizeof(ClearSet) % alignof(WordUpload) == 0, "WordUpload follows ClearSet unpadded");
__global__ void __launch_bounds__(256) k_clear_multi(ClearSet cs, WordUpload up) {
  if (blockIdx.x == 0 && up.n) {
    const uint32_t* src = reinterpret_cast<const uint32_t*>(
        (const char*)__builtin_amdgcn_kernarg_segment_ptr() + sizeof(ClearSet) +
        offsetof(WordUpload, w));
    for (uint32_t k = threadIdx.x; k < up.n; k += 256) up.dst[k] = src[k];
  }
  size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  const size_t stride = (size_t)gridDim.x * blockDim.x;
#pragma unroll
  for (int r = 0; r < kClearRanges; ++r) {
    if (r >= cs.n_ranges) break;
    for (; i < cs.n[r]; i += stride) cs.p[r][i] = 0u;
    i -= cs.n[r];  // continue the grid-stride walk into the next range
  }
}

hipError_t launch_clear_multi(const ClearSet& cs, hipStream_t s, const WordUpload* up) {
  size_t total = 0;
  for (int r = 0; r < cs.n_ranges; ++r) total += cs.n[r];
  WordUpload u;
  u.dst = nullptr;
  u.n = 0;
  if (up) u = *up;
  if (total == 0 && u.n == 0) return hipSuccess;
  const size_t blocks = total / 256 + 1;
  const unsigned grid = (unsigned)(blocks < 4096 ? blocks : 4096);
  hipLaunchKernelGGL(k_clear_multi, dim3(grid), dim3(256), 0, s, cs, u);
  return hipGetLastError();
}

// Host words to the device carried in kernel arguments, kUploadWords at a
// time (no copy from pageable host memory, which the runtime may stage
// synchronously): stream-ordered like any launch.
hipError_t launch_upload(uint32_t* dst, const void* src, size_t n_words, hipStream_t s) {
  const uint32_t* w = static_cast<const uint32_t*>(src);
  ClearSet none{};
  none.n_ranges = 0;
  for (size_t k = 0; k < n_words; k += kUploadWords) {
    WordUpload u;
    u.dst = dst + k;
    u.n = (uint32_t)std::min<size_t>(kUploadWords, n_words - k);
    std::memcpy(u.w, w + k, 4 * (size_t)u.n);
    hipLaunchKernelGGL(k_clear_multi, dim3(1), dim3(256), 0, s, none, u);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

__global__ void __launch_bounds__(256) k_activate(ModelD m, float* __restrict__ scale_out,
                                                  float* __restrict__ opacity_out) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= m.n) return;
  const int n = m.n;
#pragma unroll
  for (int k = 0; k < 3; ++k) scale_out[(size_t)k * n + i] = act_scale(m.scale[(size_t)k * n + i], m.raw);
  opacity_out[i] = act_opacity(m.opacity[i], m.raw);
}

hipError_t launch_activate(const ModelD& m, float* scale_out, float* opacity_out, hipStream_t s) {
  if (m.n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_activate, dim3(div_up((uint32_t)m.n, 256u)), dim3(256), 0, s, m, scale_out, opacity_out);
  return hipGetLastError();
}

// IEEE binary16 bit pattern to float (v_cvt_f32_f16: exact, every half is
// a float; half denormals are kept in the default floating-point mode).
__device__ __forceinline__ float half_bits(uint32_t h) {
  return (float)__builtin_bit_cast(_Float16, (uint16_t)h);
}

// Halves per codebook entry: 3 M rounded up to 16 bytes.
template <int D> constexpr int codebook_stride() { return ((3 * ((D + 1) * (D + 1) - 1)) + 7) & ~7; }

// Attribute loads per storage format: float arrays (activations applied for
// raw models) or half bit patterns of activated values.
template <int F>
__device__ __forceinline__ float ld_attr(const float* f, const uint16_t* h, size_t idx) {
  if constexpr (F == kFmtF32) return f[idx];
  else return half_bits(h[idx]);
}
template <int F> __device__ __forceinline__ float ld_scale(const ModelD& m, size_t idx) {
  if constexpr (F == kFmtF32) return act_scale(m.scale[idx], m.raw);
  else return half_bits(m.h_scale[idx]);
}

// The (D+1)^2 x 3 SH coefficients of Gaussian i, coefficient-major ([k][ch]).
template <int D, int F>
__device__ __forceinline__ void load_sh(const ModelD& m, int i, float* sh, uint32_t* counters) {
  constexpr int NC = (D + 1) * (D + 1);
  const size_t n = (size_t)m.n;
  if constexpr (F == kFmtF32) {
#pragma unroll
    for (int k = 0; k < NC * 3; ++k) sh[k] = m.sh[(size_t)k * n + i];
  } else {
#pragma unroll
    for (int ch = 0; ch < 3; ++ch) sh[ch] = half_bits(m.h_dc[(size_t)ch * n + i]);
    if constexpr (F == kFmtHalfPacked) {
#pragma unroll
      for (int k = 1; k < NC; ++k) {
        const uint32_t w = m.sh_packed[(size_t)(k - 1) * n + i];
        sh[k * 3 + 0] = m.sh_lo[0] + (float)(w & 0x7FFu) * m.sh_step[0];
        sh[k * 3 + 1] = m.sh_lo[1] + (float)((w >> 11) & 0x7FFu) * m.sh_step[1];
        sh[k * 3 + 2] = m.sh_lo[2] + (float)(w >> 22) * m.sh_step[2];
      }
    } else {
      uint32_t idx = m.sh_index[i];
      if (idx >= m.codebook_size) {
        atomicOr(&counters[kCntError], 128u);  // index outside the codebook: entry 0 is read
        idx = 0u;
      }
      constexpr int S = codebook_stride<D>();
      // the entry in 16-byte loads (8 halves each)
      const uint4* row = reinterpret_cast<const uint4*>(m.codebook + (size_t)idx * S);
#pragma unroll
      for (int q = 0; q < S / 8; ++q) {
        const uint4 w = row[q];
        const uint32_t ws[4] = {w.x, w.y, w.z, w.w};
#pragma unroll
        for (int h = 0; h < 8; ++h) {
          const int k = 3 + 8 * q + h;  // position in sh[]: coefficient-major after the 3 DC values
          if (k < NC * 3) sh[k] = half_bits((ws[h >> 1] >> (16 * (h & 1))) & 0xFFFFu);
        }
      }
    }
  }
}

// The tests a view makes before it needs more than the Gaussian's layer,
// centre and opacity: layer mask, clip planes, near plane, faded opacity.
__device__ __forceinline__ bool view_may_keep(const ViewD& V, uint32_t layer, float mx, float my, float mz,
                                              float op) {
  if (layer >= 32u || !((V.layer_mask >> layer) & 1u)) return false;
  for (int k = 0; k < V.n_clip; ++k) {
    const ClipD& c = V.clip[k];
    if (!((c.bits >> layer) & 1u)) continue;
    const float sd = ((c.n[0] * mx + c.n[1] * my) + c.n[2] * mz) + c.d;
    if (sd < 0.f) return false;
  }
  const float* W = V.R;
  const float tz = ((W[6] * mx + W[7] * my) + W[8] * mz) + V.t[2];
  if (!(tz > V.znear)) return false;
  return op * V.layer_op[layer] >= kAlphaMin;
}

// One thread per Gaussian; the Gaussian's attributes are read once and
// projected for every view of the job (stereo eyes, training views).  The
// rest of its attributes (rotation, scale, 3D filter, SH) are read only if
// some view may keep it, and then all at once: one memory round trip after
// the first instead of one per attribute group.  F selects the storage
// format of the attributes (float, or half with packed or codebook SH).
template <int D, int F>
__global__ void __launch_bounds__(256)
k_project(JobD job, const ViewD* __restrict__ views, float* __restrict__ records,
          uint32_t* __restrict__ n_tiles_out, uint4* __restrict__ tile_box, uint64_t* __restrict__ sort_keys,
          uint32_t* __restrict__ sort_vals, uint32_t* __restrict__ counters) {
  constexpr int NC = (D + 1) * (D + 1);
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  const ModelD& m = job.m;
  if (i >= m.n) return;
  const int n = m.n;
  const uint32_t layer = m.layer[i];
  const float mx = ld_attr<F>(m.mean, m.h_mean, i), my = ld_attr<F>(m.mean, m.h_mean, (size_t)n + i),
              mz = ld_attr<F>(m.mean, m.h_mean, 2 * (size_t)n + i);
  float op;
  if constexpr (F == kFmtF32) op = act_opacity(m.opacity[i], m.raw);
  else op = half_bits(m.h_opacity[i]);
  bool maybe = false;
  for (int jv = 0; jv < job.n_views && !maybe; ++jv)
    maybe = view_may_keep(views[job.view[jv]], layer, mx, my, mz, op);
  float sh[NC * 3];
  float qw = 0.f, qx = 0.f, qy = 0.f, qz = 0.f, sc0 = 0.f, sc1 = 0.f, sc2 = 0.f, f2 = 0.f;
  if (maybe) {
    qw = ld_attr<F>(m.quat, m.h_quat, i);
    qx = ld_attr<F>(m.quat, m.h_quat, (size_t)n + i);
    qy = ld_attr<F>(m.quat, m.h_quat, 2 * (size_t)n + i);
    qz = ld_attr<F>(m.quat, m.h_quat, 3 * (size_t)n + i);
    sc0 = ld_scale<F>(m, i);
    sc1 = ld_scale<F>(m, (size_t)n + i);
    sc2 = ld_scale<F>(m, 2 * (size_t)n + i);
    if (m.filter_3d) f2 = m.filter_3d[i];
    load_sh<D, F>(m, i, sh, counters);
  }
  float Rq[9];
  float qn = -1.f;  // < 0: rotation not computed yet

  for (int jv = 0; jv < job.n_views; ++jv) {
    const ViewD& V = views[job.view[jv]];
    const uint32_t r = V.rec_off + (uint32_t)i;
    uint32_t nt = 0;
    uint32_t own_key = 0xFFFFFFFFu;  // depth bits of a kept record (culled ones sort last)
    do {
      // layer activation mask
      if (layer >= 32u || !((V.layer_mask >> layer) & 1u)) break;
      // per-layer clip planes through the centre
      bool clipped = false;
      for (int k = 0; k < V.n_clip; ++k) {
        const ClipD& c = V.clip[k];
        if (!((c.bits >> layer) & 1u)) continue;
        const float sd = ((c.n[0] * mx + c.n[1] * my) + c.n[2] * mz) + c.d;
        if (sd < 0.f) { clipped = true; break; }
      }
      if (clipped) break;
      const float* W = V.R;
      const float tx = ((W[0] * mx + W[1] * my) + W[2] * mz) + V.t[0];
      const float ty = ((W[3] * mx + W[4] * my) + W[5] * mz) + V.t[1];
      const float tz = ((W[6] * mx + W[7] * my) + W[8] * mz) + V.t[2];
      if (!(tz > V.znear)) break;
      const float opv = op * V.layer_op[layer];  // the view's fading of the layer
      if (opv < kAlphaMin) break;
      if (qn < 0.f) {
        qn = sqrt_rn(((qw * qw + qx * qx) + qy * qy) + qz * qz);
        if (!(qn > 0.f)) { qn = 0.f; break; }
        qw = __fdiv_rn(qw, qn); qx = __fdiv_rn(qx, qn); qy = __fdiv_rn(qy, qn); qz = __fdiv_rn(qz, qn);
        Rq[0] = 1.f - 2.f * (qy * qy + qz * qz);
        Rq[1] = 2.f * (qx * qy - qw * qz);
        Rq[2] = 2.f * (qx * qz + qw * qy);
        Rq[3] = 2.f * (qx * qy + qw * qz);
        Rq[4] = 1.f - 2.f * (qx * qx + qz * qz);
        Rq[5] = 2.f * (qy * qz - qw * qx);
        Rq[6] = 2.f * (qx * qz - qw * qy);
        Rq[7] = 2.f * (qy * qz + qw * qx);
        Rq[8] = 1.f - 2.f * (qx * qx + qy * qy);
      }
      if (!(qn > 0.f)) break;
      // Sigma = M M^T, M = Rq diag(s)
      float s0 = sc0, s1 = sc1, s2 = sc2;
      float opf = opv;  // opacity after the Mip filters
      if (m.filter_3d) {
        // 3D filter: the Gaussian convolved with an isotropic one of variance f2
        const float q0 = s0 * s0, q1 = s1 * s1, q2 = s2 * s2;
        const float p0 = q0 + f2, p1 = q1 + f2, p2 = q2 + f2;
        s0 = sqrt_rn(p0); s1 = sqrt_rn(p1); s2 = sqrt_rn(p2);
        opf = opf * sqrt_rn(__fdiv_rn((q0 * q1) * q2, (p0 * p1) * p2));
      }
      float M[9];
#pragma unroll
      for (int rr = 0; rr < 3; ++rr) {
        M[3 * rr + 0] = Rq[3 * rr + 0] * s0;
        M[3 * rr + 1] = Rq[3 * rr + 1] * s1;
        M[3 * rr + 2] = Rq[3 * rr + 2] * s2;
      }
      float S[9];
#pragma unroll
      for (int rr = 0; rr < 3; ++rr)
#pragma unroll
        for (int cc = 0; cc < 3; ++cc)
          S[3 * rr + cc] = (M[3 * rr] * M[3 * cc] + M[3 * rr + 1] * M[3 * cc + 1]) + M[3 * rr + 2] * M[3 * cc + 2];
      // local affine approximation of the perspective map, slope clamped
      const float lim_x = __fdiv_rn(V.guard * fmaxf(V.cx, (float)V.W - V.cx), V.fx);
      const float lim_y = __fdiv_rn(V.guard * fmaxf(V.cy, (float)V.H - V.cy), V.fy);
      const float xr = fminf(fmaxf(__fdiv_rn(tx, tz), -lim_x), lim_x);
      const float yr = fminf(fmaxf(__fdiv_rn(ty, tz), -lim_y), lim_y);
      const float xc = xr * tz, yc = yr * tz;
      const float tz2 = tz * tz;
      const float J00 = __fdiv_rn(V.fx, tz);
      const float J02 = __fdiv_rn(-(V.fx * xc), tz2);
      const float J11 = __fdiv_rn(V.fy, tz);
      const float J12 = __fdiv_rn(-(V.fy * yc), tz2);
      float Tm[6];
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        Tm[c] = J00 * W[c] + J02 * W[6 + c];
        Tm[3 + c] = J11 * W[3 + c] + J12 * W[6 + c];
      }
      float U[6];
#pragma unroll
      for (int rr = 0; rr < 2; ++rr)
#pragma unroll
        for (int c = 0; c < 3; ++c)
          U[3 * rr + c] = (Tm[3 * rr] * S[c] + Tm[3 * rr + 1] * S[3 + c]) + Tm[3 * rr + 2] * S[6 + c];
      const float s00 = (U[0] * Tm[0] + U[1] * Tm[1]) + U[2] * Tm[2];
      const float s01 = (U[0] * Tm[3] + U[1] * Tm[4]) + U[2] * Tm[5];
      const float s11 = (U[3] * Tm[3] + U[4] * Tm[4]) + U[5] * Tm[5];
      const float dil = V.mip_2d ? V.mip_var : kKappa;
      const float a = s00 + dil, b = s01, c = s11 + dil;
      const float det = a * c - b * b;
      if (!(det > 0.f)) break;
      if (V.mip_2d) {
        // 2D Mip filter: the dilation's opacity compensation
        const float det0 = s00 * s11 - s01 * s01;
        opf = opf * sqrt_rn(__fdiv_rn(fmaxf(det0, 0.f), det));
      }
      if (opf < kAlphaMin) break;
      const float ca = __fdiv_rn(c, det), cb = __fdiv_rn(-b, det), cc = __fdiv_rn(a, det);
      const float u = __fdiv_rn(V.fx * tx, tz) + V.cx;
      const float v = __fdiv_rn(V.fy * ty, tz) + V.cy;
      // tile box of {q <= qmax}: clamp in float, then convert
      const float hwx = sqrt_rn(kQMax * a), hwy = sqrt_rn(kQMax * c);
      const float ftx = (float)V.tiles_x, fty = (float)V.tiles_y;
      const float inv_tile = 1.0f / (float)kTile;
      const float fx0 = fminf(fmaxf(floorf((u - hwx) * inv_tile), 0.f), ftx);
      const float fx1 = fminf(fmaxf(floorf((u + hwx) * inv_tile) + 1.f, 0.f), ftx);
      const float fy0 = fminf(fmaxf(floorf((v - hwy) * inv_tile), 0.f), fty);
      const float fy1 = fminf(fmaxf(floorf((v + hwy) * inv_tile) + 1.f, 0.f), fty);
      const int x0 = (int)fx0, x1 = (int)fx1, y0 = (int)fy0, y1 = (int)fy1;
      nt = (uint32_t)((x1 - x0) * (y1 - y0));
      if (nt == 0) break;
      // view-dependent colour from the eye centre -R^T t
      const float ccx = -((W[0] * V.t[0] + W[3] * V.t[1]) + W[6] * V.t[2]);
      const float ccy = -((W[1] * V.t[0] + W[4] * V.t[1]) + W[7] * V.t[2]);
      const float ccz = -((W[2] * V.t[0] + W[5] * V.t[1]) + W[8] * V.t[2]);
      const float ddx = mx - ccx, ddy = my - ccy, ddz = mz - ccz;
      const float dl = sqrt_rn((ddx * ddx + ddy * ddy) + ddz * ddz);
      const float dirx = __fdiv_rn(ddx, dl), diry = __fdiv_rn(ddy, dl), dirz = __fdiv_rn(ddz, dl);
      float Y[16];
      sh_basis<D>(dirx, diry, dirz, Y);
      float rgb[3];
      uint32_t clamp_bits = 0;
#pragma unroll
      for (int ch = 0; ch < 3; ++ch) {
        float acc = sh[ch] * Y[0];
#pragma unroll
        for (int k = 1; k < NC; ++k) acc = acc + sh[k * 3 + ch] * Y[k];
        float raw = acc + 0.5f;
        if (raw < 0.f) { clamp_bits |= 1u << ch; raw = 0.f; }
        rgb[ch] = raw;
      }
      float4* rec = reinterpret_cast<float4*>(records + (size_t)r * kRecordFloats);
      rec[0] = make_float4(u, v, ca, cb);
      rec[1] = make_float4(cc, opf, rgb[0], rgb[1]);
      rec[2] = make_float4(rgb[2], tz, __uint_as_float(clamp_bits), __uint_as_float(nt));
      const uint32_t base_tile = V.tile_off + (uint32_t)y0 * (uint32_t)V.tiles_x + (uint32_t)x0;
      tile_box[r] = make_uint4(base_tile, (uint32_t)(x1 - x0) | ((uint32_t)(y1 - y0) << 16),
                               __float_as_uint(tz), (uint32_t)V.tiles_x);
      own_key = __float_as_uint(tz);
    } while (false);
    if (sort_keys && (V.sort_mode == kSortOwn || V.sort_mode == kSortCamera)) {
      // the Gaussian's key in its sort unit: its own depth, or (every
      // Gaussian, kept in this view or not: a follower view may keep it) its
      // depth in the sort camera, in the order of the view's own depth
      const uint32_t key = V.sort_mode == kSortOwn
                               ? own_key
                               : __float_as_uint(((V.sort_r[0] * mx + V.sort_r[1] * my) + V.sort_r[2] * mz) + V.sort_t);
      sort_keys[V.sort_off + (uint32_t)i] = ((uint64_t)V.sort_unit << 32) | key;
      sort_vals[V.sort_off + (uint32_t)i] = r;
    }
    n_tiles_out[r] = nt;
    if (nt == 0) {
      // culled: the record's tile count slot says so (the rest is never read)
      records[(size_t)r * kRecordFloats + 11] = __uint_as_float(0u);
    }
  }
}

namespace {
template <int F>
void launch_project_fmt(const JobD& job, const ViewD* views_dev, float* records, uint32_t* n_tiles,
                        uint4* tile_box, uint64_t* sort_keys, uint32_t* sort_vals, uint32_t* counters,
                        hipStream_t s) {
  const dim3 grid(div_up((uint32_t)job.m.n, 256u)), block(256);
  switch (job.m.D) {
    case 0: hipLaunchKernelGGL((k_project<0, F>), grid, block, 0, s, job, views_dev, records, n_tiles, tile_box,
                               sort_keys, sort_vals, counters); break;
    case 1: hipLaunchKernelGGL((k_project<1, F>), grid, block, 0, s, job, views_dev, records, n_tiles, tile_box,
                               sort_keys, sort_vals, counters); break;
    case 2: hipLaunchKernelGGL((k_project<2, F>), grid, block, 0, s, job, views_dev, records, n_tiles, tile_box,
                               sort_keys, sort_vals, counters); break;
    default: hipLaunchKernelGGL((k_project<3, F>), grid, block, 0, s, job, views_dev, records, n_tiles, tile_box,
                                sort_keys, sort_vals, counters); break;
  }
}
}  // namespace

hipError_t launch_project(const JobD& job, const ViewD* views_dev, float* records, uint32_t* n_tiles,
                          uint4* tile_box, uint64_t* sort_keys, uint32_t* sort_vals, uint32_t* counters,
                          hipStream_t s) {
  if (job.m.n <= 0 || job.n_views <= 0) return hipSuccess;
  switch (job.m.fmt) {
    case kFmtHalfPacked:
      launch_project_fmt<kFmtHalfPacked>(job, views_dev, records, n_tiles, tile_box, sort_keys, sort_vals, counters, s);
      break;
    case kFmtHalfCodebook:
      launch_project_fmt<kFmtHalfCodebook>(job, views_dev, records, n_tiles, tile_box, sort_keys, sort_vals, counters,
                                           s);
      break;
    default:
      launch_project_fmt<kFmtF32>(job, views_dev, records, n_tiles, tile_box, sort_keys, sort_vals, counters, s);
      break;
  }
  return hipGetLastError();
}

}  // namespace gsr
