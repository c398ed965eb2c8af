// Backward of the projection: per Gaussian, the screen-space gradients of
// its records (one per view) are chained through the conic inverse, the EWA
// covariance J W Sigma W^T J^T, Sigma = R S S^T R^T, the quaternion
// normalisation, the perspective map of the centre and the SH colour with its
// view direction, and summed over the views.  Frozen layers (Sec. 3.2) get
// zero.  Two kernels, so that neither holds the covariance chain and the SH
// expansion at once: the geometry kernel (which also sums each record's pair
// partials and leaves its colour gradient behind), then the SH kernel, which
// adds the view-direction term to the mean and computes the activity
// 2|g_mean| + 0.1|g_sh| + 0.1|g_log s| of Sec. 3.2.2 into activity[].
#include "common.hpp"
#include "sh.hpp"

namespace gsr {

// Screen-space gradient of record r: the sum of its pairs' partials (stored
// at their emission indices, so contiguous per record) in emission order, and
// the largest alpha * T it reached.  Only pairs with alive[e] set have
// partials (the others are exactly zero and were never written); their
// loads are redirected to the zero entry at index `zero`, so the loads stay
// branch-free and adding its +0 leaves every sum bit for bit unchanged (a
// sum that starts at +0 never holds -0).
__device__ __forceinline__ void record_grad(uint32_t r, const uint32_t* __restrict__ offsets,
                                            const float* __restrict__ g_pair, const uint8_t* __restrict__ alive,
                                            uint32_t zero, uint32_t K, float* g, float& wmax) {
  for (int c = 0; c < 9; ++c) g[c] = 0.f;
  const uint32_t e0 = offsets[r], e1 = min(offsets[r + 1], K);
  // four pairs per step: their flags, then their loads, in flight at once
  for (uint32_t e = e0; e < e1; e += 4) {
    uint32_t idx[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const uint32_t q = e + (uint32_t)u;
      const bool live = alive[min(q, e1 - 1u)] != 0;
      idx[u] = q < e1 && live ? q : zero;
    }
    float4 x[12];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const float4* src = reinterpret_cast<const float4*>(g_pair + (size_t)idx[u] * 12);
      x[3 * u] = src[0];
      x[3 * u + 1] = src[1];
      x[3 * u + 2] = src[2];
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const float4 x0 = x[3 * u], x1 = x[3 * u + 1], x2 = x[3 * u + 2];
      g[0] += x0.x; g[1] += x0.y; g[2] += x0.z; g[3] += x0.w;
      g[4] += x1.x; g[5] += x1.y; g[6] += x1.z; g[7] += x1.w;
      g[8] += x2.x;
      wmax = fmaxf(wmax, x2.y);
    }
  }
}

// Geometry: opacity, and the centre / covariance chain to mean, scale and
// quaternion.  The colour gradient of each visible record (zero on clamped
// channels) is left in g_col[r][3] for the SH kernel.
__global__ void __launch_bounds__(256)
k_project_bwd_geom(JobD job, const ViewD* __restrict__ views, const float* __restrict__ records,
                   const uint32_t* __restrict__ offsets, const float* __restrict__ g_pair,
                   const uint8_t* __restrict__ alive, uint32_t cap, const uint32_t* __restrict__ counters,
                   uint32_t trainable, float* __restrict__ g_mean, float* __restrict__ g_scale,
                   float* __restrict__ g_quat, float* __restrict__ g_opacity, float* __restrict__ g_col,
                   float* __restrict__ max_contrib) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  const ModelD& m = job.m;
  if (i >= m.n) return;
  const int n = m.n;
  const uint32_t layer = m.layer[i];
  const bool train = layer < 32u && ((trainable >> layer) & 1u);
  const uint32_t K = min(counters[kCntPairs], cap);
  float wmax = 0.f;
  float gm[3] = {0.f, 0.f, 0.f}, gs[3] = {0.f, 0.f, 0.f}, gq[4] = {0.f, 0.f, 0.f, 0.f}, go = 0.f;
  if (!train && max_contrib) {
    float g[9];
    for (int jv = 0; jv < job.n_views; ++jv) {
      const uint32_t r = views[job.view[jv]].rec_off + (uint32_t)i;
      if (__float_as_uint(records[(size_t)r * kRecordFloats + 11]) != 0u) record_grad(r, offsets, g_pair, alive, cap, K, g, wmax);
    }
  }
  if (train) {
    const float mx = m.mean[i], my = m.mean[n + i], mz = m.mean[2 * n + i];
    const float s[3] = {act_scale(m.scale[i], m.raw), act_scale(m.scale[n + i], m.raw),
                        act_scale(m.scale[2 * n + i], m.raw)};
    float qw = m.quat[i], qx = m.quat[n + i], qy = m.quat[2 * n + i], qz = m.quat[3 * n + i];
    const float qn = sqrtf(qw * qw + qx * qx + qy * qy + qz * qz);
    const float iq = qn > 0.f ? 1.f / qn : 0.f;
    qw *= iq; qx *= iq; qy *= iq; qz *= iq;
    float Rq[9];
    Rq[0] = 1.f - 2.f * (qy * qy + qz * qz);
    Rq[1] = 2.f * (qx * qy - qw * qz);
    Rq[2] = 2.f * (qx * qz + qw * qy);
    Rq[3] = 2.f * (qx * qy + qw * qz);
    Rq[4] = 1.f - 2.f * (qx * qx + qz * qz);
    Rq[5] = 2.f * (qy * qz - qw * qx);
    Rq[6] = 2.f * (qx * qz - qw * qy);
    Rq[7] = 2.f * (qy * qz + qw * qx);
    Rq[8] = 1.f - 2.f * (qx * qx + qy * qy);
    float M[9], S[9];
#pragma unroll
    for (int r = 0; r < 3; ++r)
#pragma unroll
      for (int c = 0; c < 3; ++c) M[3 * r + c] = Rq[3 * r + c] * s[c];
#pragma unroll
    for (int r = 0; r < 3; ++r)
#pragma unroll
      for (int c = 0; c < 3; ++c)
        S[3 * r + c] = M[3 * r] * M[3 * c] + M[3 * r + 1] * M[3 * c + 1] + M[3 * r + 2] * M[3 * c + 2];
    float dM[9] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
    for (int jv = 0; jv < job.n_views; ++jv) {
      const ViewD& V = views[job.view[jv]];
      const uint32_t r = V.rec_off + (uint32_t)i;
      const float* rec = records + (size_t)r * kRecordFloats;
      if (__float_as_uint(rec[11]) == 0u) continue;  // culled in this view
      const uint32_t clamp_bits = __float_as_uint(rec[10]);
      float g[9];
      record_grad(r, offsets, g_pair, alive, cap, K, g, wmax);
      go += g[5];
#pragma unroll
      for (int ch = 0; ch < 3; ++ch) g_col[(size_t)r * 3 + ch] = ((clamp_bits >> ch) & 1u) ? 0.f : g[6 + ch];
      const float* W = V.R;
      const float tx = W[0] * mx + W[1] * my + W[2] * mz + V.t[0];
      const float ty = W[3] * mx + W[4] * my + W[5] * mz + V.t[1];
      const float tz = W[6] * mx + W[7] * my + W[8] * mz + V.t[2];
      // ---- conic -> 2D covariance (a, b, c)
      const float lim_x = V.guard * fmaxf(V.cx, (float)V.W - V.cx) / V.fx;
      const float lim_y = V.guard * fmaxf(V.cy, (float)V.H - V.cy) / V.fy;
      const float xr0 = tx / tz, yr0 = ty / tz;
      const bool xcl = (xr0 < -lim_x) || (xr0 > lim_x);
      const bool ycl = (yr0 < -lim_y) || (yr0 > lim_y);
      const float xr = fminf(fmaxf(xr0, -lim_x), lim_x), yr = fminf(fmaxf(yr0, -lim_y), lim_y);
      const float itz = 1.f / tz, itz2 = itz * itz, itz3 = itz2 * itz;
      const float J00 = V.fx * itz, J02 = -V.fx * xr * itz;
      const float J11 = V.fy * itz, J12 = -V.fy * yr * itz;
      float Tm[6];
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        Tm[c] = J00 * W[c] + J02 * W[6 + c];
        Tm[3 + c] = J11 * W[3 + c] + J12 * W[6 + c];
      }
      float ST0[3], ST1[3];
#pragma unroll
      for (int r2 = 0; r2 < 3; ++r2) {
        ST0[r2] = S[3 * r2] * Tm[0] + S[3 * r2 + 1] * Tm[1] + S[3 * r2 + 2] * Tm[2];
        ST1[r2] = S[3 * r2] * Tm[3] + S[3 * r2 + 1] * Tm[4] + S[3 * r2 + 2] * Tm[5];
      }
      const float a = Tm[0] * ST0[0] + Tm[1] * ST0[1] + Tm[2] * ST0[2] + kKappa;
      const float b = Tm[0] * ST1[0] + Tm[1] * ST1[1] + Tm[2] * ST1[2];
      const float c = Tm[3] * ST1[0] + Tm[4] * ST1[1] + Tm[5] * ST1[2] + kKappa;
      const float det = a * c - b * b;
      const float id2 = 1.f / (det * det);
      const float dca = g[2], dcb = g[3], dcc = g[4];
      const float da = (-c * c * dca + b * c * dcb - b * b * dcc) * id2;
      const float db = (2.f * b * c * dca - (a * c + b * b) * dcb + 2.f * a * b * dcc) * id2;
      const float dc = (-b * b * dca + a * b * dcb - a * a * dcc) * id2;
      // ---- Sigma' = T Sigma T^T
      float dT0[3], dT1[3];
#pragma unroll
      for (int r2 = 0; r2 < 3; ++r2) {
        dT0[r2] = 2.f * da * ST0[r2] + db * ST1[r2];
        dT1[r2] = db * ST0[r2] + 2.f * dc * ST1[r2];
      }
      // dSigma (symmetrised) and dM = (dS + dS^T) M
      float dS[9];
#pragma unroll
      for (int r2 = 0; r2 < 3; ++r2)
#pragma unroll
        for (int q2 = 0; q2 < 3; ++q2)
          dS[3 * r2 + q2] = da * Tm[r2] * Tm[q2] + db * Tm[r2] * Tm[3 + q2] + dc * Tm[3 + r2] * Tm[3 + q2];
#pragma unroll
      for (int r2 = 0; r2 < 3; ++r2)
#pragma unroll
        for (int k = 0; k < 3; ++k) {
          float acc = 0.f;
#pragma unroll
          for (int j = 0; j < 3; ++j) acc += (dS[3 * r2 + j] + dS[3 * j + r2]) * M[3 * j + k];
          dM[3 * r2 + k] += acc;
        }
      // ---- Jacobian and projected centre -> camera-space centre
      float dJ00 = 0.f, dJ02 = 0.f, dJ11 = 0.f, dJ12 = 0.f;
#pragma unroll
      for (int r2 = 0; r2 < 3; ++r2) {
        dJ00 += dT0[r2] * W[r2];
        dJ02 += dT0[r2] * W[6 + r2];
        dJ11 += dT1[r2] * W[3 + r2];
        dJ12 += dT1[r2] * W[6 + r2];
      }
      float dtx = 0.f, dty = 0.f, dtz = 0.f;
      dtz += -(dJ00 * V.fx + dJ11 * V.fy) * itz2;
      if (!xcl) {
        dtx += -dJ02 * V.fx * itz2;
        dtz += 2.f * dJ02 * V.fx * tx * itz3;
      } else {
        dtz += dJ02 * V.fx * xr * itz2;
      }
      if (!ycl) {
        dty += -dJ12 * V.fy * itz2;
        dtz += 2.f * dJ12 * V.fy * ty * itz3;
      } else {
        dtz += dJ12 * V.fy * yr * itz2;
      }
      dtx += g[0] * V.fx * itz;
      dtz += -g[0] * V.fx * tx * itz2;
      dty += g[1] * V.fy * itz;
      dtz += -g[1] * V.fy * ty * itz2;
      gm[0] += W[0] * dtx + W[3] * dty + W[6] * dtz;
      gm[1] += W[1] * dtx + W[4] * dty + W[7] * dtz;
      gm[2] += W[2] * dtx + W[5] * dty + W[8] * dtz;
    }
    // ---- M = Rq diag(s) -> scale, rotation -> quaternion
    float dR[9];
#pragma unroll
    for (int r = 0; r < 3; ++r)
#pragma unroll
      for (int k = 0; k < 3; ++k) {
        gs[k] += dM[3 * r + k] * Rq[3 * r + k];
        dR[3 * r + k] = dM[3 * r + k] * s[k];
      }
    float dq[4];
    dq[0] = 2.f * (-qz * dR[1] + qy * dR[2] + qz * dR[3] - qx * dR[5] - qy * dR[6] + qx * dR[7]);
    dq[1] = 2.f * (qy * dR[1] + qz * dR[2] + qy * dR[3] - 2.f * qx * dR[4] - qw * dR[5] + qz * dR[6] +
                   qw * dR[7] - 2.f * qx * dR[8]);
    dq[2] = 2.f * (-2.f * qy * dR[0] + qx * dR[1] + qw * dR[2] + qx * dR[3] + qz * dR[5] - qw * dR[6] +
                   qz * dR[7] - 2.f * qy * dR[8]);
    dq[3] = 2.f * (-2.f * qz * dR[0] - qw * dR[1] + qx * dR[2] + qw * dR[3] - 2.f * qz * dR[4] +
                   qy * dR[5] + qx * dR[6] + qy * dR[7]);
    const float qd = qw * dq[0] + qx * dq[1] + qy * dq[2] + qz * dq[3];
    gq[0] = (dq[0] - qw * qd) * iq;
    gq[1] = (dq[1] - qx * qd) * iq;
    gq[2] = (dq[2] - qy * qd) * iq;
    gq[3] = (dq[3] - qz * qd) * iq;
    if (m.raw) {  // chain rule of the activations: d exp = exp, d logistic = o (1 - o)
#pragma unroll
      for (int k = 0; k < 3; ++k) gs[k] *= s[k];
      const float o = act_opacity(m.opacity[i], 1);
      go *= o * (1.0f - o);
    }
  }
#pragma unroll
  for (int k = 0; k < 3; ++k) g_mean[(size_t)k * n + i] = gm[k];
#pragma unroll
  for (int k = 0; k < 3; ++k) g_scale[(size_t)k * n + i] = gs[k];
#pragma unroll
  for (int k = 0; k < 4; ++k) g_quat[(size_t)k * n + i] = gq[k];
  g_opacity[i] = go;
  if (max_contrib) max_contrib[i] = fmaxf(max_contrib[i], wmax);
}

// Colour: SH coefficients and, through the view direction, the mean; then
// the activity, which needs the final gradients.
template <int D>
__global__ void __launch_bounds__(256)
k_project_bwd_sh(JobD job, const ViewD* __restrict__ views, const float* __restrict__ records,
                 uint32_t trainable, const float* __restrict__ g_col, float* __restrict__ g_mean,
                 const float* __restrict__ g_scale, float* __restrict__ g_sh, float* __restrict__ activity) {
  constexpr int NC = (D + 1) * (D + 1);
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  const ModelD& m = job.m;
  if (i >= m.n) return;
  const int n = m.n;
  const uint32_t layer = m.layer[i];
  const bool train = layer < 32u && ((trainable >> layer) & 1u);
  float gsh[NC * 3];
#pragma unroll
  for (int k = 0; k < NC * 3; ++k) gsh[k] = 0.f;
  if (!train) {
#pragma unroll
    for (int k = 0; k < NC * 3; ++k) g_sh[(size_t)k * n + i] = 0.f;
    return;
  }
  const float mx = m.mean[i], my = m.mean[n + i], mz = m.mean[2 * n + i];
  float gm[3] = {0.f, 0.f, 0.f};
  for (int jv = 0; jv < job.n_views; ++jv) {
    const ViewD& V = views[job.view[jv]];
    const uint32_t r = V.rec_off + (uint32_t)i;
    if (__float_as_uint(records[(size_t)r * kRecordFloats + 11]) == 0u) continue;  // culled in this view
    const float drgb[3] = {g_col[(size_t)r * 3], g_col[(size_t)r * 3 + 1], g_col[(size_t)r * 3 + 2]};
    const float* W = V.R;
    const float ccx = -(W[0] * V.t[0] + W[3] * V.t[1] + W[6] * V.t[2]);
    const float ccy = -(W[1] * V.t[0] + W[4] * V.t[1] + W[7] * V.t[2]);
    const float ccz = -(W[2] * V.t[0] + W[5] * V.t[1] + W[8] * V.t[2]);
    const float ddx = mx - ccx, ddy = my - ccy, ddz = mz - ccz;
    const float dl = sqrtf(ddx * ddx + ddy * ddy + ddz * ddz);
    const float idl = 1.f / dl;
    const float dirx = ddx * idl, diry = ddy * idl, dirz = ddz * idl;
    float Y[16];
    sh_basis<D>(dirx, diry, dirz, Y);
    // d rgb / d dir = sum_k (sum_ch drgb_ch sh_k,ch) grad Y_k: one gradient of
    // the SH expansion with the drgb-weighted coefficients
    float e[16];
#pragma unroll
    for (int k = 0; k < NC; ++k) {
      e[k] = 0.f;
#pragma unroll
      for (int ch = 0; ch < 3; ++ch) {
        e[k] += m.sh[(size_t)(k * 3 + ch) * n + i] * drgb[ch];
        gsh[k * 3 + ch] += Y[k] * drgb[ch];
      }
    }
    if (D > 0) {
      float ddir[3];
      sh_dir_grad<D>(dirx, diry, dirz, e, ddir[0], ddir[1], ddir[2]);
      const float dd = dirx * ddir[0] + diry * ddir[1] + dirz * ddir[2];
      gm[0] += (ddir[0] - dirx * dd) * idl;
      gm[1] += (ddir[1] - diry * dd) * idl;
      gm[2] += (ddir[2] - dirz * dd) * idl;
    }
  }
  float pm = 0.f;
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    const float v = g_mean[(size_t)k * n + i] + gm[k];
    g_mean[(size_t)k * n + i] = v;
    pm += v * v;
  }
  float pc = 0.f;
#pragma unroll
  for (int k = 0; k < NC * 3; ++k) {
    g_sh[(size_t)k * n + i] = gsh[k];
    pc += gsh[k] * gsh[k];
  }
  if (activity) {
    float ps = 0.f;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      const float gl = m.raw ? g_scale[(size_t)k * n + i] : g_scale[(size_t)k * n + i] * m.scale[(size_t)k * n + i];
      ps += gl * gl;
    }
    activity[i] += 2.f * sqrtf(pm) + 0.1f * sqrtf(pc) + 0.1f * sqrtf(ps);
  }
}

hipError_t launch_project_bwd(const JobD& job, const ViewD* views_dev, const float* records,
                              const uint32_t* offsets, const float* g_pair, const uint8_t* alive,
                              uint32_t pair_capacity,
                              const uint32_t* counters, uint32_t trainable, float* g_mean, float* g_scale,
                              float* g_quat, float* g_opacity, float* g_sh, float* g_col, float* max_contrib,
                              float* activity, hipStream_t s) {
  if (job.m.n <= 0) return hipSuccess;
  const dim3 grid(div_up((uint32_t)job.m.n, 256u)), block(256);
  hipLaunchKernelGGL(k_project_bwd_geom, grid, block, 0, s, job, views_dev, records, offsets, g_pair, alive,
                     pair_capacity, counters, trainable, g_mean, g_scale, g_quat, g_opacity, g_col, max_contrib);
  switch (job.m.D) {
    case 0: hipLaunchKernelGGL(k_project_bwd_sh<0>, grid, block, 0, s, job, views_dev, records, trainable, g_col,
                               g_mean, g_scale, g_sh, activity); break;
    case 1: hipLaunchKernelGGL(k_project_bwd_sh<1>, grid, block, 0, s, job, views_dev, records, trainable, g_col,
                               g_mean, g_scale, g_sh, activity); break;
    case 2: hipLaunchKernelGGL(k_project_bwd_sh<2>, grid, block, 0, s, job, views_dev, records, trainable, g_col,
                               g_mean, g_scale, g_sh, activity); break;
    default: hipLaunchKernelGGL(k_project_bwd_sh<3>, grid, block, 0, s, job, views_dev, records, trainable, g_col,
                                g_mean, g_scale, g_sh, activity); break;
  }
  return hipGetLastError();
}

}  // namespace gsr
