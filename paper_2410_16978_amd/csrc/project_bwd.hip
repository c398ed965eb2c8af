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
// at their emission indices, so contiguous per record) in emission order,
// accumulated in double, and the largest alpha * T it reached.  Only pairs
// with alive[e] set have partials (the others are exactly zero and were never
// written); their loads are redirected to the zero entry at index `zero`, so
// the loads stay branch-free and adding its +0 leaves every sum bit for bit
// unchanged (a sum that starts at +0 never holds -0).
__device__ __forceinline__ void record_grad(uint32_t e0, uint32_t e1, const float* __restrict__ g_pair,
                                            const uint8_t* __restrict__ alive, uint32_t zero, double* g,
                                            float& wmax) {
  for (int c = 0; c < 9; ++c) g[c] = 0.0;
  if (e0 >= e1) return;
  // four pairs per step: their loads in flight at once, and with them the
  // flags of the next step's four (one load round trip per step)
  bool live[4];
#pragma unroll
  for (int u = 0; u < 4; ++u) live[u] = alive[min(e0 + (uint32_t)u, e1 - 1u)] != 0;
  for (uint32_t e = e0; e < e1; e += 4) {
    uint32_t idx[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const uint32_t q = e + (uint32_t)u;
      idx[u] = q < e1 && live[u] ? q : zero;
    }
    float4 x[12];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const float4* src = reinterpret_cast<const float4*>(g_pair + (size_t)idx[u] * 12);
      x[3 * u] = src[0];
      x[3 * u + 1] = src[1];
      x[3 * u + 2] = src[2];
    }
    uint8_t nf[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) nf[u] = alive[min(e + 4u + (uint32_t)u, e1 - 1u)];
    // keeps those flag loads here, issued before the wait for the partials
    // (left alone, the compiler moves them down to their use)
    asm volatile("" ::: "memory");
#pragma unroll
    for (int u = 0; u < 4; ++u) live[u] = nf[u] != 0;
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
// quaternion, in double: the chain rule takes differences of products of
// the covariance terms (a nearly isotropic splat's rotation gradient is a
// small difference of large ones), which float32 would leave with a relative
// error far above the per-pixel terms' own.  The kernel is bound by the
// loads of the pair partials, so the double arithmetic costs no time.  The
// colour gradient of each visible record (zero on clamped channels) is left
// in g_col[r][3] for the SH kernel.
__global__ void __launch_bounds__(256)
k_project_bwd_geom(JobD job, const ViewD* __restrict__ views, const float* __restrict__ records,
                   const uint32_t* __restrict__ offsets, const float* __restrict__ g_pair,
                   const uint8_t* __restrict__ alive, uint32_t cap, const uint32_t* __restrict__ counters,
                   uint32_t trainable, float* __restrict__ g_mean, float* __restrict__ g_scale,
                   float* __restrict__ g_quat, float* __restrict__ g_opacity, float* __restrict__ g_col,
                   float* __restrict__ max_contrib, float* __restrict__ dens_grad, float* __restrict__ dens_cnt) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  const ModelD& m = job.m;
  if (i >= m.n) return;
  const int n = m.n;
  const uint32_t layer = m.layer[i];
  const bool train = layer < 32u && ((trainable >> layer) & 1u);
  const uint32_t K = min(counters[kCntPairs], cap);
  float wmax = 0.f;
  double gm[3] = {0.0, 0.0, 0.0}, gs[3] = {0.0, 0.0, 0.0}, gq[4] = {0.0, 0.0, 0.0, 0.0}, go = 0.0;
  double dgs = 0.0, dgc = 0.0;
  if (!train && max_contrib) {
    double g[9];
    for (int jv = 0; jv < job.n_views; ++jv) {
      const uint32_t r = views[job.view[jv]].rec_off + (uint32_t)i;
      const uint32_t kept = __float_as_uint(records[(size_t)r * kRecordFloats + 11]);
      uint32_t e0 = offsets[r], e1 = offsets[r + 1];
      asm volatile("" : "+v"(e0), "+v"(e1));  // both loads issued before the test, not sunk below it
      e1 = min(e1, K);
      if (kept != 0u) record_grad(e0, e1, g_pair, alive, cap, g, wmax);
    }
  }
  if (train) {
    const double mx = m.mean[i], my = m.mean[n + i], mz = m.mean[2 * n + i];
    const double s[3] = {act_scale(m.scale[i], m.raw), act_scale(m.scale[n + i], m.raw),
                         act_scale(m.scale[2 * n + i], m.raw)};
    double qw = m.quat[i], qx = m.quat[n + i], qy = m.quat[2 * n + i], qz = m.quat[3 * n + i];
    const double qn = sqrt(qw * qw + qx * qx + qy * qy + qz * qz);
    const double iq = qn > 0.0 ? 1.0 / qn : 0.0;
    qw *= iq; qx *= iq; qy *= iq; qz *= iq;
    double Rq[9];
    Rq[0] = 1.0 - 2.0 * (qy * qy + qz * qz);
    Rq[1] = 2.0 * (qx * qy - qw * qz);
    Rq[2] = 2.0 * (qx * qz + qw * qy);
    Rq[3] = 2.0 * (qx * qy + qw * qz);
    Rq[4] = 1.0 - 2.0 * (qx * qx + qz * qz);
    Rq[5] = 2.0 * (qy * qz - qw * qx);
    Rq[6] = 2.0 * (qx * qz - qw * qy);
    Rq[7] = 2.0 * (qy * qz + qw * qx);
    Rq[8] = 1.0 - 2.0 * (qx * qx + qy * qy);
    double M[9], S[9];
#pragma unroll
    for (int r = 0; r < 3; ++r)
#pragma unroll
      for (int c = 0; c < 3; ++c) M[3 * r + c] = Rq[3 * r + c] * s[c];
#pragma unroll
    for (int r = 0; r < 3; ++r)
#pragma unroll
      for (int c = 0; c < 3; ++c)
        S[3 * r + c] = M[3 * r] * M[3 * c] + M[3 * r + 1] * M[3 * c + 1] + M[3 * r + 2] * M[3 * c + 2];
    double dM[9] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
    for (int jv = 0; jv < job.n_views; ++jv) {
      const ViewD& V = views[job.view[jv]];
      const uint32_t r = V.rec_off + (uint32_t)i;
      const float* rec = records + (size_t)r * kRecordFloats;
      // the record's flags and pair range, read together
      const uint32_t kept = __float_as_uint(rec[11]), clamp_bits = __float_as_uint(rec[10]);
      uint32_t e0 = offsets[r], e1 = offsets[r + 1];
      asm volatile("" : "+v"(e0), "+v"(e1));  // both loads issued before the test, not sunk below it
      e1 = min(e1, K);
      if (kept == 0u) continue;  // culled in this view
      double g[9];
      record_grad(e0, e1, g_pair, alive, cap, g, wmax);
      go += g[5] * (double)V.layer_op[layer];  // the record holds o times the view's factor
      {
        // density-control statistic: gradient of the projected centre in
        // normalised device coordinates (du / dx_ndc = W / 2)
        const double gx = g[0] * (0.5 * (double)V.W), gy = g[1] * (0.5 * (double)V.H);
        dgs += sqrt(gx * gx + gy * gy);
        dgc += 1.0;
      }
#pragma unroll
      for (int ch = 0; ch < 3; ++ch) g_col[(size_t)r * 3 + ch] = ((clamp_bits >> ch) & 1u) ? 0.f : (float)g[6 + ch];
      double W[9];
#pragma unroll
      for (int k = 0; k < 9; ++k) W[k] = V.R[k];
      const double fx = V.fx, fy = V.fy;
      const double tx = W[0] * mx + W[1] * my + W[2] * mz + (double)V.t[0];
      const double ty = W[3] * mx + W[4] * my + W[5] * mz + (double)V.t[1];
      const double tz = W[6] * mx + W[7] * my + W[8] * mz + (double)V.t[2];
      // ---- guard band: the clamp decision and the clamped slope exactly as
      // the projection took them (float, same operation order)
      bool xcl, ycl;
      float xr_f, yr_f;
      {
        const float* Wf = V.R;
        const float fmx = m.mean[i], fmy = m.mean[n + i], fmz = m.mean[2 * n + i];
        const float ftx = __fadd_rn(__fadd_rn(__fadd_rn(__fmul_rn(Wf[0], fmx), __fmul_rn(Wf[1], fmy)),
                                              __fmul_rn(Wf[2], fmz)), V.t[0]);
        const float fty = __fadd_rn(__fadd_rn(__fadd_rn(__fmul_rn(Wf[3], fmx), __fmul_rn(Wf[4], fmy)),
                                              __fmul_rn(Wf[5], fmz)), V.t[1]);
        const float ftz = __fadd_rn(__fadd_rn(__fadd_rn(__fmul_rn(Wf[6], fmx), __fmul_rn(Wf[7], fmy)),
                                              __fmul_rn(Wf[8], fmz)), V.t[2]);
        const float lim_x = __fdiv_rn(__fmul_rn(V.guard, fmaxf(V.cx, __fsub_rn((float)V.W, V.cx))), V.fx);
        const float lim_y = __fdiv_rn(__fmul_rn(V.guard, fmaxf(V.cy, __fsub_rn((float)V.H, V.cy))), V.fy);
        const float x0 = __fdiv_rn(ftx, ftz), y0 = __fdiv_rn(fty, ftz);
        xcl = (x0 < -lim_x) || (x0 > lim_x);
        ycl = (y0 < -lim_y) || (y0 > lim_y);
        xr_f = fminf(fmaxf(x0, -lim_x), lim_x);
        yr_f = fminf(fmaxf(y0, -lim_y), lim_y);
      }
      const double xr = xcl ? (double)xr_f : tx / tz;
      const double yr = ycl ? (double)yr_f : ty / tz;
      const double itz = 1.0 / tz, itz2 = itz * itz, itz3 = itz2 * itz;
      const double J00 = fx * itz, J02 = -fx * xr * itz;
      const double J11 = fy * itz, J12 = -fy * yr * itz;
      double Tm[6];
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        Tm[c] = J00 * W[c] + J02 * W[6 + c];
        Tm[3 + c] = J11 * W[3 + c] + J12 * W[6 + c];
      }
      double ST0[3], ST1[3];
#pragma unroll
      for (int r2 = 0; r2 < 3; ++r2) {
        ST0[r2] = S[3 * r2] * Tm[0] + S[3 * r2 + 1] * Tm[1] + S[3 * r2 + 2] * Tm[2];
        ST1[r2] = S[3 * r2] * Tm[3] + S[3 * r2 + 1] * Tm[4] + S[3 * r2 + 2] * Tm[5];
      }
      const double a = Tm[0] * ST0[0] + Tm[1] * ST0[1] + Tm[2] * ST0[2] + (double)kKappa;
      const double b = Tm[0] * ST1[0] + Tm[1] * ST1[1] + Tm[2] * ST1[2];
      const double c = Tm[3] * ST1[0] + Tm[4] * ST1[1] + Tm[5] * ST1[2] + (double)kKappa;
      const double det = a * c - b * b;
      const double id2 = 1.0 / (det * det);
      const double dca = g[2], dcb = g[3], dcc = g[4];
      const double da = (-c * c * dca + b * c * dcb - b * b * dcc) * id2;
      const double db = (2.0 * b * c * dca - (a * c + b * b) * dcb + 2.0 * a * b * dcc) * id2;
      const double dc = (-b * b * dca + a * b * dcb - a * a * dcc) * id2;
      // ---- Sigma' = T Sigma T^T
      double dT0[3], dT1[3];
#pragma unroll
      for (int r2 = 0; r2 < 3; ++r2) {
        dT0[r2] = 2.0 * da * ST0[r2] + db * ST1[r2];
        dT1[r2] = db * ST0[r2] + 2.0 * dc * ST1[r2];
      }
      // dSigma (symmetrised) and dM = (dS + dS^T) M
      double dS[9];
#pragma unroll
      for (int r2 = 0; r2 < 3; ++r2)
#pragma unroll
        for (int q2 = 0; q2 < 3; ++q2)
          dS[3 * r2 + q2] = da * Tm[r2] * Tm[q2] + db * Tm[r2] * Tm[3 + q2] + dc * Tm[3 + r2] * Tm[3 + q2];
#pragma unroll
      for (int r2 = 0; r2 < 3; ++r2)
#pragma unroll
        for (int k = 0; k < 3; ++k) {
          double acc = 0.0;
#pragma unroll
          for (int j = 0; j < 3; ++j) acc += (dS[3 * r2 + j] + dS[3 * j + r2]) * M[3 * j + k];
          dM[3 * r2 + k] += acc;
        }
      // ---- Jacobian and projected centre -> camera-space centre
      double dJ00 = 0.0, dJ02 = 0.0, dJ11 = 0.0, dJ12 = 0.0;
#pragma unroll
      for (int r2 = 0; r2 < 3; ++r2) {
        dJ00 += dT0[r2] * W[r2];
        dJ02 += dT0[r2] * W[6 + r2];
        dJ11 += dT1[r2] * W[3 + r2];
        dJ12 += dT1[r2] * W[6 + r2];
      }
      double dtx = 0.0, dty = 0.0, dtz = 0.0;
      dtz += -(dJ00 * fx + dJ11 * fy) * itz2;
      if (!xcl) {
        dtx += -dJ02 * fx * itz2;
        dtz += 2.0 * dJ02 * fx * tx * itz3;
      } else {
        dtz += dJ02 * fx * xr * itz2;
      }
      if (!ycl) {
        dty += -dJ12 * fy * itz2;
        dtz += 2.0 * dJ12 * fy * ty * itz3;
      } else {
        dtz += dJ12 * fy * yr * itz2;
      }
      dtx += g[0] * fx * itz;
      dtz += -g[0] * fx * tx * itz2;
      dty += g[1] * fy * itz;
      dtz += -g[1] * fy * ty * itz2;
      gm[0] += W[0] * dtx + W[3] * dty + W[6] * dtz;
      gm[1] += W[1] * dtx + W[4] * dty + W[7] * dtz;
      gm[2] += W[2] * dtx + W[5] * dty + W[8] * dtz;
    }
    // ---- M = Rq diag(s) -> scale, rotation -> quaternion
    double dR[9];
#pragma unroll
    for (int r = 0; r < 3; ++r)
#pragma unroll
      for (int k = 0; k < 3; ++k) {
        gs[k] += dM[3 * r + k] * Rq[3 * r + k];
        dR[3 * r + k] = dM[3 * r + k] * s[k];
      }
    double dq[4];
    dq[0] = 2.0 * (-qz * dR[1] + qy * dR[2] + qz * dR[3] - qx * dR[5] - qy * dR[6] + qx * dR[7]);
    dq[1] = 2.0 * (qy * dR[1] + qz * dR[2] + qy * dR[3] - 2.0 * qx * dR[4] - qw * dR[5] + qz * dR[6] +
                   qw * dR[7] - 2.0 * qx * dR[8]);
    dq[2] = 2.0 * (-2.0 * qy * dR[0] + qx * dR[1] + qw * dR[2] + qx * dR[3] + qz * dR[5] - qw * dR[6] +
                   qz * dR[7] - 2.0 * qy * dR[8]);
    dq[3] = 2.0 * (-2.0 * qz * dR[0] - qw * dR[1] + qx * dR[2] + qw * dR[3] - 2.0 * qz * dR[4] +
                   qy * dR[5] + qx * dR[6] + qy * dR[7]);
    const double qd = qw * dq[0] + qx * dq[1] + qy * dq[2] + qz * dq[3];
    gq[0] = (dq[0] - qw * qd) * iq;
    gq[1] = (dq[1] - qx * qd) * iq;
    gq[2] = (dq[2] - qy * qd) * iq;
    gq[3] = (dq[3] - qz * qd) * iq;
    if (m.raw) {  // chain rule of the activations: d exp = exp, d logistic = o (1 - o)
#pragma unroll
      for (int k = 0; k < 3; ++k) gs[k] *= s[k];
      const double o = act_opacity(m.opacity[i], 1);
      go *= o * (1.0 - o);
    }
  }
#pragma unroll
  for (int k = 0; k < 3; ++k) g_mean[(size_t)k * n + i] = (float)gm[k];
#pragma unroll
  for (int k = 0; k < 3; ++k) g_scale[(size_t)k * n + i] = (float)gs[k];
#pragma unroll
  for (int k = 0; k < 4; ++k) g_quat[(size_t)k * n + i] = (float)gq[k];
  g_opacity[i] = (float)go;
  if (max_contrib) max_contrib[i] = fmaxf(max_contrib[i], wmax);
  if (train && dens_grad) {
    dens_grad[i] += (float)dgs;
    dens_cnt[i] += (float)dgc;
  }
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
  double gm[3] = {0.0, 0.0, 0.0};
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
    // the SH expansion with the drgb-weighted coefficients (below)
#pragma unroll
    for (int k = 0; k < NC; ++k)
#pragma unroll
      for (int ch = 0; ch < 3; ++ch) gsh[k * 3 + ch] += Y[k] * drgb[ch];
    if (D > 0) {
      // the tangential part of the direction gradient, in double (a
      // difference of nearly parallel vectors when the gradient points along
      // the view direction)
      double ed[16];
#pragma unroll
      for (int k = 0; k < NC; ++k) {
        ed[k] = 0.0;
#pragma unroll
        for (int ch = 0; ch < 3; ++ch) ed[k] += (double)m.sh[(size_t)(k * 3 + ch) * n + i] * (double)drgb[ch];
      }
      const double dl64 = sqrt((double)ddx * ddx + (double)ddy * ddy + (double)ddz * ddz);
      const double ux = ddx / dl64, uy = ddy / dl64, uz = ddz / dl64;
      double ddir[3];
      sh_dir_grad<D>(ux, uy, uz, ed, ddir[0], ddir[1], ddir[2]);
      const double dd = ux * ddir[0] + uy * ddir[1] + uz * ddir[2];
      gm[0] += (ddir[0] - ux * dd) / dl64;
      gm[1] += (ddir[1] - uy * dd) / dl64;
      gm[2] += (ddir[2] - uz * dd) / dl64;
    }
  }
  float pm = 0.f;
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    const float v = (float)((double)g_mean[(size_t)k * n + i] + gm[k]);
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
                              float* activity, float* dens_grad, float* dens_cnt, hipStream_t s) {
  if (job.m.n <= 0) return hipSuccess;
  const dim3 grid(div_up((uint32_t)job.m.n, 256u)), block(256);
  hipLaunchKernelGGL(k_project_bwd_geom, grid, block, 0, s, job, views_dev, records, offsets, g_pair, alive,
                     pair_capacity, counters, trainable, g_mean, g_scale, g_quat, g_opacity, g_col, max_contrib,
                     dens_grad, dens_cnt);
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
