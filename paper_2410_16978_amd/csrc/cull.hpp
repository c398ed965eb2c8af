// Which 4 x 4-pixel blocks of a tile a splat can reach.
//
// A splat reaches a pixel only where o exp(-q/2) >= 1/255 (the skip rule of
// the per-pixel blend), q = a X^2 + 2 b X Y + c Y^2 at the offset (X, Y) of
// the pixel centre from the splat centre, i.e. inside the ellipse q <= K with
// K the splat's cut-off (2 ln(255 o) plus a margin, see reach_cutoff in
// blend.hip).  The blend kernels list, per wave, only the pairs whose
// ellipse meets the wave's pixel block; this file computes those memberships
// for one row of four blocks at a time from the ellipse's x-extent over the
// row's band of pixel-centre rows:
//   for fixed Y, q <= K  <=>  X in [(-b Y - s) / a, (-b Y + s) / a],
//   s = sqrt(a K - det Y^2), det = a c - b^2 > 0,
// and the right end is a concave function of Y whose maximum over the band
// is at the band point nearest the ellipse's rightmost point
// (X_r, Y_r) = (sqrt(K c / det), -b X_r / c); the left end likewise at the
// band point nearest (-X_r, -Y_r).  The band meets the ellipse at all only
// if it overlaps |Y| <= sqrt(a K / det).
//
// The result must never drop a block the ellipse meets: the interval is
// widened by 1e-3 px plus 1e-5 of its end's magnitude and the band test by
// 1e-4 of the half-height plus 1e-3 px, while the cut-off itself sits a
// 1 % + 0.05 margin above the exact threshold (about 0.5 % of the radius),
// far above the rounding of this computation; anything not finite keeps
// every block.  Host-compilable: the same function is
// exercised on the CPU by the tests.
#pragma once
#include <cstdint>

#if defined(__HIPCC__)
#define GSR_HD __host__ __device__
#else
#define GSR_HD
#include <cmath>
#endif

namespace gsr {

GSR_HD inline float cull_sqrt(float x) {
#if defined(__HIP_DEVICE_COMPILE__)
  return __builtin_amdgcn_sqrtf(x);
#else
  return std::sqrt(x);
#endif
}

GSR_HD inline float cull_rcp(float x) {
#if defined(__HIP_DEVICE_COMPILE__)
  return __builtin_amdgcn_rcpf(x);
#else
  return 1.f / x;
#endif
}

// Bits i = 0..3 of the blocks whose pixel centres span x in [x0 + 4 i,
// x0 + 4 i + 3], y in [y0, y0 + 3] that the ellipse {q <= K} around (u, v)
// with conic (a, b, c) meets.  K <= 0.05 reaches nothing.
GSR_HD inline uint32_t band_blocks(float u, float v, float a, float b, float c, float K, float x0, float y0) {
  if (!(K > 0.05f)) return 0u;
  // a c - b^2 in double (the float products are exact there): for a thin
  // ellipse the difference is far smaller than its terms
  const float det = (float)((double)a * (double)c - (double)b * (double)b);
  if (!(det > 0.f) || !(a > 0.f) || !(c > 0.f)) return 0xFu;
  const float inv_det = cull_rcp(det);
  const float Y0 = y0 - v, Y1 = Y0 + 3.f;
  const float aK = a * K;
  const float Ym = cull_sqrt(aK * inv_det) * 1.0001f + 1e-3f;
  if (Y0 > Ym || Y1 < -Ym) return 0u;
  const float Xr = cull_sqrt(K * c * inv_det);
  const float Yr = -b * Xr * cull_rcp(c);
  const float ya = fminf(fmaxf(Yr, Y0), Y1), yb = fminf(fmaxf(-Yr, Y0), Y1);
  const float ra = cull_sqrt(fmaxf(aK - det * ya * ya, 0.f));
  const float rb = cull_sqrt(fmaxf(aK - det * yb * yb, 0.f));
  const float inv_a = cull_rcp(a);
  float xmax = u + (ra - b * ya) * inv_a;
  float xmin = u - (rb + b * yb) * inv_a;
  xmax += 1e-3f + 1e-5f * fabsf(xmax);
  xmin -= 1e-3f + 1e-5f * fabsf(xmin);
  if (!(xmin <= xmax)) return 0xFu;  // not finite
  uint32_t bits = 0u;
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const float lo = x0 + 4.f * (float)i;
    bits |= (lo <= xmax && lo + 3.f >= xmin) ? (1u << i) : 0u;
  }
  return bits;
}

}  // namespace gsr
