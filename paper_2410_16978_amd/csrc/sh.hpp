// Real spherical harmonics (degree <= 3) with the Condon-Shortley phase, in
// Cartesian form on the unit sphere; Y[k] with k = l^2 + l + m.  Constants are
// the exact values rounded once to float.
#pragma once

namespace gsr {

constexpr float kShC0 = (float)0.28209479177387814347;   // 1 / (2 sqrt(pi))
constexpr float kShC1 = (float)0.48860251190291992159;   // sqrt(3 / (4 pi))
constexpr float kShC2a = (float)1.09254843059207907054;  // sqrt(15 / pi) / 2
constexpr float kShC2b = (float)0.31539156525252000603;  // sqrt(5 / pi) / 4
constexpr float kShC2c = (float)0.54627421529603953527;  // sqrt(15 / pi) / 4
constexpr float kShC3a = (float)0.59004358992664351035;  // sqrt(35 / (2 pi)) / 4
constexpr float kShC3b = (float)2.89061144264055405539;  // sqrt(105 / pi) / 2
constexpr float kShC3c = (float)0.45704579946446573616;  // sqrt(21 / (2 pi)) / 4
constexpr float kShC3d = (float)0.37317633259011539141;  // sqrt(7 / pi) / 4
constexpr float kShC3e = (float)1.44530572132027702769;  // sqrt(105 / pi) / 4

template <int D>
__device__ __forceinline__ void sh_basis(float x, float y, float z, float* Y) {
  Y[0] = kShC0;
  if (D >= 1) {
    Y[1] = (-kShC1) * y;
    Y[2] = kShC1 * z;
    Y[3] = (-kShC1) * x;
  }
  if (D >= 2) {
    const float xx = x * x, yy = y * y, zz = z * z;
    const float xy = x * y, yz = y * z, xz = x * z;
    Y[4] = kShC2a * xy;
    Y[5] = (-kShC2a) * yz;
    Y[6] = kShC2b * ((2.0f * zz - xx) - yy);
    Y[7] = (-kShC2a) * xz;
    Y[8] = kShC2c * (xx - yy);
    if (D >= 3) {
      Y[9] = (-kShC3a) * (y * (3.0f * xx - yy));
      Y[10] = kShC3b * (xy * z);
      Y[11] = (-kShC3c) * (y * ((4.0f * zz - xx) - yy));
      Y[12] = kShC3d * (z * ((2.0f * zz - 3.0f * xx) - 3.0f * yy));
      Y[13] = (-kShC3c) * (x * ((4.0f * zz - xx) - yy));
      Y[14] = kShC3e * (z * (xx - yy));
      Y[15] = (-kShC3a) * (x * (xx - 3.0f * yy));
    }
  }
}

// d/d(x, y, z) of sum_k c_k Y_k for the coefficients c (float or double).
template <int D, typename T>
__device__ __forceinline__ void sh_dir_grad(T x, T y, T z, const T* c, T& gx, T& gy, T& gz) {
  gx = T(0);
  gy = T(0);
  gz = T(0);
  if (D >= 1) {
    gy += -T(kShC1) * c[1];
    gz += T(kShC1) * c[2];
    gx += -T(kShC1) * c[3];
  }
  if (D >= 2) {
    gx += T(kShC2a) * y * c[4];
    gy += T(kShC2a) * x * c[4];
    gy += -T(kShC2a) * z * c[5];
    gz += -T(kShC2a) * y * c[5];
    gx += -T(2) * T(kShC2b) * x * c[6];
    gy += -T(2) * T(kShC2b) * y * c[6];
    gz += T(4) * T(kShC2b) * z * c[6];
    gx += -T(kShC2a) * z * c[7];
    gz += -T(kShC2a) * x * c[7];
    gx += T(2) * T(kShC2c) * x * c[8];
    gy += -T(2) * T(kShC2c) * y * c[8];
    if (D >= 3) {
      const T xx = x * x, yy = y * y, zz = z * z;
      gx += -T(6) * T(kShC3a) * x * y * c[9];
      gy += -T(kShC3a) * (T(3) * xx - T(3) * yy) * c[9];
      gx += T(kShC3b) * y * z * c[10];
      gy += T(kShC3b) * x * z * c[10];
      gz += T(kShC3b) * x * y * c[10];
      gx += T(2) * T(kShC3c) * x * y * c[11];
      gy += -T(kShC3c) * (T(4) * zz - xx - T(3) * yy) * c[11];
      gz += -T(8) * T(kShC3c) * y * z * c[11];
      gx += -T(6) * T(kShC3d) * x * z * c[12];
      gy += -T(6) * T(kShC3d) * y * z * c[12];
      gz += T(kShC3d) * (T(6) * zz - T(3) * xx - T(3) * yy) * c[12];
      gx += -T(kShC3c) * (T(4) * zz - T(3) * xx - yy) * c[13];
      gy += T(2) * T(kShC3c) * x * y * c[13];
      gz += -T(8) * T(kShC3c) * x * z * c[13];
      gx += T(2) * T(kShC3e) * x * z * c[14];
      gy += -T(2) * T(kShC3e) * y * z * c[14];
      gz += T(kShC3e) * (xx - yy) * c[14];
      gx += -T(kShC3a) * (T(3) * xx - T(3) * yy) * c[15];
      gy += T(6) * T(kShC3a) * x * y * c[15];
    }
  }
}

}  // namespace gsr
