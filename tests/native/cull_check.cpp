// CPU check of gsr::band_blocks (paper_2410_16978_amd/csrc/cull.hpp), the
// block culling of the blend kernels: over random splats (thin, round,
// rotated, large, partly or fully off the band) every 4 x 4 block whose
// pixel-centre rectangle the cut-off ellipse {q <= K} meets must be flagged,
// and a flagged block must come within 0.03 px of the ellipse (the
// widening: 1e-3 px plus 1e-5 of the coordinate).  The
// reference is the exact minimum of q over the rectangle, in double: q is a
// convex quadratic, so outside the rectangle's interior its minimum lies on
// an edge, at the clamped one-dimensional minimiser.
// Prints "misses loose checked" and exits non-zero on a miss or a loose bit.
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <random>

#include "cull.hpp"

static double q_at(double a, double b, double c, double X, double Y) { return a * X * X + 2 * b * X * Y + c * Y * Y; }

// min of q over [X0, X1] x [Y0, Y1]
static double min_q_rect(double a, double b, double c, double X0, double X1, double Y0, double Y1) {
  if (X0 <= 0 && 0 <= X1 && Y0 <= 0 && 0 <= Y1) return 0.0;
  double m = INFINITY;
  for (double X : {X0, X1}) {  // vertical edges: minimise over Y
    double Y = std::fmin(std::fmax(-b * X / c, Y0), Y1);
    m = std::fmin(m, q_at(a, b, c, X, Y));
  }
  for (double Y : {Y0, Y1}) {  // horizontal edges: minimise over X
    double X = std::fmin(std::fmax(-b * Y / a, X0), X1);
    m = std::fmin(m, q_at(a, b, c, X, Y));
  }
  return m;
}

int main(int argc, char** argv) {
  const int n = argc > 1 ? std::atoi(argv[1]) : 200000;
  std::mt19937_64 rng(1234);
  std::uniform_real_distribution<double> U(0.0, 1.0);
  long misses = 0, loose = 0, checked = 0, flagged = 0;
  for (int it = 0; it < n; ++it) {
    // covariance eigenvalues 0.3 + 10^[-1, 4.5] px^2 (the projection adds
    // 0.3 px^2), random angle; the conic is its inverse, rounded to float
    const double l1 = 0.3 + std::pow(10.0, -1.0 + 5.5 * U(rng));
    const double l2 = 0.3 + std::pow(10.0, -1.0 + 5.5 * U(rng));
    const double th = 3.14159265358979 * U(rng);
    const double cs = std::cos(th), sn = std::sin(th);
    const double sxx = l1 * cs * cs + l2 * sn * sn, syy = l1 * sn * sn + l2 * cs * cs, sxy = (l1 - l2) * cs * sn;
    const double det = sxx * syy - sxy * sxy;
    const float a = (float)(syy / det), b = (float)(-sxy / det), c = (float)(sxx / det);
    const double o = std::pow(10.0, -2.6 * U(rng));  // opacity 0.0025 .. 1
    const float K = std::fmin(11.09375f, 2.f * std::log(255.f * (float)o)) * 1.01f + 0.05f;
    // tile origin and a centre up to 3 radii away from the tile
    const double R = 3.0 * std::sqrt(std::fmax(l1, l2));
    const float tx0 = (float)(16 * (int)(U(rng) * 100)) + 0.5f, ty0 = (float)(16 * (int)(U(rng) * 100)) + 0.5f;
    const float u = (float)(tx0 + 8 + (2 * U(rng) - 1) * (R + 12)), v = (float)(ty0 + 8 + (2 * U(rng) - 1) * (R + 12));
    for (int r = 0; r < 4; ++r) {
      const float y0 = ty0 + 4.f * (float)r;
      const uint32_t bits = gsr::band_blocks(u, v, a, b, c, K, tx0, y0);
      for (int i = 0; i < 4; ++i) {
        const double X0 = (double)tx0 + 4.0 * i - u, Y0 = (double)y0 - v;
        const double mq = K > 0.05f ? min_q_rect(a, b, c, X0, X0 + 3.0, Y0, Y0 + 3.0) : INFINITY;
        const double mq_wide = K > 0.05f ? min_q_rect(a, b, c, X0 - 0.03, X0 + 3.03, Y0 - 0.03, Y0 + 3.03) : INFINITY;
        const bool set = (bits >> i) & 1u;
        ++checked;
        flagged += set;
        if (mq <= (double)K * (1.0 - 1e-5) && !set) {
          if (misses < 10)
            std::printf("miss: l %.3g %.3g th %.3f o %.3g K %.4f u %.3f v %.3f tile %.1f %.1f row %d blk %d min q %.6g\n",
                        l1, l2, th, o, K, u, v, tx0, ty0, r, i, mq);
          ++misses;
        }
        if (set && !(mq_wide <= (double)K * (1.0 + 1e-3))) {
          if (loose < 10)
            std::printf("loose: l %.3g %.3g th %.3f K %.4f row %d blk %d min q %.6g\n", l1, l2, th, K, r, i, mq_wide);
          ++loose;
        }
      }
    }
  }
  std::printf("%ld %ld %ld %ld\n", misses, loose, checked, flagged);
  return (misses || loose) ? 1 : 0;
}
