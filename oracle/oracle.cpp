// CPU oracle for the layered Gaussian-splat tile rasterizer.
//
// TEST INFRASTRUCTURE ONLY: linked by nothing in the product path; called by
// the tests, the smoke check and the benchmark's CPU-baseline leg.  Shares no
// code with the GPU path.
//
// Built with -O2 -ffp-contract=off and no fast-math, so that every float
// expression below is evaluated as written (each + - * / sqrt correctly
// rounded, in the order of the parentheses).
//
// What is computed (readings of the paper where it is silent are stated in the
// design notes and in oracle.h):
//  * per (view, Gaussian): the paper's layer visibility and cutting (Sec. 1,
//    Sec. 3.3 "only active layers", Sec. 5: the cut edge depends on the splat
//    centres) as a layer-mask bit test and centre-versus-plane tests; the
//    EWA projection of the 3D covariance, Sigma' = J W Sigma W^T J^T
//    (Zwicker et al., the splatting the paper names in Sec. 2.2.1); a
//    view-dependent spherical-harmonic colour; a conservative tile rectangle;
//  * per view: (tile, depth) keys in emission order and a stable sort;
//  * per pixel: front-to-back alpha compositing over the depth-sorted splats
//    ("analogous to Kerbl et al.", Sec. 3.3), with the 0.99 alpha clamp, the
//    1/255 cutoff and the 1e-4 transmittance stop;
//  * the exact gradient of the composited image with respect to the
//    activated Gaussian parameters, with frozen (non-trainable) layers
//    receiving none (Sec. 3.2), plus the per-Gaussian activity of
//    Sec. 3.2.2 (2|p| + 0.1|c| + 0.1|s| with p, c, s the position, colour and
//    scale gradient norms).
//
// "parity unpinned": the activity magnitudes (which norm the paper means) -
// see the design notes; everything else is pinned by the CPU tests.
#include "oracle.h"

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <vector>
#ifdef _OPENMP
#include <omp.h>
#endif

namespace {

template <typename T> struct Model {
  int n, D;
  const T *mean, *scale, *quat, *opacity, *sh;
  const uint8_t* layer;
  const T* filter3d = nullptr;  // Mip-Splatting 3D filter variances, or null
};

template <typename T> struct Consts {
  static T alpha_max() { return T(0.99); }
  static T alpha_min() { return T(1.0) / T(255.0); }
  static T t_stop() { return T(1e-4); }
  static T kappa() { return T(0.3); }
  static T qmax() { return T(11.09375); }
};

// Real spherical harmonics with the Condon-Shortley phase, Cartesian form on
// the unit sphere.  Constants are evaluated in double and rounded once.
template <typename T> struct SH {
  T c0, c1, c2a, c2b, c2c, c3a, c3b, c3c, c3d, c3e;
  SH() {
    const double pi = 3.14159265358979323846;
    c0 = T(0.5 / std::sqrt(pi));
    c1 = T(std::sqrt(3.0 / (4.0 * pi)));
    c2a = T(0.5 * std::sqrt(15.0 / pi));
    c2b = T(0.25 * std::sqrt(5.0 / pi));
    c2c = T(0.25 * std::sqrt(15.0 / pi));
    c3a = T(0.25 * std::sqrt(35.0 / (2.0 * pi)));
    c3b = T(0.5 * std::sqrt(105.0 / pi));
    c3c = T(0.25 * std::sqrt(21.0 / (2.0 * pi)));
    c3d = T(0.25 * std::sqrt(7.0 / pi));
    c3e = T(0.25 * std::sqrt(105.0 / pi));
  }
  // Y[k] for k = l^2 + l + m, l <= 3.
  void basis(T x, T y, T z, T* Y) const {
    T xx = x * x, yy = y * y, zz = z * z;
    T xy = x * y, yz = y * z, xz = x * z;
    Y[0] = c0;
    Y[1] = (-c1) * y;
    Y[2] = c1 * z;
    Y[3] = (-c1) * x;
    Y[4] = c2a * xy;
    Y[5] = (-c2a) * yz;
    Y[6] = c2b * ((T(2) * zz - xx) - yy);
    Y[7] = (-c2a) * xz;
    Y[8] = c2c * (xx - yy);
    Y[9] = (-c3a) * (y * (T(3) * xx - yy));
    Y[10] = c3b * (xy * z);
    Y[11] = (-c3c) * (y * ((T(4) * zz - xx) - yy));
    Y[12] = c3d * (z * ((T(2) * zz - T(3) * xx) - T(3) * yy));
    Y[13] = (-c3c) * (x * ((T(4) * zz - xx) - yy));
    Y[14] = c3e * (z * (xx - yy));
    Y[15] = (-c3a) * (x * (xx - T(3) * yy));
  }
  // Gradient of each polynomial with respect to (x, y, z).
  void grad(T x, T y, T z, T (*G)[3]) const {
    for (int k = 0; k < 16; ++k) G[k][0] = G[k][1] = G[k][2] = T(0);
    G[1][1] = -c1;
    G[2][2] = c1;
    G[3][0] = -c1;
    G[4][0] = c2a * y; G[4][1] = c2a * x;
    G[5][1] = -c2a * z; G[5][2] = -c2a * y;
    G[6][0] = T(-2) * c2b * x; G[6][1] = T(-2) * c2b * y; G[6][2] = T(4) * c2b * z;
    G[7][0] = -c2a * z; G[7][2] = -c2a * x;
    G[8][0] = T(2) * c2c * x; G[8][1] = T(-2) * c2c * y;
    G[9][0] = T(-6) * c3a * x * y; G[9][1] = -c3a * (T(3) * x * x - T(3) * y * y);
    G[10][0] = c3b * y * z; G[10][1] = c3b * x * z; G[10][2] = c3b * x * y;
    G[11][0] = T(2) * c3c * x * y;
    G[11][1] = -c3c * (T(4) * z * z - x * x - T(3) * y * y);
    G[11][2] = T(-8) * c3c * y * z;
    G[12][0] = T(-6) * c3d * x * z; G[12][1] = T(-6) * c3d * y * z;
    G[12][2] = c3d * (T(6) * z * z - T(3) * x * x - T(3) * y * y);
    G[13][0] = -c3c * (T(4) * z * z - T(3) * x * x - y * y);
    G[13][1] = T(2) * c3c * x * y;
    G[13][2] = T(-8) * c3c * x * z;
    G[14][0] = T(2) * c3e * x * z; G[14][1] = T(-2) * c3e * y * z; G[14][2] = c3e * (x * x - y * y);
    G[15][0] = -c3a * (T(3) * x * x - T(3) * y * y); G[15][1] = T(6) * c3a * x * y;
  }
};

template <typename T> struct Cam {
  T R[9], t[3], fx, fy, cx, cy, znear, guard;
  int W, H;
  explicit Cam(const oc_camera& c) {
    for (int i = 0; i < 9; ++i) R[i] = T(c.R[i]);
    for (int i = 0; i < 3; ++i) t[i] = T(c.t[i]);
    fx = T(c.fx); fy = T(c.fy); cx = T(c.cx); cy = T(c.cy);
    znear = T(c.znear); guard = T(c.guard);
    W = c.width; H = c.height;
  }
};

// Everything the forward derives for one (view, Gaussian); the backward
// recomputes it from the same inputs.
template <typename T> struct Proj {
  bool valid = false;
  // camera-space centre, Jacobian clamp state
  T tx, ty, tz, xr, yr;
  bool x_clamped, y_clamped;
  // rotation and covariance
  T qn, qh[4], Rq[9], M[9], S[9];
  T J00, J02, J11, J12, Tm[6];
  T a, b, c, det;
  // record
  T u, v, ca, cb, cc, op, rgb[3];
  T fade = T(1);  // the view's opacity factor of the Gaussian's layer
  uint32_t clamp = 0;
  int rect[4] = {0, 0, 0, 0};
  uint32_t ntiles = 0;
  // colour direction
  T dir[3], dlen, Y[16];
};

template <typename T>
Proj<T> project_one(const Model<T>& m, int i, const Cam<T>& cam, const oc_view& vs, int tile,
                    const SH<T>& sh) {
  Proj<T> p;
  const int n = m.n;
  const unsigned layer = m.layer[i];
  // Layer visibility: the Gaussian is drawn only if its layer is active.
  if (layer >= 32u || !((vs.layer_mask >> layer) & 1u)) return p;
  const T mx = m.mean[i], my = m.mean[n + i], mz = m.mean[2 * n + i];
  // Cutting: a plane removes the Gaussians of its layers whose centre lies on
  // its negative side.
  for (int k = 0; k < vs.n_clip; ++k) {
    const oc_clip& cp = vs.clip[k];
    if (!((cp.layer_bits >> layer) & 1u)) continue;
    T s = ((T(cp.n[0]) * mx + T(cp.n[1]) * my) + T(cp.n[2]) * mz) + T(cp.d);
    if (s < T(0)) return p;
  }
  const T* W = cam.R;
  p.tx = ((W[0] * mx + W[1] * my) + W[2] * mz) + cam.t[0];
  p.ty = ((W[3] * mx + W[4] * my) + W[5] * mz) + cam.t[1];
  p.tz = ((W[6] * mx + W[7] * my) + W[8] * mz) + cam.t[2];
  if (!(p.tz > cam.znear)) return p;
  p.op = m.opacity[i];
  // The view's opacity factor of the layer scales the opacity it is drawn
  // with; a product below the blend's skip threshold draws nothing.
  if (vs.layer_fade) {
    p.fade = T(vs.layer_opacity[layer]);
    p.op = p.op * p.fade;
  }
  if (p.op < Consts<T>::alpha_min()) return p;
  // Unit quaternion (w, x, y, z) and its rotation matrix.
  T qw = m.quat[i], qx = m.quat[n + i], qy = m.quat[2 * n + i], qz = m.quat[3 * n + i];
  p.qn = std::sqrt(((qw * qw + qx * qx) + qy * qy) + qz * qz);
  if (!(p.qn > T(0))) return p;
  qw = qw / p.qn; qx = qx / p.qn; qy = qy / p.qn; qz = qz / p.qn;
  p.qh[0] = qw; p.qh[1] = qx; p.qh[2] = qy; p.qh[3] = qz;
  T* Rq = p.Rq;
  Rq[0] = T(1) - T(2) * (qy * qy + qz * qz);
  Rq[1] = T(2) * (qx * qy - qw * qz);
  Rq[2] = T(2) * (qx * qz + qw * qy);
  Rq[3] = T(2) * (qx * qy + qw * qz);
  Rq[4] = T(1) - T(2) * (qx * qx + qz * qz);
  Rq[5] = T(2) * (qy * qz - qw * qx);
  Rq[6] = T(2) * (qx * qz - qw * qy);
  Rq[7] = T(2) * (qy * qz + qw * qx);
  Rq[8] = T(1) - T(2) * (qx * qx + qy * qy);
  // Sigma = M M^T with M = Rq diag(s).
  T s0 = m.scale[i], s1 = m.scale[n + i], s2 = m.scale[2 * n + i];
  if (m.filter3d) {
    // Mip-Splatting's 3D filter: convolving with an isotropic Gaussian of
    // variance f2 adds f2 to every principal variance (R diag(s^2) R^T +
    // f2 I = R diag(s^2 + f2) R^T); the peak scales by the ratio of the
    // square roots of the determinants, which preserves the integral.
    const T f2 = m.filter3d[i];
    const T q0 = s0 * s0, q1 = s1 * s1, q2 = s2 * s2;
    const T p0 = q0 + f2, p1 = q1 + f2, p2 = q2 + f2;
    s0 = std::sqrt(p0); s1 = std::sqrt(p1); s2 = std::sqrt(p2);
    p.op = p.op * std::sqrt(((q0 * q1) * q2) / ((p0 * p1) * p2));
  }
  for (int r = 0; r < 3; ++r) {
    p.M[3 * r + 0] = Rq[3 * r + 0] * s0;
    p.M[3 * r + 1] = Rq[3 * r + 1] * s1;
    p.M[3 * r + 2] = Rq[3 * r + 2] * s2;
  }
  for (int r = 0; r < 3; ++r)
    for (int c = 0; c < 3; ++c)
      p.S[3 * r + c] = (p.M[3 * r] * p.M[3 * c] + p.M[3 * r + 1] * p.M[3 * c + 1]) +
                       p.M[3 * r + 2] * p.M[3 * c + 2];
  // Local affine approximation of the perspective map at the centre, with the
  // centre's image-plane slope clamped to a guard band.
  const T lim_x = (cam.guard * std::max(cam.cx, T(cam.W) - cam.cx)) / cam.fx;
  const T lim_y = (cam.guard * std::max(cam.cy, T(cam.H) - cam.cy)) / cam.fy;
  T xr = p.tx / p.tz, yr = p.ty / p.tz;
  p.x_clamped = (xr < -lim_x) || (xr > lim_x);
  p.y_clamped = (yr < -lim_y) || (yr > lim_y);
  xr = std::min(std::max(xr, -lim_x), lim_x);
  yr = std::min(std::max(yr, -lim_y), lim_y);
  p.xr = xr; p.yr = yr;
  const T xc = xr * p.tz, yc = yr * p.tz;
  const T tz2 = p.tz * p.tz;
  p.J00 = cam.fx / p.tz;
  p.J02 = -(cam.fx * xc) / tz2;
  p.J11 = cam.fy / p.tz;
  p.J12 = -(cam.fy * yc) / tz2;
  // T = J W (2x3), then Sigma' = T Sigma T^T.
  T* Tm = p.Tm;
  for (int c = 0; c < 3; ++c) {
    Tm[c] = p.J00 * W[c] + p.J02 * W[6 + c];
    Tm[3 + c] = p.J11 * W[3 + c] + p.J12 * W[6 + c];
  }
  T U[6];
  for (int r = 0; r < 2; ++r)
    for (int c = 0; c < 3; ++c)
      U[3 * r + c] = (Tm[3 * r] * p.S[c] + Tm[3 * r + 1] * p.S[3 + c]) + Tm[3 * r + 2] * p.S[6 + c];
  const T s00 = (U[0] * Tm[0] + U[1] * Tm[1]) + U[2] * Tm[2];
  const T s01 = (U[0] * Tm[3] + U[1] * Tm[4]) + U[2] * Tm[5];
  const T s11 = (U[3] * Tm[3] + U[4] * Tm[4]) + U[5] * Tm[5];
  // Screen-space low-pass: the fixed dilation, or Mip-Splatting's 2D filter
  // (its variance instead, and the peak scaled so the integral is kept).
  const T dil = vs.mip_2d ? T(vs.mip_2d_var) : Consts<T>::kappa();
  p.a = s00 + dil;
  p.b = s01;
  p.c = s11 + dil;
  p.det = p.a * p.c - p.b * p.b;
  if (!(p.det > T(0))) return p;
  if (vs.mip_2d) {
    const T det0 = s00 * s11 - s01 * s01;
    p.op = p.op * std::sqrt(std::max(det0, T(0)) / p.det);
  }
  if (p.op < Consts<T>::alpha_min()) return p;
  p.ca = p.c / p.det;
  p.cb = -p.b / p.det;
  p.cc = p.a / p.det;
  p.u = (cam.fx * p.tx) / p.tz + cam.cx;
  p.v = (cam.fy * p.ty) / p.tz + cam.cy;
  // Tile rectangle of the box {q <= qmax}; clamp in float, then convert.
  const int tiles_x = (cam.W + tile - 1) / tile, tiles_y = (cam.H + tile - 1) / tile;
  const T inv_tile = T(1) / T(tile);
  const T hwx = std::sqrt(Consts<T>::qmax() * p.a);
  const T hwy = std::sqrt(Consts<T>::qmax() * p.c);
  auto clampf = [](T v, T hi) { return std::min(std::max(v, T(0)), hi); };
  const T fx0 = clampf(std::floor((p.u - hwx) * inv_tile), T(tiles_x));
  const T fx1 = clampf(std::floor((p.u + hwx) * inv_tile) + T(1), T(tiles_x));
  const T fy0 = clampf(std::floor((p.v - hwy) * inv_tile), T(tiles_y));
  const T fy1 = clampf(std::floor((p.v + hwy) * inv_tile) + T(1), T(tiles_y));
  p.rect[0] = int(fx0); p.rect[1] = int(fy0); p.rect[2] = int(fx1); p.rect[3] = int(fy1);
  p.ntiles = uint32_t((p.rect[2] - p.rect[0]) * (p.rect[3] - p.rect[1]));
  if (p.ntiles == 0) return p;
  // View-dependent colour from the eye centre c = -W^T t.
  const T ccx = -((W[0] * cam.t[0] + W[3] * cam.t[1]) + W[6] * cam.t[2]);
  const T ccy = -((W[1] * cam.t[0] + W[4] * cam.t[1]) + W[7] * cam.t[2]);
  const T ccz = -((W[2] * cam.t[0] + W[5] * cam.t[1]) + W[8] * cam.t[2]);
  const T dx = mx - ccx, dy = my - ccy, dz = mz - ccz;
  p.dlen = std::sqrt((dx * dx + dy * dy) + dz * dz);
  p.dir[0] = dx / p.dlen; p.dir[1] = dy / p.dlen; p.dir[2] = dz / p.dlen;
  sh.basis(p.dir[0], p.dir[1], p.dir[2], p.Y);
  const int nc = (m.D + 1) * (m.D + 1);
  for (int ch = 0; ch < 3; ++ch) {
    T acc = m.sh[(size_t)(0 * 3 + ch) * n + i] * p.Y[0];
    for (int k = 1; k < nc; ++k) acc = acc + m.sh[(size_t)(k * 3 + ch) * n + i] * p.Y[k];
    T raw = acc + T(0.5);
    if (raw < T(0)) { p.clamp |= 1u << ch; raw = T(0); }
    p.rgb[ch] = raw;
  }
  p.valid = true;
  return p;
}

template <typename T> struct ViewInfo {
  int tiles_x, tiles_y;
  uint64_t tile_off, rec_off, pix_off;
};

template <typename T> struct Scene {
  int n_views;
  std::vector<Model<T>> models;
  std::vector<Cam<T>> cams;
  std::vector<oc_view> views;
  std::vector<ViewInfo<T>> info;
  std::vector<Proj<T>> proj;  // all records
  // per record: the depth key the pairs are sorted by within a tile, the
  // bits of the camera-space depth as an unsigned integer; the view's own
  // depth, or that of the view's sort camera (one order shared by the eyes
  // of a stereo frame, Sec. 3.3)
  std::vector<uint32_t> sort_key;
  uint64_t total_tiles = 0, total_recs = 0, total_pix = 0;
  int tile = 16;
};

template <typename T> uint32_t depth_bits(T d);

template <typename T>
void build_scene(Scene<T>& sc, int n_views, const Model<T>* models, const oc_camera* cams,
                 const oc_view* views, int tile, const oc_camera* sort_cams = nullptr) {
  SH<T> sh;
  sc.n_views = n_views;
  sc.tile = tile;
  for (int v = 0; v < n_views; ++v) {
    sc.models.push_back(models[v]);
    sc.cams.emplace_back(cams[v]);
    sc.views.push_back(views[v]);
    ViewInfo<T> vi;
    vi.tiles_x = (cams[v].width + tile - 1) / tile;
    vi.tiles_y = (cams[v].height + tile - 1) / tile;
    vi.tile_off = sc.total_tiles;
    vi.rec_off = sc.total_recs;
    vi.pix_off = sc.total_pix;
    sc.info.push_back(vi);
    sc.total_tiles += (uint64_t)vi.tiles_x * vi.tiles_y;
    sc.total_recs += (uint64_t)models[v].n;
    sc.total_pix += (uint64_t)cams[v].width * cams[v].height;
  }
  sc.proj.resize(sc.total_recs);
  sc.sort_key.resize(sc.total_recs);
  for (int v = 0; v < n_views; ++v) {
    const Model<T>& m = sc.models[v];
    for (int i = 0; i < m.n; ++i) {
      const uint64_t r = sc.info[v].rec_off + i;
      sc.proj[r] = project_one(m, i, sc.cams[v], sc.views[v], tile, sh);
      if (sort_cams) {
        // depth of the centre in the sort camera, in the order of the
        // view's own depth
        const Cam<T> S(sort_cams[v]);
        const T mx = m.mean[i], my = m.mean[m.n + i], mz = m.mean[2 * m.n + i];
        sc.sort_key[r] = depth_bits(((S.R[6] * mx + S.R[7] * my) + S.R[8] * mz) + S.t[2]);
      } else {
        sc.sort_key[r] = sc.proj[r].valid ? depth_bits(sc.proj[r].tz) : 0u;
      }
    }
  }
}

template <typename T> uint32_t depth_bits(T d) {
  float f = float(d);
  uint32_t u;
  std::memcpy(&u, &f, 4);
  return u;
}

struct Pair {
  uint64_t tile;
  uint32_t rec;
};

// Emission order: views in order, Gaussians by index, each Gaussian's tiles
// row-major.  Sorting is stable on (tile, depth), so equal keys stay in
// emission order (ascending Gaussian index).
template <typename T> std::vector<Pair> emit_pairs(const Scene<T>& sc) {
  std::vector<Pair> pairs;
  for (int v = 0; v < sc.n_views; ++v) {
    const ViewInfo<T>& vi = sc.info[v];
    for (int i = 0; i < sc.models[v].n; ++i) {
      const Proj<T>& p = sc.proj[vi.rec_off + i];
      if (!p.valid) continue;
      for (int ty = p.rect[1]; ty < p.rect[3]; ++ty)
        for (int tx = p.rect[0]; tx < p.rect[2]; ++tx)
          pairs.push_back({vi.tile_off + (uint64_t)ty * vi.tiles_x + tx, (uint32_t)(vi.rec_off + i)});
    }
  }
  return pairs;
}

template <typename T> struct PixelOut {
  T rgb[3], T_final;
  uint32_t last = 0, n_contrib = 0;
  uint64_t evaluated = 0;
  // Smallest distance of a threshold decision from its threshold, in units of
  // that decision's tolerance (relative 1e-5 for the sign of q and the 1/255
  // cutoff, relative 1e-4 for the 1e-4 stop); below 1 the pixel is "near a
  // threshold" and a differently rounded evaluation may decide it otherwise.
  float margin = 1e30f;
};

// Front-to-back compositing of one pixel over a depth-ordered list of record
// ids.  `on_blend(k, rec, alpha, T_before, G, dx, dy, clamped)` is called for
// every blended pair.
// near (optional, [records]): set to 1 for each record one of whose decisions
// here lies below margin 1.
inline void mark_near(uint8_t* near, uint32_t rec, float m) {
  if (near && m < 1.0f) {
#pragma omp atomic write
    near[rec] = 1;
  }
}

template <typename T, typename F>
PixelOut<T> blend_pixel(const Scene<T>& sc, const uint32_t* list, size_t count, T px, T py,
                        const float* bg, F&& on_blend, uint8_t* near = nullptr) {
  PixelOut<T> o;
  T Tc = T(1);
  T C[3] = {T(0), T(0), T(0)};
  for (size_t k = 0; k < count; ++k) {
    const Proj<T>& p = sc.proj[list[k]];
    const T dx = p.u - px, dy = p.v - py;
    const T qa = p.ca * dx * dx, qc = p.cc * dy * dy, qb = T(2) * p.cb * dx * dy;
    const T q = (qa + qc) + qb;
    const T power = T(-0.5) * q;
    ++o.evaluated;
    {
      const T mag = std::fabs(qa) + std::fabs(qc) + std::fabs(qb);
      if (mag > T(0)) {
        const float m = float(std::fabs(q) / mag / T(1e-5));
        o.margin = std::min(o.margin, m);
        mark_near(near, list[k], m);
      }
    }
    if (power > T(0)) continue;
    const T G = std::exp(power);
    const T oG = p.op * G;
    {
      const float m = float(std::fabs(oG - Consts<T>::alpha_min()) / Consts<T>::alpha_min() / T(1e-5));
      o.margin = std::min(o.margin, m);
      mark_near(near, list[k], m);
    }
    const bool clamped = oG > Consts<T>::alpha_max();
    const T alpha = clamped ? Consts<T>::alpha_max() : oG;
    if (alpha < Consts<T>::alpha_min()) continue;
    const T Tn = Tc * (T(1) - alpha);
    {
      const float m = float(std::fabs(Tn - Consts<T>::t_stop()) / Consts<T>::t_stop() / T(1e-4));
      o.margin = std::min(o.margin, m);
      mark_near(near, list[k], m);
    }
    if (Tn < Consts<T>::t_stop()) break;  // this Gaussian is not blended
    const T w = alpha * Tc;
    for (int ch = 0; ch < 3; ++ch) C[ch] = C[ch] + p.rgb[ch] * w;
    on_blend(k, list[k], alpha, Tc, G, dx, dy, clamped);
    Tc = Tn;
    o.last = (uint32_t)(k + 1);
    ++o.n_contrib;
  }
  for (int ch = 0; ch < 3; ++ch) o.rgb[ch] = C[ch] + Tc * T(bg[ch]);
  o.T_final = Tc;
  return o;
}

template <typename T> struct Sorted {
  std::vector<Pair> emit, sorted;
  std::vector<uint32_t> start, end;  // per global tile
};

template <typename T> Sorted<T> sort_pairs(const Scene<T>& sc) {
  Sorted<T> s;
  s.emit = emit_pairs(sc);
  s.sorted = s.emit;
  std::stable_sort(s.sorted.begin(), s.sorted.end(), [&](const Pair& x, const Pair& y) {
    if (x.tile != y.tile) return x.tile < y.tile;
    return sc.sort_key[x.rec] < sc.sort_key[y.rec];
  });
  s.start.assign(sc.total_tiles, 0);
  s.end.assign(sc.total_tiles, 0);
  for (size_t k = 0; k < s.sorted.size(); ++k) {
    const uint64_t t = s.sorted[k].tile;
    if (k == 0 || s.sorted[k - 1].tile != t) s.start[t] = (uint32_t)k;
    if (k + 1 == s.sorted.size() || s.sorted[k + 1].tile != t) s.end[t] = (uint32_t)(k + 1);
  }
  return s;
}

// Per-pixel record lists: the tile's sorted pairs, or (brute force) every
// surviving record of the view ordered by (depth, index).
template <typename T> struct ListSource {
  const Scene<T>& sc;
  const Sorted<T>* sorted;
  std::vector<std::vector<uint32_t>> brute;  // per view
  std::vector<uint32_t> tile_vals;           // sorted vals, flat
  ListSource(const Scene<T>& s, const Sorted<T>* so, bool brute_force) : sc(s), sorted(so) {
    if (brute_force) {
      brute.resize(sc.n_views);
      for (int v = 0; v < sc.n_views; ++v) {
        const ViewInfo<T>& vi = sc.info[v];
        for (int i = 0; i < sc.models[v].n; ++i)
          if (sc.proj[vi.rec_off + i].valid) brute[v].push_back((uint32_t)(vi.rec_off + i));
        std::stable_sort(brute[v].begin(), brute[v].end(), [&](uint32_t x, uint32_t y) {
          return sc.sort_key[x] < sc.sort_key[y];
        });
      }
    } else {
      tile_vals.resize(so->sorted.size());
      for (size_t k = 0; k < so->sorted.size(); ++k) tile_vals[k] = so->sorted[k].rec;
    }
  }
  // returns list pointer, count and the index base of the list in the sorted pairs
  const uint32_t* get(int v, int x, int y, size_t* count, size_t* base) const {
    if (!brute.empty()) {
      *count = brute[v].size();
      *base = 0;
      return brute[v].data();
    }
    const ViewInfo<T>& vi = sc.info[v];
    const uint64_t t = vi.tile_off + (uint64_t)(y / sc.tile) * vi.tiles_x + (x / sc.tile);
    *base = sorted->start[t];
    *count = sorted->end[t] - sorted->start[t];
    return tile_vals.data() + *base;
  }
};

template <typename T>
int render(int n_views, const Model<T>* models, const oc_camera* cams, const oc_view* views,
           int tile, int brute_force, oc_outputs* out, int n_threads, const oc_camera* sort_cams) {
  if (n_views < 0 || !out || (tile != 8 && tile != 16 && tile != 32)) return -1;
  for (int v = 0; v < n_views; ++v) {
    if (models[v].n < 0 || models[v].D < 0 || models[v].D > 3) return -1;
    if (cams[v].width <= 0 || cams[v].height <= 0) return -1;
    if (views[v].n_clip < 0 || views[v].n_clip > 8) return -1;
  }
#ifdef _OPENMP
  if (n_threads > 0) omp_set_num_threads(n_threads);
#else
  (void)n_threads;
#endif
  Scene<T> sc;
  build_scene(sc, n_views, models, cams, views, tile, sort_cams);
  Sorted<T> so = sort_pairs(sc);
  const uint64_t K = so.sorted.size();
  out->counts[0] = K;
  out->counts[3] = sc.total_tiles;
  // records
  for (uint64_t r = 0; r < sc.total_recs; ++r) {
    const Proj<T>& p = sc.proj[r];
    if (out->rec) {
      T* rr = (T*)out->rec + 10 * r;
      if (p.valid) {
        rr[0] = p.u; rr[1] = p.v; rr[2] = p.ca; rr[3] = p.cb; rr[4] = p.cc;
        rr[5] = p.op; rr[6] = p.tz; rr[7] = p.rgb[0]; rr[8] = p.rgb[1]; rr[9] = p.rgb[2];
      } else {
        for (int k = 0; k < 10; ++k) rr[k] = T(0);
      }
    }
    if (out->rect)
      for (int k = 0; k < 4; ++k) out->rect[4 * r + k] = p.valid ? p.rect[k] : 0;
    if (out->n_tiles) out->n_tiles[r] = p.valid ? p.ntiles : 0;
    if (out->clamp) out->clamp[r] = p.valid ? p.clamp : 0;
  }
  if (out->keys_emit || out->vals_emit || out->keys || out->vals) {
    if (K > out->pair_cap) return -2;
    for (uint64_t k = 0; k < K; ++k) {
      const Pair& e = so.emit[k];
      const Pair& s = so.sorted[k];
      if (out->keys_emit) out->keys_emit[k] = (e.tile << 32) | sc.sort_key[e.rec];
      if (out->vals_emit) out->vals_emit[k] = e.rec;
      if (out->keys) out->keys[k] = (s.tile << 32) | sc.sort_key[s.rec];
      if (out->vals) out->vals[k] = s.rec;
    }
  }
  if (out->ranges)
    for (uint64_t t = 0; t < sc.total_tiles; ++t) {
      out->ranges[2 * t] = so.start[t];
      out->ranges[2 * t + 1] = so.end[t];
    }
  ListSource<T> src(sc, &so, brute_force != 0);
  uint64_t E = 0, A = 0;
  for (int v = 0; v < n_views; ++v) {
    const int W = sc.cams[v].W, H = sc.cams[v].H;
    const uint64_t po = sc.info[v].pix_off;
#pragma omp parallel for schedule(dynamic, 16) reduction(+ : E, A)
    for (int y = 0; y < H; ++y) {
      for (int x = 0; x < W; ++x) {
        size_t count, base;
        const uint32_t* list = src.get(v, x, y, &count, &base);
        PixelOut<T> o = blend_pixel(sc, list, count, T(x) + T(0.5), T(y) + T(0.5), sc.views[v].bg,
                                    [](size_t, uint32_t, T, T, T, T, T, bool) {}, out->near_rec);
        E += o.evaluated;
        A += o.n_contrib;
        const uint64_t pix = po + (uint64_t)y * W + x;
        const uint64_t pix_rgb = 3 * po + (uint64_t)y * W + x;
        if (out->rgb)
          for (int ch = 0; ch < 3; ++ch) ((T*)out->rgb)[pix_rgb + (uint64_t)ch * W * H] = o.rgb[ch];
        if (out->alpha) ((T*)out->alpha)[pix] = T(1) - o.T_final;
        if (out->final_T) ((T*)out->final_T)[pix] = o.T_final;
        if (out->last) out->last[pix] = o.last == 0 ? 0u : (uint32_t)(base + o.last);
        if (out->n_contrib) out->n_contrib[pix] = o.n_contrib;
        if (out->margin) out->margin[pix] = o.margin;
      }
    }
  }
  out->counts[1] = E;
  out->counts[2] = A;
  return 0;
}

// 2D gradient accumulators per record: u, v, conic a, b, c, opacity, r, g, b.
template <typename T> struct G2 {
  T g[9];
};

// Chain rule from the 2D gradient g2 of one record to the Gaussian's
// parameters, accumulated into gm[3], gs[3], gq[4], go, gsh[nc*3].
template <typename T>
void backward_gaussian(const Model<T>& m, int i, const Cam<T>& cam, const Proj<T>& p, const SH<T>& sh,
                       const T* g2, T* gm, T* gs, T* gq, T* go, T* gsh) {
  const int n = m.n;
  const T* W = cam.R;
  // --- opacity: the record's opacity is o times the layer's factor
  *go += p.fade * g2[5];
  // --- colour: SH coefficients and the view direction
  T drgb[3];
  for (int ch = 0; ch < 3; ++ch) drgb[ch] = ((p.clamp >> ch) & 1u) ? T(0) : g2[6 + ch];
  const int nc = (m.D + 1) * (m.D + 1);
  T ddir[3] = {T(0), T(0), T(0)};
  T Gy[16][3];
  sh.grad(p.dir[0], p.dir[1], p.dir[2], Gy);
  for (int k = 0; k < nc; ++k)
    for (int ch = 0; ch < 3; ++ch) {
      gsh[k * 3 + ch] += p.Y[k] * drgb[ch];
      const T c = m.sh[(size_t)(k * 3 + ch) * n + i];
      for (int j = 0; j < 3; ++j) ddir[j] += c * Gy[k][j] * drgb[ch];
    }
  const T* dir = p.dir;
  const T dd = dir[0] * ddir[0] + dir[1] * ddir[1] + dir[2] * ddir[2];
  for (int j = 0; j < 3; ++j) gm[j] += (ddir[j] - dir[j] * dd) / p.dlen;
  // --- conic -> (a, b, c) of the 2D covariance
  const T a = p.a, b = p.b, c = p.c, det2 = p.det * p.det;
  const T dca = g2[2], dcb = g2[3], dcc = g2[4];
  const T da = dca * (-c * c / det2) + dcb * (b * c / det2) + dcc * (-b * b / det2);
  const T db = dca * (T(2) * b * c / det2) + dcb * (-(a * c + b * b) / det2) + dcc * (T(2) * a * b / det2);
  const T dc = dca * (-b * b / det2) + dcb * (a * b / det2) + dcc * (-a * a / det2);
  // --- Sigma' = T Sigma T^T  (entries s00 = a - kappa, s01 = b, s11 = c - kappa)
  const T* Tm = p.Tm;
  const T* S = p.S;
  T ST0[3], ST1[3];
  for (int r = 0; r < 3; ++r) {
    ST0[r] = S[3 * r] * Tm[0] + S[3 * r + 1] * Tm[1] + S[3 * r + 2] * Tm[2];
    ST1[r] = S[3 * r] * Tm[3] + S[3 * r + 1] * Tm[4] + S[3 * r + 2] * Tm[5];
  }
  T dT0[3], dT1[3], dS[9];
  for (int r = 0; r < 3; ++r) {
    dT0[r] = T(2) * da * ST0[r] + db * ST1[r];
    dT1[r] = db * ST0[r] + T(2) * dc * ST1[r];
  }
  for (int r = 0; r < 3; ++r)
    for (int q = 0; q < 3; ++q)
      dS[3 * r + q] = da * Tm[r] * Tm[q] + db * Tm[r] * Tm[3 + q] + dc * Tm[3 + r] * Tm[3 + q];
  // --- Sigma = M M^T, M = Rq diag(s)
  T dM[9];
  for (int r = 0; r < 3; ++r)
    for (int k = 0; k < 3; ++k) {
      T acc = T(0);
      for (int j = 0; j < 3; ++j) acc += (dS[3 * r + j] + dS[3 * j + r]) * p.M[3 * j + k];
      dM[3 * r + k] = acc;
    }
  const T s[3] = {m.scale[i], m.scale[n + i], m.scale[2 * n + i]};
  T dR[9];
  for (int r = 0; r < 3; ++r)
    for (int k = 0; k < 3; ++k) {
      gs[k] += dM[3 * r + k] * p.Rq[3 * r + k];
      dR[3 * r + k] = dM[3 * r + k] * s[k];
    }
  // --- rotation matrix -> unit quaternion -> raw quaternion
  const T w = p.qh[0], x = p.qh[1], y = p.qh[2], z = p.qh[3];
  const T two = T(2);
  T dq[4];
  dq[0] = two * (-z * dR[1] + y * dR[2] + z * dR[3] - x * dR[5] - y * dR[6] + x * dR[7]);
  dq[1] = two * (y * dR[1] + z * dR[2] + y * dR[3] - two * x * dR[4] - w * dR[5] + z * dR[6] +
                 w * dR[7] - two * x * dR[8]);
  dq[2] = two * (-two * y * dR[0] + x * dR[1] + w * dR[2] + x * dR[3] + z * dR[5] - w * dR[6] +
                 z * dR[7] - two * y * dR[8]);
  dq[3] = two * (-two * z * dR[0] - w * dR[1] + x * dR[2] + w * dR[3] - two * z * dR[4] +
                 y * dR[5] + x * dR[6] + y * dR[7]);
  const T qd = w * dq[0] + x * dq[1] + y * dq[2] + z * dq[3];
  for (int k = 0; k < 4; ++k) gq[k] += (dq[k] - p.qh[k] * qd) / p.qn;
  // --- Jacobian and projected centre -> camera-space centre
  T dJ00 = T(0), dJ02 = T(0), dJ11 = T(0), dJ12 = T(0);
  for (int r = 0; r < 3; ++r) {
    dJ00 += dT0[r] * W[r];
    dJ02 += dT0[r] * W[6 + r];
    dJ11 += dT1[r] * W[3 + r];
    dJ12 += dT1[r] * W[6 + r];
  }
  const T tx = p.tx, ty = p.ty, tz = p.tz, tz2 = tz * tz, tz3 = tz2 * tz;
  const T fx = cam.fx, fy = cam.fy;
  T dtx = T(0), dty = T(0), dtz = T(0);
  dtz += dJ00 * (-fx / tz2) + dJ11 * (-fy / tz2);
  if (!p.x_clamped) {
    dtx += dJ02 * (-fx / tz2);
    dtz += dJ02 * (two * fx * tx / tz3);
  } else {
    dtz += dJ02 * (fx * p.xr / tz2);
  }
  if (!p.y_clamped) {
    dty += dJ12 * (-fy / tz2);
    dtz += dJ12 * (two * fy * ty / tz3);
  } else {
    dtz += dJ12 * (fy * p.yr / tz2);
  }
  const T du = g2[0], dv = g2[1];
  dtx += du * fx / tz;
  dtz += -du * fx * tx / tz2;
  dty += dv * fy / tz;
  dtz += -dv * fy * ty / tz2;
  for (int j = 0; j < 3; ++j) gm[j] += W[j] * dtx + W[3 + j] * dty + W[6 + j] * dtz;
}

// A projection's values in another floating-point type (each rounded or
// widened once).
template <typename TG, typename TF> Proj<TG> convert(const Proj<TF>& p) {
  Proj<TG> q;
  q.valid = p.valid;
  q.tx = TG(p.tx); q.ty = TG(p.ty); q.tz = TG(p.tz); q.xr = TG(p.xr); q.yr = TG(p.yr);
  q.x_clamped = p.x_clamped; q.y_clamped = p.y_clamped;
  q.qn = TG(p.qn);
  for (int k = 0; k < 4; ++k) q.qh[k] = TG(p.qh[k]);
  for (int k = 0; k < 9; ++k) { q.Rq[k] = TG(p.Rq[k]); q.M[k] = TG(p.M[k]); q.S[k] = TG(p.S[k]); }
  q.J00 = TG(p.J00); q.J02 = TG(p.J02); q.J11 = TG(p.J11); q.J12 = TG(p.J12);
  for (int k = 0; k < 6; ++k) q.Tm[k] = TG(p.Tm[k]);
  q.a = TG(p.a); q.b = TG(p.b); q.c = TG(p.c); q.det = TG(p.det);
  q.u = TG(p.u); q.v = TG(p.v); q.ca = TG(p.ca); q.cb = TG(p.cb); q.cc = TG(p.cc); q.op = TG(p.op); q.fade = TG(p.fade);
  for (int k = 0; k < 3; ++k) q.rgb[k] = TG(p.rgb[k]);
  q.clamp = p.clamp;
  for (int k = 0; k < 4; ++k) q.rect[k] = p.rect[k];
  q.ntiles = p.ntiles;
  for (int k = 0; k < 3; ++k) q.dir[k] = TG(p.dir[k]);
  q.dlen = TG(p.dlen);
  for (int k = 0; k < 16; ++k) q.Y[k] = TG(p.Y[k]);
  return q;
}

// The model's parameter arrays in another floating-point type.
template <typename TG, typename TF> struct ModelCopy {
  std::vector<TG> mean, scale, quat, opacity, sh;
  Model<TG> m;
  explicit ModelCopy(const Model<TF>& s) {
    const size_t n = (size_t)s.n, nc = (size_t)(s.D + 1) * (s.D + 1);
    mean.assign(s.mean, s.mean + 3 * n);
    scale.assign(s.scale, s.scale + 3 * n);
    quat.assign(s.quat, s.quat + 4 * n);
    opacity.assign(s.opacity, s.opacity + n);
    sh.assign(s.sh, s.sh + 3 * nc * n);
    m.n = s.n; m.D = s.D;
    m.mean = mean.data(); m.scale = scale.data(); m.quat = quat.data(); m.opacity = opacity.data();
    m.sh = sh.data(); m.layer = s.layer;
  }
};

// Exact gradient of L = sum(dL_drgb * rgb) + sum(dL_dalpha * alpha) (B1-B10
// of the design notes).  The forward - projection, pair lists and every
// per-pixel decision (skip below 1/255, the 0.99 clamp, the 1e-4 stop) - is
// the TF forward above; every quantity of the gradient (alpha, G and T of the
// blended pairs, the colour behind each of them, the per-record 2D gradients
// and the chain rule) is evaluated in TG from the TF records.  TF = TG is the
// plain float or double backward; TF = float, TG = double is the float32
// forward's gradient evaluated without float32 rounding.  With fwd_values
// the blended pairs' offsets (dx, dy), G, alpha and transmittances are the
// TF forward's own values instead (only the arithmetic after them is in TG).
// cond (optional, [(11 + 3 (D+1)^2) n], packed mean, scale, quat, opacity,
// sh like the gradients): per entry, the sum over the 2D slots of
// |d entry / d slot| times the sum over pixels of the magnitude of the
// slot's per-pixel terms, each taken with the magnitudes of its operands
// (dL/dalpha as sum_ch |G_ch| (|c_ch| T + |S_ch| / (1 - alpha)) +
// |G_A| T_final / (1 - alpha)) and weighted by the pixel's number of blended
// pairs + 16.  A float32 evaluation's per-pixel terms carry about one
// rounding per pair of the product behind T (and the colour behind) plus a
// few of their own, so cond is the scale of the error that float32 leaves
// on that entry: it errs by a small multiple of 2^-24 cond.
template <typename TF, typename TG>
int backward(int n_views, const Model<TF>& m, const oc_camera* cams, const oc_view* views, const TF* dL_drgb,
             const TF* dL_dalpha, uint32_t trainable, TG* g_mean, TG* g_scale, TG* g_quat, TG* g_opacity,
             TG* g_sh, TG* max_contrib, TG* activity, int n_threads, bool fwd_values = false,
             TG* cond = nullptr, TG* dens_grad = nullptr, TG* dens_cnt = nullptr) {
  if (n_views < 0 || m.n < 0 || m.D < 0 || m.D > 3) return -1;
  if (m.filter3d) return -1;  // the Mip filters are forward-only
  for (int v = 0; v < n_views; ++v)
    if (views[v].mip_2d) return -1;
#ifdef _OPENMP
  if (n_threads > 0) omp_set_num_threads(n_threads);
#else
  (void)n_threads;
#endif
  std::vector<Model<TF>> models(n_views, m);
  Scene<TF> sc;
  build_scene(sc, n_views, models.data(), cams, views, 16);
  Sorted<TF> so = sort_pairs(sc);
  ListSource<TF> src(sc, &so, false);
  const int n = m.n;
  // per-record 2D gradients and max contribution, accumulated per thread
  int nthr = 1;
#ifdef _OPENMP
  nthr = omp_get_max_threads();
#endif
  std::vector<std::vector<G2<TG>>> acc(nthr, std::vector<G2<TG>>(sc.total_recs, G2<TG>{}));
  std::vector<std::vector<TG>> mc(nthr, std::vector<TG>(sc.total_recs, TG(0)));
  std::vector<std::vector<G2<TG>>> accm(cond ? nthr : 0, std::vector<G2<TG>>(sc.total_recs, G2<TG>{}));
  struct Blended { uint32_t rec; TF alpha, Tb, G, dx, dy; bool clamped; };
  struct Contrib { uint32_t rec; TG alpha, Tb, G, dx, dy; bool clamped; };
  for (int v = 0; v < n_views; ++v) {
    const int W = sc.cams[v].W, H = sc.cams[v].H;
    const uint64_t po = sc.info[v].pix_off;
    // rows go to threads round-robin (a fixed assignment for a given thread
    // count), so every per-record sum is taken in the same order on every run
#pragma omp parallel for schedule(static, 1)
    for (int y = 0; y < H; ++y) {
      int tid = 0;
#ifdef _OPENMP
      tid = omp_get_thread_num();
#endif
      std::vector<Blended> bl;
      std::vector<Contrib> cl;
      for (int x = 0; x < W; ++x) {
        size_t count, base;
        const uint32_t* list = src.get(v, x, y, &count, &base);
        bl.clear();
        const PixelOut<TF> fo =
            blend_pixel(sc, list, count, TF(x) + TF(0.5), TF(y) + TF(0.5), sc.views[v].bg,
                        [&](size_t, uint32_t rec, TF alpha, TF Tb, TF G, TF dx, TF dy, bool clamped) {
                          bl.push_back({rec, alpha, Tb, G, dx, dy, clamped});
                        });
        // the blended pairs' alpha, G and transmittance in front, in TG
        cl.clear();
        const TG pxg = TG(x) + TG(0.5), pyg = TG(y) + TG(0.5);
        TG Tc = TG(1);
        for (const Blended& e : bl) {
          if (fwd_values) {
            cl.push_back({e.rec, TG(e.alpha), TG(e.Tb), TG(e.G), TG(e.dx), TG(e.dy), e.clamped});
            continue;
          }
          const Proj<TF>& p = sc.proj[e.rec];
          const TG dx = TG(p.u) - pxg, dy = TG(p.v) - pyg;
          const TG q = (TG(p.ca) * dx * dx + TG(p.cc) * dy * dy) + TG(2) * TG(p.cb) * dx * dy;
          const TG G = std::exp(TG(-0.5) * q);
          const TG alpha = e.clamped ? Consts<TG>::alpha_max() : TG(p.op) * G;
          cl.push_back({e.rec, alpha, Tc, G, dx, dy, e.clamped});
          Tc = Tc * (TG(1) - alpha);
        }
        const TG T_final = fwd_values ? TG(fo.T_final) : Tc;
        TG Gc[3];
        for (int ch = 0; ch < 3; ++ch) Gc[ch] = TG(dL_drgb[3 * po + (uint64_t)ch * W * H + (uint64_t)y * W + x]);
        const TG GA = TG(dL_dalpha[po + (uint64_t)y * W + x]);
        // suffix colour S_k = sum_{j>k} c_j alpha_j T_j + T_final * bg
        TG S[3];
        for (int ch = 0; ch < 3; ++ch) S[ch] = T_final * TG(sc.views[v].bg[ch]);
        for (size_t kk = cl.size(); kk-- > 0;) {
          const Contrib& e = cl[kk];
          const Proj<TF>& p = sc.proj[e.rec];
          G2<TG>& g = acc[tid][e.rec];
          const TG w = e.alpha * e.Tb;
          TG dalpha = GA * T_final / (TG(1) - e.alpha);
          TG dmag = std::fabs(dalpha);
          for (int ch = 0; ch < 3; ++ch) {
            const TG c = TG(p.rgb[ch]);
            g.g[6 + ch] += Gc[ch] * w;
            dalpha += Gc[ch] * (c * e.Tb - S[ch] / (TG(1) - e.alpha));
            dmag += std::fabs(Gc[ch]) * (std::fabs(c) * e.Tb + std::fabs(S[ch]) / (TG(1) - e.alpha));
            S[ch] += c * w;
          }
          if (w > mc[tid][e.rec]) mc[tid][e.rec] = w;
          const TG depth_w = TG(cl.size() + 16);
          if (cond)
            for (int ch = 0; ch < 3; ++ch) accm[tid][e.rec].g[6 + ch] += depth_w * std::fabs(Gc[ch] * w);
          if (e.clamped) continue;
          const TG op = TG(p.op), ca = TG(p.ca), cb = TG(p.cb), cc = TG(p.cc);
          g.g[5] += dalpha * e.G;
          const TG dq = dalpha * (TG(-0.5) * op * e.G);
          g.g[0] += dq * TG(2) * (ca * e.dx + cb * e.dy);
          g.g[1] += dq * TG(2) * (cb * e.dx + cc * e.dy);
          g.g[2] += dq * e.dx * e.dx;
          g.g[3] += dq * TG(2) * e.dx * e.dy;
          g.g[4] += dq * e.dy * e.dy;
          if (cond) {
            G2<TG>& a = accm[tid][e.rec];
            const TG mw = depth_w * dmag;
            const TG mq = mw * (TG(0.5) * op * e.G);
            a.g[5] += mw * e.G;
            a.g[0] += mq * TG(2) * (std::fabs(ca * e.dx) + std::fabs(cb * e.dy));
            a.g[1] += mq * TG(2) * (std::fabs(cb * e.dx) + std::fabs(cc * e.dy));
            a.g[2] += mq * e.dx * e.dx;
            a.g[3] += mq * TG(2) * std::fabs(e.dx * e.dy);
            a.g[4] += mq * e.dy * e.dy;
          }
        }
      }
    }
  }
  // reduce thread buffers in thread order
  std::vector<G2<TG>> g2(sc.total_recs, G2<TG>{});
  std::vector<G2<TG>> g2m(cond ? sc.total_recs : 0, G2<TG>{});
  std::vector<TG> mcr(sc.total_recs, TG(0));
  for (int t = 0; t < nthr; ++t)
    for (uint64_t r = 0; r < sc.total_recs; ++r) {
      for (int k = 0; k < 9; ++k) g2[r].g[k] += acc[t][r].g[k];
      if (cond)
        for (int k = 0; k < 9; ++k) g2m[r].g[k] += accm[t][r].g[k];
      mcr[r] = std::max(mcr[r], mc[t][r]);
    }
  const int nc = (m.D + 1) * (m.D + 1);
  SH<TG> sh;
  const ModelCopy<TG, TF> mg(m);
  std::vector<Cam<TG>> cams_g;
  for (int v = 0; v < n_views; ++v) cams_g.emplace_back(cams[v]);
  int i_cur = 0;
  // The chain rule differentiates the projection at the parameters: its
  // intermediate values are recomputed in TG from them (for TF = TG they
  // equal the forward's), with the forward's decisions - the guard-band
  // clamp of the Jacobian and the colour clamp bits - kept.
  auto chain_proj = [&](int v, const Proj<TF>& pf) {
    Proj<TG> pg = project_one(mg.m, i_cur, cams_g[v], sc.views[v], 16, sh);
    if (!pg.valid) return convert<TG>(pf);
    pg.x_clamped = pf.x_clamped;
    pg.y_clamped = pf.y_clamped;
    if (pf.x_clamped) pg.xr = TG(pf.xr);
    if (pf.y_clamped) pg.yr = TG(pf.yr);
    pg.clamp = pf.clamp;
    return pg;
  };
  std::vector<TG> gm(3), gs(3), gq(4), gsh(nc * 3);
  const int per = 11 + 3 * nc;  // gradient entries per Gaussian
  std::vector<TG> col(per), csum(per);
  for (int i = 0; i < n; ++i) {
    i_cur = i;
    if (cond) std::fill(csum.begin(), csum.end(), TG(0));
    TG go = TG(0);
    std::fill(gm.begin(), gm.end(), TG(0));
    std::fill(gs.begin(), gs.end(), TG(0));
    std::fill(gq.begin(), gq.end(), TG(0));
    std::fill(gsh.begin(), gsh.end(), TG(0));
    TG mcv = TG(0);
    TG dgs = TG(0), dgc = TG(0);
    const bool train = m.layer[i] < 32 && ((trainable >> m.layer[i]) & 1u);
    for (int v = 0; v < n_views; ++v) {
      const uint64_t r = sc.info[v].rec_off + i;
      if (!sc.proj[r].valid) continue;
      mcv = std::max(mcv, mcr[r]);
      if (train && sc.proj[r].ntiles > 0) {
        // densification statistic: the length of the loss gradient with
        // respect to the projected centre in normalised device coordinates
        // (x_ndc spans [-1, 1] over the width: du / dx_ndc = W / 2)
        const TG gx = g2[r].g[0] * (TG(sc.cams[v].W) / TG(2));
        const TG gy = g2[r].g[1] * (TG(sc.cams[v].H) / TG(2));
        dgs += std::sqrt(gx * gx + gy * gy);
        dgc += TG(1);
      }
      const Proj<TG> pg = train ? chain_proj(v, sc.proj[r]) : Proj<TG>();
      if (train)
        backward_gaussian(mg.m, i, cams_g[v], pg, sh, g2[r].g, gm.data(), gs.data(), gq.data(), &go, gsh.data());
      if (train && cond)
        // the chain rule is linear in the 2D gradient: column `sl` of its
        // matrix, in magnitude, times the slot's magnitude sum
        for (int sl = 0; sl < 9; ++sl) {
          if (g2m[r].g[sl] == TG(0)) continue;
          TG e[9] = {};
          e[sl] = TG(1);
          std::fill(col.begin(), col.end(), TG(0));
          backward_gaussian(mg.m, i, cams_g[v], pg, sh, e, &col[0], &col[3], &col[6], &col[10], &col[11]);
          for (int k = 0; k < per; ++k) csum[k] += std::fabs(col[k]) * g2m[r].g[sl];
        }
    }
    if (!train) {
      std::fill(gm.begin(), gm.end(), TG(0));
      std::fill(gs.begin(), gs.end(), TG(0));
      std::fill(gq.begin(), gq.end(), TG(0));
      std::fill(gsh.begin(), gsh.end(), TG(0));
      go = TG(0);
    }
    for (int j = 0; j < 3; ++j) g_mean[(size_t)j * n + i] = gm[j];
    for (int j = 0; j < 3; ++j) g_scale[(size_t)j * n + i] = gs[j];
    for (int j = 0; j < 4; ++j) g_quat[(size_t)j * n + i] = gq[j];
    g_opacity[i] = go;
    for (int k = 0; k < nc * 3; ++k) g_sh[(size_t)k * n + i] = gsh[k];
    if (cond) {
      const size_t N = (size_t)n;
      for (int k = 0; k < per; ++k) cond[(size_t)k * N + i] = csum[k];
    }
    if (max_contrib) max_contrib[i] = mcv;
    if (dens_grad) dens_grad[i] = dgs;
    if (dens_cnt) dens_cnt[i] = dgc;
    if (activity) {
      TG pm = TG(0), pc = TG(0), ps = TG(0);
      for (int j = 0; j < 3; ++j) pm += gm[j] * gm[j];
      for (int k = 0; k < nc * 3; ++k) pc += gsh[k] * gsh[k];
      for (int j = 0; j < 3; ++j) {
        const TG gl = gs[j] * mg.m.scale[(size_t)j * n + i];  // d/d log s = s * d/ds
        ps += gl * gl;
      }
      activity[i] = TG(2) * std::sqrt(pm) + TG(0.1) * std::sqrt(pc) + TG(0.1) * std::sqrt(ps);
    }
  }
  return 0;
}

template <typename T, typename MS> Model<T> to_model(const MS& s) {
  Model<T> m;
  m.n = s.n; m.D = s.sh_degree;
  m.mean = s.mean; m.scale = s.scale; m.quat = s.quat; m.opacity = s.opacity; m.sh = s.sh;
  m.layer = s.layer;
  m.filter3d = s.filter_3d;
  return m;
}

}  // namespace

extern "C" {

int oracle_render_f32(int n_views, const oc_model32* models, const oc_camera* cams,
                      const oc_view* views, int tile, int brute_force, oc_outputs* out, int n_threads,
                      const oc_camera* sort_cams) {
  std::vector<Model<float>> ms;
  for (int v = 0; v < n_views; ++v) ms.push_back(to_model<float>(models[v]));
  return render<float>(n_views, ms.data(), cams, views, tile, brute_force, out, n_threads, sort_cams);
}

int oracle_render_f64(int n_views, const oc_model64* models, const oc_camera* cams,
                      const oc_view* views, int tile, int brute_force, oc_outputs* out, int n_threads,
                      const oc_camera* sort_cams) {
  std::vector<Model<double>> ms;
  for (int v = 0; v < n_views; ++v) ms.push_back(to_model<double>(models[v]));
  return render<double>(n_views, ms.data(), cams, views, tile, brute_force, out, n_threads, sort_cams);
}

int oracle_backward_f32(int n_views, const oc_model32* model, const oc_camera* cams, const oc_view* views,
                        const float* dL_drgb, const float* dL_dalpha, uint32_t trainable, float* g_mean,
                        float* g_scale, float* g_quat, float* g_opacity, float* g_sh, float* max_contrib,
                        float* activity, int n_threads, float* dens_grad, float* dens_cnt) {
  return backward<float, float>(n_views, to_model<float>(*model), cams, views, dL_drgb, dL_dalpha, trainable,
                                g_mean, g_scale, g_quat, g_opacity, g_sh, max_contrib, activity, n_threads, false,
                                nullptr, dens_grad, dens_cnt);
}

int oracle_backward_f64(int n_views, const oc_model64* model, const oc_camera* cams, const oc_view* views,
                        const double* dL_drgb, const double* dL_dalpha, uint32_t trainable, double* g_mean,
                        double* g_scale, double* g_quat, double* g_opacity, double* g_sh,
                        double* max_contrib, double* activity, int n_threads, double* dens_grad,
                        double* dens_cnt) {
  return backward<double, double>(n_views, to_model<double>(*model), cams, views, dL_drgb, dL_dalpha, trainable,
                                  g_mean, g_scale, g_quat, g_opacity, g_sh, max_contrib, activity, n_threads, false,
                                  nullptr, dens_grad, dens_cnt);
}

int oracle_backward_exact(int n_views, const oc_model32* model, const oc_camera* cams, const oc_view* views,
                          const float* dL_drgb, const float* dL_dalpha, uint32_t trainable, double* g_mean,
                          double* g_scale, double* g_quat, double* g_opacity, double* g_sh,
                          double* max_contrib, double* activity, double* cond, int fwd_values,
                          int n_threads, double* dens_grad, double* dens_cnt) {
  return backward<float, double>(n_views, to_model<float>(*model), cams, views, dL_drgb, dL_dalpha, trainable,
                                 g_mean, g_scale, g_quat, g_opacity, g_sh, max_contrib, activity, n_threads,
                                 fwd_values != 0, cond, dens_grad, dens_cnt);
}

void oracle_sh_basis_f64(const double* dir, double* out16) {
  SH<double> sh;
  sh.basis(dir[0], dir[1], dir[2], out16);
}

void oracle_sh_basis_f32(const float* dir, float* out16) {
  SH<float> sh;
  sh.basis(dir[0], dir[1], dir[2], out16);
}

}  // extern "C"
