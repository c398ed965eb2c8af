/*
 * CPU oracle for the layered Gaussian-splat tile rasterizer.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path links or calls this
 * library; only the tests, the smoke check and the benchmark's CPU-baseline
 * leg do.  It shares no code with the GPU path.
 *
 * Plain, slow, obviously correct reference of what the rasterizer computes:
 * EWA splat projection (Zwicker et al., cited in Sec. 2.2.1), view-dependent
 * spherical-harmonic colour, the paper's per-layer visibility and cutting
 * (Sec. 1, Sec. 3.3, Sec. 5), tile/depth keys, a stable sort, per-pixel
 * front-to-back alpha compositing and its exact gradient.  Every function is
 * instantiated in float (parity) and double (finite differences).
 *
 * Conventions are the readings listed in the design notes:
 *  - pixel (i, j) is sampled at (i + 0.5, j + 0.5);
 *  - low-pass kappa = 0.3 px^2 on the 2D covariance diagonal;
 *  - splat extent: axis-aligned box of {q <= 11.09375};
 *  - alpha = min(0.99, o * exp(-q/2)); pairs with alpha < 1/255 are skipped;
 *    blending stops before a Gaussian that would bring T below 1e-4;
 *  - keys: (view tile offset + tile id) << 32 | bits(depth); stable sort.
 *
 * All pointers are host pointers; the caller owns every buffer.
 */
#ifndef GSR_ORACLE_H
#define GSR_ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct {
  float R[9];       /* world -> camera rotation, row-major */
  float t[3];       /* world -> camera translation */
  float fx, fy, cx, cy;
  int32_t width, height;
  float znear;      /* cull t_z <= znear */
  float guard;      /* Jacobian guard band, in units of the half field of view */
} oc_camera;

typedef struct {
  float n[3];
  float d;
  uint32_t layer_bits;  /* plane applies to layers whose bit is set */
} oc_clip;

typedef struct {
  uint32_t layer_mask;
  int32_t n_clip;
  oc_clip clip[8];
  float bg[3];
  /* per-layer opacity (layers shown at variable opacity, Sec. 1; fading
   * between layers, Sec. 5): when layer_fade is non-zero a Gaussian of layer
   * l is drawn with opacity o * layer_opacity[l]; zero leaves o alone */
  int32_t layer_fade;
  float layer_opacity[32];
  /* Mip-Splatting's 2D filter (forward only): when mip_2d is non-zero the
   * screen-space covariance S is dilated by mip_2d_var instead of 0.3 and the
   * opacity multiplied by sqrt(max(det S, 0) / det(S + mip_2d_var I)).  A
   * model's filter_3d (variances f^2) widens each scale to sqrt(s^2 + f^2)
   * and multiplies the opacity by sqrt(prod s^2 / prod (s^2 + f^2)).  The
   * backward rejects both. */
  int32_t mip_2d;
  float mip_2d_var;
} oc_view;

/* Gaussian arrays, structure of arrays.  mean[3][n], scale[3][n] (activated),
 * quat[4][n] (w,x,y,z), opacity[n] (activated), sh[(D+1)^2][3][n], layer[n]. */
typedef struct {
  int32_t n, sh_degree;
  const float *mean, *scale, *quat, *opacity, *sh;
  const uint8_t* layer;
  const float* filter_3d;  /* optional Mip-Splatting 3D filter variances [n], or NULL */
} oc_model32;

typedef struct {
  int32_t n, sh_degree;
  const double *mean, *scale, *quat, *opacity, *sh;
  const uint8_t* layer;
  const double* filter_3d;
} oc_model64;

/* Outputs of a render; every pointer may be NULL.  Views are concatenated in
 * call order: record r = (sum of n over earlier views) + i; pixel arrays are
 * per view [3][H][W] / [H][W]; tiles are numbered globally. */
typedef struct {
  void* rgb;            /* T[sum 3*H*W] */
  void* alpha;          /* T[sum H*W]   */
  void* final_T;        /* T[sum H*W]   */
  uint32_t* last;       /* [sum H*W] 1 + index (into the sorted pairs) of the last blended pair, 0 if none */
  uint32_t* n_contrib;  /* [sum H*W] number of blended pairs */
  float* margin;        /* [sum H*W] distance of the pixel's closest threshold decision, in units of
                           that decision's tolerance (< 1: near a threshold) */
  void* rec;            /* T[sum n][10]: u, v, conic_a, conic_b, conic_c, opacity, depth, r, g, b */
  int32_t* rect;        /* [sum n][4]: x0, y0, x1, y1 (tiles, end exclusive) */
  uint32_t* n_tiles;    /* [sum n] */
  uint32_t* clamp;      /* [sum n] bit c set when colour channel c was clamped at 0 */
  uint64_t* keys_emit;  /* [pair_cap] keys in emission order */
  uint32_t* vals_emit;  /* [pair_cap] */
  uint64_t* keys;       /* [pair_cap] sorted */
  uint32_t* vals;       /* [pair_cap] sorted */
  uint64_t pair_cap;
  uint32_t* ranges;     /* [total_tiles][2] start, end */
  uint64_t counts[4];   /* out: pairs K, evaluated pairs E, blended pairs A, total tiles */
  uint8_t* near_rec;    /* [sum n] zeroed by the caller; set to 1 for a record with a threshold decision
                           below margin 1 at some pixel */
} oc_outputs;

/* Render n_views views; view v renders models[v] with cams[v] and views[v].
 * tile: tile edge in pixels (8, 16 or 32).  brute_force != 0 ignores the
 * tiles and blends, per pixel, every surviving Gaussian sorted by
 * (depth key, index).  The depth key of a Gaussian is the bit pattern, as
 * an unsigned integer, of its camera-space depth: in the view's camera, or,
 * when sort_cams is non-NULL, in sort_cams[v] (only R and t are used; the
 * eyes of a stereo frame given the same centre camera share one depth
 * order, Sec. 3.3).  Returns 0, or -1 on bad arguments, -2 if pair_cap is
 * too small for the requested pair arrays (counts[0] then holds K). */
int oracle_render_f32(int n_views, const oc_model32* models, const oc_camera* cams,
                      const oc_view* views, int tile, int brute_force, oc_outputs* out,
                      int n_threads, const oc_camera* sort_cams);
int oracle_render_f64(int n_views, const oc_model64* models, const oc_camera* cams,
                      const oc_view* views, int tile, int brute_force, oc_outputs* out,
                      int n_threads, const oc_camera* sort_cams);

/* Gradients of L = sum(dL_drgb * rgb) + sum(dL_dalpha * alpha) over n_views
 * views of ONE model, with respect to the activated parameters.  Gaussians
 * whose layer bit is clear in trainable_layers get zero gradient.
 * g_mean[3][n], g_scale[3][n], g_quat[4][n], g_opacity[n], g_sh[(D+1)^2][3][n]
 * are overwritten.  max_contrib[n] (optional) receives the largest
 * alpha * T of each Gaussian over all pixels and views (alpha the Gaussian's
 * opacity at the pixel, T the transmittance in front of it); activity[n]
 * (optional) receives 2|g_mean| + 0.1|g_sh| + 0.1|g_log_scale|.
 * _f32 / _f64: forward and gradient in that precision.  _exact: the float32
 * forward (records, pair lists and every per-pixel decision exactly as
 * oracle_render_f32 takes them) with every quantity of the gradient
 * evaluated in double from the float32 records - the gradient of the
 * float32 forward without the float32 rounding of the backward itself.
 * fwd_values != 0 (_exact only): the blended pairs' pixel offsets, G, alpha
 * and transmittances are the float32 forward's own values, and only the
 * arithmetic after them is in double; the difference to fwd_values = 0 is
 * what the float32 rounding of those per-pixel values does to each entry.
 * cond (_exact only, optional, [(11 + 3 (D+1)^2) n] packed mean[3][n],
 * scale[3][n], quat[4][n], opacity[n], sh[(D+1)^2*3][n]): per entry, the
 * sum over its 2D screen-space slots (u, v, conic a, b, c, opacity, r, g,
 * b) of |d entry / d slot| times the sum over pixels of the magnitudes of
 * the slot's per-pixel terms (dL/dalpha taken as the sum of the magnitudes
 * of its operands), each weighted by its pixel's number of blended pairs
 * + 16: the scale of the error that float32 per-pixel arithmetic (whose
 * transmittance carries one rounding per pair) leaves on the entry.
 * dens_grad[n], dens_cnt[n] (optional): the statistic of adaptive density
 * control - over the views in which the Gaussian is visible (covers at
 * least one tile), the sum of the lengths of the gradient with respect to
 * its projected centre in normalised device coordinates ((dL/du W/2,
 * dL/dv H/2), pixels u, v) and the number of those views; zero for frozen
 * layers. */
int oracle_backward_f32(int n_views, const oc_model32* model, const oc_camera* cams,
                        const oc_view* views, const float* dL_drgb, const float* dL_dalpha,
                        uint32_t trainable_layers, float* g_mean, float* g_scale, float* g_quat,
                        float* g_opacity, float* g_sh, float* max_contrib, float* activity,
                        int n_threads, float* dens_grad, float* dens_cnt);
int oracle_backward_f64(int n_views, const oc_model64* model, const oc_camera* cams,
                        const oc_view* views, const double* dL_drgb, const double* dL_dalpha,
                        uint32_t trainable_layers, double* g_mean, double* g_scale, double* g_quat,
                        double* g_opacity, double* g_sh, double* max_contrib, double* activity,
                        int n_threads, double* dens_grad, double* dens_cnt);
int oracle_backward_exact(int n_views, const oc_model32* model, const oc_camera* cams,
                          const oc_view* views, const float* dL_drgb, const float* dL_dalpha,
                          uint32_t trainable_layers, double* g_mean, double* g_scale, double* g_quat,
                          double* g_opacity, double* g_sh, double* max_contrib, double* activity,
                          double* cond, int fwd_values, int n_threads, double* dens_grad,
                          double* dens_cnt);

/* Real spherical-harmonic basis values Y_k(dir) for k < 16 (degree <= 3),
 * float and double, for the orthonormality check. */
void oracle_sh_basis_f64(const double* dir, double* out16);
void oracle_sh_basis_f32(const float* dir, float* out16);

#ifdef __cplusplus
}
#endif
#endif
