/*
 * gsr.h - C ABI of the layered Gaussian-splat tile rasterizer (HIP, gfx950).
 *
 * The library renders scenes of anisotropic 3D Gaussians the way Gaussian
 * splatting does (the paper's renderer is "analogous to Kerbl et al.",
 * Sec. 3.3; splats are projected with the EWA approximation of Zwicker et al.
 * it cites in Sec. 2.2.1), extended with the paper's layers:
 *   - every Gaussian carries a layer id; a per-view layer-activation mask
 *     shows or hides whole layers (Sec. 1 and Sec. 3.3: only active layers
 *     are rendered);
 *   - per-layer clip planes cut through layers (Sec. 1, Sec. 5: the cut
 *     edge depends on the splat centres, so a plane removes the Gaussians
 *     of its layers whose centre lies on its negative side);
 *   - training renders frozen lower layers as background and updates only
 *     the trainable layers (Sec. 3.2), with alpha in the loss and a random
 *     background (Sec. 3.2.1), and tracks per-Gaussian activity for
 *     inactive pruning (Sec. 3.2.2).
 *
 * Pipeline per call: project (gates, EWA covariance, SH colour, tile box) ->
 * exclusive scan of tile counts -> duplicate into (tile << 32 | depth bits,
 * record) pairs -> stable LSD radix sort -> per-tile ranges -> per-tile
 * front-to-back blending (alpha = min(0.99, o exp(-q/2)), pairs below 1/255
 * skipped, stop before T would drop below 1e-4).  The backward replays the
 * blend back to front and chains to the Gaussian parameters.
 *
 * Conventions (also the CPU oracle's): OpenCV camera axes (x right, y down,
 * z forward), p_cam = R p_world + t; pixel (i, j) is sampled at
 * (i + 0.5, j + 0.5); 16 x 16 tiles; low-pass 0.3 px^2 on the 2D covariance
 * diagonal; splat extent = bounding box of {q <= 11.09375}; SH are the real
 * orthonormal harmonics with the Condon-Shortley phase, colour =
 * max(0, sum sh*Y(dir) + 0.5) with dir from the eye centre to the Gaussian.
 *
 * Memory: every array pointer is a DEVICE pointer unless marked "host".  The
 * caller owns every allocation; the library allocates nothing.  Gaussian
 * attributes are structures of arrays (one plane per component, n floats
 * each, plane-major):
 *   mean[3][n], scale[3][n] (activated, > 0), quat[4][n] (w, x, y, z; any
 *   length, normalised inside; zero culls), opacity[n] (activated, in
 *   (0, 1)), sh[(D+1)^2][3][n] (coefficient, then channel, then Gaussian),
 *   layer[n] (uint8, < 32).
 *
 * Errors: every entry point returns a gsr_status; nothing aborts or throws.
 * Arguments are validated before any launch.  Launch failures return
 * GSR_EHIP; faults inside kernels surface at the caller's next
 * synchronisation.  All work is enqueued on the caller's stream (a
 * hipStream_t passed as void*, NULL = the null stream).  Calls on distinct
 * workspaces/states may run concurrently on different streams.
 */
#ifndef GSR_H
#define GSR_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define GSR_TILE 16
#define GSR_MAX_CLIP 8
#define GSR_RECORD_FLOATS 12

typedef enum {
  GSR_OK = 0,
  GSR_EINVAL = -1,    /* bad argument (null pointer, size, degree, ...) */
  GSR_ENOSPACE = -2,  /* workspace or pair capacity too small; see the entry point */
  GSR_EHIP = -3,      /* a HIP call failed */
  GSR_EDEVICE = -4    /* a kernel reported an internal error (see gsr_forward_check) */
} gsr_status;

/* Pinhole camera (host struct). */
typedef struct {
  float R[9];          /* world -> camera rotation, row-major */
  float t[3];          /* world -> camera translation */
  float fx, fy, cx, cy;
  int32_t width, height;
  float znear;         /* Gaussians with camera depth <= znear are culled (0.2 by default) */
  float guard;         /* the Jacobian is evaluated with the centre's image-plane slope
                          clamped to guard * max(c, size - c) / f (1.3 by default) */
} gsr_camera;

/* Clip plane: for layers whose bit is set in layer_bits, a Gaussian whose
 * centre m has n.m + d < 0 is removed (Sec. 1 and Sec. 5 cutting). */
typedef struct {
  float n[3];
  float d;
  uint32_t layer_bits;
} gsr_clip_plane;

/* Per-view visibility state (host struct). */
typedef struct {
  uint32_t layer_mask;                 /* bit l set: layer l is shown */
  int32_t n_clip;                      /* 0 .. GSR_MAX_CLIP */
  gsr_clip_plane clip[GSR_MAX_CLIP];
  float bg[3];                         /* background colour composited behind the splats */
  /* Depth order of the pairs within each tile.  0: each view's own
   * camera-space depth (exact per view).  1: one order for all views of the
   * call (gsr_rasterize_forward: decided by views[0]; gsr_render_batch: by
   * the request's vs): the Gaussians are sorted once by their depth in
   * sort_cam (only its R and t are read; for stereo, the camera at the eye
   * centre), each view's pairs are emitted in that order and only grouped
   * by tile (Sec. 3.3: one sort shared by both eyes instead of one per
   * eye).  With parallel eyes and sort_cam their centre the depths agree
   * with each eye's own and the images are those of per-eye sorting; with
   * converging eyes pairs of nearly equal depth may be blended in the
   * other order.  The depth key is the bit pattern of the float depth as an
   * unsigned integer (ties: ascending Gaussian index). */
  int32_t sort_shared;
  gsr_camera sort_cam;
  /* Per-layer opacity at render time (Sec. 1: layers shown with variable
   * opacity; Sec. 5: fading between layers).  0: off.  1: a Gaussian of
   * layer l is drawn with opacity o * layer_opacity[l] (its record holds
   * that product, a product below 1/255 culls it like any too transparent
   * Gaussian, and the backward's opacity gradient is with respect to o,
   * i.e. layer_opacity[l] times that of the product).  Factors in [0, 1]. */
  int32_t layer_fade;
  float layer_opacity[32];
  /* Mip-Splatting's 2D filter (the anti-aliasing Sec. 4.4 reports trying;
   * forward only).  0: off, the screen-space covariance is dilated by 0.3 px^2.
   * 1: it is dilated by mip_2d_var px^2 instead (> 0) and the opacity is
   * multiplied by sqrt(max(det S, 0) / det(S + mip_2d_var I)), S the
   * undilated screen-space covariance (float32: det S = s00 s11 - s01 s01,
   * the quotient, its correctly rounded square root). */
  int32_t mip_2d;
  float mip_2d_var;
} gsr_view_state;

/* Compressed attributes for rendering (device arrays, structure of arrays;
 * host struct).  Sec. 4.3 renders with 16-bit floats for the point-cloud
 * parameters and either quantised spherical-harmonic coefficient triplets
 * or, "clustered", one shared set of SH coefficients per Gaussian out of a
 * K-means codebook built across all layers (Sec. 3.3).  M = (D+1)^2 - 1
 * higher coefficients per channel, D = sh_degree.  Half values are IEEE
 * binary16 bit patterns, decoded exactly (subnormals included). */
enum { GSR_FORMAT_F32 = 0, GSR_FORMAT_HALF_PACKED = 1, GSR_FORMAT_HALF_CODEBOOK = 2 };
typedef struct {
  const uint16_t* mean;     /* half[3][n] */
  const uint16_t* scale;    /* half[3][n], activated scales */
  const uint16_t* quat;     /* half[4][n], (w, x, y, z) */
  const uint16_t* opacity;  /* half[n], activated opacity */
  const uint16_t* sh_dc;    /* half[3][n]: the degree-0 coefficient of r, g, b */
  /* GSR_FORMAT_HALF_PACKED: coefficient k = 1 .. M of Gaussian i is the word
   * sh_packed[(k-1) n + i], unsigned codes q of r in bits 0-10, g in bits
   * 11-21 and b in bits 22-31; the value of channel ch is the float32
   * sh_lo[ch] + q * sh_step[ch] (the product rounded, then the sum). */
  const uint32_t* sh_packed;
  float sh_lo[3], sh_step[3];
  /* GSR_FORMAT_HALF_CODEBOOK: coefficient k = 1 .. M, channel ch of
   * Gaussian i is the half codebook[sh_index[i] S + (k - 1) 3 + ch], with
   * the entry stride S = 3M rounded up to a multiple of 8 halves (16-byte
   * entries: S = 0, 16, 24, 48 for D = 0 .. 3; the padding is not read);
   * the array is 16-byte aligned.  An index at or above codebook_size is an
   * error (the forward reads entry 0 instead and reports GSR_EDEVICE through
   * gsr_forward_check, or for every request of a gsr_render_batch call). */
  const uint16_t* sh_index; /* uint16[n] */
  const uint16_t* codebook; /* half[codebook_size][S] */
  int32_t codebook_size;    /* 1 .. 65536 */
  int32_t reserved;         /* must be 0 */
} gsr_compressed;

/* Gaussian arrays (device, structure of arrays, see above; host struct). */
typedef struct {
  int32_t n;           /* number of Gaussians, >= 0 */
  int32_t sh_degree;   /* 0 .. 3 */
  const float *mean, *scale, *quat, *opacity, *sh;
  const uint8_t* layer;
  int32_t raw;         /* 0: scale and opacity hold activated values.  1: they hold the
                          training parameters of Sec. 3.2, log-scales and opacity logits;
                          the kernels apply exp and the logistic function themselves and
                          the backward's g_scale / g_opacity are with respect to these raw
                          values. */
  int32_t format;      /* GSR_FORMAT_F32 (0): the float arrays above.  Otherwise the
                          attributes are read from *compressed (mean ... sh are not read,
                          raw must be 0); forward and batch rendering only (the backward
                          returns GSR_EINVAL).  layer is read in every format. */
  const gsr_compressed* compressed;  /* host pointer, read during the call; NULL for F32 */
  /* Mip-Splatting's 3D filter (optional, forward only; NULL: none): device
   * float[n] variances f^2.  Gaussian i is drawn with scales
   * sqrt(s_k^2 + f^2) and opacity o * sqrt((s_0^2 s_1^2) s_2^2 / ((p_0 p_1) p_2)),
   * p_k = s_k^2 + f^2 (float32, in that order, square roots correctly
   * rounded): the Gaussian convolved with an isotropic one of variance f^2. */
  const float* filter_3d;
} gsr_model;

/* Buffers that carry a forward pass to its backward (device, caller-owned;
 * host struct).  R = n_views * model.n records, P = pair_capacity,
 * X = total tiles = n_views * ceil(W/16) * ceil(H/16), Q = n_views * H * W,
 * B = batch_capacity >= P / 256 + X (see gsr_batch_capacity).
 *   records     float[R][12]  per (view, Gaussian): u, v, conic a, b, c,
 *                             opacity, r, g, b, depth, clamp bits (as uint32;
 *                             bit c = colour channel c clamped at 0), tile
 *                             count (as uint32; 0 = culled).  Record
 *                             r = v * n + i.
 *   offsets     uint32[R+1]   first pair (emission order) of each record;
 *                             offsets[R] = pair count
 *   pair_vals   uint32[2][P]  sorted record ids; which half holds the result
 *                             is recorded on the device in *sort_sel.  A
 *                             forward with checkpoints leaves in the other
 *                             half, as uint16[P], each sorted pair's mask of
 *                             the 4 x 4-pixel blocks of its tile that its
 *                             ellipse reaches (bit 4 row + column), for the
 *                             backward
 *   sort_sel    uint32[1]
 *   pair_emit   uint32[P]     emission index of each sorted pair
 *   ranges      uint32[X][2]  [start, end) of each tile's pairs
 *   pixel_state float[Q][4]   transmittance left behind the last blended
 *                             splat, then the composited colour before the
 *                             background (premultiplied r, g, b)
 *   last        uint32[Q]     1 + index of the last blended pair, 0 if none
 *   checkpoints float[B][256][4]  per 256-pair batch of a tile and pixel:
 *                             transmittance before the batch, then the
 *                             colour (r, g, b) behind the batch (the later
 *                             batches' colours plus the background times
 *                             the final transmittance); written for the
 *                             batches up to the one in which the tile's
 *                             last pixel stops (later ones are never read)
 *   batch_map   uint32[X + 1 + B]  X + 1 unused words, then for each
 *                             checkpoint batch index a word whose low 24
 *                             bits hold 1 + its tile (0: none) and whose top
 *                             byte holds the batch's work class (the
 *                             backward runs the heavier batches first);
 *                             tile t's batches have the indices
 *                             floor(ranges[t][0] / 256) + t + c
 *   counters    uint32[4]     device: pairs K, overflow flag, error flag,
 *                             reserved.  Zeroed by the caller when the state
 *                             is created.  The overflow and error words are
 *                             sticky: any call on the state may set them and
 *                             only gsr_forward_check clears them (after
 *                             reporting them), so one check after a loop of
 *                             non-synchronising calls sees every call. */
typedef struct {
  float* records;
  uint32_t* offsets;
  uint32_t* pair_vals;
  uint32_t* sort_sel;
  uint32_t* pair_emit;
  uint32_t* ranges;
  float* pixel_state;
  uint32_t* last;
  float* checkpoints;
  uint32_t* batch_map;
  uint32_t* counters;
  uint32_t pair_capacity;
  uint32_t batch_capacity;
} gsr_fwd_state;

/* Batch capacity a state needs for a pair capacity and a tile count. */
uint32_t gsr_batch_capacity(uint32_t pair_capacity, uint32_t total_tiles);

/* Optional copies of intermediate arrays for inspection (device, may all be
 * NULL; host struct).  Filled by gsr_rasterize_forward when non-NULL.  The
 * call then synchronises the stream once. */
typedef struct {
  uint32_t* n_tiles;    /* [R] tiles touched by each record */
  uint32_t* tile_box;   /* [R][4]: global id of the box's first tile, width | height << 16
                           (in tiles), depth bits, tiles per image row */
  uint64_t* keys_emit;  /* [P] keys in emission order (record order, tiles row-major) */
  uint32_t* vals_emit;  /* [P] record of each pair in emission order */
  uint64_t* keys_sorted;/* [P] */
} gsr_debug;

/* Per-stage timer (host object holding HIP events).  When a timer is passed
 * to an entry point, the library records an event pair on the caller's
 * stream around each stage it launches; gsr_timer_read synchronises on the
 * recorded events, returns the summed milliseconds and launch counts per
 * stage since the last read, and starts a new accumulation.  Recording adds
 * two event records per stage and call.  A timer must not be used from two
 * threads at once. */
typedef struct gsr_timer gsr_timer;
enum {
  GSR_STAGE_PROJECT = 0,
  GSR_STAGE_SCAN,
  GSR_STAGE_DUPLICATE,
  GSR_STAGE_SORT,
  GSR_STAGE_RANGES,
  GSR_STAGE_BLEND,
  GSR_STAGE_BLEND_BWD,     /* the backward blend kernel alone */
  GSR_STAGE_PROJECT_BWD,
  GSR_STAGE_BWD_ORDER,     /* the backward's ordering of batches, heaviest first */
  GSR_N_STAGES
};
gsr_status gsr_timer_create(gsr_timer** out);
void gsr_timer_destroy(gsr_timer* t);
gsr_status gsr_timer_read(gsr_timer* t, float* ms /* [GSR_N_STAGES] */, uint32_t* calls /* [GSR_N_STAGES] */);

/* Bytes of scratch workspace a forward or backward of n_views views of a
 * model with n Gaussians at width x height needs, for a pair capacity of
 * pair_capacity; shared_order != 0 adds the buffers of a forward with a
 * shared depth order (gsr_view_state.sort_shared: about 24 B per Gaussian
 * and 24 B per record more).  Returns 0 on bad arguments. */
size_t gsr_workspace_size(int32_t n, int32_t n_views, int32_t width, int32_t height,
                          uint32_t pair_capacity, int32_t shared_order);

/* The activated scale float[3][n] and opacity float[n] of a model exactly as
 * the kernels compute them: for model->raw = 1, exp of the log-scales and
 * the logistic function of the logits (Sec. 3.2 parameters); for raw = 0 a
 * copy.  Outputs are device arrays the caller owns.  Returns GSR_EINVAL on
 * bad arguments or a compressed model; asynchronous on stream. */
gsr_status gsr_activate(const gsr_model* model, float* scale_out, float* opacity_out, void* stream);

/* Forward render of n_views views of one model, all at the same resolution
 * (cams[v].width/height equal).  cams and views are host arrays of n_views.
 *   rgb   float[V][3][H][W]  colour composited over views[v].bg
 *   alpha float[V][H][W]     1 - final transmittance
 * The state is filled for gsr_rasterize_backward.
 * n_pairs_host: if non-NULL, the call synchronises the stream after the
 * tile-count scan, stores the exact pair count K there and returns
 * GSR_ENOSPACE without rendering when K > state->pair_capacity, or
 * GSR_EDEVICE without rendering when the state's error word is set (by this
 * call's scan or an earlier unchecked call; gsr_forward_check clears it).
 * If NULL the call never synchronises; on overflow the pairs beyond the
 * capacity are dropped, state->counters[1] is set and the image is
 * incomplete - check with gsr_forward_check after synchronising.
 * ws: scratch of at least gsr_workspace_size(...) bytes, 256-byte aligned.
 * timer: optional (NULL), see gsr_timer.  GSR_EINVAL when the total tile
 * count X is 2^24 - 1 or more (the batch map holds tiles in 24 bits).
 * With views[0].sort_shared the views share one depth order (see
 * gsr_view_state); the workspace must then be sized with shared_order set,
 * and the state can not be used for a backward. */
gsr_status gsr_rasterize_forward(const gsr_model* model, int32_t n_views, const gsr_camera* cams,
                                 const gsr_view_state* views, gsr_fwd_state* state,
                                 void* ws, size_t ws_bytes, float* rgb, float* alpha,
                                 uint32_t* n_pairs_host, const gsr_debug* debug, gsr_timer* timer,
                                 void* stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid allocation): the
 * forward of gsr_rasterize_forward (same arguments and results, no debug
 * copies, no timer) without a workspace argument.  Its scratch is a device
 * array of GSR_NOALLOC_SCRATCH_BYTES inside the library, one per GPU, held
 * until the process ends; its address is looked up on the first call on a
 * device (the device current at the call, which must own `stream`).  The
 * call allocates nothing.  Returns GSR_ENOSPACE, before any launch, when
 * the forward's scratch for these sizes (records n * n_views, the state's
 * pair capacity, the tiles of the views) exceeds that size: about 28 MB
 * for 200k Gaussians at 800 x 800 with 1M pair slots.  Every call on a GPU
 * shares its array, so calls that overlap on one GPU (other streams, other
 * threads) race and must be serialised by the caller; each call clears
 * what it needs zeroed itself (with a kernel, no memset node).  The state
 * it fills is the same as gsr_rasterize_forward's: gsr_rasterize_backward
 * takes it with its own workspace. */
#define GSR_NOALLOC_SCRATCH_BYTES (64u << 20)
gsr_status gsr_rasterize_forward_noalloc(const gsr_model* model, int32_t n_views, const gsr_camera* cams,
                                         const gsr_view_state* views, gsr_fwd_state* state, float* rgb,
                                         float* alpha, uint32_t* n_pairs_host, void* stream);

/* After non-synchronising forwards have completed (caller synchronised):
 * reads state->counters and returns GSR_OK, GSR_ENOSPACE (the pair capacity
 * was exceeded by some call since the last check; *n_pairs_host receives
 * the last call's count) or GSR_EDEVICE (a kernel reported an internal
 * error: a bounded wait gave up, or offsets and keys were inconsistent),
 * then clears the overflow and error words.  Synchronises the stream. */
gsr_status gsr_forward_check(const gsr_fwd_state* state, uint32_t* n_pairs_host, void* stream);

/* Gradients of a loss L given dL/d(rgb) float[V][3][H][W] and dL/d(alpha)
 * float[V][H][W] (either may be NULL = zero), for the forward whose state
 * is passed (same model, cameras and views).  Gradients are with respect
 * to the activated parameters (to the raw ones if model->raw) and
 * OVERWRITE grads (same layout as the
 * model arrays): g_mean[3][n], g_scale[3][n], g_quat[4][n], g_opacity[n],
 * g_sh[(D+1)^2][3][n].  Gaussians whose layer bit is clear in
 * trainable_layers receive zero (frozen layers, Sec. 3.2).
 * max_contrib float[n] (optional): max-accumulated with the largest
 *   alpha * T each Gaussian reached on any pixel (caller zeroes it to start
 *   an accumulation window).
 * activity float[n] (optional): accumulated (+=) with
 *   2 |dL/dmean| + 0.1 |dL/dsh| + 0.1 |dL/dlog scale| (Sec. 3.2.2).
 * grads->densify_grad, grads->densify_count float[n] (optional, NULL:
 *   not tracked): accumulated (+=) with the statistic of adaptive density
 *   control - per trainable Gaussian and view in which it covers at least
 *   one tile, the length of the gradient with respect to its projected
 *   centre in normalised device coordinates, |(dL/du W/2, dL/dv H/2)| (u, v
 *   in pixels), and 1 for the view.
 * ws: scratch of at least gsr_workspace_size(...) bytes.
 * The backward uses no atomics: per-pair partial gradients are summed in a
 * fixed order, so repeated calls give bitwise identical results.
 * GSR_EINVAL for views with a shared depth order (a rendering
 * approximation; training differentiates each view's own order). */
typedef struct {
  float *g_mean, *g_scale, *g_quat, *g_opacity, *g_sh;
  float *densify_grad, *densify_count;  /* optional accumulators, see above */
} gsr_grads;

gsr_status gsr_rasterize_backward(const gsr_model* model, int32_t n_views, const gsr_camera* cams,
                                  const gsr_view_state* views, const gsr_fwd_state* state,
                                  const float* dL_drgb, const float* dL_dalpha,
                                  uint32_t trainable_layers, void* ws, size_t ws_bytes,
                                  const gsr_grads* grads, float* max_contrib, float* activity,
                                  gsr_timer* timer, void* stream);

/* One render request of a batch (host struct): one or two views (stereo)
 * of models[model] sharing one view state, each written to its own
 * rgb float[3][H][W] and alpha float[H][W] (device).  Views of one request
 * may differ in resolution. */
typedef struct {
  int32_t model;
  int32_t n_views;          /* 1 or 2 */
  gsr_camera cam[2];
  gsr_view_state vs;
  float* rgb[2];
  float* alpha[2];
} gsr_request;

/* Bytes of workspace gsr_render_batch needs for these requests at a total
 * pair capacity of pair_capacity (0 on bad arguments). */
size_t gsr_batch_workspace_size(const gsr_model* models, int32_t n_models, const gsr_request* reqs,
                                int32_t n_req, uint32_t pair_capacity);

/* Render a batch of requests over resident models in one pass: one
 * projection per (model, its views), one sort over a shared tile space, one
 * blend launch over every tile of every view.  Never
 * synchronises.  req_status int32[n_req] (device) receives GSR_OK, or
 * GSR_ENOSPACE for requests whose pairs did not fit into pair_capacity
 * (their images are not written; pairs are assigned in request order, so
 * the failing requests are a suffix), or GSR_EDEVICE for every request when
 * a kernel of the call reported an internal error.  Each request's image is
 * identical to rendering it alone. */
gsr_status gsr_render_batch(const gsr_model* models, int32_t n_models, const gsr_request* reqs,
                            int32_t n_req, uint32_t pair_capacity, void* ws, size_t ws_bytes,
                            int32_t* req_status, gsr_timer* timer, void* stream);

/* One Adam step on the parameters of the Gaussians of the trainable layers
 * (Sec. 3.2: earlier layers are frozen while a layer trains; their
 * gradients are zero, so Adam leaves them unchanged: they are skipped and
 * none of their values is read or written).  groups[5] are, in order, the
 * mean [3][n], log-scale [3][n], quaternion [4][n], opacity logit [n] and
 * SH [(D+1)^2][3][n] planes, each with its gradient, first and second
 * moments (same layout) and learning rate.  Per value, t = step >= 1:
 *   m <- m + (1 - beta1) (g - m);  v <- beta2 v + (1 - beta2) g^2;
 *   p <- p - lr / (1 - beta1^t) * m / (sqrt(v) / sqrt(1 - beta2^t) + eps)
 * in float32.  activity (optional, float[n]): accumulated with the step's
 * update-norm activity, as gsr_update_activity defines it from the values
 * before and after.  Device arrays; asynchronous on stream; GSR_EINVAL on a
 * NULL array, a bad size, degree, step or hyper-parameter. */
typedef struct {
  float* param;
  const float* grad;
  float* exp_avg;
  float* exp_avg_sq;
  float lr;
} gsr_adam_group;
gsr_status gsr_adam_step(int32_t n, int32_t sh_degree, uint32_t trainable_layers, const uint8_t* layer,
                         const gsr_adam_group* groups, float beta1, float beta2, float eps, int32_t step,
                         float* activity, void* stream);

/* Inactive-pruning activity from one optimiser step (Sec. 3.2.2 tracks the
 * optimisation of each Gaussian's position, colour and scale and removes
 * Gaussians whose activity over a pruning window stays at or below a
 * threshold).  For every Gaussian whose layer bit is set in
 * trainable_layers,
 *   activity[i] += 2 |d mean_i| + 0.1 |d sh_i| + 0.1 |d log_scale_i|,
 * d = after - before of the step and |.| the Euclidean norm over the
 * Gaussian's 3, 3 (D+1)^2 and 3 values (float32, one thread per Gaussian;
 * other Gaussians untouched).
 *   mean_before/after       float[3][n]
 *   log_scale_before/after  float[3][n]
 *   sh_before/after         float[(D+1)^2][3][n], D = sh_degree <= 3
 *   layer uint8[n]; activity float[n], accumulated
 * Device arrays the caller owns; asynchronous on stream; GSR_EINVAL on a
 * NULL array (n > 0) or a bad size or degree. */
gsr_status gsr_update_activity(int32_t n, int32_t sh_degree, uint32_t trainable_layers, const float* mean_before,
                               const float* mean_after, const float* log_scale_before, const float* log_scale_after,
                               const float* sh_before, const float* sh_after, const uint8_t* layer, float* activity,
                               void* stream);

/* L1 loss of alpha-channel training (Sec. 3.2.1) and its gradient.  Per
 * view v the target colour is the target's premultiplied colour composited
 * over the view's background bg_v: target = target_rgb + (1 - target_alpha)
 * bg_v, and L = mean |rgb - target| + mean |alpha - target_alpha| (means over
 * the n_views x 3 x H x W colour and n_views x H x W alpha values).
 *   rgb, target_rgb     float[n_views][3][H][W]
 *   alpha, target_alpha float[n_views][H][W]
 *   bg_host             host float[n_views][3]; n_views <= 16
 *   loss                float[1] (NULL: loss not computed)
 *   g_loss              float[1] incoming gradient of L (NULL: 1)
 *   dL_drgb, dL_dalpha  overwritten with sign(d) g / N (both NULL: no
 *                       gradient); d the difference, N the value count
 *   ws                  gsr_l1_loss_workspace_size bytes (block partial
 *                       sums); one call at a time per ws.
 * The loss is reduced in a fixed order (bitwise reproducible). */
size_t gsr_l1_loss_workspace_size(int32_t n_views, int32_t width, int32_t height);
gsr_status gsr_l1_alpha_loss(int32_t n_views, int32_t width, int32_t height, const float* rgb, const float* alpha,
                             const float* target_rgb, const float* target_alpha, const float* bg_host, void* ws,
                             size_t ws_bytes, float* loss, const float* g_loss, float* dL_drgb, float* dL_dalpha,
                             void* stream);

/* Human-readable name of a status. */
const char* gsr_status_string(gsr_status s);

#ifdef __cplusplus
}
#endif
#endif /* GSR_H */
