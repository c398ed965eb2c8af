// Shared device-side definitions of the HIP rasterizer (gfx950, wave64).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace gsr {

constexpr int kTile = 16;
constexpr int kMaxClip = 8;
constexpr int kRecordFloats = 12;     // 48-byte splat record
constexpr int kMaxJobViews = 16;      // views projected per attribute read
constexpr int kMaxSortPasses = 8;     // 64-bit keys, 8-bit digits
constexpr int kSortThreads = 512;
constexpr int kSortWaves = kSortThreads / 64;
constexpr int kSortItems = 8;         // per thread
constexpr int kSortTile = kSortThreads * kSortItems;
constexpr int kBatch = 256;          // pairs per blend batch (one per thread of a tile block)
constexpr uint32_t kTileClasses = 34;  // tile size classes of the forward's largest-first order
// Work classes of the backward's batches (heaviest first; the last class holds
// the batches the forward never reached), kept in the top byte of the
// batch-to-tile words; the low 24 bits hold 1 + tile.
constexpr uint32_t kBatchClasses = 17;
constexpr uint32_t kBatchTileMask = 0xFFFFFFu;
constexpr uint32_t kSegWaveMax = 512;  // tiles with more pairs are depth-sorted by a whole block
constexpr int kScanThreads = 256;
constexpr int kScanItems = 16;
constexpr int kScanTile = kScanThreads * kScanItems;

// Thresholds of the compositing rule.
constexpr float kAlphaMax = 0.99f;
constexpr float kAlphaMin = 1.0f / 255.0f;
constexpr float kTStop = 1e-4f;
constexpr float kKappa = 0.3f;        // px^2 low-pass on the 2D covariance diagonal
constexpr float kQMax = 11.09375f;    // extent: box of {q <= kQMax}; > 2 ln 255

// counters[] slots
constexpr int kCntPairs = 0;
constexpr int kCntOverflow = 1;
constexpr int kCntError = 2;
constexpr int kCntReserved = 3;

struct ClipD {
  float n[3];
  float d;
  uint32_t bits;
};

// One rendered view as the kernels see it (device copy).
struct ViewD {
  float R[9], t[3];
  float fx, fy, cx, cy, znear, guard;
  int32_t W, H, tiles_x, tiles_y;
  uint32_t tile_off;   // first global tile id of the view
  uint32_t rec_off;    // first record id of the view
  uint32_t model;      // index of the model the view renders
  uint32_t request;    // request index (batch) or 0
  uint32_t layer_mask;
  int32_t n_clip;
  ClipD clip[kMaxClip];
  float bg[3];
  float* rgb;          // [3][H][W]
  float* alpha;        // [H][W]
  float* pix;          // [H][W][4]: final transmittance, colour before the background
  uint32_t* last;      // [H][W]
  // Depth order of a call that sorts Gaussians before pairing them (one
  // order shared by the eyes of a stereo frame, Sec. 3.3): kSortNone in the
  // per-tile path; a sort unit's records take slots [sort_off, sort_off + n)
  // of the Gaussian sort, keyed by (sort_unit, depth) with the depth its own
  // (kSortOwn) or the sort camera's, sort_r . mean + sort_t (kSortCamera); a
  // follower (kSortFollow) takes the order of view sort_lead.
  uint32_t sort_mode;
  uint32_t sort_unit;
  uint32_t sort_off;
  uint32_t sort_lead;
  float sort_r[3];
  float sort_t;
  float layer_op[32];  // opacity factor per layer (1 when the view has no fading)
  uint32_t mip_2d;     // Mip-Splatting 2D filter: dilation mip_var, opacity compensated
  float mip_var;
};
constexpr uint32_t kSortNone = 0, kSortOwn = 1, kSortCamera = 2, kSortFollow = 3;

constexpr int kFmtF32 = 0, kFmtHalfPacked = 1, kFmtHalfCodebook = 2;
struct ModelD {
  int32_t n, D;
  const float *mean, *scale, *quat, *opacity, *sh;
  const uint8_t* layer;
  int32_t raw;  // scale / opacity hold log-scales / logits
  int32_t fmt;  // kFmt*: where the attributes live
  // compressed attributes (half bit patterns), see gsr_compressed
  const uint16_t *h_mean, *h_scale, *h_quat, *h_opacity, *h_dc;
  const uint32_t* sh_packed;
  const uint16_t *sh_index, *codebook;
  float sh_lo[3], sh_step[3];
  uint32_t codebook_size;
  const float* filter_3d;  // Mip-Splatting 3D filter variances, or null
};

// Parameter activations of raw models: scale = exp(log-scale), opacity =
// logistic(logit) (Sec. 3.2 training parameters).
__device__ __forceinline__ float act_scale(float v, int32_t raw) { return raw ? expf(v) : v; }
__device__ __forceinline__ float act_opacity(float v, int32_t raw) { return raw ? 1.0f / (1.0f + expf(-v)) : v; }

// A model together with the (up to kMaxJobViews) views that render it; the
// projection reads each Gaussian's attributes once per job.
struct JobD {
  ModelD m;
  int32_t n_views;
  int32_t view[kMaxJobViews];
};


__host__ __device__ inline uint32_t div_up(uint32_t a, uint32_t b) { return (a + b - 1) / b; }

// Wave64 inclusive scans with DPP: Hillis-Steele within each 16-lane row
// (row_shr 1, 2, 4, 8), then row_bcast:15 and row_bcast:31 carry row totals
// into the rows above.  Lanes whose DPP source is outside the row, or whose
// row is masked off, receive the identity.
// Size class of a tile with n pairs (the forward's largest-first order).
__device__ __forceinline__ uint32_t tile_class(uint32_t n) {
  // half-octave classes, largest first: class 0 holds n >= 2^16, class
  // kTileClasses - 2 holds n = 1, the last class the empty tiles
  if (n == 0) return kTileClasses - 1;
  const uint32_t lg = 31u - (uint32_t)__clz(n);
  const uint32_t h = 2u * lg + ((lg > 0 && ((n >> (lg - 1)) & 1u)) ? 1u : 0u);  // floor(2 log2 n)
  return h >= 32u ? 0u : 32u - h;
}

__device__ __forceinline__ uint32_t wave_scan_add(uint32_t x) {
  x += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x111, 0xF, 0xF, false);
  x += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x112, 0xF, 0xF, false);
  x += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x114, 0xF, 0xF, false);
  x += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x118, 0xF, 0xF, false);
  x += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x142, 0xA, 0xF, false);
  x += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x143, 0xC, 0xF, false);
  return x;
}

// Bitwise OR over the wave, returned to every lane.
__device__ __forceinline__ uint32_t wave_or(uint32_t x) {
  x |= (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x111, 0xF, 0xF, false);
  x |= (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x112, 0xF, 0xF, false);
  x |= (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x114, 0xF, 0xF, false);
  x |= (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x118, 0xF, 0xF, false);
  x |= (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x142, 0xA, 0xF, false);
  x |= (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x143, 0xC, 0xF, false);
  return (uint32_t)__builtin_amdgcn_readlane((int)x, 63);
}

}  // namespace gsr

// ---------------------------------------------------------------------------
// Launchers (host side, defined in the .hip files).  All enqueue on `s`.
namespace gsr {

constexpr int kClearRanges = 12;
struct ClearSet {
  uint32_t* p[kClearRanges];
  size_t n[kClearRanges];
  int n_ranges;
};
// Small host data (view descriptions) carried in the kernel arguments of
// the clear launch instead of a host-to-device copy.
constexpr int kUploadWords = 4 * (int)(sizeof(ViewD) / 4);
struct WordUpload {
  uint32_t* dst;
  uint32_t n;
  uint32_t w[kUploadWords];
};
hipError_t launch_clear_multi(const ClearSet& cs, hipStream_t s, const WordUpload* up = nullptr);
hipError_t launch_upload(uint32_t* dst, const void* src, size_t n_words, hipStream_t s);
hipError_t launch_activate(const ModelD& m, float* scale_out, float* opacity_out, hipStream_t s);
hipError_t launch_clear_u32(uint32_t* p, size_t n, hipStream_t s);
hipError_t launch_project(const JobD& job, const ViewD* views_dev, float* records, uint32_t* n_tiles,
                          uint4* tile_box, uint64_t* sort_keys, uint32_t* sort_vals, uint32_t* counters,
                          hipStream_t s);
uint32_t scan_tiles(uint32_t n);
hipError_t launch_scan(const uint32_t* in, uint32_t* out, uint64_t* status, uint32_t* ticket, uint32_t n,
                       uint32_t* counters, uint32_t pair_capacity, hipStream_t s);
hipError_t launch_duplicate(const uint32_t* n_tiles, const uint32_t* offsets, const uint4* tile_box,
                            uint32_t n_rec, const uint32_t* counters, uint32_t pair_capacity,
                            uint64_t* keys, uint32_t* vals, uint32_t* rec_of, hipStream_t s,
                            const uint32_t* rec_map = nullptr);
hipError_t launch_set_u32(uint32_t* p, uint32_t value, hipStream_t s);
hipError_t launch_seq_build(const ViewD* views_dev, int n_views, uint32_t n_rec, const uint64_t* sk_a,
                            const uint64_t* sk_b, const uint32_t* sv_a, const uint32_t* sv_b, const uint32_t* sel,
                            uint32_t n_sort, const uint32_t* n_tiles, const uint4* tile_box, uint32_t* seq_rec,
                            uint32_t* n_tiles_seq, uint4* tile_box_seq, uint32_t* counters, hipStream_t s);
hipError_t launch_finalize_pairs(uint32_t* vals_a, uint32_t* vals_b, const uint64_t* keys_a, const uint64_t* keys_b,
                                 const uint32_t* sel, const uint32_t* rec_of, const uint32_t* counters,
                                 uint32_t pair_capacity, uint32_t* emit, uint64_t* keys_out, hipStream_t s);
hipError_t launch_sort(uint64_t* keys_a, uint64_t* keys_b, uint32_t* vals_a, uint32_t* vals_b,
                       const uint32_t* counters, uint32_t pair_capacity, int pass_begin, int pass_end,
                       uint32_t* hist, uint32_t* status, uint32_t* pass_ctr, uint32_t* sel_out,
                       uint32_t* error_flag, hipStream_t s, const uint32_t* sel_in = nullptr);
size_t sort_status_stride(uint32_t pair_capacity);
constexpr uint32_t kXcds = 8;  // accelerator dies per MI355X, each with its own L2
constexpr uint32_t kT12MaxPairs = 1u << 24;  // the one-pass tile grouping keeps per-block tile counts: 4 B per pair slot
bool tile_sort12(uint64_t total_tiles, uint32_t pair_capacity);
size_t tile_sort12_status_words(uint32_t pair_capacity);
hipError_t launch_tile_sort12(uint64_t* keys_a, uint64_t* keys_b, uint32_t* vals_a, uint32_t* vals_b,
                              const uint32_t* counters, uint32_t pair_capacity, uint32_t total_tiles,
                              uint32_t* totals, uint32_t* block_counts, uint32_t* ranges, uint32_t* class_count,
                              uint32_t* class_list, uint32_t* sel_out, uint32_t* error_flag, hipStream_t s);
hipError_t launch_sort_segments(uint64_t* keys_a, uint64_t* keys_b, uint32_t* vals_a, uint32_t* vals_b,
                                const uint32_t* sel, const uint32_t* ranges, uint32_t total_tiles,
                                const uint32_t* rec_of, const uint32_t* counters, uint32_t pair_capacity,
                                uint32_t* emit, uint64_t* keys_out, const uint32_t* class_count,
                                const uint32_t* class_list, uint32_t* seg_ticket, uint32_t* error_flag,
                                hipStream_t s);
hipError_t launch_tile_order(const uint32_t* ranges, uint32_t n_tiles, uint32_t* class_count,
                             uint32_t* class_list, hipStream_t s);
hipError_t launch_ranges(const uint64_t* keys_a, const uint64_t* keys_b, const uint32_t* sel,
                         uint32_t* counters, uint32_t pair_capacity, uint32_t total_tiles, uint32_t* ranges,
                         hipStream_t s);
hipError_t launch_blend_fwd_tile(const ViewD* views_dev, int n_views, uint32_t total_tiles, const float* records,
                                 uint32_t n_rec, const uint32_t* pair_vals, const uint32_t* sel, uint32_t cap,
                                 const uint32_t* ranges, uint32_t* batch_tile, uint32_t batch_cap,
                                 const int32_t* req_status, float4* ckpt, const uint32_t* class_count,
                                 const uint32_t* class_list, hipStream_t s);
uint32_t l1_loss_blocks(int n_views, int hw);
hipError_t launch_l1_loss(int n_views, int hw, const float* rgb, const float* alpha, const float* t_rgb,
                          const float* t_alpha, const float* bg_host, float* partials, float* loss,
                          const float* g_loss, float* dL_drgb, float* dL_dalpha, hipStream_t s);
// Adam over the parameter groups of a model: mean, log-scale, quaternion,
// opacity logit, SH (in that order), each planes x n floats.
constexpr int kAdamGroups = 5;
struct AdamGroupD {
  float *p, *m, *v;
  const float* grad;
  int32_t planes;
  float step_size;  // lr / (1 - beta1^t)
};
struct AdamArgs {
  AdamGroupD g[kAdamGroups];
  float one_minus_b1, b2, one_minus_b2, bc2_sqrt, eps;
};
hipError_t launch_adam(int n, const AdamArgs& a, const uint8_t* layer, uint32_t trainable, float* activity,
                       hipStream_t s);
hipError_t launch_update_activity(int n, int sh_degree, uint32_t trainable, const float* mean0, const float* mean1,
                                  const float* ls0, const float* ls1, const float* sh0, const float* sh1,
                                  const uint8_t* layer, float* activity, hipStream_t s);
hipError_t launch_batch_order(const uint32_t* batch_tile, uint32_t n_batches, uint32_t* order_cnt,
                              uint32_t* order_list, hipStream_t s);
hipError_t launch_blend_bwd(const ViewD* views_dev, int n_views, const float* records, uint32_t n_rec,
                            const uint32_t* pair_vals, const uint32_t* sel, uint32_t cap, const uint32_t* ranges,
                            const float4* ckpt, const uint32_t* batch_tile, uint32_t n_batches,
                            const uint32_t* order_cnt, const uint32_t* order_list,
                            const float* dL_drgb, const float* dL_dalpha, const uint32_t* pair_emit, float* g_pair,
                            uint8_t* alive, bool want_max, hipStream_t s);
hipError_t launch_project_bwd(const JobD& job, const ViewD* views_dev, const float* records,
                              const uint32_t* offsets, const float* g_pair, const uint8_t* alive,
                              uint32_t pair_capacity,
                              const uint32_t* counters, uint32_t trainable, float* g_mean, float* g_scale,
                              float* g_quat, float* g_opacity, float* g_sh, float* g_col, float* max_contrib,
                              float* activity, float* dens_grad, float* dens_cnt, hipStream_t s);
hipError_t launch_batch_error(const uint32_t* counters, int n_req, int32_t* req_status, hipStream_t s);
hipError_t launch_batch_status(const uint32_t* req_rec, int n_req, const uint32_t* offsets,
                               uint32_t pair_capacity, uint32_t* counters, int32_t* req_status,
                               hipStream_t s);

size_t sort_status_words(uint32_t pair_capacity);

}  // namespace gsr
