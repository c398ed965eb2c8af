// Host side of the C ABI declared in include/gsr.h: argument checks,
// workspace layout and the launch sequence of each entry point.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <mutex>
#include <vector>

#include "../../include/gsr.h"
#include "common.hpp"

using namespace gsr;

namespace {

constexpr size_t kAlign = 256;

#define HIP_TRY(expr)                      \
  do {                                     \
    if ((expr) != hipSuccess) return GSR_EHIP; \
  } while (0)

#define HIP_TRY_E(expr)                          \
  do {                                           \
    const hipError_t e_ = (expr);                \
    if (e_ != hipSuccess) return e_;             \
  } while (0)

// Lays buffers out in a byte arena; with base == nullptr it only measures.
struct Carver {
  char* base;
  size_t off = 0;
  explicit Carver(void* b) : base(static_cast<char*>(b)) {}
  template <typename T> T* take(size_t count) {
    off = (off + kAlign - 1) / kAlign * kAlign;
    T* p = base ? reinterpret_cast<T*>(base + off) : nullptr;
    off += count * sizeof(T);
    return p;
  }
};

// Sort control block: digit counts and offsets of every pass, pass tickets.
// Cleared at the start of each call.
struct SortCtl {
  uint32_t hist[kMaxSortPasses * 256];
  uint32_t pass_ctr[kMaxSortPasses];
  uint32_t scan_ticket;
  uint32_t tile_class[kTileClasses];  // tiles per size class (forward order)
  uint32_t seg_ticket;                // next large tile of the block depth sort
  uint32_t pad[6];
  uint32_t hist12[4096];              // tile counts of the one-pass tile grouping
};

struct PipeBufs {
  ViewD* views = nullptr;
  uint32_t* req_rec = nullptr;
  uint32_t* n_tiles = nullptr;
  uint32_t* offsets = nullptr;
  uint64_t* scan_status = nullptr;  // look-back words of the offsets scan
  uint4* tile_box = nullptr;
  uint64_t* keys_a = nullptr;
  uint64_t* keys_b = nullptr;
  uint32_t* rec_of = nullptr;
  SortCtl* ctl = nullptr;
  uint32_t* status = nullptr;
  uint32_t* class_list = nullptr;  // [kTileClasses][X] tiles by size class
  float* g_pair = nullptr;
  float* g_col = nullptr;    // [R][3] colour gradient of each record (backward)
  uint32_t* alive = nullptr;       // [P] bytes (as words): 1 where a pair's partials were written (backward)
  uint32_t* order_cnt = nullptr;   // [kBatchClasses] batches per work class (backward)
  uint32_t* order_list = nullptr;  // [kBatchClasses][batch capacity] batch indices by class (backward)
  // batch only (the single-call path keeps these in the caller's state)
  float* records = nullptr;
  uint32_t* vals = nullptr;
  uint32_t* ranges = nullptr;
  float* pix = nullptr;
  uint32_t* last = nullptr;
  uint32_t* counters = nullptr;
  uint32_t* sel = nullptr;
  // a shared depth order (Gaussians sorted before they are paired): their
  // keys and record ids (double-buffered), the sort's control block and
  // look-back words, words [count, selector after the depth passes,
  // selector after the unit passes], and the emission sequence
  uint64_t* gk_a = nullptr;
  uint64_t* gk_b = nullptr;
  uint32_t* gv_a = nullptr;
  uint32_t* gv_b = nullptr;
  SortCtl* gctl = nullptr;
  uint32_t* gstatus = nullptr;
  uint32_t* gwords = nullptr;
  uint32_t* seq_rec = nullptr;
  uint32_t* n_tiles_seq = nullptr;
  uint4* tile_box_seq = nullptr;
};

// Passes of the Gaussian sort of a shared depth order: 4 over the depth
// bits, then 1 or 2 over the sort unit.
constexpr int kOrderDepthPasses = 4;
int order_unit_passes(uint32_t n_units) { return n_units <= 1 ? 0 : (n_units <= 256 ? 1 : 2); }

size_t carve(Carver& c, PipeBufs& b, size_t n_views, size_t R, size_t P, size_t n_req, bool batch,
             size_t X, size_t Q, bool backward, size_t R_sort = 0) {
  b.views = c.take<ViewD>(std::max<size_t>(n_views, 1));
  b.req_rec = c.take<uint32_t>(n_req + 1);
  b.n_tiles = c.take<uint32_t>(std::max<size_t>(R, 1));
  b.scan_status = c.take<uint64_t>(scan_tiles((uint32_t)R));
  b.tile_box = c.take<uint4>(std::max<size_t>(R, 1));
  b.keys_a = c.take<uint64_t>(std::max<size_t>(P, 1));
  b.keys_b = c.take<uint64_t>(std::max<size_t>(P, 1));
  b.rec_of = c.take<uint32_t>(std::max<size_t>(P, 1));
  b.ctl = c.take<SortCtl>(1);
  b.status = c.take<uint32_t>(std::max(sort_status_words((uint32_t)P),
                                        tile_sort12(X, (uint32_t)P) ? tile_sort12_status_words((uint32_t)P) : 0));
  b.class_list = c.take<uint32_t>(kTileClasses * std::max<size_t>(X, 1));
  if (backward) {
    b.g_pair = c.take<float>(12 * (std::max<size_t>(P, 1) + 1));  // + one zero entry, index P
    b.g_col = c.take<float>(3 * std::max<size_t>(R, 1));
    b.alive = c.take<uint32_t>(std::max<size_t>(P, 1) / 4 + 1);
    b.order_cnt = c.take<uint32_t>(kBatchClasses);
    b.order_list = c.take<uint32_t>(kBatchClasses * (P / kBatch + X + 1));
  }
  if (batch) {
    b.offsets = c.take<uint32_t>(R + 1);
    b.records = c.take<float>(kRecordFloats * std::max<size_t>(R, 1));
    b.vals = c.take<uint32_t>(2 * std::max<size_t>(P, 1));
    b.ranges = c.take<uint32_t>(2 * std::max<size_t>(X, 1));
    b.pix = c.take<float>(4 * std::max<size_t>(Q, 1));
    b.last = c.take<uint32_t>(std::max<size_t>(Q, 1));
    b.counters = c.take<uint32_t>(4);
    b.sel = c.take<uint32_t>(1);
  }
  if (R_sort) {
    b.gk_a = c.take<uint64_t>(R_sort);
    b.gk_b = c.take<uint64_t>(R_sort);
    b.gv_a = c.take<uint32_t>(R_sort);
    b.gv_b = c.take<uint32_t>(R_sort);
    b.gctl = c.take<SortCtl>(1);
    b.gstatus = c.take<uint32_t>(sort_status_words((uint32_t)R_sort));
    b.gwords = c.take<uint32_t>(4);
    b.seq_rec = c.take<uint32_t>(std::max<size_t>(R, 1));
    b.n_tiles_seq = c.take<uint32_t>(std::max<size_t>(R, 1));
    b.tile_box_seq = c.take<uint4>(std::max<size_t>(R, 1));
  }
  return c.off + kAlign;
}

// One launch zeroes everything a call expects to start at zero: the sort
// control block (digit counts, tickets), the pair count (all four counter
// words for a batch, whose counters live in the workspace; a forward
// state's overflow and error words are sticky, cleared by
// gsr_forward_check), the tile ranges, the scan's and the radix passes'
// look-back words, the sorted-buffer selector and (forward) the
// batch-to-tile map.
// The global radix passes cover only the tile bits of the keys (bits 32
// up); the depth bits are sorted per tile segment.
constexpr int kDepthPasses = 4;
int tile_pass_end(uint64_t total_tiles) {
  int b = 0;
  while (b < 32 && (1ull << b) < total_tiles) ++b;
  return kDepthPasses + (b + 7) / 8;
}

// The views array goes to the device in the arguments of the clear launch
// when it is small enough (one launch), else in upload launches of their own;
// never by a copy from pageable host memory.
hipError_t upload_views(ViewD* dst, const ViewD* src, int n_views, WordUpload& up, hipStream_t s) {
  const size_t bytes = sizeof(ViewD) * (size_t)n_views;
  up.dst = nullptr;
  up.n = 0;
  if (bytes <= sizeof(up.w)) {
    up.dst = reinterpret_cast<uint32_t*>(dst);
    up.n = (uint32_t)(bytes / 4);
    std::memcpy(up.w, src, bytes);
    return hipSuccess;
  }
  return launch_upload(reinterpret_cast<uint32_t*>(dst), src, bytes / 4, s);
}

hipError_t clear_workspace(const PipeBufs& b, uint32_t* counters, bool sticky_flags, uint32_t* ranges, size_t X,
                           size_t R, uint32_t P, uint32_t* sel, hipStream_t s, const WordUpload* up,
                           uint32_t* batch_tile = nullptr, size_t n_batches = 0, uint32_t n_sort = 0) {
  ClearSet cs{};
  cs.p[0] = reinterpret_cast<uint32_t*>(b.ctl);
  cs.n[0] = sizeof(SortCtl) / 4;
  cs.p[1] = counters;
  cs.n[1] = sticky_flags ? 1 : 4;
  cs.p[2] = ranges;
  cs.n[2] = 2 * X;
  cs.p[3] = reinterpret_cast<uint32_t*>(b.scan_status);
  cs.n[3] = 2 * (size_t)scan_tiles((uint32_t)R);
  // look-back words of the tile passes, and the sorted-buffer selector
  if (tile_sort12(X, P)) {  // block counts: written before they are read, no clearing
    cs.p[4] = nullptr;
    cs.n[4] = 0;
  } else {
    const size_t stride = sort_status_stride(P);
    const int pb = kDepthPasses, pe = tile_pass_end(X);
    cs.p[4] = b.status + (size_t)pb * stride;
    cs.n[4] = (size_t)(pe - pb) * stride;
  }
  cs.p[5] = sel;
  cs.n[5] = 1;
  cs.n_ranges = 6;
  if (batch_tile && n_batches) {
    cs.p[cs.n_ranges] = batch_tile;
    cs.n[cs.n_ranges++] = n_batches;
  }
  if (b.gctl) {  // the Gaussian sort's control block, look-back words and selectors
    cs.p[cs.n_ranges] = reinterpret_cast<uint32_t*>(b.gctl);
    cs.n[cs.n_ranges++] = sizeof(SortCtl) / 4;
    cs.p[cs.n_ranges] = b.gstatus;
    cs.n[cs.n_ranges++] = sort_status_words(n_sort);
    cs.p[cs.n_ranges] = b.gwords;
    cs.n[cs.n_ranges++] = 4;
  }
  return launch_clear_multi(cs, s, up);
}

// The sort fields of view d from its view state: a shared order puts the
// sort camera's depth row in the view (a unit) or points it at its lead.
void set_sort_fields(ViewD& d, const gsr_view_state& vs, uint32_t mode, uint32_t unit, uint32_t off, uint32_t lead) {
  d.sort_mode = mode;
  d.sort_unit = unit;
  d.sort_off = off;
  d.sort_lead = lead;
  if (mode == kSortCamera) {
    d.sort_r[0] = vs.sort_cam.R[6];
    d.sort_r[1] = vs.sort_cam.R[7];
    d.sort_r[2] = vs.sort_cam.R[8];
    d.sort_t = vs.sort_cam.t[2];
  }
}

// The order stages of a call whose Gaussians are depth-sorted before they
// are paired, up to the pair count: the Gaussian sort (records written by
// the projection into gk_a / gv_a), then the emission sequence and its
// tile-count scan into `offsets` (total into counters).
hipError_t order_before_pairs(const PipeBufs& b, ViewD* views_dev, int n_views, uint32_t R, uint32_t n_sort,
                              uint32_t n_units, uint32_t* offsets, uint32_t* counters, uint32_t P, hipStream_t s) {
  uint32_t* sel = &b.gwords[1];
  HIP_TRY_E(launch_sort(b.gk_a, b.gk_b, b.gv_a, b.gv_b, b.gwords, n_sort, 0, kOrderDepthPasses, b.gctl->hist,
                        b.gstatus, b.gctl->pass_ctr, &b.gwords[1], counters + kCntError, s));
  const int up = order_unit_passes(n_units);
  if (up > 0) {
    HIP_TRY_E(launch_sort(b.gk_a, b.gk_b, b.gv_a, b.gv_b, b.gwords, n_sort, kOrderDepthPasses, kOrderDepthPasses + up,
                          b.gctl->hist, b.gstatus, b.gctl->pass_ctr, &b.gwords[2], counters + kCntError, s,
                          &b.gwords[1]));
    sel = &b.gwords[2];
  }
  HIP_TRY_E(launch_seq_build(views_dev, n_views, R, b.gk_a, b.gk_b, b.gv_a, b.gv_b, sel, n_sort, b.n_tiles,
                             b.tile_box, b.seq_rec, b.n_tiles_seq, b.tile_box_seq, counters, s));
  HIP_TRY_E(launch_scan(b.n_tiles_seq, offsets, b.scan_status, &b.ctl->scan_ticket, R, counters, P, s));
  return hipSuccess;
}

bool model_ok(const gsr_model* m) {
  if (!m || m->n < 0 || m->sh_degree < 0 || m->sh_degree > 3) return false;
  if (m->raw != 0 && m->raw != 1) return false;
  if (m->format == GSR_FORMAT_F32)
    return m->n == 0 || (m->mean && m->scale && m->quat && m->opacity && m->sh && m->layer);
  if (m->format != GSR_FORMAT_HALF_PACKED && m->format != GSR_FORMAT_HALF_CODEBOOK) return false;
  const gsr_compressed* c = m->compressed;
  if (m->raw != 0 || !c || c->reserved != 0) return false;
  if (m->n == 0) return true;
  if (!m->layer || !c->mean || !c->scale || !c->quat || !c->opacity || !c->sh_dc) return false;
  if (m->sh_degree == 0) return true;  // no higher coefficients to read
  if (m->format == GSR_FORMAT_HALF_PACKED) {
    for (int ch = 0; ch < 3; ++ch)
      if (!std::isfinite(c->sh_lo[ch]) || !std::isfinite(c->sh_step[ch])) return false;
    return c->sh_packed != nullptr;
  }
  return c->sh_index && c->codebook && c->codebook_size >= 1 && c->codebook_size <= 65536;
}

bool camera_ok(const gsr_camera& c) {
  return c.width > 0 && c.height > 0 && c.width <= 65535 * kTile && c.height <= 65535 * kTile && c.fx > 0.f &&
         c.fy > 0.f;
}

bool view_ok(const gsr_view_state& v) {
  if (v.mip_2d != 0 && (v.mip_2d != 1 || !(v.mip_2d_var > 0.f) || !std::isfinite(v.mip_2d_var))) return false;
  return v.n_clip >= 0 && v.n_clip <= GSR_MAX_CLIP && (v.sort_shared == 0 || v.sort_shared == 1);
}

uint32_t tiles_of(const gsr_camera& c) {
  return div_up((uint32_t)c.width, (uint32_t)kTile) * div_up((uint32_t)c.height, (uint32_t)kTile);
}

ViewD make_view(const gsr_camera& c, const gsr_view_state& vs) {
  ViewD v;
  std::memset(&v, 0, sizeof(v));
  std::memcpy(v.R, c.R, sizeof(v.R));
  std::memcpy(v.t, c.t, sizeof(v.t));
  v.fx = c.fx; v.fy = c.fy; v.cx = c.cx; v.cy = c.cy; v.znear = c.znear; v.guard = c.guard;
  v.W = c.width; v.H = c.height;
  v.tiles_x = (int32_t)div_up((uint32_t)c.width, (uint32_t)kTile);
  v.tiles_y = (int32_t)div_up((uint32_t)c.height, (uint32_t)kTile);
  v.layer_mask = vs.layer_mask;
  v.n_clip = vs.n_clip;
  for (int k = 0; k < vs.n_clip; ++k) {
    for (int j = 0; j < 3; ++j) v.clip[k].n[j] = vs.clip[k].n[j];
    v.clip[k].d = vs.clip[k].d;
    v.clip[k].bits = vs.clip[k].layer_bits;
  }
  for (int j = 0; j < 3; ++j) v.bg[j] = vs.bg[j];
  for (int l = 0; l < 32; ++l) v.layer_op[l] = vs.layer_fade ? vs.layer_opacity[l] : 1.f;
  v.mip_2d = vs.mip_2d ? 1u : 0u;
  v.mip_var = vs.mip_2d_var;
  return v;
}

ModelD make_model(const gsr_model& m) {
  ModelD d;
  std::memset(&d, 0, sizeof(d));
  d.n = m.n; d.D = m.sh_degree;
  d.mean = m.mean; d.scale = m.scale; d.quat = m.quat; d.opacity = m.opacity; d.sh = m.sh; d.layer = m.layer;
  d.raw = m.raw;
  d.fmt = m.format;
  d.filter_3d = m.filter_3d;
  if (m.format != GSR_FORMAT_F32 && m.compressed) {
    const gsr_compressed& c = *m.compressed;
    d.h_mean = c.mean; d.h_scale = c.scale; d.h_quat = c.quat; d.h_opacity = c.opacity; d.h_dc = c.sh_dc;
    d.sh_packed = c.sh_packed; d.sh_index = c.sh_index; d.codebook = c.codebook;
    for (int ch = 0; ch < 3; ++ch) { d.sh_lo[ch] = c.sh_lo[ch]; d.sh_step[ch] = c.sh_step[ch]; }
    d.codebook_size = (uint32_t)c.codebook_size;
  }
  return d;
}

// Jobs: the views of one model in chunks of kMaxJobViews.
std::vector<JobD> make_jobs(const ModelD& m, const std::vector<int>& view_ids) {
  std::vector<JobD> jobs;
  for (size_t i = 0; i < view_ids.size(); i += kMaxJobViews) {
    JobD j;
    std::memset(&j, 0, sizeof(j));
    j.m = m;
    j.n_views = (int32_t)std::min<size_t>(kMaxJobViews, view_ids.size() - i);
    for (int k = 0; k < j.n_views; ++k) j.view[k] = view_ids[i + k];
    jobs.push_back(j);
  }
  return jobs;
}



}  // namespace

struct gsr_timer {
  std::vector<hipEvent_t> pool;
  size_t used = 0;
  struct Mark { int stage; size_t e0, e1; };
  std::vector<Mark> marks;

  hipEvent_t next() {
    if (used == pool.size()) {
      hipEvent_t e;
      if (hipEventCreate(&e) != hipSuccess) return nullptr;
      pool.push_back(e);
    }
    return pool[used++];
  }
};

namespace {

// Event pair around one stage when a timer is attached.
struct StageScope {
  gsr_timer* t;
  int stage;
  hipStream_t s;
  size_t e0 = 0;
  bool ok = false;
  StageScope(gsr_timer* tm, int st, hipStream_t str) : t(tm), stage(st), s(str) {
    if (!t) return;
    hipEvent_t e = t->next();
    if (!e) return;
    e0 = t->used - 1;
    ok = hipEventRecord(e, s) == hipSuccess;
  }
  ~StageScope() {
    if (!t || !ok) return;
    hipEvent_t e = t->next();
    if (!e) return;
    if (hipEventRecord(e, s) == hipSuccess) t->marks.push_back({stage, e0, t->used - 1});
  }
};

bool state_ok(const gsr_fwd_state* st) {
  return st && st->records && st->offsets && st->pair_vals && st->sort_sel && st->pair_emit && st->ranges &&
         st->pixel_state && st->last && st->checkpoints && st->batch_map && st->counters &&
         st->pair_capacity < (1u << 30);
}

bool single_view_args_ok(const gsr_model* model, int32_t n_views, const gsr_camera* cams,
                         const gsr_view_state* views) {
  if (!model_ok(model) || n_views <= 0 || !cams || !views) return false;
  for (int v = 0; v < n_views; ++v) {
    if (!camera_ok(cams[v]) || !view_ok(views[v])) return false;
    if (cams[v].width != cams[0].width || cams[v].height != cams[0].height) return false;
  }
  if ((uint64_t)model->n * (uint64_t)n_views >= (1ull << 31)) return false;
  return true;
}

}  // namespace

extern "C" {

gsr_status gsr_timer_create(gsr_timer** out) {
  if (!out) return GSR_EINVAL;
  *out = new gsr_timer();
  return GSR_OK;
}

void gsr_timer_destroy(gsr_timer* t) {
  if (!t) return;
  for (hipEvent_t e : t->pool) (void)hipEventDestroy(e);
  delete t;
}

gsr_status gsr_timer_read(gsr_timer* t, float* ms, uint32_t* calls) {
  if (!t) return GSR_EINVAL;
  float acc[GSR_N_STAGES] = {0};
  uint32_t cnt[GSR_N_STAGES] = {0};
  gsr_status st = GSR_OK;
  for (const gsr_timer::Mark& m : t->marks) {
    float x = 0.f;
    if (hipEventSynchronize(t->pool[m.e1]) != hipSuccess ||
        hipEventElapsedTime(&x, t->pool[m.e0], t->pool[m.e1]) != hipSuccess) {
      st = GSR_EHIP;
      continue;
    }
    acc[m.stage] += x;
    cnt[m.stage] += 1;
  }
  t->marks.clear();
  t->used = 0;
  for (int k = 0; k < GSR_N_STAGES; ++k) {
    if (ms) ms[k] = acc[k];
    if (calls) calls[k] = cnt[k];
  }
  return st;
}

const char* gsr_status_string(gsr_status s) {
  switch (s) {
    case GSR_OK: return "ok";
    case GSR_EINVAL: return "invalid argument";
    case GSR_ENOSPACE: return "workspace or pair capacity too small";
    case GSR_EHIP: return "HIP runtime error";
    case GSR_EDEVICE: return "device-side error";
  }
  return "unknown status";
}

uint32_t gsr_batch_capacity(uint32_t pair_capacity, uint32_t total_tiles) {
  return pair_capacity / (uint32_t)kBatch + total_tiles + 1;
}

size_t gsr_workspace_size(int32_t n, int32_t n_views, int32_t width, int32_t height, uint32_t pair_capacity,
                          int32_t shared_order) {
  if (n < 0 || n_views <= 0 || width <= 0 || height <= 0 || pair_capacity >= (1u << 30)) return 0;
  Carver c(nullptr);
  PipeBufs b;
  const size_t X = (size_t)n_views * (size_t)((width + kTile - 1) / kTile) * (size_t)((height + kTile - 1) / kTile);
  return carve(c, b, (size_t)n_views, (size_t)n * n_views, pair_capacity, 0, false, X, 0, true,
               shared_order ? (size_t)std::max(n, 1) : 0);
}

gsr_status gsr_adam_step(int32_t n, int32_t sh_degree, uint32_t trainable_layers, const uint8_t* layer,
                         const gsr_adam_group* groups, float beta1, float beta2, float eps, int32_t step,
                         float* activity, void* stream) {
  if (n < 0 || sh_degree < 0 || sh_degree > 3 || !groups || step < 1) return GSR_EINVAL;
  if (!(beta1 >= 0.f && beta1 < 1.f) || !(beta2 >= 0.f && beta2 < 1.f) || !(eps >= 0.f)) return GSR_EINVAL;
  if (n == 0) return GSR_OK;
  if (!layer) return GSR_EINVAL;
  const int planes[kAdamGroups] = {3, 3, 4, 1, 3 * (sh_degree + 1) * (sh_degree + 1)};
  AdamArgs a;
  const double bc1 = 1.0 - std::pow((double)beta1, (double)step);
  const double bc2 = 1.0 - std::pow((double)beta2, (double)step);
  for (int gi = 0; gi < kAdamGroups; ++gi) {
    const gsr_adam_group& g = groups[gi];
    if (!g.param || !g.grad || !g.exp_avg || !g.exp_avg_sq || !(g.lr >= 0.f)) return GSR_EINVAL;
    a.g[gi] = AdamGroupD{g.param, g.exp_avg, g.exp_avg_sq, g.grad, planes[gi], (float)((double)g.lr / bc1)};
  }
  a.one_minus_b1 = 1.f - beta1;
  a.b2 = beta2;
  a.one_minus_b2 = 1.f - beta2;
  a.bc2_sqrt = (float)std::sqrt(bc2);
  a.eps = eps;
  HIP_TRY(launch_adam(n, a, layer, trainable_layers, activity, static_cast<hipStream_t>(stream)));
  return GSR_OK;
}

gsr_status gsr_update_activity(int32_t n, int32_t sh_degree, uint32_t trainable_layers, const float* mean_before,
                               const float* mean_after, const float* log_scale_before, const float* log_scale_after,
                               const float* sh_before, const float* sh_after, const uint8_t* layer, float* activity,
                               void* stream) {
  if (n < 0 || sh_degree < 0 || sh_degree > 3) return GSR_EINVAL;
  if (n == 0) return GSR_OK;
  if (!mean_before || !mean_after || !log_scale_before || !log_scale_after || !sh_before || !sh_after || !layer ||
      !activity)
    return GSR_EINVAL;
  HIP_TRY(launch_update_activity(n, sh_degree, trainable_layers, mean_before, mean_after, log_scale_before,
                                 log_scale_after, sh_before, sh_after, layer, activity,
                                 static_cast<hipStream_t>(stream)));
  return GSR_OK;
}

}  // extern "C"

namespace {

// The forward of gsr_rasterize_forward on a given scratch workspace; the
// layout is the forward's and the backward's (backward_layout, what
// gsr_workspace_size measures) or the forward's alone.
gsr_status forward_impl(const gsr_model* model, int32_t n_views, const gsr_camera* cams,
                        const gsr_view_state* views, gsr_fwd_state* state, void* ws, size_t ws_bytes, float* rgb,
                        float* alpha, uint32_t* n_pairs_host, const gsr_debug* debug, gsr_timer* timer,
                        void* stream, bool backward_layout) {
  if (!single_view_args_ok(model, n_views, cams, views) || !state || !ws || !rgb || !alpha) return GSR_EINVAL;
  if (!state_ok(state)) return GSR_EINVAL;
  const hipStream_t s = static_cast<hipStream_t>(stream);
  const int W = cams[0].width, H = cams[0].height;
  const uint32_t n = (uint32_t)model->n;
  const uint32_t R = n * (uint32_t)n_views;
  const uint32_t P = state->pair_capacity;
  const uint32_t tiles_per_view = tiles_of(cams[0]);
  const uint64_t X = (uint64_t)tiles_per_view * n_views;
  if (X >= kBatchTileMask || state->batch_capacity < gsr_batch_capacity(P, (uint32_t)X)) return GSR_EINVAL;
  const size_t plane = (size_t)W * H;
  // one depth order for all views: the Gaussians are sorted by their depth in
  // views[0].sort_cam before they are paired
  const bool shared = views[0].sort_shared != 0;
  const uint32_t n_sort = shared ? std::max(n, 1u) : 0u;
  Carver c(ws);
  PipeBufs b;
  if (carve(c, b, n_views, R, P, 0, false, X, 0, backward_layout, n_sort) > ws_bytes)
    return GSR_ENOSPACE;

  std::vector<ViewD> hv(n_views);
  std::vector<int> ids(n_views);
  for (int v = 0; v < n_views; ++v) {
    ViewD d = make_view(cams[v], views[v]);
    d.tile_off = (uint32_t)v * tiles_per_view;
    d.rec_off = (uint32_t)v * n;
    d.rgb = rgb + 3 * plane * v;
    d.alpha = alpha + plane * v;
    d.pix = state->pixel_state + 4 * plane * v;
    d.last = state->last + plane * v;
    if (shared) set_sort_fields(d, views[0], v == 0 ? kSortCamera : kSortFollow, 0, 0, 0);
    hv[v] = d;
    ids[v] = v;
  }
  WordUpload up;
  HIP_TRY(upload_views(b.views, hv.data(), n_views, up, s));
  HIP_TRY(clear_workspace(b, state->counters, true, state->ranges, X, R, P, state->sort_sel, s, &up,
                          state->batch_map + X + 1, state->batch_capacity, n_sort));
  if (shared) HIP_TRY(launch_set_u32(&b.gwords[0], n_sort, s));
  const ModelD md = make_model(*model);
  {
    StageScope sc(timer, GSR_STAGE_PROJECT, s);
    for (const JobD& j : make_jobs(md, ids))
      HIP_TRY(launch_project(j, b.views, state->records, b.n_tiles, b.tile_box, shared ? b.gk_a : nullptr,
                             shared ? b.gv_a : nullptr, state->counters, s));
  }
  {
    StageScope sc(timer, GSR_STAGE_SCAN, s);
    if (shared)
      HIP_TRY(order_before_pairs(b, b.views, n_views, R, n_sort, 1, state->offsets, state->counters, P, s));
    else
      HIP_TRY(launch_scan(b.n_tiles, state->offsets, b.scan_status, &b.ctl->scan_ticket, R, state->counters, P, s));
  }
  if (n_pairs_host) {
    // the pair count, and the sticky error word (this call's scan, or an
    // earlier call on this state that nobody checked)
    uint32_t cnt[3] = {0, 0, 0};
    HIP_TRY(hipMemcpyAsync(cnt, state->counters, sizeof(cnt), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    *n_pairs_host = cnt[kCntPairs];
    if (cnt[kCntError]) return GSR_EDEVICE;
    if (cnt[kCntPairs] > P) {
      HIP_TRY(launch_clear_u32(state->counters + kCntOverflow, 1, s));  // this call's overflow is reported now
      return GSR_ENOSPACE;
    }
  }
  {
    StageScope sc(timer, GSR_STAGE_DUPLICATE, s);
    if (shared)
      HIP_TRY(launch_duplicate(b.n_tiles_seq, state->offsets, b.tile_box_seq, R, state->counters, P, b.keys_a,
                               state->pair_vals, b.rec_of, s, b.seq_rec));
    else
      HIP_TRY(launch_duplicate(b.n_tiles, state->offsets, b.tile_box, R, state->counters, P, b.keys_a,
                               state->pair_vals, b.rec_of, s));
  }
  if (debug && (debug->keys_emit || debug->vals_emit)) {
    if (debug->keys_emit) HIP_TRY(hipMemcpyAsync(debug->keys_emit, b.keys_a, 8ull * P, hipMemcpyDeviceToDevice, s));
    if (debug->vals_emit) HIP_TRY(hipMemcpyAsync(debug->vals_emit, b.rec_of, 4ull * P, hipMemcpyDeviceToDevice, s));
  }
  {
    StageScope sc(timer, GSR_STAGE_SORT, s);
    if (tile_sort12(X, P))
      HIP_TRY(launch_tile_sort12(b.keys_a, b.keys_b, state->pair_vals, state->pair_vals + P, state->counters, P,
                                 (uint32_t)X, b.ctl->hist12, b.status, state->ranges, b.ctl->tile_class,
                                 b.class_list, state->sort_sel, state->counters + kCntError, s));
    else
      HIP_TRY(launch_sort(b.keys_a, b.keys_b, state->pair_vals, state->pair_vals + P, state->counters, P,
                          kDepthPasses, tile_pass_end(X), b.ctl->hist, b.status, b.ctl->pass_ctr,
                          state->sort_sel, state->counters + kCntError, s));
  }
  {
    StageScope sc(timer, GSR_STAGE_RANGES, s);
    if (!tile_sort12(X, P)) {  // (the one-pass grouping writes the ranges and classes itself)
      HIP_TRY(launch_ranges(b.keys_a, b.keys_b, state->sort_sel, state->counters, P, (uint32_t)X, state->ranges, s));
      HIP_TRY(launch_tile_order(state->ranges, (uint32_t)X, b.ctl->tile_class, b.class_list, s));
    }
  }
  {
    StageScope sc(timer, GSR_STAGE_SORT, s);
    if (shared)  // the pairs of every tile are in depth order already
      HIP_TRY(launch_finalize_pairs(state->pair_vals, state->pair_vals + P, b.keys_a, b.keys_b, state->sort_sel,
                                    b.rec_of, state->counters, P, state->pair_emit,
                                    debug ? debug->keys_sorted : nullptr, s));
    else
      HIP_TRY(launch_sort_segments(b.keys_a, b.keys_b, state->pair_vals, state->pair_vals + P, state->sort_sel,
                                   state->ranges, (uint32_t)X, b.rec_of, state->counters, P, state->pair_emit,
                                   debug ? debug->keys_sorted : nullptr, b.ctl->tile_class, b.class_list,
                                   &b.ctl->seg_ticket, state->counters + kCntError, s));
  }
  uint32_t* batch_tile = state->batch_map + X + 1;
  {
    StageScope sc(timer, GSR_STAGE_BLEND, s);
    HIP_TRY(launch_blend_fwd_tile(b.views, n_views, (uint32_t)X, state->records, R, state->pair_vals,
                                  state->sort_sel, P, state->ranges, batch_tile, state->batch_capacity,
                                  nullptr, reinterpret_cast<float4*>(state->checkpoints), b.ctl->tile_class,
                                  b.class_list, s));
  }
  if (debug) {
    if (debug->n_tiles) HIP_TRY(hipMemcpyAsync(debug->n_tiles, b.n_tiles, 4ull * R, hipMemcpyDeviceToDevice, s));
    if (debug->tile_box) HIP_TRY(hipMemcpyAsync(debug->tile_box, b.tile_box, 16ull * R, hipMemcpyDeviceToDevice, s));
    HIP_TRY(hipStreamSynchronize(s));
  }
  return GSR_OK;
}

}  // namespace

extern "C" {

gsr_status gsr_rasterize_forward(const gsr_model* model, int32_t n_views, const gsr_camera* cams,
                                 const gsr_view_state* views, gsr_fwd_state* state, void* ws, size_t ws_bytes,
                                 float* rgb, float* alpha, uint32_t* n_pairs_host, const gsr_debug* debug,
                                 gsr_timer* timer, void* stream) {
  return forward_impl(model, n_views, cams, views, state, ws, ws_bytes, rgb, alpha, n_pairs_host, debug, timer,
                      stream, true);
}

}  // extern "C"

// ---------------------------------------------------------------- no allocation
// The scratch of gsr_rasterize_forward_noalloc: a file-scope device array
// (one copy per GPU, held until the process ends).  Host code never uses the
// array's name as an address (on the host it is a stand-in symbol): each
// device's address comes from hipGetSymbolAddress, taken once per device
// with that device current and kept here.
namespace {

constexpr size_t kNoallocScratchBytes = (size_t)GSR_NOALLOC_SCRATCH_BYTES;
__device__ __align__(256) uint8_t scratch[kNoallocScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

gsr_status scratch_of_current_device(void** out) {
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess) return GSR_EHIP;
  if (dev < 0 || dev >= kMaxDevices) return GSR_EINVAL;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* ptr = nullptr;
    if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess || !ptr) return GSR_EHIP;
    g_scratch_ptr[dev] = ptr;
  }
  *out = g_scratch_ptr[dev];
  return GSR_OK;
}

}  // namespace

extern "C" {

gsr_status gsr_rasterize_forward_noalloc(const gsr_model* model, int32_t n_views, const gsr_camera* cams,
                                         const gsr_view_state* views, gsr_fwd_state* state, float* rgb,
                                         float* alpha, uint32_t* n_pairs_host, void* stream) {
  if (!single_view_args_ok(model, n_views, cams, views) || !state || !rgb || !alpha || !state_ok(state))
    return GSR_EINVAL;
  const uint64_t X = (uint64_t)tiles_of(cams[0]) * (uint64_t)n_views;
  Carver c(nullptr);
  PipeBufs b;
  const size_t need = carve(c, b, (size_t)n_views, (size_t)model->n * (size_t)n_views, state->pair_capacity, 0,
                            false, X, 0, false, views[0].sort_shared ? (size_t)std::max(model->n, 1) : 0);
  if (need > kNoallocScratchBytes) return GSR_ENOSPACE;
  void* ws = nullptr;
  const gsr_status st = scratch_of_current_device(&ws);
  if (st != GSR_OK) return st;
  return forward_impl(model, n_views, cams, views, state, ws, kNoallocScratchBytes, rgb, alpha, n_pairs_host,
                      nullptr, nullptr, stream, false);
}

gsr_status gsr_forward_check(const gsr_fwd_state* state, uint32_t* n_pairs_host, void* stream) {
  if (!state || !state->counters) return GSR_EINVAL;
  uint32_t cnt[4] = {0, 0, 0, 0};
  const hipStream_t s = static_cast<hipStream_t>(stream);
  HIP_TRY(hipMemcpyAsync(cnt, state->counters, sizeof(cnt), hipMemcpyDeviceToHost, s));
  HIP_TRY(hipStreamSynchronize(s));
  // the overflow and error words are reported once: cleared for the calls to come
  HIP_TRY(launch_clear_u32(state->counters + kCntOverflow, 2, s));
  if (n_pairs_host) *n_pairs_host = cnt[kCntPairs];
  if (cnt[kCntError]) return GSR_EDEVICE;
  if (cnt[kCntOverflow]) return GSR_ENOSPACE;
  return GSR_OK;
}

gsr_status gsr_rasterize_backward(const gsr_model* model, int32_t n_views, const gsr_camera* cams,
                                  const gsr_view_state* views, const gsr_fwd_state* state, const float* dL_drgb,
                                  const float* dL_dalpha, uint32_t trainable_layers, void* ws, size_t ws_bytes,
                                  const gsr_grads* grads, float* max_contrib, float* activity, gsr_timer* timer,
                                  void* stream) {
  if (!single_view_args_ok(model, n_views, cams, views) || !state || !ws || !grads) return GSR_EINVAL;
  if (n_views > kMaxJobViews || views[0].sort_shared || model->format != GSR_FORMAT_F32 || model->filter_3d)
    return GSR_EINVAL;
  for (int v = 0; v < n_views; ++v)
    if (views[v].mip_2d) return GSR_EINVAL;  // the Mip filters are rendered, not differentiated
  if (model->n > 0 && (!grads->g_mean || !grads->g_scale || !grads->g_quat || !grads->g_opacity || !grads->g_sh))
    return GSR_EINVAL;
  if (!state_ok(state)) return GSR_EINVAL;
  const hipStream_t s = static_cast<hipStream_t>(stream);
  const int W = cams[0].width, H = cams[0].height;
  const uint32_t n = (uint32_t)model->n;
  const uint32_t R = n * (uint32_t)n_views;
  const uint32_t P = state->pair_capacity;
  const uint32_t tiles_per_view = tiles_of(cams[0]);
  const uint64_t X = (uint64_t)tiles_per_view * n_views;
  const size_t plane = (size_t)W * H;
  Carver c(ws);
  PipeBufs b;
  if (carve(c, b, n_views, R, P, 0, false, X, 0, true) > ws_bytes)
    return GSR_ENOSPACE;
  std::vector<ViewD> hv(n_views);
  std::vector<int> ids(n_views);
  for (int v = 0; v < n_views; ++v) {
    ViewD d = make_view(cams[v], views[v]);
    d.tile_off = (uint32_t)v * tiles_per_view;
    d.rec_off = (uint32_t)v * n;
    d.pix = state->pixel_state + 4 * plane * v;
    d.last = state->last + plane * v;
    hv[v] = d;
    ids[v] = v;
  }
  if (n == 0) return GSR_OK;
  if (X >= kBatchTileMask || state->batch_capacity < gsr_batch_capacity(P, (uint32_t)X)) return GSR_EINVAL;
  // batch indices are below P / 256 + X + 1 (the order list's row length)
  const uint32_t n_batches = std::min(state->batch_capacity, gsr_batch_capacity(P, (uint32_t)X));
  {
    WordUpload up;
    HIP_TRY(upload_views(b.views, hv.data(), n_views, up, s));
    ClearSet cs{};
    cs.p[0] = b.order_cnt;
    cs.n[0] = kBatchClasses;
    cs.p[1] = b.alive;
    cs.n[1] = (size_t)P / 4 + 1;
    cs.p[2] = reinterpret_cast<uint32_t*>(b.g_pair + 12 * (size_t)P);  // the zero entry
    cs.n[2] = 12;
    cs.n_ranges = 3;
    HIP_TRY(launch_clear_multi(cs, s, up.n ? &up : nullptr));
  }
  const uint32_t* batch_tile = state->batch_map + X + 1;
  {
    StageScope sc(timer, GSR_STAGE_BWD_ORDER, s);
    HIP_TRY(launch_batch_order(batch_tile, n_batches, b.order_cnt, b.order_list, s));
  }
  {
    StageScope sc(timer, GSR_STAGE_BLEND_BWD, s);
    HIP_TRY(launch_blend_bwd(b.views, n_views, state->records, R, state->pair_vals, state->sort_sel, P,
                             state->ranges, reinterpret_cast<const float4*>(state->checkpoints), batch_tile,
                             n_batches, b.order_cnt, b.order_list, dL_drgb, dL_dalpha, state->pair_emit, b.g_pair,
                             reinterpret_cast<uint8_t*>(b.alive), max_contrib != nullptr, s));
  }
  const ModelD md = make_model(*model);
  {
    StageScope sc(timer, GSR_STAGE_PROJECT_BWD, s);
    for (const JobD& j : make_jobs(md, ids))
      HIP_TRY(launch_project_bwd(j, b.views, state->records, state->offsets, b.g_pair,
                                 reinterpret_cast<const uint8_t*>(b.alive), P,
                                 state->counters, trainable_layers, grads->g_mean, grads->g_scale, grads->g_quat,
                                 grads->g_opacity, grads->g_sh, b.g_col, max_contrib, activity,
                                 grads->densify_grad, grads->densify_count, s));
  }
  return GSR_OK;
}

// ---------------------------------------------------------------- batch
namespace {

struct BatchPlan {
  std::vector<ViewD> views;
  std::vector<uint32_t> req_rec;
  uint64_t R = 0, X = 0, Q = 0;
  // with any request sharing one depth order between its eyes, every view
  // takes the order-first path: R_sort records in n_units sort units
  bool ordered = false;
  uint64_t R_sort = 0;
  uint32_t n_units = 0;
};

bool plan_batch(const gsr_model* models, int32_t n_models, const gsr_request* reqs, int32_t n_req, BatchPlan& bp) {
  if (!models || n_models <= 0 || !reqs || n_req <= 0) return false;
  for (int m = 0; m < n_models; ++m)
    if (!model_ok(&models[m])) return false;
  bp.req_rec.assign(n_req + 1, 0);
  for (int q = 0; q < n_req; ++q) {
    const gsr_request& r = reqs[q];
    if (r.model < 0 || r.model >= n_models || r.n_views < 1 || r.n_views > 2 || !view_ok(r.vs)) return false;
    bp.req_rec[q] = (uint32_t)bp.R;
    for (int e = 0; e < r.n_views; ++e) {
      if (!camera_ok(r.cam[e]) || !r.rgb[e] || !r.alpha[e]) return false;
      ViewD d = make_view(r.cam[e], r.vs);
      d.model = (uint32_t)r.model;
      d.request = (uint32_t)q;
      d.rec_off = (uint32_t)bp.R;
      d.tile_off = (uint32_t)bp.X;
      d.rgb = r.rgb[e];
      d.alpha = r.alpha[e];
      bp.views.push_back(d);
      bp.R += (uint64_t)models[r.model].n;
      bp.X += tiles_of(r.cam[e]);
      bp.Q += (uint64_t)r.cam[e].width * r.cam[e].height;
    }
  }
  bp.req_rec[n_req] = (uint32_t)bp.R;
  for (int q = 0; q < n_req; ++q) bp.ordered = bp.ordered || reqs[q].vs.sort_shared != 0;
  if (bp.ordered) {
    // each view is a sort unit by its own depth, except the eyes of a
    // request that shares one order: the first eye sorts by the request's
    // sort camera, the second follows it
    size_t v = 0;
    for (int q = 0; q < n_req; ++q) {
      const gsr_request& r = reqs[q];
      const bool sh = r.vs.sort_shared != 0;
      for (int e = 0; e < r.n_views; ++e, ++v) {
        ViewD& d = bp.views[v];
        if (sh && e > 0) {
          set_sort_fields(d, r.vs, kSortFollow, 0, 0, (uint32_t)(v - e));
        } else {
          set_sort_fields(d, r.vs, sh ? kSortCamera : kSortOwn, bp.n_units++, (uint32_t)bp.R_sort, 0);
          bp.R_sort += (uint64_t)models[r.model].n;
        }
      }
    }
    if (bp.n_units > 65536) return false;  // two unit passes at most
  }
  return bp.R < (1ull << 31) && bp.X < (1ull << 31);
}

}  // namespace

size_t gsr_batch_workspace_size(const gsr_model* models, int32_t n_models, const gsr_request* reqs, int32_t n_req,
                                uint32_t pair_capacity) {
  BatchPlan bp;
  if (!plan_batch(models, n_models, reqs, n_req, bp) || pair_capacity >= (1u << 30)) return 0;
  Carver c(nullptr);
  PipeBufs b;
  return carve(c, b, bp.views.size(), bp.R, pair_capacity, n_req, true, bp.X, bp.Q, false,
               bp.ordered ? std::max<uint64_t>(bp.R_sort, 1) : 0);
}

gsr_status gsr_render_batch(const gsr_model* models, int32_t n_models, const gsr_request* reqs, int32_t n_req,
                            uint32_t pair_capacity, void* ws, size_t ws_bytes, int32_t* req_status, gsr_timer* timer,
                            void* stream) {
  BatchPlan bp;
  if (!plan_batch(models, n_models, reqs, n_req, bp) || !ws || !req_status || pair_capacity >= (1u << 30))
    return GSR_EINVAL;
  const hipStream_t s = static_cast<hipStream_t>(stream);
  const uint32_t P = pair_capacity;
  const uint32_t R = (uint32_t)bp.R;
  const int n_views = (int)bp.views.size();
  const uint32_t n_sort = bp.ordered ? (uint32_t)std::max<uint64_t>(bp.R_sort, 1) : 0u;
  Carver c(ws);
  PipeBufs b;
  if (carve(c, b, n_views, R, P, n_req, true, bp.X, bp.Q, false, n_sort) > ws_bytes) return GSR_ENOSPACE;
  // per-view transmittance / last index scratch
  size_t q_off = 0;
  for (ViewD& d : bp.views) {
    d.pix = b.pix + 4 * q_off;
    d.last = b.last + q_off;
    q_off += (size_t)d.W * d.H;
  }
  WordUpload up;
  HIP_TRY(upload_views(b.views, bp.views.data(), n_views, up, s));
  HIP_TRY(launch_upload(b.req_rec, bp.req_rec.data(), (size_t)n_req + 1, s));
  HIP_TRY(clear_workspace(b, b.counters, false, b.ranges, bp.X, R, P, b.sel, s, &up, nullptr, 0, n_sort));
  if (bp.ordered) HIP_TRY(launch_set_u32(&b.gwords[0], n_sort, s));
  {
    StageScope sc(timer, GSR_STAGE_PROJECT, s);
    for (int m = 0; m < n_models; ++m) {
      std::vector<int> ids;
      for (int v = 0; v < n_views; ++v)
        if ((int)bp.views[v].model == m) ids.push_back(v);
      if (ids.empty()) continue;
      const ModelD md = make_model(models[m]);
      for (const JobD& j : make_jobs(md, ids))
        HIP_TRY(launch_project(j, b.views, b.records, b.n_tiles, b.tile_box, bp.ordered ? b.gk_a : nullptr,
                               bp.ordered ? b.gv_a : nullptr, b.counters, s));
    }
  }
  {
    StageScope sc(timer, GSR_STAGE_SCAN, s);
    if (bp.ordered)
      HIP_TRY(order_before_pairs(b, b.views, n_views, R, n_sort, bp.n_units, b.offsets, b.counters, P, s));
    else
      HIP_TRY(launch_scan(b.n_tiles, b.offsets, b.scan_status, &b.ctl->scan_ticket, R, b.counters, P, s));
    // (a request's records keep their positions in the emission sequence,
    // so its pairs end at offsets[req_rec[q + 1]] in either order)
    HIP_TRY(launch_batch_status(b.req_rec, n_req, b.offsets, P, b.counters, req_status, s));
  }
  {
    StageScope sc(timer, GSR_STAGE_DUPLICATE, s);
    if (bp.ordered)
      HIP_TRY(launch_duplicate(b.n_tiles_seq, b.offsets, b.tile_box_seq, R, b.counters, P, b.keys_a, b.vals,
                               b.rec_of, s, b.seq_rec));
    else
      HIP_TRY(launch_duplicate(b.n_tiles, b.offsets, b.tile_box, R, b.counters, P, b.keys_a, b.vals, b.rec_of, s));
  }
  {
    StageScope sc(timer, GSR_STAGE_SORT, s);
    if (tile_sort12(bp.X, P))
      HIP_TRY(launch_tile_sort12(b.keys_a, b.keys_b, b.vals, b.vals + P, b.counters, P, (uint32_t)bp.X,
                                 b.ctl->hist12, b.status, b.ranges, b.ctl->tile_class, b.class_list, b.sel,
                                 b.counters + kCntError, s));
    else
      HIP_TRY(launch_sort(b.keys_a, b.keys_b, b.vals, b.vals + P, b.counters, P, kDepthPasses,
                          tile_pass_end(bp.X), b.ctl->hist, b.status, b.ctl->pass_ctr, b.sel,
                          b.counters + kCntError, s));
  }
  {
    StageScope sc(timer, GSR_STAGE_RANGES, s);
    if (!tile_sort12(bp.X, P)) {  // (the one-pass grouping writes the ranges and classes itself)
      HIP_TRY(launch_ranges(b.keys_a, b.keys_b, b.sel, b.counters, P, (uint32_t)bp.X, b.ranges, s));
      HIP_TRY(launch_tile_order(b.ranges, (uint32_t)bp.X, b.ctl->tile_class, b.class_list, s));
    }
  }
  {
    StageScope sc(timer, GSR_STAGE_SORT, s);
    if (bp.ordered)  // the pairs of every tile are in depth order already
      HIP_TRY(launch_finalize_pairs(b.vals, b.vals + P, b.keys_a, b.keys_b, b.sel, b.rec_of, b.counters, P, nullptr,
                                    nullptr, s));
    else
      HIP_TRY(launch_sort_segments(b.keys_a, b.keys_b, b.vals, b.vals + P, b.sel, b.ranges, (uint32_t)bp.X,
                                   b.rec_of, b.counters, P, nullptr, nullptr, b.ctl->tile_class, b.class_list,
                                   &b.ctl->seg_ticket, b.counters + kCntError, s));
  }
  {
    StageScope sc(timer, GSR_STAGE_BLEND, s);
    HIP_TRY(launch_blend_fwd_tile(b.views, n_views, (uint32_t)bp.X, b.records, R, b.vals, b.sel, P, b.ranges,
                                  nullptr, 0, req_status, nullptr, b.ctl->tile_class, b.class_list, s));
  }
  HIP_TRY(launch_batch_error(b.counters, n_req, req_status, s));
  return GSR_OK;
}

gsr_status gsr_activate(const gsr_model* model, float* scale_out, float* opacity_out, void* stream) {
  if (!model_ok(model) || model->format != GSR_FORMAT_F32 || (model->n > 0 && (!scale_out || !opacity_out)))
    return GSR_EINVAL;
  HIP_TRY(launch_activate(make_model(*model), scale_out, opacity_out, static_cast<hipStream_t>(stream)));
  return GSR_OK;
}

size_t gsr_l1_loss_workspace_size(int32_t n_views, int32_t width, int32_t height) {
  if (n_views <= 0 || n_views > kMaxJobViews || width <= 0 || height <= 0) return 0;
  const uint64_t hw = (uint64_t)width * (uint64_t)height;
  if (hw * (uint64_t)n_views >= (1ull << 31)) return 0;
  return 8 * (size_t)std::min<uint32_t>(l1_loss_blocks(n_views, (int)hw), 1024u);
}

gsr_status gsr_l1_alpha_loss(int32_t n_views, int32_t width, int32_t height, const float* rgb, const float* alpha,
                             const float* target_rgb, const float* target_alpha, const float* bg_host, void* ws,
                             size_t ws_bytes, float* loss, const float* g_loss, float* dL_drgb, float* dL_dalpha,
                             void* stream) {
  const size_t need = gsr_l1_loss_workspace_size(n_views, width, height);
  if (need == 0 || !rgb || !alpha || !target_rgb || !target_alpha || !bg_host || !ws) return GSR_EINVAL;
  if ((dL_drgb == nullptr) != (dL_dalpha == nullptr)) return GSR_EINVAL;
  if (ws_bytes < need) return GSR_ENOSPACE;
  HIP_TRY(launch_l1_loss(n_views, width * height, rgb, alpha, target_rgb, target_alpha, bg_host,
                         static_cast<float*>(ws), loss, g_loss, dL_drgb, dL_dalpha, static_cast<hipStream_t>(stream)));
  return GSR_OK;
}

}  // extern "C"
