// Per-tile front-to-back compositing and its backward.
//
// Per pixel, front to back: alpha = min(0.99, o exp(-q/2)) with
// q = d^T conic d; pairs with q < 0 (rounding) or alpha < 1/255 are skipped;
// a pair that would bring T below 1e-4 ends the pixel without being blended.
//
// A tile's depth-sorted pairs are handled in batches of (at most) 256: a
// batch's records are staged through LDS once and every wave builds the
// compacted list of the batch's pairs whose ellipse of possible
// alpha >= 1/255 (the conic's minimum over the wave's pixel rectangle) meets
// its pixels, and walks only that list.
//
// Forward: one block per tile walks its batches in order (below).
//
// Backward: one block per (tile, batch) - the heavy tiles' lists are walked
// by many blocks at once, one pixel per thread, each wave an 8 x 8 quadrant.
// Each block starts at the end of its batch: the transmittance there is the
// next batch's checkpoint (or the final one), the colour behind it is the
// background term plus the later batches' colours, summed from the back.  It
// walks the batch back to front, rebuilding T by division by (1 - alpha)
// (alpha <= 0.99) and carrying the upstream-weighted colour behind each pair
// normalised by the transmittance behind it (a running convex combination),
// which keeps it relatively accurate deep in a pixel's list.  The
// per-pixel gradients of each pair are summed over the wave - eight of them
// by a reduce-scatter with the lane-half and row swaps (each step halves the
// values a lane carries), the ninth and the max with DPP - the four wave sums
// in a fixed order through LDS, and written as the pair's partial gradient:
// no atomics, bitwise reproducible.
#include "common.hpp"
#include "cull.hpp"

namespace gsr {

// G = exp(-q / 2) = 2^(kPowScale q): the kernels evaluate q from the record's
// conic (b staged doubled, which is exact) and scale it once.  Staging the
// conic pre-multiplied by kPowScale would save that multiply but round each
// coefficient once per splat: the same relative error at every pixel of the
// splat, which the gradient sums over its pixels would then add up
// coherently (thin splats, whose q is a small difference of large terms,
// lose several digits that way).
constexpr float kPowScale = -0.72134752044448170368f;

struct BatchLds {
  float4 a[kBatch];    // u, v, conic a, 2 b
  float4 b[kBatch];    // conic c, opacity, r, g
  float c[kBatch];     // b
};

__device__ __forceinline__ int find_view(const ViewD* __restrict__ views, int n_views, uint32_t tile) {
  int lo = 0, hi = n_views - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (views[mid].tile_off <= tile) lo = mid; else hi = mid - 1;
  }
  return lo;
}

__device__ __forceinline__ void pixel_of(int tid, int tx, int ty, int& px, int& py) {
  const int wave = tid >> 6, lane = tid & 63;
  px = tx * kTile + (wave & 1) * 8 + (lane & 7);
  py = ty * kTile + (wave >> 1) * 8 + (lane >> 3);
}

// One pair's record in registers (loaded a batch ahead of its use).
struct Staged {
  float4 a, b;
  float c;
};

__device__ __forceinline__ Staged fetch_record(const float* __restrict__ records, uint32_t n_rec, uint32_t r,
                                               bool ok) {
  Staged st;
  st.a = make_float4(0.f, 0.f, 0.f, 0.f);
  st.b = st.a;
  st.c = 0.f;
  if (ok) {
    if (r >= n_rec) r = 0;  // never read out of range (a sort fault shows up as wrong pixels)
    const float4* rec = reinterpret_cast<const float4*>(records + (size_t)r * kRecordFloats);
    st.a = rec[0];
    st.b = rec[1];
    st.c = records[(size_t)r * kRecordFloats + 8];
  }
  return st;
}

__device__ __forceinline__ Staged fetch(const float* __restrict__ records, uint32_t n_rec,
                                        const uint32_t* __restrict__ vals, uint32_t k, bool ok) {
  return fetch_record(records, n_rec, ok ? vals[k] : 0u, ok);
}

// Cut-off of the pair's reach: o exp(-q/2) >= 1/255 needs q <= 2 ln(255 o).
// A relative margin of 1e-2 plus 0.05 on q covers the rounding of q, exp
// and this computation, so skipping a pair for pixel centres where its q
// exceeds the cut-off never changes a result.  The cut-off is negative
// (nothing reachable) when 255 o < 1.
__device__ __forceinline__ float reach_cutoff(float opacity) {
  return fminf(kQMax, 2.f * __logf(255.f * opacity)) * 1.01f + 0.05f;
}

__device__ __forceinline__ void put(BatchLds& L, const Staged& st, bool ok, int tid) {
  if (ok) {
    L.a[tid] = make_float4(st.a.x, st.a.y, st.a.z, 2.f * st.a.w);
    L.b[tid] = st.b;
    L.c[tid] = st.c;
  }
}

// A batch's records as they lie in memory (floats 0-3, 4-7 and 8 of each):
// the forward loads them from global memory straight into LDS, the next
// batch's while the current one is blended.
struct BatchRaw {
  float4 a[kBatch];  // u, v, conic a, b
  float4 b[kBatch];  // conic c, opacity, r, g
  float c[kBatch];   // b
};

// s_waitcnt operands: vmcnt(0), and lgkmcnt(0), each leaving the other
// counters alone
constexpr int kWaitVm0 = 0x0F70;
constexpr int kWaitLgkm0 = 0xC07F;

// A barrier for LDS traffic only: the wave's LDS accesses complete, then the
// block meets (the signal fences keep the compiler from moving memory
// accesses across it).  Loads into LDS in flight keep running, where
// __syncthreads would wait for them.
__device__ __forceinline__ void lds_barrier() {
  __atomic_signal_fence(__ATOMIC_SEQ_CST);
  __builtin_amdgcn_s_waitcnt(kWaitLgkm0);
  __builtin_amdgcn_s_barrier();
  __atomic_signal_fence(__ATOMIC_SEQ_CST);
}

typedef __attribute__((address_space(3))) void lds_void;

// LDS address of p as a plain number: a load into LDS aimed at it carries no
// alias information, so the compiler puts no wait for it before the reads
// that follow (it would otherwise wait before every read of the same LDS
// array, the batch in use among them).  The kernel waits for these loads
// itself, before the barrier that precedes the first read of their data.
__device__ __forceinline__ lds_void* lds_target(void* p) {
  return (lds_void*)(size_t)(uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)(size_t)(lds_void*)p);
}

// Starts the loads of one wave's 64 records of a batch into its LDS slots
// 64 w .. 64 w + 63 (w = the wave; lane l's record lands in slot 64 w + l):
// the data skips registers and has landed once the wave's vector-memory
// count has drained.  Every lane loads (a lane without a pair loads record
// 0), so the slots are always written whole.
__device__ __forceinline__ void stage_async(BatchRaw& D, const float* __restrict__ records, uint32_t n_rec,
                                            uint32_t r, bool ok) {
  if (!ok || r >= n_rec) r = 0;
  const float* g = records + (size_t)r * kRecordFloats;
  const int w0 = __builtin_amdgcn_readfirstlane((int)threadIdx.x) & ~63;
  __builtin_amdgcn_global_load_lds(g, lds_target(&D.a[w0]), 16, 0, 0);
  __builtin_amdgcn_global_load_lds(g + 4, lds_target(&D.b[w0]), 16, 0, 0);
  __builtin_amdgcn_global_load_lds(g + 8, lds_target(&D.c[w0]), 4, 0, 0);
}

// Lane permutation within rows / quads (DPP); lanes a row mask leaves out
// read 0.
template <unsigned CTRL, unsigned ROW_MASK>
__device__ __forceinline__ float dpp(float v) {
  return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, ROW_MASK, 0xF, false));
}

__device__ __forceinline__ uint64_t lanes_below() {
  const int lane = threadIdx.x & 63;
  return lane == 0 ? 0ull : (~0ull >> (64 - lane));
}

// Block memberships of a batch: thread t of a 1024-thread block takes pair
// t mod 256 and the tile's block row t / 256 and writes the 4 bits of the
// row's 4 x 4 blocks the pair's ellipse reaches (band_blocks) to
// nib[row][pair].  A tile is 4 x 4 such blocks; bit 4 row + column of a
// pair's 16-bit block mask is block (column, row).
static_assert(kBatch * 4 == 1024, "one block row per thread");

__device__ __forceinline__ void block_nibbles(const BatchRaw& L, uint8_t (*nib)[kBatch], int n, float tx0,
                                              float ty0) {
  const int j = threadIdx.x & (kBatch - 1), r = threadIdx.x >> 8;
  uint32_t bits = 0u;
  if (j < n) {
    const float4 A = L.a[j], B = L.b[j];
    bits = band_blocks(A.x, A.y, A.z, A.w, B.x, reach_cutoff(B.y), tx0, ty0 + 4.f * (float)r);
  }
  nib[r][j] = (uint8_t)bits;
}

// The wave's list of the batch's pairs (ascending, j < n) whose ellipse
// reaches its block (bit `col` of the block row's nibbles); each lane tests
// one pair per round, a ballot compacts the hits.  Returns the
// (wave-uniform) count.  Pairs not in the list cannot reach alpha >= 1/255 on
// any of the wave's pixels, so skipping them changes nothing.
__device__ __forceinline__ int wave_list(const uint8_t* nib_row, int col, uint8_t* list, int n) {
  const int lane = threadIdx.x & 63;
  int cnt = 0;
#pragma unroll
  for (int r = 0; r < kBatch / 64; ++r) {
    const int j = r * 64 + lane;
    const bool hit = j < n && ((nib_row[j] >> col) & 1u);
    const uint64_t m = __ballot(hit);
    if (hit) list[cnt + __popcll(m & lanes_below())] = (uint8_t)j;
    cnt += __popcll(m);
  }
  __builtin_amdgcn_wave_barrier();
  return cnt;
}

// Base-2 exponent kPowScale q of one pair at a pixel offset (dx, dy) =
// centre - pixel, q = a dx^2 + 2 b dx dy + c dy^2 from the staged conic;
// G = 2^power.  q is rounded exactly as its plain left-to-right evaluation
// is - (a dx) dx + (c dy) dy first, then + (2b dx) dy, no fused operations -
// which is also the reference's order: for a thin splat q is a small
// difference of terms thousands of times larger, and any other order rounds
// it differently by enough to move alpha across the 1/255 cut-off.  This file
// is compiled without implicit FMA contraction, so the forward and the
// backward evaluate this (and alpha) with the same instructions and take
// the same skip decisions.  power <= 0 is q >= 0.
__device__ __forceinline__ float pair_power(const float4 A, const float4 B, float dx, float dy) {
  const float qa = (A.z * dx) * dx, qc = (B.x * dy) * dy, qb = (A.w * dx) * dy;
  return kPowScale * ((qa + qc) + qb);
}

__device__ __forceinline__ float pair_gauss(float power) { return __builtin_amdgcn_exp2f(power); }

__device__ __forceinline__ float pair_alpha(const float4 B, float power) {
  return fminf(kAlphaMax, B.y * pair_gauss(power));
}

// Wave ballot of a condition (no round trip of the flag through a VGPR).
__device__ __forceinline__ uint64_t ballot(bool x) { return __builtin_amdgcn_ballot_w64(x); }

// ---------------------------------------------------------------- forward
// One 1024-thread block per tile walks the tile's batches in order.  Each of
// its 16 waves owns a 4 x 4 pixel sub-tile and gives every pixel a quad of
// four lanes: a step takes the next four pairs of the wave's list, one per
// lane of each quad, and advances the pixel's transmittance by the quad's
// prefix product of (1 - alpha) - four pairs per step of the serial chain
// instead of one.  The first pair (in list order) that would bring T below
// 1e-4 ends the pixel and is not blended, as are the pairs after it.  Per
// batch the records are staged once, a wave with a live pixel builds its list
// (pairs whose ellipse meets the sub-tile), and the block leaves when every
// pixel has stopped.  Per batch it stores the checkpoint (T entering the
// batch, then colour behind the batch) the backward starts from, at the
// pixel's index in the backward's 8 x 8-quadrant layout (ckpt may be null: render
// only, then batch_tile is not written).  Tile t's batches have the indices
// first_batch(t) + c, c = 0, 1, ...: distinct over the tiles and below
// P / 256 + X + 1 for any pair count P.  Each batch's word in batch_tile holds
// 1 + tile and, in the top byte, a work class for the backward's order: from
// the longest list any wave stepped through in the batch (16 classes of 16
// entries, heaviest first), the last class for batches never reached.
constexpr int kQuadPix = 4;  // sub-tile edge

// Checkpoint batch index of a tile's first batch: floor(start / 256) + t.
// Since floor((s + n) / 256) + 1 >= floor(s / 256) + ceil(n / 256), tile t + 1
// starts after tile t's last batch.
__device__ __forceinline__ uint32_t first_batch(uint32_t tile, uint32_t tile_start) {
  return tile_start / (uint32_t)kBatch + tile;
}

__device__ __forceinline__ uint32_t batch_word(uint32_t tile, uint32_t est) {
  const uint32_t cls = est == 0 ? kBatchClasses - 1 : (kBatch - min(est, (uint32_t)kBatch)) >> 4;
  return (tile + 1u) | (cls << 24);
}

// Full-mask lane permutation: every lane has a source, so no old value.
template <unsigned CTRL>
__device__ __forceinline__ float qperm(float v) {
  return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), CTRL, 0xF, 0xF, true));
}

__device__ __forceinline__ float quad_shift1(float x, int slot) {  // x of slot - 1, 1 for slot 0
  const float y = qperm<0x90>(x);                                // quad_perm [0,0,1,2]
  return slot >= 1 ? y : 1.f;
}

__device__ __forceinline__ float quad_shift2(float x, int slot) {  // x of slot - 2, 1 for slots 0, 1
  const float y = qperm<0x40>(x);                                // quad_perm [0,0,0,1]
  return slot >= 2 ? y : 1.f;
}

__device__ __forceinline__ float quad_sum(float v) {
  v += dpp<0xB1, 0xF>(v);  // quad_perm [1,0,3,2]
  v += dpp<0x4E, 0xF>(v);  // quad_perm [2,3,0,1]
  return v;
}

__device__ __forceinline__ uint32_t quad_max_u32(uint32_t v) {
  v = max(v, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0xB1, 0xF, 0xF, false));
  v = max(v, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x4E, 0xF, 0xF, false));
  return v;
}

// At most 80 SGPRs: two 1024-thread blocks per compute unit need it (with
// 81 the kernel measured 35 % slower, one block per compute unit at a time).
__global__ void __launch_bounds__(1024) __attribute__((amdgpu_num_sgpr(80)))
k_blend_tile(const ViewD* __restrict__ views, int n_views, uint32_t total_tiles, const float* __restrict__ records,
             uint32_t n_rec, const uint32_t* __restrict__ pair_vals, const uint32_t* __restrict__ sel, uint32_t cap,
             const uint32_t* __restrict__ ranges, uint32_t* __restrict__ batch_tile, uint32_t batch_cap,
             const int32_t* __restrict__ req_status, float4* __restrict__ ckpt,
             const uint32_t* __restrict__ class_count, const uint32_t* __restrict__ class_list) {
  __shared__ BatchRaw R[2];  // batch c's records in R[c & 1]
  __shared__ uint8_t lists[16][kBatch];
  __shared__ uint8_t nib[4][kBatch];
  // block b takes the b-th tile of the largest-first order (if given): the
  // class counts are read at once, the first wave finds b's class by a scan
  __shared__ uint32_t s_tile;
  uint32_t tile = blockIdx.x;
  if (class_count) {
    if (threadIdx.x < 64) {
      const uint32_t k = threadIdx.x;
      const uint32_t cnt = k < kTileClasses ? min(class_count[k], total_tiles) : 0u;
      const uint32_t inc = wave_scan_add(cnt);
      const uint32_t b = blockIdx.x;
      const bool here = k < kTileClasses && b >= inc - cnt && b < inc;
      if (here) s_tile = class_list[(size_t)k * total_tiles + (b - (inc - cnt))];
      if (__ballot(here) == 0ull && threadIdx.x == 0) s_tile = 0xFFFFFFFFu;
    }
    __syncthreads();
    tile = s_tile;
  }
  if (tile >= total_tiles) return;
  const int vi = find_view(views, n_views, tile);
  const ViewD& V = views[vi];
  if (req_status && req_status[V.request] != 0) return;  // a request that did not fit is not written
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  const int slot = lane & 3, p = lane >> 2;
  const uint32_t upto_slot = (2u << slot) - 1u;  // stop bits of the slots up to this one
  const uint32_t local = tile - V.tile_off;
  const int tx = (int)(local % (uint32_t)V.tiles_x), ty = (int)(local / (uint32_t)V.tiles_x);
  const int lx = (wave & 3) * kQuadPix + (p & 3), ly = (wave >> 2) * kQuadPix + (p >> 2);  // in the tile
  const int px = tx * kTile + lx, py = ty * kTile + ly;
  const int bidx = ((ly >> 3) * 2 + (lx >> 3)) * 64 + (ly & 7) * 8 + (lx & 7);  // backward's thread of this pixel
  const bool inside = px < V.W && py < V.H;
  const float fx = (float)px + 0.5f, fy = (float)py + 0.5f;
  const uint32_t* vals = pair_vals + (*sel ? cap : 0u);
  // a training forward leaves each sorted pair's block mask for the backward
  // in the other half of pair_vals (free once the sort is done)
  uint16_t* blk_out = ckpt ? reinterpret_cast<uint16_t*>(const_cast<uint32_t*>(pair_vals) + (*sel ? 0u : cap))
                           : nullptr;
  const uint32_t t_end = min(ranges[2 * tile + 1], cap);
  const uint32_t t_start = min(ranges[2 * tile], t_end);
  const uint32_t b0 = first_batch(tile, t_start);
  __shared__ uint32_t s_est;  // longest list stepped through in the current batch
  if (tid == 0) s_est = 0;
  uint8_t* list = lists[wave];
  float T = 1.f, C0 = 0.f, C1 = 0.f, C2 = 0.f;
  uint32_t last = 0;
  bool done = !inside;
  uint32_t n_ck = 0;  // batches processed (checkpoints written)
  // per batch parity, byte w: whether wave w still has a live pixel
  __shared__ __align__(16) uint32_t s_live[2][4];
  // Staging: waves 0-3 load the records of batch c + 1 straight into LDS
  // while batch c is blended, and the record ids of batch c + 2 into
  // registers; batch 0's loads start here.
  const bool stager = tid < kBatch;
  uint32_t rid = stager && t_start + (uint32_t)tid < t_end ? vals[t_start + tid] : 0u;
  if (stager && t_start < t_end) stage_async(R[0], records, n_rec, rid, t_start + (uint32_t)tid < t_end);
  {
    const uint32_t k = t_start + kBatch + (uint32_t)tid;
    rid = stager && k < t_end ? vals[k] : 0u;
  }
  for (uint32_t start = t_start, c = 0; start < t_end; start += kBatch, ++c) {
    // this batch's records have landed (each wave waits for its own loads);
    // the block leaves once every pixel has stopped: each wave posts its
    // flag, one barrier (which also shows the records to every wave and
    // orders the previous batch's reads of the other buffer before its
    // refill), every wave reads the sixteen posts (the other parity's posts
    // are rewritten only after the next batch's barriers)
    __builtin_amdgcn_s_waitcnt(kWaitVm0);
    {
      const bool any_live = __ballot(!done) != 0ull;
      if (lane == 0) reinterpret_cast<uint8_t*>(s_live[c & 1])[wave] = any_live ? 1 : 0;
      __syncthreads();
      const uint4 posts = *reinterpret_cast<const uint4*>(s_live[c & 1]);
      if ((posts.x | posts.y | posts.z | posts.w) == 0u) break;
    }
    if (ckpt && tid == 0 && c > 0) {
      if (b0 + c - 1 < batch_cap) batch_tile[b0 + c - 1] = batch_word(tile, s_est);
      s_est = 0;
    }
    const int n = (int)min((uint32_t)kBatch, t_end - start);
    const BatchRaw& L = R[c & 1];
    {
      const uint32_t nstart = start + kBatch;
      if (stager && nstart < t_end) stage_async(R[(c + 1) & 1], records, n_rec, rid, nstart + (uint32_t)tid < t_end);
      const uint32_t k = nstart + kBatch + (uint32_t)tid;
      rid = stager && k < t_end ? vals[k] : 0u;
    }
    block_nibbles(L, nib, n, (float)(tx * kTile) + 0.5f, (float)(ty * kTile) + 0.5f);
    lds_barrier();
    if (blk_out && tid < n)
      blk_out[start + tid] = (uint16_t)(nib[0][tid] | (nib[1][tid] << 4) | (nib[2][tid] << 8) | (nib[3][tid] << 12));
    const float T0 = T;
    float D0 = 0.f, D1 = 0.f, D2 = 0.f;
    uint32_t lst = 0;
    const int cnt = __ballot(!done) ? wave_list(nib[wave >> 2], wave & 3, list, n) : 0;
    int stepped = cnt;
    for (int t0 = 0; t0 < cnt; t0 += 4) {
      const int te = t0 + slot;
      const bool has = te < cnt;
      const int j = has ? (int)list[te] : 0;
      const float4 R4 = L.a[j], B = L.b[j];
      const float cb = L.c[j];
      const float4 A = make_float4(R4.x, R4.y, R4.z, 2.f * R4.w);  // b doubled (exact)
      const float power = pair_power(A, B, A.x - fx, A.y - fy);
      const float alpha = pair_alpha(B, power);
      const bool cand = has && !done && power <= 0.f && alpha >= kAlphaMin;
      const float f = cand ? 1.f - alpha : 1.f;
      float P = f * quad_shift1(f, slot);
      P = P * quad_shift2(P, slot);        // prod of f over slots <= slot
      const float E = quad_shift1(P, slot);  // over slots < slot
      const float Tn = T * P;
      const bool stop = cand && Tn < kTStop;
      // the quad's stop bits: a slot blends if no slot up to it stops
      const uint32_t sbits = (uint32_t)(ballot(stop) >> (lane & 60));
      const bool blend = cand && (sbits & upto_slot) == 0u;
      const float w = blend ? alpha * (T * E) : 0.f;
      D0 = fmaf(B.z, w, D0);
      D1 = fmaf(B.w, w, D1);
      D2 = fmaf(cb, w, D2);
      lst = blend ? start + (uint32_t)j + 1 : lst;
      // T after the quad's last blended slot: T times the quad's product of
      // (1 - alpha) over its blended slots (1 elsewhere; a quad that blends
      // nothing multiplies T by exactly 1)
      float g = blend ? f : 1.f;
      g *= dpp<0xB1, 0xF>(g);  // quad_perm [1,0,3,2]
      g *= dpp<0x4E, 0xF>(g);  // quad_perm [2,3,0,1]
      T *= g;
      done = done || (sbits & 0xFu) != 0u;
      if (ballot(!done) == 0ull) {
        stepped = min(cnt, t0 + 4);
        break;
      }
    }
    if (ckpt && lane == 0 && stepped > 0) atomicMax(&s_est, (uint32_t)stepped);
    D0 = quad_sum(D0);
    D1 = quad_sum(D1);
    D2 = quad_sum(D2);
    lst = quad_max_u32(lst);
    C0 += D0;
    C1 += D1;
    C2 += D2;
    last = lst ? lst : last;
    if (ckpt && slot == 0 && b0 + c < batch_cap) ckpt[(size_t)(b0 + c) * kBatch + bidx] = make_float4(T0, D0, D1, D2);
    n_ck = c + 1;
  }
  if (ckpt) {
    // the last batch reached, then the ones never reached
    __syncthreads();
    if (tid == 0 && n_ck > 0 && b0 + n_ck - 1 < batch_cap) batch_tile[b0 + n_ck - 1] = batch_word(tile, s_est);
    const uint32_t nb = (t_end - t_start + (uint32_t)kBatch - 1) / (uint32_t)kBatch;
    for (uint32_t c = n_ck + tid; c < nb; c += 1024)
      if (b0 + c < batch_cap) batch_tile[b0 + c] = batch_word(tile, 0);
  }
  if (ckpt && slot == 0) {
    // replace each batch's colour by the colour behind the batch: the
    // background under the final transmittance plus the later batches,
    // summed from the back (a batch after the pixel stopped adds 0)
    float a0 = T * V.bg[0], a1 = T * V.bg[1], a2 = T * V.bg[2];
    for (int cc = (int)n_ck - 1; cc >= 0; --cc) {
      if (b0 + (uint32_t)cc >= batch_cap) continue;
      float4* q = ckpt + (size_t)(b0 + (uint32_t)cc) * kBatch + bidx;
      const float4 d = *q;
      *q = make_float4(d.x, a0, a1, a2);
      a0 += d.y;
      a1 += d.z;
      a2 += d.w;
    }
  }
  if (!inside || slot != 0) return;
  const size_t pix = (size_t)py * V.W + px;
  const size_t plane = (size_t)V.W * V.H;
  V.rgb[pix] = fmaf(T, V.bg[0], C0);
  V.rgb[plane + pix] = fmaf(T, V.bg[1], C1);
  V.rgb[2 * plane + pix] = fmaf(T, V.bg[2], C2);
  V.alpha[pix] = 1.f - T;
  reinterpret_cast<float4*>(V.pix)[pix] = make_float4(T, C0, C1, C2);
  V.last[pix] = last;
}

hipError_t launch_blend_fwd_tile(const ViewD* views_dev, int n_views, uint32_t total_tiles, const float* records,
                                 uint32_t n_rec, const uint32_t* pair_vals, const uint32_t* sel, uint32_t cap,
                                 const uint32_t* ranges, uint32_t* batch_tile, uint32_t batch_cap,
                                 const int32_t* req_status, float4* ckpt, const uint32_t* class_count,
                                 const uint32_t* class_list, hipStream_t s) {
  if (total_tiles == 0) return hipSuccess;
  hipLaunchKernelGGL(k_blend_tile, dim3(total_tiles), dim3(1024), 0, s, views_dev, n_views, total_tiles, records,
                     n_rec, pair_vals, sel, cap, ranges, batch_tile, batch_cap, req_status, ckpt, class_count,
                     class_list);
  return hipGetLastError();
}

// ---------------------------------------------------------------- backward
// Wave64 reductions with DPP: quad swaps, half-row and row mirrors, then the
// row broadcasts 15 and 31; lane 63 ends with the result.

__device__ __forceinline__ float wave_sum63(float v) {
  v += dpp<0xB1, 0xF>(v);   // quad_perm [1,0,3,2]
  v += dpp<0x4E, 0xF>(v);   // quad_perm [2,3,0,1]
  v += dpp<0x141, 0xF>(v);  // row_half_mirror
  v += dpp<0x140, 0xF>(v);  // row_mirror
  v += dpp<0x142, 0xA>(v);  // row_bcast15 into rows 1 and 3
  v += dpp<0x143, 0xC>(v);  // row_bcast31 into rows 2 and 3
  return v;
}

template <unsigned CTRL, unsigned ROW_MASK>
__device__ __forceinline__ uint32_t dpp_u32(uint32_t v) {
  return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, CTRL, ROW_MASK, 0xF, false);
}

// For v >= 0 the float order is the order of the bit patterns: an integer
// max, which takes its DPP operand directly.
__device__ __forceinline__ float wave_max63(float v) {
  uint32_t u = __float_as_uint(v);
  u = max(u, dpp_u32<0xB1, 0xF>(u));
  u = max(u, dpp_u32<0x4E, 0xF>(u));
  u = max(u, dpp_u32<0x141, 0xF>(u));
  u = max(u, dpp_u32<0x140, 0xF>(u));
  u = max(u, dpp_u32<0x142, 0xA>(u));
  u = max(u, dpp_u32<0x143, 0xC>(u));
  return __uint_as_float(u);
}

// Reduce-scatter of two values over the wave halves: the swap exchanges the
// upper half of x with the lower half of y, so the sum holds x summed over
// lanes l and l+32 in the lower half and y (likewise) in the upper half.
__device__ __forceinline__ float swap32_add(float x, float y) {
  const auto r = __builtin_amdgcn_permlane32_swap(__float_as_uint(x), __float_as_uint(y), false, false);
  return __uint_as_float(r[0]) + __uint_as_float(r[1]);
}

// The same over 16-lane rows: rows 1 and 3 of x are exchanged with rows 0
// and 2 of y; the sum holds x (rows 0 and 2) and y (rows 1 and 3) summed over
// rows paired within each half.
__device__ __forceinline__ float swap16_add(float x, float y) {
  const auto r = __builtin_amdgcn_permlane16_swap(__float_as_uint(x), __float_as_uint(y), false, false);
  return __uint_as_float(r[0]) + __uint_as_float(r[1]);
}

// Sum over the 16 lanes of each row; every lane of the row ends with it.
__device__ __forceinline__ float row_sum16(float v) {
  v += dpp<0xB1, 0xF>(v);   // quad_perm [1,0,3,2]
  v += dpp<0x4E, 0xF>(v);   // quad_perm [2,3,0,1]
  v += dpp<0x141, 0xF>(v);  // row_half_mirror
  v += dpp<0x140, 0xF>(v);  // row_mirror
  return v;
}

// Per pair, the wave sums of: h dx, h dy, h dx^2, h dx dy, h dy^2, h, and the
// three colour weights G_ch w, plus the wave maximum of w = alpha T.  Here
// h = dL/dalpha * o * G and (dx, dy) = mean - pixel centre.  With the conic
// (a, b, c) the screen-space gradients are linear in these sums:
//   dL/du = -(a Shx + b Shy), dL/dv = -(b Shx + c Shy),
//   dL/da = -Shxx / 2, dL/db = -Shxy, dL/dc = -Shyy / 2, dL/do = Sh / o,
// so the per-pixel work needs no conic products and the conic is applied
// once per pair after the sums.
constexpr int kGradSlots = 10;

// g_pair: [P][12] per pair, at its emission index (pair_emit of its sorted
// position), so that a Gaussian's partials are contiguous: u, v, conic a,
// b, c, opacity, r, g, b, max alpha*T, 2 unused; alive[e] = 1 marks the
// entries written (pairs of batches the forward never evaluated at a live
// pixel are zero and skipped).
// The backward's block order: batches by work class, heaviest first, so that
// the longest blocks start early instead of ending the launch.  Each block
// buckets 4096 batch words; per class one atomic reserves its range of the
// class's list (order_list[k][n_batches]); the order inside a class is
// arbitrary (each batch's results do not depend on it).
constexpr uint32_t kOrderItems = 4;

__global__ void __launch_bounds__(1024)
k_batch_order(const uint32_t* __restrict__ batch_tile, uint32_t n, uint32_t* __restrict__ order_cnt,
              uint32_t* __restrict__ order_list) {
  __shared__ uint32_t s_cnt[kBatchClasses], s_base[kBatchClasses];
  const uint32_t tid = threadIdx.x;
  if (tid < kBatchClasses) s_cnt[tid] = 0;
  __syncthreads();
  const uint32_t i0 = blockIdx.x * (1024u * kOrderItems) + tid;
  uint32_t cls[kOrderItems], rank[kOrderItems];
#pragma unroll
  for (uint32_t r = 0; r < kOrderItems; ++r) {
    const uint32_t i = i0 + r * 1024u;
    const uint32_t word = i < n ? batch_tile[i] : 0u;
    cls[r] = (word & kBatchTileMask) ? min(word >> 24, kBatchClasses - 1) : kBatchClasses;
    if (cls[r] < kBatchClasses) rank[r] = atomicAdd(&s_cnt[cls[r]], 1u);
  }
  __syncthreads();
  if (tid < kBatchClasses) s_base[tid] = s_cnt[tid] ? atomicAdd(&order_cnt[tid], s_cnt[tid]) : 0u;
  __syncthreads();
#pragma unroll
  for (uint32_t r = 0; r < kOrderItems; ++r)
    if (cls[r] < kBatchClasses) order_list[(size_t)cls[r] * n + s_base[cls[r]] + rank[r]] = i0 + r * 1024u;
}

hipError_t launch_batch_order(const uint32_t* batch_tile, uint32_t n_batches, uint32_t* order_cnt,
                              uint32_t* order_list, hipStream_t s) {
  if (n_batches == 0) return hipSuccess;
  const uint32_t per = 1024u * kOrderItems;
  hipLaunchKernelGGL(k_batch_order, dim3((n_batches + per - 1) / per), dim3(1024), 0, s, batch_tile, n_batches,
                     order_cnt, order_list);
  return hipGetLastError();
}

__global__ void __launch_bounds__(256)
k_blend_bwd(const ViewD* __restrict__ views, int n_views, const float* __restrict__ records, uint32_t n_rec,
            const uint32_t* __restrict__ pair_vals, const uint32_t* __restrict__ sel, uint32_t cap,
            const uint32_t* __restrict__ ranges, const float4* __restrict__ ckpt,
            const uint32_t* __restrict__ batch_tile, uint32_t n_batches, const uint32_t* __restrict__ order_cnt,
            const uint32_t* __restrict__ order_list, const float* __restrict__ dL_drgb,
            const float* __restrict__ dL_dalpha, const uint32_t* __restrict__ pair_emit,
            float* __restrict__ g_pair, uint8_t* __restrict__ alive, int want_max) {
  __shared__ BatchLds L;
  constexpr int kSub = 64;  // pairs whose wave partials are held in LDS at a time
  // one float of padding per row: the nine lanes that store a pair's sums
  // write rows q_lane = 0..8 at one column, which then fall in different banks
  constexpr int kSubPad = kSub + 1;
  __shared__ float part[4][kGradSlots][kSubPad];
  __shared__ uint16_t s_blk[kBatch];  // block masks the forward left
  // block b takes the b-th batch of the heaviest-first order: the first wave
  // scans the class counts and finds b's class
  __shared__ uint32_t s_bi;
  if (threadIdx.x < 64) {
    const uint32_t k = threadIdx.x;
    const uint32_t cnt = k < kBatchClasses ? min(order_cnt[k], n_batches) : 0u;
    const uint32_t inc = wave_scan_add(cnt);
    const uint32_t b = blockIdx.x;
    const bool here = k < kBatchClasses && b >= inc - cnt && b < inc;
    if (here) s_bi = order_list[(size_t)k * n_batches + (b - (inc - cnt))];
    if (__ballot(here) == 0ull && threadIdx.x == 0) s_bi = 0xFFFFFFFFu;
  }
  __syncthreads();
  const uint32_t bi = s_bi;
  if (bi >= n_batches) return;
  const uint32_t word = batch_tile[bi];
  const uint32_t tile_p1 = word & kBatchTileMask;
  if (tile_p1 == 0) return;  // no tile's batch
  const uint32_t tile = tile_p1 - 1u;
  const uint32_t c = bi - first_batch(tile, ranges[2 * tile]);
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const uint32_t t_end = min(ranges[2 * tile + 1], cap);
  const uint32_t start = min(ranges[2 * tile] + c * kBatch, t_end);
  const uint32_t end = min(start + kBatch, t_end);
  const int n = (int)(end - start);
  // The forward evaluated none of this batch's pairs at a live pixel (its
  // pixels had stopped, or no pair's ellipse reaches one): every partial is
  // zero, and none is written (their alive flags stay 0).
  if ((word >> 24) == kBatchClasses - 1) return;
  const int vi = find_view(views, n_views, tile);
  const ViewD& V = views[vi];
  const uint32_t* vals = pair_vals + (*sel ? cap : 0u);

  const uint32_t local = tile - V.tile_off;
  const int tx = (int)(local % (uint32_t)V.tiles_x), ty = (int)(local / (uint32_t)V.tiles_x);
  int px, py;
  pixel_of(tid, tx, ty, px, py);
  const bool inside = px < V.W && py < V.H;
  const float fx = (float)px + 0.5f, fy = (float)py + 0.5f;
  const size_t plane = (size_t)V.W * V.H;
  const size_t pix = inside ? (size_t)py * V.W + px : 0;
  const size_t vpix = (size_t)vi * plane;  // views of one call share a resolution
  // lim: this pixel's pairs j < lim lie in front of its last blended pair
  int lim = 0;
  // With S the colour behind the current pair and T the transmittance behind
  // it, dL/dalpha = Tb (G . c) - P / (1 - alpha) where P = sum_ch G_ch S_ch -
  // GA Tfin.  The kernel carries Q = P / T instead: then dL/dalpha =
  // Tb (G . c - Q) and, per blended pair, Q <- Q + alpha (G . c - Q), a convex
  // combination of the pairs' G . c behind (and G . bg - GA), so Q keeps a
  // relative error of a few roundings however deep the pixel, and only the
  // factor Tb carries the transmittance rebuilt by division.  That division
  // runs in double: in float each of up to 256 steps back from the batch end
  // would add a rounding, several times the error a float forward leaves in
  // T, which near-cancelling per-pixel terms turn into gradient error.
  double T = 1.0;
  float Tfin = 1.f, Q = 0.f, G0 = 0.f, G1 = 0.f, G2 = 0.f, GA = 0.f;
  if (inside) {
    const uint32_t plast = V.last[pix];
    if (plast > start) {
      lim = (int)min(plast - start, (uint32_t)n);
      const float4 ps = reinterpret_cast<const float4*>(V.pix)[pix];
      Tfin = ps.x;
      // batch of the pixel's last blended pair (>= c)
      const uint32_t tile_start = ranges[2 * tile];
      const uint32_t c_last = (plast - 1 - tile_start) / kBatch;
      const float4* tck = ckpt + (size_t)(bi - c) * kBatch + tid;
      // transmittance at the end of this batch, colour behind it
      T = (c_last == c) ? Tfin : tck[(size_t)(c + 1) * kBatch].x;
      const float4 sb = tck[(size_t)c * kBatch];
      if (dL_drgb) {
        G0 = dL_drgb[3 * vpix + pix];
        G1 = dL_drgb[3 * vpix + plane + pix];
        G2 = dL_drgb[3 * vpix + 2 * plane + pix];
      }
      if (dL_dalpha) GA = dL_dalpha[vpix + pix];
      Q = __fdiv_rn(fmaf(G2, sb.w, fmaf(G1, sb.z, fmaf(G0, sb.y, -GA * Tfin))), (float)T);
    }
  }
  // thread t stages pair t and later combines its sums (sub-batch t / kSub
  // runs on wave t / kSub), so the pair's exact conic, opacity and emission
  // index stay in its registers
  const Staged mine = fetch(records, n_rec, vals, start + tid, tid < n);
  put(L, mine, tid < n, tid);
  {
    const uint16_t* blk = reinterpret_cast<const uint16_t*>(pair_vals + (*sel ? 0u : cap));
    s_blk[tid] = tid < n ? blk[start + tid] : (uint16_t)0;
  }
  uint32_t my_emit = tid < n ? pair_emit[start + tid] : 0u;
  if (my_emit >= cap) my_emit = 0;  // never write out of range (an inconsistent sort shows up as wrong gradients)
  for (int i = tid; i < 4 * kGradSlots * kSubPad; i += 256) (&part[0][0][0])[i] = 0.f;
  // the wave's 8 x 8 quadrant: 2 x 2 of the tile's 4 x 4 blocks
  const uint32_t qmask = 0x33u << (2 * (wave & 1) + 8 * (wave >> 1));
  // the wave's reach: no pair at or behind its pixels' last blended pair counts
  int n_wave = lim;
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) n_wave = max(n_wave, __shfl_xor(n_wave, off, 64));
  n_wave = __builtin_amdgcn_readfirstlane(n_wave);
  __syncthreads();

  // back to front in sub-batches of kSub pairs; after each, the four wave
  // partials of its pairs are summed in a fixed order and written out
  const int n_sub = (n + kSub - 1) / kSub;
  // where the 18-value reduce-scatter leaves each sum: rows 0-1 hold the back
  // pair of a step, rows 2-3 the front one; lane bits 3, 2 and the row's
  // parity pick one of the first eight sums, lane bit 1 the ninth
  const int row = lane >> 4;
  const int q_lane = (lane & 2) ? 8 : 2 * (((lane >> 2) & 1) * 2 + ((lane >> 3) & 1)) + (row & 1);
  const bool writer = !(lane & 1) && (!(lane & 2) || ((lane & 12) == 0 && !(row & 1)));
  const bool front = row >= 2;
  float* part_lane = &part[wave][q_lane][0];
  struct PairLds {
    float4 A, B;
    float c;
  };
  auto load = [&](int j) -> PairLds { return PairLds{L.a[j], L.b[j], L.c[j]}; };
  // one pair for this pixel: updates T and Q (back to front) and returns the
  // nine per-pixel terms; inactive pairs give zeros
  auto eval = [&](const PairLds& P, int j, bool valid, float (&v)[9], float& w) -> bool {
    // branch-free: every lane evaluates the pair, selects keep what counts
    const float4 A = P.A, B = P.B;
    const float dx = A.x - fx, dy = A.y - fy;
    const float power = pair_power(A, B, dx, dy);
    const float G = pair_gauss(power);
    const float oG = B.y * G;
    const float alpha = fminf(kAlphaMax, oG);
    const bool contrib = valid && j < lim && power <= 0.f && alpha >= kAlphaMin;
    const bool has_grad = contrib && !(oG > kAlphaMax);  // alpha not clamped: it has a gradient
    // ae is alpha where the pair blends and 0 elsewhere: with it the colour
    // weight, the Q step and the transmittance need no further selects
    const float ae = contrib ? alpha : 0.f;
    // transmittance in front of this pair: T / (1 - alpha), alpha <= 0.99,
    // the reciprocal refined by one Newton step (a few units of 2^-53)
    const double om = 1.0 - (double)ae;
    double inv1m = __builtin_amdgcn_rcp(om);
    inv1m = fma(inv1m, fma(-om, inv1m, 1.0), inv1m);
    const double Tbd = T * inv1m;
    const float Tb = (float)Tbd;
    const float gcol = fmaf(G2, P.c, fmaf(G1, B.w, G0 * B.z));  // G . c
    const float dq = gcol - Q;
    w = ae * Tb;
    Q = fmaf(ae, dq, Q);
    T = contrib ? Tbd : T;
    const float h = (Tb * dq) * (has_grad ? oG : 0.f);  // dL/dalpha o G
    const float hx = h * dx, hy = h * dy;
    v[0] = hx;
    v[1] = hy;
    v[2] = hx * dx;
    v[3] = hx * dy;
    v[4] = hy * dy;
    v[5] = h;
    v[6] = G0 * w;
    v[7] = G1 * w;
    v[8] = G2 * w;
    return contrib;
  };
  // highest pair of a wave-uniform bit set, removed from it
  auto pop = [](uint64_t& m) -> int {
    const int b = 63 - (int)__builtin_clzll(m);
    m &= ~(1ull << b);
    return b;
  };
  for (int sb = n_sub - 1; sb >= 0; --sb) {
    const int j0 = sb * kSub;
    // the wave's pairs of this sub-batch: lane l tests pair j0 + l, a ballot
    // gives the set of those that can reach alpha >= 1/255 at a pixel centre
    // of its quadrant in front of its pixels' last blended pair
    const int jl = j0 + lane;
    uint64_t m = ballot(jl < n_wave && (s_blk[jl] & qmask) != 0u);
    // two pairs per step (the second, in front, may be absent)
    while (m != 0ull) {
      const int ja = pop(m);
      const bool hb = m != 0ull;
      const int jb = hb ? pop(m) : ja;
      const PairLds pa = load(j0 + ja), pb = load(j0 + jb);
      float va[9], vb[9], wa, wb;
      const bool ca = eval(pa, j0 + ja, true, va, wa);
      const bool cb = eval(pb, j0 + jb, hb, vb, wb);
      if (ballot(ca || cb) != 0ull) {
        // reduce-scatter: halves (back | front pair), then row pairs, then
        // within rows by mirror exchanges that keep one operand per lane half
        float X[9];
#pragma unroll
        for (int q = 0; q < 9; ++q) X[q] = swap32_add(va[q], vb[q]);
        const float Y0 = swap16_add(X[0], X[1]), Y1 = swap16_add(X[2], X[3]);
        const float Y2 = swap16_add(X[4], X[5]), Y3 = swap16_add(X[6], X[7]);
        const float Y4 = swap16_add(X[8], X[8]);
        const bool b3 = lane & 8, b2 = lane & 4, b1 = lane & 2;
        const float Z0 = (b3 ? Y1 : Y0) + dpp<0x140, 0xF>(b3 ? Y0 : Y1);  // row_mirror
        const float Z1 = (b3 ? Y3 : Y2) + dpp<0x140, 0xF>(b3 ? Y2 : Y3);
        const float Z2 = Y4 + dpp<0x140, 0xF>(Y4);
        const float W0 = (b2 ? Z1 : Z0) + dpp<0x141, 0xF>(b2 ? Z0 : Z1);  // row_half_mirror
        const float W1 = Z2 + dpp<0x141, 0xF>(Z2);
        float R = (b1 ? W1 : W0) + dpp<0x4E, 0xF>(b1 ? W0 : W1);  // quad_perm [2,3,0,1]
        R += qperm<0xB1>(R);                                        // quad_perm [1,0,3,2]
        if (writer && (!front || hb)) part_lane[front ? jb : ja] = R;
        if (want_max) {
          const float mxa = wave_max63(wa);
          const float mxb = wave_max63(wb);
          if (lane == 63) {
            part[wave][9][ja] = mxa;
            if (hb) part[wave][9][jb] = mxb;
          }
        }
      }
    }
    __syncthreads();
    // each column is combined by one thread, which also zeroes it for the
    // next sub-batch (columns of no pair were never written and stay zero)
    if (tid >= j0 && tid < j0 + kSub && tid < n) {
      const int js = tid - j0;
      float m9[9], o[12];
#pragma unroll
      for (int q = 0; q < 9; ++q) m9[q] = ((part[0][q][js] + part[1][q][js]) + part[2][q][js]) + part[3][q][js];
      const float4 A = mine.a, B = mine.b;  // the conic unscaled
      o[0] = -fmaf(A.z, m9[0], A.w * m9[1]);
      o[1] = -fmaf(A.w, m9[0], B.x * m9[1]);
      o[2] = -0.5f * m9[2];
      o[3] = -m9[3];
      o[4] = -0.5f * m9[4];
      o[5] = B.y > 0.f ? m9[5] / B.y : 0.f;
      o[6] = m9[6];
      o[7] = m9[7];
      o[8] = m9[8];
      o[9] = fmaxf(fmaxf(part[0][9][js], part[1][9][js]), fmaxf(part[2][9][js], part[3][9][js]));
#pragma unroll
      for (int w = 0; w < 4; ++w)
#pragma unroll
        for (int q = 0; q < kGradSlots; ++q) part[w][q][js] = 0.f;
      o[10] = 0.f;
      o[11] = 0.f;
      float4* dst = reinterpret_cast<float4*>(g_pair + (size_t)my_emit * 12);
      dst[0] = make_float4(o[0], o[1], o[2], o[3]);
      dst[1] = make_float4(o[4], o[5], o[6], o[7]);
      dst[2] = make_float4(o[8], o[9], o[10], o[11]);
      alive[my_emit] = 1;
    }
    __syncthreads();
  }
}

hipError_t launch_blend_bwd(const ViewD* views_dev, int n_views, const float* records, uint32_t n_rec,
                            const uint32_t* pair_vals, const uint32_t* sel, uint32_t cap, const uint32_t* ranges,
                            const float4* ckpt, const uint32_t* batch_tile, uint32_t n_batches,
                            const uint32_t* order_cnt, const uint32_t* order_list, const float* dL_drgb,
                            const float* dL_dalpha, const uint32_t* pair_emit, float* g_pair, uint8_t* alive,
                            bool want_max, hipStream_t s) {
  if (n_batches == 0) return hipSuccess;
  hipLaunchKernelGGL(k_blend_bwd, dim3(n_batches), dim3(256), 0, s, views_dev, n_views, records, n_rec, pair_vals,
                     sel, cap, ranges, ckpt, batch_tile, n_batches, order_cnt, order_list, dL_drgb, dL_dalpha,
                     pair_emit, g_pair, alive, want_max ? 1 : 0);
  return hipGetLastError();
}

}  // namespace gsr
