// Integer stages between projection and blending: exclusive scan of the
// per-record tile counts, duplication into (tile << 32 | depth bits, record)
// pairs in emission order, and per-tile [start, end) ranges of the sorted
// pairs.
#include "common.hpp"

namespace gsr {

// ---------------------------------------------------------------- scan
__device__ __forceinline__ uint32_t wave_inclusive_scan(uint32_t x) { return wave_scan_add(x); }

// Block-wide exclusive scan of one value per thread (256 threads = 4 waves).
__device__ __forceinline__ uint32_t block_exclusive_scan(uint32_t x, uint32_t* lds_waves, uint32_t* total) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const uint32_t inc = wave_inclusive_scan(x);
  if (lane == 63) lds_waves[wave] = inc;
  __syncthreads();
  uint32_t wave_off = 0, tot = 0;
#pragma unroll
  for (int w = 0; w < 4; ++w) {
    const uint32_t c = lds_waves[w];
    if (w < wave) wave_off += c;
    tot += c;
  }
  __syncthreads();
  *total = tot;
  return wave_off + inc - x;
}

// Single pass with decoupled look-back: blocks take their tile index from a
// ticket (so a block only waits for blocks already running), publish the
// tile's total, and the first wave looks back over 64 predecessors at a time
// for the nearest inclusive prefix.  Status words: flag in the top 2 bits,
// 62-bit value.  The last tile writes the total K and the capacity check to
// counters.
constexpr uint64_t kScanAgg = 1ull << 62;
constexpr uint64_t kScanIncl = 2ull << 62;
constexpr uint64_t kScanValue = (1ull << 62) - 1;
constexpr uint32_t kScanSpinLimit = 1u << 22;

__global__ void __launch_bounds__(kScanThreads)
k_scan(const uint32_t* __restrict__ in, uint32_t n, uint32_t* __restrict__ out, uint64_t* __restrict__ status,
       uint32_t* __restrict__ ticket, uint32_t* __restrict__ counters, uint32_t pair_capacity) {
  __shared__ uint32_t lds[4];
  __shared__ uint32_t s_bid;
  __shared__ uint64_t s_excl;
  if (threadIdx.x == 0) s_bid = atomicAdd(ticket, 1u);
  __syncthreads();
  const uint32_t bid = s_bid;
  const uint32_t nb = gridDim.x;
  // thread t owns kScanItems consecutive items
  const uint32_t base = bid * (uint32_t)kScanTile + threadIdx.x * kScanItems;
  uint32_t v[kScanItems];
  if (base + kScanItems <= n) {
    const uint4* in4 = reinterpret_cast<const uint4*>(in + base);  // 64-byte aligned run
#pragma unroll
    for (int k = 0; k < kScanItems / 4; ++k) {
      const uint4 q = in4[k];
      v[4 * k] = q.x;
      v[4 * k + 1] = q.y;
      v[4 * k + 2] = q.z;
      v[4 * k + 3] = q.w;
    }
  } else {
#pragma unroll
    for (int k = 0; k < kScanItems; ++k) v[k] = (base + k < n) ? in[base + k] : 0u;
  }
  uint32_t sum = 0;
#pragma unroll
  for (int k = 0; k < kScanItems; ++k) sum += v[k];
  uint32_t total;
  const uint32_t local = block_exclusive_scan(sum, lds, &total);
  if (threadIdx.x < 64) {
    const int lane = threadIdx.x;
    if (lane == 0)
      __hip_atomic_store(&status[bid], (bid == 0 ? kScanIncl : kScanAgg) | total, __ATOMIC_RELAXED,
                         __HIP_MEMORY_SCOPE_AGENT);
    uint64_t excl = 0;
    if (bid > 0) {
      int j = (int)bid - 1;  // window [j - 63, j]
      uint32_t spins = 0;
      for (;;) {
        const int idx = j - lane;
        const uint64_t sv =
            idx >= 0 ? __hip_atomic_load(&status[idx], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) : kScanIncl;
        const uint64_t flag = sv & ~kScanValue;
        const uint64_t ready = __ballot(flag != 0);
        const uint64_t incl = __ballot(flag == kScanIncl);
        // lanes up to the first inclusive one, all ready: sum them
        const int first_incl = incl ? __builtin_ctzll(incl) : 64;
        const uint64_t need = first_incl < 63 ? ((2ull << first_incl) - 1) : ~0ull;
        if ((ready & need) != need) {
          if (++spins > kScanSpinLimit) {
            if (lane == 0) atomicOr(&counters[kCntError], 16u);
            break;
          }
          __builtin_amdgcn_s_sleep(1);
          continue;
        }
        uint64_t x = (lane <= first_incl && idx >= 0) ? (sv & kScanValue) : 0ull;
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) x += __shfl_xor(x, off, 64);
        excl += x;
        if (first_incl < 64) break;
        j -= 64;
      }
      if (lane == 0)
        __hip_atomic_store(&status[bid], kScanIncl | ((excl + total) & kScanValue), __ATOMIC_RELAXED,
                           __HIP_MEMORY_SCOPE_AGENT);
    }
    if (lane == 0) {
      s_excl = excl;
      if (bid == nb - 1) {
        const uint64_t K = excl + total;
        counters[kCntPairs] = K > 0xFFFFFFFFull ? 0xFFFFFFFFu : (uint32_t)K;
        if (K > pair_capacity) atomicOr(&counters[kCntOverflow], 1u);  // sticky until the caller checks
      }
    }
  }
  __syncthreads();
  uint32_t run = (uint32_t)s_excl + local;
  if (base + kScanItems <= n && (reinterpret_cast<uintptr_t>(out) & 15) == 0) {
    uint4* out4 = reinterpret_cast<uint4*>(out + base);
#pragma unroll
    for (int k = 0; k < kScanItems / 4; ++k) {
      uint4 q;
      q.x = run;
      run += v[4 * k];
      q.y = run;
      run += v[4 * k + 1];
      q.z = run;
      run += v[4 * k + 2];
      q.w = run;
      run += v[4 * k + 3];
      out4[k] = q;
    }
  } else {
#pragma unroll
    for (int k = 0; k < kScanItems; ++k) {
      if (base + k < n) out[base + k] = run;
      run += v[k];
    }
  }
  // out[n] = total, written by the thread that owns the end
  if (base <= n && n < base + kScanItems) out[n] = run;
}

uint32_t scan_tiles(uint32_t n) { return div_up(n + 1, (uint32_t)kScanTile); }

// status: scan_tiles(n) zeroed words; ticket: a zeroed counter.
hipError_t launch_scan(const uint32_t* in, uint32_t* out, uint64_t* status, uint32_t* ticket, uint32_t n,
                       uint32_t* counters, uint32_t pair_capacity, hipStream_t s) {
  hipLaunchKernelGGL(k_scan, dim3(scan_tiles(n)), dim3(kScanThreads), 0, s, in, n, out, status, ticket, counters,
                     pair_capacity);
  return hipGetLastError();
}

// ---------------------------------------------------------------- duplicate
// Each wave takes 64 consecutive records, whose pairs form one contiguous
// emission range (offsets is their exclusive scan), and writes that range
// with its lanes striding over the pairs: lane i writes pair base + i,
// finding the record that owns it by a binary search over the wave's
// offsets.  A record's tiles are row-major in its box.  Writes are
// coalesced and a large splat's pairs spread over the wave instead of one
// lane.  Pairs at or beyond min(capacity, counters[pairs]) are dropped (the
// overflow flag or the batch status already records it).  The sort carries
// each pair's emission index as its value; rec_of[e] keeps the record of
// emission index e (rec_map[j] when the records were given in another
// order, the j-th of the arrays being record rec_map[j]).
__global__ void __launch_bounds__(256)
k_duplicate(const uint32_t* __restrict__ n_tiles, const uint32_t* __restrict__ offsets,
            const uint4* __restrict__ tile_box, uint32_t n_rec, const uint32_t* __restrict__ counters,
            uint32_t pair_capacity, uint64_t* __restrict__ keys, uint32_t* __restrict__ vals,
            uint32_t* __restrict__ rec_of, const uint32_t* __restrict__ rec_map) {
  const uint32_t r = blockIdx.x * blockDim.x + threadIdx.x;
  const int lane = threadIdx.x & 63;
  const uint32_t lim = min(pair_capacity, counters[kCntPairs]);
  const bool valid = r < n_rec;
  const uint32_t cnt = valid ? n_tiles[r] : 0u;
  const uint32_t off = valid ? offsets[r] : 0xFFFFFFFFu;  // invalid lanes never own a pair
  uint4 tb = make_uint4(0u, 0u, 0u, 0u);
  if (cnt) tb = tile_box[r];
  uint32_t end = valid ? off + cnt : 0u;
#pragma unroll
  for (int s = 32; s > 0; s >>= 1) end = max(end, (uint32_t)__shfl_xor((int)end, s, 64));
  const uint32_t w0 = (uint32_t)__shfl((int)off, 0, 64);
  const uint32_t w1 = min(end, lim);
  const uint32_t r0 = r - (uint32_t)lane;
  for (uint32_t base = w0; base < w1; base += 64) {
    const uint32_t e = base + (uint32_t)lane;
    // last lane whose offset is <= e (zero-count records share the next offset)
    int lo = 0;
#pragma unroll
    for (int st = 32; st > 0; st >>= 1) {
      const uint32_t o = (uint32_t)__shfl((int)off, lo + st, 64);
      if (o <= e) lo += st;
    }
    const uint32_t o = (uint32_t)__shfl((int)off, lo, 64);
    const uint32_t bx = (uint32_t)__shfl((int)tb.x, lo, 64);
    const uint32_t by = (uint32_t)__shfl((int)tb.y, lo, 64);
    const uint32_t bz = (uint32_t)__shfl((int)tb.z, lo, 64);
    const uint32_t bw = (uint32_t)__shfl((int)tb.w, lo, 64);
    if (e < w1) {
      const uint32_t j = e - o;
      const uint32_t w = max(by & 0xFFFFu, 1u);
      uint32_t dy;
      if (j < (1u << 24)) {  // float quotient, corrected to floor(j / w)
        dy = (uint32_t)((float)j / (float)w);
        if (dy * w > j) --dy;
        if ((dy + 1) * w <= j) ++dy;
      } else {
        dy = j / w;
      }
      const uint32_t tile = bx + dy * bw + (j - dy * w);
      keys[e] = ((uint64_t)tile << 32) | bz;
      vals[e] = e;
      rec_of[e] = rec_map ? rec_map[r0 + (uint32_t)lo] : r0 + (uint32_t)lo;
    }
  }
}

hipError_t launch_duplicate(const uint32_t* n_tiles, const uint32_t* offsets, const uint4* tile_box,
                            uint32_t n_rec, const uint32_t* counters, uint32_t pair_capacity,
                            uint64_t* keys, uint32_t* vals, uint32_t* rec_of, hipStream_t s,
                            const uint32_t* rec_map) {
  if (n_rec == 0) return hipSuccess;
  hipLaunchKernelGGL(k_duplicate, dim3(div_up(n_rec, 256u)), dim3(256), 0, s, n_tiles, offsets, tile_box,
                     n_rec, counters, pair_capacity, keys, vals, rec_of, rec_map);
  return hipGetLastError();
}

// ---------------------------------------------------------------- depth order first
// Calls whose Gaussians are depth-sorted before they are paired (one order
// for the eyes of a stereo frame, Sec. 3.3) emit each view's records in the
// sorted order; a stable grouping of the pairs by tile then leaves every
// tile's pairs in depth order, with no per-tile sort.

__global__ void k_set_u32(uint32_t* p, uint32_t value) {
  if (blockIdx.x == 0 && threadIdx.x == 0) *p = value;
}

hipError_t launch_set_u32(uint32_t* p, uint32_t value, hipStream_t s) {
  hipLaunchKernelGGL(k_set_u32, dim3(1), dim3(64), 0, s, p, value);
  return hipGetLastError();
}

// View whose records include record r (views are in record order).
__device__ __forceinline__ int view_of_record(const ViewD* __restrict__ views, int n_views, uint32_t r) {
  int lo = 0, hi = n_views - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (views[mid].rec_off <= r) lo = mid; else hi = mid - 1;
  }
  return lo;
}

// Position s of the emission sequence (view by view, each view's records in
// its unit's depth order, a follower in its lead's): the record, its tile
// count, and its tile box whose depth word is the sort key (the pair keys'
// low word).  A culled record (no tiles) keeps a zero box.
__global__ void __launch_bounds__(256)
k_seq_build(const ViewD* __restrict__ views, int n_views, uint32_t n_rec, const uint64_t* __restrict__ sk_a,
            const uint64_t* __restrict__ sk_b, const uint32_t* __restrict__ sv_a, const uint32_t* __restrict__ sv_b,
            const uint32_t* __restrict__ sel, uint32_t n_sort, const uint32_t* __restrict__ n_tiles,
            const uint4* __restrict__ tile_box, uint32_t* __restrict__ seq_rec, uint32_t* __restrict__ n_tiles_seq,
            uint4* __restrict__ tile_box_seq, uint32_t* __restrict__ counters) {
  const bool side = *sel != 0;
  const uint64_t* keys = side ? sk_b : sk_a;
  const uint32_t* vals = side ? sv_b : sv_a;
  for (uint32_t s = blockIdx.x * blockDim.x + threadIdx.x; s < n_rec; s += gridDim.x * blockDim.x) {
    const int v = view_of_record(views, n_views, s);
    const ViewD& V = views[v];
    const uint32_t lead = V.sort_mode == kSortFollow ? V.sort_lead : (uint32_t)v;
    const uint32_t v_end = v + 1 < n_views ? views[v + 1].rec_off : n_rec;
    uint32_t rec = s, nt = 0, key = 0;
    bool ok = lead < (uint32_t)n_views;
    if (ok) {
      const ViewD& L = views[lead];
      const uint32_t slot = L.sort_off + (s - V.rec_off);
      ok = slot < n_sort;
      if (ok) {
        const uint32_t lead_rec = vals[slot];
        const uint32_t gi = lead_rec - L.rec_off;  // the Gaussian (wraps when out of range)
        key = (uint32_t)keys[slot];
        ok = lead_rec >= L.rec_off && V.rec_off + gi < v_end;
        if (ok) rec = V.rec_off + gi;
      }
    }
    if (!ok) atomicOr(&counters[kCntError], 64u);  // an inconsistent order: the pairs of s are dropped
    if (ok) nt = n_tiles[rec];
    uint4 tb = make_uint4(0u, 0u, 0u, 0u);
    if (nt) {
      tb = tile_box[rec];
      tb.z = key;
    }
    seq_rec[s] = rec;
    n_tiles_seq[s] = nt;
    tile_box_seq[s] = tb;
  }
}

hipError_t launch_seq_build(const ViewD* views_dev, int n_views, uint32_t n_rec, const uint64_t* sk_a,
                            const uint64_t* sk_b, const uint32_t* sv_a, const uint32_t* sv_b, const uint32_t* sel,
                            uint32_t n_sort, const uint32_t* n_tiles, const uint4* tile_box, uint32_t* seq_rec,
                            uint32_t* n_tiles_seq, uint4* tile_box_seq, uint32_t* counters, hipStream_t s) {
  if (n_rec == 0) return hipSuccess;
  uint32_t grid = div_up(n_rec, 256u);
  if (grid > 16384) grid = 16384;
  hipLaunchKernelGGL(k_seq_build, dim3(grid), dim3(256), 0, s, views_dev, n_views, n_rec, sk_a, sk_b, sv_a, sv_b,
                     sel, n_sort, n_tiles, tile_box, seq_rec, n_tiles_seq, tile_box_seq, counters);
  return hipGetLastError();
}

// After the tile grouping of depth-ordered pairs: each sorted pair's value
// (its emission index) becomes its record id; the emission index goes to
// emit and the key to keys_out (both nullable).
__global__ void __launch_bounds__(256)
k_finalize_pairs(uint32_t* __restrict__ vals_a, uint32_t* __restrict__ vals_b, const uint64_t* __restrict__ keys_a,
                 const uint64_t* __restrict__ keys_b, const uint32_t* __restrict__ sel,
                 const uint32_t* __restrict__ rec_of, uint32_t* __restrict__ counters, uint32_t pair_capacity,
                 uint32_t* __restrict__ emit, uint64_t* __restrict__ keys_out) {
  const uint32_t K = min(counters[kCntPairs], pair_capacity);
  const bool side = *sel != 0;
  uint32_t* vals = side ? vals_b : vals_a;
  const uint64_t* keys = side ? keys_b : keys_a;
  for (uint32_t k = blockIdx.x * blockDim.x + threadIdx.x; k < K; k += gridDim.x * blockDim.x) {
    uint32_t e = vals[k];
    if (e >= K) {
      atomicOr(&counters[kCntError], 64u);
      e = 0;
    }
    vals[k] = rec_of[e];
    if (emit) emit[k] = e;
    if (keys_out) keys_out[k] = keys[k];
  }
}

hipError_t launch_finalize_pairs(uint32_t* vals_a, uint32_t* vals_b, const uint64_t* keys_a, const uint64_t* keys_b,
                                 const uint32_t* sel, const uint32_t* rec_of, const uint32_t* counters,
                                 uint32_t pair_capacity, uint32_t* emit, uint64_t* keys_out, hipStream_t s) {
  if (pair_capacity == 0) return hipSuccess;
  uint32_t grid = div_up(pair_capacity, 256u);
  if (grid > 16384) grid = 16384;
  hipLaunchKernelGGL(k_finalize_pairs, dim3(grid), dim3(256), 0, s, vals_a, vals_b, keys_a, keys_b, sel, rec_of,
                     const_cast<uint32_t*>(counters), pair_capacity, emit, keys_out);
  return hipGetLastError();
}

// ---------------------------------------------------------------- ranges
__global__ void __launch_bounds__(256)
k_ranges(const uint64_t* __restrict__ keys_a, const uint64_t* __restrict__ keys_b,
         const uint32_t* __restrict__ sel, uint32_t* __restrict__ counters, uint32_t pair_capacity,
         uint32_t total_tiles, uint32_t* __restrict__ ranges) {
  const uint32_t K = min(counters[kCntPairs], pair_capacity);
  const uint64_t* keys = (*sel == 0) ? keys_a : keys_b;
  for (uint32_t k = blockIdx.x * blockDim.x + threadIdx.x; k < K; k += gridDim.x * blockDim.x) {
    const uint32_t t = (uint32_t)(keys[k] >> 32);
    if (t >= total_tiles) {
      atomicOr(&counters[kCntError], 4u);
      continue;
    }
    if (k == 0 || (uint32_t)(keys[k - 1] >> 32) != t) ranges[2 * t] = k;
    if (k + 1 == K || (uint32_t)(keys[k + 1] >> 32) != t) ranges[2 * t + 1] = k + 1;
  }
}

hipError_t launch_ranges(const uint64_t* keys_a, const uint64_t* keys_b, const uint32_t* sel,
                         uint32_t* counters, uint32_t pair_capacity, uint32_t total_tiles, uint32_t* ranges,
                         hipStream_t s) {
  if (pair_capacity == 0) return hipSuccess;
  uint32_t grid = div_up(pair_capacity, 256u);
  if (grid > 8192) grid = 8192;
  hipLaunchKernelGGL(k_ranges, dim3(grid), dim3(256), 0, s, keys_a, keys_b, sel, counters, pair_capacity,
                     total_tiles, ranges);
  return hipGetLastError();
}

// ---------------------------------------------------------------- tile order
// Tiles grouped by pair count into kTileClasses classes (largest first,
// empty tiles last), so that the forward blend starts its longest tiles
// first.  One block per 1024
// tiles: class counts per block (ballots), one addition per class and
// block reserves the block's slots in the class list.  The order within a
// class depends on the order the blocks run, which changes no result.

__global__ void __launch_bounds__(1024)
k_tile_order(const uint32_t* __restrict__ ranges, uint32_t n_tiles, uint32_t* __restrict__ class_count,
             uint32_t* __restrict__ class_list) {
  __shared__ uint32_t wc[16][kTileClasses];
  __shared__ uint32_t base[kTileClasses];
  const uint32_t t = blockIdx.x * 1024u + threadIdx.x;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  uint32_t n = 0;
  if (t < n_tiles) {
    const uint32_t s0 = ranges[2 * t], s1 = ranges[2 * t + 1];
    n = s1 > s0 ? s1 - s0 : 0u;
  }
  const uint32_t c = t < n_tiles ? tile_class(n) : kTileClasses;
  const uint64_t below = lane ? (~0ull >> (64 - lane)) : 0ull;
  uint32_t rank = 0;
#pragma unroll
  for (uint32_t k = 0; k < kTileClasses; ++k) {
    const uint64_t m = __ballot(c == k);
    if (c == k) rank = (uint32_t)__popcll(m & below);
    if (lane == 0) wc[wave][k] = (uint32_t)__popcll(m);
  }
  __syncthreads();
  if (threadIdx.x < kTileClasses) {
    uint32_t tot = 0;
    for (int w = 0; w < 16; ++w) tot += wc[w][threadIdx.x];
    base[threadIdx.x] = tot ? atomicAdd(&class_count[threadIdx.x], tot) : 0u;
  }
  __syncthreads();
  if (c < kTileClasses) {
    uint32_t pos = base[c] + rank;
    for (int w = 0; w < wave; ++w) pos += wc[w][c];
    if (pos < n_tiles) class_list[(size_t)c * n_tiles + pos] = t;
  }
}

hipError_t launch_tile_order(const uint32_t* ranges, uint32_t n_tiles, uint32_t* class_count,
                             uint32_t* class_list, hipStream_t s) {
  if (n_tiles == 0) return hipSuccess;
  hipLaunchKernelGGL(k_tile_order, dim3(div_up(n_tiles, 1024u)), dim3(1024), 0, s, ranges, n_tiles, class_count,
                     class_list);
  return hipGetLastError();
}

// ---------------------------------------------------------------- batch status
// Requests own contiguous record ranges [req_rec[q], req_rec[q+1]), so their
// pairs are contiguous in emission order.  A request whose pairs end beyond
// the capacity is marked GSR_ENOSPACE (-2) (a suffix of the requests) and the
// pair count is cut to the end of the last request that fits, so that only
// whole requests are duplicated, sorted and blended.
__global__ void k_batch_status(const uint32_t* __restrict__ req_rec, int n_req,
                               const uint32_t* __restrict__ offsets, uint32_t pair_capacity,
                               uint32_t* __restrict__ counters, int32_t* __restrict__ req_status) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  uint32_t k_fit = 0;
  for (int q = 0; q < n_req; ++q) {
    const uint32_t end = offsets[req_rec[q + 1]];
    const bool fits = end <= pair_capacity;
    req_status[q] = fits ? 0 : -2;
    if (fits) k_fit = end;
  }
  counters[kCntPairs] = k_fit;
  counters[kCntOverflow] = 0;
}

// After a batch: a device-side error anywhere in the call (the sort's or the
// scan's bounded waits, inconsistent offsets) marks every request
// GSR_EDEVICE (-4), so no image of a faulty sort is reported as good.
__global__ void k_batch_error(const uint32_t* __restrict__ counters, int n_req, int32_t* __restrict__ req_status) {
  if (counters[kCntError] == 0u) return;
  for (int q = blockIdx.x * blockDim.x + threadIdx.x; q < n_req; q += gridDim.x * blockDim.x) req_status[q] = -4;
}

hipError_t launch_batch_error(const uint32_t* counters, int n_req, int32_t* req_status, hipStream_t s) {
  if (n_req <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_batch_error, dim3(1), dim3(256), 0, s, counters, n_req, req_status);
  return hipGetLastError();
}

hipError_t launch_batch_status(const uint32_t* req_rec, int n_req, const uint32_t* offsets,
                               uint32_t pair_capacity, uint32_t* counters, int32_t* req_status,
                               hipStream_t s) {
  hipLaunchKernelGGL(k_batch_status, dim3(1), dim3(64), 0, s, req_rec, n_req, offsets, pair_capacity,
                     counters, req_status);
  return hipGetLastError();
}

}  // namespace gsr
