// Pair sort: (tile << 32 | depth bits) keys, stable, in two stages.
//
// 1. The tile digits: stable LSD radix passes over the whole pair array,
//    8-bit digits, in the single-pass-per-digit style of OneSweep (Adinets
//    and Merrill, the sort the paper's renderer derives from, Sec. 3.3): one
//    read of the keys builds the digit histograms of every pass, then each
//    pass ranks a tile of keys per block and finds the tile's global digit
//    offsets by decoupled look-back over the preceding tiles.
// 2. The depth digits, per screen tile: one block per screen tile sorts its
//    segment by the 32 depth bits with block-local LSD passes (in LDS when
//    the segment fits, else chunk by chunk through global memory), stable,
//    so that equal depths keep emission order -- the same order a stable
//    sort of the full 64-bit keys gives.  Its last pass writes the record id
//    and the emission index of every sorted pair.
//
// Wave64 details: digits are ranked with 8 ballots per round (peer masks),
// per-wave digit counters live in LDS, a chunk is re-ordered by digit in
// LDS before it is written out, so consecutive lanes write consecutive
// addresses of a digit run.  Look-back tiles are assigned in the order
// blocks start (an atomic ticket), so a block only ever waits for blocks
// that are already running; the wait is additionally bounded and reports an
// error instead of spinning forever.
#include "common.hpp"

namespace gsr {

constexpr uint32_t kFlagAgg = 1u << 30;
constexpr uint32_t kFlagIncl = 2u << 30;
constexpr uint32_t kValueMask = (1u << 30) - 1;
constexpr uint32_t kSpinLimit = 1u << 22;

__device__ __forceinline__ uint64_t lanemask_lt() {
  const int lane = threadIdx.x & 63;
  return (lane == 0) ? 0ull : (~0ull >> (64 - lane));
}

// Lanes of the wave whose valid 8-bit digit equals this lane's.
__device__ __forceinline__ uint64_t match_digit(uint32_t d, bool valid) {
  uint64_t peers = __ballot(valid);
#pragma unroll
  for (int b = 0; b < 8; ++b) {
    const bool bit = (d >> b) & 1u;
    const uint64_t bal = __ballot(bit);
    peers &= bit ? bal : ~bal;
  }
  return peers;
}

__device__ __forceinline__ uint32_t wave_incl_scan(uint32_t x) {
  const int lane = threadIdx.x & 63;
#pragma unroll
  for (int off = 1; off < 64; off <<= 1) {
    const uint32_t y = __shfl_up(x, off, 64);
    if (lane >= off) x += y;
  }
  return x;
}

// ---------------------------------------------------------------- histogram
// Digit histograms of every pass (per-wave LDS counters, merged per block
// and added to the global counts); also clears the look-back words of the
// tiles the passes will use.
__global__ void __launch_bounds__(256)
k_sort_hist(const uint64_t* __restrict__ keys, const uint32_t* __restrict__ counters, uint32_t cap,
            int pass_begin, int pass_end, uint32_t* __restrict__ hist, uint32_t* __restrict__ status,
            uint32_t nb_max) {
  __shared__ uint32_t lh[4][kMaxSortPasses * 256];
  const uint32_t K = min(counters[kCntPairs], cap);
  const int wave = threadIdx.x >> 6;
  for (int i = threadIdx.x; i < 4 * kMaxSortPasses * 256; i += 256) (&lh[0][0])[i] = 0;
  __syncthreads();
  const uint32_t stride = gridDim.x * blockDim.x;
  for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < K; i += stride) {
    const uint64_t k = keys[i];
    for (int p = pass_begin; p < pass_end; ++p)
      atomicAdd(&lh[wave][p * 256 + ((uint32_t)(k >> (8 * p)) & 255u)], 1u);
  }
  __syncthreads();
  for (int i = pass_begin * 256 + threadIdx.x; i < pass_end * 256; i += 256) {
    const uint32_t c = lh[0][i] + lh[1][i] + lh[2][i] + lh[3][i];
    if (c) atomicAdd(&hist[i], c);
  }
  // clear the look-back words of the active tiles of every pass
  const uint32_t nb = div_up(K, (uint32_t)kSortTile);
  const size_t per_pass = (size_t)nb * 256;
  const size_t total = per_pass * (size_t)(pass_end - pass_begin);
  for (size_t w = (size_t)blockIdx.x * blockDim.x + threadIdx.x; w < total; w += stride) {
    const size_t p = pass_begin + w / per_pass, rem = w % per_pass;
    status[p * (size_t)nb_max * 256 + rem] = 0u;
  }
}

// ---------------------------------------------------------------- plan
// Exclusive digit offsets per pass, passes whose keys all share one digit
// are skipped, and the ping-pong buffer of every remaining pass.
__global__ void __launch_bounds__(256)
k_sort_plan(const uint32_t* __restrict__ hist, const uint32_t* __restrict__ counters, uint32_t cap,
            int pass_begin, int pass_end, uint32_t* __restrict__ digit_off, SortPlan* __restrict__ plan,
            uint32_t* __restrict__ sel_out) {
  __shared__ uint32_t lw[4];
  __shared__ uint32_t trivial[kMaxSortPasses];
  const uint32_t K = min(counters[kCntPairs], cap);
  const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
  if (t < kMaxSortPasses) trivial[t] = 0;
  __syncthreads();
  for (int p = pass_begin; p < pass_end; ++p) {
    const uint32_t c = hist[p * 256 + t];
    const uint32_t inc = wave_incl_scan(c);
    if (lane == 63) lw[wave] = inc;
    __syncthreads();
    uint32_t off = 0;
    for (int w = 0; w < wave; ++w) off += lw[w];
    digit_off[p * 256 + t] = off + inc - c;
    if (c == K) trivial[p] = 1;  // every key has digit t (also K == 0 via c == 0 == K)
    __syncthreads();
  }
  if (t == 0) {
    uint32_t cur = 0;
    for (int p = 0; p < kMaxSortPasses; ++p) {
      const bool skip = p < pass_begin || p >= pass_end || trivial[p] || K == 0;
      plan->skip[p] = skip ? 1u : 0u;
      plan->src[p] = cur;
      if (!skip) cur ^= 1u;
    }
    plan->sel = cur;
    plan->n_passes = (uint32_t)(pass_end - pass_begin);
    *sel_out = cur;
  }
}

// ---------------------------------------------------------------- one pass
__global__ void __launch_bounds__(kSortThreads)
k_sort_pass(uint64_t* __restrict__ keys0, uint64_t* __restrict__ keys1, uint32_t* __restrict__ vals0,
            uint32_t* __restrict__ vals1, const uint32_t* __restrict__ counters, uint32_t cap,
            const SortPlan* __restrict__ plan, const uint32_t* __restrict__ digit_off,
            uint32_t* __restrict__ status, uint32_t nb_max, uint32_t* __restrict__ pass_ctr,
            uint32_t* __restrict__ err, int pass) {
  __shared__ uint32_t s_bid;
  __shared__ uint32_t wave_cnt[kSortWaves][256];
  __shared__ uint32_t s_start[256];
  __shared__ uint32_t s_global[256];
  __shared__ uint32_t s_w[4];
  __shared__ uint64_t s_keys[kSortTile];
  __shared__ uint32_t s_vals[kSortTile];

  if (plan->skip[pass]) return;
  const uint32_t K = min(counters[kCntPairs], cap);
  const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
  if (t == 0) s_bid = atomicAdd(&pass_ctr[pass], 1u);
  for (int i = t; i < kSortWaves * 256; i += kSortThreads) (&wave_cnt[0][0])[i] = 0;
  __syncthreads();
  const uint32_t bid = s_bid;
  const uint32_t base = bid * (uint32_t)kSortTile;
  if (base >= K) return;
  const uint32_t src = plan->src[pass];
  const uint64_t* kin = src ? keys1 : keys0;
  const uint32_t* vin = src ? vals1 : vals0;
  uint64_t* kout = src ? keys0 : keys1;
  uint32_t* vout = src ? vals0 : vals1;
  const int shift = 8 * pass;

  uint64_t key[kSortItems];
  uint32_t val[kSortItems];
  uint32_t rank[kSortItems];
  const uint32_t wbase = base + (uint32_t)wave * (kSortItems * 64);
#pragma unroll
  for (int r = 0; r < kSortItems; ++r) {
    const uint32_t idx = wbase + r * 64 + lane;
    const bool valid = idx < K;
    key[r] = valid ? kin[idx] : 0ull;
    val[r] = valid ? vin[idx] : 0u;
  }
  // rank within the wave, in input order (round-major, then lane)
#pragma unroll
  for (int r = 0; r < kSortItems; ++r) {
    const bool valid = (wbase + r * 64 + lane) < K;
    const uint32_t d = (uint32_t)(key[r] >> shift) & 255u;
    const uint64_t peers = match_digit(d, valid);
    const uint64_t before = peers & lanemask_lt();
    uint32_t pre = 0;
    if (valid) pre = wave_cnt[wave][d];
    __builtin_amdgcn_wave_barrier();
    if (valid && before == 0) wave_cnt[wave][d] = pre + (uint32_t)__popcll(peers);
    __builtin_amdgcn_wave_barrier();
    rank[r] = pre + (uint32_t)__popcll(before);
  }
  __syncthreads();
  // thread t < 256 owns digit t: per-wave exclusive offsets and the block count
  uint32_t cw[kSortWaves];
  uint32_t cnt = 0, inc = 0;
  uint32_t* st = status + ((size_t)pass * nb_max) * 256;
  if (t < 256) {
#pragma unroll
    for (int w = 0; w < kSortWaves; ++w) {
      cw[w] = wave_cnt[w][t];
      cnt += cw[w];
    }
    inc = wave_incl_scan(cnt);
    if (lane == 63) s_w[wave] = inc;
    // publish this tile's counts before looking back
    if (bid == 0) {
      __hip_atomic_store(&st[t], kFlagIncl | cnt, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    } else {
      __hip_atomic_store(&st[(size_t)bid * 256 + t], kFlagAgg | cnt, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
  }
  __syncthreads();
  uint32_t excl = 0;
  if (t < 256) {
    uint32_t off = 0;
    for (int w = 0; w < wave; ++w) off += s_w[w];
    s_start[t] = off + inc - cnt;
    uint32_t run = 0;
#pragma unroll
    for (int w = 0; w < kSortWaves; ++w) {
      wave_cnt[w][t] = run;
      run += cw[w];
    }
    if (bid > 0) {
      int j = (int)bid - 1;
      uint32_t spins = 0;
      while (j >= 0) {
        const uint32_t sv = __hip_atomic_load(&st[(size_t)j * 256 + t], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        const uint32_t f = sv & ~kValueMask;
        if (f == 0) {
          if (++spins > kSpinLimit) {
            atomicOr(err, 1u);
            break;
          }
          __builtin_amdgcn_s_sleep(1);
          continue;
        }
        excl += sv & kValueMask;
        if (f == kFlagIncl) break;
        --j;
      }
      __hip_atomic_store(&st[(size_t)bid * 256 + t], kFlagIncl | (excl + cnt), __ATOMIC_RELAXED,
                         __HIP_MEMORY_SCOPE_AGENT);
    }
    s_global[t] = digit_off[pass * 256 + t] + excl;
  }
  __syncthreads();
  // order the tile by digit in LDS (stable), then write digit runs out
#pragma unroll
  for (int r = 0; r < kSortItems; ++r) {
    const bool valid = (wbase + r * 64 + lane) < K;
    if (valid) {
      const uint32_t d = (uint32_t)(key[r] >> shift) & 255u;
      const uint32_t pos = s_start[d] + wave_cnt[wave][d] + rank[r];
      s_keys[pos] = key[r];
      s_vals[pos] = val[r];
    }
  }
  __syncthreads();
  const uint32_t n_items = min(K - base, (uint32_t)kSortTile);
  for (uint32_t i = t; i < n_items; i += kSortThreads) {
    const uint64_t k = s_keys[i];
    const uint32_t d = (uint32_t)(k >> shift) & 255u;
    const uint32_t dst = s_global[d] + (i - s_start[d]);
    if (dst < K) {
      kout[dst] = k;
      vout[dst] = s_vals[i];
    } else {
      atomicOr(err, 2u);  // inconsistent offsets: never write out of range
    }
  }
}

size_t sort_status_words(uint32_t pair_capacity) {
  return (size_t)kMaxSortPasses * div_up(pair_capacity > 0 ? pair_capacity : 1u, (uint32_t)kSortTile) * 256;
}

// Radix passes [pass_begin, pass_end) (bits 8 * pass_begin up) of the
// pair keys.  hist: [kMaxSortPasses][256] counts followed by
// [kMaxSortPasses][256] offsets; pass_ctr: [kMaxSortPasses]; both zero on
// entry.
hipError_t launch_sort(uint64_t* keys_a, uint64_t* keys_b, uint32_t* vals_a, uint32_t* vals_b,
                       const uint32_t* counters, uint32_t pair_capacity, int pass_begin, int pass_end,
                       uint32_t* hist, uint32_t* status, uint32_t* pass_ctr, SortPlan* plan, uint32_t* sel_out,
                       uint32_t* error_flag, hipStream_t s) {
  if (pass_begin < 0 || pass_end > kMaxSortPasses || pass_begin > pass_end) return hipErrorInvalidValue;
  const uint32_t nb_max = div_up(pair_capacity > 0 ? pair_capacity : 1u, (uint32_t)kSortTile);
  uint32_t* digit_off = hist + kMaxSortPasses * 256;
  uint32_t hist_blocks = div_up(pair_capacity > 0 ? pair_capacity : 1u, 256u * 16u);
  if (hist_blocks > 128) hist_blocks = 128;  // fewer blocks: fewer global count additions
  hipLaunchKernelGGL(k_sort_hist, dim3(hist_blocks), dim3(256), 0, s, keys_a, counters, pair_capacity, pass_begin,
                     pass_end, hist, status, nb_max);
  hipLaunchKernelGGL(k_sort_plan, dim3(1), dim3(256), 0, s, hist, counters, pair_capacity, pass_begin, pass_end,
                     digit_off, plan, sel_out);
  for (int p = pass_begin; p < pass_end; ++p)
    hipLaunchKernelGGL(k_sort_pass, dim3(nb_max), dim3(kSortThreads), 0, s, keys_a, keys_b, vals_a, vals_b,
                       counters, pair_capacity, plan, digit_off, status, nb_max, pass_ctr, error_flag, p);
  return hipGetLastError();
}

// ---------------------------------------------------------------- per-tile depth sort
constexpr int kSegThreads = 1024;
constexpr int kSegWaves = kSegThreads / 64;
constexpr int kSegItems = 8;                       // per thread and chunk
constexpr int kSegCap = kSegThreads * kSegItems;   // segments up to this size stay in LDS

struct SegLds {
  uint32_t key[kSegCap];              // depth bits of the chunk, in digit order after a pass
  uint32_t val[kSegCap];              // emission indices
  uint16_t wave_cnt[kSegWaves][256];  // per-wave digit counts, then per-wave digit offsets
  uint32_t start[256];                // first chunk position of every digit
  uint32_t run[256];                  // segment position of the next key of every digit
  uint32_t base[4][256];              // segment histograms, then exclusive offsets (large segments)
  uint32_t wsum[kSegWaves];
  uint32_t red[2][kSegWaves];
};

// Chunk positions of this thread's items when the chunk is stably ordered by
// the digit at `shift`.  Items: thread (wave, lane) holds chunk entries
// wave * I * 64 + r * 64 + lane, r < I, valid below n.  Leaves the chunk's
// digit starts in L.start and, for thread t < 256, returns the count of
// digit t.
__device__ __forceinline__ uint32_t seg_rank(SegLds& L, const uint32_t (&key)[kSegItems], int I, uint32_t n,
                                             int shift, uint32_t (&pos)[kSegItems]) {
  const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
  for (int i = t; i < kSegWaves * 256; i += kSegThreads) (&L.wave_cnt[0][0])[i] = 0;
  __syncthreads();
  uint32_t rank[kSegItems];
#pragma unroll
  for (int r = 0; r < kSegItems; ++r) {
    if (r >= I) break;
    const uint32_t idx = (uint32_t)(wave * I + r) * 64u + lane;
    const bool valid = idx < n;
    const uint32_t d = (key[r] >> shift) & 255u;
    const uint64_t peers = match_digit(d, valid);
    const uint64_t before = peers & lanemask_lt();
    uint32_t pre = 0;
    if (valid) pre = L.wave_cnt[wave][d];
    __builtin_amdgcn_wave_barrier();
    if (valid && before == 0) L.wave_cnt[wave][d] = (uint16_t)(pre + (uint32_t)__popcll(peers));
    __builtin_amdgcn_wave_barrier();
    rank[r] = pre + (uint32_t)__popcll(before);
  }
  __syncthreads();
  uint32_t cnt = 0, inc = 0;
  if (t < 256) {
    uint32_t cw[kSegWaves];
#pragma unroll
    for (int w = 0; w < kSegWaves; ++w) {
      cw[w] = L.wave_cnt[w][t];
      cnt += cw[w];
    }
    inc = wave_incl_scan(cnt);
    if (lane == 63) L.wsum[wave] = inc;
    uint32_t run = 0;
#pragma unroll
    for (int w = 0; w < kSegWaves; ++w) {
      L.wave_cnt[w][t] = (uint16_t)run;
      run += cw[w];
    }
  }
  __syncthreads();
  if (t < 256) {
    uint32_t off = 0;
    for (int w = 0; w < wave; ++w) off += L.wsum[w];
    L.start[t] = off + inc - cnt;
  }
  __syncthreads();
#pragma unroll
  for (int r = 0; r < kSegItems; ++r) {
    if (r >= I) break;
    const uint32_t idx = (uint32_t)(wave * I + r) * 64u + lane;
    const uint32_t d = (key[r] >> shift) & 255u;
    pos[r] = idx < n ? L.start[d] + L.wave_cnt[wave][d] + rank[r] : 0u;
  }
  return cnt;
}

// Bitwise OR and AND of every thread's value over the block.
__device__ __forceinline__ uint32_t seg_varying_bits(SegLds& L, uint32_t lor, uint32_t land) {
  const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    lor |= __shfl_xor(lor, off, 64);
    land &= __shfl_xor(land, off, 64);
  }
  if (lane == 0) {
    L.red[0][wave] = lor;
    L.red[1][wave] = land;
  }
  __syncthreads();
  uint32_t o = 0, a = ~0u;
#pragma unroll
  for (int w = 0; w < kSegWaves; ++w) {
    o |= L.red[0][w];
    a &= L.red[1][w];
  }
  return o ^ a;
}

// One block per screen tile; the tile's pairs [ranges[2t], ranges[2t+1])
// are already grouped by tile in emission order.  Sorts them by depth bits
// (stable) and writes vals[k] = record id, emit[k] = emission index (if
// emit), keys_out[k] = full key (if keys_out).  The keys buffer of the
// other ping-pong side is scratch for segments larger than kSegCap.
__global__ void __launch_bounds__(kSegThreads)
k_sort_segments(uint64_t* __restrict__ keys_a, uint64_t* __restrict__ keys_b, uint32_t* __restrict__ vals_a,
                uint32_t* __restrict__ vals_b, const uint32_t* __restrict__ sel, const uint32_t* __restrict__ ranges,
                const uint32_t* __restrict__ rec_of, const uint32_t* __restrict__ counters, uint32_t cap,
                uint32_t* __restrict__ emit, uint64_t* __restrict__ keys_out, uint32_t* __restrict__ err) {
  __shared__ SegLds L;
  const uint32_t tile = blockIdx.x;
  const uint32_t s0 = ranges[2 * tile], s1 = ranges[2 * tile + 1];
  if (s1 <= s0) return;
  const uint32_t K = min(counters[kCntPairs], cap);
  if (s1 > K) {
    if (threadIdx.x == 0) atomicOr(err, 32u);
    return;
  }
  const uint32_t n = s1 - s0;
  const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
  const bool side = *sel != 0;
  uint64_t* kin = side ? keys_b : keys_a;
  uint64_t* kother = side ? keys_a : keys_b;
  uint32_t* vals = side ? vals_b : vals_a;
  // final write of sorted position o (segment-relative)
  auto put = [&](uint32_t o, uint32_t depth, uint32_t e) {
    if (o >= n || e >= K) {
      atomicOr(err, 32u);
      return;
    }
    vals[s0 + o] = rec_of[e];
    if (emit) emit[s0 + o] = e;
    if (keys_out) keys_out[s0 + o] = ((uint64_t)tile << 32) | depth;
  };

  uint32_t key[kSegItems], val[kSegItems], pos[kSegItems];
  if (n <= (uint32_t)kSegCap) {
    const int I = (int)div_up(n, (uint32_t)kSegThreads);
    uint32_t lor = 0, land = ~0u;
#pragma unroll
    for (int r = 0; r < kSegItems; ++r) {
      key[r] = 0;
      val[r] = 0;
      if (r >= I) break;
      const uint32_t idx = (uint32_t)(wave * I + r) * 64u + lane;
      if (idx < n) {
        key[r] = (uint32_t)kin[s0 + idx];
        val[r] = vals[s0 + idx];
        lor |= key[r];
        land &= key[r];
      }
    }
    const uint32_t vary = seg_varying_bits(L, lor, land);
    bool moved = false;
    for (int p = 0; p < 4; ++p) {
      if (((vary >> (8 * p)) & 255u) == 0) continue;
      if (moved) {
#pragma unroll
        for (int r = 0; r < kSegItems; ++r) {
          if (r >= I) break;
          const uint32_t idx = (uint32_t)(wave * I + r) * 64u + lane;
          if (idx < n) {
            key[r] = L.key[idx];
            val[r] = L.val[idx];
          }
        }
      }
      seg_rank(L, key, I, n, 8 * p, pos);
#pragma unroll
      for (int r = 0; r < kSegItems; ++r) {
        if (r >= I) break;
        const uint32_t idx = (uint32_t)(wave * I + r) * 64u + lane;
        if (idx < n) {
          L.key[pos[r]] = key[r];
          L.val[pos[r]] = val[r];
        }
      }
      __syncthreads();
      moved = true;
    }
    if (!moved) {
#pragma unroll
      for (int r = 0; r < kSegItems; ++r) {
        if (r >= I) break;
        const uint32_t idx = (uint32_t)(wave * I + r) * 64u + lane;
        if (idx < n) put(idx, key[r], val[r]);
      }
    } else {
      for (uint32_t i = t; i < n; i += kSegThreads) put(i, L.key[i], L.val[i]);
    }
    return;
  }

  // Large segment: pack (depth, emission index) into the scratch side while
  // taking the segment's digit histograms, then run the passes chunk by
  // chunk, ping-ponging between the two key buffers; the last pass writes
  // the results.
  for (int i = t; i < 4 * 256; i += kSegThreads) (&L.base[0][0])[i] = 0;
  __syncthreads();
  uint32_t lor = 0, land = ~0u;
  for (uint32_t b0 = 0; b0 < n; b0 += kSegThreads) {
    const uint32_t i = b0 + t;
    const bool valid = i < n;
    uint32_t k = 0;
    if (valid) {
      k = (uint32_t)kin[s0 + i];
      kother[s0 + i] = ((uint64_t)k << 32) | vals[s0 + i];
      lor |= k;
      land &= k;
    }
#pragma unroll
    for (int p = 0; p < 4; ++p) {
      const uint32_t d = (k >> (8 * p)) & 255u;
      const uint64_t peers = match_digit(d, valid);
      if (valid && (peers & lanemask_lt()) == 0) atomicAdd(&L.base[p][d], (uint32_t)__popcll(peers));
    }
  }
  const uint32_t vary = seg_varying_bits(L, lor, land);  // (its barrier also publishes L.base)
  int last_pass = -1;
  for (int p = 0; p < 4; ++p)
    if ((vary >> (8 * p)) & 255u) last_pass = p;
  // exclusive digit offsets per pass
  for (int p = 0; p < 4; ++p) {
    uint32_t c = 0, inc = 0;
    if (t < 256) {
      c = L.base[p][t];
      inc = wave_incl_scan(c);
      if (lane == 63) L.wsum[wave] = inc;
    }
    __syncthreads();
    if (t < 256) {
      uint32_t off = 0;
      for (int w = 0; w < wave; ++w) off += L.wsum[w];
      L.base[p][t] = off + inc - c;
    }
    __syncthreads();
  }
  if (last_pass < 0) {
    for (uint32_t i = t; i < n; i += kSegThreads) {
      const uint64_t v = kother[s0 + i];
      put(i, (uint32_t)(v >> 32), (uint32_t)v);
    }
    return;
  }
  uint64_t* src = kother;
  uint64_t* dst = kin;
  for (int p = 0; p <= last_pass; ++p) {
    if (((vary >> (8 * p)) & 255u) == 0) continue;
    const int shift = 8 * p;
    if (t < 256) L.run[t] = L.base[p][t];
    for (uint32_t cb = 0; cb < n; cb += kSegCap) {
      const uint32_t nc = min((uint32_t)kSegCap, n - cb);
      const int I = (int)div_up(nc, (uint32_t)kSegThreads);
#pragma unroll
      for (int r = 0; r < kSegItems; ++r) {
        key[r] = 0;
        val[r] = 0;
        if (r >= I) break;
        const uint32_t idx = (uint32_t)(wave * I + r) * 64u + lane;
        if (idx < nc) {
          const uint64_t v = src[s0 + cb + idx];
          key[r] = (uint32_t)(v >> 32);
          val[r] = (uint32_t)v;
        }
      }
      const uint32_t cnt = seg_rank(L, key, I, nc, shift, pos);
#pragma unroll
      for (int r = 0; r < kSegItems; ++r) {
        if (r >= I) break;
        const uint32_t idx = (uint32_t)(wave * I + r) * 64u + lane;
        if (idx < nc) {
          L.key[pos[r]] = key[r];
          L.val[pos[r]] = val[r];
        }
      }
      __syncthreads();
      for (uint32_t i = t; i < nc; i += kSegThreads) {
        const uint32_t k = L.key[i];
        const uint32_t d = (k >> shift) & 255u;
        const uint32_t o = L.run[d] + (i - L.start[d]);
        if (p == last_pass) {
          put(o, k, L.val[i]);
        } else if (o < n) {
          dst[s0 + o] = ((uint64_t)k << 32) | L.val[i];
        } else {
          atomicOr(err, 32u);
        }
      }
      __syncthreads();
      if (t < 256) L.run[t] += cnt;
      __syncthreads();
    }
    uint64_t* tmp = src;
    src = dst;
    dst = tmp;
  }
}

// After the tile passes: per-tile depth sort, record ids and emission
// indices.  keys_out (nullable) receives the sorted 64-bit keys.
hipError_t launch_sort_segments(uint64_t* keys_a, uint64_t* keys_b, uint32_t* vals_a, uint32_t* vals_b,
                                const uint32_t* sel, const uint32_t* ranges, uint32_t total_tiles,
                                const uint32_t* rec_of, const uint32_t* counters, uint32_t pair_capacity,
                                uint32_t* emit, uint64_t* keys_out, uint32_t* error_flag, hipStream_t s) {
  if (total_tiles == 0 || pair_capacity == 0) return hipSuccess;
  hipLaunchKernelGGL(k_sort_segments, dim3(total_tiles), dim3(kSegThreads), 0, s, keys_a, keys_b, vals_a, vals_b,
                     sel, ranges, rec_of, counters, pair_capacity, emit, keys_out, error_flag);
  return hipGetLastError();
}

}  // namespace gsr
