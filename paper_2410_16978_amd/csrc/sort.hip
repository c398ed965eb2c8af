// Pair sort: (tile << 32 | depth bits) keys, stable, in two stages.
//
// 1. The tile digits: stable LSD radix passes over the whole pair array,
//    8-bit digits, in the single-pass-per-digit style of OneSweep (Adinets
//    and Merrill, the sort the paper's renderer derives from, Sec. 3.3): one
//    read of the keys counts the digits of every pass, then each pass ranks
//    a tile of keys per block and finds the tile's global digit offsets by
//    decoupled look-back over the preceding tiles.
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

#include <algorithm>

namespace gsr {

constexpr uint32_t kFlagAgg = 1u << 30;
constexpr uint32_t kFlagIncl = 2u << 30;
constexpr uint32_t kValueMask = (1u << 30) - 1;
constexpr uint32_t kSpinLimit = 1u << 22;

__device__ __forceinline__ uint64_t lanemask_lt() {
  const int lane = threadIdx.x & 63;
  return (lane == 0) ? 0ull : (~0ull >> (64 - lane));
}

// Lanes of the wave whose valid 8-bit digit equals this lane's.  Per bit b:
// s = all ones if this lane's bit is set, and the lanes that agree with it
// are ~(ballot ^ s); each half of the 64-lane mask is narrowed with one
// three-input bit operation (truth table 0x82: acc & ~(bal ^ s)).
__device__ __forceinline__ uint64_t match_digit(uint32_t d, bool valid) {
  const uint64_t vb = __ballot(valid);
  uint32_t lo = (uint32_t)vb, hi = (uint32_t)(vb >> 32);
#pragma unroll
  for (int b = 0; b < 8; ++b) {
    const uint32_t s = (uint32_t)__builtin_amdgcn_sbfe((int)d, (unsigned)b, 1u);
    const uint64_t bal = __ballot(s != 0u);
    lo = __builtin_amdgcn_bitop3_b32((uint32_t)bal, s, lo, 0x82);
    hi = __builtin_amdgcn_bitop3_b32((uint32_t)(bal >> 32), s, hi, 0x82);
  }
  return ((uint64_t)hi << 32) | lo;
}

// Digit of DBITS bits: the lanes holding the same digit (and valid).
template <int DBITS>
__device__ __forceinline__ uint64_t match_digit_bits(uint32_t d, bool valid) {
  const uint64_t vb = __ballot(valid);
  uint32_t lo = (uint32_t)vb, hi = (uint32_t)(vb >> 32);
#pragma unroll
  for (int b = 0; b < DBITS; ++b) {
    const uint32_t s = (uint32_t)__builtin_amdgcn_sbfe((int)d, (unsigned)b, 1u);
    const uint64_t bal = __ballot(s != 0u);
    lo = __builtin_amdgcn_bitop3_b32((uint32_t)bal, s, lo, 0x82);
    hi = __builtin_amdgcn_bitop3_b32((uint32_t)(bal >> 32), s, hi, 0x82);
  }
  return ((uint64_t)hi << 32) | lo;
}

__device__ __forceinline__ uint32_t wave_incl_scan(uint32_t x) { return wave_scan_add(x); }

// ---------------------------------------------------------------- histogram
// Digit counts of the passes [pass_begin, pass_end) from one read of the
// keys: a few large blocks (so that each global count takes few additions),
// per-wave LDS counts merged per block.
constexpr int kHistThreads = 1024;
constexpr int kHistWaves = kHistThreads / 64;
constexpr int kHistMaxPasses = 4;  // tile bytes

__global__ void __launch_bounds__(kHistThreads)
k_sort_hist(const uint64_t* __restrict__ keys, const uint32_t* __restrict__ counters, uint32_t cap,
            int pass_begin, int pass_end, uint32_t* __restrict__ hist) {
  __shared__ uint32_t lh[kHistWaves][kHistMaxPasses * 256];
  const uint32_t K = min(counters[kCntPairs], cap);
  const int wave = threadIdx.x >> 6;
  const int np = pass_end - pass_begin;
  for (int i = threadIdx.x; i < kHistWaves * kHistMaxPasses * 256; i += kHistThreads) (&lh[0][0])[i] = 0;
  __syncthreads();
  const uint32_t stride = gridDim.x * blockDim.x;
  uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  // four keys in flight per step
  for (; i + 3 * stride < K; i += 4 * stride) {
    uint64_t k[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) k[u] = keys[i + u * stride];
#pragma unroll
    for (int u = 0; u < 4; ++u)
      for (int q = 0; q < np; ++q)
        atomicAdd(&lh[wave][q * 256 + ((uint32_t)(k[u] >> (8 * (pass_begin + q))) & 255u)], 1u);
  }
  for (; i < K; i += stride) {
    const uint64_t k = keys[i];
    for (int q = 0; q < np; ++q)
      atomicAdd(&lh[wave][q * 256 + ((uint32_t)(k >> (8 * (pass_begin + q))) & 255u)], 1u);
  }
  __syncthreads();
  for (int i = threadIdx.x; i < np * 256; i += kHistThreads) {
    uint32_t c = 0;
#pragma unroll
    for (int w = 0; w < kHistWaves; ++w) c += lh[w][i];
    if (c) atomicAdd(&hist[pass_begin * 256 + i], c);
  }
}

int device_cus();

// ---------------------------------------------------------------- one pass
__global__ void __launch_bounds__(kSortThreads)
k_sort_pass(uint64_t* __restrict__ keys0, uint64_t* __restrict__ keys1, uint32_t* __restrict__ vals0,
            uint32_t* __restrict__ vals1, const uint32_t* __restrict__ counters, uint32_t cap,
            const uint32_t* __restrict__ hist, int pass_begin, int pass_end, uint32_t* __restrict__ sel_out,
            uint32_t* __restrict__ status, uint32_t nb_max, uint32_t* __restrict__ pass_ctr,
            uint32_t* __restrict__ err, int pass, const uint32_t* __restrict__ sel_in) {
  __shared__ uint32_t s_bid;
  __shared__ uint32_t wave_cnt[kSortWaves][256];
  __shared__ uint32_t s_start[256];
  __shared__ uint32_t s_global[256];
  __shared__ uint32_t s_w[4];
  __shared__ uint64_t s_keys[kSortTile];
  __shared__ uint32_t s_vals[kSortTile];
  __shared__ uint32_t s_triv;
  __shared__ uint32_t s_hw[4];

  const uint32_t K = min(counters[kCntPairs], cap);
  const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
  // Plan, from the digit counts of all passes (complete before the first
  // pass): a pass is a no-op when one digit holds every key; the buffers
  // alternate over the passes that move keys.  Thread t < 256 also takes
  // the exclusive global offset of digit t for this pass.
  if (t == 0) s_triv = 0;
  __syncthreads();
  // the block's ticket is drawn while the counts load (a no-op pass leaves
  // its tickets unused)
  if (t == 511 % kSortThreads) s_bid = atomicAdd(&pass_ctr[pass], 1u);
  uint32_t hc = 0, hinc = 0;
  if (t < 256) {
    // every pass's count of digit t at once (at most kHistMaxPasses passes)
    uint32_t hv[kHistMaxPasses];
#pragma unroll
    for (int q = 0; q < kHistMaxPasses; ++q) hv[q] = hist[min(pass_begin + q, pass_end - 1) * 256 + t];
#pragma unroll
    for (int q = 0; q < kHistMaxPasses; ++q) {
      if (pass_begin + q < pass_end && hv[q] == K) atomicOr(&s_triv, 1u << (pass_begin + q));
      if (pass_begin + q == pass) hc = hv[q];
    }
    hinc = wave_incl_scan(hc);
    if (lane == 63) s_hw[wave] = hinc;
  }
  __syncthreads();
  const uint32_t triv = s_triv;
  uint32_t moved_before = 0, moved_all = 0;
  for (int p = pass_begin; p < pass_end; ++p) {
    const uint32_t mv = ((triv >> p) & 1u) ? 0u : 1u;
    moved_all += mv;
    if (p < pass) moved_before += mv;
  }
  // the keys start in buffer 0, or where an earlier launch left them
  const uint32_t start = sel_in ? (*sel_in & 1u) : 0u;
  if (pass == pass_end - 1 && blockIdx.x == 0 && t == 0) *sel_out = (start + moved_all) & 1u;
  if ((triv >> pass) & 1u) return;
  for (int i = t; i < kSortWaves * 256; i += kSortThreads) (&wave_cnt[0][0])[i] = 0;
  __syncthreads();
  const uint32_t bid = s_bid;
  const uint32_t base = bid * (uint32_t)kSortTile;
  if (base >= K) return;
  const uint32_t src = (start + moved_before) & 1u;
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
      // look back four predecessors per step (block 0 is always inclusive,
      // so the walk ends at j >= 0)
      constexpr int kWin = 4;
      int j = (int)bid - 1;
      uint32_t spins = 0;
      while (j >= 0) {
        uint32_t sv[kWin];
#pragma unroll
        for (int k = 0; k < kWin; ++k)
          sv[k] = j - k >= 0 ? __hip_atomic_load(&st[(size_t)(j - k) * 256 + t], __ATOMIC_RELAXED,
                                                 __HIP_MEMORY_SCOPE_AGENT)
                             : 0u;
        int used = 0;
        bool found = false;
#pragma unroll
        for (int k = 0; k < kWin; ++k) {
          if (found || used < k) break;
          const uint32_t f = sv[k] & ~kValueMask;
          if (f == 0) break;
          excl += sv[k] & kValueMask;
          used = k + 1;
          found = f == kFlagIncl;
        }
        if (found) break;
        j -= used;
        if (used == 0) {
          if (++spins > kSpinLimit) {
            atomicOr(err, 1u);
            break;
          }
          __builtin_amdgcn_s_sleep(1);
        }
      }
      __hip_atomic_store(&st[(size_t)bid * 256 + t], kFlagIncl | (excl + cnt), __ATOMIC_RELAXED,
                         __HIP_MEMORY_SCOPE_AGENT);
    }
    uint32_t doff = hinc - hc;
    for (int w = 0; w < wave; ++w) doff += s_hw[w];
    s_global[t] = doff + excl;
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

// ---------------------------------------------------------------- 12-bit tile pass
// With at most 4096 tiles the whole tile id is one 12-bit digit: the pairs
// are grouped by tile (stably) in one counting pass instead of two 8-bit
// passes, reduce-then-scan: each block of 4096 keys counts its tiles, a scan
// turns the counts into per-block offsets (and the tile totals), and the
// pass ranks and scatters each block's keys with its offsets known - no
// chain of look-backs between blocks.
constexpr int kT12Threads = 512;
constexpr int kT12Waves = kT12Threads / 64;
constexpr int kT12Items = 8;
constexpr int kT12Tile = kT12Threads * kT12Items;  // keys per block
constexpr int kT12Digits = 4096;
constexpr int kT12Own = kT12Digits / kT12Threads;  // digits per thread
static_assert(kT12Own == 8, "eight digits per owner thread");

// Block b's tile counts into counts[b][4096].
__global__ void __launch_bounds__(kT12Threads)
k_tile_count12(const uint64_t* __restrict__ keys, const uint32_t* __restrict__ counters, uint32_t cap,
               uint32_t* __restrict__ counts) {
  __shared__ uint32_t lh[kT12Digits];
  for (int i = threadIdx.x; i < kT12Digits; i += kT12Threads) lh[i] = 0;
  __syncthreads();
  const uint32_t K = min(counters[kCntPairs], cap);
  const uint32_t base = blockIdx.x * (uint32_t)kT12Tile;
  uint32_t d[kT12Items];
#pragma unroll
  for (int r = 0; r < kT12Items; ++r) {
    const uint32_t i = base + (uint32_t)(r * kT12Threads) + threadIdx.x;
    d[r] = i < K ? (uint32_t)(keys[i] >> 32) & (uint32_t)(kT12Digits - 1) : 0xFFFFFFFFu;
  }
#pragma unroll
  for (int r = 0; r < kT12Items; ++r)
    if (d[r] != 0xFFFFFFFFu) atomicAdd(&lh[d[r]], 1u);
  __syncthreads();
  uint4* out = reinterpret_cast<uint4*>(counts + (size_t)blockIdx.x * kT12Digits);
  for (int i = threadIdx.x; i < kT12Digits / 4; i += kT12Threads)
    out[i] = make_uint4(lh[4 * i], lh[4 * i + 1], lh[4 * i + 2], lh[4 * i + 3]);
}

// counts[b][d] becomes the count of tile d in blocks before b, totals[d] the
// tile's count.  A block takes 64 tiles; sixteen threads per tile split the
// blocks holding pairs between them (sum, combine in LDS, then write the
// running offsets), loads in flight 16 at a time (one round for up to 256
// blocks, i.e. 1M pairs).  Then each tile's size
// class (the forward's largest-first order, as k_tile_order files it):
// ballot ranks per class, one addition per class and block reserves the
// block's slots.
constexpr int kT12ScanTiles = 64;
constexpr int kT12ScanSegs = 16;
constexpr int kT12ScanBatch = 16;
constexpr int kT12ScanHeadWaves = kT12ScanTiles / 64;  // waves of segment 0, which hold the totals
static_assert(kT12ScanTiles % 64 == 0 && kT12ScanTiles * kT12ScanSegs <= 1024, "scan block shape");

__global__ void __launch_bounds__(kT12ScanTiles * kT12ScanSegs)
k_tile_scan12(uint32_t* __restrict__ counts, uint32_t n_blocks, const uint32_t* __restrict__ counters,
              uint32_t cap, uint32_t* __restrict__ totals, uint32_t n_tiles, uint32_t* __restrict__ class_count,
              uint32_t* __restrict__ class_list, uint32_t* __restrict__ err) {
  __shared__ uint32_t seg_sum[kT12ScanSegs][kT12ScanTiles];
  __shared__ uint32_t wc[kT12ScanHeadWaves][kTileClasses];
  __shared__ uint32_t cbase[kTileClasses];
  const int seg = threadIdx.x / kT12ScanTiles, dl = threadIdx.x % kT12ScanTiles;
  const uint32_t d = blockIdx.x * kT12ScanTiles + dl;  // < kT12Digits: the grid is exact
  const uint32_t K = min(counters[kCntPairs], cap);
  const uint32_t nb = min(n_blocks, div_up(K, (uint32_t)kT12Tile));  // the blocks holding pairs
  const uint32_t per = div_up(nb, (uint32_t)kT12ScanSegs);
  const uint32_t b0 = min(nb, seg * per), b1 = min(nb, b0 + per);
  uint32_t sum = 0;
  for (uint32_t b = b0; b < b1; b += kT12ScanBatch) {
    uint32_t c[kT12ScanBatch];
#pragma unroll
    for (int u = 0; u < kT12ScanBatch; ++u) c[u] = b + u < b1 ? counts[(size_t)(b + u) * kT12Digits + d] : 0u;
#pragma unroll
    for (int u = 0; u < kT12ScanBatch; ++u) sum += c[u];
  }
  seg_sum[seg][dl] = sum;
  __syncthreads();
  uint32_t run = 0, total = 0;
#pragma unroll
  for (int q = 0; q < kT12ScanSegs; ++q) {
    const uint32_t v = seg_sum[q][dl];
    run += q < seg ? v : 0u;
    total += v;
  }
  for (uint32_t b = b0; b < b1; b += kT12ScanBatch) {
    uint32_t c[kT12ScanBatch];
#pragma unroll
    for (int u = 0; u < kT12ScanBatch; ++u) c[u] = b + u < b1 ? counts[(size_t)(b + u) * kT12Digits + d] : 0u;
#pragma unroll
    for (int u = 0; u < kT12ScanBatch; ++u) {
      if (b + u < b1) counts[(size_t)(b + u) * kT12Digits + d] = run;
      run += c[u];
    }
  }
  // segment 0's threads (the first kT12ScanHeadWaves waves) hold the tile totals
  const bool head = seg == 0;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  uint32_t c = kTileClasses, rank = 0;
  if (head) {
    totals[d] = total;
    if (d >= n_tiles && total) atomicOr(err, 4u);  // a key beyond the tiles
    c = d < n_tiles ? tile_class(total) : kTileClasses;
#pragma unroll
    for (uint32_t k = 0; k < kTileClasses; ++k) {
      const uint64_t m = __ballot(c == k);
      if (c == k) rank = (uint32_t)__popcll(m & lanemask_lt());
      if (lane == 0) wc[wave][k] = (uint32_t)__popcll(m);
    }
  }
  __syncthreads();
  if (threadIdx.x < kTileClasses) {
    uint32_t tot = 0;
#pragma unroll
    for (int w = 0; w < kT12ScanHeadWaves; ++w) tot += wc[w][threadIdx.x];
    cbase[threadIdx.x] = tot ? atomicAdd(&class_count[threadIdx.x], tot) : 0u;
  }
  __syncthreads();
  if (head && c < kTileClasses) {
    uint32_t pos = cbase[c] + rank;
    for (int w = 0; w < wave; ++w) pos += wc[w][c];
    if (pos < n_tiles) class_list[(size_t)c * n_tiles + pos] = d;
  }
}

__global__ void __launch_bounds__(kT12Threads)
k_tile_pass12(const uint64_t* __restrict__ kin, uint64_t* __restrict__ kout, const uint32_t* __restrict__ vin,
              uint32_t* __restrict__ vout, const uint32_t* __restrict__ counters, uint32_t cap,
              const uint32_t* __restrict__ totals, const uint32_t* __restrict__ block_off, uint32_t n_tiles,
              uint32_t* __restrict__ ranges, uint32_t* __restrict__ sel_out, uint32_t* __restrict__ err) {
  __shared__ uint16_t wave_cnt[kT12Waves][kT12Digits];  // per-wave digit counts, then offsets
  __shared__ uint64_t s_keys[kT12Tile];
  __shared__ uint32_t s_vals[kT12Tile];
  __shared__ uint16_t s_start[kT12Digits];  // block-local start of every digit
  __shared__ uint32_t s_global[kT12Digits];
  __shared__ uint32_t s_w[kT12Waves], s_h[kT12Waves];
  const uint32_t K = min(counters[kCntPairs], cap);
  const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
  if (blockIdx.x == 0 && t == 0) *sel_out = 1u;  // the result is in the second buffers
  // Workgroups go to the XCDs in turn (w -> XCD w % 8), and every tile's run
  // takes a few keys from each block, so with blocks in input order an
  // output cache line would be written in part by up to eight L2s.  Each XCD
  // takes consecutive blocks of the ones holding pairs instead: a tile's run
  // is then split between at most eight L2s in eight pieces.
  const uint32_t n_act = div_up(K, (uint32_t)kT12Tile);
  if (blockIdx.x >= n_act) return;
  const uint32_t xcd = blockIdx.x % kXcds, q = n_act / kXcds, rem = n_act % kXcds;
  const uint32_t bid = xcd * q + min(xcd, rem) + blockIdx.x / kXcds;  // a permutation of [0, n_act)
  const uint32_t base = bid * (uint32_t)kT12Tile;
  {
    uint32_t* c = reinterpret_cast<uint32_t*>(&wave_cnt[0][0]);
    for (int i = t; i < kT12Waves * kT12Digits / 2; i += kT12Threads) c[i] = 0u;
  }
  uint64_t key[kT12Items];
  uint32_t val[kT12Items], rank[kT12Items];
  const uint32_t wbase = base + (uint32_t)wave * (kT12Items * 64);
#pragma unroll
  for (int r = 0; r < kT12Items; ++r) {
    const uint32_t idx = wbase + r * 64 + lane;
    const bool valid = idx < K;
    key[r] = valid ? kin[idx] : 0ull;
    val[r] = valid ? vin[idx] : 0u;
  }
  // the tile totals and this block's offsets of the thread's eight digits
  uint32_t hg[kT12Own], bo[kT12Own];
#pragma unroll
  for (int j = 0; j < kT12Own; ++j) {
    hg[j] = totals[kT12Own * t + j];
    bo[j] = block_off[(size_t)bid * kT12Digits + kT12Own * t + j];
  }
  __syncthreads();
  // rank within the wave, in input order (round-major, then lane)
#pragma unroll
  for (int r = 0; r < kT12Items; ++r) {
    const bool valid = (wbase + r * 64 + lane) < K;
    const uint32_t d = (uint32_t)(key[r] >> 32) & (uint32_t)(kT12Digits - 1);
    const uint64_t peers = match_digit_bits<12>(d, valid);
    const uint64_t before = peers & lanemask_lt();
    uint32_t pre = 0;
    if (valid) pre = wave_cnt[wave][d];
    __builtin_amdgcn_wave_barrier();
    if (valid && before == 0) wave_cnt[wave][d] = (uint16_t)(pre + (uint32_t)__popcll(peers));
    __builtin_amdgcn_wave_barrier();
    rank[r] = pre + (uint32_t)__popcll(before);
  }
  __syncthreads();
  // owner thread t: digits 8t .. 8t + 7 - per-wave offsets and block counts
  uint32_t cnt[kT12Own];
  uint32_t own = 0, hown = 0;
#pragma unroll
  for (int j = 0; j < kT12Own; ++j) {
    const int d = kT12Own * t + j;
    uint32_t c[kT12Waves];  // all waves' counts first, so the reads are in flight together
#pragma unroll
    for (int w = 0; w < kT12Waves; ++w) c[w] = wave_cnt[w][d];
    uint32_t run = 0;
#pragma unroll
    for (int w = 0; w < kT12Waves; ++w) {
      wave_cnt[w][d] = (uint16_t)run;
      run += c[w];
    }
    cnt[j] = run;
    own += run;
    hown += hg[j];
  }
  const uint32_t inc = wave_incl_scan(own), hinc = wave_incl_scan(hown);
  if (lane == 63) {
    s_w[wave] = inc;
    s_h[wave] = hinc;
  }
  __syncthreads();
  uint32_t off = inc - own, hoff = hinc - hown;
  for (int w = 0; w < wave; ++w) {
    off += s_w[w];
    hoff += s_h[w];
  }
#pragma unroll
  for (int j = 0; j < kT12Own; ++j) {
    const int d = kT12Own * t + j;
    s_start[d] = (uint16_t)off;
    s_global[d] = hoff + bo[j];
    if (bid == 0 && (uint32_t)d < n_tiles && hg[j]) {  // the tiles' ranges, from their totals (empty: 0, 0)
      ranges[2 * d] = hoff;
      ranges[2 * d + 1] = hoff + hg[j];
    }
    off += cnt[j];
    hoff += hg[j];
  }
  __syncthreads();
  // order the block's keys by digit in LDS (stable), then write digit runs out
#pragma unroll
  for (int r = 0; r < kT12Items; ++r) {
    const bool valid = (wbase + r * 64 + lane) < K;
    if (valid) {
      const uint32_t d = (uint32_t)(key[r] >> 32) & (uint32_t)(kT12Digits - 1);
      const uint32_t pos = s_start[d] + wave_cnt[wave][d] + rank[r];
      s_keys[pos] = key[r];
      s_vals[pos] = val[r];
    }
  }
  __syncthreads();
  const uint32_t n_items = min(K - base, (uint32_t)kT12Tile);
  for (uint32_t i = t; i < n_items; i += kT12Threads) {
    const uint64_t k = s_keys[i];
    const uint32_t d = (uint32_t)(k >> 32) & (uint32_t)(kT12Digits - 1);
    const uint32_t dst = s_global[d] + (i - s_start[d]);
    if (dst < K) {
      kout[dst] = k;
      vout[dst] = s_vals[i];
    } else {
      atomicOr(err, 2u);  // inconsistent offsets: never write out of range
    }
  }
}

bool tile_sort12(uint64_t total_tiles, uint32_t pair_capacity) {
  return total_tiles <= (uint64_t)kT12Digits && pair_capacity <= kT12MaxPairs;
}

size_t tile_sort12_status_words(uint32_t pair_capacity) {
  return (size_t)div_up(pair_capacity > 0 ? pair_capacity : 1u, (uint32_t)kT12Tile) * kT12Digits;
}

// The tile grouping in one pass (tile_sort12 true): keys_a / vals_a into
// keys_b / vals_b, *sel_out = 1, the tiles' ranges and their size classes
// (class_count zero on entry; replaces k_ranges and k_tile_order).
// block_counts holds tile_sort12_status_words words, totals 4096 (neither
// needs clearing).
hipError_t launch_tile_sort12(uint64_t* keys_a, uint64_t* keys_b, uint32_t* vals_a, uint32_t* vals_b,
                              const uint32_t* counters, uint32_t pair_capacity, uint32_t total_tiles,
                              uint32_t* totals, uint32_t* block_counts, uint32_t* ranges, uint32_t* class_count,
                              uint32_t* class_list, uint32_t* sel_out, uint32_t* error_flag, hipStream_t s) {
  if (total_tiles > (uint32_t)kT12Digits) return hipErrorInvalidValue;
  const uint32_t nb = div_up(pair_capacity > 0 ? pair_capacity : 1u, (uint32_t)kT12Tile);
  hipLaunchKernelGGL(k_tile_count12, dim3(nb), dim3(kT12Threads), 0, s, keys_a, counters, pair_capacity,
                     block_counts);
  hipLaunchKernelGGL(k_tile_scan12, dim3(kT12Digits / kT12ScanTiles), dim3(kT12ScanTiles * kT12ScanSegs), 0, s,
                     block_counts, nb, counters, pair_capacity, totals, total_tiles, class_count, class_list,
                     error_flag);
  hipLaunchKernelGGL(k_tile_pass12, dim3(nb), dim3(kT12Threads), 0, s, keys_a, keys_b, vals_a, vals_b, counters,
                     pair_capacity, totals, block_counts, total_tiles, ranges, sel_out, error_flag);
  return hipGetLastError();
}

size_t sort_status_words(uint32_t pair_capacity) {
  return (size_t)kMaxSortPasses * div_up(pair_capacity > 0 ? pair_capacity : 1u, (uint32_t)kSortTile) * 256;
}

// Radix passes [pass_begin, pass_end) (bits 8 * pass_begin up) of the
// pair keys in keys_a / vals_a.  On entry hist [kMaxSortPasses][256],
// pass_ctr [kMaxSortPasses] and the passes' look-back words in status are
// zero; the digit counts go to hist.
// *sel_out receives the buffer holding the result (0: a, 1: b); with no
// pass it is left as it is.  sel_in (nullable, a word other than sel_out)
// says which buffer holds the keys on entry (an earlier launch's passes);
// the digit counts are read from keys_a, which then holds a permutation of
// the keys too.
hipError_t launch_sort(uint64_t* keys_a, uint64_t* keys_b, uint32_t* vals_a, uint32_t* vals_b,
                       const uint32_t* counters, uint32_t pair_capacity, int pass_begin, int pass_end,
                       uint32_t* hist, uint32_t* status, uint32_t* pass_ctr, uint32_t* sel_out,
                       uint32_t* error_flag, hipStream_t s, const uint32_t* sel_in) {
  if (pass_begin < 0 || pass_end > kMaxSortPasses || pass_begin > pass_end) return hipErrorInvalidValue;
  if (pass_end - pass_begin > kHistMaxPasses) return hipErrorInvalidValue;
  const uint32_t nb_max = div_up(pair_capacity > 0 ? pair_capacity : 1u, (uint32_t)kSortTile);
  if (pass_end > pass_begin) {
    // about 16 keys per thread; at most 64 blocks (few global additions per
    // count) unless the pairs need more, then up to one block per compute unit
    uint32_t hb = div_up(pair_capacity > 0 ? pair_capacity : 1u, (uint32_t)kHistThreads * 16u);
    const uint32_t hb_max = hb > 256 ? (uint32_t)std::max(64, device_cus()) : 64u;
    if (hb > hb_max) hb = hb_max;
    hipLaunchKernelGGL(k_sort_hist, dim3(hb), dim3(kHistThreads), 0, s, keys_a, counters, pair_capacity,
                       pass_begin, pass_end, hist);
  }
  for (int p = pass_begin; p < pass_end; ++p)
    hipLaunchKernelGGL(k_sort_pass, dim3(nb_max), dim3(kSortThreads), 0, s, keys_a, keys_b, vals_a, vals_b,
                       counters, pair_capacity, hist, pass_begin, pass_end, sel_out, status, nb_max, pass_ctr,
                       error_flag, p, sel_in);
  return hipGetLastError();
}

// Look-back words of pass p: status + p * sort_status_stride(P), that many.
size_t sort_status_stride(uint32_t pair_capacity) {
  return (size_t)div_up(pair_capacity > 0 ? pair_capacity : 1u, (uint32_t)kSortTile) * 256;
}

// ---------------------------------------------------------------- per-tile depth sort
constexpr int kSegItems = 8;  // keys per thread and chunk

// A sorting group is either one wave (THREADS == 64, one of several
// independent groups of a block) or the whole block.
template <int THREADS>
__device__ __forceinline__ void seg_sync() {
  if constexpr (THREADS == 64) {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  } else {
    __syncthreads();
  }
}
// The thread index, read afresh at each use: a volatile move cannot be
// hoisted, so the index arithmetic of every sorting path stays inside the
// work item that needs it instead of being kept live (and spilled) across
// the whole hand-out loop.
__device__ __forceinline__ uint32_t seg_thread() {
  uint32_t r;
  asm volatile("v_mov_b32 %0, %1" : "=v"(r) : "v"((uint32_t)threadIdx.x));
  return r;
}
template <int THREADS>
__device__ __forceinline__ int seg_tid() {  // index within the sorting group
  return (int)(seg_thread() % (unsigned)THREADS);
}

struct SegArgs {
  uint64_t* keys_a;
  uint64_t* keys_b;
  uint32_t* vals_a;
  uint32_t* vals_b;
  const uint32_t* sel;
  const uint32_t* ranges;
  const uint32_t* rec_of;
  const uint32_t* counters;
  uint32_t cap;
  uint32_t* emit;       // nullable
  uint64_t* keys_out;   // nullable
  uint32_t* err;
  uint32_t n_tiles;
  const uint32_t* class_count;  // tiles per size class, largest first (k_tile_order)
  const uint32_t* class_list;   // [kTileClasses][n_tiles]
  uint32_t* ticket;             // zero on entry: large tiles handed out after the first G
};

// Segments that fit in LDS are sorted on packed items: (depth bits minus the
// segment's smallest) << 16 | index in the segment, with digits of DBITS
// bits; only as many passes as the depth range needs (a range below
// 2^(3 DBITS) takes three).  The emission index and record id stay in LDS by
// segment index and are looked up once at the end.
// BIG: the layout of the chunked sort of segments above kCap pairs (below),
// where items carry the emission index and the segment's digit offsets and
// running positions are kept instead.
template <int THREADS, int DBITS, bool BIG = false>
struct SegLdsP {
  static constexpr int kWaves = THREADS / 64;
  static constexpr int kCap = THREADS * kSegItems;
  static constexpr int kDigits = 1 << DBITS;
  uint64_t item[kCap];
  uint32_t val[BIG ? 1 : kCap];
  uint32_t rec[BIG ? 1 : kCap];
  uint16_t cnt[kWaves][kDigits];  // per-wave digit counts, then offsets
  uint32_t start[kDigits];        // first position of every digit
  uint32_t wsum[kWaves];
  uint32_t red[2][kWaves];
  uint32_t run[BIG ? kDigits : 1];                  // segment position of every digit's next item
  uint32_t base[BIG ? 4 : 1][BIG ? kDigits : 1];  // segment digit counts, then offsets, per pass
};

// Positions of this thread's items (entries wave * I * 64 + r * 64 + lane,
// r < I, valid below n) when the segment is stably ordered by the digit at
// `shift`.  L.cnt must be zero on entry; it holds offsets on return.  With
// one digit per owner thread (THREADS >= 2^DBITS), thread t < 2^DBITS gets
// the count of digit t back.
template <int THREADS, int DBITS, bool BIG>
__device__ __forceinline__ uint32_t seg_rank_p(SegLdsP<THREADS, DBITS, BIG>& L, const uint64_t (&item)[kSegItems],
                                               int I, uint32_t n, int shift, uint32_t (&pos)[kSegItems]) {
  constexpr int D = 1 << DBITS;
  constexpr int DPT = D >= THREADS ? D / THREADS : 1;  // digits per owner thread
  constexpr int OWNERS = D / DPT;
  constexpr int W = THREADS / 64;
  const int t = seg_tid<THREADS>(), lane = t & 63, wave = t >> 6;
  uint32_t rank[kSegItems];
#pragma unroll
  for (int r = 0; r < kSegItems; ++r) {
    if (r >= I) break;
    const uint32_t idx = (uint32_t)(wave * I + r) * 64u + lane;
    const bool valid = idx < n;
    const uint32_t d = (uint32_t)(item[r] >> shift) & (uint32_t)(D - 1);
    const uint64_t peers = match_digit_bits<DBITS>(d, valid);
    const uint64_t before = peers & lanemask_lt();
    uint32_t pre = 0;
    if (valid) pre = L.cnt[wave][d];
    __builtin_amdgcn_wave_barrier();
    if (valid && before == 0) L.cnt[wave][d] = (uint16_t)(pre + (uint32_t)__popcll(peers));
    __builtin_amdgcn_wave_barrier();
    rank[r] = pre + (uint32_t)__popcll(before);
  }
  seg_sync<THREADS>();
  uint32_t dcnt[DPT];
  uint32_t own = 0, inc = 0;
  if (t < OWNERS) {
#pragma unroll
    for (int j = 0; j < DPT; ++j) {
      const int d = t * DPT + j;
      uint32_t c[W];  // all waves' counts first, so the reads are in flight together
#pragma unroll
      for (int w = 0; w < W; ++w) c[w] = L.cnt[w][d];
      uint32_t run = 0;
#pragma unroll
      for (int w = 0; w < W; ++w) {
        L.cnt[w][d] = (uint16_t)run;
        run += c[w];
      }
      dcnt[j] = run;
      own += run;
    }
    inc = wave_incl_scan(own);
    if (OWNERS > 64 && lane == 63) L.wsum[wave] = inc;
  }
  if (OWNERS > 64) seg_sync<THREADS>();
  if (t < OWNERS) {
    uint32_t off = inc - own;
    if (OWNERS > 64)
      for (int w = 0; w < wave; ++w) off += L.wsum[w];
#pragma unroll
    for (int j = 0; j < DPT; ++j) {
      L.start[t * DPT + j] = off;
      off += dcnt[j];
    }
  }
  seg_sync<THREADS>();
#pragma unroll
  for (int r = 0; r < kSegItems; ++r) {
    if (r >= I) break;
    const uint32_t idx = (uint32_t)(wave * I + r) * 64u + lane;
    const uint32_t d = (uint32_t)(item[r] >> shift) & (uint32_t)(D - 1);
    pos[r] = idx < n ? L.start[d] + L.cnt[wave][d] + rank[r] : 0u;
  }
  return (DPT == 1 && t < OWNERS) ? dcnt[0] : 0u;  // with one digit per owner: its count
}

template <int THREADS, int DBITS, bool BIG>
__device__ __forceinline__ void seg_clear_counts(SegLdsP<THREADS, DBITS, BIG>& L) {
  constexpr int kWords = THREADS / 64 * (1 << DBITS) / 2;
  uint32_t* c = reinterpret_cast<uint32_t*>(&L.cnt[0][0]);
  for (int i = seg_tid<THREADS>(); i < kWords; i += THREADS) c[i] = 0;
}

// Block-wide min and max of the thread values.
template <int THREADS, int DBITS, bool BIG>
__device__ __forceinline__ void seg_min_max(SegLdsP<THREADS, DBITS, BIG>& L, uint32_t& lo, uint32_t& hi) {
  constexpr int W = THREADS / 64;
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    lo = min(lo, (uint32_t)__shfl_xor((int)lo, off, 64));
    hi = max(hi, (uint32_t)__shfl_xor((int)hi, off, 64));
  }
  if constexpr (W > 1) {
    const int t = seg_tid<THREADS>(), wave = t >> 6;
    if ((t & 63) == 0) {
      L.red[0][wave] = lo;
      L.red[1][wave] = hi;
    }
    __syncthreads();
#pragma unroll
    for (int w = 0; w < W; ++w) {
      lo = min(lo, L.red[0][w]);
      hi = max(hi, L.red[1][w]);
    }
  }
}

// Sorts segment [s0, s0 + n), n <= kCap, stably by depth bits and writes
// vals[k] = record id, emit[k] = emission index (if emit), keys_out[k] =
// full key (if keys_out).  Groups that share the block's barriers (halves
// of a block) run in lockstep: pass_max (zero on entry, shared) makes them
// take the same number of passes (extra passes on a zero digit move
// nothing), and a group with n = 0 only takes part in the barriers.
template <int THREADS, int DBITS>
__device__ void sort_segment_lds(SegLdsP<THREADS, DBITS, false>& L, const SegArgs& a, uint32_t tile, uint32_t s0,
                                 uint32_t n, uint32_t K, uint32_t* pass_max = nullptr) {
  constexpr int kCap = SegLdsP<THREADS, DBITS>::kCap;
  static_assert(kCap <= 65536, "segment index is packed in 16 bits");
  const int t = seg_tid<THREADS>(), lane = t & 63, wave = t >> 6;
  const bool side = *a.sel != 0;
  const uint64_t* kin = side ? a.keys_b : a.keys_a;
  uint32_t* vals = side ? a.vals_b : a.vals_a;
  const int I = (int)div_up(n, (uint32_t)THREADS);
  // branch-free loads (indices clamped into the segment) so that all of
  // them are in flight at once; items past the segment (or r >= I) reload
  // its last entry, a real key, which changes neither the minimum nor the
  // maximum
  uint32_t key[kSegItems], val[kSegItems], rec[kSegItems];
  uint32_t bad = 0, lo = 0xFFFFFFFFu, hi = 0u;
  if (n > 0) {  // (uniform in the group)
#pragma unroll
    for (int r = 0; r < kSegItems; ++r) {
      const uint32_t ic = min((uint32_t)(wave * I + r) * 64u + lane, n - 1u);
      key[r] = (uint32_t)kin[s0 + ic];
      val[r] = vals[s0 + ic];
    }
#pragma unroll
    for (int r = 0; r < kSegItems; ++r) {
      bad |= val[r] >= K ? 1u : 0u;
      rec[r] = a.rec_of[min(val[r], K - 1u)];
      lo = min(lo, key[r]);
      hi = max(hi, key[r]);
    }
  } else {
#pragma unroll
    for (int r = 0; r < kSegItems; ++r) key[r] = val[r] = rec[r] = 0u;
  }
  if (bad) atomicOr(a.err, 32u);
  seg_clear_counts(L);
  seg_min_max(L, lo, hi);  // (with several waves its barrier also publishes the cleared counts)
  if constexpr (THREADS == 64) seg_sync<THREADS>();
  const uint32_t range = n > 0 ? hi - lo : 0u;
  const int bits = range ? 32 - __builtin_clz(range) : 0;
  int passes = (bits + DBITS - 1) / DBITS;
  if (pass_max) {  // groups in lockstep: the most passes any of them needs
    if (t == 0) atomicMax(pass_max, (uint32_t)passes);
    __syncthreads();
    passes = (int)*pass_max;
  }
  auto put = [&](uint32_t o, uint32_t depth, uint32_t e, uint32_t rc) {
    if (o >= n) {
      atomicOr(a.err, 32u);
      return;
    }
    vals[s0 + o] = rc;
    if (a.emit) a.emit[s0 + o] = e;
    if (a.keys_out) a.keys_out[s0 + o] = ((uint64_t)tile << 32) | depth;
  };
  if (passes == 0) {  // one depth: the emission order stands
    seg_sync<THREADS>();  // every lane has read its input before any output overwrites vals
#pragma unroll
    for (int r = 0; r < kSegItems; ++r) {
      if (r >= I) break;
      const uint32_t idx = (uint32_t)(wave * I + r) * 64u + lane;
      if (idx < n) put(idx, key[r], val[r], rec[r]);
    }
    return;
  }
  uint64_t item[kSegItems];
  uint32_t pos[kSegItems];
#pragma unroll
  for (int r = 0; r < kSegItems; ++r) {
    const uint32_t idx = (uint32_t)(wave * I + r) * 64u + lane;
    item[r] = ((uint64_t)(key[r] - lo) << 16) | (idx & 0xFFFFu);
    if (r < I && idx < n) {
      L.val[idx] = val[r];
      L.rec[idx] = rec[r];
    }
  }
  for (int p = 0; p < passes; ++p) {
    if (p > 0) {
#pragma unroll
      for (int r = 0; r < kSegItems; ++r) {
        if (r >= I) break;
        const uint32_t idx = (uint32_t)(wave * I + r) * 64u + lane;
        if (idx < n) item[r] = L.item[idx];
      }
    }
    seg_rank_p(L, item, I, n, 16 + DBITS * p, pos);
    seg_sync<THREADS>();  // all positions taken: the counts can be cleared, items moved
    if (p + 1 < passes) seg_clear_counts(L);
#pragma unroll
    for (int r = 0; r < kSegItems; ++r) {
      if (r >= I) break;
      const uint32_t idx = (uint32_t)(wave * I + r) * 64u + lane;
      if (idx < n) L.item[pos[r]] = item[r];
    }
    seg_sync<THREADS>();
  }
  for (uint32_t i = t; i < n; i += THREADS) {
    const uint64_t x = L.item[i];
    const uint32_t idx = (uint32_t)x & 0xFFFFu;
    put(i, (uint32_t)(x >> 16) + lo, L.val[idx], L.rec[idx]);
  }
}

// Segments above kCap pairs (many in the 4M and stereo workloads): LSD
// passes through global memory, one chunk of kCap items at a time, on
// packed items ((depth - segment minimum) << 32 | emission index) with
// 9-bit digits and only as many passes as the depth range needs.  One read
// finds the depth range, a second packs the items into the other key buffer
// and counts the digits of every pass; each pass then ranks a chunk in LDS
// (stable), and places each digit's items after those of the earlier chunks
// (running positions from the segment's digit offsets), ping-ponging between
// the two key buffers.  The last pass writes the results.
using SegLdsBig = SegLdsP<1024, 9, true>;

__device__ void sort_segment_big(SegLdsBig& L, const SegArgs& a, uint32_t tile, uint32_t s0, uint32_t n,
                                 uint32_t K) {
  constexpr int T = 1024, DB = 9, D = 1 << DB, kCap = SegLdsBig::kCap;
  const int t = (int)seg_thread(), lane = t & 63, wave = t >> 6;
  const bool side = *a.sel != 0;
  uint64_t* kin = side ? a.keys_b : a.keys_a;
  uint64_t* kother = side ? a.keys_a : a.keys_b;
  uint32_t* vals = side ? a.vals_b : a.vals_a;
  auto put = [&](uint32_t o, uint32_t depth, uint32_t e, uint32_t rc) {
    if (o >= n) {
      atomicOr(a.err, 32u);
      return;
    }
    vals[s0 + o] = rc;
    if (a.emit) a.emit[s0 + o] = e;
    if (a.keys_out) a.keys_out[s0 + o] = ((uint64_t)tile << 32) | depth;
  };
  constexpr uint32_t kRound = (uint32_t)T * kSegItems;
  // depth range (branch-free rounds of kSegItems keys per thread)
  uint32_t lo = 0xFFFFFFFFu, hi = 0u;
  for (uint32_t b0 = 0; b0 < n; b0 += kRound) {
    uint32_t k[kSegItems];
#pragma unroll
    for (int r = 0; r < kSegItems; ++r) k[r] = (uint32_t)kin[s0 + min(b0 + (uint32_t)(r * T + t), n - 1u)];
#pragma unroll
    for (int r = 0; r < kSegItems; ++r) {
      lo = min(lo, k[r]);
      hi = max(hi, k[r]);
    }
  }
  seg_min_max(L, lo, hi);
  const uint32_t range = hi - lo;
  const int bits = range ? 32 - __builtin_clz(range) : 0;
  const int passes = (bits + DB - 1) / DB;
  for (int i = t; i < 4 * D; i += T) (&L.base[0][0])[i] = 0u;
  seg_clear_counts(L);
  __syncthreads();
  // pack, and count the digits of every pass
  for (uint32_t b0 = 0; b0 < n; b0 += kRound) {
    uint32_t k[kSegItems], v[kSegItems];
#pragma unroll
    for (int r = 0; r < kSegItems; ++r) {
      const uint32_t ic = min(b0 + (uint32_t)(r * T + t), n - 1u);
      k[r] = (uint32_t)kin[s0 + ic] - lo;
      v[r] = vals[s0 + ic];
    }
#pragma unroll
    for (int r = 0; r < kSegItems; ++r) {
      const uint32_t i = b0 + (uint32_t)(r * T + t);
      const bool valid = i < n;
      if (valid) kother[s0 + i] = ((uint64_t)k[r] << 32) | v[r];
      for (int p = 0; p < passes; ++p) {
        const uint32_t d = (k[r] >> (DB * p)) & (uint32_t)(D - 1);
        const uint64_t peers = match_digit_bits<DB>(d, valid);
        if (valid && (peers & lanemask_lt()) == 0) atomicAdd(&L.base[p][d], (uint32_t)__popcll(peers));
      }
    }
  }
  __syncthreads();
  // exclusive digit offsets per pass (owner thread t < D holds digit t)
  for (int p = 0; p < passes; ++p) {
    uint32_t c = 0, inc = 0;
    if (t < D) {
      c = L.base[p][t];
      inc = wave_incl_scan(c);
      if (lane == 63) L.wsum[wave] = inc;
    }
    __syncthreads();
    if (t < D) {
      uint32_t off = inc - c;
      for (int w = 0; w < wave; ++w) off += L.wsum[w];
      L.base[p][t] = off;
    }
    __syncthreads();
  }
  auto record_of = [&](uint32_t e) -> uint32_t { return a.rec_of[min(e, K - 1u)]; };
  if (passes == 0) {  // one depth: the emission order stands
    for (uint32_t b0 = 0; b0 < n; b0 += 4u * T) {
      uint64_t x[4];
      uint32_t rc[4];
#pragma unroll
      for (int r = 0; r < 4; ++r) x[r] = kother[s0 + min(b0 + (uint32_t)(r * T + t), n - 1u)];
#pragma unroll
      for (int r = 0; r < 4; ++r) rc[r] = record_of((uint32_t)x[r]);
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const uint32_t i = b0 + (uint32_t)(r * T + t);
        if (i < n) put(i, (uint32_t)(x[r] >> 32) + lo, (uint32_t)x[r], rc[r]);
      }
    }
    return;
  }
  uint64_t* src = kother;
  uint64_t* dst = kin;
  for (int p = 0; p < passes; ++p) {
    const int shift = 32 + DB * p;
    const bool last = p + 1 == passes;
    if (t < D) L.run[t] = L.base[p][t];
    for (uint32_t cb = 0; cb < n; cb += kCap) {
      const uint32_t nc = min((uint32_t)kCap, n - cb);
      const int I = (int)div_up(nc, (uint32_t)T);
      uint64_t it[kSegItems];
      uint32_t pos[kSegItems];
#pragma unroll
      for (int r = 0; r < kSegItems; ++r) it[r] = src[s0 + cb + min((uint32_t)(wave * I + r) * 64u + lane, nc - 1u)];
      const uint32_t dc = seg_rank_p(L, it, I, nc, shift, pos);  // (its barriers also publish L.run)
      __syncthreads();  // all positions taken: the counts can be cleared, items moved
      seg_clear_counts(L);
#pragma unroll
      for (int r = 0; r < kSegItems; ++r) {
        if (r >= I) break;
        const uint32_t idx = (uint32_t)(wave * I + r) * 64u + lane;
        if (idx < nc) L.item[pos[r]] = it[r];
      }
      __syncthreads();
      // each digit's run of the chunk goes after the earlier chunks' items of
      // that digit (four items per thread at a time, their gathers in flight)
      for (int h = 0; h < kSegItems; h += 4) {
        uint64_t x[4];
        uint32_t rc[4];
#pragma unroll
        for (int r = 0; r < 4; ++r) x[r] = L.item[min((uint32_t)((h + r) * T + t), nc - 1u)];
        if (last) {
#pragma unroll
          for (int r = 0; r < 4; ++r) rc[r] = record_of((uint32_t)x[r]);
        }
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const uint32_t i = (uint32_t)((h + r) * T + t);
          if (i >= nc) break;
          const uint32_t d = (uint32_t)(x[r] >> shift) & (uint32_t)(D - 1);
          const uint32_t o = L.run[d] + (i - L.start[d]);
          if (last) {
            put(o, (uint32_t)(x[r] >> 32) + lo, (uint32_t)x[r], rc[r]);
          } else if (o < n) {
            dst[s0 + o] = x[r];
          } else {
            atomicOr(a.err, 32u);
          }
        }
      }
      __syncthreads();
      if (t < D) L.run[t] += dc;
      __syncthreads();
    }
    uint64_t* tmp = src;
    src = dst;
    dst = tmp;
  }
}

static_assert(kSegWaveMax == 64 * kSegItems, "a wave sorts kSegItems keys per lane");

// Segments up to kSegWaveMax pairs are sorted by one wave each (8-bit
// digits), larger ones by the whole block (9-bit digits: three passes for a
// depth range below 2^27).
constexpr int kSegWaveDigitBits = 8;
constexpr int kSegBlockDigitBits = 9;
constexpr int kSegSmallWaves = 16;           // small tiles per block item, one per wave
constexpr uint32_t kSegBlockClasses = 15;  // classes with floor(2 log2 n) >= 18, i.e. n >= 512
constexpr uint32_t kSegSingleClasses = 9;  // n >= 4096: a whole block; below, two tiles per block (halves)
constexpr int kSegHalfThreads = 512;
static_assert(kSegWaveMax == 512 && kSegBlockClasses < kTileClasses, "size classes of k_tile_order");

// One launch of G blocks of 1024 threads for every tile (the size classes of
// k_tile_order, largest first).  Items, in about descending cost: the tiles
// of at least 4096 pairs, one per block; the tiles of at most kSegWaveMax
// pairs in groups of kSegSmallWaves, one per wave (a wave on ~500 pairs
// takes about as long as a block on a large tile); then the tiles in
// between two per block, one per 512-thread half, the halves in lockstep.
// Block b starts with item b; later items go to whichever block is free
// first, so a block holding one of the largest tiles takes nothing else.
__global__ void __launch_bounds__(1024) k_sort_segments(SegArgs a) {
  __shared__ union {
    SegLdsP<1024, kSegBlockDigitBits> packed;  // a large tile that fits in LDS
    SegLdsBig chunked;                          // larger: chunks through global memory
    SegLdsP<64, kSegWaveDigitBits> small[kSegSmallWaves];
    SegLdsP<kSegHalfThreads, kSegBlockDigitBits> half[2];
  } L;
  __shared__ uint32_t s_end[kTileClasses];  // inclusive prefix of the class counts (empty tiles left out)
  __shared__ uint32_t s_next, s_passes;
  const uint32_t K = min(a.counters[kCntPairs], a.cap);
  if (threadIdx.x < 64) {
    const uint32_t k = threadIdx.x;
    const uint32_t cnt = k + 1 < kTileClasses ? min(a.class_count[k], a.n_tiles) : 0u;
    const uint32_t inc = wave_scan_add(cnt);
    if (k < kTileClasses) s_end[k] = inc;
  }
  __syncthreads();
  const uint32_t n_single = s_end[kSegSingleClasses - 1];
  const uint32_t n_big = s_end[kSegBlockClasses - 1];
  const uint32_t n_all = s_end[kTileClasses - 1];
  const uint32_t n_groups = div_up(n_all - n_big, (uint32_t)kSegSmallWaves);
  const uint32_t n_pairs = div_up(n_big - n_single, 2u);
  const uint32_t total = n_single + n_groups + n_pairs;
  // the idx-th tile of the class order (idx < n_all) and its segment
  auto segment = [&](uint32_t idx, uint32_t& tile, uint32_t& s0, uint32_t& s1) {
    uint32_t lo = 0, hi = kTileClasses - 1;  // first class with s_end > idx
    while (lo < hi) {
      const uint32_t mid = (lo + hi) >> 1;
      if (s_end[mid] > idx) hi = mid; else lo = mid + 1;
    }
    tile = a.class_list[(size_t)lo * a.n_tiles + (idx - (lo ? s_end[lo - 1] : 0u))];
    s0 = s1 = 0;
    if (tile < a.n_tiles) {
      s0 = a.ranges[2 * tile];
      s1 = a.ranges[2 * tile + 1];
    }
    return tile < a.n_tiles && s1 <= K && s0 <= s1;
  };
  for (uint32_t i = blockIdx.x; i < total;) {
    uint32_t tile = 0, s0 = 0, s1 = 0;
    if (i < n_single) {
      const bool ok = segment(i, tile, s0, s1);
      if (!ok) {
        if (threadIdx.x == 0) atomicOr(a.err, 32u);
      } else if (s1 > s0) {
        if (s1 - s0 <= (uint32_t)SegLdsP<1024, kSegBlockDigitBits>::kCap)
          sort_segment_lds(L.packed, a, tile, s0, s1 - s0, K);
        else
          sort_segment_big(L.chunked, a, tile, s0, s1 - s0, K);
      }
    } else if (i < n_single + n_groups) {
      const uint32_t wave = seg_thread() >> 6, lane = seg_thread() & 63u;
      const uint32_t idx = n_big + (i - n_single) * kSegSmallWaves + wave;
      if (idx < n_all) {
        const bool ok = segment(idx, tile, s0, s1) && s1 - s0 <= kSegWaveMax;
        if (!ok) {
          if (lane == 0) atomicOr(a.err, 32u);
        } else if (s1 > s0) {
          sort_segment_lds(L.small[wave], a, tile, s0, s1 - s0, K);
        }
      }
    } else {
      // two tiles, one per half; a half without a (valid) tile only keeps step
      const uint32_t h = seg_thread() / kSegHalfThreads;
      const uint32_t idx = n_single + 2 * (i - n_single - n_groups) + h;
      uint32_t n = 0;
      if (idx < n_big) {
        const bool ok = segment(idx, tile, s0, s1) &&
                        s1 - s0 <= (uint32_t)SegLdsP<kSegHalfThreads, kSegBlockDigitBits>::kCap;
        if (!ok) {
          if (threadIdx.x % kSegHalfThreads == 0) atomicOr(a.err, 32u);
        } else {
          n = s1 - s0;
        }
      }
      if (threadIdx.x == 0) s_passes = 0;  // (published by the first barrier inside)
      sort_segment_lds(L.half[h], a, tile, s0, n, K, &s_passes);
    }
    if (threadIdx.x == 0) s_next = gridDim.x + atomicAdd(a.ticket, 1u);
    __syncthreads();  // LDS is reused by the next item
    i = s_next;
    __syncthreads();
  }
}

int device_cus() {
  static int cus[64] = {0};
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return 256;
  if (cus[dev] == 0) {
    int c = 0;
    if (hipDeviceGetAttribute(&c, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || c <= 0) c = 256;
    cus[dev] = c;
  }
  return cus[dev];
}

// After the tile passes: per-tile depth sort, record ids and emission
// indices.  keys_out (nullable) receives the sorted 64-bit keys.
hipError_t launch_sort_segments(uint64_t* keys_a, uint64_t* keys_b, uint32_t* vals_a, uint32_t* vals_b,
                                const uint32_t* sel, const uint32_t* ranges, uint32_t total_tiles,
                                const uint32_t* rec_of, const uint32_t* counters, uint32_t pair_capacity,
                                uint32_t* emit, uint64_t* keys_out, const uint32_t* class_count,
                                const uint32_t* class_list, uint32_t* seg_ticket, uint32_t* error_flag,
                                hipStream_t s) {
  if (total_tiles == 0 || pair_capacity == 0) return hipSuccess;
  SegArgs a{keys_a, keys_b, vals_a, vals_b, sel, ranges, rec_of, counters, pair_capacity, emit, keys_out,
            error_flag, total_tiles, class_count, class_list, seg_ticket};
  const uint32_t G = std::min<uint32_t>(total_tiles, (uint32_t)std::max(1, device_cus()));
  hipLaunchKernelGGL(k_sort_segments, dim3(G), dim3(1024), 0, s, a);
  return hipGetLastError();
}

}  // namespace gsr
