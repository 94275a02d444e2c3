// Tile binning for gfx950: depth order, pair emission, stable tile sort, ranges.
//
// The per-tile lists must be ordered by (tile, fp32 depth, Gaussian index).  Rather
// than radix-sorting 64-bit (tile | depth) keys of every pair (6 passes over K
// pairs), the (view, Gaussian) entries are first sorted by depth alone (4 passes
// over V*N entries, stable, so equal depths keep index order); pairs are then
// emitted in that order and stably sorted by tile id only (ceil(log2 tiles)/8
// passes over K).  A stable sort of depth-ordered pairs by tile yields exactly the
// (tile, depth, index) order.
//
// Radix sort: least-significant-digit, 8-bit digits, reduce-then-scan.  Each
// 256-thread workgroup owns 4096 consecutive items.  Stable ranks inside a
// workgroup come from wave64 ballots (8 ballots give each lane the mask of lanes
// holding the same digit), per-wave digit counts in LDS and a running count per
// digit across the workgroup's 16 rounds.  The workgroup then places its items in
// LDS in digit order and writes each digit's run contiguously to global memory.
#include "gs_geom.h"

#pragma clang fp contract(off)

namespace gsk {
namespace {

constexpr int kThreads = 256;
constexpr int kWaves = kThreads / 64;
constexpr int kItems = kSortTileItems / kThreads;   // items per thread (16)
constexpr int kRadix = 256;

// Wave-inclusive prefix of x over lanes (DPP: shifts within rows of 16 lanes, then
// the last lane of a row broadcast into the rows after it; 0, the identity, is the
// value of lanes with no source, so each step is one DPP add).  Whole wavefronts only.
__device__ inline uint32_t wave_incl_scan(uint32_t x) {
  x += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x111, 0xf, 0xf, false);   // row_shr:1
  x += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x112, 0xf, 0xf, false);   // row_shr:2
  x += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x114, 0xf, 0xf, false);   // row_shr:4
  x += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x118, 0xf, 0xf, false);   // row_shr:8
  x += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x142, 0xa, 0xf, false);   // row_bcast:15 into rows 1, 3
  x += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x143, 0xc, 0xf, false);   // row_bcast:31 into rows 2, 3
  return x;
}

__device__ inline uint64_t lanemask_lt() {
  const unsigned lane = __lane_id();
  return lane == 0 ? 0ull : (~0ull >> (64 - lane));
}

// Mask of the active lanes whose 8-bit digit equals this lane's.
__device__ inline uint64_t match_digit(uint32_t d, bool valid) {
  uint64_t peers = __ballot(valid);
#pragma unroll
  for (int b = 0; b < 8; ++b) {
    const bool bit = (d >> b) & 1u;
    const uint64_t m = __ballot(bit);
    peers &= bit ? m : ~m;
  }
  return peers;
}

// Per-workgroup digit histogram.  Wave w of a workgroup owns items
// [base + 1024 w, base + 1024 (w + 1)) and counts them into its own LDS counters
// with non-returning atomic adds (no dependence from one 64-item round to the
// next); a round whose valid items all share one digit (the common case for the
// high digits of clustered keys) is added by one lane.
// Items to sort: n (the capacity the grids are sized for), or the count in device
// memory when there is one (never above n).
__device__ inline size_t item_count(size_t n, const unsigned long long* n_dev) {
  if (!n_dev) return n;
  const unsigned long long d = *n_dev;
  return d < (unsigned long long)n ? (size_t)d : n;
}

__global__ __launch_bounds__(kThreads) void k_radix_hist(const uint32_t* __restrict__ keys, size_t n_cap,
                                                          const unsigned long long* __restrict__ n_dev, int shift,
                                                          uint32_t* __restrict__ hist) {
  __shared__ uint32_t hw[kWaves][kRadix];
  const size_t n = item_count(n_cap, n_dev);
  // rows past the item count's blocks are never read (the scan and the scatter
  // size themselves from the same count)
  if ((size_t)blockIdx.x * kSortTileItems >= n) return;
  const int w = threadIdx.x / 64;
  for (int i = 0; i < kWaves; ++i) hw[i][threadIdx.x] = 0;
  __syncthreads();
  const size_t base = (size_t)blockIdx.x * kSortTileItems + (size_t)w * (kItems * 64) + __lane_id();
  uint32_t kk[kItems];
#pragma unroll
  for (int r = 0; r < kItems; ++r) {   // all loads in flight before any counting
    const size_t i = base + (size_t)r * 64;
    kk[r] = i < n ? keys[i] : 0u;
  }
#pragma unroll
  for (int r = 0; r < kItems; ++r) {
    const bool valid = base + (size_t)r * 64 < n;
    const uint32_t d = (kk[r] >> shift) & 0xffu;
    const uint64_t vmask = __ballot(valid);
    const uint32_t d0 = (uint32_t)__builtin_amdgcn_readfirstlane((int)d);
    if (__ballot(valid && d == d0) == vmask) {
      if (__lane_id() == 0 && vmask) atomicAdd(&hw[w][d0], (uint32_t)__popcll(vmask));
    } else if (valid) {
      atomicAdd(&hw[w][d], 1u);
    }
  }
  __syncthreads();
  uint32_t t = 0;
  for (int i = 0; i < kWaves; ++i) t += hw[i][threadIdx.x];
  hist[(size_t)blockIdx.x * kRadix + threadIdx.x] = t;
}

// The histogram table is block-major, hist[b * 256 + d].  Its scan, per digit d
// the count of items with a smaller digit plus those of digit d in earlier blocks,
// runs over chunks of blocks (at most kMaxChunks chunks) and is left in three
// parts that the scatter adds (DigitStarts): the running sum within each chunk (in
// place in the table) with the chunk's column sums, then one workgroup turning the
// chunk sums into prefixes over chunks and scanning the digit totals.
// Every pass reads rows of 256 counters (coalesced).
constexpr int kScanChunk = 16;                               // smallest chunk, and the load batch
constexpr int kMaxChunks = 128;                              // chunks grow so there are at most this many
constexpr int kChunkScanThreads = 1024;                       // k_radix_chunk_scan: 4 threads per digit
constexpr int kChunkParts = kChunkScanThreads / kRadix;

// Blocks per chunk for n_blocks blocks: a multiple of kScanChunk, at least kScanChunk.
__host__ __device__ inline int chunk_blocks(int n_blocks) {
  int cs = (n_blocks + kMaxChunks - 1) / kMaxChunks;
  cs = (cs + kScanChunk - 1) / kScanChunk * kScanChunk;
  return cs < kScanChunk ? kScanChunk : cs;
}

// Shape of one pass's digit table for n items: blocks, blocks per chunk, chunks
// (at most kMaxChunks, and at most ceil(blocks / kScanChunk)).  The kernels derive
// it from the item count they read, so a grid sized for a capacity costs only its
// empty workgroups.
struct SortGeo {
  int nb, cs, nch;
};
__host__ __device__ inline SortGeo sort_geo(size_t n) {
  SortGeo g;
  g.nb = (int)((n + kSortTileItems - 1) / kSortTileItems);
  g.cs = chunk_blocks(g.nb);
  g.nch = (g.nb + g.cs - 1) / g.cs;
  return g;
}

// Chunk rows a table for up to nb_cap blocks may need.
inline int max_chunks(int nb_cap) {
  const int c = (nb_cap + kScanChunk - 1) / kScanChunk;
  return c < kMaxChunks ? c : kMaxChunks;
}

// hist[b][d] <- digit d's count over the blocks of b's chunk before b;
// chunk_sum[c][d] <- its count over the whole chunk c.
__global__ __launch_bounds__(kRadix) void k_radix_chunk_sums(uint32_t* __restrict__ hist, size_t n_cap,
                                                              const unsigned long long* __restrict__ n_dev,
                                                              uint32_t* __restrict__ chunk_sum) {
  const SortGeo sg = sort_geo(item_count(n_cap, n_dev));
  if ((int)blockIdx.x >= sg.nch) return;
  const int cs = sg.cs;
  const int b0 = blockIdx.x * cs, b1 = min(b0 + cs, sg.nb);
  uint32_t run = 0;
  for (int b = b0; b < b1; b += kScanChunk) {
    uint32_t x[kScanChunk];
#pragma unroll
    for (int k = 0; k < kScanChunk; ++k)   // a batch of loads in flight before the stores
      x[k] = b + k < b1 ? hist[(size_t)(b + k) * kRadix + threadIdx.x] : 0u;
#pragma unroll
    for (int k = 0; k < kScanChunk; ++k) {
      if (b + k < b1) hist[(size_t)(b + k) * kRadix + threadIdx.x] = run;
      run += x[k];
    }
  }
  chunk_sum[(size_t)blockIdx.x * kRadix + threadIdx.x] = run;
}

// One workgroup, kChunkParts threads per digit d, each owning a contiguous part of
// the chunks: exclusive prefix of the chunk sums over chunks (part sums combined
// through LDS), then the exclusive scan of the digit totals over digits, stored in
// digit_base.
__global__ __launch_bounds__(kChunkScanThreads) void k_radix_chunk_scan(uint32_t* __restrict__ chunk_sum,
                                                                         size_t n_cap,
                                                                         const unsigned long long* __restrict__ n_dev,
                                                                         uint32_t* __restrict__ digit_base) {
  __shared__ uint32_t part[kChunkParts][kRadix];
  __shared__ uint32_t wsum[kRadix / 64];
  const int n_chunks = sort_geo(item_count(n_cap, n_dev)).nch;
  const int d = threadIdx.x % kRadix, pi = threadIdx.x / kRadix;
  const int per = (n_chunks + kChunkParts - 1) / kChunkParts;
  const int c0 = pi * per, c1 = min(c0 + per, n_chunks);
  uint32_t run = 0;
  for (int c = c0; c < c1; c += 8) {   // eight loads in flight per step
    uint32_t x[8];
#pragma unroll
    for (int k = 0; k < 8; ++k) x[k] = c + k < c1 ? chunk_sum[(size_t)(c + k) * kRadix + d] : 0u;
#pragma unroll
    for (int k = 0; k < 8; ++k) run += x[k];
  }
  part[pi][d] = run;
  __syncthreads();
  uint32_t pre = 0, tot = 0;
  for (int j = 0; j < kChunkParts; ++j) {
    const uint32_t v = part[j][d];
    pre += j < pi ? v : 0u;
    tot += v;
  }
  run = pre;
  for (int c = c0; c < c1; c += 8) {
    uint32_t x[8];
#pragma unroll
    for (int k = 0; k < 8; ++k) x[k] = c + k < c1 ? chunk_sum[(size_t)(c + k) * kRadix + d] : 0u;
#pragma unroll
    for (int k = 0; k < 8; ++k) {
      if (c + k < c1) chunk_sum[(size_t)(c + k) * kRadix + d] = run;
      run += x[k];
    }
  }
  if (pi == 0) {   // the first kRadix threads: exclusive scan of the digit totals
    const uint32_t incl = wave_incl_scan(tot);
    if (__lane_id() == 63) wsum[d / 64] = incl;
  }
  __syncthreads();
  if (pi == 0) {
    const uint32_t incl = wave_incl_scan(tot);
    uint32_t wpre = 0;
    for (int w = 0; w < d / 64; ++w) wpre += wsum[w];
    digit_base[d] = wpre + incl - tot;
  }
}

// Start of block b's run of digit d in a pass's output: the three parts the scan
// leaves, added by the scatter.
struct DigitStarts {
  const uint32_t* in_chunk;     // [b][d]: over the earlier blocks of b's chunk
  const uint32_t* chunk_pre;    // [c][d]: over the earlier chunks
  const uint32_t* digit_base;   // [d]: items with a smaller digit
};

// Stable scatter of one digit pass.  Items are ranked in workgroup order (wave w
// owns items [base + 1024 w, base + 1024 (w + 1)), then round, then lane): within a
// wave from ballot peer masks and the wave's running digit counters (no barrier per
// round), across waves from the counters' prefix.  The workgroup then places its
// items in LDS in digit order and writes each digit's run contiguously.
//
// Two-pass sorts of keys below 2^16 with values below 2^24 move one word per item
// between the passes: the first pass (kScatterPack, digit = key bits 0-7) writes
// (key >> 8) << 24 | value to keys_out only; the second (kScatterUnpack, digit =
// word bits 24-31, i.e. key bits 8-15) reads those words and restores the key's low
// byte from the item's position, its input being ordered by that byte: position i
// holds the largest d with low_base[d] <= i, low_base being the first pass's digit
// starts.
// The first pass of a depth sort (kScatterIota) reads its keys from the caller's
// array and forms the values itself: the entry index, with vals_in (per-entry pair
// counts) given also min(count, 255) << 24.
constexpr int kScatterPlain = 0, kScatterPack = 1, kScatterUnpack = 2, kScatterIota = 3;

// Largest d in [0, 256) with base[d] <= i (base nondecreasing, base[0] = 0).
__device__ inline uint32_t digit_at(const uint32_t* base, uint32_t i) {
  uint32_t lo = 0;
#pragma unroll
  for (uint32_t step = kRadix / 2; step > 0; step >>= 1)
    if (base[lo + step] <= i) lo += step;
  return lo;
}

// The scatter runs 512 threads (8 items each) on the same 4096-item tiles as the
// histogram: half the registers per thread of a 256-thread tile, so twice the
// wavefronts in flight.
constexpr int kScatterThreads = 512;
constexpr int kScatterWaves = kScatterThreads / 64;
constexpr int kScatterItems = kSortTileItems / kScatterThreads;

template <int MODE>
__global__ __launch_bounds__(kScatterThreads) void k_radix_scatter(const uint32_t* __restrict__ keys_in,
                                                                    const uint32_t* __restrict__ vals_in, size_t n_cap,
                                                                    const unsigned long long* __restrict__ n_dev,
                                                                    int shift, const DigitStarts starts,
                                                                    const uint32_t* __restrict__ low_base,
                                                                    uint32_t* __restrict__ keys_out,
                                                                    uint32_t* __restrict__ vals_out) {
  __shared__ uint32_t s_keys[kSortTileItems];
  __shared__ uint32_t s_vals[MODE == kScatterPack ? 1 : kSortTileItems];
  __shared__ uint8_t s_dig[MODE == kScatterPack ? kSortTileItems : 1];   // packed words lose the digit
  __shared__ uint32_t s_low[MODE == kScatterUnpack ? kRadix : 1];
  __shared__ uint32_t s_lowblk[2];
  __shared__ uint32_t wc[kScatterWaves][kRadix];   // per-wave running digit counts
  __shared__ uint32_t lstart[kRadix];              // workgroup-local start of each digit
  __shared__ uint32_t goff[kRadix];                // global start of this workgroup's run of each digit
  __shared__ uint32_t wsum[kRadix / 64];
  // Workgroups are dealt to the 8 XCDs round-robin; XCD x takes the contiguous
  // eighth x of the tiles, so each digit's output run of an eighth is written
  // through one L2 (the lines shared by neighbouring tiles' runs merge there instead
  // of reaching HBM as partial writes from two XCDs).  Grid: 8 x ceil(tiles / 8)
  // for the capacity; the eighths are those of the actual item count.
  const size_t n = item_count(n_cap, n_dev);
  const int n_tiles_sort = (int)((n + kSortTileItems - 1) / kSortTileItems);
  const int eighth = (n_tiles_sort + 7) / 8;
  if ((int)(blockIdx.x / 8) >= eighth) return;
  const int blk = (int)(blockIdx.x % 8) * eighth + (int)(blockIdx.x / 8);
  if (blk >= n_tiles_sort) return;
  const int tid = threadIdx.x;
  const int wave = tid / 64;
  const bool digit_thread = tid < kRadix;          // threads 0-255 own one digit each
  for (int i = tid; i < kScatterWaves * kRadix; i += kScatterThreads) (&wc[0][0])[i] = 0;
  if (digit_thread)
    goff[tid] = starts.in_chunk[(size_t)blk * kRadix + tid] +
                starts.chunk_pre[(size_t)(blk / sort_geo(n).cs) * kRadix + tid] + starts.digit_base[tid];
  const size_t blk0 = (size_t)blk * kSortTileItems;
  const size_t valid_items = n > blk0 ? (n - blk0 < (size_t)kSortTileItems ? n - blk0 : (size_t)kSortTileItems) : 0;
  if (MODE == kScatterUnpack) {
    if (digit_thread) s_low[tid] = low_base[tid];
    __syncthreads();
    // low bytes of the workgroup's first and last items (equal unless the
    // workgroup straddles a digit boundary)
    if (tid < 2 && valid_items > 0) s_lowblk[tid] = digit_at(s_low, (uint32_t)(blk0 + (tid ? valid_items - 1 : 0)));
  }
  __syncthreads();

  const size_t base = blk0 + (size_t)wave * (kScatterItems * 64) + __lane_id();
  uint32_t k[kScatterItems], v[kScatterItems], rank[kScatterItems];
#pragma unroll
  for (int r = 0; r < kScatterItems; ++r) {   // all loads in flight before any ranking
    const size_t i = base + (size_t)r * 64;
    k[r] = i < n ? keys_in[i] : 0xffffffffu;
    if (MODE == kScatterIota) {
      const uint32_t c = vals_in && i < n ? vals_in[i] : 0u;
      v[r] = (uint32_t)i | (vals_in ? (c < kPackSat ? c : kPackSat) << kPackShift : 0u);
    } else if (MODE != kScatterUnpack) {
      v[r] = i < n ? vals_in[i] : 0u;
    }
  }
  if (MODE == kScatterUnpack) {
    const uint32_t l0 = s_lowblk[0], l1 = s_lowblk[1];
#pragma unroll
    for (int r = 0; r < kScatterItems; ++r) {
      const size_t i = base + (size_t)r * 64;
      if (i < n) {
        const uint32_t low = l0 == l1 ? l0 : digit_at(s_low, (uint32_t)i);
        v[r] = k[r] & 0x00ffffffu;
        k[r] = ((k[r] >> 24) << 8) | low;
      } else {
        v[r] = 0u;
      }
    }
  }
  const uint64_t lt = lanemask_lt();
#pragma unroll
  for (int r = 0; r < kScatterItems; ++r) {
    const bool valid = base + (size_t)r * 64 < n;
    const uint32_t d = (k[r] >> shift) & 0xffu;
    const uint64_t peers = match_digit(d, valid);
    rank[r] = wc[wave][d] + (uint32_t)__popcll(peers & lt);
    if (valid && (peers & lt) == 0) wc[wave][d] += (uint32_t)__popcll(peers);
    __builtin_amdgcn_wave_barrier();   // the leaders' updates precede the next round's reads
  }
  __syncthreads();
  // per digit (threads 0-255, whole wavefronts): totals over waves (into wc[.][d] as
  // exclusive wave prefixes) and the exclusive scan over digits of the totals
  uint32_t tot = 0, incl = 0;
  if (digit_thread) {
    for (int w = 0; w < kScatterWaves; ++w) {
      const uint32_t c = wc[w][tid];
      wc[w][tid] = tot;
      tot += c;
    }
    incl = wave_incl_scan(tot);
    if (__lane_id() == 63) wsum[wave] = incl;
  }
  __syncthreads();
  if (digit_thread) {
    uint32_t wpre = 0;
    for (int w = 0; w < wave; ++w) wpre += wsum[w];
    lstart[tid] = wpre + incl - tot;
  }
  __syncthreads();
#pragma unroll
  for (int r = 0; r < kScatterItems; ++r) {
    if (base + (size_t)r * 64 < n) {
      const uint32_t d = (k[r] >> shift) & 0xffu;
      const uint32_t pos = lstart[d] + wc[wave][d] + rank[r];
      if (MODE == kScatterPack) {
        s_keys[pos] = ((k[r] >> 8) << 24) | v[r];
        s_dig[pos] = (uint8_t)d;
      } else {
        s_keys[pos] = k[r];
        s_vals[pos] = v[r];
      }
    }
  }
  __syncthreads();
  for (uint32_t p = tid; p < valid_items; p += kScatterThreads) {
    const uint32_t key = s_keys[p];
    const uint32_t d = MODE == kScatterPack ? (uint32_t)s_dig[p] : (key >> shift) & 0xffu;
    const size_t dst = (size_t)goff[d] + (p - lstart[d]);
    if (dst < n) {   // always true for a consistent histogram; guards the write
      keys_out[dst] = key;
      if (MODE != kScatterPack) vals_out[dst] = s_vals[p];
    }
  }
}

// ---- exclusive scan of touched[order[e]] ----
constexpr int kScanItems = 4096;

__device__ inline uint32_t block_sum_u32(uint32_t x, uint32_t* sh) {
  for (int off = 32; off > 0; off >>= 1) x += __shfl_xor(x, off);
  if (__lane_id() == 0) sh[threadIdx.x / 64] = x;
  __syncthreads();
  uint32_t t = 0;
  for (int w = 0; w < kWaves; ++w) t += sh[w];
  __syncthreads();
  return t;
}

// Count of depth-ordered entry e: touched[order[e]].  With packed != 0 the order
// entries carry min(count, 255) in their top byte (see radix_sort_depth) and only the
// saturated ones gather their count.
__device__ inline uint32_t entry_count(uint32_t o, int packed, const uint32_t* __restrict__ touched) {
  if (!packed) return touched[o];
  const uint32_t c = o >> kPackShift;
  return c == kPackSat ? touched[o & kPackRidMask] : c;
}

// Sums of the counts of every 64 consecutive depth-ordered entries (group_sums,
// one per wave of the emission) and of every kScanItems entries (block_sums).
// Thread t takes 16 consecutive entries (four 16-byte loads), four lanes a group.
__global__ __launch_bounds__(kThreads) void k_scan_reduce(const uint32_t* __restrict__ order,
                                                           const uint32_t* __restrict__ touched, size_t n,
                                                           int packed, uint32_t* __restrict__ group_sums,
                                                           uint32_t* __restrict__ block_sums) {
  static_assert(kScanItems == 16 * kThreads, "16 entries per thread");
  __shared__ uint32_t sh[kWaves];
  const size_t e0 = (size_t)blockIdx.x * kScanItems + 16 * (size_t)threadIdx.x;
  uint32_t c = 0;
  if (e0 + 16 <= n) {
    const uint4* o4 = reinterpret_cast<const uint4*>(order + e0);
    uint4 q[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) q[k] = o4[k];
#pragma unroll
    for (int k = 0; k < 4; ++k)
      c += entry_count(q[k].x, packed, touched) + entry_count(q[k].y, packed, touched) +
           entry_count(q[k].z, packed, touched) + entry_count(q[k].w, packed, touched);
  } else {
    for (size_t i = e0; i < n && i < e0 + 16; ++i) c += entry_count(order[i], packed, touched);
  }
  c += __shfl_xor(c, 1);
  c += __shfl_xor(c, 2);
  const bool lead = (threadIdx.x & 3u) == 0u;
  if (lead && e0 < n) group_sums[e0 / 64] = c;
  const uint32_t t = block_sum_u32(lead ? c : 0u, sh);
  if (threadIdx.x == 0) block_sums[blockIdx.x] = t;
}

// single workgroup: exclusive scan of block sums in 64-bit, total to *total
// Besides the scan: the binning's capacity check on the total K (thread 0, once
// every block sum is in), which also copies the status into the host-visible
// mirror; the host reads it once the stream has passed this point (see
// check_pairs).
__device__ inline void check_pairs(DevStatus* __restrict__ st, DevStatus* __restrict__ mirror,
                                   unsigned long long K, unsigned long long cap) {
  st->n_pairs = K;
  if (K > cap || K >= (1ull << 32)) {
    st->n_eff = 0ull;
    st->need_pairs = K;
    status_fail(st, GS_ERR_CAPACITY);
  } else {
    // an earlier failure (the exact pass's outcome store too small) leaves counts
    // the emission could not reproduce: then no pair is emitted either
    st->n_eff = st->code == GS_OK ? K : 0ull;
  }
  mirror->n_pairs = K;
  mirror->n_eff = st->n_eff;
  mirror->need_pairs = st->need_pairs;
  mirror->redo_count = st->redo_count;
  mirror->redo_words = st->redo_words;
  mirror->need_redo = st->need_redo;
  mirror->pad = 0u;
  __threadfence_system();
  mirror->code = st->code;
}

__global__ __launch_bounds__(1024) void k_scan_blocks(uint32_t* __restrict__ block_sums, int nb,
                                                       DevStatus* __restrict__ st, DevStatus* __restrict__ mirror,
                                                       unsigned long long cap) {
  __shared__ unsigned long long wsum[16];
  __shared__ unsigned long long carry;
  if (threadIdx.x == 0) carry = 0;
  __syncthreads();
  for (int b0 = 0; b0 < nb; b0 += 1024) {
    const int b = b0 + threadIdx.x;
    const unsigned long long x = b < nb ? block_sums[b] : 0ull;
    unsigned long long incl = x;
    for (int off = 1; off < 64; off <<= 1) {
      const unsigned long long y = __shfl_up(incl, off);
      if ((int)__lane_id() >= off) incl += y;
    }
    if (__lane_id() == 63) wsum[threadIdx.x / 64] = incl;
    __syncthreads();
    unsigned long long wpre = 0;
    for (int w = 0; w < (int)(threadIdx.x / 64); ++w) wpre += wsum[w];
    const unsigned long long c = carry;
    if (b < nb) block_sums[b] = (uint32_t)(c + wpre + incl - x);   // offsets < 2^32 checked on the host
    __syncthreads();
    if (threadIdx.x == 1023) carry = c + wpre + incl;
    __syncthreads();
  }
  if (threadIdx.x == 0) check_pairs(st, mirror, carry, cap);
}

// Inclusive max over lanes 0..l (DPP: shifts within rows of 16 lanes, then the
// last lane of a row broadcast into the rows after it).  INT_MIN, the identity,
// as the value of lanes with no source lets each step be one DPP max (lanes
// without a source keep their value).
__device__ inline int wave_incl_max(int v) {
  v = max(v, __builtin_amdgcn_update_dpp(INT_MIN, v, 0x111, 0xf, 0xf, false));   // row_shr:1
  v = max(v, __builtin_amdgcn_update_dpp(INT_MIN, v, 0x112, 0xf, 0xf, false));   // row_shr:2
  v = max(v, __builtin_amdgcn_update_dpp(INT_MIN, v, 0x114, 0xf, 0xf, false));   // row_shr:4
  v = max(v, __builtin_amdgcn_update_dpp(INT_MIN, v, 0x118, 0xf, 0xf, false));   // row_shr:8
  v = max(v, __builtin_amdgcn_update_dpp(INT_MIN, v, 0x142, 0xa, 0xf, false));   // row_bcast:15 into rows 1, 3
  v = max(v, __builtin_amdgcn_update_dpp(INT_MIN, v, 0x143, 0xc, 0xf, false));   // row_bcast:31 into rows 2, 3
  return v;
}

// Cooperative walk over the candidate pairs of 64 consecutive entries, one wave:
// entry l of the wave (lane l) has cand candidates (the tiles of its rect,
// row-major) starting at the wave-exclusive prefix excl; a round covers the
// candidates [cb, cb + 64), candidate cb + k on lane k.  Returns the entry that
// owns this lane's candidate: each entry starting inside the round marks its start
// in the wave's 64-slot scratch `own`, and a lane takes the last mark at or before
// it (`carry`, the owner of the previous round's last candidate, when the round
// opens inside an entry).  Lanes past the last candidate get a meaningless value.
__device__ inline int round_owner(uint32_t excl, uint32_t cand, uint32_t cb, int* own, int carry) {
  const unsigned lane = __lane_id();
  own[lane] = -1;
  __builtin_amdgcn_wave_barrier();
  if (cand != 0u && excl >= cb && excl - cb < 64u) own[excl - cb] = (int)lane;
  __builtin_amdgcn_wave_barrier();
  const int mark = own[lane];
  __builtin_amdgcn_wave_barrier();
  const int o = wave_incl_max(lane == 0u && mark < 0 ? carry : mark);
  return o < 0 ? 0 : o;   // only lanes past the last candidate could see no mark
}

// (tile column, row) offsets of candidate `local` in a rect nx tiles wide: the
// quotient from the hardware reciprocal (within one of the true one for the
// counts here, below 2^24), then corrected.
__device__ inline void rect_cell(uint32_t local, uint32_t nx, uint32_t& tx, uint32_t& ty) {
  ty = (uint32_t)((float)local * __builtin_amdgcn_rcpf((float)nx));
  if (ty * nx > local) --ty;
  else if ((ty + 1) * nx <= local) ++ty;
  tx = local - ty * nx;
}


// Wave-wide counter update: lane 0 adds `total` to *ctr; every lane gets the old
// value (0 and no update when total is 0).
__device__ inline unsigned long long wave_take(unsigned long long* ctr, uint32_t total) {
  unsigned long long o = 0ull;
  if (total != 0u && __lane_id() == 0u) o = atomicAdd(ctr, (unsigned long long)total);
  return (unsigned long long)__shfl((long long)o, 0);
}

// The split rule of a heavy wave (more than kSplitWave candidates): the largest
// threshold t (64 doubled up to 8192) that leaves at most kSplitWave candidates
// to the entries of at most t; the entries above it go to the chunk pass.  (64 if
// none does: entries of at most 64 candidates always stay with their wave.)
__device__ inline uint32_t split_threshold(uint32_t cand) {
  for (uint32_t t = 8192u; t > 64u; t >>= 1) {
    const uint32_t rem = (uint32_t)__builtin_amdgcn_readlane((int)wave_incl_scan(cand <= t ? cand : 0u), 63);
    if (rem <= kSplitWave) return t;
  }
  return 64u;
}

// Kept pairs per entry (index order, coalesced reads): the tiles of the entry's
// rect whose pixel-centre box meets its cutoff region.  The wave's candidates are
// spread over its lanes; runs of one entry within 64 candidates are counted with
// ballots by the run's first lane.  Each entry also gets a 16-byte EmitInfo: its
// rect and, when it has at most 64 candidates, the outcome of every test (bit i
// for the rect's i-th tile, row-major), which is all emission then has to fetch.
constexpr uint32_t kRedoMark = 1u << 31;

__global__ __launch_bounds__(kThreads) void k_count_kept(const uint32_t* __restrict__ touched,
                                                          const ushort4* __restrict__ rect,
                                                          const Record* __restrict__ rec, size_t n_entries, int n,
                                                          const ViewDev* __restrict__ views, int T, int exact_all,
                                                          uint32_t* __restrict__ kept,
                                                          EmitInfo* __restrict__ info, DevStatus* __restrict__ st,
                                                          uint32_t* __restrict__ redo_list,
                                                          uint2* __restrict__ items, size_t icap) {
  __shared__ uint32_t s_cp[kWaves][65];
  __shared__ uint32_t s_nx[kWaves][64];
  __shared__ uint32_t s_org[kWaves][64];    // rect origin (tx0 | ty0 << 16)
  __shared__ uint32_t s_wh[kWaves][64];     // view size (W | H << 16)
  __shared__ uint32_t s_k[kWaves][64];
  __shared__ uint64_t s_bits[kWaves][64];
  __shared__ int s_own[kWaves][64];
  __shared__ CutoffGeoF s_geo[kWaves][64];    // fp32 clear-case geometry
  const int w = threadIdx.x / 64;
  const unsigned lane = __lane_id();
  const size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  const uint32_t touched_e = e < n_entries ? touched[e] : 0u;
  uint32_t cand = touched_e;
  uint32_t incl = wave_incl_scan(cand);
  // a heavy wave hands its large entries to k_count_chunks (their kept[e] is
  // written as 0 below; the chunks add to it)
  if (!exact_all && (uint32_t)__builtin_amdgcn_readlane((int)incl, 63) > kSplitWave) {
    const uint32_t t = split_threshold(cand);   // (a wave-wide step: every lane takes it)
    // the wave's items are taken with one counter update
    const uint32_t nch = cand > t ? (cand + kChunk - 1u) / kChunk : 0u;
    const uint32_t nincl = wave_incl_scan(nch);
    const int list = (int)((blockIdx.x * kWaves + w) % kSplitLists);
    const unsigned long long i0 =
        wave_take(split_ctr(st, kSplitCountItems, list), (uint32_t)__builtin_amdgcn_readlane((int)nincl, 63)) +
        (nincl - nch);
    bool split = false;
    if (nch) {
      uint2* li = items + (size_t)list * icap;
      split = i0 + nch <= icap;
      for (uint32_t c = 0; c < nch && i0 + c < icap; ++c)
        li[i0 + c] = split ? make_uint2((uint32_t)e, c * kChunk) : make_uint2(~0u, 0u);
    }
    if (__ballot(split)) {
      cand = split ? 0u : cand;
      incl = wave_incl_scan(cand);
    }
  }
  const ushort4 rc = touched_e ? rect[e] : make_ushort4(0, 0, 0, 0);
  s_cp[w][lane + 1] = incl;
  if (lane == 0) s_cp[w][0] = 0u;
  s_k[w][lane] = 0u;
  s_bits[w][lane] = 0ull;
  if (cand) {
    const ViewDev& cv = views[e / (size_t)n];
    s_nx[w][lane] = (uint32_t)(rc.y - rc.x + 1);
    s_org[w][lane] = (uint32_t)rc.x | ((uint32_t)rc.z << 16);
    s_wh[w][lane] = (uint32_t)cv.W | ((uint32_t)cv.H << 16);
    s_geo[w][lane] = cutoff_geo_f(rec[e]);
  }
  __builtin_amdgcn_wave_barrier();
  const uint32_t C = s_cp[w][64];
  int carry = 0;
  for (uint32_t cb = 0; cb < C; cb += 64) {
    const uint32_t q = cb + lane;
    const bool valid = q < C;
    const int owner = round_owner(incl - cand, cand, cb, s_own[w], carry);
    carry = __builtin_amdgcn_readlane(owner, 63);
    int lo = 0;
    bool pass = false, first = false, undecided = false;
    if (valid) {
      lo = owner;
      const uint32_t li = q - s_cp[w][lo];
      first = lane == 0 || li == 0u;          // this lane opens its entry's run in the round
      uint32_t tx, ty;
      rect_cell(li, s_nx[w][lo], tx, ty);
      const uint32_t org = s_org[w][lo], wh = s_wh[w][lo];
      const int gx = (int)((org & 0xffffu) + tx), gy = (int)((org >> 16) + ty);
      const int W = (int)(wh & 0xffffu), H = (int)(wh >> 16);
      const int fast = exact_all ? -1 : tile_cutoff_fast(s_geo[w][lo], gx, gy, T, W, H);
      pass = fast > 0;
      undecided = fast < 0;   // decided by the exact pass
    }
    const uint64_t fmask = __ballot(first);
    const uint64_t pmask = __ballot(pass);
    const uint64_t umask = __ballot(undecided);
    if (first) {
      const uint64_t above = lane == 63 ? 0ull : (fmask & (~0ull << (lane + 1)));
      const unsigned next = above ? (unsigned)__builtin_ctzll(above) : 64u;
      const uint64_t run = (next == 64u ? ~0ull : ((1ull << next) - 1ull)) & (~0ull << lane);
      // the top bit flags an entry with an undecided candidate (counts stay below 2^31)
      s_k[w][lo] = (s_k[w][lo] + (uint32_t)__popcll(pmask & run)) | ((umask & run) ? kRedoMark : 0u);
      if (s_cp[w][lo + 1] - s_cp[w][lo] <= 64u)   // the run's outcomes at their rect positions
        s_bits[w][lo] |= ((pmask & run) >> lane) << (q - s_cp[w][lo]);
    }
    __builtin_amdgcn_wave_barrier();
  }
  if (e < n_entries) {
    const uint32_t k = s_k[w][lane];
    kept[e] = k & ~kRedoMark;
    EmitInfo in;
    in.rect = rc;
    in.bits = s_bits[w][lane];
    info[e] = in;
    if (k & kRedoMark) redo_list[atomicAdd(&st->redo_count, 1ull)] = (uint32_t)e;
  }
}

// Kept counts of the entries k_count_kept split into chunk items, one wave per
// item (kChunk candidates): the fp32 test as in k_count_kept, the item's passes
// added to kept[e]; an undecided candidate marks kept[e] (top bit) and the first
// chunk to mark it lists the entry for the exact pass, which rewrites its count.
__global__ __launch_bounds__(kThreads) void k_count_chunks(const ushort4* __restrict__ rect,
                                                            const Record* __restrict__ rec, int n,
                                                            const ViewDev* __restrict__ views, int T,
                                                            uint32_t* __restrict__ kept, DevStatus* __restrict__ st,
                                                            uint32_t* __restrict__ redo_list,
                                                            const uint2* __restrict__ items, size_t icap) {
  const unsigned lane = __lane_id();
  // the waves are dealt out over the lists: wave v walks list v % kSplitLists
  const size_t v = (size_t)blockIdx.x * (blockDim.x / 64) + threadIdx.x / 64;
  const int list = (int)(v % kSplitLists);
  const unsigned long long listed = *split_ctr(st, kSplitCountItems, list);
  const size_t cnt = listed < icap ? (size_t)listed : icap;
  const size_t step = (size_t)gridDim.x * (blockDim.x / 64) / kSplitLists;
  const uint2* li = items + (size_t)list * icap;
  for (size_t i = v / kSplitLists; i < cnt; i += step) {
    const uint2 it = li[i];
    if (it.x == ~0u) continue;
    const uint32_t e = it.x;
    const ushort4 rc = rect[e];
    const ViewDev& cv = views[e / (uint32_t)n];
    const CutoffGeoF geo = cutoff_geo_f(rec[e]);
    const uint32_t nx = (uint32_t)(rc.y - rc.x + 1), C = nx * (uint32_t)(rc.w - rc.z + 1);
    const uint32_t c1 = it.y + kChunk < C ? it.y + kChunk : C;
    uint32_t k = 0;
    bool undecided = false;
    for (uint32_t cb = it.y; cb < c1; cb += 64u) {
      const uint32_t li = cb + lane;
      int f = 0;
      if (li < c1) {
        uint32_t tx, ty;
        rect_cell(li, nx, tx, ty);
        f = tile_cutoff_fast(geo, (int)(rc.x + tx), (int)(rc.z + ty), T, cv.W, cv.H);
      }
      k += (uint32_t)__popcll(__ballot(f > 0));
      undecided |= __ballot(f < 0) != 0ull;
    }
    if (lane == 0) {
      if (k) atomicAdd(&kept[e], k);
      if (undecided && !(atomicOr(&kept[e], kRedoMark) & kRedoMark))
        redo_list[atomicAdd(&st->redo_count, 1ull)] = e;
    }
  }
}

// The exact pass over the entries k_count_kept listed, one wave per entry: the
// FP64 conic and cutoff are recomputed from the parameters (as the projection
// computed them) and every candidate the fp32 test cannot decide is decided by
// tile_meets_cutoff on them; the kept count and EmitInfo are rewritten.  Entries of
// more than 64 candidates keep their outcome bits in redo_bits (one bit per
// candidate, 32 per word, from an offset handed out by an atomic counter).
__global__ __launch_bounds__(kThreads) void k_count_redo(const uint32_t* __restrict__ touched,
                                                          const ushort4* __restrict__ rect,
                                                          const Record* __restrict__ rec, int n,
                                                          const ViewDev* __restrict__ views, int T, int exact_all,
                                                          const float* __restrict__ P, int stride,
                                                          uint32_t* __restrict__ kept, EmitInfo* __restrict__ info,
                                                          DevStatus* __restrict__ st,
                                                          const uint32_t* __restrict__ redo_list,
                                                          uint32_t* __restrict__ redo_bits, size_t redo_cap) {
  const unsigned lane = __lane_id();
  const unsigned long long cnt = st->redo_count;
  const size_t waves = (size_t)gridDim.x * (blockDim.x / 64);
  for (size_t i = (size_t)blockIdx.x * (blockDim.x / 64) + threadIdx.x / 64; i < cnt; i += waves) {
    const uint32_t e = redo_list[i];
    const int v = (int)(e / (uint32_t)n);
    const int g = (int)(e - (uint32_t)v * (uint32_t)n);
    const ViewDev& cv = views[v];
    const CutoffGeo ex = exact_cutoff_geo(P, stride, g, cv);
    const CutoffGeoF fg = cutoff_geo_f(rec[e]);
    const ushort4 rc = rect[e];
    const uint32_t nx = (uint32_t)(rc.y - rc.x + 1), C = touched[e];
    const bool large = C > 64u;
    size_t off = 0;
    bool room = true;
    if (large) {
      const size_t words = (C + 31u) / 32u;
      unsigned long long o = 0;
      if (lane == 0) o = atomicAdd(&st->redo_words, (unsigned long long)words);
      off = (size_t)__shfl((long long)o, 0);
      if (off + words > redo_cap) {
        room = false;
        if (lane == 0) {
          atomicMax(&st->need_redo, (unsigned long long)(off + words));
          status_fail(st, GS_ERR_CAPACITY);
        }
      }
    }
    uint32_t k = 0;
    uint64_t bits = 0ull;
    for (uint32_t cb = 0; cb < C; cb += 64u) {
      const uint32_t li = cb + lane;
      bool keep = false;
      if (li < C) {
        const uint32_t ty = li / nx, tx = li - ty * nx;
        const int gx = (int)(rc.x + tx), gy = (int)(rc.z + ty);
        const int f = exact_all ? -1 : tile_cutoff_fast(fg, gx, gy, T, cv.W, cv.H);
        keep = f >= 0 ? f != 0 : tile_meets_cutoff(ex, gx, gy, T, cv.W, cv.H);
      }
      const uint64_t m = __ballot(keep);
      k += (uint32_t)__popcll(m);
      if (!large) {
        bits = m;
      } else if (room && lane < 2u && cb / 32u + lane < (C + 31u) / 32u) {
        redo_bits[off + cb / 32u + lane] = (uint32_t)(m >> (32u * lane));
      }
    }
    if (lane == 0) {
      kept[e] = k;
      EmitInfo in;
      in.rect = rc;
      in.bits = large ? (room ? kRedoFlag | (uint64_t)off : 0ull) : bits;
      info[e] = in;
    }
  }
}

__global__ void k_status_reset(DevStatus* __restrict__ st) {
  if (threadIdx.x == 0) status_clear(st);
  split_clear(st);
}


// Pair emission, one wave per 64 consecutive depth-ordered entries.  The wave's
// pairs occupy one contiguous output range.  Its candidates (rect tiles of its
// entries, entry by entry, row-major) are spread over the lanes in rounds of 64;
// with culling on, a candidate is kept only if its tile's pixel-centre box meets
// the cutoff region (k_count_kept's outcome bits for entries of at most 64
// candidates, the same test repeated for larger ones, so the kept counts and
// offsets agree), and kept candidates are written in order at running positions
// taken from a ballot: writes are coalesced and large rects are shared by the wave.
// With culling the entry's rect comes from its EmitInfo (one 16-byte fetch).  A
// heavy wave (more than kSplitWave candidates) hands its largest entries, with
// their output ranges, to k_emit_chunks and writes the others around those ranges.
constexpr int kEmitGeoSlots = 8;   // per wave: LDS for the geometry of its large entries

__global__ __launch_bounds__(kThreads) __attribute__((amdgpu_waves_per_eu(8))) void k_emit(const uint32_t* __restrict__ order, int packed,
                                                    const uint32_t* __restrict__ touched,
                                                    const uint32_t* __restrict__ group_sums,
                                                    const uint32_t* __restrict__ block_off,
                                                    const ushort4* __restrict__ rect,
                                                    const Record* __restrict__ rec, size_t n_entries, int n,
                                                    const ViewDev* __restrict__ views,
                                                    DevStatus* __restrict__ st, int cull, int T,
                                                    const EmitInfo* __restrict__ info,
                                                    const uint32_t* __restrict__ redo_bits,
                                                    SplitEntry* __restrict__ ents, size_t ecap,
                                                    uint2* __restrict__ items, size_t icap,
                                                    uint32_t* __restrict__ pair_tile,
                                                    uint32_t* __restrict__ pair_rec) {
  __shared__ uint32_t s_cp[kWaves][65];
  __shared__ uint32_t s_dpre[kWaves][64];   // pairs of the wave's split entries before each entry
  __shared__ uint32_t s_rid[kWaves][64];
  __shared__ uint32_t s_base[kWaves][64];   // global tile id of the rect's first tile
  __shared__ uint32_t s_nx[kWaves][64];     // rect width in tiles
  __shared__ uint32_t s_tx[kWaves][64];     // tiles per row of the entry's view
  __shared__ uint32_t s_org[kWaves][64];    // rect origin (tx0 | ty0 << 16)
  __shared__ uint32_t s_wh[kWaves][64];     // view size (W | H << 16)
  __shared__ uint64_t s_bits[kWaves][64];   // test outcomes (entries of <= 64 candidates)
  __shared__ int s_own[kWaves][64];         // round_owner scratch
  __shared__ int s_slot[kWaves][64];        // entry's s_geo slot (-1: none)
  __shared__ CutoffGeoF s_geo[kWaves][kEmitGeoSlots];
  const int w = threadIdx.x / 64;
  const unsigned lane = __lane_id();
  const size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  const bool valid = e < n_entries;
  uint32_t cnt = 0, rid = 0, cand = 0;
  uint64_t bits = 0ull;
  ushort4 rc = make_ushort4(0, 0, 0, 0);
  if (valid) {
    const uint32_t o = order[e];
    rid = packed ? o & kPackRidMask : o;
    cnt = packed ? o >> kPackShift : touched[rid];   // nonzero iff the entry has pairs
    if (cnt) {
      if (cull) {
        const EmitInfo in = info[rid];
        rc = in.rect;
        bits = in.bits;
      } else {
        rc = rect[rid];
      }
      cand = (uint32_t)(rc.y - rc.x + 1) * (uint32_t)(rc.w - rc.z + 1);
    }
  }
  uint32_t incl = wave_incl_scan(cand);
  const uint32_t C_all = (uint32_t)__builtin_amdgcn_readlane((int)incl, 63);
  if (C_all == 0u) return;
  // output range of the wave (group g of 64 entries, valid since it has
  // candidates): the start of its scan block plus the sums of the block's earlier
  // groups, then its own sum
  const size_t g = ((size_t)blockIdx.x * blockDim.x + (size_t)w * 64) / 64;
  const size_t gb = g & ~(size_t)(kScanItems / 64 - 1);
  uint32_t before = gb + lane < g ? group_sums[gb + lane] : 0u;
  for (int o = 32; o > 0; o >>= 1) before += (uint32_t)__shfl_xor((int)before, o);
  const uint32_t lo_off = block_off[g / (kScanItems / 64)] + before;
  const uint32_t hi_end = lo_off + group_sums[g];
  // the pair buffers hold st->n_eff pairs (0 when they are too small for this
  // binning: then nothing is written)
  const unsigned long long K = st->n_eff;
  if (hi_end > K || hi_end < lo_off) return;
  bool any_split = false;
  uint32_t dpre = 0;
  if (C_all > kSplitWave) {
    // exact pair counts of the entries (the packed count saturates) place the
    // split entries' ranges
    const uint32_t ck = cand ? (packed && cnt == kPackSat ? touched[rid] : cnt) : 0u;
    const uint32_t cincl = wave_incl_scan(ck);
    const uint32_t t = split_threshold(cand);   // (a wave-wide step: every lane takes it)
    // the wave's entries and items are taken with one update of each counter
    const uint32_t nch = cand > t ? (cand + kChunk - 1u) / kChunk : 0u;
    const uint64_t want = __ballot(nch != 0u);
    const uint32_t nincl = wave_incl_scan(nch);
    const int list = (int)(g % kSplitLists);
    const unsigned long long j = wave_take(split_ctr(st, kSplitEmitEnts, list), (uint32_t)__popcll(want)) +
                                 (uint32_t)__popcll(want & lanemask_lt());
    const unsigned long long i0 =
        wave_take(split_ctr(st, kSplitEmitItems, list), (uint32_t)__builtin_amdgcn_readlane((int)nincl, 63)) +
        (nincl - nch);
    bool split = false;
    if (nch) {
      split = j < ecap && i0 + nch <= icap;
      const uint32_t slot = (uint32_t)((size_t)list * ecap + (size_t)j);
      if (split) {
        SplitEntry se;
        se.rid = rid;
        se.base = lo_off + cincl - ck;
        se.ctr = 0u;
        se.pad = 0u;
        ents[slot] = se;
      }
      uint2* li = items + (size_t)list * icap;
      for (uint32_t c = 0; c < nch && i0 + c < icap; ++c)
        li[i0 + c] = split ? make_uint2(slot, c * kChunk) : make_uint2(~0u, 0u);
    }
    if (__ballot(split)) {
      any_split = true;
      const uint32_t sk = split ? ck : 0u;
      dpre = wave_incl_scan(sk) - sk;
      cand = split ? 0u : cand;
      incl = wave_incl_scan(cand);
    }
  }
  s_dpre[w][lane] = dpre;
  s_cp[w][lane + 1] = incl;
  if (lane == 0) s_cp[w][0] = 0u;
  s_rid[w][lane] = rid;
  // entries of more than 64 candidates repeat the cutoff test: the first
  // kEmitGeoSlots of the wave keep its geometry in LDS, any others re-derive it per
  // candidate from the record
  const bool large = cull && cand > 64u;
  const uint64_t large_mask = __ballot(large);
  const int slot = (int)__popcll(large_mask & lanemask_lt());
  s_slot[w][lane] = large && slot < kEmitGeoSlots ? slot : -1;
  if (cand) {
    const ViewDev& cv = views[rid / (uint32_t)n];
    s_base[w][lane] = (uint32_t)cv.tile_off + (uint32_t)rc.z * (uint32_t)cv.tiles_x + rc.x;
    s_nx[w][lane] = (uint32_t)(rc.y - rc.x + 1);
    s_tx[w][lane] = (uint32_t)cv.tiles_x;
    if (cull) {
      s_bits[w][lane] = bits;
      if (large) {
        s_org[w][lane] = (uint32_t)rc.x | ((uint32_t)rc.z << 16);
        s_wh[w][lane] = (uint32_t)cv.W | ((uint32_t)cv.H << 16);
        if (slot < kEmitGeoSlots) s_geo[w][slot] = cutoff_geo_f(rec[rid]);
      }
    }
  }
  __builtin_amdgcn_wave_barrier();
  const uint32_t C = s_cp[w][64];
  if (C == 0u) return;
  uint32_t pos = lo_off;   // the next pair of the entries the wave writes itself
  int carry = 0;
  for (uint32_t cb = 0; cb < C; cb += 64) {
    const uint32_t q = cb + lane;
    bool keep = false;
    uint32_t tile = 0, r = 0;
    const int owner = round_owner(incl - cand, cand, cb, s_own[w], carry);
    carry = __builtin_amdgcn_readlane(owner, 63);
    if (q < C) {
      const int lo = owner;
      uint32_t tx, ty;
      rect_cell(q - s_cp[w][lo], s_nx[w][lo], tx, ty);
      tile = s_base[w][lo] + ty * s_tx[w][lo] + tx;
      r = s_rid[w][lo];
      keep = true;
      if (cull) {
        const uint32_t li = q - s_cp[w][lo];
        if (s_cp[w][lo + 1] - s_cp[w][lo] <= 64u) {
          keep = ((s_bits[w][lo] >> li) & 1ull) != 0ull;
        } else {
          const uint32_t org = s_org[w][lo], wh = s_wh[w][lo];
          const int sl = s_slot[w][lo];
          const uint64_t ib = s_bits[w][lo];
          if (ib & kRedoFlag) {
            // outcomes stored by the exact pass
            keep = ((redo_bits[(size_t)(ib & ~kRedoFlag) + li / 32u] >> (li & 31u)) & 1u) != 0u;
          } else {
            // the fp32 test decided every candidate of this entry in the count (else
            // the exact pass would have stored its outcomes, or reported a full
            // outcome array), and decides them the same way here
            const CutoffGeoF geo = sl >= 0 ? s_geo[w][sl] : cutoff_geo_f(rec[r]);
            keep = tile_cutoff_fast(geo, (int)((org & 0xffffu) + tx), (int)((org >> 16) + ty), T,
                                    (int)(wh & 0xffffu), (int)(wh >> 16)) > 0;
          }
        }
      }
    }
    const uint64_t kmask = __ballot(keep);
    if (keep) {
      const uint32_t dst = pos + (any_split ? s_dpre[w][owner] : 0u) + (uint32_t)__popcll(kmask & lanemask_lt());
      if (dst < hi_end) {
        pair_tile[dst] = tile;
        pair_rec[dst] = r;
      }
    }
    pos += (uint32_t)__popcll(kmask);
  }
}

// Pairs of the entries k_emit split into chunk items, one wave per item (kChunk
// candidates): the same test as k_emit's for entries of more than 64 candidates;
// the item takes its slots in the entry's range with one counter update, then
// writes its kept pairs there in candidate order.
__global__ __launch_bounds__(kThreads) void k_emit_chunks(SplitEntry* __restrict__ ents,
                                                           const uint2* __restrict__ items, size_t icap,
                                                           DevStatus* __restrict__ st,
                                                           const ushort4* __restrict__ rect,
                                                           const Record* __restrict__ rec, int n,
                                                           const ViewDev* __restrict__ views, int cull, int T,
                                                           const EmitInfo* __restrict__ info,
                                                           const uint32_t* __restrict__ redo_bits,
                                                           uint32_t* __restrict__ pair_tile,
                                                           uint32_t* __restrict__ pair_rec) {
  constexpr int R = (int)(kChunk / 64u);
  const unsigned lane = __lane_id();
  const size_t v = (size_t)blockIdx.x * (blockDim.x / 64) + threadIdx.x / 64;
  const int list = (int)(v % kSplitLists);
  const unsigned long long listed = *split_ctr(st, kSplitEmitItems, list);
  const size_t cnt = listed < icap ? (size_t)listed : icap;
  const unsigned long long K = st->n_eff;
  const size_t step = (size_t)gridDim.x * (blockDim.x / 64) / kSplitLists;
  const uint2* li = items + (size_t)list * icap;
  for (size_t i = v / kSplitLists; i < cnt; i += step) {
    const uint2 it = li[i];
    if (it.x == ~0u) continue;
    SplitEntry* se = ents + it.x;
    const uint32_t rid = se->rid, base = se->base;
    ushort4 rc;
    uint64_t ib = 0ull;
    if (cull) {
      const EmitInfo in = info[rid];
      rc = in.rect;
      ib = in.bits;
    } else {
      rc = rect[rid];
    }
    const ViewDev& cv = views[rid / (uint32_t)n];
    const bool stored = (ib & kRedoFlag) != 0ull;
    CutoffGeoF geo{};
    if (cull && !stored) geo = cutoff_geo_f(rec[rid]);
    const uint32_t nx = (uint32_t)(rc.y - rc.x + 1), C = nx * (uint32_t)(rc.w - rc.z + 1);
    const uint32_t c1 = it.y + kChunk < C ? it.y + kChunk : C;
    const uint32_t tile0 = (uint32_t)cv.tile_off + (uint32_t)rc.z * (uint32_t)cv.tiles_x + rc.x;
    uint64_t m[R];
    uint32_t tl[R];
    uint32_t total = 0;
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const uint32_t li = it.y + (uint32_t)r * 64u + lane;
      bool keep = false;
      tl[r] = 0;
      if (li < c1) {
        uint32_t tx, ty;
        rect_cell(li, nx, tx, ty);
        tl[r] = tile0 + ty * (uint32_t)cv.tiles_x + tx;
        keep = true;
        if (cull) {
          keep = stored ? ((redo_bits[(size_t)(ib & ~kRedoFlag) + li / 32u] >> (li & 31u)) & 1u) != 0u
                        : tile_cutoff_fast(geo, (int)(rc.x + tx), (int)(rc.z + ty), T, cv.W, cv.H) > 0;
        }
      }
      m[r] = __ballot(keep);
      total += (uint32_t)__popcll(m[r]);
    }
    if (total == 0u) continue;
    uint32_t s0 = 0;
    if (lane == 0) s0 = atomicAdd(&se->ctr, total);
    size_t dst0 = (size_t)base + (uint32_t)__shfl((int)s0, 0);
#pragma unroll
    for (int r = 0; r < R; ++r) {
      if ((m[r] >> lane) & 1ull) {
        const size_t dst = dst0 + (uint32_t)__popcll(m[r] & lanemask_lt());
        if (dst < K) {
          pair_tile[dst] = tl[r];
          pair_rec[dst] = rid;
        }
      }
      dst0 += (uint32_t)__popcll(m[r]);
    }
  }
}

// Tile boundaries in the sorted tile ids: each thread takes 4 consecutive ids (one
// 16-byte load) and the id before them.
__global__ void k_ranges(const uint32_t* __restrict__ tile, size_t K_cap, const unsigned long long* __restrict__ n_dev,
                         uint2* __restrict__ ranges, uint32_t n_tiles) {
  const size_t K = item_count(K_cap, n_dev);
  const size_t i0 = ((size_t)blockIdx.x * blockDim.x + threadIdx.x) * 4;
  if (i0 >= K) return;
  uint32_t t[4];
  if (i0 + 4 <= K) {
    const uint4 v = *reinterpret_cast<const uint4*>(tile + i0);
    t[0] = v.x; t[1] = v.y; t[2] = v.z; t[3] = v.w;
  } else {
    for (int k = 0; k < 4; ++k) t[k] = i0 + k < K ? tile[i0 + k] : 0xffffffffu;
  }
  uint32_t prev = i0 == 0 ? 0xffffffffu : tile[i0 - 1];
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    const size_t i = i0 + k;
    if (i >= K) break;
    if (t[k] != prev) {
      if (t[k] < n_tiles) ranges[t[k]].x = (uint32_t)i;
      if (prev < n_tiles) ranges[prev].y = (uint32_t)i;
    }
    prev = t[k];
    if (i + 1 == K && prev < n_tiles) ranges[prev].y = (uint32_t)K;
  }
}

// mode 0: keys + values, mode 1: views of the pairs
__global__ void k_compose(const uint32_t* __restrict__ tile, const uint32_t* __restrict__ rec,
                          const uint32_t* __restrict__ depth, size_t K, int n, size_t n_rec, unsigned long long* __restrict__ keys,
                          uint32_t* __restrict__ values, uint32_t* __restrict__ pviews, int mode) {
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < K; i += (size_t)gridDim.x * blockDim.x) {
    const uint32_t rid = rec[i];
    if (rid >= (uint32_t)n_rec) continue;
    if (mode == 0) {
      if (keys) keys[i] = ((unsigned long long)tile[i] << 32) | depth[rid];
      if (values) values[i] = rid % (uint32_t)n;
    } else {
      pviews[i] = rid / (uint32_t)n;
    }
  }
}

unsigned grid_for(size_t n, unsigned threads, unsigned cap = 1u << 20) {
  size_t b = (n + threads - 1) / threads;
  if (b < 1) b = 1;
  return (unsigned)(b > cap ? cap : b);
}

}  // namespace

size_t sort_hist_words(size_t n) {
  const size_t nb = (n + kSortTileItems - 1) / kSortTileItems;
  // table, chunk sums, digit bases of a pass and of the pass before it
  return (size_t)kRadix * (nb + (nb + kScanChunk - 1) / kScanChunk + 2);
}

namespace {
// Digit table of the pass at `shift` over keys and its scan, the digit starts into
// digit_base[db] (two slots: a pass and the one before it); starts(db) hands the
// scan's parts to the scatter.
// n is the capacity the grids are sized for; with n_dev the kernels sort the count
// found there (at most n) and size the table's scan from it.
struct PassScan {
  size_t n;
  const unsigned long long* n_dev;
  int n_blocks, n_chunks;
  uint32_t *hist, *chunk_sum, *digit_base[2];
  PassScan(size_t n_, const unsigned long long* n_dev_, SortScratch sc) : n(n_), n_dev(n_dev_) {
    const SortGeo g = sort_geo(n);
    n_blocks = g.nb;
    n_chunks = n_dev ? max_chunks(n_blocks) : g.nch;   // grid for any count up to n
    hist = sc.hist;
    chunk_sum = hist + (size_t)kRadix * n_blocks;
    digit_base[0] = chunk_sum + (size_t)kRadix * max_chunks(n_blocks);
    digit_base[1] = digit_base[0] + kRadix;
  }
  void run(const uint32_t* keys, int shift, int db, hipStream_t s) const {
    hipLaunchKernelGGL(k_radix_hist, dim3(n_blocks), dim3(kThreads), 0, s, keys, n, n_dev, shift, hist);
    hipLaunchKernelGGL(k_radix_chunk_sums, dim3(n_chunks), dim3(kRadix), 0, s, hist, n, n_dev, chunk_sum);
    hipLaunchKernelGGL(k_radix_chunk_scan, dim3(1), dim3(kChunkScanThreads), 0, s, chunk_sum, n, n_dev,
                       digit_base[db]);
  }
  DigitStarts starts(int db) const { return DigitStarts{hist, chunk_sum, digit_base[db]}; }
};
}  // namespace

hipError_t radix_sort_pairs(uint32_t* keys_a, uint32_t* vals_a, uint32_t* keys_b, uint32_t* vals_b, size_t n,
                            const unsigned long long* n_dev, int bits, int vals24, SortScratch scratch,
                            int* result_in_b, hipStream_t s) {
  *result_in_b = 0;
  if (n == 0 || bits <= 0) return hipSuccess;
  const PassScan ps(n, n_dev, scratch);
  const dim3 grid((unsigned)(8 * ((ps.n_blocks + 7) / 8)));   // the scatter's XCD-ordered grid
  if (bits > 8 && bits <= 16 && vals24) {
    // two passes moving one packed word between them; the result lands in *_a
    ps.run(keys_a, 0, 0, s);
    hipLaunchKernelGGL(k_radix_scatter<kScatterPack>, grid, dim3(kScatterThreads), 0, s, keys_a, vals_a, n, n_dev, 0,
                       ps.starts(0), nullptr, keys_b, nullptr);
    ps.run(keys_b, 24, 1, s);
    hipLaunchKernelGGL(k_radix_scatter<kScatterUnpack>, grid, dim3(kScatterThreads), 0, s, keys_b, nullptr, n, n_dev, 8,
                       ps.starts(1), ps.digit_base[0], keys_a, vals_a);
    return hipGetLastError();
  }
  uint32_t *ki = keys_a, *vi = vals_a, *ko = keys_b, *vo = vals_b;
  int in_b = 0;
  for (int shift = 0; shift < bits; shift += 8) {
    ps.run(ki, shift, 0, s);
    hipLaunchKernelGGL(k_radix_scatter<kScatterPlain>, grid, dim3(kScatterThreads), 0, s, ki, vi, n, n_dev, shift,
                       ps.starts(0), nullptr, ko, vo);
    uint32_t* t;
    t = ki; ki = ko; ko = t;
    t = vi; vi = vo; vo = t;
    in_b ^= 1;
  }
  *result_in_b = in_b;
  return hipGetLastError();
}

hipError_t radix_sort_depth(const uint32_t* depth, const uint32_t* count, uint32_t* keys_a, uint32_t* vals_a,
                            uint32_t* keys_b, uint32_t* vals_b, size_t n, SortScratch scratch, hipStream_t s) {
  if (n == 0) return hipSuccess;
  if (count && n > kPackMaxEntries) return hipErrorInvalidValue;
  const PassScan ps(n, nullptr, scratch);
  const dim3 grid((unsigned)(8 * ((ps.n_blocks + 7) / 8)));   // the scatter's XCD-ordered grid
  ps.run(depth, 0, 0, s);
  hipLaunchKernelGGL(k_radix_scatter<kScatterIota>, grid, dim3(kScatterThreads), 0, s, depth, count, n, nullptr, 0,
                     ps.starts(0), nullptr, keys_b, vals_b);
  uint32_t *ki = keys_b, *vi = vals_b, *ko = keys_a, *vo = vals_a;
  for (int shift = 8; shift < 32; shift += 8) {
    ps.run(ki, shift, 0, s);
    hipLaunchKernelGGL(k_radix_scatter<kScatterPlain>, grid, dim3(kScatterThreads), 0, s, ki, vi, n, nullptr, shift,
                       ps.starts(0), nullptr, ko, vo);
    uint32_t* t;
    t = ki; ki = ko; ko = t;
    t = vi; vi = vo; vo = t;
  }
  return hipGetLastError();   // three passes after the first: the result is in *_a
}

size_t scan_block_words(size_t n) { return (n + kScanItems - 1) / kScanItems + 1; }

hipError_t launch_scan_touched(const uint32_t* order, int packed, const uint32_t* touched, size_t n,
                               uint32_t* group_sums, uint32_t* block_sums, DevStatus* st, DevStatus* mirror,
                               unsigned long long cap, hipStream_t s) {
  const int nb = (int)((n + kScanItems - 1) / kScanItems);
  hipLaunchKernelGGL(k_scan_reduce, dim3(nb), dim3(kThreads), 0, s, order, touched, n, packed, group_sums,
                     block_sums);
  hipLaunchKernelGGL(k_scan_blocks, dim3(1), dim3(1024), 0, s, block_sums, nb, st, mirror, cap);
  return hipGetLastError();
}

// Workgroups of the chunk passes: enough waves for every item of a heavy scene to
// have its own (their number is known on the device only; workgroups with no item
// exit at once and cost next to nothing).
constexpr unsigned kChunkBlocks = 4096;
static_assert(kChunkBlocks * kWaves % kSplitLists == 0, "every list gets the same number of waves");

hipError_t launch_emit_pairs(const uint32_t* order, int packed, const uint32_t* touched, const uint32_t* group_sums,
                             const uint32_t* block_off, const ushort4* rect, const Record* rec, size_t n_entries,
                             int n, const ViewDev* views, DevStatus* st, int cull, int tile,
                             const EmitInfo* info, const uint32_t* redo_bits, SplitEntry* ents, uint2* items,
                             uint32_t* pair_tile, uint32_t* pair_rec, hipStream_t s) {
  if (n_entries == 0) return hipSuccess;
  const unsigned blocks = (unsigned)((n_entries + kThreads - 1) / kThreads);
  const size_t ecap = split_entry_cap(n_entries), icap = split_item_cap(n_entries);
  hipLaunchKernelGGL(k_emit, dim3(blocks), dim3(kThreads), 0, s, order, packed, touched, group_sums, block_off, rect,
                     rec, n_entries, n, views, st, cull, tile, info, redo_bits, ents, ecap, items, icap, pair_tile,
                     pair_rec);
  hipLaunchKernelGGL(k_emit_chunks, dim3(kChunkBlocks), dim3(kThreads), 0, s, ents, items, icap, st, rect,
                     rec, n, views, cull, tile, info, redo_bits, pair_tile, pair_rec);
  return hipGetLastError();
}

hipError_t launch_count_kept(const uint32_t* touched, const ushort4* rect, const Record* rec, size_t n_entries, int n,
                             const ViewDev* views, int tile, int exact_all, uint32_t* kept, EmitInfo* info,
                             DevStatus* st, uint32_t* redo_list, uint2* items, hipStream_t s) {
  if (n_entries == 0) return hipSuccess;
  const unsigned blocks = (unsigned)((n_entries + kThreads - 1) / kThreads);
  const size_t icap = split_item_cap(n_entries);
  hipLaunchKernelGGL(k_count_kept, dim3(blocks), dim3(kThreads), 0, s, touched, rect, rec, n_entries, n, views, tile,
                     exact_all, kept, info, st, redo_list, items, icap);
  if (!exact_all)
    hipLaunchKernelGGL(k_count_chunks, dim3(kChunkBlocks), dim3(kThreads), 0, s, rect, rec, n, views,
                       tile, kept, st, redo_list, items, icap);
  return hipGetLastError();
}

// Workgroups of the exact pass: its list is known on the device only (a few
// thousandths of the entries in practice; the grid-stride loop covers any number),
// and workgroups with nothing to do exit at once.
constexpr unsigned kRedoBlocks = 2048;

hipError_t launch_count_redo(const uint32_t* touched, const ushort4* rect, const Record* rec, int n,
                             const ViewDev* views, int tile, int exact_all, const float* P, int stride,
                             uint32_t* kept, EmitInfo* info, DevStatus* st, const uint32_t* redo_list,
                             uint32_t* redo_bits, size_t redo_cap, hipStream_t s) {
  hipLaunchKernelGGL(k_count_redo, dim3(kRedoBlocks), dim3(kThreads), 0, s, touched, rect, rec, n, views,
                     tile, exact_all, P,
                     stride, kept, info, st, redo_list, redo_bits, redo_cap);
  return hipGetLastError();
}

hipError_t launch_status_reset(DevStatus* st, hipStream_t s) {
  hipLaunchKernelGGL(k_status_reset, dim3(1), dim3(256), 0, s, st);
  return hipGetLastError();
}


hipError_t launch_ranges(const uint32_t* pair_tile, size_t K_cap, const unsigned long long* n_dev, uint2* ranges,
                         int n_tiles, hipStream_t s) {
  hipError_t e = launch_fill_u32(reinterpret_cast<uint32_t*>(ranges), 0u, (size_t)n_tiles * 2, s);
  if (e != hipSuccess || K_cap == 0) return e;
  const unsigned blocks = (unsigned)((K_cap + 4 * 256 - 1) / (4 * 256));
  hipLaunchKernelGGL(k_ranges, dim3(blocks), dim3(256), 0, s, pair_tile, K_cap, n_dev, ranges, (uint32_t)n_tiles);
  return hipGetLastError();
}

// ---- ordered backward: per-Gaussian sums of the per-tile partials in tile order ----

// keys[i] = entry of sorted pair i, vals[i] = i (the first min(*n_dev, K_cap) pairs)
__global__ void k_entry_keys(const uint32_t* __restrict__ pair_rec, size_t K_cap,
                             const unsigned long long* __restrict__ n_dev, uint32_t* __restrict__ keys,
                             uint32_t* __restrict__ vals) {
  const size_t K = item_count(K_cap, n_dev);
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < K; i += (size_t)gridDim.x * blockDim.x) {
    keys[i] = pair_rec[i];
    vals[i] = (uint32_t)i;
  }
}

// grad2d[e] = sum over the pair positions of entry e (ascending, i.e. in tile order)
// of the partials written by the ordered backward; zero for an entry with no pair.
__global__ void k_ordered_sum(const uint2* __restrict__ eranges, const uint32_t* __restrict__ pos,
                              const float* __restrict__ part, float* __restrict__ grad2d, size_t n_entries) {
  const size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n_entries) return;
  const uint2 r = eranges[e];
  float acc[kGrad2D];
#pragma unroll
  for (int c = 0; c < kGrad2D; ++c) acc[c] = 0.0f;
  for (uint32_t k = r.x; k < r.y; ++k) {
    const float* p = part + (size_t)pos[k] * kGrad2D;
#pragma unroll
    for (int c = 0; c < kGrad2D; ++c) acc[c] += p[c];
  }
#pragma unroll
  for (int c = 0; c < kGrad2D; ++c) grad2d[e * kGrad2D + c] = acc[c];
}

hipError_t launch_ordered_sum(const uint32_t* pair_rec, size_t K_cap, const unsigned long long* n_dev,
                              size_t n_entries, const float* part, uint32_t* keys_a, uint32_t* vals_a,
                              uint32_t* keys_b, uint32_t* vals_b, uint2* eranges, SortScratch scratch,
                              float* grad2d, hipStream_t s) {
  if (n_entries == 0) return hipSuccess;
  hipError_t e;
  int in_b = 0;
  if (K_cap > 0) {
    hipLaunchKernelGGL(k_entry_keys, dim3(grid_for(K_cap, 256, 65536)), dim3(256), 0, s, pair_rec, K_cap, n_dev,
                       keys_a, vals_a);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    int bits = 1;
    while (bits < 32 && ((size_t)1 << bits) < n_entries) ++bits;
    // stable: each entry's positions stay ascending
    if ((e = radix_sort_pairs(keys_a, vals_a, keys_b, vals_b, K_cap, n_dev, bits, 0, scratch, &in_b, s)) !=
        hipSuccess)
      return e;
  }
  if ((e = launch_ranges(in_b ? keys_b : keys_a, K_cap, n_dev, eranges, (int)n_entries, s)) != hipSuccess) return e;
  hipLaunchKernelGGL(k_ordered_sum, dim3((unsigned)((n_entries + 255) / 256)), dim3(256), 0, s, eranges,
                     in_b ? vals_b : vals_a, part, grad2d, n_entries);
  return hipGetLastError();
}

hipError_t launch_compose_keys(const uint32_t* pair_tile, const uint32_t* pair_rec, const uint32_t* depth, size_t K,
                               int n, size_t n_rec, unsigned long long* keys, uint32_t* values, uint32_t* views,
                               int mode, hipStream_t s) {
  if (K == 0) return hipSuccess;
  hipLaunchKernelGGL(k_compose, dim3(grid_for(K, 256, 65536)), dim3(256), 0, s, pair_tile, pair_rec, depth, K, n,
                     n_rec, keys, values, views, mode);
  return hipGetLastError();
}

}  // namespace gsk
