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
#include "gs_internal.h"

namespace gsk {
namespace {

constexpr int kThreads = 256;
constexpr int kWaves = kThreads / 64;
constexpr int kItems = kSortTileItems / kThreads;   // items per thread (16)
constexpr int kRadix = 256;

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

__global__ __launch_bounds__(kThreads) void k_radix_hist(const uint32_t* __restrict__ keys, size_t n, int shift,
                                                          uint32_t* __restrict__ hist, int n_blocks) {
  __shared__ uint32_t h[kRadix];
  h[threadIdx.x] = 0;
  __syncthreads();
  const size_t base = (size_t)blockIdx.x * kSortTileItems;
  for (int r = 0; r < kItems; ++r) {
    const size_t i = base + (size_t)r * kThreads + threadIdx.x;
    const bool valid = i < n;
    const uint32_t d = valid ? (keys[i] >> shift) & 0xffu : 0u;
    const uint64_t peers = match_digit(d, valid);
    // the lowest lane of each digit group adds the group's size
    if (valid && (peers & lanemask_lt()) == 0) atomicAdd(&h[d], (uint32_t)__popcll(peers));
  }
  __syncthreads();
  hist[(size_t)threadIdx.x * n_blocks + blockIdx.x] = h[threadIdx.x];
}

// digit_tot[d] = sum over blocks of hist[d][*]
__global__ __launch_bounds__(kThreads) void k_radix_digit_totals(const uint32_t* __restrict__ hist, int n_blocks,
                                                                  uint32_t* __restrict__ digit_tot) {
  __shared__ uint32_t part[kWaves];
  const uint32_t* row = hist + (size_t)blockIdx.x * n_blocks;
  uint32_t s = 0;
  for (int b = threadIdx.x; b < n_blocks; b += kThreads) s += row[b];
  for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off);
  if (__lane_id() == 0) part[threadIdx.x / 64] = s;
  __syncthreads();
  if (threadIdx.x == 0) {
    uint32_t t = 0;
    for (int w = 0; w < kWaves; ++w) t += part[w];
    digit_tot[blockIdx.x] = t;
  }
}

// In-place exclusive scan of row d of hist (over blocks), offset by the number of
// items with a smaller digit.
__global__ __launch_bounds__(kThreads) void k_radix_scan_rows(uint32_t* __restrict__ hist, int n_blocks,
                                                               const uint32_t* __restrict__ digit_tot) {
  __shared__ uint32_t wsum[kWaves];
  __shared__ uint32_t carry;
  const int d = blockIdx.x;
  // base = sum of digit_tot[0..d)
  uint32_t v = threadIdx.x < (unsigned)d ? digit_tot[threadIdx.x] : 0u;
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
  if (__lane_id() == 0) wsum[threadIdx.x / 64] = v;
  __syncthreads();
  if (threadIdx.x == 0) {
    uint32_t t = 0;
    for (int w = 0; w < kWaves; ++w) t += wsum[w];
    carry = t;
  }
  __syncthreads();
  uint32_t* row = hist + (size_t)d * n_blocks;
  for (int b0 = 0; b0 < n_blocks; b0 += kThreads) {
    const int b = b0 + threadIdx.x;
    const uint32_t x = b < n_blocks ? row[b] : 0u;
    // inclusive wave scan
    uint32_t incl = x;
    for (int off = 1; off < 64; off <<= 1) {
      const uint32_t y = __shfl_up(incl, off);
      if ((int)__lane_id() >= off) incl += y;
    }
    __syncthreads();
    if (__lane_id() == 63) wsum[threadIdx.x / 64] = incl;
    __syncthreads();
    uint32_t wpre = 0;
    for (int w = 0; w < (int)(threadIdx.x / 64); ++w) wpre += wsum[w];
    const uint32_t c = carry;
    if (b < n_blocks) row[b] = c + wpre + incl - x;
    __syncthreads();
    if (threadIdx.x == kThreads - 1) carry = c + wpre + incl;
  }
}

__global__ __launch_bounds__(kThreads) void k_radix_scatter(const uint32_t* __restrict__ keys_in,
                                                             const uint32_t* __restrict__ vals_in, size_t n, int shift,
                                                             const uint32_t* __restrict__ offsets, int n_blocks,
                                                             uint32_t* __restrict__ keys_out,
                                                             uint32_t* __restrict__ vals_out) {
  __shared__ uint32_t s_keys[kSortTileItems];
  __shared__ uint32_t s_vals[kSortTileItems];
  __shared__ uint32_t wc[kWaves][kRadix];   // per-wave digit counts of the current round
  __shared__ uint32_t run[kRadix];          // items of each digit in earlier rounds
  __shared__ uint32_t lstart[kRadix];       // workgroup-local start of each digit
  __shared__ uint32_t goff[kRadix];         // global start of this workgroup's run of each digit
  const int tid = threadIdx.x;
  const int wave = tid / 64;
  run[tid] = 0;
  for (int w = 0; w < kWaves; ++w) wc[w][tid] = 0;
  goff[tid] = offsets[(size_t)tid * n_blocks + blockIdx.x];
  __syncthreads();

  const size_t base = (size_t)blockIdx.x * kSortTileItems;
  uint32_t k[kItems], v[kItems], rank[kItems];
  const uint64_t lt = lanemask_lt();
#pragma unroll
  for (int r = 0; r < kItems; ++r) {
    const size_t i = base + (size_t)r * kThreads + tid;
    const bool valid = i < n;
    k[r] = valid ? keys_in[i] : 0xffffffffu;
    v[r] = valid ? vals_in[i] : 0u;
    const uint32_t d = (k[r] >> shift) & 0xffu;
    const uint64_t peers = match_digit(d, valid);
    const bool leader = valid && (peers & lt) == 0;
    if (leader) wc[wave][d] = (uint32_t)__popcll(peers);
    __syncthreads();
    uint32_t before = run[d];
    for (int w = 0; w < wave; ++w) before += wc[w][d];
    rank[r] = before + (uint32_t)__popcll(peers & lt);
    __syncthreads();
    uint32_t tot = 0;
    for (int w = 0; w < kWaves; ++w) {
      tot += wc[w][tid];
      wc[w][tid] = 0;
    }
    run[tid] += tot;
    __syncthreads();
  }
  // exclusive scan of run[] over digits -> local digit starts
  {
    const uint32_t x = run[tid];
    uint32_t incl = x;
    for (int off = 1; off < 64; off <<= 1) {
      const uint32_t y = __shfl_up(incl, off);
      if ((int)__lane_id() >= off) incl += y;
    }
    if (__lane_id() == 63) wc[0][wave] = incl;
    __syncthreads();
    uint32_t wpre = 0;
    for (int w = 0; w < wave; ++w) wpre += wc[0][w];
    lstart[tid] = wpre + incl - x;
    __syncthreads();
  }
  const size_t valid_items = n > base ? (n - base < (size_t)kSortTileItems ? n - base : (size_t)kSortTileItems) : 0;
#pragma unroll
  for (int r = 0; r < kItems; ++r) {
    const size_t i = base + (size_t)r * kThreads + tid;
    if (i < n) {
      const uint32_t d = (k[r] >> shift) & 0xffu;
      const uint32_t pos = lstart[d] + rank[r];
      s_keys[pos] = k[r];
      s_vals[pos] = v[r];
    }
  }
  __syncthreads();
  for (uint32_t p = tid; p < valid_items; p += kThreads) {
    const uint32_t key = s_keys[p];
    const uint32_t d = (key >> shift) & 0xffu;
    const size_t dst = (size_t)goff[d] + (p - lstart[d]);
    if (dst < n) {   // always true for a consistent histogram; guards the write
      keys_out[dst] = key;
      vals_out[dst] = s_vals[p];
    }
  }
}

__global__ void k_iota(uint32_t* __restrict__ p, size_t n) {
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
    p[i] = (uint32_t)i;
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

__global__ __launch_bounds__(kThreads) void k_scan_reduce(const uint32_t* __restrict__ order,
                                                           const uint32_t* __restrict__ touched, size_t n,
                                                           uint32_t* __restrict__ block_sums) {
  __shared__ uint32_t sh[kWaves];
  const size_t base = (size_t)blockIdx.x * kScanItems;
  uint32_t s = 0;
  for (int r = 0; r < kScanItems / kThreads; ++r) {
    const size_t i = base + (size_t)r * kThreads + threadIdx.x;
    if (i < n) s += touched[order[i]];
  }
  const uint32_t t = block_sum_u32(s, sh);
  if (threadIdx.x == 0) block_sums[blockIdx.x] = t;
}

// single workgroup: exclusive scan of block sums in 64-bit, total to *total
__global__ __launch_bounds__(1024) void k_scan_blocks(uint32_t* __restrict__ block_sums, int nb,
                                                       unsigned long long* __restrict__ total) {
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
  if (threadIdx.x == 0) *total = carry;
}

__global__ __launch_bounds__(kThreads) void k_scan_apply(const uint32_t* __restrict__ order,
                                                          const uint32_t* __restrict__ touched, size_t n,
                                                          const uint32_t* __restrict__ block_off,
                                                          uint32_t* __restrict__ offsets) {
  __shared__ uint32_t wsum[kWaves];
  __shared__ uint32_t carry;
  if (threadIdx.x == 0) carry = block_off[blockIdx.x];
  __syncthreads();
  const size_t base = (size_t)blockIdx.x * kScanItems;
  for (int r = 0; r < kScanItems / kThreads; ++r) {
    const size_t i = base + (size_t)r * kThreads + threadIdx.x;
    const uint32_t x = i < n ? touched[order[i]] : 0u;
    uint32_t incl = x;
    for (int off = 1; off < 64; off <<= 1) {
      const uint32_t y = __shfl_up(incl, off);
      if ((int)__lane_id() >= off) incl += y;
    }
    if (__lane_id() == 63) wsum[threadIdx.x / 64] = incl;
    __syncthreads();
    uint32_t wpre = 0;
    for (int w = 0; w < (int)(threadIdx.x / 64); ++w) wpre += wsum[w];
    const uint32_t c = carry;
    if (i < n) offsets[i] = c + wpre + incl - x;
    __syncthreads();
    if (threadIdx.x == kThreads - 1) carry = c + wpre + incl;
    __syncthreads();
  }
}

// One thread per depth-ordered entry writes the (tile, record) pairs of its tile rect.
__global__ __launch_bounds__(kThreads) void k_emit(const uint32_t* __restrict__ order,
                                                    const uint32_t* __restrict__ touched,
                                                    const uint32_t* __restrict__ offsets,
                                                    const ushort4* __restrict__ rect, size_t n_entries, int n,
                                                    const ViewDev* __restrict__ views, size_t K,
                                                    uint32_t* __restrict__ pair_tile, uint32_t* __restrict__ pair_rec) {
  const size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n_entries) return;
  const uint32_t rid = order[e];
  const uint32_t cnt = touched[rid];
  if (cnt == 0) return;
  const int v = (int)(rid / (uint32_t)n);
  const ushort4 rc = rect[rid];
  const uint32_t tiles_x = (uint32_t)views[v].tiles_x;
  const uint32_t toff = (uint32_t)views[v].tile_off;
  size_t o = offsets[e];
  if (o + cnt > K) return;   // never for a consistent scan; guards the writes
  for (uint32_t ty = rc.z; ty <= rc.w; ++ty)
    for (uint32_t tx = rc.x; tx <= rc.y; ++tx) {
      pair_tile[o] = toff + ty * tiles_x + tx;
      pair_rec[o] = rid;
      ++o;
    }
}

__global__ void k_ranges(const uint32_t* __restrict__ tile, size_t K, uint2* __restrict__ ranges, uint32_t n_tiles) {
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < K; i += (size_t)gridDim.x * blockDim.x) {
    const uint32_t t = tile[i];
    if (t >= n_tiles) continue;
    if (i == 0 || tile[i - 1] != t) ranges[t].x = (uint32_t)i;
    if (i == K - 1 || tile[i + 1] != t) ranges[t].y = (uint32_t)(i + 1);
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

size_t sort_hist_words(size_t n) { return (size_t)kRadix * ((n + kSortTileItems - 1) / kSortTileItems + 1); }

hipError_t radix_sort_pairs(uint32_t* keys_a, uint32_t* vals_a, uint32_t* keys_b, uint32_t* vals_b, size_t n,
                            int bits, SortScratch scratch, int* result_in_b, hipStream_t s) {
  *result_in_b = 0;
  if (n == 0 || bits <= 0) return hipSuccess;
  const int n_blocks = (int)((n + kSortTileItems - 1) / kSortTileItems);
  uint32_t *ki = keys_a, *vi = vals_a, *ko = keys_b, *vo = vals_b;
  int in_b = 0;
  for (int shift = 0; shift < bits; shift += 8) {
    hipLaunchKernelGGL(k_radix_hist, dim3(n_blocks), dim3(kThreads), 0, s, ki, n, shift, scratch.hist, n_blocks);
    hipLaunchKernelGGL(k_radix_digit_totals, dim3(kRadix), dim3(kThreads), 0, s, scratch.hist, n_blocks,
                       scratch.digit_tot);
    hipLaunchKernelGGL(k_radix_scan_rows, dim3(kRadix), dim3(kThreads), 0, s, scratch.hist, n_blocks,
                       scratch.digit_tot);
    hipLaunchKernelGGL(k_radix_scatter, dim3(n_blocks), dim3(kThreads), 0, s, ki, vi, n, shift, scratch.hist,
                       n_blocks, ko, vo);
    uint32_t* t;
    t = ki; ki = ko; ko = t;
    t = vi; vi = vo; vo = t;
    in_b ^= 1;
  }
  *result_in_b = in_b;
  return hipGetLastError();
}

hipError_t launch_iota(uint32_t* p, size_t n, hipStream_t s) {
  hipLaunchKernelGGL(k_iota, dim3(grid_for(n, 256, 65536)), dim3(256), 0, s, p, n);
  return hipGetLastError();
}

size_t scan_block_words(size_t n) { return (n + kScanItems - 1) / kScanItems + 1; }

hipError_t launch_scan_touched(const uint32_t* order, const uint32_t* touched, size_t n, uint32_t* offsets,
                               uint32_t* block_sums, unsigned long long* total, hipStream_t s) {
  const int nb = (int)((n + kScanItems - 1) / kScanItems);
  hipLaunchKernelGGL(k_scan_reduce, dim3(nb), dim3(kThreads), 0, s, order, touched, n, block_sums);
  hipLaunchKernelGGL(k_scan_blocks, dim3(1), dim3(1024), 0, s, block_sums, nb, total);
  hipLaunchKernelGGL(k_scan_apply, dim3(nb), dim3(kThreads), 0, s, order, touched, n, block_sums, offsets);
  return hipGetLastError();
}

hipError_t launch_emit_pairs(const uint32_t* order, const uint32_t* touched, const uint32_t* offsets,
                             const ushort4* rect, size_t n_entries, int n, const ViewDev* views, int V, size_t K,
                             uint32_t* pair_tile, uint32_t* pair_rec, hipStream_t s) {
  (void)V;
  hipLaunchKernelGGL(k_emit, dim3(grid_for(n_entries, kThreads)), dim3(kThreads), 0, s, order, touched, offsets, rect,
                     n_entries, n, views, K, pair_tile, pair_rec);
  return hipGetLastError();
}

hipError_t launch_ranges(const uint32_t* pair_tile, size_t K, uint2* ranges, int n_tiles, hipStream_t s) {
  hipError_t e = launch_fill_u32(reinterpret_cast<uint32_t*>(ranges), 0u, (size_t)n_tiles * 2, s);
  if (e != hipSuccess || K == 0) return e;
  hipLaunchKernelGGL(k_ranges, dim3(grid_for(K, 256, 65536)), dim3(256), 0, s, pair_tile, K, ranges,
                     (uint32_t)n_tiles);
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
