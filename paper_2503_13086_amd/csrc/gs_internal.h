// Library-internal definitions shared by the HIP kernels and the C ABI layer.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "gs.h"

namespace gsk {

// Rasterizer constants of the original 3DGS configuration (the paper defers to it
// for everything Sec. III does not state).  FP64 copies are the exact fp32 values.
constexpr double kKappa = (double)0.3f;        // 2D low-pass dilation (px^2)
constexpr double kZNear = (double)0.2f;        // near-plane cull depth
constexpr double kJacClamp = (double)1.3f;     // Jacobian clamp, in half fields of view
constexpr double kExtentSigmas = 3.0;          // extent = 3 sqrt(lambda_max)
constexpr double kCutoffFloor = -4.5;          // exponent at the 3-sigma ellipse
constexpr double kAlphaMinInv = 255.0;         // alpha >= 1/255 to contribute
constexpr float kAlphaMax = 0.99f;             // alpha cap
constexpr float kTMin = 1e-4f;                 // stop blending below this transmittance
constexpr int kTile = 16;                      // default tile edge in pixels
__host__ __device__ inline bool tile_supported(int t) { return t == 8 || t == 16 || t == 32; }
constexpr int kGrad2D = 9;                     // dL/d(u, w, a, b, c, o, r, g, b)

// Per-view constants in device memory (one entry per view).
struct ViewDev {
  float R[9];
  float t[3];
  float fx, fy, cx, cy;
  int32_t W, H;
  float bg[3];
  int32_t tile;       // tile edge in pixels (8, 16 or 32; the same for every view of a batch)
  int32_t tiles_x, tiles_y;
  int32_t tile_off;   // global id of the view's first tile
  int64_t pix_off;    // index of the view's first pixel in the concatenated image
};

// Projected splat of one (view, Gaussian), 48 bytes.  The screen centre is kept in
// FP64 so a tile can take it relative to its own origin without losing the
// sub-pixel digits an fp32 absolute coordinate would drop at 1000+ px.
struct alignas(16) Record {
  double u, w;
  float a, b, c, o;
  float tau, r, g, bl;
};
static_assert(sizeof(Record) == 48, "record layout");

__host__ __device__ inline int n_sh(int D) { return (D + 1) * (D + 1); }

// Does the cutoff region {q(dx, dy) = a dx^2 + 2 b dx dy + c dy^2 <= lim} of a
// splat centred at (u, w) meet the box spanned by the pixel centres of tile
// (gx, gy) (edge T, image W x H)?  The minimum of q over the box is 0 when the box
// holds the centre, else the smallest of the minima along the four edges (clamped
// 1-D minimisers, nbc = -b/c, nba = -b/a).  FP64, no contraction, fixed operation
// order: every kernel that asks gets the same answer.  The pair lists are defined
// by this test on the FP64 conic and cutoff of the projection (exact_cutoff_geo);
// cutoff_geo below builds the same structure from a record's fp32 copies, which
// only the fp32 clear-case test uses.
struct CutoffGeo {
  double u, w, a, b, c, nbc, nba, lim;
};

__device__ inline CutoffGeo cutoff_geo(const Record& r) {
#pragma clang fp contract(off)
  CutoffGeo g;
  g.u = r.u;
  g.w = r.w;
  g.a = r.a;
  g.b = r.b;
  g.c = r.c;
  g.nbc = -g.b / g.c;
  g.nba = -g.b / g.a;
  g.lim = -2.0 * (double)r.tau;
  return g;
}

// What the fp32 clear-case test reads (40 bytes instead of 64): the centre in FP64,
// the rest as the fp32 roundings of the FP64 values of cutoff_geo.
struct CutoffGeoF {
  double u, w;
  float a, b, c, nbc, nba, lim;
};

__device__ inline CutoffGeoF cutoff_geo_f(const Record& r) {
  const CutoffGeo g = cutoff_geo(r);
  CutoffGeoF f;
  f.u = g.u;
  f.w = g.w;
  f.a = (float)g.a;
  f.b = (float)g.b;
  f.c = (float)g.c;
  f.nbc = (float)g.nbc;
  f.nba = (float)g.nba;
  f.lim = (float)g.lim;
  return f;
}

__device__ inline double cutoff_qform(double a, double b, double c, double dx, double dy) {
#pragma clang fp contract(off)
  return ((a * dx) * dx + ((2.0 * b) * dx) * dy) + (c * dy) * dy;
}

__device__ inline bool tile_meets_cutoff(const CutoffGeo& g, int gx, int gy, int T, int W, int H) {
#pragma clang fp contract(off)
  const double dx0 = ((double)(gx * T) + 0.5) - g.u;
  const double dx1 = fmin((double)(gx * T) + ((double)T - 0.5), (double)W - 0.5) - g.u;
  const double dy0 = ((double)(gy * T) + 0.5) - g.w;
  const double dy1 = fmin((double)(gy * T) + ((double)T - 0.5), (double)H - 0.5) - g.w;
  double best = cutoff_qform(g.a, g.b, g.c, dx0, fmin(fmax(g.nbc * dx0, dy0), dy1));
  best = fmin(best, cutoff_qform(g.a, g.b, g.c, dx1, fmin(fmax(g.nbc * dx1, dy0), dy1)));
  best = fmin(best, cutoff_qform(g.a, g.b, g.c, fmin(fmax(g.nba * dy0, dx0), dx1), dy0));
  best = fmin(best, cutoff_qform(g.a, g.b, g.c, fmin(fmax(g.nba * dy1, dx0), dx1), dy1));
  if (dx0 <= 0.0 && dx1 >= 0.0 && dy0 <= 0.0 && dy1 >= 0.0) best = 0.0;
  return best <= g.lim;
}
// The same decision in fp32 where it is clear: 1 keep, 0 drop, -1 too close to call
// (then tile_meets_cutoff on the FP64 conic and cutoff decides).  The box offsets
// are taken in FP64 and rounded (signs, hence the inside test, exact); the four edge
// minima are evaluated at the same clamp points in fp32.  Against the FP64 value
// on the FP64 conic, rounding of the offsets, the products and the clamp points
// stays below 8 ulp of S, S = (|a| + |b|) Dx^2 + (|b| + |c|) Dy^2 bounding
// |a dx^2| + 2 |b dx dy| + |c dy^2| over the box (Dx, Dy the largest offsets), and
// the record's fp32 copies of a, b, c and the cutoff add at most 2^-24 S and
// 2^-23 |lim|; a result within 1e-5 S + 1e-6 |lim| of the limit is left undecided.
__device__ inline int tile_cutoff_fast(const CutoffGeoF& g, int gx, int gy, int T, int W, int H) {
#pragma clang fp contract(off)
  const float dx0 = (float)(((double)(gx * T) + 0.5) - g.u);
  const float dx1 = (float)(fmin((double)(gx * T) + ((double)T - 0.5), (double)W - 0.5) - g.u);
  const float dy0 = (float)(((double)(gy * T) + 0.5) - g.w);
  const float dy1 = (float)(fmin((double)(gy * T) + ((double)T - 0.5), (double)H - 0.5) - g.w);
  if (dx0 <= 0.0f && dx1 >= 0.0f && dy0 <= 0.0f && dy1 >= 0.0f) return g.lim >= 0.0f ? 1 : 0;   // best = 0
  const float a = g.a, b = g.b, c = g.c, nbc = g.nbc, nba = g.nba;
  auto q = [&](float dx, float dy) { return ((a * dx) * dx + ((2.0f * b) * dx) * dy) + (c * dy) * dy; };
  float best = q(dx0, __builtin_amdgcn_fmed3f(nbc * dx0, dy0, dy1));
  best = fminf(best, q(dx1, __builtin_amdgcn_fmed3f(nbc * dx1, dy0, dy1)));
  best = fminf(best, q(__builtin_amdgcn_fmed3f(nba * dy0, dx0, dx1), dy0));
  best = fminf(best, q(__builtin_amdgcn_fmed3f(nba * dy1, dx0, dx1), dy1));
  const float Dx = fmaxf(fabsf(dx0), fabsf(dx1)), Dy = fmaxf(fabsf(dy0), fabsf(dy1));
  const float S = (fabsf(a) + fabsf(b)) * (Dx * Dx) + (fabsf(b) + fabsf(c)) * (Dy * Dy);
  const float lim = g.lim;
  const float margin = 1e-5f * S + 1e-6f * fabsf(lim) + 1e-30f;
  if (best <= lim - margin) return 1;
  if (best > lim + margin) return 0;
  return -1;
}

__host__ __device__ inline int n_params(int D) { return 11 + 3 * n_sh(D); }

// Device-side status of a context: conditions kernels find while a step runs
// (reported by gs_sync_status), and the counters of the binning.  Reset at the
// start of every binning.
struct DevStatus {
  int32_t code;                   // GS_OK or the first error (GS_ERR_CAPACITY)
  uint32_t pad;
  unsigned long long n_pairs;     // pairs of the last binning (K)
  unsigned long long n_eff;       // K when the pair buffers hold it, else 0: the later kernels then do nothing
  unsigned long long need_pairs;  // pairs the last binning needed room for
  unsigned long long redo_count;  // entries whose cutoff tests the fp32 test left undecided
  unsigned long long redo_words;  // outcome words handed out to such entries of more than 64 candidates
  unsigned long long need_redo;   // outcome words they needed
};
// EmitInfo.bits of an entry of more than 64 candidates whose outcomes the exact
// pass stored: this flag | the first of its words in the outcome array.
constexpr uint64_t kRedoFlag = 1ull << 63;

__device__ inline void status_clear(DevStatus* st) {
  st->code = GS_OK;
  st->pad = 0u;
  st->n_pairs = 0ull;
  st->n_eff = 0ull;
  st->need_pairs = 0ull;
  st->redo_count = 0ull;
  st->redo_words = 0ull;
  st->need_redo = 0ull;
}

__device__ inline void status_fail(DevStatus* st, int32_t code) {
  atomicCAS(&st->code, (int32_t)GS_OK, code);
}

// ---- launchers (each file defines its own) ----
hipError_t launch_preprocess(const float* P, int n, int stride, int D, const ViewDev* views, int V,
                             Record* rec, uint32_t* depth, uint32_t* touched, ushort4* rect, DevStatus* st,
                             hipStream_t s);
hipError_t launch_preprocess_bwd(const float* P, int n, int stride, int D, const ViewDev* views, int V,
                                 const uint32_t* touched, const float* grad2d, float* grad, int accumulate,
                                 hipStream_t s);
hipError_t launch_fill_u32(uint32_t* p, uint32_t value, size_t count, hipStream_t s);

// radix sort of (uint32 key, uint32 value) pairs on bits [0, bits) of the key;
// returns which buffer (0: *_a, 1: *_b) holds the result.  vals24: every value is
// below 2^24 (then keys of 9 to 16 bits take two passes that move one packed word
// between them, and the result is in *_a; vals_b is not touched)
struct SortScratch {
  uint32_t* hist;      // sort_hist_words(n): block-major digit table, chunk sums, digit bases
};
constexpr int kSortTileItems = 4096;
size_t sort_hist_words(size_t n);
// n_dev (may be NULL): the item count in device memory, read by the kernels (at
// most n, which sizes the grids); without it n items are sorted.
hipError_t radix_sort_pairs(uint32_t* keys_a, uint32_t* vals_a, uint32_t* keys_b, uint32_t* vals_b, size_t n,
                            const unsigned long long* n_dev, int bits, int vals24, SortScratch scratch,
                            int* result_in_b, hipStream_t s);
// Stable sort of the entries 0..n-1 by depth[e] (32-bit keys, read only): values
// e, with count given e | min(count[e], 255) << 24 (n <= 2^24); result in *_a
hipError_t radix_sort_depth(const uint32_t* depth, const uint32_t* count, uint32_t* keys_a, uint32_t* vals_a,
                            uint32_t* keys_b, uint32_t* vals_b, size_t n, SortScratch scratch, hipStream_t s);
// Depth-sort values that carry the entry's pair count: index in the low 24 bits,
// min(count, 255) in the top byte (255: read the count from the per-entry array).
// Used when the entries number at most 2^24.
constexpr size_t kPackMaxEntries = (size_t)1 << 24;
constexpr int kPackShift = 24;
constexpr uint32_t kPackSat = 255u;
constexpr uint32_t kPackRidMask = 0x00ffffffu;

// Scan of the depth-ordered counts touched[order[e]]: group_sums[g] = sum over the
// 64 entries [64 g, 64 g + 64) (scan_group_words(n) words), block_sums[b] = the
// exclusive prefix at entry 4096 b (scan_block_words(n) words); the total K goes to
// st->n_pairs and is checked against the pair capacity: n_eff = K if K <= cap, K <
// 2^32 and no earlier failure, else 0 (GS_ERR_CAPACITY with need_pairs = K when K
// does not fit); then the status is copied to `mirror` (host-visible memory).
// (packed != 0: order entries come from radix_sort_depth with counts)
size_t scan_block_words(size_t n);
inline size_t scan_group_words(size_t n) { return (n + 63) / 64; }
hipError_t launch_scan_touched(const uint32_t* order, int packed, const uint32_t* touched, size_t n,
                               uint32_t* group_sums, uint32_t* block_sums, DevStatus* st, DevStatus* mirror,
                               unsigned long long cap, hipStream_t s);
// kept[e] = tiles of entry e's rect whose pixel-centre box meets its cutoff region
// (entries in index order; rect tile count in touched)
// What emission fetches per culled entry: its tile rect and, for rects of at most
// 64 tiles, which of them the cutoff region meets (bit i: the rect's i-th tile in
// row-major order).
struct alignas(16) EmitInfo {
  ushort4 rect;
  uint64_t bits;
};
// Work split for entries with large rects (near the camera, where the depth order
// puts them side by side).  A wave whose 64 entries have more than kSplitWave
// candidates in all hands its largest entries (those above the threshold that
// leaves it at most kSplitWave candidates, or all of more than 64) to a chunk pass
// instead of walking their rects itself: one item (entry, first candidate) per
// kChunk candidates, so a large rect is spread over many waves.  Items go to one
// of kSplitLists lists (by wave index), each with its own counter on its own
// 128-byte line, so heavy waves do not queue on one address; slot k of list l is
// items[l * cap + k] (x = entry, or the SplitEntry slot for the emission; y =
// first candidate; x = ~0 for a slot a full list left unused).  A full list
// leaves the entry with its wave.
constexpr uint32_t kSplitWave = 2048u;
constexpr uint32_t kChunk = 512u;
constexpr int kSplitLists = 64;
constexpr int kSplitCtrStride = 16;   // counters 16 x 8 bytes apart
// The counters sit after the status word in the same allocation: three sets of
// kSplitLists (the count's items, the emission's entries and its items).
constexpr size_t kStatusBytes = 256;
static_assert(sizeof(DevStatus) <= kStatusBytes, "status word");
constexpr size_t kStatusAllocBytes = kStatusBytes + 3 * kSplitLists * kSplitCtrStride * 8;
enum SplitSet { kSplitCountItems = 0, kSplitEmitEnts = 1, kSplitEmitItems = 2 };
__device__ inline unsigned long long* split_ctr(DevStatus* st, int set, int list) {
  return reinterpret_cast<unsigned long long*>(reinterpret_cast<char*>(st) + kStatusBytes) +
         (size_t)(set * kSplitLists + list) * kSplitCtrStride;
}
// Clears the counters (the calling workgroup's threads share the stores).
__device__ inline void split_clear(DevStatus* st) {
  for (int i = (int)threadIdx.x; i < 3 * kSplitLists; i += (int)blockDim.x)
    *split_ctr(st, i / kSplitLists, i % kSplitLists) = 0ull;
}
// An entry whose pairs the emission's chunk pass writes: its output range starts
// at `base`; `ctr` counts the pairs written so far (chunks take their slots in the
// range with atomics: within one entry's range the order does not matter, since
// its pairs go to distinct tiles and the tile sort is stable).
struct alignas(16) SplitEntry {
  uint32_t rid, base, ctr, pad;
};
// slots per list (in all about one item per 16 entries and one split entry per 64)
inline size_t split_item_cap(size_t n_entries) { return n_entries / (16 * kSplitLists) + 256; }
inline size_t split_entry_cap(size_t n_entries) { return n_entries / (64 * kSplitLists) + 64; }
// Entries where the fp32 test leaves some candidate undecided are counted without
// those candidates and listed in redo_list (count in st->redo_count); the exact
// pass launch_count_redo then recomputes their FP64 conic and cutoff from the
// parameters and rewrites their kept count and EmitInfo (for more than 64
// candidates: kRedoFlag | offset of their outcome bits in redo_bits, which holds
// redo_cap words; beyond that st reports GS_ERR_CAPACITY).
// exact_all != 0: no candidate is decided by the fp32 test (every test in FP64).
// Entries split into chunk items (items: kSplitLists * split_item_cap(n_entries)
// slots) are counted by a chunk pass in the same call.
hipError_t launch_count_kept(const uint32_t* touched, const ushort4* rect, const Record* rec, size_t n_entries, int n,
                             const ViewDev* views, int tile, int exact_all, uint32_t* kept, EmitInfo* info,
                             DevStatus* st, uint32_t* redo_list, uint2* items, hipStream_t s);
hipError_t launch_count_redo(const uint32_t* touched, const ushort4* rect, const Record* rec, int n,
                             const ViewDev* views, int tile, int exact_all, const float* P, int stride,
                             uint32_t* kept, EmitInfo* info, DevStatus* st, const uint32_t* redo_list,
                             uint32_t* redo_bits, size_t redo_cap, hipStream_t s);
// Clears the status (the projection also clears it, so a binning right after a
// gs_preprocess needs no reset launch).
hipError_t launch_status_reset(DevStatus* st, hipStream_t s);
// pairs of the depth-ordered entries order[0..n_entries): touched, group_sums and
// block_sums as scanned by launch_scan_touched; cull != 0 keeps only the rect tiles
// that meet the cutoff region (touched must then be the kept counts); writes only
// below st->n_eff pairs.  Entries split into chunk items (ents: kSplitLists *
// split_entry_cap(n_entries) slots, items: kSplitLists * split_item_cap(n_entries))
// are emitted by a chunk pass in the same call.
hipError_t launch_emit_pairs(const uint32_t* order, int packed, const uint32_t* touched, const uint32_t* group_sums,
                             const uint32_t* block_off, const ushort4* rect, const Record* rec, size_t n_entries,
                             int n, const ViewDev* views, DevStatus* st, int cull, int tile,
                             const EmitInfo* info, const uint32_t* redo_bits, SplitEntry* ents, uint2* items,
                             uint32_t* pair_tile, uint32_t* pair_rec, hipStream_t s);
// ranges of the first min(*n_dev, K_cap) sorted pairs (all K_cap without n_dev)
hipError_t launch_ranges(const uint32_t* pair_tile, size_t K_cap, const unsigned long long* n_dev, uint2* ranges,
                         int n_tiles, hipStream_t s);
hipError_t launch_compose_keys(const uint32_t* pair_tile, const uint32_t* pair_rec, const uint32_t* depth,
                               size_t K, int n, size_t n_rec, unsigned long long* keys, uint32_t* values,
                               uint32_t* views, int mode, hipStream_t s);

// n_rec: number of records (V * n); record ids at or beyond it are skipped
// forward also writes the soft count asum [P] (sum of blended alphas); the
// backward adds dL/dG [P] (may be NULL) to every blended alpha's derivative
hipError_t launch_render_fwd(const ViewDev* views, int V, int n_tiles, const uint2* ranges, const uint32_t* pair_rec,
                             const Record* rec, uint32_t n_rec, float* color, float* t_final, uint32_t* n_contrib,
                             uint32_t* last, float* asum, int tile, hipStream_t s);
// The forward walk counting per pixel the Gaussians evaluated up to termination
// (evals [P]) and per tile the list entries some pixel blended (pairs_eff [tiles]).
hipError_t launch_render_count(const ViewDev* views, int V, int n_tiles, const uint2* ranges, const uint32_t* pair_rec,
                               const Record* rec, uint32_t n_rec, uint32_t* evals, uint32_t* pairs_eff, int tile,
                               hipStream_t s);
// Probes: a streaming 16-byte-vector copy of `bytes` (a multiple of 16) and
// `blocks` x 256 threads of eight fp32 FMA chains of `iters` steps.
hipError_t launch_probe_copy(const void* src, void* dst, size_t bytes, hipStream_t s);
hipError_t launch_probe_fma(float* out, int blocks, int iters, hipStream_t s);
int64_t probe_fma_flops(int blocks, int iters);
// ordered == 0: per-tile partial sums added into grad2d[V*n][kGrad2D] with global
// atomics (grad2d zeroed first).  ordered != 0: the partial of the pair at sorted
// position i goes to grad2d[i * kGrad2D ...] (a [K][kGrad2D] buffer: every position of
// every tile list written, the same bits on every run); launch_ordered_sum then
// forms the per-entry sums.
hipError_t launch_render_bwd(const ViewDev* views, int V, int n_tiles, const uint2* ranges, const uint32_t* pair_rec,
                             const Record* rec, uint32_t n_rec, const float* t_final, const uint32_t* last,
                             const float* dL_dcolor, const float* dL_dG, float* grad2d, int tile, int ordered,
                             hipStream_t s);
// grad2d[e] = the sum, in ascending pair position (tile order), of the partials
// part[i] of the pairs i whose entry pair_rec[i] is e, for e < n_entries (zero for
// an entry with no pair): the pairs' entries are sorted stably (keys/vals a and b:
// K_cap words each, scratch sized for K_cap items), then delimited per entry
// (eranges: n_entries uint2).  K = min(*n_dev, K_cap) pairs.
hipError_t launch_ordered_sum(const uint32_t* pair_rec, size_t K_cap, const unsigned long long* n_dev,
                              size_t n_entries, const float* part, uint32_t* keys_a, uint32_t* vals_a,
                              uint32_t* keys_b, uint32_t* vals_b, uint2* eranges, SortScratch scratch,
                              float* grad2d, hipStream_t s);

// Loss over all views in 32x32-pixel tiles: loss_tiles() tiles, partials 2 doubles
// per tile; aux 9 floats per pixel for the SSIM term, or NULL for the fused SSIM
// kernel, which needs none.
int loss_tiles(const ViewDev* hviews, int V);
// Eq. 9 on the soft count asum [P]: per-view loss w std (loss_out, may be NULL)
// and dL/dG [P]; partials: V x load_chunks doubles2, stats: V doubles2
int load_chunks(const ViewDev* hviews, int V);
hipError_t launch_load_balance(const ViewDev* dviews, const ViewDev* hviews, int V, const float* asum, float w,
                               double* partials, double* stats, double* loss_out, float* dG, hipStream_t s);
hipError_t launch_loss_dev(const ViewDev* dviews, const ViewDev* hviews, int V, const float* color,
                           const float* target, float w_l1, float w_dssim, double* partials, float* aux,
                           double* loss_out, float* dL_dcolor, hipStream_t s);

struct AdamArgs {
  float lr[GS_N_GROUPS];
  float scale[GS_MAX_VIEWS];
  int n_views;          // 0: no per-view factor
  uint32_t group_mask;  // groups that take the per-view factor
  float b1, b2, eps;
};
// The Adam kernels leave every buffer untouched when st (may be NULL) reports an
// error: a step whose binning failed must not move the parameters.
hipError_t launch_adam(float* P, const float* G, float* M, float* Vv, uint32_t* step, int n, int stride, int D,
                       const AdamArgs& a, const uint32_t* touched, const DevStatus* st, hipStream_t s);

// ---- Adam pieces shared by the Adam kernel and the fused backward + Adam, so
// that both produce the same bits ----
__device__ inline int adam_row_group(int r) {
  if (r < 3) return GS_GROUP_MEAN;
  if (r < 6) return GS_GROUP_SCALE;
  if (r < 10) return GS_GROUP_ROT;
  if (r == 10) return GS_GROUP_OPACITY;
  if (r < 14) return GS_GROUP_SH_DC;
  return GS_GROUP_SH_REST;
}

// Mean of the view scales over the views that see Gaussian g (touched > 0), over
// all views when none does; 1 without view scales.
__device__ inline float adam_view_factor(const AdamArgs& a, const uint32_t* touched, int n, int g) {
  if (a.n_views <= 0) return 1.0f;
  float s = 0.0f, all = 0.0f;
  int c = 0;
  for (int v = 0; v < a.n_views; ++v) {
    all += a.scale[v];
    if (touched[(size_t)v * n + g] != 0u) {
      s += a.scale[v];
      ++c;
    }
  }
  return c > 0 ? s / (float)c : all / (float)a.n_views;
}

// Bias corrections 1 - b^k for step k (k = the element's updated step counter).
__device__ inline void adam_bias(const AdamArgs& a, uint32_t k, float& bc1, float& bc2) {
  bc1 = (float)(1.0 - pow((double)a.b1, (double)k));
  bc2 = (float)(1.0 - pow((double)a.b2, (double)k));
}

// One element: m = b1 m + (1 - b1) g, v = b2 v + (1 - b2) g^2,
// p -= lr (m / bc1) / (sqrt(v / bc2) + eps).
__device__ inline void adam_elem(float& p, float& m, float& v, float g, float lr, const AdamArgs& a, float bc1,
                                 float bc2) {
#pragma clang fp contract(off)
  const float ob1 = 1.0f - a.b1, ob2 = 1.0f - a.b2;
  m = a.b1 * m + ob1 * g;
  v = a.b2 * v + ob2 * g * g;
  p = p - lr * (m / bc1) / (sqrtf(v / bc2) + a.eps);
}

// Backward preprocess fused with the Adam step: the parameter gradient of each
// Gaussian is applied as soon as it is formed (grad written too when not NULL).
hipError_t launch_preprocess_bwd_adam(float* P, int n, int stride, int D, const ViewDev* views, int V,
                                      const uint32_t* touched, const float* grad2d, float* grad, float* M, float* Vv,
                                      uint32_t* step, const AdamArgs& a, const DevStatus* st, hipStream_t s);

}  // namespace gsk
