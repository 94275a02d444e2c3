// C ABI of the rasterizer hot path: argument checks, context state, buffer growth,
// launch sequencing and event timing.  Declarations and contracts: include/gs.h.
#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <utility>
#include <vector>

#include "gs_internal.h"

using namespace gsk;

namespace {

struct DevBuf {
  void* p = nullptr;
  size_t cap = 0;
  template <class T>
  T* as() const { return reinterpret_cast<T*>(p); }
};

enum Stage { kNone = 0, kProjected = 1, kBinned = 2, kRendered = 3 };

// Scratch of gs_loss_noalloc: the per-tile loss sums (two doubles per 32x32 loss
// tile), 1 MiB that every GPU the library runs on holds until the process ends.
// In host code this name is a host-side stand-in, not a device address: host code
// uses the per-device address gs_create looks up (scratch_ptr).
constexpr size_t kNoAllocLossTiles = 65536;
static __device__ __align__(256) double scratch[2 * kNoAllocLossTiles];

constexpr int kMaxScratchDevices = 256;
std::mutex scratch_mu;
void* scratch_ptr[kMaxScratchDevices] = {};

// Looks up this device's copy of `scratch` once (the device must be current).
bool scratch_setup(int device) {
  if (device >= kMaxScratchDevices) return true;   // gs_loss_noalloc then reports unsupported
  std::lock_guard<std::mutex> lk(scratch_mu);
  if (scratch_ptr[device]) return true;
  void* p = nullptr;
  if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return false;
  scratch_ptr[device] = p;
  return true;
}

void* scratch_for(int device) {
  if (device < 0 || device >= kMaxScratchDevices) return nullptr;
  std::lock_guard<std::mutex> lk(scratch_mu);
  return scratch_ptr[device];
}

}  // namespace

struct gs_ctx {
  int device = 0;
  std::string err;
  int stage = kNone;
  int n = 0, stride = 0, D = 0, V = 0;
  const float* params = nullptr;   // parameter array of the last gs_preprocess (read by gs_bin_sort)
  int n_tiles = 0;
  int tile = kTile;
  int64_t P = 0;
  mutable uint64_t K = 0;          // pairs of the last binning, once known on the host
  mutable bool K_known = false;    // false after a gs_bin_sort that did not wait for K
  size_t pair_cap = 0;             // pairs the pair buffers hold
  size_t pair_want = 0;            // pairs a failed binning needed (grow before the next)
  size_t redo_cap = 0;             // words of redo_bits
  size_t redo_want = 0;
  std::vector<ViewDev> hviews;
  int depth_in_b = 0, pairs_in_b = 0;
  int cull = GS_CULL_ELLIPSE;
  DevBuf views, rec, depth, touched, rect;
  DevBuf dkey[2], dval[2], groupsums, blocksums, total, hist;
  DevBuf pkey[2], pval[2], ranges;
  DevBuf tfinal, ncontrib, last, grad2d, lossp, aux, evals, pairs_eff;
  bool evals_ok = false;           // evals holds gs_render_count's counts for the current binning
  bool status_fresh = false;       // the status was cleared by the last gs_preprocess and not used since
  DevBuf asum, dG, loadp, loadst, kept, emitinfo, redo_list, redo_bits, status;
  DevBuf split_ents, split_items;  // large entries handed to the binning's chunk passes
  int bwd_order = GS_BWD_ATOMIC;
  DevBuf part, okey[2], oval[2], eranges;   // the ordered backward's partials, entry sort and ranges
  DevStatus* h_status = nullptr;   // host mirror of the device status, written by the binning's last check
  DevStatus* d_mirror = nullptr;   // its device-side address
  bool load_pending = false;   // dG holds a load-balancing gradient for the current forward
  ViewDev* h_views = nullptr;
  bool views_valid = false;   // the device views equal hviews
  unsigned long long* h_total = nullptr;
  hipEvent_t views_ev = nullptr;
  bool views_ev_pending = false;
  hipEvent_t status_ev = nullptr;  // recorded after the binning's check wrote the mirror
  bool status_ev_pending = false;
  bool prof = false;
  std::vector<std::pair<hipEvent_t, hipEvent_t>> ev[GS_N_KERNELS];
  std::vector<hipEvent_t> pool;
  size_t pool_next = 0;
};

namespace {

gs_status fail(gs_ctx* c, gs_status st, const std::string& msg) {
  if (c) c->err = msg;
  return st;
}

gs_status hip_fail(gs_ctx* c, const char* what, hipError_t e) {
  return fail(c, GS_ERR_HIP, std::string(what) + ": " + hipGetErrorString(e));
}

#define GS_HIP(c, expr)                              \
  do {                                               \
    hipError_t e_ = (expr);                          \
    if (e_ != hipSuccess) return hip_fail(c, #expr, e_); \
  } while (0)

// True while `s` is being captured into a HIP graph.  Under capture nothing may be
// allocated, waited for or copied from pageable state: the calls then require the
// buffers a previous uncaptured step sized and report GS_ERR_STATE otherwise.
bool capturing(hipStream_t s) {
  hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
  return hipStreamIsCapturing(s, &cs) == hipSuccess && cs == hipStreamCaptureStatusActive;
}

gs_status ensure(gs_ctx* c, DevBuf& b, size_t bytes, hipStream_t s) {
  if (bytes <= b.cap && b.p) return GS_OK;
  if (capturing(s))
    return fail(c, GS_ERR_STATE, "a context buffer would grow during stream capture: run one uncaptured step "
                                 "with the same sizes first");
  if (b.p) {
    GS_HIP(c, hipStreamSynchronize(s));
    GS_HIP(c, hipFree(b.p));
    b.p = nullptr;
    b.cap = 0;
  }
  size_t want = bytes + bytes / 4 + 256;
  GS_HIP(c, hipMalloc(&b.p, want));
  b.cap = want;
  return GS_OK;
}

std::vector<DevBuf*> all_bufs(gs_ctx* c) {
  return {&c->views, &c->rec, &c->depth, &c->touched, &c->rect, &c->dkey[0], &c->dkey[1], &c->dval[0],
          &c->dval[1], &c->groupsums, &c->blocksums, &c->total, &c->hist, &c->pkey[0],
          &c->pkey[1], &c->pval[0], &c->pval[1], &c->ranges, &c->tfinal, &c->ncontrib, &c->last,
          &c->grad2d, &c->lossp, &c->aux, &c->evals, &c->pairs_eff, &c->asum, &c->dG, &c->loadp, &c->loadst, &c->kept, &c->emitinfo,
          &c->redo_list, &c->redo_bits, &c->status, &c->split_ents, &c->split_items, &c->part, &c->okey[0],
          &c->okey[1], &c->oval[0], &c->oval[1], &c->eranges};
}

hipEvent_t next_event(gs_ctx* c) {
  if (c->pool_next == c->pool.size()) {
    hipEvent_t e;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    c->pool.push_back(e);
  }
  return c->pool[c->pool_next++];
}

struct Prof {
  gs_ctx* c;
  int id;
  hipStream_t s;
  hipEvent_t a = nullptr;
  Prof(gs_ctx* c_, int id_, hipStream_t s_) : c(c_), id(id_), s(s_) {
    if (c->prof && !capturing(s) && (a = next_event(c))) (void)hipEventRecord(a, s);
  }
  ~Prof() {
    if (!c->prof || !a) return;
    hipEvent_t b = next_event(c);
    if (!b) return;
    (void)hipEventRecord(b, s);
    c->ev[id].push_back({a, b});
  }
};

bool aligned(const void* p, size_t a) { return (reinterpret_cast<uintptr_t>(p) % a) == 0; }

int ceil_log2(uint64_t x) {
  int b = 0;
  while ((1ull << b) < x) ++b;
  return b;
}

gs_status check_views(gs_ctx* c, const gs_camera* cams, int n_views, int tile) {
  if (!cams) return fail(c, GS_ERR_INVALID, "cams is NULL");
  if (n_views < 1 || n_views > GS_MAX_VIEWS) return fail(c, GS_ERR_INVALID, "n_views must be in 1..64");
  if (!tile_supported(tile)) return fail(c, GS_ERR_UNSUPPORTED, "tile must be 8, 16 or 32");
  for (int v = 0; v < n_views; ++v) {
    const gs_camera& k = cams[v];
    if (k.width < 1 || k.height < 1 || k.width > GS_MAX_IMAGE_SIDE || k.height > GS_MAX_IMAGE_SIDE)
      return fail(c, GS_ERR_INVALID, "image size out of range in view " + std::to_string(v));
    if (!(std::isfinite(k.fx) && std::isfinite(k.fy) && k.fx > 0.0f && k.fy > 0.0f))
      return fail(c, GS_ERR_INVALID, "focal lengths must be finite and positive in view " + std::to_string(v));
    for (int i = 0; i < 9; ++i)
      if (!std::isfinite(k.R[i])) return fail(c, GS_ERR_INVALID, "non-finite rotation in view " + std::to_string(v));
    for (int i = 0; i < 3; ++i)
      if (!std::isfinite(k.t[i]) || !std::isfinite(k.bg[i]))
        return fail(c, GS_ERR_INVALID, "non-finite translation or background in view " + std::to_string(v));
    if (!std::isfinite(k.cx) || !std::isfinite(k.cy))
      return fail(c, GS_ERR_INVALID, "non-finite principal point in view " + std::to_string(v));
  }
  return GS_OK;
}

void build_views(const gs_camera* cams, int n_views, int tile, std::vector<ViewDev>& out, int* n_tiles, int64_t* P) {
  out.resize(n_views);
  int64_t toff = 0, poff = 0;
  for (int v = 0; v < n_views; ++v) {
    ViewDev& d = out[v];
    const gs_camera& k = cams[v];
    std::memcpy(d.R, k.R, sizeof(d.R));
    std::memcpy(d.t, k.t, sizeof(d.t));
    d.fx = k.fx; d.fy = k.fy; d.cx = k.cx; d.cy = k.cy;
    d.W = k.width; d.H = k.height;
    std::memcpy(d.bg, k.bg, sizeof(d.bg));
    d.tile = tile;
    d.tiles_x = (k.width + tile - 1) / tile;
    d.tiles_y = (k.height + tile - 1) / tile;
    d.tile_off = (int32_t)toff;
    d.pix_off = poff;
    toff += (int64_t)d.tiles_x * d.tiles_y;
    poff += (int64_t)k.width * k.height;
  }
  *n_tiles = (int)toff;
  *P = poff;
}

// Takes in the host mirror of the device status, written by the last binning's
// check: the sizes a failed binning needed (the next gs_bin_sort grows to them)
// and K.  Returns the status code, with a message for an error.
gs_status absorb_status(gs_ctx* c) {
  const DevStatus m = *c->h_status;
  if (m.code != GS_OK) {
    if (m.need_pairs > c->pair_cap && (size_t)m.need_pairs > c->pair_want) c->pair_want = (size_t)m.need_pairs;
    if (m.need_redo > c->redo_cap && (size_t)m.need_redo > c->redo_want) c->redo_want = (size_t)m.need_redo;
    c->K = 0;
    c->K_known = true;
    char buf[256];
    std::snprintf(buf, sizeof(buf),
                  "the last binning ran out of room (%llu pairs needed, %zu held; %llu outcome words needed, %zu "
                  "held); its results are void and the next gs_bin_sort grows the buffers",
                  m.need_pairs, c->pair_cap, m.need_redo, c->redo_cap);
    return fail(c, (gs_status)m.code, buf);
  }
  c->K = m.n_eff;
  c->K_known = true;
  return GS_OK;
}

// K of the last binning on the host: waits for the device when the binning did not.
gs_status resolve_pairs(const gs_ctx* cc) {
  gs_ctx* c = const_cast<gs_ctx*>(cc);
  if (c->K_known || c->stage < kBinned) return GS_OK;
  GS_HIP(c, hipSetDevice(c->device));
  GS_HIP(c, hipEventSynchronize(c->status_ev));
  c->status_ev_pending = false;
  return absorb_status(c);
}

// The raster backward into grad2d (per-entry 2D gradients), in the context's
// summation order.
gs_status raster_backward(gs_ctx* c, const float* dL_dcolor, hipStream_t s) {
  const size_t NV = (size_t)c->V * c->n;
  gs_status st;
  if ((st = ensure(c, c->grad2d, NV * kGrad2D * 4, s)) != GS_OK) return st;
  const float* dG = c->load_pending ? c->dG.as<float>() : nullptr;
  if (c->bwd_order == GS_BWD_ORDERED) {
    // one partial per pair position (the pair buffers hold pair_cap >= K pairs);
    // grids for K when the host knows it, else for the capacity
    const size_t cap = c->pair_cap > 0 ? c->pair_cap : 1;
    const size_t k_grid = c->K_known ? (size_t)c->K : c->pair_cap;
    if ((st = ensure(c, c->part, cap * kGrad2D * 4, s)) != GS_OK) return st;
    for (int i = 0; i < 2; ++i) {
      if ((st = ensure(c, c->okey[i], cap * 4, s)) != GS_OK) return st;
      if ((st = ensure(c, c->oval[i], cap * 4, s)) != GS_OK) return st;
    }
    if ((st = ensure(c, c->eranges, NV * 8, s)) != GS_OK) return st;
    Prof pr(c, GS_K_RENDER_BWD, s);
    GS_HIP(c, launch_render_bwd(c->views.as<ViewDev>(), c->V, c->n_tiles, c->ranges.as<uint2>(),
                                c->pval[c->pairs_in_b].as<uint32_t>(), c->rec.as<Record>(), (uint32_t)NV,
                                c->tfinal.as<float>(), c->last.as<uint32_t>(), dL_dcolor, dG, c->part.as<float>(),
                                c->tile, 1, s));
    SortScratch sc{c->hist.as<uint32_t>()};
    GS_HIP(c, launch_ordered_sum(c->pval[c->pairs_in_b].as<uint32_t>(), k_grid, &c->status.as<DevStatus>()->n_eff,
                                 NV, c->part.as<float>(), c->okey[0].as<uint32_t>(), c->oval[0].as<uint32_t>(),
                                 c->okey[1].as<uint32_t>(), c->oval[1].as<uint32_t>(), c->eranges.as<uint2>(), sc,
                                 c->grad2d.as<float>(), s));
    return GS_OK;
  }
  {
    Prof pr(c, GS_K_ZERO, s);
    GS_HIP(c, launch_fill_u32(c->grad2d.as<uint32_t>(), 0u, NV * kGrad2D, s));
  }
  {
    Prof pr(c, GS_K_RENDER_BWD, s);
    GS_HIP(c, launch_render_bwd(c->views.as<ViewDev>(), c->V, c->n_tiles, c->ranges.as<uint2>(),
                                c->pval[c->pairs_in_b].as<uint32_t>(), c->rec.as<Record>(), (uint32_t)NV,
                                c->tfinal.as<float>(), c->last.as<uint32_t>(), dL_dcolor, dG, c->grad2d.as<float>(),
                                c->tile, 0, s));
  }
  return GS_OK;
}

}  // namespace

extern "C" {

int32_t gs_abi_version(void) { return GS_ABI_VERSION; }

gs_status gs_create(gs_ctx** out, int32_t device) {
  if (!out) return GS_ERR_INVALID;
  *out = nullptr;
  int count = 0;
  if (hipGetDeviceCount(&count) != hipSuccess || device < 0 || device >= count) return GS_ERR_HIP;
  if (hipSetDevice(device) != hipSuccess) return GS_ERR_HIP;
  gs_ctx* c = new gs_ctx();
  c->device = device;
  if (hipHostMalloc((void**)&c->h_views, sizeof(ViewDev) * GS_MAX_VIEWS, hipHostMallocDefault) != hipSuccess ||
      hipHostMalloc((void**)&c->h_total, sizeof(unsigned long long), hipHostMallocDefault) != hipSuccess ||
      hipHostMalloc((void**)&c->h_status, sizeof(DevStatus), hipHostMallocMapped | hipHostMallocCoherent) !=
          hipSuccess ||
      hipHostGetDevicePointer((void**)&c->d_mirror, c->h_status, 0) != hipSuccess ||
      hipEventCreateWithFlags(&c->views_ev, hipEventDisableTiming) != hipSuccess ||
      hipEventCreateWithFlags(&c->status_ev, hipEventDisableTiming) != hipSuccess ||
      hipMalloc(&c->status.p, kStatusAllocBytes) != hipSuccess ||
      hipMemset(c->status.p, 0, kStatusAllocBytes) != hipSuccess || hipDeviceSynchronize() != hipSuccess ||
      !scratch_setup(device)) {
    gs_destroy(c);
    return GS_ERR_HIP;
  }
  c->status.cap = kStatusAllocBytes;
  std::memset(c->h_status, 0, sizeof(DevStatus));
  *out = c;
  return GS_OK;
}

void gs_destroy(gs_ctx* c) {
  if (!c) return;
  (void)hipSetDevice(c->device);
  (void)hipDeviceSynchronize();
  for (DevBuf* b : all_bufs(c))
    if (b->p) (void)hipFree(b->p);
  if (c->h_views) (void)hipHostFree(c->h_views);
  if (c->h_total) (void)hipHostFree(c->h_total);
  if (c->h_status) (void)hipHostFree(c->h_status);
  if (c->views_ev) (void)hipEventDestroy(c->views_ev);
  if (c->status_ev) (void)hipEventDestroy(c->status_ev);
  for (hipEvent_t e : c->pool) (void)hipEventDestroy(e);
  delete c;
}

const char* gs_last_error(const gs_ctx* c) { return c ? c->err.c_str() : "null context"; }

gs_status gs_layout(const gs_camera* cams, int32_t n_views, int32_t tile, int64_t* pix_off, int64_t* tile_off) {
  if (!cams || n_views < 1 || n_views > GS_MAX_VIEWS || tile < 1) return GS_ERR_INVALID;
  int64_t p = 0, t = 0;
  for (int v = 0; v <= n_views; ++v) {
    if (pix_off) pix_off[v] = p;
    if (tile_off) tile_off[v] = t;
    if (v == n_views) break;
    if (cams[v].width < 1 || cams[v].height < 1) return GS_ERR_INVALID;
    p += (int64_t)cams[v].width * cams[v].height;
    t += (int64_t)((cams[v].width + tile - 1) / tile) * ((cams[v].height + tile - 1) / tile);
  }
  return GS_OK;
}

gs_status gs_preprocess(gs_ctx* c, const float* params, int32_t n, int32_t stride, int32_t sh_degree,
                        const gs_camera* cams, int32_t n_views, int32_t tile, gs_stream stream) {
  if (!c) return GS_ERR_INVALID;
  c->err.clear();
  if (!params || !aligned(params, 4)) return fail(c, GS_ERR_INVALID, "params is NULL or misaligned");
  if (n < 1 || stride < n) return fail(c, GS_ERR_INVALID, "need n >= 1 and stride >= n");
  if (sh_degree < 0 || sh_degree > GS_MAX_SH_DEGREE) return fail(c, GS_ERR_INVALID, "sh_degree must be 0..3");
  gs_status st = check_views(c, cams, n_views, tile);
  if (st != GS_OK) return st;
  if ((int64_t)n_views * n >= (1ll << 31)) return fail(c, GS_ERR_CAPACITY, "n_views * n must be < 2^31");
  hipStream_t s = (hipStream_t)stream;
  GS_HIP(c, hipSetDevice(c->device));
  std::vector<ViewDev> hv;
  int n_tiles = 0;
  int64_t P = 0;
  build_views(cams, n_views, tile, hv, &n_tiles, &P);
  const size_t NV = (size_t)n_views * n;
  if ((st = ensure(c, c->views, sizeof(ViewDev) * GS_MAX_VIEWS, s)) != GS_OK) return st;
  if ((st = ensure(c, c->rec, NV * sizeof(Record), s)) != GS_OK) return st;
  if ((st = ensure(c, c->depth, NV * 4, s)) != GS_OK) return st;
  if ((st = ensure(c, c->touched, NV * 4, s)) != GS_OK) return st;
  if ((st = ensure(c, c->rect, NV * 8, s)) != GS_OK) return st;
  // the device copy of the views is only refreshed when they change (a training
  // loop passes the same cameras every step; an upload costs a copy dispatch)
  const bool same_views = c->views_valid && (int32_t)c->hviews.size() == n_views &&
                          std::memcmp(c->hviews.data(), hv.data(), sizeof(ViewDev) * n_views) == 0;
  if (!same_views) {
    if (capturing(s))
      return fail(c, GS_ERR_STATE, "the views differ from the last gs_preprocess: run one uncaptured step with "
                                   "these views before capturing");
    c->views_valid = false;
    if (c->views_ev_pending) GS_HIP(c, hipEventSynchronize(c->views_ev));
    std::memcpy(c->h_views, hv.data(), sizeof(ViewDev) * n_views);
    GS_HIP(c, hipMemcpyAsync(c->views.p, c->h_views, sizeof(ViewDev) * n_views, hipMemcpyHostToDevice, s));
    GS_HIP(c, hipEventRecord(c->views_ev, s));
    c->views_ev_pending = true;
    c->hviews = hv;   // what the device copy holds from here on
    c->views_valid = true;
  }
  {
    Prof pr(c, GS_K_PREPROCESS, s);
    GS_HIP(c, launch_preprocess(params, n, stride, sh_degree, c->views.as<ViewDev>(), n_views, c->rec.as<Record>(),
                                c->depth.as<uint32_t>(), c->touched.as<uint32_t>(), c->rect.as<ushort4>(),
                                c->status.as<DevStatus>(), s));
  }
  c->status_fresh = true;   // the projection cleared the binning status
  c->n = n; c->stride = stride; c->D = sh_degree; c->V = n_views; c->params = params;
  c->hviews = hv; c->n_tiles = n_tiles; c->tile = tile; c->P = P; c->K = 0;
  c->stage = kProjected;
  c->evals_ok = false;
  return GS_OK;
}

gs_status gs_bin_sort(gs_ctx* c, int64_t* n_pairs_out, gs_stream stream) {
  if (!c) return GS_ERR_INVALID;
  c->err.clear();
  if (c->stage < kProjected) return fail(c, GS_ERR_STATE, "gs_bin_sort needs a preceding gs_preprocess");
  hipStream_t s = (hipStream_t)stream;
  GS_HIP(c, hipSetDevice(c->device));
  const size_t NV = (size_t)c->V * c->n;
  gs_status st;
  const bool cap = capturing(s);
  if (cap && (n_pairs_out != nullptr || c->pair_cap == 0))
    return fail(c, GS_ERR_STATE, "gs_bin_sort cannot wait for K during stream capture (pass n_pairs_out = NULL "
                                 "after an uncaptured binning)");
  // what an earlier binning found too small, if the stream has passed its check
  // (read without waiting; gs_sync_status reads it after waiting)
  if (!cap && c->status_ev_pending && hipEventQuery(c->status_ev) == hipSuccess) {
    absorb_status(c);
    c->status_ev_pending = false;
  }
  for (int i = 0; i < 2; ++i) {
    if ((st = ensure(c, c->dkey[i], NV * 4, s)) != GS_OK) return st;
    if ((st = ensure(c, c->dval[i], NV * 4, s)) != GS_OK) return st;
  }
  if ((st = ensure(c, c->groupsums, scan_group_words(NV) * 4, s)) != GS_OK) return st;
  if ((st = ensure(c, c->blocksums, scan_block_words(NV) * 4, s)) != GS_OK) return st;
  if ((st = ensure(c, c->hist, sort_hist_words(NV > c->pair_cap ? NV : c->pair_cap) * 4, s)) != GS_OK) return st;
  DevStatus* dst = c->status.as<DevStatus>();
  if (!c->status_fresh) GS_HIP(c, launch_status_reset(dst, s));
  c->status_fresh = false;
  const bool cull = c->cull != GS_CULL_RECT;
  const int exact_all = c->cull == GS_CULL_ELLIPSE_EXACT ? 1 : 0;
  // pairs per entry: the rect's tiles, or with culling the tiles whose pixel-centre
  // box meets the cutoff region (counted in index order, coalesced; the candidates
  // the fp32 test cannot decide go to the exact pass)
  const uint32_t* per_entry = c->touched.as<uint32_t>();
  if ((st = ensure(c, c->split_items, kSplitLists * split_item_cap(NV) * sizeof(uint2), s)) != GS_OK) return st;
  if ((st = ensure(c, c->split_ents, kSplitLists * split_entry_cap(NV) * sizeof(SplitEntry), s)) != GS_OK)
    return st;
  if (cull) {
    Prof pr(c, GS_K_SCAN, s);
    if ((st = ensure(c, c->kept, NV * 4, s)) != GS_OK) return st;
    if ((st = ensure(c, c->emitinfo, NV * sizeof(EmitInfo), s)) != GS_OK) return st;
    if ((st = ensure(c, c->redo_list, NV * 4, s)) != GS_OK) return st;
    size_t rw = NV / 64 + 1024;
    if (rw < c->redo_want) rw = c->redo_want;
    if (rw > c->redo_cap) {
      if ((st = ensure(c, c->redo_bits, rw * 4, s)) != GS_OK) return st;
      c->redo_cap = c->redo_bits.cap / 4;
    }
    GS_HIP(c, launch_count_kept(c->touched.as<uint32_t>(), c->rect.as<ushort4>(), c->rec.as<Record>(), NV, c->n,
                                c->views.as<ViewDev>(), c->tile, exact_all, c->kept.as<uint32_t>(),
                                c->emitinfo.as<EmitInfo>(), dst, c->redo_list.as<uint32_t>(),
                                c->split_items.as<uint2>(), s));
    GS_HIP(c, launch_count_redo(c->touched.as<uint32_t>(), c->rect.as<ushort4>(), c->rec.as<Record>(), c->n,
                                c->views.as<ViewDev>(), c->tile, exact_all, c->params, c->stride,
                                c->kept.as<uint32_t>(), c->emitinfo.as<EmitInfo>(), dst, c->redo_list.as<uint32_t>(),
                                c->redo_bits.as<uint32_t>(), c->redo_cap, s));
    per_entry = c->kept.as<uint32_t>();
  }
  // depth order of all (view, Gaussian) entries (invisible ones carry the largest
  // key); up to 2^24 entries the sorted values also carry each entry's pair count
  const bool packed = NV <= kPackMaxEntries;
  {
    Prof pr(c, GS_K_DEPTH_SORT, s);
    SortScratch sc{c->hist.as<uint32_t>()};
    GS_HIP(c, radix_sort_depth(c->depth.as<uint32_t>(), packed ? per_entry : nullptr, c->dkey[0].as<uint32_t>(),
                               c->dval[0].as<uint32_t>(), c->dkey[1].as<uint32_t>(), c->dval[1].as<uint32_t>(), NV,
                               sc, s));
    c->depth_in_b = 0;
  }
  const uint32_t* order = c->dval[c->depth_in_b].as<uint32_t>();
  // The pair buffers are sized from K itself when the caller asks for K, on a
  // context's first binning, and after a binning that found them too small;
  // otherwise K stays on the device and the kernels below read it there.  Without
  // a wait the capacity is fixed before the scan, which checks K against it.
  const bool wait = n_pairs_out != nullptr || c->pair_cap == 0;
  auto grow_pairs = [&](size_t want) -> gs_status {
    gs_status g;
    for (int i = 0; i < 2; ++i) {
      if ((g = ensure(c, c->pkey[i], want * 4 + 4, s)) != GS_OK) return g;
      if ((g = ensure(c, c->pval[i], want * 4 + 4, s)) != GS_OK) return g;
    }
    size_t held = c->pkey[0].cap;
    for (DevBuf* b : {&c->pkey[1], &c->pval[0], &c->pval[1]}) held = b->cap < held ? b->cap : held;
    c->pair_cap = held / 4 - 1;
    c->pair_want = 0;
    return ensure(c, c->hist, sort_hist_words(NV > c->pair_cap ? NV : c->pair_cap) * 4, s);
  };
  if (!wait && c->pair_want > c->pair_cap && (st = grow_pairs(c->pair_want)) != GS_OK) return st;
  if ((st = ensure(c, c->ranges, (size_t)c->n_tiles * 8, s)) != GS_OK) return st;
  {
    Prof pr(c, GS_K_SCAN, s);
    // with a wait the buffers grow to K before anything reads them: no cap here
    GS_HIP(c, launch_scan_touched(order, packed ? 1 : 0, per_entry, NV, c->groupsums.as<uint32_t>(),
                                  c->blocksums.as<uint32_t>(), dst, c->d_mirror, wait ? ~0ull : c->pair_cap, s));
  }
  if (!cap) {
    GS_HIP(c, hipEventRecord(c->status_ev, s));
    c->status_ev_pending = true;
  } else {
    c->status_ev_pending = false;   // gs_sync_status waits for the stream before reading the mirror
  }
  c->K_known = false;
  if (wait) {
    GS_HIP(c, hipMemcpyAsync(c->h_total, &dst->n_pairs, 8, hipMemcpyDeviceToHost, s));
    GS_HIP(c, hipStreamSynchronize(s));
    const uint64_t K = *c->h_total;
    if (K >= (1ull << 32)) return fail(c, GS_ERR_CAPACITY, "more than 2^32 - 1 (tile, Gaussian) pairs");
    c->K = K;
    c->K_known = true;
    size_t want = (size_t)K > c->pair_want ? (size_t)K : c->pair_want;
    if ((want > c->pair_cap || c->pair_cap == 0) && (st = grow_pairs(want)) != GS_OK) return st;
  }
  const unsigned long long* n_eff = &dst->n_eff;
  // grids for K when the host knows it, else for the capacity (the kernels read the
  // count on the device either way, so a failed check sorts nothing)
  const size_t k_grid = c->K_known ? (size_t)c->K : c->pair_cap;
  {
    Prof pr(c, GS_K_EMIT, s);
    GS_HIP(c, launch_emit_pairs(order, packed ? 1 : 0, per_entry, c->groupsums.as<uint32_t>(),
                                c->blocksums.as<uint32_t>(), c->rect.as<ushort4>(), c->rec.as<Record>(), NV, c->n,
                                c->views.as<ViewDev>(), dst, cull ? 1 : 0, c->tile,
                                cull ? c->emitinfo.as<EmitInfo>() : nullptr,
                                cull ? c->redo_bits.as<uint32_t>() : nullptr, c->split_ents.as<SplitEntry>(),
                                c->split_items.as<uint2>(), c->pkey[0].as<uint32_t>(), c->pval[0].as<uint32_t>(),
                                s));
  }
  {
    Prof pr(c, GS_K_TILE_SORT, s);
    SortScratch sc{c->hist.as<uint32_t>()};
    const int bits = ceil_log2((uint64_t)c->n_tiles) < 1 ? 1 : ceil_log2((uint64_t)c->n_tiles);
    // record indices are below NV: up to 2^24 entries the two tile passes move one
    // packed word between them
    GS_HIP(c, radix_sort_pairs(c->pkey[0].as<uint32_t>(), c->pval[0].as<uint32_t>(), c->pkey[1].as<uint32_t>(),
                               c->pval[1].as<uint32_t>(), k_grid, n_eff, bits, packed ? 1 : 0, sc,
                               &c->pairs_in_b, s));
  }
  {
    Prof pr(c, GS_K_RANGES, s);
    GS_HIP(c, launch_ranges(c->pkey[c->pairs_in_b].as<uint32_t>(), k_grid, n_eff, c->ranges.as<uint2>(),
                            c->n_tiles, s));
  }
  c->stage = kBinned;
  c->evals_ok = false;
  if (n_pairs_out) *n_pairs_out = (int64_t)c->K;
  return GS_OK;
}

gs_status gs_reserve_pairs(gs_ctx* c, int64_t n_pairs, gs_stream stream) {
  if (!c) return GS_ERR_INVALID;
  c->err.clear();
  if (n_pairs < 1 || n_pairs >= (1ll << 32)) return fail(c, GS_ERR_INVALID, "n_pairs must be in 1..2^32-1");
  hipStream_t s = (hipStream_t)stream;
  GS_HIP(c, hipSetDevice(c->device));
  GS_HIP(c, hipStreamSynchronize(s));
  for (DevBuf* b : {&c->pkey[0], &c->pkey[1], &c->pval[0], &c->pval[1]}) {
    if (b->p) GS_HIP(c, hipFree(b->p));
    b->p = nullptr;
    b->cap = 0;
    GS_HIP(c, hipMalloc(&b->p, (size_t)n_pairs * 4 + 4));
    b->cap = (size_t)n_pairs * 4 + 4;
  }
  c->pair_cap = (size_t)n_pairs;
  c->pair_want = 0;
  gs_status st = ensure(c, c->hist, sort_hist_words(c->pair_cap) * 4, s);
  if (st != GS_OK) return st;
  if (c->stage > kProjected) c->stage = kProjected;   // the pair lists are gone
  return GS_OK;
}

gs_status gs_sync_status(gs_ctx* c, gs_stream stream) {
  if (!c) return GS_ERR_INVALID;
  c->err.clear();
  GS_HIP(c, hipSetDevice(c->device));
  GS_HIP(c, hipStreamSynchronize((hipStream_t)stream));
  if (c->status_ev_pending) {
    GS_HIP(c, hipEventSynchronize(c->status_ev));
    c->status_ev_pending = false;
  }
  return absorb_status(c);
}

gs_status gs_render_fwd(gs_ctx* c, float* color, gs_stream stream) {
  if (!c) return GS_ERR_INVALID;
  c->err.clear();
  if (c->stage < kBinned) return fail(c, GS_ERR_STATE, "gs_render_fwd needs a preceding gs_bin_sort");
  if (!color || !aligned(color, 4)) return fail(c, GS_ERR_INVALID, "color is NULL or misaligned");
  hipStream_t s = (hipStream_t)stream;
  GS_HIP(c, hipSetDevice(c->device));
  gs_status st;
  if ((st = ensure(c, c->tfinal, (size_t)c->P * 4, s)) != GS_OK) return st;
  if ((st = ensure(c, c->ncontrib, (size_t)c->P * 4, s)) != GS_OK) return st;
  if ((st = ensure(c, c->last, (size_t)c->P * 4, s)) != GS_OK) return st;
  if ((st = ensure(c, c->asum, (size_t)c->P * 4, s)) != GS_OK) return st;
  {
    Prof pr(c, GS_K_RENDER_FWD, s);
    GS_HIP(c, launch_render_fwd(c->views.as<ViewDev>(), c->V, c->n_tiles, c->ranges.as<uint2>(),
                                c->pval[c->pairs_in_b].as<uint32_t>(), c->rec.as<Record>(),
                                (uint32_t)((size_t)c->V * c->n), color, c->tfinal.as<float>(),
                                c->ncontrib.as<uint32_t>(), c->last.as<uint32_t>(), c->asum.as<float>(), c->tile,
                                s));
  }
  c->stage = kRendered;
  c->load_pending = false;
  return GS_OK;
}

gs_status gs_render_count(gs_ctx* c, gs_stream stream) {
  if (!c) return GS_ERR_INVALID;
  c->err.clear();
  if (c->stage < kBinned) return fail(c, GS_ERR_STATE, "gs_render_count needs a preceding gs_bin_sort");
  hipStream_t s = (hipStream_t)stream;
  GS_HIP(c, hipSetDevice(c->device));
  gs_status st;
  if ((st = ensure(c, c->evals, (size_t)c->P * 4, s)) != GS_OK) return st;
  if ((st = ensure(c, c->pairs_eff, (size_t)c->n_tiles * 4, s)) != GS_OK) return st;
  GS_HIP(c, launch_render_count(c->views.as<ViewDev>(), c->V, c->n_tiles, c->ranges.as<uint2>(),
                                c->pval[c->pairs_in_b].as<uint32_t>(), c->rec.as<Record>(),
                                (uint32_t)((size_t)c->V * c->n), c->evals.as<uint32_t>(),
                                c->pairs_eff.as<uint32_t>(), c->tile, s));
  c->evals_ok = true;
  return GS_OK;
}

gs_status gs_probe_copy(const void* src, void* dst, size_t bytes, gs_stream stream) {
  if (!src || !dst || bytes % 16 != 0 || !aligned(src, 16) || !aligned(dst, 16)) return GS_ERR_INVALID;
  return launch_probe_copy(src, dst, bytes, (hipStream_t)stream) == hipSuccess ? GS_OK : GS_ERR_HIP;
}

gs_status gs_probe_fma(float* out, int32_t blocks, int32_t iters, int64_t* flops, gs_stream stream) {
  if (!out || blocks < 1 || iters < 1 || !aligned(out, 4)) return GS_ERR_INVALID;
  if (flops) *flops = probe_fma_flops(blocks, iters);
  return launch_probe_fma(out, blocks, iters, (hipStream_t)stream) == hipSuccess ? GS_OK : GS_ERR_HIP;
}

gs_status gs_loss(gs_ctx* c, const float* color, const float* target, float w_l1, float w_dssim, double* loss_out,
                  float* dL_dcolor, gs_stream stream) {
  if (!c) return GS_ERR_INVALID;
  c->err.clear();
  if (c->stage < kProjected) return fail(c, GS_ERR_STATE, "gs_loss needs the views of a preceding gs_preprocess");
  if (!color || !target || !dL_dcolor || !aligned(color, 4) || !aligned(target, 4) || !aligned(dL_dcolor, 4))
    return fail(c, GS_ERR_INVALID, "color, target and dL_dcolor must be non-NULL and aligned");
  if (loss_out && !aligned(loss_out, 8)) return fail(c, GS_ERR_INVALID, "loss_out misaligned");
  if (!std::isfinite(w_l1) || !std::isfinite(w_dssim)) return fail(c, GS_ERR_INVALID, "non-finite loss weight");
  hipStream_t s = (hipStream_t)stream;
  GS_HIP(c, hipSetDevice(c->device));
  gs_status st;
  if ((st = ensure(c, c->lossp, (size_t)loss_tiles(c->hviews.data(), c->V) * 16, s)) != GS_OK) return st;
  if (w_dssim != 0.0f && (st = ensure(c, c->aux, (size_t)c->P * 9 * 4, s)) != GS_OK) return st;
  Prof pr(c, GS_K_LOSS, s);
  GS_HIP(c, launch_loss_dev(c->views.as<ViewDev>(), c->hviews.data(), c->V, color, target, w_l1, w_dssim,
                            c->lossp.as<double>(), w_dssim != 0.0f ? c->aux.as<float>() : nullptr, loss_out,
                            dL_dcolor, s));
  return GS_OK;
}

gs_status gs_loss_noalloc(gs_ctx* c, const float* color, const float* target, float w_l1, float w_dssim,
                          double* loss_out, float* dL_dcolor, gs_stream stream) {
  if (!c) return GS_ERR_INVALID;
  c->err.clear();
  if (c->stage < kProjected) return fail(c, GS_ERR_STATE, "gs_loss_noalloc needs the views of a preceding gs_preprocess");
  if (!color || !target || !dL_dcolor || !aligned(color, 4) || !aligned(target, 4) || !aligned(dL_dcolor, 4))
    return fail(c, GS_ERR_INVALID, "color, target and dL_dcolor must be non-NULL and aligned");
  if (loss_out && !aligned(loss_out, 8)) return fail(c, GS_ERR_INVALID, "loss_out misaligned");
  if (!std::isfinite(w_l1) || !std::isfinite(w_dssim)) return fail(c, GS_ERR_INVALID, "non-finite loss weight");
  const size_t tiles = (size_t)loss_tiles(c->hviews.data(), c->V);
  if (tiles > kNoAllocLossTiles) {
    char buf[160];
    std::snprintf(buf, sizeof buf, "gs_loss_noalloc: the views hold %zu 32x32 loss tiles, more than its %zu",
                  tiles, kNoAllocLossTiles);
    return fail(c, GS_ERR_CAPACITY, buf);
  }
  void* sp = scratch_for(c->device);
  if (!sp) return fail(c, GS_ERR_UNSUPPORTED, "gs_loss_noalloc: no scratch address for this device");
  GS_HIP(c, hipSetDevice(c->device));
  // every tile's sums are written before they are read: nothing to clear; the SSIM
  // term runs as the fused kernel, which keeps its per-pixel terms in LDS
  GS_HIP(c, launch_loss_dev(c->views.as<ViewDev>(), c->hviews.data(), c->V, color, target, w_l1, w_dssim,
                            reinterpret_cast<double*>(sp), nullptr, loss_out, dL_dcolor, (hipStream_t)stream));
  return GS_OK;
}

gs_status gs_load_balance(gs_ctx* c, float w_load, double* loss_out, gs_stream stream) {
  if (!c) return GS_ERR_INVALID;
  c->err.clear();
  if (c->stage < kRendered) return fail(c, GS_ERR_STATE, "gs_load_balance needs a preceding gs_render_fwd");
  if (loss_out && !aligned(loss_out, 8)) return fail(c, GS_ERR_INVALID, "loss_out misaligned");
  if (!std::isfinite(w_load)) return fail(c, GS_ERR_INVALID, "non-finite loss weight");
  hipStream_t s = (hipStream_t)stream;
  GS_HIP(c, hipSetDevice(c->device));
  gs_status st;
  const size_t chunks = (size_t)load_chunks(c->hviews.data(), c->V);
  if ((st = ensure(c, c->dG, (size_t)c->P * 4, s)) != GS_OK) return st;
  if ((st = ensure(c, c->loadp, chunks * c->V * 16, s)) != GS_OK) return st;
  if ((st = ensure(c, c->loadst, (size_t)c->V * 16, s)) != GS_OK) return st;
  {
    Prof pr(c, GS_K_LOAD, s);
    GS_HIP(c, launch_load_balance(c->views.as<ViewDev>(), c->hviews.data(), c->V, c->asum.as<float>(), w_load,
                                  c->loadp.as<double>(), c->loadst.as<double>(), loss_out, c->dG.as<float>(), s));
  }
  c->load_pending = w_load != 0.0f;
  return GS_OK;
}

gs_status gs_render_bwd(gs_ctx* c, const float* params, const float* dL_dcolor, float* grad, int32_t accumulate,
                        gs_stream stream) {
  if (!c) return GS_ERR_INVALID;
  c->err.clear();
  if (c->stage < kRendered) return fail(c, GS_ERR_STATE, "gs_render_bwd needs a preceding gs_render_fwd");
  if (!params || !dL_dcolor || !grad || !aligned(params, 4) || !aligned(dL_dcolor, 4) || !aligned(grad, 4))
    return fail(c, GS_ERR_INVALID, "params, dL_dcolor and grad must be non-NULL and aligned");
  hipStream_t s = (hipStream_t)stream;
  GS_HIP(c, hipSetDevice(c->device));
  gs_status st;
  if ((st = raster_backward(c, dL_dcolor, s)) != GS_OK) return st;
  {
    Prof pr(c, GS_K_PREPROCESS_BWD, s);
    GS_HIP(c, launch_preprocess_bwd(params, c->n, c->stride, c->D, c->views.as<ViewDev>(), c->V,
                                    c->touched.as<uint32_t>(), c->grad2d.as<float>(), grad, accumulate ? 1 : 0, s));
  }
  return GS_OK;
}

// Checks and packs the Adam arguments shared by gs_adam_step and gs_render_bwd_adam.
gs_status adam_args(gs_ctx* c, int32_t n, const float* lr_group, const float* view_lr_scale, int32_t n_views,
                    uint32_t group_mask, float beta1, float beta2, float eps, AdamArgs& a) {
  if (!lr_group) return fail(c, GS_ERR_INVALID, "lr_group must be non-NULL");
  if (n_views < 0 || n_views > GS_MAX_VIEWS) return fail(c, GS_ERR_INVALID, "n_views must be in 0..64");
  if (!(beta1 >= 0.0f && beta1 < 1.0f && beta2 >= 0.0f && beta2 < 1.0f && eps >= 0.0f && std::isfinite(eps)))
    return fail(c, GS_ERR_INVALID, "need 0 <= beta < 1 and finite eps >= 0");
  a = AdamArgs{};
  for (int i = 0; i < GS_N_GROUPS; ++i) {
    if (!std::isfinite(lr_group[i])) return fail(c, GS_ERR_INVALID, "non-finite learning rate");
    a.lr[i] = lr_group[i];
  }
  a.n_views = 0;
  if (n_views > 0 && view_lr_scale) {
    if (c->stage < kProjected || c->n != n || c->V != n_views)
      return fail(c, GS_ERR_STATE, "view factors need the last gs_preprocess to match n and n_views");
    for (int i = 0; i < n_views; ++i) {
      if (!std::isfinite(view_lr_scale[i])) return fail(c, GS_ERR_INVALID, "non-finite view scale");
      a.scale[i] = view_lr_scale[i];
    }
    a.n_views = n_views;
  }
  a.group_mask = group_mask;
  a.b1 = beta1; a.b2 = beta2; a.eps = eps;
  return GS_OK;
}

gs_status gs_adam_step(gs_ctx* c, float* params, const float* grad, float* m, float* v, uint32_t* step, int32_t n,
                       int32_t stride, int32_t sh_degree, const float* lr_group, const float* view_lr_scale,
                       int32_t n_views, uint32_t group_mask, float beta1, float beta2, float eps, gs_stream stream) {
  if (!c) return GS_ERR_INVALID;
  c->err.clear();
  if (!params || !grad || !m || !v || !step || !lr_group)
    return fail(c, GS_ERR_INVALID, "params, grad, m, v, step and lr_group must be non-NULL");
  if (!aligned(params, 4) || !aligned(grad, 4) || !aligned(m, 4) || !aligned(v, 4) || !aligned(step, 4))
    return fail(c, GS_ERR_INVALID, "misaligned device pointer");
  if (n < 1 || stride < n) return fail(c, GS_ERR_INVALID, "need n >= 1 and stride >= n");
  if (sh_degree < 0 || sh_degree > GS_MAX_SH_DEGREE) return fail(c, GS_ERR_INVALID, "sh_degree must be 0..3");
  AdamArgs a;
  gs_status st;
  if ((st = adam_args(c, n, lr_group, view_lr_scale, n_views, group_mask, beta1, beta2, eps, a)) != GS_OK) return st;
  hipStream_t s = (hipStream_t)stream;
  GS_HIP(c, hipSetDevice(c->device));
  Prof pr(c, GS_K_ADAM, s);
  GS_HIP(c, launch_adam(params, grad, m, v, step, n, stride, sh_degree, a,
                        a.n_views ? c->touched.as<uint32_t>() : nullptr, c->status.as<DevStatus>(), s));
  return GS_OK;
}

gs_status gs_render_bwd_adam(gs_ctx* c, float* params, const float* dL_dcolor, float* grad, float* m, float* v,
                             uint32_t* step, const float* lr_group, const float* view_lr_scale, int32_t n_views,
                             uint32_t group_mask, float beta1, float beta2, float eps, gs_stream stream) {
  if (!c) return GS_ERR_INVALID;
  c->err.clear();
  if (c->stage < kRendered) return fail(c, GS_ERR_STATE, "gs_render_bwd_adam needs a preceding gs_render_fwd");
  if (!params || !dL_dcolor || !m || !v || !step || !lr_group)
    return fail(c, GS_ERR_INVALID, "params, dL_dcolor, m, v, step and lr_group must be non-NULL");
  if (!aligned(params, 4) || !aligned(dL_dcolor, 4) || !aligned(m, 4) || !aligned(v, 4) || !aligned(step, 4) ||
      !aligned(grad, 4))
    return fail(c, GS_ERR_INVALID, "misaligned device pointer");
  AdamArgs a;
  gs_status st;
  if ((st = adam_args(c, c->n, lr_group, view_lr_scale, n_views, group_mask, beta1, beta2, eps, a)) != GS_OK)
    return st;
  hipStream_t s = (hipStream_t)stream;
  GS_HIP(c, hipSetDevice(c->device));
  if ((st = raster_backward(c, dL_dcolor, s)) != GS_OK) return st;
  {
    Prof pr(c, GS_K_BWD_ADAM, s);
    GS_HIP(c, launch_preprocess_bwd_adam(params, c->n, c->stride, c->D, c->views.as<ViewDev>(), c->V,
                                         c->touched.as<uint32_t>(), c->grad2d.as<float>(), grad, m, v, step, a,
                                         c->status.as<DevStatus>(), s));
  }
  return GS_OK;
}

gs_status gs_set_cull(gs_ctx* c, int32_t mode) {
  if (!c) return GS_ERR_INVALID;
  c->err.clear();
  if (mode != GS_CULL_RECT && mode != GS_CULL_ELLIPSE && mode != GS_CULL_ELLIPSE_EXACT)
    return fail(c, GS_ERR_INVALID, "unknown cull mode");
  c->cull = mode;
  if (c->stage > kProjected) c->stage = kProjected;   // pair lists must be rebuilt
  return GS_OK;
}

gs_status gs_set_backward_order(gs_ctx* c, int32_t mode) {
  if (!c) return GS_ERR_INVALID;
  c->err.clear();
  if (mode != GS_BWD_ATOMIC && mode != GS_BWD_ORDERED) return fail(c, GS_ERR_INVALID, "unknown backward order");
  c->bwd_order = mode;
  return GS_OK;
}

gs_status gs_buffer_size(const gs_ctx* c, int32_t which, size_t* bytes) {
  if (!c || !bytes) return GS_ERR_INVALID;
  if (which == GS_BUF_KEYS || which == GS_BUF_VALUES || which == GS_BUF_PAIR_VIEW) {
    const gs_status st = resolve_pairs(c);
    if (st != GS_OK && st != GS_ERR_CAPACITY) return st;
  }
  const size_t NV = (size_t)c->V * c->n;
  size_t b = 0;
  switch (which) {
    case GS_BUF_RECORDS: b = c->stage >= kProjected ? NV * sizeof(Record) : 0; break;
    case GS_BUF_DEPTH: case GS_BUF_TOUCHED: b = c->stage >= kProjected ? NV * 4 : 0; break;
    case GS_BUF_TILE_RECT: b = c->stage >= kProjected ? NV * 8 : 0; break;
    case GS_BUF_KEYS: b = c->stage >= kBinned ? c->K * 8 : 0; break;
    case GS_BUF_VALUES: case GS_BUF_PAIR_VIEW: b = c->stage >= kBinned ? c->K * 4 : 0; break;
    case GS_BUF_RANGES: b = c->stage >= kBinned ? (size_t)c->n_tiles * 8 : 0; break;
    case GS_BUF_EVALS: b = (c->stage >= kBinned && c->evals_ok) ? (size_t)c->P * 4 : 0; break;
    case GS_BUF_PAIRS_EFF: b = (c->stage >= kBinned && c->evals_ok) ? (size_t)c->n_tiles * 4 : 0; break;
    case GS_BUF_T_FINAL: case GS_BUF_N_CONTRIB: case GS_BUF_LAST: case GS_BUF_ALPHA_SUM:
      b = c->stage >= kRendered ? (size_t)c->P * 4 : 0;
      break;
    case GS_BUF_GRAD2D: b = (c->stage >= kRendered && c->grad2d.p) ? NV * kGrad2D * 4 : 0; break;
    default: return GS_ERR_INVALID;
  }
  *bytes = b;
  return GS_OK;
}

gs_status gs_copy_buffer(gs_ctx* c, int32_t which, void* dst, size_t bytes, gs_stream stream) {
  if (!c) return GS_ERR_INVALID;
  c->err.clear();
  size_t need = 0;
  if (gs_buffer_size(c, which, &need) != GS_OK) return fail(c, GS_ERR_INVALID, "unknown buffer id");
  if (need == 0) return fail(c, GS_ERR_STATE, "buffer not available in the current state");
  if (!dst || bytes != need) return fail(c, GS_ERR_INVALID, "dst is NULL or bytes != buffer size");
  hipStream_t s = (hipStream_t)stream;
  GS_HIP(c, hipSetDevice(c->device));
  const void* src = nullptr;
  switch (which) {
    case GS_BUF_RECORDS: src = c->rec.p; break;
    case GS_BUF_DEPTH: src = c->depth.p; break;
    case GS_BUF_TOUCHED: src = c->touched.p; break;
    case GS_BUF_TILE_RECT: src = c->rect.p; break;
    case GS_BUF_RANGES: src = c->ranges.p; break;
    case GS_BUF_T_FINAL: src = c->tfinal.p; break;
    case GS_BUF_N_CONTRIB: src = c->ncontrib.p; break;
    case GS_BUF_LAST: src = c->last.p; break;
    case GS_BUF_ALPHA_SUM: src = c->asum.p; break;
    case GS_BUF_EVALS: src = c->evals.p; break;
    case GS_BUF_PAIRS_EFF: src = c->pairs_eff.p; break;
    case GS_BUF_GRAD2D: src = c->grad2d.p; break;
    case GS_BUF_KEYS:
      GS_HIP(c, launch_compose_keys(c->pkey[c->pairs_in_b].as<uint32_t>(), c->pval[c->pairs_in_b].as<uint32_t>(),
                                    c->depth.as<uint32_t>(), c->K, c->n, (size_t)c->V * c->n, (unsigned long long*)dst,
                                    nullptr, nullptr, 0, s));
      return GS_OK;
    case GS_BUF_VALUES:
      GS_HIP(c, launch_compose_keys(c->pkey[c->pairs_in_b].as<uint32_t>(), c->pval[c->pairs_in_b].as<uint32_t>(),
                                    c->depth.as<uint32_t>(), c->K, c->n, (size_t)c->V * c->n, nullptr, (uint32_t*)dst,
                                    nullptr, 0, s));
      return GS_OK;
    case GS_BUF_PAIR_VIEW:
      GS_HIP(c, launch_compose_keys(c->pkey[c->pairs_in_b].as<uint32_t>(), c->pval[c->pairs_in_b].as<uint32_t>(),
                                    c->depth.as<uint32_t>(), c->K, c->n, (size_t)c->V * c->n, nullptr, nullptr,
                                    (uint32_t*)dst, 1, s));
      return GS_OK;
    default: return fail(c, GS_ERR_INVALID, "unknown buffer id");
  }
  GS_HIP(c, hipMemcpyAsync(dst, src, bytes, hipMemcpyDeviceToDevice, s));
  return GS_OK;
}

gs_status gs_profile_enable(gs_ctx* c, int32_t enable) {
  if (!c) return GS_ERR_INVALID;
  c->prof = enable != 0;
  if (c->prof) {
    for (auto& v : c->ev) v.clear();
    c->pool_next = 0;
  }
  return GS_OK;
}

gs_status gs_memory_bytes(const gs_ctx* c, size_t* bytes) {
  if (!c || !bytes) return GS_ERR_INVALID;
  size_t t = 0;
  for (DevBuf* b : all_bufs(const_cast<gs_ctx*>(c))) t += b->p ? b->cap : 0;
  *bytes = t;
  return GS_OK;
}

gs_status gs_profile_read(gs_ctx* c, int32_t kernel, int64_t* launches, double* total_ms) {
  if (!c || kernel < 0 || kernel >= GS_N_KERNELS || !launches || !total_ms) return GS_ERR_INVALID;
  c->err.clear();
  GS_HIP(c, hipSetDevice(c->device));
  GS_HIP(c, hipDeviceSynchronize());
  double t = 0.0;
  for (auto& pr : c->ev[kernel]) {
    float ms = 0.0f;
    GS_HIP(c, hipEventElapsedTime(&ms, pr.first, pr.second));
    t += ms;
  }
  *launches = (int64_t)c->ev[kernel].size();
  *total_ms = t;
  return GS_OK;
}

}  // extern "C"
