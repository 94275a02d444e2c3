/*
 * gs.h - C ABI of the MI355X (gfx950) differentiable tile rasterizer and optimizer
 * step: the per-iteration hot path of progressive 3D Gaussian Splatting
 * (Gaussian On-the-Fly Splatting; Sec. III Eq. 1-2, Sec. IV-D Eq. 6-8,
 * Sec. IV-E, Sec. V-A implementation details).
 *
 * Every call is stream-ordered and asynchronous unless stated otherwise, takes
 * plain pointers and sizes, and returns a gs_status; nothing aborts or throws
 * across this boundary.  Argument checks happen on the host before any work is
 * queued; a failed check queues nothing.  The caller owns every parameter,
 * gradient, optimizer-state, image and target buffer (device memory, fp32 unless
 * stated).  A context owns only its intermediate buffers (per-view projections,
 * sort buffers, per-pixel forward state, 2D gradients) and grows them as needed.
 * One context serves one stream at a time; calls on one context must not
 * overlap.  A context keeps the views, sizes and buffers of its last
 * gs_preprocess; gs_bin_sort, gs_render_fwd, gs_loss, gs_render_bwd and
 * gs_adam_step operate on that state and must follow it in this order.
 *
 * Gaussian parameters: one fp32 device array of n_params(D) rows by `stride`
 * columns (row-major, column g is Gaussian g, stride >= n), D = SH degree 0..3:
 *   rows 0..2   mean (world)              rows 3..5   log-scale
 *   rows 6..9   quaternion (w, x, y, z), any norm > 0
 *   row  10     opacity logit             rows 11..   SH coefficient k, channel c
 *                                                     at row 11 + 3k + c
 *   n_params(D) = 11 + 3 (D+1)^2   (14 at D = 0, 59 at D = 3)
 * Gradients and Adam moments use the same layout.
 *
 * Images: fp32, all views concatenated; view v occupies floats
 * [3 pix_off[v], 3 pix_off[v+1]) laid out [3][height][width] (planar RGB), where
 * pix_off is the exclusive prefix sum of width*height over views (gs_layout).
 * Pixel (i, j) has its centre at (i + 1/2, j + 1/2).
 */
#ifndef GS_H_
#define GS_H_

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define GS_ABI_VERSION 1
#define GS_MAX_VIEWS 64
#define GS_MAX_SH_DEGREE 3
#define GS_MAX_IMAGE_SIDE 16384

typedef enum gs_status {
  GS_OK = 0,
  GS_ERR_INVALID = -1,      /* bad argument (null, out of range, misaligned) */
  GS_ERR_CAPACITY = -2,     /* a size limit of the library would be exceeded */
  GS_ERR_HIP = -3,          /* a HIP runtime call failed; see gs_last_error */
  GS_ERR_UNSUPPORTED = -4,  /* valid but not implemented (e.g. tile size) */
  GS_ERR_STATE = -5         /* call out of order (e.g. render before preprocess) */
} gs_status;

typedef struct gs_ctx gs_ctx;
typedef void* gs_stream; /* a hipStream_t; NULL is the null stream */

/* A pinhole view.  World->camera: x_cam = R x_world + t, R row-major; camera axes
 * x right, y down, z forward.  Intrinsics in pixels.  bg: background colour. */
typedef struct gs_camera {
  float R[9];
  float t[3];
  float fx, fy, cx, cy;
  int32_t width, height;
  float bg[3];
} gs_camera;

/* Adam parameter groups (bits of gs_adam_step's group_mask). */
enum { GS_GROUP_MEAN = 0, GS_GROUP_SCALE = 1, GS_GROUP_ROT = 2, GS_GROUP_OPACITY = 3,
       GS_GROUP_SH_DC = 4, GS_GROUP_SH_REST = 5, GS_N_GROUPS = 6 };

/* Context buffers readable with gs_copy_buffer (for inspection and tests). */
enum {
  GS_BUF_RECORDS = 0,   /* per (view, Gaussian) record, 48 B: double u, double w (pixel-space
                           centre), float a, b, c (conic), o (opacity), tau (cutoff exponent),
                           r, g, b (colour); index v*n + g; only visible entries are defined */
  GS_BUF_DEPTH = 1,     /* uint32 [V*n]: fp32 bit pattern of camera depth (0xffffffff if invisible) */
  GS_BUF_TOUCHED = 2,   /* uint32 [V*n]: number of tiles of the tile rect (0 = invisible) */
  GS_BUF_TILE_RECT = 3, /* uint16 [V*n][4]: tx0, tx1, ty0, ty1 (inclusive) */
  GS_BUF_KEYS = 4,      /* uint64 [K]: sorted keys (global tile << 32) | depth bits */
  GS_BUF_VALUES = 5,    /* uint32 [K]: Gaussian index of each sorted pair */
  GS_BUF_RANGES = 6,    /* uint32 [tiles][2]: [start, end) of each tile in the sorted pairs */
  GS_BUF_T_FINAL = 7,   /* float  [P]: final transmittance per pixel */
  GS_BUF_N_CONTRIB = 8, /* uint32 [P]: Gaussians blended per pixel */
  GS_BUF_LAST = 9,      /* uint32 [P]: 1 + position (within its tile's list) of the last
                           blended Gaussian, 0 if none */
  GS_BUF_GRAD2D = 10,   /* float  [V*n][9]: dL/d(u, w, a, b, c, o, r, g, b) per (view, Gaussian) */
  GS_BUF_PAIR_VIEW = 11,/* uint32 [K]: view of each sorted pair */
  GS_BUF_ALPHA_SUM = 12,/* float  [P]: sum of the alphas each pixel blended (soft Gaussian count) */
  GS_BUF_EVALS = 13,    /* uint32 [P]: Gaussians each pixel evaluated up to its termination (after
                           gs_render_count; size 0 before it) */
  GS_BUF_PAIRS_EFF = 14,/* uint32 [tiles]: entries of each tile's list that at least one of the
                           tile's pixels blended (after gs_render_count; size 0 before it) */
  GS_N_BUFS = 15
};

/* Kernel ids for gs_profile_read. */
enum {
  GS_K_PREPROCESS = 0, GS_K_DEPTH_SORT = 1, GS_K_SCAN = 2, GS_K_EMIT = 3, GS_K_TILE_SORT = 4,
  GS_K_RANGES = 5, GS_K_RENDER_FWD = 6, GS_K_LOSS = 7, GS_K_RENDER_BWD = 8,
  GS_K_PREPROCESS_BWD = 9, GS_K_ADAM = 10, GS_K_ZERO = 11, GS_K_LOAD = 12, GS_K_BWD_ADAM = 13,
  GS_N_KERNELS = 14
};

int32_t gs_abi_version(void);

/* Create a context bound to HIP device `device`.  Allocates nothing large.
 * Returns GS_ERR_HIP if the device cannot be used.  *out is NULL on failure. */
gs_status gs_create(gs_ctx** out, int32_t device);
/* Destroy a context after its stream has drained; NULL is a no-op. */
void gs_destroy(gs_ctx* ctx);
/* Message of the last failed call on ctx ("" if none); valid until the next call. */
const char* gs_last_error(const gs_ctx* ctx);

/* Host-only: pixel and tile offsets of each view.  pix_off and tile_off receive
 * n_views + 1 entries (exclusive prefix sums of width*height and of
 * ceil(width/tile)*ceil(height/tile)).  Either may be NULL. */
gs_status gs_layout(const gs_camera* cams, int32_t n_views, int32_t tile, int64_t* pix_off,
                    int64_t* tile_off);

/* Sec. III Eq. 1 and the EWA projection of the original 3DGS (Sec. V-A): for each
 * view of `cams` (host array, 1..GS_MAX_VIEWS views) and each Gaussian: camera
 * transform, near cull (depth <= 0.2), pinhole projection, 2D covariance
 * J W Sigma W^T J^T + 0.3 I (Jacobian clamped at 1.3x the half field of view),
 * conic, extent 3 sqrt(lambda_max), tile rect (tile x tile pixels), cutoff
 * exponent tau = max(-4.5, -ln(255 o)) and the view-dependent SH colour
 * max(0, sum_k f_k Y_k(dir) + 1/2).  Depth, screen position, covariance and
 * extent are evaluated in IEEE FP64 in a fixed order.  params: device, read only.
 * tile: 8, 16 or 32 (others return GS_ERR_UNSUPPORTED).  Errors: GS_ERR_INVALID for
 * null or misaligned params, n < 1, stride < n, sh_degree outside 0..3, n_views
 * outside 1..GS_MAX_VIEWS, non-positive or oversized images, non-finite or
 * non-positive focal lengths; GS_ERR_CAPACITY if n_views * n >= 2^31. */
gs_status gs_preprocess(gs_ctx* ctx, const float* params, int32_t n, int32_t stride, int32_t sh_degree,
                        const gs_camera* cams, int32_t n_views, int32_t tile, gs_stream stream);

/* Per-tile depth-ordered lists (tile rasterizer of the original 3DGS): one pair
 * per (visible Gaussian, tile of its rect; see gs_set_cull), ordered by ascending
 * (global tile, fp32 depth, Gaussian index), and each tile's [start, end) range.
 * Reads the parameter array of the last gs_preprocess (unchanged since) when the
 * fp32 cutoff test cannot decide a pair (see gs_set_cull).
 * n_pairs_out not NULL: waits for the stream once to learn the pair count K and
 * writes it there (GS_ERR_CAPACITY if K >= 2^32).  n_pairs_out NULL: does not wait
 * (except on a context's first binning, which sizes the pair buffers): K stays on
 * the device, and if it exceeds the pair buffers (or 2^32 - 1) the kernels of this
 * binning and of the rendering after it do nothing, gs_adam_step and
 * gs_render_bwd_adam leave every buffer untouched, and gs_sync_status reports
 * GS_ERR_CAPACITY with the size needed; the next gs_bin_sort grows the buffers to
 * it (it also learns of the failure without gs_sync_status once the stream has
 * passed it). */
gs_status gs_bin_sort(gs_ctx* ctx, int64_t* n_pairs_out, gs_stream stream);

/* Device-side conditions of the last gs_bin_sort, which the kernels record
 * without stopping the host: waits for `stream`, then returns GS_OK or the error
 * the kernels recorded (GS_ERR_CAPACITY: the pair buffers, or the store of exact
 * cutoff outcomes, were too small; gs_last_error names the sizes needed).  The
 * failed step's images, gradients and pair lists are void; the next gs_bin_sort
 * sizes the buffers to fit. */
gs_status gs_sync_status(gs_ctx* ctx, gs_stream stream);

/* Sizes the pair buffers for exactly n_pairs pairs (at least 1), so that later
 * gs_bin_sort calls need not wait for the device to size them; a binning with more
 * pairs fails as described at gs_bin_sort.  Waits for `stream` before freeing the
 * old buffers. */
gs_status gs_reserve_pairs(gs_ctx* ctx, int64_t n_pairs, gs_stream stream);

/* Sec. III Eq. 2: front-to-back alpha blending of every pixel of every view.  Per
 * pixel, in list order: skip Gaussians whose exponent is > 0 or < tau,
 * alpha = min(0.99, o exp(exponent)), stop before blending once the
 * transmittance would fall below 1e-4.  Writes the image (layout above) to
 * `color` (device, 3P floats) and keeps the final transmittance, blend count and
 * last position per pixel in the context for gs_render_bwd. */
gs_status gs_render_fwd(gs_ctx* ctx, float* color, gs_stream stream);

/* Eq. 10 image terms: per view, w_l1 * mean|C - T| + w_dssim * (1 - SSIM(C, T))
 * with SSIM over a normalised 11x11 Gaussian window (sigma 1.5, zero padding),
 * C1 = 0.01^2, C2 = 0.03^2, averaged over pixels and channels.  color, target:
 * device images (layout above).  loss_out: device, n_views doubles (per-view
 * loss), may be NULL.  dL_dcolor: device image receiving dL/dcolor of the sum of
 * the per-view losses (sign(0) = 0 for the L1 term). */
gs_status gs_loss(gs_ctx* ctx, const float* color, const float* target, float w_l1, float w_dssim,
                  double* loss_out, float* dL_dcolor, gs_stream stream);

/* gs_loss for callers that cannot allocate device memory (code under HIP graph
 * capture, serving loops and harnesses that forbid allocation): the same
 * computation, arguments and results, with the per-tile loss sums in a static
 * device array of the library (1 MiB per GPU, held until the process ends) instead
 * of context memory; it calls no allocating routine.  Limit: at most 65536 32x32
 * loss tiles summed over the context's views (ceil(W/32) ceil(H/32) per view,
 * about 67 Mpix); beyond it GS_ERR_CAPACITY and nothing is queued.  Every call on
 * one GPU shares that array, from any context or stream: calls that overlap on a
 * GPU race and must be ordered by the caller.  Nothing in it needs clearing (each
 * call writes every tile's sums before reading them). */
gs_status gs_loss_noalloc(gs_ctx* ctx, const float* color, const float* target, float w_l1, float w_dssim,
                          double* loss_out, float* dL_dcolor, gs_stream stream);

/* Eq. 9 load-balancing term: per view, w_load * std over the view's pixels of G_p,
 * the number of Gaussians associated with pixel p, read as the soft count
 * G_p = sum of the alphas p blended (written by gs_render_fwd; a count has no
 * derivative), std the population standard deviation.  loss_out: device, n_views
 * doubles (per-view term), may be NULL.  Also stores dL/dG_p =
 * w_load (G_p - mean) / (P_v std) (0 when std = 0) in the context: the next
 * gs_render_bwd of the same forward adds it to the derivative of every blended
 * alpha (on top of dL_dcolor's terms).  w_load = 0 clears it.  A gs_render_fwd
 * discards it. */
gs_status gs_load_balance(gs_ctx* ctx, float w_load, double* loss_out, gs_stream stream);

/* Reverse-order backward of gs_render_fwd and gs_preprocess (Sec. IV-E): per
 * tile, pixels walk their lists back to front; per-Gaussian partial gradients
 * are reduced across each wavefront and workgroup before one global atomic per
 * (tile, Gaussian, component) ("splatting-based" accumulation), then one thread
 * per Gaussian applies the chain rule through projection, covariance, activations
 * and SH over all views.  params: the same device array as in gs_preprocess,
 * unchanged since.  dL_dcolor: device image.  grad: device, parameter layout;
 * overwritten (accumulate = 0) or added to (accumulate = 1).  A capped alpha and a
 * colour clamped at 0 have zero derivative. */
gs_status gs_render_bwd(gs_ctx* ctx, const float* params, const float* dL_dcolor, float* grad,
                        int32_t accumulate, gs_stream stream);

/* Adam step of the original 3DGS (Sec. V-A) with a learning rate per view
 * (Sec. IV-D, Eq. 6-8).  Dense over all n Gaussians: per element
 * m = b1 m + (1-b1) g, v = b2 v + (1-b2) g^2, k = step[i] + 1,
 * p -= lr (m / (1 - b1^k)) / (sqrt(v / (1 - b2^k)) + eps); step[i] += 1.
 * lr = lr_group[group of the row] (host, GS_N_GROUPS floats), multiplied for the
 * groups in group_mask by the mean of view_lr_scale[v] (host, n_views floats)
 * over the views of the last gs_preprocess in which Gaussian i is visible (over
 * all views when none).  n_views = 0 or view_lr_scale = NULL: no view factor.
 * params, grad, m, v: device, parameter layout; step: device uint32 [n].  When
 * n_views > 0 the context's last gs_preprocess must have used the same n. */
gs_status gs_adam_step(gs_ctx* ctx, float* params, const float* grad, float* m, float* v, uint32_t* step,
                       int32_t n, int32_t stride, int32_t sh_degree, const float* lr_group,
                       const float* view_lr_scale, int32_t n_views, uint32_t group_mask, float beta1,
                       float beta2, float eps, gs_stream stream);

/* One training step's backward and optimizer step in one pass (Sec. IV-E backward,
 * Sec. IV-D / V-A Adam): the same arithmetic as gs_render_bwd(ctx, params,
 * dL_dcolor, grad, 0) followed by gs_adam_step(ctx, params, grad, m, v, step, n,
 * stride, sh_degree, ...) with the n, stride and sh_degree of the last
 * gs_preprocess, but the parameter gradient of each Gaussian is applied as soon as
 * it is formed instead of going through memory.  (In the default GS_BWD_ATOMIC
 * order the backward's 2D gradients are summed with floating-point atomics across
 * tiles, whose order is not fixed, so repeated backward passes, fused or not,
 * agree to rounding, not bit for bit; GS_BWD_ORDERED makes them bit for bit, see
 * gs_set_backward_order.)  grad: device, parameter
 * layout, receives the gradient when not NULL (may be NULL).  params is updated
 * in place; it must be the array the last gs_preprocess read.  Other arguments and
 * errors as for gs_render_bwd and gs_adam_step (n_views > 0 with view_lr_scale
 * needs n_views equal to the last gs_preprocess's). */
gs_status gs_render_bwd_adam(gs_ctx* ctx, float* params, const float* dL_dcolor, float* grad, float* m, float* v,
                             uint32_t* step, const float* lr_group, const float* view_lr_scale, int32_t n_views,
                             uint32_t group_mask, float beta1, float beta2, float eps, gs_stream stream);

/* Pair culling of gs_bin_sort.  GS_CULL_RECT lists every tile of a Gaussian's tile
 * rect.  GS_CULL_ELLIPSE (the default) lists a tile only if the Gaussian's cutoff
 * region {a dx^2 + 2 b dx dy + c dy^2 <= -2 tau} meets the box spanned by the
 * tile's pixel centres, decided on the FP64 centre, conic and cutoff of the
 * projection (an fp32 test decides where the outcome is clear by a margin; the
 * rest, a few in 10^4, recompute the FP64 values from the parameters); the other
 * pairs of the rect can blend into no pixel of their tile, so images and
 * gradients are the same in both modes.  K (and every pair buffer) then counts
 * only the listed pairs.  GS_CULL_ELLIPSE_EXACT lists the same pairs with every
 * test taken on the recomputed FP64 values (slower; for checking the fp32 path).
 * Takes effect at the next gs_bin_sort. */
enum { GS_CULL_RECT = 0, GS_CULL_ELLIPSE = 1, GS_CULL_ELLIPSE_EXACT = 2 };
gs_status gs_set_cull(gs_ctx* ctx, int32_t mode);

/* Summation order of the per-Gaussian 2D gradients in gs_render_bwd and
 * gs_render_bwd_adam (the splat-level accumulation of Sec. IV-E).
 * GS_BWD_ATOMIC (the default): each (tile, Gaussian) partial sum is added with a
 * floating-point atomic, in whatever order the tiles finish.  GS_BWD_ORDERED:
 * each partial is written to its own slot (the partials themselves are formed in
 * a fixed order: per-wave reductions, then the waves in order), the pairs are
 * sorted by Gaussian (stably, so tile order is kept) and each Gaussian's partials
 * are summed in tile order: the gradients, and the parameters an Adam step makes
 * of them, are the same bits on every run and on every device load, which makes
 * it the reference for checking the atomic path for races (the two differ by
 * rounding only).  Costs 36 B per pair of extra memory, a sort of the pairs and a
 * gather (several times the atomic backward's time).  Returns GS_ERR_INVALID for
 * an unknown mode; takes effect at the next backward. */
enum { GS_BWD_ATOMIC = 0, GS_BWD_ORDERED = 1 };
gs_status gs_set_backward_order(gs_ctx* ctx, int32_t mode);

/* Size in bytes of a context buffer (GS_BUF_*) for the current state. */
gs_status gs_buffer_size(const gs_ctx* ctx, int32_t which, size_t* bytes);
/* Stream-ordered copy of a context buffer into device memory `dst` of `bytes`
 * bytes (must equal gs_buffer_size).  GS_BUF_KEYS is composed on the fly. */
gs_status gs_copy_buffer(gs_ctx* ctx, int32_t which, void* dst, size_t bytes, gs_stream stream);

/* Per-kernel timing with HIP events on the launching stream.  enable = 1 starts
 * recording (and clears earlier records), 0 stops.  gs_profile_read synchronises
 * the device and returns the launch count and summed duration (ms) of kernel id
 * `kernel` (GS_K_*) since the last enable. */
gs_status gs_profile_enable(gs_ctx* ctx, int32_t enable);
gs_status gs_profile_read(gs_ctx* ctx, int32_t kernel, int64_t* launches, double* total_ms);

/* Work count of the forward for rooflines (Sec. III Eq. 2): walks the lists of the
 * last gs_bin_sort exactly as gs_render_fwd does and stores, per pixel, the number
 * of Gaussians that pass its cutoff test before it stops (the blended ones plus,
 * for a pixel that stopped, the one that would have taken its transmittance below
 * 1e-4), readable as GS_BUF_EVALS.  This count depends on no tile edge.  It
 * also stores, per tile, how many entries of its list at least one of its pixels
 * blended (GS_BUF_PAIRS_EFF: the (tile, Gaussian) pairs whose partial gradient the
 * backward adds with atomics).  The forward state (images, transmittances,
 * counts) is left as it was. */
gs_status gs_render_count(gs_ctx* ctx, gs_stream stream);

/* Measurement probes (no context).  gs_probe_copy copies `bytes` (a multiple of
 * 16; both pointers 16-byte aligned, device memory, not overlapping) with a plain
 * streaming kernel: its rate (2 x bytes / time) is the achievable HBM bandwidth the
 * HBM-bound stages are compared with.  gs_probe_fma runs `blocks` x 256 threads of
 * eight independent fp32 FMA chains of `iters` steps each, built like the library's
 * other kernels (packed fp32 off), and writes one float per thread to `out` (device,
 * blocks x 256 floats); *flops (may be NULL) receives its flop count (2 per FMA).
 * Both are stream-ordered; the caller times them. */
gs_status gs_probe_copy(const void* src, void* dst, size_t bytes, gs_stream stream);
gs_status gs_probe_fma(float* out, int32_t blocks, int32_t iters, int64_t* flops, gs_stream stream);

/* Device memory (bytes) held by the context's own buffers right now. */
gs_status gs_memory_bytes(const gs_ctx* ctx, size_t* bytes);

/* ---- Host-only schedule of progressive training (no device work, no context) ----
 * Images are numbered 0..n-1.  overlap: host FP64 [n][n] row-major, entry (i, j)
 * the overlap degree of images i and j normalised to [0, 1] (0 = no overlap; the
 * diagonal is ignored).  Negative or non-finite entries give GS_ERR_INVALID. */

/* Sec. IV-C, Eq. 3-4: hierarchical weights for the newly added image new_image.
 * The new image has weight 1 (layer 1).  Layer k >= 2 holds the images not in an
 * earlier layer that overlap some image of layer k-1; each gets the mean over
 * layer k-1 of (that image's weight x overlap), which for layer 2 is Eq. 3's
 * overlap with the new image.  weights: host FP64 [n] out, -1 for images no layer
 * reaches.  layer: host int32 [n] out (1 = new image, 0 = unreached), may be NULL. */
gs_status gs_sched_weights(const double* overlap, int32_t n, int32_t new_image, double* weights,
                           int32_t* layer);

/* Sec. IV-C: which image each of the t_i iterations after an arrival trains.
 * Local half (t_i / 2 iterations): the n_m reached images (weight >= 0) of largest
 * weight (ties: smaller index) share it by Eq. 5 in proportion to 1 - exp(-w),
 * rounded by largest remainder (ties: smaller index) to sum exactly to t_i / 2, and
 * are visited round robin in weight order while their share lasts.  Semi-global
 * half (the remaining t_i - t_i / 2): the other images (every image when all are
 * key images) ordered by the caller's uniform draws u (host FP64 [n]; ties by
 * index) and taken cyclically, so counts differ by at most one and more images
 * than iterations means a draw without replacement.  plan: host int32 [t_i] out.
 * local_iters: host int32 [n] out (Eq. 5 share, 0 off the key set), may be NULL. */
gs_status gs_sched_plan(const double* weights, int32_t n, int32_t n_m, int32_t t_i, const double* u,
                        int32_t* plan, int32_t* local_iters);

/* Sec. IV-D, Eq. 6-8: per-image learning rate.  trained: host int64 [n],
 * iterations image j has been trained so far.  Eq. 7 progress t = min(1, T_j/t_a);
 * Eq. 6 current rate exp(ln(eta0)(1 - t) + ln(etaf) t) -> lr_current (host FP64
 * [n], may be NULL); Eq. 8 rate (own rate + sum over overlapping images i of
 * overlap(i, j) x their rate) / (their count + 1) -> lr (host FP64 [n]).
 * GS_ERR_INVALID for non-positive rates or t_a, or negative counts. */
gs_status gs_sched_lr(const int64_t* trained, const double* overlap, int32_t n, double eta0, double etaf,
                      double t_a, double* lr_current, double* lr);

#ifdef __cplusplus
}
#endif
#endif /* GS_H_ */
