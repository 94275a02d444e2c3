// Image loss terms of Eq. 10 and dL/dimage for gfx950.
//
// Per view: w_l1 * mean|x - y| + w_dssim * (1 - mean SSIM(x, y)), SSIM per channel
// from windowed means under a normalised 11x11 Gaussian window (sigma 1.5, zero
// padding), C1 = 0.01^2, C2 = 0.03^2.  All views share one launch of 32x32-pixel
// output tiles (256 threads); the separable window runs in two register-blocked
// passes per map (a thread filters a run of consecutive columns of a row, then a
// run of rows of a column), one map at a time through LDS.  E[x^2] and E[y^2]
// enter SSIM only through their sum (in D2), so four maps are filtered: x, y,
// x^2 + y^2 and xy.
//
// Backward: with N1 = 2 mx my + C1, N2 = 2 sxy + C2, D1 = mx^2 + my^2 + C1,
// D2 = sxx + syy + C2 and S = N1 N2 / (D1 D2), the per-pixel partials of S with
// respect to the windowed statistics (mx, E[x^2], E[xy]) are
//   A = 2 my (N2 - N1) / (D1 D2) + 2 mx S (1/D2 - 1/D1),  B = -S / D2,
//   Cc = 2 N1 / (D1 D2),
// and dS_mean/dx = (window * A + 2 x (window * B) + y (window * Cc)) / N, with 1/D1
// and 1/D2 taken once per pixel from the hardware reciprocal.
//
// Two forms of the SSIM term:
// * gs_loss: k_ssim_fwd forms the statistics over each tile (a 42x42 halo staged)
//   and stores A, B, Cc (36 B per pixel); k_ssim_bwd filters them the same way (the
//   window is symmetric) and adds the L1 term.
// * gs_loss_noalloc: k_ssim_fused does both per tile with nothing but the images,
//   the gradient and the per-tile sums in HBM: it stages the 52x52 patch that
//   reaches the tile through two windows, forms the statistics over the 42x42
//   region whose SSIM terms reach the tile, turns them into A, B, Cc there in the
//   LDS the patch occupied, and filters those over the tile.  About a third of the
//   HBM traffic, 1.4x the filtering work (the 42x42 region is recomputed by
//   neighbouring tiles); the kernel is bound by instruction issue, so on this chip
//   it is the slower of the two (0.57 against 0.45 ms at 10 Mpix).
// Loss sums are reduced per tile in FP64.
//
// The load-balancing term of Eq. 9 (kernels at the end) works on the soft
// per-pixel Gaussian count the forward writes.
#include "gs_internal.h"

namespace gsk {
namespace {

constexpr int LT = 32;              // output tile edge
constexpr int R = 5;                // window radius
constexpr int TAPS = 2 * R + 1;
constexpr int HALO = LT + 2 * R;    // 42
constexpr int HS = HALO;            // LDS row stride (unpadded: the backward then fits six workgroups per CU)
constexpr int HSEG = 8;             // horizontal outputs per thread
constexpr int VSEG = 4;             // vertical outputs per thread
constexpr int IN = LT + 4 * R;      // 52: the fused kernel's patch (two windows around the tile)
constexpr int FVSEG = 7;            // vertical outputs per thread of its 42-high forward maps
constexpr int FTASKS = HALO * (HALO / FVSEG);   // 252 threads hold its forward statistics
constexpr float kC1 = 0.01f * 0.01f;
constexpr float kC2 = 0.03f * 0.03f;

struct Win {
  float w[TAPS];
};

// global 32-tile offset of each view (n_views + 1 entries)
struct LossTiles {
  int32_t off[GS_MAX_VIEWS + 1];
};

__device__ inline double block_sum_d(double x, double* sh) {
  for (int o = 32; o > 0; o >>= 1) x += __shfl_xor(x, o);
  if (__lane_id() == 0) sh[threadIdx.x / 64] = x;
  __syncthreads();
  double t = 0.0;
  for (int w = 0; w < (int)(blockDim.x / 64); ++w) t += sh[w];
  __syncthreads();
  return t;
}

struct TileLoc {
  int v, x0, y0;
};

// Workgroups are dealt to the chip's 8 XCDs round-robin (workgroup b runs on XCD
// b mod 8), each XCD with its own L2.  Workgroup b takes tile (b mod 8) * chunk +
// b / 8, so every XCD walks a contiguous range of tiles and the halo rows that
// neighbouring tiles share are fetched into one L2.  Tiles past the end (at most
// 7 workgroups) return at once.
constexpr int kXcds = 8;

__host__ __device__ inline int xcd_tile_chunk(int n_tiles) { return (n_tiles + kXcds - 1) / kXcds; }

__device__ inline int xcd_tile(int b, int n_tiles) { return (b % kXcds) * xcd_tile_chunk(n_tiles) + b / kXcds; }

__device__ inline TileLoc loss_tile(const ViewDev* __restrict__ views, const LossTiles& lt, int V, int tile) {
  int v = 0;
  while (v + 1 < V && tile >= lt.off[v + 1]) ++v;
  const int nx = (views[v].W + LT - 1) / LT;
  const int local = tile - lt.off[v];
  return TileLoc{v, (local % nx) * LT, (local / nx) * LT};
}

// Stage a HALO x HALO patch of q planes (zero outside the image) into LDS.
template <int Q>
__device__ inline void stage_halo(float (*dst)[HALO * HS], const float* const* src, int W, int H, int x0, int y0) {
  for (int i = threadIdx.x; i < HALO * HALO; i += blockDim.x) {
    const int r = i / HALO, c = i % HALO;
    const int gx = x0 - R + c, gy = y0 - R + r;
    const bool in = gx >= 0 && gx < W && gy >= 0 && gy < H;
    const size_t p = (size_t)gy * W + gx;
#pragma unroll
    for (int q = 0; q < Q; ++q) dst[q][r * HS + c] = in ? src[q][p] : 0.0f;
  }
}

__global__ __launch_bounds__(256) void k_l1(const ViewDev* __restrict__ views, int V, LossTiles lt,
                                             const float* __restrict__ x, const float* __restrict__ y, float w_l1,
                                             float* __restrict__ grad, double2* __restrict__ partials) {
  __shared__ double sh[4];
  const int tile = xcd_tile(blockIdx.x, lt.off[V]);
  if (tile >= lt.off[V]) return;
  const TileLoc t = loss_tile(views, lt, V, tile);
  const ViewDev& cv = views[t.v];
  const size_t hw = (size_t)cv.W * cv.H;
  const size_t base = 3 * (size_t)cv.pix_off;
  const float inv = w_l1 / (float)(3 * hw);
  double s = 0.0;
  for (int i = threadIdx.x; i < LT * LT; i += blockDim.x) {
    const int px = t.x0 + i % LT, py = t.y0 + i / LT;
    if (px >= cv.W || py >= cv.H) continue;
    const size_t p = base + (size_t)py * cv.W + px;
    for (int c = 0; c < 3; ++c) {
      const float d = x[p + c * hw] - y[p + c * hw];
      s += fabs((double)d);
      grad[p + c * hw] = inv * (float)((d > 0.0f) - (d < 0.0f));
    }
  }
  const double tot = block_sum_d(s, sh);
  if (threadIdx.x == 0) partials[tile] = make_double2(tot, 0.0);
}

// Horizontal pass: out[q][r][c] (r < HALO, c < LT) = sum_k w[k] f_q(r, c + k) where the
// Q outputs are formed from the NIN staged inputs by `form`.
template <int NIN, int Q, class F>
__device__ inline void hpass(const float (*in)[HALO * HS], float (*out)[HALO * LT], const Win& win, F form) {
  const int task = threadIdx.x;
  if (task < HALO * (LT / HSEG)) {
    const int r = task / (LT / HSEG), c0 = (task % (LT / HSEG)) * HSEG;
    float acc[Q][HSEG];
#pragma unroll
    for (int q = 0; q < Q; ++q)
#pragma unroll
      for (int j = 0; j < HSEG; ++j) acc[q][j] = 0.0f;
#pragma unroll
    for (int k = 0; k < HSEG + 2 * R; ++k) {
      float v[NIN];
#pragma unroll
      for (int i = 0; i < NIN; ++i) v[i] = in[i][r * HS + c0 + k];
      float f[Q];
      form(v, f);
#pragma unroll
      for (int j = 0; j < HSEG; ++j) {
        const int tap = k - j;
        if (tap >= 0 && tap < TAPS) {
#pragma unroll
          for (int q = 0; q < Q; ++q) acc[q][j] = __fmaf_rn(win.w[tap], f[q], acc[q][j]);
        }
      }
    }
#pragma unroll
    for (int q = 0; q < Q; ++q)
#pragma unroll
      for (int j = 0; j < HSEG; ++j) out[q][r * LT + c0 + j] = acc[q][j];
  }
}

// Vertical pass for this thread's 4 output rows of one column.
template <int Q>
__device__ inline void vpass(const float (*in)[HALO * LT], const Win& win, int col, int r0, float (&res)[Q][VSEG]) {
#pragma unroll
  for (int q = 0; q < Q; ++q)
#pragma unroll
    for (int j = 0; j < VSEG; ++j) res[q][j] = 0.0f;
#pragma unroll
  for (int k = 0; k < VSEG + 2 * R; ++k) {
#pragma unroll
    for (int q = 0; q < Q; ++q) {
      const float f = in[q][(r0 + k) * LT + col];
#pragma unroll
      for (int j = 0; j < VSEG; ++j) {
        const int tap = k - j;
        if (tap >= 0 && tap < TAPS) res[q][j] = __fmaf_rn(win.w[tap], f, res[q][j]);
      }
    }
  }
}

// One windowed map of the staged planes (form makes its value from theirs) for
// this thread's VSEG outputs; the workgroup's LDS map buffer is free again on return.
template <int NIN, class F>
__device__ inline void window_map(const float (*in)[HALO * HS], float (*hb)[HALO * LT], const Win& win, int col,
                                  int r0, F form, float (&res)[VSEG]) {
  hpass<NIN, 1>(in, hb, win, form);
  __syncthreads();
  float mq[1][VSEG];
  vpass<1>(hb, win, col, r0, mq);
  // the sums are formed here: left alone, the compiler sinks them into the
  // per-pixel branches at the end and keeps every loaded tap live until then
#pragma unroll
  for (int j = 0; j < VSEG; ++j) {
    res[j] = mq[0][j];
    asm volatile("" : "+v"(res[j]));
  }
  __syncthreads();
}

// Register budgets: 8 waves per SIMD for the forward (59 VGPRs; left alone the
// compiler takes 68 and runs 7), 6 for the backward (its LDS allows 6 workgroups).
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(8))) void k_ssim_fwd(const ViewDev* __restrict__ views, int V, LossTiles lt,
                                                   const float* __restrict__ x, const float* __restrict__ y,
                                                   float* __restrict__ aux, Win win, double2* __restrict__ partials) {
  __shared__ float sin_[2][HALO * HS];
  __shared__ float hbuf[1][HALO * LT];   // the four maps one after another: 20 KB of LDS
  __shared__ double sh[4];
  const int tile = xcd_tile(blockIdx.x, lt.off[V]);
  if (tile >= lt.off[V]) return;
  const TileLoc t = loss_tile(views, lt, V, tile);
  const ViewDev& cv = views[t.v];
  const size_t hw = (size_t)cv.W * cv.H;
  const size_t base = 3 * (size_t)cv.pix_off;
  const int col = threadIdx.x % LT, r0 = (threadIdx.x / LT) * VSEG;
  double sl1 = 0.0, sss = 0.0;
  for (int ch = 0; ch < 3; ++ch) {
    const float* src[2] = {x + base + ch * hw, y + base + ch * hw};
    stage_halo<2>(sin_, src, cv.W, cv.H, t.x0, t.y0);
    __syncthreads();
    float m[4][VSEG];
    window_map<2>(sin_, hbuf, win, col, r0, [](const float* v, float* f) { f[0] = v[0]; }, m[0]);
    window_map<2>(sin_, hbuf, win, col, r0, [](const float* v, float* f) { f[0] = v[1]; }, m[1]);
    window_map<2>(sin_, hbuf, win, col, r0,
                  [](const float* v, float* f) { f[0] = __fmaf_rn(v[0], v[0], v[1] * v[1]); }, m[2]);
    window_map<2>(sin_, hbuf, win, col, r0, [](const float* v, float* f) { f[0] = v[0] * v[1]; }, m[3]);
    float* ac = aux + (size_t)cv.pix_off * 9 + (size_t)ch * 3 * hw;
#pragma unroll
    for (int j = 0; j < VSEG; ++j) {
      const int px = t.x0 + col, py = t.y0 + r0 + j;
      if (px < cv.W && py < cv.H) {
        const float mx = m[0][j], my = m[1][j];
        const float sxy = m[3][j] - mx * my;
        const float N1 = 2.0f * mx * my + kC1, N2 = 2.0f * sxy + kC2;
        const float M2 = mx * mx + my * my;
        const float D1 = M2 + kC1, D2 = (m[2][j] - M2) + kC2;
        // hardware reciprocals (1 ulp): D1, D2 >= C1 > 0
        const float r1 = __builtin_amdgcn_rcpf(D1), r2 = __builtin_amdgcn_rcpf(D2);
        const float rden = r1 * r2;
        const float S = (N1 * N2) * rden;
        const size_t p = (size_t)py * cv.W + px;
        ac[p] = 2.0f * my * (N2 - N1) * rden + 2.0f * mx * S * (r2 - r1);
        ac[p + hw] = -S * r2;
        ac[p + 2 * hw] = 2.0f * N1 * rden;
        const float xv = sin_[0][(r0 + j + R) * HS + col + R];
        const float yv = sin_[1][(r0 + j + R) * HS + col + R];
        sl1 += fabs((double)(xv - yv));
        sss += (double)S;
      }
    }
    __syncthreads();
  }
  const double t1 = block_sum_d(sl1, sh);
  const double t2 = block_sum_d(sss, sh);
  if (threadIdx.x == 0) partials[tile] = make_double2(t1, t2);
}

__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(6))) void k_ssim_bwd(const ViewDev* __restrict__ views, int V, LossTiles lt,
                                                   const float* __restrict__ x, const float* __restrict__ y,
                                                   const float* __restrict__ aux, Win win, float w_l1, float w_dssim,
                                                   float* __restrict__ grad) {
  __shared__ float sin_[3][HALO * HS];
  __shared__ float hbuf[1][HALO * LT];   // the three maps filtered one after another: 26 KB of LDS
  const int tile = xcd_tile(blockIdx.x, lt.off[V]);
  if (tile >= lt.off[V]) return;
  const TileLoc t = loss_tile(views, lt, V, tile);
  const ViewDev& cv = views[t.v];
  const size_t hw = (size_t)cv.W * cv.H;
  const size_t base = 3 * (size_t)cv.pix_off;
  const float invN = 1.0f / (float)(3 * hw);
  const int col = threadIdx.x % LT, r0 = (threadIdx.x / LT) * VSEG;
  for (int ch = 0; ch < 3; ++ch) {
    const float* ac = aux + (size_t)cv.pix_off * 9 + (size_t)ch * 3 * hw;
    const float* src[3] = {ac, ac + hw, ac + 2 * hw};
    stage_halo<3>(sin_, src, cv.W, cv.H, t.x0, t.y0);
    // this thread's image values, fetched now so the loads overlap the filtering
    float xs[VSEG], ys[VSEG];
#pragma unroll
    for (int j = 0; j < VSEG; ++j) {
      const int px = t.x0 + col, py = t.y0 + r0 + j;
      const bool in = px < cv.W && py < cv.H;
      const size_t p = base + ch * hw + (size_t)py * cv.W + px;
      xs[j] = in ? x[p] : 0.0f;
      ys[j] = in ? y[p] : 0.0f;
    }
    __syncthreads();
    float m[3][VSEG];
#pragma unroll
    for (int q = 0; q < 3; ++q)
      window_map<1>(sin_ + q, hbuf, win, col, r0, [](const float* v, float* f) { f[0] = v[0]; }, m[q]);
#pragma unroll
    for (int j = 0; j < VSEG; ++j) {
      const int px = t.x0 + col, py = t.y0 + r0 + j;
      if (px < cv.W && py < cv.H) {
        const size_t p = base + ch * hw + (size_t)py * cv.W + px;
        const float xv = xs[j], yv = ys[j];
        const float d = xv - yv;
        const float l1 = w_l1 * invN * (float)((d > 0.0f) - (d < 0.0f));
        grad[p] = l1 - w_dssim * invN * (m[0][j] + 2.0f * xv * m[1][j] + yv * m[2][j]);
      }
    }
    __syncthreads();
  }
}

// ---- fused SSIM (gs_loss_noalloc) ----

// Horizontal pass over ROWS rows of one or two staged planes (row stride IS) into
// an OW-wide map (row stride OW): out(r, c) = sum_k w[k] form(in0, in1)(r, c + k).
// A thread filters SEG consecutive columns of one row; a row's tasks start at
// min(s SEG, OW - SEG), so the last may repeat columns of the one before it, with
// bit-identical values (same operations in the same order).
template <int ROWS, int IS, int OW, int SEG, class F>
__device__ inline void row_pass(const float* in0, const float* in1, float* out, const Win& win, F form) {
  constexpr int NSEG = (OW + SEG - 1) / SEG;
  static_assert(ROWS * NSEG <= 256, "one task per thread");
  const int task = threadIdx.x;
  if (task < ROWS * NSEG) {
    const int r = task / NSEG, s = task % NSEG;
    const int c0 = min(s * SEG, OW - SEG);
    float acc[SEG];
#pragma unroll
    for (int j = 0; j < SEG; ++j) acc[j] = 0.0f;
#pragma unroll
    for (int k = 0; k < SEG + 2 * R; ++k) {
      const int q = r * IS + c0 + k;
      const float f = form(in0[q], in1 ? in1[q] : 0.0f);
#pragma unroll
      for (int j = 0; j < SEG; ++j) {
        const int tap = k - j;
        if (tap >= 0 && tap < TAPS) acc[j] = __fmaf_rn(win.w[tap], f, acc[j]);
      }
    }
#pragma unroll
    for (int j = 0; j < SEG; ++j) out[r * OW + c0 + j] = acc[j];
  }
}

// Vertical pass of an OW-wide half-filtered map for SEG consecutive rows of one
// column (rows r0 .. r0 + SEG - 1 of the result; input rows r0 .. r0 + SEG + 9).
template <int OW, int SEG>
__device__ inline void col_pass(const float* hb, const Win& win, int col, int r0, bool active, float (&res)[SEG]) {
#pragma unroll
  for (int j = 0; j < SEG; ++j) res[j] = 0.0f;
  if (!active) return;
#pragma unroll
  for (int k = 0; k < SEG + 2 * R; ++k) {
    const float f = hb[(r0 + k) * OW + col];
#pragma unroll
    for (int j = 0; j < SEG; ++j) {
      const int tap = k - j;
      if (tap >= 0 && tap < TAPS) res[j] = __fmaf_rn(win.w[tap], f, res[j]);
    }
  }
}

// The sums are formed where they are pinned (see window_map).
template <int N>
__device__ inline void pin(float (&res)[N]) {
#pragma unroll
  for (int j = 0; j < N; ++j) asm volatile("" : "+v"(res[j]));
}

// Forward statistics: maps of the 52x52 patch over the 42x42 region (rows in runs
// of FHSEG = 11: 208 row tasks; columns in runs of FVSEG = 7: 252 threads).
// Backward: maps of the 42x42 A, B, Cc planes over the 32x32 tile (runs of 6: 252
// row tasks; runs of VSEG = 4 rows: all 256 threads).
constexpr int FHRUN = 11;
constexpr int BHRUN = 6;

__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(4))) void k_ssim_fused(const ViewDev* __restrict__ views, int V, LossTiles lt,
                                               const float* __restrict__ x, const float* __restrict__ y, Win win,
                                               float w_l1, float w_dssim, float* __restrict__ grad,
                                               double2* __restrict__ partials) {
  // the staged patch (two 52x52 planes), later the A, B, Cc planes of the 42x42
  // region; two half-filtered maps (one is filled while the other is read, one
  // barrier per map): 39 KB of LDS, four workgroups per CU
  __shared__ float sp[2 * IN * IN];
  __shared__ float hb[2][IN * HALO];
  __shared__ double sh[4];
  static_assert(3 * HALO * HS <= 2 * IN * IN, "A, B, Cc planes fit where the patch was");
  static_assert(HALO * LT <= IN * HALO, "backward half-filtered maps fit");
  const int tile = xcd_tile(blockIdx.x, lt.off[V]);
  if (tile >= lt.off[V]) return;
  const TileLoc t = loss_tile(views, lt, V, tile);
  const ViewDev& cv = views[t.v];
  const size_t hw = (size_t)cv.W * cv.H;
  const size_t base = 3 * (size_t)cv.pix_off;
  const float invN = 1.0f / (float)(3 * hw);
  // forward statistics: region column fc, rows fr0 .. fr0 + 6 (threads < 252);
  // gradient: tile column col, rows r0 .. r0 + 3
  const int fc = threadIdx.x % HALO, fr0 = (threadIdx.x / HALO) * FVSEG;
  const bool factive = (int)threadIdx.x < FTASKS;
  const int col = threadIdx.x % LT, r0 = (threadIdx.x / LT) * VSEG;
  const float* X = sp;
  const float* Y = sp + IN * IN;
  double sl1 = 0.0, sss = 0.0;
  for (int ch = 0; ch < 3; ++ch) {
    const float* xc = x + base + ch * hw;
    const float* yc = y + base + ch * hw;
    for (int i = threadIdx.x; i < IN * IN; i += blockDim.x) {
      const int r = i / IN, c = i % IN;
      const int gx = t.x0 - 2 * R + c, gy = t.y0 - 2 * R + r;
      const bool in = gx >= 0 && gx < cv.W && gy >= 0 && gy < cv.H;
      const size_t p = (size_t)gy * cv.W + gx;
      sp[i] = in ? xc[p] : 0.0f;
      sp[IN * IN + i] = in ? yc[p] : 0.0f;
    }
    __syncthreads();
    float xs[VSEG], ys[VSEG];
#pragma unroll
    for (int j = 0; j < VSEG; ++j) {
      xs[j] = X[(r0 + j + 2 * R) * IN + col + 2 * R];
      ys[j] = Y[(r0 + j + 2 * R) * IN + col + 2 * R];
    }
    // windowed x, y, x^2 + y^2 (E[x^2] and E[y^2] enter S only through their sum,
    // in D2) and xy; map q's vertical pass runs beside map q + 1's horizontal one
    const auto fx = [](float a, float b) { return a; };
    const auto fy = [](float a, float b) { return b; };
    const auto fss = [](float a, float b) { return __fmaf_rn(a, a, b * b); };
    const auto fxy = [](float a, float b) { return a * b; };
    float m[4][FVSEG];
    row_pass<IN, IN, HALO, FHRUN>(X, Y, hb[0], win, fx);
    __syncthreads();
    col_pass<HALO, FVSEG>(hb[0], win, fc, fr0, factive, m[0]);
    pin(m[0]);
    row_pass<IN, IN, HALO, FHRUN>(X, Y, hb[1], win, fy);
    __syncthreads();
    col_pass<HALO, FVSEG>(hb[1], win, fc, fr0, factive, m[1]);
    pin(m[1]);
    row_pass<IN, IN, HALO, FHRUN>(X, Y, hb[0], win, fss);
    __syncthreads();
    col_pass<HALO, FVSEG>(hb[0], win, fc, fr0, factive, m[2]);
    pin(m[2]);
    row_pass<IN, IN, HALO, FHRUN>(X, Y, hb[1], win, fxy);
    __syncthreads();
    col_pass<HALO, FVSEG>(hb[1], win, fc, fr0, factive, m[3]);
    pin(m[3]);
    // every thread is past its last read of the patch (the barrier before the last
    // vertical pass): A, B, Cc go where it was
    float* pa = sp;
    if (factive) {
#pragma unroll
      for (int j = 0; j < FVSEG; ++j) {
        const int gx = t.x0 - R + fc, gy = t.y0 - R + fr0 + j;
        float A = 0.0f, B = 0.0f, Cc = 0.0f;
        if (gx >= 0 && gx < cv.W && gy >= 0 && gy < cv.H) {
          const float mx = m[0][j], my = m[1][j];
          const float sxy = m[3][j] - mx * my;
          const float N1 = 2.0f * mx * my + kC1, N2 = 2.0f * sxy + kC2;
          const float M2 = mx * mx + my * my;
          const float D1 = M2 + kC1, D2 = (m[2][j] - M2) + kC2;
          // hardware reciprocals (1 ulp): D1, D2 >= C1 > 0
          const float r1 = __builtin_amdgcn_rcpf(D1), r2 = __builtin_amdgcn_rcpf(D2);
          const float rden = r1 * r2;
          const float S = (N1 * N2) * rden;
          A = 2.0f * my * (N2 - N1) * rden + 2.0f * mx * S * (r2 - r1);
          B = -S * r2;
          Cc = 2.0f * N1 * rden;
          const int lx = fc - R, ly = fr0 + j - R;   // inside the tile: its SSIM term is counted here
          if (lx >= 0 && lx < LT && ly >= 0 && ly < LT) sss += (double)S;
        }
        const int q = (fr0 + j) * HS + fc;
        pa[q] = A;
        pa[HALO * HS + q] = B;
        pa[2 * HALO * HS + q] = Cc;
      }
    }
    __syncthreads();
    float g[3][VSEG];
    const auto fid = [](float a, float b) { return a; };
    row_pass<HALO, HS, LT, BHRUN>(pa, nullptr, hb[0], win, fid);
    __syncthreads();
    col_pass<LT, VSEG>(hb[0], win, col, r0, true, g[0]);
    pin(g[0]);
    row_pass<HALO, HS, LT, BHRUN>(pa + HALO * HS, nullptr, hb[1], win, fid);
    __syncthreads();
    col_pass<LT, VSEG>(hb[1], win, col, r0, true, g[1]);
    pin(g[1]);
    row_pass<HALO, HS, LT, BHRUN>(pa + 2 * HALO * HS, nullptr, hb[0], win, fid);
    __syncthreads();
    col_pass<LT, VSEG>(hb[0], win, col, r0, true, g[2]);
    pin(g[2]);
#pragma unroll
    for (int j = 0; j < VSEG; ++j) {
      const int px = t.x0 + col, py = t.y0 + r0 + j;
      if (px < cv.W && py < cv.H) {
        const size_t p = base + ch * hw + (size_t)py * cv.W + px;
        const float xv = xs[j], yv = ys[j];
        const float d = xv - yv;
        sl1 += fabs((double)d);
        const float l1 = w_l1 * invN * (float)((d > 0.0f) - (d < 0.0f));
        grad[p] = l1 - w_dssim * invN * (g[0][j] + 2.0f * xv * g[1][j] + yv * g[2][j]);
      }
    }
  }
  const double t1 = block_sum_d(sl1, sh);
  const double t2 = block_sum_d(sss, sh);
  if (threadIdx.x == 0) partials[tile] = make_double2(t1, t2);
}

// One workgroup per view: the view's tile partials summed in FP64.
__global__ __launch_bounds__(256) void k_loss_final(const ViewDev* __restrict__ views, LossTiles lt,
                                                     const double2* __restrict__ partials, float w_l1,
                                                     float w_dssim, int ssim, double* __restrict__ out) {
  __shared__ double sh[4];
  const int v = blockIdx.x;
  const ViewDev& cv = views[v];
  double a = 0.0, b = 0.0;
  for (int t = lt.off[v] + threadIdx.x; t < lt.off[v + 1]; t += blockDim.x) {
    const double2 pt = partials[t];
    a += pt.x;
    b += pt.y;
  }
  a = block_sum_d(a, sh);
  b = block_sum_d(b, sh);
  if (threadIdx.x == 0) {
    const double N = 3.0 * (double)cv.W * (double)cv.H;
    double l = (double)w_l1 * a / N;
    if (ssim) l += (double)w_dssim * (1.0 - b / N);
    out[v] = l;
  }
}

// ---- Eq. 9 load-balancing term on the soft per-pixel count G_p (sum of the
// alphas a pixel blended, written by the forward): per view, L = w std_p(G_p)
// (population std) and dL/dG_p = w (G_p - mean) / (P std) (0 when std = 0).
// Sums of G and G^2 are taken in FP64 per 2048-pixel chunk, then per view.
constexpr int kLoadChunk = 2048;

__global__ __launch_bounds__(256) void k_load_partial(const ViewDev* __restrict__ views,
                                                      const float* __restrict__ asum, int chunks,
                                                      double2* __restrict__ part) {
  __shared__ double sh[4];
  const ViewDev& cv = views[blockIdx.y];
  const int64_t P = (int64_t)cv.W * cv.H;
  const int64_t base = (int64_t)blockIdx.x * kLoadChunk;
  double a = 0.0, b = 0.0;
  for (int k = 0; k < kLoadChunk / 256; ++k) {
    const int64_t i = base + k * 256 + threadIdx.x;
    if (i < P) {
      const double g = (double)asum[cv.pix_off + i];
      a += g;
      b += g * g;
    }
  }
  a = block_sum_d(a, sh);
  b = block_sum_d(b, sh);
  if (threadIdx.x == 0) part[(size_t)blockIdx.y * chunks + blockIdx.x] = make_double2(a, b);
}

__global__ __launch_bounds__(256) void k_load_final(const ViewDev* __restrict__ views, int chunks,
                                                    const double2* __restrict__ part, float w,
                                                    double2* __restrict__ stats, double* __restrict__ loss_out) {
  __shared__ double sh[4];
  const int v = blockIdx.x;
  const ViewDev& cv = views[v];
  const int64_t P = (int64_t)cv.W * cv.H;
  const int nc = (int)((P + kLoadChunk - 1) / kLoadChunk);
  double a = 0.0, b = 0.0;
  for (int t = threadIdx.x; t < nc; t += blockDim.x) {
    a += part[(size_t)v * chunks + t].x;
    b += part[(size_t)v * chunks + t].y;
  }
  a = block_sum_d(a, sh);
  b = block_sum_d(b, sh);
  if (threadIdx.x == 0) {
    const double m = a / (double)P;
    const double var = fmax(b / (double)P - m * m, 0.0);
    const double sd = sqrt(var);
    stats[v] = make_double2(m, sd > 0.0 ? (double)w / ((double)P * sd) : 0.0);
    if (loss_out) loss_out[v] = (double)w * sd;
  }
}

__global__ __launch_bounds__(256) void k_load_grad(const ViewDev* __restrict__ views,
                                                   const double2* __restrict__ stats,
                                                   const float* __restrict__ asum, float* __restrict__ dG) {
  const ViewDev& cv = views[blockIdx.y];
  const int64_t P = (int64_t)cv.W * cv.H;
  const double2 st = stats[blockIdx.y];
  const int64_t base = (int64_t)blockIdx.x * kLoadChunk;
  for (int k = 0; k < kLoadChunk / 256; ++k) {
    const int64_t i = base + k * 256 + threadIdx.x;
    if (i < P) dG[cv.pix_off + i] = (float)(((double)asum[cv.pix_off + i] - st.x) * st.y);
  }
}

}  // namespace

int load_chunks(const ViewDev* hviews, int V) {
  int64_t mx = 1;
  for (int v = 0; v < V; ++v) {
    const int64_t c = ((int64_t)hviews[v].W * hviews[v].H + kLoadChunk - 1) / kLoadChunk;
    mx = c > mx ? c : mx;
  }
  return (int)mx;
}

hipError_t launch_load_balance(const ViewDev* dviews, const ViewDev* hviews, int V, const float* asum, float w,
                               double* partials, double* stats, double* loss_out, float* dG, hipStream_t s) {
  const int chunks = load_chunks(hviews, V);
  double2* part = reinterpret_cast<double2*>(partials);
  double2* st = reinterpret_cast<double2*>(stats);
  hipLaunchKernelGGL(k_load_partial, dim3(chunks, V), dim3(256), 0, s, dviews, asum, chunks, part);
  hipLaunchKernelGGL(k_load_final, dim3(V), dim3(256), 0, s, dviews, chunks, part, w, st, loss_out);
  hipLaunchKernelGGL(k_load_grad, dim3(chunks, V), dim3(256), 0, s, dviews, st, asum, dG);
  return hipGetLastError();
}

int loss_tiles(const ViewDev* hviews, int V) {
  int t = 0;
  for (int v = 0; v < V; ++v) t += ((hviews[v].W + LT - 1) / LT) * ((hviews[v].H + LT - 1) / LT);
  return t;
}

hipError_t launch_loss_dev(const ViewDev* dviews, const ViewDev* hviews, int V, const float* color,
                           const float* target, float w_l1, float w_dssim, double* partials, float* aux,
                           double* loss_out, float* dL_dcolor, hipStream_t s) {
  // aux NULL: the fused SSIM kernel (no per-pixel scratch)
  Win win;
  double g[TAPS], tot = 0.0;
  for (int k = 0; k < TAPS; ++k) {
    const double d = (double)(k - R);
    g[k] = exp(-(d * d) / (2.0 * 1.5 * 1.5));
    tot += g[k];
  }
  for (int k = 0; k < TAPS; ++k) win.w[k] = (float)(g[k] / tot);
  LossTiles lt{};
  int t = 0;
  for (int v = 0; v < V; ++v) {
    lt.off[v] = t;
    t += ((hviews[v].W + LT - 1) / LT) * ((hviews[v].H + LT - 1) / LT);
  }
  lt.off[V] = t;
  double2* part = reinterpret_cast<double2*>(partials);
  const bool ssim = w_dssim != 0.0f;
  const dim3 grid(kXcds * xcd_tile_chunk(t));   // >= t workgroups, see xcd_tile
  if (!ssim) {
    hipLaunchKernelGGL(k_l1, grid, dim3(256), 0, s, dviews, V, lt, color, target, w_l1, dL_dcolor, part);
  } else if (!aux) {
    hipLaunchKernelGGL(k_ssim_fused, grid, dim3(256), 0, s, dviews, V, lt, color, target, win, w_l1, w_dssim,
                       dL_dcolor, part);
  } else {
    hipLaunchKernelGGL(k_ssim_fwd, grid, dim3(256), 0, s, dviews, V, lt, color, target, aux, win, part);
    hipLaunchKernelGGL(k_ssim_bwd, grid, dim3(256), 0, s, dviews, V, lt, color, target, aux, win, w_l1, w_dssim,
                       dL_dcolor);
  }
  if (loss_out)
    hipLaunchKernelGGL(k_loss_final, dim3(V), dim3(256), 0, s, dviews, lt, part, w_l1, w_dssim, ssim ? 1 : 0,
                       loss_out);
  return hipGetLastError();
}

}  // namespace gsk
