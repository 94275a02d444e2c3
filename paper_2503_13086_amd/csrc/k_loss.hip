// Image loss terms of Eq. 10 and dL/dimage for gfx950.
//
// Per view: w_l1 * mean|x - y| + w_dssim * (1 - mean SSIM(x, y)), SSIM per channel
// from windowed means under a normalised 11x11 Gaussian window (sigma 1.5, zero
// padding), C1 = 0.01^2, C2 = 0.03^2.  All views share one launch, tiled like the
// rasterizer (16x16 output tiles, one thread per pixel); each workgroup stages a
// 26x26 halo of the inputs in LDS and applies the separable window in two passes.
//
// Backward: with N1 = 2 mx my + C1, N2 = 2 sxy + C2, D1 = mx^2 + my^2 + C1,
// D2 = sxx + syy + C2 and S = N1 N2 / (D1 D2), the per-pixel partials of S with
// respect to the windowed statistics (mx, E[x^2], E[xy]) are
//   A = 2 my (N2 - N1) / (D1 D2) + 2 mx S (1/D2 - 1/D1),  B = -S / D2,
//   Cc = 2 N1 / (D1 D2),
// and dS_mean/dx = (window * A + 2 x (window * B) + y (window * Cc)) / N.  The first
// kernel stores A, B, Cc; the second blurs them (the window is symmetric) and
// adds the L1 term.  Loss sums are reduced per tile in FP64.
#include "gs_internal.h"

namespace gsk {
namespace {

constexpr int T = kTile;
constexpr int R = 5;             // window radius
constexpr int HALO = T + 2 * R;  // 26
constexpr float kC1 = 0.01f * 0.01f;
constexpr float kC2 = 0.03f * 0.03f;

struct Win {
  float w[2 * R + 1];
};

__device__ inline int view_of_tile(const ViewDev* __restrict__ views, int V, int tile) {
  int v = 0;
  while (v + 1 < V && tile >= views[v + 1].tile_off) ++v;
  return v;
}

__device__ inline double block_sum_d(double x, double* sh) {
  for (int off = 32; off > 0; off >>= 1) x += __shfl_xor(x, off);
  if (__lane_id() == 0) sh[threadIdx.x / 64] = x;
  __syncthreads();
  double t = 0.0;
  for (int w = 0; w < (int)(blockDim.x / 64); ++w) t += sh[w];
  __syncthreads();
  return t;
}

__global__ __launch_bounds__(256) void k_l1(const ViewDev* __restrict__ views, int V, const float* __restrict__ x,
                                             const float* __restrict__ y, float w_l1, float* __restrict__ grad,
                                             double2* __restrict__ partials) {
  __shared__ double sh[4];
  const int tile = blockIdx.x;
  const int v = view_of_tile(views, V, tile);
  const ViewDev& cv = views[v];
  const int lt = tile - cv.tile_off;
  const int px = (lt % cv.tiles_x) * T + threadIdx.x % T;
  const int py = (lt / cv.tiles_x) * T + threadIdx.x / T;
  double s = 0.0;
  if (px < cv.W && py < cv.H) {
    const size_t hw = (size_t)cv.W * cv.H;
    const size_t off = 3 * (size_t)cv.pix_off + (size_t)py * cv.W + px;
    const float inv = w_l1 / (float)(3 * hw);
    for (int c = 0; c < 3; ++c) {
      const float d = x[off + c * hw] - y[off + c * hw];
      s += fabs((double)d);
      grad[off + c * hw] = inv * (float)((d > 0.0f) - (d < 0.0f));
    }
  }
  const double t = block_sum_d(s, sh);
  if (threadIdx.x == 0) partials[tile] = make_double2(t, 0.0);
}

// windowed sums of q quantities from a HALO x HALO LDS patch into one value per pixel
template <int Q>
__device__ inline void separable_blur(const float (*src)[HALO][HALO], float (*tmp)[HALO][T], const Win& win,
                                      float* out) {
  for (int i = threadIdx.x; i < HALO * T; i += blockDim.x) {
    const int r = i / T, c = i % T;
    for (int q = 0; q < Q; ++q) {
      float a = 0.0f;
      for (int k = 0; k <= 2 * R; ++k) a += win.w[k] * src[q][r][c + k];
      tmp[q][r][c] = a;
    }
  }
  __syncthreads();
  const int lx = threadIdx.x % T, ly = threadIdx.x / T;
  for (int q = 0; q < Q; ++q) {
    float a = 0.0f;
    for (int k = 0; k <= 2 * R; ++k) a += win.w[k] * tmp[q][ly + k][lx];
    out[q] = a;
  }
  __syncthreads();
}

__global__ __launch_bounds__(256) void k_ssim_fwd(const ViewDev* __restrict__ views, int V,
                                                   const float* __restrict__ x, const float* __restrict__ y,
                                                   float* __restrict__ aux, Win win, double2* __restrict__ partials) {
  __shared__ float src[5][HALO][HALO];
  __shared__ float tmp[5][HALO][T];
  __shared__ double sh[4];
  const int tile = blockIdx.x;
  const int v = view_of_tile(views, V, tile);
  const ViewDev& cv = views[v];
  const int lt = tile - cv.tile_off;
  const int x0 = (lt % cv.tiles_x) * T, y0 = (lt / cv.tiles_x) * T;
  const int px = x0 + threadIdx.x % T, py = y0 + threadIdx.x / T;
  const bool inside = px < cv.W && py < cv.H;
  const size_t hw = (size_t)cv.W * cv.H;
  const size_t base = 3 * (size_t)cv.pix_off;
  double sl1 = 0.0, sss = 0.0;
  for (int c = 0; c < 3; ++c) {
    const float* xc = x + base + c * hw;
    const float* yc = y + base + c * hw;
    for (int i = threadIdx.x; i < HALO * HALO; i += blockDim.x) {
      const int r = i / HALO, q = i % HALO;
      const int gx = x0 - R + q, gy = y0 - R + r;
      float a = 0.0f, b = 0.0f;
      if (gx >= 0 && gx < cv.W && gy >= 0 && gy < cv.H) {
        a = xc[(size_t)gy * cv.W + gx];
        b = yc[(size_t)gy * cv.W + gx];
      }
      src[0][r][q] = a;
      src[1][r][q] = b;
      src[2][r][q] = a * a;
      src[3][r][q] = b * b;
      src[4][r][q] = a * b;
    }
    __syncthreads();
    float m[5];
    separable_blur<5>(src, tmp, win, m);
    if (inside) {
      const float mx = m[0], my = m[1];
      const float sxx = m[2] - mx * mx, syy = m[3] - my * my, sxy = m[4] - mx * my;
      const float N1 = 2.0f * mx * my + kC1, N2 = 2.0f * sxy + kC2;
      const float D1 = mx * mx + my * my + kC1, D2 = sxx + syy + kC2;
      const float den = D1 * D2;
      const float S = (N1 * N2) / den;
      const float A = 2.0f * my * (N2 - N1) / den + 2.0f * mx * S * (1.0f / D2 - 1.0f / D1);
      const float B = -S / D2;
      const float Cc = 2.0f * N1 / den;
      const size_t p = (size_t)cv.pix_off * 9 + (size_t)c * 3 * hw + (size_t)py * cv.W + px;
      aux[p] = A;
      aux[p + hw] = B;
      aux[p + 2 * hw] = Cc;
      const float xv = src[0][threadIdx.x / T + R][threadIdx.x % T + R];
      const float yv = src[1][threadIdx.x / T + R][threadIdx.x % T + R];
      sl1 += fabs((double)(xv - yv));
      sss += (double)S;
    }
    __syncthreads();
  }
  const double t1 = block_sum_d(sl1, sh);
  const double t2 = block_sum_d(sss, sh);
  if (threadIdx.x == 0) partials[tile] = make_double2(t1, t2);
}

__global__ __launch_bounds__(256) void k_ssim_bwd(const ViewDev* __restrict__ views, int V,
                                                   const float* __restrict__ x, const float* __restrict__ y,
                                                   const float* __restrict__ aux, Win win, float w_l1, float w_dssim,
                                                   float* __restrict__ grad) {
  __shared__ float src[3][HALO][HALO];
  __shared__ float tmp[3][HALO][T];
  const int tile = blockIdx.x;
  const int v = view_of_tile(views, V, tile);
  const ViewDev& cv = views[v];
  const int lt = tile - cv.tile_off;
  const int x0 = (lt % cv.tiles_x) * T, y0 = (lt / cv.tiles_x) * T;
  const int px = x0 + threadIdx.x % T, py = y0 + threadIdx.x / T;
  const bool inside = px < cv.W && py < cv.H;
  const size_t hw = (size_t)cv.W * cv.H;
  const size_t base = 3 * (size_t)cv.pix_off;
  const float invN = 1.0f / (float)(3 * hw);
  for (int c = 0; c < 3; ++c) {
    const float* ac = aux + (size_t)cv.pix_off * 9 + (size_t)c * 3 * hw;
    for (int i = threadIdx.x; i < HALO * HALO; i += blockDim.x) {
      const int r = i / HALO, q = i % HALO;
      const int gx = x0 - R + q, gy = y0 - R + r;
      float a = 0.0f, b = 0.0f, cc = 0.0f;
      if (gx >= 0 && gx < cv.W && gy >= 0 && gy < cv.H) {
        const size_t p = (size_t)gy * cv.W + gx;
        a = ac[p];
        b = ac[p + hw];
        cc = ac[p + 2 * hw];
      }
      src[0][r][q] = a;
      src[1][r][q] = b;
      src[2][r][q] = cc;
    }
    __syncthreads();
    float m[3];
    separable_blur<3>(src, tmp, win, m);
    if (inside) {
      const size_t p = base + c * hw + (size_t)py * cv.W + px;
      const float xv = x[p], yv = y[p];
      const float d = xv - yv;
      const float l1 = w_l1 * invN * (float)((d > 0.0f) - (d < 0.0f));
      const float ds = m[0] + 2.0f * xv * m[1] + yv * m[2];
      grad[p] = l1 - w_dssim * invN * ds;
    }
    __syncthreads();
  }
}

__global__ void k_loss_final(const ViewDev* __restrict__ views, int V, const double2* __restrict__ partials,
                             float w_l1, float w_dssim, int ssim, double* __restrict__ out) {
  __shared__ double sh[4];
  for (int v = 0; v < V; ++v) {
    const ViewDev& cv = views[v];
    const int t0 = cv.tile_off, t1 = t0 + cv.tiles_x * cv.tiles_y;
    double a = 0.0, b = 0.0;
    for (int t = t0 + threadIdx.x; t < t1; t += blockDim.x) {
      a += partials[t].x;
      b += partials[t].y;
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
}

}  // namespace

hipError_t launch_loss_dev(const ViewDev* dviews, int V, int n_tiles, const float* color, const float* target,
                           float w_l1, float w_dssim, double* partials, float* aux, double* loss_out,
                           float* dL_dcolor, hipStream_t s) {
  Win win;
  double g[2 * R + 1], tot = 0.0;
  for (int k = 0; k <= 2 * R; ++k) {
    const double d = (double)(k - R);
    g[k] = exp(-(d * d) / (2.0 * 1.5 * 1.5));
    tot += g[k];
  }
  for (int k = 0; k <= 2 * R; ++k) win.w[k] = (float)(g[k] / tot);
  double2* part = reinterpret_cast<double2*>(partials);
  const bool ssim = w_dssim != 0.0f;
  if (!ssim) {
    hipLaunchKernelGGL(k_l1, dim3(n_tiles), dim3(256), 0, s, dviews, V, color, target, w_l1, dL_dcolor, part);
  } else {
    hipLaunchKernelGGL(k_ssim_fwd, dim3(n_tiles), dim3(256), 0, s, dviews, V, color, target, aux, win, part);
    hipLaunchKernelGGL(k_ssim_bwd, dim3(n_tiles), dim3(256), 0, s, dviews, V, color, target, aux, win, w_l1, w_dssim,
                       dL_dcolor);
  }
  if (loss_out)
    hipLaunchKernelGGL(k_loss_final, dim3(1), dim3(256), 0, s, dviews, V, part, w_l1, w_dssim, ssim ? 1 : 0,
                       loss_out);
  return hipGetLastError();
}
}  // namespace gsk
