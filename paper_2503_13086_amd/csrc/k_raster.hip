// Tile rasterizer forward and backward for gfx950.
//
// Forward (Sec. III Eq. 2): one 256-thread workgroup (four wave64s) per 16x16
// tile, one thread per pixel.  The tile's depth-ordered list is walked in batches
// of 256 records staged in LDS; every pixel reads each staged record by LDS
// broadcast, so a record fetched from HBM once serves all 256 pixels.  The
// workgroup stops when every pixel has stopped blending.  Screen centres arrive
// in FP64 and are made relative to the tile origin while staging, so per-pixel
// offsets are accurate fp32 numbers at any image size.
//
// Backward (Sec. IV-E): the same tiling, walking each list back to front from the
// last position any pixel of the tile blended.  Each pixel recovers its
// transmittance by division and keeps the colour accumulated behind the current
// Gaussian.  The nine per-Gaussian partials (u, w, a, b, c, o, r, g, b) are summed
// across the wavefront with DPP row shifts and row broadcasts, across the four
// wavefronts with LDS atomics, and leave the workgroup as one global atomic per
// (tile, Gaussian, component) instead of one per (pixel, Gaussian, component).
// Wavefronts in which no pixel touches a Gaussian skip its reduction.
#include "gs_internal.h"

#pragma clang fp contract(off)

namespace gsk {
namespace {

constexpr int T = kTile;
constexpr int NT = kTileThreads;

__device__ inline int view_of_tile(const ViewDev* __restrict__ views, int V, int tile) {
  int v = 0;
  while (v + 1 < V && tile >= views[v + 1].tile_off) ++v;
  return v;
}

// exponent of the 2D Gaussian at offset (dx, dy); A = -a/2, B = -b, C = -c/2
__device__ inline float gauss_power(float A, float B, float C, float dx, float dy) {
  return __fmaf_rn(A * dx, dx, __fmaf_rn(C * dy, dy, (B * dx) * dy));
}

struct TileGeom {
  int v, tx, ty, lx, ly, px, py;
  bool inside;
  double ox, oy;
};

__device__ inline TileGeom tile_geom(const ViewDev* __restrict__ views, int V, int tile) {
  TileGeom t;
  t.v = view_of_tile(views, V, tile);
  const ViewDev& cv = views[t.v];
  const int lt = tile - cv.tile_off;
  t.tx = lt % cv.tiles_x;
  t.ty = lt / cv.tiles_x;
  t.lx = threadIdx.x % T;
  t.ly = threadIdx.x / T;
  t.px = t.tx * T + t.lx;
  t.py = t.ty * T + t.ly;
  t.inside = t.px < cv.W && t.py < cv.H;
  t.ox = (double)(t.tx * T) + 0.5;
  t.oy = (double)(t.ty * T) + 0.5;
  return t;
}

// stage record `rid` for a tile with origin (ox, oy)
__device__ inline void stage(const Record* __restrict__ rec, uint32_t rid, double ox, double oy, float4& q0,
                             float4& q1, float4& q2) {
  const Record* r = rec + rid;
  const double2 uw = *reinterpret_cast<const double2*>(r);
  const float4 c = reinterpret_cast<const float4*>(r)[1];
  const float4 d = reinterpret_cast<const float4*>(r)[2];
  q0 = make_float4((float)(uw.x - ox), (float)(uw.y - oy), -0.5f * c.x, -c.y);
  q1 = make_float4(-0.5f * c.z, c.w, d.x, 0.0f);
  q2 = make_float4(d.y, d.z, d.w, 0.0f);
}

__global__ __launch_bounds__(NT) void k_render_fwd(const ViewDev* __restrict__ views, int V,
                                                    const uint2* __restrict__ ranges,
                                                    const uint32_t* __restrict__ pair_rec,
                                                    const Record* __restrict__ rec, uint32_t n_rec,
                                                    float* __restrict__ color,
                                                    float* __restrict__ t_final, uint32_t* __restrict__ n_contrib,
                                                    uint32_t* __restrict__ last) {
  __shared__ float4 s0[NT], s1[NT], s2[NT];
  const int tile = blockIdx.x;
  const TileGeom tg = tile_geom(views, V, tile);
  const uint2 rg = ranges[tile];
  const float fx = (float)tg.lx, fy = (float)tg.ly;
  float Tr = 1.0f, C0 = 0.0f, C1 = 0.0f, C2 = 0.0f;
  uint32_t cnt = 0, lastp = 0;
  bool done = !tg.inside;
  for (uint32_t base = rg.x; base < rg.y; base += NT) {
    const uint32_t m = min((uint32_t)NT, rg.y - base);
    __syncthreads();
    if (threadIdx.x < m) {
      const uint32_t rid = pair_rec[base + threadIdx.x];
      if (rid < n_rec) {
        stage(rec, rid, tg.ox, tg.oy, s0[threadIdx.x], s1[threadIdx.x], s2[threadIdx.x]);
      } else {   // never for a consistent sort: an entry that no pixel accepts
        s0[threadIdx.x] = make_float4(0.f, 0.f, 0.f, 0.f);
        s1[threadIdx.x] = make_float4(0.f, 0.f, 1.f, 0.f);
        s2[threadIdx.x] = make_float4(0.f, 0.f, 0.f, 0.f);
      }
    }
    __syncthreads();
    if (!done) {
      for (uint32_t j = 0; j < m; ++j) {
        const float4 a0 = s0[j];
        const float4 a1 = s1[j];
        const float dx = a0.x - fx, dy = a0.y - fy;
        const float power = gauss_power(a0.z, a0.w, a1.x, dx, dy);
        if (power > 0.0f || power < a1.z) continue;
        const float og = a1.y * __expf(power);
        const float alpha = fminf(kAlphaMax, og);
        const float Tn = Tr * (1.0f - alpha);
        if (Tn < kTMin) {
          done = true;
          break;
        }
        const float4 a2 = s2[j];
        const float wgt = alpha * Tr;
        C0 += a2.x * wgt;
        C1 += a2.y * wgt;
        C2 += a2.z * wgt;
        Tr = Tn;
        ++cnt;
        lastp = base - rg.x + j + 1;
      }
    }
    if (__syncthreads_and(done)) break;
  }
  if (tg.inside) {
    const ViewDev& cv = views[tg.v];
    const size_t hw = (size_t)cv.W * cv.H;
    const size_t pix = (size_t)tg.py * cv.W + tg.px;
    float* img = color + 3 * (size_t)cv.pix_off;
    img[pix] = C0 + Tr * cv.bg[0];
    img[hw + pix] = C1 + Tr * cv.bg[1];
    img[2 * hw + pix] = C2 + Tr * cv.bg[2];
    const size_t gp = (size_t)cv.pix_off + pix;
    t_final[gp] = Tr;
    n_contrib[gp] = cnt;
    last[gp] = lastp;
  }
}

// Sum of v over the wavefront, valid in lane 63 (GFX9 DPP: row shifts, then row broadcasts).
__device__ inline float wave_sum_lane63(float v) {
  v += __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x111, 0xf, 0xf, true));  // row_shr:1
  v += __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x112, 0xf, 0xf, true));  // row_shr:2
  v += __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x114, 0xf, 0xf, true));  // row_shr:4
  v += __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x118, 0xf, 0xf, true));  // row_shr:8
  v += __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x142, 0xa, 0xf, false)); // row_bcast:15
  v += __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x143, 0xc, 0xf, false)); // row_bcast:31
  return v;
}

__global__ __launch_bounds__(NT) void k_render_bwd(const ViewDev* __restrict__ views, int V,
                                                    const uint2* __restrict__ ranges,
                                                    const uint32_t* __restrict__ pair_rec,
                                                    const Record* __restrict__ rec, uint32_t n_rec,
                                                    const float* __restrict__ t_final,
                                                    const uint32_t* __restrict__ last,
                                                    const float* __restrict__ dL_dcolor, float* __restrict__ grad2d) {
  __shared__ float4 s0[NT], s1[NT], s2[NT];
  __shared__ uint32_t srid[NT];
  __shared__ float acc[NT][kGrad2D];
  __shared__ uint32_t smax[NT / 64];
  const int tile = blockIdx.x;
  const TileGeom tg = tile_geom(views, V, tile);
  const ViewDev& cv = views[tg.v];
  const uint2 rg = ranges[tile];
  const float fx = (float)tg.lx, fy = (float)tg.ly;

  float Tr = 0.0f, S0 = 0.0f, S1 = 0.0f, S2 = 0.0f, g0 = 0.0f, g1 = 0.0f, g2 = 0.0f;
  uint32_t lp = 0;
  if (tg.inside) {
    const size_t hw = (size_t)cv.W * cv.H;
    const size_t pix = (size_t)tg.py * cv.W + tg.px;
    const size_t gp = (size_t)cv.pix_off + pix;
    Tr = t_final[gp];
    lp = last[gp];
    const float* gimg = dL_dcolor + 3 * (size_t)cv.pix_off;
    g0 = gimg[pix];
    g1 = gimg[hw + pix];
    g2 = gimg[2 * hw + pix];
    S0 = Tr * cv.bg[0];
    S1 = Tr * cv.bg[1];
    S2 = Tr * cv.bg[2];
  }
  uint32_t mx = lp;
  for (int off = 32; off > 0; off >>= 1) mx = max(mx, (uint32_t)__shfl_xor((int)mx, off));
  if (__lane_id() == 0) smax[threadIdx.x / 64] = mx;
  for (int k = 0; k < kGrad2D; ++k) acc[threadIdx.x][k] = 0.0f;
  __syncthreads();
  int jmax = 0;
  for (int w = 0; w < NT / 64; ++w) jmax = max(jmax, (int)smax[w]);

  for (int end = jmax; end > 0; end -= NT) {
    const int beg = end > NT ? end - NT : 0;
    const int m = end - beg;
    __syncthreads();
    if ((int)threadIdx.x < m) {
      const uint32_t rid = pair_rec[rg.x + beg + threadIdx.x];
      srid[threadIdx.x] = rid;
      if (rid < n_rec) {
        stage(rec, rid, tg.ox, tg.oy, s0[threadIdx.x], s1[threadIdx.x], s2[threadIdx.x]);
      } else {   // never for a consistent sort: an entry that no pixel accepts
        s0[threadIdx.x] = make_float4(0.f, 0.f, 0.f, 0.f);
        s1[threadIdx.x] = make_float4(0.f, 0.f, 1.f, 0.f);
        s2[threadIdx.x] = make_float4(0.f, 0.f, 0.f, 0.f);
      }
    }
    __syncthreads();
    for (int j = m - 1; j >= 0; --j) {
      bool on = tg.inside && (uint32_t)(beg + j) < lp;
      float pu = 0.f, pw = 0.f, pa = 0.f, pb = 0.f, pc = 0.f, po = 0.f, pr = 0.f, pg = 0.f, pbl = 0.f;
      if (on) {
        const float4 a0 = s0[j];
        const float4 a1 = s1[j];
        const float dx = a0.x - fx, dy = a0.y - fy;
        const float power = gauss_power(a0.z, a0.w, a1.x, dx, dy);
        if (power > 0.0f || power < a1.z) {
          on = false;
        } else {
          const float4 a2 = s2[j];
          const float G = __expf(power);
          const float og = a1.y * G;
          const bool capped = og > kAlphaMax;
          const float alpha = capped ? kAlphaMax : og;
          const float oma = 1.0f - alpha;
          Tr = Tr / oma;                    // transmittance in front of this Gaussian
          const float wgt = alpha * Tr;
          pr = g0 * wgt;
          pg = g1 * wgt;
          pbl = g2 * wgt;
          const float dLda = g0 * (a2.x * Tr - S0 / oma) + g1 * (a2.y * Tr - S1 / oma) + g2 * (a2.z * Tr - S2 / oma);
          S0 += a2.x * wgt;
          S1 += a2.y * wgt;
          S2 += a2.z * wgt;
          if (!capped) {
            const float dpow = dLda * og;
            po = dLda * G;
            pu = dpow * (2.0f * a0.z * dx + a0.w * dy);
            pw = dpow * (a0.w * dx + 2.0f * a1.x * dy);
            pa = dpow * (-0.5f * dx * dx);
            pb = dpow * (-(dx * dy));
            pc = dpow * (-0.5f * dy * dy);
          }
        }
      }
      if (__ballot(on) != 0ull) {
        pu = wave_sum_lane63(pu);
        pw = wave_sum_lane63(pw);
        pa = wave_sum_lane63(pa);
        pb = wave_sum_lane63(pb);
        pc = wave_sum_lane63(pc);
        po = wave_sum_lane63(po);
        pr = wave_sum_lane63(pr);
        pg = wave_sum_lane63(pg);
        pbl = wave_sum_lane63(pbl);
        if (__lane_id() == 63) {
          float* a = acc[j];
          atomicAdd(a + 0, pu);
          atomicAdd(a + 1, pw);
          atomicAdd(a + 2, pa);
          atomicAdd(a + 3, pb);
          atomicAdd(a + 4, pc);
          atomicAdd(a + 5, po);
          atomicAdd(a + 6, pr);
          atomicAdd(a + 7, pg);
          atomicAdd(a + 8, pbl);
        }
      }
    }
    __syncthreads();
    if ((int)threadIdx.x < m) {
      float* a = acc[threadIdx.x];
      const uint32_t rid = srid[threadIdx.x];
      float* dst = grad2d + (size_t)rid * kGrad2D;
      for (int k = 0; k < kGrad2D; ++k) {
        const float x = a[k];
        if (x != 0.0f && rid < n_rec) unsafeAtomicAdd(dst + k, x);
        a[k] = 0.0f;
      }
    }
  }
}

}  // namespace

hipError_t launch_render_fwd(const ViewDev* views, int V, int n_tiles, const uint2* ranges, const uint32_t* pair_rec,
                             const Record* rec, uint32_t n_rec, float* color, float* t_final, uint32_t* n_contrib,
                             uint32_t* last, hipStream_t s) {
  if (n_tiles <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_render_fwd, dim3(n_tiles), dim3(NT), 0, s, views, V, ranges, pair_rec, rec, n_rec, color,
                     t_final, n_contrib, last);
  return hipGetLastError();
}

hipError_t launch_render_bwd(const ViewDev* views, int V, int n_tiles, const uint2* ranges, const uint32_t* pair_rec,
                             const Record* rec, uint32_t n_rec, const float* t_final, const uint32_t* last,
                             const float* dL_dcolor, float* grad2d, hipStream_t s) {
  if (n_tiles <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_render_bwd, dim3(n_tiles), dim3(NT), 0, s, views, V, ranges, pair_rec, rec, n_rec, t_final,
                     last, dL_dcolor, grad2d);
  return hipGetLastError();
}

}  // namespace gsk
