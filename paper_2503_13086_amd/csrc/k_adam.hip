// Fused dense Adam step with a learning rate per view, for gfx950.
//
// The optimizer of the original 3DGS configuration (Sec. V-A) with the per-image
// learning rate of Sec. IV-D (Eq. 6-8): one thread per Gaussian computes its
// bias corrections from its own step counter (Gaussians appended later start at
// step 0) and its view factor (mean of the per-view scales over the views that
// see it), then streams its parameter rows: each row is a coalesced read of
// param, grad, m, v and a write of param, m, v.
#include "gs_internal.h"

namespace gsk {
namespace {

__device__ inline int row_group(int r) {
  if (r < 3) return GS_GROUP_MEAN;
  if (r < 6) return GS_GROUP_SCALE;
  if (r < 10) return GS_GROUP_ROT;
  if (r == 10) return GS_GROUP_OPACITY;
  if (r < 14) return GS_GROUP_SH_DC;
  return GS_GROUP_SH_REST;
}

__global__ __launch_bounds__(256) void k_adam(float* __restrict__ P, const float* __restrict__ G,
                                               float* __restrict__ M, float* __restrict__ Vv,
                                               uint32_t* __restrict__ step, int n, int stride, int rows, AdamArgs a,
                                               const uint32_t* __restrict__ touched) {
  const int g = blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= n) return;
  const uint32_t k = step[g] + 1u;
  step[g] = k;
  const float bc1 = (float)(1.0 - pow((double)a.b1, (double)k));
  const float bc2 = (float)(1.0 - pow((double)a.b2, (double)k));
  float factor = 1.0f;
  if (a.n_views > 0) {
    float s = 0.0f, all = 0.0f;
    int c = 0;
    for (int v = 0; v < a.n_views; ++v) {
      all += a.scale[v];
      if (touched[(size_t)v * n + g] != 0u) {
        s += a.scale[v];
        ++c;
      }
    }
    factor = c > 0 ? s / (float)c : all / (float)a.n_views;
  }
  const float ob1 = 1.0f - a.b1, ob2 = 1.0f - a.b2;
  for (int r = 0; r < rows; ++r) {
    const int grp = row_group(r);
    const float lr = ((a.group_mask >> grp) & 1u) ? a.lr[grp] * factor : a.lr[grp];
    const size_t i = (size_t)r * stride + g;
    const float gi = G[i];
    const float m = a.b1 * M[i] + ob1 * gi;
    const float v = a.b2 * Vv[i] + ob2 * gi * gi;
    M[i] = m;
    Vv[i] = v;
    P[i] = P[i] - lr * (m / bc1) / (sqrtf(v / bc2) + a.eps);
  }
}

}  // namespace

hipError_t launch_adam(float* P, const float* G, float* M, float* Vv, uint32_t* step, int n, int stride, int D,
                       const AdamArgs& a, const uint32_t* touched, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_adam, dim3((n + 255) / 256), dim3(256), 0, s, P, G, M, Vv, step, n, stride, n_params(D), a,
                     touched);
  return hipGetLastError();
}

}  // namespace gsk
