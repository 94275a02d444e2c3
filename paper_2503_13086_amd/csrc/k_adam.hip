// Fused dense Adam step with a learning rate per view, for gfx950.
//
// The optimizer of the original 3DGS configuration (Sec. V-A) with the per-image
// learning rate of Sec. IV-D (Eq. 6-8): one thread per Gaussian computes its
// bias corrections from its own step counter (Gaussians appended later start at
// step 0) and its view factor (mean of the per-view scales over the views that
// see it), then streams its parameter rows: each row is a coalesced read of
// param, grad, m, v and a write of param, m, v.  A step whose binning reported an
// error on the device (pair buffers too small) writes nothing.
#include "gs_internal.h"

namespace gsk {
namespace {

__global__ __launch_bounds__(256) void k_adam(float* __restrict__ P, const float* __restrict__ G,
                                               float* __restrict__ M, float* __restrict__ Vv,
                                               uint32_t* __restrict__ step, int n, int stride, int rows, AdamArgs a,
                                               const uint32_t* __restrict__ touched,
                                               const DevStatus* __restrict__ st) {
  const int g = blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= n) return;
  if (st && st->code != GS_OK) return;
  const uint32_t k = step[g] + 1u;
  step[g] = k;
  float bc1, bc2;
  adam_bias(a, k, bc1, bc2);
  const float factor = adam_view_factor(a, touched, n, g);
  for (int r = 0; r < rows; ++r) {
    const int grp = adam_row_group(r);
    const float lr = ((a.group_mask >> grp) & 1u) ? a.lr[grp] * factor : a.lr[grp];
    const size_t i = (size_t)r * stride + g;
    float p = P[i], m = M[i], v = Vv[i];
    adam_elem(p, m, v, G[i], lr, a, bc1, bc2);
    M[i] = m;
    Vv[i] = v;
    P[i] = p;
  }
}

}  // namespace

hipError_t launch_adam(float* P, const float* G, float* M, float* Vv, uint32_t* step, int n, int stride, int D,
                       const AdamArgs& a, const uint32_t* touched, const DevStatus* st, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_adam, dim3((n + 255) / 256), dim3(256), 0, s, P, G, M, Vv, step, n, stride, n_params(D), a,
                     touched, st);
  return hipGetLastError();
}

}  // namespace gsk
