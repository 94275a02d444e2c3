// Per-Gaussian projection (forward) and its chain rule (backward) for gfx950.
//
// Forward: Sec. III Eq. 1 (covariance R S S^T R^T) and the EWA splatting of the
// original 3DGS configuration (Sec. V-A): camera transform, near cull, pinhole
// projection, clamped projection Jacobian, 2D covariance J W Sigma W^T J^T + 0.3 I,
// conic, extent 3 sqrt(lambda_max), tile rect, cutoff exponent and SH colour.
// One thread per Gaussian reads its parameters once (planar rows, coalesced) and
// loops over the views, so parameter traffic does not grow with the view count.
// The geometry is evaluated in FP64 (CDNA4 issues FP64 FMA at the non-packed FP32
// rate), so depth, screen position and extent come out exactly as an IEEE FP64
// evaluation in the same operation order (contraction is off in this file); the
// SH colour, which no discrete decision depends on, is fp32 (FP64 coefficients
// held across the view loop cost 96 registers).
//
// Backward: one thread per Gaussian recomputes the forward quantities per view in
// fp32 (gradients carry no discrete decision; visibility is the forward's
// tiles-touched count), applies the chain rule from the per-view 2D gradients
// (u, w, a, b, c, o, rgb) to mean, covariance, opacity and SH coefficients, sums
// the views, takes covariance to log-scale and quaternion in FP64 once, and
// writes each gradient once.
#include "gs_geom.h"

#pragma clang fp contract(off)

namespace gsk {
namespace {

// Real SH basis of the 3DGS lineage (order k = l^2 + l + m), constants from
// sqrt((2l+1)/(4 pi) (l-|m|)!/(l+|m|)!) times the Cartesian polynomial factors.
constexpr double kPi = 3.14159265358979323846;
template <typename F>
__device__ inline void sh_eval(int D, F x, F y, F z, F* Y) {
  const F c0 = (F)(0.5 * sqrt(1.0 / kPi));
  Y[0] = c0;
  if (D < 1) return;
  const F c1 = (F)sqrt(3.0 / (4.0 * kPi));
  Y[1] = -c1 * y;
  Y[2] = c1 * z;
  Y[3] = -c1 * x;
  if (D < 2) return;
  const F xx = x * x, yy = y * y, zz = z * z;
  const F c2a = (F)(0.5 * sqrt(15.0 / kPi)), c2b = (F)(0.25 * sqrt(5.0 / kPi)), c2c = (F)(0.25 * sqrt(15.0 / kPi));
  Y[4] = c2a * (x * y);
  Y[5] = -c2a * (y * z);
  Y[6] = c2b * ((F)2 * zz - xx - yy);
  Y[7] = -c2a * (x * z);
  Y[8] = c2c * (xx - yy);
  if (D < 3) return;
  const F c3a = (F)(0.25 * sqrt(35.0 / (2.0 * kPi))), c3b = (F)(0.5 * sqrt(105.0 / kPi));
  const F c3c = (F)(0.25 * sqrt(21.0 / (2.0 * kPi))), c3d = (F)(0.25 * sqrt(7.0 / kPi));
  const F c3e = (F)(0.25 * sqrt(105.0 / kPi));
  Y[9] = -c3a * y * ((F)3 * xx - yy);
  Y[10] = c3b * (x * y) * z;
  Y[11] = -c3c * y * ((F)4 * zz - xx - yy);
  Y[12] = c3d * z * ((F)2 * zz - (F)3 * xx - (F)3 * yy);
  Y[13] = -c3c * x * ((F)4 * zz - xx - yy);
  Y[14] = c3e * z * (xx - yy);
  Y[15] = -c3a * x * (xx - (F)3 * yy);
}

// dL/d(direction) from dL/dY_k (gradient of each basis polynomial); evaluated in
// fp32 by the backward
__device__ inline void sh_grad_dir(int D, float x, float y, float z, const float* gY, float* gd) {
  gd[0] = gd[1] = gd[2] = 0.0f;
  if (D < 1) return;
  const float c1 = (float)sqrt(3.0 / (4.0 * kPi));
  gd[1] += -c1 * gY[1];
  gd[2] += c1 * gY[2];
  gd[0] += -c1 * gY[3];
  if (D < 2) return;
  const float xx = x * x, yy = y * y, zz = z * z;
  const float c2a = (float)(0.5 * sqrt(15.0 / kPi)), c2b = (float)(0.25 * sqrt(5.0 / kPi));
  const float c2c = (float)(0.25 * sqrt(15.0 / kPi));
  gd[0] += c2a * y * gY[4];            gd[1] += c2a * x * gY[4];
  gd[1] += -c2a * z * gY[5];           gd[2] += -c2a * y * gY[5];
  gd[0] += -2.0f * c2b * x * gY[6];    gd[1] += -2.0f * c2b * y * gY[6];  gd[2] += 4.0f * c2b * z * gY[6];
  gd[0] += -c2a * z * gY[7];           gd[2] += -c2a * x * gY[7];
  gd[0] += 2.0f * c2c * x * gY[8];     gd[1] += -2.0f * c2c * y * gY[8];
  if (D < 3) return;
  const float c3a = (float)(0.25 * sqrt(35.0 / (2.0 * kPi))), c3b = (float)(0.5 * sqrt(105.0 / kPi));
  const float c3c = (float)(0.25 * sqrt(21.0 / (2.0 * kPi))), c3d = (float)(0.25 * sqrt(7.0 / kPi));
  const float c3e = (float)(0.25 * sqrt(105.0 / kPi));
  gd[0] += -c3a * 6.0f * x * y * gY[9];
  gd[1] += -c3a * 3.0f * (xx - yy) * gY[9];
  gd[0] += c3b * y * z * gY[10];
  gd[1] += c3b * x * z * gY[10];
  gd[2] += c3b * x * y * gY[10];
  gd[0] += -c3c * (-2.0f * x * y) * gY[11];
  gd[1] += -c3c * (4.0f * zz - xx - 3.0f * yy) * gY[11];
  gd[2] += -c3c * (8.0f * y * z) * gY[11];
  gd[0] += c3d * (-6.0f * x * z) * gY[12];
  gd[1] += c3d * (-6.0f * y * z) * gY[12];
  gd[2] += c3d * (6.0f * zz - 3.0f * xx - 3.0f * yy) * gY[12];
  gd[0] += -c3c * (4.0f * zz - 3.0f * xx - yy) * gY[13];
  gd[1] += -c3c * (-2.0f * x * y) * gY[13];
  gd[2] += -c3c * (8.0f * x * z) * gY[13];
  gd[0] += c3e * 2.0f * x * z * gY[14];
  gd[1] += -c3e * 2.0f * y * z * gY[14];
  gd[2] += c3e * (xx - yy) * gY[14];
  gd[0] += -c3a * 3.0f * (xx - yy) * gY[15];
  gd[1] += -c3a * (-6.0f * x * y) * gY[15];
}


// Unit direction from the camera centre to the Gaussian in fp32 (feeds only the
// SH colour).
__device__ inline void camera_dir_f(const float m[3], const ViewDev& V, float dir[3]) {
  float oc[3];
  for (int k = 0; k < 3; ++k) oc[k] = -((V.R[k] * V.t[0] + V.R[3 + k] * V.t[1]) + V.R[6 + k] * V.t[2]);
  const float d0 = m[0] - oc[0], d1 = m[1] - oc[1], d2 = m[2] - oc[2];
  const float inv = 1.0f / sqrtf((d0 * d0 + d1 * d1) + d2 * d2);
  dir[0] = d0 * inv; dir[1] = d1 * inv; dir[2] = d2 * inv;
}

template <int D>
// st (may be NULL): the binning status and the split counters after it, cleared
// here for the binning that follows.
__global__ __launch_bounds__(256) void k_preprocess(const float* __restrict__ P, int n, int stride,
                                                     const ViewDev* __restrict__ views, int V,
                                                     Record* __restrict__ rec, uint32_t* __restrict__ depth,
                                                     uint32_t* __restrict__ touched, ushort4* __restrict__ rect,
                                                     DevStatus* __restrict__ st) {
  if (st && blockIdx.x == 0) {
    if (threadIdx.x == 0) status_clear(st);
    split_clear(st);
  }
  const int g = blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= n) return;
  Gauss G;
  load_gauss(P, stride, g, G);
  const double tau = cutoff_tau(G.o);
  constexpr int K = (D + 1) * (D + 1);
  float f[3 * K];
#pragma unroll
  for (int i = 0; i < 3 * K; ++i) f[i] = P[(size_t)(11 + i) * stride + g];
  const float m[3] = {(float)G.m[0], (float)G.m[1], (float)G.m[2]};
  for (int v = 0; v < V; ++v) {
    const ViewDev& cv = views[v];
    Proj p;
    project(G, cv, p);
    const size_t idx = (size_t)v * n + g;
    if (!p.visible) {
      depth[idx] = 0xffffffffu;
      touched[idx] = 0u;
      rect[idx] = make_ushort4(0, 0, 0, 0);
      continue;
    }
    // colour in fp32 (no discrete decision depends on it; error a few 1e-7)
    float dir[3];
    camera_dir_f(m, cv, dir);
    float Y[16];
    sh_eval(D, dir[0], dir[1], dir[2], Y);
    float col[3];
#pragma unroll
    for (int ch = 0; ch < 3; ++ch) {
      float acc = 0.5f;
#pragma unroll
      for (int k = 0; k < K; ++k) acc = __fmaf_rn(f[3 * k + ch], Y[k], acc);
      col[ch] = acc < 0.0f ? 0.0f : acc;
    }
    depth[idx] = __float_as_uint((float)p.tz);
    touched[idx] = (uint32_t)((p.tx1 - p.tx0 + 1) * (p.ty1 - p.ty0 + 1));
    rect[idx] = make_ushort4((unsigned short)p.tx0, (unsigned short)p.tx1, (unsigned short)p.ty0,
                             (unsigned short)p.ty1);
    double2* r2 = reinterpret_cast<double2*>(rec + idx);
    r2[0] = make_double2(p.u, p.w);
    float4* r4 = reinterpret_cast<float4*>(rec + idx);
    r4[1] = make_float4((float)p.a, (float)p.b, (float)p.c, (float)G.o);
    r4[2] = make_float4((float)tau, col[0], col[1], col[2]);
  }
}

// ---- backward, in fp32 (gradients carry no discrete decision; visibility comes
// from the forward's tiles-touched count) ----
struct GaussF {
  float m[3];
  float Sig[3][3];
};

__device__ inline void gauss_geom_f(const float* __restrict__ P, int stride, int g, GaussF& G) {
#pragma clang fp contract(fast)
  for (int i = 0; i < 3; ++i) G.m[i] = P[(size_t)i * stride + g];
  float sc[3];
  for (int i = 0; i < 3; ++i) sc[i] = expf(P[(size_t)(3 + i) * stride + g]);
  const float qw = P[(size_t)6 * stride + g], qx = P[(size_t)7 * stride + g];
  const float qy = P[(size_t)8 * stride + g], qz = P[(size_t)9 * stride + g];
  const float inv = 1.0f / sqrtf(qw * qw + qx * qx + qy * qy + qz * qz);
  const float w = qw * inv, x = qx * inv, y = qy * inv, z = qz * inv;
  const float Rq[3][3] = {{1.0f - 2.0f * (y * y + z * z), 2.0f * (x * y - w * z), 2.0f * (x * z + w * y)},
                          {2.0f * (x * y + w * z), 1.0f - 2.0f * (x * x + z * z), 2.0f * (y * z - w * x)},
                          {2.0f * (x * z - w * y), 2.0f * (y * z + w * x), 1.0f - 2.0f * (x * x + y * y)}};
  float M[3][3];
  for (int k = 0; k < 3; ++k)
    for (int l = 0; l < 3; ++l) M[k][l] = Rq[k][l] * sc[l];
  for (int k = 0; k < 3; ++k)
    for (int l = 0; l < 3; ++l) G.Sig[k][l] = M[k][0] * M[l][0] + M[k][1] * M[l][1] + M[k][2] * M[l][2];
}

// The nine 2D gradients of one (view, Gaussian) entry, zeros for an entry the view
// does not touch (one branch for the whole row).
__device__ inline void load_grad2d(const float* __restrict__ src, uint32_t touched, float (&out)[kGrad2D]) {
  if (touched != 0u) {
#pragma unroll
    for (int k = 0; k < kGrad2D; ++k) out[k] = src[k];
  } else {
#pragma unroll
    for (int k = 0; k < kGrad2D; ++k) out[k] = 0.0f;
  }
}

// With adam != 0 the gradient is applied at once (params updated in place, `out`
// written only when not NULL); otherwise it goes to `out` (or is added to it).
// One kernel serves both so that the gradient is the same machine arithmetic
// either way.  The parameters are read before this thread writes any of them,
// and a thread touches only its own Gaussian's column.
template <int D>
__global__ __launch_bounds__(256) void k_preprocess_bwd(float* P, int n, int stride,
                                                         const ViewDev* __restrict__ views, int V,
                                                         const uint32_t* __restrict__ touched,
                                                         const float* __restrict__ grad2d, float* out,
                                                         int accumulate, int adam, float* M, float* Vv,
                                                         uint32_t* step, AdamArgs a, const DevStatus* st) {
#pragma clang fp contract(fast)
  const int g = blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= n) return;
  if (adam && st && st->code != GS_OK) return;   // the binning of this step failed: leave the state
  constexpr int K = (D + 1) * (D + 1);
  // the loads of the view loop run ahead of it: the touched flag of view v + 2 and
  // the 2D gradient of view v + 1 are in flight while view v is processed (at two
  // waves per SIMD nothing else would cover their latency)
  uint32_t t_next = V > 0 ? touched[g] : 0u;                  // view v + 1
  uint32_t t_after = V > 1 ? touched[(size_t)n + g] : 0u;     // view v + 2
  const uint32_t step_old = adam ? step[g] : 0u;
  GaussF G;
  gauss_geom_f(P, stride, g, G);

  float gm[3] = {0.f, 0.f, 0.f};       // dL/dmean
  float gSig[3][3] = {{0.f}};          // symmetric dL/dSigma accumulated over views
  float go = 0.f;                      // dL/dopacity
  float gf[3 * K];                     // dL/dSH
  float f[3 * K];                      // SH coefficients, held across the views
#pragma unroll
  for (int i = 0; i < 3 * K; ++i) {
    gf[i] = 0.f;
    f[i] = P[(size_t)(11 + i) * stride + g];
  }

  // the per-view learning-rate factor of the fused step (the mean of the scales of
  // the views that see the Gaussian, else of all), summed in view order as
  // adam_view_factor does, from the flags the loop reads anyway
  const bool fold_factor = adam && a.n_views == V;
  float fs = 0.0f, fall = 0.0f;
  int fc = 0;
  float g2n[kGrad2D];
  load_grad2d(grad2d + (size_t)g * kGrad2D, t_next, g2n);
  for (int v = 0; v < V; ++v) {
    const uint32_t t_cur = t_next;
    float g2[kGrad2D];
#pragma unroll
    for (int k = 0; k < kGrad2D; ++k) g2[k] = g2n[k];
    t_next = t_after;
    if (v + 1 < V) load_grad2d(grad2d + ((size_t)(v + 1) * n + g) * kGrad2D, t_next, g2n);
    t_after = v + 2 < V ? touched[(size_t)(v + 2) * n + g] : 0u;
    if (fold_factor) {
      fall += a.scale[v];
      if (t_cur != 0u) {
        fs += a.scale[v];
        ++fc;
      }
    }
    if (t_cur == 0u) continue;
    const ViewDev& cv = views[v];
    const float gu = g2[0], gw = g2[1], ga = g2[2], gb = g2[3], gc = g2[4];
    go += g2[5];
    const float grgb[3] = {g2[6], g2[7], g2[8]};
    float Wr[3][3];
    for (int i = 0; i < 3; ++i)
      for (int j = 0; j < 3; ++j) Wr[i][j] = cv.R[3 * i + j];

    // colour: raw = 1/2 + sum_k f_k Y_k(dir), clamped at 0 (zero derivative when
    // clamped); dir from the camera centre -W^T t to the mean
    float oc[3];
    for (int k = 0; k < 3; ++k) oc[k] = -(Wr[0][k] * cv.t[0] + Wr[1][k] * cv.t[1] + Wr[2][k] * cv.t[2]);
    const float d0 = G.m[0] - oc[0], d1 = G.m[1] - oc[1], d2 = G.m[2] - oc[2];
    const float dn = sqrtf(d0 * d0 + d1 * d1 + d2 * d2);
    const float dir[3] = {d0 / dn, d1 / dn, d2 / dn};
    float Y[16];
    sh_eval<float>(D, dir[0], dir[1], dir[2], Y);
    float graw[3];
#pragma unroll
    for (int ch = 0; ch < 3; ++ch) {
      float acc = 0.5f;
#pragma unroll
      for (int k = 0; k < K; ++k) acc += f[3 * k + ch] * Y[k];
      graw[ch] = acc < 0.0f ? 0.0f : grgb[ch];
    }
    float gY[16];
#pragma unroll
    for (int k = 0; k < K; ++k) {
      gY[k] = 0.0f;
#pragma unroll
      for (int ch = 0; ch < 3; ++ch) {
        gf[3 * k + ch] += graw[ch] * Y[k];
        gY[k] += graw[ch] * f[3 * k + ch];
      }
    }
    float gdir[3];
    sh_grad_dir(D, dir[0], dir[1], dir[2], gY, gdir);
    const float dd = gdir[0] * dir[0] + gdir[1] * dir[1] + gdir[2] * dir[2];
    for (int k = 0; k < 3; ++k) gm[k] += (gdir[k] - dir[k] * dd) / dn;

    // projection (the forward's formulas; the clamp state is re-derived)
    const float tx = Wr[0][0] * G.m[0] + Wr[0][1] * G.m[1] + Wr[0][2] * G.m[2] + cv.t[0];
    const float ty = Wr[1][0] * G.m[0] + Wr[1][1] * G.m[1] + Wr[1][2] * G.m[2] + cv.t[1];
    const float tz = Wr[2][0] * G.m[0] + Wr[2][1] * G.m[1] + Wr[2][2] * G.m[2] + cv.t[2];
    const float fx = cv.fx, fy = cv.fy;
    const float limx = ((float)kJacClamp * (0.5f * (float)cv.W)) / fx;
    const float limy = ((float)kJacClamp * (0.5f * (float)cv.H)) / fy;
    const float rx = tx / tz, ry = ty / tz;
    const bool clx = !(rx >= -limx && rx <= limx), cly = !(ry >= -limy && ry <= limy);
    const float txc = tz * fminf(fmaxf(rx, -limx), limx), tyc = tz * fminf(fmaxf(ry, -limy), limy);
    const float J00 = fx / tz, J02 = -(fx * txc) / (tz * tz);
    const float J11 = fy / tz, J12 = -(fy * tyc) / (tz * tz);
    float T0[3], T1[3];
    for (int k = 0; k < 3; ++k) {
      T0[k] = J00 * Wr[0][k] + J02 * Wr[2][k];
      T1[k] = J11 * Wr[1][k] + J12 * Wr[2][k];
    }
    float ST0[3], ST1[3];
    for (int k = 0; k < 3; ++k) {
      ST0[k] = G.Sig[k][0] * T0[0] + G.Sig[k][1] * T0[1] + G.Sig[k][2] * T0[2];
      ST1[k] = G.Sig[k][0] * T1[0] + G.Sig[k][1] * T1[1] + G.Sig[k][2] * T1[2];
    }
    const float S00 = ST0[0] * T0[0] + ST0[1] * T0[1] + ST0[2] * T0[2] + (float)kKappa;
    const float S01 = ST0[0] * T1[0] + ST0[1] * T1[1] + ST0[2] * T1[2];
    const float S11 = ST1[0] * T1[0] + ST1[1] * T1[1] + ST1[2] * T1[2] + (float)kKappa;
    const float idet = 1.0f / (S00 * S11 - S01 * S01);
    const float A00 = S11 * idet, A01 = -S01 * idet, A11 = S00 * idet;

    // conic (a, b, c) = inverse of S -> dL/dS = -A Gc A, Gc = [[ga, gb/2], [gb/2, gc]]
    const float H00 = ga * A00 + 0.5f * gb * A01, H01 = ga * A01 + 0.5f * gb * A11;
    const float H10 = 0.5f * gb * A00 + gc * A01, H11 = 0.5f * gb * A01 + gc * A11;  // Gc A
    const float gS00 = -(A00 * H00 + A01 * H10);
    const float gS11 = -(A01 * H01 + A11 * H11);
    const float gS01 = -2.0f * (A00 * H01 + A01 * H11);   // S01 appears in both off-diagonal slots

    // S = T Sigma T^T (+ kappa I): dL/dSigma (symmetric part) and dL/dT
    for (int k = 0; k < 3; ++k)
      for (int l = 0; l < 3; ++l)
        gSig[k][l] += gS00 * T0[k] * T0[l] + 0.5f * gS01 * (T0[k] * T1[l] + T1[k] * T0[l]) + gS11 * T1[k] * T1[l];
    float gT0[3], gT1[3];
    for (int k = 0; k < 3; ++k) {
      gT0[k] = 2.0f * gS00 * ST0[k] + gS01 * ST1[k];
      gT1[k] = gS01 * ST0[k] + 2.0f * gS11 * ST1[k];
    }
    // T0 = J00 W0 + J02 W2, T1 = J11 W1 + J12 W2 (W = view rotation rows)
    float gJ00 = 0.f, gJ02 = 0.f, gJ11 = 0.f, gJ12 = 0.f;
    for (int k = 0; k < 3; ++k) {
      gJ00 += gT0[k] * Wr[0][k];
      gJ02 += gT0[k] * Wr[2][k];
      gJ11 += gT1[k] * Wr[1][k];
      gJ12 += gT1[k] * Wr[2][k];
    }
    const float tz2 = tz * tz, tz3 = tz2 * tz;
    float gt[3] = {0.f, 0.f, 0.f};
    // u = fx tx / tz + cx, w = fy ty / tz + cy
    gt[0] += gu * fx / tz;
    gt[1] += gw * fy / tz;
    gt[2] += -(gu * fx * tx + gw * fy * ty) / tz2;
    // J00 = fx / tz, J11 = fy / tz
    gt[2] += -(gJ00 * fx + gJ11 * fy) / tz2;
    // J02 = -fx txc / tz^2 with txc = tx (free) or tz * (+-lim) (clamped)
    if (!clx) {
      gt[0] += -gJ02 * fx / tz2;
      gt[2] += gJ02 * 2.0f * fx * txc / tz3;
    } else {
      gt[2] += gJ02 * fx * txc / tz3;
    }
    if (!cly) {
      gt[1] += -gJ12 * fy / tz2;
      gt[2] += gJ12 * 2.0f * fy * tyc / tz3;
    } else {
      gt[2] += gJ12 * fy * tyc / tz3;
    }
    // t = W mean + t_v
    for (int k = 0; k < 3; ++k) gm[k] += Wr[0][k] * gt[0] + Wr[1][k] * gt[1] + Wr[2][k] * gt[2];
  }

  // Sigma = M M^T -> dL/dM = 2 sym(dL/dSigma) M; M = Rq diag(s); then the
  // activations (FP64, once per Gaussian)
  Gauss H;
  load_gauss(P, stride, g, H);
  double gs[3] = {0, 0, 0};
  double gR[3][3];
  for (int k = 0; k < 3; ++k)
    for (int j = 0; j < 3; ++j) {
      const double gM = 2.0 * ((double)gSig[k][0] * H.M[0][j] + (double)gSig[k][1] * H.M[1][j] +
                               (double)gSig[k][2] * H.M[2][j]);
      gs[j] += gM * H.Rq[k][j];
      gR[k][j] = gM * H.s[j];
    }
  const double w = H.q[0], x = H.q[1], y = H.q[2], z = H.q[3];
  double gq[4];
  gq[0] = 2.0 * (-z * gR[0][1] + y * gR[0][2] + z * gR[1][0] - x * gR[1][2] - y * gR[2][0] + x * gR[2][1]);
  gq[1] = 2.0 * (y * gR[0][1] + z * gR[0][2] + y * gR[1][0] - 2.0 * x * gR[1][1] - w * gR[1][2] + z * gR[2][0] +
                 w * gR[2][1] - 2.0 * x * gR[2][2]);
  gq[2] = 2.0 * (-2.0 * y * gR[0][0] + x * gR[0][1] + w * gR[0][2] + x * gR[1][0] + z * gR[1][2] - w * gR[2][0] +
                 z * gR[2][1] - 2.0 * y * gR[2][2]);
  gq[3] = 2.0 * (-2.0 * z * gR[0][0] - w * gR[0][1] + x * gR[0][2] + w * gR[1][0] - 2.0 * z * gR[1][1] +
                 y * gR[1][2] + x * gR[2][0] + y * gR[2][1]);
  const double qd = gq[0] * w + gq[1] * x + gq[2] * y + gq[3] * z;

  double outv[11];
  for (int k = 0; k < 3; ++k) outv[k] = gm[k];
  for (int k = 0; k < 3; ++k) outv[3 + k] = gs[k] * H.s[k];
  for (int k = 0; k < 4; ++k) outv[6 + k] = (gq[k] - H.q[k] * qd) / H.qn;
  outv[10] = (double)go * H.o * (1.0 - H.o);
  if (adam) {
    const uint32_t k = step_old + 1u;
    step[g] = k;
    float bc1, bc2;
    adam_bias(a, k, bc1, bc2);
    const float factor = fold_factor ? (fc > 0 ? fs / (float)fc : fall / (float)a.n_views)
                                     : adam_view_factor(a, touched, n, g);
    constexpr int ROWS = 11 + 3 * K, B = 8;
    float grv[ROWS];
#pragma unroll
    for (int r = 0; r < ROWS; ++r) grv[r] = r < 11 ? (float)outv[r] : gf[r - 11];
    // rows in groups of B, the loads of the next group issued before this group's
    // arithmetic and stores (rows of one thread never alias: each group's loads
    // precede its own stores, and no group reads another's rows)
    float np[B], nm[B], nv[B];
#pragma unroll
    for (int j = 0; j < B; ++j) {
      if (j < ROWS) {
        const size_t i = (size_t)j * stride + g;
        np[j] = P[i];
        nm[j] = M[i];
        nv[j] = Vv[i];
      }
    }
#pragma unroll
    for (int r0 = 0; r0 < ROWS; r0 += B) {
      float pp[B], mm[B], vv[B];
#pragma unroll
      for (int j = 0; j < B; ++j) {
        pp[j] = np[j];
        mm[j] = nm[j];
        vv[j] = nv[j];
      }
#pragma unroll
      for (int j = 0; j < B; ++j) {
        if (r0 + B + j < ROWS) {
          const size_t i = (size_t)(r0 + B + j) * stride + g;
          np[j] = P[i];
          nm[j] = M[i];
          nv[j] = Vv[i];
        }
      }
#pragma unroll
      for (int j = 0; j < B; ++j) {
        const int r = r0 + j;
        if (r < ROWS) {
          const int grp = adam_row_group(r);
          const float lr = ((a.group_mask >> grp) & 1u) ? a.lr[grp] * factor : a.lr[grp];
          adam_elem(pp[j], mm[j], vv[j], grv[r], lr, a, bc1, bc2);
          const size_t i = (size_t)r * stride + g;
          if (out) out[i] = grv[r];
          P[i] = pp[j];
          M[i] = mm[j];
          Vv[i] = vv[j];
        }
      }
    }
    return;
  }
  for (int r = 0; r < 11; ++r) {
    float* dst = out + (size_t)r * stride + g;
    *dst = accumulate ? *dst + (float)outv[r] : (float)outv[r];
  }
#pragma unroll
  for (int i = 0; i < 3 * K; ++i) {
    float* dst = out + (size_t)(11 + i) * stride + g;
    *dst = accumulate ? *dst + gf[i] : gf[i];
  }
}

__global__ void k_fill_u32(uint32_t* __restrict__ p, uint32_t value, size_t count) {
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < count; i += (size_t)gridDim.x * blockDim.x)
    p[i] = value;
}

}  // namespace

hipError_t launch_preprocess(const float* P, int n, int stride, int D, const ViewDev* views, int V, Record* rec,
                             uint32_t* depth, uint32_t* touched, ushort4* rect, DevStatus* st, hipStream_t s) {
  const int blocks = (n + 255) / 256;
  switch (D) {
    case 0: hipLaunchKernelGGL(k_preprocess<0>, dim3(blocks), dim3(256), 0, s, P, n, stride, views, V, rec, depth, touched, rect, st); break;
    case 1: hipLaunchKernelGGL(k_preprocess<1>, dim3(blocks), dim3(256), 0, s, P, n, stride, views, V, rec, depth, touched, rect, st); break;
    case 2: hipLaunchKernelGGL(k_preprocess<2>, dim3(blocks), dim3(256), 0, s, P, n, stride, views, V, rec, depth, touched, rect, st); break;
    default: hipLaunchKernelGGL(k_preprocess<3>, dim3(blocks), dim3(256), 0, s, P, n, stride, views, V, rec, depth, touched, rect, st); break;
  }
  return hipGetLastError();
}

hipError_t launch_bwd(float* P, int n, int stride, int D, const ViewDev* views, int V, const uint32_t* touched,
                      const float* grad2d, float* grad, int accumulate, int adam, float* M, float* Vv, uint32_t* step,
                      const AdamArgs& a, const DevStatus* st, hipStream_t s) {
  const int blocks = (n + 255) / 256;
  switch (D) {
    case 0: hipLaunchKernelGGL(k_preprocess_bwd<0>, dim3(blocks), dim3(256), 0, s, P, n, stride, views, V, touched, grad2d, grad, accumulate, adam, M, Vv, step, a, st); break;
    case 1: hipLaunchKernelGGL(k_preprocess_bwd<1>, dim3(blocks), dim3(256), 0, s, P, n, stride, views, V, touched, grad2d, grad, accumulate, adam, M, Vv, step, a, st); break;
    case 2: hipLaunchKernelGGL(k_preprocess_bwd<2>, dim3(blocks), dim3(256), 0, s, P, n, stride, views, V, touched, grad2d, grad, accumulate, adam, M, Vv, step, a, st); break;
    default: hipLaunchKernelGGL(k_preprocess_bwd<3>, dim3(blocks), dim3(256), 0, s, P, n, stride, views, V, touched, grad2d, grad, accumulate, adam, M, Vv, step, a, st); break;
  }
  return hipGetLastError();
}

hipError_t launch_preprocess_bwd(const float* P, int n, int stride, int D, const ViewDev* views, int V,
                                 const uint32_t* touched, const float* grad2d, float* grad, int accumulate,
                                 hipStream_t s) {
  // the plain backward reads the parameters only
  return launch_bwd(const_cast<float*>(P), n, stride, D, views, V, touched, grad2d, grad, accumulate, 0, nullptr,
                    nullptr, nullptr, AdamArgs{}, nullptr, s);
}

hipError_t launch_preprocess_bwd_adam(float* P, int n, int stride, int D, const ViewDev* views, int V,
                                      const uint32_t* touched, const float* grad2d, float* grad, float* M, float* Vv,
                                      uint32_t* step, const AdamArgs& a, const DevStatus* st, hipStream_t s) {
  return launch_bwd(P, n, stride, D, views, V, touched, grad2d, grad, 0, 1, M, Vv, step, a, st, s);
}

hipError_t launch_fill_u32(uint32_t* p, uint32_t value, size_t count, hipStream_t s) {
  if (count == 0) return hipSuccess;
  size_t blocks = (count + 255) / 256;
  if (blocks > 65536) blocks = 65536;
  hipLaunchKernelGGL(k_fill_u32, dim3((unsigned)blocks), dim3(256), 0, s, p, value, count);
  return hipGetLastError();
}

}  // namespace gsk
