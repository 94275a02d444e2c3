// FP64 per-view geometry of one Gaussian, shared by the projection kernel and
// the binning kernels' exact cutoff test.  Sec. III Eq. 1 (covariance
// R S S^T R^T) and the EWA splatting of the original 3DGS configuration
// (Sec. V-A): camera transform, near cull, pinhole projection, clamped projection
// Jacobian, 2D covariance J W Sigma W^T J^T + 0.3 I, conic, extent
// 3 sqrt(lambda_max), tile rect and cutoff exponent.  Every value is an IEEE FP64
// evaluation in a fixed operation order with contraction off, so any kernel that
// includes this header derives the same bits from the same fp32 parameters.
#pragma once

#include "gs_internal.h"

namespace gsk {

// View-independent quantities of one Gaussian.
struct Gauss {
  double m[3];
  double s[3];
  double q[4];     // unit quaternion w, x, y, z
  double qn;       // |q| before normalisation
  double o;        // opacity
  double Rq[3][3];
  double M[3][3];  // Rq diag(s)
  double Sig[3][3];
};

__device__ inline void load_gauss(const float* __restrict__ P, int stride, int g, Gauss& G) {
#pragma clang fp contract(off)
  for (int i = 0; i < 3; ++i) G.m[i] = (double)P[(size_t)i * stride + g];
  for (int i = 0; i < 3; ++i) G.s[i] = exp((double)P[(size_t)(3 + i) * stride + g]);
  const double qw = P[(size_t)6 * stride + g], qx = P[(size_t)7 * stride + g];
  const double qy = P[(size_t)8 * stride + g], qz = P[(size_t)9 * stride + g];
  G.qn = sqrt(((qw * qw + qx * qx) + qy * qy) + qz * qz);
  const double w = qw / G.qn, x = qx / G.qn, y = qy / G.qn, z = qz / G.qn;
  G.q[0] = w; G.q[1] = x; G.q[2] = y; G.q[3] = z;
  G.o = 1.0 / (1.0 + exp(-(double)P[(size_t)10 * stride + g]));
  G.Rq[0][0] = 1.0 - 2.0 * (y * y + z * z);
  G.Rq[0][1] = 2.0 * (x * y - w * z);
  G.Rq[0][2] = 2.0 * (x * z + w * y);
  G.Rq[1][0] = 2.0 * (x * y + w * z);
  G.Rq[1][1] = 1.0 - 2.0 * (x * x + z * z);
  G.Rq[1][2] = 2.0 * (y * z - w * x);
  G.Rq[2][0] = 2.0 * (x * z - w * y);
  G.Rq[2][1] = 2.0 * (y * z + w * x);
  G.Rq[2][2] = 1.0 - 2.0 * (x * x + y * y);
  for (int k = 0; k < 3; ++k)
    for (int j = 0; j < 3; ++j) G.M[k][j] = G.Rq[k][j] * G.s[j];
  for (int k = 0; k < 3; ++k)
    for (int l = 0; l < 3; ++l)
      G.Sig[k][l] = (G.M[k][0] * G.M[l][0] + G.M[k][1] * G.M[l][1]) + G.M[k][2] * G.M[l][2];
}

// Per-view quantities of one Gaussian.
struct Proj {
  bool visible;
  bool clx, cly;       // Jacobian clamp active on x / y
  double tx, ty, tz;   // camera-space mean (tz replaced by 1 when culled)
  double u, w;
  double txc, tyc;
  double J00, J02, J11, J12;
  double T0[3], T1[3];
  double S00, S01, S11;
  double a, b, c;
  double r;
  int tx0, tx1, ty0, ty1;
};

__device__ inline void project(const Gauss& G, const ViewDev& V, Proj& p) {
#pragma clang fp contract(off)
  double R[3][3], t[3];
  for (int i = 0; i < 3; ++i) {
    for (int j = 0; j < 3; ++j) R[i][j] = (double)V.R[3 * i + j];
    t[i] = (double)V.t[i];
  }
  const double fx = V.fx, fy = V.fy, cx = V.cx, cy = V.cy;
  const double tx = ((R[0][0] * G.m[0] + R[0][1] * G.m[1]) + R[0][2] * G.m[2]) + t[0];
  const double ty = ((R[1][0] * G.m[0] + R[1][1] * G.m[1]) + R[1][2] * G.m[2]) + t[1];
  const double tz0 = ((R[2][0] * G.m[0] + R[2][1] * G.m[1]) + R[2][2] * G.m[2]) + t[2];
  const bool in_front = tz0 > kZNear;
  const double tz = in_front ? tz0 : 1.0;
  p.tx = tx; p.ty = ty; p.tz = tz;
  p.u = (fx * tx) / tz + cx;
  p.w = (fy * ty) / tz + cy;
  const double limx = (kJacClamp * (0.5 * (double)V.W)) / fx;
  const double limy = (kJacClamp * (0.5 * (double)V.H)) / fy;
  const double rx = tx / tz, ry = ty / tz;
  p.clx = !(rx >= -limx && rx <= limx);
  p.cly = !(ry >= -limy && ry <= limy);
  p.txc = tz * fmin(fmax(rx, -limx), limx);
  p.tyc = tz * fmin(fmax(ry, -limy), limy);
  p.J00 = fx / tz;
  p.J02 = -(fx * p.txc) / (tz * tz);
  p.J11 = fy / tz;
  p.J12 = -(fy * p.tyc) / (tz * tz);
  for (int k = 0; k < 3; ++k) {
    p.T0[k] = p.J00 * R[0][k] + p.J02 * R[2][k];
    p.T1[k] = p.J11 * R[1][k] + p.J12 * R[2][k];
  }
  double U0[3], U1[3];
  for (int l = 0; l < 3; ++l) {
    U0[l] = (p.T0[0] * G.Sig[0][l] + p.T0[1] * G.Sig[1][l]) + p.T0[2] * G.Sig[2][l];
    U1[l] = (p.T1[0] * G.Sig[0][l] + p.T1[1] * G.Sig[1][l]) + p.T1[2] * G.Sig[2][l];
  }
  p.S00 = ((U0[0] * p.T0[0] + U0[1] * p.T0[1]) + U0[2] * p.T0[2]) + kKappa;
  p.S01 = (U0[0] * p.T1[0] + U0[1] * p.T1[1]) + U0[2] * p.T1[2];
  p.S11 = ((U1[0] * p.T1[0] + U1[1] * p.T1[1]) + U1[2] * p.T1[2]) + kKappa;
  const double det = p.S00 * p.S11 - p.S01 * p.S01;
  const bool det_ok = det > 0.0;
  const double dets = det_ok ? det : 1.0;
  p.a = p.S11 / dets;
  p.b = -p.S01 / dets;
  p.c = p.S00 / dets;
  const double dd = p.S00 - p.S11;
  const double lam = 0.5 * (p.S00 + p.S11) + sqrt(0.25 * (dd * dd) + p.S01 * p.S01);
  p.r = kExtentSigmas * sqrt(lam);
  // pixel rect: centres within [u - r, u + r] x [w - r, w + r] inside the image
  const double xlo = ceil((p.u - p.r) - 0.5), xhi = floor((p.u + p.r) - 0.5);
  const double ylo = ceil((p.w - p.r) - 0.5), yhi = floor((p.w + p.r) - 0.5);
  const int W = V.W, H = V.H;
  const int i0 = isnan(xlo) ? W : (int)fmin(fmax(xlo, 0.0), (double)W);
  const int i1 = isnan(xhi) ? -1 : (int)fmin(fmax(xhi, -1.0), (double)(W - 1));
  const int j0 = isnan(ylo) ? H : (int)fmin(fmax(ylo, 0.0), (double)H);
  const int j1 = isnan(yhi) ? -1 : (int)fmin(fmax(yhi, -1.0), (double)(H - 1));
  p.visible = in_front && det_ok && i0 <= i1 && j0 <= j1;
  p.tx0 = i0 / V.tile; p.tx1 = i1 / V.tile;
  p.ty0 = j0 / V.tile; p.ty1 = j1 / V.tile;
}

// Cutoff exponent tau = max(-4.5, -ln(255 o)): the exponent at which a splat's
// alpha falls to 1/255, floored at the 3-sigma ellipse.
__device__ inline double cutoff_tau(double o) {
#pragma clang fp contract(off)
  const double tau = -log(kAlphaMinInv * o);
  return tau < kCutoffFloor ? kCutoffFloor : tau;
}

// The cutoff region of Gaussian g in view V from its FP64 conic and cutoff (the
// definition the pair lists follow); only called where the fp32 clear-case test
// cannot decide, so the projection is recomputed from the parameters instead of
// being stored.
__device__ __noinline__ inline CutoffGeo exact_cutoff_geo(const float* __restrict__ P, int stride, int g,
                                                           const ViewDev& V) {
#pragma clang fp contract(off)
  Gauss G;
  load_gauss(P, stride, g, G);
  Proj p;
  project(G, V, p);
  CutoffGeo c;
  c.u = p.u;
  c.w = p.w;
  c.a = p.a;
  c.b = p.b;
  c.c = p.c;
  c.nbc = -c.b / c.c;
  c.nba = -c.b / c.a;
  c.lim = -2.0 * cutoff_tau(G.o);
  return c;
}

}  // namespace gsk
