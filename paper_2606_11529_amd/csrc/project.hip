// Projection of 3D Gaussians (listing "Implementation of XPR-3DGS",
// function project) and its backward, one thread per (view, Gaussian).
//
// Inputs are structure-of-arrays, so each component load of a wave is one
// coalesced 256-byte read; the kernel is bound by HBM traffic (236 bytes in,
// 64 bytes out per Gaussian at SH degree 3), not by its arithmetic.
#include "xpr_internal.h"

namespace xpr {

// Real spherical harmonics (Condon-Shortley phase kept; m = -l..l), values
// of the closed forms sqrt((2l+1)/(4 pi) (l-|m|)!/(l+|m|)!) (times sqrt 2
// for m != 0) and the Cartesian polynomials they multiply.
constexpr float kY0 = 0.28209479177387814f;   // 1 / (2 sqrt(pi))
constexpr float kY1 = 0.48860251190291992f;   // sqrt(3 / (4 pi))
constexpr float kY2a = 1.0925484305920792f;   // sqrt(15 / pi) / 2
constexpr float kY2b = 0.31539156525252005f;  // sqrt(5 / pi) / 4
constexpr float kY2c = 0.54627421529603959f;  // sqrt(15 / pi) / 4
constexpr float kY3a = 0.59004358992664352f;  // sqrt(35 / (2 pi)) / 4
constexpr float kY3b = 2.8906114426405538f;   // sqrt(105 / pi) / 2
constexpr float kY3c = 0.45704579946446577f;  // sqrt(21 / (2 pi)) / 4
constexpr float kY3d = 0.37317633259011546f;  // sqrt(7 / pi) / 4
constexpr float kY3e = 1.4453057213202769f;   // sqrt(105 / pi) / 4

template <int DEG>
__device__ __forceinline__ void sh_basis(float x, float y, float z, float* Y) {
  Y[0] = kY0;
  if (DEG >= 1) {
    Y[1] = -kY1 * y;
    Y[2] = kY1 * z;
    Y[3] = -kY1 * x;
  }
  if (DEG >= 2) {
    const float xx = x * x, yy = y * y, zz = z * z;
    Y[4] = kY2a * x * y;
    Y[5] = -kY2a * y * z;
    Y[6] = kY2b * (2.f * zz - xx - yy);
    Y[7] = -kY2a * x * z;
    Y[8] = kY2c * (xx - yy);
    if (DEG >= 3) {
      Y[9] = -kY3a * y * (3.f * xx - yy);
      Y[10] = kY3b * x * y * z;
      Y[11] = -kY3c * y * (4.f * zz - xx - yy);
      Y[12] = kY3d * z * (2.f * zz - 3.f * xx - 3.f * yy);
      Y[13] = -kY3c * x * (4.f * zz - xx - yy);
      Y[14] = kY3e * z * (xx - yy);
      Y[15] = -kY3a * x * (xx - 3.f * yy);
    }
  }
}

// Gradient of sum_j w_j Y_j with respect to (x, y, z).
template <int DEG>
__device__ __forceinline__ void sh_basis_vjp(float x, float y, float z, const float* w,
                                             float& gx, float& gy, float& gz) {
  gx = gy = gz = 0.f;
  if (DEG >= 1) {
    gy -= kY1 * w[1];
    gz += kY1 * w[2];
    gx -= kY1 * w[3];
  }
  if (DEG >= 2) {
    gx += kY2a * y * w[4];
    gy += kY2a * x * w[4];
    gy -= kY2a * z * w[5];
    gz -= kY2a * y * w[5];
    gx -= 2.f * kY2b * x * w[6];
    gy -= 2.f * kY2b * y * w[6];
    gz += 4.f * kY2b * z * w[6];
    gx -= kY2a * z * w[7];
    gz -= kY2a * x * w[7];
    gx += 2.f * kY2c * x * w[8];
    gy -= 2.f * kY2c * y * w[8];
  }
  if (DEG >= 3) {
    const float xx = x * x, yy = y * y, zz = z * z;
    gx -= 6.f * kY3a * x * y * w[9];
    gy -= kY3a * (3.f * xx - 3.f * yy) * w[9];
    gx += kY3b * y * z * w[10];
    gy += kY3b * x * z * w[10];
    gz += kY3b * x * y * w[10];
    gx += 2.f * kY3c * x * y * w[11];
    gy -= kY3c * (4.f * zz - xx - 3.f * yy) * w[11];
    gz -= 8.f * kY3c * y * z * w[11];
    gx -= 6.f * kY3d * x * z * w[12];
    gy -= 6.f * kY3d * y * z * w[12];
    gz += kY3d * (6.f * zz - 3.f * xx - 3.f * yy) * w[12];
    gx -= kY3c * (4.f * zz - 3.f * xx - yy) * w[13];
    gy += 2.f * kY3c * x * y * w[13];
    gz -= 8.f * kY3c * x * z * w[13];
    gx += 2.f * kY3e * x * z * w[14];
    gy -= 2.f * kY3e * y * z * w[14];
    gz += kY3e * (xx - yy) * w[14];
    gx -= kY3a * (3.f * xx - 3.f * yy) * w[15];
    gy += 6.f * kY3a * x * y * w[15];
  }
}

// Everything the forward computes for one (view, Gaussian), kept so the
// backward can reuse it after recomputation. The geometric chain runs in
// FP64: on CDNA4 a double FMA issues at the per-lane rate of an unpacked
// float one and this kernel is bound by HBM traffic, so the extra precision
// is free, and it keeps the 2x2 inverse (condition numbers up to ~1e5 for
// needle-like Gaussians near the camera) and its derivative accurate.
struct ProjState {
  double t[3];           // camera-space mean
  double qn[4], qinv;    // unit quaternion, 1/|q|
  double Rq[9];          // rotation of the Gaussian
  double s[3];           // scales
  double Sig[6];         // 3D covariance 00 01 02 11 12 22
  double rx, ry;         // (clamped) tx/tz, ty/tz
  bool clampx, clampy;
  double T0[3], T1[3];   // rows of J W
  double a, b, c, det;   // low-passed 2D covariance
  double con0, con1, con2;
  double u, v;
  int rect[4];
  int tc;
  double dir[3], dinv;   // unit view direction, 1/distance
};

// STREAM_SH: the forward projection reads the SH coefficients (192 of its
// 236 bytes per Gaussian at degree 3) exactly once, so it loads them
// non-temporally and they do not displace cached data (measured: 188 ->
// 173 us for 3M Gaussians; the same for means, quaternions and scales, or
// streaming stores of the backward's gradients, was slower). The backward
// reads them a second time and keeps the default.
template <int DEG, bool STREAM_SH = false>
__device__ __forceinline__ void project_core(const Batch& B, const ViewDev& V, const SceneDev& S,
                                             int i, ProjState& P, float* colour, float* raw) {
  const double mx = S.means[i], my = S.means[S.ld + i], mz = S.means[2 * S.ld + i];
  double R[9];
#pragma unroll
  for (int k = 0; k < 9; ++k) R[k] = V.R[k];
  P.t[0] = R[0] * mx + R[1] * my + R[2] * mz + (double)V.t[0];
  P.t[1] = R[3] * mx + R[4] * my + R[5] * mz + (double)V.t[1];
  P.t[2] = R[6] * mx + R[7] * my + R[8] * mz + (double)V.t[2];
  const double tx = P.t[0], ty = P.t[1], tz = P.t[2];
  const double fx = V.fx, fy = V.fy;

  // Sigma = Rq diag(s^2) Rq^T
  const double qw = S.quats[i], qx = S.quats[S.ld + i], qy = S.quats[2 * S.ld + i],
               qz = S.quats[3 * S.ld + i];
  const double qlen = sqrt(qw * qw + qx * qx + qy * qy + qz * qz);
  P.qinv = 1.0 / qlen;
  const double w = qw * P.qinv, x = qx * P.qinv, y = qy * P.qinv, z = qz * P.qinv;
  P.qn[0] = w; P.qn[1] = x; P.qn[2] = y; P.qn[3] = z;
  double* Q = P.Rq;
  Q[0] = 1.0 - 2.0 * (y * y + z * z); Q[1] = 2.0 * (x * y - w * z); Q[2] = 2.0 * (x * z + w * y);
  Q[3] = 2.0 * (x * y + w * z); Q[4] = 1.0 - 2.0 * (x * x + z * z); Q[5] = 2.0 * (y * z - w * x);
  Q[6] = 2.0 * (x * z - w * y); Q[7] = 2.0 * (y * z + w * x); Q[8] = 1.0 - 2.0 * (x * x + y * y);
  P.s[0] = S.scales[i]; P.s[1] = S.scales[S.ld + i]; P.s[2] = S.scales[2 * S.ld + i];
  double M[9];
#pragma unroll
  for (int r = 0; r < 3; ++r)
#pragma unroll
    for (int k = 0; k < 3; ++k) M[3 * r + k] = Q[3 * r + k] * P.s[k];
  P.Sig[0] = M[0] * M[0] + M[1] * M[1] + M[2] * M[2];
  P.Sig[1] = M[0] * M[3] + M[1] * M[4] + M[2] * M[5];
  P.Sig[2] = M[0] * M[6] + M[1] * M[7] + M[2] * M[8];
  P.Sig[3] = M[3] * M[3] + M[4] * M[4] + M[5] * M[5];
  P.Sig[4] = M[3] * M[6] + M[4] * M[7] + M[5] * M[8];
  P.Sig[5] = M[6] * M[6] + M[7] * M[7] + M[8] * M[8];

  // EWA: T = J W with J the perspective Jacobian at the clamped direction.
  const double limx = (double)B.fov_clip * V.W / (2.0 * fx);
  const double limy = (double)B.fov_clip * V.H / (2.0 * fy);
  double rx = tx / tz, ry = ty / tz;
  P.clampx = P.clampy = false;
  if (B.fov_clip > 0.f) {
    P.clampx = rx < -limx || rx > limx;
    P.clampy = ry < -limy || ry > limy;
    rx = fmin(limx, fmax(-limx, rx));
    ry = fmin(limy, fmax(-limy, ry));
  }
  P.rx = rx; P.ry = ry;
  const double j00 = fx / tz, j02 = -fx * rx / tz;
  const double j11 = fy / tz, j12 = -fy * ry / tz;
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    P.T0[k] = j00 * R[k] + j02 * R[6 + k];
    P.T1[k] = j11 * R[3 + k] + j12 * R[6 + k];
  }
  const double* Sg = P.Sig;
  const double S0[3] = {Sg[0] * P.T0[0] + Sg[1] * P.T0[1] + Sg[2] * P.T0[2],
                        Sg[1] * P.T0[0] + Sg[3] * P.T0[1] + Sg[4] * P.T0[2],
                        Sg[2] * P.T0[0] + Sg[4] * P.T0[1] + Sg[5] * P.T0[2]};
  const double S1[3] = {Sg[0] * P.T1[0] + Sg[1] * P.T1[1] + Sg[2] * P.T1[2],
                        Sg[1] * P.T1[0] + Sg[3] * P.T1[1] + Sg[4] * P.T1[2],
                        Sg[2] * P.T1[0] + Sg[4] * P.T1[1] + Sg[5] * P.T1[2]};
  const double lp = B.lowpass;
  P.a = P.T0[0] * S0[0] + P.T0[1] * S0[1] + P.T0[2] * S0[2] + lp;
  P.b = P.T0[0] * S1[0] + P.T0[1] * S1[1] + P.T0[2] * S1[2];
  P.c = P.T1[0] * S1[0] + P.T1[1] * S1[1] + P.T1[2] * S1[2] + lp;
  P.det = P.a * P.c - P.b * P.b;
  const double dinv = P.det > 0.0 ? 1.0 / P.det : 0.0;
  P.con0 = P.c * dinv;
  P.con1 = -P.b * dinv;
  P.con2 = P.a * dinv;
  P.u = fx * tx / tz + (double)V.cx - 0.5;
  P.v = fy * ty / tz + (double)V.cy - 0.5;

  // Extents, radius, tile rect, tile count: the 3-sigma radius of the
  // largest eigenvalue, or (opacity-aware) the half-widths of the ellipse
  // where o G = alpha_min.
  const float o = S.opac[i];
  double ex, ey, rad;
  if (B.opacity_extents) {
    const double lvl = 2.0 * log((double)o / (double)B.alpha_min);
    ex = lvl > 0.0 ? sqrt(lvl * P.a) : 0.0;
    ey = lvl > 0.0 ? sqrt(lvl * P.c) : 0.0;
    rad = fmax(ex, ey);
  } else {
    const double mid = 0.5 * (P.a + P.c);
    const double lam = mid + sqrt(fmax(0.0, mid * mid - P.det));
    rad = ceil(3.0 * sqrt(lam));
    ex = ey = rad;
  }
  const double tw = B.tile_w, th = B.tile_h;
  const double txn = V.tiles_x, tyn = V.tiles_y;
  P.rect[0] = (int)fmin(txn, fmax(0.0, floor((P.u - ex) / tw)));
  P.rect[1] = (int)fmin(tyn, fmax(0.0, floor((P.v - ey) / th)));
  P.rect[2] = (int)fmin(txn, fmax(0.0, floor((P.u + ex) / tw) + 1.0));
  P.rect[3] = (int)fmin(tyn, fmax(0.0, floor((P.v + ey) / th) + 1.0));
  const int area = (P.rect[2] - P.rect[0]) * (P.rect[3] - P.rect[1]);
  const bool visible = tz > (double)B.z_near && P.det > 0.0 && o >= B.alpha_min && rad > 0.0 &&
                       area > 0;
  P.tc = visible ? area : 0;

  // View-dependent colour (SH in float: a well-conditioned sum).
  const double cpx = -(R[0] * V.t[0] + R[3] * V.t[1] + R[6] * V.t[2]);
  const double cpy = -(R[1] * V.t[0] + R[4] * V.t[1] + R[7] * V.t[2]);
  const double cpz = -(R[2] * V.t[0] + R[5] * V.t[1] + R[8] * V.t[2]);
  const double dx = mx - cpx, dy = my - cpy, dz = mz - cpz;
  P.dinv = 1.0 / sqrt(dx * dx + dy * dy + dz * dz);
  P.dir[0] = dx * P.dinv; P.dir[1] = dy * P.dinv; P.dir[2] = dz * P.dinv;
  float Y[16];
  sh_basis<DEG>((float)P.dir[0], (float)P.dir[1], (float)P.dir[2], Y);
  constexpr int NB = (DEG + 1) * (DEG + 1);
#pragma unroll
  for (int ch = 0; ch < 3; ++ch) {
    float acc = 0.5f;
#pragma unroll
    for (int j = 0; j < NB; ++j) {
      const float* p = S.sh + (size_t)(3 * j + ch) * S.ld + i;
      acc += (STREAM_SH ? __builtin_nontemporal_load(p) : *p) * Y[j];
    }
    raw[ch] = acc;
    colour[ch] = fmaxf(0.f, acc);
  }
}

template <int DEG>
__global__ __launch_bounds__(256) void k_project(Batch B, float4* __restrict__ splat,
                                                 float* __restrict__ depth,
                                                 short4* __restrict__ rect,
                                                 int32_t* __restrict__ tc) {
  const ViewDev& V = B.v[blockIdx.y];
  const SceneDev& S = B.s[V.scene];
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i >= S.n) return;
  ProjState P;
  float col[3], raw[3];
  project_core<DEG, true>(B, V, S, i, P, col, raw);
  const int r = V.rec_off + i;
  const float o = S.opac[i];
  splat[3 * (size_t)r + 0] =
      make_float4((float)P.u, (float)P.v, (float)(-0.5 * P.con0), (float)(-P.con1));
  splat[3 * (size_t)r + 1] = make_float4((float)(-0.5 * P.con2), o, col[0], col[1]);
  splat[3 * (size_t)r + 2] = make_float4(col[2], 0.f, 0.f, 0.f);
  depth[r] = (float)P.t[2];
  rect[r] = P.tc > 0 ? make_short4((short)P.rect[0], (short)P.rect[1], (short)P.rect[2],
                                   (short)P.rect[3])
                     : make_short4(0, 0, 0, 0);
  tc[r] = P.tc;
}

// Backward of Rq(q / |q|), the rotation of the normalised quaternion
// (w, x, y, z) = qn: dL/dq added to gq from dL/dRq (row-major) in gR.
__device__ __forceinline__ void quat_vjp(const double* qn, double qinv, const double* gR,
                                         double* gq) {
  const double w = qn[0], x = qn[1], y = qn[2], z = qn[3];
  const double gw = 2.0 * (-z * gR[1] + y * gR[2] + z * gR[3] - x * gR[5] - y * gR[6] + x * gR[7]);
  const double gx = 2.0 * (y * gR[1] + z * gR[2] + y * gR[3] - w * gR[5] + z * gR[6] + w * gR[7]) -
                    4.0 * x * (gR[4] + gR[8]);
  const double gy = 2.0 * (x * gR[1] + w * gR[2] + x * gR[3] + z * gR[5] - w * gR[6] + z * gR[7]) -
                    4.0 * y * (gR[0] + gR[8]);
  const double gz = 2.0 * (-w * gR[1] + x * gR[2] + w * gR[3] + y * gR[5] + x * gR[6] + y * gR[7]) -
                    4.0 * z * (gR[0] + gR[4]);
  const double qd = w * gw + x * gx + y * gy + z * gz;
  gq[0] += (gw - w * qd) * qinv;
  gq[1] += (gx - x * qd) * qinv;
  gq[2] += (gy - y * qd) * qinv;
  gq[3] += (gz - z * qd) * qinv;
}

__device__ __forceinline__ GradDev grad_dest(int sidx, const GradDev& G0, const GradDev& G1,
                                             const GradDev& G2, const GradDev& G3,
                                             const GradDev& G4, const GradDev& G5,
                                             const GradDev& G6, const GradDev& G7) {
  switch (sidx) {
    case 0: return G0;
    case 1: return G1;
    case 2: return G2;
    case 3: return G3;
    case 4: return G4;
    case 5: return G5;
    case 6: return G6;
    default: return G7;
  }
}

// Writes (or, with accumulate, adds) one Gaussian's parameter gradients;
// overwriting also zeroes the SH coefficients above the rendered degree.
template <int NB>
__device__ __forceinline__ void store_param_grads(const GradDev& G, const SceneDev& S, int i,
                                                  const double (&gmu)[3], const double (&gs)[3],
                                                  const double (&gq)[4], float go,
                                                  const float (&gsh)[NB][3], int accumulate) {
  const size_t ld = S.ld;
  if (accumulate) {
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      G.means[k * ld + i] += (float)gmu[k];
      G.scales[k * ld + i] += (float)gs[k];
    }
#pragma unroll
    for (int k = 0; k < 4; ++k) G.quats[k * ld + i] += (float)gq[k];
    G.opac[i] += go;
#pragma unroll
    for (int j = 0; j < NB; ++j)
#pragma unroll
      for (int ch = 0; ch < 3; ++ch) G.sh[(3 * j + ch) * ld + i] += gsh[j][ch];
  } else {
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      G.means[k * ld + i] = (float)gmu[k];
      G.scales[k * ld + i] = (float)gs[k];
    }
#pragma unroll
    for (int k = 0; k < 4; ++k) G.quats[k * ld + i] = (float)gq[k];
    G.opac[i] = go;
#pragma unroll
    for (int j = 0; j < NB; ++j)
#pragma unroll
      for (int ch = 0; ch < 3; ++ch) G.sh[(3 * j + ch) * ld + i] = gsh[j][ch];
    for (int j = NB; j < S.K; ++j)
      for (int ch = 0; ch < 3; ++ch) G.sh[(3 * j + ch) * ld + i] = 0.f;
  }
}

// Backward of the projection for one Gaussian of scene blockIdx.y, summed
// over the views that render it. grad2d [records][9] holds dL/d(u, v, A, B,
// C, o, r, g, b). Chain: shader data -> conic -> 2D covariance -> (J W,
// Sigma) -> (camera-space mean, scales, rotation -> quaternion); mean2D ->
// camera-space mean -> world mean; colour -> SH coefficients and direction.
// Writes (or, with accumulate, adds) one Gaussian's mean, scale, quaternion
// and opacity gradients. The SH gradients were written view by view
// (sh_out: at least one view wrote them); overwriting zeroes those no view
// wrote and those above the rendered degree (NB coefficients).
__device__ __forceinline__ void store_geom_grads(const GradDev& G, const SceneDev& S, int i,
                                                 const double (&gmu)[3], const double (&gs)[3],
                                                 const double (&gq)[4], float go, int accumulate,
                                                 bool sh_out, int NB) {
  const size_t ld = S.ld;
  if (accumulate) {
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      G.means[k * ld + i] += (float)gmu[k];
      G.scales[k * ld + i] += (float)gs[k];
    }
#pragma unroll
    for (int k = 0; k < 4; ++k) G.quats[k * ld + i] += (float)gq[k];
    G.opac[i] += go;
  } else {
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      G.means[k * ld + i] = (float)gmu[k];
      G.scales[k * ld + i] = (float)gs[k];
    }
#pragma unroll
    for (int k = 0; k < 4; ++k) G.quats[k * ld + i] = (float)gq[k];
    G.opac[i] = go;
    for (int j = sh_out ? NB : 0; j < S.K; ++j)
      for (int ch = 0; ch < 3; ++ch) G.sh[(3 * j + ch) * ld + i] = 0.f;
  }
}

// The SH part of one view's projection backward: colour = max(0, 0.5 +
// sum_j sh_j Y_j(dir)) with the channels' gradients gr (zero where the
// record's colour, max(0, raw), is 0). Writes dL/dsh (stores on the first
// view unless accumulating, adds after) and returns dL/ddir through wsum;
// each coefficient is read once.
template <int DEG>
__device__ __forceinline__ void sh_backward(const SceneDev& S, const GradDev& G, int i,
                                            const float (&Y)[16], float gr0, float gr1, float gr2,
                                            bool add, float (&wsum)[16]) {
  constexpr int NB = (DEG + 1) * (DEG + 1);
  const size_t ld = S.ld;
#pragma unroll
  for (int j = 0; j < NB; ++j) wsum[j] = 0.f;
#pragma unroll
  for (int ch = 0; ch < 3; ++ch) {
    const float gr = ch == 0 ? gr0 : (ch == 1 ? gr1 : gr2);
#pragma unroll
    for (int j = 0; j < NB; ++j) {
      const size_t o = (size_t)(3 * j + ch) * ld + i;
      const float v = Y[j] * gr;
      if (add)
        G.sh[o] += v;
      else
        G.sh[o] = v;
      wsum[j] += S.sh[o] * gr;
    }
  }
}

template <int DEG>
__global__ __launch_bounds__(256) void k_project_bwd(Batch B, const float* __restrict__ grad2d,
                                                     const int32_t* __restrict__ tc,
                                                     GradDev G0, GradDev G1, GradDev G2,
                                                     GradDev G3, GradDev G4, GradDev G5,
                                                     GradDev G6, GradDev G7, int accumulate) {
  const int sidx = blockIdx.y;
  const SceneDev& S = B.s[sidx];
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i >= S.n) return;
  constexpr int NB = (DEG + 1) * (DEG + 1);
  double gmu[3] = {0.0, 0.0, 0.0}, gs[3] = {0.0, 0.0, 0.0}, gq[4] = {0.0, 0.0, 0.0, 0.0};
  float go = 0.f;
  float gsh[NB][3];
#pragma unroll
  for (int j = 0; j < NB; ++j) gsh[j][0] = gsh[j][1] = gsh[j][2] = 0.f;

  for (int vi = 0; vi < B.n_views; ++vi) {
    const ViewDev& V = B.v[vi];
    if (V.scene != sidx) continue;
    const int r = V.rec_off + i;
    if (tc[r] == 0) continue;
    const float* g = grad2d + 9 * (size_t)r;
    const double gu = g[0], gv = g[1], gA = g[2], gB = g[3], gC = g[4];
    const float gcol[3] = {g[6], g[7], g[8]};
    go += g[5];
    ProjState P;
    float col[3], raw[3];
    project_core<DEG>(B, V, S, i, P, col, raw);
    double R[9];
#pragma unroll
    for (int k = 0; k < 9; ++k) R[k] = V.R[k];
    const double fx = V.fx, fy = V.fy;

    // colour = max(0, 0.5 + sum_j sh_j Y_j(dir))
    float Y[16];
    const float dxf = (float)P.dir[0], dyf = (float)P.dir[1], dzf = (float)P.dir[2];
    sh_basis<DEG>(dxf, dyf, dzf, Y);
    float graw[3];
#pragma unroll
    for (int ch = 0; ch < 3; ++ch) graw[ch] = raw[ch] > 0.f ? gcol[ch] : 0.f;
    float wsum[16];
#pragma unroll
    for (int j = 0; j < NB; ++j) {
      float acc = 0.f;
#pragma unroll
      for (int ch = 0; ch < 3; ++ch) {
        gsh[j][ch] += Y[j] * graw[ch];
        acc += S.sh[(size_t)(3 * j + ch) * S.ld + i] * graw[ch];
      }
      wsum[j] = acc;
    }
    float gdxf, gdyf, gdzf;
    sh_basis_vjp<DEG>(dxf, dyf, dzf, wsum, gdxf, gdyf, gdzf);
    const double gdx = gdxf, gdy = gdyf, gdz = gdzf;
    const double dd = P.dir[0] * gdx + P.dir[1] * gdy + P.dir[2] * gdz;
    gmu[0] += (gdx - P.dir[0] * dd) * P.dinv;
    gmu[1] += (gdy - P.dir[1] * dd) * P.dinv;
    gmu[2] += (gdz - P.dir[2] * dd) * P.dinv;

    // conic entries: con0 = c/det, con1 = -b/det, con2 = a/det
    const double gk0 = -0.5 * gA, gk1 = -gB, gk2 = -0.5 * gC;
    const double a = P.a, b = P.b, c = P.c;
    const double id2 = 1.0 / (P.det * P.det);
    const double ga = (-c * c * gk0 + b * c * gk1 - b * b * gk2) * id2;
    const double gb = (2.0 * b * c * gk0 - (a * c + b * b) * gk1 + 2.0 * a * b * gk2) * id2;
    const double gc = (-b * b * gk0 + a * b * gk1 - a * a * gk2) * id2;

    // a = T0 Sig T0, b = T0 Sig T1, c = T1 Sig T1 (Sig symmetric)
    const double* T0 = P.T0;
    const double* T1 = P.T1;
    const double* Sg = P.Sig;
    const double ST0[3] = {Sg[0] * T0[0] + Sg[1] * T0[1] + Sg[2] * T0[2],
                           Sg[1] * T0[0] + Sg[3] * T0[1] + Sg[4] * T0[2],
                           Sg[2] * T0[0] + Sg[4] * T0[1] + Sg[5] * T0[2]};
    const double ST1[3] = {Sg[0] * T1[0] + Sg[1] * T1[1] + Sg[2] * T1[2],
                           Sg[1] * T1[0] + Sg[3] * T1[1] + Sg[4] * T1[2],
                           Sg[2] * T1[0] + Sg[4] * T1[1] + Sg[5] * T1[2]};
    double gT0[3], gT1[3];
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      gT0[k] = 2.0 * ga * ST0[k] + gb * ST1[k];
      gT1[k] = gb * ST0[k] + 2.0 * gc * ST1[k];
    }
    // symmetric dL/dSigma (full matrix G + G^T)
    double Gs[3][3];
#pragma unroll
    for (int r2 = 0; r2 < 3; ++r2)
#pragma unroll
      for (int s2 = 0; s2 < 3; ++s2)
        Gs[r2][s2] = 2.0 * ga * T0[r2] * T0[s2] + gb * (T0[r2] * T1[s2] + T1[r2] * T0[s2]) +
                     2.0 * gc * T1[r2] * T1[s2];

    // T = J W: only J00, J02, J11, J12 are non-zero
    const double gJ00 = gT0[0] * R[0] + gT0[1] * R[1] + gT0[2] * R[2];
    const double gJ02 = gT0[0] * R[6] + gT0[1] * R[7] + gT0[2] * R[8];
    const double gJ11 = gT1[0] * R[3] + gT1[1] * R[4] + gT1[2] * R[5];
    const double gJ12 = gT1[0] * R[6] + gT1[1] * R[7] + gT1[2] * R[8];
    const double tx = P.t[0], ty = P.t[1], tz = P.t[2];
    const double iz = 1.0 / tz, iz2 = iz * iz;
    double gtx = 0.0, gty = 0.0, gtz = 0.0;
    gtz += -fx * iz2 * gJ00 + fx * P.rx * iz2 * gJ02 - fy * iz2 * gJ11 + fy * P.ry * iz2 * gJ12;
    const double grx = -fx * iz * gJ02, gry = -fy * iz * gJ12;
    if (!P.clampx) { gtx += grx * iz; gtz -= grx * tx * iz2; }
    if (!P.clampy) { gty += gry * iz; gtz -= gry * ty * iz2; }
    // mean2D
    gtx += gu * fx * iz;
    gtz -= gu * fx * tx * iz2;
    gty += gv * fy * iz;
    gtz -= gv * fy * ty * iz2;
    // t = W mu + t_w
#pragma unroll
    for (int k = 0; k < 3; ++k) gmu[k] += R[k] * gtx + R[3 + k] * gty + R[6 + k] * gtz;

    // Sigma = M M^T, M = Rq diag(s): dL/dM = Gs M
    const double* Rq = P.Rq;
    double gR[9];
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      double acc = 0.0;
#pragma unroll
      for (int r2 = 0; r2 < 3; ++r2) {
        const double gM =
            (Gs[r2][0] * Rq[k] + Gs[r2][1] * Rq[3 + k] + Gs[r2][2] * Rq[6 + k]) * P.s[k];
        acc += gM * Rq[3 * r2 + k];
        gR[3 * r2 + k] = gM * P.s[k];
      }
      gs[k] += acc;
    }
    quat_vjp(P.qn, P.qinv, gR, gq);
  }

  store_param_grads<NB>(grad_dest(sidx, G0, G1, G2, G3, G4, G5, G6, G7), S, i, gmu, gs, gq, go,
                        gsh, accumulate);
}

// 3DGUT projection (listing "Implementation of XPR-3DGUT", project), one
// thread per (view, Gaussian), in FP64 like the EWA path. The unscented
// transform of the 3D Gaussian (n = 3, alpha = 1, beta = 2, kappa = 0, so
// lambda = 0): sigma points mu and mu +- sqrt(3) s_j R e_j, mean weights 0
// (centre) and 1/6, covariance weights 2 (centre) and 1/6, each point taken
// through the pinhole projection f X / Z + c; a Gaussian with a sigma point
// at camera depth <= z_near is not visible. The 2D covariance gets the
// low-pass, the opacity the Mip-Splatting factor sqrt(det_orig / det), and
// the bounding box is placed at mean2D - 1/2 (pixel (i, j) is the ray
// through (i + 1/2, j + 1/2)). Record layout (24 floats):
//   (u, v, A, B) (C, o', r, g) (b, ro) (M00 M01 M02 M10) (M11 M12 M20 M21)
//   (M22, bx, by, 0)
// with (u, v) = mean2D - 1/2, (A, B, C) the scaled conic as for 3DGS, ro the
// camera position in the Gaussian's canonical frame, M = S^-1 R^T, and
// bx, by (bit patterns) the pixel box of gut_pixel_box for the compositing
// kernels' per-wave lists.
//
// The pixel box: a ray can only come within d^2 <= 9 of the centre if it
// meets the ellipsoid (x - mu)^T Sigma^-1 (x - mu) <= 9, whose image is
// bounded by the tangent planes through the camera centre. In camera
// coordinates the ellipsoid is {x : (x - c)^T E^-1 (x - c) <= 1} with
// E = 9 N N^T and c = -N ro for N = R_cam M^-1, and the plane X = a Z
// touches it iff K00 - 2 a K02 + a^2 K22 = 0 for K = E - c c^T
// = N (9 I - ro ro^T) N^T (likewise Y = b Z with K11, K12, K22), so the
// image lies in x in fx [a1, a2] + cx (and y alike) when K22 < 0 (the
// ellipsoid in front of the camera plane). Taken in float64 from the
// record's float32 M and ro (the values the compositing reads), widened by
// 1% + 0.05 px and rounded outward to the pixel columns X0 .. X1 and rows
// Y0 .. Y1 whose centres it may hold, as int16 pairs bx = X0 | X1 << 16,
// by = Y0 | Y1 << 16 (the whole int16 range when the bound does not exist:
// K22 >= 0, det M = 0 or a NaN). Computed once per record instead of per
// (tile, record) in the compositing kernels.
__device__ __forceinline__ void gut_pixel_box(const double* m, const double* ro,
                                              const ViewDev& V, uint32_t& bx, uint32_t& by) {
  constexpr uint32_t kAll = 0x7fff8000u;  // -32768 | 32767 << 16
  bx = by = kAll;
  // M^-1 by the adjugate
  const double c00 = m[4] * m[8] - m[5] * m[7], c01 = m[5] * m[6] - m[3] * m[8],
               c02 = m[3] * m[7] - m[4] * m[6];
  const double det = m[0] * c00 + m[1] * c01 + m[2] * c02;
  if (!(fabs(det) > 0.0)) return;
  const double id = 1.0 / det;
  const double inv[9] = {c00 * id, (m[2] * m[7] - m[1] * m[8]) * id,
                         (m[1] * m[5] - m[2] * m[4]) * id, c01 * id,
                         (m[0] * m[8] - m[2] * m[6]) * id, (m[2] * m[3] - m[0] * m[5]) * id,
                         c02 * id, (m[1] * m[6] - m[0] * m[7]) * id,
                         (m[0] * m[4] - m[1] * m[3]) * id};
  double N[9];  // R_cam M^-1
#pragma unroll
  for (int r = 0; r < 3; ++r)
#pragma unroll
    for (int c = 0; c < 3; ++c)
      N[3 * r + c] = (double)V.R[3 * r] * inv[c] + (double)V.R[3 * r + 1] * inv[3 + c] +
                     (double)V.R[3 * r + 2] * inv[6 + c];
  // K = N (9 I - ro ro^T) N^T: entries 00, 02, 22, 11, 12
  double Nro[3];
#pragma unroll
  for (int r = 0; r < 3; ++r)
    Nro[r] = N[3 * r] * ro[0] + N[3 * r + 1] * ro[1] + N[3 * r + 2] * ro[2];
  auto kk = [&](int i, int j) {
    return 9.0 * (N[3 * i] * N[3 * j] + N[3 * i + 1] * N[3 * j + 1] + N[3 * i + 2] * N[3 * j + 2]) -
           Nro[i] * Nro[j];
  };
  const double k22 = kk(2, 2);
  if (!(k22 < 0.0)) return;
  const double k00 = kk(0, 0), k02 = kk(0, 2), k11 = kk(1, 1), k12 = kk(1, 2);
  const double dx = fmax(k02 * k02 - k00 * k22, 0.0), dy = fmax(k12 * k12 - k11 * k22, 0.0);
  // roots of K00 - 2 a K02 + a^2 K22 = 0: (K02 -/+ sqrt(dx)) / K22
  const double ax0 = (k02 + sqrt(dx)) / k22, ax1 = (k02 - sqrt(dx)) / k22;
  const double ay0 = (k12 + sqrt(dy)) / k22, ay1 = (k12 - sqrt(dy)) / k22;
  // image box of the ray points x + 1/2, widened
  const double ux0 = (double)V.fx * fmin(ax0, ax1) + (double)V.cx,
               ux1 = (double)V.fx * fmax(ax0, ax1) + (double)V.cx;
  const double uy0 = (double)V.fy * fmin(ay0, ay1) + (double)V.cy,
               uy1 = (double)V.fy * fmax(ay0, ay1) + (double)V.cy;
  const double wx = 0.01 * (ux1 - ux0) + 0.05, wy = 0.01 * (uy1 - uy0) + 0.05;
  // pixel i's centre is i + 1/2: columns floor(lo - 1/2) .. ceil(hi - 1/2)
  // hold every centre in [lo, hi]; clamped to int16 (views are at most
  // 16384 pixels wide), a NaN bound opens the box
  auto lo16 = [](double x) -> uint32_t {
    x = floor(x);
    const int v = !(x >= -32768.0) ? -32768 : (x > 32767.0 ? 32767 : (int)x);
    return (uint32_t)(uint16_t)(int16_t)v;
  };
  auto hi16 = [](double x) -> uint32_t {
    x = ceil(x);
    const int v = !(x <= 32767.0) ? 32767 : (x < -32768.0 ? -32768 : (int)x);
    return (uint32_t)(uint16_t)(int16_t)v;
  };
  bx = lo16(ux0 - wx - 0.5) | (hi16(ux1 + wx - 0.5) << 16);
  by = lo16(uy0 - wy - 0.5) | (hi16(uy1 + wy - 0.5) << 16);
}

template <int DEG>
__global__ __launch_bounds__(256) void k_project_gut(Batch B, float4* __restrict__ splat,
                                                     float* __restrict__ depth,
                                                     short4* __restrict__ rect,
                                                     int32_t* __restrict__ tc) {
  const ViewDev& V = B.v[blockIdx.y];
  const SceneDev& S = B.s[V.scene];
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i >= S.n) return;
  const double mu[3] = {S.means[i], S.means[S.ld + i], S.means[2 * S.ld + i]};
  double R[9];
#pragma unroll
  for (int k = 0; k < 9; ++k) R[k] = V.R[k];
  const double qw = S.quats[i], qx = S.quats[S.ld + i], qy = S.quats[2 * S.ld + i],
               qz = S.quats[3 * S.ld + i];
  const double qinv = 1.0 / sqrt(qw * qw + qx * qx + qy * qy + qz * qz);
  const double w = qw * qinv, x = qx * qinv, y = qy * qinv, z = qz * qinv;
  const double Q[9] = {1.0 - 2.0 * (y * y + z * z), 2.0 * (x * y - w * z), 2.0 * (x * z + w * y),
                       2.0 * (x * y + w * z), 1.0 - 2.0 * (x * x + z * z), 2.0 * (y * z - w * x),
                       2.0 * (x * z - w * y), 2.0 * (y * z + w * x), 1.0 - 2.0 * (x * x + y * y)};
  const double s[3] = {S.scales[i], S.scales[S.ld + i], S.scales[2 * S.ld + i]};
  const double fx = V.fx, fy = V.fy, cx = V.cx, cy = V.cy;
  const double k3 = 1.7320508075688772;  // sqrt(3)
  // sigma points in camera space: centre, then +-sqrt(3) s_j (R column j)
  bool front = true;
  double zc = 0.0, px[7], py[7];
#pragma unroll
  for (int p = 0; p < 7; ++p) {
    double X[3] = {mu[0], mu[1], mu[2]};
    if (p > 0) {
      const int j = (p - 1) >> 1;
      const double sg = ((p - 1) & 1) ? -k3 : k3;
#pragma unroll
      for (int c = 0; c < 3; ++c) X[c] += sg * s[j] * Q[3 * c + j];
    }
    const double cxp = R[0] * X[0] + R[1] * X[1] + R[2] * X[2] + (double)V.t[0];
    const double cyp = R[3] * X[0] + R[4] * X[1] + R[5] * X[2] + (double)V.t[1];
    const double czp = R[6] * X[0] + R[7] * X[1] + R[8] * X[2] + (double)V.t[2];
    if (p == 0) zc = czp;
    front = front && czp > (double)B.z_near;
    px[p] = fx * cxp / czp + cx;
    py[p] = fy * cyp / czp + cy;
  }
  double mx = 0.0, my = 0.0;
#pragma unroll
  for (int p = 1; p < 7; ++p) {
    mx += px[p] / 6.0;
    my += py[p] / 6.0;
  }
  double cxx = 0.0, cxy = 0.0, cyy = 0.0;
#pragma unroll
  for (int p = 0; p < 7; ++p) {
    const double wc = p == 0 ? 2.0 : 1.0 / 6.0;
    const double dx = px[p] - mx, dy = py[p] - my;
    cxx += wc * dx * dx;
    cxy += wc * dx * dy;
    cyy += wc * dy * dy;
  }
  const double det0 = cxx * cyy - cxy * cxy;
  const double a = cxx + (double)B.lowpass, b = cxy, c = cyy + (double)B.lowpass;
  const double det = a * c - b * b;
  const double dinv = det > 0.0 ? 1.0 / det : 0.0;
  const double o = det > 0.0 ? (double)S.opac[i] * sqrt(fmax(det0, 0.0) * dinv) : 0.0;
  const double u = mx - 0.5, v = my - 0.5;
  double ex, ey, rad;
  if (B.opacity_extents) {
    const double lvl = o > 0.0 ? 2.0 * log(o / (double)B.alpha_min) : -1.0;
    ex = lvl > 0.0 ? sqrt(lvl * a) : 0.0;
    ey = lvl > 0.0 ? sqrt(lvl * c) : 0.0;
    rad = fmax(ex, ey);
  } else {
    const double mid = 0.5 * (a + c);
    rad = ceil(3.0 * sqrt(mid + sqrt(fmax(0.0, mid * mid - det))));
    ex = ey = rad;
  }
  const double tw = B.tile_w, th = B.tile_h;
  const double txn = V.tiles_x, tyn = V.tiles_y;
  const int x0 = (int)fmin(txn, fmax(0.0, floor((u - ex) / tw)));
  const int y0 = (int)fmin(tyn, fmax(0.0, floor((v - ey) / th)));
  const int x1 = (int)fmin(txn, fmax(0.0, floor((u + ex) / tw) + 1.0));
  const int y1 = (int)fmin(tyn, fmax(0.0, floor((v + ey) / th) + 1.0));
  const int area = (x1 - x0) * (y1 - y0);
  const bool visible = front && det > 0.0 && o > (double)B.alpha_min && rad > 0.0 && area > 0;
  // shader data: M = S^-1 R^T (row r = column r of R over s_r), camera
  // position in the canonical frame
  double M[9];
#pragma unroll
  for (int r = 0; r < 3; ++r)
#pragma unroll
    for (int k = 0; k < 3; ++k) M[3 * r + k] = Q[3 * k + r] / s[r];
  const double cpx = -(R[0] * V.t[0] + R[3] * V.t[1] + R[6] * V.t[2]);
  const double cpy = -(R[1] * V.t[0] + R[4] * V.t[1] + R[7] * V.t[2]);
  const double cpz = -(R[2] * V.t[0] + R[5] * V.t[1] + R[8] * V.t[2]);
  const double d0 = cpx - mu[0], d1 = cpy - mu[1], d2 = cpz - mu[2];
  const double ro0 = M[0] * d0 + M[1] * d1 + M[2] * d2;
  const double ro1 = M[3] * d0 + M[4] * d1 + M[5] * d2;
  const double ro2 = M[6] * d0 + M[7] * d1 + M[8] * d2;
  // view-dependent colour, as for 3DGS
  const double dn = 1.0 / sqrt(d0 * d0 + d1 * d1 + d2 * d2);
  float Y[16];
  sh_basis<DEG>((float)(-d0 * dn), (float)(-d1 * dn), (float)(-d2 * dn), Y);
  constexpr int NB = (DEG + 1) * (DEG + 1);
  float col[3];
#pragma unroll
  for (int ch = 0; ch < 3; ++ch) {
    float acc = 0.5f;
#pragma unroll
    for (int j = 0; j < NB; ++j)  // read once: streaming loads, as in the EWA projection
      acc += __builtin_nontemporal_load(S.sh + (size_t)(3 * j + ch) * S.ld + i) * Y[j];
    col[ch] = fmaxf(0.f, acc);
  }
  const size_t r = (size_t)V.rec_off + i;
  float4* out = splat + 6 * r;
  float Mf[9];
#pragma unroll
  for (int k = 0; k < 9; ++k) Mf[k] = (float)M[k];
  const float rof[3] = {(float)ro0, (float)ro1, (float)ro2};
  uint32_t bx = 0u, by = 0u;
  if (visible) {
    const double md[9] = {Mf[0], Mf[1], Mf[2], Mf[3], Mf[4], Mf[5], Mf[6], Mf[7], Mf[8]};
    const double rod[3] = {rof[0], rof[1], rof[2]};
    gut_pixel_box(md, rod, V, bx, by);
  }
  out[0] = make_float4((float)u, (float)v, (float)(-0.5 * c * dinv), (float)(b * dinv));
  out[1] = make_float4((float)(-0.5 * a * dinv), (float)o, col[0], col[1]);
  out[2] = make_float4(col[2], rof[0], rof[1], rof[2]);
  out[3] = make_float4(Mf[0], Mf[1], Mf[2], Mf[3]);
  out[4] = make_float4(Mf[4], Mf[5], Mf[6], Mf[7]);
  out[5] = make_float4(Mf[8], __uint_as_float(bx), __uint_as_float(by), 0.f);
  depth[r] = (float)zc;
  rect[r] = visible ? make_short4((short)x0, (short)y0, (short)x1, (short)y1)
                    : make_short4(0, 0, 0, 0);
  tc[r] = visible ? area : 0;
}

// Backward of the 3DGUT projection, one thread per scene Gaussian over the
// views of its scene (blockIdx.y = scene), in FP64 like the forward: from
// dL/d(o', colour, ro, M) [record][16] to the gradients of the means,
// activated scales and opacity, raw quaternion and SH coefficients. The
// chain, for a visible record:
//   ro = M (campos - mu) at fixed M: dL/dmu -= M^T dL/dro;
//   M = S^-1 R^T with the centre fixed (the record gradient's dL/dM):
//     dL/dR_cr += dL/dM_rc / s_r and dL/ds_r -= sum_c dL/dM_rc R_cr / s_r^2;
//   o' = o comp, comp = sqrt(det_orig / det) of the unscented transform's
//     2D covariance before and after the low-pass: dL/do = comp dL/do', and
//     through det_orig and det to the covariance, its weighted deviations,
//     the seven projected sigma points and so to mu, s and R;
//   the colour as for 3DGS (clamped channels pass nothing).
template <int DEG>
__global__ __launch_bounds__(256, 2) void k_project_bwd_gut(Batch B,
                                                            const float* __restrict__ splat,
                                                            const float* __restrict__ grad,
                                                            const int32_t* __restrict__ tc,
                                                         GradDev G0, GradDev G1, GradDev G2,
                                                         GradDev G3, GradDev G4, GradDev G5,
                                                         GradDev G6, GradDev G7, int accumulate) {
  const int sidx = blockIdx.y;
  const SceneDev& S = B.s[sidx];
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i >= S.n) return;
  constexpr int NB = (DEG + 1) * (DEG + 1);
  const GradDev G = grad_dest(sidx, G0, G1, G2, G3, G4, G5, G6, G7);
  const size_t ld = S.ld;
  double gmu[3] = {0.0, 0.0, 0.0}, gs[3] = {0.0, 0.0, 0.0}, gq[4] = {0.0, 0.0, 0.0, 0.0};
  double gR[9] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
  float go = 0.f;
  // the SH gradient goes straight to memory, view by view (this thread owns
  // Gaussian i): the first view stores unless accumulating, later ones add
  bool sh_out = false;
  // the Gaussian's frame, as the forward forms it
  const double mu[3] = {S.means[i], S.means[ld + i], S.means[2 * ld + i]};
  const double q0 = S.quats[i], q1 = S.quats[ld + i], q2 = S.quats[2 * ld + i],
               q3 = S.quats[3 * ld + i];
  const double qinv = 1.0 / sqrt(q0 * q0 + q1 * q1 + q2 * q2 + q3 * q3);
  const double qn[4] = {q0 * qinv, q1 * qinv, q2 * qinv, q3 * qinv};
  const double w = qn[0], x = qn[1], y = qn[2], z = qn[3];
  const double Q[9] = {1.0 - 2.0 * (y * y + z * z), 2.0 * (x * y - w * z), 2.0 * (x * z + w * y),
                       2.0 * (x * y + w * z), 1.0 - 2.0 * (x * x + z * z), 2.0 * (y * z - w * x),
                       2.0 * (x * z - w * y), 2.0 * (y * z + w * x), 1.0 - 2.0 * (x * x + y * y)};
  const double s[3] = {S.scales[i], S.scales[ld + i], S.scales[2 * ld + i]};
  const double is[3] = {1.0 / s[0], 1.0 / s[1], 1.0 / s[2]};
  const double opac = S.opac[i];
  const double k3 = 1.7320508075688772;  // sqrt(3)
  const double lp = B.lowpass;

  for (int vi = 0; vi < B.n_views; ++vi) {
    const ViewDev& V = B.v[vi];
    if (V.scene != sidx) continue;
    const int r = V.rec_off + i;
    // a record the view does not see adds nothing, but the first view still
    // stores its zero SH gradient, in the same store instruction as the
    // visible lanes (two partial stores to one line would write it twice)
    const bool vis = tc[r] != 0;
    if (!vis && (sh_out || accumulate)) continue;
    const float* g = grad + 16 * (size_t)r;
    double R[9];
#pragma unroll
    for (int k = 0; k < 9; ++k) R[k] = V.R[k];
    const double fx = V.fx, fy = V.fy;
    const double cp[3] = {-(R[0] * V.t[0] + R[3] * V.t[1] + R[6] * V.t[2]),
                          -(R[1] * V.t[0] + R[4] * V.t[1] + R[7] * V.t[2]),
                          -(R[2] * V.t[0] + R[5] * V.t[1] + R[8] * V.t[2])};

    // colour = max(0, 0.5 + sum_j sh_j Y_j(dir)), dir = (mu - campos) / |.|;
    // a channel passes its gradient where the record's colour is positive
    // (the forward stored max(0, raw): positive exactly when raw is)
    {
      const double d[3] = {cp[0] - mu[0], cp[1] - mu[1], cp[2] - mu[2]};
      const double dn = 1.0 / sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
      const double dir[3] = {-d[0] * dn, -d[1] * dn, -d[2] * dn};
      const float dxf = (float)dir[0], dyf = (float)dir[1], dzf = (float)dir[2];
      float Y[16];
      sh_basis<DEG>(dxf, dyf, dzf, Y);
      const float* col = splat + 24 * (size_t)r + 6;  // (r, g, b) of the 24-float record
      float wsum[16];
      sh_backward<DEG>(S, G, i, Y, vis && col[0] > 0.f ? g[1] : 0.f,
                       vis && col[1] > 0.f ? g[2] : 0.f, vis && col[2] > 0.f ? g[3] : 0.f,
                       sh_out || accumulate, wsum);
      sh_out = true;
      if (!vis) continue;
      float gdxf, gdyf, gdzf;
      sh_basis_vjp<DEG>(dxf, dyf, dzf, wsum, gdxf, gdyf, gdzf);
      const double gd[3] = {gdxf, gdyf, gdzf};
      const double dd = dir[0] * gd[0] + dir[1] * gd[1] + dir[2] * gd[2];
#pragma unroll
      for (int c = 0; c < 3; ++c) gmu[c] += (gd[c] - dir[c] * dd) * dn;
    }

    // ro = M (campos - mu) at fixed M, M_ac = Q_ca / s_a with the centre fixed
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      const double gro = g[4 + a];
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        const double Mac = Q[3 * c + a] * is[a];
        const double gM = g[7 + 3 * a + c];
        gmu[c] -= Mac * gro;
        gR[3 * c + a] += gM * is[a];
        gs[a] -= gM * Mac * is[a];
      }
    }

    // o' = o comp over the seven sigma points. Each pass below recomputes
    // the points (mu and mu +- sqrt(3) s_j Q e_j) and their normalised camera
    // coordinates (x / z, y / z) instead of keeping them: four cheap passes
    // (mean, covariance, the covariance gradient's point sums, the chain
    // back to mu, s and R) in few registers.
    auto point = [&](int j, double sg, double& u, double& v, double& iz) {
      double X[3] = {mu[0], mu[1], mu[2]};
      if (j >= 0) {
#pragma unroll
        for (int c = 0; c < 3; ++c) X[c] += sg * s[j] * Q[3 * c + j];
      }
      iz = 1.0 / (R[6] * X[0] + R[7] * X[1] + R[8] * X[2] + (double)V.t[2]);
      u = (R[0] * X[0] + R[1] * X[1] + R[2] * X[2] + (double)V.t[0]) * iz;
      v = (R[3] * X[0] + R[4] * X[1] + R[5] * X[2] + (double)V.t[1]) * iz;
    };
    constexpr double k6 = 1.0 / 6.0;
    double mu_u = 0.0, mu_v = 0.0;
#pragma unroll 1
    for (int p = 1; p < 7; ++p) {
      double u, v, iz;
      point((p - 1) >> 1, ((p - 1) & 1) ? -k3 : k3, u, v, iz);
      mu_u += u;
      mu_v += v;
    }
    mu_u *= k6;
    mu_v *= k6;
    // 2D covariance of the deviations (pixels) from the mean
    double cxx = 0.0, cxy = 0.0, cyy = 0.0;
#pragma unroll 1
    for (int p = 0; p < 7; ++p) {
      double u, v, iz;
      point((p - 1) >> 1, ((p - 1) & 1) ? -k3 : k3, u, v, iz);
      const double wc = p == 0 ? 2.0 : k6;
      const double dx = fx * (u - mu_u), dy = fy * (v - mu_v);
      cxx += wc * dx * dx;
      cxy += wc * dx * dy;
      cyy += wc * dy * dy;
    }
    const double det0 = cxx * cyy - cxy * cxy;
    const double det = (cxx + lp) * (cyy + lp) - cxy * cxy;
    const double comp = det > 0.0 ? sqrt(fmax(det0, 0.0) / det) : 0.0;
    go += (float)(comp * (double)g[0]);
    if (det0 > 0.0 && det > 0.0) {
      const double gcomp = opac * (double)g[0];
      const double gdet0 = gcomp * comp / (2.0 * det0), gdet = -gcomp * comp / (2.0 * det);
      const double gxx = gdet0 * cyy + gdet * (cyy + lp);
      const double gyy = gdet0 * cxx + gdet * (cxx + lp);
      const double gxy = -2.0 * cxy * (gdet0 + gdet);
      // dL/d(deviation) of point p is wc (2 dx gxx + dy gxy, 2 dy gyy + dx gxy);
      // the mean's share goes back through the mean weights (0 for the
      // centre, 1/6 for the others), so every point needs their sum sD
      double sDx = 0.0, sDy = 0.0;
#pragma unroll 1
      for (int p = 0; p < 7; ++p) {
        double u, v, iz;
        point((p - 1) >> 1, ((p - 1) & 1) ? -k3 : k3, u, v, iz);
        const double wc = p == 0 ? 2.0 : k6;
        const double dx = fx * (u - mu_u), dy = fy * (v - mu_v);
        sDx += wc * (2.0 * dx * gxx + dy * gxy);
        sDy += wc * (2.0 * dy * gyy + dx * gxy);
      }
      sDx *= k6;
      sDy *= k6;
      // through px = fx x / z + cx, py = fy y / z + cy to the point, then
      // to mu (every point) and to s_j, Q e_j (the axis points)
      auto back = [&](int p, double* gX) {
        double u, v, iz;
        point((p - 1) >> 1, ((p - 1) & 1) ? -k3 : k3, u, v, iz);
        const double wc = p == 0 ? 2.0 : k6;
        const double dx = fx * (u - mu_u), dy = fy * (v - mu_v);
        double gPx = wc * (2.0 * dx * gxx + dy * gxy), gPy = wc * (2.0 * dy * gyy + dx * gxy);
        if (p > 0) {
          gPx -= sDx;
          gPy -= sDy;
        }
        const double g0 = fx * iz * gPx, g1 = fy * iz * gPy,
                     g2 = -(fx * u * gPx + fy * v * gPy) * iz;
#pragma unroll
        for (int c = 0; c < 3; ++c) {
          gX[c] = R[c] * g0 + R[3 + c] * g1 + R[6 + c] * g2;
          gmu[c] += gX[c];
        }
      };
      double gX[3];
      back(0, gX);
#pragma unroll
      for (int j = 0; j < 3; ++j) {
#pragma unroll 1
        for (int h = 0; h < 2; ++h) {
          const double sg = h ? -k3 : k3;
          back(1 + 2 * j + h, gX);
#pragma unroll
          for (int c = 0; c < 3; ++c) {
            gs[j] += sg * gX[c] * Q[3 * c + j];
            gR[3 * c + j] += sg * s[j] * gX[c];
          }
        }
      }
    }
  }
  quat_vjp(qn, qinv, gR, gq);
  store_geom_grads(G, S, i, gmu, gs, gq, go, accumulate, sh_out, NB);
}

// LinPrim projection (listing "Implementation of XPR-LinPrim", project),
// one thread per (view, Gaussian slot holding an octahedron: scales are its
// half-extents), in FP64. A = J3 R_w2c R diag(s) maps the octahedron's
// local frame to (x_px, y_px, tau) with tau the Euclidean depth from the
// centre; J3 stacks the perspective Jacobian rows on the unit viewing
// direction. The footprint lies in mu_2D +- (ex, ey) with ex = max_k |A_0k|,
// ey = max_k |A_1k| (the projected vertices), the sort depth is |mu_c|,
// sigma = -log(1 - 0.99 o) / (2 s_min) with o clipped to [0, 0.999], and
// the rows c_k of A^-1 are the slab data. Visible: centre in front
// (z > z_near), A invertible, s_min > 0, footprint on the tile grid.
// Record layout (20 floats):
//   (u, v, sigma, r) (g, b, ex, ey) (c00 c01 c02 c10) (c11 c12 c20 c21)
//   (c22, 0, 0, 0)    with (u, v) = mu_2D - 1/2
template <int DEG>
__global__ __launch_bounds__(256) void k_project_lin(Batch B, float4* __restrict__ splat,
                                                     float* __restrict__ depth,
                                                     short4* __restrict__ rect,
                                                     int32_t* __restrict__ tc) {
  const ViewDev& V = B.v[blockIdx.y];
  const SceneDev& S = B.s[V.scene];
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i >= S.n) return;
  const double mu[3] = {S.means[i], S.means[S.ld + i], S.means[2 * S.ld + i]};
  double R[9];
#pragma unroll
  for (int k = 0; k < 9; ++k) R[k] = V.R[k];
  const double x = R[0] * mu[0] + R[1] * mu[1] + R[2] * mu[2] + (double)V.t[0];
  const double y = R[3] * mu[0] + R[4] * mu[1] + R[5] * mu[2] + (double)V.t[1];
  const double z = R[6] * mu[0] + R[7] * mu[1] + R[8] * mu[2] + (double)V.t[2];
  const double d = sqrt(x * x + y * y + z * z);
  const double qw = S.quats[i], qx = S.quats[S.ld + i], qy = S.quats[2 * S.ld + i],
               qz = S.quats[3 * S.ld + i];
  const double qinv = 1.0 / sqrt(qw * qw + qx * qx + qy * qy + qz * qz);
  const double w = qw * qinv, a = qx * qinv, b = qy * qinv, c = qz * qinv;
  const double Q[9] = {1.0 - 2.0 * (b * b + c * c), 2.0 * (a * b - w * c), 2.0 * (a * c + w * b),
                       2.0 * (a * b + w * c), 1.0 - 2.0 * (a * a + c * c), 2.0 * (b * c - w * a),
                       2.0 * (a * c - w * b), 2.0 * (b * c + w * a), 1.0 - 2.0 * (a * a + b * b)};
  const double s[3] = {S.scales[i], S.scales[S.ld + i], S.scales[2 * S.ld + i]};
  const double smin = fmin(s[0], fmin(s[1], s[2]));
  const double fx = V.fx, fy = V.fy;
  const double J[9] = {fx / z, 0.0, -fx * x / (z * z), 0.0, fy / z, -fy * y / (z * z),
                       x / d, y / d, z / d};
  double A[9];
#pragma unroll
  for (int r = 0; r < 3; ++r)
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      // (J R_w2c Rq)[r][k] s[k]
      double acc = 0.0;
#pragma unroll
      for (int m = 0; m < 3; ++m)
        acc += J[3 * r + m] * (R[3 * m] * Q[k] + R[3 * m + 1] * Q[3 + k] + R[3 * m + 2] * Q[6 + k]);
      A[3 * r + k] = acc * s[k];
    }
  const double c00 = A[4] * A[8] - A[5] * A[7], c01 = A[5] * A[6] - A[3] * A[8],
               c02 = A[3] * A[7] - A[4] * A[6];
  const double det = A[0] * c00 + A[1] * c01 + A[2] * c02;
  const bool inv_ok = z > (double)B.z_near && smin > 0.0 && fabs(det) > 0.0 && isfinite(det);
  const double id = inv_ok ? 1.0 / det : 0.0;
  const double C[9] = {c00 * id, (A[2] * A[7] - A[1] * A[8]) * id, (A[1] * A[5] - A[2] * A[4]) * id,
                       c01 * id, (A[0] * A[8] - A[2] * A[6]) * id, (A[2] * A[3] - A[0] * A[5]) * id,
                       c02 * id, (A[1] * A[6] - A[0] * A[7]) * id, (A[0] * A[4] - A[1] * A[3]) * id};
  const double ex = fmax(fabs(A[0]), fmax(fabs(A[1]), fabs(A[2])));
  const double ey = fmax(fabs(A[3]), fmax(fabs(A[4]), fabs(A[5])));
  const double o = fmin(0.999, fmax(0.0, (double)S.opac[i]));
  const double sigma = smin > 0.0 ? -log1p(-0.99 * o) / (2.0 * smin) : 0.0;
  const double u = fx * x / z + (double)V.cx - 0.5, v = fy * y / z + (double)V.cy - 0.5;
  const double tw = B.tile_w, th = B.tile_h;
  const double txn = V.tiles_x, tyn = V.tiles_y;
  const int x0 = (int)fmin(txn, fmax(0.0, floor((u - ex) / tw)));
  const int y0 = (int)fmin(tyn, fmax(0.0, floor((v - ey) / th)));
  const int x1 = (int)fmin(txn, fmax(0.0, floor((u + ex) / tw) + 1.0));
  const int y1 = (int)fmin(tyn, fmax(0.0, floor((v + ey) / th) + 1.0));
  const int area = (x1 - x0) * (y1 - y0);
  const bool visible = inv_ok && fmax(ex, ey) > 0.0 && area > 0 && d > (double)B.z_near;
  // view-dependent colour, as for 3DGS
  const double cpx = -(R[0] * V.t[0] + R[3] * V.t[1] + R[6] * V.t[2]);
  const double cpy = -(R[1] * V.t[0] + R[4] * V.t[1] + R[7] * V.t[2]);
  const double cpz = -(R[2] * V.t[0] + R[5] * V.t[1] + R[8] * V.t[2]);
  const double dx = mu[0] - cpx, dy = mu[1] - cpy, dz = mu[2] - cpz;
  const double dn = 1.0 / sqrt(dx * dx + dy * dy + dz * dz);
  float Y[16];
  sh_basis<DEG>((float)(dx * dn), (float)(dy * dn), (float)(dz * dn), Y);
  constexpr int NB = (DEG + 1) * (DEG + 1);
  float col[3];
#pragma unroll
  for (int ch = 0; ch < 3; ++ch) {
    float acc = 0.5f;
#pragma unroll
    for (int j = 0; j < NB; ++j)  // read once: streaming loads, as in the EWA projection
      acc += __builtin_nontemporal_load(S.sh + (size_t)(3 * j + ch) * S.ld + i) * Y[j];
    col[ch] = fmaxf(0.f, acc);
  }
  const size_t r = (size_t)V.rec_off + i;
  float4* out = splat + 5 * r;
  out[0] = make_float4((float)u, (float)v, (float)sigma, col[0]);
  out[1] = make_float4(col[1], col[2], (float)ex, (float)ey);
  out[2] = make_float4((float)C[0], (float)C[1], (float)C[2], (float)C[3]);
  out[3] = make_float4((float)C[4], (float)C[5], (float)C[6], (float)C[7]);
  out[4] = make_float4((float)C[8], 0.f, 0.f, 0.f);
  depth[r] = (float)d;
  rect[r] = visible ? make_short4((short)x0, (short)y0, (short)x1, (short)y1)
                    : make_short4(0, 0, 0, 0);
  tc[r] = visible ? area : 0;
}

// Backward of the LinPrim projection, one thread per scene Gaussian over the
// views of its scene (blockIdx.y = scene), in FP64 like the forward: from
// dL/d(u, v, sigma, colour, c0, c1, c2) [record][16] to the gradients of the
// means, half-extent scales, opacity, raw quaternion and SH coefficients.
// For a visible record:
//   mean2D = (fx x / z + cx, fy y / z + cy) of the camera-space centre;
//   sigma = -log(1 - 0.99 o) / (2 s_min), o the opacity clipped to
//     [0, 0.999] (no gradient where the clip holds; the s_min term goes to
//     the first smallest scale);
//   C = A^-1 with A = J3 R_w2c Rq diag(s): dL/dA = -C^T dL/dC C^T, then
//     dL/ds_k = sum_r dL/dA_rk (J3 W)_rk, dL/dJ3 and dL/dW from
//     dL/d(J3 W) = dL/dA diag(s), J3's perspective rows and unit viewing
//     direction to (x, y, z), dL/dRq = R_w2c^T dL/dW;
//   the colour as for 3DGS (clamped channels, read from the record, pass
//     nothing).
template <int DEG>
__global__ __launch_bounds__(256) void k_project_bwd_lin(Batch B, const float* __restrict__ splat,
                                                         const float* __restrict__ grad,
                                                         const int32_t* __restrict__ tc,
                                                         GradDev G0, GradDev G1, GradDev G2,
                                                         GradDev G3, GradDev G4, GradDev G5,
                                                         GradDev G6, GradDev G7, int accumulate) {
  const int sidx = blockIdx.y;
  const SceneDev& S = B.s[sidx];
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i >= S.n) return;
  constexpr int NB = (DEG + 1) * (DEG + 1);
  const GradDev G = grad_dest(sidx, G0, G1, G2, G3, G4, G5, G6, G7);
  const size_t ld = S.ld;
  double gmu[3] = {0.0, 0.0, 0.0}, gs[3] = {0.0, 0.0, 0.0}, gq[4] = {0.0, 0.0, 0.0, 0.0};
  double gR[9] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
  float go = 0.f;
  bool sh_out = false;
  const double mu[3] = {S.means[i], S.means[ld + i], S.means[2 * ld + i]};
  const double q0 = S.quats[i], q1 = S.quats[ld + i], q2 = S.quats[2 * ld + i],
               q3 = S.quats[3 * ld + i];
  const double qinv = 1.0 / sqrt(q0 * q0 + q1 * q1 + q2 * q2 + q3 * q3);
  const double qn[4] = {q0 * qinv, q1 * qinv, q2 * qinv, q3 * qinv};
  const double w = qn[0], a = qn[1], b = qn[2], c = qn[3];
  const double Q[9] = {1.0 - 2.0 * (b * b + c * c), 2.0 * (a * b - w * c), 2.0 * (a * c + w * b),
                       2.0 * (a * b + w * c), 1.0 - 2.0 * (a * a + c * c), 2.0 * (b * c - w * a),
                       2.0 * (a * c - w * b), 2.0 * (b * c + w * a), 1.0 - 2.0 * (a * a + b * b)};
  const double s[3] = {S.scales[i], S.scales[ld + i], S.scales[2 * ld + i]};
  int jmin = 0;
  if (s[1] < s[jmin]) jmin = 1;
  if (s[2] < s[jmin]) jmin = 2;
  const double smin = s[jmin];
  const double op = S.opac[i];
  const double o = fmin(0.999, fmax(0.0, op));
  const double sigma = -log1p(-0.99 * o) / (2.0 * smin);
  const double dsig_do = (op > 0.0 && op < 0.999) ? 0.99 / ((1.0 - 0.99 * o) * 2.0 * smin) : 0.0;

  for (int vi = 0; vi < B.n_views; ++vi) {
    const ViewDev& V = B.v[vi];
    if (V.scene != sidx) continue;
    const int r = V.rec_off + i;
    // a record the view does not see adds nothing, but the first view still
    // stores its zero SH gradient, in the same store instruction as the
    // visible lanes (two partial stores to one line would write it twice)
    const bool vis = tc[r] != 0;
    if (!vis && (sh_out || accumulate)) continue;
    const float* g = grad + 16 * (size_t)r;
    double R[9];
#pragma unroll
    for (int k = 0; k < 9; ++k) R[k] = V.R[k];

    // colour = max(0, 0.5 + sum_j sh_j Y_j(dir)), dir = (mu - campos) / |.|
    {
      const double cp[3] = {-(R[0] * V.t[0] + R[3] * V.t[1] + R[6] * V.t[2]),
                            -(R[1] * V.t[0] + R[4] * V.t[1] + R[7] * V.t[2]),
                            -(R[2] * V.t[0] + R[5] * V.t[1] + R[8] * V.t[2])};
      const double dv[3] = {mu[0] - cp[0], mu[1] - cp[1], mu[2] - cp[2]};
      const double dn = 1.0 / sqrt(dv[0] * dv[0] + dv[1] * dv[1] + dv[2] * dv[2]);
      const double dir[3] = {dv[0] * dn, dv[1] * dn, dv[2] * dn};
      const float dxf = (float)dir[0], dyf = (float)dir[1], dzf = (float)dir[2];
      float Y[16];
      sh_basis<DEG>(dxf, dyf, dzf, Y);
      const float* col = splat + 20 * (size_t)r + 3;  // (r, g, b) of the 20-float record
      float wsum[16];
      sh_backward<DEG>(S, G, i, Y, vis && col[0] > 0.f ? g[3] : 0.f,
                       vis && col[1] > 0.f ? g[4] : 0.f, vis && col[2] > 0.f ? g[5] : 0.f,
                       sh_out || accumulate, wsum);
      sh_out = true;
      if (!vis) continue;
      float gdxf, gdyf, gdzf;
      sh_basis_vjp<DEG>(dxf, dyf, dzf, wsum, gdxf, gdyf, gdzf);
      const double gd[3] = {gdxf, gdyf, gdzf};
      const double dd = dir[0] * gd[0] + dir[1] * gd[1] + dir[2] * gd[2];
#pragma unroll
      for (int k = 0; k < 3; ++k) gmu[k] += (gd[k] - dir[k] * dd) * dn;
    }

    const double fx = V.fx, fy = V.fy;
    const double x = R[0] * mu[0] + R[1] * mu[1] + R[2] * mu[2] + (double)V.t[0];
    const double y = R[3] * mu[0] + R[4] * mu[1] + R[5] * mu[2] + (double)V.t[1];
    const double z = R[6] * mu[0] + R[7] * mu[1] + R[8] * mu[2] + (double)V.t[2];
    const double d = sqrt(x * x + y * y + z * z);
    const double iz = 1.0 / z, iz2 = iz * iz;
    double gx = 0.0, gy = 0.0, gz = 0.0;  // dL/d(x, y, z)

    // mean2D
    const double gu = g[0], gv = g[1];
    gx += gu * fx * iz;
    gy += gv * fy * iz;
    gz -= (gu * fx * x + gv * fy * y) * iz2;

    // sigma
    go += (float)(g[2] * dsig_do);
    gs[jmin] -= g[2] * sigma / smin;

    // A = J3 Wm diag(s), Wm = R_w2c Rq, C = A^-1 (as the forward forms them)
    const double J[9] = {fx * iz, 0.0, -fx * x * iz2, 0.0, fy * iz, -fy * y * iz2,
                         x / d, y / d, z / d};
    double Wm[9], JW[9], A[9];
#pragma unroll
    for (int rr = 0; rr < 3; ++rr)
#pragma unroll
      for (int k = 0; k < 3; ++k)
        Wm[3 * rr + k] = R[3 * rr] * Q[k] + R[3 * rr + 1] * Q[3 + k] + R[3 * rr + 2] * Q[6 + k];
#pragma unroll
    for (int rr = 0; rr < 3; ++rr)
#pragma unroll
      for (int k = 0; k < 3; ++k) {
        JW[3 * rr + k] = J[3 * rr] * Wm[k] + J[3 * rr + 1] * Wm[3 + k] + J[3 * rr + 2] * Wm[6 + k];
        A[3 * rr + k] = JW[3 * rr + k] * s[k];
      }
    const double c00 = A[4] * A[8] - A[5] * A[7], c01 = A[5] * A[6] - A[3] * A[8],
                 c02 = A[3] * A[7] - A[4] * A[6];
    const double id = 1.0 / (A[0] * c00 + A[1] * c01 + A[2] * c02);
    const double C[9] = {c00 * id, (A[2] * A[7] - A[1] * A[8]) * id,
                         (A[1] * A[5] - A[2] * A[4]) * id, c01 * id,
                         (A[0] * A[8] - A[2] * A[6]) * id, (A[2] * A[3] - A[0] * A[5]) * id,
                         c02 * id, (A[1] * A[6] - A[0] * A[7]) * id,
                         (A[0] * A[4] - A[1] * A[3]) * id};
    // dL/dA = -C^T dL/dC C^T
    double T1[9];
#pragma unroll
    for (int rr = 0; rr < 3; ++rr)
#pragma unroll
      for (int k = 0; k < 3; ++k)
        T1[3 * rr + k] = (double)g[6 + 3 * rr] * C[3 * k] + (double)g[7 + 3 * rr] * C[3 * k + 1] +
                         (double)g[8 + 3 * rr] * C[3 * k + 2];
    double GJW[9];
#pragma unroll
    for (int rr = 0; rr < 3; ++rr)
#pragma unroll
      for (int k = 0; k < 3; ++k) {
        const double ga = -(C[rr] * T1[k] + C[3 + rr] * T1[3 + k] + C[6 + rr] * T1[6 + k]);
        gs[k] += ga * JW[3 * rr + k];
        GJW[3 * rr + k] = ga * s[k];
      }
    // dL/dJ = GJW Wm^T, dL/dWm = J^T GJW, dL/dRq = R_w2c^T dL/dWm
    double GJ[9], GW[9];
#pragma unroll
    for (int rr = 0; rr < 3; ++rr)
#pragma unroll
      for (int k = 0; k < 3; ++k) {
        GJ[3 * rr + k] = GJW[3 * rr] * Wm[3 * k] + GJW[3 * rr + 1] * Wm[3 * k + 1] +
                         GJW[3 * rr + 2] * Wm[3 * k + 2];
        GW[3 * rr + k] = J[rr] * GJW[k] + J[3 + rr] * GJW[3 + k] + J[6 + rr] * GJW[6 + k];
      }
#pragma unroll
    for (int rr = 0; rr < 3; ++rr)
#pragma unroll
      for (int k = 0; k < 3; ++k)
        gR[3 * rr + k] += R[rr] * GW[k] + R[3 + rr] * GW[3 + k] + R[6 + rr] * GW[6 + k];
    // J3 with respect to (x, y, z)
    const double iz3 = iz2 * iz;
    gz += -GJ[0] * fx * iz2 + GJ[2] * 2.0 * fx * x * iz3 - GJ[4] * fy * iz2 +
          GJ[5] * 2.0 * fy * y * iz3;
    gx -= GJ[2] * fx * iz2;
    gy -= GJ[5] * fy * iz2;
    const double id_ = 1.0 / d;
    const double e[3] = {x * id_, y * id_, z * id_};
    const double ge = GJ[6] * e[0] + GJ[7] * e[1] + GJ[8] * e[2];
    gx += (GJ[6] - e[0] * ge) * id_;
    gy += (GJ[7] - e[1] * ge) * id_;
    gz += (GJ[8] - e[2] * ge) * id_;
    // (x, y, z) = R_w2c mu + t
#pragma unroll
    for (int k = 0; k < 3; ++k) gmu[k] += R[k] * gx + R[3 + k] * gy + R[6 + k] * gz;
  }
  quat_vjp(qn, qinv, gR, gq);
  store_geom_grads(G, S, i, gmu, gs, gq, go, accumulate, sh_out, NB);
}

// Launchers ------------------------------------------------------------------

hipError_t launch_project(const Batch& B, int max_n, float* splat, float* depth, int16_t* rect,
                          int32_t* tc, hipStream_t st) {
  if (max_n <= 0) return hipSuccess;
  dim3 grid((max_n + 255) / 256, B.n_views);
  float4* sp = reinterpret_cast<float4*>(splat);
  short4* rc = reinterpret_cast<short4*>(rect);
  if (B.method == XPR_METHOD_LINPRIM) {
    switch (B.sh_degree) {
      case 0: hipLaunchKernelGGL(k_project_lin<0>, grid, dim3(256), 0, st, B, sp, depth, rc, tc); break;
      case 1: hipLaunchKernelGGL(k_project_lin<1>, grid, dim3(256), 0, st, B, sp, depth, rc, tc); break;
      case 2: hipLaunchKernelGGL(k_project_lin<2>, grid, dim3(256), 0, st, B, sp, depth, rc, tc); break;
      default: hipLaunchKernelGGL(k_project_lin<3>, grid, dim3(256), 0, st, B, sp, depth, rc, tc); break;
    }
    return hipGetLastError();
  }
  if (B.method == XPR_METHOD_3DGUT) {
    switch (B.sh_degree) {
      case 0: hipLaunchKernelGGL(k_project_gut<0>, grid, dim3(256), 0, st, B, sp, depth, rc, tc); break;
      case 1: hipLaunchKernelGGL(k_project_gut<1>, grid, dim3(256), 0, st, B, sp, depth, rc, tc); break;
      case 2: hipLaunchKernelGGL(k_project_gut<2>, grid, dim3(256), 0, st, B, sp, depth, rc, tc); break;
      default: hipLaunchKernelGGL(k_project_gut<3>, grid, dim3(256), 0, st, B, sp, depth, rc, tc); break;
    }
    return hipGetLastError();
  }
  switch (B.sh_degree) {
    case 0: hipLaunchKernelGGL(k_project<0>, grid, dim3(256), 0, st, B, sp, depth, rc, tc); break;
    case 1: hipLaunchKernelGGL(k_project<1>, grid, dim3(256), 0, st, B, sp, depth, rc, tc); break;
    case 2: hipLaunchKernelGGL(k_project<2>, grid, dim3(256), 0, st, B, sp, depth, rc, tc); break;
    default: hipLaunchKernelGGL(k_project<3>, grid, dim3(256), 0, st, B, sp, depth, rc, tc); break;
  }
  return hipGetLastError();
}

hipError_t launch_project_bwd(const Batch& B, int max_n, const float* splat, const float* grad2d,
                              const int32_t* tc, const GradDev* G, int accumulate, hipStream_t st) {
  if (max_n <= 0) return hipSuccess;
  dim3 grid((max_n + 255) / 256, B.n_scenes);
  if (B.method == XPR_METHOD_LINPRIM) {
#define XPR_PBL(D)                                                                         \
  hipLaunchKernelGGL(k_project_bwd_lin<D>, grid, dim3(256), 0, st, B, splat, grad2d, tc, G[0], \
                     G[1], G[2], G[3], G[4], G[5], G[6], G[7], accumulate)
    switch (B.sh_degree) {
      case 0: XPR_PBL(0); break;
      case 1: XPR_PBL(1); break;
      case 2: XPR_PBL(2); break;
      default: XPR_PBL(3); break;
    }
#undef XPR_PBL
    return hipGetLastError();
  }
  if (B.method == XPR_METHOD_3DGUT) {
#define XPR_PBG(D)                                                                         \
  hipLaunchKernelGGL(k_project_bwd_gut<D>, grid, dim3(256), 0, st, B, splat, grad2d, tc, G[0], \
                     G[1], G[2], G[3], G[4], G[5], G[6], G[7], accumulate)
    switch (B.sh_degree) {
      case 0: XPR_PBG(0); break;
      case 1: XPR_PBG(1); break;
      case 2: XPR_PBG(2); break;
      default: XPR_PBG(3); break;
    }
#undef XPR_PBG
    return hipGetLastError();
  }
#define XPR_PB(D)                                                                             \
  hipLaunchKernelGGL(k_project_bwd<D>, grid, dim3(256), 0, st, B, grad2d, tc, G[0], G[1],        \
                     G[2], G[3], G[4], G[5], G[6], G[7], accumulate)
  switch (B.sh_degree) {
    case 0: XPR_PB(0); break;
    case 1: XPR_PB(1); break;
    case 2: XPR_PB(2); break;
    default: XPR_PB(3); break;
  }
#undef XPR_PB
  return hipGetLastError();
}

}  // namespace xpr
