// Projection of 3D Gaussians (listing "Implementation of XPR-3DGS",
// function project) and its backward, one thread per (view, Gaussian).
//
// Inputs are structure-of-arrays, so each component load of a wave is one
// coalesced 256-byte read; the kernel is bound by HBM traffic (236 bytes in,
// 64 bytes out per Gaussian at SH degree 3), not by its ~400 flops.
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
// backward can reuse it after recomputation.
struct ProjState {
  float t[3];            // camera-space mean
  float qn[4], qinv;     // unit quaternion, 1/|q|
  float Rq[9];           // rotation of the Gaussian
  float s[3];            // scales
  float Sig[6];          // 3D covariance 00 01 02 11 12 22
  float rx, ry;          // (clamped) tx/tz, ty/tz
  bool clampx, clampy;
  float T0[3], T1[3];    // rows of J W
  float a, b, c, det;    // low-passed 2D covariance
  float con0, con1, con2;
  float u, v;
  int rect[4];
  int tc;
  float dir[3], dinv;    // unit view direction, 1/distance
};

template <int DEG>
__device__ __forceinline__ void project_core(const Batch& B, const ViewDev& V, const SceneDev& S,
                                             int i, ProjState& P, float* colour, float* raw) {
  const float mx = S.means[i], my = S.means[S.ld + i], mz = S.means[2 * S.ld + i];
  P.t[0] = V.R[0] * mx + V.R[1] * my + V.R[2] * mz + V.t[0];
  P.t[1] = V.R[3] * mx + V.R[4] * my + V.R[5] * mz + V.t[1];
  P.t[2] = V.R[6] * mx + V.R[7] * my + V.R[8] * mz + V.t[2];
  const float tx = P.t[0], ty = P.t[1], tz = P.t[2];

  // Sigma = Rq diag(s^2) Rq^T
  const float qw = S.quats[i], qx = S.quats[S.ld + i], qy = S.quats[2 * S.ld + i],
              qz = S.quats[3 * S.ld + i];
  const float qlen = sqrtf(qw * qw + qx * qx + qy * qy + qz * qz);
  P.qinv = 1.f / qlen;
  const float w = qw * P.qinv, x = qx * P.qinv, y = qy * P.qinv, z = qz * P.qinv;
  P.qn[0] = w; P.qn[1] = x; P.qn[2] = y; P.qn[3] = z;
  float* R = P.Rq;
  R[0] = 1.f - 2.f * (y * y + z * z); R[1] = 2.f * (x * y - w * z); R[2] = 2.f * (x * z + w * y);
  R[3] = 2.f * (x * y + w * z); R[4] = 1.f - 2.f * (x * x + z * z); R[5] = 2.f * (y * z - w * x);
  R[6] = 2.f * (x * z - w * y); R[7] = 2.f * (y * z + w * x); R[8] = 1.f - 2.f * (x * x + y * y);
  P.s[0] = S.scales[i]; P.s[1] = S.scales[S.ld + i]; P.s[2] = S.scales[2 * S.ld + i];
  float M[9];
#pragma unroll
  for (int r = 0; r < 3; ++r)
#pragma unroll
    for (int k = 0; k < 3; ++k) M[3 * r + k] = R[3 * r + k] * P.s[k];
  P.Sig[0] = M[0] * M[0] + M[1] * M[1] + M[2] * M[2];
  P.Sig[1] = M[0] * M[3] + M[1] * M[4] + M[2] * M[5];
  P.Sig[2] = M[0] * M[6] + M[1] * M[7] + M[2] * M[8];
  P.Sig[3] = M[3] * M[3] + M[4] * M[4] + M[5] * M[5];
  P.Sig[4] = M[3] * M[6] + M[4] * M[7] + M[5] * M[8];
  P.Sig[5] = M[6] * M[6] + M[7] * M[7] + M[8] * M[8];

  // EWA: T = J W with J the perspective Jacobian at the clamped direction.
  const float limx = B.fov_clip * (float)V.W / (2.f * V.fx);
  const float limy = B.fov_clip * (float)V.H / (2.f * V.fy);
  float rx = tx / tz, ry = ty / tz;
  P.clampx = P.clampy = false;
  if (B.fov_clip > 0.f) {
    P.clampx = rx < -limx || rx > limx;
    P.clampy = ry < -limy || ry > limy;
    rx = fminf(limx, fmaxf(-limx, rx));
    ry = fminf(limy, fmaxf(-limy, ry));
  }
  P.rx = rx; P.ry = ry;
  const float j00 = V.fx / tz, j02 = -V.fx * rx / tz;
  const float j11 = V.fy / tz, j12 = -V.fy * ry / tz;
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    P.T0[k] = j00 * V.R[k] + j02 * V.R[6 + k];
    P.T1[k] = j11 * V.R[3 + k] + j12 * V.R[6 + k];
  }
  const float* Sg = P.Sig;
  const float S0[3] = {Sg[0] * P.T0[0] + Sg[1] * P.T0[1] + Sg[2] * P.T0[2],
                       Sg[1] * P.T0[0] + Sg[3] * P.T0[1] + Sg[4] * P.T0[2],
                       Sg[2] * P.T0[0] + Sg[4] * P.T0[1] + Sg[5] * P.T0[2]};
  const float S1[3] = {Sg[0] * P.T1[0] + Sg[1] * P.T1[1] + Sg[2] * P.T1[2],
                       Sg[1] * P.T1[0] + Sg[3] * P.T1[1] + Sg[4] * P.T1[2],
                       Sg[2] * P.T1[0] + Sg[4] * P.T1[1] + Sg[5] * P.T1[2]};
  P.a = P.T0[0] * S0[0] + P.T0[1] * S0[1] + P.T0[2] * S0[2] + B.lowpass;
  P.b = P.T0[0] * S1[0] + P.T0[1] * S1[1] + P.T0[2] * S1[2];
  P.c = P.T1[0] * S1[0] + P.T1[1] * S1[1] + P.T1[2] * S1[2] + B.lowpass;
  P.det = P.a * P.c - P.b * P.b;
  const float dinv = P.det > 0.f ? 1.f / P.det : 0.f;
  P.con0 = P.c * dinv;
  P.con1 = -P.b * dinv;
  P.con2 = P.a * dinv;
  P.u = V.fx * tx / tz + V.cx - 0.5f;
  P.v = V.fy * ty / tz + V.cy - 0.5f;

  // 3-sigma radius of the largest eigenvalue, tile rect, tile count.
  const float mid = 0.5f * (P.a + P.c);
  const float lam = mid + sqrtf(fmaxf(0.f, mid * mid - P.det));
  const float rad = ceilf(3.f * sqrtf(lam));
  const float itw = 1.f / (float)B.tile_w, ith = 1.f / (float)B.tile_h;
  const float txn = (float)V.tiles_x, tyn = (float)V.tiles_y;
  P.rect[0] = (int)fminf(txn, fmaxf(0.f, floorf((P.u - rad) * itw)));
  P.rect[1] = (int)fminf(tyn, fmaxf(0.f, floorf((P.v - rad) * ith)));
  P.rect[2] = (int)fminf(txn, fmaxf(0.f, floorf((P.u + rad) * itw) + 1.f));
  P.rect[3] = (int)fminf(tyn, fmaxf(0.f, floorf((P.v + rad) * ith) + 1.f));
  const int area = (P.rect[2] - P.rect[0]) * (P.rect[3] - P.rect[1]);
  const float o = S.opac[i];
  const bool visible = tz > B.z_near && P.det > 0.f && o >= B.alpha_min && rad > 0.f && area > 0;
  P.tc = visible ? area : 0;

  // View-dependent colour.
  const float cpx = -(V.R[0] * V.t[0] + V.R[3] * V.t[1] + V.R[6] * V.t[2]);
  const float cpy = -(V.R[1] * V.t[0] + V.R[4] * V.t[1] + V.R[7] * V.t[2]);
  const float cpz = -(V.R[2] * V.t[0] + V.R[5] * V.t[1] + V.R[8] * V.t[2]);
  const float dx = mx - cpx, dy = my - cpy, dz = mz - cpz;
  P.dinv = 1.f / sqrtf(dx * dx + dy * dy + dz * dz);
  P.dir[0] = dx * P.dinv; P.dir[1] = dy * P.dinv; P.dir[2] = dz * P.dinv;
  float Y[16];
  sh_basis<DEG>(P.dir[0], P.dir[1], P.dir[2], Y);
  constexpr int NB = (DEG + 1) * (DEG + 1);
#pragma unroll
  for (int ch = 0; ch < 3; ++ch) {
    float acc = 0.5f;
#pragma unroll
    for (int j = 0; j < NB; ++j) acc += S.sh[(size_t)(3 * j + ch) * S.ld + i] * Y[j];
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
  project_core<DEG>(B, V, S, i, P, col, raw);
  const int r = V.rec_off + i;
  const float o = S.opac[i];
  splat[3 * (size_t)r + 0] = make_float4(P.u, P.v, -0.5f * P.con0, -P.con1);
  splat[3 * (size_t)r + 1] = make_float4(-0.5f * P.con2, o, col[0], col[1]);
  splat[3 * (size_t)r + 2] = make_float4(col[2], 0.f, 0.f, 0.f);
  depth[r] = P.t[2];
  rect[r] = P.tc > 0 ? make_short4((short)P.rect[0], (short)P.rect[1], (short)P.rect[2],
                                   (short)P.rect[3])
                     : make_short4(0, 0, 0, 0);
  tc[r] = P.tc;
}

// Backward of the projection for one Gaussian of scene blockIdx.y, summed
// over the views that render it. grad2d [records][9] holds dL/d(u, v, A, B,
// C, o, r, g, b). Chain: shader data -> conic -> 2D covariance -> (J W,
// Sigma) -> (camera-space mean, scales, rotation -> quaternion); mean2D ->
// camera-space mean -> world mean; colour -> SH coefficients and direction.
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
  float gmu[3] = {0.f, 0.f, 0.f}, gs[3] = {0.f, 0.f, 0.f}, gq[4] = {0.f, 0.f, 0.f, 0.f};
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
    const float gu = g[0], gv = g[1], gA = g[2], gB = g[3], gC = g[4];
    const float gcol[3] = {g[6], g[7], g[8]};
    go += g[5];
    ProjState P;
    float col[3], raw[3];
    project_core<DEG>(B, V, S, i, P, col, raw);

    // colour = max(0, 0.5 + sum_j sh_j Y_j(dir))
    float Y[16];
    sh_basis<DEG>(P.dir[0], P.dir[1], P.dir[2], Y);
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
    float gdx, gdy, gdz;
    sh_basis_vjp<DEG>(P.dir[0], P.dir[1], P.dir[2], wsum, gdx, gdy, gdz);
    const float dd = P.dir[0] * gdx + P.dir[1] * gdy + P.dir[2] * gdz;
    gmu[0] += (gdx - P.dir[0] * dd) * P.dinv;
    gmu[1] += (gdy - P.dir[1] * dd) * P.dinv;
    gmu[2] += (gdz - P.dir[2] * dd) * P.dinv;

    // conic entries: con0 = c/det, con1 = -b/det, con2 = a/det
    const float gk0 = -0.5f * gA, gk1 = -gB, gk2 = -0.5f * gC;
    const float a = P.a, b = P.b, c = P.c;
    const float id2 = 1.f / (P.det * P.det);
    const float ga = (-c * c * gk0 + b * c * gk1 - b * b * gk2) * id2;
    const float gb = (2.f * b * c * gk0 - (a * c + b * b) * gk1 + 2.f * a * b * gk2) * id2;
    const float gc = (-b * b * gk0 + a * b * gk1 - a * a * gk2) * id2;

    // a = T0 Sig T0, b = T0 Sig T1, c = T1 Sig T1 (Sig symmetric)
    const float* T0 = P.T0;
    const float* T1 = P.T1;
    const float* Sg = P.Sig;
    const float ST0[3] = {Sg[0] * T0[0] + Sg[1] * T0[1] + Sg[2] * T0[2],
                          Sg[1] * T0[0] + Sg[3] * T0[1] + Sg[4] * T0[2],
                          Sg[2] * T0[0] + Sg[4] * T0[1] + Sg[5] * T0[2]};
    const float ST1[3] = {Sg[0] * T1[0] + Sg[1] * T1[1] + Sg[2] * T1[2],
                          Sg[1] * T1[0] + Sg[3] * T1[1] + Sg[4] * T1[2],
                          Sg[2] * T1[0] + Sg[4] * T1[1] + Sg[5] * T1[2]};
    float gT0[3], gT1[3];
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      gT0[k] = 2.f * ga * ST0[k] + gb * ST1[k];
      gT1[k] = gb * ST0[k] + 2.f * gc * ST1[k];
    }
    // symmetric dL/dSigma (full matrix G + G^T): Gs[r][s] for r <= s
    float Gs[3][3];
#pragma unroll
    for (int r2 = 0; r2 < 3; ++r2)
#pragma unroll
      for (int s2 = 0; s2 < 3; ++s2)
        Gs[r2][s2] = 2.f * ga * T0[r2] * T0[s2] + gb * (T0[r2] * T1[s2] + T1[r2] * T0[s2]) +
                     2.f * gc * T1[r2] * T1[s2];

    // T = J W: only J00, J02, J11, J12 are non-zero
    const float gJ00 = gT0[0] * V.R[0] + gT0[1] * V.R[1] + gT0[2] * V.R[2];
    const float gJ02 = gT0[0] * V.R[6] + gT0[1] * V.R[7] + gT0[2] * V.R[8];
    const float gJ11 = gT1[0] * V.R[3] + gT1[1] * V.R[4] + gT1[2] * V.R[5];
    const float gJ12 = gT1[0] * V.R[6] + gT1[1] * V.R[7] + gT1[2] * V.R[8];
    const float tx = P.t[0], ty = P.t[1], tz = P.t[2];
    const float iz = 1.f / tz, iz2 = iz * iz;
    float gtx = 0.f, gty = 0.f, gtz = 0.f;
    gtz += -V.fx * iz2 * gJ00 + V.fx * P.rx * iz2 * gJ02 - V.fy * iz2 * gJ11 +
           V.fy * P.ry * iz2 * gJ12;
    const float grx = -V.fx * iz * gJ02, gry = -V.fy * iz * gJ12;
    if (!P.clampx) { gtx += grx * iz; gtz -= grx * tx * iz2; }
    if (!P.clampy) { gty += gry * iz; gtz -= gry * ty * iz2; }
    // mean2D
    gtx += gu * V.fx * iz;
    gtz -= gu * V.fx * tx * iz2;
    gty += gv * V.fy * iz;
    gtz -= gv * V.fy * ty * iz2;
    // t = W mu + t_w
#pragma unroll
    for (int k = 0; k < 3; ++k) gmu[k] += V.R[k] * gtx + V.R[3 + k] * gty + V.R[6 + k] * gtz;

    // Sigma = M M^T, M = Rq diag(s): dL/dM = Gs M
    const float* Rq = P.Rq;
    float gR[9];
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      float acc = 0.f;
#pragma unroll
      for (int r2 = 0; r2 < 3; ++r2) {
        const float gM = (Gs[r2][0] * Rq[k] + Gs[r2][1] * Rq[3 + k] + Gs[r2][2] * Rq[6 + k]) * P.s[k];
        acc += gM * Rq[3 * r2 + k];
        gR[3 * r2 + k] = gM * P.s[k];
      }
      gs[k] += acc;
    }
    // Rq(q) -> unit quaternion -> raw quaternion
    const float w = P.qn[0], x = P.qn[1], y = P.qn[2], z = P.qn[3];
    const float gw = 2.f * (-z * gR[1] + y * gR[2] + z * gR[3] - x * gR[5] - y * gR[6] + x * gR[7]);
    const float gx = 2.f * (y * gR[1] + z * gR[2] + y * gR[3] - w * gR[5] + z * gR[6] + w * gR[7]) -
                     4.f * x * (gR[4] + gR[8]);
    const float gy = 2.f * (x * gR[1] + w * gR[2] + x * gR[3] + z * gR[5] - w * gR[6] + z * gR[7]) -
                     4.f * y * (gR[0] + gR[8]);
    const float gz = 2.f * (-w * gR[1] + x * gR[2] + w * gR[3] + y * gR[5] + x * gR[6] + y * gR[7]) -
                     4.f * z * (gR[0] + gR[4]);
    const float qd = w * gw + x * gx + y * gy + z * gz;
    gq[0] += (gw - w * qd) * P.qinv;
    gq[1] += (gx - x * qd) * P.qinv;
    gq[2] += (gy - y * qd) * P.qinv;
    gq[3] += (gz - z * qd) * P.qinv;
  }

  GradDev G;
  switch (sidx) {
    case 0: G = G0; break;
    case 1: G = G1; break;
    case 2: G = G2; break;
    case 3: G = G3; break;
    case 4: G = G4; break;
    case 5: G = G5; break;
    case 6: G = G6; break;
    default: G = G7; break;
  }
  const size_t ld = S.ld;
  if (accumulate) {
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      G.means[k * ld + i] += gmu[k];
      G.scales[k * ld + i] += gs[k];
    }
#pragma unroll
    for (int k = 0; k < 4; ++k) G.quats[k * ld + i] += gq[k];
    G.opac[i] += go;
#pragma unroll
    for (int j = 0; j < NB; ++j)
#pragma unroll
      for (int ch = 0; ch < 3; ++ch) G.sh[(3 * j + ch) * ld + i] += gsh[j][ch];
  } else {
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      G.means[k * ld + i] = gmu[k];
      G.scales[k * ld + i] = gs[k];
    }
#pragma unroll
    for (int k = 0; k < 4; ++k) G.quats[k * ld + i] = gq[k];
    G.opac[i] = go;
#pragma unroll
    for (int j = 0; j < NB; ++j)
#pragma unroll
      for (int ch = 0; ch < 3; ++ch) G.sh[(3 * j + ch) * ld + i] = gsh[j][ch];
    for (int j = NB; j < S.K; ++j)
      for (int ch = 0; ch < 3; ++ch) G.sh[(3 * j + ch) * ld + i] = 0.f;
  }
}

// Launchers ------------------------------------------------------------------

hipError_t launch_project(const Batch& B, int max_n, float* splat, float* depth, int16_t* rect,
                          int32_t* tc, hipStream_t st) {
  if (max_n <= 0) return hipSuccess;
  dim3 grid((max_n + 255) / 256, B.n_views);
  float4* sp = reinterpret_cast<float4*>(splat);
  short4* rc = reinterpret_cast<short4*>(rect);
  switch (B.sh_degree) {
    case 0: hipLaunchKernelGGL(k_project<0>, grid, dim3(256), 0, st, B, sp, depth, rc, tc); break;
    case 1: hipLaunchKernelGGL(k_project<1>, grid, dim3(256), 0, st, B, sp, depth, rc, tc); break;
    case 2: hipLaunchKernelGGL(k_project<2>, grid, dim3(256), 0, st, B, sp, depth, rc, tc); break;
    default: hipLaunchKernelGGL(k_project<3>, grid, dim3(256), 0, st, B, sp, depth, rc, tc); break;
  }
  return hipGetLastError();
}

hipError_t launch_project_bwd(const Batch& B, int max_n, const float* grad2d, const int32_t* tc,
                              const GradDev* G, int accumulate, hipStream_t st) {
  if (max_n <= 0) return hipSuccess;
  dim3 grid((max_n + 255) / 256, B.n_scenes);
#define XPR_PB(D)                                                                          \
  hipLaunchKernelGGL(k_project_bwd<D>, grid, dim3(256), 0, st, B, grad2d, tc, G[0], G[1], \
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
