// FP64 CPU oracle for tile-based splatting of 3D Gaussians (3DGS), forward
// and backward.
//
// TEST INFRASTRUCTURE ONLY. Only the tests, the smoke check and the bench's
// CPU-baseline leg may load this library. The GPU path shares no code,
// header, table or helper with it.
//
// What it computes follows the paper (XPR, arxiv 2606.11529):
//   * Background section: 3D Gaussian G(x) with covariance R S S^T R^T,
//     opacity o, SH colour; alpha blending c = sum c_i a_i T_i with
//     T_i = prod_{j<i} (1 - a_j) and termination on low transmittance.
//   * Listing "Implementation of XPR-3DGS", function project: world->camera,
//     EWA 2D covariance, conic, extents/radius, tile-space bounding box,
//     tile count, visibility flag, colour, shader data (mu2D, -0.5*con00,
//     -con01, -0.5*con11, o, c); function evaluate: power and alpha.
//   * Section "Rasterizer": replicate by prefix sum, tile id
//     t = y*W' + x with x = xmin + (r mod w), y = ymin + floor(r/w), sort by
//     (tile id, depth), per-tile segment bounds; optionally tile_cull of the
//     XPR-3DGS listing per replicated pair, culled pairs moved to a sentinel
//     tile (the largest-response test the XPR-3DGS section describes).
//   * Section "Shader", Algorithm 1: per-pixel front-to-back loop over the
//     tile's list, gate and accumulate.
//   * Listing "Implementation of XPR-3DGUT" (forward only): unscented-
//     transform projection, pixel_info (ray direction) and the ray-based
//     evaluate at tau_max; tile_cull with the extended tile bounds.
//   * Listing "Implementation of XPR-LinPrim" (forward): the linear map A of
//     each octahedron, slab-pair ray intersection, Beer-Lambert opacity, and
//     tile_cull with the per-tile chord bound of the XPR-LinPrim section.
// Readings where the paper is silent (pixel sample position, low-pass 0.3,
// 3-sigma radius from the largest eigenvalue, conservative rect rounding,
// alpha clamp 0.99, stop at T < 1e-4 before blending, ties by index, SH
// basis with Condon-Shortley phase, +0.5 colour offset and clamp at 0,
// off-screen Jacobian clamp 1.3*tan(fov/2)) are listed with the design notes.
//
// The backward is the analytic derivative of the forward above (the paper
// differentiates its pipeline with JAX autodiff, section "Key Interfaces"):
// gate, stop and rect decisions are piecewise constant (zero derivative), and
// the clamps (Jacobian clamp, colour >= 0, alpha <= 0.99) take the true
// one-sided derivative.
//
// All array arguments are plain host arrays. Per-Gaussian SoA inputs are
// [k][n] (component-major) in double precision; the caller casts float32
// inputs exactly.

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <vector>
#ifdef _OPENMP
#include <omp.h>
#include <parallel/algorithm>
#endif

namespace {

// ----------------------------------------------------------------------------
// Real spherical harmonics up to degree 3, orthonormal on the unit sphere,
// with the Condon-Shortley phase kept: for m > 0 the function is
// sqrt(2) Re Y_l^m, for m < 0 it is sqrt(2) Im Y_l^|m|, ordered m = -l..l.
// Normalisation constants from the closed forms sqrt((2l+1)/(4pi) (l-m)!/(l+m)!).
// ----------------------------------------------------------------------------
struct ShConst {
  double k0, k1, k2a, k2b, k2c, k3a, k3b, k3c, k3d, k3e;
  ShConst() {
    const double pi = 3.14159265358979323846;
    k0 = 0.5 / std::sqrt(pi);
    k1 = std::sqrt(3.0 / (4.0 * pi));
    k2a = 0.5 * std::sqrt(15.0 / pi);
    k2b = 0.25 * std::sqrt(5.0 / pi);
    k2c = 0.25 * std::sqrt(15.0 / pi);
    k3a = 0.25 * std::sqrt(35.0 / (2.0 * pi));
    k3b = 0.5 * std::sqrt(105.0 / pi);
    k3c = 0.25 * std::sqrt(21.0 / (2.0 * pi));
    k3d = 0.25 * std::sqrt(7.0 / pi);
    k3e = 0.25 * std::sqrt(105.0 / pi);
  }
};
const ShConst SHK;

// Y[j] and dY[j][0..2] = dY_j/d(x,y,z) for j < (deg+1)^2, at unit direction d.
void sh_basis(int deg, const double d[3], double* Y, double (*dY)[3]) {
  const double x = d[0], y = d[1], z = d[2];
  const ShConst& k = SHK;
  auto set = [&](int j, double v, double gx, double gy, double gz) {
    Y[j] = v;
    if (dY) { dY[j][0] = gx; dY[j][1] = gy; dY[j][2] = gz; }
  };
  set(0, k.k0, 0, 0, 0);
  if (deg < 1) return;
  set(1, -k.k1 * y, 0, -k.k1, 0);
  set(2, k.k1 * z, 0, 0, k.k1);
  set(3, -k.k1 * x, -k.k1, 0, 0);
  if (deg < 2) return;
  set(4, k.k2a * x * y, k.k2a * y, k.k2a * x, 0);
  set(5, -k.k2a * y * z, 0, -k.k2a * z, -k.k2a * y);
  set(6, k.k2b * (2 * z * z - x * x - y * y), -2 * k.k2b * x, -2 * k.k2b * y, 4 * k.k2b * z);
  set(7, -k.k2a * x * z, -k.k2a * z, 0, -k.k2a * x);
  set(8, k.k2c * (x * x - y * y), 2 * k.k2c * x, -2 * k.k2c * y, 0);
  if (deg < 3) return;
  set(9, -k.k3a * y * (3 * x * x - y * y), -6 * k.k3a * x * y, -k.k3a * (3 * x * x - 3 * y * y), 0);
  set(10, k.k3b * x * y * z, k.k3b * y * z, k.k3b * x * z, k.k3b * x * y);
  set(11, -k.k3c * y * (4 * z * z - x * x - y * y), 2 * k.k3c * x * y,
      -k.k3c * (4 * z * z - x * x - 3 * y * y), -8 * k.k3c * y * z);
  set(12, k.k3d * z * (2 * z * z - 3 * x * x - 3 * y * y), -6 * k.k3d * x * z, -6 * k.k3d * y * z,
      k.k3d * (6 * z * z - 3 * x * x - 3 * y * y));
  set(13, -k.k3c * x * (4 * z * z - x * x - y * y), -k.k3c * (4 * z * z - 3 * x * x - y * y),
      2 * k.k3c * x * y, -8 * k.k3c * x * z);
  set(14, k.k3e * z * (x * x - y * y), 2 * k.k3e * x * z, -2 * k.k3e * y * z, k.k3e * (x * x - y * y));
  set(15, -k.k3a * x * (x * x - 3 * y * y), -k.k3a * (3 * x * x - 3 * y * y), 6 * k.k3a * x * y, 0);
}

// ----------------------------------------------------------------------------
// Small dense helpers (row-major 3x3).
// ----------------------------------------------------------------------------
struct Cam {
  double R[9], t[3], fx, fy, cx, cy;
  int W, H;
};

Cam read_cam(const double* c, int W, int H) {
  Cam k;
  for (int i = 0; i < 9; ++i) k.R[i] = c[i];
  for (int i = 0; i < 3; ++i) k.t[i] = c[9 + i];
  k.fx = c[12]; k.fy = c[13]; k.cx = c[14]; k.cy = c[15];
  k.W = W; k.H = H;
  return k;
}

// Rotation matrix of a unit quaternion (w, x, y, z).
void quat_to_rot(const double q[4], double Rq[9]) {
  const double w = q[0], x = q[1], y = q[2], z = q[3];
  Rq[0] = 1 - 2 * (y * y + z * z); Rq[1] = 2 * (x * y - w * z);     Rq[2] = 2 * (x * z + w * y);
  Rq[3] = 2 * (x * y + w * z);     Rq[4] = 1 - 2 * (x * x + z * z); Rq[5] = 2 * (y * z - w * x);
  Rq[6] = 2 * (x * z - w * y);     Rq[7] = 2 * (y * z + w * x);     Rq[8] = 1 - 2 * (x * x + y * y);
}

// d Rq[k] / d q[c] for c = w, x, y, z.
void quat_to_rot_jac(const double q[4], double dR[9][4]) {
  const double w = q[0], x = q[1], y = q[2], z = q[3];
  const double J[9][4] = {
      {0, 0, -4 * y, -4 * z},      {-2 * z, 2 * y, 2 * x, -2 * w}, {2 * y, 2 * z, 2 * w, 2 * x},
      {2 * z, 2 * y, 2 * x, 2 * w}, {0, -4 * x, 0, -4 * z},        {-2 * x, -2 * w, 2 * z, 2 * y},
      {-2 * y, 2 * z, -2 * w, 2 * x}, {2 * x, 2 * w, 2 * z, 2 * y}, {0, -4 * x, -4 * y, 0}};
  std::memcpy(dR, J, sizeof(J));
}

// Forward quantities of one Gaussian under one camera, kept for the backward.
struct Proj {
  double tcam[3];        // camera-space mean
  double qn[4], qnorm;   // normalised quaternion, norm of the raw one
  double Rq[9];          // rotation of the Gaussian
  double s[3];           // scales
  double Sigma[9];       // 3D covariance
  double rho[2];         // clamped tx/tz, ty/tz
  bool clampx, clampy;
  double T[6];           // 2x3 J*W
  double a, b, c;        // low-passed 2D covariance
  double det;
  double con[3];         // conic (inverse covariance) entries 00, 01, 11
  double u, v;           // mean2D
  double lambda, radius;
  int rect[4];           // x0 y0 x1 y1 (tiles, half-open)
  int tc;
  bool visible;
  double dir[3], dirnorm;  // unit view direction and distance
  double raw[3], colour[3];
  double Y[16];
  bool guard;
};

// Is x within tol of an integer?
bool near_int(double x, double tol) { return std::fabs(x - std::nearbyint(x)) <= tol; }

// Projection of Gaussian i (Listing "XPR-3DGS", project).
void project_one(int64_t i, int64_t n, const double* means, const double* scales,
                 const double* quats, const double* opac, const double* sh, int K,
                 const Cam& cam, const double* cfg, int tile_w, int tile_h, int deg, Proj& P) {
  const double lowpass = cfg[0], alpha_min = cfg[1], z_near = cfg[2], fov_clip = cfg[3];
  const bool opacity_extents = cfg[4] != 0.0;
  const int tiles_x = (cam.W + tile_w - 1) / tile_w;
  const int tiles_y = (cam.H + tile_h - 1) / tile_h;
  std::memset(&P, 0, sizeof(P));
  const double mu[3] = {means[i], means[n + i], means[2 * n + i]};
  // world -> camera
  for (int r = 0; r < 3; ++r)
    P.tcam[r] = cam.R[3 * r] * mu[0] + cam.R[3 * r + 1] * mu[1] + cam.R[3 * r + 2] * mu[2] + cam.t[r];
  const double tx = P.tcam[0], ty = P.tcam[1], tz = P.tcam[2];
  const double o = opac[i];
  // 3D covariance Sigma = Rq S S^T Rq^T from the normalised quaternion.
  const double q[4] = {quats[i], quats[n + i], quats[2 * n + i], quats[3 * n + i]};
  P.qnorm = std::sqrt(q[0] * q[0] + q[1] * q[1] + q[2] * q[2] + q[3] * q[3]);
  for (int c = 0; c < 4; ++c) P.qn[c] = q[c] / P.qnorm;
  quat_to_rot(P.qn, P.Rq);
  for (int c = 0; c < 3; ++c) P.s[c] = scales[c * n + i];
  double M[9];
  for (int r = 0; r < 3; ++r)
    for (int c = 0; c < 3; ++c) M[3 * r + c] = P.Rq[3 * r + c] * P.s[c];
  for (int r = 0; r < 3; ++r)
    for (int c = 0; c < 3; ++c)
      P.Sigma[3 * r + c] = M[3 * r] * M[3 * c] + M[3 * r + 1] * M[3 * c + 1] + M[3 * r + 2] * M[3 * c + 2];

  bool in_front = tz > z_near;
  P.guard = std::fabs(tz - z_near) <= 1e-9 * std::max(1.0, std::fabs(z_near)) ||
            std::fabs(o - alpha_min) <= 1e-9 * alpha_min;
  if (in_front) {
    // EWA: J (perspective Jacobian at the clamped direction) times W.
    const double limx = fov_clip * cam.W / (2.0 * cam.fx);
    const double limy = fov_clip * cam.H / (2.0 * cam.fy);
    double rx = tx / tz, ry = ty / tz;
    if (fov_clip > 0) {
      P.clampx = rx < -limx || rx > limx;
      P.clampy = ry < -limy || ry > limy;
      rx = std::min(limx, std::max(-limx, rx));
      ry = std::min(limy, std::max(-limy, ry));
    }
    P.rho[0] = rx; P.rho[1] = ry;
    const double J[6] = {cam.fx / tz, 0, -cam.fx * rx / tz, 0, cam.fy / tz, -cam.fy * ry / tz};
    for (int r = 0; r < 2; ++r)
      for (int c = 0; c < 3; ++c)
        P.T[3 * r + c] = J[3 * r] * cam.R[c] + J[3 * r + 1] * cam.R[3 + c] + J[3 * r + 2] * cam.R[6 + c];
    // cov2D = T Sigma T^T + lowpass I
    double ST0[3], ST1[3];
    for (int r = 0; r < 3; ++r) {
      ST0[r] = P.Sigma[3 * r] * P.T[0] + P.Sigma[3 * r + 1] * P.T[1] + P.Sigma[3 * r + 2] * P.T[2];
      ST1[r] = P.Sigma[3 * r] * P.T[3] + P.Sigma[3 * r + 1] * P.T[4] + P.Sigma[3 * r + 2] * P.T[5];
    }
    P.a = P.T[0] * ST0[0] + P.T[1] * ST0[1] + P.T[2] * ST0[2] + lowpass;
    P.b = P.T[0] * ST1[0] + P.T[1] * ST1[1] + P.T[2] * ST1[2];
    P.c = P.T[3] * ST1[0] + P.T[4] * ST1[1] + P.T[5] * ST1[2] + lowpass;
    P.det = P.a * P.c - P.b * P.b;
    if (std::fabs(P.det) <= 1e-9 * P.a * P.c) P.guard = true;
    if (P.det > 0) {
      P.con[0] = P.c / P.det;
      P.con[1] = -P.b / P.det;
      P.con[2] = P.a / P.det;
    }
    // mean2D: pixel (i, j) is sampled at (i, j), so the continuous image
    // point f*X/Z + c is shifted by one half pixel.
    P.u = cam.fx * tx / tz + cam.cx - 0.5;
    P.v = cam.fy * ty / tz + cam.cy - 0.5;
    // Extents (compute_extents of the listing): the 3-sigma radius of the
    // largest eigenvalue in both directions, or, opacity-aware, the
    // half-widths of the ellipse 0.5 d^T conic d = log(o / alpha_min) where
    // o G falls to alpha_min: sqrt(2 log(o / alpha_min) cov_xx) and likewise
    // with cov_yy (the extreme x of that ellipse); the radius is their
    // maximum (compute_radius).
    const double mid = 0.5 * (P.a + P.c);
    P.lambda = mid + std::sqrt(std::max(0.0, mid * mid - P.det));
    const double r3 = 3.0 * std::sqrt(P.lambda);
    double ex, ey;
    if (opacity_extents) {
      const double lvl = 2.0 * std::log(o / alpha_min);
      ex = lvl > 0.0 ? std::sqrt(lvl * P.a) : 0.0;
      ey = lvl > 0.0 ? std::sqrt(lvl * P.c) : 0.0;
      P.radius = std::max(ex, ey);
    } else {
      P.radius = std::ceil(r3);
      ex = ey = P.radius;
    }
    // Tile-space bounding box, half-open: covers every pixel sample within
    // the box of half-widths (ex, ey) around mean2D.
    const double fx0 = (P.u - ex) / tile_w, fx1 = (P.u + ex) / tile_w;
    const double fy0 = (P.v - ey) / tile_h, fy1 = (P.v + ey) / tile_h;
    auto clampi = [](double x, int lo, int hi) {
      return (int)std::min<double>(hi, std::max<double>(lo, x));
    };
    P.rect[0] = clampi(std::floor(fx0), 0, tiles_x);
    P.rect[1] = clampi(std::floor(fy0), 0, tiles_y);
    P.rect[2] = clampi(std::floor(fx1) + 1, 0, tiles_x);
    P.rect[3] = clampi(std::floor(fy1) + 1, 0, tiles_y);
    P.tc = (P.rect[2] - P.rect[0]) * (P.rect[3] - P.rect[1]);
    // Guard band of the parity protocol: the radius or a rect boundary within
    // 1e-9 (relative) of an integer, where a float64 computation in another
    // operation order may round the other way.
    const double g = 1e-9;
    if ((!opacity_extents && near_int(r3, g * std::max(1.0, r3))) ||
        near_int(fx0, g * std::max(1.0, std::fabs(fx0))) ||
        near_int(fx1, g * std::max(1.0, std::fabs(fx1))) ||
        near_int(fy0, g * std::max(1.0, std::fabs(fy0))) ||
        near_int(fy1, g * std::max(1.0, std::fabs(fy1))))
      P.guard = true;
  }
  P.visible = in_front && P.det > 0 && o >= alpha_min && P.radius > 0 && P.tc > 0;
  if (!P.visible) P.tc = 0;

  // View-dependent colour from the SH coefficients.
  const double cp[3] = {
      -(cam.R[0] * cam.t[0] + cam.R[3] * cam.t[1] + cam.R[6] * cam.t[2]),
      -(cam.R[1] * cam.t[0] + cam.R[4] * cam.t[1] + cam.R[7] * cam.t[2]),
      -(cam.R[2] * cam.t[0] + cam.R[5] * cam.t[1] + cam.R[8] * cam.t[2])};
  double dv[3] = {mu[0] - cp[0], mu[1] - cp[1], mu[2] - cp[2]};
  P.dirnorm = std::sqrt(dv[0] * dv[0] + dv[1] * dv[1] + dv[2] * dv[2]);
  for (int c = 0; c < 3; ++c) P.dir[c] = dv[c] / P.dirnorm;
  sh_basis(deg, P.dir, P.Y, nullptr);
  const int nb = (deg + 1) * (deg + 1);
  for (int ch = 0; ch < 3; ++ch) {
    double acc = 0.5;
    for (int j = 0; j < nb; ++j) acc += sh[(int64_t)(j * 3 + ch) * n + i] * P.Y[j];
    P.raw[ch] = acc;
    P.colour[ch] = std::max(0.0, acc);
  }
  (void)K;
}

// tile_cull of one (Gaussian, tile) pair (Listing "XPR-3DGS", tile_cull; the
// XPR-3DGS section states the test): the largest contribution o G(x) over
// the tile is reached at the point of the tile where the power
// 0.5 (x - mu)^T conic (x - mu) is smallest, which is mu itself when mu lies
// in the tile and otherwise a point on a tile edge facing mu; the pair is
// kept iff that smallest power is at most log(o / alpha_min).
//
// Readings: the tile is the box spanned by its pixel samples,
// [tx tw, tx tw + tw - 1] x [ty th, ty th + th - 1] clipped to the image
// (pixel (i, j) is sampled at (i, j)); a conic that is not positive
// definite (possible once rounded to float32) has no bounded footprint and
// its pairs are kept. guard marks a smallest power within 1e-9 (relative)
// of the level, where another float64 evaluation order may decide the other
// way.
struct CullTest {
  bool keep, guard;
  double power, level;
};

CullTest tile_cull_one(const double* rec, int tx, int ty, int W, int H, int tile_w, int tile_h,
                       double alpha_min, int ext = 0) {
  // ext = 1 for 3DGUT: its tile_cull first moves tile_max out by one pixel
  // in x and y (the ray offset adjustment of Listing "XPR-3DGUT")
  const double X0 = (double)tx * tile_w, X1 = std::min(X0 + tile_w - 1, W - 1.0) + ext;
  const double Y0 = (double)ty * tile_h, Y1 = std::min(Y0 + tile_h - 1, H - 1.0) + ext;
  const double u = rec[0], v = rec[1];
  // conic entries from the shader data (-0.5 con00, -con01, -0.5 con11)
  const double a = -2.0 * rec[2], b = -rec[3], c = -2.0 * rec[4], o = rec[5];
  CullTest r{true, false, 0.0, std::log(o / alpha_min)};
  if (!(a > 0.0 && a * c - b * b > 0.0)) return r;
  auto q = [&](double dx, double dy) { return a * dx * dx + 2.0 * b * dx * dy + c * dy * dy; };
  auto clampd = [](double x, double lo, double hi) { return std::min(hi, std::max(lo, x)); };
  const bool out_x = u < X0 || u > X1, out_y = v < Y0 || v > Y1;
  double best = 0.0;
  if (out_x || out_y) {
    best = INFINITY;
    if (out_x) {
      // vertical edge facing mu: q along it is smallest at dy = -b dx / c
      const double dx = (u < X0 ? X0 : X1) - u;
      const double y = clampd(v - b * dx / c, Y0, Y1);
      best = std::min(best, q(dx, y - v));
    }
    if (out_y) {
      // horizontal edge facing mu: smallest at dx = -b dy / a
      const double dy = (v < Y0 ? Y0 : Y1) - v;
      const double x = clampd(u - b * dy / a, X0, X1);
      best = std::min(best, q(x - u, dy));
    }
  }
  r.power = 0.5 * best;
  r.keep = r.power <= r.level;
  r.guard = std::fabs(r.power - r.level) <= 1e-9 * std::max(1.0, std::fabs(r.level));
  return r;
}

// ----------------------------------------------------------------------------
// 3DGUT (Listing "Implementation of XPR-3DGUT"): unscented-transform
// projection and per-pixel ray evaluation.
//
// Readings: the unscented transform of n = 3 dimensions with alpha = 1,
// beta = 2, kappa = 0, so lambda = 0: sigma points mu and
// mu +- sqrt(3) s_j R e_j (j = 0..2), mean weights 0 (centre) and 1/6,
// covariance weights 2 (centre) and 1/6; the 2D points are the pinhole
// projections f X / Z + c; a Gaussian with a sigma point at camera depth
// <= z_near is not visible (the projection is undefined there); the opacity
// compensation of the low-pass (Mip-Splatting) is sqrt(det_orig / det).
// ----------------------------------------------------------------------------
struct GutProj {
  double u, v, A, B, C, o;  // 2D cull data (mean2D - 1/2, scaled conic), adjusted opacity
  double colour[3];
  double ro[3], M[9];       // canonical ray origin, M = S^-1 R^T (row-major)
  double a, b, c;           // low-passed 2D covariance
  double depth;
  int rect[4];
  int tc;
  bool guard;
};

void project_gut_one(int64_t i, int64_t n, const double* means, const double* scales,
                     const double* quats, const double* opac, const double* sh, const Cam& cam,
                     const double* cfg, int tile_w, int tile_h, int deg, GutProj& G) {
  const double lowpass = cfg[0], alpha_min = cfg[1], z_near = cfg[2];
  const bool opacity_extents = cfg[3] != 0.0;
  const int tiles_x = (cam.W + tile_w - 1) / tile_w;
  const int tiles_y = (cam.H + tile_h - 1) / tile_h;
  std::memset(&G, 0, sizeof(G));
  const double mu[3] = {means[i], means[n + i], means[2 * n + i]};
  const double q[4] = {quats[i], quats[n + i], quats[2 * n + i], quats[3 * n + i]};
  const double qn = std::sqrt(q[0] * q[0] + q[1] * q[1] + q[2] * q[2] + q[3] * q[3]);
  const double qu[4] = {q[0] / qn, q[1] / qn, q[2] / qn, q[3] / qn};
  double Rq[9];
  quat_to_rot(qu, Rq);
  const double s[3] = {scales[i], scales[n + i], scales[2 * n + i]};
  // sigma points: centre, then +- sqrt(3) s_j times column j of Rq
  double X[7][3];
  for (int c = 0; c < 3; ++c) X[0][c] = mu[c];
  const double k = std::sqrt(3.0);
  for (int j = 0; j < 3; ++j)
    for (int sg = 0; sg < 2; ++sg)
      for (int c = 0; c < 3; ++c)
        X[1 + 2 * j + sg][c] = mu[c] + (sg ? -1.0 : 1.0) * k * s[j] * Rq[3 * c + j];
  const double wm[7] = {0.0, 1.0 / 6, 1.0 / 6, 1.0 / 6, 1.0 / 6, 1.0 / 6, 1.0 / 6};
  const double wc[7] = {2.0, 1.0 / 6, 1.0 / 6, 1.0 / 6, 1.0 / 6, 1.0 / 6, 1.0 / 6};
  double P2[7][2];
  bool front = true;
  double zc = 0.0;
  for (int p = 0; p < 7; ++p) {
    double y[3];
    for (int r = 0; r < 3; ++r)
      y[r] = cam.R[3 * r] * X[p][0] + cam.R[3 * r + 1] * X[p][1] + cam.R[3 * r + 2] * X[p][2] +
             cam.t[r];
    if (p == 0) zc = y[2];
    if (!(y[2] > z_near)) front = false;
    if (std::fabs(y[2] - z_near) <= 1e-9 * std::max(1.0, z_near)) G.guard = true;
    P2[p][0] = cam.fx * y[0] / y[2] + cam.cx;
    P2[p][1] = cam.fy * y[1] / y[2] + cam.cy;
  }
  G.depth = zc;
  double m2[2] = {0.0, 0.0};
  for (int p = 0; p < 7; ++p) {
    m2[0] += wm[p] * P2[p][0];
    m2[1] += wm[p] * P2[p][1];
  }
  double cxx = 0.0, cxy = 0.0, cyy = 0.0;
  for (int p = 0; p < 7; ++p) {
    const double dx = P2[p][0] - m2[0], dy = P2[p][1] - m2[1];
    cxx += wc[p] * dx * dx;
    cxy += wc[p] * dx * dy;
    cyy += wc[p] * dy * dy;
  }
  const double det_orig = cxx * cyy - cxy * cxy;
  G.a = cxx + lowpass;
  G.b = cxy;
  G.c = cyy + lowpass;
  const double det = G.a * G.c - G.b * G.b;
  if (std::fabs(det) <= 1e-9 * G.a * G.c) G.guard = true;
  double con[3] = {0.0, 0.0, 0.0};
  if (det > 0) {
    con[0] = G.c / det;
    con[1] = -G.b / det;
    con[2] = G.a / det;
  }
  const double o = opac[i] * (det > 0 ? std::sqrt(std::max(det_orig, 0.0) / det) : 0.0);
  G.o = o;
  if (std::fabs(o - alpha_min) <= 1e-9 * alpha_min) G.guard = true;
  // the bounding box is placed at mean2D - 1/2 (ray offset): pixel (i, j)
  // is the ray through (i + 1/2, j + 1/2)
  G.u = m2[0] - 0.5;
  G.v = m2[1] - 0.5;
  G.A = -0.5 * con[0];
  G.B = -con[1];
  G.C = -0.5 * con[2];
  double ex, ey, rad;
  if (opacity_extents) {
    const double lvl = o > 0 ? 2.0 * std::log(o / alpha_min) : -1.0;
    ex = lvl > 0.0 ? std::sqrt(lvl * G.a) : 0.0;
    ey = lvl > 0.0 ? std::sqrt(lvl * G.c) : 0.0;
    rad = std::max(ex, ey);
  } else {
    const double mid = 0.5 * (G.a + G.c);
    const double lam = mid + std::sqrt(std::max(0.0, mid * mid - det));
    const double r3 = 3.0 * std::sqrt(lam);
    if (near_int(r3, 1e-9 * std::max(1.0, r3))) G.guard = true;
    rad = std::ceil(r3);
    ex = ey = rad;
  }
  const double fx0 = (G.u - ex) / tile_w, fx1 = (G.u + ex) / tile_w;
  const double fy0 = (G.v - ey) / tile_h, fy1 = (G.v + ey) / tile_h;
  auto clampi = [](double x, int lo, int hi) {
    return (int)std::min<double>(hi, std::max<double>(lo, x));
  };
  G.rect[0] = clampi(std::floor(fx0), 0, tiles_x);
  G.rect[1] = clampi(std::floor(fy0), 0, tiles_y);
  G.rect[2] = clampi(std::floor(fx1) + 1, 0, tiles_x);
  G.rect[3] = clampi(std::floor(fy1) + 1, 0, tiles_y);
  const double g = 1e-9;
  if (near_int(fx0, g * std::max(1.0, std::fabs(fx0))) ||
      near_int(fx1, g * std::max(1.0, std::fabs(fx1))) ||
      near_int(fy0, g * std::max(1.0, std::fabs(fy0))) ||
      near_int(fy1, g * std::max(1.0, std::fabs(fy1))))
    G.guard = true;
  const int area = (G.rect[2] - G.rect[0]) * (G.rect[3] - G.rect[1]);
  const bool visible = front && det > 0 && o > alpha_min && rad > 0 && area > 0;
  G.tc = visible ? area : 0;
  // shader data: M = S^-1 R^T and the camera position in canonical space
  for (int r = 0; r < 3; ++r)
    for (int c = 0; c < 3; ++c) G.M[3 * r + c] = Rq[3 * c + r] / s[r];
  const double cp[3] = {
      -(cam.R[0] * cam.t[0] + cam.R[3] * cam.t[1] + cam.R[6] * cam.t[2]),
      -(cam.R[1] * cam.t[0] + cam.R[4] * cam.t[1] + cam.R[7] * cam.t[2]),
      -(cam.R[2] * cam.t[0] + cam.R[5] * cam.t[1] + cam.R[8] * cam.t[2])};
  for (int r = 0; r < 3; ++r)
    G.ro[r] = G.M[3 * r] * (cp[0] - mu[0]) + G.M[3 * r + 1] * (cp[1] - mu[1]) +
              G.M[3 * r + 2] * (cp[2] - mu[2]);
  // view-dependent colour, as for 3DGS
  double dv[3] = {mu[0] - cp[0], mu[1] - cp[1], mu[2] - cp[2]};
  const double dn = std::sqrt(dv[0] * dv[0] + dv[1] * dv[1] + dv[2] * dv[2]);
  for (int c = 0; c < 3; ++c) dv[c] /= dn;
  double Y[16];
  sh_basis(deg, dv, Y, nullptr);
  const int nb = (deg + 1) * (deg + 1);
  for (int ch = 0; ch < 3; ++ch) {
    double acc = 0.5;
    for (int j = 0; j < nb; ++j) acc += sh[(int64_t)(j * 3 + ch) * n + i] * Y[j];
    G.colour[ch] = std::max(0.0, acc);
  }
}

// pixel_info of 3DGUT: the world-space unit direction of the ray through
// pixel (px, py), i.e. through (px + 1/2, py + 1/2).
void gut_ray(const Cam& cam, int px, int py, double rd[3]) {
  double dc[3] = {(px + 0.5 - cam.cx) / cam.fx, (py + 0.5 - cam.cy) / cam.fy, 1.0};
  const double nn = std::sqrt(dc[0] * dc[0] + dc[1] * dc[1] + dc[2] * dc[2]);
  for (int c = 0; c < 3; ++c) dc[c] /= nn;
  for (int c = 0; c < 3; ++c)
    rd[c] = cam.R[c] * dc[0] + cam.R[3 + c] * dc[1] + cam.R[6 + c] * dc[2];
}

// evaluate of 3DGUT: the largest response of the canonical Gaussian
// exp(-|x|^2 / 2) along the ray ro + tau M rd, reached at
// tau_max = -(ro . rdc) / (rdc . rdc).
double gut_response(const double* ro, const double* M, const double rd[3]) {
  double rdc[3];
  for (int r = 0; r < 3; ++r) rdc[r] = M[3 * r] * rd[0] + M[3 * r + 1] * rd[1] + M[3 * r + 2] * rd[2];
  const double tau = -(ro[0] * rdc[0] + ro[1] * rdc[1] + ro[2] * rdc[2]) /
                     (rdc[0] * rdc[0] + rdc[1] * rdc[1] + rdc[2] * rdc[2]);
  double d2 = 0.0;
  for (int r = 0; r < 3; ++r) {
    const double x = ro[r] + tau * rdc[r];
    d2 += x * x;
  }
  return std::exp(-0.5 * d2);
}

// ----------------------------------------------------------------------------
// LinPrim (Listing "Implementation of XPR-LinPrim", forward): octahedra
// {mu + R diag(s) u : |u|_1 <= 1} with homogeneous density, projected by
// the linear map A = J3 R_w2c R diag(s) to (x_px, y_px, tau) (tau the
// Euclidean depth relative to the centre), evaluated by intersecting the
// pixel ray with the four slab pairs |n_i . (dx, dy, tau)| <= 1,
// n_i = c0 +- c1 +- c2 (c_k the rows of A^-1), opacity by Beer-Lambert.
//
// Readings: J3 stacks the perspective Jacobian rows (fx/z, 0, -fx x/z^2),
// (0, fy/z, -fy y/z^2) on the unit viewing direction mu_c / |mu_c| (the
// derivative of the Euclidean distance); the extents are the largest
// |A_0k| and |A_1k| (the projected vertices mu_2D +- A e_k bound the
// footprint) and compute_radius their maximum; the depth is |mu_c|; a
// primitive is visible only if its centre is in front (z_c > z_near), A is
// invertible and s_min > 0; a slab with |n_z| < 1e-10 does not constrain
// tau where |n_x dx + n_y dy| <= 1 and excludes the pixel elsewhere.
// ----------------------------------------------------------------------------
struct LinProj {
  double u2, v2;     // mu_2D (f x / z + c)
  double c[9];       // rows of A^-1
  double sigma, ex, ey, depth;
  double colour[3];
  int rect[4];
  int tc;
  bool guard;
};

bool inv3(const double* m, double* inv) {
  const double c00 = m[4] * m[8] - m[5] * m[7], c01 = m[5] * m[6] - m[3] * m[8],
               c02 = m[3] * m[7] - m[4] * m[6];
  const double det = m[0] * c00 + m[1] * c01 + m[2] * c02;
  if (!(std::fabs(det) > 0.0) || !std::isfinite(det)) return false;
  const double id = 1.0 / det;
  inv[0] = c00 * id; inv[1] = (m[2] * m[7] - m[1] * m[8]) * id; inv[2] = (m[1] * m[5] - m[2] * m[4]) * id;
  inv[3] = c01 * id; inv[4] = (m[0] * m[8] - m[2] * m[6]) * id; inv[5] = (m[2] * m[3] - m[0] * m[5]) * id;
  inv[6] = c02 * id; inv[7] = (m[1] * m[6] - m[0] * m[7]) * id; inv[8] = (m[0] * m[4] - m[1] * m[3]) * id;
  return true;
}

void project_lin_one(int64_t i, int64_t n, const double* means, const double* scales,
                     const double* quats, const double* opac, const double* sh, const Cam& cam,
                     const double* cfg, int tile_w, int tile_h, int deg, LinProj& L) {
  const double z_near = cfg[2];
  const int tiles_x = (cam.W + tile_w - 1) / tile_w;
  const int tiles_y = (cam.H + tile_h - 1) / tile_h;
  std::memset(&L, 0, sizeof(L));
  const double mu[3] = {means[i], means[n + i], means[2 * n + i]};
  double mc[3];
  for (int r = 0; r < 3; ++r)
    mc[r] = cam.R[3 * r] * mu[0] + cam.R[3 * r + 1] * mu[1] + cam.R[3 * r + 2] * mu[2] + cam.t[r];
  const double x = mc[0], y = mc[1], z = mc[2];
  const double d = std::sqrt(x * x + y * y + z * z);
  L.depth = d;
  if (std::fabs(z - z_near) <= 1e-9 * std::max(1.0, z_near)) L.guard = true;
  const double q[4] = {quats[i], quats[n + i], quats[2 * n + i], quats[3 * n + i]};
  const double qn = std::sqrt(q[0] * q[0] + q[1] * q[1] + q[2] * q[2] + q[3] * q[3]);
  const double qu[4] = {q[0] / qn, q[1] / qn, q[2] / qn, q[3] / qn};
  double Rq[9];
  quat_to_rot(qu, Rq);
  const double s[3] = {scales[i], scales[n + i], scales[2 * n + i]};
  const double smin = std::min(s[0], std::min(s[1], s[2]));
  // A = J3 R_w2c Rq diag(s)
  const double J[9] = {cam.fx / z, 0.0, -cam.fx * x / (z * z), 0.0, cam.fy / z,
                       -cam.fy * y / (z * z), x / d, y / d, z / d};
  double W[9], A[9];
  for (int r = 0; r < 3; ++r)
    for (int c = 0; c < 3; ++c)
      W[3 * r + c] = cam.R[3 * r] * Rq[c] + cam.R[3 * r + 1] * Rq[3 + c] + cam.R[3 * r + 2] * Rq[6 + c];
  for (int r = 0; r < 3; ++r)
    for (int c = 0; c < 3; ++c)
      A[3 * r + c] = (J[3 * r] * W[c] + J[3 * r + 1] * W[3 + c] + J[3 * r + 2] * W[6 + c]) * s[c];
  const bool inv_ok = z > z_near && smin > 0.0 && inv3(A, L.c);
  L.u2 = cam.fx * x / z + cam.cx;
  L.v2 = cam.fy * y / z + cam.cy;
  L.ex = std::max(std::fabs(A[0]), std::max(std::fabs(A[1]), std::fabs(A[2])));
  L.ey = std::max(std::fabs(A[3]), std::max(std::fabs(A[4]), std::fabs(A[5])));
  const double r = std::max(L.ex, L.ey);
  const double o = std::min(0.999, std::max(0.0, opac[i]));
  L.sigma = smin > 0.0 ? -std::log1p(-0.99 * o) / (2.0 * smin) : 0.0;
  const double u = L.u2 - 0.5, v = L.v2 - 0.5;
  const double fx0 = (u - L.ex) / tile_w, fx1 = (u + L.ex) / tile_w;
  const double fy0 = (v - L.ey) / tile_h, fy1 = (v + L.ey) / tile_h;
  auto clampi = [](double t, int lo, int hi) {
    return (int)std::min<double>(hi, std::max<double>(lo, t));
  };
  L.rect[0] = clampi(std::floor(fx0), 0, tiles_x);
  L.rect[1] = clampi(std::floor(fy0), 0, tiles_y);
  L.rect[2] = clampi(std::floor(fx1) + 1, 0, tiles_x);
  L.rect[3] = clampi(std::floor(fy1) + 1, 0, tiles_y);
  const double g = 1e-9;
  if (near_int(fx0, g * std::max(1.0, std::fabs(fx0))) ||
      near_int(fx1, g * std::max(1.0, std::fabs(fx1))) ||
      near_int(fy0, g * std::max(1.0, std::fabs(fy0))) ||
      near_int(fy1, g * std::max(1.0, std::fabs(fy1))))
    L.guard = true;
  const int area = (L.rect[2] - L.rect[0]) * (L.rect[3] - L.rect[1]);
  const bool visible = inv_ok && r > 0 && area > 0 && d > z_near;
  L.tc = visible ? area : 0;
  double dv[3] = {mu[0], mu[1], mu[2]};
  const double cp[3] = {
      -(cam.R[0] * cam.t[0] + cam.R[3] * cam.t[1] + cam.R[6] * cam.t[2]),
      -(cam.R[1] * cam.t[0] + cam.R[4] * cam.t[1] + cam.R[7] * cam.t[2]),
      -(cam.R[2] * cam.t[0] + cam.R[5] * cam.t[1] + cam.R[8] * cam.t[2])};
  for (int k = 0; k < 3; ++k) dv[k] -= cp[k];
  const double dn = std::sqrt(dv[0] * dv[0] + dv[1] * dv[1] + dv[2] * dv[2]);
  for (int k = 0; k < 3; ++k) dv[k] /= dn;
  double Y[16];
  sh_basis(deg, dv, Y, nullptr);
  const int nb = (deg + 1) * (deg + 1);
  for (int ch = 0; ch < 3; ++ch) {
    double acc = 0.5;
    for (int j = 0; j < nb; ++j) acc += sh[(int64_t)(j * 3 + ch) * n + i] * Y[j];
    L.colour[ch] = std::max(0.0, acc);
  }
}

// Chord of the ray through pixel-centre offset (dx, dy) inside the slabs:
// [enter, exit] = intersection over i of {tau : |n_i . (dx, dy, tau)| <= 1};
// returns exit - enter, or a value <= 0 when empty.
double lin_chord(const double* c, double dx, double dy) {
  double enter = -INFINITY, exit_ = INFINITY;
  for (int i = 0; i < 4; ++i) {
    const double e1 = (i & 2) ? -1.0 : 1.0, e2 = (i & 1) ? -1.0 : 1.0;
    const double nx = c[0] + e1 * c[3] + e2 * c[6];
    const double ny = c[1] + e1 * c[4] + e2 * c[7];
    const double nz = c[2] + e1 * c[5] + e2 * c[8];
    const double w = nx * dx + ny * dy;
    if (std::fabs(nz) >= 1e-10) {
      const double m = -w / nz, h = 1.0 / std::fabs(nz);
      enter = std::max(enter, m - h);
      exit_ = std::min(exit_, m + h);
    } else if (std::fabs(w) > 1.0) {
      return -1.0;
    }
  }
  return exit_ - enter;
}

// tile_cull of one (octahedron, tile) pair (Listing "XPR-LinPrim",
// tile_cull; the per-tile upper bound and cull predicate of the XPR-LinPrim
// section). Every chord over the tile is at most
//   bound = max(0, min over ordered slab pairs (i, j) of
//               [max over the box corners of (m_i - m_j) + h_i + h_j])
// with m_i = -(n_ix dx + n_iy dy) / n_iz and h_i = 1 / |n_iz| at each corner
// (dx, dy) = corner - u; a slab with |n_iz| < 1e-10 leaves tau free and is
// dropped from the minimum (its gaps are +infinity). The pair is culled iff
// sigma bound < -log(1 - alpha_min).
//
// Readings: the box is the pixel-sample box of the 3DGS cull,
// [tx tw, min(tx tw + tw - 1, W - 1)] x [ty th, min(ty th + th - 1, H - 1)],
// with the sample of pixel x at x + 1/2, so that its offset from mu_2D is
// x - u (u = mu_2D - 1/2). power holds sigma bound, level the threshold;
// guard marks sigma bound within 1e-9 (relative) of the threshold.
CullTest lin_cull_one(const double* rec, int tx, int ty, int W, int H, int tile_w, int tile_h,
                      double alpha_min) {
  const double X0 = (double)tx * tile_w, X1 = std::min(X0 + tile_w - 1, W - 1.0);
  const double Y0 = (double)ty * tile_h, Y1 = std::min(Y0 + tile_h - 1, H - 1.0);
  const double u = rec[0], v = rec[1], sigma = rec[2];
  const double* c = rec + 8;  // rows c0, c1, c2 of A^-1
  const double cx[4] = {X0 - u, X0 - u, X1 - u, X1 - u};
  const double cy[4] = {Y0 - v, Y1 - v, Y0 - v, Y1 - v};
  double m[4][4], h[4];
  bool flat[4];
  for (int i = 0; i < 4; ++i) {
    const double e1 = (i & 2) ? -1.0 : 1.0, e2 = (i & 1) ? -1.0 : 1.0;
    const double nx = c[0] + e1 * c[3] + e2 * c[6];
    const double ny = c[1] + e1 * c[4] + e2 * c[7];
    const double nz = c[2] + e1 * c[5] + e2 * c[8];
    flat[i] = !(std::fabs(nz) >= 1e-10);
    h[i] = flat[i] ? INFINITY : 1.0 / std::fabs(nz);
    for (int k = 0; k < 4; ++k) m[i][k] = flat[i] ? 0.0 : -(nx * cx[k] + ny * cy[k]) / nz;
  }
  double best = INFINITY;
  for (int i = 0; i < 4; ++i)
    for (int j = 0; j < 4; ++j) {
      if (flat[i] || flat[j]) continue;
      double mx = -INFINITY;
      for (int k = 0; k < 4; ++k) mx = std::max(mx, m[i][k] - m[j][k]);
      best = std::min(best, mx + h[i] + h[j]);
    }
  const double bound = std::max(0.0, best);
  CullTest r{true, false, sigma * bound, -std::log(1.0 - alpha_min)};
  r.keep = r.power >= r.level;
  r.guard = std::fabs(r.power - r.level) <= 1e-9 * r.level;
  return r;
}

}  // namespace

extern "C" {

int orc_version(void) { return 1; }

int orc_num_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}

// Threads of the later parallel regions (n >= 1).
void orc_set_num_threads(int n) {
#ifdef _OPENMP
  omp_set_num_threads(n < 1 ? 1 : n);
#else
  (void)n;
#endif
}

// Real SH basis values (and gradients w.r.t. the direction if dY != NULL) at
// a unit direction d. Y has (deg+1)^2 entries, dY 3 per entry.
void orc_sh_basis(int deg, const double* d, double* Y, double* dY) {
  double dYl[16][3];
  sh_basis(deg, d, Y, dY ? dYl : nullptr);
  if (dY)
    for (int j = 0; j < (deg + 1) * (deg + 1); ++j)
      for (int c = 0; c < 3; ++c) dY[3 * j + c] = dYl[j][c];
}

// Projection of n Gaussians (Listing "XPR-3DGS", project).
//   means [3][n], scales [3][n], quats [4][n], opac [n], sh [K][3][n]
//   cam: R (9, row-major world->camera), t (3), fx, fy, cx, cy
//   cfg: lowpass, alpha_min, z_near, fov_clip
// Outputs (any may be NULL):
//   rec [n][9]: u, v, -0.5*con00, -con01, -0.5*con11, o, r, g, b (shader data)
//   cov [n][3]: a, b, c of the low-passed 2D covariance
//   depth [n], rect [n][4] (x0, y0, x1, y1), tc [n], radius [n], guard [n]
void orc_project(int64_t n, const double* means, const double* scales, const double* quats,
                 const double* opac, const double* sh, int K, const double* camv, int W, int H,
                 const double* cfg, int tile_w, int tile_h, int deg, double* rec, double* cov,
                 double* depth, int32_t* rect, int32_t* tc, int32_t* radius, uint8_t* guard) {
  const Cam cam = read_cam(camv, W, H);
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < n; ++i) {
    Proj P;
    project_one(i, n, means, scales, quats, opac, sh, K, cam, cfg, tile_w, tile_h, deg, P);
    if (rec) {
      double* r = rec + 9 * i;
      r[0] = P.u; r[1] = P.v;
      r[2] = -0.5 * P.con[0]; r[3] = -P.con[1]; r[4] = -0.5 * P.con[2];
      r[5] = opac[i];
      r[6] = P.colour[0]; r[7] = P.colour[1]; r[8] = P.colour[2];
    }
    if (cov) { cov[3 * i] = P.a; cov[3 * i + 1] = P.b; cov[3 * i + 2] = P.c; }
    if (depth) depth[i] = P.tcam[2];
    if (rect) for (int c = 0; c < 4; ++c) rect[4 * i + c] = P.rect[c];
    if (tc) tc[i] = P.tc;
    if (radius) radius[i] = (int32_t)P.radius;
    if (guard) guard[i] = P.guard ? 1 : 0;
  }
}

// Binning (section "Rasterizer"): prefix sum of the tile counts, replicate,
// tile id per replicated entry, sort by (tile id, depth) with ties to the
// lower Gaussian index, per-tile [start, end).
//   depth [n] (sorted on the float32 value of each entry), rect [n][4], tc [n]
//   offsets [n] (exclusive prefix sum of tc, may be NULL)
//   keys [cap]: tile << 32 | float32 bits of depth (may be NULL)
//   vals [cap]: Gaussian index, ranges [tiles_x*tiles_y][2]
// With cull_rec [n][rec_stride] (shader data, may be NULL) every replicated pair
// also goes through tile_cull (Listing "XPR-3DGS") and a culled pair gets
// the sentinel tile id tiles_x*tiles_y, so it sorts after every real tile
// and belongs to no range; *n_kept counts the pairs not culled, *n_guard the
// pairs whose decision is in the guard band, pair_guard [cap] (may be NULL)
// flags them in sorted order. W, H, tile_w, tile_h and alpha_min are only
// read with cull_rec; rec_stride is 9 (3DGS), 21 (3DGUT, whose cull uses
// tile bounds extended by ext = 1) or 17 (LinPrim, the chord bound).
// Returns I = sum tc; writes the lists only when I <= cap.
int64_t orc_bin(int64_t n, const double* depth, const int32_t* rect, const int32_t* tc,
                int tiles_x, int tiles_y, int64_t cap, int64_t* offsets, uint64_t* keys,
                int32_t* vals, int32_t* ranges, const double* cull_rec, int rec_stride, int ext,
                int W, int H, int tile_w, int tile_h, double alpha_min, int64_t* n_kept,
                int64_t* n_guard, uint8_t* pair_guard) {
  std::vector<int64_t> off(n + 1, 0);
  for (int64_t i = 0; i < n; ++i) off[i + 1] = off[i] + tc[i];
  const int64_t I = off[n];
  if (offsets) for (int64_t i = 0; i < n; ++i) offsets[i] = off[i];
  if (I > cap) return I;
  const uint32_t sentinel = (uint32_t)tiles_x * (uint32_t)tiles_y;
  struct Pair { uint32_t tile; float depth; int32_t idx; uint8_t guard; };
  std::vector<Pair> pairs(I);
#pragma omp parallel for schedule(dynamic, 1024)
  for (int64_t i = 0; i < n; ++i) {
    const int x0 = rect[4 * i], y0 = rect[4 * i + 1], x1 = rect[4 * i + 2];
    const int w = x1 - x0;
    for (int64_t r = 0; r < tc[i]; ++r) {
      const int x = x0 + (int)(r % w);
      const int y = y0 + (int)(r / w);
      uint32_t tile = (uint32_t)(y * tiles_x + x);
      uint8_t g = 0;
      if (cull_rec) {
        const double* cr = cull_rec + (int64_t)rec_stride * i;
        const CullTest t = rec_stride == 17
                               ? lin_cull_one(cr, x, y, W, H, tile_w, tile_h, alpha_min)
                               : tile_cull_one(cr, x, y, W, H, tile_w, tile_h, alpha_min, ext);
        if (!t.keep) tile = sentinel;
        g = t.guard ? 1 : 0;
      }
      pairs[off[i] + r] = Pair{tile, (float)depth[i], (int32_t)i, g};
    }
  }
  auto less = [](const Pair& p, const Pair& q) {
    if (p.tile != q.tile) return p.tile < q.tile;
    if (p.depth != q.depth) return p.depth < q.depth;
    return p.idx < q.idx;
  };
#ifdef _OPENMP
  __gnu_parallel::sort(pairs.begin(), pairs.end(), less);
#else
  std::sort(pairs.begin(), pairs.end(), less);
#endif
  const int64_t T = (int64_t)tiles_x * tiles_y;
  for (int64_t t = 0; t < 2 * T; ++t) ranges[t] = 0;
  int64_t kept = 0, guards = 0;
  for (int64_t k = 0; k < I; ++k) {
    const Pair& p = pairs[k];
    if (keys) {
      uint32_t bits;
      std::memcpy(&bits, &p.depth, 4);
      keys[k] = ((uint64_t)p.tile << 32) | bits;
    }
    vals[k] = p.idx;
    if (pair_guard) pair_guard[k] = p.guard;
    guards += p.guard;
    if (p.tile == sentinel) continue;
    ++kept;
    if (k == 0 || pairs[k - 1].tile != p.tile) ranges[2 * p.tile] = (int32_t)k;
    if (k == I - 1 || pairs[k + 1].tile != p.tile) ranges[2 * p.tile + 1] = (int32_t)(k + 1);
  }
  if (n_kept) *n_kept = kept;
  if (n_guard) *n_guard = guards;
  return I;
}

// tile_cull of m (primitive, tile) pairs: rec [m][rec_stride] shader data
// (9: 3DGS/3DGUT cull columns, 17: LinPrim), txy [m][2] tile coordinates,
// ext the tile-bound extension (0 for 3DGS, 1 for 3DGUT); keep, power
// (3DGS: smallest 0.5 q over the tile, level log(o / alpha_min); LinPrim:
// sigma times the chord bound, level -log(1 - alpha_min)) and guard per pair
// (any output may be NULL).
void orc_tile_cull(int64_t m, const double* rec, int rec_stride, const int32_t* txy, int W,
                   int H, int tile_w, int tile_h, double alpha_min, int ext, uint8_t* keep,
                   double* power, double* level, uint8_t* guard) {
  for (int64_t k = 0; k < m; ++k) {
    const double* r = rec + (int64_t)rec_stride * k;
    const CullTest t =
        rec_stride == 17
            ? lin_cull_one(r, txy[2 * k], txy[2 * k + 1], W, H, tile_w, tile_h, alpha_min)
            : tile_cull_one(r, txy[2 * k], txy[2 * k + 1], W, H, tile_w, tile_h, alpha_min, ext);
    if (keep) keep[k] = t.keep ? 1 : 0;
    if (power) power[k] = t.power;
    if (level) level[k] = t.level;
    if (guard) guard[k] = t.guard ? 1 : 0;
  }
}

// Forward compositing (Algorithm 1 with the 3DGS evaluate): for pixel (x, y)
// of tile t, walk the tile's list front to back:
//   P = A dx^2 + B dx dy + C dy^2 with dx = x - u, dy = y - v (shader data)
//   skip if P > 0; alpha = min(alpha_max, o e^P); skip if alpha < alpha_min;
//   stop (without blending) if T (1 - alpha) < t_min; else C += c alpha T,
//   T *= 1 - alpha.
// Output C + T bg.
//
// A decision is in the guard band when its operand lies within the float32
// rounding bound of its threshold, so that a float32 evaluation may take it
// either way. With u = 2^-24 and S the sum of the absolute power terms
// (the power's rounding grows with S, not with |P|: a needle-like conic
// cancels large terms): the P > 0 gate when |P| <= max(1e-6, 2 * 7 S u);
// the alpha gate when |alpha - alpha_min| <= max(1e-4 alpha_min,
// 2 (7 S + 3) u alpha); the stop rule when |T (1 - alpha) - t_min| <=
// max(1e-3, 2 s u) t_min, s the T sensitivity below including this entry.
// For a pixel with such decisions the walk is repeated once per decision
// with that decision alone inverted; the largest change of any colour
// channel (and of T) summed over these walks is the pixel's ambiguous
// contribution.
struct PixelWalk {
  double C[3], T;
  int32_t last, count, neval, nguard;
  double tsens;  // sum over blended entries of alpha/(1-alpha) (7 S + 3) + 2
};

// flip: ordinal of the guard decision to invert (-1: none).
static PixelWalk walk_pixel(int px, int py, const double* rec, const int32_t* vals, int32_t start,
                     int32_t end, double alpha_min, double alpha_max, double t_min, int flip) {
  PixelWalk w{{0, 0, 0}, 1.0, 0, 0, 0, 0, 1.0};
  auto decide = [&](bool near, bool value) {
    if (!near) return value;
    return (w.nguard++ == flip) ? !value : value;
  };
  w.neval = end - start;
  for (int32_t k = start; k < end; ++k) {
    const double* r = rec + 9 * (int64_t)vals[k];
    const double dx = px - r[0], dy = py - r[1];
    const double t0 = r[2] * dx * dx, t1 = r[3] * dx * dy, t2 = r[4] * dy * dy;
    const double P = t0 + t1 + t2;
    const double S = std::fabs(t0) + std::fabs(t1) + std::fabs(t2);
    const double u = 0x1p-24;
    if (decide(std::fabs(P) <= std::max(1e-6, 14.0 * S * u), P > 0)) continue;
    const double raw = r[5] * std::exp(P);
    const double alpha = std::min(alpha_max, raw);
    if (decide(std::fabs(alpha - alpha_min) <=
                   std::max(1e-4 * alpha_min, 2.0 * (7.0 * S + 3.0) * u * alpha),
               alpha < alpha_min))
      continue;
    // Sensitivity of T to float32 evaluation (in units of u): alpha carries
    // a relative error of at most about 7u S plus 3u (the roundings of dx,
    // dy, the products and sums of the power, exp and the opacity product),
    // amplified by alpha / (1 - alpha) in 1 - alpha; the update of T adds
    // two roundings. A clamped alpha is the constant alpha_max.
    const double sens =
        w.tsens + (raw >= alpha_max ? 0.0 : alpha / (1.0 - alpha) * (7.0 * S + 3.0)) + 2.0;
    const double Tn = w.T * (1.0 - alpha);
    if (decide(std::fabs(Tn - t_min) <= std::max(1e-3, 2.0 * sens * u) * t_min, Tn < t_min)) {
      w.neval = k - start + 1;
      break;
    }
    for (int c = 0; c < 3; ++c) w.C[c] += r[6 + c] * alpha * w.T;
    w.tsens = sens;
    w.T = Tn;
    w.last = k - start + 1;
    ++w.count;
  }
  return w;
}

// rec [n][9], vals, ranges as produced by orc_bin
// cfg: alpha_min, alpha_max, t_min, bg0, bg1, bg2
// Outputs (all but img may be NULL):
//   img [3][H][W], Tfinal [H][W], ncontrib [H][W] (1-based position of the
//   last blended entry, 0 if none), nblend [H][W] (number blended),
//   guard [H][W] (1 where a decision sits within the guard band),
//   neval [H][W] (list entries the pixel evaluates: the position of the
//   entry that stops it, else the list length),
//   tsens [H][W] (the sensitivity above, in units of 2^-24),
//   amb [2][H][W] (ambiguous contribution: colour, then T; 0 off the guard
//   band).
void orc_render_fwd(int W, int H, int tile_w, int tile_h, const double* rec, const int32_t* vals,
                    const int32_t* ranges, const double* cfg, double* img, double* Tfinal,
                    int32_t* ncontrib, int32_t* nblend, uint8_t* guard, int32_t* neval,
                    double* tsens, double* amb) {
  const double alpha_min = cfg[0], alpha_max = cfg[1], t_min = cfg[2];
  const double bg[3] = {cfg[3], cfg[4], cfg[5]};
  const int tiles_x = (W + tile_w - 1) / tile_w;
  const int tiles_y = (H + tile_h - 1) / tile_h;
  const int64_t WH = (int64_t)W * H;
#pragma omp parallel for schedule(dynamic, 1)
  for (int t = 0; t < tiles_x * tiles_y; ++t) {
    const int tx = t % tiles_x, ty = t / tiles_x;
    const int32_t start = ranges[2 * t], end = ranges[2 * t + 1];
    for (int py = ty * tile_h; py < std::min(H, (ty + 1) * tile_h); ++py)
      for (int px = tx * tile_w; px < std::min(W, (tx + 1) * tile_w); ++px) {
        const PixelWalk w =
            walk_pixel(px, py, rec, vals, start, end, alpha_min, alpha_max, t_min, -1);
        const int64_t p = (int64_t)py * W + px;
        for (int c = 0; c < 3; ++c) img[(int64_t)c * WH + p] = w.C[c] + w.T * bg[c];
        if (Tfinal) Tfinal[p] = w.T;
        if (ncontrib) ncontrib[p] = w.last;
        if (nblend) nblend[p] = w.count;
        if (guard) guard[p] = w.nguard > 0 ? 1 : 0;
        if (neval) neval[p] = w.neval;
        if (tsens) tsens[p] = w.tsens;
        if (amb) {
          double ac = 0.0, at = 0.0;
          for (int f = 0; f < w.nguard; ++f) {
            const PixelWalk v =
                walk_pixel(px, py, rec, vals, start, end, alpha_min, alpha_max, t_min, f);
            double d = 0.0;
            for (int c = 0; c < 3; ++c)
              d = std::max(d, std::fabs((v.C[c] + v.T * bg[c]) - (w.C[c] + w.T * bg[c])));
            ac += d;
            at += std::fabs(v.T - w.T);
          }
          amb[p] = ac;
          amb[WH + p] = at;
        }
      }
  }
}

// 3DGUT projection of n Gaussians (Listing "XPR-3DGUT", project).
//   cfg: lowpass, alpha_min, z_near, opacity_extents (0/1)
// Outputs (any may be NULL): rec [n][21] = u, v, A, B, C, o', r, g, b
// (2D cull data and colour, laid out like the 3DGS shader data), ro (3),
// M (9, row-major); cov [n][3]; depth [n]; rect [n][4]; tc [n]; guard [n].
void orc_project_gut(int64_t n, const double* means, const double* scales, const double* quats,
                     const double* opac, const double* sh, const double* camv, int W, int H,
                     const double* cfg, int tile_w, int tile_h, int deg, double* rec, double* cov,
                     double* depth, int32_t* rect, int32_t* tc, uint8_t* guard) {
  const Cam cam = read_cam(camv, W, H);
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < n; ++i) {
    GutProj G;
    project_gut_one(i, n, means, scales, quats, opac, sh, cam, cfg, tile_w, tile_h, deg, G);
    if (rec) {
      double* r = rec + 21 * i;
      const double v9[9] = {G.u, G.v, G.A, G.B, G.C, G.o, G.colour[0], G.colour[1], G.colour[2]};
      for (int c = 0; c < 9; ++c) r[c] = v9[c];
      for (int c = 0; c < 3; ++c) r[9 + c] = G.ro[c];
      for (int c = 0; c < 9; ++c) r[12 + c] = G.M[c];
    }
    if (cov) { cov[3 * i] = G.a; cov[3 * i + 1] = G.b; cov[3 * i + 2] = G.c; }
    if (depth) depth[i] = G.depth;
    if (rect) for (int c = 0; c < 4; ++c) rect[4 * i + c] = G.rect[c];
    if (tc) tc[i] = G.tc;
    if (guard) guard[i] = G.guard ? 1 : 0;
  }
}

// 3DGUT forward compositing (Algorithm 1 with the 3DGUT pixel_info and
// evaluate): per pixel the ray direction rd; per listed record the response
// along the ray, alpha = o' response, skipped unless response > 0.0113
// (the listing's validity threshold) and, as for 3DGS, alpha =
// min(alpha_max, alpha) >= alpha_min; same stop rule and blending.
//   rec [n][21], vals / ranges from orc_bin, camv the camera (pixel_info)
//   cfg: alpha_min, alpha_max, t_min, bg0, bg1, bg2; outputs as orc_render_fwd
void orc_render_fwd_gut(int W, int H, int tile_w, int tile_h, const double* rec,
                        const int32_t* vals, const int32_t* ranges, const double* camv,
                        const double* cfg, double* img, double* Tfinal, int32_t* ncontrib,
                        int32_t* nblend, uint8_t* guard, int32_t* neval) {
  const Cam cam = read_cam(camv, W, H);
  const double alpha_min = cfg[0], alpha_max = cfg[1], t_min = cfg[2];
  const double bg[3] = {cfg[3], cfg[4], cfg[5]};
  const double valid_min = 0.0113;
  const int tiles_x = (W + tile_w - 1) / tile_w;
  const int tiles_y = (H + tile_h - 1) / tile_h;
#pragma omp parallel for schedule(dynamic, 1)
  for (int t = 0; t < tiles_x * tiles_y; ++t) {
    const int tx = t % tiles_x, ty = t / tiles_x;
    const int32_t start = ranges[2 * t], end = ranges[2 * t + 1];
    for (int py = ty * tile_h; py < std::min(H, (ty + 1) * tile_h); ++py)
      for (int px = tx * tile_w; px < std::min(W, (tx + 1) * tile_w); ++px) {
        double rd[3];
        gut_ray(cam, px, py, rd);
        double T = 1.0, C[3] = {0, 0, 0};
        int32_t last = 0, count = 0, ne = end - start;
        bool g = false;
        for (int32_t k = start; k < end; ++k) {
          const double* r = rec + 21 * (int64_t)vals[k];
          const double resp = gut_response(r + 9, r + 12, rd);
          if (std::fabs(resp - valid_min) <= 1e-6 * valid_min) g = true;
          if (!(resp > valid_min)) continue;
          const double alpha = std::min(alpha_max, r[5] * resp);
          if (std::fabs(alpha - alpha_min) <= 1e-4 * alpha_min) g = true;
          if (alpha < alpha_min) continue;
          const double Tn = T * (1.0 - alpha);
          if (std::fabs(Tn - t_min) <= 1e-3 * t_min) g = true;
          if (Tn < t_min) {
            ne = k - start + 1;
            break;
          }
          for (int c = 0; c < 3; ++c) C[c] += r[6 + c] * alpha * T;
          T = Tn;
          last = k - start + 1;
          ++count;
        }
        const int64_t p = (int64_t)py * W + px;
        for (int c = 0; c < 3; ++c) img[(int64_t)c * W * H + p] = C[c] + T * bg[c];
        if (Tfinal) Tfinal[p] = T;
        if (ncontrib) ncontrib[p] = last;
        if (nblend) nblend[p] = count;
        if (guard) guard[p] = g ? 1 : 0;
        if (neval) neval[p] = ne;
      }
  }
}

// The 3DGUT response along the ray through pixel (px, py) for m records
// rec [m][21] (one pixel per record): out [m].
void orc_gut_response(int64_t m, const double* rec, const int32_t* pxy, const double* camv,
                      int W, int H, double* out) {
  const Cam cam = read_cam(camv, W, H);
  for (int64_t k = 0; k < m; ++k) {
    double rd[3];
    gut_ray(cam, pxy[2 * k], pxy[2 * k + 1], rd);
    out[k] = gut_response(rec + 21 * k + 9, rec + 21 * k + 12, rd);
  }
}

// LinPrim projection of n octahedra (Listing "XPR-LinPrim", project).
//   cfg: lowpass (unused), alpha_min, z_near, unused
// rec [n][17] = u, v (mu_2D - 1/2), sigma, r, g, b, ex, ey, c0 (3), c1 (3),
// c2 (3); depth [n] (Euclidean); rect [n][4]; tc [n]; guard [n].
void orc_project_lin(int64_t n, const double* means, const double* scales, const double* quats,
                     const double* opac, const double* sh, const double* camv, int W, int H,
                     const double* cfg, int tile_w, int tile_h, int deg, double* rec,
                     double* depth, int32_t* rect, int32_t* tc, uint8_t* guard) {
  const Cam cam = read_cam(camv, W, H);
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < n; ++i) {
    LinProj L;
    project_lin_one(i, n, means, scales, quats, opac, sh, cam, cfg, tile_w, tile_h, deg, L);
    if (rec) {
      double* r = rec + 17 * i;
      const double v8[8] = {L.u2 - 0.5, L.v2 - 0.5, L.sigma, L.colour[0], L.colour[1],
                            L.colour[2], L.ex, L.ey};
      for (int k = 0; k < 8; ++k) r[k] = v8[k];
      for (int k = 0; k < 9; ++k) r[8 + k] = L.c[k];
    }
    if (depth) depth[i] = L.depth;
    if (rect) for (int k = 0; k < 4; ++k) rect[4 * i + k] = L.rect[k];
    if (tc) tc[i] = L.tc;
    if (guard) guard[i] = L.guard ? 1 : 0;
  }
}

// Chord lengths for m (record, pixel) pairs: rec [m][17], pxy [m][2].
void orc_lin_chord(int64_t m, const double* rec, const int32_t* pxy, double* out) {
  for (int64_t k = 0; k < m; ++k) {
    const double* r = rec + 17 * k;
    // pixel centre px + 1/2 minus mu_2D = px - u with u = mu_2D - 1/2
    out[k] = lin_chord(r + 8, pxy[2 * k] - r[0], pxy[2 * k + 1] - r[1]);
  }
}

// LinPrim forward compositing (Algorithm 1 with the XPR-LinPrim evaluate):
// per listed record alpha = 1 - exp(-sigma chord) for a positive chord
// (valid always), then alpha = min(alpha_max, alpha) >= alpha_min, the stop
// rule and blending of the 3DGS path.
void orc_render_fwd_lin(int W, int H, int tile_w, int tile_h, const double* rec,
                        const int32_t* vals, const int32_t* ranges, const double* cfg,
                        double* img, double* Tfinal, int32_t* ncontrib, int32_t* nblend,
                        uint8_t* guard, int32_t* neval) {
  const double alpha_min = cfg[0], alpha_max = cfg[1], t_min = cfg[2];
  const double bg[3] = {cfg[3], cfg[4], cfg[5]};
  const int tiles_x = (W + tile_w - 1) / tile_w;
  const int tiles_y = (H + tile_h - 1) / tile_h;
#pragma omp parallel for schedule(dynamic, 1)
  for (int t = 0; t < tiles_x * tiles_y; ++t) {
    const int tx = t % tiles_x, ty = t / tiles_x;
    const int32_t start = ranges[2 * t], end = ranges[2 * t + 1];
    for (int py = ty * tile_h; py < std::min(H, (ty + 1) * tile_h); ++py)
      for (int px = tx * tile_w; px < std::min(W, (tx + 1) * tile_w); ++px) {
        double T = 1.0, C[3] = {0, 0, 0};
        int32_t last = 0, count = 0, ne = end - start;
        bool g = false;
        for (int32_t k = start; k < end; ++k) {
          const double* r = rec + 17 * (int64_t)vals[k];
          const double ch = lin_chord(r + 8, px - r[0], py - r[1]);
          if (!(ch > 0.0)) continue;
          const double alpha = std::min(alpha_max, -std::expm1(-r[2] * ch));
          if (std::fabs(alpha - alpha_min) <= 1e-4 * alpha_min) g = true;
          if (alpha < alpha_min) continue;
          const double Tn = T * (1.0 - alpha);
          if (std::fabs(Tn - t_min) <= 1e-3 * t_min) g = true;
          if (Tn < t_min) {
            ne = k - start + 1;
            break;
          }
          for (int c = 0; c < 3; ++c) C[c] += r[3 + c] * alpha * T;
          T = Tn;
          last = k - start + 1;
          ++count;
        }
        const int64_t p = (int64_t)py * W + px;
        for (int c = 0; c < 3; ++c) img[(int64_t)c * W * H + p] = C[c] + T * bg[c];
        if (Tfinal) Tfinal[p] = T;
        if (ncontrib) ncontrib[p] = last;
        if (nblend) nblend[p] = count;
        if (guard) guard[p] = g ? 1 : 0;
        if (neval) neval[p] = ne;
      }
  }
}

// Backward of the compositing: given dL/dimg [3][H][W], the derivative of
// L with respect to each Gaussian's shader data, summed over pixels:
//   grad [n][9] = dL/d(u, v, A, B, C, o, r, g, b), A = -0.5 con00,
//   B = -con01, C = -0.5 con11.
// Each pixel re-runs its forward walk and then differentiates
//   C = sum_i c_i a_i T_i + T_final bg, T_i = prod_{j<i} (1 - a_j)
// in reverse order. grad is overwritten.
void orc_render_bwd(int W, int H, int tile_w, int tile_h, int64_t n, const double* rec,
                    const int32_t* vals, const int32_t* ranges, const double* cfg,
                    const double* dimg, double* grad) {
  const double alpha_min = cfg[0], alpha_max = cfg[1], t_min = cfg[2];
  const double bg[3] = {cfg[3], cfg[4], cfg[5]};
  const int tiles_x = (W + tile_w - 1) / tile_w;
  const int tiles_y = (H + tile_h - 1) / tile_h;
  int nthreads = 1;
#ifdef _OPENMP
  nthreads = omp_get_max_threads();
#endif
  std::vector<std::vector<double>> part(nthreads);
#pragma omp parallel
  {
    int tid = 0;
#ifdef _OPENMP
    tid = omp_get_thread_num();
#endif
    std::vector<double>& acc = part[tid];
    acc.assign((size_t)n * 9, 0.0);
    struct Step { int64_t g; double alpha, T, eP, dx, dy; bool clamped; };
    std::vector<Step> steps;
#pragma omp for schedule(dynamic, 1)
    for (int t = 0; t < tiles_x * tiles_y; ++t) {
      const int tx = t % tiles_x, ty = t / tiles_x;
      const int32_t start = ranges[2 * t], end = ranges[2 * t + 1];
      for (int py = ty * tile_h; py < std::min(H, (ty + 1) * tile_h); ++py)
        for (int px = tx * tile_w; px < std::min(W, (tx + 1) * tile_w); ++px) {
          steps.clear();
          double T = 1.0;
          for (int32_t k = start; k < end; ++k) {
            const int64_t gi = vals[k];
            const double* r = rec + 9 * gi;
            const double dx = px - r[0], dy = py - r[1];
            const double P = r[2] * dx * dx + r[3] * dx * dy + r[4] * dy * dy;
            if (P > 0) continue;
            const double eP = std::exp(P);
            const double raw = r[5] * eP;
            const double alpha = std::min(alpha_max, raw);
            if (alpha < alpha_min) continue;
            const double Tn = T * (1.0 - alpha);
            if (Tn < t_min) break;
            steps.push_back(Step{gi, alpha, T, eP, dx, dy, raw > alpha_max});
            T = Tn;
          }
          const double Tfin = T;
          const int64_t p = (int64_t)py * W + px;
          const double G[3] = {dimg[p], dimg[(int64_t)W * H + p], dimg[2 * (int64_t)W * H + p]};
          const double bgG = bg[0] * G[0] + bg[1] * G[1] + bg[2] * G[2];
          double S[3] = {0, 0, 0};  // colour behind, normalised by the transmittance
          for (int s = (int)steps.size() - 1; s >= 0; --s) {
            const Step& st = steps[s];
            const double* r = rec + 9 * st.g;
            double* ga = acc.data() + 9 * st.g;
            double dalpha = 0;
            for (int c = 0; c < 3; ++c) {
              ga[6 + c] += st.alpha * st.T * G[c];
              dalpha += st.T * (r[6 + c] - S[c]) * G[c];
            }
            dalpha -= Tfin * bgG / (1.0 - st.alpha);
            for (int c = 0; c < 3; ++c) S[c] = st.alpha * r[6 + c] + (1.0 - st.alpha) * S[c];
            if (st.clamped) continue;
            const double dP = st.alpha * dalpha;   // alpha = o e^P
            ga[5] += st.eP * dalpha;
            const double A = r[2], B = r[3], Cc = r[4];
            ga[0] += dP * (-(2 * A * st.dx + B * st.dy));
            ga[1] += dP * (-(2 * Cc * st.dy + B * st.dx));
            ga[2] += dP * st.dx * st.dx;
            ga[3] += dP * st.dx * st.dy;
            ga[4] += dP * st.dy * st.dy;
          }
        }
    }
  }
  for (int64_t k = 0; k < n * 9; ++k) {
    double s = 0;
    for (int th = 0; th < nthreads; ++th)
      if (!part[th].empty()) s += part[th][k];
    grad[k] = s;
  }
}

// Backward of the projection: from dL/d(shader data) [n][9] to the gradient
// of L with respect to the inputs (activated scales and opacity, raw
// quaternion). Outputs are [k][n] like the inputs and are overwritten.
void orc_project_bwd(int64_t n, const double* means, const double* scales, const double* quats,
                     const double* opac, const double* sh, int K, const double* camv, int W, int H,
                     const double* cfg, int tile_w, int tile_h, int deg, const double* grad,
                     double* g_means, double* g_scales, double* g_quats, double* g_opac,
                     double* g_sh) {
  const Cam cam = read_cam(camv, W, H);
  const int nb = (deg + 1) * (deg + 1);
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < n; ++i) {
    for (int c = 0; c < 3; ++c) { g_means[c * n + i] = 0; g_scales[c * n + i] = 0; }
    for (int c = 0; c < 4; ++c) g_quats[c * n + i] = 0;
    g_opac[i] = 0;
    for (int j = 0; j < K; ++j)
      for (int ch = 0; ch < 3; ++ch) g_sh[(int64_t)(j * 3 + ch) * n + i] = 0;
    Proj P;
    project_one(i, n, means, scales, quats, opac, sh, K, cam, cfg, tile_w, tile_h, deg, P);
    if (!P.visible) continue;
    const double* g = grad + 9 * i;
    double gmu[3] = {0, 0, 0};

    // Colour: colour = max(0, 0.5 + sum_j sh_j Y_j(dir)), dir = (mu - campos)/|.|
    double Y[16], dY[16][3];
    sh_basis(deg, P.dir, Y, dY);
    double graw[3];
    for (int ch = 0; ch < 3; ++ch) graw[ch] = P.raw[ch] > 0 ? g[6 + ch] : 0.0;
    double gdir[3] = {0, 0, 0};
    for (int j = 0; j < nb; ++j)
      for (int ch = 0; ch < 3; ++ch) {
        g_sh[(int64_t)(j * 3 + ch) * n + i] = Y[j] * graw[ch];
        const double w = sh[(int64_t)(j * 3 + ch) * n + i] * graw[ch];
        for (int c = 0; c < 3; ++c) gdir[c] += w * dY[j][c];
      }
    const double dd = P.dir[0] * gdir[0] + P.dir[1] * gdir[1] + P.dir[2] * gdir[2];
    for (int c = 0; c < 3; ++c) gmu[c] += (gdir[c] - P.dir[c] * dd) / P.dirnorm;

    // Opacity.
    g_opac[i] = g[5];

    // Conic entries from the shader data A = -0.5 con00, B = -con01, C = -0.5 con11.
    const double gk00 = -0.5 * g[2], gk01 = -g[3], gk11 = -0.5 * g[4];
    // con00 = c/det, con01 = -b/det, con11 = a/det, det = a c - b^2.
    const double a = P.a, b = P.b, c = P.c, d2 = P.det * P.det;
    const double ga = gk00 * (-c * c / d2) + gk01 * (b * c / d2) + gk11 * (-b * b / d2);
    const double gb = gk00 * (2 * b * c / d2) + gk01 * (-(a * c + b * b) / d2) + gk11 * (2 * a * b / d2);
    const double gc = gk00 * (-b * b / d2) + gk01 * (a * b / d2) + gk11 * (-a * a / d2);

    // cov2D entries a = T0 Sigma T0^T, b = T0 Sigma T1^T, c = T1 Sigma T1^T.
    const double* T0 = P.T;
    const double* T1 = P.T + 3;
    double gSigma[9];
    for (int r = 0; r < 3; ++r)
      for (int s = 0; s < 3; ++s)
        gSigma[3 * r + s] = ga * T0[r] * T0[s] + gb * T0[r] * T1[s] + gc * T1[r] * T1[s];
    double ST0[3], ST1[3];
    for (int r = 0; r < 3; ++r) {
      ST0[r] = P.Sigma[3 * r] * T0[0] + P.Sigma[3 * r + 1] * T0[1] + P.Sigma[3 * r + 2] * T0[2];
      ST1[r] = P.Sigma[3 * r] * T1[0] + P.Sigma[3 * r + 1] * T1[1] + P.Sigma[3 * r + 2] * T1[2];
    }
    double gT[6];
    for (int r = 0; r < 3; ++r) {
      gT[r] = 2 * ga * ST0[r] + gb * ST1[r];
      gT[3 + r] = gb * ST0[r] + 2 * gc * ST1[r];
    }
    // T = J W  ->  dL/dJ = dL/dT W^T
    double gJ[6];
    for (int r = 0; r < 2; ++r)
      for (int s = 0; s < 3; ++s)
        gJ[3 * r + s] = gT[3 * r] * cam.R[3 * s] + gT[3 * r + 1] * cam.R[3 * s + 1] +
                        gT[3 * r + 2] * cam.R[3 * s + 2];
    // J00 = fx/tz, J02 = -fx rho_x/tz, J11 = fy/tz, J12 = -fy rho_y/tz
    const double tx = P.tcam[0], ty = P.tcam[1], tz = P.tcam[2];
    double gt[3] = {0, 0, 0};
    gt[2] += gJ[0] * (-cam.fx / (tz * tz)) + gJ[2] * (cam.fx * P.rho[0] / (tz * tz)) +
             gJ[4] * (-cam.fy / (tz * tz)) + gJ[5] * (cam.fy * P.rho[1] / (tz * tz));
    const double grx = gJ[2] * (-cam.fx / tz), gry = gJ[5] * (-cam.fy / tz);
    if (!P.clampx) { gt[0] += grx / tz; gt[2] += grx * (-tx / (tz * tz)); }
    if (!P.clampy) { gt[1] += gry / tz; gt[2] += gry * (-ty / (tz * tz)); }
    // mean2D
    gt[0] += g[0] * cam.fx / tz;
    gt[2] += g[0] * (-cam.fx * tx / (tz * tz));
    gt[1] += g[1] * cam.fy / tz;
    gt[2] += g[1] * (-cam.fy * ty / (tz * tz));
    // t = W mu + t_w
    for (int c = 0; c < 3; ++c)
      gmu[c] += cam.R[c] * gt[0] + cam.R[3 + c] * gt[1] + cam.R[6 + c] * gt[2];
    for (int c = 0; c < 3; ++c) g_means[c * n + i] = gmu[c];

    // Sigma = M M^T, M = Rq S:  dL/dM = (G + G^T) M
    double M[9];
    for (int r = 0; r < 3; ++r)
      for (int s = 0; s < 3; ++s) M[3 * r + s] = P.Rq[3 * r + s] * P.s[s];
    double gM[9];
    for (int r = 0; r < 3; ++r)
      for (int s = 0; s < 3; ++s) {
        double acc = 0;
        for (int k = 0; k < 3; ++k) acc += (gSigma[3 * r + k] + gSigma[3 * k + r]) * M[3 * k + s];
        gM[3 * r + s] = acc;
      }
    double gR[9];
    for (int s = 0; s < 3; ++s) {
      double acc = 0;
      for (int r = 0; r < 3; ++r) {
        acc += gM[3 * r + s] * P.Rq[3 * r + s];
        gR[3 * r + s] = gM[3 * r + s] * P.s[s];
      }
      g_scales[s * n + i] = acc;
    }
    double dR[9][4];
    quat_to_rot_jac(P.qn, dR);
    double gqn[4] = {0, 0, 0, 0};
    for (int k = 0; k < 9; ++k)
      for (int c = 0; c < 4; ++c) gqn[c] += gR[k] * dR[k][c];
    const double qd = P.qn[0] * gqn[0] + P.qn[1] * gqn[1] + P.qn[2] * gqn[2] + P.qn[3] * gqn[3];
    for (int c = 0; c < 4; ++c) g_quats[c * n + i] = (gqn[c] - P.qn[c] * qd) / P.qnorm;
  }
}


// ----------------------------------------------------------------------------
// 3DGUT backward. The forward (Listing XPR-3DGUT: the unscented-transform
// project, pixel_info and evaluate, blended by Algorithm 1) differentiated
// by hand, as the paper obtains it by automatic differentiation (section Key
// Interfaces). The shader data's derivative is taken with respect to the 16
// values the evaluation reads: the adjusted opacity o', the colour (3), the
// canonical ray origin ro (3) and M = S^-1 R^T (9, row-major); the 2D mean
// and conic of the record only place the rect, which is piecewise constant.
// The derivative with respect to M holds the Gaussian's centre fixed, i.e.
// ro = M d moves with M for d = M^-1 ro (the camera position minus the
// centre): dL/dM|centre = dL/dM|ro + dL/dro d^T. The two terms on the right
// are each about |d| / |x| times larger than their sum (x below), so
// forming the sum per pixel in float64 keeps the scale and rotation
// gradients that follow from it well conditioned when the per-record sums
// are stored in float32.
// ----------------------------------------------------------------------------

// dL/d(o', r, g, b, ro, M|centre) per record [n][16] from dL/dimage
// [3][H][W]: per pixel the blended entries are found front to back (as in
// orc_render_fwd_gut), then walked back with the colour behind S, as in
// orc_render_bwd. With resp = exp(-d2 / 2), d2 = |p|^2 for p = ro - t w,
// w = M rd (rd the pixel's world ray) and t = (ro . w) / |w|^2 (p is the
// canonical offset of the ray's closest point from the centre, and t is
// stationary there): dL/do' = resp dL/dalpha, dL/dd2 = -resp o' dL/dalpha
// / 2, dd2/dro = 2 p, and with the centre fixed p = M x for the world
// offset x = d - t rd of the closest point, so dd2/dM = 2 p x^T.
void orc_render_bwd_gut(int W, int H, int tile_w, int tile_h, int64_t n, const double* rec,
                        const int32_t* vals, const int32_t* ranges, const double* camv,
                        const double* cfg, const double* dimg, double* grad) {
  const Cam cam = read_cam(camv, W, H);
  const double alpha_min = cfg[0], alpha_max = cfg[1], t_min = cfg[2];
  const double bg[3] = {cfg[3], cfg[4], cfg[5]};
  const double valid_min = 0.0113;
  const int tiles_x = (W + tile_w - 1) / tile_w;
  const int tiles_y = (H + tile_h - 1) / tile_h;
  int nthreads = 1;
#ifdef _OPENMP
  nthreads = omp_get_max_threads();
#endif
  std::vector<std::vector<double>> part(nthreads);
#pragma omp parallel
  {
    int tid = 0;
#ifdef _OPENMP
    tid = omp_get_thread_num();
#endif
    std::vector<double>& acc = part[tid];
    acc.assign((size_t)n * 16, 0.0);
    struct Step { int64_t g; double alpha, T, resp; bool clamped; };
    std::vector<Step> steps;
#pragma omp for schedule(dynamic, 1)
    for (int t = 0; t < tiles_x * tiles_y; ++t) {
      const int tx = t % tiles_x, ty = t / tiles_x;
      const int32_t start = ranges[2 * t], end = ranges[2 * t + 1];
      for (int py = ty * tile_h; py < std::min(H, (ty + 1) * tile_h); ++py)
        for (int px = tx * tile_w; px < std::min(W, (tx + 1) * tile_w); ++px) {
          double rd[3];
          gut_ray(cam, px, py, rd);
          steps.clear();
          double T = 1.0;
          for (int32_t k = start; k < end; ++k) {
            const int64_t gi = vals[k];
            const double* r = rec + 21 * gi;
            const double resp = gut_response(r + 9, r + 12, rd);
            if (!(resp > valid_min)) continue;
            const double raw = r[5] * resp;
            const double alpha = std::min(alpha_max, raw);
            if (alpha < alpha_min) continue;
            const double Tn = T * (1.0 - alpha);
            if (Tn < t_min) break;
            steps.push_back(Step{gi, alpha, T, resp, raw > alpha_max});
            T = Tn;
          }
          const double Tfin = T;
          const int64_t p = (int64_t)py * W + px;
          const double G[3] = {dimg[p], dimg[(int64_t)W * H + p], dimg[2 * (int64_t)W * H + p]};
          const double bgG = bg[0] * G[0] + bg[1] * G[1] + bg[2] * G[2];
          double S[3] = {0, 0, 0};
          for (int si = (int)steps.size() - 1; si >= 0; --si) {
            const Step& st = steps[si];
            const double* r = rec + 21 * st.g;
            double* ga = acc.data() + 16 * st.g;
            double dalpha = 0;
            for (int c = 0; c < 3; ++c) {
              ga[1 + c] += st.alpha * st.T * G[c];
              dalpha += st.T * (r[6 + c] - S[c]) * G[c];
            }
            dalpha -= Tfin * bgG / (1.0 - st.alpha);
            for (int c = 0; c < 3; ++c) S[c] = st.alpha * r[6 + c] + (1.0 - st.alpha) * S[c];
            if (st.clamped) continue;
            ga[0] += st.resp * dalpha;
            const double dd2 = -0.5 * st.resp * r[5] * dalpha;
            const double* ro = r + 9;
            const double* M = r + 12;
            double w[3], Minv[9], d[3], x[3], pv[3];
            for (int a = 0; a < 3; ++a) w[a] = M[3 * a] * rd[0] + M[3 * a + 1] * rd[1] + M[3 * a + 2] * rd[2];
            const double rw = ro[0] * w[0] + ro[1] * w[1] + ro[2] * w[2];
            const double ww = w[0] * w[0] + w[1] * w[1] + w[2] * w[2];
            const double t = rw / ww;
            if (!inv3(M, Minv)) continue;  // not reached: a blended record has M invertible
            for (int a = 0; a < 3; ++a) d[a] = Minv[3 * a] * ro[0] + Minv[3 * a + 1] * ro[1] + Minv[3 * a + 2] * ro[2];
            for (int a = 0; a < 3; ++a) x[a] = d[a] - t * rd[a];
            for (int a = 0; a < 3; ++a) pv[a] = M[3 * a] * x[0] + M[3 * a + 1] * x[1] + M[3 * a + 2] * x[2];
            for (int a = 0; a < 3; ++a) {
              ga[4 + a] += 2.0 * dd2 * pv[a];
              for (int b = 0; b < 3; ++b) ga[7 + 3 * a + b] += 2.0 * dd2 * pv[a] * x[b];
            }
          }
        }
    }
  }
  for (int64_t k = 0; k < n * 16; ++k) {
    double s = 0;
    for (int th = 0; th < nthreads; ++th)
      if (!part[th].empty()) s += part[th][k];
    grad[k] = s;
  }
}

// Backward of the 3DGUT projection: from dL/d(o', colour, ro, M|centre)
// [n][16] (as orc_render_bwd_gut writes it) to the gradients of the inputs
// (activated scales and opacity, raw quaternion), [k][n] like the inputs,
// overwritten. Through o' = o comp, comp = sqrt(det_orig / det), the
// unscented transform's 2D covariance and its seven projected sigma points;
// through ro = M (campos - mu) at fixed M (dL/dmu = -M^T dL/dro) and
// M = S^-1 R^T with the centre fixed (the dL/dM given); through the colour
// as for 3DGS. Gaussians that are not visible get zero.
void orc_project_bwd_gut(int64_t n, const double* means, const double* scales,
                         const double* quats, const double* opac, const double* sh, int K,
                         const double* camv, int W, int H, const double* cfg, int tile_w,
                         int tile_h, int deg, const double* grad, double* g_means,
                         double* g_scales, double* g_quats, double* g_opac, double* g_sh) {
  const Cam cam = read_cam(camv, W, H);
  const double lowpass = cfg[0];
  const int nb = (deg + 1) * (deg + 1);
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < n; ++i) {
    for (int c = 0; c < 3; ++c) { g_means[c * n + i] = 0; g_scales[c * n + i] = 0; }
    for (int c = 0; c < 4; ++c) g_quats[c * n + i] = 0;
    g_opac[i] = 0;
    for (int j = 0; j < K; ++j)
      for (int ch = 0; ch < 3; ++ch) g_sh[(int64_t)(j * 3 + ch) * n + i] = 0;
    GutProj Gp;
    project_gut_one(i, n, means, scales, quats, opac, sh, cam, cfg, tile_w, tile_h, deg, Gp);
    if (Gp.tc == 0) continue;
    const double* g = grad + 16 * i;
    const double mu[3] = {means[i], means[n + i], means[2 * n + i]};
    const double q[4] = {quats[i], quats[n + i], quats[2 * n + i], quats[3 * n + i]};
    const double qnorm = std::sqrt(q[0] * q[0] + q[1] * q[1] + q[2] * q[2] + q[3] * q[3]);
    const double qn[4] = {q[0] / qnorm, q[1] / qnorm, q[2] / qnorm, q[3] / qnorm};
    double Rq[9];
    quat_to_rot(qn, Rq);
    const double s[3] = {scales[i], scales[n + i], scales[2 * n + i]};
    const double cp[3] = {
        -(cam.R[0] * cam.t[0] + cam.R[3] * cam.t[1] + cam.R[6] * cam.t[2]),
        -(cam.R[1] * cam.t[0] + cam.R[4] * cam.t[1] + cam.R[7] * cam.t[2]),
        -(cam.R[2] * cam.t[0] + cam.R[5] * cam.t[1] + cam.R[8] * cam.t[2])};
    double gmu[3] = {0, 0, 0}, gs[3] = {0, 0, 0}, gR[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};

    // colour = max(0, 0.5 + sum_j sh_j Y_j(dir)), dir = (mu - campos) / |.|
    double dv[3] = {mu[0] - cp[0], mu[1] - cp[1], mu[2] - cp[2]};
    const double dn = std::sqrt(dv[0] * dv[0] + dv[1] * dv[1] + dv[2] * dv[2]);
    for (int c = 0; c < 3; ++c) dv[c] /= dn;
    double Y[16], dY[16][3];
    sh_basis(deg, dv, Y, dY);
    double gdir[3] = {0, 0, 0};
    for (int ch = 0; ch < 3; ++ch) {
      double raw = 0.5;
      for (int j = 0; j < nb; ++j) raw += sh[(int64_t)(j * 3 + ch) * n + i] * Y[j];
      const double gr = raw > 0 ? g[1 + ch] : 0.0;
      for (int j = 0; j < nb; ++j) {
        g_sh[(int64_t)(j * 3 + ch) * n + i] = Y[j] * gr;
        const double wgt = sh[(int64_t)(j * 3 + ch) * n + i] * gr;
        for (int c = 0; c < 3; ++c) gdir[c] += wgt * dY[j][c];
      }
    }
    const double dd = dv[0] * gdir[0] + dv[1] * gdir[1] + dv[2] * gdir[2];
    for (int c = 0; c < 3; ++c) gmu[c] += (gdir[c] - dv[c] * dd) / dn;

    // ro = M (campos - mu) at fixed M; then M[r][c] = Rq[c][r] / s[r], whose
    // derivative (the centre fixed) the record gradient holds
    double gM[9];
    for (int k = 0; k < 9; ++k) gM[k] = g[7 + k];
    for (int r = 0; r < 3; ++r)
      for (int c = 0; c < 3; ++c) gmu[c] -= Gp.M[3 * r + c] * g[4 + r];
    for (int r = 0; r < 3; ++r)
      for (int c = 0; c < 3; ++c) {
        gR[3 * c + r] += gM[3 * r + c] / s[r];
        gs[r] -= gM[3 * r + c] * Rq[3 * c + r] / (s[r] * s[r]);
      }

    // o' = o comp, comp = sqrt(max(det_orig, 0) / det) over the sigma points
    const double k3 = std::sqrt(3.0);
    double X[7][3];
    for (int c = 0; c < 3; ++c) X[0][c] = mu[c];
    for (int j = 0; j < 3; ++j)
      for (int sg = 0; sg < 2; ++sg)
        for (int c = 0; c < 3; ++c)
          X[1 + 2 * j + sg][c] = mu[c] + (sg ? -1.0 : 1.0) * k3 * s[j] * Rq[3 * c + j];
    const double wm[7] = {0.0, 1.0 / 6, 1.0 / 6, 1.0 / 6, 1.0 / 6, 1.0 / 6, 1.0 / 6};
    const double wc[7] = {2.0, 1.0 / 6, 1.0 / 6, 1.0 / 6, 1.0 / 6, 1.0 / 6, 1.0 / 6};
    double Yc[7][3], P2[7][2];
    for (int p = 0; p < 7; ++p) {
      for (int r = 0; r < 3; ++r)
        Yc[p][r] = cam.R[3 * r] * X[p][0] + cam.R[3 * r + 1] * X[p][1] + cam.R[3 * r + 2] * X[p][2] +
                   cam.t[r];
      P2[p][0] = cam.fx * Yc[p][0] / Yc[p][2] + cam.cx;
      P2[p][1] = cam.fy * Yc[p][1] / Yc[p][2] + cam.cy;
    }
    double m2[2] = {0, 0};
    for (int p = 0; p < 7; ++p) { m2[0] += wm[p] * P2[p][0]; m2[1] += wm[p] * P2[p][1]; }
    double D[7][2], cxx = 0, cxy = 0, cyy = 0;
    for (int p = 0; p < 7; ++p) {
      D[p][0] = P2[p][0] - m2[0];
      D[p][1] = P2[p][1] - m2[1];
      cxx += wc[p] * D[p][0] * D[p][0];
      cxy += wc[p] * D[p][0] * D[p][1];
      cyy += wc[p] * D[p][1] * D[p][1];
    }
    const double det0 = cxx * cyy - cxy * cxy;
    const double det = (cxx + lowpass) * (cyy + lowpass) - cxy * cxy;
    const double comp = det > 0 ? std::sqrt(std::max(det0, 0.0) / det) : 0.0;
    g_opac[i] = comp * g[0];
    if (det0 > 0 && det > 0) {
      const double gcomp = opac[i] * g[0];
      const double gdet0 = gcomp * comp / (2.0 * det0), gdet = -gcomp * comp / (2.0 * det);
      const double gxx = gdet0 * cyy + gdet * (cyy + lowpass);
      const double gyy = gdet0 * cxx + gdet * (cxx + lowpass);
      const double gxy = -2.0 * cxy * (gdet0 + gdet);
      double gD[7][2], sD[2] = {0, 0};
      for (int p = 0; p < 7; ++p) {
        gD[p][0] = wc[p] * (2.0 * D[p][0] * gxx + D[p][1] * gxy);
        gD[p][1] = wc[p] * (2.0 * D[p][1] * gyy + D[p][0] * gxy);
        sD[0] += gD[p][0];
        sD[1] += gD[p][1];
      }
      for (int p = 0; p < 7; ++p) {
        const double gPx = gD[p][0] - wm[p] * sD[0], gPy = gD[p][1] - wm[p] * sD[1];
        const double z = Yc[p][2];
        const double gy[3] = {cam.fx / z * gPx, cam.fy / z * gPy,
                              -(cam.fx * Yc[p][0] * gPx + cam.fy * Yc[p][1] * gPy) / (z * z)};
        double gX[3];
        for (int c = 0; c < 3; ++c)
          gX[c] = cam.R[c] * gy[0] + cam.R[3 + c] * gy[1] + cam.R[6 + c] * gy[2];
        for (int c = 0; c < 3; ++c) gmu[c] += gX[c];
        if (p == 0) continue;
        const int j = (p - 1) / 2;
        const double sign = ((p - 1) % 2) ? -1.0 : 1.0;
        for (int c = 0; c < 3; ++c) {
          gs[j] += sign * k3 * gX[c] * Rq[3 * c + j];
          gR[3 * c + j] += sign * k3 * s[j] * gX[c];
        }
      }
    }
    for (int c = 0; c < 3; ++c) {
      g_means[c * n + i] = gmu[c];
      g_scales[c * n + i] = gs[c];
    }
    double dR[9][4];
    quat_to_rot_jac(qn, dR);
    double gqn[4] = {0, 0, 0, 0};
    for (int k = 0; k < 9; ++k)
      for (int c = 0; c < 4; ++c) gqn[c] += gR[k] * dR[k][c];
    const double qd = qn[0] * gqn[0] + qn[1] * gqn[1] + qn[2] * gqn[2] + qn[3] * gqn[3];
    for (int c = 0; c < 4; ++c) g_quats[c * n + i] = (gqn[c] - qn[c] * qd) / qnorm;
  }
}


// ----------------------------------------------------------------------------
// LinPrim backward. The forward (Listing XPR-LinPrim: project and evaluate,
// blended by Algorithm 1) differentiated by hand, as the paper obtains it by
// automatic differentiation (section Key Interfaces). The record gradient
// holds the 15 values evaluate reads -- u, v (mu_2D - 1/2), sigma, the
// colour (3), the rows c0, c1, c2 of A^-1 (9) -- and a 16th slot that stays
// zero: [n][16]. ex, ey only place the rect (piecewise constant).
// ----------------------------------------------------------------------------

// The chord of lin_chord with the slabs that bound it: the entry point is
// max over slabs of m_i - h_i (slab *ia), the exit min of m_i + h_i (slab
// *ib); the first slab reaching the extreme is taken. Returns the chord
// (<= 0 when the ray misses); slabs with |n_z| < 1e-10 bound neither.
double lin_chord_slabs(const double* c, double dx, double dy, int* ia, int* ib) {
  double enter = -INFINITY, exit_ = INFINITY;
  *ia = *ib = -1;
  for (int i = 0; i < 4; ++i) {
    const double e1 = (i & 2) ? -1.0 : 1.0, e2 = (i & 1) ? -1.0 : 1.0;
    const double nx = c[0] + e1 * c[3] + e2 * c[6];
    const double ny = c[1] + e1 * c[4] + e2 * c[7];
    const double nz = c[2] + e1 * c[5] + e2 * c[8];
    const double w = nx * dx + ny * dy;
    if (std::fabs(nz) >= 1e-10) {
      const double m = -w / nz, h = 1.0 / std::fabs(nz);
      if (m - h > enter) { enter = m - h; *ia = i; }
      if (m + h < exit_) { exit_ = m + h; *ib = i; }
    } else if (std::fabs(w) > 1.0) {
      return -1.0;
    }
  }
  return exit_ - enter;
}

// dL/d(u, v, sigma, r, g, b, c0, c1, c2, 0) per record [n][16] from
// dL/dimage [3][H][W]. Per pixel the blended entries are found front to back
// (as in orc_render_fwd_lin), then walked back with the colour behind, as
// in orc_render_bwd. With e = exp(-sigma chord) and alpha = 1 - e (not
// clamped): dL/dsigma = e chord dL/dalpha, dL/dchord = e sigma dL/dalpha.
// chord = (m_b + h_b) - (m_a - h_a) for the exit slab b and entry slab a,
// m = -(n_x dx + n_y dy) / n_z, h = 1 / |n_z|, n_i = c0 +- c1 +- c2 and
// (dx, dy) = (x - u, y - v):
//   dm/dn = (-dx / n_z, -dy / n_z, -m / n_z), dh/dn_z = -sgn(n_z) h^2,
//   dm/du = n_x / n_z, dm/dv = n_y / n_z.
void orc_render_bwd_lin(int W, int H, int tile_w, int tile_h, int64_t n, const double* rec,
                        const int32_t* vals, const int32_t* ranges, const double* cfg,
                        const double* dimg, double* grad) {
  const double alpha_min = cfg[0], alpha_max = cfg[1], t_min = cfg[2];
  const double bg[3] = {cfg[3], cfg[4], cfg[5]};
  const int tiles_x = (W + tile_w - 1) / tile_w;
  const int tiles_y = (H + tile_h - 1) / tile_h;
  int nthreads = 1;
#ifdef _OPENMP
  nthreads = omp_get_max_threads();
#endif
  std::vector<std::vector<double>> part(nthreads);
#pragma omp parallel
  {
    int tid = 0;
#ifdef _OPENMP
    tid = omp_get_thread_num();
#endif
    std::vector<double>& acc = part[tid];
    acc.assign((size_t)n * 16, 0.0);
    struct Step { int64_t g; double alpha, T, chord; int ia, ib; bool clamped; };
    std::vector<Step> steps;
#pragma omp for schedule(dynamic, 1)
    for (int t = 0; t < tiles_x * tiles_y; ++t) {
      const int tx = t % tiles_x, ty = t / tiles_x;
      const int32_t start = ranges[2 * t], end = ranges[2 * t + 1];
      for (int py = ty * tile_h; py < std::min(H, (ty + 1) * tile_h); ++py)
        for (int px = tx * tile_w; px < std::min(W, (tx + 1) * tile_w); ++px) {
          steps.clear();
          double T = 1.0;
          for (int32_t k = start; k < end; ++k) {
            const int64_t gi = vals[k];
            const double* r = rec + 17 * gi;
            int ia, ib;
            const double ch = lin_chord_slabs(r + 8, px - r[0], py - r[1], &ia, &ib);
            if (!(ch > 0.0)) continue;
            const double raw = -std::expm1(-r[2] * ch);
            const double alpha = std::min(alpha_max, raw);
            if (alpha < alpha_min) continue;
            const double Tn = T * (1.0 - alpha);
            if (Tn < t_min) break;
            steps.push_back(Step{gi, alpha, T, ch, ia, ib, raw > alpha_max});
            T = Tn;
          }
          const double Tfin = T;
          const int64_t p = (int64_t)py * W + px;
          const double G[3] = {dimg[p], dimg[(int64_t)W * H + p], dimg[2 * (int64_t)W * H + p]};
          const double bgG = bg[0] * G[0] + bg[1] * G[1] + bg[2] * G[2];
          double S[3] = {0, 0, 0};
          for (int si = (int)steps.size() - 1; si >= 0; --si) {
            const Step& st = steps[si];
            const double* r = rec + 17 * st.g;
            double* ga = acc.data() + 16 * st.g;
            double dalpha = 0;
            for (int c = 0; c < 3; ++c) {
              ga[3 + c] += st.alpha * st.T * G[c];
              dalpha += st.T * (r[3 + c] - S[c]) * G[c];
            }
            dalpha -= Tfin * bgG / (1.0 - st.alpha);
            for (int c = 0; c < 3; ++c) S[c] = st.alpha * r[3 + c] + (1.0 - st.alpha) * S[c];
            if (st.clamped) continue;
            const double e = std::exp(-r[2] * st.chord);
            ga[2] += e * st.chord * dalpha;
            const double dch = e * r[2] * dalpha;
            const double* c = r + 8;
            const double dx = px - r[0], dy = py - r[1];
            // exit slab (kappa = +1) and entry slab (kappa = -1)
            for (int side = 0; side < 2; ++side) {
              const int i = side == 0 ? st.ib : st.ia;
              const double kappa = side == 0 ? 1.0 : -1.0;
              const double e1 = (i & 2) ? -1.0 : 1.0, e2 = (i & 1) ? -1.0 : 1.0;
              const double nx = c[0] + e1 * c[3] + e2 * c[6];
              const double ny = c[1] + e1 * c[4] + e2 * c[7];
              const double nz = c[2] + e1 * c[5] + e2 * c[8];
              const double m = -(nx * dx + ny * dy) / nz, h = 1.0 / std::fabs(nz);
              const double sg = nz > 0 ? 1.0 : -1.0;
              // d chord / d n_i: kappa dm/dn + dh/dn (h enters the chord with +)
              const double gn[3] = {dch * kappa * (-dx / nz), dch * kappa * (-dy / nz),
                                    dch * (kappa * (-m / nz) - sg * h * h)};
              for (int k = 0; k < 3; ++k) {
                ga[6 + k] += gn[k];
                ga[9 + k] += e1 * gn[k];
                ga[12 + k] += e2 * gn[k];
              }
              ga[0] += dch * kappa * nx / nz;
              ga[1] += dch * kappa * ny / nz;
            }
          }
        }
    }
  }
  for (int64_t k = 0; k < n * 16; ++k) {
    double s = 0;
    for (int th = 0; th < nthreads; ++th)
      if (!part[th].empty()) s += part[th][k];
    grad[k] = s;
  }
}

// Backward of the LinPrim projection: from dL/d(u, v, sigma, colour, c0,
// c1, c2) [n][16] to the gradients of the inputs (means, scales as
// half-extents, opacity, raw quaternion, SH), [k][n], overwritten; not
// visible: zero. Through mu_2D = (fx x / z + cx, fy y / z + cy) of the
// camera-space centre (x, y, z); sigma = -log(1 - 0.99 o) / (2 s_min) with
// o = min(0.999, max(0, opacity)) (no gradient where the clip holds, the
// whole s_min term to the smallest scale); C = A^-1 for
// A = J3 R_w2c Rq diag(s) (dL/dA = -C^T dL/dC C^T), J3's perspective rows
// and unit viewing direction differentiated with respect to (x, y, z);
// the colour as for 3DGS.
void orc_project_bwd_lin(int64_t n, const double* means, const double* scales,
                         const double* quats, const double* opac, const double* sh, int K,
                         const double* camv, int W, int H, const double* cfg, int tile_w,
                         int tile_h, int deg, const double* grad, double* g_means,
                         double* g_scales, double* g_quats, double* g_opac, double* g_sh) {
  const Cam cam = read_cam(camv, W, H);
  const int nb = (deg + 1) * (deg + 1);
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < n; ++i) {
    for (int c = 0; c < 3; ++c) { g_means[c * n + i] = 0; g_scales[c * n + i] = 0; }
    for (int c = 0; c < 4; ++c) g_quats[c * n + i] = 0;
    g_opac[i] = 0;
    for (int j = 0; j < K; ++j)
      for (int ch = 0; ch < 3; ++ch) g_sh[(int64_t)(j * 3 + ch) * n + i] = 0;
    LinProj L;
    project_lin_one(i, n, means, scales, quats, opac, sh, cam, cfg, tile_w, tile_h, deg, L);
    if (L.tc == 0) continue;
    const double* g = grad + 16 * i;
    const double mu[3] = {means[i], means[n + i], means[2 * n + i]};
    const double q[4] = {quats[i], quats[n + i], quats[2 * n + i], quats[3 * n + i]};
    const double qnorm = std::sqrt(q[0] * q[0] + q[1] * q[1] + q[2] * q[2] + q[3] * q[3]);
    const double qn[4] = {q[0] / qnorm, q[1] / qnorm, q[2] / qnorm, q[3] / qnorm};
    double Rq[9];
    quat_to_rot(qn, Rq);
    const double s[3] = {scales[i], scales[n + i], scales[2 * n + i]};
    double mc[3];
    for (int r = 0; r < 3; ++r)
      mc[r] = cam.R[3 * r] * mu[0] + cam.R[3 * r + 1] * mu[1] + cam.R[3 * r + 2] * mu[2] + cam.t[r];
    const double x = mc[0], y = mc[1], z = mc[2];
    const double d = std::sqrt(x * x + y * y + z * z);
    double gmc[3] = {0, 0, 0}, gmu[3] = {0, 0, 0}, gs[3] = {0, 0, 0}, gRq[9] = {0};

    // mean2D (u = mu_2D.x - 1/2, v likewise)
    gmc[0] += g[0] * cam.fx / z;
    gmc[1] += g[1] * cam.fy / z;
    gmc[2] += -g[0] * cam.fx * x / (z * z) - g[1] * cam.fy * y / (z * z);

    // sigma
    int jmin = 0;
    for (int j = 1; j < 3; ++j)
      if (s[j] < s[jmin]) jmin = j;
    const double o = std::min(0.999, std::max(0.0, opac[i]));
    const double smin = s[jmin];
    if (opac[i] > 0.0 && opac[i] < 0.999) g_opac[i] = g[2] * 0.99 / ((1.0 - 0.99 * o) * 2.0 * smin);
    gs[jmin] += -g[2] * L.sigma / smin;

    // colour = max(0, 0.5 + sum_j sh_j Y_j(dir)), dir = (mu - campos) / |.|
    const double cp[3] = {
        -(cam.R[0] * cam.t[0] + cam.R[3] * cam.t[1] + cam.R[6] * cam.t[2]),
        -(cam.R[1] * cam.t[0] + cam.R[4] * cam.t[1] + cam.R[7] * cam.t[2]),
        -(cam.R[2] * cam.t[0] + cam.R[5] * cam.t[1] + cam.R[8] * cam.t[2])};
    double dv[3] = {mu[0] - cp[0], mu[1] - cp[1], mu[2] - cp[2]};
    const double dn = std::sqrt(dv[0] * dv[0] + dv[1] * dv[1] + dv[2] * dv[2]);
    for (int c = 0; c < 3; ++c) dv[c] /= dn;
    double Y[16], dY[16][3];
    sh_basis(deg, dv, Y, dY);
    double gdir[3] = {0, 0, 0};
    for (int ch = 0; ch < 3; ++ch) {
      double raw = 0.5;
      for (int j = 0; j < nb; ++j) raw += sh[(int64_t)(j * 3 + ch) * n + i] * Y[j];
      const double gr = raw > 0 ? g[3 + ch] : 0.0;
      for (int j = 0; j < nb; ++j) {
        g_sh[(int64_t)(j * 3 + ch) * n + i] = Y[j] * gr;
        const double wgt = sh[(int64_t)(j * 3 + ch) * n + i] * gr;
        for (int c = 0; c < 3; ++c) gdir[c] += wgt * dY[j][c];
      }
    }
    const double dd = dv[0] * gdir[0] + dv[1] * gdir[1] + dv[2] * gdir[2];
    for (int c = 0; c < 3; ++c) gmu[c] += (gdir[c] - dv[c] * dd) / dn;

    // C = A^-1 (rows c0, c1, c2): dL/dA = -C^T dL/dC C^T
    const double* C = L.c;
    const double* GC = g + 6;
    double T1[9], GA[9];
    for (int r = 0; r < 3; ++r)  // T1 = dL/dC C^T
      for (int c = 0; c < 3; ++c)
        T1[3 * r + c] = GC[3 * r] * C[3 * c] + GC[3 * r + 1] * C[3 * c + 1] + GC[3 * r + 2] * C[3 * c + 2];
    for (int r = 0; r < 3; ++r)  // GA = -C^T T1
      for (int c = 0; c < 3; ++c)
        GA[3 * r + c] = -(C[r] * T1[c] + C[3 + r] * T1[3 + c] + C[6 + r] * T1[6 + c]);
    // A = J3 Wm diag(s), Wm = R_w2c Rq
    const double J[9] = {cam.fx / z, 0.0, -cam.fx * x / (z * z), 0.0, cam.fy / z,
                         -cam.fy * y / (z * z), x / d, y / d, z / d};
    double Wm[9], JW[9];
    for (int r = 0; r < 3; ++r)
      for (int c = 0; c < 3; ++c)
        Wm[3 * r + c] = cam.R[3 * r] * Rq[c] + cam.R[3 * r + 1] * Rq[3 + c] + cam.R[3 * r + 2] * Rq[6 + c];
    for (int r = 0; r < 3; ++r)
      for (int c = 0; c < 3; ++c)
        JW[3 * r + c] = J[3 * r] * Wm[c] + J[3 * r + 1] * Wm[3 + c] + J[3 * r + 2] * Wm[6 + c];
    double GJW[9];
    for (int r = 0; r < 3; ++r)
      for (int c = 0; c < 3; ++c) {
        gs[c] += GA[3 * r + c] * JW[3 * r + c];
        GJW[3 * r + c] = GA[3 * r + c] * s[c];
      }
    double GJ[9], GW[9];
    for (int r = 0; r < 3; ++r)
      for (int c = 0; c < 3; ++c) {
        GJ[3 * r + c] = GJW[3 * r] * Wm[3 * c] + GJW[3 * r + 1] * Wm[3 * c + 1] + GJW[3 * r + 2] * Wm[3 * c + 2];
        GW[3 * r + c] = J[r] * GJW[c] + J[3 + r] * GJW[3 + c] + J[6 + r] * GJW[6 + c];
      }
    for (int r = 0; r < 3; ++r)  // Wm = R_w2c Rq: dL/dRq = R_w2c^T dL/dWm
      for (int c = 0; c < 3; ++c)
        gRq[3 * r + c] = cam.R[r] * GW[c] + cam.R[3 + r] * GW[3 + c] + cam.R[6 + r] * GW[6 + c];
    // J3 with respect to (x, y, z)
    const double z2 = z * z, z3 = z2 * z;
    gmc[2] += -GJ[0] * cam.fx / z2 + GJ[2] * 2.0 * cam.fx * x / z3 - GJ[4] * cam.fy / z2 +
              GJ[5] * 2.0 * cam.fy * y / z3;
    gmc[0] += -GJ[2] * cam.fx / z2;
    gmc[1] += -GJ[5] * cam.fy / z2;
    const double e[3] = {x / d, y / d, z / d};
    const double ge = GJ[6] * e[0] + GJ[7] * e[1] + GJ[8] * e[2];
    for (int c = 0; c < 3; ++c) gmc[c] += (GJ[6 + c] - e[c] * ge) / d;
    // mc = R_w2c mu + t
    for (int c = 0; c < 3; ++c)
      gmu[c] += cam.R[c] * gmc[0] + cam.R[3 + c] * gmc[1] + cam.R[6 + c] * gmc[2];

    for (int c = 0; c < 3; ++c) {
      g_means[c * n + i] = gmu[c];
      g_scales[c * n + i] = gs[c];
    }
    double dR[9][4];
    quat_to_rot_jac(qn, dR);
    double gqn[4] = {0, 0, 0, 0};
    for (int k = 0; k < 9; ++k)
      for (int c = 0; c < 4; ++c) gqn[c] += gRq[k] * dR[k][c];
    const double qd = qn[0] * gqn[0] + qn[1] * gqn[1] + qn[2] * gqn[2] + qn[3] * gqn[3];
    for (int c = 0; c < 4; ++c) g_quats[c * n + i] = (gqn[c] - qn[c] * qd) / qnorm;
  }
}

}  // extern "C"
