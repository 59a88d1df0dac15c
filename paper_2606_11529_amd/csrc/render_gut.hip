// Forward compositing of 3DGUT: Algorithm 1 of the paper with the
// pixel_info and evaluate of the listing "Implementation of XPR-3DGUT".
//
// One workgroup per tile, one thread per pixel (256 threads for 16x16
// tiles, 64 for 8x8). pixel_info: the world-space unit direction rd of the
// ray through (x + 1/2, y + 1/2), once per pixel. evaluate, per list entry:
// in the Gaussian's canonical frame the ray is ro + tau M rd (ro and
// M = S^-1 R^T from the record); its closest approach to the centre,
// at tau_max = -(ro . rdc) / (rdc . rdc) with rdc = M rd, has squared
// distance d^2 = |ro|^2 - (ro . rdc)^2 / (rdc . rdc), and the response is
// exp(-d^2 / 2). For small Gaussians seen from afar |ro| is in the
// thousands while the d^2 that matters is a few units, so d^2 is formed in
// float64 (a float32 ray direction alone would move it by ~1e-4); the
// exponential, the gates and the blending are float32 as for 3DGS:
// skipped unless the response exceeds 0.0113 (the listing's validity
// threshold, d^2 < 8.97), alpha = min(alpha_max, o' response) >= alpha_min,
// stop before blending when T (1 - alpha) < t_min.
#include "xpr_internal.h"

namespace xpr {

constexpr int kGutBatch = 128;
constexpr float kGutValid = 0.0113f;
constexpr float kGutHalfLog2e = 0.72134752044448170f;  // log2(e) / 2
// d^2 above this cannot pass the validity threshold (2 ln(1 / 0.0113) =
// 8.966, with margin for the float32 rounding of the response)
constexpr double kGutD2Max = 9.0;

struct GutStage {
  float4 g0[kGutBatch];    // ro, o'
  float4 g1[kGutBatch];    // M00 M01 M02 M10
  float4 g2[kGutBatch];    // M11 M12 M20 M21
  float4 g3[kGutBatch];    // M22, r, g, b
  double ro2[kGutBatch];   // |ro|^2
};

template <int TW, int TH>
__global__ __launch_bounds__(TW* TH) void k_render_fwd_gut(
    Batch B, const float4* __restrict__ splat, const int32_t* __restrict__ vals,
    const int2* __restrict__ ranges, float* __restrict__ image, float* __restrict__ Tfin,
    int32_t* __restrict__ ncon, int32_t* __restrict__ tile_work, const int32_t* order) {
  constexpr int NT = TW * TH;
  __shared__ GutStage S;
  const int g = order ? order[blockIdx.x] : (int)blockIdx.x;
  const ViewDev& V = B.v[view_of_tile(B, g)];
  const int lt = g - V.tile_off;
  const int ty = lt / V.tiles_x, tx = lt - ty * V.tiles_x;
  const int px = tx * TW + (int)(threadIdx.x % TW);
  const int py = ty * TH + (int)(threadIdx.x / TW);
  const bool inside = px < V.W && py < V.H;
  const int2 rg = ranges[g];
  const float amax = B.alpha_max, amin = B.alpha_min, tmin = B.t_min;
  // pixel_info: world ray direction through the pixel centre, R^T dc
  double rd0, rd1, rd2;
  {
    const double dcx = ((double)px + 0.5 - (double)V.cx) / (double)V.fx;
    const double dcy = ((double)py + 0.5 - (double)V.cy) / (double)V.fy;
    const double inv = 1.0 / sqrt(dcx * dcx + dcy * dcy + 1.0);
    const double ex = dcx * inv, ey = dcy * inv, ez = inv;
    rd0 = (double)V.R[0] * ex + (double)V.R[3] * ey + (double)V.R[6] * ez;
    rd1 = (double)V.R[1] * ex + (double)V.R[4] * ey + (double)V.R[7] * ez;
    rd2 = (double)V.R[2] * ex + (double)V.R[5] * ey + (double)V.R[8] * ez;
  }
  float T = 1.f, C0 = 0.f, C1 = 0.f, C2 = 0.f;
  int last = 0;
  bool done = !inside;
  int walked = 0;
  const int stride = splat_stride4(B);
  for (int base = rg.x; base < rg.y; base += kGutBatch) {
    if (__syncthreads_count(!done) == 0) break;
    const int nb = min(kGutBatch, rg.y - base);
    walked = nb + (base - rg.x);
    for (int k = threadIdx.x; k < nb; k += NT) {
      const float4* q = splat + (size_t)stride * (size_t)vals[base + k];
      const float4 q1 = q[1], q2 = q[2], q3 = q[3], q4 = q[4], q5 = q[5];
      S.g0[k] = make_float4(q2.y, q2.z, q2.w, q1.y);
      S.g1[k] = q3;
      S.g2[k] = q4;
      S.g3[k] = make_float4(q5.x, q1.z, q1.w, q2.x);
      S.ro2[k] = (double)q2.y * q2.y + (double)q2.z * q2.z + (double)q2.w * q2.w;
    }
    __syncthreads();
    for (int i0 = 0; i0 < nb; i0 += 8) {
      if (__ballot(!done) == 0) break;
      const int iend = min(i0 + 8, nb);
      for (int k = i0; k < iend; ++k) {
        const float4 a = S.g0[k], m1 = S.g1[k], m2 = S.g2[k], m3 = S.g3[k];
        const double r0 = (double)m1.x * rd0 + (double)m1.y * rd1 + (double)m1.z * rd2;
        const double r1 = (double)m1.w * rd0 + (double)m2.x * rd1 + (double)m2.y * rd2;
        const double r2 = (double)m2.z * rd0 + (double)m2.w * rd1 + (double)m3.x * rd2;
        const double dot = (double)a.x * r0 + (double)a.y * r1 + (double)a.z * r2;
        const double nrm = r0 * r0 + r1 * r1 + r2 * r2;
        const double d2 = fmax(S.ro2[k] - dot * dot / nrm, 0.0);
        const bool near = !done && d2 < kGutD2Max;
        if (__ballot(near) == 0) continue;
        const float resp = __builtin_amdgcn_exp2f(-kGutHalfLog2e * (float)d2);
        const float alpha = fminf(amax, __fmul_rn(a.w, resp));
        const bool use = near && resp > kGutValid && alpha >= amin;
        const float Tn = T * (1.f - alpha);
        const bool blend = use && Tn >= tmin;
        const float w = blend ? alpha * T : 0.f;
        C0 += m3.y * w;
        C1 += m3.z * w;
        C2 += m3.w * w;
        T = blend ? Tn : T;
        last = blend ? base + k - rg.x + 1 : last;
        done = done || (use && !blend);
      }
    }
  }
  if (inside) {
    const size_t WH = (size_t)V.W * V.H;
    const size_t p = (size_t)py * V.W + px;
    float* img = image + 3 * (size_t)V.pix_off;
    img[p] = C0 + T * B.bg[0];
    img[WH + p] = C1 + T * B.bg[1];
    img[2 * WH + p] = C2 + T * B.bg[2];
    Tfin[(size_t)V.pix_off + p] = T;
    ncon[(size_t)V.pix_off + p] = last;
  }
  if (tile_work && threadIdx.x == 0) tile_work[g] = walked;
}

hipError_t launch_render_fwd_gut(const Batch& B, const float* splat, const int32_t* vals,
                                 const int32_t* ranges, const int32_t* order, float* image,
                                 float* Tfin, int32_t* ncon, int32_t* tile_work, hipStream_t st) {
  if (B.total_tiles <= 0) return hipSuccess;
  const float4* sp = reinterpret_cast<const float4*>(splat);
  const int2* rg = reinterpret_cast<const int2*>(ranges);
  const dim3 grid(B.total_tiles);
  if (B.tile_w == 8)
    hipLaunchKernelGGL((k_render_fwd_gut<8, 8>), grid, dim3(64), 0, st, B, sp, vals, rg, image,
                       Tfin, ncon, tile_work, order);
  else
    hipLaunchKernelGGL((k_render_fwd_gut<16, 16>), grid, dim3(256), 0, st, B, sp, vals, rg,
                       image, Tfin, ncon, tile_work, order);
  return hipGetLastError();
}

}  // namespace xpr
