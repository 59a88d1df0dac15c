// Forward compositing of 3DGUT: Algorithm 1 of the paper with the
// pixel_info and evaluate of the listing "Implementation of XPR-3DGUT".
//
// One workgroup per tile, one thread per pixel (256 threads for 16x16
// tiles, 64 for 8x8, 1024 for 32x32). pixel_info: the world-space unit direction rd of the
// ray through (x + 1/2, y + 1/2), once per pixel. evaluate, per list entry:
// in the Gaussian's canonical frame the ray is ro + tau M rd (ro and
// M = S^-1 R^T from the record); its closest approach to the centre,
// at tau_max = -(ro . rdc) / (rdc . rdc) with rdc = M rd, has squared
// distance d^2 = |ro|^2 - (ro . rdc)^2 / (rdc . rdc), and the response is
// exp(-d^2 / 2), evaluated as ro . rdc = (M^T ro) . rd and
// rdc . rdc = rd^T (M^T M) rd with M^T ro and M^T M formed once per staged
// record and the six products of rd's components once per pixel (9
// multiply-adds per entry instead of 15). For small Gaussians seen from
// afar |ro| is in the thousands while the d^2 that matters is a few units,
// so d^2 is formed in
// float64 (a float32 ray direction alone would move it by ~1e-4); the
// exponential, the gates and the blending are float32 as for 3DGS:
// skipped unless the response exceeds 0.0113 (the listing's validity
// threshold, d^2 < 8.97), alpha = min(alpha_max, o' response) >= alpha_min,
// stop before blending when T (1 - alpha) < t_min.
//
// Per-wave record lists: each record carries the pixel box (int16 column
// and row bounds, from the projection) that holds every pixel whose ray can
// come within d^2 <= 9 of its centre; each staged record gets the mask of
// the waves whose pixel rows meet that box (none when the box misses the
// tile's columns), and each wave walks only its records, in list order;
// the per-lane test still decides.
#include "xpr_internal.h"

namespace xpr {

constexpr int kGutBatch = 128;
constexpr float kGutValid = 0.0113f;
constexpr float kGutHalfLog2e = 0.72134752044448170f;  // log2(e) / 2
// d^2 above this cannot pass the validity threshold (2 ln(1 / 0.0113) =
// 8.966, with margin for the float32 rounding of the response)
constexpr double kGutD2Max = 9.0;

struct GutRec {
  double w[3];   // M^T ro
  double q[6];   // M^T M: 00 11 22 01 02 12
  double ro2;    // |ro|^2
  float o, r, g, b;
};

template <int NW>
struct GutStage {
  // one bit per wave: 4 waves at 16x16 tiles, 16 at 32x32
  using mask_t = std::conditional_t<(NW > 8), uint16_t, uint8_t>;
  GutRec rec[kGutBatch];
  mask_t mask[kGutBatch];
  uint16_t list[NW][kGutBatch];
};

// Mask of the waves (rows of RPW pixels from y0) that meet the record's
// pixel box (bx, by: int16 pairs X0 | X1 << 16, Y0 | Y1 << 16); x0 .. x1 are
// the tile's pixel columns.
__device__ __forceinline__ uint32_t gut_wave_mask(uint32_t bx, uint32_t by, int x0, int x1,
                                                  int y0, int rpw, int nw) {
  const int X0 = (int16_t)(bx & 0xffffu), X1 = (int16_t)(bx >> 16);
  const int Y0 = (int16_t)(by & 0xffffu), Y1 = (int16_t)(by >> 16);
  if (X1 < x0 || X0 > x1) return 0u;
  uint32_t msk = 0u;
  for (int w = 0; w < nw; ++w) {
    const int r0 = y0 + w * rpw;
    if (Y1 >= r0 && Y0 <= r0 + rpw - 1) msk |= 1u << w;
  }
  return msk;
}

// With COUNT the tile also counts the definition's work into tile_work
// [g][2]: per pixel the entries evaluated (up to and including the one that
// stops it, else the whole list) and the entries blended.
template <int TW, int TH, bool COUNT = false>
__global__ __launch_bounds__(TW* TH)
__attribute__((amdgpu_waves_per_eu(TW * TH >= 256 ? 7 : 1))) void k_render_fwd_gut(
    Batch B, const float4* __restrict__ splat, const int32_t* __restrict__ vals,
    const int2* __restrict__ ranges, float* __restrict__ image, float* __restrict__ Tfin,
    int32_t* __restrict__ ncon, int32_t* __restrict__ tile_work, const int32_t* order) {
  constexpr int NT = TW * TH;
  constexpr int NW = (NT + 63) / 64;
  constexpr int RPW = 64 / TW;  // pixel rows per wave
  __shared__ GutStage<NW> S;
  const int g = order ? order[blockIdx.x] : (int)blockIdx.x;
  const ViewDev& V = B.v[view_of_tile(B, g)];
  const int lt = g - V.tile_off;
  const int ty = lt / V.tiles_x, tx = lt - ty * V.tiles_x;
  const int px = tx * TW + (int)(threadIdx.x % TW);
  const int py = ty * TH + (int)(threadIdx.x / TW);
  const bool inside = px < V.W && py < V.H;
  const int2 rg = ranges[g];
  const float amax = B.alpha_max, amin = B.alpha_min, tmin = B.t_min;
  const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
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
  const double p00 = rd0 * rd0, p11 = rd1 * rd1, p22 = rd2 * rd2;
  const double p01 = 2.0 * rd0 * rd1, p02 = 2.0 * rd0 * rd2, p12 = 2.0 * rd1 * rd2;
  float T = 1.f, C0 = 0.f, C1 = 0.f, C2 = 0.f;
  int last = 0;
  int stop = 0, nbl = 0;  // COUNT only
  // a finished pixel (or one outside the image) carries lift = +inf, which
  // fails every later test; kept in a vector register (a carried boolean
  // becomes a lane mask updated by scalar instructions on every record)
  float lift = inside ? 0.f : __builtin_inff();
  const int stride = splat_stride4(B);
  for (int base = rg.x; base < rg.y; base += kGutBatch) {
    if (__syncthreads_count(lift == 0.f) == 0) break;
    const int nb = min(kGutBatch, rg.y - base);
    for (int k = threadIdx.x; k < nb; k += NT) {
      const float4* q = splat + (size_t)stride * (size_t)vals[base + k];
      const float4 q1 = q[1], q2 = q[2], q3 = q[3], q4 = q[4], q5 = q[5];
      const double m[9] = {q3.x, q3.y, q3.z, q3.w, q4.x, q4.y, q4.z, q4.w, q5.x};
      const double ro[3] = {q2.y, q2.z, q2.w};
      GutRec& G = S.rec[k];
#pragma unroll
      for (int c = 0; c < 3; ++c) G.w[c] = m[c] * ro[0] + m[3 + c] * ro[1] + m[6 + c] * ro[2];
      auto mm = [&](int a, int b) { return m[a] * m[b] + m[3 + a] * m[3 + b] + m[6 + a] * m[6 + b]; };
      G.q[0] = mm(0, 0); G.q[1] = mm(1, 1); G.q[2] = mm(2, 2);
      G.q[3] = mm(0, 1); G.q[4] = mm(0, 2); G.q[5] = mm(1, 2);
      G.ro2 = ro[0] * ro[0] + ro[1] * ro[1] + ro[2] * ro[2];
      G.o = q1.y; G.r = q1.z; G.g = q1.w; G.b = q2.x;
      S.mask[k] = (typename GutStage<NW>::mask_t)gut_wave_mask(
          __float_as_uint(q5.y), __float_as_uint(q5.z), tx * TW, tx * TW + TW - 1, ty * TH, RPW, NW);
    }
    __syncthreads();
    // this wave's records of the batch, in list order
    int cnt = 0;
    {
      const uint64_t lt_mask = lane == 0 ? 0ull : (~0ull >> (64 - lane));
      for (int i0 = 0; i0 < nb; i0 += 64) {
        const int k = i0 + lane;
        const bool hit = k < nb && ((S.mask[k] >> wv) & 1u);
        const uint64_t m = __ballot(hit);
        if (hit) S.list[wv][cnt + __popcll(m & lt_mask)] = (uint16_t)k;
        cnt += __popcll(m);
      }
    }
    __syncthreads();
    for (int i0 = 0; i0 < cnt; i0 += 8) {
      if (__ballot(lift == 0.f) == 0) break;
      const int iend = min(i0 + 8, cnt);
      int knext = S.list[wv][i0];
      for (int i = i0; i < iend; ++i) {
        // the next list entry is read one step ahead, so the record's reads
        // do not wait behind the read of its index
        const int k = knext;
        if (i + 1 < iend) knext = S.list[wv][i + 1];
        const GutRec& G = S.rec[k];
        const double dot = G.w[0] * rd0 + G.w[1] * rd1 + G.w[2] * rd2;
        const double nrm = G.q[0] * p00 + G.q[1] * p11 + G.q[2] * p22 + G.q[3] * p01 +
                           G.q[4] * p02 + G.q[5] * p12;
        // 1 / nrm: hardware reciprocal, then two Newton steps
        double rn = __builtin_amdgcn_rcp(nrm);
        rn = fma(rn, fma(-nrm, rn, 1.0), rn);
        rn = fma(rn, fma(-nrm, rn, 1.0), rn);
        const double d2 = fmax(G.ro2 - dot * dot * rn, 0.0);
        const bool near = d2 + (double)lift < kGutD2Max;
        if (__ballot(near) == 0) continue;
        const float resp = __builtin_amdgcn_exp2f(-kGutHalfLog2e * (float)d2);
        const float alpha = fminf(amax, __fmul_rn(G.o, resp));
        const bool use = near && resp > kGutValid && alpha >= amin;
        const float Tn = T * (1.f - alpha);
        const bool blend = use && Tn >= tmin;
        const float w = blend ? alpha * T : 0.f;
        C0 += G.r * w;
        C1 += G.g * w;
        C2 += G.b * w;
        T = blend ? Tn : T;
        last = blend ? base + k - rg.x + 1 : last;
        if (COUNT) {
          stop = (use && !blend) ? base + k - rg.x + 1 : stop;
          nbl += blend ? 1 : 0;
        }
        lift = (use && !blend) ? __builtin_inff() : lift;
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
  if (COUNT) {
    __shared__ int32_t s_cnt[2];
    store_tile_work(inside ? (stop > 0 ? stop : rg.y - rg.x) : 0, inside ? nbl : 0, s_cnt,
                    tile_work, g);
  }
}

hipError_t launch_render_fwd_gut(const Batch& B, const float* splat, const int32_t* vals,
                                 const int32_t* ranges, const int32_t* order, float* image,
                                 float* Tfin, int32_t* ncon, int32_t* tile_work, hipStream_t st) {
  if (B.total_tiles <= 0) return hipSuccess;
  const float4* sp = reinterpret_cast<const float4*>(splat);
  const int2* rg = reinterpret_cast<const int2*>(ranges);
  const dim3 grid(B.total_tiles);
  if (tile_work) {
    if (B.tile_w == 8)
      hipLaunchKernelGGL((k_render_fwd_gut<8, 8, true>), grid, dim3(64), 0, st, B, sp, vals, rg, image,
                         Tfin, ncon, tile_work, order);
    else if (B.tile_w == 32)
      hipLaunchKernelGGL((k_render_fwd_gut<32, 32, true>), grid, dim3(1024), 0, st, B, sp, vals, rg,
                         image, Tfin, ncon, tile_work, order);
    else
      hipLaunchKernelGGL((k_render_fwd_gut<16, 16, true>), grid, dim3(256), 0, st, B, sp, vals, rg,
                         image, Tfin, ncon, tile_work, order);
    return hipGetLastError();
  }
  if (B.tile_w == 8)
    hipLaunchKernelGGL((k_render_fwd_gut<8, 8>), grid, dim3(64), 0, st, B, sp, vals, rg, image,
                       Tfin, ncon, nullptr, order);
  else if (B.tile_w == 32)
    hipLaunchKernelGGL((k_render_fwd_gut<32, 32>), grid, dim3(1024), 0, st, B, sp, vals, rg,
                       image, Tfin, ncon, nullptr, order);
  else
    hipLaunchKernelGGL((k_render_fwd_gut<16, 16>), grid, dim3(256), 0, st, B, sp, vals, rg,
                       image, Tfin, ncon, nullptr, order);
  return hipGetLastError();
}


// Backward of the 3DGUT compositing. The gradient of each record is taken
// with respect to the 16 values evaluate reads: the adjusted opacity o',
// the colour (3), the canonical ray origin ro (3) and M = S^-1 R^T (9,
// row-major), as grad [record][16] in that order; the derivative with
// respect to M holds the Gaussian's centre fixed (ro = M d moves with M,
// d = M^-1 ro the camera position minus the centre).
//
// Per pixel the blended entries are those at list positions <= n_contrib
// that pass the forward's tests (the forward stops at the first entry it
// would keep but cannot blend, which lies past n_contrib). They are walked
// last first with T recovered as T / (1 - alpha) from T_final and the
// colour behind accumulated, as for 3DGS; every decision (d^2 < 9,
// response > 0.0113, alpha >= alpha_min) is taken in the forward's exact
// arithmetic. With resp = exp(-d^2 / 2), alpha = min(alpha_max, o' resp),
// and dL/dalpha from the blending:
//   dL/do' = resp dL/dalpha,   dL/dd^2 = -alpha dL/dalpha / 2
// (both zero where alpha is clamped). d^2 = |p|^2 for p = ro - t w with
// w = M rd and t = (ro . w) / |w|^2 (p is the canonical offset of the ray's
// closest point from the centre; t is stationary there), so
//   dd^2/dro = 2 p   (M fixed),   dd^2/dM_ab = 2 p_a x_b   (centre fixed)
// with x = d - t rd the world offset of the closest point and p = M x.
// The two parts of the centre-fixed derivative (through w and through ro)
// are each about |d| / |x| larger than their sum, which is why it is formed
// here per pixel, in float64 (x and p; d once per staged record), and not
// from float32 sums later. The rest is float32. Each lane holds its pixel's
// 16 terms; the wave sums them with lane swaps (reduce16) and four lanes
// add them to grad with float atomics.
struct GutBwdRec {
  double m[9];
  double d[3];  // M^-1 ro
  int32_t id;
};

template <int NW>
struct GutBwdStage {
  GutStage<NW> f;  // the forward's staged data, masks and wave lists
  GutBwdRec b[kGutBatch];
};

template <int TW, int TH>
__global__ __launch_bounds__(TW* TH)
__attribute__((amdgpu_waves_per_eu(TW * TH >= 256 ? 5 : 1))) void k_render_bwd_gut(
    Batch B, const float4* __restrict__ splat, const int32_t* __restrict__ vals,
    const int2* __restrict__ ranges, const float* __restrict__ dimg,
    const float* __restrict__ Tfin, const int32_t* __restrict__ ncon, float* __restrict__ grad,
    const int32_t* order) {
  constexpr int NT = TW * TH;
  constexpr int NW = (NT + 63) / 64;
  constexpr int RPW = 64 / TW;
  __shared__ GutBwdStage<NW> S;
  __shared__ int32_t s_maxlast;
  const int g = order ? order[blockIdx.x] : (int)blockIdx.x;
  const ViewDev& V = B.v[view_of_tile(B, g)];
  const int lt = g - V.tile_off;
  const int ty = lt / V.tiles_x, tx = lt - ty * V.tiles_x;
  const int px = tx * TW + (int)(threadIdx.x % TW);
  const int py = ty * TH + (int)(threadIdx.x / TW);
  const bool inside = px < V.W && py < V.H;
  const int2 rg = ranges[g];
  const float amax = B.alpha_max, amin = B.alpha_min;
  const int wv = threadIdx.x >> 6;
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
  const double p00 = rd0 * rd0, p11 = rd1 * rd1, p22 = rd2 * rd2;
  const double p01 = 2.0 * rd0 * rd1, p02 = 2.0 * rd0 * rd2, p12 = 2.0 * rd1 * rd2;
  float T = 1.f, G0 = 0.f, G1 = 0.f, G2 = 0.f;
  int mylast = 0;
  if (inside) {
    const size_t WH = (size_t)V.W * V.H;
    const size_t p = (size_t)py * V.W + px;
    const float* gi = dimg + 3 * (size_t)V.pix_off;
    T = Tfin[(size_t)V.pix_off + p];
    mylast = ncon[(size_t)V.pix_off + p];
    G0 = gi[p];
    G1 = gi[WH + p];
    G2 = gi[2 * WH + p];
  }
  const float TfbG = T * (B.bg[0] * G0 + B.bg[1] * G1 + B.bg[2] * G2);
  float S0 = 0.f, S1 = 0.f, S2 = 0.f;
  if (threadIdx.x == 0) s_maxlast = 0;
  __syncthreads();
  if (mylast > 0) atomicMax(&s_maxlast, mylast);
  __syncthreads();
  const int end = rg.x + min(s_maxlast, rg.y - rg.x);
  int wlast = mylast;
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) wlast = max(wlast, __shfl_xor(wlast, o, 64));
  const int stride = splat_stride4(B);
  for (int hi = end; hi > rg.x; hi -= kGutBatch) {
    const int lo = max(rg.x, hi - kGutBatch);
    const int nb = hi - lo;
    __syncthreads();
    for (int k = threadIdx.x; k < nb; k += NT) {
      const int id = vals[lo + k];
      const float4* q = splat + (size_t)stride * (size_t)id;
      const float4 q1 = q[1], q2 = q[2], q3 = q[3], q4 = q[4], q5 = q[5];
      GutBwdRec& R = S.b[k];
      const double m[9] = {q3.x, q3.y, q3.z, q3.w, q4.x, q4.y, q4.z, q4.w, q5.x};
      const double ro[3] = {q2.y, q2.z, q2.w};
#pragma unroll
      for (int c = 0; c < 9; ++c) R.m[c] = m[c];
      {
        // M^-1 ro by the adjugate (a staged record has det M != 0: its
        // scales are finite and positive)
        const double c00 = m[4] * m[8] - m[5] * m[7], c01 = m[5] * m[6] - m[3] * m[8],
                     c02 = m[3] * m[7] - m[4] * m[6];
        const double idet = 1.0 / (m[0] * c00 + m[1] * c01 + m[2] * c02);
        R.d[0] = (c00 * ro[0] + (m[2] * m[7] - m[1] * m[8]) * ro[1] +
                  (m[1] * m[5] - m[2] * m[4]) * ro[2]) * idet;
        R.d[1] = (c01 * ro[0] + (m[0] * m[8] - m[2] * m[6]) * ro[1] +
                  (m[2] * m[3] - m[0] * m[5]) * ro[2]) * idet;
        R.d[2] = (c02 * ro[0] + (m[1] * m[6] - m[0] * m[7]) * ro[1] +
                  (m[0] * m[4] - m[1] * m[3]) * ro[2]) * idet;
      }
      R.id = id;
      GutRec& G = S.f.rec[k];
#pragma unroll
      for (int c = 0; c < 3; ++c) G.w[c] = m[c] * ro[0] + m[3 + c] * ro[1] + m[6 + c] * ro[2];
      auto mm = [&](int a, int b) { return m[a] * m[b] + m[3 + a] * m[3 + b] + m[6 + a] * m[6 + b]; };
      G.q[0] = mm(0, 0); G.q[1] = mm(1, 1); G.q[2] = mm(2, 2);
      G.q[3] = mm(0, 1); G.q[4] = mm(0, 2); G.q[5] = mm(1, 2);
      G.ro2 = ro[0] * ro[0] + ro[1] * ro[1] + ro[2] * ro[2];
      G.o = q1.y; G.r = q1.z; G.g = q1.w; G.b = q2.x;
      S.f.mask[k] = (typename GutStage<NW>::mask_t)gut_wave_mask(
          __float_as_uint(q5.y), __float_as_uint(q5.z), tx * TW, tx * TW + TW - 1, ty * TH, RPW, NW);
    }
    __syncthreads();
    // this wave's records of the batch within its walk, in list order
    int cnt = 0;
    {
      const int lane = threadIdx.x & 63;
      const uint64_t lt_mask = lanemask_lt();
      const int kmax = wlast + rg.x - lo - 1;
      for (int i0 = 0; i0 < nb; i0 += 64) {
        const int k = i0 + lane;
        const bool hit = k < nb && k <= kmax && ((S.f.mask[k] >> wv) & 1u);
        const uint64_t msk = __ballot(hit);
        if (hit) S.f.list[wv][cnt + __popcll(msk & lt_mask)] = (uint16_t)k;
        cnt += __popcll(msk);
      }
    }
    __syncthreads();
    for (int i = cnt - 1; i >= 0; --i) {
      const int k = S.f.list[wv][i];
      const int pos = lo + k - rg.x + 1;
      const GutRec& G = S.f.rec[k];
      // the forward's arithmetic, operation for operation
      const double dot = G.w[0] * rd0 + G.w[1] * rd1 + G.w[2] * rd2;
      const double nrm = G.q[0] * p00 + G.q[1] * p11 + G.q[2] * p22 + G.q[3] * p01 +
                         G.q[4] * p02 + G.q[5] * p12;
      double rn = __builtin_amdgcn_rcp(nrm);
      rn = fma(rn, fma(-nrm, rn, 1.0), rn);
      rn = fma(rn, fma(-nrm, rn, 1.0), rn);
      const double d2 = fmax(G.ro2 - dot * dot * rn, 0.0);
      const bool near = pos <= mylast && d2 < kGutD2Max;
      if (__ballot(near) == 0) continue;
      const float resp = __builtin_amdgcn_exp2f(-kGutHalfLog2e * (float)d2);
      const float raw = __fmul_rn(G.o, resp);
      float alpha = fminf(amax, raw);
      alpha = (near && resp > kGutValid && alpha >= amin) ? alpha : 0.f;
      if (__ballot(alpha > 0.f) == 0) continue;
      const float inv = __builtin_amdgcn_rcpf(1.f - alpha);
      T = T * inv;
      const float w = alpha * T;
      float X[16];
      X[1] = w * G0;
      X[2] = w * G1;
      X[3] = w * G2;
      const float d0 = G.r - S0, d1 = G.g - S1, dc2 = G.b - S2;
      const float da = T * (d0 * G0 + d1 * G1 + dc2 * G2) - TfbG * inv;
      S0 += alpha * d0;
      S1 += alpha * d1;
      S2 += alpha * dc2;
      const bool unclamped = raw <= amax && alpha > 0.f;
      X[0] = unclamped ? resp * da : 0.f;
      const float dA = unclamped ? alpha * da : 0.f;  // -2 dL/dd^2
      // x = d - t rd and p = M x in float64 (selected, not multiplied, to
      // zero on the lanes that do not use the entry, whose t may not be
      // finite)
      const GutBwdRec& Rb = S.b[k];
      const double t = dot * rn;
      const double x0 = Rb.d[0] - t * rd0, x1 = Rb.d[1] - t * rd1, x2 = Rb.d[2] - t * rd2;
      const float xf0 = unclamped ? (float)x0 : 0.f, xf1 = unclamped ? (float)x1 : 0.f,
                  xf2 = unclamped ? (float)x2 : 0.f;
#pragma unroll
      for (int a = 0; a < 3; ++a) {
        const double pa = Rb.m[3 * a] * x0 + Rb.m[3 * a + 1] * x1 + Rb.m[3 * a + 2] * x2;
        const float qa = unclamped ? -dA * (float)pa : 0.f;  // 2 dL/dd^2 p_a
        X[4 + a] = qa;
        X[7 + 3 * a] = qa * xf0;
        X[8 + 3 * a] = qa * xf1;
        X[9 + 3 * a] = qa * xf2;
      }
      reduce16(X, grad + 16 * (size_t)Rb.id);
    }
  }
}

hipError_t launch_render_bwd_gut(const Batch& B, const float* splat, const int32_t* vals,
                                 const int32_t* ranges, const int32_t* order, const float* dimg,
                                 const float* Tfin, const int32_t* ncon, float* grad,
                                 hipStream_t st) {
  if (B.total_tiles <= 0) return hipSuccess;
  const float4* sp = reinterpret_cast<const float4*>(splat);
  const int2* rg = reinterpret_cast<const int2*>(ranges);
  const dim3 grid(B.total_tiles);
  if (B.tile_w == 8)
    hipLaunchKernelGGL((k_render_bwd_gut<8, 8>), grid, dim3(64), 0, st, B, sp, vals, rg, dimg,
                       Tfin, ncon, grad, order);
  else if (B.tile_w == 32)
    hipLaunchKernelGGL((k_render_bwd_gut<32, 32>), grid, dim3(1024), 0, st, B, sp, vals, rg,
                       dimg, Tfin, ncon, grad, order);
  else
    hipLaunchKernelGGL((k_render_bwd_gut<16, 16>), grid, dim3(256), 0, st, B, sp, vals, rg, dimg,
                       Tfin, ncon, grad, order);
  return hipGetLastError();
}

}  // namespace xpr
