// Forward compositing of LinPrim: Algorithm 1 of the paper with the
// evaluate of the listing "Implementation of XPR-LinPrim".
//
// One workgroup per tile, one thread per pixel (256 threads for 16x16
// tiles, 64 for 8x8, 1024 for 32x32). For pixel (x, y) the offset from the record's
// projected centre is (dx, dy) = (x + 1/2 - mu_2D) = (x - u, y - v). The
// octahedron is the intersection of the slabs |n_i . (dx, dy, tau)| <= 1,
// n_i = c0 +- c1 +- c2 (c_k the rows of A^-1): slab i holds
// tau in [m_i - h_i, m_i + h_i] with m_i = -(n_ix dx + n_iy dy) / n_iz and
// h_i = 1 / |n_iz|, so the ray's chord is min_i (m_i + h_i) -
// max_i (m_i - h_i) when positive; a slab with |n_iz| < 1e-10 does not
// bound tau and excludes the pixel when |n_ix dx + n_iy dy| > 1. The slope
// coefficients -n_ix / n_iz, -n_iy / n_iz and h_i are formed in float64
// once per staged record, the chord per pixel in float64 (anisotropic
// octahedra make the float32 chord lose ~1e-5 of alpha), Beer-Lambert
// alpha = 1 - exp(-sigma chord) and the gates, stop rule and blending of the
// 3DGS path in float32.
//
// Per-wave lists: the footprint lies in |dx| <= ex, |dy| <= ey (the
// projected vertices of the octahedron), so each staged record gets the
// mask of the waves whose pixel rows meet that box (widened by 0.05 px) and
// each wave walks only its records, in list order.
#include "xpr_internal.h"

namespace xpr {

constexpr int kLinBatch = 128;
constexpr float kLog2eLin = 1.4426950408889634f;

struct LinRec {
  double a[4], b[4], h[4];  // m_i = a_i dx + b_i dy; h_i < 0 marks a slab with n_z ~ 0
  double u, v;
  float sigma, r, g, bl;
  int32_t flat, pad;  // flat: some slab has n_z ~ 0 (the general chord below)
};

template <int NW>
struct LinStage {
  LinRec rec[kLinBatch];
  // one bit per wave: 4 waves at 16x16 tiles, 16 at 32x32
  using mask_t = std::conditional_t<(NW > 8), uint16_t, uint8_t>;
  mask_t mask[kLinBatch];
  uint16_t list[NW][kLinBatch];
};

// With COUNT the tile also counts the definition's work into tile_work
// [g][2]: per pixel the entries evaluated (up to and including the one that
// stops it, else the whole list) and the entries blended.
template <int TW, int TH, bool COUNT = false>
__global__ __launch_bounds__(TW* TH) void k_render_fwd_lin(
    Batch B, const float4* __restrict__ splat, const int32_t* __restrict__ vals,
    const int2* __restrict__ ranges, float* __restrict__ image, float* __restrict__ Tfin,
    int32_t* __restrict__ ncon, int32_t* __restrict__ tile_work, const int32_t* order) {
  constexpr int NT = TW * TH;
  constexpr int NW = (NT + 63) / 64;
  constexpr int RPW = 64 / TW;  // pixel rows per wave
  __shared__ LinStage<NW> S;
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
  const double fpx = (double)px, fpy = (double)py;
  float T = 1.f, C0 = 0.f, C1 = 0.f, C2 = 0.f;
  int last = 0;
  int stop = 0, nbl = 0;  // COUNT only
  // a finished pixel (or one outside the image) carries lift = +inf, which
  // fails every later test; kept in a vector register (a carried boolean
  // becomes a lane mask updated by scalar instructions on every record)
  float lift = inside ? 0.f : __builtin_inff();
  const int stride = splat_stride4(B);
  const int x0 = tx * TW, x1 = tx * TW + TW - 1, y0 = ty * TH;
  for (int base = rg.x; base < rg.y; base += kLinBatch) {
    if (__syncthreads_count(lift == 0.f) == 0) break;
    const int nb = min(kLinBatch, rg.y - base);
    for (int k = threadIdx.x; k < nb; k += NT) {
      const float4* q = splat + (size_t)stride * (size_t)vals[base + k];
      const float4 q0 = q[0], q1 = q[1], q2 = q[2], q3 = q[3], q4 = q[4];
      const double c[9] = {q2.x, q2.y, q2.z, q2.w, q3.x, q3.y, q3.z, q3.w, q4.x};
      LinRec& L = S.rec[k];
      int flat_any = 0;
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const double e1 = (i & 2) ? -1.0 : 1.0, e2 = (i & 1) ? -1.0 : 1.0;
        const double nx = c[0] + e1 * c[3] + e2 * c[6];
        const double ny = c[1] + e1 * c[4] + e2 * c[7];
        const double nz = c[2] + e1 * c[5] + e2 * c[8];
        const bool flat = !(fabs(nz) >= 1e-10);
        L.a[i] = flat ? nx : -nx / nz;
        L.b[i] = flat ? ny : -ny / nz;
        L.h[i] = flat ? -1.0 : 1.0 / fabs(nz);
        flat_any |= flat ? 1 : 0;
      }
      L.flat = flat_any;
      L.u = q0.x;
      L.v = q0.y;
      L.sigma = q0.z;
      L.r = q0.w;
      L.g = q1.x;
      L.bl = q1.y;
      // waves whose pixel rows meet the footprint box
      const double ex = (double)q1.z + 0.05, ey = (double)q1.w + 0.05;
      uint32_t msk = 0u;
      if (L.u + ex >= (double)x0 && L.u - ex <= (double)x1) {
        for (int w = 0; w < NW; ++w) {
          const double r0 = (double)(y0 + w * RPW), r1 = r0 + (double)(RPW - 1);
          if (L.v + ey >= r0 && L.v - ey <= r1) msk |= 1u << w;
        }
      }
      S.mask[k] = (typename LinStage<NW>::mask_t)msk;
    }
    __syncthreads();
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
        const LinRec& L = S.rec[k];
        const double dx = fpx - L.u, dy = fpy - L.v;
        double chord;
        if (!L.flat) {  // one record per wave step: a uniform branch
          double m = L.a[0] * dx + L.b[0] * dy;
          double enter = m - L.h[0], exit_ = m + L.h[0];
#pragma unroll
          for (int j = 1; j < 4; ++j) {
            m = L.a[j] * dx + L.b[j] * dy;
            enter = fmax(enter, m - L.h[j]);
            exit_ = fmin(exit_, m + L.h[j]);
          }
          chord = exit_ - enter;
        } else {
          double enter = -INFINITY, exit_ = INFINITY;
          bool miss = false;
#pragma unroll
          for (int j = 0; j < 4; ++j) {
            const double m = L.a[j] * dx + L.b[j] * dy, h = L.h[j];
            const bool fl = h < 0.0;
            enter = fl ? enter : fmax(enter, m - h);
            exit_ = fl ? exit_ : fmin(exit_, m + h);
            miss = miss || (fl && fabs(m) > 1.0);
          }
          chord = miss ? -1.0 : exit_ - enter;
        }
        const bool hitp = chord - (double)lift > 0.0;
        if (__ballot(hitp) == 0) continue;
        const float alpha =
            fminf(amax, 1.f - __builtin_amdgcn_exp2f(-L.sigma * kLog2eLin * (float)chord));
        const bool use = hitp && alpha >= amin;
        const float Tn = T * (1.f - alpha);
        const bool blend = use && Tn >= tmin;
        const float w = blend ? alpha * T : 0.f;
        C0 += L.r * w;
        C1 += L.g * w;
        C2 += L.bl * w;
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

hipError_t launch_render_fwd_lin(const Batch& B, const float* splat, const int32_t* vals,
                                 const int32_t* ranges, const int32_t* order, float* image,
                                 float* Tfin, int32_t* ncon, int32_t* tile_work, hipStream_t st) {
  if (B.total_tiles <= 0) return hipSuccess;
  const float4* sp = reinterpret_cast<const float4*>(splat);
  const int2* rg = reinterpret_cast<const int2*>(ranges);
  const dim3 grid(B.total_tiles);
  if (tile_work) {
    if (B.tile_w == 8)
      hipLaunchKernelGGL((k_render_fwd_lin<8, 8, true>), grid, dim3(64), 0, st, B, sp, vals, rg, image,
                         Tfin, ncon, tile_work, order);
    else if (B.tile_w == 32)
      hipLaunchKernelGGL((k_render_fwd_lin<32, 32, true>), grid, dim3(1024), 0, st, B, sp, vals, rg,
                         image, Tfin, ncon, tile_work, order);
    else
      hipLaunchKernelGGL((k_render_fwd_lin<16, 16, true>), grid, dim3(256), 0, st, B, sp, vals, rg,
                         image, Tfin, ncon, tile_work, order);
    return hipGetLastError();
  }
  if (B.tile_w == 8)
    hipLaunchKernelGGL((k_render_fwd_lin<8, 8>), grid, dim3(64), 0, st, B, sp, vals, rg, image,
                       Tfin, ncon, nullptr, order);
  else if (B.tile_w == 32)
    hipLaunchKernelGGL((k_render_fwd_lin<32, 32>), grid, dim3(1024), 0, st, B, sp, vals, rg,
                       image, Tfin, ncon, nullptr, order);
  else
    hipLaunchKernelGGL((k_render_fwd_lin<16, 16>), grid, dim3(256), 0, st, B, sp, vals, rg,
                       image, Tfin, ncon, nullptr, order);
  return hipGetLastError();
}


// Backward of the LinPrim compositing. The gradient of each record is taken
// with respect to the 15 values evaluate reads -- u, v (mu_2D - 1/2),
// sigma, the colour (3) and the rows c0, c1, c2 of A^-1 (9) -- as grad
// [record][16] with the 16th left zero.
//
// Per pixel the blended entries are those at list positions <= n_contrib
// whose chord is positive and alpha >= alpha_min (the forward's exact
// arithmetic decides); they are walked last first with T recovered as
// T / (1 - alpha) and the colour behind accumulated, as for 3DGS. With
// e = exp(-sigma chord) (alpha = 1 - e when not clamped):
//   dL/dsigma = e chord dL/dalpha,   dL/dchord = e sigma dL/dalpha.
// The chord is (m_b + h_b) - (m_a - h_a) for the exit slab b (the first
// reaching the minimum of m_i + h_i) and the entry slab a (the first
// reaching the maximum of m_i - h_i), m_i = -(n_ix dx + n_iy dy) / n_iz,
// h_i = 1 / |n_iz|. With s_i = 1 / n_iz and kappa = +1 (exit), -1 (entry):
//   dchord/dn_i = (-kappa dx s_i, -kappa dy s_i, -s_i (kappa m_i + h_i)),
//   dchord/du = -kappa (-n_ix s_i), likewise v,
// and n_i = c0 + e1 c1 + e2 c2 spreads dL/dn_i to the rows. These terms are
// formed in float64 (with dx, dy, m as the forward forms them), the rest
// in float32; each wave sums its lanes' 16 terms with lane swaps
// (reduce16) and four lanes add them to grad with float atomics.
struct LinBwdRec {
  double s[4];  // 1 / n_iz (0 for a slab with n_z ~ 0)
  int32_t id;
};

template <int NW>
struct LinBwdStage {
  LinStage<NW> f;  // the forward's staged data, masks and wave lists
  LinBwdRec b[kLinBatch];
};

template <int TW, int TH>
__global__ __launch_bounds__(TW* TH) void k_render_bwd_lin(
    Batch B, const float4* __restrict__ splat, const int32_t* __restrict__ vals,
    const int2* __restrict__ ranges, const float* __restrict__ dimg,
    const float* __restrict__ Tfin, const int32_t* __restrict__ ncon, float* __restrict__ grad,
    const int32_t* order) {
  constexpr int NT = TW * TH;
  constexpr int NW = (NT + 63) / 64;
  constexpr int RPW = 64 / TW;
  __shared__ LinBwdStage<NW> S;
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
  const double fpx = (double)px, fpy = (double)py;
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
  const int x0 = tx * TW, x1 = tx * TW + TW - 1, y0 = ty * TH;
  for (int hi = end; hi > rg.x; hi -= kLinBatch) {
    const int lo = max(rg.x, hi - kLinBatch);
    const int nb = hi - lo;
    __syncthreads();
    for (int k = threadIdx.x; k < nb; k += NT) {
      const int id = vals[lo + k];
      const float4* q = splat + (size_t)stride * (size_t)id;
      const float4 q0 = q[0], q1 = q[1], q2 = q[2], q3 = q[3], q4 = q[4];
      const double c[9] = {q2.x, q2.y, q2.z, q2.w, q3.x, q3.y, q3.z, q3.w, q4.x};
      LinRec& L = S.f.rec[k];
      LinBwdRec& Lb = S.b[k];
      int flat_any = 0;
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const double e1 = (i & 2) ? -1.0 : 1.0, e2 = (i & 1) ? -1.0 : 1.0;
        const double nx = c[0] + e1 * c[3] + e2 * c[6];
        const double ny = c[1] + e1 * c[4] + e2 * c[7];
        const double nz = c[2] + e1 * c[5] + e2 * c[8];
        const bool flat = !(fabs(nz) >= 1e-10);
        L.a[i] = flat ? nx : -nx / nz;
        L.b[i] = flat ? ny : -ny / nz;
        L.h[i] = flat ? -1.0 : 1.0 / fabs(nz);
        Lb.s[i] = flat ? 0.0 : 1.0 / nz;
        flat_any |= flat ? 1 : 0;
      }
      L.flat = flat_any;
      L.u = q0.x;
      L.v = q0.y;
      L.sigma = q0.z;
      L.r = q0.w;
      L.g = q1.x;
      L.bl = q1.y;
      Lb.id = id;
      const double ex = (double)q1.z + 0.05, ey = (double)q1.w + 0.05;
      uint32_t msk = 0u;
      if (L.u + ex >= (double)x0 && L.u - ex <= (double)x1) {
        for (int w = 0; w < NW; ++w) {
          const double r0 = (double)(y0 + w * RPW), r1 = r0 + (double)(RPW - 1);
          if (L.v + ey >= r0 && L.v - ey <= r1) msk |= 1u << w;
        }
      }
      S.f.mask[k] = (typename LinStage<NW>::mask_t)msk;
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
      if (__ballot(pos <= mylast) == 0) continue;
      const LinRec& L = S.f.rec[k];
      // the forward's chord, operation for operation, with the bounding slabs
      const double dx = fpx - L.u, dy = fpy - L.v;
      double chord;
      int ia = 0, ib = 0;
      if (!L.flat) {
        double m = L.a[0] * dx + L.b[0] * dy;
        double enter = m - L.h[0], exit_ = m + L.h[0];
#pragma unroll
        for (int j = 1; j < 4; ++j) {
          m = L.a[j] * dx + L.b[j] * dy;
          const double en = m - L.h[j], xn = m + L.h[j];
          ia = en > enter ? j : ia;
          ib = xn < exit_ ? j : ib;
          enter = fmax(enter, en);
          exit_ = fmin(exit_, xn);
        }
        chord = exit_ - enter;
      } else {
        double enter = -INFINITY, exit_ = INFINITY;
        bool miss = false;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          const double m = L.a[j] * dx + L.b[j] * dy, h = L.h[j];
          const bool fl = h < 0.0;
          ia = (!fl && m - h > enter) ? j : ia;
          ib = (!fl && m + h < exit_) ? j : ib;
          enter = fl ? enter : fmax(enter, m - h);
          exit_ = fl ? exit_ : fmin(exit_, m + h);
          miss = miss || (fl && fabs(m) > 1.0);
        }
        chord = miss ? -1.0 : exit_ - enter;
      }
      const bool hitp = pos <= mylast && chord > 0.0;
      if (__ballot(hitp) == 0) continue;
      const float ef = __builtin_amdgcn_exp2f(-L.sigma * kLog2eLin * (float)chord);
      const float raw = 1.f - ef;
      float alpha = fminf(amax, raw);
      alpha = (hitp && alpha >= amin) ? alpha : 0.f;
      if (__ballot(alpha > 0.f) == 0) continue;
      const float inv = __builtin_amdgcn_rcpf(1.f - alpha);
      T = T * inv;
      const float w = alpha * T;
      float X[16];
      X[3] = w * G0;
      X[4] = w * G1;
      X[5] = w * G2;
      X[15] = 0.f;
      const float d0 = L.r - S0, d1 = L.g - S1, dc2 = L.bl - S2;
      const float da = T * (d0 * G0 + d1 * G1 + dc2 * G2) - TfbG * inv;
      S0 += alpha * d0;
      S1 += alpha * d1;
      S2 += alpha * dc2;
      const bool unclamped = raw <= amax && alpha > 0.f;
      const float ed = unclamped ? ef * da : 0.f;
      X[2] = unclamped ? ed * (float)chord : 0.f;
      // dL/dchord, then through the exit (kappa = +1) and entry (-1) slabs
      const double dch = (double)(ed * L.sigma);
      const LinBwdRec& Lb = S.b[k];
      double gn[3] = {0.0, 0.0, 0.0}, gc1[3] = {0.0, 0.0, 0.0}, gc2[3] = {0.0, 0.0, 0.0};
      double gu = 0.0, gv = 0.0;
#pragma unroll
      for (int side = 0; side < 2; ++side) {
        const int j = side == 0 ? ib : ia;
        const double kap = side == 0 ? 1.0 : -1.0;
        const double sj = Lb.s[j];
        const double mj = L.a[j] * dx + L.b[j] * dy;
        const double t0 = -kap * dx * sj * dch, t1 = -kap * dy * sj * dch,
                     t2 = -sj * (kap * mj + L.h[j]) * dch;
        const double e1 = (j & 2) ? -1.0 : 1.0, e2 = (j & 1) ? -1.0 : 1.0;
        gn[0] += t0; gn[1] += t1; gn[2] += t2;
        gc1[0] += e1 * t0; gc1[1] += e1 * t1; gc1[2] += e1 * t2;
        gc2[0] += e2 * t0; gc2[1] += e2 * t1; gc2[2] += e2 * t2;
        // m_j = a_j dx + b_j dy with dx = x - u
        gu -= kap * L.a[j] * dch;
        gv -= kap * L.b[j] * dch;
      }
      // lanes not using the entry select zeros (their chord may be -1)
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        X[6 + c] = unclamped ? (float)gn[c] : 0.f;
        X[9 + c] = unclamped ? (float)gc1[c] : 0.f;
        X[12 + c] = unclamped ? (float)gc2[c] : 0.f;
      }
      X[0] = unclamped ? (float)gu : 0.f;
      X[1] = unclamped ? (float)gv : 0.f;
      reduce16(X, grad + 16 * (size_t)Lb.id);
    }
  }
}

hipError_t launch_render_bwd_lin(const Batch& B, const float* splat, const int32_t* vals,
                                 const int32_t* ranges, const int32_t* order, const float* dimg,
                                 const float* Tfin, const int32_t* ncon, float* grad,
                                 hipStream_t st) {
  if (B.total_tiles <= 0) return hipSuccess;
  const float4* sp = reinterpret_cast<const float4*>(splat);
  const int2* rg = reinterpret_cast<const int2*>(ranges);
  const dim3 grid(B.total_tiles);
  if (B.tile_w == 8)
    hipLaunchKernelGGL((k_render_bwd_lin<8, 8>), grid, dim3(64), 0, st, B, sp, vals, rg, dimg,
                       Tfin, ncon, grad, order);
  else if (B.tile_w == 32)
    hipLaunchKernelGGL((k_render_bwd_lin<32, 32>), grid, dim3(1024), 0, st, B, sp, vals, rg,
                       dimg, Tfin, ncon, grad, order);
  else
    hipLaunchKernelGGL((k_render_bwd_lin<16, 16>), grid, dim3(256), 0, st, B, sp, vals, rg, dimg,
                       Tfin, ncon, grad, order);
  return hipGetLastError();
}

}  // namespace xpr
