// Per-pixel compositing (Algorithm 1 of the paper with the 3DGS evaluate of
// the listing "Implementation of XPR-3DGS") and its backward.
//
// One workgroup per tile. Each thread owns PPT vertically adjacent pixels of
// its tile column (a 16x16 tile is 256/PPT threads: four wave64s at PPT=1,
// one wave64 covering the whole tile at PPT=4; an 8x8 tile is one wave64 at
// PPT=1, a 32x32 tile four wave64s of 8 rows at PPT=4). The tile's
// depth-sorted list is walked in batches of BATCH splat records staged in
// LDS; every thread reads each record once (an LDS broadcast) and applies it
// to its PPT pixels, so LDS reads, loop control and, in the backward, the cross-lane
// gradient reduction are shared by PPT pixel evaluations. The workgroup
// leaves the loop as soon as no pixel is still active, checked once per batch
// (the batch-boundary exit check of Algorithm 1). The loop body is plain FP32
// VALU work: the kernels are bound by VALU issue, not by memory.
#include <algorithm>

#include "xpr_internal.h"

namespace xpr {

// Records are staged in LDS with the conic scaled by log2(e), so the power
// comes out in base-2 units and alpha = min(alpha_max, o 2^P2) needs no
// extra multiply, and with a per-record power threshold
//   thr = log2(alpha_min / o) - 2^-10,
// below which o 2^P2 < alpha_min holds with a wide margin over the rounding
// of exp2 and of the product: such pairs are skipped before exp2 is taken
// (whole waves skip it when all their lanes are below). Every pair at or
// above thr takes the exact test, so the accept decisions are the ones the
// plain alpha < alpha_min gate takes on the same P2. Staged layout:
//   s0 = (u, v, A', B'), s1 = (C', thr, o, red), s2 = (green, blue).
constexpr float kLog2e = 1.4426950408889634f;
constexpr float kLn2 = 0.6931471805599453f;
constexpr float kThrMargin = 1.0f / 1024.0f;

__device__ __forceinline__ void stage_record(const float4* __restrict__ splat, size_t r,
                                             float alpha_min, float4& o0, float4& o1,
                                             float2& o2) {
  const float4 p0 = splat[3 * r];
  const float4 p1 = splat[3 * r + 1];
  const float p2 = splat[3 * r + 2].x;
  o0 = make_float4(p0.x, p0.y, p0.z * kLog2e, p0.w * kLog2e);
  o1 = make_float4(p1.x * kLog2e, __log2f(alpha_min / p1.y) - kThrMargin, p1.y, p1.z);
  o2 = make_float2(p1.w, p2);
}

// The evaluate of the listing on the staged record: power P2 = A' dx^2 +
// B' dx dy + C' dy^2 (base 2), written with explicit roundings so the
// forward and backward kernels take bit-identical decisions.
__device__ __forceinline__ float power2(float dx, float dy, float4 a, float c) {
  return __fmaf_rn(a.z, __fmul_rn(dx, dx),
                   __fmaf_rn(a.w, __fmul_rn(dx, dy), __fmul_rn(c, __fmul_rn(dy, dy))));
}

// Per-wave record lists. A record can only pass its threshold test at
// pixels inside a box around its centre: for a negative definite base-2
// power P2 = A' dx^2 + B' dx dy + C' dy^2, P2 >= thr (thr < 0) implies
//   dx^2 <= thr / (A' - B'^2 / (4 C')),   dy^2 <= thr / (C' - B'^2 / (4 A')).
// Each staged record gets a mask of the waves whose pixel rectangle meets
// that box (computed in FP64 and widened by 1% + 0.05 px, far beyond the
// rounding of the FP32 power; near-singular conics get every wave) and on
// which the power's maximum reaches the threshold: P2 is concave, so its
// maximum over the rectangle (dx in [X0, X1], dy in [Y0, Y1]) is 0 when the
// centre lies inside, else the largest of the four edge maxima, each a
// one-variable quadratic maximised at its clamped vertex (dy = -B' dx /
// (2 C') on an edge of fixed dx, likewise dx). The comparison allows
// 1e-5 S + 1e-6 below the threshold, S the largest sum of the power's
// absolute terms over the rectangle, against an FP32 evaluation error of
// about 1e-6 S. Each wave walks only its own records, in list order. The
// per-lane threshold test still decides every pair, so this only skips
// (wave, record) iterations in which no lane could pass.
template <int BATCH, int NW>
struct Stage {
  float4 s0[BATCH];
  float4 s1[BATCH];
  float2 s2[BATCH];
  uint8_t mask[BATCH];
  uint16_t list[NW][BATCH];
  int32_t rec[BATCH];
};

__device__ __forceinline__ uint32_t wave_mask(float4 a, float4 b, int x0, int x1, int y0, int rpw,
                                              int nw) {
  const uint32_t all = (1u << nw) - 1u;
  const double A = a.z, Bc = a.w, C = b.x, thr = b.y;
  if (thr >= 0.0) return 0u;  // o < alpha_min: no pixel can pass
  if (!(thr < 0.0) || !(A < 0.0) || !(C < 0.0)) return all;
  const double det4 = 4.0 * A * C - Bc * Bc;
  if (!(det4 > 1e-3 * 4.0 * A * C)) return all;
  // two divisions per record; the vertices below use their reciprocals
  // (a rounding of ~1e-16 relative in a vertex moves the edge maximum by a
  // second-order amount, far inside the 1e-6 margin)
  const double idet = 1.0 / det4, i4ac = 1.0 / (4.0 * A * C);
  const double ex = sqrt(thr * 4.0 * C * idet) * 1.01 + 0.05;
  const double ey = sqrt(thr * 4.0 * A * idet) * 1.01 + 0.05;
  if (!(a.x + ex >= (double)x0 && a.x - ex <= (double)x1)) return 0u;
  const double X0 = (double)x0 - (double)a.x, X1 = (double)x1 - (double)a.x;
  const double mx = fmax(fabs(X0), fabs(X1));
  auto pw = [&](double dx, double dy) { return A * dx * dx + Bc * dx * dy + C * dy * dy; };
  // vertex of the power along an edge of fixed dx: dy = -B' dx / (2 C')
  // (likewise dx = -B' dy / (2 A')), before clamping to the wave's rows
  const double kc = -Bc * (2.0 * A) * i4ac, ka = -Bc * (2.0 * C) * i4ac;
  const double va = X0 * kc, vb = X1 * kc;
  uint32_t m = 0u;
  for (int w = 0; w < nw; ++w) {
    const double r0 = (double)(y0 + w * rpw), r1 = r0 + (double)(rpw - 1);
    if (!(a.y + ey >= r0 && a.y - ey <= r1)) continue;
    const double Y0 = r0 - (double)a.y, Y1 = r1 - (double)a.y;
    double best;
    if (X0 <= 0.0 && X1 >= 0.0 && Y0 <= 0.0 && Y1 >= 0.0) {
      best = 0.0;
    } else {
      const double ya = fmin(Y1, fmax(Y0, va));
      const double yb = fmin(Y1, fmax(Y0, vb));
      const double xa = fmin(X1, fmax(X0, Y0 * ka));
      const double xb = fmin(X1, fmax(X0, Y1 * ka));
      best = fmax(fmax(pw(X0, ya), pw(X1, yb)), fmax(pw(xa, Y0), pw(xb, Y1)));
    }
    const double my = fmax(fabs(Y0), fabs(Y1));
    const double S = -A * mx * mx + fabs(Bc) * mx * my - C * my * my;
    if (best >= thr - (1e-5 * S + 1e-6)) m |= 1u << w;
  }
  return m;
}

// Builds this wave's ordered list of the staged records [0, nb) whose mask
// has the wave's bit (and, for the backward, whose list position is within
// the wave's walk); returns its length.
template <int BATCH, int NW>
__device__ __forceinline__ int build_wave_list(Stage<BATCH, NW>& S, int nb, int wv,
                                               int max_k) {
  const int lane = threadIdx.x & 63;
  const uint64_t lt = lanemask_lt();
  int cnt = 0;
  for (int i0 = 0; i0 < nb; i0 += 64) {
    const int k = i0 + lane;
    const bool hit = k < nb && k <= max_k && ((S.mask[k] >> wv) & 1u);
    const uint64_t m = __ballot(hit);
    if (hit) S.list[wv][cnt + __popcll(m & lt)] = (uint16_t)k;
    cnt += __popcll(m);
  }
  return cnt;
}

// With COUNT the tile also counts the work the definition performs: per
// pixel the list entries it evaluates (up to and including the one that
// stops it, else the whole list) and the entries it blends, summed over the
// tile's pixels into tile_work [g][2] (s_cnt: two ints of LDS).
template <int TW, int TH, int BATCH, int PPT, bool COUNT>
__device__ __forceinline__ void fwd_tile(const Batch& B, int g, const float4* __restrict__ splat,
                                         const int32_t* __restrict__ vals,
                                         const int2* __restrict__ ranges,
                                         float* __restrict__ image, float* __restrict__ Tfin,
                                         int32_t* __restrict__ ncon,
                                         int32_t* __restrict__ tile_work,
                                         Stage<BATCH, (TW * TH / PPT + 63) / 64>& S,
                                         int32_t* s_cnt) {
  constexpr int NT = TW * TH / PPT;
  constexpr int NW = (NT + 63) / 64;
  constexpr int RPW = 64 * PPT / TW;  // pixel rows per wave
  const ViewDev& V = B.v[view_of_tile(B, g)];
  const int lt = g - V.tile_off;
  const int ty = lt / V.tiles_x, tx = lt - ty * V.tiles_x;
  const int px = tx * TW + (int)(threadIdx.x % TW);
  const int py0 = ty * TH + (int)(threadIdx.x / TW) * PPT;
  const int2 rg = ranges[g];
  const float fpx = (float)px;
  const float amax = B.alpha_max, amin = B.alpha_min, tmin = B.t_min;
  float T[PPT], C0[PPT], C1[PPT], C2[PPT], lift[PPT];
  int last[PPT];
  int stop[PPT], nbl[PPT];  // COUNT only: stopping position, entries blended
  int nalive = 0;
#pragma unroll
  for (int j = 0; j < PPT; ++j) {
    T[j] = 1.f;
    C0[j] = C1[j] = C2[j] = 0.f;
    last[j] = 0;
    stop[j] = nbl[j] = 0;
    const bool inside = px < V.W && py0 + j < V.H;
    lift[j] = inside ? 0.f : __builtin_inff();
  }
  for (int base = rg.x; base < rg.y; base += BATCH) {
    nalive = 0;
#pragma unroll
    for (int j = 0; j < PPT; ++j) nalive += lift[j] == 0.f ? 1 : 0;
    if (__syncthreads_count(nalive > 0) == 0) break;
    for (int k = threadIdx.x; k < BATCH; k += NT) {
      const int idx = base + k;
      if (idx < rg.y) {
        stage_record(splat, (size_t)vals[idx], amin, S.s0[k], S.s1[k], S.s2[k]);
        S.mask[k] = (uint8_t)wave_mask(S.s0[k], S.s1[k], tx * TW, tx * TW + TW - 1, ty * TH, RPW,
                                       NW);
      }
    }
    __syncthreads();
    // The walk over the batch is branch-free per lane: a lane's decisions
    // become selects, and only wave-uniform conditions branch (all lanes
    // finished; no lane at or above the record's power threshold).
    // Divergent branches would cost a scalar exec-mask sequence per
    // condition per record, and the scalar unit has no more issue slots
    // than the vector unit. A finished pixel adds +inf to every record's
    // threshold (a live one adds 0), so it never passes the test again.
    const int nb = min(BATCH, rg.y - base);
    const int wv = threadIdx.x >> 6;
    const int cnt = build_wave_list(S, nb, wv, BATCH);
    __syncthreads();
    for (int i0 = 0; i0 < cnt; i0 += 8) {
      bool alive = false;
#pragma unroll
      for (int j = 0; j < PPT; ++j) alive = alive || lift[j] == 0.f;
      if (__ballot(alive) == 0) break;
      const int iend = min(i0 + 8, cnt);
      for (int i = i0; i < iend; ++i) {
        const int k = S.list[wv][i];
        const float4 a = S.s0[k];
        const float4 b = S.s1[k];
        const float dx = __fsub_rn(fpx, a.x);
        float P2[PPT];
        bool anyp = false;
#pragma unroll
        for (int j = 0; j < PPT; ++j) {
          P2[j] = power2(dx, __fsub_rn((float)(py0 + j), a.y), a, b.x);
          anyp = anyp || P2[j] >= b.y + lift[j];
        }
        if (__ballot(anyp) == 0) continue;
        const float2 gb = S.s2[k];
        const int idx = base + k - rg.x + 1;
#pragma unroll
        for (int j = 0; j < PPT; ++j) {
          // finished pixels and P2 > 0 get alpha 0, which fails alpha >= amin
          float alpha = fminf(amax, __fmul_rn(b.z, __builtin_amdgcn_exp2f(P2[j])));
          alpha = P2[j] + lift[j] > 0.f ? 0.f : alpha;
          const bool use = alpha >= amin;
          const float Tn = T[j] * (1.f - alpha);
          const bool blend = use && Tn >= tmin;
          const float w = blend ? alpha * T[j] : 0.f;
          C0[j] += b.w * w;
          C1[j] += gb.x * w;
          C2[j] += gb.y * w;
          T[j] = blend ? Tn : T[j];
          last[j] = blend ? idx : last[j];
          if (COUNT) {
            stop[j] = (use && !blend) ? idx : stop[j];
            nbl[j] += blend ? 1 : 0;
          }
          lift[j] = (use && !blend) ? __builtin_inff() : lift[j];
        }
      }
    }
  }
  const size_t WH = (size_t)V.W * V.H;
  float* img = image + 3 * (size_t)V.pix_off;
#pragma unroll
  for (int j = 0; j < PPT; ++j) {
    const int py = py0 + j;
    if (px < V.W && py < V.H) {
      const size_t p = (size_t)py * V.W + px;
      img[p] = C0[j] + T[j] * B.bg[0];
      img[WH + p] = C1[j] + T[j] * B.bg[1];
      img[2 * WH + p] = C2[j] + T[j] * B.bg[2];
      Tfin[(size_t)V.pix_off + p] = T[j];
      ncon[(size_t)V.pix_off + p] = last[j];
    }
  }
  if (COUNT) {
    int ev = 0, bl = 0;
#pragma unroll
    for (int j = 0; j < PPT; ++j) {
      if (px < V.W && py0 + j < V.H) {
        ev += stop[j] > 0 ? stop[j] : rg.y - rg.x;
        bl += nbl[j];
      }
    }
    store_tile_work(ev, bl, s_cnt, tile_work, g);
  }
}

// Tile scheduling: with PERSIST the grid is sized to the device and each
// workgroup takes the next tile of ``order`` from an atomic counter until
// the list is exhausted; otherwise workgroup b renders order[b] (or tile b).
__device__ __forceinline__ int next_tile(int* s_next, int32_t* qhead) {
  __syncthreads();
  if (threadIdx.x == 0) *s_next = atomicAdd(qhead, 1);
  __syncthreads();
  return *s_next;
}

template <int TW, int TH, int BATCH, int PPT, bool PERSIST, bool COUNT = false>
__global__ __launch_bounds__(TW* TH / PPT) void k_render_fwd(
    Batch B, const float4* __restrict__ splat, const int32_t* __restrict__ vals,
    const int2* __restrict__ ranges, float* __restrict__ image, float* __restrict__ Tfin,
    int32_t* __restrict__ ncon, int32_t* __restrict__ tile_work, const int32_t* order,
    int32_t* qhead) {
  __shared__ Stage<BATCH, (TW * TH / PPT + 63) / 64> S;
  __shared__ int32_t s_cnt[2];
  if (!PERSIST) {
    const int g = order ? order[blockIdx.x] : (int)blockIdx.x;
    fwd_tile<TW, TH, BATCH, PPT, COUNT>(B, g, splat, vals, ranges, image, Tfin, ncon, tile_work,
                                        S, s_cnt);
    return;
  }
  __shared__ int s_next;
  for (int q = next_tile(&s_next, qhead); q < B.total_tiles; q = next_tile(&s_next, qhead))
    fwd_tile<TW, TH, BATCH, PPT, COUNT>(B, order[q], splat, vals, ranges, image, Tfin, ncon,
                                        tile_work, S, s_cnt);
}

// Backward of the compositing. Each pixel walks its list in reverse from
// its last blended entry, recovering T_i = T_{i+1} / (1 - a_i) and the
// colour behind S_i, and forms
//   dL/dc_i = a_i T_i G,  dL/da_i = T_i (c_i - S_i).G - T_final (bg.G)/(1 - a_i)
//   dL/do = e^P dL/da, dL/dP = a dL/da (zero when a is clamped)
//   dL/du = -dL/dP (2A dx + B dy), dL/dv = -dL/dP (2C dy + B dx),
//   dL/d(A, B, C) = dL/dP (dx^2, dx dy, dy^2).
// Each lane first sums the nine values over its PPT pixels; the wave then
// sums them over its lanes with DPP and one lane adds them to
// grad2d [record][9] with float atomics. Waves where no pixel uses the entry
// skip both.
// Sum over the 64 lanes of a wave of nine values for each of two records X
// and Y, added to gx[0..8] and gy[0..8] with float atomics (a record whose
// flag is false is skipped). The two records are reduced together with the
// gfx950 lane swaps: permlane32 swaps of (X_i, Y_i) leave X_i folded to 32
// lanes in the lower half and Y_i in the upper half of one register;
// permlane16 swaps of register pairs then fold to one row of 16 lanes per
// (record, value), so 5 registers hold all 18 values, a row of 16 lanes
// each; four DPP steps sum each row, and lane 15 of row r issues that row's
// atomics: row 0 X_0,2,4,6,8; row 1 X_1,3,5,7; row 2 Y_0,2,4,6,8; row 3
// Y_1,3,5,7. 48 lane-parallel instructions instead of 2 x 9 full-wave
// reductions.
__device__ __forceinline__ void reduce_pair(const float (&X)[9], const float (&Y)[9], bool ax,
                                            bool ay, float* gx, float* gy) {
  float Z[9];
#pragma unroll
  for (int i = 0; i < 9; ++i) Z[i] = fold32(X[i], Y[i]);
  float W[5];
#pragma unroll
  for (int m = 0; m < 4; ++m) W[m] = row_sum16(fold16(Z[2 * m], Z[2 * m + 1]));
  W[4] = row_sum16(fold16(Z[8], 0.f));
  const int lane = threadIdx.x & 63;
  if ((lane & 15) == 15) {
    const int row = lane >> 4;
    const bool isy = row >= 2;
    if (isy ? ay : ax) {
      float* dst = (isy ? gy : gx) + (row & 1);
#pragma unroll
      for (int m = 0; m < 4; ++m) atomicAdd(dst + 2 * m, W[m]);
      if ((row & 1) == 0) atomicAdd(dst + 8, W[4]);
    }
  }
}

// The backward of the pixel rows [y_off, y_off + TROWS) of tile g (TROWS =
// TH: the whole tile).
template <int TW, int TH, int TROWS, int BATCH, int PPT>
__device__ __forceinline__ void bwd_tile(const Batch& B, int g, int y_off,
                                         const float4* __restrict__ splat,
                                         const int32_t* __restrict__ vals,
                                         const int2* __restrict__ ranges,
                                         const float* __restrict__ dimg,
                                         const float* __restrict__ Tfin,
                                         const int32_t* __restrict__ ncon,
                                         float* __restrict__ grad2d,
                                         Stage<BATCH, (TW * TROWS / PPT + 63) / 64>& S,
                                         int32_t* s_maxlast_p) {
  constexpr int NT = TW * TROWS / PPT;
  constexpr int NW = (NT + 63) / 64;
  constexpr int RPW = 64 * PPT / TW;  // pixel rows per wave
  // One wave over the whole row span (16x16 at 4 pixels per lane): a lane's
  // PPT pixels lie in PPT bands of NT / TW rows (pixel j in band j), and a
  // band whose pixels no lane has in play for a record skips that record's
  // gradient arithmetic. Several waves keep each wave's rows contiguous
  // (PPT consecutive rows per lane) for the per-wave record lists.
  constexpr bool BANDS = NW == 1 && PPT > 1;
  constexpr int kRowStep = BANDS ? NT / TW : 1;
  int32_t& s_maxlast = *s_maxlast_p;
  const ViewDev& V = B.v[view_of_tile(B, g)];
  const int lt = g - V.tile_off;
  const int ty = lt / V.tiles_x, tx = lt - ty * V.tiles_x;
  const int px = tx * TW + (int)(threadIdx.x % TW);
  // pixel j of this lane is row py0 + j * kRowStep
  const int py0 = ty * TH + y_off + (int)(threadIdx.x / TW) * (BANDS ? 1 : PPT);
  const int2 rg = ranges[g];
  const float fpx = (float)px;
  const float amax = B.alpha_max, amin = B.alpha_min;
  const size_t WH = (size_t)V.W * V.H;
  const float* gi = dimg + 3 * (size_t)V.pix_off;
  float T[PPT], TfbG[PPT], G0[PPT], G1[PPT], G2[PPT], S0[PPT], S1[PPT], S2[PPT];
  int last[PPT];
  int mylast = 0;
#pragma unroll
  for (int j = 0; j < PPT; ++j) {
    const int py = py0 + j * kRowStep;
    T[j] = 1.f;
    G0[j] = G1[j] = G2[j] = 0.f;
    last[j] = 0;
    if (px < V.W && py < V.H) {
      const size_t p = (size_t)py * V.W + px;
      T[j] = Tfin[(size_t)V.pix_off + p];
      last[j] = ncon[(size_t)V.pix_off + p];
      G0[j] = gi[p];
      G1[j] = gi[WH + p];
      G2[j] = gi[2 * WH + p];
    }
    S0[j] = S1[j] = S2[j] = 0.f;
    // T_final (bg . G), the background's share of dL/dalpha before 1/(1-alpha)
    TfbG[j] = T[j] * (B.bg[0] * G0[j] + B.bg[1] * G1[j] + B.bg[2] * G2[j]);
    mylast = max(mylast, last[j]);
  }
  __syncthreads();
  if (threadIdx.x == 0) s_maxlast = 0;
  __syncthreads();
  if (mylast > 0) atomicMax(&s_maxlast, mylast);
  __syncthreads();
  const int end = rg.x + min(s_maxlast, rg.y - rg.x);
  // A tile whose walk is much longer than the typical few hundred entries
  // would finish last while sharing its SIMD with lighter waves: its waves
  // get a higher issue priority (per wave, reset at the end of the tile).
  // The walk is known here (the last blended position over the tile).
  const int walk = end - rg.x;
  if (walk >= 3072)
    __builtin_amdgcn_s_setprio(3);
  else if (walk >= 1536)
    __builtin_amdgcn_s_setprio(2);
  else if (walk >= 768)
    __builtin_amdgcn_s_setprio(1);
  int lo = 0;
  // Per-lane sums of the nine gradient terms of staged record kk over this
  // lane's PPT pixels, into g; returns whether any lane of the wave used it.
  // Branch-free per lane, as in the forward: pixels past their last blended
  // entry or below the record's threshold get alpha 0, which makes every
  // update an exact no-op (T * rcp(1) = T, S unchanged, all terms 0).
  auto contrib = [&](int kk, float (&g)[9]) -> bool {
#pragma unroll
    for (int i = 0; i < 9; ++i) g[i] = 0.f;
    const int pos = lo + kk - rg.x + 1;
    if (__ballot(pos <= mylast) == 0) return false;
    const float4 a = S.s0[kk];
    const float4 b = S.s1[kk];
    const float dx = __fsub_rn(fpx, a.x);
    float P2[PPT], dy[PPT];
    bool anyp = false;
#pragma unroll
    for (int j = 0; j < PPT; ++j) {
      dy[j] = __fsub_rn((float)(py0 + j * kRowStep), a.y);
      P2[j] = power2(dx, dy[j], a, b.x);
      const float thr = pos <= last[j] ? b.y : __builtin_inff();
      anyp = anyp || P2[j] >= thr;
      P2[j] = P2[j] >= thr ? P2[j] : __builtin_inff();  // inf: not in play
    }
    if (__ballot(anyp) == 0) return false;
    const float2 c = S.s2[kk];
    const float cr = b.w, cg = c.x, cb = c.y;
    // per-record terms of the conic gradient that do not depend on the row
    const float hu = 2.f * a.z * dx, hv = a.w * dx, dx2 = dx * dx;
    bool any = false;
#pragma unroll
    for (int j = 0; j < PPT; ++j) {
      // a band no lane has in play: every update below is a no-op there
      if (BANDS && __ballot(P2[j] != __builtin_inff()) == 0) continue;
      const float eP = __builtin_amdgcn_exp2f(P2[j]);
      const float raw = __fmul_rn(b.z, eP);
      float alpha = fminf(amax, raw);
      alpha = (P2[j] > 0.f || alpha < amin) ? 0.f : alpha;  // covers P2 = inf
      any = any || alpha > 0.f;
      const float inv = __builtin_amdgcn_rcpf(1.f - alpha);
      T[j] = T[j] * inv;
      const float w = alpha * T[j];
      g[6] += w * G0[j];
      g[7] += w * G1[j];
      g[8] += w * G2[j];
      // colour minus the colour behind; S_i = S_{i+1} + alpha (c - S_{i+1})
      const float d0 = cr - S0[j], d1 = cg - S1[j], d2 = cb - S2[j];
      const float da = T[j] * (d0 * G0[j] + d1 * G1[j] + d2 * G2[j]) - TfbG[j] * inv;
      S0[j] += alpha * d0;
      S1[j] += alpha * d1;
      S2[j] += alpha * d2;
      // dL/dP in natural-log units (zero when alpha is clamped); the staged
      // conic carries log2(e)
      const float dP = raw <= amax ? alpha * da : 0.f;
      const float dPn = dP * kLn2;
      g[5] += raw <= amax && alpha > 0.f ? eP * da : 0.f;
      g[0] -= dPn * (hu + a.w * dy[j]);
      g[1] -= dPn * (2.f * b.x * dy[j] + hv);
      g[2] += dP * dx2;
      g[3] += dP * dx * dy[j];
      g[4] += dP * dy[j] * dy[j];
    }
    return __ballot(any) != 0;
  };
  // the last list position any pixel of this wave blended
  int wlast = mylast;
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) wlast = max(wlast, __shfl_xor(wlast, o, 64));
  const int wv = threadIdx.x >> 6;
  for (int hi = end; hi > rg.x; hi -= BATCH) {
    lo = max(rg.x, hi - BATCH);
    __syncthreads();
    for (int k = threadIdx.x; k < hi - lo; k += NT) {
      const int r = vals[lo + k];
      S.rec[k] = r;
      stage_record(splat, (size_t)r, amin, S.s0[k], S.s1[k], S.s2[k]);
      S.mask[k] = (uint8_t)wave_mask(S.s0[k], S.s1[k], tx * TW, tx * TW + TW - 1,
                                     ty * TH + y_off, RPW, NW);
    }
    __syncthreads();
    const int cnt = build_wave_list(S, hi - lo, wv, wlast + rg.x - lo - 1);
    __syncthreads();
    // The wave's records, last first, two at a time (the reverse order the
    // recovery of T needs); their 2 x 9 per-lane sums are reduced over the
    // wave together (reduce_pair).
    for (int i = cnt - 1; i >= 0; i -= 2) {
      const int kx = S.list[wv][i];
      const int ky = i >= 1 ? S.list[wv][i - 1] : kx;
      float X[9], Y[9];
      const bool ax = contrib(kx, X);
      const bool ay = i >= 1 && contrib(ky, Y);
      if (!ax && !ay) continue;
      if (!ay) {
#pragma unroll
        for (int q = 0; q < 9; ++q) Y[q] = 0.f;
      }
      reduce_pair(X, Y, ax, ay, grad2d + 9 * (size_t)S.rec[kx], grad2d + 9 * (size_t)S.rec[ky]);
    }
  }
  __builtin_amdgcn_s_setprio(0);
}

template <int TW, int TH, int BATCH, int PPT, bool PERSIST>
__global__ __launch_bounds__(TW* TH / PPT) void k_render_bwd(
    Batch B, const float4* __restrict__ splat, const int32_t* __restrict__ vals,
    const int2* __restrict__ ranges, const float* __restrict__ dimg,
    const float* __restrict__ Tfin, const int32_t* __restrict__ ncon,
    float* __restrict__ grad2d, const int32_t* order, int32_t* qhead) {
  __shared__ Stage<BATCH, (TW * TH / PPT + 63) / 64> S;
  __shared__ int32_t s_maxlast;
  if (!PERSIST) {
    const int g = order ? order[blockIdx.x] : (int)blockIdx.x;
    bwd_tile<TW, TH, TH, BATCH, PPT>(B, g, 0, splat, vals, ranges, dimg, Tfin, ncon, grad2d, S,
                                     &s_maxlast);
    return;
  }
  __shared__ int s_next;
  for (int q = next_tile(&s_next, qhead); q < B.total_tiles; q = next_tile(&s_next, qhead))
    bwd_tile<TW, TH, TH, BATCH, PPT>(B, order[q], 0, splat, vals, ranges, dimg, Tfin, ncon,
                                     grad2d, S, &s_maxlast);
}

// Backward with heavy tiles split (16x16 tiles). A first kernel finds each
// tile's walk -- the largest n_contrib over its pixels -- and gives the
// tiles whose walk reaches split_walk a slot in a short list (at most
// kSplitMaxHeavy; tiles beyond it stay whole). Such a tile is walked as four
// 16x4 bands at one pixel per lane, by four one-wave workgroups each with
// its own walk and record list, instead of by one wave at four pixels per
// lane: its waves would otherwise walk thousands of entries long after the
// other tiles are done. The grid is 3 kSplitMaxHeavy workgroups for bands
// 1..3 of the listed tiles (first, so they start early; those past the
// list's length return at once), then one per tile: band 0 of a listed
// tile, else the whole tile. Split metadata (int32): [0] list length,
// [kSplitHeavyOff + h] the listed tiles, [kSplitSlotOff + g] tile g's slot
// or -1.
constexpr int kSplitMaxHeavy = 64;
constexpr int kSplitHeavyOff = 64;
constexpr int kSplitSlotOff = kSplitHeavyOff + kSplitMaxHeavy;

__global__ __launch_bounds__(256) void k_tile_walks(Batch B, const int32_t* __restrict__ ncon,
                                                    int split_walk, int32_t* __restrict__ meta) {
  const int g = (int)blockIdx.x * 4 + (int)(threadIdx.x >> 6);
  if (g >= B.total_tiles) return;
  const int lane = (int)(threadIdx.x & 63u);
  const ViewDev& V = B.v[view_of_tile(B, g)];
  const int lt = g - V.tile_off;
  const int ty = lt / V.tiles_x, tx = lt - ty * V.tiles_x;
  const int px = tx * 16 + (lane & 15);
  const int py0 = ty * 16 + (lane >> 4) * 4;
  int walk = 0;
#pragma unroll
  for (int j = 0; j < 4; ++j)
    if (px < V.W && py0 + j < V.H)
      walk = max(walk, ncon[(size_t)V.pix_off + (size_t)(py0 + j) * V.W + px]);
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) walk = max(walk, __shfl_xor(walk, o, 64));
  if (lane == 0) {
    int slot = -1;
    if (walk >= split_walk) {
      const int h = atomicAdd(&meta[0], 1);
      if (h < kSplitMaxHeavy) {
        meta[kSplitHeavyOff + h] = g;
        slot = h;
      }
    }
    meta[kSplitSlotOff + g] = slot;
  }
}

template <int BATCH>
__global__ __launch_bounds__(64) void k_render_bwd_split(
    Batch B, const float4* __restrict__ splat, const int32_t* __restrict__ vals,
    const int2* __restrict__ ranges, const float* __restrict__ dimg,
    const float* __restrict__ Tfin, const int32_t* __restrict__ ncon,
    float* __restrict__ grad2d, const int32_t* order, const int32_t* __restrict__ meta) {
  __shared__ Stage<BATCH, 1> S;
  __shared__ int32_t s_maxlast;
  constexpr int NX = 3 * kSplitMaxHeavy;
  int g, band;
  if ((int)blockIdx.x < NX) {
    const int h = (int)blockIdx.x / 3;
    if (h >= min(meta[0], kSplitMaxHeavy)) return;
    g = meta[kSplitHeavyOff + h];
    band = 1 + (int)blockIdx.x % 3;
  } else {
    const int q = (int)blockIdx.x - NX;
    g = order ? order[q] : q;
    if (meta[kSplitSlotOff + g] < 0) {
      bwd_tile<16, 16, 16, BATCH, 4>(B, g, 0, splat, vals, ranges, dimg, Tfin, ncon, grad2d, S,
                                     &s_maxlast);
      return;
    }
    band = 0;
  }
  bwd_tile<16, 16, 4, BATCH, 1>(B, g, 4 * band, splat, vals, ranges, dimg, Tfin, ncon, grad2d, S,
                                &s_maxlast);
}

size_t split_meta_bytes(int64_t tiles) {
  return (((size_t)(kSplitSlotOff + tiles) * sizeof(int32_t)) + 255) & ~(size_t)255;
}

// Launchers ------------------------------------------------------------------

struct RenderArgs {
  const float4* splat;
  const int32_t* vals;
  const int2* ranges;
  float* image;
  float* Tfin;
  int32_t* ncon;
  int32_t* tile_work;
  const float* dimg;
  const float* Tfin_in;
  const int32_t* ncon_in;
  float* grad2d;
  const int32_t* order;
  int32_t* qhead;
  bool persistent;
};

__global__ void k_zero_i32(int32_t* p) {
  if (threadIdx.x == 0) *p = 0;
}

// Workgroups that fill the device once: resident blocks per CU x CUs.
template <typename K>
static int persistent_grid(K kernel, int threads) {
  int dev = 0, cus = 0, per_cu = 0;
  if (hipGetDevice(&dev) != hipSuccess) return 0;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
    return 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kernel, threads, 0) != hipSuccess)
    return 0;
  return std::max(1, per_cu) * std::max(1, cus);
}

template <int TW, int TH, int BATCH, int PPT>
static void launch_one(const Batch& B, const RenderArgs& A, bool bwd, hipStream_t st) {
  const int threads = TW * TH / PPT;
  if (A.persistent) {
    hipLaunchKernelGGL(k_zero_i32, dim3(1), dim3(64), 0, st, A.qhead);
    if (bwd) {
      auto k = k_render_bwd<TW, TH, BATCH, PPT, true>;
      const int grid = std::min(B.total_tiles, persistent_grid(k, threads));
      hipLaunchKernelGGL(k, dim3(std::max(grid, 1)), dim3(threads), 0, st, B, A.splat, A.vals,
                         A.ranges, A.dimg, A.Tfin_in, A.ncon_in, A.grad2d, A.order, A.qhead);
    } else {
      auto k = k_render_fwd<TW, TH, BATCH, PPT, true>;
      const int grid = std::min(B.total_tiles, persistent_grid(k, threads));
      hipLaunchKernelGGL(k, dim3(std::max(grid, 1)), dim3(threads), 0, st, B, A.splat, A.vals,
                         A.ranges, A.image, A.Tfin, A.ncon, A.tile_work, A.order, A.qhead);
    }
    return;
  }
  const dim3 grid(B.total_tiles), block(threads);
  if (bwd)
    hipLaunchKernelGGL((k_render_bwd<TW, TH, BATCH, PPT, false>), grid, block, 0, st, B, A.splat,
                       A.vals, A.ranges, A.dimg, A.Tfin_in, A.ncon_in, A.grad2d, A.order,
                       A.qhead);
  else
    hipLaunchKernelGGL((k_render_fwd<TW, TH, BATCH, PPT, false>), grid, block, 0, st, B, A.splat,
                       A.vals, A.ranges, A.image, A.Tfin, A.ncon, A.tile_work, A.order, A.qhead);
}

template <int TW, int TH, int PPT>
static void launch_batch(const Batch& B, int lds_batch, const RenderArgs& A, bool bwd,
                         hipStream_t st) {
  switch (lds_batch) {
    case 64: launch_one<TW, TH, 64, PPT>(B, A, bwd, st); break;
    case 128: launch_one<TW, TH, 128, PPT>(B, A, bwd, st); break;
    case 512: launch_one<TW, TH, 512, PPT>(B, A, bwd, st); break;
    default: launch_one<TW, TH, 256, PPT>(B, A, bwd, st); break;
  }
}

// The counting forward: index order, LDS batch 256, one pixel per thread
// (four per thread at 32x32); the work counts and the image do not depend
// on the launch shape.
static void launch_count(const Batch& B, const RenderArgs& A, hipStream_t st) {
  const dim3 grid(B.total_tiles);
  if (B.tile_w == 8)
    hipLaunchKernelGGL((k_render_fwd<8, 8, 256, 1, false, true>), grid, dim3(64), 0, st, B,
                       A.splat, A.vals, A.ranges, A.image, A.Tfin, A.ncon, A.tile_work,
                       nullptr, nullptr);
  else if (B.tile_w == 32)
    hipLaunchKernelGGL((k_render_fwd<32, 32, 256, 4, false, true>), grid, dim3(256), 0, st, B,
                       A.splat, A.vals, A.ranges, A.image, A.Tfin, A.ncon, A.tile_work,
                       nullptr, nullptr);
  else
    hipLaunchKernelGGL((k_render_fwd<16, 16, 256, 1, false, true>), grid, dim3(256), 0, st, B,
                       A.splat, A.vals, A.ranges, A.image, A.Tfin, A.ncon, A.tile_work,
                       nullptr, nullptr);
}

static void launch_render(const Batch& B, int lds_batch, int ppt, const RenderArgs& A, bool bwd,
                          hipStream_t st) {
  if (!bwd && A.tile_work) {
    launch_count(B, A, st);
    return;
  }
  if (B.tile_w == 8) {
    launch_batch<8, 8, 1>(B, lds_batch, A, bwd, st);
    return;
  }
  if (B.tile_w == 32) {  // 4 pixels per thread: 256 threads, 4 waves of 8 rows
    launch_batch<32, 32, 4>(B, lds_batch, A, bwd, st);
    return;
  }
  switch (ppt) {
    case 2: launch_batch<16, 16, 2>(B, lds_batch, A, bwd, st); break;
    case 4: launch_batch<16, 16, 4>(B, lds_batch, A, bwd, st); break;
    default: launch_batch<16, 16, 1>(B, lds_batch, A, bwd, st); break;
  }
}

hipError_t launch_render_fwd(const Batch& B, int lds_batch, int ppt, bool persistent,
                             const float* splat, const int32_t* vals, const int32_t* ranges,
                             int32_t* order, float* image, float* Tfin, int32_t* ncon,
                             int32_t* tile_work, hipStream_t st) {
  if (B.total_tiles <= 0) return hipSuccess;
  RenderArgs A{};
  A.splat = reinterpret_cast<const float4*>(splat);
  A.vals = vals;
  A.ranges = reinterpret_cast<const int2*>(ranges);
  A.image = image;
  A.Tfin = Tfin;
  A.ncon = ncon;
  A.tile_work = tile_work;
  A.order = order;
  A.qhead = order ? order + B.total_tiles : nullptr;
  A.persistent = persistent && order;
  launch_render(B, lds_batch, ppt, A, false, st);
  return hipGetLastError();
}

template <int BATCH>
static void launch_bwd_split(const Batch& B, const RenderArgs& A, int32_t* meta, hipStream_t st) {
  hipLaunchKernelGGL((k_render_bwd_split<BATCH>), dim3(3 * kSplitMaxHeavy + B.total_tiles),
                     dim3(64), 0, st, B, A.splat, A.vals, A.ranges, A.dimg, A.Tfin_in, A.ncon_in,
                     A.grad2d, A.order, meta);
}

hipError_t launch_render_bwd(const Batch& B, int lds_batch, int ppt, bool persistent,
                             int split_walk, int32_t* split_meta, const float* splat,
                             const int32_t* vals, const int32_t* ranges, int32_t* order,
                             const float* dimg, const float* Tfin, const int32_t* ncon,
                             float* grad2d, hipStream_t st) {
  if (B.total_tiles <= 0) return hipSuccess;
  RenderArgs A{};
  A.splat = reinterpret_cast<const float4*>(splat);
  A.vals = vals;
  A.ranges = reinterpret_cast<const int2*>(ranges);
  A.dimg = dimg;
  A.Tfin_in = Tfin;
  A.ncon_in = ncon;
  A.grad2d = grad2d;
  A.order = order;
  A.qhead = order ? order + B.total_tiles : nullptr;
  A.persistent = persistent && order;
  if (split_walk > 0 && split_meta && !A.persistent && B.tile_w == 16 && ppt == 4) {
    hipLaunchKernelGGL(k_zero_i32, dim3(1), dim3(64), 0, st, split_meta);
    hipLaunchKernelGGL(k_tile_walks, dim3((B.total_tiles + 3) / 4), dim3(256), 0, st, B,
                       A.ncon_in, split_walk, split_meta);
    switch (lds_batch) {
      case 64: launch_bwd_split<64>(B, A, split_meta, st); break;
      case 128: launch_bwd_split<128>(B, A, split_meta, st); break;
      case 512: launch_bwd_split<512>(B, A, split_meta, st); break;
      default: launch_bwd_split<256>(B, A, split_meta, st); break;
    }
    return hipGetLastError();
  }
  launch_render(B, lds_batch, ppt, A, true, st);
  return hipGetLastError();
}

}  // namespace xpr
