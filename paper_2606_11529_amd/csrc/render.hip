// Per-pixel compositing (Algorithm 1 of the paper with the 3DGS evaluate of
// the listing "Implementation of XPR-3DGS") and its backward.
//
// One workgroup per tile: a TW x TH tile is TW*TH threads (16x16 = four
// wave64s), one pixel per thread. The tile's depth-sorted list is walked in
// batches of BATCH splat records staged in LDS (each thread loads at most
// BATCH / (TW*TH) records, then every thread reads each record as a
// broadcast); the whole workgroup leaves the loop as soon as no pixel is
// still active, checked once per batch (the batch-boundary exit check of
// Algorithm 1). The loop body is plain FP32 VALU work: the kernels are
// bound by VALU issue, not by memory.
#include "xpr_internal.h"

namespace xpr {

// The evaluate of the listing: power P = A dx^2 + B dx dy + C dy^2 and
// alpha = min(alpha_max, o e^P). Written with explicit roundings so the
// forward and backward kernels take bit-identical decisions.
struct Eval {
  float dx, dy, P, eP, raw, alpha;
};

__device__ __forceinline__ Eval evaluate(float px, float py, float4 a, float4 b, float alpha_max) {
  Eval e;
  e.dx = __fsub_rn(px, a.x);
  e.dy = __fsub_rn(py, a.y);
  e.P = __fmaf_rn(a.z, __fmul_rn(e.dx, e.dx),
                  __fmaf_rn(a.w, __fmul_rn(e.dx, e.dy), __fmul_rn(b.x, __fmul_rn(e.dy, e.dy))));
  e.eP = __expf(e.P);
  e.raw = __fmul_rn(b.y, e.eP);
  e.alpha = fminf(alpha_max, e.raw);
  return e;
}

template <int TW, int TH, int BATCH>
__global__ __launch_bounds__(TW* TH) void k_render_fwd(Batch B, const float4* __restrict__ splat,
                                                       const int32_t* __restrict__ vals,
                                                       const int2* __restrict__ ranges,
                                                       float* __restrict__ image,
                                                       float* __restrict__ Tfin,
                                                       int32_t* __restrict__ ncon,
                                                       int32_t* __restrict__ tile_work) {
  constexpr int NT = TW * TH;
  __shared__ float4 s0[BATCH];
  __shared__ float4 s1[BATCH];
  __shared__ float s2[BATCH];
  const int g = blockIdx.x;
  const ViewDev& V = B.v[view_of_tile(B, g)];
  const int lt = g - V.tile_off;
  const int ty = lt / V.tiles_x, tx = lt - ty * V.tiles_x;
  const int px = tx * TW + (int)(threadIdx.x % TW);
  const int py = ty * TH + (int)(threadIdx.x / TW);
  const bool inside = px < V.W && py < V.H;
  const int2 rg = ranges[g];
  const float fpx = (float)px, fpy = (float)py;
  const float amax = B.alpha_max, amin = B.alpha_min, tmin = B.t_min;
  float T = 1.f, C0 = 0.f, C1 = 0.f, C2 = 0.f;
  int last = 0;
  bool done = !inside;
  int walked = 0;
  for (int base = rg.x; base < rg.y; base += BATCH) {
    if (__syncthreads_count(!done) == 0) break;
    walked = min(BATCH, rg.y - base) + (base - rg.x);
    for (int k = threadIdx.x; k < BATCH; k += NT) {
      const int idx = base + k;
      if (idx < rg.y) {
        const size_t r = (size_t)vals[idx];
        s0[k] = splat[3 * r];
        s1[k] = splat[3 * r + 1];
        s2[k] = splat[3 * r + 2].x;
      }
    }
    __syncthreads();
    if (!done) {
      const int nb = min(BATCH, rg.y - base);
      for (int k = 0; k < nb; ++k) {
        const float4 a = s0[k];
        const float4 b = s1[k];
        const Eval e = evaluate(fpx, fpy, a, b, amax);
        if (e.P > 0.f || e.alpha < amin) continue;
        const float Tn = T * (1.f - e.alpha);
        if (Tn < tmin) {
          done = true;
          break;
        }
        const float w = e.alpha * T;
        C0 += b.z * w;
        C1 += b.w * w;
        C2 += s2[k] * w;
        T = Tn;
        last = base + k - rg.x + 1;
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

// Backward of the compositing. Each pixel walks its list in reverse from
// its last blended entry, recovering T_i = T_{i+1} / (1 - a_i) and the
// colour behind S_i, and forms
//   dL/dc_i = a_i T_i G,  dL/da_i = T_i (c_i - S_i).G - T_final (bg.G)/(1 - a_i)
//   dL/do = e^P dL/da, dL/dP = a dL/da (zero when a is clamped)
//   dL/du = -dL/dP (2A dx + B dy), dL/dv = -dL/dP (2C dy + B dx),
//   dL/d(A, B, C) = dL/dP (dx^2, dx dy, dy^2).
// The nine per-pixel values are summed over the wave with DPP and added to
// grad2d [record][9] with one lane's float atomics; waves where no pixel
// uses the entry skip both.
template <int TW, int TH, int BATCH>
__global__ __launch_bounds__(TW* TH) void k_render_bwd(Batch B, const float4* __restrict__ splat,
                                                       const int32_t* __restrict__ vals,
                                                       const int2* __restrict__ ranges,
                                                       const float* __restrict__ dimg,
                                                       const float* __restrict__ Tfin,
                                                       const int32_t* __restrict__ ncon,
                                                       float* __restrict__ grad2d) {
  constexpr int NT = TW * TH;
  __shared__ float4 s0[BATCH];
  __shared__ float4 s1[BATCH];
  __shared__ float s2[BATCH];
  __shared__ int32_t srec[BATCH];
  __shared__ int32_t s_maxlast;
  const int g = blockIdx.x;
  const ViewDev& V = B.v[view_of_tile(B, g)];
  const int lt = g - V.tile_off;
  const int ty = lt / V.tiles_x, tx = lt - ty * V.tiles_x;
  const int px = tx * TW + (int)(threadIdx.x % TW);
  const int py = ty * TH + (int)(threadIdx.x / TW);
  const bool inside = px < V.W && py < V.H;
  const int2 rg = ranges[g];
  const float fpx = (float)px, fpy = (float)py;
  const float amax = B.alpha_max, amin = B.alpha_min;
  const size_t WH = (size_t)V.W * V.H;
  const size_t p = (size_t)py * V.W + px;
  float T = 1.f, G0 = 0.f, G1 = 0.f, G2 = 0.f;
  int last = 0;
  if (inside) {
    T = Tfin[(size_t)V.pix_off + p];
    last = ncon[(size_t)V.pix_off + p];
    const float* gi = dimg + 3 * (size_t)V.pix_off;
    G0 = gi[p];
    G1 = gi[WH + p];
    G2 = gi[2 * WH + p];
  }
  if (threadIdx.x == 0) s_maxlast = 0;
  __syncthreads();
  if (last > 0) atomicMax(&s_maxlast, last);
  __syncthreads();
  const int end = rg.x + min(s_maxlast, rg.y - rg.x);
  const float Tf = T;
  const float bgG = B.bg[0] * G0 + B.bg[1] * G1 + B.bg[2] * G2;
  float S0 = 0.f, S1 = 0.f, S2 = 0.f;
  for (int hi = end; hi > rg.x; hi -= BATCH) {
    const int lo = max(rg.x, hi - BATCH);
    __syncthreads();
    for (int k = threadIdx.x; k < hi - lo; k += NT) {
      const int r = vals[lo + k];
      srec[k] = r;
      s0[k] = splat[3 * (size_t)r];
      s1[k] = splat[3 * (size_t)r + 1];
      s2[k] = splat[3 * (size_t)r + 2].x;
    }
    __syncthreads();
    for (int k = hi - lo - 1; k >= 0; --k) {
      const float4 a = s0[k];
      const float4 b = s1[k];
      const int pos = lo + k - rg.x + 1;
      const Eval e = evaluate(fpx, fpy, a, b, amax);
      const bool use = pos <= last && !(e.P > 0.f) && !(e.alpha < amin);
      if (__ballot(use) == 0) continue;
      float gu = 0.f, gv = 0.f, gA = 0.f, gB = 0.f, gC = 0.f, go = 0.f;
      float gr = 0.f, gg = 0.f, gb = 0.f;
      if (use) {
        const float c2 = s2[k];
        T = T / (1.f - e.alpha);
        const float w = e.alpha * T;
        gr = w * G0;
        gg = w * G1;
        gb = w * G2;
        const float da = T * ((b.z - S0) * G0 + (b.w - S1) * G1 + (c2 - S2) * G2) -
                         Tf * bgG / (1.f - e.alpha);
        S0 = e.alpha * b.z + (1.f - e.alpha) * S0;
        S1 = e.alpha * b.w + (1.f - e.alpha) * S1;
        S2 = e.alpha * c2 + (1.f - e.alpha) * S2;
        if (e.raw <= amax) {
          const float dP = e.alpha * da;
          go = e.eP * da;
          gu = -dP * (2.f * a.z * e.dx + a.w * e.dy);
          gv = -dP * (2.f * b.x * e.dy + a.w * e.dx);
          gA = dP * e.dx * e.dx;
          gB = dP * e.dx * e.dy;
          gC = dP * e.dy * e.dy;
        }
      }
      gu = wave_sum_lane63(gu);
      gv = wave_sum_lane63(gv);
      gA = wave_sum_lane63(gA);
      gB = wave_sum_lane63(gB);
      gC = wave_sum_lane63(gC);
      go = wave_sum_lane63(go);
      gr = wave_sum_lane63(gr);
      gg = wave_sum_lane63(gg);
      gb = wave_sum_lane63(gb);
      if ((threadIdx.x & 63) == 63) {
        float* dst = grad2d + 9 * (size_t)srec[k];
        atomicAdd(dst + 0, gu);
        atomicAdd(dst + 1, gv);
        atomicAdd(dst + 2, gA);
        atomicAdd(dst + 3, gB);
        atomicAdd(dst + 4, gC);
        atomicAdd(dst + 5, go);
        atomicAdd(dst + 6, gr);
        atomicAdd(dst + 7, gg);
        atomicAdd(dst + 8, gb);
      }
    }
  }
}

// Launchers ------------------------------------------------------------------

template <int TW, int TH>
static hipError_t launch_fwd_t(const Batch& B, int lds_batch, const float* splat,
                               const int32_t* vals, const int32_t* ranges, float* image,
                               float* Tfin, int32_t* ncon, int32_t* tw, hipStream_t st) {
  const dim3 grid(B.total_tiles), block(TW * TH);
  const float4* sp = reinterpret_cast<const float4*>(splat);
  const int2* rg = reinterpret_cast<const int2*>(ranges);
  switch (lds_batch) {
    case 64: hipLaunchKernelGGL((k_render_fwd<TW, TH, 64>), grid, block, 0, st, B, sp, vals, rg, image, Tfin, ncon, tw); break;
    case 128: hipLaunchKernelGGL((k_render_fwd<TW, TH, 128>), grid, block, 0, st, B, sp, vals, rg, image, Tfin, ncon, tw); break;
    case 512: hipLaunchKernelGGL((k_render_fwd<TW, TH, 512>), grid, block, 0, st, B, sp, vals, rg, image, Tfin, ncon, tw); break;
    default: hipLaunchKernelGGL((k_render_fwd<TW, TH, 256>), grid, block, 0, st, B, sp, vals, rg, image, Tfin, ncon, tw); break;
  }
  return hipGetLastError();
}

template <int TW, int TH>
static hipError_t launch_bwd_t(const Batch& B, int lds_batch, const float* splat,
                               const int32_t* vals, const int32_t* ranges, const float* dimg,
                               const float* Tfin, const int32_t* ncon, float* grad2d,
                               hipStream_t st) {
  const dim3 grid(B.total_tiles), block(TW * TH);
  const float4* sp = reinterpret_cast<const float4*>(splat);
  const int2* rg = reinterpret_cast<const int2*>(ranges);
  switch (lds_batch) {
    case 64: hipLaunchKernelGGL((k_render_bwd<TW, TH, 64>), grid, block, 0, st, B, sp, vals, rg, dimg, Tfin, ncon, grad2d); break;
    case 128: hipLaunchKernelGGL((k_render_bwd<TW, TH, 128>), grid, block, 0, st, B, sp, vals, rg, dimg, Tfin, ncon, grad2d); break;
    case 512: hipLaunchKernelGGL((k_render_bwd<TW, TH, 512>), grid, block, 0, st, B, sp, vals, rg, dimg, Tfin, ncon, grad2d); break;
    default: hipLaunchKernelGGL((k_render_bwd<TW, TH, 256>), grid, block, 0, st, B, sp, vals, rg, dimg, Tfin, ncon, grad2d); break;
  }
  return hipGetLastError();
}

hipError_t launch_render_fwd(const Batch& B, int lds_batch, const float* splat,
                             const int32_t* vals, const int32_t* ranges, float* image, float* Tfin,
                             int32_t* ncon, int32_t* tile_work, hipStream_t st) {
  if (B.total_tiles <= 0) return hipSuccess;
  if (B.tile_w == 8)
    return launch_fwd_t<8, 8>(B, lds_batch, splat, vals, ranges, image, Tfin, ncon, tile_work, st);
  return launch_fwd_t<16, 16>(B, lds_batch, splat, vals, ranges, image, Tfin, ncon, tile_work, st);
}

hipError_t launch_render_bwd(const Batch& B, int lds_batch, const float* splat,
                             const int32_t* vals, const int32_t* ranges, const float* dimg,
                             const float* Tfin, const int32_t* ncon, float* grad2d,
                             hipStream_t st) {
  if (B.total_tiles <= 0) return hipSuccess;
  if (B.tile_w == 8)
    return launch_bwd_t<8, 8>(B, lds_batch, splat, vals, ranges, dimg, Tfin, ncon, grad2d, st);
  return launch_bwd_t<16, 16>(B, lds_batch, splat, vals, ranges, dimg, Tfin, ncon, grad2d, st);
}

}  // namespace xpr
