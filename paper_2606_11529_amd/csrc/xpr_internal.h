// Internal declarations of the gfx950 kernels behind include/xpr.h.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <type_traits>

#include "xpr.h"

namespace xpr {

constexpr int kWave = 64;

// Scene as the kernels see it (kernel-argument copy of xpr_scene).
struct SceneDev {
  const float* means;
  const float* scales;
  const float* quats;
  const float* opac;
  const float* sh;
  int32_t n, ld, K, pad;
};

// One view: camera, image/tile sizes and its offsets in the concatenated
// per-record, per-tile and per-pixel buffers.
struct ViewDev {
  float R[9], t[3];
  float fx, fy, cx, cy;
  int16_t W, H, tiles_x, tiles_y;
  int32_t scene, rec_off, tile_off, pix_off;
};
static_assert(sizeof(ViewDev) == 88, "view descriptor layout");

// Whole batch, passed by value as a kernel argument.
struct Batch {
  SceneDev s[XPR_MAX_SCENES];
  ViewDev v[XPR_MAX_VIEWS];
  int32_t n_views, n_scenes;
  int32_t total_rec, total_tiles;
  int32_t tile_w, tile_h;
  int32_t sh_degree, opacity_extents;
  float lowpass, alpha_min, alpha_max, t_min, z_near, fov_clip;
  float bg[3];
  int32_t method;  // XPR_METHOD_3DGS, XPR_METHOD_3DGUT or XPR_METHOD_LINPRIM
};
// Gradient destinations of every scene (project backward).
struct GradDev {
  float* means;
  float* scales;
  float* quats;
  float* opac;
  float* sh;
};
// Kernel arguments stay below the 4 KiB kernarg limit.
static_assert(sizeof(Batch) + sizeof(GradDev) * XPR_MAX_SCENES + 64 <= 4096,
              "kernel argument block too large");

// Splat record stride in float4 units: 12 floats for 3DGS, 24 for 3DGUT,
// 20 for LinPrim.
__device__ __host__ __forceinline__ int splat_stride4(const Batch& B) {
  return B.method == XPR_METHOD_3DGUT ? 6 : (B.method == XPR_METHOD_LINPRIM ? 5 : 3);
}

// View owning global tile g (views are few; a scalar linear scan).
__device__ __forceinline__ int view_of_tile(const Batch& B, int g) {
  int v = 0;
  for (int k = 1; k < B.n_views; ++k)
    if (g >= B.v[k].tile_off) v = k;
  return v;
}

// Workgroups are dispatched round-robin over the 8 XCDs of an MI355X
// (workgroup b runs on XCD b % 8), and each XCD has its own L2. This
// bijection of [0, n) gives XCD x a contiguous range of work items, so
// neighbouring items (adjacent partitions of a sort, whose partial cache
// lines at run boundaries then merge in one L2) share an L2. Only for blocks
// of uniform cost: it hands each XCD one contiguous stretch of the work, so
// uneven work (image tiles, records of very different footprint) would pile
// up on some XCDs. Correct for any dispatch order; only locality changes.
__device__ __forceinline__ int xcd_swizzle(int b, int n) {
  const int x = b & 7, k = b >> 3;
  const int per = n >> 3, rem = n & 7;
  return x * per + min(x, rem) + k;
}

// Cross-lane helpers (wave64).
template <int CTRL, int ROW_MASK = 0xf, int BANK_MASK = 0xf>
__device__ __forceinline__ float dpp_f(float x) {
  return __int_as_float(
      __builtin_amdgcn_update_dpp(0, __float_as_int(x), CTRL, ROW_MASK, BANK_MASK, true));
}

// Sum over the 64 lanes; the total lands in lane 63 (other lanes hold
// partial sums). Butterflies inside each row of 16 lanes, then the two
// row broadcasts of the gfx9 DPP.
__device__ __forceinline__ float wave_sum_lane63(float x) {
  x += dpp_f<0xB1>(x);          // quad_perm [1,0,3,2]
  x += dpp_f<0x4E>(x);          // quad_perm [2,3,0,1]
  x += dpp_f<0x141>(x);         // row_half_mirror
  x += dpp_f<0x140>(x);         // row_mirror: every lane holds its row sum
  x += dpp_f<0x142, 0xa>(x);    // row_bcast:15 into rows 1 and 3
  x += dpp_f<0x143, 0xc>(x);    // row_bcast:31 into rows 2 and 3
  return x;
}

// gfx950 lane swaps (v_permlane32_swap, v_permlane16_swap) for reducing
// several values over a wave at once. fold32(x, y): lanes 0..31 hold
// x[l] + x[l + 32], lanes 32..63 hold y[l - 32] + y[l]. fold16(c, d): of
// the four 16-lane rows, row 0 holds c's rows 0 + 1, row 1 d's rows 0 + 1,
// row 2 c's rows 2 + 3 and row 3 d's rows 2 + 3. row_sum16: every lane
// gets the sum over its row.
__device__ __forceinline__ float fold32(float x, float y) {
  const auto r = __builtin_amdgcn_permlane32_swap(__float_as_uint(x), __float_as_uint(y), false,
                                                  false);
  return __uint_as_float(r[0]) + __uint_as_float(r[1]);
}

__device__ __forceinline__ float fold16(float x, float y) {
  const auto r = __builtin_amdgcn_permlane16_swap(__float_as_uint(x), __float_as_uint(y), false,
                                                  false);
  return __uint_as_float(r[0]) + __uint_as_float(r[1]);
}

__device__ __forceinline__ float row_sum16(float x) {
  x += dpp_f<0xB1>(x);   // quad_perm [1,0,3,2]
  x += dpp_f<0x4E>(x);   // quad_perm [2,3,0,1]
  x += dpp_f<0x141>(x);  // row_half_mirror
  x += dpp_f<0x140>(x);  // row_mirror: every lane holds its row sum
  return x;
}

// Sum over the 64 lanes of X[0..15], added to dst[0..15] with float
// atomics: fold32 leaves X_i in rows 0-1 and X_{i+8} in rows 2-3, fold16 of
// (Z_2m, Z_2m+1) then gives row 0 X_2m, row 1 X_2m+1, row 2 X_2m+8 and row 3
// X_2m+9; lane 15 of each row issues its four atomics.
__device__ __forceinline__ void reduce16(const float (&X)[16], float* dst) {
  float Z[8];
#pragma unroll
  for (int i = 0; i < 8; ++i) Z[i] = fold32(X[i], X[i + 8]);
  float W[4];
#pragma unroll
  for (int m = 0; m < 4; ++m) W[m] = row_sum16(fold16(Z[2 * m], Z[2 * m + 1]));
  const int lane = threadIdx.x & 63;
  if ((lane & 15) == 15) {
    const int row = lane >> 4;
    float* d = dst + (row & 1) + 8 * (row >> 1);
#pragma unroll
    for (int m = 0; m < 4; ++m) atomicAdd(d + 2 * m, W[m]);
  }
}

__device__ __forceinline__ float lane63(float x) {
  return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(x), 63));
}

__device__ __forceinline__ uint64_t lanemask_lt() {
  const int lane = threadIdx.x & (kWave - 1);
  return lane == 0 ? 0ull : (~0ull >> (64 - lane));
}

// Host-side launch helpers (api.hip).
const char* set_error(const char* fmt, ...);

// Work counts of the counting forward: the workgroup's sums of its
// threads' evaluated and blended list entries go to tile_work [g][2]
// (s_cnt: two ints of LDS). Every thread of the workgroup calls it.
__device__ __forceinline__ void store_tile_work(int ev, int bl, int32_t* s_cnt,
                                                int32_t* tile_work, int g) {
  __syncthreads();
  if (threadIdx.x == 0) s_cnt[0] = s_cnt[1] = 0;
  __syncthreads();
  atomicAdd(&s_cnt[0], ev);
  atomicAdd(&s_cnt[1], bl);
  __syncthreads();
  if (threadIdx.x == 0) {
    tile_work[2 * (size_t)g] = s_cnt[0];
    tile_work[2 * (size_t)g + 1] = s_cnt[1];
  }
}

}  // namespace xpr
