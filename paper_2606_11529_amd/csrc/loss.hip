// The training objective of the benchmarked step: L1 loss between the
// rendered image and a target, L = (1/n) sum |C - target| over the n = 3HW
// colour values, and its gradient dL/dC = sign(C - target) / n (sign(0) = 0),
// the input of the compositing backward. One pass over the pixels: HBM-bound,
// 8 B read and 4 B written per value.
#include "xpr_internal.h"

namespace xpr {

__device__ __forceinline__ float sgn(float d) { return d > 0.f ? 1.f : (d < 0.f ? -1.f : 0.f); }

// Grid-stride over float4 groups when VEC (all three pointers 16-byte
// aligned), then the tail; each thread keeps four groups' loads in flight.
// One float atomic per block for the loss: a few hundred blocks of 1024
// threads, since same-address atomics serialise.
constexpr int kLossThreads = 1024;
constexpr int kLossUnroll = 4;

template <bool VEC>
__global__ __launch_bounds__(kLossThreads) void k_l1_loss(const float* __restrict__ img,
                                                          const float* __restrict__ tgt,
                                                          int64_t n, float inv_n,
                                                          float* __restrict__ loss,
                                                          float* __restrict__ dimg) {
  __shared__ float s_wave[kLossThreads / 64];
  const int64_t stride = (int64_t)gridDim.x * kLossThreads;
  const int64_t tid = (int64_t)blockIdx.x * kLossThreads + threadIdx.x;
  float s = 0.f;
  int64_t done = 0;
  if (VEC) {
    const int64_t nv = n / 4;
    const float4* a4 = reinterpret_cast<const float4*>(img);
    const float4* b4 = reinterpret_cast<const float4*>(tgt);
    float4* g4 = reinterpret_cast<float4*>(dimg);
    for (int64_t i0 = tid; i0 < nv; i0 += kLossUnroll * stride) {
      float4 a[kLossUnroll], b[kLossUnroll];
#pragma unroll
      for (int u = 0; u < kLossUnroll; ++u) {
        const int64_t i = min(i0 + u * stride, nv - 1);
        a[u] = a4[i];
        b[u] = b4[i];
      }
#pragma unroll
      for (int u = 0; u < kLossUnroll; ++u) {
        const int64_t i = i0 + u * stride;
        if (i < nv) {
          const float d0 = a[u].x - b[u].x, d1 = a[u].y - b[u].y;
          const float d2 = a[u].z - b[u].z, d3 = a[u].w - b[u].w;
          s += fabsf(d0) + fabsf(d1) + fabsf(d2) + fabsf(d3);
          g4[i] = make_float4(sgn(d0) * inv_n, sgn(d1) * inv_n, sgn(d2) * inv_n,
                              sgn(d3) * inv_n);
        }
      }
    }
    done = nv * 4;
  }
  for (int64_t i = done + tid; i < n; i += stride) {
    const float d = img[i] - tgt[i];
    s += fabsf(d);
    dimg[i] = sgn(d) * inv_n;
  }
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) s += __shfl_xor(s, o, 64);
  if ((threadIdx.x & 63) == 0) s_wave[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) {
    float t = 0.f;
#pragma unroll
    for (int w = 0; w < kLossThreads / 64; ++w) t += s_wave[w];
    atomicAdd(loss, t * inv_n);
  }
}

__global__ void k_set_f32(float* p, float v) {
  if (threadIdx.x == 0) *p = v;
}

hipError_t launch_l1_loss(const float* img, const float* tgt, int64_t n, float* loss,
                          float* dimg, hipStream_t st) {
  hipLaunchKernelGGL(k_set_f32, dim3(1), dim3(64), 0, st, loss, 0.f);
  if (n <= 0) return hipGetLastError();
  const bool vec = ((uintptr_t)img % 16 == 0) && ((uintptr_t)tgt % 16 == 0) &&
                   ((uintptr_t)dimg % 16 == 0);
  const int64_t work = vec ? (n + 3) / 4 : n;
  const int grid = (int)std::min<int64_t>((work + kLossThreads - 1) / kLossThreads, 256);
  const float inv_n = (float)(1.0 / (double)n);
  if (vec)
    hipLaunchKernelGGL(k_l1_loss<true>, dim3(grid), dim3(kLossThreads), 0, st, img, tgt, n,
                       inv_n, loss, dimg);
  else
    hipLaunchKernelGGL(k_l1_loss<false>, dim3(grid), dim3(kLossThreads), 0, st, img, tgt, n,
                       inv_n, loss, dimg);
  return hipGetLastError();
}

}  // namespace xpr
