// Binning (section "Rasterizer" of the paper): exclusive prefix sum of the
// per-record tile counts, replication of each record once per tile of its
// rect with tile id G_v + y tx + x (row-major in the rect), stable LSD radix
// sort by (tile id, depth), and per-tile [start, end) ranges.
//
// All kernels here are bound by HBM traffic. The radix sort is a
// reduce-then-scan LSD sort with 8-bit digits: per pass a histogram kernel,
// a device-wide scan of the digit-major block counts, and a scatter kernel
// that ranks the 4096 keys of a block stably in LDS (wave64 ballots give the
// rank among lanes holding the same digit) and writes them out in digit
// order, so global stores are contiguous runs per digit.
#include <algorithm>
#include <cmath>

#include "xpr_internal.h"

namespace xpr {

constexpr int kScanItems = 16;
constexpr int kScanTile = 256 * kScanItems;
constexpr int kSortItems = 16;
constexpr int kSortTile = 256 * kSortItems;  // keys per scatter block
constexpr int kSortWaves = 4;
// threads of a radix scatter block (kSortTile keys, 8 per thread: about
// 75 VGPRs, six waves per SIMD, against 124 and four with 256 threads)
constexpr int kRadixThreads = 512;
// threads of a first-tile-pass block (kSortTile pairs generated in LDS)
constexpr int kPairThreads = 512;
// threads of a first-pass histogram block (one sort block's records: about
// a hundred and fifty at this workload, so one wave)
constexpr int kHistThreads = 64;

// ---------------------------------------------------------------------------
// Block-level helpers (256 threads = 4 waves unless they take NT).

__device__ __forceinline__ uint32_t wave_incl_scan(uint32_t x) {
  const int lane = threadIdx.x & 63;
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    const uint32_t y = __shfl_up(x, d, 64);
    if (lane >= d) x += y;
  }
  return x;
}

// Inclusive scan over the 64 lanes with DPP (no LDS crossbar): prefix sums
// inside each row of 16 lanes (row_shr 1, 2, 4, 8, sources outside the row
// read 0), then row 0's total into row 1 and row 2's into row 3
// (row_bcast:15), then the total of rows 0-1 into rows 2 and 3
// (row_bcast:31). Every lane must be active.
template <int CTRL, int ROW_MASK = 0xf>
__device__ __forceinline__ uint32_t dpp_u(uint32_t x) {
  return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, CTRL, ROW_MASK, 0xf, true);
}
__device__ __forceinline__ uint32_t wave_incl_scan_dpp(uint32_t x) {
  x += dpp_u<0x111>(x);
  x += dpp_u<0x112>(x);
  x += dpp_u<0x114>(x);
  x += dpp_u<0x118>(x);
  x += dpp_u<0x142, 0xa>(x);
  x += dpp_u<0x143, 0xc>(x);
  return x;
}
__device__ __forceinline__ uint32_t lane63_u(uint32_t x) {
  return (uint32_t)__builtin_amdgcn_readlane((int)x, 63);
}

// Exclusive scan of one value per thread over a 256-thread block.
__device__ __forceinline__ uint32_t block_excl_scan256(uint32_t x, uint32_t* s_wave,
                                                       uint32_t* total) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const uint32_t inc = wave_incl_scan(x);
  if (lane == 63) s_wave[w] = inc;
  __syncthreads();
  uint32_t off = 0;
  for (int k = 0; k < w; ++k) off += s_wave[k];
  if (total) *total = s_wave[0] + s_wave[1] + s_wave[2] + s_wave[3];
  __syncthreads();
  return off + inc - x;
}

// Exclusive scan of one value per thread over an NT-thread block.
template <int NT>
__device__ __forceinline__ uint32_t block_excl_scan(uint32_t x, uint32_t* s_wave) {
  constexpr int NW = NT / 64;
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const uint32_t inc = wave_incl_scan(x);
  if (lane == 63) s_wave[w] = inc;
  __syncthreads();
  uint32_t off = 0;
#pragma unroll
  for (int k = 0; k < NW; ++k) off += k < w ? s_wave[k] : 0u;
  __syncthreads();
  return off + inc - x;
}

// Exclusive running maximum of one value per thread over a 256-thread block.
__device__ __forceinline__ uint32_t block_excl_max256(uint32_t x, uint32_t* s_wave) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  uint32_t inc = x;
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    const uint32_t y = __shfl_up(inc, d, 64);
    if (lane >= d) inc = max(inc, y);
  }
  uint32_t ex = __shfl_up(inc, 1, 64);
  if (lane == 0) ex = 0;
  if (lane == 63) s_wave[w] = inc;
  __syncthreads();
  for (int k = 0; k < w; ++k) ex = max(ex, s_wave[k]);
  __syncthreads();
  return ex;
}

// Exclusive running maximum of one value per thread over an NT-thread block.
template <int NT>
__device__ __forceinline__ uint32_t block_excl_max(uint32_t x, uint32_t* s_wave) {
  constexpr int NW = NT / 64;
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  uint32_t inc = x;
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    const uint32_t y = __shfl_up(inc, d, 64);
    if (lane >= d) inc = max(inc, y);
  }
  uint32_t ex = __shfl_up(inc, 1, 64);
  if (lane == 0) ex = 0;
  if (lane == 63) s_wave[w] = inc;
  __syncthreads();
#pragma unroll
  for (int k = 0; k < NW; ++k)
    if (k < w) ex = max(ex, s_wave[k]);
  __syncthreads();
  return ex;
}

__device__ __forceinline__ uint64_t block_sum256_u64(uint64_t x, uint64_t* s_wave) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
#pragma unroll
  for (int d = 32; d >= 1; d >>= 1) x += __shfl_xor(x, d, 64);
  if (lane == 0) s_wave[w] = x;
  __syncthreads();
  const uint64_t t = s_wave[0] + s_wave[1] + s_wave[2] + s_wave[3];
  __syncthreads();
  return t;
}

// ---------------------------------------------------------------------------
// Device-wide exclusive scan of n uint32 values (n known on the host), two
// kernels: block sums, then block scans, each block adding the sum of the
// preceding block sums (the grand total, if wanted, from the last block).

struct LoadArray {
  const uint32_t* p;
  __device__ __forceinline__ uint32_t operator()(int64_t i) const { return p[i]; }
};
struct LoadCount {  // tile counts of records, in record order
  const int32_t* tc;
  __device__ __forceinline__ uint32_t operator()(int64_t i) const { return (uint32_t)tc[i]; }
};

struct LoadMask {  // p[i] & m
  const uint32_t* p;
  uint32_t m;
  __device__ __forceinline__ uint32_t operator()(int64_t i) const { return p[i] & m; }
};
struct LoadShift {  // p[i] >> s
  const uint32_t* p;
  int s;
  __device__ __forceinline__ uint32_t operator()(int64_t i) const { return p[i] >> s; }
};
struct LoadGather {  // p[idx[i]]
  const uint32_t* p;
  const uint32_t* idx;
  __device__ __forceinline__ uint32_t operator()(int64_t i) const { return p[idx[i]]; }
};

template <class L>
__global__ __launch_bounds__(256) void k_scan_reduce(L load, int64_t n, uint64_t* partials) {
  __shared__ uint64_t s_wave[4];
  const int64_t base = (int64_t)blockIdx.x * kScanTile;
  // all loads first (indices clamped, out-of-range items weighted 0)
  uint32_t x[kScanItems];
#pragma unroll
  for (int j = 0; j < kScanItems; ++j) x[j] = load(min(base + j * 256 + threadIdx.x, n - 1));
  uint64_t s = 0;
#pragma unroll
  for (int j = 0; j < kScanItems; ++j)
    if (base + j * 256 + threadIdx.x < n) s += x[j];
  s = block_sum256_u64(s, s_wave);
  if (threadIdx.x == 0) partials[blockIdx.x] = s;
}

template <class L>
__global__ __launch_bounds__(256) void k_scan_down(L load, int64_t n, const uint64_t* partials,
                                                   uint32_t* out, int64_t* total) {
  // 16 items per thread, staged through LDS with one pad word per 16 so the
  // per-thread contiguous reads are free of bank conflicts.
  __shared__ uint32_t s[kScanTile + kScanTile / 16];
  __shared__ uint32_t s_wave[4];
  __shared__ uint64_t s_wave64[4];
  const int64_t base = (int64_t)blockIdx.x * kScanTile;
  const int t = threadIdx.x;
  {
    uint32_t y[kScanItems];
#pragma unroll
    for (int j = 0; j < kScanItems; ++j) y[j] = load(min(base + j * 256 + t, n - 1));
#pragma unroll
    for (int j = 0; j < kScanItems; ++j) {
      const int i = j * 256 + t;
      s[i + (i >> 4)] = (base + i < n) ? y[j] : 0u;
    }
  }
  __syncthreads();
  uint32_t x[kScanItems];
  uint32_t run = 0;
#pragma unroll
  for (int j = 0; j < kScanItems; ++j) {
    x[j] = s[17 * t + j];
    run += x[j];
  }
  uint32_t excl = block_excl_scan256(run, s_wave, nullptr);
  // this block's offset: the sum of the preceding blocks' totals (a few
  // hundred at most), summed here instead of in a separate scan launch
  uint64_t pre = 0;
  for (int64_t b = t; b < (int64_t)blockIdx.x; b += 256) pre += partials[b];
  const uint64_t boff64 = block_sum256_u64(pre, s_wave64);
  if (total && t == 0 && blockIdx.x == gridDim.x - 1)
    *total = (int64_t)(boff64 + partials[blockIdx.x]);
  const uint32_t boff = (uint32_t)boff64;
#pragma unroll
  for (int j = 0; j < kScanItems; ++j) {
    const uint32_t v = x[j];
    s[17 * t + j] = boff + excl;
    excl += v;
  }
  __syncthreads();
#pragma unroll
  for (int j = 0; j < kScanItems; ++j) {
    const int i = j * 256 + t;
    if (base + i < n) out[base + i] = s[i + (i >> 4)];
  }
}

template <class L>
static hipError_t device_scan(L load, int64_t n, uint32_t* out, uint64_t* partials,
                              int64_t* total, hipStream_t st) {
  if (n <= 0) {
    return hipSuccess;
  }
  const int64_t nb = (n + kScanTile - 1) / kScanTile;
  hipLaunchKernelGGL(k_scan_reduce<L>, dim3(nb), dim3(256), 0, st, load, n, partials);
  hipLaunchKernelGGL(k_scan_down<L>, dim3(nb), dim3(256), 0, st, load, n, partials, out, total);
  return hipGetLastError();
}

// Exclusive scan of each digit's block counts of a radix pass, in place
// (counts[d nb + b] becomes the count of digit d in blocks before b), and
// each digit's total over all blocks (tot[d]). The scatter kernels turn the
// totals into digit starts themselves. A digit's column is cut into chunks
// of kScanTile counts: with one chunk (up to 4096 sort blocks, 16M keys) a
// single launch scans every column; longer columns take a reduce launch over
// all chunks, then a scan launch whose chunks add the sums of the earlier
// chunks of their column.
__global__ __launch_bounds__(256) void k_digit_reduce(const uint32_t* __restrict__ counts, int nb,
                                                      int nchunk, uint32_t* __restrict__ csum) {
  __shared__ uint64_t s_wave[4];
  const int d = blockIdx.x / nchunk, ch = blockIdx.x - d * nchunk;
  const uint32_t* c = counts + (int64_t)d * nb;
  const int base = ch * kScanTile;
  uint32_t x[kScanItems];
#pragma unroll
  for (int j = 0; j < kScanItems; ++j) {
    const int i = base + j * 256 + (int)threadIdx.x;
    x[j] = i < nb ? c[i] : 0u;
  }
  uint64_t s = 0;
#pragma unroll
  for (int j = 0; j < kScanItems; ++j) s += x[j];
  s = block_sum256_u64(s, s_wave);
  if (threadIdx.x == 0) csum[blockIdx.x] = (uint32_t)s;
}

// csum: the chunk sums of k_digit_reduce, or null with one chunk per column.
__global__ __launch_bounds__(256) void k_digit_scan(uint32_t* __restrict__ counts, int nb,
                                                    int nchunk, const uint32_t* __restrict__ csum,
                                                    uint32_t* __restrict__ tot) {
  __shared__ uint32_t s[kScanTile + kScanTile / 16];
  __shared__ uint32_t s_wave[4];
  const int d = blockIdx.x / nchunk, ch = blockIdx.x - d * nchunk;
  uint32_t* c = counts + (int64_t)d * nb;
  const int base = ch * kScanTile;
  const int t = threadIdx.x;
  // the sums of the column's earlier chunks (a few at most)
  uint32_t carry = 0;
  if (csum)
    for (int k = 0; k < ch; ++k) carry += csum[d * nchunk + k];
  {
    uint32_t y[kScanItems];
#pragma unroll
    for (int j = 0; j < kScanItems; ++j) {
      const int i = base + j * 256 + t;
      y[j] = i < nb ? c[i] : 0u;
    }
#pragma unroll
    for (int j = 0; j < kScanItems; ++j) {
      const int i = j * 256 + t;
      s[i + (i >> 4)] = y[j];
    }
  }
  __syncthreads();
  uint32_t x[kScanItems];
  uint32_t run = 0;
#pragma unroll
  for (int j = 0; j < kScanItems; ++j) {
    x[j] = s[17 * t + j];
    run += x[j];
  }
  uint32_t total;
  uint32_t excl = carry + block_excl_scan256(run, s_wave, &total);
#pragma unroll
  for (int j = 0; j < kScanItems; ++j) {
    s[17 * t + j] = excl;
    excl += x[j];
  }
  __syncthreads();
#pragma unroll
  for (int j = 0; j < kScanItems; ++j) {
    const int i = j * 256 + t;
    if (base + i < nb) c[base + i] = s[i + (i >> 4)];
  }
  if (t == 0 && ch == nchunk - 1) tot[d] = carry + total;
}

// csum: nchunk * radix words of scratch (unused with one chunk).
static hipError_t digit_scan(uint32_t* counts, int nb, int radix, uint32_t* tot, uint32_t* csum,
                             hipStream_t st) {
  if (nb <= 0) return hipSuccess;
  const int nchunk = (nb + kScanTile - 1) / kScanTile;
  if (nchunk > 1)
    hipLaunchKernelGGL(k_digit_reduce, dim3(radix * nchunk), dim3(256), 0, st, counts, nb, nchunk,
                       csum);
  hipLaunchKernelGGL(k_digit_scan, dim3(radix * nchunk), dim3(256), 0, st, counts, nb, nchunk,
                     nchunk > 1 ? csum : (const uint32_t*)nullptr, tot);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Small utility kernels.

__global__ void k_fill_u32(uint32_t* p, int64_t n, uint32_t v) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

// Zero fill in 16-byte stores (the backward's gradient buffer: 9 floats per
// record, a pure write stream).
__global__ void k_zero_x4(uint4* p, int64_t n4) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n4) p[i] = make_uint4(0u, 0u, 0u, 0u);
}

__global__ void k_set_i64(int64_t* p, int64_t v) {
  if (threadIdx.x == 0) *p = v;
}

// Depth-presort keys: the float bits of the depth (positive floats order
// like their bit patterns); records that touch no tile sort last.
// Depth keys of the presort (a record that touches no tile gets the key
// 0xffffffff, which no depth has) with the identity permutation, and the
// first radix pass's digit counts (bits 0-7) of each sort block of
// kSortTile keys, written digit-major like k_radix_hist; also zeroes the
// pair count that k_sorted_rects accumulates.
__global__ __launch_bounds__(256) void k_depth_keys(const float* __restrict__ depth,
                                                    const int32_t* __restrict__ tc, int64_t n,
                                                    uint32_t* __restrict__ key,
                                                    uint32_t* __restrict__ perm,
                                                    int64_t* n_isect,
                                                    uint32_t* __restrict__ counts, int nblocks) {
  constexpr int COPIES = 8;
  __shared__ uint32_t h[COPIES][256];
  const int t = threadIdx.x;
  for (int k = t; k < COPIES * 256; k += 256) (&h[0][0])[k] = 0;
  if (blockIdx.x == 0 && t == 0) *n_isect = 0;
  const int64_t base = (int64_t)blockIdx.x * kSortTile;
  float dd[kSortItems];
  int32_t cc[kSortItems];
#pragma unroll
  for (int j = 0; j < kSortItems; ++j) {
    const int64_t i = min(base + j * 256 + t, n - 1);
    dd[j] = depth[i];
    cc[j] = tc[i];
  }
  __syncthreads();
  uint32_t* mine = h[t & (COPIES - 1)];
#pragma unroll
  for (int j = 0; j < kSortItems; ++j) {
    const int64_t i = base + j * 256 + t;
    if (i < n) {
      const uint32_t k = cc[j] > 0 ? __float_as_uint(dd[j]) : 0xffffffffu;
      key[i] = k;
      perm[i] = (uint32_t)i;
      atomicAdd(&mine[k & 255u], 1u);
    }
  }
  __syncthreads();
  uint32_t c = 0;
#pragma unroll
  for (int k = 0; k < COPIES; ++k) c += h[k][t];
  counts[(int64_t)t * nblocks + blockIdx.x] = c;
}

// ---------------------------------------------------------------------------
// Replication: block b covers records [256 b, 256 b + 256) in the (possibly
// depth-permuted) order; its pairs occupy [off[first], off[last] + tc[last]),
// and threads stride over that range, locating their record by binary search
// in LDS, so every wave writes contiguous pairs whatever the tile counts.

template <bool PERM, bool KEY64>
__global__ __launch_bounds__(256) void k_duplicate(Batch B, const short4* __restrict__ rect,
                                                   const int32_t* __restrict__ tc,
                                                   const float* __restrict__ depth,
                                                   const uint32_t* __restrict__ perm,
                                                   const uint32_t* __restrict__ offsets,
                                                   int64_t n_rec, int64_t cap,
                                                   void* __restrict__ keys_out,
                                                   uint32_t* __restrict__ vals_out) {
  __shared__ uint32_t s_off[257];
  __shared__ short4 s_rect[256];
  __shared__ uint32_t s_rec[256];
  __shared__ int32_t s_tbase[256];
  __shared__ int32_t s_tx[256];
  __shared__ uint32_t s_depth[256];
  const int t = threadIdx.x;
  // no XCD swizzle here: blocks hold very different pair counts (the front
  // of the depth order has the largest footprints), and round-robin
  // dispatch spreads them evenly over the XCDs
  const int blk = blockIdx.x;
  const int64_t i = (int64_t)blk * 256 + t;
  const int64_t last = min(n_rec, (int64_t)blk * 256 + 256) - 1;
  if (i <= last) {
    const uint32_t r = PERM ? perm[i] : (uint32_t)i;
    int v = 0;
    for (int k = 1; k < B.n_views; ++k)
      if ((int32_t)r >= B.v[k].rec_off) v = k;
    s_rec[t] = r;
    s_off[t] = offsets[i];
    s_rect[t] = rect[r];
    s_tbase[t] = B.v[v].tile_off;
    s_tx[t] = B.v[v].tiles_x;
    s_depth[t] = __float_as_uint(depth[r]);
    if (i == last) s_off[256] = offsets[i] + (uint32_t)tc[r];
  }
  __syncthreads();
  const int nvalid = (int)(last - (int64_t)blk * 256 + 1);
  if (t >= nvalid) s_off[t] = s_off[256];
  __syncthreads();
  const uint32_t beg = s_off[0], end = s_off[256];
  for (uint32_t p = beg + t; p < end; p += 256) {
    // last j with s_off[j] <= p
    int lo = 0, hi = 255;
    while (lo < hi) {
      const int mid = (lo + hi + 1) >> 1;
      if (s_off[mid] <= p) lo = mid; else hi = mid - 1;
    }
    const short4 rc = s_rect[lo];
    const uint32_t local = p - s_off[lo];
    const uint32_t w = (uint32_t)(rc.z - rc.x);
    const uint32_t yy = local / w;
    const uint32_t xx = local - yy * w;
    const uint32_t tile = (uint32_t)s_tbase[lo] + ((uint32_t)rc.y + yy) * (uint32_t)s_tx[lo] +
                          (uint32_t)rc.x + xx;
    if (p < cap) {
      if (KEY64)
        static_cast<uint64_t*>(keys_out)[p] = ((uint64_t)tile << 32) | s_depth[lo];
      else
        static_cast<uint32_t*>(keys_out)[p] = tile;
      vals_out[p] = s_rec[lo];
    }
  }
}

// ---------------------------------------------------------------------------
// LSD radix sort with BITS-bit digits (7 or 8).

template <int BITS, typename K>
__device__ __forceinline__ uint32_t digit_of(K k, int shift) {
  return (uint32_t)(k >> shift) & ((1u << BITS) - 1u);
}

// Lanes of the wave holding the same BITS-bit digit (among active lanes).
// Per bit, s is the bit sign-extended (0 or all ones: one bitfield extract),
// the ballot compares s itself (the compare intrinsic keeps the compiler
// from re-deriving the bit with a shift and a second compare), and the
// lanes with the bit set keep the ballot, the others its complement:
// lo &= ~(ballot ^ s) in each 32-bit half, one gfx950 three-input bit
// operation (truth table 0x90 on (lo, ballot, s)), written as the builtin
// because the compiler otherwise splits it into xor and or chains. Four
// VALU instructions per bit.
template <int BITS>
__device__ __forceinline__ uint64_t match_digit(uint32_t d, bool active) {
  const uint64_t a = __ballot(active);
  uint32_t lo = (uint32_t)a, hi = (uint32_t)(a >> 32);
#pragma unroll
  for (int b = 0; b < BITS; ++b) {
    const uint32_t s = (uint32_t)__builtin_amdgcn_sbfe((int)d, b, 1);
    const uint64_t bb = __builtin_amdgcn_uicmp(s, 0u, 33);  // 33: not equal
    lo = __builtin_amdgcn_bitop3_b32(lo, (uint32_t)bb, s, 0x90);
    hi = __builtin_amdgcn_bitop3_b32(hi, (uint32_t)(bb >> 32), s, 0x90);
  }
  return ((uint64_t)hi << 32) | lo;
}

__device__ __forceinline__ int64_t clamp_n(const int64_t* n_dev, int64_t cap) {
  const int64_t n = n_dev ? *n_dev : cap;
  return n < cap ? n : cap;
}

// Partition of sort block b when the grid holds nblocks blocks but only the
// first ceil(n / kSortTile) hold items (a grid sized from a capacity): the
// live blocks are XCD-swizzled among themselves, so every XCD gets its share
// of the real work, and the rest map to themselves (their digit counts are
// zero).
__device__ __forceinline__ int live_swizzle(int b, int nblocks, int64_t n) {
  const int64_t need = (n + kSortTile - 1) / kSortTile;
  const int live = need < nblocks ? (int)need : nblocks;
  return b < live ? xcd_swizzle(b, live) : b;
}

// Digit counts of one block of kSortTile keys, written digit-major
// (counts[d * nblocks + b]) for the scan. Eight lane-indexed copies of the
// histogram keep LDS atomic collisions at most 8-way.
template <int BITS, typename K>
__global__ __launch_bounds__(256) void k_radix_hist(const K* __restrict__ keys,
                                                    const int64_t* n_dev, int64_t cap, int shift,
                                                    uint32_t* __restrict__ counts, int nblocks) {
  constexpr int RADIX = 1 << BITS;
  constexpr int COPIES = 8;
  __shared__ uint32_t h[COPIES][RADIX];
  const int t = threadIdx.x;
  for (int k = t; k < COPIES * RADIX; k += 256) (&h[0][0])[k] = 0;
  __syncthreads();
  const int64_t n = clamp_n(n_dev, cap);
  const int part = live_swizzle(blockIdx.x, nblocks, n);
  const int64_t base = (int64_t)part * kSortTile;
  uint32_t* mine = h[t & (COPIES - 1)];
  if (base < n) {
    // all loads first (indices clamped into the list), then the counting:
    // a load-use pair per item would serialise the memory latencies
    K kk[kSortItems];
#pragma unroll
    for (int j = 0; j < kSortItems; ++j) kk[j] = keys[min(base + j * 256 + t, n - 1)];
#pragma unroll
    for (int j = 0; j < kSortItems; ++j)
      if (base + j * 256 + t < n) atomicAdd(&mine[digit_of<BITS>(kk[j], shift)], 1u);
  }
  __syncthreads();
  for (int d = t; d < RADIX; d += 256) {
    uint32_t c = 0;
#pragma unroll
    for (int k = 0; k < COPIES; ++k) c += h[k][d];
    counts[(int64_t)d * nblocks + part] = c;
  }
}

// Writes a block's keys, ranked into digit order in LDS, to their global
// runs. With RANGES (the last pass over tile keys) the output is the final
// order, so a tile's pairs form one contiguous span across all blocks: each
// block records where the tiles it holds begin and end inside it, and the
// minimum start / maximum end over blocks are the tile ranges. Keys are only
// stored when kout is given. With aux_dst, aux_dst[g] = aux_src[value] is
// stored beside each value (a per-record quantity carried into sorted
// order).
template <int BITS, typename KS, typename KO, bool RANGES, int NT = 256>
__device__ __forceinline__ void write_sorted(const KS* skey, const uint32_t* sval,
                                             const uint32_t* gbase, int nvalid, int shift,
                                             KO* __restrict__ kout, uint32_t* __restrict__ vout,
                                             int2* __restrict__ ranges,
                                             const int32_t* __restrict__ aux_src,
                                             uint32_t* __restrict__ aux_dst) {
  for (int k = threadIdx.x; k < nvalid; k += NT) {
    const KS kk = skey[k];
    const uint32_t g = gbase[digit_of<BITS>(kk, shift)] + (uint32_t)k;
    if (!RANGES || kout) kout[g] = (KO)kk;
    const uint32_t v = sval[k];
    vout[g] = v;
    if (aux_dst) aux_dst[g] = (uint32_t)aux_src[v];
    if (RANGES) {
      const uint32_t tile = (uint32_t)kk;
      if (k == 0 || (uint32_t)skey[k - 1] != tile) atomicMin(&ranges[tile].x, (int)g);
      if (k == nvalid - 1 || (uint32_t)skey[k + 1] != tile) atomicMax(&ranges[tile].y, (int)g + 1);
    }
  }
}

// Stable scatter of one block of kSortTile keys on NT threads (NT / 64
// waves, kSortTile / NT keys per thread): rank the block's keys by digit in
// LDS (per wave, slot by slot, the wave64 ballot match gives the rank among
// lanes with the same digit), then write them out in digit order so each
// digit's run is a contiguous global store. More threads hold fewer keys
// each: fewer registers per thread, more waves per CU.
template <int BITS, typename K, bool RANGES, int NT>
__global__ __launch_bounds__(NT) void k_radix_scatter(const K* __restrict__ kin,
                                                      const uint32_t* __restrict__ vin,
                                                      K* __restrict__ kout,
                                                      uint32_t* __restrict__ vout,
                                                      const int64_t* n_dev, int64_t cap,
                                                      int shift,
                                                      const uint32_t* __restrict__ offsets,
                                                      const uint32_t* __restrict__ dtot,
                                                      int nblocks, int2* __restrict__ ranges,
                                                      const int32_t* __restrict__ aux_src,
                                                      uint32_t* __restrict__ aux_dst) {
  constexpr int RADIX = 1 << BITS;
  constexpr int NW = NT / 64;
  constexpr int IT = kSortTile / NT;
  static_assert(RADIX <= NT && IT * NT == kSortTile, "radix scatter shape");
  __shared__ uint32_t wcnt[NW][RADIX];
  __shared__ uint32_t gbase[RADIX];  // global offset of the digit's run minus its block start
  __shared__ uint32_t s_wave[NW];
  __shared__ K skey[kSortTile];
  __shared__ uint32_t sval[kSortTile];
  const int t = threadIdx.x, w = t >> 6, lane = t & 63;
  for (int k = t; k < NW * RADIX; k += NT) (&wcnt[0][0])[k] = 0;
  __syncthreads();
  const int64_t n = clamp_n(n_dev, cap);
  const int part = live_swizzle(blockIdx.x, nblocks, n);
  const int64_t bbase = (int64_t)part * kSortTile;
  if (bbase >= n) return;  // whole block beyond the list: no counts, nothing to write
  const int64_t base = bbase + w * (64 * IT);
  const uint64_t lt = lanemask_lt();
  K key[IT];
  uint32_t val[IT];
  uint32_t lofs[IT];
  // all loads first (indices clamped into the list), then the ranking
#pragma unroll
  for (int j = 0; j < IT; ++j) {
    const int64_t idx = min(base + j * 64 + lane, n - 1);
    key[j] = kin[idx];
    val[j] = vin[idx];
  }
  // digit t's total and its count in earlier blocks
  const uint32_t my_tot = t < RADIX ? dtot[t] : 0u;
  const uint32_t my_off = t < RADIX ? offsets[(int64_t)t * nblocks + part] : 0u;
#pragma unroll
  for (int j = 0; j < IT; ++j) {
    const bool ok = base + j * 64 + lane < n;
    const uint32_t d = digit_of<BITS>(key[j], shift);
    const uint64_t m = match_digit<BITS>(d, ok);
    const uint32_t before = wcnt[w][d];
    lofs[j] = before + (uint32_t)__popcll(m & lt);
    if (ok && (m & lt) == 0) wcnt[w][d] = before + (uint32_t)__popcll(m);
  }
  __syncthreads();
  // digit t: the waves' counts, the block's exclusive start, per-wave starts
  uint32_t c[NW], tot = 0;
#pragma unroll
  for (int q = 0; q < NW; ++q) {
    c[q] = t < RADIX ? wcnt[q][t] : 0u;
    tot += c[q];
  }
  const uint32_t start = block_excl_scan<NT>(tot, s_wave);
  const uint32_t dstart = block_excl_scan<NT>(my_tot, s_wave);
  if (t < RADIX) {
    gbase[t] = dstart + my_off - start;
    uint32_t s = start;
#pragma unroll
    for (int q = 0; q < NW; ++q) {
      wcnt[q][t] = s;
      s += c[q];
    }
  }
  __syncthreads();
#pragma unroll
  for (int j = 0; j < IT; ++j) {
    const int64_t idx = base + j * 64 + lane;
    if (idx < n) {
      const uint32_t pos = wcnt[w][digit_of<BITS>(key[j], shift)] + lofs[j];
      skey[pos] = key[j];
      sval[pos] = val[j];
    }
  }
  __syncthreads();
  const int64_t rem = n - bbase;
  const int nvalid = rem <= 0 ? 0 : (rem < kSortTile ? (int)rem : kSortTile);
  write_sorted<BITS, K, K, RANGES, NT>(skey, sval, gbase, nvalid, shift, kout, vout, ranges,
                                       aux_src, aux_dst);
}

// ---------------------------------------------------------------------------
// Replication fused into the first pass of the tile sort (depth-presort
// path). The pairs are never stored unsorted: the first pass's histogram and
// scatter each regenerate the pairs of their sort block from the records.
// Sort block b owns pairs [b T, b T + T) of the depth-ordered pair sequence
// (T = kSortTile); first[b] is the record (depth-order position) holding its
// first pair, and first[b + 1] the one holding the pair after its last, so
// records first[b] .. first[b + 1] hold all of its pairs.

// The rect of every record in depth order (perm: the record at each depth-
// order position, key its sorted depth key): one gather of the rect per
// visible record, all of a thread's 16 in flight together, so the pair
// records below read their rects contiguously. A record's tile count is its
// rect's area (the projection gives a record that touches no tile an empty
// rect and the key 0xffffffff, which no depth has). Each block of kSortTile
// positions writes its total tile count to partials[b] and adds it to
// *n_isect (zeroed by k_depth_keys), so the pair count is known when the
// depth presort ends and k_pair_records scans the counts itself. tc_sorted
// (the counts in depth order) is written when given.
__global__ __launch_bounds__(256) void k_sorted_rects(const short4* __restrict__ rect,
                                                      const uint32_t* __restrict__ key,
                                                      const uint32_t* __restrict__ perm,
                                                      int64_t n_rec,
                                                      short4* __restrict__ rect_sorted,
                                                      uint32_t* __restrict__ tc_sorted,
                                                      uint64_t* __restrict__ partials,
                                                      int64_t* n_isect) {
  __shared__ uint64_t s_wave[4];
  const int t = threadIdx.x;
  const int64_t base = (int64_t)blockIdx.x * kSortTile;
  uint32_t kk[kSortItems], pp[kSortItems];
#pragma unroll
  for (int i = 0; i < kSortItems; ++i) {
    const int64_t j = min(base + i * 256 + t, n_rec - 1);
    kk[i] = key[j];
    pp[i] = perm[j];
  }
  short4 rc[kSortItems];
#pragma unroll
  for (int i = 0; i < kSortItems; ++i) {
    rc[i] = make_short4(0, 0, 0, 0);
    if (base + i * 256 + t < n_rec && kk[i] != 0xffffffffu) rc[i] = rect[pp[i]];
  }
  uint64_t s = 0;
#pragma unroll
  for (int i = 0; i < kSortItems; ++i) {
    const int64_t j = base + i * 256 + t;
    if (j < n_rec) {
      const uint32_t tc = (uint32_t)((rc[i].z - rc[i].x) * (rc[i].w - rc[i].y));
      rect_sorted[j] = rc[i];
      if (tc_sorted) tc_sorted[j] = tc;
      s += tc;
    }
  }
  s = block_sum256_u64(s, s_wave);
  if (t == 0) {
    partials[blockIdx.x] = s;
    atomicAdd(reinterpret_cast<unsigned long long*>(n_isect), (unsigned long long)s);
  }
}

// One pass over the records in depth order, kSortTile per block (wave w
// takes positions base + 1024 w + 64 i + lane): a record's pair offset is
// the tile count of all earlier records, from the block totals of
// k_sorted_rects and wave scans of the counts. Writes the packed record
// each sort block reads contiguously (pair offset, record id, tile id of
// the rect's top-left corner, rect width | tiles_x << 16), and first[b] for
// every block b with b T < n, plus first[ceil(n / T)] = the record holding
// pair n - 1, where n = min(I, capacity).
__global__ __launch_bounds__(256) void k_pair_records(Batch B,
                                                      const short4* __restrict__ rect_sorted,
                                                      const uint32_t* __restrict__ perm,
                                                      const uint64_t* __restrict__ partials,
                                                      int64_t n_rec, const int64_t* n_isect,
                                                      int64_t cap, uint4* __restrict__ packed,
                                                      uint32_t* __restrict__ first) {
  __shared__ uint64_t s_wave64[4];
  __shared__ uint32_t s_wtot[4];
  const int t = threadIdx.x, w = t >> 6, lane = t & 63;
  const int64_t wbase = (int64_t)blockIdx.x * kSortTile + w * (64 * kSortItems);
  short4 rc[kSortItems];
  uint32_t rid[kSortItems];
#pragma unroll
  for (int i = 0; i < kSortItems; ++i) {
    const int64_t j = min(wbase + i * 64 + lane, n_rec - 1);
    rc[i] = rect_sorted[j];
    rid[i] = perm[j];
  }
  // the tile counts of all earlier blocks
  uint64_t pre = 0;
  for (int b = t; b < (int)blockIdx.x; b += 256) pre += partials[b];
  const uint64_t boff = block_sum256_u64(pre, s_wave64);
  const int64_t n = clamp_n(n_isect, cap);
  // the wave's exclusive scan of its 1024 counts, then the waves' offsets
  uint32_t ex[kSortItems];
  uint32_t carry = 0;
#pragma unroll
  for (int i = 0; i < kSortItems; ++i) {
    const uint32_t tc = wbase + i * 64 + lane < n_rec
                            ? (uint32_t)((rc[i].z - rc[i].x) * (rc[i].w - rc[i].y))
                            : 0u;
    const uint32_t inc = wave_incl_scan_dpp(tc);
    ex[i] = carry + inc - tc;
    carry += lane63_u(inc);
  }
  if (lane == 0) s_wtot[w] = carry;
  __syncthreads();
  uint32_t woff = 0;
  for (int k = 0; k < w; ++k) woff += s_wtot[k];
#pragma unroll
  for (int i = 0; i < kSortItems; ++i) {
    const int64_t j = wbase + i * 64 + lane;
    if (j >= n_rec) continue;
    const int64_t o = (int64_t)(boff + woff + ex[i]);
    const uint32_t tc = (uint32_t)((rc[i].z - rc[i].x) * (rc[i].w - rc[i].y));
    const int64_t e = min(o + (int64_t)tc, n);
    if (e <= o) continue;
    const uint32_t r = rid[i];
    int v = 0;
    for (int q = 1; q < B.n_views; ++q)
      if ((int32_t)r >= B.v[q].rec_off) v = q;
    const uint32_t tx = (uint32_t)B.v[v].tiles_x;
    packed[j] = make_uint4((uint32_t)o, r,
                           (uint32_t)B.v[v].tile_off + (uint32_t)rc[i].y * tx + (uint32_t)rc[i].x,
                           (uint32_t)(rc[i].z - rc[i].x) | (tx << 16));
    for (int64_t b = (o + kSortTile - 1) / kSortTile; b * kSortTile < e; ++b)
      first[b] = (uint32_t)j;
    if (e == n) first[(n + kSortTile - 1) / kSortTile] = (uint32_t)j;
  }
}

// ---------------------------------------------------------------------------
// Per-(Gaussian, tile) cull (tile_cull of XPR-3DGS, the StopThePop-style
// test of the XPR-3DGS section): a pair is kept iff the power
// 0.5 (x - mu)^T conic (x - mu), minimised over the tile's pixel-sample box
// [tx tw, tx tw + tw - 1] x [ty th, ty th + th - 1] (clipped to the image),
// is at most log(o / alpha_min). For 3DGUT (tile_cull of XPR-3DGUT) the box
// is first extended by one pixel in x and y, on the UT footprint and o'.
//
// Equivalently, the tile meets the ellipse E = {q(d) <= 2 log(o / alpha_min)}
// with q(d) = a dx^2 + 2 b dx dy + c dy^2. E is convex, so in each tile row
// the kept tiles are the ones whose x range meets the x extent [xl, xr] of
// E inside the row's y strip, a single run of columns found in closed form:
// from (a dx + b dy)^2 = a q - det dy^2, the chord of E at height dy spans
// dx = (-b dy -/+ sqrt(a lvl - det dy^2)) / a, its right end is concave in
// dy with its peak at the rightmost point of E (dy = -b ex / c), so the
// strip's xr is that end at the peak clamped into the strip (likewise xl).
// Evaluated in float64 from the float32 shader data, without contracted
// multiply-adds, so that the count and emit passes (separate kernels) take
// bit-identical decisions; a conic that is not positive definite has no
// bounded footprint and keeps its whole rect.

__device__ __forceinline__ int view_of_record(const Batch& B, int r) {
  int v = 0;
  for (int q = 1; q < B.n_views; ++q)
    if (r >= B.v[q].rec_off) v = q;
  return v;
}

struct RowGeom {
  double u, v, b, det;  // mean2D, conic entry b, det = a c - b^2
  double aq, pk, ey;    // a lvl, b ex / c, half height of E
  double inv_a;
  int32_t x0, x1, y0, pd;  // rect columns [x0, x1), first rect row, positive definite
  int32_t wm1, hm1;        // W - 1, H - 1 of the view
  int32_t rec, tile0;      // record id, tile id of the view's tile (0, 0)
  int32_t tiles_x, ext;     // ext: tile boxes extended by one pixel (3DGUT)
};

// Cull constants of one record (lvl = 2 log(o / alpha_min), ex the half
// width of E); q is the record's splat data.
__device__ __forceinline__ void make_geom(RowGeom& G, const Batch& B, int r,
                                          const float4* __restrict__ q, const short4 rc, double) {
#pragma clang fp contract(off)
  const float4 s0 = q[0], s1 = q[1];
  const int v = view_of_record(B, r);
  const double a = -2.0 * (double)s0.z, b = -(double)s0.w, c = -2.0 * (double)s1.x;
  G.u = s0.x;
  G.v = s0.y;
  G.b = b;
  // a c and b^2 are exact products of float32 values, so the sign of det is
  G.det = a * c - b * b;
  G.pd = a > 0.0 && G.det > 0.0 ? 1 : 0;
  const double lvl = 2.0 * log((double)s1.y / (double)B.alpha_min);
  const double id = 1.0 / G.det;
  const double ex = G.pd ? sqrt(lvl * c * id) : 0.0;
  G.ey = G.pd ? sqrt(lvl * a * id) : 0.0;
  G.aq = a * lvl;
  G.pk = b * ex / c;
  G.inv_a = 1.0 / a;
  G.x0 = rc.x;
  G.x1 = rc.z;
  G.y0 = rc.y;
  G.wm1 = B.v[v].W - 1;
  G.hm1 = B.v[v].H - 1;
  G.rec = r;
  G.tile0 = B.v[v].tile_off;
  G.tiles_x = B.v[v].tiles_x;
  G.ext = B.method == XPR_METHOD_3DGUT ? 1 : 0;
}

// Kept columns [*lo, *hi) of rect row ty. Tile sizes are powers of two, so
// the scalings by 1 / tw are exact.
__device__ __forceinline__ void cull_row(const RowGeom& G, int ty, int tw, int th, double inv_tw,
                                         int* lo, int* hi) {
#pragma clang fp contract(off)
  if (!G.pd) {
    *lo = G.x0;
    *hi = G.x1;
    return;
  }
  const double y0 = (double)ty * th;
  const double y1 = fmin(y0 + (th - 1), (double)G.hm1) + G.ext;
  const double d0 = fmax(y0 - G.v, -G.ey), d1 = fmin(y1 - G.v, G.ey);
  const double dr = fmin(fmax(-G.pk, d0), d1), dl = fmin(fmax(G.pk, d0), d1);
  const double xr = G.u + (-G.b * dr + sqrt(fmax(G.aq - G.det * dr * dr, 0.0))) * G.inv_a;
  const double xl = G.u + (-G.b * dl - sqrt(fmax(G.aq - G.det * dl * dl, 0.0))) * G.inv_a;
  // tile tx is kept iff tx tw <= xr and min(tx tw + tw - 1, W - 1) + ext >= xl
  const bool none = d0 > d1 || xl > (double)(G.wm1 + G.ext) || xr < 0.0;
  const double c_hi = floor(fmin(xr, 1e6) * inv_tw) + 1.0;
  const double c_lo = ceil((fmax(xl, -1e6) - (tw - 1) - G.ext) * inv_tw);
  const int h = min(G.x1, (int)c_hi), l = max(G.x0, (int)c_lo);
  *lo = l;
  *hi = none ? l : max(l, h);
}

// LinPrim (tile_cull of XPR-LinPrim, the per-tile chord bound of the
// XPR-LinPrim section): a pair is kept iff sigma * bound >= -log(1 -
// alpha_min), with
//   bound = max(0, min over ordered slab pairs (i, j) of
//               [max over the box corners of (m_i - m_j) + h_i + h_j]),
// m_i = a_i dx + b_i dy (a_i = -n_ix / n_iz, b_i = -n_iy / n_iz),
// h_i = 1 / |n_iz|, on the pixel-sample box of the 3DGS cull; a slab with
// |n_iz| < 1e-10 is dropped (h = +inf, a = b = 0). With lam = req / sigma
// the test is: 2 min h_i >= lam and every off-diagonal gap >= lam.
//
// The corners form the product {dx0, dx1} x {dy0, dy1}, so the gap of
// (i, j) is max(D dx0, D dx1) + max(Bd dy0, Bd dy1) + h_i + h_j with
// D = a_i - a_j, Bd = b_i - b_j, and (j, i) has the negated slopes. In a
// tile row dy0, dy1 are fixed and dx1 = dx0 + tw - 1 with dx0 = X0 - u (X0
// the tile's first pixel column), so for D != 0 the two gaps of a slab pair
// (the one with positive x slope reaches its maximum at dx1, the other at
// dx0) are >= lam exactly when, with th = lam - h_i - h_j and q = 1 / D,
//   X0 >= lc - max(bq dy0, bq dy1),  lc = (u - tw + 1) + th |q|,
//   X0 <= uc - min(bq dy0, bq dy1),  uc = u - th |q|,   bq = Bd q,
// whatever the sign of D: a row keeps the tiles whose X0 lies in the
// intersection of these intervals (one run; the gaps are affine in X0).
// A pair with D = 0 is a yes/no condition on the row (max(Bd dy) >= th and
// -min(Bd dy) >= th). A last tile column clipped by the image border has
// dx1 = W - 1 - u: its lower bounds are checked at X0 = W - tw.
struct LinGeom {
  double lc[6], uc[6], bq[6];  // slab pairs i < j with a_i != a_j
  double zb[6], zt[6];         // pairs with a_i == a_j: Bd and th (read when zm != 0)
  double v;                    // mu_2D.y - 1/2
  int32_t zm, none;            // mask of the a_i == a_j pairs; 2 min h < lam
  int32_t x0, x1, y0, wm1;     // rect columns [x0, x1), first rect row, W - 1
  int32_t hm1, rec;            // H - 1, record id
  int32_t tile0, tiles_x;      // tile id of the view's tile (0, 0), tiles per row
};

// 1 / d from the hardware reciprocal and two Newton-Raphson steps (about one
// ulp; d finite and normal).
__device__ __forceinline__ double rcp_nr(double d) {
  double x = __builtin_amdgcn_rcp(d);
  double e = fma(-d, x, 1.0);
  x = fma(x, e, x);
  e = fma(-d, x, 1.0);
  return fma(x, e, x);
}

__device__ __forceinline__ void make_geom(LinGeom& G, const Batch& B, int r,
                                          const float4* __restrict__ q, const short4 rc,
                                          double req) {
#pragma clang fp contract(off)
  const float4 q0 = q[0], q2 = q[2], q3 = q[3], q4 = q[4];
  const double c[9] = {q2.x, q2.y, q2.z, q2.w, q3.x, q3.y, q3.z, q3.w, q4.x};
  const int v = view_of_record(B, r);
  const double u = q0.x, sigma = q0.z;
  G.v = q0.y;
  const double lam = sigma > 0.0 ? req * rcp_nr(sigma) : INFINITY;
  double a[4], b[4], h[4], hm = INFINITY;
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const double e1 = (i & 2) ? -1.0 : 1.0, e2 = (i & 1) ? -1.0 : 1.0;
    const double nx = c[0] + e1 * c[3] + e2 * c[6];
    const double ny = c[1] + e1 * c[4] + e2 * c[7];
    const double nz = c[2] + e1 * c[5] + e2 * c[8];
    const bool flat = !(fabs(nz) >= 1e-10);
    const double rz = rcp_nr(flat ? 1.0 : nz);
    a[i] = flat ? 0.0 : -nx * rz;
    b[i] = flat ? 0.0 : -ny * rz;
    h[i] = flat ? INFINITY : fabs(rz);
    hm = fmin(hm, h[i]);
  }
  G.none = hm + hm >= lam ? 0 : 1;
  const double ul = u - (double)(B.tile_w - 1);
  int zm = 0, p = 0;
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = i + 1; j < 4; ++j, ++p) {
      const double D = a[i] - a[j], Bd = b[i] - b[j];
      const double th = lam - (h[i] + h[j]);
      const bool z = D == 0.0;
      const double qd = rcp_nr(z ? 1.0 : D), aq = fabs(qd);
      G.lc[p] = z ? -1e300 : ul + th * aq;
      G.uc[p] = z ? 1e300 : u - th * aq;
      G.bq[p] = z ? 0.0 : Bd * qd;
      G.zb[p] = Bd;
      G.zt[p] = th;
      zm |= z ? 1 << p : 0;
    }
  G.zm = zm;
  G.x0 = rc.x;
  G.x1 = rc.z;
  G.y0 = rc.y;
  G.wm1 = B.v[v].W - 1;
  G.hm1 = B.v[v].H - 1;
  G.rec = r;
  G.tile0 = B.v[v].tile_off;
  G.tiles_x = B.v[v].tiles_x;
}

// The LinPrim cull threshold -log(1 - alpha_min), formed on the host.
inline double lin_req(const Batch& B) { return -std::log(1.0 - (double)B.alpha_min); }

// Kept columns [*lo, *hi) of rect row ty.
__device__ __forceinline__ void cull_row(const LinGeom& G, int ty, int tw, int th, double inv_tw,
                                         int* lo, int* hi) {
#pragma clang fp contract(off)
  const double dy0 = (double)ty * th - G.v;
  const double dy1 = fmin((double)ty * th + (th - 1), (double)G.hm1) - G.v;
  double xl = -1e9, xr = 1e9;  // X0 must lie in [xl, xr]
#pragma unroll
  for (int p = 0; p < 6; ++p) {
    const double t0 = G.bq[p] * dy0, t1 = G.bq[p] * dy1;
    xl = fmax(xl, G.lc[p] - fmax(t0, t1));
    xr = fmin(xr, G.uc[p] - fmin(t0, t1));
  }
  bool none = G.none != 0;
  if (G.zm != 0) {
#pragma unroll
    for (int p = 0; p < 6; ++p) {
      const double t0 = G.zb[p] * dy0, t1 = G.zb[p] * dy1;
      const bool bad = fmax(t0, t1) < G.zt[p] || -fmin(t0, t1) < G.zt[p];
      none = none || (((G.zm >> p) & 1) && bad);
    }
  }
  const int c_lo = (int)ceil(fmin(fmax(xl, -1e9), 1e9) * inv_tw);
  const int c_hi = (int)floor(fmin(fmax(xr, -1e9), 1e9) * inv_tw) + 1;
  const int l = max(G.x0, c_lo);
  int h = none ? l : max(l, min(G.x1, c_hi));
  // the last tile column, if the image border clips its box
  if (h > l && h == G.tiles_x && (h - 1) * tw + (tw - 1) > G.wm1 &&
      !((double)(G.wm1 - (tw - 1)) >= xl))
    --h;
  *lo = l;
  *hi = h;
}

// The rows of the rects of a wave's 64 records, spread over its lanes: lane
// l's record has h rows (0 when it keeps nothing), pre = the wave's
// exclusive scan of h, and item q of the flattened row sequence belongs to
// the last record g with pre[g] <= q. Calls f(g, ty, lo, hi) for every item
// of every chunk of 64 (valid = false past the end, then lo = hi); the loop
// is wave-uniform. geo / pre are this wave's 64 LDS entries.
template <class Geo, class F>
__device__ __forceinline__ void wave_rows(const Geo* geo, const uint32_t* pre, uint32_t total,
                                          int tw, int th, F f) {
  const int lane = threadIdx.x & 63;
  const double inv_tw = 1.0 / tw;
  for (uint32_t base = 0; base < total; base += 64) {
    const uint32_t q = base + (uint32_t)lane;
    int g = 0, lo = 0, hi = 0, ty = 0;
    const bool valid = q < total;
    if (valid) {
#pragma unroll
      for (int step = 32; step >= 1; step >>= 1)
        if (pre[g + step] <= q) g += step;
      ty = geo[g].y0 + (int)(q - pre[g]);
      cull_row(geo[g], ty, tw, th, inv_tw, &lo, &hi);
    }
    f(valid, g, ty, lo, hi);
  }
}

// Count pass of the cull (record order): kept pairs kc and kept rows per
// record, written as kc | rows << pack_bits (pack_bits > 0) or to two arrays,
// and the depth-presort keys (records keeping no pair sort last).
template <class Geo>
__global__ __launch_bounds__(256) void k_cull_count(Batch B, const float4* __restrict__ splat,
                                                    const short4* __restrict__ rect,
                                                    const int32_t* __restrict__ tc,
                                                    const float* __restrict__ depth, int64_t n,
                                                    int pack_bits, uint32_t* __restrict__ kc,
                                                    uint32_t* __restrict__ nrow,
                                                    uint32_t* __restrict__ key,
                                                    uint32_t* __restrict__ perm, double req) {
  __shared__ Geo geo[256];
  __shared__ uint32_t pre[256], s_kc[256], s_nr[256];
  const int t = threadIdx.x, wb = t & ~63;
  const int64_t i = (int64_t)blockIdx.x * 256 + t;
  uint32_t h = 0;
  if (i < n && tc[i] > 0) {
    const short4 rc = rect[i];
    make_geom(geo[t], B, (int)i, splat + (int64_t)splat_stride4(B) * i, rc, req);
    h = (uint32_t)(rc.w - rc.y);
  }
  s_kc[t] = 0;
  s_nr[t] = 0;
  const uint32_t inc = wave_incl_scan_dpp(h);
  pre[t] = inc - h;
  const uint32_t total = lane63_u(inc);
  __syncthreads();
  wave_rows(geo + wb, pre + wb, total, B.tile_w, B.tile_h,
            [&](bool valid, int g, int, int lo, int hi) {
              if (valid && hi > lo) {
                atomicAdd(&s_kc[wb + g], (uint32_t)(hi - lo));
                atomicAdd(&s_nr[wb + g], 1u);
              }
            });
  __syncthreads();
  if (i >= n) return;
  const uint32_t c = s_kc[t], rows = s_nr[t];
  if (pack_bits > 0) {
    kc[i] = c | (rows << pack_bits);
  } else {
    kc[i] = c;
    nrow[i] = rows;
  }
  key[i] = c > 0 ? __float_as_uint(depth[i]) : 0xffffffffu;
  perm[i] = (uint32_t)i;
}

// Emit pass of the cull (depth order): one packed record per kept row (pair
// offset, record id, tile id of the row's first kept tile, run length |
// tiles_x << 16), and first[] as k_pair_records writes it. A wave's rows are
// flattened in depth order, so their pair offsets and record slots are the
// wave's bases (offsets / roff at its first position) plus running sums.
template <class Geo>
__global__ __launch_bounds__(256) void k_cull_emit(Batch B, const float4* __restrict__ splat,
                                                   const short4* __restrict__ rect,
                                                   const uint32_t* __restrict__ kcs,
                                                   const uint32_t* __restrict__ perm,
                                                   const uint32_t* __restrict__ offsets,
                                                   const uint32_t* __restrict__ roff,
                                                   uint32_t kc_mask, int64_t n_rec,
                                                   const int64_t* n_isect, int64_t cap,
                                                   uint4* __restrict__ packed,
                                                   uint32_t* __restrict__ first, double req) {
  __shared__ Geo geo[256];
  __shared__ uint32_t pre[256];
  const int t = threadIdx.x, lane = t & 63, wb = t & ~63;
  const int64_t j = (int64_t)blockIdx.x * 256 + t;
  const int64_t jw = (int64_t)blockIdx.x * 256 + wb;
  uint32_t h = 0;
  if (j < n_rec && (kcs[j] & kc_mask) > 0) {
    const uint32_t r = perm[j];
    const short4 rc = rect[r];
    make_geom(geo[t], B, (int)r, splat + (int64_t)splat_stride4(B) * r, rc, req);
    h = (uint32_t)(rc.w - rc.y);
  }
  const uint32_t inc = wave_incl_scan_dpp(h);
  pre[t] = inc - h;
  const uint32_t total = lane63_u(inc);
  __syncthreads();
  if (jw >= n_rec || total == 0) return;
  const int64_t n = clamp_n(n_isect, cap);
  int64_t pbase = offsets[jw];
  uint32_t rbase = roff[jw];
  wave_rows(geo + wb, pre + wb, total, B.tile_w, B.tile_h,
            [&](bool valid, int g, int ty, int lo, int hi) {
              // run length (<= 2048 tile columns, so a chunk's sum < 2^20)
              // and kept flag, scanned together
              const uint32_t w = valid ? (uint32_t)(hi - lo) : 0u;
              const uint32_t x = w | (w > 0 ? 1u << 20 : 0u);
              const uint32_t ix = wave_incl_scan_dpp(x);
              const uint32_t iw = ix & 0xfffffu, ir = ix >> 20;
              const int64_t o = pbase + (int64_t)(iw - w);
              if (w > 0 && o < n) {
                const Geo& G = geo[wb + g];
                const uint32_t k = rbase + ir - 1u;
                packed[k] = make_uint4((uint32_t)o, (uint32_t)G.rec,
                                       (uint32_t)(G.tile0 + ty * G.tiles_x + lo),
                                       w | ((uint32_t)G.tiles_x << 16));
                const int64_t oe = min(o + (int64_t)w, n);
                for (int64_t b = (o + kSortTile - 1) / kSortTile; b * kSortTile < oe; ++b)
                  first[b] = k;
                if (oe == n) first[(n + kSortTile - 1) / kSortTile] = k;
              }
              const uint32_t tot = lane63_u(ix);
              pbase += tot & 0xfffffu;
              rbase += tot >> 20;
            });
  (void)lane;
}

// The LinPrim cull passes, one record per lane: octahedron rects span few
// tile rows (about two on average) and the row test is a closed form, so a
// lane walks its own record's rows with the slab data in registers (no LDS
// staging, no cross-lane search). Same outputs as k_cull_count /
// k_cull_emit. The count pass also keeps, in record order, the runs of a
// record whose kept rows are at most 3 consecutive ones: runs[i] = (first
// kept row | rows << 16, lo | hi << 16 of each row), else (0xffffffff, ...);
// the emit pass (depth order) then gathers those 16 bytes instead of the
// splat and rect, and rebuilds the runs only for the other records.
__global__ __launch_bounds__(256) void k_cull_count_lin(Batch B, const float4* __restrict__ splat,
                                                        const short4* __restrict__ rect,
                                                        const int32_t* __restrict__ tc,
                                                        const float* __restrict__ depth,
                                                        int64_t n, int pack_bits,
                                                        uint32_t* __restrict__ kc,
                                                        uint32_t* __restrict__ nrow,
                                                        uint32_t* __restrict__ key,
                                                        uint32_t* __restrict__ perm,
                                                        uint4* __restrict__ runs, double req) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= n) return;
  uint32_t c = 0, rows = 0, first_row = 0;
  uint32_t rw0 = 0, rw1 = 0, rw2 = 0;
  bool gap = false;
  if (tc[i] > 0) {
    const short4 rc = rect[i];
    LinGeom G;
    make_geom(G, B, (int)i, splat + (int64_t)splat_stride4(B) * i, rc, req);
    const double inv_tw = ldexp(1.0, -__builtin_ctz(B.tile_w));  // tile sizes are powers of 2
    for (int ty = rc.y; ty < rc.w; ++ty) {
      int lo, hi;
      cull_row(G, ty, B.tile_w, B.tile_h, inv_tw, &lo, &hi);
      if (hi <= lo) continue;
      const uint32_t w = (uint32_t)lo | ((uint32_t)hi << 16);
      if (rows == 0) first_row = (uint32_t)ty;
      gap = gap || (uint32_t)ty != first_row + rows;
      rw0 = rows == 0 ? w : rw0;
      rw1 = rows == 1 ? w : rw1;
      rw2 = rows == 2 ? w : rw2;
      c += (uint32_t)(hi - lo);
      ++rows;
    }
  }
  runs[i] = rows > 0 && rows <= 3 && !gap ? make_uint4(first_row | (rows << 16), rw0, rw1, rw2)
                                          : make_uint4(0xffffffffu, 0u, 0u, 0u);
  if (pack_bits > 0) {
    kc[i] = c | (rows << pack_bits);
  } else {
    kc[i] = c;
    nrow[i] = rows;
  }
  key[i] = c > 0 ? __float_as_uint(depth[i]) : 0xffffffffu;
  perm[i] = (uint32_t)i;
}

__global__ __launch_bounds__(256) void k_cull_emit_lin(Batch B, const float4* __restrict__ splat,
                                                       const short4* __restrict__ rect,
                                                       const uint32_t* __restrict__ kcs,
                                                       const uint32_t* __restrict__ perm,
                                                       const uint32_t* __restrict__ offsets,
                                                       const uint32_t* __restrict__ roff,
                                                       uint32_t kc_mask, int64_t n_rec,
                                                       const int64_t* n_isect, int64_t cap,
                                                       const uint4* __restrict__ runs,
                                                       uint4* __restrict__ packed,
                                                       uint32_t* __restrict__ first, double req) {
  const int64_t j = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (j >= n_rec || (kcs[j] & kc_mask) == 0) return;
  const uint32_t r = perm[j];
  const int64_t n = clamp_n(n_isect, cap);
  int64_t o = offsets[j];
  uint32_t k = roff[j];
  const int v = view_of_record(B, (int)r);
  const int tile0 = B.v[v].tile_off, tiles_x = B.v[v].tiles_x;
  auto put = [&](int ty, int lo, int hi) {
    const uint32_t w = (uint32_t)(hi - lo);
    packed[k] = make_uint4((uint32_t)o, r, (uint32_t)(tile0 + ty * tiles_x + lo),
                           w | ((uint32_t)tiles_x << 16));
    const int64_t oe = min(o + (int64_t)w, n);
    for (int64_t b = (o + kSortTile - 1) / kSortTile; b * kSortTile < oe; ++b) first[b] = k;
    if (oe == n) first[(n + kSortTile - 1) / kSortTile] = k;
    o += w;
    ++k;
  };
  const uint4 ru = runs[r];
  if (ru.x != 0xffffffffu) {
    const int ty0 = (int)(ru.x & 0xffffu), rows = (int)(ru.x >> 16);
    const uint32_t rw[3] = {ru.y, ru.z, ru.w};
#pragma unroll
    for (int q = 0; q < 3; ++q)
      if (q < rows && o < n) put(ty0 + q, (int)(rw[q] & 0xffffu), (int)(rw[q] >> 16));
    return;
  }
  const short4 rc = rect[r];
  LinGeom G;
  make_geom(G, B, (int)r, splat + (int64_t)splat_stride4(B) * r, rc, req);
  const double inv_tw = ldexp(1.0, -__builtin_ctz(B.tile_w));
  for (int ty = rc.y; ty < rc.w && o < n; ++ty) {
    int lo, hi;
    cull_row(G, ty, B.tile_w, B.tile_h, inv_tw, &lo, &hi);
    if (hi > lo) put(ty, lo, hi);
  }
}

// Up to N packed records of a sort block, staged in LDS: the item offset of
// each record and its payload words (the third one only when the record
// kind reads it).
template <int N, bool C>
struct RecChunk {
  uint32_t off[N + 1];
  uint32_t a[N];
  uint32_t b[N];
  uint32_t c[C ? N : 1];
};

// What a packed record generates. Items of a record form a grid of
// width(k) columns in row-major order; item (yy, xx) gets a sort key and a
// value. j is the record's depth-order position.
//
// Tile pairs: packed = (pair offset, record id, tile id of the rect's top-
// left corner, rect width | tiles_x << 16); key = tile id, value = record.
struct PairItems {
  using Chunk = RecChunk<256, true>;
  static constexpr int kStage = 256;
  static __device__ __forceinline__ uint32_t width(uint4 q) { return q.w & 0xffffu; }
  static __device__ __forceinline__ uint32_t key0(uint4 q) { return q.z; }
  static __device__ __forceinline__ uint32_t stride(uint4 q) { return q.w >> 16; }
  static __device__ __forceinline__ void item(uint4 q, uint32_t, uint32_t yy, uint32_t xx,
                                              uint32_t& key, uint32_t& val) {
    key = q.z + yy * (q.w >> 16) + xx;
    val = q.y;
  }
};

// Band entries (one per tile row of the rect and band of kBandWidth tile
// columns it touches): packed = (entry offset, band id of the first entry,
// bands per rect row | bands per view row << 16, x0 | x1 << 16 with the
// rect's tile columns [x0, x1)); key = band id, value = j | xlo << 23 |
// (xhi - 1) << 27 with [xlo, xhi) the rect's columns inside the band.
constexpr int kBandWidth = 16;

struct BandItems {
  using Chunk = RecChunk<256, true>;
  static constexpr int kStage = 256;
  static __device__ __forceinline__ uint32_t width(uint4 q) { return q.z & 0xffffu; }
  static __device__ __forceinline__ uint32_t key0(uint4 q) { return q.y; }
  static __device__ __forceinline__ uint32_t stride(uint4 q) { return q.z >> 16; }
  static __device__ __forceinline__ void item(uint4 q, uint32_t j, uint32_t yy, uint32_t xx,
                                              uint32_t& key, uint32_t& val) {
    key = q.y + yy * (q.z >> 16) + xx;
    const int x0 = (int)(q.w & 0xffffu), x1 = (int)(q.w >> 16);
    const int b0 = ((x0 / kBandWidth) + (int)xx) * kBandWidth;
    const uint32_t xlo = (uint32_t)max(x0 - b0, 0);
    const uint32_t xhi = (uint32_t)min(x1 - b0, kBandWidth);
    val = j | (xlo << 23) | ((xhi - 1u) << 27);
  }
};

// Kept rows of the per-(Gaussian, tile) cull: packed = (pair offset, record
// id, tile id of the row's first kept tile, -); a one-row grid, so no width
// is needed (any width beyond the row keeps xx = item - offset). Records
// average a few pairs, so a sort block holds about a thousand: up to 2048
// are staged in LDS.
struct RowItems {
  using Chunk = RecChunk<2048, false>;
  static constexpr int kStage = 2048;
  static __device__ __forceinline__ uint32_t width(uint4) { return 1u << 30; }
  static __device__ __forceinline__ uint32_t key0(uint4 q) { return q.z; }
  static __device__ __forceinline__ uint32_t stride(uint4) { return 0u; }
  static __device__ __forceinline__ void item(uint4 q, uint32_t, uint32_t, uint32_t xx,
                                              uint32_t& key, uint32_t& val) {
    key = q.z + xx;
    val = q.y;
  }
};

// LDS position of slot s in the pair staging arrays: one pad word per 16
// slots, so a thread owning 16 consecutive slots and its neighbours hit
// distinct banks.
__device__ __forceinline__ int spad(int s) { return s + (s >> 4); }
constexpr int kSortTilePad = kSortTile + kSortTile / 16;
// The same with one pad word per IT slots (a thread of an NT-thread block
// owns IT = kSortTile / NT consecutive slots).
template <int IT>
__device__ __forceinline__ int spad_n(int s) { return s + s / IT; }
template <int IT>
constexpr int sort_tile_pad_n() { return kSortTile + kSortTile / IT; }

// Calls emit(slot, key, value) once for every item of sort block `part`
// (slot = item index - part T; items at or beyond n are skipped); Items says
// what a record's grid of items is. Must be called by all NT threads of the
// block. `marks` is LDS scratch of sort_tile_pad_n<IT>() words, IT =
// kSortTile / NT.
//
// Each record marks the slot of its first item, and a block-wide running
// maximum over the slots gives every slot its record; thread t then handles
// slots IT t .. IT t + IT - 1, stepping through its record's grid and
// dividing only for its first slot (every later record change starts a
// record at its first item). A block holds at most T + 1 records; up to
// Items::kStage are staged in LDS, beyond that they are read from the
// packed array (L2-resident).
template <class Items, int NT = 256, class Emit>
__device__ __forceinline__ void gen_block_pairs(const uint4* __restrict__ packed,
                                                const uint32_t* __restrict__ first, int part,
                                                int64_t n, typename Items::Chunk& S,
                                                uint32_t* marks,
                                                uint32_t* s_wave, Emit emit) {
  constexpr int IT = kSortTile / NT;  // consecutive slots per thread
  const int t = threadIdx.x;
  const uint32_t lo = (uint32_t)part * kSortTile;
  const uint32_t hi = (uint32_t)min(n, (int64_t)lo + kSortTile);
  const int nslots = (int)(hi - lo);
  const uint32_t j0 = first[part], j1 = first[part + 1];
  const uint32_t nrec = j1 - j0 + 1;
  constexpr bool kC = sizeof(S.c) > sizeof(uint32_t);
  const bool in_lds = nrec <= (uint32_t)Items::kStage;
  if (in_lds) {
    // all loads first, then the LDS stores
    constexpr int R = (Items::kStage + NT - 1) / NT;
    uint4 q[R];
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const uint32_t k = (uint32_t)(t + NT * r);
      if (k < nrec) q[r] = packed[j0 + k];
    }
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const uint32_t k = (uint32_t)(t + NT * r);
      if (k < nrec) {
        S.off[k] = q[r].x;
        S.a[k] = q[r].y;
        S.b[k] = q[r].z;
        if (kC) S.c[k] = q[r].w;
      }
    }
  }
#pragma unroll
  for (int i = 0; i < IT; ++i) marks[spad_n<IT>(IT * t + i)] = 0u;
  __syncthreads();
  // (the staged and the unstaged case take separate loops: a pointer that
  // may address either LDS or global memory would make every read a flat
  // load that waits for all outstanding loads)
  auto mark = [&](uint32_t k, uint32_t o) {
    const uint32_t s0 = (o > lo ? o : lo) - lo;
    if (s0 < (uint32_t)nslots) marks[spad_n<IT>((int)s0)] = k + 1u;
  };
  if (in_lds) {
    for (uint32_t k = (uint32_t)t; k < nrec; k += (uint32_t)NT) mark(k, S.off[k]);
  } else {
    for (uint32_t k = (uint32_t)t; k < nrec; k += (uint32_t)NT) mark(k, packed[j0 + k].x);
  }
  __syncthreads();
  uint32_t m[IT];
  uint32_t run = 0;
#pragma unroll
  for (int i = 0; i < IT; ++i) {
    run = max(run, marks[spad_n<IT>(IT * t + i)]);
    m[i] = run;
  }
  const uint32_t pre = block_excl_max<NT>(run, s_wave);
  auto walk = [&](auto rec) {
    int kprev = (int)max(pre, m[0]) - 1;
    uint4 q = rec(kprev);
    uint32_t xx = 0, yy = 0;
    {
      const uint32_t w0 = Items::width(q);
      const uint32_t local = lo + (uint32_t)(IT * t) - q.x;
      yy = local / w0;
      xx = local - yy * w0;
    }
#pragma unroll
    for (int i = 0; i < IT; ++i) {
      const int s = IT * t + i;
      const int k = (int)max(pre, m[i]) - 1;
      if (i > 0) {
        const bool nk = k != kprev;
        if (nk) q = rec(k);
        const uint32_t w = Items::width(q);
        const uint32_t x1 = xx + 1u;
        const bool wrap = x1 == w;
        xx = nk || wrap ? 0u : x1;
        yy = nk ? 0u : (wrap ? yy + 1u : yy);
        kprev = k;
      }
      if (s < nslots) {
        uint32_t key, val;
        Items::item(q, j0 + (uint32_t)k, yy, xx, key, val);
        emit(s, key, val);
      }
    }
  };
  if (in_lds)
    walk([&](int k) { return make_uint4(S.off[k], S.a[k], S.b[k], kC ? S.c[k] : 0u); });
  else
    walk([&](int k) { return packed[j0 + (uint32_t)k]; });
}

// First-pass histogram (digit = low BITS bits of the key) of each sort
// block, counted from its records without generating the items: record k
// of the block holds items [max(o_k, lo), min(o_(k+1), hi)) of the block's
// range [lo, hi) (records are contiguous in item order; the block's last
// record runs to hi), a run of rows of its grid, and each row segment is a
// run of consecutive keys t0 .. t0 + len - 1, whose low BITS bits take
// every digit len >> BITS times plus the cyclic run of len mod RADIX digits
// from t0 mod RADIX once. The runs go into an LDS difference array (at
// most three atomics per row segment instead of one per item), whose
// prefix sums are the counts; written digit-major like k_radix_hist.
template <int BITS, class Items, int NT>
__global__ __launch_bounds__(NT) void k_pair_hist(const uint4* __restrict__ packed,
                                                   const uint32_t* __restrict__ first,
                                                   const int64_t* n_isect, int64_t cap,
                                                   uint32_t* __restrict__ counts, int nblocks) {
  constexpr int RADIX = 1 << BITS;
  constexpr int DPT = (RADIX + NT - 1) / NT;
  constexpr int NW = NT / 64;
  __shared__ int32_t D[RADIX];
  __shared__ uint32_t s_wave[NW];
  const int t = threadIdx.x;
  for (int k = t; k < RADIX; k += NT) D[k] = 0;
  const int64_t n = clamp_n(n_isect, cap);
  const int part = live_swizzle(blockIdx.x, nblocks, n);
  __syncthreads();
  uint32_t whole = 0;  // sum of len >> BITS over this thread's segments
  if ((int64_t)part * kSortTile < n) {
    const uint32_t lo = (uint32_t)part * kSortTile;
    const uint32_t hi = (uint32_t)min(n, (int64_t)lo + kSortTile);
    const uint32_t j0 = first[part], j1 = first[part + 1];
    for (uint32_t k = j0 + (uint32_t)t; k <= j1; k += (uint32_t)NT) {
      const uint4 q = packed[k];
      const uint32_t o = q.x;
      const uint32_t end = k < j1 ? min(packed[k + 1].x, hi) : hi;
      const uint32_t beg = max(o, lo);
      if (beg >= end) continue;
      const uint32_t w = Items::width(q), stride = Items::stride(q), z = Items::key0(q);
      const uint32_t a = beg - o, b = end - o;  // items [a, b) of the record's grid
      uint32_t y = a / w;
      uint32_t xa = a - y * w;
      const uint32_t ylast = (b - 1u) / w;
      for (; y <= ylast; ++y) {
        const uint32_t xb = y == ylast ? b - y * w : w;
        const uint32_t t0 = z + y * stride + xa, len = xb - xa;
        whole += len >> BITS;
        const uint32_t r = len & (RADIX - 1), s = t0 & (RADIX - 1);
        if (r != 0u) {
          atomicAdd(&D[s], 1);
          if (s + r < (uint32_t)RADIX) {
            atomicAdd(&D[s + r], -1);
          } else if (s + r > (uint32_t)RADIX) {
            atomicAdd(&D[0], 1);
            atomicAdd(&D[s + r - RADIX], -1);
          }
        }
        xa = 0;
      }
    }
  }
  uint32_t all = 0;
  {
    // block sum of the whole-cycle counts
    const uint32_t inc = wave_incl_scan(whole);
    if ((t & 63) == 63) s_wave[t >> 6] = inc;
    __syncthreads();
#pragma unroll
    for (int q = 0; q < NW; ++q) all += s_wave[q];
    __syncthreads();
  }
  // counts = all + inclusive prefix sums of D; thread t holds digits
  // [DPT t, DPT t + DPT)
  int32_t dv[DPT], run = 0;
#pragma unroll
  for (int i = 0; i < DPT; ++i) {
    const int d = DPT * t + i;
    dv[i] = d < RADIX ? D[d] : 0;
    run += dv[i];
  }
  int32_t pre = (int32_t)block_excl_scan<NT>((uint32_t)run, s_wave);
#pragma unroll
  for (int i = 0; i < DPT; ++i) {
    const int d = DPT * t + i;
    pre += dv[i];
    if (d < RADIX) counts[(int64_t)d * nblocks + part] = all + (uint32_t)pre;
  }
}

// First-pass scatter from regenerated pairs: the block's pairs are laid out
// in LDS in pair order, then ranked and written exactly like k_radix_scatter
// (digit = low BITS bits). With RANGES this is also the last pass.
template <int BITS, bool RANGES, typename KO, class Items, int NT>
__global__ __launch_bounds__(NT) void k_pair_scatter(
    const uint4* __restrict__ packed, const uint32_t* __restrict__ first, const int64_t* n_isect,
    int64_t cap, const uint32_t* __restrict__ doff, const uint32_t* __restrict__ dtot,
    int nblocks, KO* __restrict__ kout,
    uint32_t* __restrict__ vout, int2* __restrict__ ranges) {
  constexpr int RADIX = 1 << BITS;
  constexpr int NW = NT / 64;
  constexpr int IT = kSortTile / NT;
  constexpr int PADN = sort_tile_pad_n<IT>();
  __shared__ typename Items::Chunk S;
  __shared__ uint32_t wcnt[NW][RADIX];
  __shared__ uint32_t gbase[RADIX];
  __shared__ uint32_t s_wave[NW];
  // pairs in slot order at spad(slot) (sval doubles as the generator's
  // marks), then the ranked block in plain order; keys in the output key
  // type (16-bit tile ids take half the LDS: four blocks per CU, not three)
  __shared__ KO skey[PADN];
  __shared__ uint32_t sval[PADN];
  const int t = threadIdx.x, w = t >> 6, lane = t & 63;
  const int64_t n = clamp_n(n_isect, cap);
  const int part = live_swizzle(blockIdx.x, nblocks, n);
  const int64_t bbase = (int64_t)part * kSortTile;
  if (bbase >= n) return;  // whole block beyond the list: no counts, nothing to write
  const int nvalid = (int)min((int64_t)kSortTile, n - bbase);
  for (int k = t; k < NW * RADIX; k += NT) (&wcnt[0][0])[k] = 0;
  // thread t owns digits [DPT t, DPT t + DPT); the block's digit offsets do
  // not depend on the items: fetch them early
  constexpr int DPT = (RADIX + NT - 1) / NT;
  uint32_t my_off[DPT], my_tot[DPT], tot_sum = 0;
#pragma unroll
  for (int i = 0; i < DPT; ++i) {
    const int d = DPT * t + i;
    my_off[i] = d < RADIX ? doff[(int64_t)d * nblocks + part] : 0u;
    my_tot[i] = d < RADIX ? dtot[d] : 0u;
    tot_sum += my_tot[i];
  }
  gen_block_pairs<Items, NT>(packed, first, part, n, S, sval, s_wave,
                             [&](int slot, uint32_t key, uint32_t val) {
                               skey[spad_n<IT>(slot)] = (KO)key;
                               sval[spad_n<IT>(slot)] = val;
                             });
  __syncthreads();
  const uint64_t lt = lanemask_lt();
  uint32_t key[IT], val[IT], lofs[IT];
#pragma unroll
  for (int j = 0; j < IT; ++j) {
    const int slot = w * (64 * IT) + j * 64 + lane;
    const bool ok = slot < nvalid;
    key[j] = ok ? skey[spad_n<IT>(slot)] : 0u;
    val[j] = ok ? sval[spad_n<IT>(slot)] : 0u;
    const uint32_t d = key[j] & (RADIX - 1);
    const uint64_t m = match_digit<BITS>(d, ok);
    const uint32_t before = wcnt[w][d];
    lofs[j] = before + (uint32_t)__popcll(m & lt);
    if (ok && (m & lt) == 0) wcnt[w][d] = before + (uint32_t)__popcll(m);
  }
  __syncthreads();
  uint32_t cw[DPT][NW], tot = 0;
#pragma unroll
  for (int i = 0; i < DPT; ++i) {
    const int d = DPT * t + i;
#pragma unroll
    for (int q = 0; q < NW; ++q) {
      cw[i][q] = d < RADIX ? wcnt[q][d] : 0u;
      tot += cw[i][q];
    }
  }
  uint32_t start = block_excl_scan<NT>(tot, s_wave);
  uint32_t dstart = block_excl_scan<NT>(tot_sum, s_wave);
#pragma unroll
  for (int i = 0; i < DPT; ++i) {
    const int d = DPT * t + i;
    const uint32_t sd = start;  // the digit's start in the block
#pragma unroll
    for (int q = 0; q < NW; ++q) {
      if (d < RADIX) wcnt[q][d] = start;
      start += cw[i][q];
    }
    if (d < RADIX) gbase[d] = dstart + my_off[i] - sd;
    dstart += my_tot[i];
  }
  __syncthreads();
#pragma unroll
  for (int j = 0; j < IT; ++j) {
    const int slot = w * (64 * IT) + j * 64 + lane;
    if (slot < nvalid) {
      const uint32_t pos = wcnt[w][key[j] & (RADIX - 1)] + lofs[j];
      skey[pos] = (KO)key[j];
      sval[pos] = val[j];
    }
  }
  __syncthreads();
  write_sorted<BITS, KO, KO, RANGES, NT>(skey, sval, gbase, nvalid, 0, kout, vout, ranges,
                                         nullptr, nullptr);
}

// ---------------------------------------------------------------------------
// Single-pass ("onesweep") radix passes with decoupled look-back
// (XPR_SORT_ONESWEEP). The digit counts of every pass are taken up front in
// one pass over the data (for the tile passes, from the records' rects
// without generating the pairs), so no pass needs a histogram kernel or a
// device-wide scan of block counts. A block takes the next partition id from
// an atomic counter (ids follow the order in which blocks start, so a block
// only ever waits for partitions held by blocks already running), ranks its
// 4096 keys in LDS as in k_radix_scatter, publishes its per-digit counts,
// and finds, per digit, the count of the same digit in all earlier
// partitions by walking back over their published words until one holds an
// inclusive prefix; it then publishes its own inclusive prefix and writes its
// keys at digit start + prefix + rank. A status word is flag << 30 | count
// (0 = not yet published, 1 = the partition's own count, 2 = inclusive
// prefix), so one 32-bit atomic load reads both. Waits are bounded: past the
// limit the block records an error and goes on, and the driver turns the
// error into a failed binning instead of a hang.
constexpr uint32_t kLbAgg = 1u << 30;
constexpr uint32_t kLbInc = 2u << 30;
constexpr uint32_t kLbCount = kLbAgg - 1u;
constexpr int kLbSpinLimit = 1 << 22;
constexpr int kSweepMaxPasses = 4;

struct Sweep {
  uint32_t* status;      // [partitions][RADIX] look-back words, zero before the pass
  uint32_t* counter;     // partition counter, zero before the pass
  const uint32_t* hist;  // [RADIX] digit counts of the pass over the whole list
  uint32_t* err;         // nonzero after a look-back wait hit its limit
};

__device__ __forceinline__ uint32_t lb_load(const uint32_t* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void lb_store(uint32_t* p, uint32_t v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// The block's partition id (all threads).
__device__ __forceinline__ int sweep_part(uint32_t* counter, int* s_part) {
  if (threadIdx.x == 0) *s_part = (int)atomicAdd(counter, 1u);
  __syncthreads();
  return *s_part;
}

// Publishes the block's count of digit t (thread t < RADIX): as an
// inclusive prefix for partition 0, else as its own count. Called as soon
// as the counts are known, so that later partitions find it early.
template <int RADIX>
__device__ __forceinline__ void sweep_publish(const Sweep& sw, int part, uint32_t tot) {
  const int t = threadIdx.x;
  if (t < RADIX) lb_store(sw.status + (size_t)part * RADIX + t, (part == 0 ? kLbInc : kLbAgg) | tot);
}

// Called by all threads after sweep_publish: returns, for thread t <
// RADIX, where the block's run of digit t starts in the output (digit start
// over the whole list plus the count of digit t in earlier partitions), and
// publishes the inclusive prefix. The walk back reads kLbWindow earlier
// partitions' words at once (independent loads), then takes them in order.
constexpr int kLbWindow = 4;
template <int RADIX>
__device__ __forceinline__ uint32_t sweep_offset(const Sweep& sw, int part, uint32_t tot,
                                                 uint32_t* s_wave) {
  const int t = threadIdx.x;
  const uint32_t dstart = block_excl_scan256(t < RADIX ? sw.hist[t] : 0u, s_wave, nullptr);
  if (t >= RADIX || part == 0) return t < RADIX ? dstart : 0u;
  uint32_t excl = 0u;
  int p = part - 1;
  int spins = 0;
  bool done = false;
  while (!done && p >= 0) {
    uint32_t w[kLbWindow];
#pragma unroll
    for (int i = 0; i < kLbWindow; ++i)
      w[i] = p - i >= 0 ? lb_load(sw.status + (size_t)(p - i) * RADIX + t) : (kLbInc | 0u);
#pragma unroll
    for (int i = 0; i < kLbWindow; ++i) {
      if (done) break;
      const uint32_t flag = w[i] >> 30;
      if (flag == 0u) break;  // not yet published: read again from p
      excl += w[i] & kLbCount;
      --p;
      if (flag == 2u) done = true;
    }
    if (!done && p >= 0 && (lb_load(sw.status + (size_t)p * RADIX + t) >> 30) == 0u) {
      if (++spins > kLbSpinLimit) {
        atomicOr(sw.err, 1u);
        break;
      }
      __builtin_amdgcn_s_sleep(1);
    }
  }
  lb_store(sw.status + (size_t)part * RADIX + t, kLbInc | ((excl + tot) & kLbCount));
  return dstart + excl;
}

// write_sorted with a bound: with a pair list larger than its capacity the
// digit starts can point past it, and nothing may be written there.
template <int BITS, typename KS, typename KO, bool RANGES>
__device__ __forceinline__ void write_sorted_capped(const KS* skey, const uint32_t* sval,
                                                    const uint32_t* gbase, int nvalid, int shift,
                                                    int64_t cap, KO* __restrict__ kout,
                                                    uint32_t* __restrict__ vout,
                                                    int2* __restrict__ ranges,
                                                    const int32_t* __restrict__ aux_src,
                                                    uint32_t* __restrict__ aux_dst) {
  for (int k = threadIdx.x; k < nvalid; k += 256) {
    const KS kk = skey[k];
    const uint32_t g = gbase[digit_of<BITS>(kk, shift)] + (uint32_t)k;
    if ((int64_t)g >= cap) continue;
    if (!RANGES || kout) kout[g] = (KO)kk;
    const uint32_t v = sval[k];
    vout[g] = v;
    if (aux_dst) aux_dst[g] = (uint32_t)aux_src[v];
    if (RANGES) {
      const uint32_t tile = (uint32_t)kk;
      if (k == 0 || (uint32_t)skey[k - 1] != tile) atomicMin(&ranges[tile].x, (int)g);
      if (k == nvalid - 1 || (uint32_t)skey[k + 1] != tile) atomicMax(&ranges[tile].y, (int)g + 1);
    }
  }
}

// One onesweep pass over keys in memory: k_radix_scatter with the digit
// offsets from the look-back.
template <int BITS, typename K, bool RANGES>
__global__ __launch_bounds__(256) void k_sweep_scatter(const K* __restrict__ kin,
                                                       const uint32_t* __restrict__ vin,
                                                       K* __restrict__ kout,
                                                       uint32_t* __restrict__ vout,
                                                       const int64_t* n_dev, int64_t cap,
                                                       int shift, Sweep sw,
                                                       int2* __restrict__ ranges,
                                                       const int32_t* __restrict__ aux_src,
                                                       uint32_t* __restrict__ aux_dst) {
  constexpr int RADIX = 1 << BITS;
  __shared__ uint32_t wcnt[kSortWaves][RADIX];
  __shared__ uint32_t gbase[RADIX];
  __shared__ uint32_t s_wave[4];
  __shared__ int s_part;
  __shared__ K skey[kSortTile];
  __shared__ uint32_t sval[kSortTile];
  const int t = threadIdx.x, w = t >> 6, lane = t & 63;
  const int part = sweep_part(sw.counter, &s_part);
  const int64_t n = clamp_n(n_dev, cap);
  const int64_t bbase = (int64_t)part * kSortTile;
  if (bbase >= n) return;  // partitions past the list: nobody waits for them
  for (int k = t; k < kSortWaves * RADIX; k += 256) (&wcnt[0][0])[k] = 0;
  for (int k = t; k < RADIX; k += 256) gbase[k] = 0u;
  const int64_t base = bbase + w * (64 * kSortItems);
  const uint64_t lt = lanemask_lt();
  K key[kSortItems];
  uint32_t val[kSortItems];
  uint32_t lofs[kSortItems];
#pragma unroll
  for (int j = 0; j < kSortItems; ++j) {
    const int64_t idx = min(base + j * 64 + lane, n - 1);
    key[j] = kin[idx];
    val[j] = vin[idx];
  }
  __syncthreads();
  // the block's digit counts first, published before the ranking
#pragma unroll
  for (int j = 0; j < kSortItems; ++j)
    if (base + j * 64 + lane < n) atomicAdd(&gbase[digit_of<BITS>(key[j], shift)], 1u);
  __syncthreads();
  sweep_publish<RADIX>(sw, part, t < RADIX ? gbase[t] : 0u);
#pragma unroll
  for (int j = 0; j < kSortItems; ++j) {
    const bool ok = base + j * 64 + lane < n;
    const uint32_t d = digit_of<BITS>(key[j], shift);
    const uint64_t m = match_digit<BITS>(d, ok);
    const uint32_t before = wcnt[w][d];
    lofs[j] = before + (uint32_t)__popcll(m & lt);
    if (ok && (m & lt) == 0) wcnt[w][d] = before + (uint32_t)__popcll(m);
  }
  __syncthreads();
  uint32_t c0 = 0, c1 = 0, c2 = 0, c3 = 0;
  if (t < RADIX) {
    c0 = wcnt[0][t];
    c1 = wcnt[1][t];
    c2 = wcnt[2][t];
    c3 = wcnt[3][t];
  }
  const uint32_t tot = c0 + c1 + c2 + c3;
  const uint32_t start = block_excl_scan256(tot, s_wave, nullptr);
  const uint32_t gofs = sweep_offset<RADIX>(sw, part, tot, s_wave);
  if (t < RADIX) {
    gbase[t] = gofs - start;
    wcnt[0][t] = start;
    wcnt[1][t] = start + c0;
    wcnt[2][t] = start + c0 + c1;
    wcnt[3][t] = start + c0 + c1 + c2;
  }
  __syncthreads();
#pragma unroll
  for (int j = 0; j < kSortItems; ++j) {
    const int64_t idx = base + j * 64 + lane;
    if (idx < n) {
      const uint32_t pos = wcnt[w][digit_of<BITS>(key[j], shift)] + lofs[j];
      skey[pos] = key[j];
      sval[pos] = val[j];
    }
  }
  __syncthreads();
  const int64_t rem = n - bbase;
  const int nvalid = rem < kSortTile ? (int)rem : kSortTile;
  write_sorted_capped<BITS, K, K, RANGES>(skey, sval, gbase, nvalid, shift, cap, kout, vout,
                                          ranges, aux_src, aux_dst);
}

// First tile pass of the onesweep path: k_pair_scatter with the digit
// offsets from the look-back.
template <int BITS, bool RANGES, typename KO>
__global__ __launch_bounds__(256) void k_sweep_pair_scatter(
    const uint4* __restrict__ packed, const uint32_t* __restrict__ first, const int64_t* n_isect,
    int64_t cap, Sweep sw, KO* __restrict__ kout, uint32_t* __restrict__ vout,
    int2* __restrict__ ranges) {
  constexpr int RADIX = 1 << BITS;
  __shared__ typename PairItems::Chunk S;
  __shared__ uint32_t wcnt[kSortWaves][RADIX];
  __shared__ uint32_t gbase[RADIX];
  __shared__ uint32_t s_wave[4];
  __shared__ int s_part;
  __shared__ uint32_t skey[kSortTilePad];
  __shared__ uint32_t sval[kSortTilePad];
  const int t = threadIdx.x, w = t >> 6, lane = t & 63;
  const int part = sweep_part(sw.counter, &s_part);
  const int64_t n = clamp_n(n_isect, cap);
  const int64_t bbase = (int64_t)part * kSortTile;
  if (bbase >= n) return;
  const int nvalid = (int)min((int64_t)kSortTile, n - bbase);
  for (int k = t; k < kSortWaves * RADIX; k += 256) (&wcnt[0][0])[k] = 0;
  for (int k = t; k < RADIX; k += 256) gbase[k] = 0u;
  gen_block_pairs<PairItems>(packed, first, part, n, S, sval, s_wave,
                             [&](int slot, uint32_t key, uint32_t val) {
                               skey[spad(slot)] = key;
                               sval[spad(slot)] = val;
                               atomicAdd(&gbase[key & (RADIX - 1)], 1u);
                             });
  __syncthreads();
  sweep_publish<RADIX>(sw, part, t < RADIX ? gbase[t] : 0u);
  const uint64_t lt = lanemask_lt();
  uint32_t key[kSortItems], val[kSortItems], lofs[kSortItems];
#pragma unroll
  for (int j = 0; j < kSortItems; ++j) {
    const int slot = w * (64 * kSortItems) + j * 64 + lane;
    const bool ok = slot < nvalid;
    key[j] = ok ? skey[spad(slot)] : 0u;
    val[j] = ok ? sval[spad(slot)] : 0u;
    const uint32_t d = key[j] & (RADIX - 1);
    const uint64_t m = match_digit<BITS>(d, ok);
    const uint32_t before = wcnt[w][d];
    lofs[j] = before + (uint32_t)__popcll(m & lt);
    if (ok && (m & lt) == 0) wcnt[w][d] = before + (uint32_t)__popcll(m);
  }
  __syncthreads();
  uint32_t c0 = 0, c1 = 0, c2 = 0, c3 = 0;
  if (t < RADIX) {
    c0 = wcnt[0][t];
    c1 = wcnt[1][t];
    c2 = wcnt[2][t];
    c3 = wcnt[3][t];
  }
  const uint32_t tot = c0 + c1 + c2 + c3;
  const uint32_t start = block_excl_scan256(tot, s_wave, nullptr);
  const uint32_t gofs = sweep_offset<RADIX>(sw, part, tot, s_wave);
  if (t < RADIX) {
    gbase[t] = gofs - start;
    wcnt[0][t] = start;
    wcnt[1][t] = start + c0;
    wcnt[2][t] = start + c0 + c1;
    wcnt[3][t] = start + c0 + c1 + c2;
  }
  __syncthreads();
#pragma unroll
  for (int j = 0; j < kSortItems; ++j) {
    const int slot = w * (64 * kSortItems) + j * 64 + lane;
    if (slot < nvalid) {
      const uint32_t pos = wcnt[w][key[j] & (RADIX - 1)] + lofs[j];
      skey[pos] = key[j];
      sval[pos] = val[j];
    }
  }
  __syncthreads();
  write_sorted_capped<BITS, uint32_t, KO, RANGES>(skey, sval, gbase, nvalid, 0, cap, kout, vout,
                                                  ranges, nullptr, nullptr);
}

// Depth-presort keys (as k_depth_keys) for 16 records per thread, with the
// digit counts of the four 8-bit passes over all of them added to
// hist [4][256] (zero before).
__global__ __launch_bounds__(256) void k_depth_keys_hist(const float* __restrict__ depth,
                                                         const int32_t* __restrict__ tc,
                                                         int64_t n, uint32_t* __restrict__ key,
                                                         uint32_t* __restrict__ perm,
                                                         uint32_t* __restrict__ hist) {
  __shared__ uint32_t h[4][256];
  const int t = threadIdx.x;
  for (int k = t; k < 4 * 256; k += 256) (&h[0][0])[k] = 0u;
  __syncthreads();
  const int64_t base = (int64_t)blockIdx.x * kSortTile;
#pragma unroll 4
  for (int j = 0; j < kSortItems; ++j) {
    const int64_t i = base + j * 256 + t;
    if (i < n) {
      const uint32_t k = tc[i] > 0 ? __float_as_uint(depth[i]) : 0xffffffffu;
      key[i] = k;
      perm[i] = (uint32_t)i;
#pragma unroll
      for (int p = 0; p < 4; ++p) atomicAdd(&h[p][(k >> (8 * p)) & 255u], 1u);
    }
  }
  __syncthreads();
  for (int k = t; k < 4 * 256; k += 256) {
    const uint32_t c = (&h[0][0])[k];
    if (c) atomicAdd(hist + k, c);
  }
}

// Digit counts of the tile keys of the pairs [a, a + len) of one rect row
// (consecutive tile ids), pairs of the list only; hist rows of 256 per pass.
// The first pass's digits of a run of consecutive ids are consecutive
// modulo the radix: a difference array (diff, RADIX + 1 words) takes the
// run in two updates (plus full cycles in `cyc`); later passes change digit
// at most once per 2^shift ids.
__device__ __forceinline__ void hist_run(uint32_t a, uint32_t len, int dbits, int passes,
                                         int* diff, uint32_t* cyc, uint32_t* h) {
  const uint32_t radix = 1u << dbits, mask = radix - 1u;
  const uint32_t full = len >> dbits, rem = len & mask;
  if (full) atomicAdd(cyc, full);
  if (rem) {
    const uint32_t lo = a & mask, hi = lo + rem;
    atomicAdd(&diff[lo], 1);
    if (hi <= radix) {
      atomicAdd(&diff[hi], -1);
    } else {
      atomicAdd(&diff[radix], -1);
      atomicAdd(&diff[0], 1);
      atomicAdd(&diff[hi - radix], -1);
    }
  }
  for (int p = 1; p < passes; ++p) {
    const int sh = p * dbits;
    uint32_t x = a;
    const uint32_t e = a + len;
    while (x < e) {
      const uint32_t seg = min(e, ((x >> sh) + 1u) << sh);
      atomicAdd(&h[p * 256 + ((x >> sh) & mask)], seg - x);
      x = seg;
    }
  }
}

// k_pair_records for 16 records per thread, adding the digit counts of all
// tile passes over the list's pairs to hist [passes][256] (zero before).
__global__ __launch_bounds__(256) void k_pair_records_hist(
    Batch B, const short4* __restrict__ rect, const uint32_t* __restrict__ tc_sorted,
    const uint32_t* __restrict__ perm, const uint32_t* __restrict__ offsets, int64_t n_rec,
    const int64_t* n_isect, int64_t cap, int dbits, int passes, uint4* __restrict__ packed,
    uint32_t* __restrict__ first, uint32_t* __restrict__ hist) {
  __shared__ int diff[257];
  __shared__ uint32_t cyc;
  __shared__ uint32_t h[kSweepMaxPasses * 256];
  const int t = threadIdx.x;
  for (int k = t; k < 257; k += 256) diff[k] = 0;
  for (int k = t; k < kSweepMaxPasses * 256; k += 256) h[k] = 0u;
  if (t == 0) cyc = 0u;
  __syncthreads();
  const int64_t n = clamp_n(n_isect, cap);
  const int64_t base = (int64_t)blockIdx.x * kSortTile;
  for (int jj = 0; jj < kSortItems; ++jj) {
    const int64_t j = base + jj * 256 + t;
    if (j >= n_rec) break;
    const int64_t o = offsets[j];
    const int64_t e = min(o + (int64_t)tc_sorted[j], n);
    if (e <= o) continue;
    const uint32_t r = perm[j];
    int v = 0;
    for (int q = 1; q < B.n_views; ++q)
      if ((int32_t)r >= B.v[q].rec_off) v = q;
    const short4 rc = rect[r];
    const uint32_t tx = (uint32_t)B.v[v].tiles_x;
    const uint32_t t0 = (uint32_t)B.v[v].tile_off + (uint32_t)rc.y * tx + (uint32_t)rc.x;
    const uint32_t wdt = (uint32_t)(rc.z - rc.x);
    packed[j] = make_uint4((uint32_t)o, r, t0, wdt | (tx << 16));
    for (int64_t b = (o + kSortTile - 1) / kSortTile; b * kSortTile < e; ++b)
      first[b] = (uint32_t)j;
    if (e == n) first[(n + kSortTile - 1) / kSortTile] = (uint32_t)j;
    // the record's pairs in the list: whole rows, then part of one
    const int64_t cnt = e - o;
    const uint32_t rows = (uint32_t)(cnt / wdt), last = (uint32_t)(cnt - (int64_t)rows * wdt);
    for (uint32_t y = 0; y < rows; ++y) hist_run(t0 + y * tx, wdt, dbits, passes, diff, &cyc, h);
    if (last) hist_run(t0 + rows * tx, last, dbits, passes, diff, &cyc, h);
  }
  __syncthreads();
  // first pass: prefix sum of the difference array, plus the full cycles
  const uint32_t radix = 1u << dbits;
  int run = 0;
  if (t < (int)radix) {
    for (int k = 0; k <= t; ++k) run += diff[k];
    h[t] = (uint32_t)run + cyc;
  }
  __syncthreads();
  for (int k = t; k < passes * 256; k += 256) {
    const uint32_t c = h[k];
    if (c && (k & 255) < (int)radix) atomicAdd(hist + k, c);
  }
}

// A failed look-back poisons the pair count, so the caller's capacity check
// (which every caller makes) reports it; the synchronous entry point also
// reads err itself.
__global__ void k_sweep_check(const uint32_t* err, int64_t* n_isect) {
  if (threadIdx.x == 0 && *err != 0u) *n_isect = (int64_t)1 << 62;
}

// Digit width for sorting `bits` bits: 7 when that needs no more passes than
// 8 (longer per-digit runs in the scatter, one ballot fewer per key).
static inline int radix_digit_bits(int bits) { return (bits + 6) / 7 == (bits + 7) / 8 ? 7 : 8; }

// Number of passes radix_sort makes for `bits`.
static inline int radix_passes(int bits) {
  const int d = radix_digit_bits(bits);
  return (bits + d - 1) / d;
}

template <int BITS, typename K>
static hipError_t radix_pass(K* k0, uint32_t* v0, K* k1, uint32_t* v1, const int64_t* n_dev,
                             int64_t cap, int nb, int shift, uint32_t* counts,
                             uint32_t* dtot, uint32_t* csum, int2* ranges,
                             const int32_t* aux_src, uint32_t* aux_dst, hipStream_t st,
                             bool counted) {
  if (!counted)
    hipLaunchKernelGGL((k_radix_hist<BITS, K>), dim3(nb), dim3(256), 0, st, k0, n_dev, cap, shift,
                       counts, nb);
  hipError_t e = digit_scan(counts, nb, 1 << BITS, dtot, csum, st);
  if (e != hipSuccess) return e;
  constexpr int NT = kRadixThreads;
  if (ranges)
    hipLaunchKernelGGL((k_radix_scatter<BITS, K, true, NT>), dim3(nb), dim3(NT), 0, st, k0, v0,
                       k1, v1, n_dev, cap, shift, counts, dtot, nb, ranges, aux_src, aux_dst);
  else
    hipLaunchKernelGGL((k_radix_scatter<BITS, K, false, NT>), dim3(nb), dim3(NT), 0, st, k0, v0,
                       k1, v1, n_dev, cap, shift, counts, dtot, nb, (int2*)nullptr, aux_src,
                       aux_dst);
  return hipGetLastError();
}

// Sorts (keys, vals) of length n_dev (<= cap) on bits [0, bits). The data
// starts in (k0, v0) and ping-pongs with (k1, v1); returns via *k_out/*v_out
// where it ended. grid_n bounds the number of keys (host known). The last
// pass can build tile ranges and carry aux_src[value] into aux_dst.
template <typename K>
static hipError_t radix_sort(K* k0, uint32_t* v0, K* k1, uint32_t* v1, const int64_t* n_dev,
                             int64_t cap, int64_t grid_n, int bits, uint32_t* counts,
                             uint32_t* dtot, uint32_t* csum, K** k_out, uint32_t** v_out,
                             hipStream_t st,
                             int first_shift = 0, int2* ranges = nullptr,
                             bool keys_last = true, const int32_t* aux_src = nullptr,
                             uint32_t* aux_dst = nullptr, bool first_counted = false) {
  *k_out = k0;
  *v_out = v0;
  if (grid_n <= 0) return hipSuccess;
  const int nb = (int)((grid_n + kSortTile - 1) / kSortTile);
  const int dbits = radix_digit_bits(bits);
  for (int shift = first_shift; shift < bits; shift += dbits) {
    const bool last = shift + dbits >= bits;
    int2* rg = last ? ranges : nullptr;
    K* kdst = (last && !keys_last && ranges) ? nullptr : k1;
    const int32_t* as = last ? aux_src : nullptr;
    uint32_t* ad = last ? aux_dst : nullptr;
    // each pass ranks exactly the bits it places (the last one may have
    // fewer than dbits left: one ballot per bit saved per key)
    const int pb = std::min(dbits, bits - shift);
    // the first pass's counts may come with the keys
    const bool counted = first_counted && shift == first_shift;
    hipError_t e;
    switch (pb) {
      case 8: e = radix_pass<8, K>(k0, v0, kdst, v1, n_dev, cap, nb, shift, counts, dtot, csum, rg,
                                   as, ad, st, counted); break;
      case 7: e = radix_pass<7, K>(k0, v0, kdst, v1, n_dev, cap, nb, shift, counts, dtot, csum, rg,
                                   as, ad, st, counted); break;
      case 6: e = radix_pass<6, K>(k0, v0, kdst, v1, n_dev, cap, nb, shift, counts, dtot, csum, rg,
                                   as, ad, st, counted); break;
      case 5: e = radix_pass<5, K>(k0, v0, kdst, v1, n_dev, cap, nb, shift, counts, dtot, csum, rg,
                                   as, ad, st, counted); break;
      default: e = radix_pass<4, K>(k0, v0, kdst, v1, n_dev, cap, nb, shift, counts, dtot, csum, rg,
                                    as, ad, st, counted); break;
    }
    if (e != hipSuccess) return e;
    K* tk = k0; k0 = k1; k1 = tk;
    uint32_t* tv = v0; v0 = v1; v1 = tv;
  }
  *k_out = k0;
  *v_out = v0;
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Tile ranges from sorted keys (tile in the high part for 64-bit keys). Each
// thread reads 4 consecutive keys plus the one before them and writes the
// starts and ends of the tiles that change inside that window.
template <typename K>
__device__ __forceinline__ uint32_t tile_of(K k) {
  return (uint32_t)(k >> (sizeof(K) == 8 ? 32 : 0));
}

template <typename K>
__global__ void k_ranges(const K* __restrict__ keys, const int64_t* n_dev, int64_t cap,
                         int total_tiles, int2* __restrict__ ranges) {
  const int64_t n = clamp_n(n_dev, cap);
  const int64_t i0 = 4 * ((int64_t)blockIdx.x * blockDim.x + threadIdx.x);
  if (i0 >= n) return;
  uint32_t t[5];
  t[0] = i0 > 0 ? tile_of(keys[i0 - 1]) : 0xffffffffu;
#pragma unroll
  for (int j = 0; j < 4; ++j) t[j + 1] = i0 + j < n ? tile_of(keys[i0 + j]) : 0xffffffffu;
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    const int64_t i = i0 + j;
    if (i >= n) break;
    const uint32_t cur = t[j + 1];
    if (cur >= (uint32_t)total_tiles) continue;
    if (t[j] != cur) ranges[cur].x = (int)i;
    const uint32_t nxt = j < 3 ? t[j + 2] : (i + 1 < n ? tile_of(keys[i + 1]) : 0xffffffffu);
    if (nxt != cur) ranges[cur].y = (int)(i + 1);
  }
}

// Ranges built by atomic min/max: start from (INT_MAX, 0), and give tiles
// that received no pair the empty range (0, 0).
__global__ void k_ranges_init(int2* ranges, int tiles) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t < tiles) ranges[t] = make_int2(0x7fffffff, 0);
}

__global__ void k_ranges_fix(int2* ranges, int tiles) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t < tiles && ranges[t].x == 0x7fffffff) ranges[t] = make_int2(0, 0);
}

// 64-bit output keys of the presort path: tile << 32 | depth bits.
template <typename KT>
__global__ void k_make_keys64(const KT* __restrict__ tiles, const uint32_t* __restrict__ vals,
                              const float* __restrict__ depth, const int64_t* n_dev, int64_t cap,
                              uint64_t* __restrict__ keys) {
  const int64_t n = clamp_n(n_dev, cap);
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  keys[i] = ((uint64_t)tiles[i] << 32) | __float_as_uint(depth[vals[i]]);
}

__global__ void k_copy_u64(const uint64_t* __restrict__ a, const int64_t* n_dev, int64_t cap,
                           uint64_t* __restrict__ b) {
  const int64_t n = clamp_n(n_dev, cap);
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) b[i] = a[i];
}

__global__ void k_copy_u32(const uint32_t* __restrict__ a, const int64_t* n_dev, int64_t cap,
                           uint32_t* __restrict__ b) {
  const int64_t n = clamp_n(n_dev, cap);
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) b[i] = a[i];
}

// ---------------------------------------------------------------------------
// Workspace layout and the binning driver.

static inline size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

// Band entries are distributed in chunks of kBandChunk entries of one band.
constexpr int kBandChunk = 1024;
static inline int64_t band_chunk_bound(int64_t cap, int64_t bands) {
  return cap / kBandChunk + bands + 1;
}

struct BinWs {
  uint32_t* okey[2];   // [tiles]  (tile order)
  uint32_t* oval[2];   // [tiles]
  uint32_t* offsets;   // [n_rec]
  uint64_t* partials;  // scan block sums
  uint32_t* counts;    // [256 * nb]
  uint32_t* dtot;      // [1024]    digit totals of a radix pass
  uint32_t* csum;      // [radix * chunks]  chunk sums of the digit columns
  uint32_t* vals_alt;  // [cap]
  uint32_t* dkey[2];   // [n_rec]   (presort)
  uint32_t* perm[2];   // [n_rec]   (presort)
  uint32_t* tkey[2];   // [cap]     (presort)
  uint32_t* first;     // [cap / kSortTile + 2]  (presort)
  uint4* packed;       // [n_rec]   (presort); [max(n_rec, cap)] row records with the cull
  uint32_t* tcs;       // [n_rec]   tile counts in depth order (presort)
  short4* rect_s;      // [n_rec]   rects in depth order (presort without the cull)
  // per-(Gaussian, tile) cull
  uint32_t* kc;        // [n_rec]   kept pairs per record
  uint32_t* nrow;      // [n_rec]   kept rows per record
  uint32_t* roff;      // [n_rec]   first row record, depth order
  uint4* runs;         // [n_rec]   kept runs of up to 3 rows (the LinPrim count pass)
  // band binning
  int64_t* n_ent;      // [1] band entries
  int64_t* n_chunk;    // [1] chunks
  int2* branges;       // [tiles]   entry range per band
  uint32_t* nch;       // [tiles]   chunks per band
  uint32_t* cstart;    // [tiles]   first chunk of each band
  int2* desc;          // [chunks]  (band, first entry)
  uint32_t* ccnt;      // [chunks][16] per chunk and band column: covering entries
  uint32_t* coff;      // [chunks][16] output offset of the chunk's entries per column
  uint32_t* ttot;      // [tiles * 16] per band column: pairs
  uint32_t* tbase;     // [tiles * 16] exclusive scan of ttot
  uint64_t* key64[2];  // [cap]     (full)
  // onesweep passes (zeroed together at the start of the binning)
  uint32_t* sweep;     // start of the zeroed region
  size_t sweep_bytes;
  uint32_t* hist_d;    // [4][256]  depth passes
  uint32_t* hist_t;    // [4][256]  tile passes
  uint32_t* counters;  // [16]      partition counters (depth 0..3, tile 4..7)
  uint32_t* err;       // [1]
  uint32_t* status_d;  // [4][parts of n_rec][256]
  uint32_t* status_t;  // [passes][parts of cap][2^dbits]
  int64_t parts_d, parts_t;
  int t_radix;
  size_t bytes;
};

static inline int tile_id_bits(int64_t tiles) {
  int bits = 1;
  while (bits < 31 && ((int64_t)1 << bits) < tiles) ++bits;
  return bits;
}

static BinWs bin_ws_layout(int64_t n_rec, int64_t cap, int64_t tiles, int sort_mode, bool cull,
                           char* base) {
  BinWs L{};
  size_t off = 0;
  auto take = [&](size_t bytes) -> char* {
    char* p = base ? base + off : nullptr;
    off += align256(bytes);
    return p;
  };
  const int64_t nb_max =
      (std::max(std::max(cap, n_rec), tiles) + kSortTile - 1) / kSortTile + 1;
  for (int k = 0; k < 2; ++k) L.okey[k] = (uint32_t*)take(4 * (size_t)std::max<int64_t>(tiles, 1));
  for (int k = 0; k < 2; ++k) L.oval[k] = (uint32_t*)take(4 * (size_t)std::max<int64_t>(tiles, 1));
  // digit counts per sort block: up to 1024 digits in the band pass
  const int64_t radix_max = sort_mode == XPR_SORT_BANDS ? 1024 : 256;
  const int64_t scan_n = std::max<int64_t>(radix_max * nb_max, n_rec);
  const int64_t nparts = (scan_n + kScanTile - 1) / kScanTile + 1;
  L.offsets = (uint32_t*)take(4 * (size_t)std::max<int64_t>(n_rec, 1));
  L.partials = (uint64_t*)take(8 * (size_t)nparts);
  L.counts = (uint32_t*)take(4 * (size_t)(radix_max * nb_max));
  L.dtot = (uint32_t*)take(4 * 1024);
  L.csum = (uint32_t*)take(4 * (size_t)(radix_max * ((nb_max + kScanTile - 1) / kScanTile)));
  L.vals_alt = (uint32_t*)take(4 * (size_t)std::max<int64_t>(std::max(cap, n_rec), 1));
  if (sort_mode == XPR_SORT_PRESORT || sort_mode == XPR_SORT_BANDS ||
      sort_mode == XPR_SORT_ONESWEEP) {
    for (int k = 0; k < 2; ++k) L.dkey[k] = (uint32_t*)take(4 * (size_t)std::max<int64_t>(n_rec, 1));
    for (int k = 0; k < 2; ++k) L.perm[k] = (uint32_t*)take(4 * (size_t)std::max<int64_t>(n_rec, 1));
    for (int k = 0; k < 2; ++k) L.tkey[k] = (uint32_t*)take(4 * (size_t)std::max<int64_t>(cap, 1));
    L.first = (uint32_t*)take(4 * (size_t)(cap / kSortTile + 2));
    // with the cull a record yields one packed record per kept row, and every
    // kept row holds at least one of the <= cap pairs
    L.packed = (uint4*)take(16 * (size_t)std::max<int64_t>(cull ? std::max(n_rec, cap) : n_rec, 1));
    L.tcs = (uint32_t*)take(4 * (size_t)std::max<int64_t>(n_rec, 1));
    if (!cull) L.rect_s = (short4*)take(8 * (size_t)std::max<int64_t>(n_rec, 1));
    if (cull) {
      L.kc = (uint32_t*)take(4 * (size_t)std::max<int64_t>(n_rec, 1));
      L.nrow = (uint32_t*)take(4 * (size_t)std::max<int64_t>(n_rec, 1));
      L.roff = (uint32_t*)take(4 * (size_t)std::max<int64_t>(n_rec, 1));
      L.runs = (uint4*)take(16 * (size_t)std::max<int64_t>(n_rec, 1));
    }
    if (sort_mode == XPR_SORT_BANDS) {
      const int64_t T1 = std::max<int64_t>(tiles, 1);
      const int64_t nchunk = band_chunk_bound(cap, T1);
      L.n_ent = (int64_t*)take(8);
      L.n_chunk = (int64_t*)take(8);
      L.branges = (int2*)take(8 * (size_t)T1);
      L.nch = (uint32_t*)take(4 * (size_t)T1);
      L.cstart = (uint32_t*)take(4 * (size_t)T1);
      L.desc = (int2*)take(8 * (size_t)nchunk);
      L.ccnt = (uint32_t*)take(4 * (size_t)nchunk * kBandWidth);
      L.coff = (uint32_t*)take(4 * (size_t)nchunk * kBandWidth);
      L.ttot = (uint32_t*)take(4 * (size_t)T1 * kBandWidth);
      L.tbase = (uint32_t*)take(4 * (size_t)T1 * kBandWidth);
    }
  } else {
    for (int k = 0; k < 2; ++k) L.key64[k] = (uint64_t*)take(8 * (size_t)std::max<int64_t>(cap, 1));
  }
  if (sort_mode == XPR_SORT_ONESWEEP) {
    const int tb = tile_id_bits(std::max<int64_t>(tiles, 1));
    L.parts_d = (n_rec + kSortTile - 1) / kSortTile + 1;
    L.parts_t = (cap + kSortTile - 1) / kSortTile + 1;
    L.t_radix = 1 << radix_digit_bits(tb);
    const size_t head = 4 * (4 * 256 + 4 * 256 + 16 + 64);
    const size_t sd = 4 * (size_t)4 * L.parts_d * 256;
    const size_t st = 4 * (size_t)radix_passes(tb) * L.parts_t * L.t_radix;
    char* r = take(head + sd + st);
    L.sweep = (uint32_t*)r;
    L.sweep_bytes = align256(head + sd + st);
    if (r) {
      L.hist_d = (uint32_t*)r;
      L.hist_t = L.hist_d + 4 * 256;
      L.counters = L.hist_t + 4 * 256;
      L.err = L.counters + 16;
      L.status_d = L.err + 64;
      L.status_t = L.status_d + (size_t)4 * L.parts_d * 256;
    }
  }
  L.bytes = off;
  return L;
}

// The onesweep look-back words hold counts below 2^30.
static inline int effective_mode(int sort_mode, bool cull, int64_t cap, int64_t n_rec) {
  if (cull) return XPR_SORT_PRESORT;
  if (sort_mode == XPR_SORT_ONESWEEP &&
      (cap >= ((int64_t)1 << 30) || n_rec >= ((int64_t)1 << 30)))
    return XPR_SORT_PRESORT;
  return sort_mode;
}

size_t bin_workspace_bytes(int64_t n_rec, int64_t cap, int64_t tiles, int sort_mode, bool cull) {
  return bin_ws_layout(n_rec, cap, tiles, effective_mode(sort_mode, cull, cap, n_rec), cull,
                       nullptr).bytes;
}

static inline int grid1(int64_t n, int bs = 256) { return (int)((n + bs - 1) / bs); }

// Kept pairs and kept rows of a record travel through the depth presort as
// one word, kc | rows << bits, when both fit (kc <= tiles of the view, rows
// <= its tile rows); 0 = they do not, rows are then gathered separately.
static int cull_pack_bits(const Batch& B) {
  int64_t tiles = 1, ty = 1;
  for (int v = 0; v < B.n_views; ++v) {
    tiles = std::max<int64_t>(tiles, (int64_t)B.v[v].tiles_x * B.v[v].tiles_y);
    ty = std::max<int64_t>(ty, B.v[v].tiles_y);
  }
  int kb = 1, rb = 1;
  while (((int64_t)1 << kb) <= tiles) ++kb;
  while (((int64_t)1 << rb) <= ty) ++rb;
  return kb + rb <= 32 ? kb : 0;
}

// Phase 1: everything up to a known I (the prefix sum of the counts, in
// depth order for the presort path). Phase 2: replication, pair sort, ranges.
hipError_t bin_phase1(const Batch& B, int sort_mode, bool cull, const float* splat,
                      const int16_t* rect, const float* depth, const int32_t* tc,
                      int64_t n_rec, int64_t cap,
                      int64_t* n_isect, void* ws, hipStream_t st, const uint32_t** perm_out) {
  sort_mode = effective_mode(sort_mode, cull, cap, n_rec);
  BinWs L = bin_ws_layout(n_rec, cap, B.total_tiles, sort_mode, cull, (char*)ws);
  *perm_out = nullptr;
  if (n_rec == 0) {
    hipLaunchKernelGGL(k_set_i64, dim3(1), dim3(64), 0, st, n_isect, (int64_t)0);
    return hipGetLastError();
  }
  if (sort_mode == XPR_SORT_ONESWEEP) {
    // zero the histograms, counters, error word and look-back words of
    // every pass (a fill kernel: the step may be captured in a graph)
    hipLaunchKernelGGL(k_zero_x4, dim3(grid1((int64_t)(L.sweep_bytes / 16))), dim3(256), 0, st,
                       reinterpret_cast<uint4*>(L.sweep), (int64_t)(L.sweep_bytes / 16));
    hipLaunchKernelGGL(k_depth_keys_hist, dim3((int)((n_rec + kSortTile - 1) / kSortTile)),
                       dim3(256), 0, st, depth, tc, n_rec, L.dkey[0], L.perm[0], L.hist_d);
    const int nb = (int)((n_rec + kSortTile - 1) / kSortTile);
    uint32_t *k0 = L.dkey[0], *v0 = L.perm[0], *k1 = L.dkey[1], *v1 = L.perm[1];
    for (int p = 0; p < 4; ++p) {
      const Sweep sw{L.status_d + (size_t)p * L.parts_d * 256, L.counters + p,
                     L.hist_d + 256 * p, L.err};
      hipLaunchKernelGGL((k_sweep_scatter<8, uint32_t, false>), dim3(nb), dim3(256), 0, st, k0,
                         v0, k1, v1, (const int64_t*)nullptr, n_rec, 8 * p, sw, (int2*)nullptr,
                         p == 3 ? tc : nullptr, p == 3 ? L.tcs : nullptr);
      std::swap(k0, k1);
      std::swap(v0, v1);
    }
    *perm_out = v0;
    return device_scan(LoadArray{L.tcs}, n_rec, L.offsets, L.partials, n_isect, st);
  }
  if (sort_mode == XPR_SORT_PRESORT || sort_mode == XPR_SORT_BANDS) {
    const int32_t* counts = tc;
    const int pb = cull ? cull_pack_bits(B) : 0;
    if (cull) {
      if (B.method == XPR_METHOD_LINPRIM)
        hipLaunchKernelGGL(k_cull_count_lin, dim3(grid1(n_rec)), dim3(256), 0, st, B,
                           reinterpret_cast<const float4*>(splat),
                           reinterpret_cast<const short4*>(rect), tc, depth, n_rec, pb, L.kc,
                           L.nrow, L.dkey[0], L.perm[0], L.runs, lin_req(B));
      else
        hipLaunchKernelGGL(k_cull_count<RowGeom>, dim3(grid1(n_rec)), dim3(256), 0, st, B,
                           reinterpret_cast<const float4*>(splat),
                           reinterpret_cast<const short4*>(rect), tc, depth, n_rec, pb, L.kc,
                           L.nrow, L.dkey[0], L.perm[0], lin_req(B));
      counts = reinterpret_cast<const int32_t*>(L.kc);
    } else {
      const int nbk = (int)((n_rec + kSortTile - 1) / kSortTile);
      hipLaunchKernelGGL(k_depth_keys, dim3(nbk), dim3(256), 0, st, depth, tc, n_rec, L.dkey[0],
                         L.perm[0], n_isect, L.counts, nbk);
    }
    uint32_t *ko, *vo;
    // with the cull the kept-pair counts ride along the last pass; without
    // it the rects and tile counts are gathered afterwards in one kernel
    hipError_t e = radix_sort<uint32_t>(L.dkey[0], L.perm[0], L.dkey[1], L.perm[1], nullptr, n_rec,
                                        n_rec, 32, L.counts, L.dtot, L.csum, &ko, &vo, st, 0,
                                        nullptr, true, cull ? counts : nullptr,
                                        cull ? L.tcs : nullptr, !cull);
    if (e != hipSuccess) return e;
    *perm_out = vo;
    if (!cull) {
      // the band path reads the counts in depth order; the pair path
      // derives them from the rects
      hipLaunchKernelGGL(k_sorted_rects, dim3((int)((n_rec + kSortTile - 1) / kSortTile)),
                         dim3(256), 0, st, reinterpret_cast<const short4*>(rect), ko, vo, n_rec,
                         L.rect_s, sort_mode == XPR_SORT_BANDS ? L.tcs : nullptr, L.partials,
                         n_isect);
      return hipGetLastError();
    }
    if (pb > 0) {
      e = device_scan(LoadMask{L.tcs, (1u << pb) - 1u}, n_rec, L.offsets, L.partials, n_isect, st);
      if (e != hipSuccess) return e;
      return device_scan(LoadShift{L.tcs, pb}, n_rec, L.roff, L.partials, nullptr, st);
    }
    e = device_scan(LoadArray{L.tcs}, n_rec, L.offsets, L.partials, n_isect, st);
    if (e != hipSuccess) return e;
    return device_scan(LoadGather{L.nrow, vo}, n_rec, L.roff, L.partials, nullptr, st);
  }
  return device_scan(LoadCount{tc}, n_rec, L.offsets, L.partials, n_isect, st);
}

// Tiles by decreasing list length (ties by tile id): a stable sort of
// 65535 - min(length, 65535).
__global__ void k_tile_len_keys(const int2* __restrict__ ranges, int tiles, uint32_t* key,
                                uint32_t* val) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= tiles) return;
  const int2 r = ranges[t];
  key[t] = 65535u - (uint32_t)min(r.y - r.x, 65535);
  val[t] = (uint32_t)t;
}

static hipError_t tile_order_lpt(const Batch& B, const BinWs& L, const int2* ranges,
                                 int32_t* order, hipStream_t st) {
  const int64_t T = B.total_tiles;
  if (T <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_tile_len_keys, dim3(grid1(T)), dim3(256), 0, st, ranges, (int)T,
                     L.okey[0], L.oval[0]);
  uint32_t *ko, *vo;
  hipError_t e = radix_sort<uint32_t>(L.okey[0], L.oval[0], L.okey[1], L.oval[1], nullptr, T, T,
                                      16, L.counts, L.dtot, L.csum, &ko, &vo, st);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_copy_u32, dim3(grid1(T)), dim3(256), 0, st, vo, (const int64_t*)nullptr, T,
                     (uint32_t*)order);
  return hipGetLastError();
}

static inline bool tiles_16bit(int64_t tiles) { return tiles <= 65536; }

// Depth-presort path, after phase 1: replication fused into the first pass
// of the tile-id sort, the remaining passes on tile keys of type KT (16 bits
// when the tile ids fit), tile ranges built by the last pass. The pass
// count's parity picks the first output buffer so the last pass lands in
// the caller's vals.
template <typename KT>
static hipError_t pair_sort(const Batch& B, int tile_bits, const float* depth, const short4* rc,
                            const float* splat, const uint32_t* perm, int64_t n_rec, int64_t cap,
                            int64_t grid_n,
                            const int64_t* n_isect, uint64_t* keys_out, uint32_t* vals_u,
                            int2* ranges, const BinWs& L, hipStream_t st) {
  const int dbits = radix_digit_bits(tile_bits);
  const int passes = radix_passes(tile_bits);
  const bool one = passes == 1;
  uint32_t* v1 = (passes % 2 == 1) ? vals_u : L.vals_alt;
  uint32_t* v2 = (passes % 2 == 1) ? L.vals_alt : vals_u;
  KT* tk0 = reinterpret_cast<KT*>(L.tkey[0]);
  KT* tk1 = reinterpret_cast<KT*>(L.tkey[1]);
  const int tiles = B.total_tiles;
  hipLaunchKernelGGL(k_ranges_init, dim3(grid1(tiles)), dim3(256), 0, st, ranges, tiles);
  if (splat) {  // per-(Gaussian, tile) cull: one record per kept row
    const int pb = cull_pack_bits(B);
    const uint32_t kmask = pb > 0 ? (1u << pb) - 1u : 0xffffffffu;
    if (B.method == XPR_METHOD_LINPRIM)
      hipLaunchKernelGGL(k_cull_emit_lin, dim3(grid1(n_rec)), dim3(256), 0, st, B,
                         reinterpret_cast<const float4*>(splat), rc, L.tcs, perm, L.offsets,
                         L.roff, kmask, n_rec, n_isect, cap, L.runs, L.packed, L.first,
                         lin_req(B));
    else
      hipLaunchKernelGGL(k_cull_emit<RowGeom>, dim3(grid1(n_rec)), dim3(256), 0, st, B,
                         reinterpret_cast<const float4*>(splat), rc, L.tcs, perm, L.offsets,
                         L.roff, kmask, n_rec, n_isect, cap, L.packed, L.first, lin_req(B));
  } else
    hipLaunchKernelGGL(k_pair_records, dim3((int)((n_rec + kSortTile - 1) / kSortTile)),
                       dim3(256), 0, st, B, L.rect_s, perm, L.partials, n_rec, n_isect, cap,
                       L.packed, L.first);
  const int nb = (int)((grid_n + kSortTile - 1) / kSortTile);
  KT* k1 = (one && !keys_out) ? nullptr : tk0;
#define XPR_PAIR_HIST(BITS, ITEMS)                                                          \
  hipLaunchKernelGGL((k_pair_hist<BITS, ITEMS, kHistThreads>), dim3(nb), dim3(kHistThreads), 0,  \
                     st, L.packed, L.first,                                                   \
                     n_isect, cap, L.counts, nb)
  if (dbits == 7) {
    if (splat) XPR_PAIR_HIST(7, RowItems); else XPR_PAIR_HIST(7, PairItems);
  } else {
    if (splat) XPR_PAIR_HIST(8, RowItems); else XPR_PAIR_HIST(8, PairItems);
  }
#undef XPR_PAIR_HIST
  hipError_t e = digit_scan(L.counts, nb, 1 << dbits, L.dtot, L.csum, st);
  if (e != hipSuccess) return e;
#define XPR_PAIR_SCATTER(BITS, LAST, ITEMS)                                                 \
  hipLaunchKernelGGL((k_pair_scatter<BITS, LAST, KT, ITEMS, kPairThreads>), dim3(nb),           \
                     dim3(kPairThreads), 0, st,                                               \
                     L.packed,                                                               \
                     L.first, n_isect, cap, L.counts, L.dtot, nb, k1, v1,                   \
                     LAST ? ranges : (int2*)nullptr)
#define XPR_PAIR_SCATTER_I(BITS, LAST)                                                      \
  do {                                                                                      \
    if (splat) XPR_PAIR_SCATTER(BITS, LAST, RowItems);                                      \
    else XPR_PAIR_SCATTER(BITS, LAST, PairItems);                                           \
  } while (0)
  if (dbits == 7) {
    if (one) XPR_PAIR_SCATTER_I(7, true); else XPR_PAIR_SCATTER_I(7, false);
  } else {
    if (one) XPR_PAIR_SCATTER_I(8, true); else XPR_PAIR_SCATTER_I(8, false);
  }
#undef XPR_PAIR_SCATTER_I
#undef XPR_PAIR_SCATTER
  KT* ko = tk0;
  uint32_t* vo = v1;
  if (!one) {
    e = radix_sort<KT>(tk0, v1, tk1, v2, n_isect, cap, grid_n, tile_bits, L.counts, L.dtot,
                       L.csum, &ko, &vo, st, dbits, ranges, keys_out != nullptr);
    if (e != hipSuccess) return e;
  }
  hipLaunchKernelGGL(k_ranges_fix, dim3(grid1(tiles)), dim3(256), 0, st, ranges, tiles);
  if (keys_out)
    hipLaunchKernelGGL(k_make_keys64<KT>, dim3(grid1(grid_n)), dim3(256), 0, st, ko, vo, depth,
                       n_isect, cap, keys_out);
  if (vo != vals_u) return hipErrorUnknown;  // the pass parity above guarantees vo == vals
  return hipGetLastError();
}

// Onesweep path after phase 1 (XPR_SORT_ONESWEEP): the records' pass over
// the depth order also takes the digit counts of every tile pass, the first
// pass generates the pairs in LDS (as k_pair_scatter), each pass is one
// kernel, the last writes the ranges.
template <typename KT>
static hipError_t pair_sort_sweep(const Batch& B, int tile_bits, const float* depth,
                                  const short4* rc, const uint32_t* perm, int64_t n_rec,
                                  int64_t cap, int64_t grid_n, const int64_t* n_isect,
                                  uint64_t* keys_out, uint32_t* vals_u, int2* ranges,
                                  const BinWs& L, hipStream_t st) {
  const int dbits = radix_digit_bits(tile_bits);
  const int passes = radix_passes(tile_bits);
  if (passes > kSweepMaxPasses || (1 << dbits) != L.t_radix) return hipErrorInvalidValue;
  uint32_t* v1 = (passes % 2 == 1) ? vals_u : L.vals_alt;
  uint32_t* v2 = (passes % 2 == 1) ? L.vals_alt : vals_u;
  KT* tk0 = reinterpret_cast<KT*>(L.tkey[0]);
  KT* tk1 = reinterpret_cast<KT*>(L.tkey[1]);
  const int tiles = B.total_tiles;
  hipLaunchKernelGGL(k_ranges_init, dim3(grid1(tiles)), dim3(256), 0, st, ranges, tiles);
  hipLaunchKernelGGL(k_pair_records_hist, dim3((int)((n_rec + kSortTile - 1) / kSortTile)),
                     dim3(256), 0, st, B, rc, L.tcs, perm, L.offsets, n_rec, n_isect, cap, dbits,
                     passes, L.packed, L.first, L.hist_t);
  const int nb = (int)((grid_n + kSortTile - 1) / kSortTile);
  auto sweep_of = [&](int p) {
    return Sweep{L.status_t + (size_t)p * L.parts_t * L.t_radix, L.counters + 4 + p,
                 L.hist_t + 256 * p, L.err};
  };
  const bool one = passes == 1;
  KT* k1 = (one && !keys_out) ? nullptr : tk0;
#define XPR_SWEEP_PAIR(BITS, LAST)                                                          \
  hipLaunchKernelGGL((k_sweep_pair_scatter<BITS, LAST, KT>), dim3(nb), dim3(256), 0, st,    \
                     L.packed, L.first, n_isect, cap, sweep_of(0), k1, v1,                  \
                     LAST ? ranges : (int2*)nullptr)
  if (dbits == 7) {
    if (one) XPR_SWEEP_PAIR(7, true); else XPR_SWEEP_PAIR(7, false);
  } else {
    if (one) XPR_SWEEP_PAIR(8, true); else XPR_SWEEP_PAIR(8, false);
  }
#undef XPR_SWEEP_PAIR
  KT* ka = tk0;
  KT* kb = tk1;
  uint32_t* va = v1;
  uint32_t* vb = v2;
  for (int p = 1; p < passes; ++p) {
    const int shift = p * dbits;
    const bool last = p == passes - 1;
    const int pb = std::min(dbits, tile_bits - shift);
    KT* kdst = (last && !keys_out) ? nullptr : kb;
    int2* rg = last ? ranges : nullptr;
    const Sweep sw = sweep_of(p);
#define XPR_SWEEP(BITS)                                                                     \
  do {                                                                                      \
    if (last)                                                                               \
      hipLaunchKernelGGL((k_sweep_scatter<BITS, KT, true>), dim3(nb), dim3(256), 0, st, ka, \
                         va, kdst, vb, n_isect, cap, shift, sw, rg, (const int32_t*)nullptr, \
                         (uint32_t*)nullptr);                                               \
    else                                                                                    \
      hipLaunchKernelGGL((k_sweep_scatter<BITS, KT, false>), dim3(nb), dim3(256), 0, st,    \
                         ka, va, kdst, vb, n_isect, cap, shift, sw, rg,                     \
                         (const int32_t*)nullptr, (uint32_t*)nullptr);                      \
  } while (0)
    switch (pb) {
      case 8: XPR_SWEEP(8); break;
      case 7: XPR_SWEEP(7); break;
      case 6: XPR_SWEEP(6); break;
      case 5: XPR_SWEEP(5); break;
      case 4: XPR_SWEEP(4); break;
      case 3: XPR_SWEEP(3); break;
      case 2: XPR_SWEEP(2); break;
      default: XPR_SWEEP(1); break;
    }
#undef XPR_SWEEP
    std::swap(ka, kb);
    std::swap(va, vb);
  }
  hipLaunchKernelGGL(k_ranges_fix, dim3(grid1(tiles)), dim3(256), 0, st, ranges, tiles);
  if (keys_out)
    hipLaunchKernelGGL(k_make_keys64<KT>, dim3(grid1(grid_n)), dim3(256), 0, st, ka, va, depth,
                       n_isect, cap, keys_out);
  hipLaunchKernelGGL(k_sweep_check, dim3(1), dim3(64), 0, st, L.err, (int64_t*)n_isect);
  if (va != vals_u) return hipErrorUnknown;  // the pass parity above guarantees va == vals
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Band binning (depth-presort path, XPR_SORT_BANDS). The stable sort by
// (tile id, depth) is done in two stages that exploit the rect shape of a
// record's tiles. A band is one tile row by kBandWidth tile columns of one
// view; band ids run in tile-id order (view, row, column band).
//  1. Every record yields one entry per (row, band) of its rect, carrying
//     its depth position j and its column range inside the band; the
//     entries (about pairs / 4) are radix-sorted stably by band id, the
//     replication fused into the first pass as for pairs.
//  2. The entries of each band are cut into chunks of kBandChunk. Per chunk
//     and band column, the covering entries are counted with one wave64
//     ballot per (item, column); scans over (band, column) give each tile
//     its output range and each chunk its offset inside it; then the same
//     ballots rank the covering entries of every (wave, column) and they
//     write their record ids, in depth order, as coalesced runs.
// The result (vals, tile ranges, optional keys) is identical to the pair
// sort's: the low 4 bits of the tile key are placed by the counting step
// instead of a scatter pass, and 61M pairs are written once.

__device__ __forceinline__ void view_bands(const Batch& B, int v, int& nbx, int& boff) {
  boff = 0;
  for (int q = 0; q < v; ++q)
    boff += (int)B.v[q].tiles_y * (((int)B.v[q].tiles_x + kBandWidth - 1) / kBandWidth);
  nbx = ((int)B.v[v].tiles_x + kBandWidth - 1) / kBandWidth;
}

// Packed band record and entry count per depth-ordered record. ne aliases
// the tile counts it is computed from (read before written, same index).
__global__ void k_band_records(Batch B, const short4* __restrict__ rect, const uint32_t* tcs,
                               const uint32_t* __restrict__ perm, int64_t n_rec,
                               uint4* __restrict__ packed, uint32_t* ne) {
  const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= n_rec) return;
  if (tcs[j] == 0u) {
    ne[j] = 0u;
    return;
  }
  const uint32_t r = perm[j];
  int v = 0;
  for (int q = 1; q < B.n_views; ++q)
    if ((int32_t)r >= B.v[q].rec_off) v = q;
  const short4 rc = rect[r];
  int nbx, boff;
  view_bands(B, v, nbx, boff);
  const int bx0 = rc.x / kBandWidth, bx1 = (rc.z - 1) / kBandWidth;
  const uint32_t nbr = (uint32_t)(bx1 - bx0 + 1);
  packed[j] = make_uint4(0u, (uint32_t)(boff + rc.y * nbx + bx0), nbr | ((uint32_t)nbx << 16),
                         (uint32_t)rc.x | ((uint32_t)rc.z << 16));
  ne[j] = (uint32_t)(rc.w - rc.y) * nbr;
}

// Entry offsets into the packed records and the sort-block map (as
// k_pair_records does for pairs), n = min(entries, capacity).
__global__ void k_band_first(const uint32_t* __restrict__ ne, const uint32_t* __restrict__ eoff,
                             int64_t n_rec, const int64_t* n_ent, int64_t cap,
                             uint4* __restrict__ packed, uint32_t* __restrict__ first) {
  const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= n_rec) return;
  const int64_t n = clamp_n(n_ent, cap);
  const int64_t o = eoff[j];
  const int64_t e = min(o + (int64_t)ne[j], n);
  if (e <= o) return;
  packed[j].x = (uint32_t)o;
  for (int64_t b = (o + kSortTile - 1) / kSortTile; b * kSortTile < e; ++b) first[b] = (uint32_t)j;
  if (e == n) first[(n + kSortTile - 1) / kSortTile] = (uint32_t)j;
}

__global__ void k_band_nchunks(const int2* __restrict__ br, int nbk, uint32_t* __restrict__ nch) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b < nbk) nch[b] = (uint32_t)((br[b].y - br[b].x + kBandChunk - 1) / kBandChunk);
}

__global__ void k_band_desc(const int2* __restrict__ br, const uint32_t* __restrict__ nch,
                            const uint32_t* __restrict__ cstart, int nbk,
                            int2* __restrict__ desc) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= nbk) return;
  const uint32_t c0 = cstart[b];
  for (uint32_t i = 0; i < nch[b]; ++i)
    desc[c0 + i] = make_int2(b, br[b].x + (int)i * kBandChunk);
}

// Chunk entry i = 256 w + 64 item + lane of wave w. The values of a
// thread's 4 items and, per wave, the number of covering entries per band
// column (lane-uniform).
struct ChunkItems {
  uint32_t xlo[4], xhi[4];
  bool ok[4];
};

__device__ __forceinline__ void chunk_load(const uint32_t* __restrict__ ev, int first, int end,
                                           ChunkItems& it, uint32_t* jpos) {
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  uint32_t v[4];
#pragma unroll
  for (int q = 0; q < 4; ++q) v[q] = ev[min(first + 256 * w + 64 * q + lane, end - 1)];
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    it.ok[q] = first + 256 * w + 64 * q + lane < end;
    it.xlo[q] = (v[q] >> 23) & 15u;
    it.xhi[q] = ((v[q] >> 27) & 15u) + 1u;
    if (jpos) jpos[q] = v[q] & 0x7fffffu;
  }
}

__device__ __forceinline__ void chunk_wave_counts(const ChunkItems& it, uint32_t (&acc)[kBandWidth]) {
#pragma unroll
  for (int x = 0; x < kBandWidth; ++x) acc[x] = 0u;
#pragma unroll
  for (int q = 0; q < 4; ++q)
#pragma unroll
    for (int x = 0; x < kBandWidth; ++x)
      acc[x] += (uint32_t)__popcll(__ballot(it.ok[q] && it.xlo[q] <= (uint32_t)x &&
                                            (uint32_t)x < it.xhi[q]));
}

__global__ __launch_bounds__(256) void k_band_count(const int2* __restrict__ desc,
                                                    const int64_t* n_chunk,
                                                    const int2* __restrict__ br,
                                                    const uint32_t* __restrict__ ev,
                                                    uint32_t* __restrict__ ccnt) {
  __shared__ uint32_t wc[4][kBandWidth];
  const int c = blockIdx.x;
  if ((int64_t)c >= *n_chunk) return;
  const int2 d = desc[c];
  const int end = min(d.y + kBandChunk, br[d.x].y);
  ChunkItems it;
  chunk_load(ev, d.y, end, it, nullptr);
  uint32_t acc[kBandWidth];
  chunk_wave_counts(it, acc);
  const int w = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0)
#pragma unroll
    for (int x = 0; x < kBandWidth; ++x) wc[w][x] = acc[x];
  __syncthreads();
  if (threadIdx.x < kBandWidth) {
    const int x = threadIdx.x;
    ccnt[(int64_t)c * kBandWidth + x] = wc[0][x] + wc[1][x] + wc[2][x] + wc[3][x];
  }
}

// Per (band, column): pairs over the band's chunks.
__global__ void k_band_totals(const uint32_t* __restrict__ cstart,
                              const uint32_t* __restrict__ nch, int nbk,
                              const uint32_t* __restrict__ ccnt, uint32_t* __restrict__ ttot) {
  const int id = blockIdx.x * blockDim.x + threadIdx.x;
  if (id >= nbk * kBandWidth) return;
  const int b = id / kBandWidth, x = id - b * kBandWidth;
  const uint32_t c0 = cstart[b], c1 = c0 + nch[b];
  uint32_t s = 0;
  for (uint32_t c = c0; c < c1; ++c) s += ccnt[(size_t)c * kBandWidth + x];
  ttot[id] = s;
}

// Chunk offsets per column, and the tile ranges ((0, 0) when empty).
__global__ void k_band_offsets(Batch B, const uint32_t* __restrict__ cstart,
                               const uint32_t* __restrict__ nch, int nbk,
                               const uint32_t* __restrict__ ccnt,
                               const uint32_t* __restrict__ ttot,
                               const uint32_t* __restrict__ tbase, uint32_t* __restrict__ coff,
                               int2* __restrict__ ranges) {
  const int id = blockIdx.x * blockDim.x + threadIdx.x;
  if (id >= nbk * kBandWidth) return;
  const int b = id / kBandWidth, x = id - b * kBandWidth;
  uint32_t run = tbase[id];
  const uint32_t c0 = cstart[b], c1 = c0 + nch[b];
  for (uint32_t c = c0; c < c1; ++c) {
    coff[(size_t)c * kBandWidth + x] = run;
    run += ccnt[(size_t)c * kBandWidth + x];
  }
  int v = 0, boff = 0, nbx = 0;
  for (;; ++v) {
    nbx = ((int)B.v[v].tiles_x + kBandWidth - 1) / kBandWidth;
    const int nv = (int)B.v[v].tiles_y * nbx;
    if (b < boff + nv || v == B.n_views - 1) break;
    boff += nv;
  }
  const int ty = (b - boff) / nbx, band = (b - boff) - ty * nbx;
  const int tx = band * kBandWidth + x;
  if (tx < (int)B.v[v].tiles_x) {
    const int tile = B.v[v].tile_off + ty * (int)B.v[v].tiles_x + tx;
    const uint32_t n = ttot[id];
    ranges[tile] = n ? make_int2((int)tbase[id], (int)(tbase[id] + n)) : make_int2(0, 0);
  }
}

// Writes each chunk's records into its tiles' lists: per (wave, item,
// column) the covering lanes take consecutive slots after the chunk's
// offset and the earlier waves' and items' counts.
__global__ __launch_bounds__(256) void k_band_emit(Batch B, const int2* __restrict__ desc,
                                                   const int64_t* n_chunk,
                                                   const int2* __restrict__ br,
                                                   const uint32_t* __restrict__ ev,
                                                   const uint32_t* __restrict__ perm,
                                                   const uint32_t* __restrict__ coff, int64_t cap,
                                                   uint32_t* __restrict__ vals,
                                                   uint64_t* __restrict__ keys,
                                                   const float* __restrict__ depth) {
  __shared__ uint32_t wc[4][kBandWidth];
  const int c = blockIdx.x;
  if ((int64_t)c >= *n_chunk) return;
  const int2 d = desc[c];
  const int end = min(d.y + kBandChunk, br[d.x].y);
  ChunkItems it;
  uint32_t jpos[4];
  chunk_load(ev, d.y, end, it, jpos);
  uint32_t rec[4];
#pragma unroll
  for (int q = 0; q < 4; ++q) rec[q] = perm[jpos[q]];
  uint32_t acc[kBandWidth];
  chunk_wave_counts(it, acc);
  const int w = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0)
#pragma unroll
    for (int x = 0; x < kBandWidth; ++x) wc[w][x] = acc[x];
  __syncthreads();
  uint32_t pos[kBandWidth];
#pragma unroll
  for (int x = 0; x < kBandWidth; ++x) {
    uint32_t p = coff[(size_t)c * kBandWidth + x];
    for (int q = 0; q < w; ++q) p += wc[q][x];
    pos[x] = p;
  }
  // tile id of column 0 of this band (for the optional 64-bit keys)
  int tile0 = 0;
  if (keys) {
    int v = 0, boff = 0, nbx = 0;
    for (;; ++v) {
      nbx = ((int)B.v[v].tiles_x + kBandWidth - 1) / kBandWidth;
      const int nv = (int)B.v[v].tiles_y * nbx;
      if (d.x < boff + nv || v == B.n_views - 1) break;
      boff += nv;
    }
    const int ty = (d.x - boff) / nbx, band = (d.x - boff) - ty * nbx;
    tile0 = B.v[v].tile_off + ty * (int)B.v[v].tiles_x + band * kBandWidth;
  }
  const uint64_t lt = lanemask_lt();
#pragma unroll
  for (int q = 0; q < 4; ++q) {
#pragma unroll
    for (int x = 0; x < kBandWidth; ++x) {
      const bool cov = it.ok[q] && it.xlo[q] <= (uint32_t)x && (uint32_t)x < it.xhi[q];
      const uint64_t m = __ballot(cov);
      const uint32_t p = pos[x] + (uint32_t)__popcll(m & lt);
      if (cov && (int64_t)p < cap) {
        vals[p] = rec[q];
        if (keys) keys[p] = ((uint64_t)(uint32_t)(tile0 + x) << 32) | __float_as_uint(depth[rec[q]]);
      }
      pos[x] += (uint32_t)__popcll(m);
    }
  }
}

static inline int bits_for(int64_t n) {
  int b = 1;
  while (((int64_t)1 << b) < n) ++b;
  return b;
}

static int band_count(const Batch& B) {
  int nbk = 0;
  for (int v = 0; v < B.n_views; ++v)
    nbk += (int)B.v[v].tiles_y * (((int)B.v[v].tiles_x + kBandWidth - 1) / kBandWidth);
  return nbk;
}

static hipError_t band_sort(const Batch& B, const float* depth, const short4* rc,
                            const uint32_t* perm, int64_t n_rec, int64_t cap, int64_t grid_n,
                            uint64_t* keys_out, uint32_t* vals_u, int2* ranges, const BinWs& L,
                            hipStream_t st) {
  const int nbk = band_count(B);
  // 1. entries per record, their offsets, the sort-block map
  hipLaunchKernelGGL(k_band_records, dim3(grid1(n_rec)), dim3(256), 0, st, B, rc, L.tcs, perm,
                     n_rec, L.packed, L.tcs);
  hipError_t e = device_scan(LoadArray{L.tcs}, n_rec, L.offsets, L.partials, L.n_ent, st);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_band_first, dim3(grid1(n_rec)), dim3(256), 0, st, L.tcs, L.offsets, n_rec,
                     (const int64_t*)L.n_ent, cap, L.packed, L.first);
  // 2. entries sorted by band; the last pass leaves them in vals_alt (the
  // caller's vals serve as the other buffer until the final write)
  // up to 10 band bits in one pass (1024 buckets), else 7/8-bit digits
  const int bits = bits_for(nbk);
  const int dbits = bits <= 10 ? std::max(bits, 7) : radix_digit_bits(bits);
  const int passes = bits <= 10 ? 1 : radix_passes(bits);
  const bool one = passes == 1;
  uint32_t* v1 = (passes % 2 == 1) ? L.vals_alt : vals_u;
  uint32_t* v2 = (passes % 2 == 1) ? vals_u : L.vals_alt;
  uint16_t* tk0 = reinterpret_cast<uint16_t*>(L.tkey[0]);
  uint16_t* tk1 = reinterpret_cast<uint16_t*>(L.tkey[1]);
  hipLaunchKernelGGL(k_ranges_init, dim3(grid1(nbk)), dim3(256), 0, st, L.branges, nbk);
  const int nb = (int)((grid_n + kSortTile - 1) / kSortTile);
#define XPR_BAND_HIST(BITS)                                                                   \
  hipLaunchKernelGGL((k_pair_hist<BITS, BandItems, kHistThreads>), dim3(nb), dim3(kHistThreads),  \
                     0, st, L.packed,                                                         \
                     L.first, (const int64_t*)L.n_ent, cap, L.counts, nb)
  switch (dbits) {
    case 7: XPR_BAND_HIST(7); break;
    case 8: XPR_BAND_HIST(8); break;
    case 9: XPR_BAND_HIST(9); break;
    default: XPR_BAND_HIST(10); break;
  }
#undef XPR_BAND_HIST
  e = digit_scan(L.counts, nb, 1 << dbits, L.dtot, L.csum, st);
  if (e != hipSuccess) return e;
  uint16_t* k1 = one ? nullptr : tk0;
#define XPR_BAND_SCATTER(BITS, LAST)                                                          \
  hipLaunchKernelGGL((k_pair_scatter<BITS, LAST, uint16_t, BandItems, kPairThreads>), dim3(nb),  \
                     dim3(kPairThreads), 0,                                                   \
                     st, L.packed, L.first, (const int64_t*)L.n_ent, cap, L.counts, L.dtot, nb, k1, \
                     v1,                                                                       \
                     LAST ? L.branges : (int2*)nullptr)
  switch (dbits) {
    case 7: if (one) XPR_BAND_SCATTER(7, true); else XPR_BAND_SCATTER(7, false); break;
    case 8: if (one) XPR_BAND_SCATTER(8, true); else XPR_BAND_SCATTER(8, false); break;
    case 9: XPR_BAND_SCATTER(9, true); break;
    default: XPR_BAND_SCATTER(10, true); break;
  }
#undef XPR_BAND_SCATTER
  uint16_t* ko = tk0;
  uint32_t* vo = v1;
  if (!one) {
    e = radix_sort<uint16_t>(tk0, v1, tk1, v2, (const int64_t*)L.n_ent, cap, grid_n, bits,
                             L.counts, L.dtot, L.csum, &ko, &vo, st, dbits, L.branges, false);
    if (e != hipSuccess) return e;
  }
  if (vo != L.vals_alt) return hipErrorUnknown;  // the pass parity above guarantees it
  hipLaunchKernelGGL(k_ranges_fix, dim3(grid1(nbk)), dim3(256), 0, st, L.branges, nbk);
  // 3. chunks of each band's entries
  hipLaunchKernelGGL(k_band_nchunks, dim3(grid1(nbk)), dim3(256), 0, st, L.branges, nbk, L.nch);
  e = device_scan(LoadArray{L.nch}, nbk, L.cstart, L.partials, L.n_chunk, st);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_band_desc, dim3(grid1(nbk)), dim3(256), 0, st, L.branges, L.nch, L.cstart,
                     nbk, L.desc);
  const int64_t nch_bound = band_chunk_bound(grid_n, nbk);
  hipLaunchKernelGGL(k_band_count, dim3(nch_bound), dim3(256), 0, st, L.desc,
                     (const int64_t*)L.n_chunk, L.branges, L.vals_alt, L.ccnt);
  // 4. tile ranges and chunk offsets
  const int ncol = nbk * kBandWidth;
  hipLaunchKernelGGL(k_band_totals, dim3(grid1(ncol)), dim3(256), 0, st, L.cstart, L.nch, nbk,
                     L.ccnt, L.ttot);
  e = device_scan(LoadArray{L.ttot}, ncol, L.tbase, L.partials, nullptr, st);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_band_offsets, dim3(grid1(ncol)), dim3(256), 0, st, B, L.cstart, L.nch, nbk,
                     L.ccnt, L.ttot, L.tbase, L.coff, ranges);
  // 5. the records into their tiles' lists
  hipLaunchKernelGGL(k_band_emit, dim3(nch_bound), dim3(256), 0, st, B, L.desc,
                     (const int64_t*)L.n_chunk, L.branges, L.vals_alt, perm, L.coff, cap, vals_u,
                     keys_out, depth);
  return hipGetLastError();
}

hipError_t bin_phase2(const Batch& B, int sort_mode, bool cull, const float* splat,
                      int tile_bits, const float* depth, const int16_t* rect, const int32_t* tc,
                      const uint32_t* perm, int64_t n_rec,
                      int64_t cap, int64_t grid_n, const int64_t* n_isect, uint64_t* keys_out,
                      int32_t* vals, int2* ranges, int32_t* tile_order, void* ws, size_t ws_bytes,
                      hipStream_t st) {
  (void)ws_bytes;
  sort_mode = effective_mode(sort_mode, cull, cap, n_rec);
  BinWs L = bin_ws_layout(n_rec, cap, B.total_tiles, sort_mode, cull, (char*)ws);
  const float* cull_splat = cull ? splat : nullptr;
  const bool band_ok =
      sort_mode == XPR_SORT_BANDS && band_count(B) <= 65536 && n_rec < ((int64_t)1 << 23);
  // the presort and onesweep paths initialise every tile range themselves
  const bool own_init = n_rec > 0 && grid_n > 0 &&
                        (sort_mode == XPR_SORT_ONESWEEP ||
                         ((sort_mode == XPR_SORT_PRESORT || sort_mode == XPR_SORT_BANDS) &&
                          !band_ok));
  if (!own_init)
    hipLaunchKernelGGL(k_fill_u32, dim3(grid1(2 * (int64_t)B.total_tiles)), dim3(256), 0, st,
                       (uint32_t*)ranges, 2 * (int64_t)B.total_tiles, 0u);
  if (n_rec == 0 || grid_n == 0) {
    if (tile_order) return tile_order_lpt(B, L, ranges, tile_order, st);
    return hipGetLastError();
  }
  const short4* rc = reinterpret_cast<const short4*>(rect);
  uint32_t* vals_u = reinterpret_cast<uint32_t*>(vals);
  const int nbd = grid1(n_rec);
  if (sort_mode == XPR_SORT_ONESWEEP) {
    const hipError_t e =
        tiles_16bit(B.total_tiles)
            ? pair_sort_sweep<uint16_t>(B, tile_bits, depth, rc, perm, n_rec, cap, grid_n,
                                        n_isect, keys_out, vals_u, ranges, L, st)
            : pair_sort_sweep<uint32_t>(B, tile_bits, depth, rc, perm, n_rec, cap, grid_n,
                                        n_isect, keys_out, vals_u, ranges, L, st);
    if (e != hipSuccess) return e;
  } else if (band_ok) {
    const hipError_t e = band_sort(B, depth, rc, perm, n_rec, cap, grid_n, keys_out, vals_u,
                                   ranges, L, st);
    if (e != hipSuccess) return e;
  } else if (sort_mode == XPR_SORT_PRESORT || sort_mode == XPR_SORT_BANDS) {
    const hipError_t e =
        tiles_16bit(B.total_tiles)
            ? pair_sort<uint16_t>(B, tile_bits, depth, rc, cull_splat, perm, n_rec, cap, grid_n,
                                  n_isect, keys_out, vals_u, ranges, L, st)
            : pair_sort<uint32_t>(B, tile_bits, depth, rc, cull_splat, perm, n_rec, cap, grid_n,
                                  n_isect, keys_out, vals_u, ranges, L, st);
    if (e != hipSuccess) return e;
  } else {
    const int bits = 32 + tile_bits;
    const int passes = radix_passes(bits);
    uint32_t* v_start = (passes % 2 == 0) ? vals_u : L.vals_alt;
    uint32_t* v_other = (passes % 2 == 0) ? L.vals_alt : vals_u;
    hipLaunchKernelGGL((k_duplicate<false, true>), dim3(nbd), dim3(256), 0, st, B, rc, tc, depth,
                       (const uint32_t*)nullptr, L.offsets, n_rec, cap, (void*)L.key64[0], v_start);
    uint64_t* ko;
    uint32_t* vo;
    hipError_t e = radix_sort<uint64_t>(L.key64[0], v_start, L.key64[1], v_other, n_isect, cap,
                                        grid_n, bits, L.counts, L.dtot, L.csum, &ko, &vo, st);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_ranges<uint64_t>, dim3(grid1((grid_n + 3) / 4)), dim3(256), 0, st, ko,
                       n_isect, cap, B.total_tiles, ranges);
    if (keys_out)
      hipLaunchKernelGGL(k_copy_u64, dim3(grid1(grid_n)), dim3(256), 0, st, ko, n_isect, cap,
                         keys_out);
    if (vo != vals_u)
      hipLaunchKernelGGL(k_copy_u32, dim3(grid1(grid_n)), dim3(256), 0, st, vo, n_isect, cap,
                         vals_u);
  }
  if (tile_order) return tile_order_lpt(B, L, ranges, tile_order, st);
  return hipGetLastError();
}

hipError_t fill_zero_f32(float* p, int64_t n, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  // 16-byte stores over the aligned multiple of 4 floats, then the rest
  const int64_t n4 = ((uintptr_t)p & 15u) == 0 ? n / 4 : 0;
  if (n4 > 0)
    hipLaunchKernelGGL(k_zero_x4, dim3(grid1(n4)), dim3(256), 0, st, reinterpret_cast<uint4*>(p),
                       n4);
  const int64_t rest = n - 4 * n4;
  if (rest > 0)
    hipLaunchKernelGGL(k_fill_u32, dim3(grid1(rest)), dim3(256), 0, st,
                       reinterpret_cast<uint32_t*>(p + 4 * n4), rest, 0u);
  return hipGetLastError();
}

}  // namespace xpr
