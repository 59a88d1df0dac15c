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

#include "xpr_internal.h"

namespace xpr {

constexpr int kScanItems = 16;
constexpr int kScanTile = 256 * kScanItems;
constexpr int kSortItems = 16;
constexpr int kSortTile = 256 * kSortItems;  // keys per scatter block
constexpr int kSortWaves = 4;

// ---------------------------------------------------------------------------
// Block-level helpers (256 threads = 4 waves).

__device__ __forceinline__ uint32_t wave_incl_scan(uint32_t x) {
  const int lane = threadIdx.x & 63;
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    const uint32_t y = __shfl_up(x, d, 64);
    if (lane >= d) x += y;
  }
  return x;
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
// Device-wide exclusive scan of n uint32 values (n known on the host),
// three kernels: block sums, scan of block sums, block scans + offset.

struct LoadArray {
  const uint32_t* p;
  __device__ __forceinline__ uint32_t operator()(int64_t i) const { return p[i]; }
};
struct LoadCount {  // tile counts of records, in record order
  const int32_t* tc;
  __device__ __forceinline__ uint32_t operator()(int64_t i) const { return (uint32_t)tc[i]; }
};
struct LoadCountPerm {  // tile counts of records, in depth order
  const int32_t* tc;
  const uint32_t* perm;
  __device__ __forceinline__ uint32_t operator()(int64_t i) const {
    return (uint32_t)tc[perm[i]];
  }
};

template <class L>
__global__ __launch_bounds__(256) void k_scan_reduce(L load, int64_t n, uint64_t* partials) {
  __shared__ uint64_t s_wave[4];
  const int64_t base = (int64_t)blockIdx.x * kScanTile;
  uint64_t s = 0;
#pragma unroll
  for (int j = 0; j < kScanItems; ++j) {
    const int64_t i = base + j * 256 + threadIdx.x;
    if (i < n) s += load(i);
  }
  s = block_sum256_u64(s, s_wave);
  if (threadIdx.x == 0) partials[blockIdx.x] = s;
}

// Single block: in-place exclusive scan of the block sums; the grand total
// goes to *total (if not null).
__global__ __launch_bounds__(1024) void k_scan_partials(uint64_t* partials, int64_t nparts,
                                                        int64_t* total) {
  __shared__ uint64_t s_wave[16];
  __shared__ uint64_t s_carry;
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  if (threadIdx.x == 0) s_carry = 0;
  __syncthreads();
  for (int64_t base = 0; base < nparts; base += 1024) {
    const int64_t i = base + threadIdx.x;
    const uint64_t x = i < nparts ? partials[i] : 0;
    uint64_t inc = x;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
      const uint64_t y = __shfl_up(inc, d, 64);
      if (lane >= d) inc += y;
    }
    if (lane == 63) s_wave[w] = inc;
    __syncthreads();
    uint64_t off = s_carry;
    for (int k = 0; k < w; ++k) off += s_wave[k];
    if (i < nparts) partials[i] = off + inc - x;
    __syncthreads();
    if (threadIdx.x == 0) {
      uint64_t t = 0;
      for (int k = 0; k < 16; ++k) t += s_wave[k];
      s_carry += t;
    }
    __syncthreads();
  }
  if (threadIdx.x == 0 && total) *total = (int64_t)s_carry;
}

template <class L>
__global__ __launch_bounds__(256) void k_scan_down(L load, int64_t n, const uint64_t* partials,
                                                   uint32_t* out) {
  // 16 items per thread, staged through LDS with one pad word per 16 so the
  // per-thread contiguous reads are free of bank conflicts.
  __shared__ uint32_t s[kScanTile + kScanTile / 16];
  __shared__ uint32_t s_wave[4];
  const int64_t base = (int64_t)blockIdx.x * kScanTile;
  const int t = threadIdx.x;
#pragma unroll
  for (int j = 0; j < kScanItems; ++j) {
    const int i = j * 256 + t;
    s[i + (i >> 4)] = (base + i < n) ? load(base + i) : 0u;
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
  const uint32_t boff = (uint32_t)partials[blockIdx.x];
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
  hipLaunchKernelGGL(k_scan_partials, dim3(1), dim3(1024), 0, st, partials, nb, total);
  hipLaunchKernelGGL(k_scan_down<L>, dim3(nb), dim3(256), 0, st, load, n, partials, out);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Small utility kernels.

__global__ void k_fill_u32(uint32_t* p, int64_t n, uint32_t v) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

__global__ void k_set_i64(int64_t* p, int64_t v) {
  if (threadIdx.x == 0) *p = v;
}

// Depth-presort keys: the float bits of the depth (positive floats order
// like their bit patterns); records that touch no tile sort last.
__global__ void k_depth_keys(const float* depth, const int32_t* tc, int64_t n, uint32_t* key,
                             uint32_t* perm) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  key[i] = tc[i] > 0 ? __float_as_uint(depth[i]) : 0xffffffffu;
  perm[i] = (uint32_t)i;
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
  const int64_t i = (int64_t)blockIdx.x * 256 + t;
  const int64_t last = min(n_rec, (int64_t)blockIdx.x * 256 + 256) - 1;
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
  const int nvalid = (int)(last - (int64_t)blockIdx.x * 256 + 1);
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
template <int BITS>
__device__ __forceinline__ uint64_t match_digit(uint32_t d, bool active) {
  uint64_t m = __ballot(active);
#pragma unroll
  for (int b = 0; b < BITS; ++b) {
    const bool bit = (d >> b) & 1u;
    const uint64_t bb = __ballot(bit);
    m &= bit ? bb : ~bb;
  }
  return m;
}

__device__ __forceinline__ int64_t clamp_n(const int64_t* n_dev, int64_t cap) {
  const int64_t n = n_dev ? *n_dev : cap;
  return n < cap ? n : cap;
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
  const int64_t base = (int64_t)blockIdx.x * kSortTile;
  uint32_t* mine = h[t & (COPIES - 1)];
#pragma unroll 4
  for (int j = 0; j < kSortItems; ++j) {
    const int64_t idx = base + j * 256 + t;
    if (idx < n) atomicAdd(&mine[digit_of<BITS>(keys[idx], shift)], 1u);
  }
  __syncthreads();
  if (t < RADIX) {
    uint32_t c = 0;
#pragma unroll
    for (int k = 0; k < COPIES; ++k) c += h[k][t];
    counts[(int64_t)t * nblocks + blockIdx.x] = c;
  }
}

// Stable scatter of one block: rank the block's keys by digit in LDS (per
// wave, slot by slot, the wave64 ballot match gives the rank among lanes
// with the same digit), then write them out in digit order so each digit's
// run is a contiguous global store.
template <int BITS, typename K>
__global__ __launch_bounds__(256) void k_radix_scatter(const K* __restrict__ kin,
                                                       const uint32_t* __restrict__ vin,
                                                       K* __restrict__ kout,
                                                       uint32_t* __restrict__ vout,
                                                       const int64_t* n_dev, int64_t cap,
                                                       int shift,
                                                       const uint32_t* __restrict__ offsets,
                                                       int nblocks) {
  constexpr int RADIX = 1 << BITS;
  __shared__ uint32_t wcnt[kSortWaves][RADIX];
  __shared__ uint32_t gbase[RADIX];  // global offset of the digit's run minus its block start
  __shared__ uint32_t s_wave[4];
  __shared__ K skey[kSortTile];
  __shared__ uint32_t sval[kSortTile];
  const int t = threadIdx.x, w = t >> 6, lane = t & 63;
  for (int k = t; k < kSortWaves * RADIX; k += 256) (&wcnt[0][0])[k] = 0;
  __syncthreads();
  const int64_t n = clamp_n(n_dev, cap);
  const int64_t bbase = (int64_t)blockIdx.x * kSortTile;
  const int64_t base = bbase + w * (64 * kSortItems);
  const uint64_t lt = lanemask_lt();
  K key[kSortItems];
  uint32_t val[kSortItems];
  uint32_t lofs[kSortItems];
#pragma unroll
  for (int j = 0; j < kSortItems; ++j) {
    const int64_t idx = base + j * 64 + lane;
    const bool ok = idx < n;
    key[j] = ok ? kin[idx] : (K)0;
    val[j] = ok ? vin[idx] : 0u;
    const uint32_t d = digit_of<BITS>(key[j], shift);
    const uint64_t m = match_digit<BITS>(d, ok);
    const uint32_t before = wcnt[w][d];
    lofs[j] = before + (uint32_t)__popcll(m & lt);
    if (ok && (m & lt) == 0) wcnt[w][d] = before + (uint32_t)__popcll(m);
  }
  __syncthreads();
  // digit t: block totals, exclusive block start, per-wave starts
  uint32_t c0 = 0, c1 = 0, c2 = 0, c3 = 0;
  if (t < RADIX) {
    c0 = wcnt[0][t];
    c1 = wcnt[1][t];
    c2 = wcnt[2][t];
    c3 = wcnt[3][t];
  }
  const uint32_t start = block_excl_scan256(c0 + c1 + c2 + c3, s_wave, nullptr);
  if (t < RADIX) {
    gbase[t] = offsets[(int64_t)t * nblocks + blockIdx.x] - start;
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
  const int nvalid = rem <= 0 ? 0 : (rem < kSortTile ? (int)rem : kSortTile);
  for (int k = t; k < nvalid; k += 256) {
    const K kk = skey[k];
    const uint32_t g = gbase[digit_of<BITS>(kk, shift)] + (uint32_t)k;
    kout[g] = kk;
    vout[g] = sval[k];
  }
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
                             uint64_t* partials, hipStream_t st) {
  hipLaunchKernelGGL((k_radix_hist<BITS, K>), dim3(nb), dim3(256), 0, st, k0, n_dev, cap, shift,
                     counts, nb);
  hipError_t e = device_scan(LoadArray{counts}, (int64_t)nb << BITS, counts, partials, nullptr, st);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL((k_radix_scatter<BITS, K>), dim3(nb), dim3(256), 0, st, k0, v0, k1, v1, n_dev,
                     cap, shift, counts, nb);
  return hipGetLastError();
}

// Sorts (keys, vals) of length n_dev (<= cap) on bits [0, bits). The data
// starts in (k0, v0) and ping-pongs with (k1, v1); returns via *k_out/*v_out
// where it ended. grid_n bounds the number of keys (host known).
template <typename K>
static hipError_t radix_sort(K* k0, uint32_t* v0, K* k1, uint32_t* v1, const int64_t* n_dev,
                             int64_t cap, int64_t grid_n, int bits, uint32_t* counts,
                             uint64_t* partials, K** k_out, uint32_t** v_out, hipStream_t st) {
  *k_out = k0;
  *v_out = v0;
  if (grid_n <= 0) return hipSuccess;
  const int nb = (int)((grid_n + kSortTile - 1) / kSortTile);
  const int dbits = radix_digit_bits(bits);
  for (int shift = 0; shift < bits; shift += dbits) {
    hipError_t e = dbits == 7
                       ? radix_pass<7, K>(k0, v0, k1, v1, n_dev, cap, nb, shift, counts, partials, st)
                       : radix_pass<8, K>(k0, v0, k1, v1, n_dev, cap, nb, shift, counts, partials, st);
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

// 64-bit output keys of the presort path: tile << 32 | depth bits.
__global__ void k_make_keys64(const uint32_t* __restrict__ tiles, const uint32_t* __restrict__ vals,
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

struct BinWs {
  uint32_t* okey[2];   // [tiles]  (tile order)
  uint32_t* oval[2];   // [tiles]
  uint32_t* offsets;   // [n_rec]
  uint64_t* partials;  // scan block sums
  uint32_t* counts;    // [256 * nb]
  uint32_t* vals_alt;  // [cap]
  uint32_t* dkey[2];   // [n_rec]   (presort)
  uint32_t* perm[2];   // [n_rec]   (presort)
  uint32_t* tkey[2];   // [cap]     (presort)
  uint64_t* key64[2];  // [cap]     (full)
  size_t bytes;
};

static BinWs bin_ws_layout(int64_t n_rec, int64_t cap, int64_t tiles, int sort_mode, char* base) {
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
  const int64_t scan_n = std::max<int64_t>(256 * nb_max, n_rec);
  const int64_t nparts = (scan_n + kScanTile - 1) / kScanTile + 1;
  L.offsets = (uint32_t*)take(4 * (size_t)std::max<int64_t>(n_rec, 1));
  L.partials = (uint64_t*)take(8 * (size_t)nparts);
  L.counts = (uint32_t*)take(4 * (size_t)(256 * nb_max));
  L.vals_alt = (uint32_t*)take(4 * (size_t)std::max<int64_t>(std::max(cap, n_rec), 1));
  if (sort_mode == XPR_SORT_PRESORT) {
    for (int k = 0; k < 2; ++k) L.dkey[k] = (uint32_t*)take(4 * (size_t)std::max<int64_t>(n_rec, 1));
    for (int k = 0; k < 2; ++k) L.perm[k] = (uint32_t*)take(4 * (size_t)std::max<int64_t>(n_rec, 1));
    for (int k = 0; k < 2; ++k) L.tkey[k] = (uint32_t*)take(4 * (size_t)std::max<int64_t>(cap, 1));
  } else {
    for (int k = 0; k < 2; ++k) L.key64[k] = (uint64_t*)take(8 * (size_t)std::max<int64_t>(cap, 1));
  }
  L.bytes = off;
  return L;
}

size_t bin_workspace_bytes(int64_t n_rec, int64_t cap, int64_t tiles, int sort_mode) {
  return bin_ws_layout(n_rec, cap, tiles, sort_mode, nullptr).bytes;
}

static inline int grid1(int64_t n, int bs = 256) { return (int)((n + bs - 1) / bs); }

// Phase 1: everything up to a known I (the prefix sum of the counts, in
// depth order for the presort path). Phase 2: replication, pair sort, ranges.
hipError_t bin_phase1(const Batch& B, int sort_mode, const float* depth, const int32_t* tc,
                      int64_t n_rec, int64_t cap, int64_t* n_isect, void* ws, hipStream_t st,
                      const uint32_t** perm_out) {
  BinWs L = bin_ws_layout(n_rec, cap, B.total_tiles, sort_mode, (char*)ws);
  *perm_out = nullptr;
  if (n_rec == 0) {
    hipLaunchKernelGGL(k_set_i64, dim3(1), dim3(64), 0, st, n_isect, (int64_t)0);
    return hipGetLastError();
  }
  if (sort_mode == XPR_SORT_PRESORT) {
    hipLaunchKernelGGL(k_depth_keys, dim3(grid1(n_rec)), dim3(256), 0, st, depth, tc, n_rec,
                       L.dkey[0], L.perm[0]);
    uint32_t *ko, *vo;
    hipError_t e = radix_sort<uint32_t>(L.dkey[0], L.perm[0], L.dkey[1], L.perm[1], nullptr, n_rec,
                                        n_rec, 32, L.counts, L.partials, &ko, &vo, st);
    if (e != hipSuccess) return e;
    *perm_out = vo;
    return device_scan(LoadCountPerm{tc, vo}, n_rec, L.offsets, L.partials, n_isect, st);
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
                                      16, L.counts, L.partials, &ko, &vo, st);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_copy_u32, dim3(grid1(T)), dim3(256), 0, st, vo, (const int64_t*)nullptr, T,
                     (uint32_t*)order);
  return hipGetLastError();
}

hipError_t bin_phase2(const Batch& B, int sort_mode, int tile_bits, const float* depth,
                      const int16_t* rect, const int32_t* tc, const uint32_t* perm, int64_t n_rec,
                      int64_t cap, int64_t grid_n, const int64_t* n_isect, uint64_t* keys_out,
                      int32_t* vals, int2* ranges, int32_t* tile_order, void* ws, size_t ws_bytes,
                      hipStream_t st) {
  (void)ws_bytes;
  BinWs L = bin_ws_layout(n_rec, cap, B.total_tiles, sort_mode, (char*)ws);
  hipLaunchKernelGGL(k_fill_u32, dim3(grid1(2 * (int64_t)B.total_tiles)), dim3(256), 0, st,
                     (uint32_t*)ranges, 2 * (int64_t)B.total_tiles, 0u);
  if (n_rec == 0 || grid_n == 0) {
    if (tile_order) return tile_order_lpt(B, L, ranges, tile_order, st);
    return hipGetLastError();
  }
  const short4* rc = reinterpret_cast<const short4*>(rect);
  uint32_t* vals_u = reinterpret_cast<uint32_t*>(vals);
  const int nbd = grid1(n_rec);
  if (sort_mode == XPR_SORT_PRESORT) {
    const int passes = radix_passes(tile_bits);
    // start so that the last pass lands in the caller's vals
    uint32_t* v_start = (passes % 2 == 0) ? vals_u : L.vals_alt;
    uint32_t* v_other = (passes % 2 == 0) ? L.vals_alt : vals_u;
    hipLaunchKernelGGL((k_duplicate<true, false>), dim3(nbd), dim3(256), 0, st, B, rc, tc, depth,
                       perm, L.offsets, n_rec, cap, (void*)L.tkey[0], v_start);
    uint32_t *ko, *vo;
    hipError_t e = radix_sort<uint32_t>(L.tkey[0], v_start, L.tkey[1], v_other, n_isect, cap,
                                        grid_n, tile_bits, L.counts, L.partials, &ko, &vo, st);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_ranges<uint32_t>, dim3(grid1((grid_n + 3) / 4)), dim3(256), 0, st, ko,
                       n_isect, cap, B.total_tiles, ranges);
    if (keys_out)
      hipLaunchKernelGGL(k_make_keys64, dim3(grid1(grid_n)), dim3(256), 0, st, ko, vo, depth,
                         n_isect, cap, keys_out);
    if (vo != vals_u)
      hipLaunchKernelGGL(k_copy_u32, dim3(grid1(grid_n)), dim3(256), 0, st, vo, n_isect, cap,
                         vals_u);
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
                                        grid_n, bits, L.counts, L.partials, &ko, &vo, st);
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
  hipLaunchKernelGGL(k_fill_u32, dim3(grid1(n)), dim3(256), 0, st, (uint32_t*)p, n, 0u);
  return hipGetLastError();
}

}  // namespace xpr
