// pp_sort.hpp -- scans, stable LSD radix passes and compaction for term arrays (gfx950).
//
// A radix pass moves whole terms (all x/z word planes, the coefficient and the order tag)
// by one digit of a key computed on the fly (a group hash, or a word of the canonical key).
// Each 256-thread block owns a 4096-term tile: a histogram kernel writes per-(digit, tile)
// counts, an exclusive scan turns them into global offsets, and the scatter kernel ranks
// the tile stably (wavefront ballots find the lanes that share a digit; per-wave running
// counts keep tile order), stages each plane in LDS in digit order and writes it out in
// runs of consecutive addresses.
#pragma once

#include "pp_common.hpp"

namespace pp {

constexpr int kSortBlock = 256;
constexpr int kSortItems = 16;
constexpr int kSortTile = kSortBlock * kSortItems;  // 4096 terms per block
constexpr int kMaxDigitBits = 10;
constexpr int kMaxBins = 1 << kMaxDigitBits;

__device__ __forceinline__ uint64_t lanemask_lt() {
  const unsigned lane = __lane_id();
  return lane == 0 ? 0ULL : (~0ULL >> (64 - lane));
}

// Exclusive scan of one value per thread over a block of BLOCK threads.  `tmp` holds
// BLOCK/64 entries.  Ends with a barrier, so `tmp` may be reused at once.
template <int BLOCK, class T>
__device__ __forceinline__ T block_exclusive_scan(T v, T* tmp, T* total) {
  const int lane = threadIdx.x & 63;
  const int wid = threadIdx.x >> 6;
  T x = v;
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    T y = __shfl_up(x, d, 64);
    if (lane >= d) x += y;
  }
  if (lane == 63) tmp[wid] = x;
  __syncthreads();
  T wbase = 0, tot = 0;
#pragma unroll
  for (int w = 0; w < BLOCK / 64; ++w) {
    T t = tmp[w];
    if (w < wid) wbase += t;
    tot += t;
  }
  __syncthreads();
  if (total) *total = tot;
  return wbase + x - v;
}

// ---------------------------------------------------------------------------------------
// Exclusive scan of a uint32 array (length < 2^31), tiles of 4096.
// ---------------------------------------------------------------------------------------
__global__ void __launch_bounds__(kSortBlock) k_scan_sums(const uint32_t* in, uint64_t n, uint32_t* sums) {
  __shared__ uint32_t tmp[kSortBlock / 64];
  const uint64_t base = (uint64_t)blockIdx.x * kSortTile;
  uint32_t s = 0;
  for (int k = 0; k < kSortItems; ++k) {
    const uint64_t i = base + (uint64_t)k * kSortBlock + threadIdx.x;
    if (i < n) s += in[i];
  }
  uint32_t tot;
  block_exclusive_scan<kSortBlock>(s, tmp, &tot);
  if (threadIdx.x == 0) sums[blockIdx.x] = tot;
}

__global__ void __launch_bounds__(kSortBlock) k_scan_apply(uint32_t* data, uint64_t n, const uint32_t* sums) {
  __shared__ uint32_t tmp[kSortBlock / 64];
  const uint64_t base = (uint64_t)blockIdx.x * kSortTile + (uint64_t)threadIdx.x * kSortItems;
  uint32_t v[kSortItems];
  uint32_t s = 0;
#pragma unroll
  for (int k = 0; k < kSortItems; ++k) {
    const uint64_t i = base + k;
    v[k] = i < n ? data[i] : 0u;
    s += v[k];
  }
  uint32_t ex = block_exclusive_scan<kSortBlock>(s, tmp, (uint32_t*)nullptr);
  if (sums) ex += sums[blockIdx.x];
#pragma unroll
  for (int k = 0; k < kSortItems; ++k) {
    const uint64_t i = base + k;
    if (i < n) data[i] = ex;
    ex += v[k];
  }
}

// Output-region bases of tiles: out[t] = exclusive prefix of 2 * len[t], and *total = the
// sum of 2 * len.  Blocks of kSortTile entries: k_bases_sums writes each block's sum.  With
// few blocks (raw_sums = 1) each block of k_bases_apply adds up the sums of the blocks
// before it itself, so no scan of the sums runs in between; otherwise the sums have been
// scanned like exclusive_scan_u32 and each block reads its own.
__global__ void __launch_bounds__(kSortBlock) k_bases_sums(const uint32_t* len, uint64_t n, uint32_t* sums) {
  __shared__ uint32_t tmp[kSortBlock / 64];
  const uint64_t base = (uint64_t)blockIdx.x * kSortTile;
  uint32_t s = 0;
  for (int k = 0; k < kSortItems; ++k) {
    const uint64_t i = base + (uint64_t)k * kSortBlock + threadIdx.x;
    if (i < n) s += 2u * len[i];
  }
  uint32_t tot;
  block_exclusive_scan<kSortBlock>(s, tmp, &tot);
  if (threadIdx.x == 0) sums[blockIdx.x] = tot;
}

constexpr uint32_t kBasesRawMax = 1024;   // most blocks whose sums k_bases_apply adds up itself

__global__ void __launch_bounds__(kSortBlock) k_bases_apply(const uint32_t* len, uint64_t n, const uint32_t* sums,
                                                            int raw_sums, uint32_t* out, unsigned long long* total) {
  __shared__ uint32_t tmp[kSortBlock / 64];
  const uint64_t base = (uint64_t)blockIdx.x * kSortTile + (uint64_t)threadIdx.x * kSortItems;
  uint32_t v[kSortItems];
  uint32_t s = 0;
#pragma unroll
  for (int k = 0; k < kSortItems; ++k) {
    const uint64_t i = base + k;
    v[k] = i < n ? 2u * len[i] : 0u;
    s += v[k];
  }
  uint32_t ex = block_exclusive_scan<kSortBlock>(s, tmp, (uint32_t*)nullptr);
  if (sums && raw_sums) {   // uniform: the barriers of the scan below are reached by every thread
    uint32_t p = 0, before = 0;
    for (uint32_t b = threadIdx.x; b < blockIdx.x; b += kSortBlock) p += sums[b];
    block_exclusive_scan<kSortBlock>(p, tmp, &before);
    ex += before;
  } else if (sums) {
    ex += sums[blockIdx.x];
  }
#pragma unroll
  for (int k = 0; k < kSortItems; ++k) {
    const uint64_t i = base + k;
    if (i < n) out[i] = ex;
    if (i == n - 1) *total = (unsigned long long)ex + v[k];
    ex += v[k];
  }
}

// scratch must hold scan_scratch_words(n) uint32 values.
inline uint64_t scan_scratch_words(uint64_t n) {
  uint64_t tot = 0;
  while (n > (uint64_t)kSortTile) {
    n = (n + kSortTile - 1) / kSortTile;
    tot += n + 64;
  }
  return tot + 64;
}

inline void exclusive_scan_u32(uint32_t* data, uint64_t n, uint32_t* scratch, hipStream_t st) {
  if (n == 0) return;
  const uint64_t nb = (n + kSortTile - 1) / kSortTile;
  if (nb == 1) {
    hipLaunchKernelGGL(k_scan_apply, dim3(1), dim3(kSortBlock), 0, st, data, n, (const uint32_t*)nullptr);
    return;
  }
  hipLaunchKernelGGL(k_scan_sums, dim3((unsigned)nb), dim3(kSortBlock), 0, st, data, n, scratch);
  exclusive_scan_u32(scratch, nb, scratch + nb + 64, st);
  hipLaunchKernelGGL(k_scan_apply, dim3((unsigned)nb), dim3(kSortBlock), 0, st, data, n, scratch);
}

// ---------------------------------------------------------------------------------------
// Digit sources.
// ---------------------------------------------------------------------------------------
template <int W>
struct HashDigits {   // bits [shift, shift+bits) of the group hash of (x & mx, z & mz)
  GroupMask gm;
  int shift;
  int bits;
  template <class CT>
  __device__ __forceinline__ uint32_t digit(const Terms<CT>& t, uint64_t i) const {
    uint64_t xs[W], zs[W];
#pragma unroll
    for (int w = 0; w < W; ++w) {
      xs[w] = t.x[w * t.stride + i];
      zs[w] = t.z[w * t.stride + i];
    }
    const uint64_t h = group_hash<W>(xs, zs, gm.mx, gm.mz);
    return (uint32_t)(h >> shift) & ((1u << bits) - 1u);
  }
};

template <int W>
struct WordDigits {   // bits [shift, shift+bits) of one key plane: 0..W-1 x words, W..2W-1 z words, 2W order
  int plane;
  int shift;
  int bits;
  template <class CT>
  __device__ __forceinline__ uint32_t digit(const Terms<CT>& t, uint64_t i) const {
    uint64_t v;
    if (plane < W) v = t.x[plane * t.stride + i];
    else if (plane < 2 * W) v = t.z[(plane - W) * t.stride + i];
    else v = t.o[i];
    return (uint32_t)(v >> shift) & ((1u << bits) - 1u);
  }
};

template <class CT>
__device__ __forceinline__ uint64_t coef_bits(CT v);
template <>
__device__ __forceinline__ uint64_t coef_bits<double>(double v) { return (uint64_t)__double_as_longlong(v); }
template <>
__device__ __forceinline__ uint64_t coef_bits<float>(float v) { return (uint64_t)(uint32_t)__float_as_uint(v); }
template <class CT>
__device__ __forceinline__ CT coef_from_bits(uint64_t b);
template <>
__device__ __forceinline__ double coef_from_bits<double>(uint64_t b) { return __longlong_as_double((long long)b); }
template <>
__device__ __forceinline__ float coef_from_bits<float>(uint64_t b) { return __uint_as_float((uint32_t)b); }

// Plane p of term i as 64 raw bits: 0..W-1 x, W..2W-1 z, 2W coefficient, 2W+1 order.
template <int W, class CT>
__device__ __forceinline__ uint64_t load_plane(const Terms<CT>& t, int p, uint64_t i) {
  if (p < W) return t.x[p * t.stride + i];
  if (p < 2 * W) return t.z[(p - W) * t.stride + i];
  if (p == 2 * W) return coef_bits<CT>(t.c[i]);
  return t.o[i];
}
template <int W, class CT>
__device__ __forceinline__ void store_plane(const Terms<CT>& t, int p, uint64_t i, uint64_t v) {
  if (p < W) t.x[p * t.stride + i] = v;
  else if (p < 2 * W) t.z[(p - W) * t.stride + i] = v;
  else if (p == 2 * W) t.c[i] = coef_from_bits<CT>(v);
  else t.o[i] = (uint8_t)v;
}

// ---------------------------------------------------------------------------------------
// Radix pass: histogram.  counts is digit-major: counts[d * nblocks + block].
// ---------------------------------------------------------------------------------------
template <int W, class CT, class DS>
__global__ void __launch_bounds__(kSortBlock) k_radix_hist(Terms<CT> in, uint64_t n, DS ds, int bins,
                                                           uint32_t* counts, uint32_t nblocks) {
  __shared__ uint32_t h[kMaxBins];
  for (int b = threadIdx.x; b < bins; b += kSortBlock) h[b] = 0;
  __syncthreads();
  const uint64_t base = (uint64_t)blockIdx.x * kSortTile;
  for (int k = 0; k < kSortItems; ++k) {
    const uint64_t i = base + (uint64_t)k * kSortBlock + threadIdx.x;
    if (i < n) atomicAdd(&h[ds.digit(in, i)], 1u);
  }
  __syncthreads();
  for (int b = threadIdx.x; b < bins; b += kSortBlock) counts[(uint64_t)b * nblocks + blockIdx.x] = h[b];
}

// ---------------------------------------------------------------------------------------
// Radix pass: stable scatter.  offs = exclusive scan of counts (same layout).
// ---------------------------------------------------------------------------------------
template <int W, class CT, bool ORD, class DS>
__global__ void __launch_bounds__(kSortBlock) k_radix_scatter(Terms<CT> in, Terms<CT> out, uint64_t n, DS ds,
                                                              int bits, const uint32_t* offs, uint32_t nblocks) {
  constexpr int NW = kSortBlock / 64;
  __shared__ uint32_t wcnt[NW][kMaxBins];
  __shared__ uint32_t goff[kMaxBins];
  __shared__ uint32_t lstart[kMaxBins];
  __shared__ uint16_t sdig[kSortTile];
  __shared__ uint64_t stage[kSortTile];
  __shared__ uint32_t stmp[NW];
  const int bins = 1 << bits;
  const int lane = threadIdx.x & 63;
  const int wid = threadIdx.x >> 6;
  for (int j = threadIdx.x; j < NW * kMaxBins; j += kSortBlock) (&wcnt[0][0])[j] = 0;
  __syncthreads();
  const uint64_t base = (uint64_t)blockIdx.x * kSortTile;
  const uint64_t lt = lanemask_lt();
  uint32_t rank[kSortItems];
  uint16_t dig[kSortItems];
#pragma unroll
  for (int k = 0; k < kSortItems; ++k) {
    const uint64_t i = base + (uint64_t)wid * (kSortItems * 64) + (uint64_t)k * 64 + lane;
    const bool valid = i < n;
    const uint32_t d = valid ? ds.digit(in, i) : 0u;
    uint64_t peers = __ballot(valid);
    for (int b = 0; b < bits; ++b) {
      const bool bit = (d >> b) & 1u;
      const uint64_t bal = __ballot(bit);
      peers &= bit ? bal : ~bal;
    }
    uint32_t r = 0;
    if (valid) {
      const uint32_t before = wcnt[wid][d];
      r = before + (uint32_t)__popcll(peers & lt);
      if ((peers & lt) == 0) wcnt[wid][d] = before + (uint32_t)__popcll(peers);
    }
    __builtin_amdgcn_wave_barrier();
    rank[k] = r;
    dig[k] = (uint16_t)d;
  }
  __syncthreads();
  // Scan over (digit, wave) in digit-major order.
  constexpr int BPT = kMaxBins / kSortBlock;
  uint32_t tsum = 0;
#pragma unroll
  for (int j = 0; j < BPT; ++j) {
    const int b = threadIdx.x * BPT + j;
    if (b < bins)
      for (int w = 0; w < NW; ++w) tsum += wcnt[w][b];
  }
  uint32_t run = block_exclusive_scan<kSortBlock>(tsum, stmp, (uint32_t*)nullptr);
#pragma unroll
  for (int j = 0; j < BPT; ++j) {
    const int b = threadIdx.x * BPT + j;
    if (b < bins) {
      lstart[b] = run;
      for (int w = 0; w < NW; ++w) {
        const uint32_t c = wcnt[w][b];
        wcnt[w][b] = run;
        run += c;
      }
      goff[b] = offs[(uint64_t)b * nblocks + blockIdx.x];
    }
  }
  __syncthreads();
  uint32_t lpos[kSortItems];
#pragma unroll
  for (int k = 0; k < kSortItems; ++k) {
    const uint64_t i = base + (uint64_t)wid * (kSortItems * 64) + (uint64_t)k * 64 + lane;
    lpos[k] = 0xffffffffu;
    if (i < n) {
      lpos[k] = wcnt[wid][dig[k]] + rank[k];
      sdig[lpos[k]] = dig[k];
    }
  }
  __syncthreads();
  const uint32_t tile_n = (uint32_t)((n - base) < (uint64_t)kSortTile ? (n - base) : (uint64_t)kSortTile);
  constexpr int NPLANES = 2 * W + 1 + (ORD ? 1 : 0);
  for (int p = 0; p < NPLANES; ++p) {
#pragma unroll
    for (int k = 0; k < kSortItems; ++k) {
      const uint64_t i = base + (uint64_t)wid * (kSortItems * 64) + (uint64_t)k * 64 + lane;
      if (lpos[k] != 0xffffffffu) stage[lpos[k]] = load_plane<W, CT>(in, p, i);
    }
    __syncthreads();
    for (uint32_t j = threadIdx.x; j < tile_n; j += kSortBlock) {
      const uint32_t d = sdig[j];
      const uint64_t g = (uint64_t)goff[d] + (j - lstart[d]);
      if (g < n) store_plane<W, CT>(out, p, g, stage[j]);
    }
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------------------
// Stream compaction of whole terms by a keep flag (flags -> exclusive positions in place).
// ---------------------------------------------------------------------------------------
template <int W, class CT, bool ORD>
__global__ void k_compact_scatter(Terms<CT> in, Terms<CT> out, uint64_t n, const uint8_t* keep,
                                  const uint32_t* pos) {
  const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n || !keep[i]) return;
  const uint64_t j = pos[i];
  if (j >= out.stride) return;
#pragma unroll
  for (int w = 0; w < W; ++w) {
    out.x[w * out.stride + j] = in.x[w * in.stride + i];
    out.z[w * out.stride + j] = in.z[w * in.stride + i];
  }
  out.c[j] = in.c[i];
  if (ORD) out.o[j] = in.o[i];
}

__global__ void k_flags_to_u32(const uint8_t* f, uint32_t* v, uint64_t n) {
  const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) v[i] = f[i];
}

}  // namespace pp
