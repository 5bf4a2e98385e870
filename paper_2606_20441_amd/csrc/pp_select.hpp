// Device-side cut of the cap between the gates of a run (Section I.A's truncation to the
// K largest terms after every non-Clifford gate).  The cut is the K-th term of the order
// |c| descending, then canonical key ascending (x words from the most significant down,
// then z words, then the order tag); a term survives iff it does not come after it.
//
// The selection reads a tiled buffer's live slots only, and the host waits for none of it.
// It is a fixed chain of launches; each reads the state the previous ones left in SelState
// and returns at once when it has nothing to do:
//  * k_sel_win: reads the live count the gate pass left on the device (nothing more to do
//    when the sum is within the cap), then a histogram of the |c| keys over a window of 2048
//    bins around the previous cut (before the first cut: one bin per octave, every key);
//  * k_sel_pick (one workgroup): the bin holding the K-th term, or, when the window missed
//    it, the passes start from the top bits;
//  * twice k_sel_pass, each followed by a pick of its bin: 15 more bits of |c|, while the
//    bucket of the K-th term holds more than a few thousand terms;
//  * k_sel_rest (one workgroup): the pick after the second pass, then whatever is left, in
//    the rare case it is not done: more bits of |c|, then the canonical key words, which
//    split a bucket of exactly equal |c|;
//  * k_sel_gather: the bucket's terms;
//  * k_sel_rank (one workgroup): sorts them in LDS in the cut order and writes the K-th as
//    the pending cut, which the next gate pass reads from device memory.
#pragma once

#include "pp_common.hpp"
#include "pp_gate.hpp"
#include "pp_misc.hpp"

namespace pp {

// Window bins start at 2^shift keys and narrow by one bit after each cut whose window bucket
// was still too large to gather, down to 2^min_shift.  A window that misses the cut widens by
// two bits; if that miss also left the two passes short, so that the one-workgroup sweeps had
// to finish the job (FP64 keys of a large sum), the wider window becomes the new floor: such
// a miss costs far more than the passes a narrow window saves.
constexpr int kSelMinShift = 4;

// Candidates ranked in LDS: (8 + 16 W + 1) bytes each.
template <int W>
constexpr uint32_t sel_gather() { return W == 1 ? 4096u : (W == 2 ? 2048u : 1024u); }

// Words of the composite key: 0 = |c| key (larger first), 1..W = x words W-1..0, W+1..2W =
// z words W-1..0, 2W+1 = order tag (smaller first for all but word 0).
constexpr int kSelWords = 2 * PP_MAXW + 2;
constexpr int kSelBits = 15;                 // bits per pass after the window (128 KiB of LDS)
constexpr int kSelBins = 1 << kSelBits;

struct SelState {
  // kept from one cut to the next
  unsigned long long hint_key;   // |c| key of the last cut
  int hint_valid;
  int hint_shift;                // window bins of 2^hint_shift keys
  int min_shift;                 // the narrowest bins the window may take
  int missed;                    // the window of the current cut missed it
  // one cut
  unsigned long long K;          // the cap
  int active;                    // 1: the sum exceeds the cap and a cut is being selected
  int word, hi;                  // word being narrowed; its bits at and above `hi` are fixed
  int done;                      // the bucket is small enough to gather
  unsigned int count_eq;         // terms in the bucket
  unsigned int gcount;           // candidates gathered
  unsigned long long need;       // rank (1-based) of the boundary inside the bucket
  unsigned long long px[kSelWords], pm[kSelWords];   // fixed bits of each word
  // statistics, read by the host after a run
  unsigned long long n_capped, n_cuts, n_passes, n_misses, n_rest, n_errors;
  CutDev cut;                    // the pending cut (has = 0: none)
  unsigned int hist[kSelBins];   // global histogram, all zero between passes
};

// Value of composite word w of slot i (key: its |c| key).
template <int W, class CT, bool ORD>
__device__ __forceinline__ uint64_t sel_word(const Terms<CT>& t, uint64_t i, uint64_t key, int w) {
  if (w == 0) return key;
  if (w <= W) return t.x[(uint64_t)(W - w) * t.stride + i];
  if (w <= 2 * W) return t.z[(uint64_t)(2 * W - w) * t.stride + i];
  return ORD ? (uint64_t)t.o[i] : 0ULL;
}

// Slot i lies in the current bucket: words before `word` equal their fixed values, and
// `word` matches its fixed bits.
template <int W, class CT, bool ORD>
__device__ __forceinline__ bool sel_in_bucket(const Terms<CT>& t, uint64_t i, uint64_t key, int word,
                                              const SelState* ss) {
  if ((key & ss->pm[0]) != ss->px[0]) return false;
  for (int w = 1; w <= word; ++w)
    if ((sel_word<W, CT, ORD>(t, i, key, w) & ss->pm[w]) != ss->px[w]) return false;
  return true;
}

// One 256-thread workgroup: the bin of `counts` (bins entries in LDS, in bin order) holding
// the need-th term, counting from the top bin when `descending`, else from bin 0; `need`
// becomes the rank inside that bin and `count` its size.  Returns -1 when the bins hold
// fewer than `need` terms.  lsum: 256 words of LDS scratch.
__device__ __forceinline__ int sel_pick_bin(const unsigned int* counts, int bins, bool descending,
                                            unsigned long long& need, unsigned int& count,
                                            unsigned long long* lsum) {
  const int tid = threadIdx.x;
  const int per = (bins + 255) / 256;
  auto at = [&](int b) { return counts[descending ? bins - 1 - b : b]; };   // b-th bin in rank order
  unsigned long long s = 0;
  for (int b = tid * per; b < min(bins, (tid + 1) * per); ++b) s += at(b);
  lsum[tid] = s;
  __syncthreads();
  for (int d = 1; d < 256; d <<= 1) {
    const unsigned long long v = tid >= d ? lsum[tid - d] : 0ULL;
    __syncthreads();
    lsum[tid] += v;
    __syncthreads();
  }
  __shared__ int s_bin;
  __shared__ unsigned long long s_before;
  if (tid == 0) s_bin = -1;
  __syncthreads();
  const unsigned long long before = tid > 0 ? lsum[tid - 1] : 0ULL;
  if (before < need && lsum[tid] >= need) {
    unsigned long long c = before;
    for (int b = tid * per; b < min(bins, (tid + 1) * per); ++b) {
      if (c + at(b) >= need) {
        s_bin = b;
        s_before = c;
        break;
      }
      c += at(b);
    }
  }
  __syncthreads();
  const int r = s_bin;
  const unsigned long long sb = s_before;
  __syncthreads();
  if (r < 0) return -1;
  need -= sb;
  count = at(r);
  return descending ? bins - 1 - r : r;
}

// State after the bits of a pass are fixed at bin d (bits at [shift, shift + bits)); a word
// whose bits are all fixed hands over to the next one.
template <int W, bool ORD>
__device__ __forceinline__ void sel_fix(SelState* ss, int word, int shift, int bits, int d, unsigned long long need,
                                        unsigned int count) {
  constexpr uint32_t G = sel_gather<W>();
  ss->need = need;
  ss->count_eq = count;
  ss->px[word] |= (unsigned long long)d << shift;
  ss->pm[word] |= (unsigned long long)((1 << bits) - 1) << shift;
  ss->n_passes += 1;
  if (shift > 0) {
    ss->hi = shift;
  } else if (word + 1 < 2 * W + 1 + (ORD ? 1 : 0)) {
    ss->word = word + 1;
    ss->hi = (word + 1 == 2 * W + 1) ? 8 : 64;
    ss->px[word + 1] = 0;
    ss->pm[word + 1] = 0;
  } else {
    ss->word = word + 1;   // every word fixed: the bucket is one term
    ss->hi = 0;
  }
  ss->done = count <= G;
}

// The window of the first histogram: 2048 bins of 2^sh keys from lo, around the previous cut
// (returns true), or, before the first cut, over every key (bins of one octave of |c|).
template <class CT>
__device__ __forceinline__ bool sel_window(const SelState* ss, int& sh, unsigned long long& lo) {
  constexpr int KB = sizeof(CT) == 8 ? 63 : 31;
  if (!ss->hint_valid) {
    sh = KB - 11;
    lo = 0ULL;
    return false;
  }
  sh = ss->hint_shift;
  const unsigned long long hk = ss->hint_key, half = 1024ULL << sh;
  lo = hk > half ? ((hk - half) >> sh) << sh : 0ULL;
  return true;
}

// The pick after the window histogram (stage 0) or after a pass (stage 1), by one
// workgroup.  lh: LDS for the bins (2049 at stage 0, kSelBins at stage 1).
__device__ __forceinline__ unsigned int sel_hist_at(const SelState* ss, int b) { return ss->hist[b]; }

template <int W, class CT, bool ORD>
__device__ void sel_pick(SelState* ss, int stage, unsigned long long K, unsigned int* lh, unsigned long long* lsum) {
  constexpr int KB = sizeof(CT) == 8 ? 63 : 31;
  constexpr uint32_t G = sel_gather<W>();
  const int tid = threadIdx.x;
  if (stage == 0) {
    bool hit = false;
    {
      int sh;
      unsigned long long lo;
      const bool hinted = sel_window<CT>(ss, sh, lo);
      for (int b = tid; b < 2049; b += 256) lh[b] = sel_hist_at(ss, b);
      __syncthreads();
      unsigned long long need = K;
      unsigned int count = 0;
      // rank order: the overflow bin (keys above the window) first, then the bins from the top
      const int r = sel_pick_bin(lh, 2049, true, need, count, lsum);
      hit = r >= 0 && r < 2048;
      if (tid == 0) {
        if (hit) {
          ss->need = need;
          ss->count_eq = count;
          ss->word = 0;
          ss->px[0] = lo + ((unsigned long long)r << sh);
          ss->pm[0] = ~0ULL << sh;
          ss->hi = sh;
          ss->done = count <= G;
          if (hinted && count > G && ss->hint_shift > ss->min_shift) ss->hint_shift -= 1;   // finer bins next time
        } else {
          ss->n_misses += 1;
          ss->missed = 1;
          ss->hint_shift = min(ss->hint_shift + 2, KB - kSelBits);   // a wider window next time
        }
      }
      for (int b = tid; b < 2049; b += 256) ss->hist[b] = 0;
    }
    if (!hit && tid == 0) {
      // the passes start from the top bits of |c|
      ss->need = K;
      ss->word = 0;
      ss->px[0] = 0;
      ss->pm[0] = 0;
      ss->hi = KB;
      ss->done = 0;
    }
    return;
  }
  // after a pass over the next bits of word 0
  if (ss->active != 1 || ss->done || ss->word != 0) return;
  const int hi = ss->hi, bits = min(kSelBits, hi), shift = hi - bits, bins = 1 << bits;
  for (int b = tid; b < bins; b += 256) lh[b] = sel_hist_at(ss, b);
  __syncthreads();
  unsigned long long need = ss->need;
  unsigned int count = 0;
  int d = sel_pick_bin(lh, bins, true, need, count, lsum);
  if (tid == 0) {
    if (d < 0) {
      ss->n_errors += 1;   // the bucket lost terms: nothing sensible to fix
      ss->active = -1;
    } else {
      sel_fix<W, ORD>(ss, 0, shift, bits, d, need, count);
    }
  }
  for (int b = tid; b < bins; b += 256) ss->hist[b] = 0;
}

// Live count, and the window histogram around the previous cut.
template <int W, class CT, bool ORD>
__global__ void __launch_bounds__(256) k_sel_win(const CT* c, TileView tv, const unsigned long long* live2,
                                                 unsigned long long K, SelState* ss) {
  __shared__ uint32_t h[2049];
  const unsigned long long n_live = *live2 / 2;   // the pass's output extent is twice its live terms
  if (n_live <= K) {
    if (blockIdx.x == 0 && threadIdx.x == 0) {
      ss->active = 0;
      ss->cut.has = 0;
    }
    return;
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    ss->active = 1;
    ss->missed = 0;
    ss->K = K;
    ss->gcount = 0;
    ss->n_capped += n_live - K;
    ss->n_cuts += 1;
  }
  int sh;
  unsigned long long lo;
  sel_window<CT>(ss, sh, lo);
  for (int b = threadIdx.x; b < 2049; b += 256) h[b] = 0;
  __syncthreads();
  uint32_t above = 0;   // most keys lie above a window near the cut: counted in a register
  tile_visit<CT>(c, tv, [&](uint64_t, uint64_t k) {
    if (k >= lo) {
      const uint64_t d = (k - lo) >> sh;
      if (d >= 2048) ++above;
      else atomicAdd(&h[d], 1u);
    }
  });
  for (int d = 32; d >= 1; d >>= 1) above += __shfl_xor(above, d, 64);
  if ((threadIdx.x & 63) == 0 && above) atomicAdd(&h[2048], above);
  __syncthreads();
  for (int b = threadIdx.x; b < 2049; b += 256)
    if (h[b]) atomicAdd(&ss->hist[b], h[b]);
}

// The next kSelBits bits of |c| inside the bucket, while the bucket is large.
template <int W, class CT, bool ORD>
__global__ void __launch_bounds__(256) k_sel_pass(const CT* c, TileView tv, SelState* ss) {
  __shared__ unsigned int h[kSelBins];
  if (ss->active != 1 || ss->done || ss->word != 0) return;
  const int hi = ss->hi, bits = min(kSelBits, hi), shift = hi - bits, bins = 1 << bits;
  const unsigned long long px = ss->px[0], pm = ss->pm[0];
  for (int b = threadIdx.x; b < bins; b += 256) h[b] = 0;
  __syncthreads();
  tile_visit<CT>(c, tv, [&](uint64_t, uint64_t k) {
    if ((k & pm) == px) atomicAdd(&h[(k >> shift) & (uint64_t)(bins - 1)], 1u);
  });
  __syncthreads();
  for (int b = threadIdx.x; b < bins; b += 256)
    if (h[b]) atomicAdd(&ss->hist[b], h[b]);
}

// One 256-thread workgroup after k_sel_win (stage 0) or after a k_sel_pass (stage 1).  (A
// pick run by the last workgroup of the sweep itself needs a device-scope fence in every
// workgroup, which writes back the L2 each time: four times slower than this launch.)
template <int W, class CT, bool ORD>
__global__ void __launch_bounds__(256) k_sel_pick(SelState* ss, int stage) {
  __shared__ unsigned int lh[kSelBins];
  __shared__ unsigned long long lsum[256];
  if (stage == 0) {
    if (ss->active != 1) return;
    sel_pick<W, CT, ORD>(ss, 0, ss->K, lh, lsum);
  } else {
    sel_pick<W, CT, ORD>(ss, 1, 0ULL, lh, lsum);
  }
}

// One 256-thread workgroup: the pick after the last pass, then whatever that leaves undone
// (a bucket of exactly equal |c|, split by the strings, or low bits of |c| after a window
// that missed): each further pass is a sweep of all tiles by this one workgroup.
template <int W, class CT, bool ORD>
__global__ void __launch_bounds__(256) k_sel_rest(Terms<CT> t, TileView tv, SelState* ss) {
  constexpr int NWORDS = 2 * W + 1 + (ORD ? 1 : 0);
  __shared__ unsigned int lh[kSelBins];
  __shared__ unsigned long long lsum[256];
  sel_pick<W, CT, ORD>(ss, 1, 0ULL, lh, lsum);
  __syncthreads();   // the pick's state, written by thread 0, is read by every thread below
  if (ss->active != 1 || ss->done) return;
  if (threadIdx.x == 0) {
    ss->n_rest += 1;
    if (ss->missed) ss->min_shift = max(ss->min_shift, ss->hint_shift);   // never that narrow again
  }
  for (;;) {
    __syncthreads();
    const int word = ss->word;
    if (ss->done || word >= NWORDS) break;
    const int hi = ss->hi, bits = min(kSelBits, hi), shift = hi - bits, bins = 1 << bits;
    for (int b = threadIdx.x; b < bins; b += 256) lh[b] = 0;
    __syncthreads();
    tile_visit<CT>(t.c, tv, [&](uint64_t i, uint64_t k) {
      if (!sel_in_bucket<W, CT, ORD>(t, i, k, word, ss)) return;
      atomicAdd(&lh[(sel_word<W, CT, ORD>(t, i, k, word) >> shift) & (uint64_t)(bins - 1)], 1u);
    });
    __syncthreads();
    unsigned long long need = ss->need;
    unsigned int count = 0;
    const int d = sel_pick_bin(lh, bins, word == 0, need, count, lsum);
    if (threadIdx.x == 0) {
      if (d < 0) {
        ss->n_errors += 1;
        ss->active = -1;
      } else {
        sel_fix<W, ORD>(ss, word, shift, bits, d, need, count);
      }
    }
    __syncthreads();
    if (ss->active != 1) break;
  }
}

// The bucket's terms (at most sel_gather<W>()).
template <int W, class CT, bool ORD>
__global__ void __launch_bounds__(256) k_sel_gather(Terms<CT> t, TileView tv, SelState* ss, Terms<CT> gb) {
  constexpr int NWORDS = 2 * W + 1 + (ORD ? 1 : 0);
  constexpr uint32_t G = sel_gather<W>();
  if (ss->active != 1) return;
  const int word = min(ss->word, NWORDS - 1);
  const unsigned long long px0 = ss->px[0], pm0 = ss->pm[0];
  tile_visit<CT>(t.c, tv, [&](uint64_t i, uint64_t k) {
    if ((k & pm0) != px0) return;
    if (word > 0 && !sel_in_bucket<W, CT, ORD>(t, i, k, word, ss)) return;
    const unsigned int j = atomicAdd(&ss->gcount, 1u);
    if (j >= G) return;
#pragma unroll
    for (int w = 0; w < W; ++w) {
      gb.x[(uint64_t)w * gb.stride + j] = t.x[(uint64_t)w * t.stride + i];
      gb.z[(uint64_t)w * gb.stride + j] = t.z[(uint64_t)w * t.stride + i];
    }
    gb.c[j] = t.c[i];
    if (ORD) gb.o[j] = t.o[i];
  });
}

// One 256-thread workgroup: the need-th of the gathered candidates in the cut order, written
// as the pending cut.  A radix select over the |c| bits the bucket has not fixed yet
// (11 bits a step, stopping once one candidate is left); candidates of exactly equal |c|
// are then ranked by their canonical keys.
template <int W, class CT, bool ORD>
__global__ void __launch_bounds__(256) k_sel_rank(SelState* ss, Terms<CT> gb) {
  constexpr uint32_t G = sel_gather<W>();
  constexpr int KB = sizeof(CT) == 8 ? 63 : 31;
  __shared__ uint64_t key[G];
  __shared__ unsigned int hist[2048];
  __shared__ unsigned long long lsum[256];
  __shared__ uint16_t ties[G];
  __shared__ unsigned int s_nt;
  __shared__ int s_pick;
  if (ss->active != 1) return;
  const uint32_t n = min(ss->gcount, G);
  unsigned long long need = ss->need;
  const int tid = threadIdx.x;
  if (n == 0 || need < 1 || need > n || ss->gcount != ss->count_eq) {
    // the selection lost its boundary: no cut, flagged for the host
    if (tid == 0) {
      ss->cut.has = 0;
      ss->active = -1;
      ss->n_errors += 1;
    }
    return;
  }
  for (uint32_t i = tid; i < n; i += 256) key[i] = abs_key<CT>(gb.c[i]);
  // bits of |c| still open: below `hi` while word 0 is being narrowed, none once it is fixed
  int hi = ss->word == 0 ? ss->hi : 0;
  if (hi > KB) hi = KB;
  uint64_t pfx = 0, pmask = 0;
  unsigned int count = n;
  __syncthreads();
  while (hi > 0 && count > 1) {
    const int bits = min(11, hi), shift = hi - bits, bins = 1 << bits;
    for (int b = tid; b < bins; b += 256) hist[b] = 0;
    __syncthreads();
    for (uint32_t i = tid; i < n; i += 256)
      if ((key[i] & pmask) == pfx) atomicAdd(&hist[(key[i] >> shift) & (uint64_t)(bins - 1)], 1u);
    __syncthreads();
    const int d = sel_pick_bin(hist, bins, true, need, count, lsum);
    pfx |= (uint64_t)(d < 0 ? 0 : d) << shift;
    pmask |= (uint64_t)(bins - 1) << shift;
    hi = shift;
    __syncthreads();
  }
  // the candidates left: one, or several of exactly equal |c| ranked by their strings
  if (tid == 0) {
    s_nt = 0;
    s_pick = -1;
  }
  __syncthreads();
  for (uint32_t i = tid; i < n; i += 256)
    if ((key[i] & pmask) == pfx) ties[atomicAdd(&s_nt, 1u)] = (uint16_t)i;
  __syncthreads();
  const uint32_t nt = s_nt;
  auto canon_less = [&](uint32_t a, uint32_t b) -> bool {
#pragma unroll
    for (int w = W - 1; w >= 0; --w) {
      const uint64_t xa = gb.x[(uint64_t)w * gb.stride + a], xb = gb.x[(uint64_t)w * gb.stride + b];
      if (xa != xb) return xa < xb;
    }
#pragma unroll
    for (int w = W - 1; w >= 0; --w) {
      const uint64_t za = gb.z[(uint64_t)w * gb.stride + a], zb = gb.z[(uint64_t)w * gb.stride + b];
      if (za != zb) return za < zb;
    }
    return ORD ? gb.o[a] < gb.o[b] : false;
  };
  if (nt == 1) {
    if (tid == 0) s_pick = ties[0];
  } else {
    for (uint32_t u = tid; u < nt; u += 256) {
      const uint32_t a = ties[u];
      unsigned long long r = 0;
      for (uint32_t v = 0; v < nt; ++v)
        if (v != u && canon_less(ties[v], a)) ++r;
      if (r == need - 1) s_pick = (int)a;
    }
  }
  __syncthreads();
  if (tid == 0) {
    const int bi = s_pick;
    if (bi < 0) {
      ss->cut.has = 0;
      ss->active = -1;
      ss->n_errors += 1;
      return;
    }
    CutDev c{};
    c.has = 1;
    c.val = key[bi];
    for (int w = 0; w < W; ++w) {
      c.x[w] = gb.x[(uint64_t)w * gb.stride + bi];
      c.z[w] = gb.z[(uint64_t)w * gb.stride + bi];
    }
    c.o = ORD ? gb.o[bi] : 0u;
    ss->cut = c;
    ss->hint_key = c.val;
    ss->hint_valid = 1;
  }
}

// A fresh state: no cut pending, no window yet (bins of 2^shift keys once there is one).
__global__ void k_sel_init(SelState* ss, int shift) {
  if (threadIdx.x == 0) {
    ss->hint_valid = 0;
    ss->hint_key = 0;
    ss->hint_shift = shift;
    ss->min_shift = kSelMinShift;
    ss->missed = 0;
    ss->active = 0;
    ss->cut.has = 0;
  }
  for (int b = threadIdx.x; b < kSelBins; b += blockDim.x) ss->hist[b] = 0;
}

// Statistics read by the host: start again from zero.
__global__ void k_sel_reset_stats(SelState* ss) {
  if (threadIdx.x == 0) ss->n_capped = ss->n_cuts = ss->n_passes = ss->n_misses = ss->n_rest = ss->n_errors = 0;
}

// No cut pending (after a Clifford gate, which the cap does not follow).
__global__ void k_sel_clear(SelState* ss) {
  if (threadIdx.x == 0) {
    ss->active = 0;
    ss->cut.has = 0;
  }
}

}  // namespace pp
