// pp_gate.hpp -- one rotation over persistent tiles, with the truncation of the previous
// gate applied on load (gfx950).
//
// When the cap (keep the largest K_O terms, Section I.A) binds after every non-Clifford
// gate, each gate needs a device-wide selection before the next one can start.  The
// terms are grouped once per run of gates by a hash of the bits no gate of the run changes,
// and cut into tiles of whole groups.  Every gate is then one pass over the same tiles:
// a workgroup loads its tile, drops the terms below the previous gate's cut, pairs each
// anticommuting string with its partner through an LDS hash table, applies the cos/sin
// branching (Section I, Eq. evolve_gate, and the Euclid appendix's backward rule), drops
// |c| < eps, and writes its survivors back as one contiguous range, which is the same
// tile at the next gate.  A per-term 32-bit hash (GF(2)-linear in the string, so a
// partner's hash is one XOR away) travels with the terms.
#pragma once

#include "pp_common.hpp"
#include "pp_layer.hpp"
#include "pp_misc.hpp"

namespace pp {

constexpr int kDropSlots = 64;   // spread accumulators: one address per workgroup is a serial queue

// The cut of a cap: the boundary term (the K-th in the order |c| descending, then canonical
// key ascending) and the rule "kept iff it does not come after the boundary".  Canonical
// key order: x words from the most significant word down, then z words, then the order tag.
struct CutDev {
  int has;
  uint32_t o;
  uint64_t val;               // |c| bits of the boundary term
  uint64_t x[PP_MAXW], z[PP_MAXW];
};

template <int W>
__device__ __forceinline__ bool canon_le(const uint64_t* kx, const uint64_t* kz, uint32_t ko, const CutDev& b) {
#pragma unroll
  for (int w = W - 1; w >= 0; --w)
    if (kx[w] != b.x[w]) return kx[w] < b.x[w];
#pragma unroll
  for (int w = W - 1; w >= 0; --w)
    if (kz[w] != b.z[w]) return kz[w] < b.z[w];
  return ko <= b.o;
}

// Survives the cut (exact zeros never do).
template <int W, class CT>
__device__ __forceinline__ bool cut_keeps(CT v, const uint64_t* kx, const uint64_t* kz, uint32_t ko,
                                          const CutDev& cut) {
  if (v == (CT)0) return false;
  if (!cut.has) return true;
  const uint64_t k = abs_key<CT>(v);
  if (k != cut.val) return k > cut.val;
  return canon_le<W>(kx, kz, ko, cut);
}

template <class CT>
struct Gate1Args {
  Terms<CT> in;
  Terms<CT> out;
  uint32_t* hscr;               // per-slot hash scratch of `out` (the oversize kernel only)
  const uint32_t* t_start;      // tile ranges in `in`
  const uint32_t* t_len;
  const uint32_t* t_list;       // optional: list entry -> tile
  uint32_t t_count;             // list entries (tiles) to process
  const uint32_t* t_count_dev;  // if set: the count, read on the device (t_count bounds it)
  const uint32_t* o_base;       // start of each tile's output region (2 * t_len slots)
  uint32_t* o_start;            // tile ranges in `out` (same tile index)
  uint32_t* o_len;
  int zero_on_ovf;              // a tile that does not fit zeroes its region (nobody retries it here)
  GateDev g;
  double eps;                   // threshold after the gate (0: none)
  CutDev cut;                   // the previous gate's cap, applied on load
  const CutDev* cutp;           // if set, that cut is read from here on the device instead
  // Sine order (sine_on, non-Clifford gates only): the tag counts sines.  The cos part of
  // (P, t) keeps its tag, the sin part goes to (RP, t + 1) and is dropped above sine_max.
  int sine_on;
  int sine_max;
  double* cscr;                 // per-slot coefficient scratch of `out` (the oversize kernel, sine order)
  uint32_t* ovf_tiles;          // tiles that did not fit in LDS
  uint32_t* ovf_count;
  double* dropped;              // [kDropSlots]: sum of |c| removed (cut and threshold)
  unsigned long long* io;       // [2][kDropSlots]: terms loaded / written by completed tiles
};

// The pending cut of a gate pass: from device memory (written there by the device-side
// selection of the previous gate) or from the launch arguments.
template <class CT>
__device__ __forceinline__ CutDev gate_cut(const Gate1Args<CT>& a) {
  if (!a.cutp) return a.cut;
  return *a.cutp;
}

// A tile handed to another path: its output range is left empty (length 0).
template <class CT>
__device__ void zero_region(const Gate1Args<CT>& a, uint32_t tile, uint32_t n0) {
  (void)n0;
  if (threadIdx.x == 0) {
    a.o_start[tile] = (uint32_t)a.o_base[tile];
    a.o_len[tile] = 0;
  }
}

// A tile copied through with only the pending cut applied (order kept).
template <int W, class CT, bool ORD, int BLOCK>
__device__ void pass_through(const Gate1Args<CT>& a, const CutDev& cut, uint32_t tile, uint32_t t0, uint32_t n0) {
  constexpr int NW = BLOCK / 64;
  __shared__ uint32_t p_wsum[NW];
  __shared__ double p_drop[NW];
  const int tid = threadIdx.x, lane = tid & 63;
  auto keep = [&](uint64_t src) {
    const CT v = a.in.c[src];
    if (v == (CT)0) return false;
    if (fabs((double)v) < a.eps) return false;   // the threshold after a non-Clifford gate
    if (!cut.has) return true;
    uint64_t kx[W], kz[W];
#pragma unroll
    for (int w = 0; w < W; ++w) { kx[w] = a.in.x[w * a.in.stride + src]; kz[w] = a.in.z[w * a.in.stride + src]; }
    return cut_keeps<W, CT>(v, kx, kz, ORD ? a.in.o[src] : 0u, cut);
  };
  // count survivors per contiguous chunk of the tile
  const uint32_t chunk = (n0 + BLOCK - 1) / BLOCK;
  const uint32_t lo = tid * chunk < n0 ? tid * chunk : n0;
  const uint32_t hi = lo + chunk < n0 ? lo + chunk : n0;
  uint32_t cnt = 0;
  double lost = 0.0;
  for (uint32_t i = lo; i < hi; ++i) {
    if (keep((uint64_t)t0 + i)) ++cnt;
    else lost += fabs((double)a.in.c[(uint64_t)t0 + i]);
  }
  uint32_t incl = cnt;
  for (int d = 1; d < 64; d <<= 1) {
    const uint32_t v = __shfl_up(incl, d, 64);
    if (lane >= d) incl += v;
  }
  for (int d = 32; d >= 1; d >>= 1) lost += __shfl_xor(lost, d, 64);
  if (lane == 63) p_wsum[tid >> 6] = incl;
  if (lane == 0) p_drop[tid >> 6] = lost;
  __syncthreads();
  uint32_t before = 0, total = 0;
  for (int w = 0; w < NW; ++w) {
    before += (w < (tid >> 6)) ? p_wsum[w] : 0u;
    total += p_wsum[w];
  }
  const uint64_t base = a.o_base[tile];
  if (tid == 0) {
    a.o_start[tile] = (uint32_t)base;
    a.o_len[tile] = total;
    double v = 0.0;
    for (int w = 0; w < NW; ++w) v += p_drop[w];
    if (v != 0.0) atomicAdd(&a.dropped[blockIdx.x % kDropSlots], v);
    atomicAdd(&a.io[blockIdx.x % kDropSlots], (unsigned long long)n0);
    atomicAdd(&a.io[kDropSlots + blockIdx.x % kDropSlots], (unsigned long long)total);
  }
  uint64_t dst = base + before + incl - cnt;
  for (uint32_t i = lo; i < hi; ++i) {
    const uint64_t src = (uint64_t)t0 + i;
    if (!keep(src)) continue;
#pragma unroll
    for (int w = 0; w < W; ++w) {
      a.out.x[w * a.out.stride + dst] = a.in.x[w * a.in.stride + src];
      a.out.z[w * a.out.stride + dst] = a.in.z[w * a.in.stride + src];
    }
    a.out.c[dst] = a.in.c[src];
    if (ORD) a.out.o[dst] = a.in.o[src];
    ++dst;
  }
}

// Smallest power of two above n: an open-addressing table of that size holding at most n
// keys always has an empty slot, so every probe sequence ends.
constexpr int pow2_above(int n) { return n < 1 ? 1 : 2 * pow2_above(n / 2); }

// A uniform read of a table that no kernel writes while this one runs, through the
// constant address space: a scalar load, counted apart from the vector loads and stores,
// so waiting for it does not drain them.
__device__ __forceinline__ uint32_t ld_uniform(const uint32_t* p, uint32_t i) {
  return ((const __attribute__((address_space(4))) uint32_t*)p)[i];
}

// One tile's terms in registers: entry r of thread tid is term r * BLOCK + tid of the tile.
template <int W, class CT, int R>
struct G1Regs {
  uint64_t x[R][W], z[R][W];
  CT c[R];
  uint32_t o[R];
};

// Issue the loads of a tile's terms (nothing for a tile above CAP, which takes another path).
template <int W, class CT, bool ORD, int CAP, int BLOCK>
__device__ __forceinline__ void g1_fetch(const Gate1Args<CT>& a, G1Regs<W, CT, CAP / BLOCK>& g, uint32_t t0,
                                         uint32_t n0) {
  constexpr int R = CAP / BLOCK;
#pragma unroll
  for (int r = 0; r < R; ++r) {
    const uint32_t i = (uint32_t)r * BLOCK + threadIdx.x;
    const bool in = n0 <= (uint32_t)CAP && i < n0;
    const uint64_t src = (uint64_t)t0 + (in ? i : 0u);
#pragma unroll
    for (int w = 0; w < W; ++w) {
      g.x[r][w] = in ? a.in.x[w * a.in.stride + src] : 0ULL;
      g.z[r][w] = in ? a.in.z[w * a.in.stride + src] : 0ULL;
    }
    g.c[r] = in ? a.in.c[src] : (CT)0;
    g.o[r] = (ORD && in) ? (uint32_t)a.in.o[src] : 0u;
  }
}

// The gate on whole tiles, one workgroup per tile at a time.  The grid is persistent: a
// workgroup takes the tiles blockIdx.x, blockIdx.x + gridDim.x, ... of the list (t_count
// entries) and loads the next tile's terms while it compacts and writes the current one;
// tile ranges are read two tiles ahead.
template <int W, class CT, bool ORD, int CAP, int BLOCK>
__global__ void __launch_bounds__(BLOCK) k_gate1(Gate1Args<CT> a) {
  constexpr int R = CAP / BLOCK;
  constexpr int H = pow2_above(CAP);
  static_assert(H > CAP && (H & (H - 1)) == 0 && R * BLOCK == CAP, "tile shape");
  constexpr int NW = BLOCK / 64;
  constexpr uint32_t EMPTY = 0xffffffffu;
  // Table slot of a (string hash, order tag): the top bits of a multiplicative mix, which
  // depend on every bit of the key.  (The strings of a class differ in a few bits, and the
  // low bits of their linear hashes are correlated.)
  constexpr int HB = __builtin_ctz((unsigned)H);
  auto slot_of = [](uint32_t h, uint32_t o) -> uint32_t {
    return ((h ^ (o * 0x9e3779b9u)) * 0x85ebca6bu) >> (32 - HB);
  };
  __shared__ uint64_t sx[W][CAP];
  __shared__ uint64_t sz[W][CAP];
  __shared__ CT sc[CAP];
  __shared__ uint32_t sh[CAP];
  __shared__ uint8_t so[ORD ? CAP : 1];
  __shared__ uint32_t hidx[H];
  __shared__ uint32_t s_new, s_ovf, s_any;
  __shared__ uint32_t s_slice[R * NW];
  __shared__ uint32_t s_total;
  __shared__ double s_drop[NW];

  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const uint32_t count = a.t_count_dev ? min(*a.t_count_dev, a.t_count) : a.t_count;
  const uint32_t G = gridDim.x;
  uint32_t li = blockIdx.x;
  if (li >= count) return;
  auto tile_at = [&](uint32_t l) { return a.t_list ? ld_uniform(a.t_list, l) : l; };

  uint64_t m[2 * W];
#pragma unroll
  for (int w = 0; w < 2 * W; ++w) m[w] = a.g.m[w];
  const double cs = a.g.cs, snd = a.g.sn_dir;
  const uint32_t gh = a.g.khash;
  const int pw = a.g.pivot_word, pb = a.g.pivot_bit;
  const double thr = a.eps;
  const CutDev cut = gate_cut(a);

  // current tile and the next one (ranges), the current tile's terms in flight
  uint32_t tile = tile_at(li), t0 = ld_uniform(a.t_start, tile), n0 = ld_uniform(a.t_len, tile);
  uint32_t tile_n = 0, t0_n = 0, n0_n = 0;
  if (li + G < count) {
    tile_n = tile_at(li + G);
    t0_n = ld_uniform(a.t_start, tile_n);
    n0_n = ld_uniform(a.t_len, tile_n);
  }
  G1Regs<W, CT, R> cur;
  g1_fetch<W, CT, ORD, CAP, BLOCK>(a, cur, t0, n0);
  // the workgroup's statistics (thread 0), added to the global counters once at the end
  double acc_drop = 0.0;
  unsigned long long acc_in = 0, acc_out = 0;

  // One tile with its terms in `cur`.  Once the gate has read them, `cur` receives the next
  // tile's terms, which arrive while this tile is compacted and written.
  for (;;) {
    const bool more = li + G < count;
    uint32_t tile_nn = 0, t0_nn = 0, n0_nn = 0;
    if (li + 2 * G < count) {
      tile_nn = tile_at(li + 2 * G);
      t0_nn = ld_uniform(a.t_start, tile_nn);
      n0_nn = ld_uniform(a.t_len, tile_nn);
    }
    const uint64_t base = ld_uniform(a.o_base, tile);
    double lost = 0.0;
    if (n0 > (uint32_t)CAP) {
      if (more) g1_fetch<W, CT, ORD, CAP, BLOCK>(a, cur, t0_n, n0_n);
      // Too large for LDS.  If no term of the tile anticommutes with the gate, the tile
      // passes through unchanged apart from the pending cut; otherwise it is reported.
      if (tid == 0) s_any = 0;
      __syncthreads();
      bool any = false;
      for (uint32_t i = tid; i < n0 && !any; i += BLOCK) {
        uint64_t kx[W], kz[W];
#pragma unroll
        for (int w = 0; w < W; ++w) {
          kx[w] = a.in.x[w * a.in.stride + t0 + i];
          kz[w] = a.in.z[w * a.in.stride + t0 + i];
        }
        any = anticommutes<W>(kx, kz, m) != 0;
      }
      if (any) s_any = 1;
      __syncthreads();
      if (s_any || BLOCK < 256) {
        if (tid == 0) a.ovf_tiles[atomicAdd(a.ovf_count, 1u)] = tile;
        if (a.zero_on_ovf) zero_region(a, tile, n0);
      } else {
        pass_through<W, CT, ORD, BLOCK>(a, cut, tile, t0, n0);
      }
    } else {
      for (int j = tid; j < H; j += BLOCK) hidx[j] = EMPTY;
      if (tid == 0) { s_new = 0; s_ovf = 0; }
      __syncthreads();

      // ---- stage, cut, insert ----------------------------------------------------------------
      // Only strings that anticommute with the gate branch, and a partner iRP anticommutes
      // too, so only they enter the table (and need a hash); with a Clifford angle no
      // partner is looked up at all.
      const bool pairs = cs != 0.0 && snd != 0.0;
      uint32_t hh[R];   // key hashes of this thread's anticommuting terms
      bool an[R];       // anticommutes with the gate
#pragma unroll
      for (int r = 0; r < R; ++r) {
        const uint32_t i = (uint32_t)r * BLOCK + tid;
        an[r] = anticommutes<W>(cur.x[r], cur.z[r], m) != 0;
        hh[r] = an[r] ? key_hash<W>(cur.x[r], cur.z[r]) : 0u;
        if (i >= n0) continue;
#pragma unroll
        for (int w = 0; w < W; ++w) { sx[w][i] = cur.x[r][w]; sz[w][i] = cur.z[r][w]; }
        if (ORD) so[i] = (uint8_t)cur.o[r];
        const CT cv = cur.c[r];
        if (cv != (CT)0 && !cut_keeps<W, CT>(cv, cur.x[r], cur.z[r], cur.o[r], cut)) {
          lost += fabs((double)cv);
          cur.c[r] = (CT)0;
        }
        sh[i] = hh[r];
        sc[i] = cur.c[r];
        if (pairs && an[r] && cur.c[r] != (CT)0) {
          uint32_t slot = slot_of(hh[r], cur.o[r]);
          while (atomicCAS(&hidx[slot], EMPTY, i) != EMPTY) slot = (slot + 1) & (H - 1);
        }
      }
      __syncthreads();

      // ---- the gate ----------------------------------------------------------------------------
      const bool sine = ORD && a.sine_on && pairs;
      CT nsc[R];
      uint32_t upd = 0;
#pragma unroll
      for (int r = 0; r < R; ++r) {
        const uint32_t i = (uint32_t)r * BLOCK + tid;
        const double ci = (double)cur.c[r];
        if (i >= n0 || ci == 0.0) continue;
        if (!an[r]) {
          // untouched, but the threshold after a non-Clifford gate covers every term
          if (fabs(ci) < thr) { lost += fabs(ci); sc[i] = (CT)0; }
          continue;
        }
        if (snd == 0.0) {            // cos = +-1, sin = 0: a sign, no branching
          sc[i] = (CT)(ci * cs);
          continue;
        }
        const bool neg_i = irp_negative<W>(cur.x[r], cur.z[r], m, a.g.rr_phase);
        uint64_t qx[W], qz[W];
#pragma unroll
        for (int w = 0; w < W; ++w) { qx[w] = cur.x[r][w] ^ m[w]; qz[w] = cur.z[r][w] ^ m[W + w]; }
        if (cs == 0.0) {             // sin = +-1: P -> +-iRP in place (a permutation of strings)
#pragma unroll
          for (int w = 0; w < W; ++w) { sx[w][i] = qx[w]; sz[w][i] = qz[w]; }
          sh[i] = hh[r] ^ gh;
          sc[i] = (CT)((neg_i ? -ci : ci) * snd);
          continue;
        }
        if (sine) {
          // sine order: (Q, s) becomes cos c(Q, s) plus the sin part of (RQ, s - 1); the sin
          // part of (Q, s) starts (RQ, s + 1) when no entry of that string and tag exists
          // (an existing one takes it as its own incoming part).  Originals are read here,
          // the new values written after the barrier.
          const uint32_t hq = hh[r] ^ gh;
          const uint32_t t = cur.o[r];
          auto find = [&](uint32_t tag) -> uint32_t {
            uint32_t sl = slot_of(hq, tag);
            for (;;) {
              const uint32_t k = hidx[sl];
              if (k == EMPTY) return EMPTY;
              if (sh[k] == hq && so[k] == tag) {
                bool eq = true;
#pragma unroll
                for (int w = 0; w < W; ++w) eq = eq && sx[w][k] == qx[w] && sz[w][k] == qz[w];
                if (eq) return k;
              }
              sl = (sl + 1) & (H - 1);
            }
          };
          double ni = ci * cs;
          if (t > 0) {
            const uint32_t j = find(t - 1);
            if (j != EMPTY) {
              const double cj = (double)sc[j];
              const bool neg_j = irp_negative<W>(qx, qz, m, a.g.rr_phase);
              ni += (neg_j ? -cj : cj) * snd;
            }
          }
          if (fabs(ni) < thr || ni == 0.0) { lost += fabs(ni); ni = 0.0; }
          nsc[r] = (CT)ni;
          upd |= 1u << r;
          if ((int)t + 1 <= a.sine_max && find(t + 1) == EMPTY) {
            const double nq = (neg_i ? -ci : ci) * snd;
            if (fabs(nq) < thr || nq == 0.0) {
              lost += fabs(nq);
            } else {
              const uint32_t k = n0 + atomicAdd(&s_new, 1u);
              if (k < (uint32_t)CAP) {
#pragma unroll
                for (int w = 0; w < W; ++w) { sx[w][k] = qx[w]; sz[w][k] = qz[w]; }
                sh[k] = hq;
                so[k] = (uint8_t)(t + 1);
                sc[k] = (CT)nq;
              } else {
                s_ovf = 1;
              }
            }
          }
          continue;
        }
        // non-Clifford: find the partner string (same order tag) in the tile
        const uint32_t hq = hh[r] ^ gh;
        uint32_t slot = slot_of(hq, cur.o[r]);
        uint32_t j = EMPTY;
        for (;;) {
          const uint32_t k = hidx[slot];
          if (k == EMPTY) break;
          if (sh[k] == hq) {
            bool eq = !ORD || so[k] == cur.o[r];
#pragma unroll
            for (int w = 0; w < W; ++w) eq = eq && sx[w][k] == qx[w] && sz[w][k] == qz[w];
            if (eq) { j = k; break; }
          }
          slot = (slot + 1) & (H - 1);
        }
        if (j != EMPTY) {
          // both present: the member with the pivot bit clear updates the pair
          const uint64_t pv = pw < W ? pick<W>(cur.x[r], pw) : pick<W>(cur.z[r], pw - W);
          if ((pv >> pb) & 1ULL) continue;
          const double cj = (double)sc[j];
          const bool neg_j = irp_negative<W>(qx, qz, m, a.g.rr_phase);
          double ni = ci * cs + (neg_j ? -cj : cj) * snd;
          double nj = cj * cs + (neg_i ? -ci : ci) * snd;
          if (fabs(ni) < thr || ni == 0.0) { lost += fabs(ni); ni = 0.0; }
          if (fabs(nj) < thr || nj == 0.0) { lost += fabs(nj); nj = 0.0; }
          sc[i] = (CT)ni;
          sc[j] = (CT)nj;
        } else {
          double ni = ci * cs;
          const double nq = (neg_i ? -ci : ci) * snd;
          if (fabs(ni) < thr || ni == 0.0) { lost += fabs(ni); ni = 0.0; }
          sc[i] = (CT)ni;
          if (fabs(nq) < thr || nq == 0.0) {
            lost += fabs(nq);
          } else {
            const uint32_t k = n0 + atomicAdd(&s_new, 1u);
            if (k < (uint32_t)CAP) {
#pragma unroll
              for (int w = 0; w < W; ++w) { sx[w][k] = qx[w]; sz[w][k] = qz[w]; }
              sh[k] = hq;
              if (ORD) so[k] = (uint8_t)cur.o[r];
              sc[k] = (CT)nq;
            } else {
              s_ovf = 1;
            }
          }
        }
      }
      if (sine) {
        __syncthreads();   // every original has been read
#pragma unroll
        for (int r = 0; r < R; ++r)
          if ((upd >> r) & 1u) sc[(uint32_t)r * BLOCK + tid] = nsc[r];
      }
      if (more) g1_fetch<W, CT, ORD, CAP, BLOCK>(a, cur, t0_n, n0_n);
      __syncthreads();
      if (s_ovf) {
        if (tid == 0) a.ovf_tiles[atomicAdd(a.ovf_count, 1u)] = tile;
        if (a.zero_on_ovf) zero_region(a, tile, n0);
      } else {
        const uint32_t n = n0 + s_new;
        // ---- compact and write -------------------------------------------------------------------
        // Entry i = r * BLOCK + tid: the survivors of one (r, wavefront) slice are ranked by a
        // ballot, the slices in entry order by their counts, so the tile's order is kept,
        // LDS reads are consecutive and the global writes of a wavefront are contiguous.
        const int wv = tid >> 6;
        const uint64_t below = (1ULL << lane) - 1ULL;
        uint64_t bal[R];
#pragma unroll
        for (int r = 0; r < R; ++r) {
          const uint32_t i = (uint32_t)r * BLOCK + tid;
          bal[r] = __ballot(i < n && sc[i] != (CT)0);
          if (lane == 0) s_slice[r * NW + wv] = (uint32_t)__popcll(bal[r]);
        }
        double lsum = lost;
        for (int d = 32; d >= 1; d >>= 1) lsum += __shfl_xor(lsum, d, 64);
        if (lane == 0) s_drop[wv] = lsum;
        __syncthreads();
        uint32_t pre[R];
        uint32_t total = 0;
        if constexpr (NW <= 4) {
#pragma unroll
          for (int r = 0; r < R; ++r) {
            uint32_t before = 0;
#pragma unroll
            for (int w = 0; w < NW; ++w) before += w < wv ? s_slice[r * NW + w] : 0u;
            pre[r] = total + before;
#pragma unroll
            for (int w = 0; w < NW; ++w) total += s_slice[r * NW + w];
          }
        } else {
          // one wavefront scans the R * NW (<= 64) slice counts in place
          static_assert(R * NW <= 64, "slice scan");
          if (wv == 0) {
            const uint32_t v = lane < R * NW ? s_slice[lane] : 0u;
            uint32_t incl = v;
            for (int d = 1; d < 64; d <<= 1) {
              const uint32_t u = __shfl_up(incl, d, 64);
              if (lane >= d) incl += u;
            }
            if (lane < R * NW) s_slice[lane] = incl - v;
            if (lane == R * NW - 1) s_total = incl;
          }
          __syncthreads();
#pragma unroll
          for (int r = 0; r < R; ++r) pre[r] = s_slice[r * NW + wv];
          total = s_total;
        }
        // the tile's output region holds 2 * n0 slots (a gate at most doubles a tile); the
        // slots after its `total` survivors are left unused (every later sweep reads the
        // tile ranges, never the whole buffer)
        if (tid == 0) {
          a.o_start[tile] = (uint32_t)base;
          a.o_len[tile] = total;
          for (int w = 0; w < NW; ++w) acc_drop += s_drop[w];
          acc_in += n0;
          acc_out += total;
        }
#pragma unroll
        for (int r = 0; r < R; ++r) {
          if (!((bal[r] >> lane) & 1ULL)) continue;
          const uint32_t i = (uint32_t)r * BLOCK + tid;
          const uint64_t dst = base + pre[r] + (uint32_t)__popcll(bal[r] & below);
#pragma unroll
          for (int w = 0; w < W; ++w) {
            a.out.x[w * a.out.stride + dst] = sx[w][i];
            a.out.z[w * a.out.stride + dst] = sz[w][i];
          }
          a.out.c[dst] = sc[i];
          if (ORD) a.out.o[dst] = so[i];
        }
      }
    }
    __syncthreads();   // the tile's LDS is free
    li += G;
    tile = tile_n;
    t0 = t0_n;
    n0 = n0_n;
    tile_n = tile_nn;
    t0_n = t0_nn;
    n0_n = n0_nn;
    if (!more) break;
  }
  if (tid == 0) {
    if (acc_drop != 0.0) atomicAdd(&a.dropped[blockIdx.x % kDropSlots], acc_drop);
    if (acc_in) atomicAdd(&a.io[blockIdx.x % kDropSlots], acc_in);
    if (acc_out) atomicAdd(&a.io[kDropSlots + blockIdx.x % kDropSlots], acc_out);
  }
}

// A tile too large for LDS that the gate touches: a 1024-thread workgroup works in the
// tile's own output region (2 * n0 slots) with an open-addressing table in global memory,
// then compacts the region in place.  Same arithmetic as k_gate1.  Tables: either given
// (table[off[b] .. off[b] + hsize[b]) for list entry b, hsize a power of two >= 2 * n0,
// preset to ~0; one workgroup per entry), or, with `cursor` set, carved out of `table`
// (table_cap words) on the device, one per tile, by a persistent grid that reads the
// entry count on the device; a table that does not fit sets *err and its tile is skipped.
template <int W, class CT, bool ORD>
__device__ void gate1_big_tile(const Gate1Args<CT>& a, uint32_t li, uint32_t* table, const uint64_t* off,
                               const uint32_t* hsize, unsigned long long* cursor, unsigned long long table_cap,
                               unsigned int* err) {
  constexpr int BLOCK = 1024;
  constexpr int NW = BLOCK / 64;
  constexpr uint32_t EMPTY = 0xffffffffu;
  __shared__ uint32_t s_new;
  __shared__ uint32_t s_wsum[NW];
  __shared__ uint32_t s_done;
  __shared__ double s_drop[NW];
  __shared__ unsigned long long s_off;
  __shared__ uint32_t s_hsize;
  const int tid = threadIdx.x, lane = tid & 63;
  const uint32_t tile = a.t_list[li];
  const uint64_t t0 = a.t_start[tile];
  const uint32_t n0 = a.t_len[tile];
  const uint64_t base = a.o_base[tile];
  if (cursor) {
    if (tid == 0) {
      uint32_t h = 64;
      while (h < 2 * n0) h <<= 1;
      const unsigned long long o = atomicAdd(cursor, (unsigned long long)h);
      s_off = o;
      s_hsize = o + h <= table_cap ? h : 0u;
      if (!s_hsize) atomicOr(err, 1u);
    }
    __syncthreads();
    if (!s_hsize) return;
    for (uint32_t j = tid; j < s_hsize; j += BLOCK) table[s_off + j] = EMPTY;
  } else if (tid == 0) {
    s_off = off[li];
    s_hsize = hsize[li];
  }
  __syncthreads();
  uint32_t* tab = table + s_off;
  const uint32_t hm = s_hsize - 1;
  const int hb = __builtin_ctz(s_hsize);   // the table has 2^hb slots (hb >= 6)
  // slot of a (string hash, order tag): the top bits of a multiplicative mix, as in k_gate1
  auto bslot = [hb](uint32_t hh, uint32_t o) -> uint32_t {
    return ((hh ^ (o * 0x9e3779b9u)) * 0x85ebca6bu) >> (32 - hb);
  };
  uint64_t m[2 * W];
#pragma unroll
  for (int w = 0; w < 2 * W; ++w) m[w] = a.g.m[w];
  const double cs = a.g.cs, snd = a.g.sn_dir, thr = a.eps;
  const uint32_t gh = a.g.khash;
  const int pw = a.g.pivot_word, pb = a.g.pivot_bit;
  const CutDev cut = gate_cut(a);
  Terms<CT> o = a.out;
  if (tid == 0) { s_new = 0; s_done = 0; }
  double lost = 0.0;
  auto okey = [&](uint64_t j, uint64_t* kx, uint64_t* kz) {
#pragma unroll
    for (int w = 0; w < W; ++w) { kx[w] = o.x[w * o.stride + j]; kz[w] = o.z[w * o.stride + j]; }
  };
  // copy into the region, apply the pending cut, insert the live terms
  for (uint32_t i = tid; i < n0; i += BLOCK) {
    uint64_t kx[W], kz[W];
#pragma unroll
    for (int w = 0; w < W; ++w) {
      kx[w] = a.in.x[w * a.in.stride + t0 + i];
      kz[w] = a.in.z[w * a.in.stride + t0 + i];
      o.x[w * o.stride + base + i] = kx[w];
      o.z[w * o.stride + base + i] = kz[w];
    }
    const uint32_t oi = ORD ? a.in.o[t0 + i] : 0u;
    if (ORD) o.o[base + i] = (uint8_t)oi;
    const uint32_t h = key_hash<W>(kx, kz);
    a.hscr[base + i] = h;
    const CT cv = a.in.c[t0 + i];
    CT keep = cv;
    if (cv != (CT)0 && !cut_keeps<W, CT>(cv, kx, kz, oi, cut)) {
      lost += fabs((double)cv);
      keep = (CT)0;
    }
    o.c[base + i] = keep;
    if (keep != (CT)0) {
      uint32_t slot = bslot(h, oi);
      while (atomicCAS(&tab[slot], EMPTY, i) != EMPTY) slot = (slot + 1) & hm;
    }
  }
  __syncthreads();
  // sine order: new coefficients go to cscr first (originals are read by other threads) and
  // are copied back after the barrier
  const bool sine = ORD && a.sine_on && cs != 0.0 && snd != 0.0;
  if (sine)
    for (uint32_t i = tid; i < n0; i += BLOCK) a.cscr[base + i] = (double)o.c[base + i];
  __syncthreads();
  // the gate
  for (uint32_t i = tid; i < n0; i += BLOCK) {
    const double ci = (double)o.c[base + i];
    if (ci == 0.0) continue;
    uint64_t kx[W], kz[W];
    okey(base + i, kx, kz);
    if (!anticommutes<W>(kx, kz, m)) {
      if (fabs(ci) < thr) {   // threshold on every term
        lost += fabs(ci);
        o.c[base + i] = (CT)0;
        if (sine) a.cscr[base + i] = 0.0;
      }
      continue;
    }
    if (snd == 0.0) {
      o.c[base + i] = (CT)(ci * cs);
      continue;
    }
    const uint32_t oi = ORD ? o.o[base + i] : 0u;
    const uint32_t h = a.hscr[base + i];
    const bool neg_i = irp_negative<W>(kx, kz, m, a.g.rr_phase);
    uint64_t qx[W], qz[W];
#pragma unroll
    for (int w = 0; w < W; ++w) { qx[w] = kx[w] ^ m[w]; qz[w] = kz[w] ^ m[W + w]; }
    if (cs == 0.0) {
#pragma unroll
      for (int w = 0; w < W; ++w) { o.x[w * o.stride + base + i] = qx[w]; o.z[w * o.stride + base + i] = qz[w]; }
      a.hscr[base + i] = h ^ gh;
      o.c[base + i] = (CT)((neg_i ? -ci : ci) * snd);
      continue;
    }
    const uint32_t hq = h ^ gh;
    if (sine) {
      // as in k_gate1: (Q, s) takes cos c(Q, s) plus the sin part of (RQ, s - 1); a sin part
      // without an entry (RQ, s + 1) starts one
      auto find = [&](uint32_t tag) -> uint32_t {
        uint32_t sl = bslot(hq, tag);
        for (;;) {
          const uint32_t k = tab[sl];
          if (k == EMPTY) return EMPTY;
          if (a.hscr[base + k] == hq && o.o[base + k] == tag) {
            uint64_t px[W], pz[W];
            okey(base + k, px, pz);
            bool eq = true;
#pragma unroll
            for (int w = 0; w < W; ++w) eq = eq && px[w] == qx[w] && pz[w] == qz[w];
            if (eq) return k;
          }
          sl = (sl + 1) & hm;
        }
      };
      double ni = ci * cs;
      if (oi > 0) {
        const uint32_t j = find(oi - 1);
        if (j != EMPTY) {
          const double cj = (double)o.c[base + j];
          const bool neg_j = irp_negative<W>(qx, qz, m, a.g.rr_phase);
          ni += (neg_j ? -cj : cj) * snd;
        }
      }
      if (fabs(ni) < thr || ni == 0.0) { lost += fabs(ni); ni = 0.0; }
      a.cscr[base + i] = ni;
      if ((int)oi + 1 <= a.sine_max && find(oi + 1) == EMPTY) {
        const double nq = (neg_i ? -ci : ci) * snd;
        if (fabs(nq) < thr || nq == 0.0) {
          lost += fabs(nq);
        } else {
          const uint64_t k = base + n0 + atomicAdd(&s_new, 1u);   // at most one child per term
#pragma unroll
          for (int w = 0; w < W; ++w) { o.x[w * o.stride + k] = qx[w]; o.z[w * o.stride + k] = qz[w]; }
          o.o[k] = (uint8_t)(oi + 1);
          o.c[k] = (CT)nq;
          a.hscr[k] = hq;
        }
      }
      continue;
    }
    uint32_t slot = bslot(hq, oi);
    uint32_t j = EMPTY;
    for (;;) {
      const uint32_t k = tab[slot];
      if (k == EMPTY) break;
      if (a.hscr[base + k] == hq && (!ORD || o.o[base + k] == oi)) {
        uint64_t px[W], pz[W];
        okey(base + k, px, pz);
        bool eq = true;
#pragma unroll
        for (int w = 0; w < W; ++w) eq = eq && px[w] == qx[w] && pz[w] == qz[w];
        if (eq) { j = k; break; }
      }
      slot = (slot + 1) & hm;
    }
    if (j != EMPTY) {
      const uint64_t pv = pw < W ? pick<W>(kx, pw) : pick<W>(kz, pw - W);
      if ((pv >> pb) & 1ULL) continue;
      const double cj = (double)o.c[base + j];
      const bool neg_j = irp_negative<W>(qx, qz, m, a.g.rr_phase);
      double ni = ci * cs + (neg_j ? -cj : cj) * snd;
      double nj = cj * cs + (neg_i ? -ci : ci) * snd;
      if (fabs(ni) < thr || ni == 0.0) { lost += fabs(ni); ni = 0.0; }
      if (fabs(nj) < thr || nj == 0.0) { lost += fabs(nj); nj = 0.0; }
      o.c[base + i] = (CT)ni;
      o.c[base + j] = (CT)nj;
    } else {
      double ni = ci * cs;
      const double nq = (neg_i ? -ci : ci) * snd;
      if (fabs(ni) < thr || ni == 0.0) { lost += fabs(ni); ni = 0.0; }
      o.c[base + i] = (CT)ni;
      if (fabs(nq) < thr || nq == 0.0) {
        lost += fabs(nq);
      } else {
        const uint64_t k = base + n0 + atomicAdd(&s_new, 1u);   // at most one child per term: fits 2 * n0
#pragma unroll
        for (int w = 0; w < W; ++w) { o.x[w * o.stride + k] = qx[w]; o.z[w * o.stride + k] = qz[w]; }
        if (ORD) o.o[k] = (uint8_t)oi;
        o.c[k] = (CT)nq;
        a.hscr[k] = hq;
      }
    }
  }
  __syncthreads();
  if (sine) {
    for (uint32_t i = tid; i < n0; i += BLOCK) o.c[base + i] = (CT)a.cscr[base + i];
    __syncthreads();
  }
  // compact the region in place, chunk by chunk (destinations never pass their sources)
  const uint32_t n = n0 + s_new;
  uint32_t written = 0;
  for (uint32_t c0 = 0; c0 < n; c0 += BLOCK) {
    const uint32_t i = c0 + tid;
    const bool live = i < n && o.c[base + i] != (CT)0;
    uint64_t kx[W], kz[W];
    CT cv = (CT)0;
    uint32_t h = 0, oi = 0;
    if (live) {
      okey(base + i, kx, kz);
      cv = o.c[base + i];
      h = a.hscr[base + i];
      if (ORD) oi = o.o[base + i];
    }
    const uint64_t bal = __ballot(live);
    const uint32_t below = (uint32_t)__popcll(bal & ((1ULL << lane) - 1ULL));
    if (lane == 0) s_wsum[tid >> 6] = (uint32_t)__popcll(bal);
    __syncthreads();
    uint32_t before = 0, total = 0;
    for (int w = 0; w < NW; ++w) {
      before += (w < (tid >> 6)) ? s_wsum[w] : 0u;
      total += s_wsum[w];
    }
    if (live) {
      const uint64_t d = base + written + before + below;
#pragma unroll
      for (int w = 0; w < W; ++w) { o.x[w * o.stride + d] = kx[w]; o.z[w * o.stride + d] = kz[w]; }
      o.c[d] = cv;
      if (ORD) o.o[d] = (uint8_t)oi;
      a.hscr[d] = h;
    }
    written += total;
    __syncthreads();
  }
  for (int d = 32; d >= 1; d >>= 1) lost += __shfl_xor(lost, d, 64);
  if (lane == 0) s_drop[tid >> 6] = lost;
  __syncthreads();
  if (tid == 0) {
    a.o_start[tile] = (uint32_t)base;
    a.o_len[tile] = written;
    double v = 0.0;
    for (int w = 0; w < NW; ++w) v += s_drop[w];
    if (v != 0.0) atomicAdd(&a.dropped[li % kDropSlots], v);
    if (a.io) {
      atomicAdd(&a.io[li % kDropSlots], (unsigned long long)n0);
      atomicAdd(&a.io[kDropSlots + li % kDropSlots], (unsigned long long)written);
    }
  }
  (void)s_done;
}

template <int W, class CT, bool ORD>
__global__ void __launch_bounds__(1024) k_gate1_big(Gate1Args<CT> a, uint32_t* table, const uint64_t* off,
                                                    const uint32_t* hsize, unsigned long long* cursor,
                                                    unsigned long long table_cap, unsigned int* err,
                                                    unsigned long long* big_terms) {
  const uint32_t count = a.t_count_dev ? min(*a.t_count_dev, a.t_count) : a.t_count;
  for (uint32_t li = blockIdx.x; li < count; li += gridDim.x) {
    __syncthreads();   // the previous tile's readers of the shared words are done
    if (big_terms && threadIdx.x == 0) atomicAdd(big_terms, (unsigned long long)a.t_len[a.t_list[li]]);
    gate1_big_tile<W, CT, ORD>(a, li, table, off, hsize, cursor, table_cap, err);
  }
}

// Sort tiles by size: empty tiles get their (empty) output record here, tiles of at most
// small_max terms go to list 0, of at most mid_max to list 1, the others to list 2.
__global__ void k_route_tiles(const uint32_t* len, uint32_t ntiles, uint32_t small_max, uint32_t mid_max,
                              const uint32_t* o_base, uint32_t* o_start, uint32_t* o_len, uint32_t* list0,
                              uint32_t* list1, uint32_t* list2, uint32_t* counts) {
  const uint32_t t = blockIdx.x * blockDim.x + threadIdx.x;
  const uint32_t l = t < ntiles ? len[t] : 0u;
  if (t < ntiles && l == 0) {
    o_start[t] = o_base[t];
    o_len[t] = 0;
  }
  const int lane = threadIdx.x & 63;
  const uint64_t lt = (1ULL << lane) - 1ULL;
  const int cls = l <= small_max ? 0 : (l <= mid_max ? 1 : 2);
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    const bool mine = t < ntiles && l > 0 && cls == k;
    const uint64_t bal = __ballot(mine);
    if (!bal) continue;
    const int leader = __ffsll((unsigned long long)bal) - 1;
    uint32_t base = 0;
    if (lane == leader) base = atomicAdd(&counts[k], (uint32_t)__popcll(bal));
    base = __shfl(base, leader, 64);
    if (mine) (k == 0 ? list0 : (k == 1 ? list1 : list2))[base + (uint32_t)__popcll(bal & lt)] = t;
  }
}

// Tile ranges from tile starts ([ntiles + 1] prefix form).
__global__ void k_tile_ranges(const uint32_t* starts, uint32_t ntiles, uint32_t* start, uint32_t* len) {
  const uint32_t t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= ntiles) return;
  start[t] = starts[t];
  len[t] = starts[t + 1] - starts[t];
}

// keep[i] = the term survives the pending cut (and is not an exact zero).
template <int W, class CT, bool ORD>
__global__ void k_cut_keep(Terms<CT> t, uint64_t n, CutDev cut, uint32_t* keep, double* dropped) {
  double lost = 0.0;
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (uint64_t)gridDim.x * blockDim.x) {
    const CT v = t.c[i];
    bool k = v != (CT)0;
    if (k && cut.has) {
      uint64_t kx[W], kz[W];
#pragma unroll
      for (int w = 0; w < W; ++w) { kx[w] = t.x[w * t.stride + i]; kz[w] = t.z[w * t.stride + i]; }
      k = cut_keeps<W, CT>(v, kx, kz, ORD ? t.o[i] : 0u, cut);
    }
    keep[i] = k ? 1u : 0u;
    if (!k) lost += fabs((double)v);
  }
  add_dropped(lost, dropped);
}

// Gather the terms whose |c| bits match `prefix` on `pmask` (the candidates for the
// boundary of a cap) into `g` (capacity gcap); *cnt counts all matches.
template <int W, class CT, bool ORD>
__global__ void k_gather_bucket(Terms<CT> t, uint64_t n, uint64_t pmask, uint64_t prefix, Terms<CT> g, uint64_t gcap,
                                uint32_t* cnt) {
  const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const bool hit = i < n && t.c[i] != (CT)0 && (abs_key<CT>(t.c[i]) & pmask) == prefix;
  const uint64_t bal = __ballot(hit);
  if (!bal) return;
  const int lane = threadIdx.x & 63;
  const int leader = __ffsll((unsigned long long)bal) - 1;
  uint32_t base = 0;
  if (lane == leader) base = atomicAdd(cnt, (uint32_t)__popcll(bal));
  base = __shfl(base, leader, 64);
  if (!hit) return;
  const uint64_t j = base + (uint64_t)__popcll(bal & ((1ULL << lane) - 1ULL));
  if (j >= gcap) return;
#pragma unroll
  for (int w = 0; w < W; ++w) { g.x[w * g.stride + j] = t.x[w * t.stride + i]; g.z[w * g.stride + j] = t.z[w * t.stride + i]; }
  g.c[j] = t.c[i];
  if (ORD) g.o[j] = t.o[i];
}

// ------------------------------------------------------------------------------------------
// Sweeps over the live slots of a tiled buffer.  Between the gates of a run, tile t holds its
// terms in slots [start[t], start[t] + len[t]) of its own output region; the rest of the
// region is unused and never read, so these sweeps walk the tile ranges instead of the
// whole buffer.
// ------------------------------------------------------------------------------------------
struct TileView {
  const uint32_t* start;
  const uint32_t* len;
  uint32_t ntiles;
};

// Call f(slot, key) with the |c| key of every live slot.  A wavefront takes sixteen
// consecutive tiles: lanes 0..15 load their ranges in one request, the sixteen ranges are
// read into scalar registers (readlane, before any branch: a shuffle from a lane that a
// branch has switched off returns 0), and the first 128 keys of all sixteen tiles are loaded
// (32 loads in flight per lane) before any is used; the rest of tiles longer than 128
// follows in a loop.
template <class CT, class F>
__device__ __forceinline__ void tile_visit(const CT* c, const TileView tv, F&& f) {
  const int lane = threadIdx.x & 63;
  const uint32_t wave = (blockIdx.x * blockDim.x + threadIdx.x) >> 6;
  const uint32_t nw = (gridDim.x * blockDim.x) >> 6;
  for (uint64_t t0 = (uint64_t)wave * 16; t0 < tv.ntiles; t0 += (uint64_t)nw * 16) {
    uint32_t my_s = 0, my_l = 0;
    if (lane < 16 && t0 + lane < tv.ntiles) {
      my_s = tv.start[t0 + lane];
      my_l = tv.len[t0 + lane];
    }
    uint32_t ts[16], tl[16];
#pragma unroll
    for (int u = 0; u < 16; ++u) {
      ts[u] = (uint32_t)__builtin_amdgcn_readlane((int)my_s, u);
      tl[u] = (uint32_t)__builtin_amdgcn_readlane((int)my_l, u);
    }
    uint64_t k[2][16];
#pragma unroll
    for (int r = 0; r < 2; ++r)
#pragma unroll
      for (int u = 0; u < 16; ++u) {
        const uint32_t i = (uint32_t)lane + 64u * r;
        k[r][u] = i < tl[u] ? abs_key<CT>(c[(uint64_t)ts[u] + i]) : 0ULL;
      }
#pragma unroll
    for (int r = 0; r < 2; ++r)
#pragma unroll
      for (int u = 0; u < 16; ++u)
        if (k[r][u]) f((uint64_t)ts[u] + (uint64_t)lane + 64u * r, k[r][u]);
#pragma unroll
    for (int u = 0; u < 16; ++u)
      for (uint32_t i = 128 + lane; i < tl[u]; i += 64) {
        const uint64_t kk = abs_key<CT>(c[(uint64_t)ts[u] + i]);
        if (kk) f((uint64_t)ts[u] + i, kk);
      }
  }
}

// As k_abs_hist_win over the live slots of the tiles.
template <class CT>
__global__ void __launch_bounds__(256) k_abs_hist_win_tiles(const CT* c, TileView tv, uint64_t lo, int shift,
                                                            uint32_t* hist) {
  __shared__ uint32_t h[2049];
  for (int b = threadIdx.x; b < 2049; b += 256) h[b] = 0;
  __syncthreads();
  uint32_t above = 0;   // most keys lie above a window near the cut: counted in a register
  tile_visit<CT>(c, tv, [&](uint64_t, uint64_t k) {
    if (k >= lo) {
      const uint64_t d = (k - lo) >> shift;
      if (d >= 2048) ++above;
      else atomicAdd(&h[d], 1u);
    }
  });
  for (int d = 32; d >= 1; d >>= 1) above += __shfl_xor(above, d, 64);
  if ((threadIdx.x & 63) == 0 && above) atomicAdd(&h[2048], above);
  __syncthreads();
  for (int b = threadIdx.x; b < 2049; b += 256)
    if (h[b]) atomicAdd(&hist[b], h[b]);
}

// As k_abs_hist over the live slots of the tiles.
template <class CT>
__global__ void __launch_bounds__(256) k_abs_hist_tiles(const CT* c, TileView tv, int shift, int bits, uint64_t pmask,
                                                        uint64_t prefix, uint32_t* hist) {
  __shared__ uint32_t h[2048];
  const int bins = 1 << bits;
  for (int b = threadIdx.x; b < bins; b += 256) h[b] = 0;
  __syncthreads();
  tile_visit<CT>(c, tv, [&](uint64_t, uint64_t k) {
    if ((k & pmask) == prefix) atomicAdd(&h[(k >> shift) & (uint64_t)(bins - 1)], 1u);
  });
  __syncthreads();
  for (int b = threadIdx.x; b < bins; b += 256)
    if (h[b]) atomicAdd(&hist[b], h[b]);
}

// As k_gather_bucket over the live slots of the tiles (the candidates are few: one atomic
// each).
template <int W, class CT, bool ORD>
__global__ void k_gather_bucket_tiles(Terms<CT> t, TileView tv, uint64_t pmask, uint64_t prefix, Terms<CT> g,
                                      uint64_t gcap, uint32_t* cnt) {
  tile_visit<CT>(t.c, tv, [&](uint64_t i, uint64_t key) {
    if ((key & pmask) != prefix) return;
    const CT v = t.c[i];
    const uint64_t j = atomicAdd(cnt, 1u);
    if (j >= gcap) return;
#pragma unroll
    for (int w = 0; w < W; ++w) { g.x[w * g.stride + j] = t.x[w * t.stride + i]; g.z[w * g.stride + j] = t.z[w * t.stride + i]; }
    g.c[j] = v;
    if (ORD) g.o[j] = t.o[i];
  });
}

// keep[i] = 1 for the live slots that survive the pending cut (the caller clears keep over
// the whole buffer first, so unused slots stay 0).
template <int W, class CT, bool ORD>
__global__ void k_cut_keep_tiles(Terms<CT> t, TileView tv, CutDev cut0, const CutDev* cutp, uint32_t* keep,
                                 double* dropped) {
  const CutDev cut = cutp ? *cutp : cut0;
  double lost = 0.0;
  tile_visit<CT>(t.c, tv, [&](uint64_t i, uint64_t key) {
    bool k = true;
    if (cut.has) {
      if (key != cut.val) {
        k = key > cut.val;
      } else {
        uint64_t kx[W], kz[W];
#pragma unroll
        for (int w = 0; w < W; ++w) { kx[w] = t.x[w * t.stride + i]; kz[w] = t.z[w * t.stride + i]; }
        k = canon_le<W>(kx, kz, ORD ? t.o[i] : 0u, cut);
      }
    }
    if (k) keep[i] = 1u;
    else lost += fabs((double)t.c[i]);
  });
  add_dropped(lost, dropped);
}

}  // namespace pp
