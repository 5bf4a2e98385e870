// pp_layer.hpp -- fused per-layer propagation of grouped terms in LDS (gfx950).
//
// A layer's gates never change some bits of a term: rotations about X-type Paulis keep z,
// Z-type ones keep x, a single general rotation keeps everything but one pivot bit.  After
// the terms are grouped by a hash of those invariant bits (LSD radix passes), every group
// is closed under the layer: all branching, merging and thresholding of its members stays
// inside it.  One workgroup loads a tile of whole groups into an LDS hash table and applies
// every gate of the layer in order -- cos/sin branching (Section I, Eq. evolve_gate, and the
// backward rule of the Euclid appendix), accumulation of duplicate strings (Appendix B's
// A'[P'] += c'), the |c| < eps threshold after each non-Clifford gate -- then the inverse
// Pauli-Lindblad rescale or its error-order expansion (Eq. evolve_noise; Appendix C's
// expansion in the number of errors), and writes the survivors to HBM once.  A tile whose
// terms outgrow LDS reports itself and is finished by the per-gate path.
#pragma once

#include "pp_common.hpp"
#include "pp_sort.hpp"

#include <type_traits>

namespace pp {

template <int W>
struct LayerCfg;
template <>
struct LayerCfg<1> { static constexpr int CAP = 4096, BLOCK = 1024, GATES = 64; };
template <>
struct LayerCfg<2> { static constexpr int CAP = 2048, BLOCK = 1024, GATES = 64; };
template <>
struct LayerCfg<3> { static constexpr int CAP = 2048, BLOCK = 1024, GATES = 32; };
template <>
struct LayerCfg<4> { static constexpr int CAP = 1024, BLOCK = 512, GATES = 64; };

constexpr int kMaxPowerSums = 4;   // error-order mode supports max_order <= 4
constexpr uint32_t kOvfOutput = 0x80000000u;   // overflow-list flag: output space, not LDS

template <class CT>
struct LayerArgs {
  Terms<CT> in;
  Terms<CT> out;
  const uint32_t* tile_start;   // [ntiles + 1]
  const uint32_t* tile_list;    // optional: blockIdx.x -> tile index
  const GateDev* gates;         // in application order
  int ngates;
  double eps;                   // threshold after each non-Clifford gate (0: none)
  int gate_kind;                // 0 X-type run, 1 Z-type run, 2 general gate
  int any_nonclifford;          // the gate list holds a non-Clifford gate
  int has_noise;
  NoiseDev noise;
  double eps_noise;             // threshold after the noise expansion (error-order mode)
  const uint32_t* htab;          // linear-hash tables (kHashTabWords)
  unsigned long long* out_count;
  unsigned long long* out_fail;  // smallest start refused for lack of output space
  uint32_t* ovf_tiles;
  uint32_t* ovf_count;
  // statistics, each spread over kStatSlots addresses (one workgroup adds to slot
  // blockIdx.x % kStatSlots; a single address would serialise the workgroups)
  double* dropped;              // sum of |c| removed by thresholds
  unsigned int* peak;           // largest live count seen in a tile
  unsigned long long* peak_sum; // sum over tiles of each tile's largest live count during the gates
};
constexpr int kStatSlots = 64;

// Compact per-W gate record staged in LDS by the fused kernel.
template <int W>
struct GateC {
  uint64_t m[2 * W];
  double cs, sn_dir;
  uint32_t hash;
  int16_t type, clifford, pivot_word, pivot_bit, rr_phase, w0, b0, w1, b1, pad;
};
template <int W>
__device__ __forceinline__ GateC<W> to_compact(const GateDev& g) {
  GateC<W> c;
#pragma unroll
  for (int w = 0; w < 2 * W; ++w) c.m[w] = w < W ? g.m[w] : g.m[W + (w - W)];
  c.cs = g.cs;
  c.sn_dir = g.sn_dir;
  c.hash = g.hash;
  c.type = (int16_t)g.type;
  c.clifford = (int16_t)g.clifford;
  c.pivot_word = (int16_t)g.pivot_word;
  c.pivot_bit = (int16_t)g.pivot_bit;
  c.rr_phase = (int16_t)g.rr_phase;
  c.w0 = (int16_t)g.w0;
  c.b0 = (int16_t)g.b0;
  c.w1 = (int16_t)g.w1;
  c.b1 = (int16_t)g.b1;
  c.pad = 0;
  return c;
}

// ------------------------------------------------------------------------------------------
// Pauli helpers on register copies of a key.
// ------------------------------------------------------------------------------------------
template <int W>
__device__ __forceinline__ uint64_t pick(const uint64_t* v, int w) {
  uint64_t r = v[0];
#pragma unroll
  for (int k = 1; k < W; ++k)
    if (w == k) r = v[k];
  return r;
}

// <P, R>: parity of |x_P & z_R| + |z_P & x_R|.
template <int W>
__device__ __forceinline__ int anticommutes(const uint64_t* px, const uint64_t* pz, const uint64_t* m) {
  uint64_t acc = 0;
#pragma unroll
  for (int w = 0; w < W; ++w) acc ^= (px[w] & m[W + w]) ^ (pz[w] & m[w]);
  return __popcll(acc) & 1;
}

// Sign s of i R P = s Q for anticommuting Hermitian Paulis, Q = (x_P ^ x_R, z_P ^ z_R):
// R P = i^{|xR&zR|} i^{|xP&zP|} (-1)^{|zR&xP|} X^{xQ} Z^{zQ} and Q = i^{|xQ&zQ|} X^{xQ} Z^{zQ},
// so i R P = i^{1 + |xR&zR| + |xP&zP| + 2|zR&xP| - |xQ&zQ|} Q (an even power here).
template <int W>
__device__ __forceinline__ bool irp_negative(const uint64_t* px, const uint64_t* pz, const uint64_t* m,
                                             int rr_phase) {
  int ph = 1 + rr_phase;
#pragma unroll
  for (int w = 0; w < W; ++w) {
    const uint64_t qx = px[w] ^ m[w];
    const uint64_t qz = pz[w] ^ m[W + w];
    ph += __popcll(px[w] & pz[w]) + 2 * __popcll(m[W + w] & px[w]) + 3 * __popcll(qx & qz);
  }
  return (ph & 3) == 2;
}

// Power sums p_j = sum over generators anticommuting with P of v_k^j (error-order mode,
// v_k = x_k) or the plain sum of lambda_k (greedy mode, one value).
template <int W>
__device__ __forceinline__ void noise_sums(const uint64_t* px, const uint64_t* pz, const NoiseDev& nd,
                                           int np, double* p) {
#pragma unroll
  for (int j = 0; j < kMaxPowerSums; ++j) p[j] = 0.0;
  for (int s = 0; s < nd.nsup; ++s) {
    const SupportDev sp = nd.sup[s];
    uint32_t pat = (uint32_t)((pick<W>(px, sp.w0) >> sp.b0) & 1u) | (uint32_t)(((pick<W>(pz, sp.w0) >> sp.b0) & 1u) << 1);
    if (sp.w1 >= 0)
      pat |= (uint32_t)(((pick<W>(px, sp.w1) >> sp.b1) & 1u) << 2) | (uint32_t)(((pick<W>(pz, sp.w1) >> sp.b1) & 1u) << 3);
    if (pat) {
      const double* t = nd.tab + sp.table + (size_t)pat * np;
      for (int j = 0; j < np; ++j) p[j] += t[j];
    }
  }
  for (int d = 0; d < nd.ndirect; ++d) {
    const uint64_t* m = nd.dm + (size_t)d * 2 * W;
    if (anticommutes<W>(px, pz, m))
      for (int j = 0; j < np; ++j) p[j] += nd.dval[(size_t)d * np + j];
  }
}

// Greedy-mode factor of a string: the product, over the generators that anticommute with
// it, of their fidelity factors 1 - 2q_k (Eq. evolve_noise), multiplied one at a time in
// generator-list order.  Supports are listed in that order with their generators'
// factor indices in per-pattern slots (padding points at a 1.0, an exact no-op);
// generators handled directly come after them.
template <int W>
__device__ __forceinline__ uint32_t support_pattern(const uint64_t* px, const uint64_t* pz, const SupportDev& sp) {
  uint32_t pat = (uint32_t)((pick<W>(px, sp.w0) >> sp.b0) & 1u) | (uint32_t)(((pick<W>(pz, sp.w0) >> sp.b0) & 1u) << 1);
  if (sp.w1 >= 0)
    pat |= (uint32_t)(((pick<W>(px, sp.w1) >> sp.b1) & 1u) << 2) | (uint32_t)(((pick<W>(pz, sp.w1) >> sp.b1) & 1u) << 3);
  return pat;
}

// qoff/qent: the supports listed per qubit (NoiseDev), or null to visit every support.
template <int W>
__device__ __forceinline__ double noise_factor(const uint64_t* px, const uint64_t* pz, const double* tab,
                                               const SupportDev* sup, const int32_t* qoff, const uint32_t* qent,
                                               const NoiseDev& nd) {
  // Greedy mode: the product over runs of generators on the same qubits of each run's
  // product for the string's local pattern (pattern 0: exactly 1.0, skipped).  Only runs
  // on the string's non-identity qubits can differ from 1: with the per-qubit lists the
  // string visits just those, each once (a two-qubit run at its first qubit when that one
  // is set, else at its second), in qubit order.
  double prod = 1.0;
  if (qoff) {
#pragma unroll
    for (int w = 0; w < W; ++w) {
      uint64_t live = px[w] | pz[w];
      while (live) {
        const int q = 64 * w + (int)__builtin_ctzll(live);
        live &= live - 1;
        if (q >= nd.nq) break;
        for (int e = qoff[q]; e < qoff[q + 1]; ++e) {
          const uint32_t en = qent[e];
          const SupportDev sp = sup[en & 0x7fffffffu];
          if ((en >> 31) && (((pick<W>(px, sp.w0) | pick<W>(pz, sp.w0)) >> sp.b0) & 1u)) continue;
          prod *= tab[sp.table + (int)support_pattern<W>(px, pz, sp)];
        }
      }
    }
  } else {
    for (int s = 0; s < nd.nsup; ++s) {
      const SupportDev sp = sup[s];
      const uint32_t pat = support_pattern<W>(px, pz, sp);
      if (pat) prod *= tab[sp.table + (int)pat];
    }
  }
  if (nd.ndirect > 0) {
    double run = 1.0;
    for (int d = 0; d < nd.ndirect; ++d) {
      if (d > 0 && nd.drun[d]) {
        prod *= run;
        run = 1.0;
      }
      const uint64_t* m = nd.dm + (size_t)d * 2 * W;
      if (anticommutes<W>(px, pz, m)) run *= nd.dval[d];
    }
    prod *= run;
  }
  return prod;
}

// Elementary symmetric sums e_0..e_M of the anticommuting x_k from power sums (Newton).
__device__ __forceinline__ void elementary_from_power(const double* p, int M, double* e) {
  e[0] = 1.0;
  if (M >= 1) e[1] = p[0];
  if (M >= 2) e[2] = (e[1] * p[0] - p[1]) / 2.0;
  if (M >= 3) e[3] = (e[2] * p[0] - e[1] * p[1] + p[2]) / 3.0;
  if (M >= 4) e[4] = (e[3] * p[0] - e[2] * p[1] + e[1] * p[2] - p[3]) / 4.0;
}

// ------------------------------------------------------------------------------------------
// The fused layer kernel.
// ------------------------------------------------------------------------------------------
// Two shapes of the same kernel: one wavefront with a 256-entry table (first attempt: many
// small tiles, barriers are wavefront-local, tiles skip the gates none of their terms sees)
// and a 1024-thread workgroup with the LayerCfg table (tiles whose groups outgrow 256).
template <int W>
struct SmallCfg { static constexpr int CAP = 256, BLOCK = 64, GATES = 64; };

template <int W, class CT, bool ORD, int CAP, int BLOCK, int GATES>
__global__ void __launch_bounds__(BLOCK) k_layer(LayerArgs<CT> a) {
  constexpr int H = 2 * CAP;
  constexpr int R = CAP / BLOCK;
  constexpr uint32_t EMPTY = 0xffffffffu;

  __shared__ uint64_t sx[W][CAP];
  __shared__ uint64_t sz[W][CAP];
  __shared__ CT sc[CAP];
  __shared__ uint32_t sh[CAP];       // linear hash of each entry's string (order not included)
  __shared__ uint8_t so[ORD ? CAP : 1];
  __shared__ uint32_t hidx[H];       // (16-bit fingerprint << 16) | entry index, or EMPTY
  __shared__ uint32_t s_cnt[3];      // appends of processed gate k land in s_cnt[k % 3]
  __shared__ uint32_t s_dead[3];     // entries zeroed by processed gate k
  __shared__ int s_ldelta[3];        // change of the live count by processed gate k (appends aside)
  __shared__ uint32_t s_tdrop;       // entries zeroed by the tile-wide threshold (cumulative)
  __shared__ uint32_t s_ovf;
  __shared__ unsigned long long s_or[2 * W];
  __shared__ uint32_t stmp[BLOCK / 64];
  __shared__ unsigned long long s_base;
  __shared__ double s_drop[BLOCK / 64];
  __shared__ GateC<W> sgate[GATES];   // a chunk of the gate list

  const int tid = threadIdx.x;
  const uint32_t tile = a.tile_list ? a.tile_list[blockIdx.x] : blockIdx.x;
  const uint32_t t0 = a.tile_start[tile];
  const uint32_t t1 = a.tile_start[tile + 1];
  if (t1 <= t0) return;
  const uint32_t n0 = t1 - t0;
  if (n0 > (uint32_t)CAP) {
    if (tid == 0) {
      const uint32_t k = atomicAdd(a.ovf_count, 1u);
      a.ovf_tiles[k] = tile;
    }
    return;
  }

  // Slot = the top bits of a multiplicative mix of the full hash (the strings of a tile's
  // classes differ in a few bits, and the low bits of their linear hashes are correlated),
  // fingerprint = its high 16 bits (kept in the slot so most probes are resolved without
  // reading the stored key).
  static_assert((H & (H - 1)) == 0, "table size");
  constexpr int HB = __builtin_ctz((unsigned)H);
  auto full_hash = [](uint32_t hs, uint32_t o) -> uint32_t { return ORD ? hs ^ ord_hash(o) : hs; };
  auto slot_of = [](uint32_t fh) -> uint32_t { return (fh * 0x85ebca6bu) >> (32 - HB); };
  auto fp_of = [](uint32_t fh) -> uint32_t { return fh >> 16; };
  auto same_key = [&](uint32_t idx, const uint64_t* kx, const uint64_t* kz, uint32_t o) -> bool {
    bool eq = true;
#pragma unroll
    for (int w = 0; w < W; ++w) eq = eq && sx[w][idx] == kx[w] && sz[w][idx] == kz[w];
    if (ORD) eq = eq && so[idx] == o;
    return eq;
  };
  // Resolve a probe sequence whose first slot value v was already read.
  auto resolve = [&](uint32_t s, uint32_t fp, uint32_t v, const uint64_t* kx, const uint64_t* kz,
                     uint32_t o) -> uint32_t {
    for (int probe = 0; probe < H; ++probe) {
      if (v == EMPTY) return EMPTY;
      if ((v >> 16) == fp) {
        const uint32_t idx = v & 0xffffu;
        if (same_key(idx, kx, kz, o)) return idx;
      }
      s = (s + 1) & (H - 1);
      v = hidx[s];
    }
    return EMPTY;
  };
  auto lookup_h = [&](uint32_t fh, const uint64_t* kx, const uint64_t* kz, uint32_t o) -> uint32_t {
    const uint32_t s = slot_of(fh);
    return resolve(s, fp_of(fh), hidx[s], kx, kz, o);
  };
  auto insert_h = [&](uint32_t i, uint32_t fh) {
    uint32_t s = slot_of(fh);
    const uint32_t v = (fp_of(fh) << 16) | i;
    for (int probe = 0; probe < H; ++probe) {
      if (atomicCAS(&hidx[s], EMPTY, v) == EMPTY) return;
      s = (s + 1) & (H - 1);
    }
  };
  auto insert = [&](uint32_t i) { insert_h(i, full_hash(sh[i], ORD ? (uint32_t)so[i] : 0u)); };
  auto load_key = [&](uint32_t i, uint64_t* kx, uint64_t* kz) {
#pragma unroll
    for (int w = 0; w < W; ++w) { kx[w] = sx[w][i]; kz[w] = sz[w][i]; }
  };

  // ---- load the tile -----------------------------------------------------------------------
  uint64_t lor[2 * W];
#pragma unroll
  for (int w = 0; w < 2 * W; ++w) lor[w] = 0;
  for (uint32_t i = tid; i < n0; i += BLOCK) {
    uint64_t kx[W], kz[W];
#pragma unroll
    for (int w = 0; w < W; ++w) {
      kx[w] = a.in.x[w * a.in.stride + t0 + i];
      kz[w] = a.in.z[w * a.in.stride + t0 + i];
      sx[w][i] = kx[w];
      sz[w][i] = kz[w];
      lor[w] |= kx[w];
      lor[W + w] |= kz[w];
    }
    sc[i] = a.in.c[t0 + i];
    if (ORD) so[i] = a.in.o[t0 + i];
    sh[i] = lin_hash<W>(kx, kz, a.htab);
  }
  for (uint32_t j = tid; j < (uint32_t)H; j += BLOCK) hidx[j] = EMPTY;
  if (tid < 2 * W) s_or[tid] = 0;
  if (tid < 3) { s_cnt[tid] = 0; s_dead[tid] = 0; s_ldelta[tid] = 0; }
  if (tid == 0) { s_ovf = 0; s_tdrop = 0; }
  __syncthreads();
#pragma unroll
  for (int w = 0; w < 2 * W; ++w) {
    uint64_t v = lor[w];
    for (int d = 32; d >= 1; d >>= 1) v |= __shfl_xor(v, d, 64);
    if ((tid & 63) == 0 && v) atomicOr(&s_or[w], (unsigned long long)v);
  }
  for (uint32_t i = tid; i < n0; i += BLOCK) insert(i);
  __syncthreads();
  // x bits and z bits present anywhere in the tile: a gate R can only act on the tile if
  // (x_any & z_R) | (z_any & x_R) is nonzero.  X-type (Z-type) runs never change z (x),
  // so the half of this mask those gates test stays exact; a general gate is alone in its run.
  uint64_t orx[W], orz[W];
#pragma unroll
  for (int w = 0; w < W; ++w) { orx[w] = s_or[w]; orz[w] = s_or[W + w]; }

  uint32_t n = n0;
  uint32_t peak = n0;
  uint32_t live_peak = n0;   // largest count of live entries after any gate
  int64_t live = n0;         // entries with c != 0 (exact: every change is counted)
  uint32_t tdrop_seen = 0;
  uint32_t dead = 0;
  double dropped = 0.0;
  bool thresholded_all = false;
  int gi = 0;   // processed-gate counter (rotates the shared counters)

  // Keys and hashes of the entries this thread owns (entry i belongs to thread i % BLOCK).
  uint64_t rkx[R][W], rkz[R][W];
  uint32_t rko[R], rh[R];
  auto reload = [&](uint32_t lo, uint32_t hi) {
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const uint32_t i = (uint32_t)r * BLOCK + tid;
      if (i >= lo && i < hi) {
#pragma unroll
        for (int w = 0; w < W; ++w) { rkx[r][w] = sx[w][i]; rkz[r][w] = sz[w][i]; }
        rko[r] = ORD ? so[i] : 0u;
        rh[r] = sh[i];
      }
    }
  };
  reload(0, n);

  // Compaction of entries [0, nn) keeping c != 0 and !(|c| < thr); optionally rebuilds the
  // hash index.  Uniform call.
  auto compact = [&](uint32_t nn, double thr, bool rebuild) -> uint32_t {
    uint64_t rx[R][W], rz[R][W];
    CT rc[R];
    uint8_t ro[R];
    uint32_t rhh[R];
    bool keep[R];
    uint32_t cnt = 0;
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const uint32_t i = (uint32_t)r * BLOCK + tid;
      keep[r] = false;
      if (i < nn) {
#pragma unroll
        for (int w = 0; w < W; ++w) { rx[r][w] = sx[w][i]; rz[r][w] = sz[w][i]; }
        rc[r] = sc[i];
        ro[r] = ORD ? so[i] : 0;
        rhh[r] = sh[i];
        const double v = (double)rc[r];
        keep[r] = v != 0.0 && !(fabs(v) < thr);
        if (!keep[r]) dropped += fabs(v);
        cnt += keep[r] ? 1u : 0u;
      }
    }
    uint32_t total;
    uint32_t pos = block_exclusive_scan<BLOCK>(cnt, stmp, &total);
#pragma unroll
    for (int r = 0; r < R; ++r) {
      if (keep[r]) {
#pragma unroll
        for (int w = 0; w < W; ++w) { sx[w][pos] = rx[r][w]; sz[w][pos] = rz[r][w]; }
        sc[pos] = rc[r];
        if (ORD) so[pos] = ro[r];
        sh[pos] = rhh[r];
        ++pos;
      }
    }
    if (rebuild) {
      for (uint32_t j = tid; j < (uint32_t)H; j += BLOCK) hidx[j] = EMPTY;
      __syncthreads();
      for (uint32_t i = tid; i < total; i += BLOCK) insert(i);
    }
    __syncthreads();
    return total;
  };

  auto overflow_exit = [&]() {
    if (tid == 0) {
      const uint32_t k = atomicAdd(a.ovf_count, 1u);
      a.ovf_tiles[k] = tile;
    }
  };

  // The threshold after the first non-Clifford gate also reaches terms that gate left alone
  // (later ones cannot fall below it: magnitudes change only where a gate acts).
  auto threshold_all = [&]() {
    thresholded_all = true;
    if (!(a.eps > 0.0)) return;
    int nd = 0;
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const uint32_t i = (uint32_t)r * BLOCK + tid;
      if (i < n) {
        const double v = (double)sc[i];
        if (v != 0.0 && fabs(v) < a.eps) {
          dropped += fabs(v);
          sc[i] = (CT)0.0;
          ++nd;
        }
      }
    }
    int ndw = nd;
    for (int d = 32; d >= 1; d >>= 1) ndw += __shfl_xor(ndw, d, 64);
    if ((tid & 63) == 0 && ndw) atomicAdd(&s_tdrop, (uint32_t)ndw);
    if (__syncthreads_or(nd)) dead += 1;   // barrier; zeros now exist, so compaction may run
    live -= (int64_t)(s_tdrop - tdrop_seen);
    tdrop_seen = s_tdrop;
  };

  // One gate over the tile: stage 1 tests anticommutation and prefetches the partner's first
  // slot, stage 2 resolves and updates (a pair by its member with the pivot bit clear), stage
  // 3 appends the sin children of terms without partner.  TYPE selects the bit-level forms
  // of the test, the flip and the sign of i R P for single-qubit X and for Z Z rotations.
  auto gate_pass = [&](auto type_tag, const GateC<W>& G, uint32_t nn) {
    constexpr int TYPE = decltype(type_tag)::value;
    uint64_t m[2 * W];
#pragma unroll
    for (int w = 0; w < 2 * W; ++w) m[w] = G.m[w];
    const double cs = G.cs;
    const double snd = G.sn_dir;
    const double thr = G.clifford ? 0.0 : a.eps;
    const uint32_t ghash = G.hash;
    const int w0 = G.w0, b0 = G.b0, w1 = G.w1, b1 = G.b1;
    const int slot = (gi - 1) % 3;
    auto anti_of = [&](const uint64_t* kx, const uint64_t* kz) -> bool {
      if constexpr (TYPE == GATE_X1) return (pick<W>(kz, w0) >> b0) & 1u;
      else if constexpr (TYPE == GATE_ZZ) return ((pick<W>(kx, w0) >> b0) ^ (pick<W>(kx, w1) >> b1)) & 1u;
      else return anticommutes<W>(kx, kz, m);
    };
    auto flip = [&](const uint64_t* kx, const uint64_t* kz, uint64_t* qx, uint64_t* qz) {
#pragma unroll
      for (int w = 0; w < W; ++w) { qx[w] = kx[w]; qz[w] = kz[w]; }
      if constexpr (TYPE == GATE_X1) {
#pragma unroll
        for (int w = 0; w < W; ++w) if (w == w0) qx[w] ^= 1ULL << b0;
      } else if constexpr (TYPE == GATE_ZZ) {
#pragma unroll
        for (int w = 0; w < W; ++w) {
          if (w == w0) qz[w] ^= 1ULL << b0;
          if (w == w1) qz[w] ^= 1ULL << b1;
        }
      } else {
#pragma unroll
        for (int w = 0; w < W; ++w) { qx[w] ^= m[w]; qz[w] ^= m[W + w]; }
      }
    };
    // sign of i R P = -Q for an anticommuting P (see irp_negative for the general rule):
    // X_j: negative iff P has X or Y... i.e. x_j = 1 (Y -> Z);  Z_a Z_b: negative iff the
    // qubit carrying x has z = 0 there.
    auto neg_of = [&](const uint64_t* kx, const uint64_t* kz) -> bool {
      if constexpr (TYPE == GATE_X1) return (pick<W>(kx, w0) >> b0) & 1u;
      else if constexpr (TYPE == GATE_ZZ) {
        const bool xa = (pick<W>(kx, w0) >> b0) & 1u;
        const uint64_t zq = xa ? (pick<W>(kz, w0) >> b0) : (pick<W>(kz, w1) >> b1);
        return (zq & 1u) == 0;
      } else return irp_negative<W>(kx, kz, m, G.rr_phase);
    };
    auto is_leader = [&](const uint64_t* kx, const uint64_t* kz) -> bool {
      if constexpr (TYPE == GATE_X1) return ((pick<W>(kx, w0) >> b0) & 1u) == 0;
      else if constexpr (TYPE == GATE_ZZ) return ((pick<W>(kz, w0) >> b0) & 1u) == 0;
      else {
        const uint64_t piv = G.pivot_word < W ? pick<W>(kx, G.pivot_word) : pick<W>(kz, G.pivot_word - W);
        return ((piv >> G.pivot_bit) & 1u) == 0;
      }
    };

    bool act[R];
    uint32_t hs[R], hf[R], hv[R];
    double cv[R];
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const uint32_t i = (uint32_t)r * BLOCK + tid;
      act[r] = false;
      if ((uint32_t)r * BLOCK >= nn) continue;   // uniform: the whole round is empty
      act[r] = i < nn && anti_of(rkx[r], rkz[r]);
      hs[r] = 0; hf[r] = 0; hv[r] = EMPTY; cv[r] = 0.0;
      if (act[r]) {
        cv[r] = (double)sc[i];
        if (snd != 0.0) {
          const uint32_t fh = full_hash(rh[r] ^ ghash, rko[r]);
          hs[r] = slot_of(fh);
          hf[r] = fp_of(fh);
          hv[r] = hidx[hs[r]];
        }
      }
    }
    bool app[R];
    double childv[R];
    uint32_t zeroed = 0;
    int dl = 0;   // live-count change from updates in place
#pragma unroll
    for (int r = 0; r < R; ++r) {
      app[r] = false;
      childv[r] = 0.0;
      if (!act[r]) continue;
      const uint32_t i = (uint32_t)r * BLOCK + tid;
      const double c = cv[r];
      if (snd == 0.0) {   // sin = 0: the Pauli is only scaled (Clifford, |cos| = 1)
        sc[i] = (CT)(c * cs);
        continue;
      }
      uint64_t qx[W], qz[W];
      flip(rkx[r], rkz[r], qx, qz);
      const uint32_t p = resolve(hs[r], hf[r], hv[r], qx, qz, rko[r]);
      if (p == EMPTY) {
        if (c == 0.0) continue;
        const bool neg_i = neg_of(rkx[r], rkz[r]);
        double ni = c * cs;
        const double child = (neg_i ? -c : c) * snd;
        if (ni == 0.0 || fabs(ni) < thr) {
          dropped += fabs(ni);
          ni = 0.0;
          ++zeroed;
          --dl;
        }
        sc[i] = (CT)ni;
        if (!(fabs(child) < thr) && child != 0.0) {
          app[r] = true;
          childv[r] = child;
        } else {
          dropped += fabs(child);
        }
      } else {
        if (!is_leader(rkx[r], rkz[r])) continue;   // the partner leads this pair
        const bool neg_i = neg_of(rkx[r], rkz[r]);
        const bool neg_p = neg_of(qx, qz);
        const double cp = (double)sc[p];
        double ni = c * cs + (neg_p ? -cp : cp) * snd;
        double np = cp * cs + (neg_i ? -c : c) * snd;
        if (fabs(ni) < thr || ni == 0.0) {
          dropped += fabs(ni);
          if (c != 0.0) ++zeroed;
          ni = 0.0;
        }
        if (fabs(np) < thr || np == 0.0) {
          dropped += fabs(np);
          if (cp != 0.0) ++zeroed;
          np = 0.0;
        }
        dl += (ni != 0.0) - (c != 0.0) + (np != 0.0) - (cp != 0.0);
        sc[i] = (CT)ni;
        sc[p] = (CT)np;
      }
    }
    // stage 3: one shared-counter atomic per wavefront for its queued children
    const uint64_t lt = lanemask_lt();
    const int lane = tid & 63;
#pragma unroll
    for (int r = 0; r < R; ++r) {
      if ((uint32_t)r * BLOCK >= nn) continue;
      const uint64_t bal = __ballot(app[r]);
      if (bal == 0) continue;
      const int leader = __ffsll((unsigned long long)bal) - 1;
      uint32_t base = 0;
      if (lane == leader) base = atomicAdd(&s_cnt[slot], (uint32_t)__popcll(bal));
      base = __shfl(base, leader, 64);
      if (app[r]) {
        const uint32_t j = nn + base + (uint32_t)__popcll(bal & lt);
        if (j < (uint32_t)CAP) {
          uint64_t qx[W], qz[W];
          flip(rkx[r], rkz[r], qx, qz);
#pragma unroll
          for (int w = 0; w < W; ++w) { sx[w][j] = qx[w]; sz[w][j] = qz[w]; }
          if (ORD) so[j] = (uint8_t)rko[r];
          sc[j] = (CT)childv[r];
          const uint32_t hq = rh[r] ^ ghash;
          sh[j] = hq;
          __threadfence_block();
          insert_h(j, full_hash(hq, rko[r]));
        } else {
          s_ovf = 1;
        }
      }
    }
    uint32_t zs = zeroed;
    for (int d = 32; d >= 1; d >>= 1) zs += __shfl_xor(zs, d, 64);
    if (lane == 0 && zs) atomicAdd(&s_dead[slot], zs);
    for (int d = 32; d >= 1; d >>= 1) dl += __shfl_xor(dl, d, 64);
    if (lane == 0 && dl) atomicAdd(&s_ldelta[slot], dl);
  };

  // ---- gates: one pass and one barrier per gate ------------------------------------------------
  for (int g = 0; g < a.ngates; ++g) {
    if (g % GATES == 0) {   // stage the next chunk of gate records
      __syncthreads();
      const int cnt = a.ngates - g < GATES ? a.ngates - g : GATES;
      for (int j = tid; j < cnt; j += BLOCK) sgate[j] = to_compact<W>(a.gates[g + j]);
      __syncthreads();
    }
    const GateC<W> G = sgate[g % GATES];
    const bool clifford = G.clifford != 0;
    uint64_t touch = 0;
#pragma unroll
    for (int w = 0; w < W; ++w) touch |= (orx[w] & G.m[W + w]) | (orz[w] & G.m[w]);
    if (!touch) {   // no entry of this tile anticommutes with the gate
      if (!clifford && !thresholded_all) threshold_all();
      continue;
    }
    // reclaim zeroed slots when the table is filling up and enough of them are dead
    if (n > (uint32_t)(3 * CAP / 4) && dead * 8 > n) {
      n = compact(n, 0.0, true);
      dead = 0;
      reload(0, n);
    }
    const int slot = gi % 3;
    if (tid == 0) { s_cnt[(gi + 1) % 3] = 0; s_dead[(gi + 1) % 3] = 0; s_ldelta[(gi + 1) % 3] = 0; }
    ++gi;
    if (G.type == GATE_X1) gate_pass(std::integral_constant<int, GATE_X1>{}, G, n);
    else if (G.type == GATE_ZZ) gate_pass(std::integral_constant<int, GATE_ZZ>{}, G, n);
    else gate_pass(std::integral_constant<int, GATE_GENERIC>{}, G, n);
    __syncthreads();
    if (s_ovf) {
      overflow_exit();
      return;
    }
    const uint32_t n_old = n;
    n += s_cnt[slot];
    dead += s_dead[slot];
    live += (int64_t)s_cnt[slot] + s_ldelta[slot];
    peak = n > peak ? n : peak;
    if (n > n_old) reload(n_old, n);
    if (!clifford && !thresholded_all) threshold_all();
    live_peak = live > (int64_t)live_peak ? (uint32_t)live : live_peak;
  }
  if (a.any_nonclifford && !thresholded_all) threshold_all();

  // ---- noise -------------------------------------------------------------------------------
  if (a.has_noise) {
    const NoiseDev nd = a.noise;
    if (nd.mode == 0) {
      for (int r = 0; r < R; ++r) {
        const uint32_t i = (uint32_t)r * BLOCK + tid;
        if (i >= n) break;
        const double c = (double)sc[i];
        if (c == 0.0) continue;
        uint64_t kx[W], kz[W];
        load_key(i, kx, kz);
        sc[i] = (CT)(c * noise_factor<W>(kx, kz, nd.tab, nd.sup, nd.qoff, nd.qent, nd));
      }
      __syncthreads();
    } else if (ORD) {
      const int M = nd.max_order;
      __syncthreads();
      if (tid == 0) s_cnt[0] = 0;
      __syncthreads();
      for (int r = 0; r < R; ++r) {
        const uint32_t i = (uint32_t)r * BLOCK + tid;
        if (i >= n) break;
        uint64_t kx[W], kz[W];
        load_key(i, kx, kz);
        const uint32_t oi = so[i];
        const uint32_t hstr = sh[i];
        bool leader = true;
        for (uint32_t o = 0; o < oi && leader; ++o)
          if (lookup_h(full_hash(hstr, o), kx, kz, o) != EMPTY) leader = false;
        if (!leader) continue;
        double p[kMaxPowerSums], e[kMaxPowerSums + 1];
        noise_sums<W>(kx, kz, nd, M, p);
        elementary_from_power(p, M, e);
        uint32_t idx[kMaxPowerSums + 1];
        double val[kMaxPowerSums + 1];
#pragma unroll
        for (int o = 0; o <= kMaxPowerSums; ++o) {
          idx[o] = EMPTY;
          val[o] = 0.0;
          if (o <= M && (uint32_t)o >= oi) {
            idx[o] = lookup_h(full_hash(hstr, (uint32_t)o), kx, kz, (uint32_t)o);
            val[o] = idx[o] == EMPTY ? 0.0 : (double)sc[idx[o]];
          }
        }
#pragma unroll
        for (int o = kMaxPowerSums; o >= 0; --o) {
          if (o > M) continue;
          double acc = 0.0;
          for (int j = 0; j <= o; ++j) acc += val[o - j] * e[j];
          if (idx[o] != EMPTY) {
            sc[idx[o]] = (CT)acc;
          } else if (acc != 0.0) {
            const uint32_t j = n + atomicAdd(&s_cnt[0], 1u);
            if (j < (uint32_t)CAP) {
#pragma unroll
              for (int w = 0; w < W; ++w) { sx[w][j] = kx[w]; sz[w][j] = kz[w]; }
              so[j] = (uint8_t)o;
              sc[j] = (CT)acc;
              sh[j] = hstr;
            } else {
              s_ovf = 1;
            }
          }
        }
      }
      __syncthreads();
      if (s_ovf) {
        overflow_exit();
        return;
      }
      n += s_cnt[0];
      peak = n > peak ? n : peak;
      __syncthreads();
      n = compact(n, a.eps_noise, false);
    }
  }

  // ---- pack the live entries and write them out ---------------------------------------------
  n = compact(n, 0.0, false);
  if (tid == 0) {
    // One fetch-add per tile.  Ranges are handed out in order, so when the buffer runs out
    // every tile from the first that does not fit on is refused; the host keeps the prefix
    // below the smallest refused start (out_fail) and retries the refused tiles.
    const unsigned long long old = n ? atomicAdd(a.out_count, (unsigned long long)n) : 0ULL;
    if (old + n <= a.out.stride) {
      s_base = old;
    } else {
      s_base = ~0ULL;
      atomicMin(a.out_fail, old);
    }
  }
  {
    double v = dropped;
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) v += __shfl_xor(v, d, 64);
    if ((tid & 63) == 0) s_drop[tid >> 6] = v;
  }
  __syncthreads();
  const unsigned long long base = s_base;
  if (base == ~0ULL) {
    if (tid == 0) {
      const uint32_t k = atomicAdd(a.ovf_count, 1u);
      a.ovf_tiles[k] = tile | kOvfOutput;
    }
    return;
  }
  if (tid == 0) {
    double v = 0.0;
    for (int w = 0; w < BLOCK / 64; ++w) v += s_drop[w];
    const uint32_t slot = blockIdx.x % kStatSlots;
    if (v != 0.0) atomicAdd(&a.dropped[slot], v);
    atomicMax(&a.peak[slot], peak);
    if (a.peak_sum) atomicAdd(&a.peak_sum[slot], (unsigned long long)live_peak);
  }
  for (uint32_t i = tid; i < n; i += BLOCK) {
    const uint64_t j = base + i;
#pragma unroll
    for (int w = 0; w < W; ++w) {
      a.out.x[w * a.out.stride + j] = sx[w][i];
      a.out.z[w * a.out.stride + j] = sz[w][i];
    }
    a.out.c[j] = sc[i];
    if (ORD) a.out.o[j] = so[i];
  }
}

// Tile boundaries without walking long classes: flag the first term of every class, list
// the flagged positions (a scan), and give tile t the first class start at or after t * T.
template <int W, class CT>
__global__ void k_class_flags(Terms<CT> t, uint64_t n, GroupMask gm, uint64_t kmask, uint32_t* flag) {
  const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  auto hk = [&](uint64_t j) {
    uint64_t xs[W], zs[W];
#pragma unroll
    for (int w = 0; w < W; ++w) { xs[w] = t.x[w * t.stride + j]; zs[w] = t.z[w * t.stride + j]; }
    return group_hash<W>(xs, zs, gm.mx, gm.mz) & kmask;
  };
  flag[i] = (i == 0 || hk(i) != hk(i - 1)) ? 1u : 0u;
}

__global__ void k_scatter_flagged(const uint32_t* flag, const uint32_t* pos, uint64_t n, uint32_t* list) {
  const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n && flag[i]) list[pos[i]] = (uint32_t)i;
}

__global__ void k_tile_starts(const uint32_t* bnd, uint32_t nb, uint64_t n, uint64_t T, uint32_t ntiles,
                              uint32_t* start) {
  const uint32_t t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t > ntiles) return;
  const uint64_t target = (uint64_t)t * T;
  if (t == 0) { start[0] = 0; return; }
  if (target >= n) { start[t] = (uint32_t)n; return; }
  uint32_t lo = 0, hi = nb;   // first boundary >= target
  while (lo < hi) {
    const uint32_t mid = (lo + hi) >> 1;
    if (bnd[mid] < target) lo = mid + 1;
    else hi = mid;
  }
  start[t] = lo < nb ? bnd[lo] : (uint32_t)n;
}

// ------------------------------------------------------------------------------------------
// Elementwise kernels.
// ------------------------------------------------------------------------------------------
// Bytes of LDS a noise descriptor needs when staged (table, then supports).
inline size_t noise_lds_bytes(const NoiseDev& nd) {
  return (size_t)nd.ntab * sizeof(double) + (size_t)nd.nsup * sizeof(SupportDev) +
         (nd.nq ? (size_t)(nd.nq + 1) * 4 + (size_t)nd.nqent * 4 : 0);
}
constexpr size_t kNoiseLdsMax = 64 * 1024;

// LDS layout of a staged noise descriptor: tab (doubles), supports, then (when built) the
// per-qubit support lists.
__device__ __forceinline__ void stage_noise(const NoiseDev& nd, double* stab, SupportDev* ssup) {
  for (int j = threadIdx.x; j < nd.ntab; j += blockDim.x) stab[j] = nd.tab[j];
  for (int j = threadIdx.x; j < nd.nsup; j += blockDim.x) ssup[j] = nd.sup[j];
  if (nd.nq) {
    int32_t* qo = (int32_t*)(ssup + nd.nsup);
    uint32_t* qe = (uint32_t*)(qo + nd.nq + 1);
    for (int j = threadIdx.x; j <= nd.nq; j += blockDim.x) qo[j] = nd.qoff[j];
    for (int j = threadIdx.x; j < nd.nqent; j += blockDim.x) qe[j] = nd.qent[j];
  }
}
__device__ __forceinline__ const int32_t* staged_qoff(const NoiseDev& nd, const SupportDev* ssup) {
  return nd.nq ? (const int32_t*)(ssup + nd.nsup) : nullptr;
}
__device__ __forceinline__ const uint32_t* staged_qent(const NoiseDev& nd, const SupportDev* ssup) {
  return nd.nq ? (const uint32_t*)((const int32_t*)(ssup + nd.nsup) + nd.nq + 1) : nullptr;
}

// A layer made only of Clifford rotations maps every string to one string (no merging):
// apply the gates (staged in LDS) in order in registers, optionally followed by the
// greedy-mode rescale (tables staged in dynamic LDS after the gates).
template <int W, class CT, bool ORD>
__global__ void __launch_bounds__(1024) k_clifford(Terms<CT> t, uint64_t n, const GateDev* gates, int ngates,
                                                  int has_noise, NoiseDev nd) {
  extern __shared__ double dsm[];
  GateDev* sg = (GateDev*)dsm;
  double* stab = (double*)(sg + ngates);
  SupportDev* ssup = (SupportDev*)(stab + (has_noise ? nd.ntab : 0));
  for (int j = threadIdx.x; j < ngates; j += blockDim.x) sg[j] = gates[j];
  if (has_noise) stage_noise(nd, stab, ssup);
  __syncthreads();
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (uint64_t)gridDim.x * blockDim.x) {
    uint64_t kx[W], kz[W];
#pragma unroll
    for (int w = 0; w < W; ++w) { kx[w] = t.x[w * t.stride + i]; kz[w] = t.z[w * t.stride + i]; }
    double c = (double)t.c[i];
    for (int g = 0; g < ngates; ++g) {
      uint64_t m[2 * W];
#pragma unroll
      for (int w = 0; w < 2 * W; ++w) m[w] = sg[g].m[w];
      if (!anticommutes<W>(kx, kz, m)) continue;
      const double snd = sg[g].sn_dir;
      if (snd == 0.0) {
        c = c * sg[g].cs;
      } else {
        const bool neg = irp_negative<W>(kx, kz, m, sg[g].rr_phase);
        c = (neg ? -c : c) * snd;
#pragma unroll
        for (int w = 0; w < W; ++w) { kx[w] ^= m[w]; kz[w] ^= m[W + w]; }
      }
    }
    if (has_noise) c = c * noise_factor<W>(kx, kz, stab, ssup, staged_qoff(nd, ssup), staged_qent(nd, ssup), nd);
#pragma unroll
    for (int w = 0; w < W; ++w) { t.x[w * t.stride + i] = kx[w]; t.z[w * t.stride + i] = kz[w]; }
    t.c[i] = (CT)c;
  }
}

template <int W, class CT>
__global__ void __launch_bounds__(1024) k_noise_greedy(Terms<CT> t, uint64_t n, NoiseDev nd) {
  extern __shared__ double dsm[];
  double* stab = dsm;
  SupportDev* ssup = (SupportDev*)(stab + nd.ntab);
  stage_noise(nd, stab, ssup);
  __syncthreads();
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (uint64_t)gridDim.x * blockDim.x) {
    uint64_t kx[W], kz[W];
#pragma unroll
    for (int w = 0; w < W; ++w) { kx[w] = t.x[w * t.stride + i]; kz[w] = t.z[w * t.stride + i]; }
    const double c = (double)t.c[i];
    t.c[i] = (CT)(c * noise_factor<W>(kx, kz, stab, ssup, staged_qoff(nd, ssup), staged_qent(nd, ssup), nd));
  }
}

}  // namespace pp
