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

namespace pp {

template <int W>
struct LayerCfg;
template <>
struct LayerCfg<1> { static constexpr int CAP = 4096, BLOCK = 512; };
template <>
struct LayerCfg<2> { static constexpr int CAP = 2048, BLOCK = 512; };
template <>
struct LayerCfg<3> { static constexpr int CAP = 2048, BLOCK = 512; };
template <>
struct LayerCfg<4> { static constexpr int CAP = 1024, BLOCK = 256; };

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
  unsigned long long* out_count;
  uint32_t* ovf_tiles;
  uint32_t* ovf_count;
  double* dropped;              // sum of |c| removed by thresholds
  unsigned int* peak;           // largest live count seen in a tile
};

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
template <int W, class CT, bool ORD>
__global__ void __launch_bounds__(LayerCfg<W>::BLOCK) k_layer(LayerArgs<CT> a) {
  constexpr int CAP = LayerCfg<W>::CAP;
  constexpr int BLOCK = LayerCfg<W>::BLOCK;
  constexpr int H = 2 * CAP;
  constexpr int R = CAP / BLOCK;
  constexpr uint32_t EMPTY = 0xffffffffu;

  __shared__ uint64_t sx[W][CAP];
  __shared__ uint64_t sz[W][CAP];
  __shared__ CT sc[CAP];
  __shared__ uint8_t so[ORD ? CAP : 1];
  __shared__ uint32_t hidx[H];
  __shared__ uint32_t s_cnt[3];      // appends of gate g land in s_cnt[g % 3]
  __shared__ uint32_t s_dead[3];     // entries zeroed by gate g
  __shared__ uint32_t s_ovf;
  __shared__ unsigned long long s_or[2 * W];
  __shared__ uint32_t stmp[BLOCK / 64];
  __shared__ unsigned long long s_base;
  __shared__ double s_drop[BLOCK / 64];

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

  auto slot_of = [&](const uint64_t* kx, const uint64_t* kz, uint32_t o) -> uint32_t {
    uint64_t h = 0x9e3779b97f4a7c15ULL * (o + 1);
#pragma unroll
    for (int w = 0; w < W; ++w) {
      h = (h ^ kx[w]) * 0xff51afd7ed558ccdULL;
      h = (h ^ kz[w]) * 0xc4ceb9fe1a85ec53ULL;
    }
    return (uint32_t)(h >> 40) & (H - 1);
  };
  auto same_key = [&](uint32_t idx, const uint64_t* kx, const uint64_t* kz, uint32_t o) -> bool {
    bool eq = true;
#pragma unroll
    for (int w = 0; w < W; ++w) eq = eq && sx[w][idx] == kx[w] && sz[w][idx] == kz[w];
    if (ORD) eq = eq && so[idx] == o;
    return eq;
  };
  auto lookup = [&](const uint64_t* kx, const uint64_t* kz, uint32_t o) -> uint32_t {
    uint32_t h = slot_of(kx, kz, o);
    for (int probe = 0; probe < H; ++probe) {
      const uint32_t idx = hidx[h];
      if (idx == EMPTY) return EMPTY;
      if (same_key(idx, kx, kz, o)) return idx;
      h = (h + 1) & (H - 1);
    }
    return EMPTY;
  };
  auto insert_key = [&](uint32_t i, const uint64_t* kx, const uint64_t* kz, uint32_t o) {
    uint32_t h = slot_of(kx, kz, o);
    for (int probe = 0; probe < H; ++probe) {
      if (atomicCAS(&hidx[h], EMPTY, i) == EMPTY) return;
      h = (h + 1) & (H - 1);
    }
  };
  auto insert = [&](uint32_t i) {
    uint64_t kx[W], kz[W];
#pragma unroll
    for (int w = 0; w < W; ++w) { kx[w] = sx[w][i]; kz[w] = sz[w][i]; }
    insert_key(i, kx, kz, ORD ? so[i] : 0u);
  };
  auto load_key = [&](uint32_t i, uint64_t* kx, uint64_t* kz) {
#pragma unroll
    for (int w = 0; w < W; ++w) { kx[w] = sx[w][i]; kz[w] = sz[w][i]; }
  };

  // ---- load the tile -----------------------------------------------------------------------
  uint64_t lor[2 * W];
#pragma unroll
  for (int w = 0; w < 2 * W; ++w) lor[w] = 0;
  for (uint32_t i = tid; i < n0; i += BLOCK) {
#pragma unroll
    for (int w = 0; w < W; ++w) {
      const uint64_t xv = a.in.x[w * a.in.stride + t0 + i];
      const uint64_t zv = a.in.z[w * a.in.stride + t0 + i];
      sx[w][i] = xv;
      sz[w][i] = zv;
      lor[w] |= xv;
      lor[W + w] |= zv;
    }
    sc[i] = a.in.c[t0 + i];
    if (ORD) so[i] = a.in.o[t0 + i];
  }
  for (uint32_t j = tid; j < (uint32_t)H; j += BLOCK) hidx[j] = EMPTY;
  if (tid < 2 * W) s_or[tid] = 0;
  if (tid < 3) { s_cnt[tid] = 0; s_dead[tid] = 0; }
  if (tid == 0) s_ovf = 0;
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
  // (x_any & z_R) | (z_any & x_R) is nonzero.  Gates keep the group's invariant bits, so
  // for X-type (Z-type) runs the z (x) part of this mask stays exact; otherwise it is
  // refreshed below after every gate that moved bits.
  uint64_t orx[W], orz[W];
#pragma unroll
  for (int w = 0; w < W; ++w) { orx[w] = s_or[w]; orz[w] = s_or[W + w]; }

  uint32_t n = n0;
  uint32_t peak = n0;
  uint32_t dead = 0;
  double dropped = 0.0;
  bool thresholded_all = false;
  int gi = 0;   // processed-gate counter (rotates the shared counters)

  // Compaction of entries [0, nn) keeping c != 0 and !(|c| < thr); optionally rebuilds the
  // hash index.  Uniform call.
  auto compact = [&](uint32_t nn, double thr, bool rebuild) -> uint32_t {
    uint64_t rx[R][W], rz[R][W];
    CT rc[R];
    uint8_t ro[R];
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
    for (int r = 0; r < R; ++r) {
      const uint32_t i = (uint32_t)r * BLOCK + tid;
      if (i >= n) break;
      const double v = (double)sc[i];
      if (v != 0.0 && fabs(v) < a.eps) {
        dropped += fabs(v);
        sc[i] = (CT)0.0;
        ++nd;
      }
    }
    if (__syncthreads_or(nd)) dead += 1;   // barrier; zeros now exist, so compaction may run
  };

  // ---- gates: one pass and one barrier per gate ------------------------------------------------
  for (int g = 0; g < a.ngates; ++g) {
    uint64_t m[2 * W];
#pragma unroll
    for (int w = 0; w < 2 * W; ++w) m[w] = a.gates[g].m[w];
    const bool clifford = a.gates[g].clifford != 0;
    uint64_t touch = 0;
#pragma unroll
    for (int w = 0; w < W; ++w) touch |= (orx[w] & m[W + w]) | (orz[w] & m[w]);
    if (!touch) {   // no entry of this tile anticommutes with the gate
      if (!clifford && !thresholded_all) threshold_all();
      continue;
    }
    const double cs = a.gates[g].cs;
    const double snd = a.gates[g].sn_dir;
    const int pw = a.gates[g].pivot_word;
    const int pb = a.gates[g].pivot_bit;
    const int rrp = a.gates[g].rr_phase;
    const double thr = clifford ? 0.0 : a.eps;
    const int slot = gi % 3;
    // keep room: at most n appends can happen in this gate
    if (n + n > (uint32_t)CAP && dead > 0) {
      n = compact(n, 0.0, true);
      dead = 0;
    }
    if (tid == 0) { s_cnt[(gi + 1) % 3] = 0; s_dead[(gi + 1) % 3] = 0; }
    ++gi;
    for (int r = 0; r < R; ++r) {
      const uint32_t i = (uint32_t)r * BLOCK + tid;
      if (i >= n) break;
      uint64_t kx[W], kz[W];
      load_key(i, kx, kz);
      if (!anticommutes<W>(kx, kz, m)) continue;
      const double c = (double)sc[i];
      if (snd == 0.0) {   // sin = 0: the Pauli is only scaled (Clifford, |cos| = 1)
        sc[i] = (CT)(c * cs);
        continue;
      }
      uint64_t qx[W], qz[W];
#pragma unroll
      for (int w = 0; w < W; ++w) { qx[w] = kx[w] ^ m[w]; qz[w] = kz[w] ^ m[W + w]; }
      const uint32_t oi = ORD ? so[i] : 0u;
      const uint32_t p = lookup(qx, qz, oi);
      const bool neg_i = irp_negative<W>(kx, kz, m, rrp);
      if (p == EMPTY) {
        if (c == 0.0) continue;
        double ni = c * cs;
        const double child = (neg_i ? -c : c) * snd;
        if (ni == 0.0 || fabs(ni) < thr) {
          dropped += fabs(ni);
          ni = 0.0;
          atomicAdd(&s_dead[slot], 1u);
        }
        sc[i] = (CT)ni;
        if (!(fabs(child) < thr) && child != 0.0) {
          const uint32_t j = n + atomicAdd(&s_cnt[slot], 1u);
          if (j < (uint32_t)CAP) {
#pragma unroll
            for (int w = 0; w < W; ++w) { sx[w][j] = qx[w]; sz[w][j] = qz[w]; }
            if (ORD) so[j] = (uint8_t)oi;
            sc[j] = (CT)child;
            __threadfence_block();
            insert_key(j, qx, qz, oi);
          } else {
            s_ovf = 1;
          }
        } else {
          dropped += fabs(child);
        }
      } else {
        const uint64_t piv = pw < W ? pick<W>(kx, pw) : pick<W>(kz, pw - W);
        if ((piv >> pb) & 1u) continue;   // the partner leads this pair
        const bool neg_p = irp_negative<W>(qx, qz, m, rrp);
        const double cp = (double)sc[p];
        double ni = c * cs + (neg_p ? -cp : cp) * snd;
        double np = cp * cs + (neg_i ? -c : c) * snd;
        if (fabs(ni) < thr || ni == 0.0) {
          dropped += fabs(ni);
          if (c != 0.0) atomicAdd(&s_dead[slot], 1u);
          ni = 0.0;
        }
        if (fabs(np) < thr || np == 0.0) {
          dropped += fabs(np);
          if (cp != 0.0) atomicAdd(&s_dead[slot], 1u);
          np = 0.0;
        }
        sc[i] = (CT)ni;
        sc[p] = (CT)np;
      }
    }
    __syncthreads();
    if (s_ovf) {
      overflow_exit();
      return;
    }
    n += s_cnt[slot];
    dead += s_dead[slot];
    peak = n > peak ? n : peak;
    if (!clifford && !thresholded_all) threshold_all();
    if (a.gate_kind == 2) {
      // a general gate moves both x and z bits: refresh the OR masks from the live entries
#pragma unroll
      for (int w = 0; w < W; ++w) { orx[w] |= m[w]; orz[w] |= m[W + w]; }
    }
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
        double p[kMaxPowerSums];
        noise_sums<W>(kx, kz, nd, 1, p);
        sc[i] = (CT)(c * exp(2.0 * nd.sign * p[0]));
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
        bool leader = true;
        for (uint32_t o = 0; o < oi && leader; ++o)
          if (lookup(kx, kz, o) != EMPTY) leader = false;
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
            idx[o] = lookup(kx, kz, (uint32_t)o);
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
    unsigned long long old = *((volatile unsigned long long*)a.out_count);
    unsigned long long got = ~0ULL;
    while (old + n <= a.out.stride) {
      const unsigned long long prev = atomicCAS(a.out_count, old, old + n);
      if (prev == old) { got = old; break; }
      old = prev;
    }
    s_base = got;
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
    if (v != 0.0) atomicAdd(a.dropped, v);
    atomicMax(a.peak, peak);
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

// ------------------------------------------------------------------------------------------
// Tile boundaries after the group-hash sort: tile t starts at the first class boundary at or
// after t * T (class = equal low k bits of the group hash).
// ------------------------------------------------------------------------------------------
template <int W, class CT>
__global__ void k_tiles(Terms<CT> t, uint64_t n, GroupMask gm, uint64_t kmask, uint64_t T, uint32_t ntiles,
                        uint32_t* start) {
  const uint32_t tile = blockIdx.x * blockDim.x + threadIdx.x;
  if (tile > ntiles) return;
  if (tile == 0) { start[0] = 0; return; }
  uint64_t i = (uint64_t)tile * T;
  if (i >= n) { start[tile] = (uint32_t)n; return; }
  auto hk = [&](uint64_t j) {
    uint64_t xs[W], zs[W];
#pragma unroll
    for (int w = 0; w < W; ++w) { xs[w] = t.x[w * t.stride + j]; zs[w] = t.z[w * t.stride + j]; }
    return group_hash<W>(xs, zs, gm.mx, gm.mz) & kmask;
  };
  const uint64_t prev = hk(i - 1);
  while (i < n && hk(i) == prev) ++i;
  start[tile] = (uint32_t)i;
}

// ------------------------------------------------------------------------------------------
// Elementwise kernels.
// ------------------------------------------------------------------------------------------
// Bytes of LDS a noise descriptor needs when staged (table, then supports).
inline size_t noise_lds_bytes(int ntab, int nsup) {
  return (size_t)ntab * sizeof(double) + (size_t)nsup * sizeof(SupportDev);
}
constexpr size_t kNoiseLdsMax = 64 * 1024;

// Greedy-mode rescale with the support tables staged in LDS: the exponent is a sum of one
// table value per support (one or two qubits) plus the generators with larger support.
template <int W>
__device__ __forceinline__ double noise_exponent_lds(const uint64_t* px, const uint64_t* pz, const double* stab,
                                                     const SupportDev* ssup, const NoiseDev& nd) {
  double acc = 0.0;
  for (int s = 0; s < nd.nsup; ++s) {
    const SupportDev sp = ssup[s];
    uint32_t pat = (uint32_t)((pick<W>(px, sp.w0) >> sp.b0) & 1u) | (uint32_t)(((pick<W>(pz, sp.w0) >> sp.b0) & 1u) << 1);
    if (sp.w1 >= 0)
      pat |= (uint32_t)(((pick<W>(px, sp.w1) >> sp.b1) & 1u) << 2) | (uint32_t)(((pick<W>(pz, sp.w1) >> sp.b1) & 1u) << 3);
    acc += stab[sp.table + pat];   // pattern 0 (identity on the support) holds 0
  }
  for (int d = 0; d < nd.ndirect; ++d) {
    const uint64_t* m = nd.dm + (size_t)d * 2 * W;
    if (anticommutes<W>(px, pz, m)) acc += nd.dval[d];
  }
  return acc;
}

__device__ __forceinline__ void stage_noise(const NoiseDev& nd, double* stab, SupportDev* ssup) {
  for (int j = threadIdx.x; j < nd.ntab; j += blockDim.x) stab[j] = nd.tab[j];
  for (int j = threadIdx.x; j < nd.nsup; j += blockDim.x) ssup[j] = nd.sup[j];
}

// A layer made only of Clifford rotations maps every string to one string (no merging):
// apply the gates (staged in LDS) in order in registers, optionally followed by the
// greedy-mode rescale (tables staged in dynamic LDS after the gates).
template <int W, class CT, bool ORD>
__global__ void __launch_bounds__(256) k_clifford(Terms<CT> t, uint64_t n, const GateDev* gates, int ngates,
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
    if (has_noise) c = c * exp(2.0 * nd.sign * noise_exponent_lds<W>(kx, kz, stab, ssup, nd));
#pragma unroll
    for (int w = 0; w < W; ++w) { t.x[w * t.stride + i] = kx[w]; t.z[w * t.stride + i] = kz[w]; }
    t.c[i] = (CT)c;
  }
}

template <int W, class CT>
__global__ void __launch_bounds__(256) k_noise_greedy(Terms<CT> t, uint64_t n, NoiseDev nd) {
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
    t.c[i] = (CT)(c * exp(2.0 * nd.sign * noise_exponent_lds<W>(kx, kz, stab, ssup, nd)));
  }
}

}  // namespace pp
