// pp_misc.hpp -- per-gate path, segmented merge, cap selection, expectation (gfx950).
#pragma once

#include "pp_common.hpp"
#include "pp_layer.hpp"
#include "pp_sort.hpp"

namespace pp {

// ------------------------------------------------------------------------------------------
// Per-gate path (tiles that outgrow LDS, and general gates): every term writes two slots --
// itself (cos part, or unchanged if it commutes) and its sin child (or a zero placeholder) --
// then a canonical sort and a segmented sum merge equal strings.  sine_max >= 0 (sine-order
// mode): the sin child of a non-Clifford gate carries tag + 1 and is zeroed above sine_max.
// ------------------------------------------------------------------------------------------
template <int W, class CT, bool ORD>
__global__ void k_expand_gate(Terms<CT> in, uint64_t n, GateDev G, Terms<CT> out, int sine_max) {
  const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  uint64_t kx[W], kz[W], m[2 * W];
#pragma unroll
  for (int w = 0; w < W; ++w) { kx[w] = in.x[w * in.stride + i]; kz[w] = in.z[w * in.stride + i]; }
#pragma unroll
  for (int w = 0; w < 2 * W; ++w) m[w] = G.m[w];
  const double c = (double)in.c[i];
  const uint8_t o = ORD ? in.o[i] : 0;
  uint8_t ob = o;
  const uint64_t a = 2 * i, b = 2 * i + 1;
  double ca = c, cb = 0.0;
  uint64_t bx[W], bz[W];
#pragma unroll
  for (int w = 0; w < W; ++w) { bx[w] = kx[w]; bz[w] = kz[w]; }
  if (anticommutes<W>(kx, kz, m)) {
    ca = c * G.cs;
    if (G.sn_dir != 0.0) {
      const bool neg = irp_negative<W>(kx, kz, m, G.rr_phase);
      cb = (neg ? -c : c) * G.sn_dir;
#pragma unroll
      for (int w = 0; w < W; ++w) { bx[w] = kx[w] ^ m[w]; bz[w] = kz[w] ^ m[W + w]; }
      if (ORD && sine_max >= 0 && !G.clifford) {
        ob = (uint8_t)(o + 1);
        if ((int)ob > sine_max) cb = 0.0;
      }
    }
  }
#pragma unroll
  for (int w = 0; w < W; ++w) {
    out.x[w * out.stride + a] = kx[w];
    out.z[w * out.stride + a] = kz[w];
    out.x[w * out.stride + b] = bx[w];
    out.z[w * out.stride + b] = bz[w];
  }
  out.c[a] = (CT)ca;
  out.c[b] = (CT)cb;
  if (ORD) { out.o[a] = o; out.o[b] = ob; }
}

// Error-order noise for the per-gate path: term (P, o) writes M+1 slots (P, o+j, c e_j) for
// o + j <= M and zero placeholders otherwise.
template <int W, class CT, bool ORD>
__global__ void k_expand_noise(Terms<CT> in, uint64_t n, NoiseDev nd, Terms<CT> out) {
  const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int M = nd.max_order;
  uint64_t kx[W], kz[W];
#pragma unroll
  for (int w = 0; w < W; ++w) { kx[w] = in.x[w * in.stride + i]; kz[w] = in.z[w * in.stride + i]; }
  const double c = (double)in.c[i];
  const int o = ORD ? in.o[i] : 0;
  double p[kMaxPowerSums], e[kMaxPowerSums + 1];
  noise_sums<W>(kx, kz, nd, M, p);
  elementary_from_power(p, M, e);
  for (int j = 0; j <= M; ++j) {
    const uint64_t s = i * (uint64_t)(M + 1) + j;
#pragma unroll
    for (int w = 0; w < W; ++w) { out.x[w * out.stride + s] = kx[w]; out.z[w * out.stride + s] = kz[w]; }
    const bool ok = o + j <= M;
    out.c[s] = (CT)(ok ? c * e[j] : 0.0);
    if (ORD) out.o[s] = (uint8_t)(ok ? o + j : o);
  }
}

// Sum `v` over the (256-thread) block and add it to *dst once per block (dst may be null).
// Kernels using it run a grid-stride loop over a bounded grid, so the atomics stay few.
__device__ __forceinline__ void add_dropped(double v, double* dst) {
  __shared__ double part[4];
  for (int d = 32; d >= 1; d >>= 1) v += __shfl_xor(v, d, 64);
  if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = v;
  __syncthreads();
  if (threadIdx.x == 0 && dst) {
    const double t = (part[0] + part[1]) + (part[2] + part[3]);
    if (t != 0.0) atomicAdd(dst, t);
  }
}

template <int W, class CT, bool ORD>
__device__ __forceinline__ bool same_term(const Terms<CT>& t, uint64_t a, uint64_t b) {
  bool eq = true;
#pragma unroll
  for (int w = 0; w < W; ++w)
    eq = eq && t.x[w * t.stride + a] == t.x[w * t.stride + b] && t.z[w * t.stride + a] == t.z[w * t.stride + b];
  if (ORD) eq = eq && t.o[a] == t.o[b];
  return eq;
}

// Phase of a product of Hermitian Paulis, A B = i^k (A xor B), k mod 4.  Per qubit,
// XY = iZ, YZ = iX and ZX = iY contribute +i, the reverse orders -i, all other pairs 1.
template <int W>
__device__ __forceinline__ int herm_mul_phase(const uint64_t* ax, const uint64_t* az, const uint64_t* bx,
                                              const uint64_t* bz) {
  int k = 0;
#pragma unroll
  for (int w = 0; w < W; ++w) {
    const uint64_t aX = ax[w] & ~az[w], aY = ax[w] & az[w], aZ = ~ax[w] & az[w];
    const uint64_t bX = bx[w] & ~bz[w], bY = bx[w] & bz[w], bZ = ~bx[w] & bz[w];
    k += popc64((aX & bY) | (aY & bZ) | (aZ & bX)) - popc64((aX & bZ) | (aY & bX) | (aZ & bY));
  }
  return k & 3;
}

// Pair p (0-based) of the K(K-1)/2 unordered pairs a < b listed row by row (a = 0: b = 1..K-1,
// then a = 1, ...): row a starts at a (2K - a - 1) / 2.  The row comes from the quadratic's
// root in FP64 and is then corrected to the exact integer row, so any K below 2^26 works.
__device__ __forceinline__ void pair_of_index(uint64_t p, uint64_t K, uint32_t& a, uint32_t& b) {
  auto start = [&](uint64_t r) { return r * (2 * K - r - 1) / 2; };
  const double t = 2.0 * (double)K - 1.0;
  const double disc = t * t - 8.0 * (double)p;
  int64_t r = (int64_t)floor((t - sqrt(disc > 0.0 ? disc : 0.0)) * 0.5);
  if (r < 0) r = 0;
  if (r > (int64_t)K - 2) r = (int64_t)K - 2;
  while (r > 0 && start((uint64_t)r) > p) --r;
  while ((uint64_t)r + 1 < K - 1 && start((uint64_t)r + 1) <= p) ++r;
  a = (uint32_t)r;
  b = (uint32_t)(r + 1 + (int64_t)(p - start((uint64_t)r)));
}

// Expansion of one propagated antinoise map (Section I.A, Eq. applyantinoise):
// O -> id O + q E' O E' with E' = sum_a e_a P_a (K terms, in `e`; id = 1 - q for one map,
// other values for the terms of a batch).  Term i of O owns S = 1 + K(K-1)/2 consecutive
// output slots:
//  * slot 0: P_i with c_i [id + q sum_a e_a^2 (-1)^{<P_a, P_i>}]  (P_a P P_a = +-P);
//  * slot 1 + j, pair (a, b) = pair_of_index(j) with a < b: the two orders are adjoints of
//    each other, so P_a P P_b + P_b P P_a = 2 Re(i^k) R for P_a P P_b = i^k R: 2 q e_a e_b c_i
//    times +1 (k = 0) or -1 (k = 2), and 0 for odd k.
// keep[t] flags the nonzero slots, which are compacted before the canonical sort.
// Grid-stride over n * S slots, so consecutive threads write consecutive slots of every
// plane.
template <int W, class CT, bool ORD>
__global__ void k_expand_antinoise(Terms<CT> in, uint64_t n, Terms<CT> e, uint32_t K, uint64_t S, double q,
                                   double id, Terms<CT> out, uint32_t* keep) {
  const uint64_t total = n * S;
  for (uint64_t t = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; t < total;
       t += (uint64_t)gridDim.x * blockDim.x) {
    const uint64_t i = t / S;
    const uint64_t j = t - i * S;
    uint64_t px[W], pz[W], rx[W], rz[W];
#pragma unroll
    for (int w = 0; w < W; ++w) {
      px[w] = in.x[(size_t)w * in.stride + i];
      pz[w] = in.z[(size_t)w * in.stride + i];
      rx[w] = px[w];
      rz[w] = pz[w];
    }
    const double c = (double)in.c[i];
    double v = 0.0;
    if (j == 0) {
      double s = 0.0;
      for (uint32_t a = 0; a < K; ++a) {
        int par = 0;
#pragma unroll
        for (int w = 0; w < W; ++w)
          par += popc64(e.x[(size_t)w * e.stride + a] & pz[w]) + popc64(e.z[(size_t)w * e.stride + a] & px[w]);
        const double ea = (double)e.c[a];
        s += (par & 1) ? -ea * ea : ea * ea;
      }
      v = c * (id + q * s);
    } else {
      uint32_t a, b;
      pair_of_index(j - 1, K, a, b);
      uint64_t ax[W], az[W], bx[W], bz[W], tx[W], tz[W];
#pragma unroll
      for (int w = 0; w < W; ++w) {
        ax[w] = e.x[(size_t)w * e.stride + a];
        az[w] = e.z[(size_t)w * e.stride + a];
        bx[w] = e.x[(size_t)w * e.stride + b];
        bz[w] = e.z[(size_t)w * e.stride + b];
        tx[w] = ax[w] ^ px[w];
        tz[w] = az[w] ^ pz[w];
      }
      const int k = (herm_mul_phase<W>(ax, az, px, pz) + herm_mul_phase<W>(tx, tz, bx, bz)) & 3;
      if (!(k & 1)) v = (k == 0 ? 2.0 : -2.0) * q * (double)e.c[a] * (double)e.c[b] * c;
#pragma unroll
      for (int w = 0; w < W; ++w) {
        rx[w] = tx[w] ^ bx[w];
        rz[w] = tz[w] ^ bz[w];
      }
    }
#pragma unroll
    for (int w = 0; w < W; ++w) {
      out.x[(size_t)w * out.stride + t] = rx[w];
      out.z[(size_t)w * out.stride + t] = rz[w];
    }
    out.c[t] = (CT)v;
    if (ORD) out.o[t] = in.o[i];
    keep[t] = (CT)v != (CT)0 ? 1u : 0u;
  }
}

// ---- most significant products only (Appendix B, heuristic conjugation) --------------------
// The K(K-1)/2 unordered pairs a < b of E' (the products limited; the products with a = b
// are always kept) get the sort key x = ~bits(|e_a| |e_b|) (non-negative doubles order like
// their bit patterns, so ascending keys are descending magnitudes) and z = a << 32 | b, then
// are put in canonical order by the library's radix sort.
template <int W, class CT>
__global__ void k_pair_keys(const CT* ec, uint64_t K, uint64_t P, Terms<double> out) {
  for (uint64_t p = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; p < P; p += (uint64_t)gridDim.x * blockDim.x) {
    uint32_t a, b;
    pair_of_index(p, K, a, b);
    const double m = fabs((double)ec[a]) * fabs((double)ec[b]);
    out.x[p] = ~(uint64_t)__double_as_longlong(m);
    out.z[p] = ((uint64_t)a << 32) | b;
#pragma unroll
    for (int w = 1; w < W; ++w) {
      out.x[(size_t)w * out.stride + p] = 0;
      out.z[(size_t)w * out.stride + p] = 0;
    }
    out.c[p] = 0.0;
    out.o[p] = 0;
  }
}

// From the sorted pairs: magnitudes pm[p], indices pidx[p] = a << 32 | b, and each pair's
// weight w[p] (its ordered triplets per term: 1 for a = b, 2 otherwise).
__global__ void k_pair_tables(Terms<double> srt, uint64_t P, double* pm, uint64_t* pidx, uint32_t* w) {
  const uint64_t p = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= P) return;
  const uint64_t z = srt.z[p];
  pm[p] = __longlong_as_double((long long)~srt.x[p]);
  pidx[p] = z;
  w[p] = (z >> 32) == (z & 0xffffffffULL) ? 1u : 2u;
}

// cw[p] = weights before pair p (ws: their exclusive scan), cw[P] = all of them.
__global__ void k_pair_cw(const uint32_t* ws, const uint64_t* pidx, uint64_t P, uint64_t* cw) {
  const uint64_t p = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= P) return;
  cw[p] = ws[p];
  if (p == P - 1) {
    const uint64_t z = pidx[p];
    cw[P] = (uint64_t)ws[p] + ((z >> 32) == (z & 0xffffffffULL) ? 1u : 2u);
  }
}

// Unordered pairs p = (a <= b) of E' terms are sorted on the host by pm[p] = |e_a| |e_b|,
// largest first; cw[p] = sum of the pair weights before p (1 for a = b, 2 otherwise: the
// number of ordered triplets).  A triplet's magnitude is mu = |c_s| pm[p], non-increasing
// in p for a fixed term s, so the pairs with mu >= tau form a prefix of the list.
__device__ __forceinline__ uint32_t topk_prefix(double ac, const double* pm, uint32_t P, double tau) {
  uint32_t lo = 0, hi = P;   // first p with ac * pm[p] < tau
  while (lo < hi) {
    const uint32_t mid = lo + (hi - lo) / 2;
    if (ac * pm[mid] >= tau) lo = mid + 1; else hi = mid;
  }
  return lo;
}

// One workgroup: tau = the largest value with at least k triplets of mu >= tau, by
// bisection on the bit pattern of tau (order-preserving for non-negative doubles).  Every
// round ends in barriers that all waves reach; at most 64 rounds.
template <class CT>
__global__ void __launch_bounds__(1024) k_topk_cut(const CT* c, uint64_t n, const double* pm, const uint64_t* cw,
                                                   uint32_t P, uint64_t k, uint64_t hi_bits, double* tau_out) {
  __shared__ unsigned long long part[16];
  __shared__ uint64_t s_lo, s_hi;
  if (threadIdx.x == 0) { s_lo = 0; s_hi = hi_bits; }
  __syncthreads();
  for (int round = 0; round < 64; ++round) {
    const uint64_t lo = s_lo, hi = s_hi;
    if (hi - lo <= 1) break;
    const uint64_t mid = lo + (hi - lo) / 2;
    const double tau = __longlong_as_double((long long)mid);
    unsigned long long cnt = 0;
    for (uint64_t s = threadIdx.x; s < n; s += blockDim.x) cnt += cw[topk_prefix(fabs((double)c[s]), pm, P, tau)];
    for (int off = 32; off > 0; off >>= 1) cnt += __shfl_down(cnt, off);
    if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = cnt;
    __syncthreads();
    if (threadIdx.x == 0) {
      unsigned long long tot = 0;
      for (int w = 0; w < (int)(blockDim.x >> 6); ++w) tot += part[w];
      if (tot >= k) s_lo = mid; else s_hi = mid;
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) *tau_out = __longlong_as_double((long long)s_lo);
}

// Slots of term s: 1 (the (1 - q) c_s P_s part) + the pairs kept for it.  `total` (zeroed
// by the host) receives their exact 64-bit sum, one atomic per wavefront, so the host can
// reject an expansion whose 32-bit offsets would wrap.
template <class CT>
__global__ void k_topk_lens(const CT* c, uint64_t n, const double* pm, uint32_t P, const double* tau,
                            uint32_t* lens, unsigned long long* total) {
  const uint64_t s = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  unsigned long long v = 0;
  if (s < n) {
    v = 1u + topk_prefix(fabs((double)c[s]), pm, P, *tau);
    lens[s] = (uint32_t)v;
  }
  for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off);
  if ((threadIdx.x & 63) == 0 && v) atomicAdd(total, v);
}

// Expansion with the kept pairs only.  off[s] = first slot of term s (exclusive scan of
// lens).  Slot 0 of a term: P with c [(1 - q) + q sum_a e_a^2 (-1)^{<P_a, P>}] (every
// diagonal product, as in the exact update).  Pair (a, b), a < b: both orders,
// 2 Re(i^k) q e_a e_b c on R for P_a P P_b = i^k R.
template <int W, class CT, bool ORD>
__global__ void k_expand_topk(Terms<CT> in, uint64_t n, const uint32_t* off, uint64_t total, Terms<CT> e,
                              uint32_t K, const uint64_t* pidx, double q, Terms<CT> out, uint32_t* keep) {
  for (uint64_t t = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; t < total;
       t += (uint64_t)gridDim.x * blockDim.x) {
    uint64_t lo = 0, hi = n;   // last s with off[s] <= t
    while (hi - lo > 1) {
      const uint64_t mid = lo + (hi - lo) / 2;
      if ((uint64_t)off[mid] <= t) lo = mid; else hi = mid;
    }
    const uint64_t i = lo;
    const uint64_t j = t - off[i];
    uint64_t px[W], pz[W], rx[W], rz[W];
#pragma unroll
    for (int w = 0; w < W; ++w) {
      px[w] = in.x[(size_t)w * in.stride + i];
      pz[w] = in.z[(size_t)w * in.stride + i];
      rx[w] = px[w];
      rz[w] = pz[w];
    }
    const double c = (double)in.c[i];
    double v;
    if (j == 0) {
      double sd = 0.0;
      for (uint32_t a = 0; a < K; ++a) {
        int par = 0;
#pragma unroll
        for (int w = 0; w < W; ++w)
          par += popc64(e.x[(size_t)w * e.stride + a] & pz[w]) + popc64(e.z[(size_t)w * e.stride + a] & px[w]);
        const double ea = (double)e.c[a];
        sd += (par & 1) ? -ea * ea : ea * ea;
      }
      v = c * ((1.0 - q) + q * sd);
    } else {
      const uint64_t pr = pidx[j - 1];
      const uint32_t a = (uint32_t)(pr >> 32), b = (uint32_t)pr;
      uint64_t ax[W], az[W], bx[W], bz[W], tx[W], tz[W];
#pragma unroll
      for (int w = 0; w < W; ++w) {
        ax[w] = e.x[(size_t)w * e.stride + a];
        az[w] = e.z[(size_t)w * e.stride + a];
        bx[w] = e.x[(size_t)w * e.stride + b];
        bz[w] = e.z[(size_t)w * e.stride + b];
        tx[w] = ax[w] ^ px[w];
        tz[w] = az[w] ^ pz[w];
      }
      const double ea = (double)e.c[a], eb = (double)e.c[b];
      if (a == b) {
        int par = 0;
#pragma unroll
        for (int w = 0; w < W; ++w) par += popc64(ax[w] & pz[w]) + popc64(az[w] & px[w]);
        v = (par & 1) ? -(q * ea * ea * c) : q * ea * ea * c;
      } else {
        const int k = (herm_mul_phase<W>(ax, az, px, pz) + herm_mul_phase<W>(tx, tz, bx, bz)) & 3;
        v = (k & 1) ? 0.0 : (k == 0 ? 2.0 : -2.0) * q * ea * eb * c;
#pragma unroll
        for (int w = 0; w < W; ++w) {
          rx[w] = tx[w] ^ bx[w];
          rz[w] = tz[w] ^ bz[w];
        }
      }
    }
#pragma unroll
    for (int w = 0; w < W; ++w) {
      out.x[(size_t)w * out.stride + t] = rx[w];
      out.z[(size_t)w * out.stride + t] = rz[w];
    }
    out.c[t] = (CT)v;
    if (ORD) out.o[t] = in.o[i];
    keep[t] = (CT)v != (CT)0 ? 1u : 0u;
  }
}

template <int W, class CT, bool ORD>
__device__ __forceinline__ double reduce_run(Terms<CT>& t, uint64_t n, uint64_t i, double thr, uint32_t* keep) {
  if (i > 0 && same_term<W, CT, ORD>(t, i, i - 1)) { keep[i] = 0; return 0.0; }
  double s;
  if (sizeof(CT) == 8) {
    s = (double)t.c[i];
    for (uint64_t j = i + 1; j < n && same_term<W, CT, ORD>(t, i, j); ++j) s += (double)t.c[j];
  } else {
    float sum = (float)t.c[i], comp = 0.0f;   // Kahan summation in FP32
    for (uint64_t j = i + 1; j < n && same_term<W, CT, ORD>(t, i, j); ++j) {
      const float y = (float)t.c[j] - comp;
      const float tt = sum + y;
      comp = (tt - sum) - y;
      sum = tt;
    }
    s = (double)sum;
  }
  t.c[i] = (CT)s;
  const bool k = s != 0.0 && !(fabs(s) < thr);
  keep[i] = k ? 1u : 0u;
  return k ? 0.0 : fabs(s);
}


// On a sorted array: the first entry of each run of equal (string, order) sums its run
// (compensated in FP32), stores the sum in place and flags it if nonzero and |sum| >= thr.
template <int W, class CT, bool ORD>
__global__ void k_reduce_runs(Terms<CT> t, uint64_t n, double thr, uint32_t* keep, double* dropped) {
  double lost = 0.0;
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (uint64_t)gridDim.x * blockDim.x)
    lost += reduce_run<W, CT, ORD>(t, n, i, thr, keep);
  add_dropped(lost, dropped);
}

// keep flags from a threshold on |c| (exact zeros always dropped)
template <class CT>
__global__ void k_threshold_flags(const CT* c, uint64_t n, double thr, uint32_t* keep, double* dropped) {
  double lost = 0.0;
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (uint64_t)gridDim.x * blockDim.x) {
    const double v = (double)c[i];
    const bool k = v != 0.0 && !(fabs(v) < thr);
    keep[i] = k ? 1u : 0u;
    lost += k ? 0.0 : fabs(v);
  }
  add_dropped(lost, dropped);
}

// out[pos[i]] = in[i] for keep[i]; pos = exclusive scan of keep (kept in a separate array).
template <int W, class CT, bool ORD>
__global__ void k_compact(Terms<CT> in, Terms<CT> out, uint64_t n, const uint32_t* keep, const uint32_t* pos) {
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

// Copy terms [src, src+len) of `in` to `out` at dst (ranges from a list).
template <int W, class CT, bool ORD>
__global__ void k_copy_ranges(Terms<CT> in, Terms<CT> out, const uint32_t* src, const uint32_t* len,
                              const uint64_t* dst, int nranges) {
  const int r = blockIdx.x;
  if (r >= nranges) return;
  for (uint32_t k = threadIdx.x; k < len[r]; k += blockDim.x) {
    const uint64_t i = (uint64_t)src[r] + k;
    const uint64_t j = dst[r] + k;
    if (j >= out.stride) return;
#pragma unroll
    for (int w = 0; w < W; ++w) {
      out.x[w * out.stride + j] = in.x[w * in.stride + i];
      out.z[w * out.stride + j] = in.z[w * in.stride + i];
    }
    out.c[j] = in.c[i];
    if (ORD) out.o[j] = in.o[i];
  }
}

template <int W, class CT, bool ORD>
__global__ void k_copy(Terms<CT> in, uint64_t i0, Terms<CT> out, uint64_t j0, uint64_t n) {
  const uint64_t k = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= n) return;
  const uint64_t i = i0 + k, j = j0 + k;
  if (j >= out.stride) return;
#pragma unroll
  for (int w = 0; w < W; ++w) {
    out.x[w * out.stride + j] = in.x[w * in.stride + i];
    out.z[w * out.stride + j] = in.z[w * in.stride + i];
  }
  out.c[j] = in.c[i];
  if (ORD) out.o[j] = in.o[i];
}

// OR and AND of every key plane (to find which digit ranges of the canonical key vary).
template <int W, class CT, bool ORD>
__global__ void k_key_span(Terms<CT> t, uint64_t n, unsigned long long* or_and /*[2][2W+1]*/) {
  constexpr int NP = 2 * W + 1;
  uint64_t vo[NP], va[NP];
#pragma unroll
  for (int p = 0; p < NP; ++p) { vo[p] = 0; va[p] = ~0ULL; }
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (uint64_t)gridDim.x * blockDim.x) {
#pragma unroll
    for (int w = 0; w < W; ++w) {
      const uint64_t a = t.x[w * t.stride + i], b = t.z[w * t.stride + i];
      vo[w] |= a; va[w] &= a;
      vo[W + w] |= b; va[W + w] &= b;
    }
    const uint64_t o = ORD ? t.o[i] : 0;
    vo[2 * W] |= o; va[2 * W] &= o;
  }
#pragma unroll
  for (int p = 0; p < NP; ++p) {
    uint64_t a = vo[p], b = va[p];
    for (int d = 32; d >= 1; d >>= 1) {
      a |= __shfl_xor(a, d, 64);
      b &= __shfl_xor(b, d, 64);
    }
    if ((threadIdx.x & 63) == 0) {
      atomicOr(&or_and[p], (unsigned long long)a);
      atomicAnd(&or_and[NP + p], (unsigned long long)b);
    }
  }
}

// ------------------------------------------------------------------------------------------
// Cap: radix select on |c| bits, most significant digit first.
// ------------------------------------------------------------------------------------------
template <class CT>
__device__ __forceinline__ uint64_t abs_key(CT v) {
  return coef_bits<CT>(v) & (sizeof(CT) == 8 ? 0x7fffffffffffffffULL : 0x7fffffffULL);
}

// Visit the |c| keys of c[0..n) over a grid-stride loop of 256-thread blocks, eight loads
// in flight per thread.
template <class CT, class F>
__device__ __forceinline__ void grid_keys(const CT* c, uint64_t n, F&& f) {
  const uint64_t stride = (uint64_t)gridDim.x * 256;
  uint64_t i = (uint64_t)blockIdx.x * 256 + threadIdx.x;
  for (; i + 7 * stride < n; i += 8 * stride) {
    uint64_t k[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) k[u] = abs_key<CT>(c[i + u * stride]);
#pragma unroll
    for (int u = 0; u < 8; ++u) f(k[u]);
  }
  for (; i < n; i += stride) f(abs_key<CT>(c[i]));
}

template <class CT>
__global__ void __launch_bounds__(256) k_abs_hist(const CT* c, uint64_t n, int shift, int bits,
                                                  uint64_t pmask, uint64_t prefix, uint32_t* hist) {
  __shared__ uint32_t h[2048];
  const int bins = 1 << bits;
  for (int b = threadIdx.x; b < bins; b += 256) h[b] = 0;
  __syncthreads();
  uint32_t zeros = 0;   // unused slots (c = 0) are many: counted in a register, not in LDS
  auto add = [&](uint64_t k) {
    if ((k & pmask) == prefix) {
      if (k == 0) ++zeros;
      else atomicAdd(&h[(k >> shift) & (uint64_t)(bins - 1)], 1u);
    }
  };
  grid_keys<CT>(c, n, add);
  for (int d = 32; d >= 1; d >>= 1) zeros += __shfl_xor(zeros, d, 64);
  if ((threadIdx.x & 63) == 0 && zeros) atomicAdd(&h[0], zeros);
  __syncthreads();
  for (int b = threadIdx.x; b < bins; b += 256)
    if (h[b]) atomicAdd(&hist[b], h[b]);
}

// Histogram of |c| keys over the window [lo, lo + 2048 * 2^shift): bins of 2^shift keys,
// hist[2048] counts the keys above the window (lo is a multiple of 2^shift).
template <class CT>
__global__ void __launch_bounds__(256) k_abs_hist_win(const CT* c, uint64_t n, uint64_t lo, int shift,
                                                      uint32_t* hist) {
  __shared__ uint32_t h[2049];
  for (int b = threadIdx.x; b < 2049; b += 256) h[b] = 0;
  __syncthreads();
  // counted in registers: most keys lie above a window near the cut, and unused slots (c = 0)
  // are many
  uint32_t above = 0, zeros = 0;
  auto add = [&](uint64_t k) {
    if (k >= lo) {
      const uint64_t d = (k - lo) >> shift;
      if (d >= 2048) ++above;
      else if (k == 0) ++zeros;
      else atomicAdd(&h[d], 1u);
    }
  };
  grid_keys<CT>(c, n, add);
  for (int d = 32; d >= 1; d >>= 1) {
    above += __shfl_xor(above, d, 64);
    zeros += __shfl_xor(zeros, d, 64);
  }
  if ((threadIdx.x & 63) == 0 && above) atomicAdd(&h[2048], above);
  if ((threadIdx.x & 63) == 0 && zeros) atomicAdd(&h[0], zeros);
  __syncthreads();
  for (int b = threadIdx.x; b < 2049; b += 256)
    if (h[b]) atomicAdd(&hist[b], h[b]);
}

// keep: |c| > tau, or |c| == tau and marked; ties flagged for the tie-break list.  Only the
// key bits in pmask take part (the selection may stop at a bucket that is kept whole).
template <class CT>
__global__ void k_cap_flags(const CT* c, uint64_t n, uint64_t tau, uint64_t pmask, uint32_t* keep, uint32_t* tie,
                            double* dropped) {
  double lost = 0.0;
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (uint64_t)gridDim.x * blockDim.x) {
    const uint64_t k = abs_key<CT>(c[i]) & pmask;
    keep[i] = k > tau ? 1u : 0u;
    tie[i] = k == tau ? 1u : 0u;
    lost += k < tau ? fabs((double)c[i]) : 0.0;
  }
  add_dropped(lost, dropped);
}

// Gather tied terms' keys with their index stored as the coefficient (double).
template <int W, class CT, bool ORD>
__global__ void k_gather_ties(Terms<CT> in, uint64_t n, const uint32_t* tie, const uint32_t* pos, Terms<double> out) {
  const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n || !tie[i]) return;
  const uint64_t j = pos[i];
  if (j >= out.stride) return;
#pragma unroll
  for (int w = 0; w < W; ++w) {
    out.x[w * out.stride + j] = in.x[w * in.stride + i];
    out.z[w * out.stride + j] = in.z[w * in.stride + i];
  }
  out.c[j] = (double)i;
  out.o[j] = ORD ? in.o[i] : 0;
}

template <class CT>
__global__ void k_mark_ties(const double* idx, uint64_t r, uint32_t* keep, uint64_t n) {
  const uint64_t j = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= r) return;
  const uint64_t i = (uint64_t)idx[j];
  if (i < n) keep[i] = 1u;
}

// ------------------------------------------------------------------------------------------
// Expectation <b|O|b>: per-block FP64 partial sums, then one block in fixed order.
// ------------------------------------------------------------------------------------------
template <int W, class CT>
__global__ void __launch_bounds__(256) k_expect(Terms<CT> t, uint64_t n, GroupMask basis, double* partial) {
  __shared__ double s[4];
  double acc = 0.0;
  for (uint64_t i = (uint64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (uint64_t)gridDim.x * 256) {
    bool diag = true;
    int par = 0;
#pragma unroll
    for (int w = 0; w < W; ++w) {
      diag = diag && t.x[w * t.stride + i] == 0;
      par += __popcll(t.z[w * t.stride + i] & basis.mz[w]);
    }
    if (diag) {
      const double v = (double)t.c[i];
      acc += (par & 1) ? -v : v;
    }
  }
  for (int d = 32; d >= 1; d >>= 1) acc += __shfl_xor(acc, d, 64);
  if ((threadIdx.x & 63) == 0) s[threadIdx.x >> 6] = acc;
  __syncthreads();
  if (threadIdx.x == 0) partial[blockIdx.x] = (s[0] + s[1]) + (s[2] + s[3]);
}

// keep[i] = 1 for diagonal strings (x = 0): the only ones with a nonzero <b|P|b>.
template <int W, class CT>
__global__ void k_diag_flags(Terms<CT> t, uint64_t n, uint32_t* keep) {
  const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  uint64_t any = 0;
#pragma unroll
  for (int w = 0; w < W; ++w) any |= t.x[w * t.stride + i];
  keep[i] = any == 0;
}

__global__ void k_sum_partials(const double* partial, int nb, double* out) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    double a = 0.0;
    for (int i = 0; i < nb; ++i) a += partial[i];
    *out = a;
  }
}

// ------------------------------------------------------------------------------------------
// Conversions for FP32 storage.
// ------------------------------------------------------------------------------------------
template <class CT>
__global__ void k_from_f64(const double* src, CT* dst, uint64_t n) {
  const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) dst[i] = (CT)src[i];
}
template <class CT>
__global__ void k_to_f64(const CT* src, double* dst, uint64_t n) {
  const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) dst[i] = (double)src[i];
}

__global__ void k_or_flags(uint32_t* a, const uint32_t* b, uint64_t n) {
  const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) a[i] |= b[i];
}

__global__ void k_fill_u32(uint32_t* p, uint64_t n, uint32_t v) {
  const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

}  // namespace pp
