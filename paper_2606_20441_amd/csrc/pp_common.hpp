// pp_common.hpp -- shared device/host definitions of the gfx950 Pauli-propagation library.
//
// Term storage (HBM): structure of arrays with one plane per 64-bit word, so a wavefront's
// load of one plane is 64 consecutive 8-byte words:
//   x[w * stride + i], z[w * stride + i]   (w = 0..W-1)   Pauli bits of term i
//   c[i]                                    coefficient (double, or float)
//   o[i]                                    error-order tag (error-order mode only)
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#define PP_MAXW 4

namespace pp {

constexpr int kWave = 64;

template <class CT>
struct Terms {
  uint64_t* x;      // [W][stride]
  uint64_t* z;      // [W][stride]
  CT* c;            // [stride]
  uint8_t* o;       // [stride] or nullptr
  uint64_t stride;  // plane stride (capacity)
};

// One rotation as the kernels see it.  m[0..W-1] = x mask, m[W..2W-1] = z mask.
// Noise of one layer, decomposed by generator support on the host:
//  * `nsup` supports of one or two qubits, each with a table over the 4 or 16 local
//    Pauli patterns giving, for the generators on that support that anticommute with
//    the pattern, the product of their factors f_k in list order (greedy mode: one run
//    of consecutive generators on the same qubits) or the power sums of x_k = f_k - 1
//    (error-order mode);
//  * `ndirect` generators tested one by one (larger supports).
struct SupportDev {
  int16_t w0, b0, w1, b1;   // word/bit of the two qubits (w1 < 0: single qubit)
  int32_t table;            // offset into the value table
  int32_t pad;
};

struct NoiseDev {
  int nsup;
  int ndirect;
  int ntab;                 // doubles in `tab`
  int sign;                 // +1 inverse map, -1 channel
  int mode;                 // 0 greedy, 1 error order
  int max_order;
  const SupportDev* sup;
  const double* tab;        // per support and pattern: greedy, the run's product; error order, max_order power sums
  const uint64_t* dm;       // direct generators: [ndirect][2W]
  const double* dval;       // greedy: fidelity factor; error order: max_order powers of x_k
  const uint8_t* drun;      // greedy, direct generators: 1 where a run on new qubits starts
  // greedy mode: the supports listed per qubit (CSR over n qubits; entry = support index,
  // top bit set when the qubit is the support's second one), so that a string visits only
  // the supports on its non-identity qubits; null when not built
  int nq;                   // qubits with lists (0: none)
  int nqent;
  const int32_t* qoff;      // [nq + 1]
  const uint32_t* qent;     // [nqent]
};

__device__ __forceinline__ int popc64(uint64_t v) { return __popcll(v); }

__device__ __host__ __forceinline__ uint64_t mix64(uint64_t v) {
  v ^= v >> 31;
  v *= 0x7fb5d329728ea185ULL;
  v ^= v >> 27;
  v *= 0x81dadef4bc2dd44dULL;
  v ^= v >> 33;
  return v;
}

enum GateType { GATE_GENERIC = 0, GATE_X1 = 1, GATE_ZZ = 2 };

struct GateDev {
  uint64_t m[2 * PP_MAXW];
  double cs;          // cos(theta) (exact for Clifford angles)
  double sn_dir;      // +sin(theta) for U^dag P U, -sin(theta) for U P U^dag
  int pivot_word;     // word (0..2W-1) of the lowest set bit of m; pair leader has it clear
  int pivot_bit;
  int rr_phase;       // |x_R & z_R| mod 4
  int clifford;       // 1: exact angle, no threshold afterwards
  int type;           // GATE_X1: R = X on qubit (w0,b0); GATE_ZZ: R = Z Z on (w0,b0), (w1,b1)
  int w0, b0, w1, b1; // for GATE_ZZ (w0,b0) is the lower qubit (the pivot)
  uint32_t hash;      // linear key hash of the flip mask (x = m[0..W), z = m[W..2W))
  uint32_t khash;     // key_hash of the flip mask
};

// GF(2)-linear 32-bit hash of a Pauli key: XOR of one table word per key byte.  Linear, so
// the hash of P xor R is hash(P) xor hash(R): a partner's hash costs one XOR.
constexpr int kHashTabWords = 2 * PP_MAXW * 8 * 256;   // [plane][byte][value]; z planes at PP_MAXW
template <int W>
__device__ __host__ __forceinline__ uint32_t lin_hash(const uint64_t* kx, const uint64_t* kz, const uint32_t* tab) {
  uint32_t h = 0;
  for (int w = 0; w < W; ++w)
    for (int k = 0; k < 8; ++k) {
      h ^= tab[((w * 8) + k) * 256 + (uint32_t)((kx[w] >> (8 * k)) & 255u)];
      h ^= tab[(((PP_MAXW + w) * 8) + k) * 256 + (uint32_t)((kz[w] >> (8 * k)) & 255u)];
    }
  return h;
}

// A GF(2)-linear 32-bit hash computed in registers (rotations, xor-shifts and a fold are
// all linear): key_hash(P xor R) = key_hash(P) xor key_hash(R).  Used where the table hash
// would need a per-term plane in memory; a match is always confirmed on the full key.
__device__ __host__ __forceinline__ uint64_t kh_rotl(uint64_t v, int r) { return (v << r) | (v >> (64 - r)); }
template <int W>
__device__ __host__ __forceinline__ uint32_t key_hash(const uint64_t* kx, const uint64_t* kz) {
  uint64_t y = 0;
#pragma unroll
  for (int w = 0; w < W; ++w) {
    uint64_t v = kx[w] ^ kh_rotl(kz[w], 32);
    v ^= v << 13;
    v ^= v >> 7;
    v ^= v << 17;
    y ^= w == 0 ? v : kh_rotl(v, 11 * w);
  }
  y ^= y >> 29;
  return (uint32_t)(y ^ (y >> 32));
}

__device__ __host__ __forceinline__ uint32_t ord_hash(uint32_t o) {
  return o ? (uint32_t)(mix64(0x5851f42d4c957f2dULL + o) >> 32) : 0u;
}

// Group hash: the bits of (x & mx, z & mz) that a layer's gates can never change.
template <int W>
__device__ __forceinline__ uint64_t group_hash(const uint64_t* xs, const uint64_t* zs,
                                               const uint64_t* mx, const uint64_t* mz) {
  uint64_t h = 0x243f6a8885a308d3ULL;
#pragma unroll
  for (int w = 0; w < W; ++w) {
    h = mix64(h ^ (xs[w] & mx[w]));
    h = mix64(h + (zs[w] & mz[w]));
  }
  return h;
}

struct GroupMask {
  uint64_t mx[PP_MAXW];
  uint64_t mz[PP_MAXW];
};

}  // namespace pp
