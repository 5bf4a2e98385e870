// pp_oracle.cpp -- plain CPU FP64 reference for noise-canceling Pauli propagation.
//
// TEST INFRASTRUCTURE ONLY: the test suite, the package smoke check and the benchmark's
// CPU-baseline leg load this library; the product path never does.  It shares no code,
// header or table with the HIP library.  It is written to be read against the paper
// (Eddins et al., "Computing noise-canceling observables via Pauli propagation"), not to
// be fast: one hash map of (string, order) -> coefficient, rebuilt after every gate.
//
// Pinned by the CPU tests against: explicit 2^n x 2^n matrices (Pauli products and the
// rotation rule), a dense density-matrix / superoperator brute force at <= 9 qubits
// (the trace identity of Section I.B at zero threshold), the one-qubit worked example of
// Appendix "Invalidity of applying certain lightcone reductions before PNA", the Clifford
// closed form of Appendix A, channel-times-inverse identity, unitary round trips and
// brute-force truncation on random arrays.
#include "pp_oracle.h"

#include <algorithm>
#include <cmath>
#include <complex>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <unordered_map>
#include <vector>

namespace {

constexpr int kMaxWords = 4;

struct Key {
  uint64_t x[kMaxWords];
  uint64_t z[kMaxWords];
  uint8_t o;
};

bool operator==(const Key& a, const Key& b) {
  return std::memcmp(a.x, b.x, sizeof a.x) == 0 && std::memcmp(a.z, b.z, sizeof a.z) == 0 &&
         a.o == b.o;
}

uint64_t mix64(uint64_t v) {  // splitmix64 finaliser
  v ^= v >> 30; v *= 0xbf58476d1ce4e5b9ULL;
  v ^= v >> 27; v *= 0x94d049bb133111ebULL;
  v ^= v >> 31;
  return v;
}

struct KeyHash {
  size_t operator()(const Key& k) const {
    uint64_t h = 0x9e3779b97f4a7c15ULL ^ k.o;
    for (int w = 0; w < kMaxWords; ++w) h = mix64(h ^ k.x[w]) + 0x632be59bd9b4e019ULL;
    for (int w = 0; w < kMaxWords; ++w) h = mix64(h ^ k.z[w]) + 0x2545f4914f6cdd1dULL;
    return (size_t)h;
  }
};

using Map = std::unordered_map<Key, double, KeyHash>;

[[noreturn]] void fail(const char* what) {
  std::fprintf(stderr, "pp_oracle: %s\n", what);
  std::abort();
}

// Canonical order: x words from the most significant word down, then z words, then order.
bool canonical_less(const Key& a, const Key& b) {
  for (int w = kMaxWords - 1; w >= 0; --w)
    if (a.x[w] != b.x[w]) return a.x[w] < b.x[w];
  for (int w = kMaxWords - 1; w >= 0; --w)
    if (a.z[w] != b.z[w]) return a.z[w] < b.z[w];
  return a.o < b.o;
}

int popc(uint64_t v) { return __builtin_popcountll(v); }

}  // namespace

struct or_sum {
  int n = 0;
  int W = 0;
  Map m;
};

namespace {

// Symplectic product <P, R> (Section I, below Eq. evolve_gate: 0 if P and R commute, 1
// if they anticommute).  X^a Z^b X^c Z^d = (-1)^{|b&c|} X^{a^c} Z^{b^d}, so the two
// orders of the product differ by (-1)^{|x_P & z_R| + |z_P & x_R|}.
int anticommutes(const Key& p, const uint64_t* rx, const uint64_t* rz, int W) {
  int s = 0;
  for (int w = 0; w < W; ++w) s += popc(p.x[w] & rz[w]) + popc(p.z[w] & rx[w]);
  return s & 1;
}

// i R P for anticommuting Hermitian Paulis R = i^{|xR&zR|} X^xR Z^zR and
// P = i^{|xP&zP|} X^xP Z^zP equals s * Q with Q = (xR^xP, zR^zP) in Hermitian form and
// s = +-1: R P = i^{|xR&zR| + |xP&zP|} (-1)^{|zR&xP|} X^xQ Z^zQ
//          = i^{|xR&zR| + |xP&zP| + 2|zR&xP| - |xQ&zQ|} Q,
// so i R P = i^e Q with e = 1 + |xR&zR| + |xP&zP| + 2|zR&xP| - |xQ&zQ| (e even here).
int irp_sign(const Key& p, const uint64_t* rx, const uint64_t* rz, int W, Key* q) {
  *q = p;
  int e = 1;
  for (int w = 0; w < W; ++w) {
    q->x[w] = p.x[w] ^ rx[w];
    q->z[w] = p.z[w] ^ rz[w];
    e += popc(rx[w] & rz[w]) + popc(p.x[w] & p.z[w]) + 2 * popc(rz[w] & p.x[w]) -
         popc(q->x[w] & q->z[w]);
  }
  e = ((e % 4) + 4) % 4;
  if (e == 0) return 1;
  if (e == 2) return -1;
  fail("i R P is not Hermitian: R and P commute");
}

// Exact cos/sin at multiples of pi/2; otherwise libm.  Returns 1 for a Clifford angle.
int angle_cos_sin(double theta, double* c, double* s) {
  const double k = theta / (M_PI / 2);
  const double r = std::nearbyint(k);
  if (std::fabs(k - r) < 1e-12) {
    long m = ((long)r % 4 + 4) % 4;
    static const double cs[4][2] = {{1, 0}, {0, 1}, {-1, 0}, {0, -1}};
    *c = cs[m][0];
    *s = cs[m][1];
    return 1;
  }
  *c = std::cos(theta);
  *s = std::sin(theta);
  return 0;
}

Key make_key(int W, const uint64_t* x, const uint64_t* z, uint8_t o) {
  Key k;
  std::memset(&k, 0, sizeof k);
  for (int w = 0; w < W; ++w) { k.x[w] = x[w]; k.z[w] = z[w]; }
  k.o = o;
  return k;
}

void erase_zeros(Map& m) {
  for (auto it = m.begin(); it != m.end();) {
    if (it->second == 0.0) it = m.erase(it); else ++it;
  }
}

void threshold(Map& m, double eps) {
  for (auto it = m.begin(); it != m.end();) {
    if (std::fabs(it->second) < eps) it = m.erase(it); else ++it;
  }
}

// Rotation past one gate (Section I, Eq. evolve_gate forward; the Appendix on Euclid
// theory gives the backward form): a commuting P is kept; an anticommuting P becomes
//   forward  U P U^dag = cos(theta) P - sin(theta) (i R P)
//   backward U^dag P U = cos(theta) P + sin(theta) (i R P)
// and duplicated strings are accumulated (Appendix B's A'[P'] += c').
// With sine_max >= 0 (the sine-order mode) the tag counts the sine factors along a term's
// path, the CPT order kappa = k + 2p of the Euclid appendix (k steps, p bubbles, each step
// one sin): the sin child of a non-Clifford rotation gets tag + 1 and is dropped above
// sine_max.  Clifford rotations are exact frame changes and do not count.
int rotate(or_sum* s, const uint64_t* rx, const uint64_t* rz, double theta, int dir, int sine_max = -1) {
  if (dir != 1 && dir != -1) fail("dir must be +1 or -1");
  double cs, sn;
  const int clifford = angle_cos_sin(theta, &cs, &sn);
  Map out;
  out.reserve(s->m.size() * 2 + 16);
  for (const auto& kv : s->m) {
    const Key& p = kv.first;
    const double c = kv.second;
    if (!anticommutes(p, rx, rz, s->W)) {
      out[p] += c;
      continue;
    }
    if (cs != 0.0) out[p] += c * cs;
    if (sn != 0.0) {
      Key q;
      const int sg = irp_sign(p, rx, rz, s->W, &q);
      const double child = (dir == 1 ? 1.0 : -1.0) * sg * c;
      if (sine_max >= 0 && !clifford) {
        if (p.o + 1 > sine_max) continue;
        q.o = (uint8_t)(p.o + 1);
      }
      out[q] += child * sn;
    }
  }
  erase_zeros(out);
  s->m.swap(out);
  return clifford;
}

// Per-generator Pauli fidelity of one local Pauli-Lindblad channel: E(.)E applied with
// probability p = (1 - e^{-2 lambda})/2 multiplies an anticommuting P by 1 - 2p
// (Section I, the channel definition and Eq. evolve_noise).  The inverse negates lambda,
// giving the quasi-probability q = (1 - e^{2 lambda})/2 <= 0 and factor 1 - 2q.
double fidelity_factor(double lambda, int sign) {
  // sign = -1: the channel, p = (1 - e^{-2 lambda})/2; sign = +1: its inverse, lambda -> -lambda.
  const double q = (1.0 - std::exp(2.0 * sign * lambda)) / 2.0;
  return 1.0 - 2.0 * q;
}

void noise(or_sum* s, int n_gen, const uint64_t* ex, const uint64_t* ez, const double* lambda,
           int sign, int mode, int max_order) {
  if (sign != 1 && sign != -1) fail("noise sign must be +1 or -1");
  if (n_gen <= 0) return;
  std::vector<double> f(n_gen);
  for (int k = 0; k < n_gen; ++k) {
    if (!(lambda[k] >= 0.0) || !std::isfinite(lambda[k])) fail("lambda must be finite and >= 0");
    f[k] = fidelity_factor(lambda[k], sign);
  }
  const int W = s->W;
  if (mode == 0) {
    // The layer's channel is the composition of its local channels, one per generator
    // (Section I, the noise model), so Eq. evolve_noise is applied generator by generator in
    // list order: an anticommuting P is multiplied by that generator's f_k.
    for (auto& kv : s->m) {
      for (int k = 0; k < n_gen; ++k)
        if (anticommutes(kv.first, ex + (size_t)k * W, ez + (size_t)k * W, W)) kv.second *= f[k];
    }
    return;
  }
  if (mode != 1) fail("noise mode must be 0 or 1");
  if (max_order < 0 || max_order > 255) fail("max_order out of range");
  // prod_k (1 + x_k) over anticommuting k, x_k = f_k - 1, written as sum_j e_j with e_j the
  // elementary symmetric polynomial of degree j in those x_k; a term of order o receives
  // e_j at order o + j <= max_order (Appendix C orders terms by the number of errors
  // acting on the observable; the Euclid appendix linearises 1/f as 1 + eps).
  Map out;
  out.reserve(s->m.size() * (size_t)(max_order + 1) + 16);
  std::vector<double> e((size_t)max_order + 1);
  for (const auto& kv : s->m) {
    const Key& p = kv.first;
    const int o = p.o;
    if (o > max_order) continue;
    const int jmax = max_order - o;
    std::fill(e.begin(), e.end(), 0.0);
    e[0] = 1.0;
    for (int k = 0; k < n_gen; ++k) {
      if (!anticommutes(p, ex + (size_t)k * W, ez + (size_t)k * W, W)) continue;
      const double xk = std::expm1(2.0 * sign * lambda[k]);   // f_k - 1 without cancellation
      for (int j = jmax; j >= 1; --j) e[j] += e[j - 1] * xk;
    }
    for (int j = 0; j <= jmax; ++j) {
      Key q = p;
      q.o = (uint8_t)(o + j);
      out[q] += kv.second * e[j];
    }
  }
  erase_zeros(out);
  s->m.swap(out);
}

// Greedy truncation (Section I.A): drop |c| < eps, then keep at most max_terms of the
// largest |c|; equal magnitudes are ranked by the canonical key (smaller first).
void truncate(or_sum* s, double eps, int64_t max_terms) {
  if (!(eps >= 0.0)) fail("eps must be >= 0");
  if (eps > 0.0) threshold(s->m, eps);
  if (max_terms > 0 && (int64_t)s->m.size() > max_terms) {
    std::vector<std::pair<Key, double>> v(s->m.begin(), s->m.end());
    std::sort(v.begin(), v.end(), [](const std::pair<Key, double>& a, const std::pair<Key, double>& b) {
      const double fa = std::fabs(a.second), fb = std::fabs(b.second);
      if (fa != fb) return fa > fb;
      return canonical_less(a.first, b.first);
    });
    v.resize((size_t)max_terms);
    Map keep;
    keep.reserve(v.size() * 2);
    for (auto& kv : v) keep.emplace(kv.first, kv.second);
    s->m.swap(keep);
  }
}

// Product of two Hermitian Paulis, A B = i^e C with C = (xA ^ xB, zA ^ zB) in Hermitian
// form: A = i^{|xA&zA|} X^xA Z^zA, and moving Z^zA past X^xB gives (-1)^{|zA&xB|}, so
// e = |xA&zA| + |xB&zB| + 2|zA&xB| - |xC&zC| (mod 4).  C keeps A's order tag.
int pauli_mul(const Key& a, const Key& b, int W, Key* c) {
  *c = a;
  int e = 0;
  for (int w = 0; w < W; ++w) {
    c->x[w] = a.x[w] ^ b.x[w];
    c->z[w] = a.z[w] ^ b.z[w];
    e += popc(a.x[w] & a.z[w]) + popc(b.x[w] & b.z[w]) + 2 * popc(a.z[w] & b.x[w]) -
         popc(c->x[w] & c->z[w]);
  }
  return ((e % 4) + 4) % 4;
}

// Propagated antinoise absorbed into the observable (Section I.A, Eq. applyantinoise): the
// inverse map of one generator, carried to the end of the circuit, applies the evolved
// error E' = sum_a e_a P_a with quasi-probability q, so O -> (1 - q) O + q E' O E'.
// E' O E' is written out as the plain sum over ordered pairs (a, b) of e_a e_b P_a P P_b
// for every term P of O, in complex arithmetic; the result is Hermitian, so every
// imaginary part must cancel.  Exact zeros are dropped; nothing else is truncated here.
void antinoise(or_sum* s, const or_sum* e, double q) {
  if (e->W != s->W || e->n != s->n) fail("E' and O must have the same qubit count");
  if (!std::isfinite(q)) fail("q must be finite");
  const int W = s->W;
  std::vector<std::pair<Key, double>> ev(e->m.begin(), e->m.end());
  std::unordered_map<Key, std::complex<double>, KeyHash> acc;
  acc.reserve(s->m.size() * (ev.size() * ev.size() + 1) + 16);
  static const std::complex<double> ipow[4] = {{1, 0}, {0, 1}, {-1, 0}, {0, -1}};
  double scale = 0.0;
  for (const auto& kv : s->m) {
    const Key& p = kv.first;
    const double c = kv.second;
    acc[p] += (1.0 - q) * c;
    for (const auto& ea : ev) {
      for (const auto& eb : ev) {
        Key t, r;
        const int k1 = pauli_mul(ea.first, p, W, &t);
        const int k2 = pauli_mul(t, eb.first, W, &r);
        r.o = p.o;
        const double w = q * ea.second * eb.second * c;
        acc[r] += w * ipow[(k1 + k2) & 3];
        scale = std::max(scale, std::fabs(w));
      }
    }
  }
  Map out;
  out.reserve(acc.size() * 2 + 16);
  for (const auto& kv : acc) {
    if (std::fabs(kv.second.imag()) > 1e-12 * std::max(1.0, scale)) fail("E' O E' is not Hermitian");
    if (kv.second.real() != 0.0) out.emplace(kv.first, kv.second.real());
  }
  s->m.swap(out);
}

// Approximate conjugation by the most significant products (Appendix B, the heuristic
// conjugation of large Pauli sums): E' O E' is a sum of products P_a P P_b over index
// triplets (a, term of O, b) with magnitudes mu = |c| (|e_a| |e_b|).  Reading used here:
// the products with a = b (P_a P P_a = +-P), which together with (1 - q) O make up the
// part of the update that leaves every term on its own string (for an E' of unit weight,
// exactly O where E' commutes with it; compare the commutator form of Appendix A), are
// always kept; the limit applies to the triplets with a != b, of which the k largest mu
// are kept, every triplet tied with the k-th as well (both orders of a pair have equal mu,
// so they stay together and the result is Hermitian).  k <= 0, or k at least the number of
// such triplets, keeps all: the exact update.  Written as the definition: every off-diagonal
// triplet's mu, sorted, the k-th taken as the cut.
void antinoise_topk(or_sum* s, const or_sum* e, double q, int64_t k) {
  if (e->W != s->W || e->n != s->n) fail("E' and O must have the same qubit count");
  if (!std::isfinite(q)) fail("q must be finite");
  const int W = s->W;
  std::vector<std::pair<Key, double>> ev(e->m.begin(), e->m.end());
  std::vector<std::pair<Key, double>> ov(s->m.begin(), s->m.end());
  double cut = 0.0;
  const uint64_t n_trip = (uint64_t)ov.size() * ev.size() * (ev.size() ? ev.size() - 1 : 0);
  if (k > 0 && (uint64_t)k < n_trip) {
    std::vector<double> mu;
    mu.reserve(n_trip);
    for (const auto& p : ov)
      for (size_t a = 0; a < ev.size(); ++a)
        for (size_t b = 0; b < ev.size(); ++b)
          if (a != b) mu.push_back(std::fabs(p.second) * (std::fabs(ev[a].second) * std::fabs(ev[b].second)));
    std::sort(mu.begin(), mu.end(), [](double x, double y) { return x > y; });
    cut = mu[(size_t)k - 1];
  }
  std::unordered_map<Key, std::complex<double>, KeyHash> acc;
  static const std::complex<double> ipow[4] = {{1, 0}, {0, 1}, {-1, 0}, {0, -1}};
  double scale = 0.0;
  for (const auto& kv : ov) {
    const Key& p = kv.first;
    const double c = kv.second;
    acc[p] += (1.0 - q) * c;
    for (size_t a = 0; a < ev.size(); ++a) {
      for (size_t b = 0; b < ev.size(); ++b) {
        const auto& ea = ev[a];
        const auto& eb = ev[b];
        if (a != b && !(std::fabs(c) * (std::fabs(ea.second) * std::fabs(eb.second)) >= cut)) continue;
        Key t, r;
        const int k1 = pauli_mul(ea.first, p, W, &t);
        const int k2 = pauli_mul(t, eb.first, W, &r);
        r.o = p.o;
        const double w = q * ea.second * eb.second * c;
        acc[r] += w * ipow[(k1 + k2) & 3];
        scale = std::max(scale, std::fabs(w));
      }
    }
  }
  Map out;
  out.reserve(acc.size() * 2 + 16);
  for (const auto& kv : acc) {
    if (std::fabs(kv.second.imag()) > 1e-12 * std::max(1.0, scale)) fail("kept products are not Hermitian");
    if (kv.second.real() != 0.0) out.emplace(kv.first, kv.second.real());
  }
  s->m.swap(out);
}

// A batch of C commuting antinoise maps expanded in the number of errors (Appendix C):
// with a_c = q_c / (1 - q_c) and C_c(X) = E'_c X E'_c, the exact product
// prod_c (1 - q_c)(1 + a_c C_c) O is approximated by
//   O0 = O prod_c (1 - q_c),   O1 = sum_c a_c C_c(O0),
//   O2 = 1/2 sum_c (a_c C_c(O1') - a_c^2 O0)     (order 2 only),
// returning O0 + O1 (+ O2), where O1' is O1 with |c| < eps1 dropped (the input of the
// second-order pass only; eps1 = 0 keeps it whole).  Reading: the appendix's overbarred error carries the factor
// whose square is q/(1 - q), negative for an inverse map, which is what the exact product
// gives; its printed |q| drops that sign.  C = 1 is exact.  Each C_c is the plain double
// sum over ordered pairs (as in antinoise).
Map conj_sum(const Map& x, const or_sum* e, double scale, int W) {
  std::unordered_map<Key, std::complex<double>, KeyHash> acc;
  static const std::complex<double> ipow[4] = {{1, 0}, {0, 1}, {-1, 0}, {0, -1}};
  std::vector<std::pair<Key, double>> ev(e->m.begin(), e->m.end());
  for (const auto& kv : x)
    for (const auto& ea : ev)
      for (const auto& eb : ev) {
        Key t, r;
        const int k1 = pauli_mul(ea.first, kv.first, W, &t);
        const int k2 = pauli_mul(t, eb.first, W, &r);
        r.o = kv.first.o;
        acc[r] += scale * ea.second * eb.second * kv.second * ipow[(k1 + k2) & 3];
      }
  Map out;
  for (const auto& kv : acc) {
    if (std::fabs(kv.second.imag()) > 1e-12 * std::max(1.0, std::fabs(scale))) fail("E' X E' is not Hermitian");
    if (kv.second.real() != 0.0) out.emplace(kv.first, kv.second.real());
  }
  return out;
}

void antinoise_batch(or_sum* s, int C, const or_sum* const* e, const double* q, int order, double eps1) {
  if (C < 1) fail("a batch needs at least one map");
  if (order != 1 && order != 2) fail("order must be 1 or 2");
  const int W = s->W;
  double p0 = 1.0;
  for (int c = 0; c < C; ++c) {
    if (e[c]->W != s->W || e[c]->n != s->n) fail("E' and O must have the same qubit count");
    p0 *= 1.0 - q[c];
  }
  Map o0;
  for (const auto& kv : s->m) o0[kv.first] = kv.second * p0;
  Map o1;
  for (int c = 0; c < C; ++c) {
    const double a = q[c] / (1.0 - q[c]);
    for (const auto& kv : conj_sum(o0, e[c], a, W)) o1[kv.first] += kv.second;
  }
  Map out = o0;
  for (const auto& kv : o1) out[kv.first] += kv.second;
  if (order == 2) {
    if (eps1 > 0.0) threshold(o1, eps1);
    double a2 = 0.0;
    for (int c = 0; c < C; ++c) {
      const double a = q[c] / (1.0 - q[c]);
      a2 += a * a;
      for (const auto& kv : conj_sum(o1, e[c], 0.5 * a, W)) out[kv.first] += kv.second;
    }
    for (const auto& kv : o0) out[kv.first] -= 0.5 * a2 * kv.second;
  }
  erase_zeros(out);
  s->m.swap(out);
}

void apply_layer(or_sum* s, int n_gates, const uint64_t* gx, const uint64_t* gz, const double* theta,
                 int dir, int n_gen, const uint64_t* ex, const uint64_t* ez, const double* lambda,
                 int noise_sign, int noise_after_gates, double eps, int64_t max_terms, int mode,
                 int max_order) {
  const int W = s->W;
  // Truncation of intermediate results (Section I.A): terms with |c| < eps are dropped and
  // at most max_terms of the largest |c| are kept.  Reading used here: both are applied
  // after every non-Clifford gate (merge, then threshold, then cap), and in the error-order
  // mode also after the noise layer.  Clifford gates and the greedy mode's inverse noise
  // never lower a magnitude, so nothing is truncated after them.  Mode 2 (sine order)
  // rescales like the greedy mode and counts sines in the tag (see rotate).
  const bool truncating = eps > 0.0 || max_terms > 0;
  auto do_noise = [&]() {
    if (n_gen <= 0) return;
    noise(s, n_gen, ex, ez, lambda, noise_sign, mode == 2 ? 0 : mode, max_order);
    if (mode == 1 && truncating) truncate(s, eps, max_terms);
  };
  if (!noise_after_gates) do_noise();
  // A layer's gates are in time order.  U^dag P U for U = U_G ... U_1 conjugates by U_G
  // first, so the backward pass walks the list in reverse; the forward pass in order.
  for (int i = 0; i < n_gates; ++i) {
    const int g = dir == 1 ? n_gates - 1 - i : i;
    const int clifford = rotate(s, gx + (size_t)g * W, gz + (size_t)g * W, theta[g], dir, mode == 2 ? max_order : -1);
    if (!clifford && truncating) truncate(s, eps, max_terms);
  }
  if (noise_after_gates) do_noise();
}

}  // namespace

extern "C" {

or_sum* or_create(int n_qubits, int64_t n, const uint64_t* x, const uint64_t* z, const double* c,
                  const uint8_t* ord) {
  if (n_qubits <= 0 || n_qubits > 64 * kMaxWords) fail("n_qubits out of range");
  if (n < 0) fail("negative term count");
  or_sum* s = new or_sum;
  s->n = n_qubits;
  s->W = (n_qubits + 63) / 64;
  const int W = s->W;
  // Bits above n_qubits in the last word must be clear.
  const int top = n_qubits - 64 * (W - 1);
  const uint64_t top_mask = top == 64 ? ~0ULL : ((1ULL << top) - 1);
  s->m.reserve((size_t)n * 2 + 16);
  for (int64_t i = 0; i < n; ++i) {
    if ((x[(size_t)i * W + W - 1] & ~top_mask) || (z[(size_t)i * W + W - 1] & ~top_mask))
      fail("string has bits above n_qubits");
    if (!std::isfinite(c[i])) fail("non-finite coefficient");
    Key k = make_key(W, x + (size_t)i * W, z + (size_t)i * W, ord ? ord[i] : 0);
    s->m[k] += c[i];
  }
  erase_zeros(s->m);
  return s;
}

or_sum* or_clone(const or_sum* s) { return new or_sum(*s); }

void or_free(or_sum* s) { delete s; }

int64_t or_size(const or_sum* s) { return (int64_t)s->m.size(); }

void or_export(const or_sum* s, uint64_t* x, uint64_t* z, double* c, uint8_t* ord) {
  std::vector<std::pair<Key, double>> v(s->m.begin(), s->m.end());
  std::sort(v.begin(), v.end(), [](const std::pair<Key, double>& a, const std::pair<Key, double>& b) {
    return canonical_less(a.first, b.first);
  });
  const int W = s->W;
  for (size_t i = 0; i < v.size(); ++i) {
    for (int w = 0; w < W; ++w) {
      if (x) x[i * W + w] = v[i].first.x[w];
      if (z) z[i * W + w] = v[i].first.z[w];
    }
    if (c) c[i] = v[i].second;
    if (ord) ord[i] = v[i].first.o;
  }
}

int or_rotate(or_sum* s, const uint64_t* rx, const uint64_t* rz, double theta, int dir) {
  return rotate(s, rx, rz, theta, dir);
}

void or_noise(or_sum* s, int n_gen, const uint64_t* ex, const uint64_t* ez, const double* lambda,
              int sign, int mode, int max_order) {
  noise(s, n_gen, ex, ez, lambda, sign, mode, max_order);
}

void or_truncate(or_sum* s, double eps, int64_t max_terms) { truncate(s, eps, max_terms); }

void or_antinoise(or_sum* s, const or_sum* eprime, double q) { antinoise(s, eprime, q); }

void or_antinoise_batch(or_sum* s, int C, const or_sum* const* eprimes, const double* q, int order,
                        double eps1) {
  antinoise_batch(s, C, eprimes, q, order, eps1);
}

void or_antinoise_topk(or_sum* s, const or_sum* eprime, double q, int64_t k) {
  antinoise_topk(s, eprime, q, k);
}

void or_apply_layer(or_sum* s, int n_gates, const uint64_t* gx, const uint64_t* gz,
                    const double* theta, int dir, int n_gen, const uint64_t* ex, const uint64_t* ez,
                    const double* lambda, int noise_sign, int noise_after_gates, double eps,
                    int64_t max_terms, int mode, int max_order) {
  apply_layer(s, n_gates, gx, gz, theta, dir, n_gen, ex, ez, lambda, noise_sign, noise_after_gates,
              eps, max_terms, mode, max_order);
}

// O~ = D O, D = (C_ideal C_noisy^{-1})^dag (Section I.B).  With C_noisy = N_M G_M ... N_1 G_1
// and C_ideal = G_M ... G_1 (channels on states), C_ideal C_noisy^{-1} =
// G_M..G_2 N_1^{-1} G_2^{-1} N_2^{-1} ... G_M^{-1} N_M^{-1} (the G_1 pair cancels), and the
// adjoint of that product, applied to O, walks it from the left end inwards in reverse:
// G_M^dag .. G_2^dag (backward, noiseless), then N_1^{-1}, then for m = 2..M the adjoint of
// G_m^{-1} (forward conjugation U P U^dag) followed by N_m^{-1} (Pauli maps are self-adjoint).
or_sum* or_noise_canceling(const or_sum* obs, int n_layers, const int* n_gates, const uint64_t* gx,
                           const uint64_t* gz, const double* theta, const int* n_gen,
                           const uint64_t* ex, const uint64_t* ez, const double* lambda, double eps,
                           int64_t max_terms, int mode, int max_order) {
  if (n_layers <= 0) fail("need at least one layer");
  const int W = obs->W;
  std::vector<size_t> g_off((size_t)n_layers + 1, 0), e_off((size_t)n_layers + 1, 0);
  for (int m = 0; m < n_layers; ++m) {
    g_off[m + 1] = g_off[m] + (size_t)n_gates[m];
    e_off[m + 1] = e_off[m] + (size_t)n_gen[m];
  }
  or_sum* s = new or_sum(*obs);
  auto layer = [&](int m, int dir, bool with_gates, bool with_noise) {
    apply_layer(s, with_gates ? n_gates[m] : 0, gx + g_off[m] * W, gz + g_off[m] * W,
                theta + g_off[m], dir, with_noise ? n_gen[m] : 0, ex + e_off[m] * W,
                ez + e_off[m] * W, lambda + e_off[m], +1, 1, eps, max_terms, mode, max_order);
  };
  // The sine-order mode expands D over every gate of C_ideal, the first layer's included
  // (the Euclid appendix's diagrams run over j = 1..N in both halves), so it keeps the
  // G_1^dag G_1 pair: with a cut on the number of sines its two halves no longer cancel.
  const int first = mode == 2 ? 0 : 1;
  for (int m = n_layers - 1; m >= first; --m) layer(m, +1, true, false);  // G_M^dag .. G_2^dag (.. G_1^dag)
  layer(0, -1, first == 0, true);                                         // (G_1, then) N_1^{-1}
  for (int m = 1; m < n_layers; ++m) layer(m, -1, true, true);            // G_m, then N_m^{-1}
  return s;
}

double or_expectation(const or_sum* s, const uint64_t* basis) {
  std::vector<std::pair<Key, double>> v(s->m.begin(), s->m.end());
  std::sort(v.begin(), v.end(), [](const std::pair<Key, double>& a, const std::pair<Key, double>& b) {
    return canonical_less(a.first, b.first);
  });
  long double acc = 0.0L;
  for (const auto& kv : v) {
    bool diag = true;
    int par = 0;
    for (int w = 0; w < s->W; ++w) {
      if (kv.first.x[w]) diag = false;
      if (basis) par += popc(kv.first.z[w] & basis[w]);
    }
    if (!diag) continue;
    acc += (par & 1) ? -(long double)kv.second : (long double)kv.second;
  }
  return (double)acc;
}

double or_norm2(const or_sum* s) {
  long double acc = 0.0L;
  for (const auto& kv : s->m) acc += (long double)kv.second * kv.second;
  return (double)acc;
}

}  // extern "C"
