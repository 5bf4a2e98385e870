/*
 * pp_oracle.h -- plain CPU FP64 reference for noise-canceling Pauli propagation.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the package's smoke check and the
 * CPU-baseline leg of the benchmark may load this library.  The product path never
 * links, loads or calls it, and it shares no code with the HIP library.
 *
 * What it computes (Eddins et al., "Computing noise-canceling observables via Pauli
 * propagation"):
 *   - Pauli rotation past U = exp(-i theta R / 2), forward U P U^dag (Section I,
 *     Eq. evolve_gate) and backward U^dag P U (Appendix "Details on Euclid theory",
 *     the backward rule beside Eq. evolve_noise_fid);
 *   - Pauli-Lindblad channels and their inverses on a Pauli, (1 - 2q)^<P,E> P
 *     (Section I, Eq. evolve_noise, with p = (1 - e^{-2 lambda})/2 and lambda -> -lambda
 *     for the inverse);
 *   - the noise-canceling observable O~ = D O with D = (C_ideal C_noisy^{-1})^dag
 *     (Section I.B, the trace identity), under greedy |c| truncation (Section I.A)
 *     or with the inverse-noise factors expanded in powers of the error generators
 *     and cut at a maximum order (Appendix C's expansion in the number of errors);
 *   - <b| O~ |b> on a computational basis state.
 *
 * Strings: x and z bit vectors of W = ceil(n/64) uint64 words, qubit q in word q/64,
 * bit q%64; the Pauli is the Hermitian i^{|x&z|} X^x Z^z (Y = (1,1)).  n <= 256.
 * Every array argument is host memory owned by the caller.  Functions abort the
 * process with a message on invalid input (this is a checker, not a product).
 */
#ifndef PP_ORACLE_H
#define PP_ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct or_sum or_sum;   /* a Pauli sum: map (x, z, order) -> real coefficient */

/* Build a sum from n terms; duplicated (string, order) entries are added and exact
 * zeros dropped.  ord may be NULL (all orders 0). */
or_sum* or_create(int n_qubits, int64_t n, const uint64_t* x, const uint64_t* z,
                  const double* c, const uint8_t* ord);
or_sum* or_clone(const or_sum* s);
void    or_free(or_sum* s);
int64_t or_size(const or_sum* s);
/* Export in canonical order: x words (word W-1 most significant) first, then z words,
 * then order.  Any of the output pointers may be NULL. */
void    or_export(const or_sum* s, uint64_t* x, uint64_t* z, double* c, uint8_t* ord);

/* One Pauli rotation, no truncation.  dir = +1: U^dag P U (Heisenberg, backward);
 * dir = -1: U P U^dag (forward). Returns 1 if the angle was treated as Clifford. */
int     or_rotate(or_sum* s, const uint64_t* rx, const uint64_t* rz, double theta, int dir);

/* One Pauli-Lindblad layer (all generators), no truncation.  sign = +1 applies the
 * inverse map, sign = -1 the channel itself.  mode 0: the local channels one after the
 * other in list order, each multiplying an anticommuting string by its f_k; mode 1: expand
 * the product in the anticommuting generators' (f_k - 1) and keep total order <= max_order,
 * tagging each term with its order. */
void    or_noise(or_sum* s, int n_gen, const uint64_t* ex, const uint64_t* ez,
                 const double* lambda, int sign, int mode, int max_order);

/* Drop |c| < eps; then, if more than max_terms remain (max_terms > 0), keep the
 * max_terms largest |c| (ties: smaller canonical key first). */
void    or_truncate(or_sum* s, double eps, int64_t max_terms);
/* O -> (1 - q) O + q E' O E' for E' = eprime (Section I.A, Eq. applyantinoise); exact zeros
 * dropped, no other truncation.  eprime must have the same qubit count. */
void    or_antinoise(or_sum* s, const or_sum* eprime, double q);
/* As or_antinoise, with E' O E' limited to the products P_i P P_j (i != j) of the k largest
 * |alpha||beta_i||beta_j| (Appendix B's heuristic conjugation); ties with the k-th kept; the
 * products with i = j (P_i P P_i = +-P) are always kept. */
void    or_antinoise_topk(or_sum* s, const or_sum* eprime, double q, int64_t k);
/* A batch of C commuting antinoise maps to first (order 1) or second (order 2) order in
 * the number of errors (Appendix C); exact for C = 1; the second-order pass takes the
 * first-order part with |c| < eps1 dropped; no other truncation. */
void    or_antinoise_batch(or_sum* s, int C, const or_sum* const* eprimes, const double* q, int order,
                           double eps1);

/* One circuit layer with the truncation schedule of the propagation:
 *   [noise if !noise_after_gates] ; gates (dir = +1: reverse list order, U^dag P U;
 *   dir = -1: list order, U P U^dag), after every non-Clifford gate: drop |c| < eps, then
 *   keep the max_terms largest (max_terms > 0) ; [noise if noise_after_gates].  In mode 1
 *   the same truncation follows the noise.  Mode 2 (sine order): noise as in mode 0, and
 *   the tag counts the sine factors of a term's path (the sin child of a non-Clifford
 *   rotation gets tag + 1; tags above max_order are dropped).  n_gates or n_gen may be 0. */
void    or_apply_layer(or_sum* s, int n_gates, const uint64_t* gx, const uint64_t* gz,
                       const double* theta, int dir, int n_gen, const uint64_t* ex,
                       const uint64_t* ez, const double* lambda, int noise_sign,
                       int noise_after_gates, double eps, int64_t max_terms, int mode,
                       int max_order);

/* The noise-canceling observable of a layered circuit (layer m = gates G_m then noise
 * N_m, m = 1..M, arrays concatenated over layers):
 *   O~ = N_M^{-1} G_M ... N_2^{-1} G_2 N_1^{-1} G_2^dag ... G_M^dag (O)
 * i.e. backward (Heisenberg) through G_M..G_2, then N_1^{-1}, then for m = 2..M forward
 * through G_m and N_m^{-1}.  In mode 2 (sine order) the first layer's pair is kept:
 * backward through G_M..G_1, then forward through G_1 and N_1^{-1}, then as above (the
 * Euclid appendix expands D over every gate of C_ideal).  Truncation as in
 * or_apply_layer, per layer call. */
or_sum* or_noise_canceling(const or_sum* obs, int n_layers, const int* n_gates,
                           const uint64_t* gx, const uint64_t* gz, const double* theta,
                           const int* n_gen, const uint64_t* ex, const uint64_t* ez,
                           const double* lambda, double eps, int64_t max_terms, int mode,
                           int max_order);

/* <b| S |b> = sum over terms with x = 0 of c (-1)^{|z & b|}; basis = W words or NULL (|0>). */
double  or_expectation(const or_sum* s, const uint64_t* basis);
/* Sum of c^2 (the Pauli 2-norm squared, invariant under unitary conjugation). */
double  or_norm2(const or_sum* s);

#ifdef __cplusplus
}
#endif
#endif
