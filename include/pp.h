/*
 * pp.h -- C ABI of the MI355X (gfx950) noise-canceling Pauli-propagation library.
 *
 * The library computes the noise-canceling observable O~ = D O,
 * D = (C_ideal C_noisy^{-1})^dag, of Eddins et al., "Computing noise-canceling
 * observables via Pauli propagation" (Section I.B, the trace identity
 * <O> = Tr[D O rho] with rho = C_noisy |0><0|), by Heisenberg-picture Pauli
 * propagation of a real-coefficient Pauli sum held on the GPU.  A caller drives it
 * one circuit layer at a time (pp_apply_layer); the order of layers that realises D
 * for a layered circuit is the caller's (the Python package provides it).
 *
 * Pauli strings.  A string on n qubits is two bit vectors x, z of W = ceil(n/64)
 * little-endian uint64 words each (qubit q in word q/64, bit q%64); the operator is
 * the Hermitian Pauli i^{|x&z|} X^x Z^z, so (x_q, z_q) = (1,1) is Y.  1 <= n <= 256.
 * Host arrays of strings are row-major [count][W].
 *
 * Conventions for every entry point:
 *  - Ownership: host arrays passed in are read during the call only; the caller keeps
 *    them.  Device memory is owned by the library (allocated through the allocator
 *    given to pp_ctx_create, else hipMalloc) and released by pp_destroy.
 *  - Errors: every call returns a pp_status; no C++ exception crosses the ABI.  A
 *    validation failure (PP_ERR_INVALID, PP_ERR_UNSUPPORTED) leaves the observable
 *    unchanged.  PP_ERR_OOM or PP_ERR_DEVICE leaves it unusable (destroy it).
 *    pp_last_error() returns a thread-local message for the last failure.
 *  - Streams: all GPU work is enqueued on the context's stream.  pp_apply_layer and
 *    pp_truncate synchronise that stream internally to read term counts (the arrays
 *    are resized per layer), so they return with the layer complete.  Inside a layer
 *    whose cap binds, the gates' passes and the cut after each of them are selected and
 *    applied on the device: the host enqueues gate after gate without waiting, and reads
 *    each gate's counters (statistics, retiling decisions) while the next one runs.
 *    pp_size, pp_expectation and pp_export return host values and therefore also
 *    synchronise.
 *  - Threads: a context and its observables must be used by one host thread at a time;
 *    different contexts may be driven concurrently from different threads.
 */
#ifndef PP_H
#define PP_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  PP_OK = 0,
  PP_ERR_INVALID = 1,      /* bad argument; nothing changed */
  PP_ERR_OOM = 2,          /* device allocation failed; observable unusable */
  PP_ERR_DEVICE = 3,       /* HIP runtime error; observable unusable */
  PP_ERR_UNSUPPORTED = 4   /* valid but not supported by this build; nothing changed */
} pp_status;

/* Coefficient storage.  PP_F64: FP64 throughout.  PP_F32_KAHAN: FP32 coefficients in
 * HBM; each rotation's cos/sin combination is evaluated in FP64 and rounded once,
 * duplicate-string merges use compensated (Kahan) sums, inverse-noise scale factors
 * are accumulated in FP64 and the expectation value is reduced in FP64. */
typedef enum { PP_F64 = 0, PP_F32_KAHAN = 1 } pp_precision;

/* Truncation mode.  PP_MODE_GREEDY: propagated noise absorption's greedy truncation
 * (Section I.A): drop |c| < eps and keep at most max_terms of the largest |c|.
 * PP_MODE_ERROR_ORDER: each term carries an error-order tag (uint8); every inverse
 * Pauli-Lindblad layer multiplies a Pauli P by prod_{k: <P,E_k>=1} (1 + x_k),
 * x_k = f_k - 1 with f_k the generator's inverse fidelity factor, and that product is
 * expanded in powers of the x_k: a term of order o receives the degree-j elementary
 * symmetric sum of its anticommuting x_k at order o + j, orders above max_order are
 * dropped, and terms are merged by (string, order) (the expansion in the number of
 * errors of Appendix C; the Euclid appendix's first-order form 1/f ~ 1 + eps).
 * PP_MODE_SINE_ORDER: the tag counts the sine factors along a term's path, the CPT order
 * kappa = k + 2p of the Euclid appendix (k steps and p bubbles, one sine per step): the
 * sin child of a non-Clifford rotation gets tag + 1 and is dropped above max_order
 * (0..250), Clifford rotations do not count, the noise rescales as in PP_MODE_GREEDY, and
 * terms merge by (string, tag).  With max_terms > 0 the gates of a layer go through the
 * tiled gate passes with the cap's cut on the device, as in PP_MODE_GREEDY; without a cap,
 * through the per-gate sort-and-merge path.  pp_apply_layer writes each layer in the
 * Clifford interaction picture of the Euclid appendix before propagating: a rotation by
 * theta becomes the exact Clifford rotation by the nearest multiple k pi/2 followed by one
 * by the residual theta - k pi/2 (at most pi/4, so every counted sine is at most
 * 1/sqrt 2); whole turns are dropped.  <O~> sums all tags.
 * The Euclid appendix expands D over every gate of C_ideal, the first layer's included, so
 * a caller building D in this mode keeps the G_1^dag G_1 pair. */
typedef enum { PP_MODE_GREEDY = 0, PP_MODE_ERROR_ORDER = 1, PP_MODE_SINE_ORDER = 2 } pp_mode;

/* Direction of a gate layer.  PP_HEISENBERG: P -> U^dag P U = cos P + sin (i R P) for
 * anticommuting P (backward rule of the Euclid appendix); gates are applied in reverse
 * list order.  PP_FORWARD: P -> U P U^dag = cos P - sin (i R P) (Section I,
 * Eq. evolve_gate); gates in list order.  U = exp(-i theta R / 2). */
typedef enum { PP_HEISENBERG = 1, PP_FORWARD = -1 } pp_dir;

typedef struct {
  double eps;          /* drop |c| < eps after every non-Clifford gate (>= 0) */
  int64_t max_terms;   /* after every non-Clifford gate (after the eps threshold) keep at
                          most this many of the largest |c| (0 = no cap); ties in |c| go
                          to the smaller canonical key (Section I.A's K_O) */
  int max_order;       /* PP_MODE_ERROR_ORDER: highest kept order (0..250) */
} pp_trunc;

/* One circuit layer.  Gates: n_gates Pauli rotations R_g (gx, gz: [n_gates][W]) with
 * angles theta[g].  Angles within 1e-12 of a multiple of pi/2 are Clifford and use
 * exact cos/sin in {0, +-1}; nothing is truncated after a Clifford gate.
 * Noise: n_gen Pauli-Lindblad generators E_k (ex, ez: [n_gen][W]) with strengths
 * lambda[k] >= 0 (Section I: the local channel applies E_k with probability
 * p_k = (1 - e^{-2 lambda_k})/2).  noise_sign = +1 applies the inverse map
 * (Eq. evolve_noise: an anticommuting P is multiplied by 1 - 2 q_k = e^{2 lambda_k});
 * -1 applies the channel (factor e^{-2 lambda_k}).  noise_after_gates selects whether
 * the noise map follows (1) or precedes (0) the gates.  Either count may be 0. */
typedef struct {
  int n_gates;
  const uint64_t* gx;
  const uint64_t* gz;
  const double* theta;
  int dir;                 /* pp_dir */
  int n_gen;
  const uint64_t* ex;
  const uint64_t* ez;
  const double* lambda;
  int noise_sign;          /* +1 inverse map, -1 channel */
  int noise_after_gates;   /* 1: gates then noise; 0: noise then gates */
} pp_layer;

typedef struct pp_ctx pp_ctx;
typedef struct pp_obs pp_obs;

/* Device allocator hooks (e.g. a framework's caching allocator).  alloc returns NULL
 * on failure; release may be called with any pointer alloc returned. */
typedef void* (*pp_alloc_fn)(size_t bytes, void* user);
typedef void (*pp_release_fn)(void* ptr, void* user);

/* Create a context on HIP device `device` that enqueues on `hip_stream` (a
 * hipStream_t; NULL = the null stream).  alloc/release may both be NULL (then
 * hipMalloc/hipFree with an internal buffer cache).  *out receives the handle. */
pp_status pp_ctx_create(int device, void* hip_stream, pp_alloc_fn alloc, pp_release_fn release,
                        void* user, pp_ctx** out);
void pp_ctx_destroy(pp_ctx* ctx);

/* Create an observable O = sum_i coeff[i] P_i on the device (step "create": the host
 * strings are copied, duplicated strings are summed and exact zeros dropped; Appendix B's
 * accumulate-and-deduplicate).  n_terms >= 0; x, z: [n_terms][W] host arrays with no bits
 * at or above n_qubits; coeff finite.  trunc configures every later pp_apply_layer. */
pp_status pp_create_observable(pp_ctx* ctx, int n_qubits, int64_t n_terms, const uint64_t* x,
                               const uint64_t* z, const double* coeff, pp_precision precision,
                               pp_mode mode, pp_trunc trunc, pp_obs** out);

/* Replace the terms of an existing observable, as pp_create_observable would set them
 * (duplicates summed, exact zeros dropped, tags zero), keeping its context, qubit count,
 * precision, mode, truncation and device buffers.  For callers that propagate many small
 * sums in turn (the forward-evolved errors of PNA) without creating and freeing an
 * observable each time.  Arguments and errors as pp_create_observable's; on an error the
 * previous terms may be lost (the observable then holds no terms). */
pp_status pp_set_terms(pp_obs* obs, int64_t n_terms, const uint64_t* x, const uint64_t* z, const double* coeff);

/* Propagate through one layer (gates, then or preceded by, a Pauli-Lindblad map):
 * rotation branching per gate with the cos/sin split (Eq. evolve_gate and its backward
 * form), duplicate strings merged after every gate, and after every non-Clifford gate
 * |c| < eps dropped and then the max_terms cap (Section I.A's truncation of intermediate
 * results); the inverse-noise rescale by exp(2 noise_sign sum_{k anticommuting} lambda_k)
 * (Eq. evolve_noise), not followed by a truncation in PP_MODE_GREEDY; in
 * PP_MODE_ERROR_ORDER the expansion described above, followed by the eps threshold per
 * (string, order) and the max_terms cap. */
pp_status pp_apply_layer(pp_obs* obs, const pp_layer* layer);

/* Absorb one propagated antinoise map into the observable (Section I.A, Eq.
 * applyantinoise): O -> (1 - q) O + q E' O E'.  E' = sum_a e_a P_a is the observable
 * `eprime`, normally one noise generator E evolved to the end of the circuit, U E U^dag
 * (Eq. channel_prop; pp_apply_layer with PP_FORWARD over the later layers, noise off).
 * lambda is that generator's strength (finite, 0 <= lambda <= 300, else PP_ERR_INVALID);
 * the library takes the inverse map's quasi-probability q = (1 - e^{2 lambda})/2 <= 0
 * (Section I: the channel applies E with probability (1 - e^{-2 lambda})/2, the inverse
 * negates lambda).
 * Each term of O expands into 1 + K(K-1)/2 strings for K = |E'| (P itself, and one string
 * per unordered pair of E' terms), duplicates are merged, then |c| < eps and the max_terms
 * cap of obs's pp_trunc are applied; eprime is not changed.  Both observables must share
 * the context, qubit count and precision (PP_ERR_INVALID otherwise) and be in
 * PP_MODE_GREEDY (PP_ERR_UNSUPPORTED otherwise).  PP_ERR_UNSUPPORTED as well when
 * K > 4096 or the expansion exceeds 2^31 - 1 strings; obs is then unchanged. */
pp_status pp_apply_antinoise(pp_obs* obs, const pp_obs* eprime, double lambda);

/* A batch of n_maps commuting antinoise maps (e.g. generators of one layer) absorbed at
 * once, expanded in the number of errors (Appendix C): with a_c = q_c / (1 - q_c) and
 * C_c(X) = E'_c X E'_c, O0 = O prod (1 - q_c), O1 = sum_c a_c C_c(O0), and for order 2
 * also O2 = 1/2 sum_c (a_c C_c(O1') - a_c^2 O0), where O1' is O1 without its terms below
 * obs's eps (the second pass's input only); O becomes O0 + O1 (+ O2), then |c| < eps and
 * the max_terms cap of obs's pp_trunc apply.  Exact for n_maps = 1; the error of a
 * batch is of order (q C)^2 (order 1) or (q C)^3 (order 2).  eprimes: n_maps observables
 * sharing O's context, qubit count and precision, in PP_MODE_GREEDY; lambda: the n_maps
 * generators' strengths (host array, each as for pp_apply_antinoise), q_c taken from
 * lambda_c as there.  All maps of the batch are expanded into one buffer and merged
 * once, instead of one sort per map.  Errors as pp_apply_antinoise (PP_ERR_INVALID for
 * n_maps < 1 or order not 1 or 2). */
pp_status pp_apply_antinoise_batch(pp_obs* obs, const pp_obs* const* eprimes, const double* lambda, int n_maps,
                                   int order);

/* As pp_apply_antinoise, with E' O E' approximated by its most significant products
 * (Appendix B, the heuristic conjugation of large Pauli sums): of the products P_a P P_b
 * with a != b over ordered triplets (a, term of O, b), only those whose magnitude
 * |c_P| (|e_a| |e_b|) is among the max_products largest enter; every product tied with
 * the max_products-th is kept as well, so both orders of a pair stay together and the
 * result is Hermitian.  The (1 - q) O part and the products with a = b (P_a P P_a = +-P,
 * which cancel (1 - q) on terms that commute with E') are exact, so a walk of limited
 * updates does not inflate O.  max_products <= 0, or at least |O| K (K - 1), gives
 * pp_apply_antinoise's result.  The pair magnitudes are sorted on the device; K <= 16384
 * (PP_ERR_UNSUPPORTED otherwise).  Only the kept products are expanded, so the 2^31 - 1
 * limit applies to |O| + (kept unordered pairs); other arguments and errors as
 * pp_apply_antinoise. */
pp_status pp_apply_antinoise_topk(pp_obs* obs, const pp_obs* eprime, double lambda, int64_t max_products);

/* Explicit greedy truncation: drop |c| < eps, then keep the max_terms largest |c|
 * (0 = no cap; ties to the smaller canonical key).  E.g. the K_M leading terms of
 * Section I.C's estimation step. */
pp_status pp_truncate(pp_obs* obs, double eps, int64_t max_terms);

/* <b| O |b> = sum over terms with x = 0 of c (-1)^{|z & b|} (Section I.B's <O> for a
 * computational-basis state), reduced in FP64 on the device; basis: W host words, or
 * NULL for |0...0>.  In PP_MODE_ERROR_ORDER all orders are summed. */
pp_status pp_expectation(pp_obs* obs, const uint64_t* basis, double* out);

/* For callers that cannot allocate device memory (code under HIP graph capture, tight
 * serving loops, harnesses that forbid hipMalloc): pp_expectation without any allocation.
 * Same arguments, result and errors as pp_expectation, up to the order of the FP64 sum (the
 * terms' storage order here, canonical order there: the two differ by rounding only).  The
 * block partials live in a fixed device array of 2080 doubles (16.6 KB) per GPU, held until
 * the process ends; the workgroups stride over the terms, so an observable of any size fits
 * in it.  Every call on one GPU shares that array: calls that overlap on one GPU (several
 * host threads, or several streams) race and must be serialised by the caller.  The array's
 * address is taken when the first context is created on a device. */
pp_status pp_expectation_noalloc(pp_obs* obs, const uint64_t* basis, double* out);

/* Current number of terms (distinct (string, order) entries). */
pp_status pp_size(pp_obs* obs, int64_t* out);

/* Copy all terms to host arrays sized by pp_size: x, z [n][W], c [n] (FP64), ord [n]
 * (0 in greedy mode), in canonical order: x words compared from word W-1 down, then z
 * words likewise, then order.  Any output pointer may be NULL. */
pp_status pp_export(pp_obs* obs, uint64_t* x, uint64_t* z, double* c, uint8_t* ord);

void pp_destroy(pp_obs* obs);

/* Thread-local message of the last failed call on this thread ("" if none). */
const char* pp_last_error(void);

/* ---- instrumentation (not part of the method) ---------------------------------------
 * When enabled, every kernel launch of the context is bracketed by HIP events on the
 * context's stream, and per-kernel-name totals (launch count, summed device time,
 * summed algorithmic bytes) are accumulated until read.  pp_timing_read fills up to
 * `cap` records and returns the number of distinct kernel names. */
typedef struct {
  char name[48];
  int64_t launches;
  double total_ms;
  double algo_bytes;     /* terms loaded plus terms written by the launches, times the term
                            size: one read and one write of what each pass handled */
  double items;          /* terms processed (term-updates for layer kernels) */
  double layer_bytes;    /* the launches' share of their layer calls' algorithmic bytes
                            (N_in + N_out) B: algo_bytes / G for the passes of a layer whose G
                            gates run one pass each, algo_bytes otherwise */
} pp_kernel_stat;

pp_status pp_timing_enable(pp_ctx* ctx, int enable);
int pp_timing_read(pp_ctx* ctx, pp_kernel_stat* out, int cap, int reset);

/* Per-layer counters of the last pp_apply_layer on this observable. */
typedef struct {
  int64_t n_in;            /* terms entering the layer */
  int64_t n_out;           /* terms after the layer */
  int64_t n_peak;          /* largest intermediate count */
  int64_t n_fallback;      /* terms routed to the per-gate path */
  int64_t n_capped;        /* terms removed by the caps of this layer */
  double dropped_l1;       /* sum of |c| removed by thresholds and the cap */
} pp_layer_stats;

pp_status pp_last_layer_stats(pp_obs* obs, pp_layer_stats* out);

#ifdef __cplusplus
}
#endif
#endif /* PP_H */
