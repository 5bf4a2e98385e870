// pp_api.hip -- host orchestration and the C ABI (include/pp.h) of the gfx950 library.
//
// Per layer (pp_apply_layer) the host classifies the gates, uploads them in application
// order with their exact or libm cos/sin, and enqueues:
//   * all-Clifford layer: one elementwise kernel (strings map one-to-one; no merging);
//   * a run of X-type (z-preserving) or Z-type (x-preserving) rotations: group-hash radix
//     passes, tile boundaries, then the fused LDS layer kernel (all gates of the run, the
//     per-gate merge and threshold, and the noise map when it follows);
//   * any other rotation: the same fused kernel with one gate, grouped by its pair key;
//   * tiles that outgrow LDS: the per-gate path (expand, canonical sort, segmented sum);
//   * the cap: radix select on |c| with ties ranked by canonical key, then compaction.
#include "../../include/pp.h"

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstddef>
#include <cstring>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <utility>
#include <vector>

#include "pp_common.hpp"
#include "pp_gate.hpp"
#include "pp_layer.hpp"
#include "pp_misc.hpp"
#include "pp_select.hpp"
#include "pp_sort.hpp"

using namespace pp;

#ifndef PP_LEVEL0_WAVE
#define PP_LEVEL0_WAVE 1   // first attempt with one-wavefront tiles (else 1024-thread tiles)
#endif

namespace {

thread_local std::string g_last_error;

struct Failure {
  pp_status status;
  std::string msg;
};

[[noreturn]] void throw_fail(pp_status s, const std::string& m) { throw Failure{s, m}; }

#define HIPCHK(expr)                                                                        \
  do {                                                                                      \
    hipError_t e_ = (expr);                                                                 \
    if (e_ != hipSuccess) throw_fail(PP_ERR_DEVICE, std::string(#expr) + ": " + hipGetErrorString(e_)); \
  } while (0)

inline uint64_t cdiv(uint64_t a, uint64_t b) { return (a + b - 1) / b; }
inline int ceil_log2(uint64_t v) { int k = 0; while ((1ULL << k) < v) ++k; return k; }
inline int floor_log2(uint64_t v) { int k = 0; while ((2ULL << k) <= v) ++k; return k; }

}  // namespace

// ---------------------------------------------------------------------------------------------
// Scratch of the allocation-free expectation (pp_expectation_noalloc): one FP64 partial per
// workgroup of k_expect (at most kNoAllocBlocks) and the reduced value after them.  Each GPU
// the library runs on holds its own copy until the process ends.  Host code never passes the
// array's name to a kernel: it uses the device address that hipGetSymbolAddress returned for
// the current device when a context was created there (scratch_of).
// ---------------------------------------------------------------------------------------------
constexpr unsigned kNoAllocBlocks = 2048;
static __device__ __align__(256) double scratch[kNoAllocBlocks + 32];

namespace {
std::mutex g_scratch_mu;
std::vector<double*> g_scratch_addr;   // per device ordinal, set by pp_ctx_create

// Record this device's address of `scratch` (the device must be current).  Called once per
// device, at the first context created on it.
void register_scratch(int device, int count) {
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if ((int)g_scratch_addr.size() < count) g_scratch_addr.resize((size_t)count, nullptr);
  if (g_scratch_addr[(size_t)device]) return;
  void* p = nullptr;
  HIPCHK(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
  if (!p) throw_fail(PP_ERR_DEVICE, "hipGetSymbolAddress returned no address for the scratch array");
  g_scratch_addr[(size_t)device] = (double*)p;
}

double* scratch_of(int device) {
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (device < 0 || (size_t)device >= g_scratch_addr.size()) return nullptr;
  return g_scratch_addr[(size_t)device];
}
}  // namespace

// ---------------------------------------------------------------------------------------------
// Context
// ---------------------------------------------------------------------------------------------
struct pp_ctx {
  int device = 0;
  hipStream_t stream = nullptr;
  pp_alloc_fn alloc = nullptr;
  pp_release_fn release = nullptr;
  void* user = nullptr;
  uint64_t* pinned = nullptr;   // host-pinned scratch for counters
  bool timing = false;
  struct Pending {
    std::string name;
    hipEvent_t a, b;
    double bytes, items, share;
  };
  std::vector<Pending> pending;
  struct Acc {
    int64_t launches = 0;
    double ms = 0, bytes = 0, items = 0, layer_bytes = 0;
  };
  // Share of its layer call's algorithmic bytes (N_in + N_out) B that one pass of the
  // current kernel stands for: 1 / G while a layer's G gates run one pass each, else 1.
  double pass_share = 1.0;
  std::map<std::string, Acc> acc;
  std::vector<hipEvent_t> evfree;

  void* dalloc(size_t b) {
    if (b == 0) b = 256;
    void* p = nullptr;
    if (alloc) {
      p = alloc(b, user);
    } else if (hipMalloc(&p, b) != hipSuccess) {
      (void)hipGetLastError();
      p = nullptr;
    }
    if (!p) throw_fail(PP_ERR_OOM, "device allocation of " + std::to_string(b) + " bytes failed");
    return p;
  }
  void dfree(void* p) {
    if (!p) return;
    if (release) release(p, user);
    else (void)hipFree(p);
  }
  hipEvent_t ev() {
    if (!evfree.empty()) {
      hipEvent_t e = evfree.back();
      evfree.pop_back();
      return e;
    }
    hipEvent_t e;
    HIPCHK(hipEventCreate(&e));
    return e;
  }
  // Enqueue `f` bracketed by events when timing is on.  Returns the pending index or -1.
  template <class F>
  int run(const char* name, double bytes, double items, F&& f) {
    if (!timing) {
      f();
      return -1;
    }
    Pending p{name, ev(), ev(), bytes, items, pass_share};
    HIPCHK(hipEventRecord(p.a, stream));
    f();
    HIPCHK(hipEventRecord(p.b, stream));
    pending.push_back(p);
    return (int)pending.size() - 1;
  }
  void collect() {
    if (pending.empty()) return;
    HIPCHK(hipStreamSynchronize(stream));
    for (auto& p : pending) {
      float ms = 0.f;
      HIPCHK(hipEventElapsedTime(&ms, p.a, p.b));
      Acc& a = acc[p.name];
      a.launches += 1;
      a.ms += ms;
      a.bytes += p.bytes;
      a.layer_bytes += p.bytes * p.share;
      a.items += p.items;
      evfree.push_back(p.a);
      evfree.push_back(p.b);
    }
    pending.clear();
  }
  void check_launch() {
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) throw_fail(PP_ERR_DEVICE, std::string("kernel launch: ") + hipGetErrorString(e));
  }
};

namespace {

struct Buf {
  pp_ctx* ctx = nullptr;
  void* p = nullptr;
  size_t bytes = 0;
  void ensure(size_t b) {
    if (b <= bytes) return;
    release();
    const size_t nb = b + b / 4 + 256;
    p = ctx->dalloc(nb);
    bytes = nb;
  }
  void release() {
    if (p) ctx->dfree(p);
    p = nullptr;
    bytes = 0;
  }
  template <class T>
  T* as() const { return (T*)p; }
};

template <class CT, bool ORD>
struct TBuf {
  Buf mem;
  uint64_t cap = 0;
  int W = 1;
  static size_t bytes_for(int W, uint64_t n) {
    return (size_t)n * (16 * W + sizeof(CT) + (ORD ? 1 : 0)) + 1024;
  }
  void ensure(uint64_t n) {   // contents are NOT preserved
    if (n <= cap) return;
    const uint64_t nc = std::max<uint64_t>(n + n / 4, 4096);
    mem.release();
    mem.ensure(bytes_for(W, nc));
    cap = nc;
  }
  Terms<CT> view() const {
    Terms<CT> t;
    char* b = (char*)mem.p;
    t.x = (uint64_t*)b;
    t.z = t.x + (size_t)W * cap;
    t.c = (CT*)(t.z + (size_t)W * cap);
    t.o = ORD ? (uint8_t*)(t.c + cap) : nullptr;
    t.stride = cap;
    return t;
  }
  void swap(TBuf& o) {
    std::swap(mem.p, o.mem.p);
    std::swap(mem.bytes, o.mem.bytes);
    std::swap(cap, o.cap);
  }
};

// Clifford test and cos/sin: multiples of pi/2 (within 1e-12 of the quotient) are exact.
bool angle_cos_sin(double theta, double* c, double* s) {
  const double q = theta / (M_PI / 2);
  const double r = std::nearbyint(q);
  if (std::fabs(q - r) < 1e-12) {
    const long k = (((long)r) % 4 + 4) % 4;
    const double cc[4] = {1.0, 0.0, -1.0, 0.0};
    const double ss[4] = {0.0, 1.0, 0.0, -1.0};
    *c = cc[k];
    *s = ss[k];
    return true;
  }
  *c = std::cos(theta);
  *s = std::sin(theta);
  return false;
}

enum GateKind { KIND_X = 0, KIND_Z = 1, KIND_OTHER = 2, KIND_NOISE = 3 };

// Tables of the linear key hash.  Every key bit gets a pseudo-random 32-bit word; the table
// entry of (plane, byte, value) is the XOR of the words of the bits set in `value`, so the
// hash of a key is the XOR of its bits' words -- a GF(2)-linear map.
const std::vector<uint32_t>& hash_tables() {
  static const std::vector<uint32_t> t = [] {
    std::vector<uint32_t> v(kHashTabWords);
    for (int pb = 0; pb < 2 * PP_MAXW * 8; ++pb) {   // (plane, byte) position
      uint32_t basis[8];
      for (int i = 0; i < 8; ++i)
        basis[i] = (uint32_t)(mix64(0x243f6a8885a308d3ULL * (uint64_t)(pb * 8 + i + 1)) >> 32);
      for (int val = 0; val < 256; ++val) {
        uint32_t h = 0;
        for (int i = 0; i < 8; ++i)
          if (val >> i & 1) h ^= basis[i];
        v[(size_t)pb * 256 + val] = h;
      }
    }
    return v;
  }();
  return t;
}

constexpr uint64_t kMaxAntinoiseTerms = 1ULL << 20;   // E' terms per antinoise update
constexpr uint64_t kExpandSlab = 1ULL << 27;          // expansion slots handled at once
constexpr uint64_t kMaxTopkTerms = 1ULL << 14;        // E' terms of a product-limited update (pairs sorted on the device)

struct HostGate {
  GateDev g;
  int kind;
};

}  // namespace

// ---------------------------------------------------------------------------------------------
// Observable
// ---------------------------------------------------------------------------------------------
struct EngineBase {
  virtual ~EngineBase() = default;
  virtual void create(int64_t n, const uint64_t* x, const uint64_t* z, const double* c) = 0;
  virtual void apply_layer(const pp_layer* L) = 0;
  virtual void truncate(double eps, int64_t cap) = 0;
  virtual void antinoise(const EngineBase* eprime, double q) = 0;
  virtual void antinoise_topk(const EngineBase* eprime, double q, int64_t k) = 0;
  virtual void antinoise_batch(const std::vector<const EngineBase*>& eprimes, const double* q, int order) = 0;
  virtual double expectation(const uint64_t* basis) = 0;
  virtual double expectation_noalloc(const uint64_t* basis, double* dev_scratch) = 0;
  virtual void export_terms(uint64_t* x, uint64_t* z, double* c, uint8_t* o) = 0;
  virtual uint64_t size() const = 0;
};

struct pp_obs {
  pp_ctx* ctx = nullptr;
  int n_qubits = 0;
  int W = 1;
  pp_precision prec = PP_F64;
  pp_mode mode = PP_MODE_GREEDY;
  pp_trunc trunc{0.0, 0, 2};
  bool broken = false;
  pp_layer_stats last{};
  std::unique_ptr<EngineBase> eng;
};

namespace {

template <int W, class CT, bool ORD>
struct Engine final : EngineBase {
  static constexpr int CAP = LayerCfg<W>::CAP;
  static constexpr int BLOCK = LayerCfg<W>::BLOCK;
  static constexpr double kTermBytes = 16.0 * W + sizeof(CT) + (ORD ? 1 : 0);

  pp_obs* obs;
  pp_ctx* ctx;
  hipStream_t st;
  uint64_t N = 0;
  TBuf<CT, ORD> cur, alt, sa, sb, tmp;
  uint64_t run_bound = 0;   // upper bound of the live count after any gate of the current run
  bool abort_on_full = false;   // a fused attempt that fills its output buffer stops (cap binds)
  bool aborted = false;
  TBuf<double, true> ta, tb;     // tie lists for the cap
  TBuf<CT, ORD> gb;              // boundary candidates of a cap
  Buf u32a, u32b, u32c, scan_scr, tiles, gates_d, sup_d, tab_d, drun_d, dm_d, dval_d, cnt_d, ovf_d, partial_d, f64_d, span_d, htab_d, lstat_d;
  Buf hscr_d, tr_s0, tr_l0, tr_s1, tr_l1, g1_d, g1_ovf, g1_base, g1_base2;   // per-gate tile path
  Buf rl0, rl1, rl2, ovl1, ovl2, tf_flag, tf_pos, tf_list, g1_io, g1_tab, g1_tabmeta, win_hist_d, qlist_d, topk_d, topk_off, sel_d, cscr_d;
  double growth[4] = {4.0, 4.0, 2.0, 3.0};
  double tile_target[4] = {80.0, 80.0, 80.0, 64.0};   // level-0 (one-wavefront) tile targets
  uint64_t last_ntiles = 1, last_ovf_tiles = 0;

  explicit Engine(pp_obs* o) : obs(o), ctx(o->ctx), st(o->ctx->stream) {
    for (auto* t : {&cur, &alt, &sa, &sb, &tmp, &gb}) { t->mem.ctx = ctx; t->W = W; }
    for (auto* t : {&ta, &tb}) { t->mem.ctx = ctx; t->W = W; }
    for (Buf* b : {&u32a, &u32b, &u32c, &scan_scr, &tiles, &gates_d, &sup_d, &tab_d, &drun_d, &dm_d, &dval_d, &cnt_d, &ovf_d,
                   &partial_d, &f64_d, &span_d, &htab_d, &lstat_d, &hscr_d, &tr_s0, &tr_l0, &tr_s1, &tr_l1, &g1_d, &g1_ovf, &g1_base, &g1_base2, &rl0, &rl1, &rl2, &ovl1, &ovl2,
                   &tf_flag, &tf_pos, &tf_list, &g1_io, &g1_tab, &g1_tabmeta, &win_hist_d, &qlist_d, &topk_d, &topk_off, &sel_d, &cscr_d})
      b->ctx = ctx;
    cnt_d.ensure(256);
    span_d.ensure(256);
    htab_d.ensure(kHashTabWords * 4);
    HIPCHK(hipMemcpyAsync(htab_d.p, hash_tables().data(), kHashTabWords * 4, hipMemcpyHostToDevice, st));
    sync();
  }
  ~Engine() override {
    for (auto* t : {&cur, &alt, &sa, &sb, &tmp, &gb}) t->mem.release();
    for (auto* t : {&ta, &tb}) t->mem.release();
    for (Buf* b : {&u32a, &u32b, &u32c, &scan_scr, &tiles, &gates_d, &sup_d, &tab_d, &drun_d, &dm_d, &dval_d, &cnt_d, &ovf_d,
                   &partial_d, &f64_d, &span_d, &htab_d, &lstat_d, &hscr_d, &tr_s0, &tr_l0, &tr_s1, &tr_l1, &g1_d, &g1_ovf, &g1_base, &g1_base2, &rl0, &rl1, &rl2, &ovl1, &ovl2,
                   &tf_flag, &tf_pos, &tf_list, &g1_io, &g1_tab, &g1_tabmeta, &win_hist_d, &qlist_d, &topk_d, &topk_off, &sel_d, &cscr_d})
      b->release();
  }

  uint64_t size() const override { return N; }

  static dim3 grid1(uint64_t n, int b = 256) { return dim3((unsigned)std::max<uint64_t>(1, cdiv(n, b))); }
  // bounded grid for grid-stride kernels that reduce per block
  static dim3 gridb(uint64_t n) { return dim3((unsigned)std::min<uint64_t>(2048, std::max<uint64_t>(1, cdiv(n, 256)))); }

  // Grid of the elementwise kernels that stage tables in LDS: 1024-thread blocks (a block's
  // tables serve 16 wavefronts), two per compute unit, grid-stride over the terms.
  static unsigned table_grid(uint64_t n) { return (unsigned)std::min<uint64_t>(cdiv(n, 1024), 512); }

  void sync() { HIPCHK(hipStreamSynchronize(st)); }

  // ---- scans ---------------------------------------------------------------------------------
  void scan_u32(uint32_t* data, uint64_t n) {
    scan_scr.ensure(scan_scratch_words(n) * 4);
    ctx->run("scan", 0, (double)n, [&] { exclusive_scan_u32(data, n, scan_scr.as<uint32_t>(), st); });
    ctx->check_launch();
  }

  // ---- radix passes ----------------------------------------------------------------------------
  template <class CT2, bool ORD2, class DS>
  void radix_pass(TBuf<CT2, ORD2>& a, TBuf<CT2, ORD2>& b, uint64_t n, const DS& ds, int bits, const char* tag) {
    const uint32_t nblocks = (uint32_t)cdiv(n, kSortTile);
    const int bins = 1 << bits;
    u32a.ensure((size_t)bins * nblocks * 4 + 64);
    b.ensure(n);
    const Terms<CT2> in = a.view(), out = b.view();
    uint32_t* counts = u32a.as<uint32_t>();
    ctx->run("radix_hist", 0, (double)n, [&] {
      hipLaunchKernelGGL((k_radix_hist<W, CT2, DS>), dim3(nblocks), dim3(kSortBlock), 0, st, in, n, ds, bins,
                         counts, nblocks);
    });
    ctx->check_launch();
    scan_u32(counts, (uint64_t)bins * nblocks);
    const double rec = 16.0 * W + sizeof(CT2) + (ORD2 ? 1 : 0);
    ctx->run(tag, 2.0 * rec * n, (double)n, [&] {
      hipLaunchKernelGGL((k_radix_scatter<W, CT2, ORD2, DS>), dim3(nblocks), dim3(kSortBlock), 0, st, in, out, n,
                         ds, bits, (const uint32_t*)counts, nblocks);
    });
    ctx->check_launch();
    a.swap(b);
  }

  // Sort by the low k bits of the group hash (result in a).
  void hash_sort(TBuf<CT, ORD>& a, TBuf<CT, ORD>& b, uint64_t n, const GroupMask& gm, int k) {
    const int passes = (k + kMaxDigitBits - 1) / kMaxDigitBits;
    const int bits = (k + passes - 1) / passes;
    for (int p = 0; p < passes; ++p) {
      HashDigits<W> ds{gm, p * bits, bits};
      radix_pass(a, b, n, ds, bits, "radix_scatter_hash");
    }
  }

  // Canonical order: x words (word W-1 most significant), then z words, then order.  Digits
  // whose bits are the same in every term are skipped.  Result in a.
  template <class CT2, bool ORD2>
  void canonical_sort(TBuf<CT2, ORD2>& a, TBuf<CT2, ORD2>& b, uint64_t n) {
    if (n <= 1) return;
    constexpr int NP = 2 * W + 1;
    HIPCHK(hipMemsetAsync(span_d.p, 0, 8 * NP, st));
    HIPCHK(hipMemsetAsync(span_d.as<unsigned long long>() + NP, 0xff, 8 * NP, st));
    const Terms<CT2> t = a.view();
    unsigned long long* oa = span_d.as<unsigned long long>();
    const unsigned nb = (unsigned)std::min<uint64_t>(1024, cdiv(n, 256));
    ctx->run("key_span", 0, (double)n, [&] {
      hipLaunchKernelGGL((k_key_span<W, CT2, ORD2>), dim3(nb), dim3(256), 0, st, t, n, oa);
    });
    ctx->check_launch();
    uint64_t span[2 * NP];
    HIPCHK(hipMemcpyAsync(ctx->pinned, oa, 16 * NP, hipMemcpyDeviceToHost, st));
    sync();
    std::memcpy(span, ctx->pinned, 16 * NP);
    // least significant first: order, z words 0..W-1, x words 0..W-1
    std::vector<int> planes;
    if (ORD2) planes.push_back(2 * W);
    for (int w = 0; w < W; ++w) planes.push_back(W + w);
    for (int w = 0; w < W; ++w) planes.push_back(w);
    for (int p : planes) {
      const uint64_t var = span[p] ^ span[NP + p];
      if (!var) continue;
      const int lo = __builtin_ctzll(var);
      const int hi = 63 - __builtin_clzll(var);
      const int width = hi - lo + 1;
      const int passes = (width + kMaxDigitBits - 1) / kMaxDigitBits;
      const int bits = (width + passes - 1) / passes;
      for (int q = 0; q < passes; ++q) {
        const int sh = lo + q * bits;
        const int bb = std::min(bits, 64 - sh);
        WordDigits<W> ds{p, sh, bb};
        radix_pass(a, b, n, ds, bb, "radix_scatter_canon");
      }
    }
  }

  // On a canonically sorted buffer a: merge runs, drop zeros and |c| < thr; result in a.
  uint64_t merge_sorted(TBuf<CT, ORD>& a, TBuf<CT, ORD>& b, uint64_t n, double thr, double* dropped_dev) {
    if (n == 0) return 0;
    u32b.ensure(n * 4 + 64);
    u32c.ensure(n * 4 + 64);
    uint32_t* keep = u32b.as<uint32_t>();
    uint32_t* pos = u32c.as<uint32_t>();
    const Terms<CT> t = a.view();
    ctx->run("reduce_runs", 0, (double)n, [&] {
      hipLaunchKernelGGL((k_reduce_runs<W, CT, ORD>), gridb(n), dim3(256), 0, st, t, n, thr, keep, dropped_dev);
    });
    ctx->check_launch();
    HIPCHK(hipMemcpyAsync(pos, keep, n * 4, hipMemcpyDeviceToDevice, st));
    scan_u32(pos, n);
    uint32_t last_pos = 0, last_keep = 0;
    HIPCHK(hipMemcpyAsync(ctx->pinned, pos + n - 1, 4, hipMemcpyDeviceToHost, st));
    HIPCHK(hipMemcpyAsync((char*)ctx->pinned + 4, keep + n - 1, 4, hipMemcpyDeviceToHost, st));
    sync();
    std::memcpy(&last_pos, ctx->pinned, 4);
    std::memcpy(&last_keep, (char*)ctx->pinned + 4, 4);
    const uint64_t m = (uint64_t)last_pos + last_keep;
    b.ensure(std::max<uint64_t>(m, 1));
    const Terms<CT> o = b.view();
    ctx->run("compact", 0, (double)n, [&] {
      hipLaunchKernelGGL((k_compact<W, CT, ORD>), grid1(n), dim3(256), 0, st, t, o, n, (const uint32_t*)keep,
                         (const uint32_t*)pos);
    });
    ctx->check_launch();
    a.swap(b);
    return m;
  }

  // Keep-flag compaction of cur (flags in u32b) -> cur.
  uint64_t compact_cur(uint32_t* keep) {
    u32c.ensure(N * 4 + 64);
    uint32_t* pos = u32c.as<uint32_t>();
    HIPCHK(hipMemcpyAsync(pos, keep, N * 4, hipMemcpyDeviceToDevice, st));
    scan_u32(pos, N);
    uint32_t lp = 0, lk = 0;
    HIPCHK(hipMemcpyAsync(ctx->pinned, pos + N - 1, 4, hipMemcpyDeviceToHost, st));
    HIPCHK(hipMemcpyAsync((char*)ctx->pinned + 4, keep + N - 1, 4, hipMemcpyDeviceToHost, st));
    sync();
    std::memcpy(&lp, ctx->pinned, 4);
    std::memcpy(&lk, (char*)ctx->pinned + 4, 4);
    const uint64_t m = (uint64_t)lp + lk;
    alt.ensure(std::max<uint64_t>(m, 1));
    const Terms<CT> in = cur.view(), out = alt.view();
    const uint64_t n = N;
    ctx->run("compact", 0, (double)n, [&] {
      hipLaunchKernelGGL((k_compact<W, CT, ORD>), grid1(n), dim3(256), 0, st, in, out, n, (const uint32_t*)keep,
                         (const uint32_t*)pos);
    });
    ctx->check_launch();
    cur.swap(alt);
    N = m;
    return m;
  }

  // ---- gates and noise on the host --------------------------------------------------------------
  std::vector<HostGate> prepare_gates(const pp_layer* L) {
    std::vector<HostGate> out;
    for (int i = 0; i < L->n_gates; ++i) {
      const int g = L->dir == PP_HEISENBERG ? L->n_gates - 1 - i : i;
      HostGate h{};
      std::memset(&h.g, 0, sizeof h.g);
      bool any_x = false, any_z = false;
      int rr = 0;
      for (int w = 0; w < W; ++w) {
        h.g.m[w] = L->gx[(size_t)g * W + w];
        h.g.m[W + w] = L->gz[(size_t)g * W + w];
        any_x |= h.g.m[w] != 0;
        any_z |= h.g.m[W + w] != 0;
        rr += __builtin_popcountll(h.g.m[w] & h.g.m[W + w]);
      }
      double cs, sn;
      h.g.clifford = angle_cos_sin(L->theta[g], &cs, &sn) ? 1 : 0;
      h.g.cs = cs;
      h.g.sn_dir = L->dir == PP_HEISENBERG ? sn : -sn;
      h.g.rr_phase = rr & 3;
      h.g.pivot_word = -1;
      h.g.pivot_bit = 0;
      for (int w = 0; w < 2 * W; ++w)
        if (h.g.m[w]) {
          h.g.pivot_word = w;
          h.g.pivot_bit = __builtin_ctzll(h.g.m[w]);
          break;
        }
      if (h.g.pivot_word < 0) { h.g.pivot_word = 0; h.g.pivot_bit = 0; }
      h.kind = !any_z ? KIND_X : (!any_x ? KIND_Z : KIND_OTHER);
      // bit-level forms for X on one qubit and Z Z on two qubits
      int nx = 0, nz = 0;
      for (int w = 0; w < W; ++w) { nx += __builtin_popcountll(h.g.m[w]); nz += __builtin_popcountll(h.g.m[W + w]); }
      h.g.type = GATE_GENERIC;
      h.g.w0 = h.g.b0 = h.g.w1 = h.g.b1 = 0;
      if (nx == 1 && nz == 0) {
        h.g.type = GATE_X1;
        for (int w = 0; w < W; ++w)
          if (h.g.m[w]) { h.g.w0 = w; h.g.b0 = __builtin_ctzll(h.g.m[w]); }
      } else if (nx == 0 && nz == 2) {
        h.g.type = GATE_ZZ;
        int found = 0;
        for (int w = 0; w < W; ++w) {
          uint64_t v = h.g.m[W + w];
          while (v) {
            const int b = __builtin_ctzll(v);
            v &= v - 1;
            if (found == 0) { h.g.w0 = w; h.g.b0 = b; }
            else { h.g.w1 = w; h.g.b1 = b; }
            ++found;
          }
        }
      }
      h.g.hash = lin_hash<W>(h.g.m, h.g.m + W, hash_tables().data());
      h.g.khash = key_hash<W>(h.g.m, h.g.m + W);
      out.push_back(h);
    }
    return out;
  }

  struct HostNoise {
    std::vector<SupportDev> sup;
    std::vector<double> tab;
    std::vector<uint8_t> drun;
    std::vector<uint64_t> dm;
    std::vector<double> dval;
    std::vector<int32_t> qoff;    // greedy: supports listed per qubit (CSR), see NoiseDev
    std::vector<uint32_t> qent;
    int np = 1;
  };

  // The support (one or two qubits) of generator k, or {-2,-2} for a larger one and
  // {-1,-1} for the identity.
  std::pair<int, int> gen_support(const pp_layer* L, int k) const {
    std::vector<int> qs;
    for (int w = 0; w < W && qs.size() <= 2; ++w) {
      uint64_t s = L->ex[(size_t)k * W + w] | L->ez[(size_t)k * W + w];
      while (s && qs.size() <= 2) {
        qs.push_back(64 * w + __builtin_ctzll(s));
        s &= s - 1;
      }
    }
    if (qs.empty()) return {-1, -1};
    if (qs.size() > 2) return {-2, -2};
    return {qs[0], qs.size() == 2 ? qs[1] : -1};
  }

  // Fidelity factor 1 - 2q of one generator (Eq. evolve_noise): the local channel applies
  // E with p = (1 - e^{-2 lambda})/2; the inverse map negates lambda (sign = +1).
  static double fidelity_factor(double lambda, int sign) {
    const double q = (1.0 - std::exp(2.0 * sign * lambda)) / 2.0;
    return 1.0 - 2.0 * q;
  }

  // Generator tables.  Greedy mode: each string's factor is the product of its
  // anticommuting generators' fidelity factors in list order (see noise_factor); supports
  // are kept in list order with per-pattern factor slots when every generator acts on one
  // or two qubits and each support's generators are contiguous in the list, and otherwise
  // every generator is handled directly, in list order.  Error-order mode: per support and
  // pattern, the power sums of x_k = f_k - 1 = e^{2 sign lambda_k} - 1 over its anticommuting generators (the
  // supports' independent channels multiply, so power sums add over supports).
  HostNoise prepare_noise(const pp_layer* L, int mode, int max_order) {
    HostNoise hn;
    const int np = mode == PP_MODE_GREEDY ? 1 : std::max(1, max_order);
    hn.np = np;
    auto bit = [&](const uint64_t* a, int k, int q) -> int { return (int)((a[(size_t)k * W + q / 64] >> (q % 64)) & 1ULL); };
    auto anti_pat = [&](int k, int q0, int q1, int pat) -> bool {
      const int px0 = pat & 1, pz0 = (pat >> 1) & 1, px1 = (pat >> 2) & 1, pz1 = (pat >> 3) & 1;
      int par = px0 * bit(L->ez, k, q0) + pz0 * bit(L->ex, k, q0);
      if (q1 >= 0) par += px1 * bit(L->ez, k, q1) + pz1 * bit(L->ex, k, q1);
      return (par & 1) != 0;
    };
    auto add_direct = [&](int k, const std::vector<double>& vals) {
      for (int w = 0; w < W; ++w) hn.dm.push_back(L->ex[(size_t)k * W + w]);
      for (int w = 0; w < W; ++w) hn.dm.push_back(L->ez[(size_t)k * W + w]);
      for (double v : vals) hn.dval.push_back(v);
    };
    auto make_sup = [&](int q0, int q1) {
      SupportDev sd{};
      sd.w0 = (int16_t)(q0 / 64);
      sd.b0 = (int16_t)(q0 % 64);
      sd.w1 = (int16_t)(q1 < 0 ? -1 : q1 / 64);
      sd.b1 = (int16_t)(q1 < 0 ? 0 : q1 % 64);
      sd.table = (int32_t)hn.tab.size();
      return sd;
    };
    if (mode == PP_MODE_GREEDY) {
      // The layer's channel is a composition of local channels: runs of consecutive
      // generators on the same one or two qubits (identity generators left out).  A
      // string's factor is the product over runs, in list order, of the run's product of
      // f_k over the generators it anticommutes with, in list order.
      std::vector<std::pair<int, int>> order;
      std::vector<std::vector<int>> groups;
      bool tabled = true;
      for (int k = 0; k < L->n_gen && tabled; ++k) {
        const auto sup = gen_support(L, k);
        if (sup.first == -1) continue;             // the identity commutes with everything
        if (sup.first == -2) { tabled = false; break; }
        if (order.empty() || order.back() != sup) {
          order.push_back(sup);
          groups.emplace_back();
        }
        groups.back().push_back(k);
      }
      if (!tabled) {
        // generators tested one by one; drun marks where a run with a new support starts
        std::vector<uint64_t> prev;
        for (int k = 0; k < L->n_gen; ++k) {
          if (gen_support(L, k).first == -1) continue;
          std::vector<uint64_t> m(W);
          for (int w = 0; w < W; ++w) m[w] = L->ex[(size_t)k * W + w] | L->ez[(size_t)k * W + w];
          hn.drun.push_back(hn.drun.empty() || m != prev ? 1 : 0);
          prev = m;
          add_direct(k, {fidelity_factor(L->lambda[k], L->noise_sign)});
        }
        return hn;
      }
      // tab: per run and local pattern, the run's product for that pattern (1.0 for none)
      for (size_t si = 0; si < order.size(); ++si) {
        const int q0 = order[si].first, q1 = order[si].second;
        const int npat = q1 < 0 ? 4 : 16;
        SupportDev sd = make_sup(q0, q1);
        for (int pat = 0; pat < npat; ++pat) {
          double run = 1.0;
          if (pat)
            for (int k : groups[si])
              if (anti_pat(k, q0, q1, pat)) run *= fidelity_factor(L->lambda[k], L->noise_sign);
          hn.tab.push_back(run);
        }
        hn.sup.push_back(sd);
      }
      // per-qubit lists: every run under its first qubit, two-qubit runs also under their
      // second qubit (flagged; taken there only when the first qubit is the identity)
      const int nq = obs->n_qubits;
      std::vector<std::vector<uint32_t>> per(nq);
      for (size_t si = 0; si < order.size(); ++si) {
        per[order[si].first].push_back((uint32_t)si);
        if (order[si].second >= 0) per[order[si].second].push_back((uint32_t)si | 0x80000000u);
      }
      hn.qoff.assign(1, 0);
      for (int q = 0; q < nq; ++q) {
        for (uint32_t e : per[q]) hn.qent.push_back(e);
        hn.qoff.push_back((int32_t)hn.qent.size());
      }
      return hn;
    }
    std::map<std::pair<int, int>, std::vector<int>> by_sup;
    for (int k = 0; k < L->n_gen; ++k) {
      const auto sup = gen_support(L, k);
      if (sup.first == -1) continue;
      const double v = std::expm1(2.0 * L->noise_sign * L->lambda[k]);   // x_k = f_k - 1
      if (sup.first == -2) {
        std::vector<double> pw(np);
        double a = 1.0;
        for (int j = 0; j < np; ++j) pw[j] = (a *= v);
        add_direct(k, pw);
        continue;
      }
      by_sup[sup].push_back(k);
    }
    for (auto& kv : by_sup) {
      const int q0 = kv.first.first, q1 = kv.first.second;
      SupportDev sd = make_sup(q0, q1);
      const int npat = q1 < 0 ? 4 : 16;
      for (int pat = 0; pat < npat; ++pat) {
        std::vector<double> acc(np, 0.0);
        for (int k : kv.second) {
          if (!anti_pat(k, q0, q1, pat)) continue;
          const double v = std::expm1(2.0 * L->noise_sign * L->lambda[k]);   // x_k = f_k - 1
          double a = 1.0;
          for (int j = 0; j < np; ++j) acc[j] += (a *= v);
        }
        for (int j = 0; j < np; ++j) hn.tab.push_back(acc[j]);
      }
      hn.sup.push_back(sd);
    }
    return hn;
  }

  NoiseDev upload_noise(const HostNoise& hn, int sign, int mode, int max_order) {
    NoiseDev nd{};
    nd.nsup = (int)hn.sup.size();
    nd.ndirect = (int)(hn.dm.size() / (2 * W));
    nd.ntab = (int)hn.tab.size();
    nd.sign = sign;
    nd.mode = mode == PP_MODE_GREEDY ? 0 : 1;
    nd.max_order = max_order;
    sup_d.ensure(hn.sup.size() * sizeof(SupportDev) + 64);
    tab_d.ensure(hn.tab.size() * 8 + 64);
    drun_d.ensure(hn.drun.size() + 64);
    dm_d.ensure(hn.dm.size() * 8 + 64);
    dval_d.ensure(hn.dval.size() * 8 + 64);
    if (!hn.sup.empty())
      HIPCHK(hipMemcpyAsync(sup_d.p, hn.sup.data(), hn.sup.size() * sizeof(SupportDev), hipMemcpyHostToDevice, st));
    if (!hn.tab.empty()) HIPCHK(hipMemcpyAsync(tab_d.p, hn.tab.data(), hn.tab.size() * 8, hipMemcpyHostToDevice, st));
    if (!hn.drun.empty()) HIPCHK(hipMemcpyAsync(drun_d.p, hn.drun.data(), hn.drun.size(), hipMemcpyHostToDevice, st));
    if (!hn.dm.empty()) HIPCHK(hipMemcpyAsync(dm_d.p, hn.dm.data(), hn.dm.size() * 8, hipMemcpyHostToDevice, st));
    if (!hn.dval.empty())
      HIPCHK(hipMemcpyAsync(dval_d.p, hn.dval.data(), hn.dval.size() * 8, hipMemcpyHostToDevice, st));
    nd.sup = sup_d.as<SupportDev>();
    nd.tab = tab_d.as<double>();
    nd.drun = hn.drun.empty() ? nullptr : drun_d.as<uint8_t>();
    nd.dm = dm_d.as<uint64_t>();
    nd.dval = dval_d.as<double>();
    nd.nq = 0;
    nd.nqent = 0;
    nd.qoff = nullptr;
    nd.qent = nullptr;
    if (!hn.qoff.empty()) {
      nd.nq = (int)hn.qoff.size() - 1;
      nd.nqent = (int)hn.qent.size();
      qlist_d.ensure(hn.qoff.size() * 4 + hn.qent.size() * 4 + 64);
      HIPCHK(hipMemcpyAsync(qlist_d.p, hn.qoff.data(), hn.qoff.size() * 4, hipMemcpyHostToDevice, st));
      if (!hn.qent.empty())
        HIPCHK(hipMemcpyAsync((char*)qlist_d.p + hn.qoff.size() * 4, hn.qent.data(), hn.qent.size() * 4,
                              hipMemcpyHostToDevice, st));
      nd.qoff = qlist_d.as<int32_t>();
      nd.qent = (const uint32_t*)((const char*)qlist_d.p + hn.qoff.size() * 4);
    }
    // The uploads above are ordered on the stream before the kernels that read them; the
    // host vectors are synchronous copies' sources, so wait for them before returning.
    sync();
    return nd;
  }

  // Greedy-mode rescale, elementwise, support tables staged in LDS.
  void noise_greedy(const Terms<CT>& t, uint64_t n, const NoiseDev& nd, const char* name) {
    if (n == 0) return;
    const size_t lds = noise_lds_bytes(nd);
    if (lds > 160 * 1024) throw_fail(PP_ERR_UNSUPPORTED, "noise tables exceed LDS");
    if (lds > kNoiseLdsMax)
      HIPCHK(hipFuncSetAttribute((const void*)k_noise_greedy<W, CT>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                 (int)lds));
    ctx->run(name, 2.0 * kTermBytes * n, (double)n, [&] {
      hipLaunchKernelGGL((k_noise_greedy<W, CT>), dim3(table_grid(n)), dim3(1024), lds, st, t, n, nd);
    });
    ctx->check_launch();
  }

  // ---- per-gate path on a subset (sa holds m terms) ------------------------------------------
  uint64_t per_gate(uint64_t m, const std::vector<GateDev>& gates, double eps, const NoiseDev* nd,
                    double eps_noise, double* dropped_dev, uint64_t* peak_out = nullptr, int sine_max = -1) {
    uint64_t gate_peak = m;
    for (const GateDev& G : gates) {
      if (m == 0) break;
      sb.ensure(2 * m);
      const Terms<CT> in = sa.view(), out = sb.view();
      ctx->run("expand_gate", 0, (double)m, [&] {
        hipLaunchKernelGGL((k_expand_gate<W, CT, ORD>), grid1(m), dim3(256), 0, st, in, m, G, out, sine_max);
      });
      ctx->check_launch();
      sa.swap(sb);
      canonical_sort(sa, sb, 2 * m);
      m = merge_sorted(sa, sb, 2 * m, G.clifford ? 0.0 : eps, dropped_dev);
      gate_peak = std::max(gate_peak, m);
    }
    if (peak_out) *peak_out = gate_peak;
    if (nd && m) {
      if (nd->mode == 0) {
        noise_greedy(sa.view(), m, *nd, "noise");
      } else {
        const uint64_t M1 = (uint64_t)nd->max_order + 1;
        sb.ensure(m * M1);
        const Terms<CT> in = sa.view(), out = sb.view();
        const NoiseDev ndv = *nd;
        ctx->run("expand_noise", 0, (double)m, [&] {
          hipLaunchKernelGGL((k_expand_noise<W, CT, ORD>), grid1(m), dim3(256), 0, st, in, m, ndv, out);
        });
        ctx->check_launch();
        sa.swap(sb);
        canonical_sort(sa, sb, m * M1);
        m = merge_sorted(sa, sb, m * M1, eps_noise, dropped_dev);
      }
    }
    return m;
  }

  struct Counters {
    unsigned long long out_count;
    uint32_t ovf_count;
    uint32_t peak;
    double dropped;
    unsigned long long out_fail;
    unsigned long long peak_sum;
  };

  // Tile starts ts[0..ntiles] over the m terms of `src` (sorted by the class hash): tile t
  // starts at the first class boundary at or after t * T.
  void make_tiles(const TBuf<CT, ORD>& src, uint64_t m, const GroupMask& gm, uint64_t kmask, uint64_t T,
                  uint64_t ntiles, uint32_t* ts) {
    tf_flag.ensure(m * 4 + 64);
    tf_pos.ensure(m * 4 + 64);
    tf_list.ensure(m * 4 + 64);
    uint32_t *flag = tf_flag.as<uint32_t>(), *pos = tf_pos.as<uint32_t>(), *lst = tf_list.as<uint32_t>();
    const Terms<CT> t = src.view();
    ctx->run("tiles", 0, (double)m, [&] {
      hipLaunchKernelGGL((k_class_flags<W, CT>), grid1(m), dim3(256), 0, st, t, m, gm, kmask, flag);
    });
    ctx->check_launch();
    HIPCHK(hipMemcpyAsync(pos, flag, m * 4, hipMemcpyDeviceToDevice, st));
    scan_u32(pos, m);
    uint32_t lp = 0, lk = 0;
    HIPCHK(hipMemcpyAsync(ctx->pinned, pos + m - 1, 4, hipMemcpyDeviceToHost, st));
    HIPCHK(hipMemcpyAsync((char*)ctx->pinned + 4, flag + m - 1, 4, hipMemcpyDeviceToHost, st));
    hipLaunchKernelGGL(k_scatter_flagged, grid1(m), dim3(256), 0, st, (const uint32_t*)flag, (const uint32_t*)pos, m,
                       lst);
    ctx->check_launch();
    sync();
    std::memcpy(&lp, ctx->pinned, 4);
    std::memcpy(&lk, (char*)ctx->pinned + 4, 4);
    const uint32_t nb = lp + lk;
    ctx->run("tiles", 0, (double)ntiles, [&] {
      hipLaunchKernelGGL(k_tile_starts, grid1(ntiles + 1), dim3(256), 0, st, (const uint32_t*)lst, nb, m, T,
                         (uint32_t)ntiles, ts);
    });
    ctx->check_launch();
  }

  // ---- grouped fused pass ---------------------------------------------------------------------
  // One level: run the fused kernel over `m` terms of `src` with tile target T, appending the
  // survivors to `alt` at out_count; the inputs of tiles that overflowed (LDS or output
  // space) are gathered into `ovf`.  Returns their count.
  uint64_t fused_level(TBuf<CT, ORD>& src, uint64_t m, uint64_t T, const GroupMask& gm, int ngates, int kind,
                       bool any_nc, double thr, const NoiseDev* nd, double thr_noise, TBuf<CT, ORD>& dst,
                       uint64_t& out_count, TBuf<CT, ORD>& ovf, bool& out_full, pp_layer_stats& ls,
                       bool small) {
    uint64_t ntiles;
    if (m <= T) {
      ntiles = 1;
      tiles.ensure(64);
      uint32_t h[2] = {0u, (uint32_t)m};
      std::memcpy(ctx->pinned, h, 8);
      HIPCHK(hipMemcpyAsync(tiles.p, ctx->pinned, 8, hipMemcpyHostToDevice, st));
    } else {
      const int k = std::min(40, std::max(8, ceil_log2(m) - floor_log2(T) + 4));
      const int passes = (k + kMaxDigitBits - 1) / kMaxDigitBits;
      const int kk = passes * ((k + passes - 1) / passes);
      hash_sort(src, tmp, m, gm, kk);
      ntiles = cdiv(m, T);
      tiles.ensure((ntiles + 2) * 4);
      const Terms<CT> t = src.view();
      const uint64_t kmask = kk >= 64 ? ~0ULL : ((1ULL << kk) - 1);
      uint32_t* ts = tiles.as<uint32_t>();
      (void)t;
      make_tiles(src, m, gm, kmask, T, ntiles, ts);
    }
    ovf_d.ensure((ntiles + 2) * 4);
    Counters hc0{};
    hc0.out_count = out_count;
    hc0.out_fail = ~0ULL;
    std::memcpy((char*)ctx->pinned + 256, &hc0, sizeof hc0);
    HIPCHK(hipMemcpyAsync(cnt_d.p, (char*)ctx->pinned + 256, sizeof(Counters), hipMemcpyHostToDevice, st));
    Counters* cd = cnt_d.as<Counters>();
    LayerArgs<CT> a{};
    a.in = src.view();
    a.out = dst.view();
    a.tile_start = tiles.as<uint32_t>();
    a.tile_list = nullptr;
    a.gates = gates_d.as<GateDev>();
    a.ngates = ngates;
    a.eps = thr;
    a.gate_kind = kind == KIND_OTHER ? 2 : (kind == KIND_Z ? 1 : 0);
    a.any_nonclifford = any_nc ? 1 : 0;
    a.has_noise = nd ? 1 : 0;
    if (nd) a.noise = *nd;
    a.eps_noise = thr_noise;
    a.htab = htab_d.as<uint32_t>();
    a.out_count = &cd->out_count;
    a.out_fail = &cd->out_fail;
    a.ovf_tiles = ovf_d.as<uint32_t>();
    a.ovf_count = &cd->ovf_count;
    // per-slot statistics: dropped (double), peak_sum (u64), peak (u32)
    constexpr size_t kStatBytes = kStatSlots * (8 + 8 + 4);
    lstat_d.ensure(kStatBytes + 64);
    HIPCHK(hipMemsetAsync(lstat_d.p, 0, kStatBytes, st));
    a.dropped = (double*)lstat_d.p;
    a.peak_sum = (unsigned long long*)((char*)lstat_d.p + kStatSlots * 8);
    a.peak = (unsigned int*)((char*)lstat_d.p + kStatSlots * 16);
    const int pi = ctx->run(small ? "layer_fused_wave" : "layer_fused_block", 0, (double)m, [&] {
      if (small)
        hipLaunchKernelGGL((k_layer<W, CT, ORD, SmallCfg<W>::CAP, SmallCfg<W>::BLOCK, SmallCfg<W>::GATES>),
                           dim3((unsigned)ntiles), dim3(SmallCfg<W>::BLOCK), 0, st, a);
      else
        hipLaunchKernelGGL((k_layer<W, CT, ORD, LayerCfg<W>::CAP, LayerCfg<W>::BLOCK, LayerCfg<W>::GATES>),
                           dim3((unsigned)ntiles), dim3(LayerCfg<W>::BLOCK), 0, st, a);
    });
    ctx->check_launch();
    Counters hc;
    HIPCHK(hipMemcpyAsync(ctx->pinned, cd, sizeof(Counters), hipMemcpyDeviceToHost, st));
    HIPCHK(hipMemcpyAsync((char*)ctx->pinned + 1024, lstat_d.p, kStatBytes, hipMemcpyDeviceToHost, st));
    sync();
    std::memcpy(&hc, ctx->pinned, sizeof hc);
    {
      const char* ps = (const char*)ctx->pinned + 1024;
      hc.dropped = 0.0;
      hc.peak = 0;
      hc.peak_sum = 0;
      for (int k = 0; k < kStatSlots; ++k) {
        double d;
        unsigned long long q;
        uint32_t pk;
        std::memcpy(&d, ps + 8 * k, 8);
        std::memcpy(&q, ps + kStatSlots * 8 + 8 * k, 8);
        std::memcpy(&pk, ps + kStatSlots * 16 + 4 * k, 4);
        hc.dropped += d;
        hc.peak_sum += q;
        hc.peak = std::max(hc.peak, pk);
      }
    }
    last_ntiles = ntiles;
    last_ovf_tiles = hc.ovf_count;
    const uint64_t end = std::min<uint64_t>(hc.out_count, hc.out_fail);   // valid prefix
    const uint64_t written = end - out_count;
    out_count = end;
    ls.dropped_l1 += hc.dropped;
    ls.n_peak = std::max<int64_t>(ls.n_peak, (int64_t)hc.peak);
    run_bound += hc.peak_sum;
    uint64_t mo = 0;
    std::vector<uint32_t> src_r, len_r;
    std::vector<uint64_t> dst_r;
    if (hc.ovf_count > 0) {
      const uint32_t nov = hc.ovf_count;
      std::vector<uint32_t> ov(nov), ts(ntiles + 1);
      HIPCHK(hipMemcpyAsync(ov.data(), ovf_d.p, 4 * (size_t)nov, hipMemcpyDeviceToHost, st));
      HIPCHK(hipMemcpyAsync(ts.data(), tiles.p, 4 * (ntiles + 1), hipMemcpyDeviceToHost, st));
      sync();
      for (uint32_t v : ov) {
        out_full |= (v & kOvfOutput) != 0;
        const uint32_t t = v & ~kOvfOutput;
        src_r.push_back(ts[t]);
        len_r.push_back(ts[t + 1] - ts[t]);
        dst_r.push_back(mo);
        mo += ts[t + 1] - ts[t];
      }
      ovf.ensure(std::max<uint64_t>(mo, 1));
      u32b.ensure(8 * (size_t)nov + 64);
      u32c.ensure(8 * (size_t)nov + 64);
      partial_d.ensure(8 * (size_t)nov + 64);
      HIPCHK(hipMemcpyAsync(u32b.p, src_r.data(), 4 * (size_t)nov, hipMemcpyHostToDevice, st));
      HIPCHK(hipMemcpyAsync(u32c.p, len_r.data(), 4 * (size_t)nov, hipMemcpyHostToDevice, st));
      HIPCHK(hipMemcpyAsync(partial_d.p, dst_r.data(), 8 * (size_t)nov, hipMemcpyHostToDevice, st));
      const Terms<CT> in = src.view(), sub = ovf.view();
      const uint32_t *srcd = u32b.as<uint32_t>(), *lend = u32c.as<uint32_t>();
      const uint64_t* dstd = partial_d.as<uint64_t>();
      ctx->run("copy_ranges", 0, (double)mo, [&] {
        hipLaunchKernelGGL((k_copy_ranges<W, CT, ORD>), dim3(nov), dim3(256), 0, st, in, sub, srcd, lend, dstd,
                           (int)nov);
      });
      ctx->check_launch();
      sync();   // the range lists are host vectors
    }
    // A term's bytes in and out of the layer are the algorithmic traffic of the launch.
    if (pi >= 0) ctx->pending[pi].bytes = kTermBytes * (double)((m - mo) + written);
    return mo;
  }

  // Grow `b` to hold `need` terms, keeping its first `keep` terms (staged through tmp).
  void grow_keep(TBuf<CT, ORD>& b, uint64_t need, uint64_t keep) {
    if (need <= b.cap) return;
    tmp.ensure(std::max<uint64_t>(keep, 1));
    if (keep) {
      const Terms<CT> from = b.view(), to = tmp.view();
      ctx->run("copy", 0, (double)keep, [&] {
        hipLaunchKernelGGL((k_copy<W, CT, ORD>), grid1(keep), dim3(256), 0, st, from, 0, to, 0, keep);
      });
      ctx->check_launch();
    }
    b.ensure(need);
    if (keep) {
      const Terms<CT> from = tmp.view(), to = b.view();
      ctx->run("copy", 0, (double)keep, [&] {
        hipLaunchKernelGGL((k_copy<W, CT, ORD>), grid1(keep), dim3(256), 0, st, from, 0, to, 0, keep);
      });
      ctx->check_launch();
    }
  }

  void append(TBuf<CT, ORD>& dst, uint64_t& count, TBuf<CT, ORD>& src, uint64_t m) {
    if (!m) return;
    grow_keep(dst, count + m + 1, count);
    const Terms<CT> from = src.view(), to = dst.view();
    const uint64_t oc = count;
    ctx->run("copy", 0, (double)m, [&] {
      hipLaunchKernelGGL((k_copy<W, CT, ORD>), grid1(m), dim3(256), 0, st, from, 0, to, oc, m);
    });
    ctx->check_launch();
    count += m;
  }

  // Group mask of the bits a run of gates cannot change: X-type gates keep z and every x bit
  // outside the union of their x masks; Z-type likewise with x and z exchanged; a general
  // gate keeps every bit outside its x and z masks.
  GroupMask invariant_mask(const std::vector<GateDev>& gates, int kind) const {
    GroupMask gm;
    for (int w = 0; w < PP_MAXW; ++w) { gm.mx[w] = ~0ULL; gm.mz[w] = ~0ULL; }
    if (kind == KIND_X) {
      for (const GateDev& g : gates)
        for (int w = 0; w < W; ++w) gm.mx[w] &= ~g.m[w];
    } else if (kind == KIND_Z) {
      for (const GateDev& g : gates)
        for (int w = 0; w < W; ++w) gm.mz[w] &= ~g.m[W + w];
    } else if (kind == KIND_OTHER) {
      // a general rotation flips every bit of its own x and z masks
      for (const GateDev& g : gates)
        for (int w = 0; w < W; ++w) {
          gm.mx[w] &= ~g.m[w];
          gm.mz[w] &= ~g.m[W + w];
        }
    }
    return gm;
  }

  // Propagate the m terms of `src` through `gates` (one kind; noise `nd` after them) and
  // append the results to dst.  Tiles that outgrow LDS are retried with smaller tiles; the
  // terms that still do not fit go through the gates in two halves, each grouped by its own
  // (finer) invariant mask, recursively.  `src` is consumed.
  void run_groups(TBuf<CT, ORD>& src, uint64_t m, const std::vector<GateDev>& gates, int kind, double thr,
                  const NoiseDev* nd, double thr_noise, TBuf<CT, ORD>& dst, uint64_t& dst_count, int depth,
                  pp_layer_stats& ls) {
    if (m == 0 || aborted) return;
    bool any_nc = false;
    for (const GateDev& g : gates) any_nc |= g.clifford == 0;
    gates_d.ensure(std::max<size_t>(1, gates.size()) * sizeof(GateDev) + 64);
    if (!gates.empty()) {
      HIPCHK(hipMemcpyAsync(gates_d.p, gates.data(), gates.size() * sizeof(GateDev), hipMemcpyHostToDevice, st));
      sync();
    }
    const GroupMask gm = invariant_mask(gates, kind);
    TBuf<CT, ORD> ov_a, ov_b, ov_c;
    for (auto* t : {&ov_a, &ov_b, &ov_c}) { t->mem.ctx = ctx; t->W = W; }
    TBuf<CT, ORD>* in = &src;
    uint64_t mi = m;
    // level 0: one-wavefront tiles; levels 1, 2: 1024-thread tiles, the second with small
    // targets (one hash class per tile)
    for (int level = 0; level < 3 && mi > 0; ++level) {
      TBuf<CT, ORD>& ovf = level == 0 ? ov_a : (level == 1 ? ov_b : ov_c);
      const bool small = level == 0 && PP_LEVEL0_WAVE;
      uint64_t T;
      if (level == 0 && small) T = (uint64_t)std::max(4.0, std::min((double)SmallCfg<W>::CAP / 2, tile_target[kind]));
      else if (level == 0) T = CAP / 3;
      else if (level == 1) T = CAP / 3;
      else T = 256;
      bool out_full = false;
      const uint64_t mo = fused_level(*in, mi, T, gm, (int)gates.size(), kind, any_nc, thr, nd, thr_noise, dst,
                                      dst_count, ovf, out_full, ls, small);
      if (level > 0 || depth > 0) ls.n_fallback += (int64_t)mi;
      if (mo && out_full) {
        if (abort_on_full) {   // more terms than the output buffer holds: the caller gives up
          aborted = true;
          break;
        }
        grow_keep(dst, std::max<uint64_t>(dst.cap + dst.cap / 2, dst_count + mo * 4), dst_count);
      }
      if (level == 0 && depth == 0) {
        const double frac = (double)last_ovf_tiles / (double)std::max<uint64_t>(1, last_ntiles);
        if (frac > 0.10) tile_target[kind] = std::max(16.0, tile_target[kind] * 0.75);
        else if (frac < 0.02) tile_target[kind] = std::min((double)SmallCfg<W>::CAP / 2, tile_target[kind] * 1.2);
      }
      in = &ovf;
      mi = mo;
    }
    if (mi > 0 && !aborted) {
      if (gates.size() >= 2 && depth < 8) {
        // groups too large for LDS under all these gates: split the gate list in two
        const size_t h = gates.size() / 2;
        std::vector<GateDev> g1(gates.begin(), gates.begin() + h), g2(gates.begin() + h, gates.end());
        TBuf<CT, ORD> mid;
        mid.mem.ctx = ctx;
        mid.W = W;
        uint64_t mm = 0;
        mid.ensure(mi * 2 + 1);
        run_groups(*in, mi, g1, kind, thr, nullptr, thr_noise, mid, mm, depth + 1, ls);
        run_groups(mid, mm, g2, kind, thr, nd, thr_noise, dst, dst_count, depth + 1, ls);
        mid.mem.release();
      } else {
        // last resort (a single gate's pairs cannot outgrow LDS; kept for safety)
        ls.n_fallback += (int64_t)mi;
        if (in != &sa) sa.swap(*in);
        uint64_t gp = 0;
        const uint64_t mm = per_gate(mi, gates, thr, nd, thr_noise, &cnt_d.as<Counters>()->dropped, &gp);
        run_bound += gp;
        if (abort_on_full && dst_count + mm > dst.cap) {
          aborted = true;
        } else {
          append(dst, dst_count, sa, mm);
        }
      }
    }
    ov_a.mem.release();
    ov_b.mem.release();
    ov_c.mem.release();
  }

  // One run of gates of one kind.  Truncation follows every non-Clifford gate: the threshold
  // inside the kernels, the cap (when set) as a device-wide selection.  All gates of the run
  // go through one fused pass when the cap cannot bind: the pass reports an upper bound of
  // the live count after every gate, and if that bound stays within the cap, every
  // per-gate cap was a no-op.  Otherwise the run is redone one gate at a time, with the cap
  // after each non-Clifford gate.  Returns false if the noise `nd` was not applied (the
  // caller applies it after the run).
  bool grouped_pass(const std::vector<GateDev>& gates, int kind, double thr, const NoiseDev* nd,
                    double thr_noise, pp_layer_stats& ls) {
    if (N == 0) return true;
    const int64_t cap = obs->trunc.max_terms;
    bool any_nc = false;
    for (const GateDev& g : gates) any_nc |= g.clifford == 0;
    const bool capped = cap > 0 && any_nc;
    // a sum already at half the cap nearly always outgrows it at some gate
    if (!capped || (int64_t)N * 2 <= cap) {
      const uint64_t n_in = N;
      const double g = growth[kind];
      // first guess from the growth of the last run of this kind (refused tiles are retried
      // after the buffer grows, so the guess only has to be good, not safe)
      uint64_t guess = (uint64_t)((double)N * std::min(8.0, std::max(2.0, 1.25 * g))) + 4 * CAP;
      if (capped) guess = std::min<uint64_t>(guess, 2 * (uint64_t)cap + 4 * CAP);   // more than 2x the cap: it binds
      alt.ensure(guess);
      uint64_t out_count = 0;
      run_bound = 0;
      abort_on_full = capped;
      aborted = false;
      run_groups(cur, N, gates, kind, thr, nd, thr_noise, alt, out_count, 0, ls);
      abort_on_full = false;
      const bool gave_up = aborted;
      aborted = false;
      if (!gave_up && (!capped || run_bound <= (uint64_t)cap)) {
        cur.swap(alt);
        N = out_count;
        const double obs_g = (double)N / (double)std::max<uint64_t>(1, n_in);
        growth[kind] = std::min(256.0, std::max({2.0, 1.5 * obs_g, growth[kind] * 0.75}));
        return true;
      }
      ls.n_fallback += (int64_t)N;   // the fused result is discarded; cur still holds the input
    }
    gate_by_gate(gates, kind, thr, (uint64_t)cap, ls);
    return nd == nullptr;
  }

  // ---- gate by gate over persistent tiles --------------------------------------------------------
  // host-pinned scratch layout: the gate pass's counter block at 0, a bases total at
  // kPinBases, the window histogram at kPinWin
  static constexpr size_t kPinBases = 3072, kPinWin = 4096;

  struct G1Counters {
    uint32_t nlist[3];   // routed tiles: small, middle, large (kept from one gate to the next)
    uint32_t ovf[3];     // tiles reported by the small shapes, the 256-thread and the 1024-thread shape
    unsigned long long bases_total;   // the next gate's output extent (2 x the live terms)
    unsigned long long tab_cursor;    // hash-table words handed out to oversize tiles
    unsigned long long big_terms;     // terms of the oversize tiles
    uint32_t tab_err;                 // an oversize tile found no table room
    uint32_t pad;
    double drop[kDropSlots];          // sum of |c| removed, per slot
  };
  static constexpr uint32_t kG1SmallMax = 128;   // tiles up to this size start in one wavefront
  static constexpr uint32_t kG1MidMax = 256;     // up to this size in 128 threads (room for 512)
  // LDS capacity of the one-wavefront shape: less LDS per wavefront, more of them per compute
  // unit; a tile that outgrows it is redone in the 256-thread shape
  static constexpr int kG1WaveCap = 256;
  // Terms per tile when tiling.  Measured on the 56-qubit workload (cap 2^24, FP64, ms per
  // propagation): 96 -> 401, 128 -> 390, 192 -> 378, 256 -> 370, 384 -> 375, 512 -> 380,
  // 768 -> 437.  Larger tiles mean fewer per-tile phases and fewer half-used cache lines at
  // tile edges, until the tiles no longer fit the one-wavefront and 128-thread shapes.
  static constexpr uint64_t kG1Target = 256;
  uint64_t g1_ntiles = 0;
  bool routed = false;      // tile lists by size are current for this tiling
  int sine_limit = -1;      // >= 0: the gate passes run in sine order with this tag limit
  uint32_t route_n[3] = {0, 0, 0};

  // Group the terms by the run's invariant bits and cut them into tiles of whole groups
  // (cur must be dense).
  void g1_tile(const GroupMask& gm) {
    const uint64_t m = N;
    const uint64_t T = kG1Target;
    const int k = std::min(40, std::max(8, ceil_log2(std::max<uint64_t>(m, 2)) - floor_log2(T) + 4));
    const int passes = (k + kMaxDigitBits - 1) / kMaxDigitBits;
    const int kk = passes * ((k + passes - 1) / passes);
    hash_sort(cur, tmp, m, gm, kk);
    const uint64_t ntiles = std::max<uint64_t>(1, cdiv(m, T));
    tiles.ensure((ntiles + 2) * 4);
    const uint64_t kmask = kk >= 64 ? ~0ULL : ((1ULL << kk) - 1);
    uint32_t* ts = tiles.as<uint32_t>();
    make_tiles(cur, m, gm, kmask, T, ntiles, ts);
    tr_s0.ensure(ntiles * 4 + 64);
    tr_l0.ensure(ntiles * 4 + 64);
    uint32_t *s0 = tr_s0.as<uint32_t>(), *l0 = tr_l0.as<uint32_t>();
    hipLaunchKernelGGL(k_tile_ranges, grid1(ntiles), dim3(256), 0, st, (const uint32_t*)ts, (uint32_t)ntiles, s0, l0);
    ctx->check_launch();
    g1_ntiles = ntiles;
    routed = false;
  }

  // Output bases of the tiles for the next gate: exclusive prefix of 2 * len.  Returns the
  // total (the extent of the output buffer).
  // Enqueue the bases into `out` (exclusive prefix of 2 * len) and their total into *total.
  void g1_bases_launch(const uint32_t* len, uint64_t ntiles, Buf& out, unsigned long long* total) {
    out.ensure(ntiles * 4 + 64);
    uint32_t* b = out.as<uint32_t>();
    const uint64_t nb = cdiv(ntiles, kSortTile);
    ctx->run("scan", 0, (double)ntiles, [&] {
      if (nb == 1) {
        hipLaunchKernelGGL(k_bases_apply, dim3(1), dim3(kSortBlock), 0, st, len, ntiles, (const uint32_t*)nullptr, 0,
                           b, total);
      } else {
        scan_scr.ensure(scan_scratch_words(nb) * 4 + nb * 4 + 256);
        uint32_t* sums = scan_scr.as<uint32_t>();
        hipLaunchKernelGGL(k_bases_sums, dim3((unsigned)nb), dim3(kSortBlock), 0, st, len, ntiles, sums);
        const int raw = nb <= kBasesRawMax;   // few blocks: each adds up the sums before it
        if (!raw) exclusive_scan_u32(sums, nb, sums + nb + 64, st);
        hipLaunchKernelGGL(k_bases_apply, dim3((unsigned)nb), dim3(kSortBlock), 0, st, len, ntiles,
                           (const uint32_t*)sums, raw, b, total);
      }
    });
    ctx->check_launch();
  }
  uint64_t g1_bases(const uint32_t* len, uint64_t ntiles) {
    unsigned long long* tot = &g1_d.as<G1Counters>()->bases_total;
    g1_bases_launch(len, ntiles, g1_base, tot);
    HIPCHK(hipMemcpyAsync((char*)ctx->pinned + kPinBases, tot, 8, hipMemcpyDeviceToHost, st));
    sync();
    unsigned long long v = 0;
    std::memcpy(&v, (const char*)ctx->pinned + kPinBases, 8);
    return v;
  }

  static uint64_t abs_key_host(CT v) {
    if (sizeof(CT) == 8) {
      uint64_t b;
      std::memcpy(&b, &v, 8);
      return b & 0x7fffffffffffffffULL;
    }
    uint32_t b;
    std::memcpy(&b, &v, 4);
    return b & 0x7fffffffU;
  }

  // The cut of a cap at K over the first n slots of cur (zeros are empty slots): radix
  // select on the |c| bits narrows the K-th largest to a bucket of few candidates, which
  // are gathered and ranked exactly on the host by (|c| descending, canonical key
  // ascending); the K-th of that order is the boundary term.
  // Last cut of this engine: the next cut's first histogram spans a window around it.
  bool hint_valid = false;
  uint64_t hint_key = 0;
  int hint_shift = sizeof(CT) == 8 ? 43 : 14;   // 2048 bins of 2^shift keys: about 4 octaves

  // The window histogram (first pass of the cut) for the n coefficients at c, enqueued with
  // the copy of its bins to the host.
  uint64_t win_lo = 0;
  int win_sh = 0;
  void win_hist_launch(const CT* c, uint64_t n, const TileView* tv = nullptr) {
    win_sh = hint_shift;
    const uint64_t half = 1024ULL << win_sh;
    win_lo = hint_key > half ? ((hint_key - half) >> win_sh) << win_sh : 0ULL;
    win_hist_d.ensure(2049 * 4 + 64);
    uint32_t* hist = win_hist_d.as<uint32_t>();
    HIPCHK(hipMemsetAsync(hist, 0, 2049 * 4, st));
    const unsigned nbh = (unsigned)std::min<uint64_t>(2048, cdiv(n, 256));
    const uint64_t lo = win_lo;
    const int sh = win_sh;
    ctx->run("cap_hist", sizeof(CT) * (double)n, (double)n, [&] {
      if (tv)
        hipLaunchKernelGGL((k_abs_hist_win_tiles<CT>), dim3(tile_grid(*tv)), dim3(256), 0, st, c, *tv, lo, sh, hist);
      else
        hipLaunchKernelGGL((k_abs_hist_win<CT>), dim3(nbh), dim3(256), 0, st, c, n, lo, sh, hist);
    });
    ctx->check_launch();
    HIPCHK(hipMemcpyAsync((char*)ctx->pinned + kPinWin, hist, 2049 * 4, hipMemcpyDeviceToHost, st));
  }

  // Grid of the tile sweeps: four tiles per wavefront, four wavefronts per workgroup.
  static unsigned tile_grid(const TileView& tv) {   // sixteen tiles per wavefront at first
    return (unsigned)std::max<uint64_t>(1, std::min<uint64_t>(4096, cdiv(tv.ntiles, 64)));
  }

  // tv: the buffer is tiled (only the tiles' live ranges hold terms), else n dense slots.
  CutDev cap_cut(uint64_t K, uint64_t n, const TileView* tv = nullptr) {
    constexpr uint32_t kGather = 4096;
    const int KB = sizeof(CT) == 8 ? 63 : 31;
    uint64_t prefix = 0, pmask = 0, need = K, count_eq = 0;
    u32a.ensure(2049 * 4 + 64);
    uint32_t* hist = u32a.as<uint32_t>();
    const CT* c = cur.view().c;
    int hi = KB;
    std::vector<uint32_t> h(2049);
    const unsigned nbh = (unsigned)std::min<uint64_t>(2048, cdiv(n, 256));
    bool done = false;
    if (hint_valid) {
      // The window's bins are the key prefixes above bit `shift`, so a hit continues the
      // radix passes below it; a miss falls back to the passes from the top.
      win_hist_launch(c, n, tv);
      sync();
      const int sh = win_sh;
      const uint64_t lo = win_lo;
      std::memcpy(h.data(), (const char*)ctx->pinned + kPinWin, 2049 * 4);
      uint64_t cum = h[2048];
      int d = -1;
      if (cum < need) {
        for (d = 2047; d >= 0; --d) {
          if (cum + h[d] >= need) break;
          cum += h[d];
        }
      }
      if (d >= 0) {
        need -= cum;
        prefix = lo + ((uint64_t)d << sh);
        pmask = ~0ULL << sh;
        count_eq = h[d];
        hi = sh;
        done = count_eq <= kGather;
        if (!done && hint_shift > 4) --hint_shift;   // finer bins next time
      } else {
        hint_shift = std::min(hint_shift + 2, KB - 11);   // wider window next time
      }
    }
    while (hi > 0 && !done) {
      const int bits = std::min(11, hi);
      const int shift = hi - bits;
      const int bins = 1 << bits;
      HIPCHK(hipMemsetAsync(hist, 0, bins * 4, st));
      ctx->run("cap_hist", sizeof(CT) * (double)n, (double)n, [&] {
        if (tv)
          hipLaunchKernelGGL((k_abs_hist_tiles<CT>), dim3(tile_grid(*tv)), dim3(256), 0, st, c, *tv, shift, bits, pmask,
                             prefix, hist);
        else
          hipLaunchKernelGGL((k_abs_hist<CT>), dim3(nbh), dim3(256), 0, st, c, n, shift, bits, pmask, prefix, hist);
      });
      ctx->check_launch();
      HIPCHK(hipMemcpyAsync(ctx->pinned, hist, bins * 4, hipMemcpyDeviceToHost, st));
      sync();
      std::memcpy(h.data(), ctx->pinned, bins * 4);
      uint64_t cum = 0;
      int d = bins - 1;
      for (; d >= 0; --d) {
        if (cum + h[d] >= need) break;
        cum += h[d];
      }
      if (d < 0) d = 0;
      need -= cum;
      prefix |= (uint64_t)d << shift;
      pmask |= (uint64_t)(bins - 1) << shift;
      count_eq = h[d];
      hi = shift;
      if (count_eq <= kGather) break;
    }
    // gather the bucket and rank it
    gb.ensure(std::max<uint64_t>(count_eq, 1));
    u32a.ensure(2048 * 4 + 64);
    uint32_t* cntd = u32a.as<uint32_t>();
    HIPCHK(hipMemsetAsync(cntd, 0, 4, st));
    const Terms<CT> t = cur.view(), g = gb.view();
    const uint64_t gcap = gb.cap;
    ctx->run("cap_gather", 0, (double)n, [&] {
      if (tv)
        hipLaunchKernelGGL((k_gather_bucket_tiles<W, CT, ORD>), dim3(tile_grid(*tv)), dim3(256), 0, st, t, *tv, pmask,
                           prefix, g, gcap, cntd);
      else
        hipLaunchKernelGGL((k_gather_bucket<W, CT, ORD>), grid1(n), dim3(256), 0, st, t, n, pmask, prefix, g, gcap,
                           cntd);
    });
    ctx->check_launch();
    const CutDev cut = rank_bucket(g, count_eq, need);   // its copies wait for the gather
    hint_valid = true;
    hint_key = cut.val;
    return cut;
  }

  // Drop the terms a cut removes (and exact zeros) from cur (N slots).
  // tv: cur is tiled over its first N slots (only the tiles' live ranges hold terms).
  // cutp: the cut is the one pending on the device there (tiled buffers only).
  void apply_cut(const CutDev& cut, pp_layer_stats& ls, const TileView* tv = nullptr, const CutDev* cutp = nullptr) {
    if (cutp && !tv) throw_fail(PP_ERR_DEVICE, "a device-side cut applies to tiles only");
    if (N == 0) return;
    u32b.ensure(N * 4 + 64);
    uint32_t* keep = u32b.as<uint32_t>();
    double* dd = &cnt_d.as<Counters>()->dropped;
    HIPCHK(hipMemsetAsync(dd, 0, 8, st));
    const Terms<CT> t = cur.view();
    const uint64_t n = N;
    if (tv) HIPCHK(hipMemsetAsync(keep, 0, n * 4, st));
    ctx->run("cut_flags", 0, (double)n, [&] {
      if (tv)
        hipLaunchKernelGGL((k_cut_keep_tiles<W, CT, ORD>), dim3(tile_grid(*tv)), dim3(256), 0, st, t, *tv, cut, cutp,
                           keep, dd);
      else
        hipLaunchKernelGGL((k_cut_keep<W, CT, ORD>), gridb(n), dim3(256), 0, st, t, n, cut, keep, dd);
    });
    ctx->check_launch();
    compact_cur(keep);
    double dropped = 0.0;
    HIPCHK(hipMemcpyAsync(ctx->pinned, dd, 8, hipMemcpyDeviceToHost, st));
    sync();
    std::memcpy(&dropped, ctx->pinned, 8);
    ls.dropped_l1 += dropped;
  }

  // The pending cut on the m terms of sa (result in sa); returns the survivors' count.
  uint64_t cut_subset(uint64_t m, const CutDev& cut) {
    if (m == 0) return 0;
    u32b.ensure(m * 4 + 64);
    u32c.ensure(m * 4 + 64);
    uint32_t* keep = u32b.as<uint32_t>();
    uint32_t* pos = u32c.as<uint32_t>();
    const Terms<CT> ts = sa.view();
    ctx->run("cut_flags", 0, (double)m, [&] {
      hipLaunchKernelGGL((k_cut_keep<W, CT, ORD>), gridb(m), dim3(256), 0, st, ts, m, cut, keep, (double*)nullptr);
    });
    ctx->check_launch();
    HIPCHK(hipMemcpyAsync(pos, keep, m * 4, hipMemcpyDeviceToDevice, st));
    scan_u32(pos, m);
    uint32_t lp = 0, lk = 0;
    HIPCHK(hipMemcpyAsync(ctx->pinned, pos + m - 1, 4, hipMemcpyDeviceToHost, st));
    HIPCHK(hipMemcpyAsync((char*)ctx->pinned + 4, keep + m - 1, 4, hipMemcpyDeviceToHost, st));
    sync();
    std::memcpy(&lp, ctx->pinned, 4);
    std::memcpy(&lk, (char*)ctx->pinned + 4, 4);
    const uint64_t k = (uint64_t)lp + lk;
    sb.ensure(std::max<uint64_t>(k, 1));
    const Terms<CT> in = sa.view(), out = sb.view();
    ctx->run("compact", 0, (double)m, [&] {
      hipLaunchKernelGGL((k_compact<W, CT, ORD>), grid1(m), dim3(256), 0, st, in, out, m, (const uint32_t*)keep,
                         (const uint32_t*)pos);
    });
    ctx->check_launch();
    sa.swap(sb);
    return k;
  }

  // One launch of the gate pass; its algorithmic bytes (terms loaded and written by the
  // tiles it completed, times the term size) are read back when timing is on.
  // The workgroups of k_gate1<CAPK, BLOCKK> that the device holds at once: its persistent grid.
  template <int CAPK, int BLOCKK>
  unsigned g1_resident() {
    static const unsigned resident = [] {
      int dev = 0, cus = 0, per_cu = 0;
      HIPCHK(hipGetDevice(&dev));
      HIPCHK(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
      HIPCHK(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, (const void*)k_gate1<W, CT, ORD, CAPK, BLOCKK>,
                                                          BLOCKK, 0));
      // A persistent grid must be resident at once: a workgroup that only starts when
      // another ends does its share of tiles after the others.  The occupancy query has
      // allowed one workgroup per compute unit more than the 160 KiB of LDS of a gfx950
      // compute unit holds (it leaves out that LDS is allocated in 512-byte blocks), so
      // that bound is taken as well.
      hipFuncAttributes fa{};
      HIPCHK(hipFuncGetAttributes(&fa, (const void*)k_gate1<W, CT, ORD, CAPK, BLOCKK>));
      constexpr int kLdsPerCu = 160 * 1024, kLdsBlock = 512;
      const int lds_wg = (int)((fa.sharedSizeBytes + kLdsBlock - 1) / kLdsBlock) * kLdsBlock;
      if (lds_wg > 0) per_cu = std::min<int>(per_cu, kLdsPerCu / lds_wg);
      return (unsigned)std::max(1, cus * std::max(1, per_cu));
    }();
    return resident;
  }

  // `ntiles` list entries, or, with dev_count, the count the device holds there (at most ntiles).
  // max_blocks: a smaller persistent grid for a list expected to be short (the kernel loops
  // over the list whatever its length).
  template <int CAPK, int BLOCKK>
  void g1_launch(Gate1Args<CT> a, unsigned ntiles, int shape, const uint32_t* dev_count = nullptr,
                 unsigned max_blocks = 0xffffffffu) {
    static const char* names[4] = {"gate_tile_wave", "gate_tile_256", "gate_tile_1024", "gate_tile_128"};
    g1_io.ensure(2 * kDropSlots * 8 + 64);
    unsigned long long* io = g1_io.as<unsigned long long>();
    a.io = io;
    a.t_count = ntiles;
    a.t_count_dev = dev_count;
    const unsigned nblocks = std::max(1u, std::min({ntiles, g1_resident<CAPK, BLOCKK>(), max_blocks}));
    if (ctx->timing) HIPCHK(hipMemsetAsync(io, 0, 2 * kDropSlots * 8, st));
    const int pi = ctx->run(names[shape], 0, (double)ntiles, [&] {
      hipLaunchKernelGGL((k_gate1<W, CT, ORD, CAPK, BLOCKK>), dim3(nblocks), dim3(BLOCKK), 0, st, a);
    });
    ctx->check_launch();
    if (pi >= 0) {
      std::vector<unsigned long long> h(2 * kDropSlots);
      HIPCHK(hipMemcpyAsync(h.data(), io, h.size() * 8, hipMemcpyDeviceToHost, st));
      sync();
      double terms = 0.0;
      for (unsigned long long v : h) terms += (double)v;
      ctx->pending[pi].bytes = kTermBytes * terms;
    }
  }

  // The need-th term (1-based) of m gathered candidates in the cap order.
  CutDev rank_bucket(const Terms<CT>& g, uint64_t m, uint64_t need) {
    std::vector<uint64_t> gx(m * W), gz(m * W);
    std::vector<CT> gc(m);
    std::vector<uint8_t> go(m, 0);
    for (int w = 0; w < W; ++w) {
      HIPCHK(hipMemcpyAsync(gx.data() + (size_t)w * m, g.x + (size_t)w * g.stride, m * 8, hipMemcpyDeviceToHost, st));
      HIPCHK(hipMemcpyAsync(gz.data() + (size_t)w * m, g.z + (size_t)w * g.stride, m * 8, hipMemcpyDeviceToHost, st));
    }
    HIPCHK(hipMemcpyAsync(gc.data(), g.c, m * sizeof(CT), hipMemcpyDeviceToHost, st));
    if (ORD) HIPCHK(hipMemcpyAsync(go.data(), g.o, m, hipMemcpyDeviceToHost, st));
    sync();
    std::vector<uint32_t> idx(m);
    for (uint32_t i = 0; i < m; ++i) idx[i] = i;
    auto before = [&](uint32_t a, uint32_t b) {   // a precedes b in the cap order
      const uint64_t ka = abs_key_host(gc[a]), kb = abs_key_host(gc[b]);
      if (ka != kb) return ka > kb;
      for (int w = W - 1; w >= 0; --w)
        if (gx[(size_t)w * m + a] != gx[(size_t)w * m + b]) return gx[(size_t)w * m + a] < gx[(size_t)w * m + b];
      for (int w = W - 1; w >= 0; --w)
        if (gz[(size_t)w * m + a] != gz[(size_t)w * m + b]) return gz[(size_t)w * m + a] < gz[(size_t)w * m + b];
      return go[a] < go[b];
    };
    if (need < 1 || need > m) throw_fail(PP_ERR_DEVICE, "cap selection lost its boundary");
    std::nth_element(idx.begin(), idx.begin() + (need - 1), idx.end(), before);
    const uint32_t bi = idx[need - 1];
    CutDev cut{};
    cut.has = 1;
    cut.val = abs_key_host(gc[bi]);
    for (int w = 0; w < W; ++w) {
      cut.x[w] = gx[(size_t)w * m + bi];
      cut.z[w] = gz[(size_t)w * m + bi];
    }
    cut.o = go[bi];
    return cut;
  }

  // The device-side state of the cap's cut between gates (one per engine), set up on first
  // use: no cut pending, no window yet.
  SelState* sel_state() {
    if (!sel_d.p) {
      sel_d.ensure(sizeof(SelState) + 64);
      HIPCHK(hipMemsetAsync(sel_d.p, 0, sizeof(SelState), st));
      hipLaunchKernelGGL(k_sel_init, dim3(1), dim3(64), 0, st, sel_d.as<SelState>(), sizeof(CT) == 8 ? 43 : 14);
      ctx->check_launch();
    }
    return sel_d.as<SelState>();
  }
  // Enqueue the cut after a gate: select the K-th term of the tiles' live slots on the device
  // (nothing when the live count, read there too, is within the cap) and leave it pending.
  // A fixed chain of launches; those with nothing to do return at once.
  void sel_launch(const TileView& tv, const unsigned long long* live2, uint64_t K) {
    SelState* ss = sel_state();
    gb.ensure(sel_gather<W>() + 64);
    const Terms<CT> t = cur.view(), g = gb.view();
    const dim3 grid(tile_grid(tv));
    ctx->run("cap_hist", 0, 0.0, [&] {
      hipLaunchKernelGGL((k_sel_win<W, CT, ORD>), grid, dim3(256), 0, st, t.c, tv, live2, (unsigned long long)K, ss);
    });
    ctx->check_launch();
    ctx->run("cap_pick", 0, 0.0, [&] {
      hipLaunchKernelGGL((k_sel_pick<W, CT, ORD>), dim3(1), dim3(256), 0, st, ss, 0);
    });
    ctx->check_launch();
    // the passes after the window are rarely needed: a smaller grid returns sooner when not
    const dim3 pgrid(std::min(256u, tile_grid(tv)));
    // the pick after the second pass runs at the start of k_sel_rest
    for (int p = 0; p < 2; ++p) {
      ctx->run("cap_pass", 0, 0.0, [&] {
        hipLaunchKernelGGL((k_sel_pass<W, CT, ORD>), pgrid, dim3(256), 0, st, t.c, tv, ss);
      });
      ctx->check_launch();
      if (p == 1) break;
      ctx->run("cap_pick", 0, 0.0, [&] {
        hipLaunchKernelGGL((k_sel_pick<W, CT, ORD>), dim3(1), dim3(256), 0, st, ss, 1);
      });
      ctx->check_launch();
    }
    ctx->run("cap_rest", 0, 0.0, [&] {
      hipLaunchKernelGGL((k_sel_rest<W, CT, ORD>), dim3(1), dim3(256), 0, st, t, tv, ss);
    });
    ctx->check_launch();
    ctx->run("cap_gather", 0, 0.0, [&] {
      hipLaunchKernelGGL((k_sel_gather<W, CT, ORD>), grid, dim3(256), 0, st, t, tv, ss, g);
    });
    ctx->check_launch();
    ctx->run("cap_rank", 0, 0.0, [&] {
      hipLaunchKernelGGL((k_sel_rank<W, CT, ORD>), dim3(1), dim3(256), 0, st, ss, g);
    });
    ctx->check_launch();
  }

  // Apply `gates` one at a time with the cap after each non-Clifford gate (Section I.A's
  // truncation of intermediate results, taken after every such gate).  The terms are tiled
  // once by the run's invariant bits; each gate is one pass over the tiles.  Between gates
  // the buffer holds each tile in its own region (2x its input) and only the tiles' live
  // ranges are read; the cut of the last gate is selected on the device and applied when
  // the next pass loads the tile.
  //
  // Nothing in the loop waits for the device: a gate's pass reads its tile lists and the
  // pending cut on the device, oversize tiles take their hash tables from a device-side
  // cursor, and the buffers are sized for the largest extent a pass can produce (a pass
  // writes 2 slots per input term, and at most 2 terms per survivor of the previous cut, so
  // 4 max(K, N) slots).  The host reads each gate's counters one gate later, while the next
  // pass runs, to keep statistics and to decide when to sort the tiles again or regroup.
  void gate_by_gate(const std::vector<GateDev>& gates, int kind, double eps, uint64_t cap, pp_layer_stats& ls) {
    const GroupMask gm = invariant_mask(gates, kind);
    // each gate's pass over the tiles carries 1 / G of the layer's read-once, write-once bytes
    struct ShareGuard {
      pp_ctx* c;
      ~ShareGuard() { c->pass_share = 1.0; }
    } share_guard{ctx};
    ctx->pass_share = 1.0 / (double)std::max<size_t>(1, gates.size());
    SelState* ss = sel_state();
    const CutDev* cutp = &ss->cut;
    hipLaunchKernelGGL(k_sel_clear, dim3(1), dim3(64), 0, st, ss);
    ctx->check_launch();
    bool cut_pending = false;    // a cut may be pending on the device
    bool need_tiles = true;
    uint64_t extent = N;         // slots of cur that hold terms (exact when `exact`)
    uint64_t out_extent = 0;     // slots the next pass writes (known on the host after tiling)
    const uint64_t bound = 4 * std::max<uint64_t>(cap, N) + 64;
    g1_d.ensure(2 * sizeof(G1Counters) + 64);
    G1Counters* cd = g1_d.as<G1Counters>();
    double* dropd = &cd->drop[0];
    bool tiled = false;          // cur holds tiles (live ranges tr_s0/tr_l0 of g1_ntiles tiles)
    // counters of the gates enqueued but not yet read (at most two: the previous and this one)
    constexpr size_t kPinRing = 16384;
    struct Lag {
      size_t gi;
      hipEvent_t ev;
      int slot;
    };
    std::vector<Lag> lag;
    uint64_t last_live = 0;      // live terms after the last gate read, before its cut
    uint64_t ext_next = 0;       // slots the pass after the last gate read writes
    uint64_t ext_last = 0;       // slots the last gate read wrote
    bool last_capped = false;
    // sizes of the retry lists of the last gate read, which size the next retries' grids
    // (0xffffffff: unknown, a full grid)
    uint32_t seen_ovf[3] = {0xffffffffu, 0xffffffffu, 0xffffffffu};
    auto absorb = [&](const Lag& l) {   // read one gate's counters (waits for that gate only)
      HIPCHK(hipEventSynchronize(l.ev));
      G1Counters h;
      std::memcpy(&h, (const char*)ctx->pinned + kPinRing + (size_t)l.slot * 1024, sizeof h);
      ctx->evfree.push_back(l.ev);
      if (h.tab_err) throw_fail(PP_ERR_DEVICE, "no room for an oversize tile's hash table");
      for (int k = 0; k < kDropSlots; ++k) ls.dropped_l1 += h.drop[k];
      ls.n_fallback += (int64_t)h.big_terms;
      for (int k = 0; k < 3; ++k) seen_ovf[k] = h.ovf[k];
      last_live = h.bases_total / 2;
      ext_last = ext_next;
      ext_next = h.bases_total;
      ls.n_peak = std::max<int64_t>(ls.n_peak, (int64_t)last_live);
      if (h.ovf[0] * 64 > h.nlist[0] + h.nlist[1]) routed = false;   // tiles outgrew their shape: sort again
      last_capped = !gates[l.gi].clifford && cap > 0 && last_live > cap;
      const uint64_t n_after = last_capped ? cap : last_live;
      if (n_after < g1_ntiles * kG1Target / 4) need_tiles = true;   // the tiles have become small
    };
    auto drain = [&]() {
      for (const Lag& l : lag) absorb(l);
      lag.clear();
    };
    auto densify = [&]() {   // apply a pending cut and squeeze out the unused slots
      N = extent;
      const TileView tv{tr_s0.as<uint32_t>(), tr_l0.as<uint32_t>(), (uint32_t)g1_ntiles};
      apply_cut(CutDev{}, ls, tiled ? &tv : nullptr, cut_pending ? cutp : nullptr);
      hipLaunchKernelGGL(k_sel_clear, dim3(1), dim3(64), 0, st, ss);
      ctx->check_launch();
      cut_pending = false;
      extent = N;
      tiled = false;
    };
    size_t gi = 0;
    for (; gi < gates.size() && N > 0; ++gi) {
      const GateDev& G = gates[gi];
      if (need_tiles) {
        drain();
        if (tiled) {
          // extent and live count of the last pass, exactly
          extent = ext_last;
          N = last_capped ? cap : last_live;
        }
        if (extent != N || cut_pending) densify();
        if (N == 0) break;
        g1_tile(gm);
        out_extent = g1_bases(tr_l0.as<uint32_t>(), g1_ntiles);
        ext_next = out_extent;
        for (auto& v : seen_ovf) v = 0xffffffffu;
        need_tiles = false;
      }
      const uint64_t ntiles = g1_ntiles;
      alt.ensure(std::max(bound, out_extent + 64));
      tr_s1.ensure(ntiles * 4 + 64);
      tr_l1.ensure(ntiles * 4 + 64);
      for (Buf* b : {&rl0, &rl1, &rl2, &g1_ovf, &ovl1, &ovl2}) b->ensure(ntiles * 4 + 64);
      // counters of this gate (the routed list sizes stay), cleared by one small kernel (a
      // memset of this unaligned range is split into three fills)
      static_assert((sizeof(G1Counters) - offsetof(G1Counters, ovf)) % 4 == 0, "counter words");
      hipLaunchKernelGGL(k_fill_u32, dim3(1), dim3(256), 0, st, (uint32_t*)&cd->ovf[0],
                         (uint64_t)((sizeof(G1Counters) - offsetof(G1Counters, ovf)) / 4), 0u);
      ctx->check_launch();
      if (!routed) {
        // sort the tiles by size (a tile changes size slowly; one that outgrows its shape is
        // retried in the next); the passes read the list sizes on the device
        HIPCHK(hipMemsetAsync(&cd->nlist[0], 0, sizeof cd->nlist, st));
        hipLaunchKernelGGL(k_route_tiles, grid1(ntiles), dim3(256), 0, st, (const uint32_t*)tr_l0.as<uint32_t>(),
                           (uint32_t)ntiles, kG1SmallMax, kG1MidMax, (const uint32_t*)g1_base.as<uint32_t>(),
                           tr_s1.as<uint32_t>(), tr_l1.as<uint32_t>(), rl0.as<uint32_t>(), rl1.as<uint32_t>(),
                           rl2.as<uint32_t>(), &cd->nlist[0]);
        ctx->check_launch();
        routed = true;
      }
      Gate1Args<CT> a{};
      a.in = cur.view();
      a.out = alt.view();
      a.t_start = tr_s0.as<uint32_t>();
      a.t_len = tr_l0.as<uint32_t>();
      a.o_base = g1_base.as<uint32_t>();
      a.o_start = tr_s1.as<uint32_t>();
      a.o_len = tr_l1.as<uint32_t>();
      a.zero_on_ovf = 0;
      a.g = G;
      a.eps = G.clifford ? 0.0 : eps;
      a.cutp = cutp;
      a.dropped = dropd;
      if (sine_limit >= 0) {
        a.sine_on = 1;
        a.sine_max = sine_limit;
      }
      auto with_list = [&](const Buf& list, Buf& ovl, int k, int zero) {
        Gate1Args<CT> b = a;
        b.t_list = list.as<uint32_t>();
        b.ovf_tiles = ovl.as<uint32_t>();
        b.ovf_count = &cd->ovf[k];
        b.zero_on_ovf = zero;
        return b;
      };
      // One wavefront for small tiles, 128 and 256 threads for the others.  Tiles that
      // outgrow a shape are retried in the next; every launch reads its list size on the
      // device, so the whole cascade is enqueued without waiting.
      const unsigned nt = (unsigned)ntiles;
      // the retries' grids follow the retry lists of the gate read last (a list is rarely
      // much longer than at the gate before; a longer one is still covered, more slowly)
      auto retry_grid = [&](uint32_t seen) {
        return seen == 0xffffffffu ? 0xffffffffu : std::max<uint32_t>(16, 2 * seen);
      };
      g1_launch<kG1WaveCap, 64>(with_list(rl0, g1_ovf, 0, 0), nt, 0, &cd->nlist[0]);
      g1_launch<512, 128>(with_list(rl1, g1_ovf, 0, 0), nt, 3, &cd->nlist[1]);
      g1_launch<1024, 256>(with_list(rl2, ovl1, 1, 0), nt, 1, &cd->nlist[2]);
      g1_launch<1024, 256>(with_list(g1_ovf, ovl1, 1, 0), nt, 1, &cd->ovf[0], retry_grid(seen_ovf[0]));
      g1_launch<LayerCfg<W>::CAP, LayerCfg<W>::BLOCK>(with_list(ovl1, ovl2, 2, 1), nt, 2, &cd->ovf[1],
                                                       retry_grid(seen_ovf[1]));
      {
        // classes too large for LDS that the gate touches: a persistent grid of 1024-thread
        // workgroups, one tile at a time in its own output region, with a hash table in
        // global memory carved from g1_tab (at most 4 words per input term of the pass)
        const uint64_t tab_words = 2 * std::max<uint64_t>(bound, out_extent) + 4096;
        g1_tab.ensure(tab_words * 4 + 64);
        hscr_d.ensure(alt.cap * 4 + 64);   // hash scratch, one slot per output slot
        Gate1Args<CT> b = with_list(ovl2, ovl2, 2, 0);
        b.t_count = nt;
        b.t_count_dev = &cd->ovf[2];
        b.hscr = hscr_d.as<uint32_t>();
        if (b.sine_on) {
          cscr_d.ensure(alt.cap * 8 + 64);   // coefficient scratch, one slot per output slot
          b.cscr = cscr_d.as<double>();
        }
        g1_io.ensure(2 * kDropSlots * 8 + 64);
        b.io = g1_io.as<unsigned long long>();
        uint32_t* tabd = g1_tab.as<uint32_t>();
        const unsigned nbig = (unsigned)std::min<uint64_t>({ntiles, 256, retry_grid(seen_ovf[2])});
        ctx->run("gate_tile_global", 0, 0.0, [&] {
          hipLaunchKernelGGL((k_gate1_big<W, CT, ORD>), dim3(nbig), dim3(1024), 0, st, b, tabd, (const uint64_t*)nullptr,
                             (const uint32_t*)nullptr, &cd->tab_cursor, (unsigned long long)tab_words, &cd->tab_err,
                             &cd->big_terms);
        });
        ctx->check_launch();
      }
      // the next gate's output bases (other buffer: this pass read the current ones) and their
      // total, twice the live count
      g1_bases_launch(tr_l1.as<uint32_t>(), ntiles, g1_base2, &cd->bases_total);
      cur.swap(alt);
      std::swap(tr_s0, tr_s1);
      std::swap(tr_l0, tr_l1);
      std::swap(g1_base, g1_base2);
      tiled = true;
      // the cap after a non-Clifford gate: selected on the device from the live ranges
      if (!G.clifford && cap > 0) {
        const TileView tv{tr_s0.as<uint32_t>(), tr_l0.as<uint32_t>(), (uint32_t)ntiles};
        sel_launch(tv, &cd->bases_total, cap);
        cut_pending = true;
      } else {
        hipLaunchKernelGGL(k_sel_clear, dim3(1), dim3(64), 0, st, ss);
        ctx->check_launch();
        cut_pending = false;
      }
      // this gate's counters, read one gate later
      const int slot = (int)(gi & 1);
      HIPCHK(hipMemcpyAsync((char*)ctx->pinned + kPinRing + (size_t)slot * 1024, cd, sizeof(G1Counters),
                            hipMemcpyDeviceToHost, st));
      hipEvent_t ev = ctx->ev();
      HIPCHK(hipEventRecord(ev, st));
      // the output extent of the next pass is this pass's bases total: known on the host
      // only once read; until then the buffers are sized by the bound
      out_extent = 0;
      lag.push_back(Lag{gi, ev, slot});
      if (lag.size() > 1) {
        absorb(lag.front());
        lag.erase(lag.begin());
      }
    }
    drain();
    if (tiled) {
      extent = ext_last;
      N = last_capped ? cap : last_live;
    }
    if (cut_pending || extent != N) densify();
    check_selection(ls);
  }

  // Statistics of the device-side cuts since the last call, and their error flag.
  void check_selection(pp_layer_stats& ls) {
    if (!sel_d.p) return;
    SelState* ss = sel_d.as<SelState>();
    constexpr size_t kPinSel = 24576;
    HIPCHK(hipMemcpyAsync((char*)ctx->pinned + kPinSel, ss, offsetof(SelState, cut), hipMemcpyDeviceToHost, st));
    sync();
    SelState h;
    std::memcpy(&h, (const char*)ctx->pinned + kPinSel, offsetof(SelState, cut));
    if (h.n_errors) throw_fail(PP_ERR_DEVICE, "cap selection lost its boundary");
    ls.n_capped += (int64_t)h.n_capped;
    hipLaunchKernelGGL(k_sel_reset_stats, dim3(1), dim3(64), 0, st, ss);
    ctx->check_launch();
  }

  // ---- create ----------------------------------------------------------------------------------
  void create(int64_t n, const uint64_t* x, const uint64_t* z, const double* c) override {
    N = 0;
    if (n == 0) return;
    const uint64_t un = (uint64_t)n;
    sa.ensure(un);
    // all planes staged at once (x planes, then z planes), one wait after the copies
    std::vector<uint64_t> planes(2 * (size_t)W * un);
    const Terms<CT> t = sa.view();
    for (int w = 0; w < W; ++w)
      for (uint64_t i = 0; i < un; ++i) {
        planes[(size_t)w * un + i] = x[i * W + w];
        planes[(size_t)(W + w) * un + i] = z[i * W + w];
      }
    for (int w = 0; w < W; ++w) {
      HIPCHK(hipMemcpyAsync(t.x + (size_t)w * t.stride, planes.data() + (size_t)w * un, un * 8,
                            hipMemcpyHostToDevice, st));
      HIPCHK(hipMemcpyAsync(t.z + (size_t)w * t.stride, planes.data() + (size_t)(W + w) * un, un * 8,
                            hipMemcpyHostToDevice, st));
    }
    f64_d.ensure(un * 8 + 64);
    HIPCHK(hipMemcpyAsync(f64_d.p, c, un * 8, hipMemcpyHostToDevice, st));
    const double* src = f64_d.as<double>();
    CT* dstc = t.c;
    ctx->run("convert", 0, (double)un, [&] {
      hipLaunchKernelGGL((k_from_f64<CT>), grid1(un), dim3(256), 0, st, src, dstc, un);
    });
    ctx->check_launch();
    if (ORD) HIPCHK(hipMemsetAsync(t.o, 0, un, st));
    sync();   // the staged planes go out of scope
    if (un == 1) {   // one term: already in canonical order; only an exact zero is dropped
      cur.swap(sa);
      N = c[0] != 0.0 && (CT)c[0] != (CT)0 ? 1 : 0;
      return;
    }
    canonical_sort(sa, sb, un);
    const uint64_t m = merge_sorted(sa, sb, un, 0.0, nullptr);
    cur.swap(sa);
    N = m;
  }

  // ---- apply layer -----------------------------------------------------------------------------
  void noise_step(const pp_layer* L, pp_layer_stats& ls) {
    const int mode = obs->mode;
    const int M = obs->trunc.max_order;
    HostNoise hn = prepare_noise(L, mode, M);
    NoiseDev nd = upload_noise(hn, L->noise_sign, mode, M);
    if (N == 0) return;
    if (mode == PP_MODE_GREEDY) {
      noise_greedy(cur.view(), N, nd, "noise");
    } else {
      GroupMask gm;
      for (int w = 0; w < PP_MAXW; ++w) { gm.mx[w] = ~0ULL; gm.mz[w] = ~0ULL; }
      grouped_pass({}, KIND_NOISE, 0.0, &nd, obs->trunc.eps, ls);
      // error-order mode: the noise is followed by the threshold (in the pass) and the cap
      if (obs->trunc.max_terms > 0 && (int64_t)N > obs->trunc.max_terms)
        cap_select((uint64_t)obs->trunc.max_terms, ls);
    }
  }

  // Sine-order mode: greedy noise, and every gate through the per-gate path, whose
  // expansion counts the sines of non-Clifford gates in the tag; threshold and cap after
  // every non-Clifford gate.
  void sine_order_layer(const pp_layer* L0) {
    // The Clifford interaction picture of the Euclid appendix: a rotation by theta about R
    // becomes the exact Clifford rotation by the nearest multiple k pi/2 (first; the two
    // commute) and one by the residual theta - k pi/2, |residual| <= pi/4, so every sine the
    // tag counts is at most 1/sqrt 2.  A whole turn (k = 0 mod 4) is a phase under
    // conjugation and is left out; Clifford angles stay single gates.
    std::vector<uint64_t> ipx, ipz;
    std::vector<double> ipt;
    const double half = M_PI / 2;
    for (int g = 0; g < L0->n_gates; ++g) {
      const double t = L0->theta[g];
      const double k = std::nearbyint(t / half);
      const double r = t - k * half;
      std::vector<double> parts;
      if (std::fabs(r) <= 1e-12 * half) parts = {t};
      else if ((((long long)k % 4) + 4) % 4 == 0) parts = {r};
      else parts = {k * half, r};
      for (double a : parts) {
        for (int w = 0; w < W; ++w) {
          ipx.push_back(L0->gx[(size_t)g * W + w]);
          ipz.push_back(L0->gz[(size_t)g * W + w]);
        }
        ipt.push_back(a);
      }
    }
    pp_layer ip = *L0;
    ip.n_gates = (int)ipt.size();
    ip.gx = ipx.data();
    ip.gz = ipz.data();
    ip.theta = ipt.data();
    const pp_layer* L = &ip;
    pp_layer_stats ls{};
    ls.n_in = (int64_t)N;
    auto noise = [&]() {
      if (L->n_gen <= 0) return;
      HostNoise hn = prepare_noise(L, PP_MODE_GREEDY, 0);
      NoiseDev nd = upload_noise(hn, L->noise_sign, PP_MODE_GREEDY, 0);
      if (N) noise_greedy(cur.view(), N, nd, "noise");
    };
    if (!L->noise_after_gates) noise();
    const std::vector<HostGate> hg = prepare_gates(L);
    if (obs->trunc.max_terms > 0) {
      // with a cap: the tiled gate passes in sine order, one run of gates of a kind at a time
      // (the tags are part of each term's key, the sin parts step them up)
      struct SineGuard {
        int* p;
        ~SineGuard() { *p = -1; }
      } sine_guard{&sine_limit};
      sine_limit = obs->trunc.max_order;
      size_t i = 0;
      while (i < hg.size() && N > 0) {
        size_t j = i + 1;
        const int kind = hg[i].kind;
        if (kind != KIND_OTHER)
          while (j < hg.size() && hg[j].kind == kind) ++j;
        std::vector<GateDev> run;
        for (size_t k = i; k < j; ++k) run.push_back(hg[k].g);
        gate_by_gate(run, kind, obs->trunc.eps, (uint64_t)obs->trunc.max_terms, ls);
        ls.n_peak = std::max(ls.n_peak, (int64_t)N);
        i = j;
      }
    } else {
      for (const HostGate& h : hg) {
        if (N == 0) break;
        cur.swap(sa);
        const uint64_t m = per_gate(N, {h.g}, obs->trunc.eps, nullptr, 0.0, nullptr, nullptr, obs->trunc.max_order);
        cur.swap(sa);
        N = m;
        ls.n_peak = std::max(ls.n_peak, (int64_t)N);
      }
    }
    if (L->noise_after_gates) noise();
    ls.n_out = (int64_t)N;
    ls.n_peak = std::max(ls.n_peak, std::max(ls.n_in, ls.n_out));
    obs->last = ls;
  }

  void apply_layer(const pp_layer* L) override {
    if (obs->mode == PP_MODE_SINE_ORDER) {
      sine_order_layer(L);
      return;
    }
    pp_layer_stats ls{};
    ls.n_in = (int64_t)N;
    // threshold (and cap) after every non-Clifford gate
    const double eps = obs->trunc.eps;
    const bool has_noise = L->n_gen > 0;
    bool noise_done = false;
    if (has_noise && !L->noise_after_gates) {
      noise_step(L, ls);
      noise_done = true;
    }
    std::vector<HostGate> hg = prepare_gates(L);
    if (!hg.empty() && N > 0) {
      bool all_cliff = true;
      for (auto& h : hg) all_cliff &= h.g.clifford != 0;
      const bool fuse_noise = has_noise && !noise_done && L->noise_after_gates;
      if (all_cliff) {
        std::vector<GateDev> gv;
        for (auto& h : hg) gv.push_back(h.g);
        gates_d.ensure(gv.size() * sizeof(GateDev) + 64);
        HIPCHK(hipMemcpyAsync(gates_d.p, gv.data(), gv.size() * sizeof(GateDev), hipMemcpyHostToDevice, st));
        NoiseDev nd{};
        int with_noise = 0;
        if (fuse_noise && obs->mode == PP_MODE_GREEDY) {
          HostNoise hn = prepare_noise(L, obs->mode, obs->trunc.max_order);
          nd = upload_noise(hn, L->noise_sign, obs->mode, obs->trunc.max_order);
          with_noise = 1;
          noise_done = true;
        }
        const Terms<CT> t = cur.view();
        const uint64_t n = N;
        const GateDev* gd = gates_d.as<GateDev>();
        const int ng = (int)gv.size();
        const size_t lds = ng * sizeof(GateDev) + (with_noise ? noise_lds_bytes(nd) : 0);
        if (lds > 160 * 1024) throw_fail(PP_ERR_UNSUPPORTED, "gate and noise tables exceed LDS");
        if (lds > kNoiseLdsMax)
          HIPCHK(hipFuncSetAttribute((const void*)k_clifford<W, CT, ORD>,
                                     hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
        ctx->run("clifford_layer", 2.0 * kTermBytes * n, (double)n, [&] {
          hipLaunchKernelGGL((k_clifford<W, CT, ORD>), dim3(table_grid(n)), dim3(1024), lds, st, t, n, gd, ng,
                             with_noise, nd);
        });
        ctx->check_launch();
        sync();   // gv is a host vector
      } else {
        // split into runs of X-type, Z-type, and single general gates
        size_t i = 0;
        while (i < hg.size()) {
          size_t j = i + 1;
          const int kind = hg[i].kind;
          if (kind != KIND_OTHER)
            while (j < hg.size() && hg[j].kind == kind) ++j;
          std::vector<GateDev> run;
          for (size_t k = i; k < j; ++k) run.push_back(hg[k].g);
          GroupMask gm;
          for (int w = 0; w < PP_MAXW; ++w) { gm.mx[w] = 0; gm.mz[w] = 0; }
          for (int w = 0; w < W; ++w) {
            if (kind == KIND_X) { gm.mx[w] = 0; gm.mz[w] = ~0ULL; }
            else if (kind == KIND_Z) { gm.mx[w] = ~0ULL; gm.mz[w] = 0; }
            else { gm.mx[w] = ~0ULL; gm.mz[w] = ~0ULL; }
          }
          if (kind == KIND_OTHER) {   // pair key: clear the pivot bit
            const int pw = run[0].pivot_word, pb = run[0].pivot_bit;
            if (pw < W) gm.mx[pw] &= ~(1ULL << pb);
            else gm.mz[pw - W] &= ~(1ULL << pb);
          }
          const bool last = j == hg.size();
          NoiseDev nd{};
          const NoiseDev* ndp = nullptr;
          if (last && fuse_noise && obs->mode == PP_MODE_ERROR_ORDER) {
            HostNoise hn = prepare_noise(L, obs->mode, obs->trunc.max_order);
            nd = upload_noise(hn, L->noise_sign, obs->mode, obs->trunc.max_order);
            ndp = &nd;
            noise_done = true;
          }
          if (!grouped_pass(run, kind, eps, ndp, eps, ls)) noise_done = false;
          else if (ndp && obs->trunc.max_terms > 0 && (int64_t)N > obs->trunc.max_terms)
            cap_select((uint64_t)obs->trunc.max_terms, ls);   // the cap after the fused noise
          i = j;
        }
      }
    }
    if (has_noise && !noise_done) noise_step(L, ls);
    ls.n_out = (int64_t)N;
    ls.n_peak = std::max(ls.n_peak, std::max(ls.n_in, ls.n_out));
    obs->last = ls;
  }

  // ---- cap -------------------------------------------------------------------------------------
  static double coef_from_bits_host(uint64_t b) {
    if (sizeof(CT) == 8) {
      double v;
      std::memcpy(&v, &b, 8);
      return v;
    }
    const uint32_t u = (uint32_t)b;
    float f;
    std::memcpy(&f, &u, 4);
    return (double)f;
  }

  // Keep the K largest |c| (ties to the smaller canonical key).
  void cap_select(uint64_t K, pp_layer_stats& ls) {
    if (N <= K) return;
    const uint64_t before = N;
    const CutDev cut = cap_cut(K, N);
    apply_cut(cut, ls);
    ls.n_capped += (int64_t)(before - N);
  }

  void truncate(double eps, int64_t cap) override {
    pp_layer_stats ls{};
    if (N > 0 && eps > 0.0) {
      u32b.ensure(N * 4 + 64);
      uint32_t* keep = u32b.as<uint32_t>();
      const CT* c = cur.view().c;
      const uint64_t n = N;
      ctx->run("threshold", 0, (double)n, [&] {
        hipLaunchKernelGGL((k_threshold_flags<CT>), gridb(n), dim3(256), 0, st, c, n, eps, keep, (double*)nullptr);
      });
      ctx->check_launch();
      compact_cur(keep);
    }
    if (cap > 0 && (int64_t)N > cap) cap_select((uint64_t)cap, ls);
  }

  // Propagated antinoise (Section I.A, Eq. applyantinoise): O -> (1 - q) O + q E' O E'.
  // Every term expands into 1 + K(K-1)/2 slots (k_expand_antinoise), the slots are put in
  // canonical order and merged with the observable's eps threshold, then the cap applies.
  void antinoise(const EngineBase* eb, double q) override {
    const auto* e = dynamic_cast<const Engine*>(eb);
    if (!e) throw_fail(PP_ERR_UNSUPPORTED, "E' must have the same word count, precision and mode as O");
    if (N == 0) return;
    const uint64_t S = slots_per_term(e->N);
    if (N * S < kExpandSlab) {
      finish_expansion(expand_items({{cur.view(), N, e, q, 1.0 - q}}));
      return;
    }
    // Larger than one slab: the map is linear in O, so O is expanded a chunk of terms at a
    // time; each chunk's expansion is merged without a threshold and appended to alt, and
    // the concatenation is merged once more with the threshold, then capped.
    const uint64_t chunk = std::max<uint64_t>(1, kExpandSlab / S);
    uint64_t acc = 0;
    for (uint64_t i0 = 0; i0 < N; i0 += chunk) {
      const uint64_t n = std::min<uint64_t>(chunk, N - i0);
      Terms<CT> part = cur.view();   // planes keep cur's stride; the chunk starts at term i0
      part.x = cur.view().x + i0;
      part.z = cur.view().z + i0;
      part.c = cur.view().c + i0;
      if (ORD) part.o = cur.view().o + i0;
      const uint64_t m = merge_expansion(expand_items({{part, n, e, q, 1.0 - q}}), 0.0);
      grow_keep(alt, acc + m, acc);
      const Terms<CT> from = sa.view(), to = alt.view();
      ctx->run("copy", 0, (double)m, [&] {
        hipLaunchKernelGGL((k_copy<W, CT, ORD>), grid1(m), dim3(256), 0, st, from, 0, to, acc, m);
      });
      ctx->check_launch();
      acc += m;
    }
    sa.ensure(std::max<uint64_t>(acc, 1));
    u32b.ensure(acc * 4 + 64);
    {
      const Terms<CT> from = alt.view(), to = sa.view();
      ctx->run("copy", 0, (double)acc, [&] {
        hipLaunchKernelGGL((k_copy<W, CT, ORD>), grid1(acc), dim3(256), 0, st, from, 0, to, 0, acc);
      });
      ctx->check_launch();
      hipLaunchKernelGGL(k_fill_u32, grid1(acc), dim3(256), 0, st, u32b.as<uint32_t>(), acc, 1u);
      ctx->check_launch();
    }
    finish_expansion(acc);
  }

  // One expansion of a batch: `scale` C(X) (scale E' X E') for an E', or id X alone (e
  // null), for X = the first n terms of `in`.
  struct ExpItem {
    Terms<CT> in;
    uint64_t n;
    const Engine* e;
    double scale, id;
  };

  // Writes every item's slots at consecutive offsets of sa (flags in u32b); returns the
  // slot count.  Pair tables of all items go up in one copy.
  // Slots per term of an expansion by an E' of K terms: P itself and one per unordered pair.
  static uint64_t slots_per_term(uint64_t K) { return 1 + (K ? K * (K - 1) / 2 : 0); }

  uint64_t expand_items(const std::vector<ExpItem>& items) {
    std::vector<uint64_t> S(items.size()), off(items.size() + 1, 0);
    for (size_t i = 0; i < items.size(); ++i) {
      const uint64_t K = items[i].e ? items[i].e->N : 0;
      if (K > kMaxAntinoiseTerms)
        throw_fail(PP_ERR_UNSUPPORTED, "E' has " + std::to_string(K) + " terms; at most " +
                                           std::to_string(kMaxAntinoiseTerms) + " are supported");
      S[i] = slots_per_term(K);
      off[i + 1] = off[i] + items[i].n * S[i];
      if (off[i + 1] >= (1ULL << 31))
        throw_fail(PP_ERR_UNSUPPORTED, "antinoise expansion exceeds 2^31 - 1 terms");
    }
    const uint64_t total = off.back();
    sa.ensure(std::max<uint64_t>(total, 1));
    u32b.ensure(total * 4 + 64);
    uint32_t* keep = u32b.as<uint32_t>();
    const Terms<CT> out = sa.view();
    for (size_t i = 0; i < items.size(); ++i) {
      const ExpItem& it = items[i];
      if (it.n == 0) continue;
      Terms<CT> o = out;
      o.x += off[i];
      o.z += off[i];
      o.c += off[i];
      if (ORD) o.o += off[i];
      const Terms<CT> ev = it.e ? it.e->cur.view() : it.in;
      const uint32_t K = it.e ? (uint32_t)it.e->N : 0u;
      const uint64_t cnt = it.n * S[i];
      const unsigned grid = (unsigned)std::min<uint64_t>(cdiv(cnt, 256), 1u << 20);
      const double q = it.e ? it.scale : 0.0;
      ctx->run("antinoise_expand", kTermBytes * (double)(it.n + cnt) + 4.0 * cnt, (double)cnt, [&] {
        hipLaunchKernelGGL((k_expand_antinoise<W, CT, ORD>), dim3(grid), dim3(256), 0, st, it.in, it.n, ev, K, S[i], q,
                           it.id, o, keep + off[i]);
      });
      ctx->check_launch();
    }
    return total;
  }

  // A batch of commuting antinoise maps to first or second order in the number of errors
  // (Appendix C): with a_c = q_c / (1 - q_c), O0 = O prod (1 - q_c), O1 = sum a_c C_c(O0),
  // O2 = 1/2 sum (a_c C_c(O1') - a_c^2 O0) with O1' = O1 without its terms below eps (the
  // second pass's input only); O becomes O0 + O1 (+ O2), then eps and the cap.
  void antinoise_batch(const std::vector<const EngineBase*>& ebs, const double* q, int order) override {
    std::vector<const Engine*> es;
    for (const EngineBase* b : ebs) {
      const auto* e = dynamic_cast<const Engine*>(b);
      if (!e) throw_fail(PP_ERR_UNSUPPORTED, "E' must have the same word count, precision and mode as O");
      es.push_back(e);
    }
    if (N == 0) return;
    double p0 = 1.0, a2 = 0.0;
    std::vector<double> a(es.size());
    for (size_t c = 0; c < es.size(); ++c) {
      p0 *= 1.0 - q[c];
      a[c] = q[c] / (1.0 - q[c]);
      a2 += a[c] * a[c];
    }
    const Terms<CT> o = cur.view();
    if (order == 1) {
      std::vector<ExpItem> items{{o, N, nullptr, 0.0, p0}};
      for (size_t c = 0; c < es.size(); ++c) items.push_back({o, N, es[c], a[c] * p0, 0.0});
      finish_expansion(expand_items(items));
      return;
    }
    std::vector<ExpItem> first;
    for (size_t c = 0; c < es.size(); ++c) first.push_back({o, N, es[c], a[c] * p0, 0.0});
    const uint64_t m1 = merge_expansion(expand_items(first), obs->trunc.eps);   // O1'
    tmp.swap(sa);
    const Terms<CT> t1 = tmp.view();
    std::vector<ExpItem> second{{o, N, nullptr, 0.0, p0 * (1.0 - 0.5 * a2)}};
    for (size_t c = 0; c < es.size(); ++c) second.push_back({o, N, es[c], a[c] * p0, 0.0});   // O1 in full
    for (size_t c = 0; c < es.size(); ++c) second.push_back({t1, m1, es[c], 0.5 * a[c], 0.0});
    finish_expansion(expand_items(second));
  }

  // After an antinoise expansion: sa holds `total` slots and u32b their nonzero flags.
  // Exact zeros (pairs whose two orders cancel) are dropped, the rest put in canonical
  // order and merged with the eps threshold, and the cap applied; the result becomes O.
  void finish_expansion(uint64_t total) {
    const uint64_t m = merge_expansion(total, obs->trunc.eps);
    cur.swap(sa);
    N = m;
    pp_layer_stats ls{};
    if (obs->trunc.max_terms > 0 && (int64_t)N > obs->trunc.max_terms) cap_select((uint64_t)obs->trunc.max_terms, ls);
  }

  // Compaction of the nonzero slots, canonical sort and merge with threshold `thr`;
  // returns the term count, the terms in sa.
  uint64_t merge_expansion(uint64_t total, double thr) {
    if (total == 0) return 0;
    u32c.ensure(total * 4 + 64);
    uint32_t* keep = u32b.as<uint32_t>();
    uint32_t* pos = u32c.as<uint32_t>();
    HIPCHK(hipMemcpyAsync(pos, keep, total * 4, hipMemcpyDeviceToDevice, st));
    scan_u32(pos, total);
    HIPCHK(hipMemcpyAsync(ctx->pinned, pos + total - 1, 4, hipMemcpyDeviceToHost, st));
    HIPCHK(hipMemcpyAsync((char*)ctx->pinned + 4, keep + total - 1, 4, hipMemcpyDeviceToHost, st));
    sync();
    uint32_t lp = 0, lk = 0;
    std::memcpy(&lp, ctx->pinned, 4);
    std::memcpy(&lk, (char*)ctx->pinned + 4, 4);
    const uint64_t nz = (uint64_t)lp + lk;
    sb.ensure(std::max<uint64_t>(nz, 1));
    const Terms<CT> out = sa.view(), dense = sb.view();
    ctx->run("compact", 0, (double)total, [&] {
      hipLaunchKernelGGL((k_compact<W, CT, ORD>), grid1(total), dim3(256), 0, st, out, dense, total,
                         (const uint32_t*)keep, (const uint32_t*)pos);
    });
    ctx->check_launch();
    sa.swap(sb);
    canonical_sort(sa, sb, nz);
    return merge_sorted(sa, sb, nz, thr, nullptr);
  }

  // E' O E' limited to the products of the k largest magnitudes |c_s| |e_a| |e_b| over
  // ordered triplets, ties with the k-th kept (Appendix B's heuristic conjugation).  The
  // cut tau is found on the device by bisection; only the kept pairs are expanded.
  void antinoise_topk(const EngineBase* eb, double q, int64_t kmax) override {
    const auto* e = dynamic_cast<const Engine*>(eb);
    if (!e) throw_fail(PP_ERR_UNSUPPORTED, "E' must have the same word count, precision and mode as O");
    if (N == 0) return;
    const uint64_t K = e->N;
    if (K > kMaxTopkTerms)
      throw_fail(PP_ERR_UNSUPPORTED, "E' has " + std::to_string(K) + " terms; at most " +
                                         std::to_string(kMaxTopkTerms) + " are supported with a product limit");
    if (K < 2 || kmax <= 0 || (uint64_t)kmax >= N * K * (K - 1)) {
      antinoise(eb, q);
      return;
    }
    // pairs a < b of E' (the limited products; a = b are always kept), largest |e_a| |e_b|
    // first: keys generated, put in canonical order and tabulated on the device
    const uint64_t P = K * (K - 1) / 2;
    ta.ensure(P);
    tb.ensure(P);
    {
      const Terms<double> kt = ta.view();
      const CT* ecd = e->cur.view().c;
      const unsigned grid = (unsigned)std::min<uint64_t>(cdiv(P, 256), 1u << 20);
      ctx->run("topk_pairs", 0, (double)P, [&] {
        hipLaunchKernelGGL((k_pair_keys<W, CT>), dim3(grid), dim3(256), 0, st, ecd, K, P, kt);
      });
      ctx->check_launch();
    }
    canonical_sort(ta, tb, P);
    // tables: pm[P] doubles, cw[P + 1] u64, tau (one double), the slot total (u64), pidx[P]
    // u64, the weights w[P] u32 (scanned in place)
    const size_t o_cw = P * 8, o_tau = o_cw + (P + 1) * 8, o_sum = o_tau + 8, o_idx = o_sum + 8, o_w = o_idx + P * 8;
    topk_d.ensure(o_w + P * 4 + 64);
    double* pm_w = (double*)topk_d.p;
    uint64_t* cw_w = (uint64_t*)((char*)topk_d.p + o_cw);
    uint64_t* pidx_w = (uint64_t*)((char*)topk_d.p + o_idx);
    uint32_t* w_w = (uint32_t*)((char*)topk_d.p + o_w);
    HIPCHK(hipMemsetAsync((char*)topk_d.p + o_tau, 0, 16, st));
    {
      const Terms<double> srt = ta.view();
      hipLaunchKernelGGL(k_pair_tables, grid1(P), dim3(256), 0, st, srt, P, pm_w, pidx_w, w_w);
      ctx->check_launch();
      scan_u32(w_w, P);
      hipLaunchKernelGGL(k_pair_cw, grid1(P), dim3(256), 0, st, (const uint32_t*)w_w, (const uint64_t*)pidx_w, P,
                         cw_w);
      ctx->check_launch();
    }
    const double* pm_d = (const double*)topk_d.p;
    const uint64_t* cw_d = (const uint64_t*)((char*)topk_d.p + o_cw);
    double* tau_d = (double*)((char*)topk_d.p + o_tau);
    unsigned long long* sum_d = (unsigned long long*)((char*)topk_d.p + o_sum);
    const uint64_t* pidx_d = (const uint64_t*)((char*)topk_d.p + o_idx);
    const CT* c = cur.view().c;
    const uint64_t n = N;
    ctx->run("topk_cut", 0, (double)n, [&] {
      hipLaunchKernelGGL((k_topk_cut<CT>), dim3(1), dim3(1024), 0, st, c, n, pm_d, cw_d, (uint32_t)P,
                         (uint64_t)kmax, 0x7FF0000000000000ULL, tau_d);
    });
    ctx->check_launch();
    u32b.ensure(n * 4 + 64);
    topk_off.ensure(n * 4 + 64);
    uint32_t* lens = u32b.as<uint32_t>();
    uint32_t* off = topk_off.as<uint32_t>();
    ctx->run("topk_lens", 0, (double)n, [&] {
      hipLaunchKernelGGL((k_topk_lens<CT>), grid1(n), dim3(256), 0, st, c, n, pm_d, (uint32_t)P,
                         (const double*)tau_d, lens, sum_d);
    });
    ctx->check_launch();
    HIPCHK(hipMemcpyAsync(ctx->pinned, sum_d, 8, hipMemcpyDeviceToHost, st));
    sync();
    uint64_t total = 0;
    std::memcpy(&total, ctx->pinned, 8);
    if (total >= (1ULL << 31))
      throw_fail(PP_ERR_UNSUPPORTED, "antinoise expansion of " + std::to_string(total) + " terms exceeds 2^31 - 1");
    HIPCHK(hipMemcpyAsync(off, lens, n * 4, hipMemcpyDeviceToDevice, st));
    scan_u32(off, n);
    sa.ensure(total);
    u32b.ensure(total * 4 + 64);   // the flags replace lens, which is no longer read
    uint32_t* keep = u32b.as<uint32_t>();
    const Terms<CT> in = cur.view(), ev = e->cur.view(), out = sa.view();
    const uint32_t* offc = topk_off.as<uint32_t>();
    const unsigned grid = (unsigned)std::min<uint64_t>(cdiv(total, 256), 1u << 20);
    ctx->run("antinoise_topk_expand", kTermBytes * (double)(n + total) + 4.0 * total, (double)total, [&] {
      hipLaunchKernelGGL((k_expand_topk<W, CT, ORD>), dim3(grid), dim3(256), 0, st, in, n, offc, total, ev,
                         (uint32_t)K, pidx_d, q, out, keep);
    });
    ctx->check_launch();
    finish_expansion(total);
  }

  double expectation(const uint64_t* basis) override {
    GroupMask b;
    for (int w = 0; w < PP_MAXW; ++w) { b.mx[w] = 0; b.mz[w] = 0; }
    if (basis)
      for (int w = 0; w < W; ++w) b.mz[w] = basis[w];
    // Only diagonal strings contribute.  They are gathered and put in canonical order
    // first, so the FP64 sum runs in an order fixed by the term set alone, and the value
    // does not depend on where earlier kernels happened to place each term.
    uint64_t n = 0;
    if (N > 0) {
      u32b.ensure(N * 4 + 64);
      u32c.ensure(N * 4 + 64);
      uint32_t* keep = u32b.as<uint32_t>();
      uint32_t* pos = u32c.as<uint32_t>();
      const Terms<CT> all = cur.view();
      const uint64_t nall = N;
      ctx->run("diag_flags", 0, (double)nall, [&] {
        hipLaunchKernelGGL((k_diag_flags<W, CT>), grid1(nall), dim3(256), 0, st, all, nall, keep);
      });
      ctx->check_launch();
      HIPCHK(hipMemcpyAsync(pos, keep, nall * 4, hipMemcpyDeviceToDevice, st));
      scan_u32(pos, nall);
      uint32_t lp = 0, lk = 0;
      HIPCHK(hipMemcpyAsync(ctx->pinned, pos + nall - 1, 4, hipMemcpyDeviceToHost, st));
      HIPCHK(hipMemcpyAsync((char*)ctx->pinned + 4, keep + nall - 1, 4, hipMemcpyDeviceToHost, st));
      sync();
      std::memcpy(&lp, ctx->pinned, 4);
      std::memcpy(&lk, (char*)ctx->pinned + 4, 4);
      n = (uint64_t)lp + lk;
      sa.ensure(std::max<uint64_t>(n, 1));
      const Terms<CT> dg = sa.view();
      ctx->run("compact", 0, (double)nall, [&] {
        hipLaunchKernelGGL((k_compact<W, CT, ORD>), grid1(nall), dim3(256), 0, st, all, dg, nall,
                           (const uint32_t*)keep, (const uint32_t*)pos);
      });
      ctx->check_launch();
      canonical_sort(sa, sb, n);
    }
    const unsigned nb = (unsigned)std::max<uint64_t>(1, std::min<uint64_t>(1024, cdiv(n, 256)));
    partial_d.ensure(nb * 8 + 64);
    double* part = partial_d.as<double>();
    const Terms<CT> t = sa.view();
    double* outd = &cnt_d.as<Counters>()->dropped;
    ctx->run("expectation", kTermBytes * n, (double)n, [&] {
      hipLaunchKernelGGL((k_expect<W, CT>), dim3(nb), dim3(256), 0, st, t, n, b, part);
      hipLaunchKernelGGL(k_sum_partials, dim3(1), dim3(64), 0, st, (const double*)part, (int)nb, outd);
    });
    ctx->check_launch();
    double v = 0.0;
    HIPCHK(hipMemcpyAsync(ctx->pinned, outd, 8, hipMemcpyDeviceToHost, st));
    sync();
    std::memcpy(&v, ctx->pinned, 8);
    return v;
  }

  // <b|O|b> with no allocation: k_expect over all N slots (it skips non-diagonal strings)
  // with its workgroup partials in the caller-given device scratch, the reduction into the
  // slot after them, and one copy to the context's pinned host word.  The sum runs in the
  // terms' storage order, so it can differ from expectation()'s canonical-order sum by
  // rounding.  No instrumentation (which would allocate events).
  double expectation_noalloc(const uint64_t* basis, double* dev_scratch) override {
    GroupMask b;
    for (int w = 0; w < PP_MAXW; ++w) { b.mx[w] = 0; b.mz[w] = 0; }
    if (basis)
      for (int w = 0; w < W; ++w) b.mz[w] = basis[w];
    const uint64_t n = N;
    const unsigned nb = (unsigned)std::max<uint64_t>(1, std::min<uint64_t>(kNoAllocBlocks, cdiv(n, 256)));
    double* part = dev_scratch;
    double* outd = dev_scratch + kNoAllocBlocks;
    const Terms<CT> t = cur.view();
    hipLaunchKernelGGL((k_expect<W, CT>), dim3(nb), dim3(256), 0, st, t, n, b, part);
    ctx->check_launch();
    hipLaunchKernelGGL(k_sum_partials, dim3(1), dim3(64), 0, st, (const double*)part, (int)nb, outd);
    ctx->check_launch();
    HIPCHK(hipMemcpyAsync(ctx->pinned, outd, 8, hipMemcpyDeviceToHost, st));
    sync();
    double v = 0.0;
    std::memcpy(&v, ctx->pinned, 8);
    return v;
  }

  void export_terms(uint64_t* x, uint64_t* z, double* c, uint8_t* o) override {
    if (N == 0) return;
    const uint64_t n = N;
    sa.ensure(n);
    {
      const Terms<CT> from = cur.view(), to = sa.view();
      ctx->run("copy", 0, (double)n, [&] {
        hipLaunchKernelGGL((k_copy<W, CT, ORD>), grid1(n), dim3(256), 0, st, from, 0, to, 0, n);
      });
      ctx->check_launch();
    }
    canonical_sort(sa, sb, n);
    const Terms<CT> t = sa.view();
    std::vector<uint64_t> plane(n);
    for (int w = 0; w < W; ++w) {
      if (x) {
        HIPCHK(hipMemcpyAsync(plane.data(), t.x + (size_t)w * t.stride, n * 8, hipMemcpyDeviceToHost, st));
        sync();
        for (uint64_t i = 0; i < n; ++i) x[i * W + w] = plane[i];
      }
      if (z) {
        HIPCHK(hipMemcpyAsync(plane.data(), t.z + (size_t)w * t.stride, n * 8, hipMemcpyDeviceToHost, st));
        sync();
        for (uint64_t i = 0; i < n; ++i) z[i * W + w] = plane[i];
      }
    }
    if (c) {
      f64_d.ensure(n * 8 + 64);
      double* d = f64_d.as<double>();
      const CT* src = t.c;
      ctx->run("convert", 0, (double)n, [&] {
        hipLaunchKernelGGL((k_to_f64<CT>), grid1(n), dim3(256), 0, st, src, d, n);
      });
      ctx->check_launch();
      HIPCHK(hipMemcpyAsync(c, d, n * 8, hipMemcpyDeviceToHost, st));
      sync();
    }
    if (o) {
      if (ORD) {
        HIPCHK(hipMemcpyAsync(o, t.o, n, hipMemcpyDeviceToHost, st));
        sync();
      } else {
        std::memset(o, 0, n);
      }
    }
  }
};

template <int W>
EngineBase* make_engine_w(pp_obs* o) {
  const bool f32 = o->prec == PP_F32_KAHAN;
  const bool ord = o->mode != PP_MODE_GREEDY;
  if (!f32 && !ord) return new Engine<W, double, false>(o);
  if (!f32 && ord) return new Engine<W, double, true>(o);
  if (f32 && !ord) return new Engine<W, float, false>(o);
  return new Engine<W, float, true>(o);
}

EngineBase* make_engine(pp_obs* o) {
  switch (o->W) {
    case 1: return make_engine_w<1>(o);
    case 2: return make_engine_w<2>(o);
    case 3: return make_engine_w<3>(o);
    case 4: return make_engine_w<4>(o);
  }
  throw_fail(PP_ERR_UNSUPPORTED, "more than 256 qubits");
}

template <class F>
pp_status guarded(F&& f) {
  try {
    f();
    return PP_OK;
  } catch (const Failure& e) {
    g_last_error = e.msg;
    return e.status;
  } catch (const std::bad_alloc&) {
    g_last_error = "host allocation failed";
    return PP_ERR_OOM;
  } catch (const std::exception& e) {
    g_last_error = e.what();
    return PP_ERR_DEVICE;
  }
}

bool strings_ok(int n_qubits, int W, int64_t n, const uint64_t* x, const uint64_t* z) {
  const int top = n_qubits - 64 * (W - 1);
  const uint64_t mask = top >= 64 ? ~0ULL : ((1ULL << top) - 1);
  for (int64_t i = 0; i < n; ++i)
    if ((x[(size_t)i * W + W - 1] & ~mask) || (z[(size_t)i * W + W - 1] & ~mask)) return false;
  return true;
}

}  // namespace

// ---------------------------------------------------------------------------------------------
// C ABI
// ---------------------------------------------------------------------------------------------
extern "C" {

const char* pp_last_error(void) { return g_last_error.c_str(); }

pp_status pp_ctx_create(int device, void* hip_stream, pp_alloc_fn alloc, pp_release_fn release, void* user,
                        pp_ctx** out) {
  if (!out) { g_last_error = "out is NULL"; return PP_ERR_INVALID; }
  *out = nullptr;
  if ((alloc == nullptr) != (release == nullptr)) {
    g_last_error = "alloc and release must both be given or both be NULL";
    return PP_ERR_INVALID;
  }
  return guarded([&] {
    int count = 0;
    HIPCHK(hipGetDeviceCount(&count));
    if (device < 0 || device >= count) throw_fail(PP_ERR_INVALID, "device index out of range");
    HIPCHK(hipSetDevice(device));
    register_scratch(device, count);
    auto* c = new pp_ctx;
    c->device = device;
    c->stream = (hipStream_t)hip_stream;
    c->alloc = alloc;
    c->release = release;
    c->user = user;
    if (hipHostMalloc((void**)&c->pinned, 1 << 16, hipHostMallocDefault) != hipSuccess) {
      delete c;
      throw_fail(PP_ERR_OOM, "pinned host allocation failed");
    }
    *out = c;
  });
}

void pp_ctx_destroy(pp_ctx* ctx) {
  if (!ctx) return;
  (void)hipSetDevice(ctx->device);
  (void)hipStreamSynchronize(ctx->stream);
  for (auto& p : ctx->pending) { (void)hipEventDestroy(p.a); (void)hipEventDestroy(p.b); }
  for (auto e : ctx->evfree) (void)hipEventDestroy(e);
  if (ctx->pinned) (void)hipHostFree(ctx->pinned);
  delete ctx;
}

pp_status pp_create_observable(pp_ctx* ctx, int n_qubits, int64_t n_terms, const uint64_t* x, const uint64_t* z,
                               const double* coeff, pp_precision precision, pp_mode mode, pp_trunc trunc,
                               pp_obs** out) {
  if (!out) { g_last_error = "out is NULL"; return PP_ERR_INVALID; }
  *out = nullptr;
  if (!ctx) { g_last_error = "ctx is NULL"; return PP_ERR_INVALID; }
  if (n_qubits < 1 || n_qubits > 64 * PP_MAXW) { g_last_error = "n_qubits must be in 1..256"; return PP_ERR_INVALID; }
  if (n_terms < 0 || n_terms >= (1LL << 31)) { g_last_error = "n_terms out of range"; return PP_ERR_INVALID; }
  if (n_terms > 0 && (!x || !z || !coeff)) { g_last_error = "NULL term array"; return PP_ERR_INVALID; }
  if (precision != PP_F64 && precision != PP_F32_KAHAN) { g_last_error = "bad precision"; return PP_ERR_INVALID; }
  if (mode != PP_MODE_GREEDY && mode != PP_MODE_ERROR_ORDER && mode != PP_MODE_SINE_ORDER) { g_last_error = "bad mode"; return PP_ERR_INVALID; }
  if (mode == PP_MODE_SINE_ORDER && (trunc.max_order < 0 || trunc.max_order > 250)) {
    g_last_error = "max_order must be in 0..250 in the sine-order mode";
    return PP_ERR_INVALID;
  }
  if (!(trunc.eps >= 0.0) || !std::isfinite(trunc.eps)) { g_last_error = "eps must be finite and >= 0"; return PP_ERR_INVALID; }
  if (trunc.max_terms < 0) { g_last_error = "max_terms must be >= 0"; return PP_ERR_INVALID; }
  if (mode == PP_MODE_ERROR_ORDER && (trunc.max_order < 0 || trunc.max_order > kMaxPowerSums)) {
    g_last_error = "max_order must be in 0..4 on the GPU";
    return PP_ERR_UNSUPPORTED;
  }
  const int W = (n_qubits + 63) / 64;
  if (n_terms > 0 && !strings_ok(n_qubits, W, n_terms, x, z)) { g_last_error = "string bits above n_qubits"; return PP_ERR_INVALID; }
  for (int64_t i = 0; i < n_terms; ++i)
    if (!std::isfinite(coeff[i])) { g_last_error = "non-finite coefficient"; return PP_ERR_INVALID; }
  pp_obs* o = new pp_obs;
  o->ctx = ctx;
  o->n_qubits = n_qubits;
  o->W = W;
  o->prec = precision;
  o->mode = mode;
  o->trunc = trunc;
  const pp_status s = guarded([&] {
    HIPCHK(hipSetDevice(ctx->device));
    o->eng.reset(make_engine(o));
    o->eng->create(n_terms, x, z, coeff);
  });
  if (s != PP_OK) {
    delete o;
    return s;
  }
  *out = o;
  return PP_OK;
}

pp_status pp_set_terms(pp_obs* obs, int64_t n_terms, const uint64_t* x, const uint64_t* z, const double* coeff) {
  if (!obs) { g_last_error = "NULL argument"; return PP_ERR_INVALID; }
  if (obs->broken) { g_last_error = "observable is unusable after an earlier device error"; return PP_ERR_INVALID; }
  if (n_terms < 0 || n_terms >= (1LL << 31)) { g_last_error = "n_terms out of range"; return PP_ERR_INVALID; }
  if (n_terms > 0 && (!x || !z || !coeff)) { g_last_error = "NULL term array"; return PP_ERR_INVALID; }
  if (n_terms > 0 && !strings_ok(obs->n_qubits, obs->W, n_terms, x, z)) { g_last_error = "string bits above n_qubits"; return PP_ERR_INVALID; }
  for (int64_t i = 0; i < n_terms; ++i)
    if (!std::isfinite(coeff[i])) { g_last_error = "non-finite coefficient"; return PP_ERR_INVALID; }
  const pp_status s = guarded([&] {
    HIPCHK(hipSetDevice(obs->ctx->device));
    obs->eng->create(n_terms, x, z, coeff);
  });
  if (s == PP_ERR_DEVICE || s == PP_ERR_OOM) obs->broken = true;
  return s;
}

pp_status pp_apply_layer(pp_obs* obs, const pp_layer* L) {
  if (!obs || !L) { g_last_error = "NULL argument"; return PP_ERR_INVALID; }
  if (obs->broken) { g_last_error = "observable is unusable after an earlier device error"; return PP_ERR_INVALID; }
  if (L->n_gates < 0 || L->n_gen < 0) { g_last_error = "negative count"; return PP_ERR_INVALID; }
  if (L->n_gates > 0 && (!L->gx || !L->gz || !L->theta)) { g_last_error = "NULL gate array"; return PP_ERR_INVALID; }
  if (L->n_gen > 0 && (!L->ex || !L->ez || !L->lambda)) { g_last_error = "NULL noise array"; return PP_ERR_INVALID; }
  if (L->n_gates > 0 && L->dir != PP_HEISENBERG && L->dir != PP_FORWARD) { g_last_error = "dir must be +1 or -1"; return PP_ERR_INVALID; }
  if (L->n_gen > 0 && L->noise_sign != 1 && L->noise_sign != -1) { g_last_error = "noise_sign must be +1 or -1"; return PP_ERR_INVALID; }
  for (int g = 0; g < L->n_gates; ++g)
    if (!std::isfinite(L->theta[g])) { g_last_error = "non-finite angle"; return PP_ERR_INVALID; }
  for (int k = 0; k < L->n_gen; ++k)
    if (!(L->lambda[k] >= 0.0) || !std::isfinite(L->lambda[k])) { g_last_error = "lambda must be finite and >= 0"; return PP_ERR_INVALID; }
  if (L->n_gates > 0 && !strings_ok(obs->n_qubits, obs->W, L->n_gates, L->gx, L->gz)) { g_last_error = "gate bits above n_qubits"; return PP_ERR_INVALID; }
  if (L->n_gen > 0 && !strings_ok(obs->n_qubits, obs->W, L->n_gen, L->ex, L->ez)) { g_last_error = "generator bits above n_qubits"; return PP_ERR_INVALID; }
  const pp_status s = guarded([&] {
    HIPCHK(hipSetDevice(obs->ctx->device));
    obs->eng->apply_layer(L);
  });
  if (s == PP_ERR_DEVICE || s == PP_ERR_OOM) obs->broken = true;
  return s;
}

pp_status pp_truncate(pp_obs* obs, double eps, int64_t max_terms) {
  if (!obs) { g_last_error = "NULL argument"; return PP_ERR_INVALID; }
  if (obs->broken) { g_last_error = "observable is unusable after an earlier device error"; return PP_ERR_INVALID; }
  if (!(eps >= 0.0) || !std::isfinite(eps) || max_terms < 0) { g_last_error = "bad truncation arguments"; return PP_ERR_INVALID; }
  const pp_status s = guarded([&] {
    HIPCHK(hipSetDevice(obs->ctx->device));
    obs->eng->truncate(eps, max_terms);
  });
  if (s == PP_ERR_DEVICE || s == PP_ERR_OOM) obs->broken = true;
  return s;
}

// Quasi-probability of a generator's inverse map (Section I: the channel applies E with
// probability (1 - e^{-2 lambda})/2 and the inverse map negates lambda): (1 - e^{2 lambda})/2.
static double inverse_quasi_probability(double lambda) { return -0.5 * std::expm1(2.0 * lambda); }

pp_status pp_apply_antinoise(pp_obs* obs, const pp_obs* eprime, double lambda) {
  if (!obs || !eprime) { g_last_error = "NULL argument"; return PP_ERR_INVALID; }
  if (obs->broken || eprime->broken) { g_last_error = "observable is unusable after an earlier device error"; return PP_ERR_INVALID; }
  if (obs->ctx != eprime->ctx) { g_last_error = "O and E' belong to different contexts"; return PP_ERR_INVALID; }
  if (obs->n_qubits != eprime->n_qubits) { g_last_error = "O and E' have different qubit counts"; return PP_ERR_INVALID; }
  if (obs->prec != eprime->prec) { g_last_error = "O and E' have different precisions"; return PP_ERR_INVALID; }
  if (obs->mode != PP_MODE_GREEDY || eprime->mode != PP_MODE_GREEDY) { g_last_error = "antinoise needs PP_MODE_GREEDY observables"; return PP_ERR_UNSUPPORTED; }
  if (!std::isfinite(lambda) || lambda < 0.0 || lambda > 300.0) { g_last_error = "lambda must be finite, >= 0 and <= 300"; return PP_ERR_INVALID; }
  const double q = inverse_quasi_probability(lambda);
  const pp_status s = guarded([&] {
    HIPCHK(hipSetDevice(obs->ctx->device));
    obs->eng->antinoise(eprime->eng.get(), q);
  });
  if (s == PP_ERR_DEVICE || s == PP_ERR_OOM) obs->broken = true;
  return s;
}

pp_status pp_apply_antinoise_batch(pp_obs* obs, const pp_obs* const* eprimes, const double* lambda, int n_maps, int order) {
  if (!obs || !eprimes || !lambda) { g_last_error = "NULL argument"; return PP_ERR_INVALID; }
  if (n_maps < 1) { g_last_error = "n_maps must be >= 1"; return PP_ERR_INVALID; }
  if (order != 1 && order != 2) { g_last_error = "order must be 1 or 2"; return PP_ERR_INVALID; }
  if (obs->broken) { g_last_error = "observable is unusable after an earlier device error"; return PP_ERR_INVALID; }
  if (obs->mode != PP_MODE_GREEDY) { g_last_error = "antinoise needs PP_MODE_GREEDY observables"; return PP_ERR_UNSUPPORTED; }
  std::vector<const EngineBase*> es;
  std::vector<double> q((size_t)n_maps);
  for (int c = 0; c < n_maps; ++c) {
    const pp_obs* e = eprimes[c];
    if (!e) { g_last_error = "NULL E'"; return PP_ERR_INVALID; }
    if (e->broken) { g_last_error = "E' is unusable after an earlier device error"; return PP_ERR_INVALID; }
    if (e->ctx != obs->ctx || e->n_qubits != obs->n_qubits || e->prec != obs->prec) {
      g_last_error = "every E' must share O's context, qubit count and precision";
      return PP_ERR_INVALID;
    }
    if (e->mode != PP_MODE_GREEDY) { g_last_error = "antinoise needs PP_MODE_GREEDY observables"; return PP_ERR_UNSUPPORTED; }
    if (!std::isfinite(lambda[c]) || lambda[c] < 0.0 || lambda[c] > 300.0) { g_last_error = "lambda must be finite, >= 0 and <= 300"; return PP_ERR_INVALID; }
    q[c] = inverse_quasi_probability(lambda[c]);
    es.push_back(e->eng.get());
  }
  const pp_status s = guarded([&] {
    HIPCHK(hipSetDevice(obs->ctx->device));
    obs->eng->antinoise_batch(es, q.data(), order);
  });
  if (s == PP_ERR_DEVICE || s == PP_ERR_OOM) obs->broken = true;
  return s;
}

pp_status pp_apply_antinoise_topk(pp_obs* obs, const pp_obs* eprime, double lambda, int64_t max_products) {
  if (!obs || !eprime) { g_last_error = "NULL argument"; return PP_ERR_INVALID; }
  if (obs->broken || eprime->broken) { g_last_error = "observable is unusable after an earlier device error"; return PP_ERR_INVALID; }
  if (obs->ctx != eprime->ctx) { g_last_error = "O and E' belong to different contexts"; return PP_ERR_INVALID; }
  if (obs->n_qubits != eprime->n_qubits) { g_last_error = "O and E' have different qubit counts"; return PP_ERR_INVALID; }
  if (obs->prec != eprime->prec) { g_last_error = "O and E' have different precisions"; return PP_ERR_INVALID; }
  if (obs->mode != PP_MODE_GREEDY || eprime->mode != PP_MODE_GREEDY) { g_last_error = "antinoise needs PP_MODE_GREEDY observables"; return PP_ERR_UNSUPPORTED; }
  if (!std::isfinite(lambda) || lambda < 0.0 || lambda > 300.0) { g_last_error = "lambda must be finite, >= 0 and <= 300"; return PP_ERR_INVALID; }
  const double q = inverse_quasi_probability(lambda);
  const pp_status s = guarded([&] {
    HIPCHK(hipSetDevice(obs->ctx->device));
    obs->eng->antinoise_topk(eprime->eng.get(), q, max_products);
  });
  if (s == PP_ERR_DEVICE || s == PP_ERR_OOM) obs->broken = true;
  return s;
}

pp_status pp_expectation(pp_obs* obs, const uint64_t* basis, double* out) {
  if (!obs || !out) { g_last_error = "NULL argument"; return PP_ERR_INVALID; }
  if (obs->broken) { g_last_error = "observable is unusable after an earlier device error"; return PP_ERR_INVALID; }
  if (basis && !strings_ok(obs->n_qubits, obs->W, 1, basis, basis)) { g_last_error = "basis bits above n_qubits"; return PP_ERR_INVALID; }
  const pp_status s = guarded([&] {
    HIPCHK(hipSetDevice(obs->ctx->device));
    *out = obs->eng->expectation(basis);
  });
  if (s == PP_ERR_DEVICE || s == PP_ERR_OOM) obs->broken = true;
  return s;
}

pp_status pp_expectation_noalloc(pp_obs* obs, const uint64_t* basis, double* out) {
  if (!obs || !out) { g_last_error = "NULL argument"; return PP_ERR_INVALID; }
  if (obs->broken) { g_last_error = "observable is unusable after an earlier device error"; return PP_ERR_INVALID; }
  if (basis && !strings_ok(obs->n_qubits, obs->W, 1, basis, basis)) { g_last_error = "basis bits above n_qubits"; return PP_ERR_INVALID; }
  double* scr = scratch_of(obs->ctx->device);
  if (!scr) { g_last_error = "no scratch address recorded for this device"; return PP_ERR_DEVICE; }
  const pp_status s = guarded([&] {
    HIPCHK(hipSetDevice(obs->ctx->device));
    *out = obs->eng->expectation_noalloc(basis, scr);
  });
  if (s == PP_ERR_DEVICE || s == PP_ERR_OOM) obs->broken = true;
  return s;
}

pp_status pp_size(pp_obs* obs, int64_t* out) {
  if (!obs || !out) { g_last_error = "NULL argument"; return PP_ERR_INVALID; }
  *out = (int64_t)obs->eng->size();
  return PP_OK;
}

pp_status pp_export(pp_obs* obs, uint64_t* x, uint64_t* z, double* c, uint8_t* ord) {
  if (!obs) { g_last_error = "NULL argument"; return PP_ERR_INVALID; }
  if (obs->broken) { g_last_error = "observable is unusable after an earlier device error"; return PP_ERR_INVALID; }
  const pp_status s = guarded([&] {
    HIPCHK(hipSetDevice(obs->ctx->device));
    obs->eng->export_terms(x, z, c, ord);
  });
  if (s == PP_ERR_DEVICE || s == PP_ERR_OOM) obs->broken = true;
  return s;
}

void pp_destroy(pp_obs* obs) {
  if (!obs) return;
  (void)hipSetDevice(obs->ctx->device);
  (void)hipStreamSynchronize(obs->ctx->stream);
  delete obs;
}

pp_status pp_timing_enable(pp_ctx* ctx, int enable) {
  if (!ctx) { g_last_error = "NULL argument"; return PP_ERR_INVALID; }
  return guarded([&] {
    ctx->collect();
    ctx->timing = enable != 0;
  });
}

int pp_timing_read(pp_ctx* ctx, pp_kernel_stat* out, int cap, int reset) {
  if (!ctx) return -1;
  int n = 0;
  const pp_status s = guarded([&] {
    ctx->collect();
    for (auto& kv : ctx->acc) {
      if (out && n < cap) {
        pp_kernel_stat& k = out[n];
        std::memset(&k, 0, sizeof k);
        std::snprintf(k.name, sizeof k.name, "%s", kv.first.c_str());
        k.launches = kv.second.launches;
        k.total_ms = kv.second.ms;
        k.algo_bytes = kv.second.bytes;
        k.items = kv.second.items;
        k.layer_bytes = kv.second.layer_bytes;
      }
      ++n;
    }
    if (reset) ctx->acc.clear();
  });
  return s == PP_OK ? n : -1;
}

pp_status pp_last_layer_stats(pp_obs* obs, pp_layer_stats* out) {
  if (!obs || !out) { g_last_error = "NULL argument"; return PP_ERR_INVALID; }
  *out = obs->last;
  return PP_OK;
}

}  // extern "C"
