// Host orchestration and C ABI of libpbpqlp.so (declared in include/pbpqlp.h).
//
// One call enqueues the whole method on the caller's stream with no host
// synchronization:  sketch -> (orth, A^T pass, orth, A pass) x q -> orth ->
// projection B^T = A^T Q -> QR of B^T -> QR of R^T -> Q Qt, following
// Algorithm 1 of the paper applied to A^T.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <climits>
#include <cmath>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/pbpqlp.h"
#include "common.h"
#include "kernels.h"
#include "launch.h"
#include "tune.h"

using namespace pbq;

namespace pbq {
Recorder*& current_recorder() {
  static thread_local Recorder* r = nullptr;
  return r;
}
}  // namespace pbq

namespace {

inline int64_t rup(int64_t x, int64_t a) { return (x + a - 1) / a * a; }

// Bump allocator over one workspace block; with base == nullptr it only sizes.
struct Bump {
  char* base = nullptr;
  size_t off = 0;
  void* take(size_t bytes) {
    off = (size_t)rup((int64_t)off, 256);
    void* p = base ? base + off : nullptr;
    off += bytes;
    return p;
  }
};

#define PBQ_CHECK(expr)                       \
  do {                                        \
    hipError_t e_ = (expr);                   \
    if (e_ != hipSuccess) return PBPQLP_EHIP; \
  } while (0)

int resolve_mode(pbpqlp_dtype dt, int prec, bool* ok) {
  *ok = true;
  if (dt == PBPQLP_F64) {
    if (prec != PBPQLP_PREC_NATIVE) *ok = false;
    return M_F64;
  }
  switch (prec) {
    case PBPQLP_PREC_NATIVE: return M_F32;
    case PBPQLP_PREC_BF16: return M_BF16;
    case PBPQLP_PREC_FP16: return M_F16;
    case PBPQLP_PREC_BF16X3: return M_BF16X3;
  }
  *ok = false;
  return M_F32;
}

// Relative pivot threshold below which a Cholesky column counts as
// dependent: the larger of (32 u_data)^2 (a residual below 32 rounding units
// of the data is noise) and max(16 l, 4 len) u_64, the noise level of a
// pivot computed from an FP64 Gram: each Gram entry sums len products, and
// the pivot of an exactly dependent column carries that rounding (up to
// about 2 len u_64 relative to its diagonal, depending on the summation order).
double dep_eps(bool f64, int l, int64_t len) {
  const double u64 = 1.1102230246251565e-16, u32 = 5.9604644775390625e-08;
  const double ud = f64 ? u64 : u32;
  const double n = 16.0 * l > 4.0 * (double)len ? 16.0 * l : 4.0 * (double)len;
  const double a = (32.0 * ud) * (32.0 * ud), b = n * u64;
  return a > b ? a : b;
}

// Widest sketch of the single-problem path (the blocked l x l stages); the
// batched path stays at 256.
constexpr int kMaxWideL = 16384;

struct Split {
  int S;
  int64_t chunk;
};

// Cost terms of one streaming pass, for plan_split.
struct PassCost {
  double a_bytes = 0, flops = 0, out_bytes = 0, peak = 1;
  bool k1_even = false;   // K1 in a 16-bit mode: evens a ragged last round out without a split
};

// Contraction split of one streaming pass over `blocks` A-side workgroups
// (one eight-wave block per CU at a time).  Among the splits that keep at
// least 4 stages of 64 per split (and 64 at most), the one of least estimated
// time: the pass's work (its A bytes over the HBM rate the kernels reach, or
// its flops over the matrix-core peak, whichever bounds it) spread over the
// ceil(T / CUs) rounds of T = blocks S workgroups, a partly busy round
// running at the rate its CUs reach (HBM-bound passes saturate at ~90% of
// the CUs, matrix-core bound ones scale with them), plus the S partial
// results written and read back by the reduction and its launch.
Split plan_split(int64_t blocks, int64_t klen, int forced, const PassCost& pc = PassCost()) {
  const int64_t maxS = std::min<int64_t>(64, std::max<int64_t>(1, klen / 256));
  int64_t S = 1;
  if (forced > 0) {
    S = std::min<int64_t>(forced, maxS);
  } else {
    constexpr double kBw = 6.2e12;
    const double cus = (double)device_cus();
    const double tm = pc.a_bytes / kBw, tc = pc.flops / pc.peak;
    const bool mem = tm >= tc;
    const double base = mem ? tm : tc;
    auto rate = [&](double nb) { return std::min(1.0, mem ? nb / (0.9 * cus) : nb / cus); };
    double best = 0.0;
    for (int64_t s = 1; s <= maxS; ++s) {
      const double T = (double)blocks * (double)s;
      double t;
      if (s == 1 && pc.k1_even && T > cus) {
        t = base;
      } else {
        const double full = std::floor(T / cus), rest = T - full * cus;
        t = full * (cus / T) * base / rate(cus) + (rest > 0 ? (rest / T) * base / rate(rest) : 0.0);
      }
      if (s > 1) t += 2.0 * (double)s * pc.out_bytes / kBw + 4e-6;
      if (s == 1 || t < best) {
        best = t;
        S = s;
      }
    }
  }
  int64_t chunk = rup((klen + S - 1) / S, 64);
  S = (klen + chunk - 1) / chunk;
  if (S < 1) S = 1;
  return {(int)S, chunk};
}

// ---------------------------------------------------------------------------
// Optional event tracing of hot-path kernels (pbpqlp_trace_*).
// ---------------------------------------------------------------------------
struct TraceRec {
  std::string name;
  double bytes = 0, flops = 0;
  hipEvent_t a = nullptr, b = nullptr;
};
std::mutex g_trace_mu;
std::vector<TraceRec> g_trace;
size_t g_trace_n = 0;
int g_trace_level = 0;  // 0 off, 1 streaming products, 2 all hot-path kernels

// Set while an allocation-free call runs on this thread: no trace events are
// created then (creating them is the one allocation tracing would make).
thread_local bool t_no_trace = false;

struct TraceScope {
  TraceRec* rec = nullptr;
  hipStream_t st;
  TraceScope(const char* name, double bytes, double flops, hipStream_t s, int level = 2) : st(s) {
    if (g_trace_level < level || pbq::current_recorder() || t_no_trace) return;
    std::lock_guard<std::mutex> lk(g_trace_mu);
    if (g_trace_n == g_trace.size()) {
      TraceRec r;
      if (hipEventCreate(&r.a) != hipSuccess || hipEventCreate(&r.b) != hipSuccess) return;
      g_trace.push_back(r);
    }
    rec = &g_trace[g_trace_n++];
    rec->name = name;
    rec->bytes = bytes;
    rec->flops = flops;
    (void)hipEventRecord(rec->a, st);
  }
  ~TraceScope() {
    if (rec) (void)hipEventRecord(rec->b, st);
  }
};

const char* mode_name(int mode) {
  switch (mode) {
    case M_F64: return "f64";
    case M_F32: return "f32";
    case M_BF16: return "bf16";
    case M_F16: return "fp16";
    case M_BF16X3: return "bf16x3";
  }
  return "?";
}

// Power-of-two lift of an FP16 operand: unit-norm columns have entries of
// about len^-1/2, lifted to about 1 (exact, undone on the product).
float fp16_lift(bool unit_columns, int64_t xlen) {
  return unit_columns ? std::ldexp(1.0f, (int)std::floor(0.5 * std::log2((double)xlen))) : 1.0f;
}

// Everything one factorization needs, carved from one workspace block.
struct Ctx {
  // problem: A is m x n (lda) as stored.  The method runs on M = A, or on
  // M = A^T when tv (the paper's own orientation): M's rows and columns are
  // mM x nM, and a product with M or M^T is a pass with A or A^T.
  int64_t m = 0, n = 0, lda = 0;
  bool tv = false;
  int l = 0, lp = 0, lp32 = 0, q = 0;
  bool f64 = false;
  size_t el = 4;           // bytes of one data element
  int64_t ldm = 0, ldn = 0, ldS = 0;
  int mode_sketch = 0, mode_power = 0, mode_proj = 0;
  float fp16_scale = 1.0f;
  int forced_split = 0;
  int gram_target = 256;   // Gram workgroups to aim at (fewer per problem in a batch)
  uint64_t seed = 0;
  const void* omega_in = nullptr;  // caller's sketch matrix (row-major n x l), or generated
  int64_t ldo_in = 0;
  // splits: the sketch pass's grid sizes the ||A||_F^2 partials
  int k1_blocks = 0, k1_splits = 1;
  size_t part_bytes = 0;
  // buffers
  void *Om = nullptr, *Y = nullptr, *Qm = nullptr, *W1m = nullptr, *Zn = nullptr, *Pn = nullptr,
       *W1n = nullptr;
  void *Xhi = nullptr, *Xlo = nullptr, *part = nullptr;
  double *normA = nullptr, *gpart = nullptr, *G = nullptr, *R1 = nullptr, *R2 = nullptr,
         *Rfin = nullptr, *M1 = nullptr, *Qt64 = nullptr, *U = nullptr;
  void *Ra = nullptr, *Dinv = nullptr, *Ra64 = nullptr, *Dinv64 = nullptr, *Qt32 = nullptr;
  int* dep = nullptr;
  int* ident = nullptr;   // a later sweep's factor was the identity (device flag)
  int* far = nullptr;     // the Gram reduction's identity-test flags (lp x gram_far_cols)
  // which operand the 16-bit buffers Xhi/Xlo hold (written by a conversion, or
  // by the last apply of an orth() for the pass that follows it)
  const void* conv_X = nullptr;
  int conv_mode = 0;
  float conv_xs = 1.0f;
  double* rowsq = nullptr;
  uint64_t ncall = 0;
  // optional outputs: R of the projection's QR (row-major, ldr_out) and the
  // numerical rank estimated from the L-values
  double* r_out = nullptr;
  int64_t ldr_out = 0;
  double rank_tol = 0.0;
  int* rank_out = nullptr;
  // host-resident A (Section IV-E, A stored externally): every pass streams
  // row panels of panel_rows rows through two device staging buffers
  const char* A_host = nullptr;
  int64_t panel_rows = 0;
  int npanels = 0;
  void* stage[2] = {nullptr, nullptr};
  hipStream_t cs = nullptr;            // copy stream
  hipEvent_t ev_copied[2] = {nullptr, nullptr}, ev_used[2] = {nullptr, nullptr};
  int panel_seq = 0;                   // panels streamed so far (buffer = panel_seq & 1)
  // pageable A: rows go through two pinned bounce buffers first (a host copy,
  // then an asynchronous copy that keeps the copy stream's order)
  bool bounce = false;
  void* bounce_buf[2] = {nullptr, nullptr};
  hipEvent_t ev_bounce[2] = {nullptr, nullptr};
  // sparse A in CSR (Section IV-E): both products are row-gather products
  bool sparse = false;
  const int64_t* rowptr = nullptr;
  const int32_t* colind = nullptr;
  const void* vals = nullptr;
  int64_t nnz = 0;
  int nsq = 1;            // ||A||_F^2 partials
  int64_t* ptr_t = nullptr;
  int32_t* idx_t = nullptr;
  void* vals_t = nullptr;
  void* tscratch = nullptr;  // the stable sort of the transpose
  void* Xrm = nullptr;    // row-major copy of the l-column operand (lp32 wide)
  void* Yrm = nullptr;    // row-major product of one 256-column slice
  void* spart = nullptr;  // partial rows of the nonzero-balanced product
  int ldyr() const { return lp32 < kMaxL ? lp32 : kMaxL; }
  // sketches wider than 256 columns: the l x l stages are blocked by 256
  bool wide = false;
  double* gdiag = nullptr;             // the Gram's diagonal before the blocked updates
  int nbw() const { return (lp + kMaxL - 1) / kMaxL; }
  // apply forms, diagonal-block inverses and dependence flags of block J
  void* ra_blk(bool f64, int J) const {
    return (char*)(f64 ? Ra64 : Ra) + (size_t)J * kMaxL * kMaxL * (f64 ? 8 : el);
  }
  void* dinv_blk(bool f64, int J) const {
    return (char*)(f64 ? Dinv64 : Dinv) + (size_t)J * (kMaxL / 16) * 256 * (f64 ? 8 : el);
  }
  int* dep_blk(int J) const { return dep + (size_t)J * (kMaxL + 16); }

  int64_t mM() const { return tv ? n : m; }
  int64_t nM() const { return tv ? m : n; }
  int64_t ldmM() const { return tv ? ldn : ldm; }
  int64_t ldnM() const { return tv ? ldm : ldn; }
  // Split plan of a pass in compute mode `mode` (grid blocks depend on it).
  Split split_for(int mode, bool trans) const {
    const int64_t rb = stream_span(mode, trans);
    const int64_t mr = panel_rows > 0 ? panel_rows : m;   // rows one launch sees
    const int64_t len = trans ? n : mr, klen = trans ? mr : n;
    // one launch covers at most kMaxL columns of the operand
    const double w = (double)std::min(lp, kMaxL);
    PassCost pc;
    pc.a_bytes = (double)len * (double)klen * el;
    pc.flops = 2.0 * (double)len * (double)klen * w * (mode == M_BF16X3 ? 3.0 : 1.0);
    pc.out_bytes = (double)len * w * el;
    pc.peak = mode == M_F64 ? 78.6e12 : mode == M_F32 ? 157.3e12 : 2.5e15;
    pc.k1_even = !trans && (mode == M_BF16 || mode == M_F16);
    Split sp = plan_split((len + rb - 1) / rb, klen, forced_split, pc);
    // the A^T X panels of a host-resident A keep every split partial until the
    // last panel: at most 64 partials in all
    if (panel_rows > 0 && trans && (int64_t)sp.S * npanels > 64) {
      const int S = (int)(64 / npanels) > 0 ? (int)(64 / npanels) : 1;
      sp = plan_split((len + rb - 1) / rb, klen, S, pc);
    }
    return sp;
  }
  // Partials one pass keeps: split partials of one launch, or, for A^T X over
  // host panels, those of every panel.
  int64_t partial_slots(int mode, bool trans) const {
    const Split sp = split_for(mode, trans);
    if (panel_rows > 0 && trans) return (int64_t)sp.S * npanels;
    return sp.S > 1 ? sp.S : 0;
  }
  // Sizes of the split partials and the ||A||^2 partials for the passes this
  // context will run: the sketch M X, the power passes (both directions) and
  // the projection M^T X.  ||A||_F^2 is accumulated on the one of the sketch
  // and the projection that is a product A X: the sketch for M = A, the
  // projection for M = A^T.
  void plan_buffers(bool sketch, bool power, bool proj) {
    part_bytes = 0;
    if (sparse) {
      k1_blocks = nsq;
      k1_splits = 1;
      return;
    }
    auto need = [&](int mode, bool trans) {
      const size_t b = (size_t)partial_slots(mode, trans) * lp * (trans ? ldn : ldm) * el;
      if (b > part_bytes) part_bytes = b;
    };
    if (sketch) need(mode_sketch, tv);
    if (power) {
      need(mode_power, false);
      need(mode_power, true);
    }
    if (proj) need(mode_proj, !tv);
    const int nmode = tv ? mode_proj : mode_sketch;
    k1_splits = split_for(nmode, false).S;
    if (panel_rows > 0) {
      // every panel but the last holds panel_rows rows
      k1_blocks = (int)(stream_k1_grid(nmode, panel_rows, k1_splits) * (npanels - 1) +
                        stream_k1_grid(nmode, m - panel_rows * (npanels - 1), k1_splits));
    } else {
      k1_blocks = (int)stream_k1_grid(nmode, m, k1_splits);
    }
  }

  void carve(Bump& b, bool need16) {
    const int64_t ldmax = ldm > ldn ? ldm : ldn;
    Om = b.take((size_t)lp32 * ldnM() * el);
    Y = b.take((size_t)lp32 * ldmM() * el);
    Qm = b.take((size_t)lp32 * ldmM() * el);
    W1m = b.take((size_t)lp32 * ldmM() * el);
    Zn = b.take((size_t)lp32 * ldnM() * el);
    Pn = b.take((size_t)lp32 * ldnM() * el);
    W1n = b.take((size_t)lp32 * ldnM() * el);
    if (need16) {
      Xhi = b.take((size_t)lp32 * ldmax * 2);
      Xlo = b.take((size_t)lp32 * ldmax * 2);
    }
    part = b.take(part_bytes);
    normA = (double*)b.take((size_t)k1_blocks * k1_splits * sizeof(double));
    size_t gp = gram_partial_elems(m, lp, gram_target);
    const size_t gpn = gram_partial_elems(n, lp, gram_target),
                 gps = gram_partial_elems(l, lp, gram_target);
    if (gpn > gp) gp = gpn;
    if (gps > gp) gp = gps;
    gpart = (double*)b.take(gp * sizeof(double));
    G = (double*)b.take((size_t)lp * lp * 8);
    R1 = (double*)b.take((size_t)lp * lp * 8);
    R2 = (double*)b.take((size_t)lp * lp * 8);
    U = (double*)b.take((size_t)lp * lp * 8);
    Rfin = (double*)b.take((size_t)lp32 * ldS * 8);
    M1 = (double*)b.take((size_t)lp32 * ldS * 8);
    Qt64 = (double*)b.take((size_t)lp32 * ldS * 8);
    Qt32 = b.take((size_t)lp32 * ldS * 4);
    // wide sketches keep one 256 x 256 apply form per diagonal block
    const size_t nra = wide ? (size_t)nbw() * kMaxL * kMaxL : (size_t)lp * lp;
    const size_t ndv = wide ? (size_t)nbw() * (kMaxL / 16) * 256 : (size_t)(lp / 16) * 256;
    const size_t ndep = wide ? (size_t)nbw() * (kMaxL + 16) : (size_t)lp + 1;
    Ra = b.take(nra * el);
    Dinv = b.take(ndv * el);
    Ra64 = b.take(nra * 8);
    Dinv64 = b.take(ndv * 8);
    dep = (int*)b.take(ndep * sizeof(int));
    rowsq = (double*)b.take((size_t)lp * sizeof(double));
    ident = (int*)b.take(sizeof(int));
    far = (int*)b.take((size_t)lp * gram_far_cols(lp) * sizeof(int));
    gdiag = wide ? (double*)b.take((size_t)lp * sizeof(double)) : nullptr;
    if (panel_rows > 0) {
      stage[0] = b.take((size_t)panel_rows * lda * el);
      stage[1] = b.take((size_t)panel_rows * lda * el);
    }
    if (sparse) {
      ptr_t = (int64_t*)b.take((size_t)(n + 1) * sizeof(int64_t));
      idx_t = (int32_t*)b.take((size_t)nnz * sizeof(int32_t));
      vals_t = b.take((size_t)nnz * el);
      tscratch = b.take(csr_transpose_scratch_bytes(nnz, n));
      Xrm = b.take((size_t)(m > n ? m : n) * lp32 * el);
      Yrm = b.take((size_t)(m > n ? m : n) * ldyr() * el);
      spart = b.take((size_t)spmm_part_rows(nnz) * ldyr() * el);
    }
  }
};

// Every matrix must be aligned to its element type.
bool aligned(const void* p, size_t el) { return ((uintptr_t)p % el) == 0; }

bool valid_args(int64_t m, int64_t n, int k, int p, int q) {
  if (m < 1 || n < 1 || k < 1 || p < 0 || q < 0 || q > 16) return false;
  const int64_t l = (int64_t)k + p;
  return l <= m && l <= n;
}

pbpqlp_status setup(Ctx& c, int64_t m, int64_t n, int64_t lda, pbpqlp_dtype dt, int k, int p,
                    int q, const pbpqlp_opts* opts, bool batched = false, bool tv = false) {
  if (dt != PBPQLP_F64 && dt != PBPQLP_F32) return PBPQLP_EINVAL;
  if (!valid_args(m, n, k, p, q) || lda < n) return PBPQLP_EINVAL;
  const int l = k + p;
  if (l > (batched ? kMaxL : kMaxWideL)) return PBPQLP_EUNSUPPORTED;
  pbpqlp_opts o;
  pbpqlp_default_opts(&o);
  if (opts) o = *opts;
  c.m = m; c.n = n; c.lda = lda; c.q = q; c.tv = tv;
  c.l = l; c.lp = (int)rup(l, 16); c.lp32 = (int)rup(l, 32);
  c.wide = c.lp > kMaxL;
  c.f64 = dt == PBPQLP_F64;
  c.el = c.f64 ? 8 : 4;
  c.ldm = rup(m, 64); c.ldn = rup(n, 64); c.ldS = rup(c.lp, 64);
  bool ok1, ok2, ok3;
  c.mode_sketch = resolve_mode(dt, o.sketch_prec, &ok1);
  c.mode_power = resolve_mode(dt, o.power_prec, &ok2);
  c.mode_proj = resolve_mode(dt, o.proj_prec, &ok3);
  if (!ok1 || !ok2 || !ok3) return c.f64 ? PBPQLP_EUNSUPPORTED : PBPQLP_EINVAL;
  c.fp16_scale = (float)(o.fp16_scale_a > 0 ? o.fp16_scale_a : 1.0);
  if (o.split_k < -1 || o.gram_workgroups < 0) return PBPQLP_EINVAL;
  int split = o.split_k, gram = o.gram_workgroups;
  if (!batched && (split == 0 || gram == 0)) {
    TunePlan t;
    if (tune_lookup(tune_key((int)dt, o.sketch_prec, o.power_prec, o.proj_prec, l, m, n, false), &t)) {
      if (split == 0) split = t.split_k;
      if (gram == 0) gram = t.gram_wg;
    }
  }
  c.forced_split = split > 0 ? split : 0;
  if (gram > 0) c.gram_target = gram;
  c.plan_buffers(true, q > 0, true);
  return PBPQLP_OK;
}

bool needs16(const Ctx& c) {
  return c.mode_sketch >= M_BF16 || c.mode_power >= M_BF16 || c.mode_proj >= M_BF16;
}

// The launch of a product over columns [j0, j0 + 256) of X and of the result
// (the whole product when l <= 256).
StreamArgs slice_args(const Ctx& c, const StreamArgs& a, int mode, int j0) {
  StreamArgs s = a;
  const int w32 = c.lp32 - j0 < kMaxL ? c.lp32 - j0 : kMaxL;
  s.lp32 = w32;
  s.lp = c.lp - j0 < w32 ? c.lp - j0 : w32;
  const size_t xel = mode >= M_BF16 ? 2 : c.el;
  s.X = (const char*)a.X + (size_t)j0 * a.ldx * xel;
  if (a.Xlo) s.Xlo = (const char*)a.Xlo + (size_t)j0 * a.ldx * xel;
  return s;
}

// One pass over a host-resident A (Section IV-E: with A stored externally each
// product with A or A^T is one more pass over it).  Row panels of panel_rows
// rows are copied on the copy stream into two device staging buffers in turn;
// the compute stream waits for each copy, and a copy into a buffer waits until
// the kernel that read the buffer's previous panel is done.  A X: each panel
// gives its rows of the result (through its own split partials when the
// contraction is split).  A^T X: each panel's split partials stay in their
// own slots and one reduction in a fixed order sums all of them at the end.
pbpqlp_status host_pass(Ctx& c, bool trans, int mode, StreamArgs a, int64_t xlen, void* out,
                        int64_t ldo, double* normA, hipStream_t st) {
  const Split sp = c.split_for(mode, trans);
  const int64_t rb = stream_span(mode, trans);
  const int64_t olen = trans ? c.n : c.m;
  const double xb = (mode >= M_BF16) ? 2.0 : (double)c.el;
  int64_t slot = 0;
  int64_t nblk = 0;   // row blocks of the panels done so far (||A||^2 partial offset)
  for (int pi = 0; pi < c.npanels; ++pi) {
    const int64_t r0 = (int64_t)pi * c.panel_rows;
    const int64_t rows = std::min(c.panel_rows, c.m - r0);
    const int b = c.panel_seq++ & 1;
    // the copy waits for the last kernel that read this buffer
    PBQ_CHECK(hipStreamWaitEvent(c.cs, c.ev_used[b], 0));
    if (c.bounce) {
      // the bounce buffer is free once its previous copy to the device is done
      PBQ_CHECK(hipEventSynchronize(c.ev_bounce[b]));
      const size_t rb_bytes = (size_t)c.n * c.el;
      for (int64_t i = 0; i < rows; ++i)
        std::memcpy((char*)c.bounce_buf[b] + (size_t)i * rb_bytes,
                    c.A_host + (size_t)(r0 + i) * c.lda * c.el, rb_bytes);
      PBQ_CHECK(hipMemcpy2DAsync(c.stage[b], (size_t)c.lda * c.el, c.bounce_buf[b], rb_bytes, rb_bytes,
                                 (size_t)rows, hipMemcpyHostToDevice, c.cs));
      PBQ_CHECK(hipEventRecord(c.ev_bounce[b], c.cs));
    } else {
      PBQ_CHECK(hipMemcpy2DAsync(c.stage[b], (size_t)c.lda * c.el, c.A_host + (size_t)r0 * c.lda * c.el,
                                 (size_t)c.lda * c.el, (size_t)c.n * c.el, (size_t)rows,
                                 hipMemcpyHostToDevice, c.cs));
    }
    PBQ_CHECK(hipEventRecord(c.ev_copied[b], c.cs));
    PBQ_CHECK(hipStreamWaitEvent(st, c.ev_copied[b], 0));
    // the same split count for every panel (the last may be shorter)
    const Split ps = plan_split(trans ? (c.n + rb - 1) / rb : (rows + rb - 1) / rb, trans ? rows : c.n, sp.S);
    for (int j0 = 0; j0 < c.lp32; j0 += kMaxL) {
      StreamArgs pa = slice_args(c, a, mode, j0);
      pa.A = c.stage[b];
      pa.m = rows;
      if (trans) {
        // A^T X contracts over the panel's rows: the matching rows of X
        const size_t xel = mode >= M_BF16 ? 2 : c.el;
        pa.X = (const char*)pa.X + (size_t)r0 * xel;
        if (pa.Xlo) pa.Xlo = (const char*)pa.Xlo + (size_t)r0 * xel;
      }
      pa.splits = ps.S;
      pa.chunk = ps.chunk;
      pa.normA = (normA && j0 == 0) ? normA + nblk * ps.S : nullptr;
      pa.ldo = ldo;
      const size_t jo = (size_t)j0 * ldo * c.el;
      if (trans) {
        pa.out = (char*)c.part + (size_t)slot * c.lp * ldo * c.el + jo;
        pa.split_stride = (int64_t)c.lp * ldo;
      } else if (ps.S == 1) {
        pa.out = (char*)out + (size_t)r0 * c.el + jo;
        pa.split_stride = 0;
      } else {
        pa.out = (char*)c.part + jo;
        pa.split_stride = (int64_t)c.lp * ldo;
      }
      const int w = pa.lp < c.l - j0 ? pa.lp : c.l - j0;
      {
        const double bytes = (double)rows * c.n * c.el + (double)(trans ? rows : xlen) * w * xb *
                             (mode == M_BF16X3 ? 2 : 1) + (double)(trans ? c.n : rows) * w * c.el;
        std::string nm = std::string(trans ? "k2_" : "k1_") + mode_name(mode) + "_panel";
        TraceScope ts(nm.c_str(), bytes, 2.0 * rows * c.n * w, st, 1);
        PBQ_CHECK(launch_stream(trans, mode, pa, st));
      }
      if (!trans && ps.S > 1) {
        TraceScope ts("splitk_reduce", (double)(ps.S + 1) * rows * w * c.el, 0.0, st);
        // only this panel's rows (the last panel also zeroes the padding rows)
        const int64_t wl = pi == c.npanels - 1 ? ldo - r0 : rows;
        PBQ_CHECK(launch_splitk_reduce(c.f64, (char*)c.part + jo, pa.split_stride, ps.S, ldo, pa.lp, rows,
                                       (char*)out + (size_t)r0 * c.el + jo, ldo, st, wl));
      }
    }
    if (trans) slot += ps.S;
    PBQ_CHECK(hipEventRecord(c.ev_used[b], st));
    nblk += stream_k1_grid(mode, rows, ps.S);
  }
  if (trans) {
    for (int j0 = 0; j0 < c.lp32; j0 += kMaxL) {
      const int wl = c.lp - j0 < kMaxL ? c.lp - j0 : kMaxL;
      const size_t jo = (size_t)j0 * ldo * c.el;
      TraceScope ts("splitk_reduce", (double)(slot + 1) * olen * wl * c.el, 0.0, st);
      PBQ_CHECK(launch_splitk_reduce(c.f64, (char*)c.part + jo, (int64_t)c.lp * ldo, (int)slot, ldo, wl, olen,
                                     (char*)out + jo, ldo, st));
    }
  }
  return PBPQLP_OK;
}

// One pass with a sparse A: the operand is copied row-major (its padding
// columns are 0 from the set-up), then out = A X with A's CSR or A^T X with
// the CSR of A^T, 256 columns per launch.
pbpqlp_status sparse_pass(Ctx& c, bool trans, const void* X, int64_t ldx, int64_t xlen, void* out,
                          int64_t ldo, hipStream_t st) {
  {
    TraceScope ts("sp_rowmajor", 2.0 * xlen * c.l * c.el, 0.0, st);
    PBQ_CHECK(launch_cm_to_rm(c.f64, X, ldx, xlen, c.l, c.Xrm, c.lp32, st));
  }
  const int64_t rows = trans ? c.n : c.m, cols = trans ? c.m : c.n;
  for (int j0 = 0; j0 < c.lp; j0 += kMaxL) {
    const int w = c.lp - j0 < kMaxL ? c.lp - j0 : kMaxL;
    const double bytes = (double)c.nnz * (c.el + 4) + (double)rows * 8 + (double)c.nnz * w * c.el +
                         (double)rows * w * c.el;
    TraceScope ts(trans ? "k2_spmm" : "k1_spmm", bytes, 2.0 * c.nnz * w, st, 1);
    void* oj = (char*)out + (size_t)j0 * ldo * c.el;
    if (trans)
      PBQ_CHECK(launch_spmm(c.f64, c.ptr_t, c.idx_t, c.vals_t, rows, cols, c.nnz, c.Xrm, c.lp32, j0, w, c.Yrm,
                            c.ldyr(), c.spart, oj, ldo, st));
    else
      PBQ_CHECK(launch_spmm(c.f64, c.rowptr, c.colind, c.vals, rows, cols, c.nnz, c.Xrm, c.lp32, j0, w, c.Yrm,
                            c.ldyr(), c.spart, oj, ldo, st));
  }
  return PBPQLP_OK;
}

// One A-streaming pass: out (column-major, ld) = A X (trans=0) or A^T X.
pbpqlp_status stream_pass(Ctx& c, bool trans, int mode, const void* A, const void* X,
                          int64_t ldx, int64_t xlen, bool unit_columns, void* out, int64_t ldo,
                          double* normA, hipStream_t st) {
  if (c.sparse) return sparse_pass(c, trans, X, ldx, xlen, out, ldo, st);
  StreamArgs a;
  a.A = A; a.lda = c.lda; a.m = c.m; a.n = c.n;
  a.lp = c.lp;
  a.lp32 = c.lp32;
  a.a_scale = 1.0f;
  a.out_scale = 1.0f;
  if (mode >= M_BF16) {
    float xs = 1.0f;
    if (mode == M_F16) {
      a.a_scale = c.fp16_scale;
      xs = fp16_lift(unit_columns, xlen);
      a.out_scale = 1.0f / (a.a_scale * xs);
    }
    // the 16-bit copy may already be there: the orth() that produced X wrote it
    if (!(c.conv_X == X && c.conv_mode == mode && c.conv_xs == xs)) {
      TraceScope ts("convert", (double)xlen * c.l * (4.0 + (mode == M_BF16X3 ? 4.0 : 2.0)), 0.0, st);
      PBQ_CHECK(launch_convert(mode, (const float*)X, ldx, xlen, c.l, c.lp32, xs, c.Xhi, c.Xlo, st));
      c.conv_X = X;
      c.conv_mode = mode;
      c.conv_xs = xs;
    }
    a.X = c.Xhi;
    a.Xlo = c.Xlo;
  } else {
    a.X = X;
    a.Xlo = nullptr;
  }
  a.ldx = ldx;
  if (c.A_host) return host_pass(c, trans, mode, a, xlen, out, ldo, normA, st);
  const Split sp = c.split_for(mode, trans);
  const int64_t olen = trans ? c.n : c.m;
  const double xb = (mode >= M_BF16) ? 2.0 : (double)c.el;
  // at most 256 columns of X per launch: wider sketches take several launches
  for (int j0 = 0; j0 < c.lp32; j0 += kMaxL) {
    StreamArgs sa = slice_args(c, a, mode, j0);
    sa.splits = sp.S;
    sa.chunk = sp.chunk;
    sa.normA = j0 == 0 ? normA : nullptr;
    sa.ldo = ldo;
    char* outj = (char*)out + (size_t)j0 * ldo * c.el;
    char* partj = (char*)c.part + (size_t)j0 * ldo * c.el;
    if (sp.S == 1) {
      sa.out = outj;
      sa.split_stride = 0;
    } else {
      sa.out = partj;
      sa.split_stride = (int64_t)c.lp * ldo;
    }
    const int w = sa.lp < c.l - j0 ? sa.lp : c.l - j0;
    {
      const double bytes = (double)c.m * c.n * c.el + (double)xlen * w * xb * (mode == M_BF16X3 ? 2 : 1) +
                           (double)olen * w * c.el;
      std::string nm = std::string(trans ? "k2_" : "k1_") + mode_name(mode);
      TraceScope ts(nm.c_str(), bytes, 2.0 * c.m * c.n * w, st, 1);
      PBQ_CHECK(launch_stream(trans, mode, sa, st));
    }
    if (sp.S > 1) {
      TraceScope ts("splitk_reduce", (double)(sp.S + 1) * olen * w * c.el, 0.0, st);
      PBQ_CHECK(launch_splitk_reduce(c.f64, partj, sa.split_stride, sp.S, ldo, sa.lp, olen, outj, ldo, st));
    }
  }
  return PBPQLP_OK;
}

// Blocked upper Cholesky G = Rt^T Rt (lp x lp, FP64) for lp > 256, blocks of
// 256: each diagonal block (already updated by the earlier blocks) is
// factored by the single-workgroup Cholesky with the dependence test measured
// against the Gram's own diagonal; the block's row of Rt is the triangular
// solve R_J,K = R_JJ^-T G_J,K (the tall apply on the FP64 matrix cores, the
// rows of dependent columns set to 0), and the trailing upper triangle takes
// G_K,K' -= R_J,K^T R_J,K' on the FP64 matrix cores.  Outputs: Rt (lower part
// 0), and per diagonal block its apply form, inverses and dependence flags in
// the storage type of the tall matrix.
pbpqlp_status chol_wide(Ctx& c, bool f64, double eps, double* Rt, void* info, hipStream_t st) {
  const int lp = c.lp, l = c.l, nb = c.nbw();
  double* G = c.G;
  PBQ_CHECK(launch_save_diag(G, lp, l, lp, c.gdiag, st));
  PBQ_CHECK(launch_fill_zero(Rt, (size_t)lp * lp * sizeof(double), st));
  for (int J = 0; J < nb; ++J) {
    const int j0 = J * kMaxL;
    const int bJ = lp - j0 < kMaxL ? lp - j0 : kMaxL;
    const int lJ = l - j0 < bJ ? (l - j0 > 0 ? l - j0 : 0) : bJ;
    const int64_t rest = lp - (j0 + bJ);
    {
      TraceScope ts("chol", (double)bJ * bJ * 8 * 2, (double)bJ * bJ * bJ / 3.0, st);
      PBQ_CHECK(launch_chol(true, G + (size_t)j0 * lp + j0, lp, lJ, bJ, eps, Rt + (size_t)j0 * lp + j0, lp,
                            c.ra_blk(true, J), c.dinv_blk(true, J), c.dep_blk(J), info, st, c.gdiag + j0));
    }
    if (!f64) {
      PBQ_CHECK(launch_cast_f32((const double*)c.ra_blk(true, J), (float*)c.ra_blk(false, J), (int64_t)bJ * bJ, st));
      PBQ_CHECK(launch_cast_f32((const double*)c.dinv_blk(true, J), (float*)c.dinv_blk(false, J),
                                (int64_t)(bJ / 16) * 256, st));
    }
    if (rest <= 0) continue;
    const size_t off = (size_t)j0 * lp + j0 + bJ;
    {
      // R_J,K^T = G_K,J R_JJ^-1: column c of the tall operand is row j0 + c
      TraceScope ts("chol_panel", 2.0 * rest * bJ * 8, (double)rest * bJ * bJ, st);
      PBQ_CHECK(launch_apply(true, G + off, lp, rest, bJ, lJ, c.ra_blk(true, J), c.dinv_blk(true, J),
                             c.dep_blk(J), c.seed, Rt + off, lp, nullptr, 0, st, rest));
      PBQ_CHECK(launch_zero_dep_rows(Rt + off, lp, bJ, rest, c.dep_blk(J), st));
    }
    {
      const size_t t0 = (size_t)(j0 + bJ);
      TraceScope ts("chol_update", (double)rest * rest * 8 * 2, (double)rest * rest * bJ, st);
      PBQ_CHECK(launch_gemm(1, rest, rest, bJ, Rt + off, 1, lp, Rt + off, lp, 1, G + t0 * lp + t0,
                            G + t0 * lp + t0, lp, 1, -1.0, 1.0, true, st));
    }
  }
  return PBPQLP_OK;
}

// Q = Y Rt^-1 for lp > 256 by column blocks of 256: block J first takes
// Y_J - Q_<J Rt_<J,J (a matrix-core product), then the single-block apply
// with block J's apply form (dependent columns completed as in the narrow
// path).  dst may be written in place of the block being solved.
pbpqlp_status apply_wide(Ctx& c, bool f64, const void* src, int64_t ld, int64_t len, const double* Rt,
                         uint64_t cseed, void* dst, void* rm, int64_t ldrm, hipStream_t st,
                         const Emit16& em = Emit16()) {
  const int lp = c.lp, l = c.l, nb = c.nbw();
  const size_t el = f64 ? 8 : c.el;
  for (int J = 0; J < nb; ++J) {
    const int j0 = J * kMaxL;
    const int bJ = lp - j0 < kMaxL ? lp - j0 : kMaxL;
    const int lJ = l - j0 < bJ ? (l - j0 > 0 ? l - j0 : 0) : bJ;
    const void* srcJ = (const char*)src + (size_t)j0 * ld * el;
    void* dstJ = (char*)dst + (size_t)j0 * ld * el;
    if (J > 0) {
      TraceScope ts("apply_update", 2.0 * len * bJ * el, 2.0 * len * j0 * bJ, st);
      PBQ_CHECK(launch_gemm(f64 ? 1 : 3, len, bJ, j0, dst, 1, ld, Rt + j0, lp, 1, srcJ, dstJ, 1, ld, -1.0, 1.0,
                            false, st));
      srcJ = dstJ;
    }
    TraceScope ts("apply", 2.0 * len * bJ * el, (double)len * bJ * bJ, st);
    Emit16 ej = em;
    if (ej.mode) {
      ej.hi = (char*)em.hi + (size_t)j0 * ld * 2;
      ej.lo = (char*)em.lo + (size_t)j0 * ld * 2;
    }
    PBQ_CHECK(launch_apply(f64, srcJ, ld, len, bJ, lJ, c.ra_blk(f64, J), c.dinv_blk(f64, J), c.dep_blk(J),
                           cseed + (uint64_t)J, dstJ, ld, rm ? (char*)rm + (size_t)j0 * el : nullptr, ldrm, st,
                           -1, nullptr, ej));
  }
  return PBPQLP_OK;
}

pbpqlp_status orth_wide(Ctx& c, bool f64, const void* X, int64_t ld, int64_t len, int passes, void* out,
                        void* tmp, double* Rkeep, int64_t ldrk, void* rm, int64_t ldrm, void* info,
                        hipStream_t st, bool small, const Emit16& em) {
  const double eps = dep_eps(f64, c.l, len);
  const void* src = X;
  for (int ps = 0; ps < passes; ++ps) {
    const bool last = ps == passes - 1;
    void* dst = last ? out : tmp;
    double* Rt = ps == 0 ? c.R1 : c.R2;
    const uint64_t cseed = c.seed ^ (0x9E3779B97F4A7C15ull * (++c.ncall));
    const double el = f64 ? 8.0 : (double)c.el;
    {
      TraceScope ts(small ? "gram_ll" : "gram", (double)len * c.l * el, (double)len * c.l * c.l, st);
      PBQ_CHECK(launch_gram(f64, src, ld, len, c.lp, c.gpart, c.G, c.lp, c.gram_target, st));
    }
    pbpqlp_status s = chol_wide(c, f64, eps, Rt, info, st);
    if (s) return s;
    s = apply_wide(c, f64, src, ld, len, Rt, cseed, dst, last ? rm : nullptr, ldrm, st, last ? em : Emit16());
    if (s) return s;
    src = dst;
  }
  if (Rkeep) {
    TraceScope ts("r2r1", 3.0 * c.lp * c.lp * 8, 2.0 * c.lp * c.lp * c.lp, st);
    if (passes == 1)
      PBQ_CHECK(launch_copy_mat(c.R1, c.lp, c.lp, c.lp, Rkeep, ldrk, 1, st));
    else
      PBQ_CHECK(launch_gemm(1, c.lp, c.lp, c.lp, c.R2, c.lp, 1, c.R1, c.lp, 1, nullptr, Rkeep, ldrk, 1, 1.0, 0.0,
                            false, st));
  }
  return PBPQLP_OK;
}

// orth()/qr() of a column-major tall matrix X (lp32 x ld, len rows of the
// tall matrix) by `passes` CholeskyQR sweeps.  Result in `out` (column-major)
// and optionally row-major `rm` (ld_rm).  Rkeep (lp x lp, FP64) receives the
// accumulated triangular factor when non-null.
pbpqlp_status orth(Ctx& c, bool f64, const void* X, int64_t ld, int64_t len, int passes,
                   void* out, void* tmp, double* Rkeep, int64_t ldrk, void* rm, int64_t ldrm,
                   void* info, hipStream_t st, bool small = false, int next_mode = M_F32) {
  // the last apply also writes the 16-bit copy the next pass multiplies with
  Emit16 em;
  if (!f64 && next_mode >= M_BF16) {
    em.hi = c.Xhi;
    em.lo = c.Xlo;
    em.mode = next_mode;
    em.xs = next_mode == M_F16 ? fp16_lift(true, len) : 1.0f;
  }
  if (em.mode) {
    c.conv_X = out;
    c.conv_mode = em.mode;
    c.conv_xs = em.xs;
  } else if (c.conv_X == out) {
    c.conv_X = nullptr;   // out is rewritten without its 16-bit copy
  }
  if (c.wide) return orth_wide(c, f64, X, ld, len, passes, out, tmp, Rkeep, ldrk, rm, ldrm, info, st, small, em);
  const double eps = dep_eps(f64, c.l, len);
  void* Ra = f64 ? c.Ra64 : c.Ra;
  void* Dv = f64 ? c.Dinv64 : c.Dinv;
  const void* src = X;
  for (int ps = 0; ps < passes; ++ps) {
    const bool last = ps == passes - 1;
    void* dst = last ? out : tmp;
    double* Rt = ps == 0 ? c.R1 : c.R2;
    const uint64_t cseed = c.seed ^ (0x9E3779B97F4A7C15ull * (++c.ncall));
    const double el = f64 ? 8.0 : (double)c.el;
    // a later sweep whose input is already orthonormal to the rounding of its
    // storage takes the identity factor, decided on the device: the Gram
    // reduction flags entries off the identity, the Cholesky reads the flags,
    // the sweep's apply and R2 R1 become copies.  FP32 data: a sweep's own
    // FP32 substitution leaves |Q^T Q - I| at about 3 u32 for l up to 256
    // (l-term sums), so an input within 4 u32 is as orthonormal as another
    // sweep would make it
    int* idf = ps > 0 ? c.ident : nullptr;
    int* farf = ps > 0 ? c.far : nullptr;
    const double itol = f64 ? 2e-14 : 4.0 * 5.9604644775390625e-08;
    {
      TraceScope ts(small ? "gram_ll" : "gram", (double)len * c.l * el, (double)len * c.l * c.l, st);
      PBQ_CHECK(launch_gram(f64, src, ld, len, c.lp, c.gpart, c.G, c.lp, c.gram_target, st, farf, c.l, itol));
    }
    {
      TraceScope ts(small ? "chol_ll" : "chol", (double)c.l * c.l * 8 * 2, (double)c.l * c.l * c.l / 3.0, st);
      PBQ_CHECK(launch_chol(f64, c.G, c.lp, c.l, c.lp, eps, Rt, c.lp, Ra, Dv, c.dep, info, st, nullptr, idf, farf));
    }
    {
      TraceScope ts(small ? "apply_ll" : "apply", 2.0 * len * c.l * el, (double)len * c.l * c.l, st);
      PBQ_CHECK(launch_apply(f64, src, ld, len, c.lp, c.l, Ra, Dv, c.dep, cseed, dst, ld,
                             last ? rm : nullptr, ldrm, st, -1, idf, last ? em : Emit16()));
    }
    src = dst;
  }
  if (Rkeep) {
    TraceScope ts("r2r1", 3.0 * c.lp * c.lp * 8, 2.0 * c.lp * c.lp * c.lp, st);
    if (passes == 1)
      PBQ_CHECK(launch_copy_mat(c.R1, c.lp, c.lp, c.lp, Rkeep, ldrk, 1, st));
    else
      PBQ_CHECK(launch_small_gemm(c.lp, c.lp, c.lp, c.R2, c.lp, 0, c.R1, c.lp, 0, Rkeep, ldrk, 0, st, c.ident));
  }
  return PBPQLP_OK;
}

// The l x l stage: R^T = Qt U (U = L^T) by two FP64 CholeskyQR sweeps of the
// l x l matrix R^T, whose column-major storage is R itself (row-major).
pbpqlp_status small_qr(Ctx& c, const double* Rrow, int64_t ldr, void* info, hipStream_t st) {
  return orth(c, true, Rrow, ldr, c.l, 2, c.Qt64, c.M1, c.U, c.lp, nullptr, 0, info, st, true);
}

// The whole method on M (M = A, or M = A^T for the paper's orientation).
// Q (mM x l) receives Q Qt and P (nM x l) the orthonormal factor of the
// projection, so that M ~= Q L^T P^T.  A product M X is a pass with A when
// M = A and with A^T when M = A^T; M^T X the other way round.
pbpqlp_status run_factor(Ctx& c, const void* A, void* Q, int64_t ldq, double* L, int64_t ldl,
                         void* P, int64_t ldp, pbpqlp_info* info, hipStream_t st) {
  const bool tM = c.tv, tMt = !c.tv;   // direction of the passes with A for M X and M^T X
  const int64_t mM = c.mM(), nM = c.nM(), ldmM = c.ldmM(), ldnM = c.ldnM();
  {
    TraceScope ts("info", 0.0, 0.0, st);
    PBQ_CHECK(launch_info_init(info, c.l, c.q, st));
  }
  if (c.sparse) {
    // CSR of A^T (stable), ||A||_F^2 from the values, zero padding of the
    // row-major operand copy
    TraceScope ts("csr_transpose", (double)c.nnz * (2 * (c.el + 4) + 40) + (double)c.n * 12, 0.0, st);
    PBQ_CHECK(launch_fill_zero(c.Xrm, (size_t)(c.m > c.n ? c.m : c.n) * c.lp32 * c.el, st));
    PBQ_CHECK(launch_csr_transpose(c.f64, c.rowptr, c.colind, c.vals, c.m, c.n, c.nnz, c.tscratch, c.ptr_t,
                                   c.idx_t, c.vals_t, &info->status_flags, st));
    PBQ_CHECK(launch_sumsq(c.f64, c.vals, c.nnz, c.nsq, c.normA, st));
  }
  // S0: sketch matrix, column-major (lp32 x ldnM): generated, or the caller's
  {
    TraceScope ts("omega", (double)nM * c.l * c.el, 0.0, st);
    if (c.omega_in)
      PBQ_CHECK(launch_rm_to_cm(c.f64, c.omega_in, c.ldo_in, nM, c.l, c.lp32, c.Om, ldnM, st));
    else
      PBQ_CHECK(c.wide ? launch_omega_big(c.f64, nM, c.l, c.lp32, c.seed, c.Om, ldnM, st)
                       : launch_omega_cm(c.f64, nM, c.l, c.lp32, c.seed, c.Om, ldnM, st));
  }
  // S1: Y = M Omega (+ ||A||_F^2 when this pass is A X)
  pbpqlp_status s;
  s = stream_pass(c, tM, c.mode_sketch, A, c.Om, ldnM, nM, c.omega_in != nullptr, c.Y, ldmM,
                  tM ? nullptr : c.normA, st);
  if (s) return s;
  s = orth(c, c.f64, c.Y, ldmM, mM, c.q == 0 ? 2 : 1, c.Qm, c.W1m, nullptr, 0, nullptr, 0, info, st, false,
           c.q > 0 ? c.mode_power : c.mode_proj);
  if (s) return s;
  // S3: power iterations with re-orthonormalization after each product
  for (int i = 1; i <= c.q; ++i) {
    s = stream_pass(c, tMt, c.mode_power, A, c.Qm, ldmM, mM, true, c.Zn, ldnM, nullptr, st);
    if (s) return s;
    s = orth(c, c.f64, c.Zn, ldnM, nM, 1, c.Pn, c.W1n, nullptr, 0, nullptr, 0, info, st, false, c.mode_power);
    if (s) return s;
    s = stream_pass(c, tM, c.mode_power, A, c.Pn, ldnM, nM, true, c.Y, ldmM, nullptr, st);
    if (s) return s;
    s = orth(c, c.f64, c.Y, ldmM, mM, i == c.q ? 2 : 1, c.Qm, c.W1m, nullptr, 0, nullptr, 0, info, st, false,
             i < c.q ? c.mode_power : c.mode_proj);
    if (s) return s;
  }
  // S4: projection M^T Q (+ ||A||_F^2 when this pass is A X);  S5: = P R
  // (P written row-major to the caller)
  s = stream_pass(c, tMt, c.mode_proj, A, c.Qm, ldmM, mM, true, c.Zn, ldnM, tMt ? nullptr : c.normA, st);
  if (s) return s;
  s = orth(c, c.f64, c.Zn, ldnM, nM, 2, c.Pn, c.W1n, c.Rfin, c.ldS, P, ldp, info, st);
  if (s) return s;
  if (c.r_out) PBQ_CHECK(launch_copy_mat(c.Rfin, c.ldS, c.l, c.l, c.r_out, c.ldr_out, 1, st));
  // S6: R^T = Qt L^T
  s = small_qr(c, c.Rfin, c.ldS, info, st);
  if (s) return s;
  {
    TraceScope ts("write_l", 2.0 * c.l * c.l * 8, 0.0, st);
    PBQ_CHECK(launch_write_lower_t(c.U, c.lp, c.l, L, ldl, c.rowsq, st));
  }
  // S7: Q Qt, written row-major to the caller; Qt (column-major FP64) is first
  // transposed to row-major in the data type (M1 is free once small_qr is done)
  void* Mr = c.f64 ? (void*)c.M1 : c.Qt32;
  {
    TraceScope ts("transpose", (double)c.lp * c.lp * (8.0 + c.el), 0.0, st);
    PBQ_CHECK(launch_transpose_cast(c.f64, c.Qt64, c.ldS, c.lp, c.lp, Mr, c.ldS, st));
  }
  {
    TraceScope ts("right_mul", 2.0 * mM * c.l * c.el, 2.0 * mM * c.l * c.l, st);
    if (c.wide)
      PBQ_CHECK(launch_gemm(c.f64 ? 1 : 0, mM, c.l, c.l, c.Qm, 1, ldmM, Mr, c.ldS, 1, nullptr, Q, ldq, 1, 1.0,
                            0.0, false, st));
    else
      PBQ_CHECK(launch_right_mul(c.f64, c.Qm, ldmM, mM, c.lp, c.l, Mr, c.ldS, nullptr, 0, Q, ldq, st));
  }
  // S8: result record; numerical rank from the L-values
  {
    TraceScope ts("info", 0.0, 0.0, st);
    PBQ_CHECK(launch_info_finalize(info, c.normA, c.k1_blocks * c.k1_splits, c.rowsq, c.l, st));
  }
  if (c.rank_out) PBQ_CHECK(launch_rank_estimate(L, ldl, c.l, c.rank_tol, c.rank_out, st));
  return PBPQLP_OK;
}

struct ScratchGuard {
  void* p = nullptr;
  hipStream_t s = nullptr;
  ~ScratchGuard() {
    if (p) (void)hipFreeAsync(p, s);
  }
};

pbpqlp_status alloc_scratch(ScratchGuard& g, size_t bytes, hipStream_t st) {
  g.s = st;
  if (hipMallocAsync(&g.p, bytes > 0 ? bytes : 256, st) != hipSuccess) {
    g.p = nullptr;
    return PBPQLP_ENOMEM;
  }
  return PBPQLP_OK;
}

}  // namespace

// ---------------------------------------------------------------------------
// Batches: the single-problem orchestration is recorded once per problem and
// the records become grouped launches (see launch.h).  Problems with the same
// launch sequence (the same q) form a class; launch j of every problem in a
// class runs in one kernel launch per distinct kernel (shape class), with the
// per-problem parameters in a device array and blockIdx.z selecting the
// problem.  Stream order between consecutive launches keeps each problem's
// dependencies.
// ---------------------------------------------------------------------------
namespace {

struct BatchGroup {
  const void* fn;
  dim3 grid, block;
  size_t psize, offset;  // parameter block size and its offset in the device array
  int count;
};

}  // namespace

struct pbpqlp_batch {
  int count = 0;
  void* ws = nullptr;
  size_t ws_bytes = 0;
  void* dparams = nullptr;
  size_t dparams_bytes = 0;
  std::vector<BatchGroup> groups;
  hipStream_t cap = nullptr;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  int use_graph = 1;
  std::vector<int> gram_wg;   // per problem
};

namespace {

// Gram workgroups per problem in a batch: the problems already fill the chip
// together, so each Gram splits only while the batch is small.
int batch_gram_target(int count) {
  const int t = (4096 + count - 1) / count;
  return t < 512 ? t : 512;
}

void batch_free(pbpqlp_batch* b) {
  if (!b) return;
  if (b->exec) (void)hipGraphExecDestroy(b->exec);
  if (b->graph) (void)hipGraphDestroy(b->graph);
  if (b->cap) (void)hipStreamDestroy(b->cap);
  if (b->dparams) (void)hipFree(b->dparams);
  if (b->ws) (void)hipFree(b->ws);
  delete b;
}

pbpqlp_status batch_launch_all(pbpqlp_batch* b, hipStream_t st) {
  alignas(16) unsigned char zero[512] = {};
  for (const BatchGroup& g : b->groups) {
    void* dptr = (char*)b->dparams + g.offset;
    void* args[2] = {&dptr, zero};
    if (g.psize > sizeof(zero)) return PBPQLP_EHIP;
    dim3 grid(g.grid.x, g.grid.y, (unsigned)g.count);
    if (hipLaunchKernel(g.fn, grid, g.block, args, 0, st) != hipSuccess) return PBPQLP_EHIP;
  }
  return hipGetLastError() == hipSuccess ? PBPQLP_OK : PBPQLP_EHIP;
}

}  // namespace

extern "C" {

const char* pbpqlp_status_string(pbpqlp_status s) {
  switch (s) {
    case PBPQLP_OK: return "PBPQLP_OK";
    case PBPQLP_EINVAL: return "PBPQLP_EINVAL: invalid argument";
    case PBPQLP_ENOMEM: return "PBPQLP_ENOMEM: workspace too small or allocation failed";
    case PBPQLP_EHIP: return "PBPQLP_EHIP: HIP runtime error";
    case PBPQLP_EUNSUPPORTED: return "PBPQLP_EUNSUPPORTED: outside the library's limits";
  }
  return "PBPQLP: unknown status";
}

int pbpqlp_version(void) { return 100; }

void pbpqlp_default_opts(pbpqlp_opts* o) {
  if (!o) return;
  std::memset(o, 0, sizeof(*o));
  o->sketch_prec = o->power_prec = o->proj_prec = PBPQLP_PREC_NATIVE;
  o->fp16_scale_a = 1.0;
}

pbpqlp_status pbpqlp_workspace_size(int64_t m, int64_t n, int k, int p, pbpqlp_dtype dt,
                                    const pbpqlp_opts* opts, size_t* bytes) {
  if (!bytes) return PBPQLP_EINVAL;
  // sized for q >= 1 (the power passes may split differently from the
  // others) and for both orientations
  size_t most = 0;
  for (int tv = 0; tv < 2; ++tv) {
    Ctx c;
    pbpqlp_status s = setup(c, m, n, n, dt, k, p, 1, opts, false, tv != 0);
    if (s) return s;
    Bump b;
    c.carve(b, needs16(c));
    b.take(sizeof(pbpqlp_info));
    if (b.off + 256 > most) most = b.off + 256;
  }
  *bytes = most;
  return PBPQLP_OK;
}

}  // extern "C"

namespace {

// Optional parts of a factorization call: orientation, R, numerical rank.
struct Extras {
  bool tv = false;            // run on A^T (the paper's orientation)
  double* R = nullptr;
  int64_t ldr = 0;
  double rank_tol = 0.0;
  int* rank = nullptr;
};

pbpqlp_status factor_impl(const void* A, int64_t m, int64_t n, int64_t lda, pbpqlp_dtype dt,
                          const void* Omega, int64_t ldo, int k, int p, int q, uint64_t seed,
                          void* Q, int64_t ldq, double* L, int64_t ldl, void* P, int64_t ldp,
                          const pbpqlp_opts* opts, pbpqlp_info* d_info, void* stream,
                          const Extras& ex = Extras()) {
  if (!A || !Q || !L || !P) return PBPQLP_EINVAL;
  Ctx c;
  pbpqlp_status s = setup(c, m, n, lda, dt, k, p, q, opts, false, ex.tv);
  if (s) return s;
  if (ex.R) {
    if (ex.ldr < c.l || !aligned(ex.R, 8) || (const void*)ex.R == A || (void*)ex.R == Q ||
        (void*)ex.R == P || ex.R == L)
      return PBPQLP_EINVAL;
    c.r_out = ex.R;
    c.ldr_out = ex.ldr;
  }
  if (ex.rank) {
    if (!(ex.rank_tol >= 0.0) || !aligned(ex.rank, 4)) return PBPQLP_EINVAL;
    c.rank_tol = ex.rank_tol;
    c.rank_out = ex.rank;
  }
  if (ldq < c.l || ldl < c.l || ldp < c.l) return PBPQLP_EINVAL;
  if (Q == A || P == A || (const void*)L == A || Q == P) return PBPQLP_EINVAL;
  if (!aligned(A, c.el) || !aligned(Q, c.el) || !aligned(P, c.el) || !aligned(L, 8))
    return PBPQLP_EINVAL;
  if (Omega) {
    if (ldo < c.l || !aligned(Omega, c.el) || Omega == Q || Omega == P || Omega == (const void*)L)
      return PBPQLP_EINVAL;
    c.omega_in = Omega;
    c.ldo_in = ldo;
  }
  c.seed = seed;
  hipStream_t st = (hipStream_t)stream;
  const bool n16 = needs16(c);
  Bump sizer;
  c.carve(sizer, n16);
  sizer.take(sizeof(pbpqlp_info));
  const size_t need = sizer.off + 256;   // + alignment slack for an unaligned caller block
  ScratchGuard g;
  char* base;
  size_t avail;
  if (opts && opts->workspace) {
    base = (char*)opts->workspace;
    avail = opts->workspace_bytes;
    if (avail < need) return PBPQLP_ENOMEM;
  } else {
    s = alloc_scratch(g, need, st);
    if (s) return s;
    base = (char*)g.p;
    avail = need;
  }
  Bump b;
  b.base = (char*)(((uintptr_t)base + 255) & ~(uintptr_t)255);
  c.carve(b, n16);
  pbpqlp_info* own = (pbpqlp_info*)b.take(sizeof(pbpqlp_info));
  if ((size_t)(b.base + b.off - base) > avail) return PBPQLP_ENOMEM;
  pbpqlp_info* info = d_info ? d_info : own;
  // on M = A^T the method's Q (n x l) is the caller's P and its P (m x l) the
  // caller's Q: A = M^T ~= P_M L Q_M^T
  if (c.tv) return run_factor(c, A, P, ldp, L, ldl, Q, ldq, info, st);
  return run_factor(c, A, Q, ldq, L, ldl, P, ldp, info, st);
}

// Rows per staged panel of a host-resident A: the caller's count rounded up to
// a multiple of 256, or about 256 MiB of rows; never more than m rounded up.
int64_t host_panel_rows(int64_t m, int64_t lda, size_t el, int64_t want) {
  int64_t r = want > 0 ? want : (int64_t)((256ull << 20) / ((size_t)lda * el));
  r = rup(r < 1 ? 1 : r, 256);
  const int64_t mr = rup(m, 256);
  return r < mr ? r : mr;
}

// Streams and events of one host-resident call; destroyed at the end of the
// call, after the copy stream has finished (the compute stream's waits were
// enqueued before).
struct HostRes {
  hipStream_t cs = nullptr;
  hipEvent_t ev[6] = {nullptr, nullptr, nullptr, nullptr, nullptr, nullptr};
  void* bounce[2] = {nullptr, nullptr};
  ~HostRes() {
    if (cs) (void)hipStreamSynchronize(cs);
    for (hipEvent_t e : ev)
      if (e) (void)hipEventDestroy(e);
    for (void* p : bounce)
      if (p) (void)hipHostFree(p);
    if (cs) (void)hipStreamDestroy(cs);
  }
};

// True for host memory the runtime can copy from asynchronously (allocated
// with hipHostMalloc or registered); pageable memory reports otherwise.  The
// query's error on pageable memory is cleared so no later call reports it.
bool host_pinned(const void* p) {
  hipPointerAttribute_t at;
  const hipError_t e = hipPointerGetAttributes(&at, p);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    return false;
  }
  return at.type == hipMemoryTypeHost;
}

pbpqlp_status host_setup(Ctx& c, int64_t m, int64_t n, int64_t lda, pbpqlp_dtype dt, int k, int p,
                         int q, int64_t panel_rows, const pbpqlp_opts* opts) {
  pbpqlp_status s = setup(c, m, n, lda, dt, k, p, q, opts, false, false);
  if (s) return s;
  if (panel_rows < 0) return PBPQLP_EINVAL;
  c.panel_rows = host_panel_rows(m, lda, c.el, panel_rows);
  c.npanels = (int)((m + c.panel_rows - 1) / c.panel_rows);
  c.plan_buffers(true, q > 0, true);
  return PBPQLP_OK;
}

pbpqlp_status csr_setup(Ctx& c, int64_t m, int64_t n, int64_t nnz, pbpqlp_dtype dt, int k, int p, int q,
                        const pbpqlp_opts* opts) {
  if (nnz < 0 || nnz >= INT32_MAX || m >= INT32_MAX || n >= INT32_MAX) return PBPQLP_EINVAL;
  pbpqlp_status s = setup(c, m, n, n, dt, k, p, q, opts, false, false);
  if (s) return s;
  const int native = c.f64 ? M_F64 : M_F32;
  if (c.mode_sketch != native || c.mode_power != native || c.mode_proj != native) return PBPQLP_EUNSUPPORTED;
  c.sparse = true;
  c.nnz = nnz;
  const int64_t ns = (nnz + 4095) / 4096;
  c.nsq = (int)(ns < 1 ? 1 : (ns > 256 ? 256 : ns));
  c.plan_buffers(true, q > 0, true);
  return PBPQLP_OK;
}

}  // namespace

extern "C" {

pbpqlp_status pbpqlp_workspace_size_csr(int64_t m, int64_t n, int64_t nnz, int k, int p, pbpqlp_dtype dt,
                                        const pbpqlp_opts* opts, size_t* bytes) {
  if (!bytes) return PBPQLP_EINVAL;
  Ctx c;
  pbpqlp_status s = csr_setup(c, m, n, nnz, dt, k, p, 1, opts);
  if (s) return s;
  Bump b;
  c.carve(b, false);
  b.take(sizeof(pbpqlp_info));
  *bytes = b.off + 256;
  return PBPQLP_OK;
}

pbpqlp_status pbpqlp_factor_csr(const int64_t* rowptr, const int32_t* colind, const void* vals, int64_t m,
                                int64_t n, int64_t nnz, pbpqlp_dtype dt, int k, int p, int q, uint64_t seed,
                                void* Q, int64_t ldq, double* L, int64_t ldl, void* P, int64_t ldp,
                                const pbpqlp_opts* opts, pbpqlp_info* d_info, void* stream) {
  if (!rowptr || (nnz > 0 && (!colind || !vals)) || !Q || !L || !P) return PBPQLP_EINVAL;
  Ctx c;
  pbpqlp_status s = csr_setup(c, m, n, nnz, dt, k, p, q, opts);
  if (s) return s;
  if (ldq < c.l || ldl < c.l || ldp < c.l || Q == P) return PBPQLP_EINVAL;
  if (!aligned(rowptr, 8) || !aligned(colind, 4) || !aligned(vals, c.el) || !aligned(Q, c.el) ||
      !aligned(P, c.el) || !aligned(L, 8))
    return PBPQLP_EINVAL;
  c.rowptr = rowptr;
  c.colind = colind;
  c.vals = vals;
  c.seed = seed;
  hipStream_t st = (hipStream_t)stream;
  Bump sizer;
  c.carve(sizer, false);
  sizer.take(sizeof(pbpqlp_info));
  const size_t need = sizer.off + 256;
  ScratchGuard g;
  char* base;
  size_t avail;
  if (opts && opts->workspace) {
    base = (char*)opts->workspace;
    avail = opts->workspace_bytes;
    if (avail < need) return PBPQLP_ENOMEM;
  } else {
    s = alloc_scratch(g, need, st);
    if (s) return s;
    base = (char*)g.p;
    avail = need;
  }
  Bump b;
  b.base = (char*)(((uintptr_t)base + 255) & ~(uintptr_t)255);
  c.carve(b, false);
  pbpqlp_info* own = (pbpqlp_info*)b.take(sizeof(pbpqlp_info));
  if ((size_t)(b.base + b.off - base) > avail) return PBPQLP_ENOMEM;
  return run_factor(c, nullptr, Q, ldq, L, ldl, P, ldp, d_info ? d_info : own, st);
}

pbpqlp_status pbpqlp_workspace_size_host(int64_t m, int64_t n, int64_t lda, int k, int p,
                                         pbpqlp_dtype dt, int64_t panel_rows,
                                         const pbpqlp_opts* opts, size_t* bytes) {
  if (!bytes) return PBPQLP_EINVAL;
  Ctx c;
  pbpqlp_status s = host_setup(c, m, n, lda, dt, k, p, 1, panel_rows, opts);
  if (s) return s;
  Bump b;
  c.carve(b, needs16(c));
  b.take(sizeof(pbpqlp_info));
  *bytes = b.off + 256;
  return PBPQLP_OK;
}

pbpqlp_status pbpqlp_factor_host(const void* A_host, int64_t m, int64_t n, int64_t lda,
                                 pbpqlp_dtype dt, int k, int p, int q, uint64_t seed,
                                 int64_t panel_rows, void* Q, int64_t ldq, double* L, int64_t ldl,
                                 void* P, int64_t ldp, const pbpqlp_opts* opts, pbpqlp_info* d_info,
                                 void* stream) {
  if (!A_host || !Q || !L || !P) return PBPQLP_EINVAL;
  Ctx c;
  pbpqlp_status s = host_setup(c, m, n, lda, dt, k, p, q, panel_rows, opts);
  if (s) return s;
  if (ldq < c.l || ldl < c.l || ldp < c.l || Q == P) return PBPQLP_EINVAL;
  if (!aligned(A_host, c.el) || !aligned(Q, c.el) || !aligned(P, c.el) || !aligned(L, 8))
    return PBPQLP_EINVAL;
  c.seed = seed;
  c.A_host = (const char*)A_host;
  hipStream_t st = (hipStream_t)stream;
  const bool n16 = needs16(c);
  Bump sizer;
  c.carve(sizer, n16);
  sizer.take(sizeof(pbpqlp_info));
  const size_t need = sizer.off + 256;
  ScratchGuard g;
  char* base;
  size_t avail;
  if (opts && opts->workspace) {
    base = (char*)opts->workspace;
    avail = opts->workspace_bytes;
    if (avail < need) return PBPQLP_ENOMEM;
  } else {
    s = alloc_scratch(g, need, st);
    if (s) return s;
    base = (char*)g.p;
    avail = need;
  }
  Bump b;
  b.base = (char*)(((uintptr_t)base + 255) & ~(uintptr_t)255);
  c.carve(b, n16);
  pbpqlp_info* own = (pbpqlp_info*)b.take(sizeof(pbpqlp_info));
  if ((size_t)(b.base + b.off - base) > avail) return PBPQLP_ENOMEM;
  pbpqlp_info* info = d_info ? d_info : own;
  HostRes hr;
  if (hipStreamCreateWithFlags(&hr.cs, hipStreamNonBlocking) != hipSuccess) return PBPQLP_EHIP;
  for (hipEvent_t& e : hr.ev)
    if (hipEventCreateWithFlags(&e, hipEventDisableTiming) != hipSuccess) return PBPQLP_EHIP;
  c.cs = hr.cs;
  c.ev_copied[0] = hr.ev[0];
  c.ev_copied[1] = hr.ev[1];
  c.ev_used[0] = hr.ev[2];
  c.ev_used[1] = hr.ev[3];
  c.ev_bounce[0] = hr.ev[4];
  c.ev_bounce[1] = hr.ev[5];
  if (!host_pinned(A_host)) {
    c.bounce = true;
    for (int i = 0; i < 2; ++i) {
      if (hipHostMalloc(&hr.bounce[i], (size_t)c.panel_rows * c.n * c.el, hipHostMallocDefault) != hipSuccess) {
        hr.bounce[i] = nullptr;
        return PBPQLP_ENOMEM;
      }
      c.bounce_buf[i] = hr.bounce[i];
      if (hipEventRecord(c.ev_bounce[i], c.cs) != hipSuccess) return PBPQLP_EHIP;
    }
  }
  // the staging buffers are free once the work already on the stream is done
  if (hipEventRecord(c.ev_used[0], st) != hipSuccess || hipEventRecord(c.ev_used[1], st) != hipSuccess)
    return PBPQLP_EHIP;
  return run_factor(c, nullptr, Q, ldq, L, ldl, P, ldp, info, st);
}

pbpqlp_status pbpqlp_factor(const void* A, int64_t m, int64_t n, int64_t lda, pbpqlp_dtype dt,
                            int k, int p, int q, uint64_t seed, void* Q, int64_t ldq, double* L,
                            int64_t ldl, void* P, int64_t ldp, const pbpqlp_opts* opts,
                            pbpqlp_info* d_info, void* stream) {
  return factor_impl(A, m, n, lda, dt, nullptr, 0, k, p, q, seed, Q, ldq, L, ldl, P, ldp, opts,
                     d_info, stream);
}

}  // extern "C"

// ---------------------------------------------------------------------------
// Allocation-free factorization.  The workspace is one file-scope device
// array; every GPU the library runs on holds its own copy for the life of the
// process.  Host code never passes the array's name to a kernel: the device
// address of the current device's copy is looked up once per device with
// hipGetSymbolAddress and used from then on.
// ---------------------------------------------------------------------------
static __device__ __align__(256) unsigned char scratch[PBPQLP_NOALLOC_SCRATCH_BYTES];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

pbpqlp_status scratch_of_current_device(void** out) {
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) return PBPQLP_EHIP;
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* ptr = nullptr;
    if (hipGetSymbolAddress((void**)&ptr, HIP_SYMBOL(scratch)) != hipSuccess || !ptr) return PBPQLP_EHIP;
    g_scratch_ptr[dev] = ptr;
  }
  *out = g_scratch_ptr[dev];
  return PBPQLP_OK;
}

struct NoTrace {
  NoTrace() { t_no_trace = true; }
  ~NoTrace() { t_no_trace = false; }
};

}  // namespace

extern "C" {

pbpqlp_status pbpqlp_factor_noalloc(const void* A, int64_t m, int64_t n, int64_t lda,
                                    pbpqlp_dtype dt, int k, int p, int q, uint64_t seed, void* Q,
                                    int64_t ldq, double* L, int64_t ldl, void* P, int64_t ldp,
                                    const pbpqlp_opts* opts, pbpqlp_info* d_info, void* stream) {
  pbpqlp_opts o;
  pbpqlp_default_opts(&o);
  if (opts) o = *opts;
  o.workspace = nullptr;
  o.workspace_bytes = 0;
  // the bound of pbpqlp_workspace_size holds for every q and lda; sizes are
  // checked before anything touches the device
  size_t need = 0;
  pbpqlp_status s = pbpqlp_workspace_size(m, n, k, p, dt, &o, &need);
  if (s) return s;
  if (need > (size_t)PBPQLP_NOALLOC_SCRATCH_BYTES) return PBPQLP_EUNSUPPORTED;
  void* ptr = nullptr;
  s = scratch_of_current_device(&ptr);
  if (s) return s;
  o.workspace = ptr;
  o.workspace_bytes = (size_t)PBPQLP_NOALLOC_SCRATCH_BYTES;
  NoTrace nt;
  return factor_impl(A, m, n, lda, dt, nullptr, 0, k, p, q, seed, Q, ldq, L, ldl, P, ldp, &o, d_info,
                     stream);
}

pbpqlp_status pbpqlp_factor_rr(const void* A, int64_t m, int64_t n, int64_t lda, pbpqlp_dtype dt,
                               int k, int p, int q, uint64_t seed, void* Q, int64_t ldq, double* L,
                               int64_t ldl, void* P, int64_t ldp, const pbpqlp_opts* opts,
                               pbpqlp_rr* rr, pbpqlp_info* d_info, void* stream) {
  if (!rr) return PBPQLP_EINVAL;
  Extras ex;
  switch (rr->orientation) {
    case PBPQLP_ORIENT_AT: ex.tv = false; break;
    case PBPQLP_ORIENT_A: ex.tv = true; break;
    case PBPQLP_ORIENT_AUTO: ex.tv = m >= n; break;
    default: return PBPQLP_EINVAL;
  }
  ex.R = rr->R;
  ex.ldr = rr->ldr;
  ex.rank = rr->d_rank;
  ex.rank_tol = rr->rank_tol;
  const pbpqlp_status s = factor_impl(A, m, n, lda, dt, nullptr, 0, k, p, q, seed, Q, ldq, L, ldl, P,
                                      ldp, opts, d_info, stream, ex);
  if (s == PBPQLP_OK) rr->orientation_used = ex.tv ? PBPQLP_ORIENT_A : PBPQLP_ORIENT_AT;
  return s;
}

pbpqlp_status pbpqlp_factor_sketch(const void* A, int64_t m, int64_t n, int64_t lda,
                                   pbpqlp_dtype dt, const void* Omega, int64_t ldo, int k, int p,
                                   int q, void* Q, int64_t ldq, double* L, int64_t ldl, void* P,
                                   int64_t ldp, const pbpqlp_opts* opts, pbpqlp_info* d_info,
                                   void* stream) {
  if (!Omega) return PBPQLP_EINVAL;
  // the seed still drives the completion of dependent columns
  return factor_impl(A, m, n, lda, dt, Omega, ldo, k, p, q, 0x5EEDull, Q, ldq, L, ldl, P, ldp,
                     opts, d_info, stream);
}

pbpqlp_status pbpqlp_omega(int64_t n, int l, uint64_t seed, pbpqlp_dtype dt, void* Omega,
                           int64_t ldo, void* stream) {
  if (!Omega || n < 1 || l < 1 || ldo < l) return PBPQLP_EINVAL;
  if (dt != PBPQLP_F64 && dt != PBPQLP_F32) return PBPQLP_EINVAL;
  if (l > kMaxWideL) return PBPQLP_EUNSUPPORTED;
  const bool f64 = dt == PBPQLP_F64;
  if (!aligned(Omega, f64 ? 8 : 4)) return PBPQLP_EINVAL;
  // the factorization's own generator (column-major), then the caller's layout
  hipStream_t st = (hipStream_t)stream;
  const int lp32 = (int)rup(l, 32);
  const int64_t ld = rup(n, 64);
  ScratchGuard g;
  pbpqlp_status s = alloc_scratch(g, (size_t)lp32 * ld * (f64 ? 8 : 4), st);
  if (s) return s;
  PBQ_CHECK(lp32 > kMaxL ? launch_omega_big(f64, n, l, lp32, seed, g.p, ld, st)
                         : launch_omega_cm(f64, n, l, lp32, seed, g.p, ld, st));
  PBQ_CHECK(launch_cm_to_rm(f64, g.p, ld, n, l, Omega, ldo, st));
  return PBPQLP_OK;
}

pbpqlp_status pbpqlp_matmul(int trans, const void* A, int64_t m, int64_t n, int64_t lda,
                            pbpqlp_dtype dt, const void* X, int64_t ldx, int l, int prec,
                            double fp16_scale_a, void* Y, int64_t ldy, void* stream) {
  if (!A || !X || !Y || l < 1 || m < 1 || n < 1 || lda < n || ldx < l || ldy < l)
    return PBPQLP_EINVAL;
  {
    const size_t el = dt == PBPQLP_F64 ? 8 : 4;
    if (!aligned(A, el) || !aligned(X, el) || !aligned(Y, el)) return PBPQLP_EINVAL;
  }
  if (l > kMaxL) return PBPQLP_EUNSUPPORTED;
  pbpqlp_opts o;
  pbpqlp_default_opts(&o);
  o.sketch_prec = o.power_prec = o.proj_prec = prec;
  o.fp16_scale_a = fp16_scale_a;
  Ctx c;
  // setup() checks l <= min(m, n); a bare product only needs l <= 256
  c.m = m; c.n = n; c.lda = lda; c.l = l; c.lp = (int)rup(l, 16); c.lp32 = (int)rup(l, 32);
  c.f64 = dt == PBPQLP_F64;
  if (dt != PBPQLP_F64 && dt != PBPQLP_F32) return PBPQLP_EINVAL;
  c.el = c.f64 ? 8 : 4;
  c.ldm = rup(m, 64); c.ldn = rup(n, 64); c.ldS = rup(c.lp, 64);
  bool ok;
  const int mode = resolve_mode(dt, prec, &ok);
  if (!ok) return c.f64 ? PBPQLP_EUNSUPPORTED : PBPQLP_EINVAL;
  c.mode_sketch = c.mode_power = c.mode_proj = mode;
  c.fp16_scale = (float)(fp16_scale_a > 0 ? fp16_scale_a : 1.0);
  c.plan_buffers(!trans, false, trans != 0);
  hipStream_t st = (hipStream_t)stream;
  const int64_t xlen = trans ? m : n, ylen = trans ? n : m;
  const int64_t ldxi = trans ? c.ldm : c.ldn, ldyo = trans ? c.ldn : c.ldm;
  // scratch: Xt, Yt, 16-bit copies, split partials (one carve sizes and hands out)
  const int64_t ldmax = c.ldm > c.ldn ? c.ldm : c.ldn;
  void *Xt = nullptr, *Yt = nullptr;
  auto carve = [&](Bump& b) {
    Xt = b.take((size_t)c.lp32 * ldxi * c.el);
    Yt = b.take((size_t)c.lp32 * ldyo * c.el);
    c.Xhi = b.take((size_t)c.lp32 * ldmax * 2);
    c.Xlo = b.take((size_t)c.lp32 * ldmax * 2);
    c.part = b.take(c.part_bytes);
    c.normA = (double*)b.take((size_t)c.k1_blocks * c.k1_splits * 8);
  };
  Bump sz;
  carve(sz);
  ScratchGuard g;
  pbpqlp_status s = alloc_scratch(g, sz.off + 256, st);
  if (s) return s;
  Bump b;
  b.base = (char*)g.p;
  carve(b);
  PBQ_CHECK(launch_rm_to_cm(c.f64, X, ldx, xlen, l, c.lp32, Xt, ldxi, st));
  s = stream_pass(c, trans != 0, mode, A, Xt, ldxi, xlen, false, Yt, ldyo, nullptr, st);
  if (s) return s;
  PBQ_CHECK(launch_cm_to_rm(c.f64, Yt, ldyo, ylen, l, Y, ldy, st));
  return PBPQLP_OK;
}

pbpqlp_status pbpqlp_orth(const void* Y, int64_t rows, int l, int64_t ldy, pbpqlp_dtype dt,
                          int passes, void* Q, int64_t ldq, double* R, int64_t ldr,
                          pbpqlp_info* d_info, void* stream) {
  if (!Y || !Q || l < 1 || rows < l || ldy < l || ldq < l || (R && ldr < l)) return PBPQLP_EINVAL;
  if (passes < 1 || passes > 2) return PBPQLP_EINVAL;
  if (dt != PBPQLP_F64 && dt != PBPQLP_F32) return PBPQLP_EINVAL;
  if (l > kMaxL) return PBPQLP_EUNSUPPORTED;
  Ctx c;
  c.m = rows; c.n = rows; c.l = l; c.lp = (int)rup(l, 16); c.lp32 = (int)rup(l, 32);
  c.f64 = dt == PBPQLP_F64;
  c.el = c.f64 ? 8 : 4;
  c.ldm = rup(rows, 64);
  c.seed = 0x5EEDull;
  hipStream_t st = (hipStream_t)stream;
  void *Xt = nullptr, *Out = nullptr, *Tmp = nullptr;
  double* Rk = nullptr;
  pbpqlp_info* info = d_info;
  // the same carve sizes the scratch and hands out its pieces
  auto carve = [&](Bump& b) {
    Xt = b.take((size_t)c.lp32 * c.ldm * c.el);
    Out = b.take((size_t)c.lp32 * c.ldm * c.el);
    Tmp = b.take((size_t)c.lp32 * c.ldm * c.el);
    c.gpart = (double*)b.take(gram_partial_elems(rows, c.lp, c.gram_target) * 8);
    c.G = (double*)b.take((size_t)c.lp * c.lp * 8);
    c.R1 = (double*)b.take((size_t)c.lp * c.lp * 8);
    c.R2 = (double*)b.take((size_t)c.lp * c.lp * 8);
    Rk = (double*)b.take((size_t)c.lp * c.lp * 8);
    c.Ra = b.take((size_t)c.lp * c.lp * 8);
    c.Dinv = b.take((size_t)(c.lp / 16) * 256 * 8);
    c.Ra64 = b.take((size_t)c.lp * c.lp * 8);
    c.Dinv64 = b.take((size_t)(c.lp / 16) * 256 * 8);
    c.dep = (int*)b.take((size_t)(c.lp + 1) * 4);
    c.ident = (int*)b.take(sizeof(int));
    c.far = (int*)b.take((size_t)c.lp * gram_far_cols(c.lp) * sizeof(int));
    void* own = b.take(sizeof(pbpqlp_info));
    if (!d_info) info = (pbpqlp_info*)own;
  };
  Bump sz;
  carve(sz);
  ScratchGuard g;
  pbpqlp_status s = alloc_scratch(g, sz.off + 256, st);
  if (s) return s;
  Bump b;
  b.base = (char*)g.p;
  carve(b);
  if (!d_info) PBQ_CHECK(launch_info_init(info, l, 0, st));
  PBQ_CHECK(launch_rm_to_cm(c.f64, Y, ldy, rows, l, c.lp32, Xt, c.ldm, st));
  s = orth(c, c.f64, Xt, c.ldm, rows, passes, Out, Tmp, R ? Rk : nullptr, c.lp, Q, ldq, info, st);
  if (s) return s;
  if (R) PBQ_CHECK(launch_copy_mat(Rk, c.lp, l, l, R, ldr, 1, st));
  return PBPQLP_OK;
}

pbpqlp_status pbpqlp_small_qr(const double* R, int l, int64_t ldr, double* Qt, int64_t ldqt,
                              double* L, int64_t ldl, pbpqlp_info* d_info, void* stream) {
  if (!R || !Qt || !L || l < 1 || ldr < l || ldqt < l || ldl < l) return PBPQLP_EINVAL;
  if (l > kMaxL) return PBPQLP_EUNSUPPORTED;
  Ctx c;
  c.l = l; c.lp = (int)rup(l, 16); c.lp32 = (int)rup(l, 32);
  c.f64 = true; c.el = 8;
  c.ldS = rup(c.lp, 64);
  c.seed = 0x5A11ull;
  hipStream_t st = (hipStream_t)stream;
  pbpqlp_info* info = d_info;
  auto carve = [&](Bump& b) {
    c.Rfin = (double*)b.take((size_t)c.lp32 * c.ldS * 8);
    c.M1 = (double*)b.take((size_t)c.lp32 * c.ldS * 8);
    c.Qt64 = (double*)b.take((size_t)c.lp32 * c.ldS * 8);
    c.gpart = (double*)b.take(gram_partial_elems(l, c.lp, c.gram_target) * 8);
    c.G = (double*)b.take((size_t)c.lp * c.lp * 8);
    c.R1 = (double*)b.take((size_t)c.lp * c.lp * 8);
    c.R2 = (double*)b.take((size_t)c.lp * c.lp * 8);
    c.U = (double*)b.take((size_t)c.lp * c.lp * 8);
    c.Ra64 = c.Ra = b.take((size_t)c.lp * c.lp * 8);
    c.Dinv64 = c.Dinv = b.take((size_t)(c.lp / 16) * 256 * 8);
    c.dep = (int*)b.take((size_t)(c.lp + 1) * 4);
    c.ident = (int*)b.take(sizeof(int));
    c.far = (int*)b.take((size_t)c.lp * gram_far_cols(c.lp) * sizeof(int));
    void* own = b.take(sizeof(pbpqlp_info));
    if (!d_info) info = (pbpqlp_info*)own;
  };
  Bump sz;
  carve(sz);
  ScratchGuard g;
  pbpqlp_status s = alloc_scratch(g, sz.off + 256, st);
  if (s) return s;
  Bump b;
  b.base = (char*)g.p;
  carve(b);
  if (!d_info) PBQ_CHECK(launch_info_init(info, l, 0, st));
  PBQ_CHECK(launch_fill_zero(c.Rfin, (size_t)c.lp32 * c.ldS * 8, st));
  PBQ_CHECK(launch_copy_mat(R, ldr, l, l, c.Rfin, c.ldS, 1, st));
  s = small_qr(c, c.Rfin, c.ldS, info, st);
  if (s) return s;
  PBQ_CHECK(launch_cm_to_rm(true, c.Qt64, c.ldS, l, l, Qt, ldqt, st));
  PBQ_CHECK(launch_write_lower_t(c.U, c.lp, l, L, ldl, nullptr, st));
  return PBPQLP_OK;
}

void pbpqlp_trace_enable(int level) { g_trace_level = level < 0 ? 0 : level; }

void pbpqlp_trace_reset(void) {
  std::lock_guard<std::mutex> lk(g_trace_mu);
  g_trace_n = 0;
}

int pbpqlp_trace_count(void) {
  std::lock_guard<std::mutex> lk(g_trace_mu);
  return (int)g_trace_n;
}

pbpqlp_status pbpqlp_trace_get(int i, char* name, int name_len, double* bytes, double* flops,
                               float* ms) {
  std::lock_guard<std::mutex> lk(g_trace_mu);
  if (i < 0 || (size_t)i >= g_trace_n) return PBPQLP_EINVAL;
  const TraceRec& r = g_trace[i];
  if (name && name_len > 0) {
    std::strncpy(name, r.name.c_str(), (size_t)name_len - 1);
    name[name_len - 1] = 0;
  }
  if (bytes) *bytes = r.bytes;
  if (flops) *flops = r.flops;
  if (ms) {
    if (hipEventElapsedTime(ms, r.a, r.b) != hipSuccess) return PBPQLP_EHIP;
  }
  return PBPQLP_OK;
}

pbpqlp_status pbpqlp_batch_create(int count, const pbpqlp_problem* problems, pbpqlp_dtype dt,
                                  const pbpqlp_opts* opts, pbpqlp_batch** out) {
  if (!out || count < 1 || !problems) return PBPQLP_EINVAL;
  *out = nullptr;
  pbpqlp_opts o;
  pbpqlp_default_opts(&o);
  if (opts) o = *opts;
  o.split_k = 1;               // one contraction split: every problem runs the same launch sequence
  o.workspace = nullptr;
  o.workspace_bytes = 0;
  std::vector<Ctx> ctx((size_t)count);
  std::vector<size_t> off((size_t)count);
  size_t total = 0;
  // a batch tuned for the class of its first problem
  int tuned_gram = 0;
  if (o.gram_workgroups == 0) {
    TunePlan t;
    const pbpqlp_problem& p0 = problems[0];
    if (tune_lookup(tune_key((int)dt, o.sketch_prec, o.power_prec, o.proj_prec, p0.k + p0.p, p0.m,
                             p0.n, true), &t))
      tuned_gram = t.gram_wg;
  }
  for (int i = 0; i < count; ++i) {
    const pbpqlp_problem& pr = problems[i];
    if (!pr.A || !pr.Q || !pr.L || !pr.P) return PBPQLP_EINVAL;
    Ctx& c = ctx[(size_t)i];
    pbpqlp_status s = setup(c, pr.m, pr.n, pr.lda, dt, pr.k, pr.p, pr.q, &o, true);
    if (s) return s;
    if (pr.ldq < c.l || pr.ldl < c.l || pr.ldp < c.l) return PBPQLP_EINVAL;
    if (pr.Q == pr.A || pr.P == pr.A || pr.Q == pr.P) return PBPQLP_EINVAL;
    if (!aligned(pr.A, c.el) || !aligned(pr.Q, c.el) || !aligned(pr.P, c.el) ||
        !aligned(pr.L, 8))
      return PBPQLP_EINVAL;
    c.seed = pr.seed;
    if (o.gram_workgroups == 0) c.gram_target = tuned_gram > 0 ? tuned_gram : batch_gram_target(count);
    Bump sizer;
    c.carve(sizer, needs16(c));
    sizer.take(sizeof(pbpqlp_info));
    off[(size_t)i] = total;
    total += (size_t)rup((int64_t)sizer.off, 256);
  }
  pbpqlp_batch* b = new pbpqlp_batch();
  b->count = count;
  for (const Ctx& c : ctx) b->gram_wg.push_back(c.gram_target);
  b->ws_bytes = total;
  if (hipMalloc(&b->ws, total > 0 ? total : 256) != hipSuccess) {
    batch_free(b);
    return PBPQLP_ENOMEM;
  }
  // record every problem's launch sequence
  std::vector<Recorder> recs((size_t)count);
  for (int i = 0; i < count; ++i) {
    const pbpqlp_problem& pr = problems[i];
    Ctx& c = ctx[(size_t)i];
    Bump bp;
    bp.base = (char*)b->ws + off[(size_t)i];
    c.carve(bp, needs16(c));
    pbpqlp_info* own = (pbpqlp_info*)bp.take(sizeof(pbpqlp_info));
    current_recorder() = &recs[(size_t)i];
    const pbpqlp_status s = run_factor(c, pr.A, pr.Q, pr.ldq, pr.L, pr.ldl, pr.P, pr.ldp,
                                       pr.info ? pr.info : own, nullptr);
    current_recorder() = nullptr;
    if (s) {
      batch_free(b);
      return s;
    }
  }
  // classes of identical sequences (same q), then one group per (slot, kernel)
  std::map<int, std::vector<int>> classes;
  for (int i = 0; i < count; ++i) classes[problems[i].q].push_back(i);
  std::vector<unsigned char> host;
  for (auto& kv : classes) {
    const std::vector<int>& members = kv.second;
    const size_t L = recs[(size_t)members[0]].recs.size();
    for (int i : members)
      if (recs[(size_t)i].recs.size() != L) {
        batch_free(b);
        return PBPQLP_EUNSUPPORTED;
      }
    for (size_t j = 0; j < L; ++j) {
      std::vector<const void*> fns;
      for (int i : members) {
        const void* f = recs[(size_t)i].recs[j].fn;
        bool seen = false;
        for (const void* g : fns) seen = seen || g == f;
        if (!seen) fns.push_back(f);
      }
      for (const void* f : fns) {
        BatchGroup g{};
        g.fn = f;
        g.count = 0;
        for (int i : members) {
          const LaunchRec& r = recs[(size_t)i].recs[j];
          if (r.fn != f) continue;
          if (g.count == 0) {
            g.block = r.block;
            g.psize = r.params.size();
            g.grid = dim3(0, 0, 1);
            host.resize((host.size() + 255) & ~(size_t)255);
            g.offset = host.size();
          }
          g.grid.x = r.grid.x > g.grid.x ? r.grid.x : g.grid.x;
          g.grid.y = r.grid.y > g.grid.y ? r.grid.y : g.grid.y;
          host.insert(host.end(), r.params.begin(), r.params.end());
          ++g.count;
        }
        b->groups.push_back(g);
      }
    }
  }
  b->dparams_bytes = host.size();
  if (hipMalloc(&b->dparams, host.size() > 0 ? host.size() : 256) != hipSuccess ||
      hipMemcpy(b->dparams, host.data(), host.size(), hipMemcpyHostToDevice) != hipSuccess) {
    batch_free(b);
    return PBPQLP_ENOMEM;
  }
  // capture the grouped launches once; runs replay the graph
  if (hipStreamCreateWithFlags(&b->cap, hipStreamNonBlocking) != hipSuccess) {
    batch_free(b);
    return PBPQLP_EHIP;
  }
  if (hipStreamBeginCapture(b->cap, hipStreamCaptureModeThreadLocal) != hipSuccess) {
    batch_free(b);
    return PBPQLP_EHIP;
  }
  const pbpqlp_status ls = batch_launch_all(b, b->cap);
  const hipError_t ce = hipStreamEndCapture(b->cap, &b->graph);
  if (ls || ce != hipSuccess || hipGraphInstantiate(&b->exec, b->graph, nullptr, nullptr, 0) != hipSuccess) {
    batch_free(b);
    return PBPQLP_EHIP;
  }
  *out = b;
  return PBPQLP_OK;
}

pbpqlp_status pbpqlp_batch_run(pbpqlp_batch* b, void* stream) {
  if (!b) return PBPQLP_EINVAL;
  hipStream_t st = (hipStream_t)stream;
  if (b->use_graph) return hipGraphLaunch(b->exec, st) == hipSuccess ? PBPQLP_OK : PBPQLP_EHIP;
  return batch_launch_all(b, st);
}

pbpqlp_status pbpqlp_batch_set_graph(pbpqlp_batch* b, int use_graph) {
  if (!b) return PBPQLP_EINVAL;
  b->use_graph = use_graph ? 1 : 0;
  return PBPQLP_OK;
}

pbpqlp_status pbpqlp_batch_stats(const pbpqlp_batch* b, int* launches, size_t* workspace_bytes) {
  if (!b) return PBPQLP_EINVAL;
  if (launches) *launches = (int)b->groups.size();
  if (workspace_bytes) *workspace_bytes = b->ws_bytes;
  return PBPQLP_OK;
}

pbpqlp_status pbpqlp_batch_problem_plan(const pbpqlp_batch* b, int i, int* split_k,
                                        int* gram_workgroups) {
  if (!b || i < 0 || i >= b->count) return PBPQLP_EINVAL;
  if (split_k) *split_k = 1;
  if (gram_workgroups) *gram_workgroups = b->gram_wg[(size_t)i];
  return PBPQLP_OK;
}

void pbpqlp_batch_destroy(pbpqlp_batch* b) { batch_free(b); }

pbpqlp_status pbpqlp_factor_batched(int count, const pbpqlp_problem* problems, pbpqlp_dtype dt,
                                    const pbpqlp_opts* opts, void* stream) {
  pbpqlp_batch* b = nullptr;
  pbpqlp_status s = pbpqlp_batch_create(count, problems, dt, opts, &b);
  if (s) return s;
  s = pbpqlp_batch_run(b, stream);
  if (hipStreamSynchronize((hipStream_t)stream) != hipSuccess && !s) s = PBPQLP_EHIP;
  pbpqlp_batch_destroy(b);
  return s;
}

}  // extern "C"
