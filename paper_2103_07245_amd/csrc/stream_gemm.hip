// A-streaming products of PbP-QLP on gfx950 matrix cores.
//
// These are the passes that dominate the method's cost (Section IV-E: the
// cost is dominated by the multiplications of A and A^T with d-column
// matrices; 2q+2 of them):
//   K1  Y = A X      (eq. (c) for A^T, i.e. the sketch, and the A-side power step)
//   K2  Z = A^T X    (the A^T-side power step and the projection, eq. (D))
// A (m x n, row-major, FP32 or FP64) is read exactly once per pass and never
// touches LDS; the l-column operand X (column-major, compute type) is staged
// through a double-buffered LDS ring shared by the block's waves and re-read from
// L2 by every block.  Both kernels split the contraction over the grid's y
// dimension ("split-K") so small matrices still fill 256 CUs; the partial
// results are summed by splitk_reduce in a fixed order (deterministic).
//
// One kernel serves both directions.  A matrix-core step computes
// D[p][q] += sum_k Aop[p][k] Bop[k][q]:
//   K1: Aop = A (p = row of A, a 16-byte row-contiguous load per lane),
//       Bop = X (q = column of X);  D = (A X)[rows, cols].
//   K2: Aop = X^T (p = column of X), Bop = A (q = column of A): each lane
//       loads RT consecutive columns of V rows of A, so the transpose happens
//       in registers;  D = (A^T X)^T[cols of X, cols of A].
// Lane group g of a step owns the V contraction indices g V .. g V + V - 1 of
// that step in both operands, so each lane's X fragment is one 16-byte LDS
// read.  Full stages run without bounds checks (rows or columns of A past the
// edge are clamped onto valid memory and discarded at the store); only the
// ragged last stage of a split takes masked loads.
//
// Modes: F64 (v_mfma_f64_16x16x4), F32 (v_mfma_f32_16x16x4), BF16 / FP16
// (v_mfma_f32_16x16x32_{bf16,f16}, FP32 accumulate; A converted in
// registers), BF16X3 (hi*hi + hi*lo + lo*hi of bfloat16 splits).
#include <atomic>
#include <type_traits>

#include "common.h"
#include "kernels.h"
#include "launch.h"

namespace pbq {

template <int MODE> struct Tr;
template <> struct Tr<M_F64> {
  typedef double TA; typedef double TC; typedef double TACC;
  static constexpr int V = 2, RT = 1, XN = 1, NW = 8;
  static constexpr int RT1 = 1, NS1 = 2;
};
template <> struct Tr<M_F32> {
  typedef float TA; typedef float TC; typedef float TACC;
  static constexpr int V = 4, RT = 2, XN = 1, NW = 8;
  static constexpr int RT1 = 2, NS1 = 2;
};
template <> struct Tr<M_BF16> {
  typedef float TA; typedef __bf16 TC; typedef float TACC;
  static constexpr int V = 8, RT = 2, XN = 1, NW = 8;
  static constexpr int RT1 = 2, NS1 = 2;
};
template <> struct Tr<M_F16> {
  typedef float TA; typedef _Float16 TC; typedef float TACC;
  static constexpr int V = 8, RT = 2, XN = 1, NW = 8;
  static constexpr int RT1 = 2, NS1 = 2;
};
template <> struct Tr<M_BF16X3> {
  typedef float TA; typedef __bf16 TC; typedef float TACC;
  static constexpr int V = 8, RT = 2, XN = 2, NW = 8;
  static constexpr int RT1 = 2, NS1 = 2;
};

// Every mode moves 16 bytes of compute-type operand per lane per step
// (KS = 4 V contraction indices); a stage is NS steps (two for A^T X and the
// two-stage K1, Tr::NS1 for the general K1), 64 NS bytes per X column.
// RT: 16-row (K1) or paired-column (K2) sub-tiles per wave; the general K1
// takes Tr::RT1.
constexpr int kPitch = 128 + 16;  // LDS bytes per X column of a two-step stage, padded against bank conflicts
constexpr int kGroup = 4;         // X column tiles per scheduling group

typedef uint32_t u32x2 __attribute__((ext_vector_type(2)));
// The same vectors at element alignment: rows of A need only be aligned to
// their element type (the matrix cores' global loads take dword-aligned
// multi-dword addresses).
typedef u32x4 u32x4_e __attribute__((aligned(4)));
typedef u32x2 u32x2_e __attribute__((aligned(4)));

__device__ __forceinline__ float u2f(uint32_t x) { return __uint_as_float(x); }

// Convert 8 FP32 values (two 16-byte groups) to the 16-bit compute type.
template <int MODE>
__device__ __forceinline__ void to16(const u32x4& a, const u32x4& b, float s, u32x4& hi, u32x4& lo) {
  float f[8] = {u2f(a.x), u2f(a.y), u2f(a.z), u2f(a.w), u2f(b.x), u2f(b.y), u2f(b.z), u2f(b.w)};
  if constexpr (MODE == M_F16) {
    union { u32x4 v; f16x8 h; } u;
#pragma unroll
    for (int i = 0; i < 8; ++i) u.h[i] = (_Float16)(f[i] * s);
    hi = u.v;
  } else {
    union { u32x4 v; bf16x8 h; } u, w;
#pragma unroll
    for (int i = 0; i < 8; ++i) {
      u.h[i] = (__bf16)f[i];
      if constexpr (MODE == M_BF16X3) w.h[i] = (__bf16)(f[i] - (float)u.h[i]);
    }
    hi = u.v;
    if constexpr (MODE == M_BF16X3) lo = w.v;
  }
}

template <int MODE>
__device__ __forceinline__ void mma16(const u32x4& a, const u32x4& b, f32x4& c) {
  if constexpr (MODE == M_F16) {
    union { u32x4 v; f16x8 h; } ua, ub;
    ua.v = a; ub.v = b;
    c = mma_f16(ua.h, ub.h, c);
  } else {
    union { u32x4 v; bf16x8 h; } ua, ub;
    ua.v = a; ub.v = b;
    c = mma_bf16(ua.h, ub.h, c);
  }
}

// acc += Aop * Bop for one 16-byte operand slice pair (one step).
template <int MODE, typename ACC>
__device__ __forceinline__ void step_mma(const u32x4& ahi, const u32x4& alo, const u32x4& bhi,
                                         const u32x4& blo, ACC& acc) {
  if constexpr (MODE == M_F64) {
    union { u32x4 v; double d[2]; } ua, ub;
    ua.v = ahi; ub.v = bhi;
    acc = mma_f64(ua.d[0], ub.d[0], acc);
    acc = mma_f64(ua.d[1], ub.d[1], acc);
  } else if constexpr (MODE == M_F32) {
    acc = mma_f32(u2f(ahi.x), u2f(bhi.x), acc);
    acc = mma_f32(u2f(ahi.y), u2f(bhi.y), acc);
    acc = mma_f32(u2f(ahi.z), u2f(bhi.z), acc);
    acc = mma_f32(u2f(ahi.w), u2f(bhi.w), acc);
  } else if constexpr (MODE == M_BF16X3) {
    mma16<MODE>(ahi, bhi, acc);
    mma16<MODE>(ahi, blo, acc);
    mma16<MODE>(alo, bhi, acc);
  } else {
    mma16<MODE>(ahi, bhi, acc);
  }
}

template <typename T> struct AccOf;
template <> struct AccOf<float> { typedef f32x4 type; };
template <> struct AccOf<double> { typedef f64x4 type; };

// K1 store: rows acc_row(g, r) of a 16-row tile starting at `tile_row`,
// column `col`: out[col * ld + tile_row + acc_row(g, r)].
template <typename T, typename ACC>
__device__ __forceinline__ void store_rows(T* out, int64_t ld, int64_t col, int64_t tile_row, int g,
                                           int64_t rend, const ACC& v, float scale) {
  T* p = out + col * ld + tile_row;
  if constexpr (sizeof(T) == 4) {
    const int64_t r0 = tile_row + 4 * g;
    if (r0 + 3 < rend) {
      f32x4 w = {v[0] * scale, v[1] * scale, v[2] * scale, v[3] * scale};
      *(f32x4*)(p + 4 * g) = w;
      return;
    }
  }
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const int rr = acc_row<T>(g, r);
    if (tile_row + rr < rend) p[rr] = (T)(v[r] * scale);
  }
}

// Rows of A that K1 block b (of gx) multiplies: the m rows are cut
// into 16-row groups, block b takes groups [b N / gx, (b + 1) N / gx) of the
// N = ceil(m / 16), i.e. its rows [16 g0, rend), and wave w sub-tile rt the
// group g0 + rt NW + w (first row tile_r[rt]; groups past the block's end are
// clamped away by the caller).  With gx >= ceil(m / (16 NW RT)) no block has
// more than NW RT groups; a grid of more blocks than that evens the work of
// the blocks out (every row block is within one group of the others).  Groups
// go round the waves, so the two waves that share a SIMD (w, w + 4) hold
// every fourth group and a block short of groups still keeps its SIMDs even.
template <int NW, int RT>
__device__ __forceinline__ void k1_rows(int64_t m, unsigned b, unsigned gx, int wave, int64_t& g0, int64_t& rend,
                                        int64_t* tile_r) {
  const int64_t ngr = (m + 15) >> 4;
  g0 = (int64_t)b * ngr / gx;
  const int64_t g1 = ((int64_t)b + 1) * ngr / gx;
  rend = min(m, 16 * g1);
#pragma unroll
  for (int rt = 0; rt < RT; ++rt) tile_r[rt] = 16 * (g0 + rt * NW + wave);
}

// Kernel arguments (by value).
struct StreamParams {
  const void* A;
  int64_t lda, m, n;
  const void* X;
  const void* Xlo;
  int64_t ldx;
  int lp;               // output columns stored (multiple of 16)
  void* out;
  int64_t ldo, split_stride, chunk;
  double* normA;
  float a_scale, out_scale;
  PBQ_GRID;
};

// ---------------------------------------------------------------------------
// grid (ceil(len / (16 RT NW)), S), 64 NW threads (NW = 8 waves: two per
// SIMD; BF16X3 then spills a few registers per lane, which costs less than the
// memory latency a single wave per SIMD leaves exposed).  Wave w owns the
// A-side tiles: for K2 the columns 16 RT (NW blockIdx.x + w) .. + 16 RT, for
// K1 the row groups k1_rows gives it.  The eight waves (one block per CU)
// share one X stage.
// Full stages load A with element-aligned vector loads; only the ragged last
// stage of a split masks its loads.  K2 with n % RT != 0 (VEC = false): the
// lane holding the last, unpaired column loads the pair that ends there and
// moves that column into its first slot (one select per load).
// ---------------------------------------------------------------------------
template <int MODE, int NT, bool TRANS, bool VEC, bool B>
__global__ __launch_bounds__(64 * Tr<MODE>::NW, 2) void stream_kernel(const StreamParams* pb,
                                                                                       StreamParams ps) {
  bool past;
  const StreamParams p = kparams<B>(pb, ps, past);
  if (past) return;
  // Block order (single launches): workgroups are dealt to the eight XCDs
  // round-robin by linear id.  With a grid of a multiple of 8 blocks and one
  // split or at least eight, XCD x takes the x-th eighth of them in
  // split-major order: a contiguous eighth of A's rows, or the rows of the
  // l-column operand of a split or two, which then stay in its L2.  With two
  // to four splits the round-robin order measured as fast or faster (C2
  // 2.664 vs 2.674 ms; C3 2.967 vs 2.863 ms the other way).
  unsigned bx = blockIdx.x, by = blockIdx.y;
  if constexpr (!B) {
    const unsigned N = p.gx * p.gy;
    if ((N & 7) == 0 && (p.gy == 1 || p.gy >= 8)) {
      const unsigned L = blockIdx.x + p.gx * blockIdx.y;
      const unsigned g = (L & 7) * (N >> 3) + (L >> 3);
      bx = g % p.gx;
      by = g / p.gx;
    }
  }
  typedef Tr<MODE> TR;
  typedef typename TR::TA TA;
  typedef typename TR::TC TC;
  typedef typename TR::TACC TACC;
  typedef typename AccOf<TACC>::type ACC;
  constexpr int V = TR::V, KS = 4 * V, XN = TR::XN;
  constexpr int RT = TRANS ? TR::RT : TR::RT1;      // sub-tiles per wave
  constexpr int NS = TRANS ? 2 : TR::NS1;           // steps per stage
  constexpr int KC = NS * KS;                       // contraction indices per stage
  constexpr int PITCH = 64 * NS + 16;               // LDS bytes per X column, padded against bank conflicts
  constexpr int CPC = 4 * NS;                       // 16-byte X chunks per column per stage
  constexpr int NBUF = 2;                           // X ring depth in LDS
  constexpr int NW = TR::NW, NTH = 64 * NW;
  constexpr int NCH = NT * 16 * CPC;                // 16-byte X chunks per stage
  constexpr int XCH = (NCH + NTH - 1) / NTH;        // per thread
  constexpr int EA = 16 / (int)sizeof(TA);          // A elements per 16-byte load (K1)
  constexpr int NLA = (V * (int)sizeof(TA)) / 16;   // 16-byte A loads per lane per step (K1)
  constexpr int NAR = TRANS ? NS * V : NS * RT * NLA; // A registers-loads per lane per stage
  static_assert(NT % 2 == 0, "NT must be even");
  // a chunk index q < NCH is valid; only the last j can overflow
  auto xch_ok = [&](int j, int q) { return j < XCH - 1 || NCH % NTH == 0 || q < NCH; };
  static_assert(!TRANS || RT * sizeof(TA) == 8, "K2 loads 8 bytes of A per row per lane");
  __shared__ __attribute__((aligned(16))) char xs[NBUF][XN][NT * 16 * PITCH];

  const TA* __restrict__ A = (const TA*)p.A;
  const TC* __restrict__ Xc = (const TC*)p.X;
  const TC* __restrict__ Xl = (const TC*)p.Xlo;
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63, li = lane & 15, lg = lane >> 4;
  // A-side position of this lane: K1 a row of A per (rt), K2 RT columns.
  const int64_t a0 = ((int64_t)bx * NW + wave) * (16 * RT);
  const int64_t alen = TRANS ? p.n : p.m;           // extent of the A-side dimension
  const int64_t kb = (int64_t)by * p.chunk;
  const int64_t ke = min(TRANS ? p.m : p.n, kb + p.chunk);
  const int nst = (int)((ke - kb + KC - 1) / KC);
  // K2 needs RT columns for its paired loads; a narrower A runs masked only
  const int nfull = (TRANS && alen < RT) ? 0 : (int)((ke - kb) / KC);

  // K1: this block's rows [16 g0, rend) and its sub-tiles' first rows (tile_r);
  // clamped A-side indices (always valid memory), validity kept for normA.
  int64_t g0 = 0, rend = alen, tile_r[RT], arow[RT];
  bool rowok[RT];
  if constexpr (!TRANS) k1_rows<NW, RT>(p.m, bx, p.gx, wave, g0, rend, tile_r);
#pragma unroll
  for (int rt = 0; rt < RT; ++rt) {
    if constexpr (TRANS) tile_r[rt] = a0 + 16 * rt;
    const int64_t r = tile_r[rt] + li;
    rowok[rt] = r < rend;
    arow[rt] = rowok[rt] ? r : rend - 1;
  }
  // K2: this lane's RT consecutive columns start at acol; its loads start at
  // acol_ld = min(acol, alen - RT) so that a pair never leaves the row, and
  // sh marks the lane whose first column is the last, unpaired one (odd n)
  int64_t acol_ld = a0 + li * RT;
  bool sh = false;
  if (TRANS && acol_ld + RT > alen) {
    const int64_t c = alen > RT ? alen - RT : 0;
    sh = !VEC && RT == 2 && c + 1 == acol_ld;
    acol_ld = c;
  }

  ACC acc[RT][NT];
#pragma unroll
  for (int r = 0; r < RT; ++r)
#pragma unroll
    for (int c = 0; c < NT; ++c) acc[r][c] = ACC{0, 0, 0, 0};

  // the next stage, prefetched into registers
  u32x4 an[TRANS ? 1 : NAR];   // K1: 16-byte A loads
  u32x2 at[TRANS ? NAR : 1];   // K2: 8-byte A loads (RT consecutive columns of one row)
  u32x4 xn[XN][XCH];
  double nrm = 0.0;

  // ---- loads of one stage starting at contraction index k0
  auto load_x = [&](int64_t k0, bool full) __attribute__((always_inline)) {
#pragma unroll
    for (int j = 0; j < XCH; ++j) {
      const int q = tid + NTH * j;
      if (!xch_ok(j, q)) continue;
      const int c = q / CPC, part = q % CPC;
      constexpr int EX = 16 / (int)sizeof(TC);
      const int64_t k = k0 + part * EX;
      const int64_t off = (int64_t)c * p.ldx + k;
#pragma unroll
      for (int x = 0; x < XN; ++x) {
        const TC* src = x == 0 ? Xc : Xl;
        if (full) {
          xn[x][j] = ld16(src + off);
        } else {
          union { u32x4 v; TC e[EX]; } u;
#pragma unroll
          for (int e = 0; e < EX; ++e) u.e[e] = (k + e < ke) ? src[off + e] : TC(0);
          xn[x][j] = u.v;
        }
      }
    }
  };
  auto load_a = [&](int64_t k0, bool full) __attribute__((always_inline)) {
    if constexpr (!TRANS) {
#pragma unroll
      for (int rt = 0; rt < RT; ++rt)
#pragma unroll
        for (int st = 0; st < NS; ++st)
#pragma unroll
          for (int h = 0; h < NLA; ++h) {
            const int64_t k = k0 + st * KS + lg * V + h * EA;
            const TA* src = A + arow[rt] * p.lda + k;
            u32x4& d = an[(rt * NS + st) * NLA + h];
            if (full) {
              d = *(const u32x4_e*)src;
            } else {
              union { u32x4 v; TA e[EA]; } u;
#pragma unroll
              for (int e = 0; e < EA; ++e) u.e[e] = (k + e < ke) ? src[e] : TA(0);
              d = u.v;
            }
          }
    } else {
#pragma unroll
      for (int st = 0; st < NS; ++st)
#pragma unroll
        for (int e = 0; e < V; ++e) {
          const int64_t i = k0 + st * KS + lg * V + e;
          u32x2& d = at[st * V + e];
          if (full) {
            d = *(const u32x2_e*)(A + i * p.lda + acol_ld);
            if (sh) d.x = d.y;
          } else {
            union { u32x2 v; TA e2[RT]; } u;
#pragma unroll
            for (int t = 0; t < RT; ++t)
              u.e2[t] = (i < ke && acol_ld + t < alen) ? A[i * p.lda + acol_ld + t] : TA(0);
            d = u.v;
            if (sh) d.x = d.y;
          }
        }
    }
  };

  if (nst > 0) {
    load_x(kb, nfull > 0);
    load_a(kb, nfull > 0);
  }
  // one stage: its X and A come from the registers, which then take the next
  // stage; the X ring in LDS alternates between two buffers.  NextFull tells
  // that stage s + 1 is full: its prefetch is then unmasked straight-line code.
  // (A masked/unmasked choice per load inside the loop makes the compiler wait
  // for every outstanding load before each new one.)
  auto stage = [&](int s, auto next_full) __attribute__((always_inline)) {
    const int64_t k0 = kb + (int64_t)s * KC;
    const int buf = s & 1;
    // X(s) -> LDS
#pragma unroll
    for (int j = 0; j < XCH; ++j) {
      const int q = tid + NTH * j;
      if (!xch_ok(j, q)) continue;
      const int c = q / CPC, part = q % CPC;
#pragma unroll
      for (int x = 0; x < XN; ++x) st16(&xs[buf][x][c * PITCH + part * 16], xn[x][j]);
    }
    // A(s) -> compute-type fragments afr[rt][st] (hi and, for BF16X3, lo)
    u32x4 ahi[RT][NS], alo[RT][NS];
#pragma unroll
    for (int rt = 0; rt < RT; ++rt)
#pragma unroll
      for (int st = 0; st < NS; ++st) {
        u32x4 g0, g1;  // the V A values of this lane for (rt, st), as raw TA bits
        if constexpr (!TRANS) {
          g0 = an[(rt * NS + st) * NLA];
          g1 = NLA > 1 ? an[(rt * NS + st) * NLA + NLA - 1] : g0;
          if (p.normA) {
            // rows past the edge repeat the last row: weight 0 (no lane branch)
            const double wgt = rowok[rt] ? 1.0 : 0.0;
            if constexpr (sizeof(TA) == 8) {
              union { u32x4 v; double d[2]; } u;
              u.v = g0;
              nrm += wgt * (u.d[0] * u.d[0] + u.d[1] * u.d[1]);
            } else {
#pragma unroll
              for (int h = 0; h < NLA; ++h) {
                const u32x4 v = an[(rt * NS + st) * NLA + h];
                const double x0 = u2f(v.x), x1 = u2f(v.y), x2 = u2f(v.z), x3 = u2f(v.w);
                nrm += wgt * (x0 * x0 + x1 * x1 + x2 * x2 + x3 * x3);
              }
            }
          }
        } else {
          // element e of the fragment is row (lg V + e), column acol + rt
          if constexpr (sizeof(TA) == 8) {
            g0 = u32x4{at[st * V + 0].x, at[st * V + 0].y, at[st * V + 1].x, at[st * V + 1].y};
            g1 = g0;
          } else {
            uint32_t w[8];
#pragma unroll
            for (int e = 0; e < V; ++e) w[e] = rt == 0 ? at[st * V + e].x : at[st * V + e].y;
            g0 = u32x4{w[0], w[1], w[2], w[3]};
            g1 = V > 4 ? u32x4{w[4 % V], w[5 % V], w[6 % V], w[7 % V]} : g0;
          }
        }
        if constexpr (MODE == M_F64 || MODE == M_F32) {
          ahi[rt][st] = g0;
          alo[rt][st] = g0;
        } else {
          to16<MODE>(g0, g1, p.a_scale, ahi[rt][st], alo[rt][st]);
        }
      }
    // prefetch stage s + 1 (its loads stay in flight across the barrier)
    if constexpr (decltype(next_full)::value) {
      load_x(k0 + KC, true);
      load_a(k0 + KC, true);
    } else if (s + 1 < nst) {
      const bool full = s + 1 < nfull;
      load_x(k0 + KC, full);
      load_a(k0 + KC, full);
    }
    lds_barrier();
    if constexpr (XN == 2) {
      // split-BF16x3: six products per X fragment pair; the pair of the next
      // column tile is read before the products of this one are issued
      auto frag = [&](int t, u32x4& h, u32x4& l) __attribute__((always_inline)) {
        const int boff = (16 * (t % NT) + li) * PITCH + (t / NT) * 64 + lg * 16;
        h = *(const u32x4*)&xs[buf][0][boff];
        l = *(const u32x4*)&xs[buf][1][boff];
      };
      u32x4 fh, fl;
      frag(0, fh, fl);
#pragma unroll
      for (int t = 0; t < NS * NT; ++t) {
        const int st = t / NT, ct = t % NT;
        u32x4 nh = fh, nl = fl;
        if (t + 1 < NS * NT) frag(t + 1, nh, nl);
        __builtin_amdgcn_sched_barrier(0);
#pragma unroll
        for (int rt = 0; rt < RT; ++rt) {
          if constexpr (!TRANS)
            step_mma<MODE>(ahi[rt][st], alo[rt][st], fh, fl, acc[rt][ct]);
          else
            step_mma<MODE>(fh, fl, ahi[rt][st], alo[rt][st], acc[rt][ct]);
        }
        __builtin_amdgcn_sched_barrier(0);
        fh = nh;
        fl = nl;
      }
    } else {
#pragma unroll
      for (int st = 0; st < NS; ++st) {
#pragma unroll
        for (int ct = 0; ct < NT; ++ct) {
          // keep at most kGroup X fragments in flight: the scheduler would
          // otherwise hoist every LDS read of the step and spill accumulators
          if (ct % kGroup == 0 && (ct > 0 || st > 0)) __builtin_amdgcn_sched_barrier(0);
          const int boff = (16 * ct + li) * PITCH + st * 64 + lg * 16;
          const u32x4 xhi = *(const u32x4*)&xs[buf][0][boff];
#pragma unroll
          for (int rt = 0; rt < RT; ++rt) {
            if constexpr (!TRANS)
              step_mma<MODE>(ahi[rt][st], alo[rt][st], xhi, xhi, acc[rt][ct]);
            else
              step_mma<MODE>(xhi, xhi, ahi[rt][st], alo[rt][st], acc[rt][ct]);
          }
        }
      }
    }
  };
  int s = 0;
  for (; s + 1 < nfull; ++s) stage(s, std::true_type());
  for (; s < nst; ++s) stage(s, std::false_type());

  TACC* out = (TACC*)p.out + (int64_t)by * p.split_stride;
  const int Tst = p.lp >> 4;
  if constexpr (!TRANS) {
#pragma unroll
    for (int rt = 0; rt < RT; ++rt)
#pragma unroll
      for (int ct = 0; ct < NT; ++ct)
        if (ct < Tst)
          store_rows<TACC>(out, p.ldo, 16 * ct + li, tile_r[rt], lg, rend, acc[rt][ct], p.out_scale);
  } else {
    const int64_t j = a0 + li * RT;  // unclamped: lanes past the edge store nothing
#pragma unroll
    for (int ct = 0; ct < NT; ++ct)
      if (ct < Tst)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int64_t c = 16 * ct + acc_row<TACC>(lg, r);
          TACC* dst = out + c * p.ldo + j;
          if constexpr (RT == 2) {
            if (j + 1 < alen) {
              typedef float f32x2 __attribute__((ext_vector_type(2)));
              *(f32x2*)dst = f32x2{acc[0][ct][r] * p.out_scale, acc[1][ct][r] * p.out_scale};
            } else if (j < alen) {
              dst[0] = acc[0][ct][r] * p.out_scale;
            }
          } else {
            if (j < alen) dst[0] = (TACC)(acc[0][ct][r] * p.out_scale);
          }
        }
  }

  if (!TRANS && p.normA) {
    __shared__ double red[NW];
    nrm = wave_sum(nrm);
    if (lane == 0) red[wave] = nrm;
    lds_barrier();
    if (tid == 0) {
      double t = 0.0;
#pragma unroll
      for (int w = 0; w < NW; ++w) t += red[w];
      p.normA[by * p.gx + bx] = t;
    }
  }
}

// ---------------------------------------------------------------------------
// K1 (Y = A X) with two stages of A in flight per wave.  Rows of A are
// 16-byte aligned; each stage's A tile of a wave is NAR 16-byte loads per
// lane.  Even stages land in registers; odd stages go from HBM straight into
// a per-wave LDS slot (global_load_lds, no register cost) and are read back
// when used.  The steady state (all stages full) runs two stages per
// iteration as straight-line code, so the wait counts stay exact: a wave
// waits for the stage it is about to use, never for the one behind it.
// Stage barriers order only LDS (the X ring); the slot is private to its
// wave and guarded by that wave's own vmcnt / lgkmcnt waits.
// ---------------------------------------------------------------------------
__device__ __forceinline__ void ring_barrier() {
  // LDS writes of this wave complete, then the workgroup barrier; no wait on
  // vector memory (the next stages' loads stay in flight)
  asm volatile("s_waitcnt lgkmcnt(0)\n\ts_barrier" ::: "memory");
}

template <int MODE, int NT, bool NORM, bool B>
__global__ __launch_bounds__(64 * Tr<MODE>::NW, 2) void stream_k1_kernel(const StreamParams* pb,
                                                                       StreamParams ps) {
  bool past;
  const StreamParams p = kparams<B>(pb, ps, past);
  if (past) return;
  typedef Tr<MODE> TR;
  typedef typename TR::TA TA;
  typedef typename TR::TC TC;
  typedef typename TR::TACC TACC;
  typedef typename AccOf<TACC>::type ACC;
  constexpr int V = TR::V, KS = 4 * V, KC = 2 * KS, RT = TR::RT;
  static_assert(TR::XN == 1, "split-BF16x3 keeps the general kernel");
  static_assert(TR::RT1 == TR::RT && TR::NS1 == 2, "the two-stage K1 keeps two-step stages of RT sub-tiles");
  constexpr int NW = TR::NW, NTH = 64 * NW;
  constexpr int XCH = (NT * 128 + NTH - 1) / NTH;
  constexpr int EA = 16 / (int)sizeof(TA);
  constexpr int NLA = (V * (int)sizeof(TA)) / 16;
  constexpr int NAR = 2 * RT * NLA;
  static_assert(NLA <= 2, "a fragment is at most two 16-byte loads");
  // every thread moves XCH chunks; chunks past the NT * 16 live columns re-read
  // the last column into padding columns of the ring (no divergent branch)
  constexpr int XCOLS = XCH * NTH / 8;
  __shared__ __attribute__((aligned(16))) char xs[2][XCOLS * kPitch];
  __shared__ __attribute__((aligned(16))) u32x4 aslot[NW * NAR * 64];

  const TA* __restrict__ A = (const TA*)p.A;
  const TC* __restrict__ Xc = (const TC*)p.X;
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63, li = lane & 15, lg = lane >> 4;
  u32x4* const myslot = &aslot[wave * NAR * 64];
  const int64_t kb = (int64_t)blockIdx.y * p.chunk;
  const int64_t ke = min(p.n, kb + p.chunk);
  const int nst = (int)((ke - kb + KC - 1) / KC);
  const int nfull = (int)((ke - kb) / KC);
  int64_t g0, rend, tile_r[RT], arow[RT];
  bool rowok[RT];
  k1_rows<NW, RT>(p.m, blockIdx.x, p.gx, wave, g0, rend, tile_r);
#pragma unroll
  for (int rt = 0; rt < RT; ++rt) {
    const int64_t r = tile_r[rt] + li;
    rowok[rt] = r < rend;
    arow[rt] = rowok[rt] ? r : rend - 1;
  }
  // NORM: the sketch pass also accumulates ||A||_F^2 (p.normA set)
  constexpr bool want_norm = NORM;
  ACC acc[RT][NT];
#pragma unroll
  for (int r = 0; r < RT; ++r)
#pragma unroll
    for (int c = 0; c < NT; ++c) acc[r][c] = ACC{0, 0, 0, 0};
  u32x4 an[NAR];
  u32x4 xn[XCH];
  double nrm = 0.0;

  auto load_x = [&](int64_t k0, bool full) __attribute__((always_inline)) {
#pragma unroll
    for (int j = 0; j < XCH; ++j) {
      const int q = tid + NTH * j;
      const int c = min(q >> 3, NT * 16 - 1), part = q & 7;
      constexpr int EX = 16 / (int)sizeof(TC);
      const int64_t k = k0 + part * EX;
      const TC* src = Xc + (int64_t)c * p.ldx + k;
      if (full) {
        xn[j] = ld16(src);
      } else {
        union { u32x4 v; TC e[EX]; } u;
#pragma unroll
        for (int e = 0; e < EX; ++e) u.e[e] = (k + e < ke) ? src[e] : TC(0);
        xn[j] = u.v;
      }
    }
  };
  auto a_src = [&](int rt, int st, int h, int64_t k0) __attribute__((always_inline)) {
    return A + arow[rt] * p.lda + k0 + st * KS + lg * V + h * EA;
  };
  auto load_a = [&](int64_t k0, bool full, u32x4* dst) __attribute__((always_inline)) {
#pragma unroll
    for (int rt = 0; rt < RT; ++rt)
#pragma unroll
      for (int st = 0; st < 2; ++st)
#pragma unroll
        for (int h = 0; h < NLA; ++h) {
          const TA* src = a_src(rt, st, h, k0);
          u32x4& d = dst[(rt * 2 + st) * NLA + h];
          if (full) {
            d = ld16(src);
          } else {
            const int64_t k = k0 + st * KS + lg * V + h * EA;
            union { u32x4 v; TA e[EA]; } u;
#pragma unroll
            for (int e = 0; e < EA; ++e) u.e[e] = (k + e < ke) ? src[e] : TA(0);
            d = u.v;
          }
        }
  };
  auto dma_a = [&](int64_t k0) __attribute__((always_inline)) {
#pragma unroll
    for (int rt = 0; rt < RT; ++rt)
#pragma unroll
      for (int st = 0; st < 2; ++st)
#pragma unroll
        for (int h = 0; h < NLA; ++h)
          __builtin_amdgcn_global_load_lds(
              (const void*)a_src(rt, st, h, k0),
              (__attribute__((address_space(3))) void*)(myslot + 64 * ((rt * 2 + st) * NLA + h)), 16, 0, 0);
  };
  auto store_x = [&](int buf) __attribute__((always_inline)) {
#pragma unroll
    for (int j = 0; j < XCH; ++j) {
      const int q = tid + NTH * j;
      const int c = q >> 3, part = q & 7;
      st16(&xs[buf][c * kPitch + part * 16], xn[j]);
    }
  };
  u32x4 ahi[RT][2], alo[RT][2];
  auto convert = [&](auto get) __attribute__((always_inline)) {
#pragma unroll
    for (int rt = 0; rt < RT; ++rt)
#pragma unroll
      for (int st = 0; st < 2; ++st) {
        const u32x4 g0 = get((rt * 2 + st) * NLA);
        const u32x4 g1 = NLA > 1 ? get((rt * 2 + st) * NLA + NLA - 1) : g0;
        if (want_norm) {
          // rows past the edge repeat the last row: weight 0
          const double wgt = rowok[rt] ? 1.0 : 0.0;
          if constexpr (sizeof(TA) == 8) {
            union { u32x4 v; double d[2]; } u;
            u.v = g0;
            nrm += wgt * (u.d[0] * u.d[0] + u.d[1] * u.d[1]);
          } else {
#pragma unroll
            for (int h = 0; h < NLA; ++h) {
              const u32x4 v = h == 0 ? g0 : g1;
              const double x0 = u2f(v.x), x1 = u2f(v.y), x2 = u2f(v.z), x3 = u2f(v.w);
              nrm += wgt * (x0 * x0 + x1 * x1 + x2 * x2 + x3 * x3);
            }
          }
        }
        if constexpr (MODE == M_F64 || MODE == M_F32) {
          ahi[rt][st] = g0;
          alo[rt][st] = g0;
        } else {
          to16<MODE>(g0, g1, p.a_scale, ahi[rt][st], alo[rt][st]);
        }
        __builtin_amdgcn_sched_barrier(0);
      }
  };
  auto compute = [&](int buf) __attribute__((always_inline)) {
#pragma unroll
    for (int st = 0; st < 2; ++st) {
#pragma unroll
      for (int ct = 0; ct < NT; ++ct) {
        if (ct % kGroup == 0 && (ct > 0 || st > 0)) __builtin_amdgcn_sched_barrier(0);
        const int boff = (16 * ct + li) * kPitch + st * 64 + lg * 16;
        const u32x4 xhi = *(const u32x4*)&xs[buf][boff];
#pragma unroll
        for (int rt = 0; rt < RT; ++rt) step_mma<MODE>(ahi[rt][st], alo[rt][st], xhi, xhi, acc[rt][ct]);
      }
    }
  };
  auto from_regs = [&](int j) { return an[j]; };
  auto from_slot = [&](int j) { return myslot[64 * j + lane]; };

  // prologue: X(0), A(0) -> registers; A(1) -> slot when full
  if (nst > 0) {
    load_x(kb, nfull > 0);
    load_a(kb, nfull > 0, an);
    if (nfull > 1) dma_a(kb + KC);
  }
  int s = 0;
  // steady state: stages s (registers) and s + 1 (slot) full, and the two
  // stages prefetched here (s + 2 into registers, s + 3 into the slot) full
  for (; s + 3 < nfull; s += 2) {
    const int64_t k0 = kb + (int64_t)s * KC;
    // even stage s
    store_x(0);
    convert(from_regs);
    load_x(k0 + KC, true);
    load_a(k0 + 2 * KC, true, an);
    ring_barrier();
    compute(0);
    // odd stage s + 1: its slot loads are older than the NAR loads of A(s + 2)
    store_x(1);
    asm volatile("s_waitcnt vmcnt(%0)" ::"n"(NAR) : "memory");
    convert(from_slot);
    load_x(k0 + 2 * KC, true);
    asm volatile("s_waitcnt lgkmcnt(0)" ::: "memory");   // slot read before it refills
    dma_a(k0 + 3 * KC);
    ring_barrier();
    compute(1);
  }
  // remaining stages, one at a time: stage t's A sits in the registers (even
  // t), in the slot (odd t, full) or is loaded now (odd t, ragged)
  for (; s < nst; ++s) {
    const int64_t k0 = kb + (int64_t)s * KC;
    const int buf = s & 1;
    store_x(buf);
    if ((s & 1) == 0) {
      convert(from_regs);
    } else if (s < nfull) {
      asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
      convert(from_slot);
    } else {
      u32x4 tail[NAR];
      load_a(k0, false, tail);
      convert([&](int j) { return tail[j]; });
    }
    if (s + 1 < nst) load_x(k0 + KC, s + 1 < nfull);
    if (s + 2 < nst) {
      if ((s & 1) == 0) {
        load_a(k0 + 2 * KC, s + 2 < nfull, an);
      } else if (s + 2 < nfull) {
        asm volatile("s_waitcnt lgkmcnt(0)" ::: "memory");
        dma_a(k0 + 2 * KC);
      }
    }
    ring_barrier();
    compute(buf);
  }

  TACC* out = (TACC*)p.out + (int64_t)blockIdx.y * p.split_stride;
  const int Tst = p.lp >> 4;
#pragma unroll
  for (int rt = 0; rt < RT; ++rt)
#pragma unroll
    for (int ct = 0; ct < NT; ++ct)
      if (ct < Tst) store_rows<TACC>(out, p.ldo, 16 * ct + li, tile_r[rt], lg, rend, acc[rt][ct], p.out_scale);
  if (want_norm) {
    __shared__ double red[NW];
    nrm = wave_sum(nrm);
    if (lane == 0) red[wave] = nrm;
    lds_barrier();
    if (tid == 0) {
      double t = 0.0;
#pragma unroll
      for (int w = 0; w < NW; ++w) t += red[w];
      p.normA[blockIdx.y * p.gx + blockIdx.x] = t;
    }
  }
}

// ---------------------------------------------------------------------------
// Launchers
// ---------------------------------------------------------------------------
template <int MODE, int NT, bool TRANS>
static hipError_t launch_nt(const StreamArgs& a, bool vec, hipStream_t s) {
  typedef Tr<MODE> TR;
  const int span = stream_span(MODE, TRANS);
  const int64_t gx = TRANS ? (a.n + span - 1) / span : stream_k1_grid(MODE, a.m, a.splits);
  dim3 grid((unsigned)gx, (unsigned)a.splits);
  StreamParams p;
  p.A = a.A; p.lda = a.lda; p.m = a.m; p.n = a.n;
  p.X = a.X; p.Xlo = a.Xlo; p.ldx = a.ldx; p.lp = a.lp;
  p.out = a.out; p.ldo = a.ldo; p.split_stride = a.split_stride; p.chunk = a.chunk;
  p.normA = TRANS ? nullptr : a.normA;
  p.a_scale = a.a_scale; p.out_scale = a.out_scale;
  // the two-stage K1 for the matrix-core bound FP32 and FP64 modes where its
  // registers fit; the 16-bit modes stream faster through the general kernel
  // (measured per instantiation)
  constexpr bool two = MODE == M_F64 || (MODE == M_F32 && NT <= 14);
  constexpr bool two_norm = two && !(MODE == M_F32 && NT == 14);
  if constexpr (!TRANS && TR::XN == 1 && two) {
    if (vec && p.normA && two_norm)
      return launch_k(stream_k1_kernel<MODE, NT, true, false>, stream_k1_kernel<MODE, NT, true, true>, grid,
                      dim3(64 * TR::NW), s, p);
    if (vec && !p.normA)
      return launch_k(stream_k1_kernel<MODE, NT, false, false>, stream_k1_kernel<MODE, NT, false, true>, grid,
                      dim3(64 * TR::NW), s, p);
  }
  if (vec || !TRANS)
    return launch_k(stream_kernel<MODE, NT, TRANS, true, false>, stream_kernel<MODE, NT, TRANS, true, true>,
                    grid, dim3(64 * TR::NW), s, p);
  if constexpr (TRANS)
    return launch_k(stream_kernel<MODE, NT, TRANS, false, false>, stream_kernel<MODE, NT, TRANS, false, true>,
                    grid, dim3(64 * TR::NW), s, p);
  return hipErrorInvalidValue;
}

template <int MODE, bool TRANS>
static hipError_t dispatch_nt(const StreamArgs& a, bool vec, hipStream_t s) {
  switch (a.lp32 / 16) {
    case 2: return launch_nt<MODE, 2, TRANS>(a, vec, s);
    case 4: return launch_nt<MODE, 4, TRANS>(a, vec, s);
    case 6: return launch_nt<MODE, 6, TRANS>(a, vec, s);
    case 8: return launch_nt<MODE, 8, TRANS>(a, vec, s);
    case 10: return launch_nt<MODE, 10, TRANS>(a, vec, s);
    case 12: return launch_nt<MODE, 12, TRANS>(a, vec, s);
    case 14: return launch_nt<MODE, 14, TRANS>(a, vec, s);
    case 16: return launch_nt<MODE, 16, TRANS>(a, vec, s);
  }
  return hipErrorInvalidValue;
}

template <int MODE>
static hipError_t dispatch_dir(bool trans, const StreamArgs& a, hipStream_t s) {
  typedef Tr<MODE> TR;
  if (((uintptr_t)a.A % sizeof(typename TR::TA)) != 0) return hipErrorInvalidValue;
  // K1: 16-byte aligned rows take the two-stage kernel (odd stages' A tiles
  // through LDS), others the general one with element-aligned loads; K2
  // pairs columns: an odd last column takes the shifted-pair path
  const bool vec = trans ? a.n % TR::RT == 0
                         : ((uintptr_t)a.A % 16 == 0 && (a.lda * (int64_t)sizeof(typename TR::TA)) % 16 == 0);
  return trans ? dispatch_nt<MODE, true>(a, vec, s) : dispatch_nt<MODE, false>(a, vec, s);
}

template <int MODE> static int span_of(bool trans) {
  typedef Tr<MODE> TR;
  return 16 * (trans ? TR::RT : TR::RT1) * TR::NW;
}
int stream_span(int mode, bool trans) {
  switch (mode) {
    case M_F64: return span_of<M_F64>(trans);
    case M_F32: return span_of<M_F32>(trans);
    case M_BF16: return span_of<M_BF16>(trans);
    case M_F16: return span_of<M_F16>(trans);
    default: return span_of<M_BF16X3>(trans);
  }
}
int device_cus() {
  static std::atomic<int> cached[64];
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) dev = 0;
  int v = cached[dev].load(std::memory_order_relaxed);
  if (v <= 0) {
    if (hipDeviceGetAttribute(&v, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || v <= 0) v = 256;
    cached[dev].store(v, std::memory_order_relaxed);
  }
  return v;
}

int64_t stream_k1_grid(int mode, int64_t rows, int splits) {
  const int64_t span = stream_span(mode, false);
  const int64_t b0 = (rows + span - 1) / span;
  const int64_t cus = device_cus();
  // one block per CU at a time: for the HBM-bound 16-bit modes a ragged last
  // round becomes whole rounds of smaller row blocks (the FP32 and FP64 modes
  // are matrix-core bound, and a block's clamped sub-tiles cost them as much
  // as full ones)
  if (splits == 1 && b0 > cus && (mode == M_BF16 || mode == M_F16)) return (b0 + cus - 1) / cus * cus;
  return b0;
}


hipError_t launch_stream(bool trans, int mode, const StreamArgs& a, hipStream_t s) {
  if (a.lp32 < 32 || a.lp32 > 256 || a.lp32 % 32 != 0 || a.lp > a.lp32) return hipErrorInvalidValue;
  switch (mode) {
    case M_F64: return dispatch_dir<M_F64>(trans, a, s);
    case M_F32: return dispatch_dir<M_F32>(trans, a, s);
    case M_BF16: return dispatch_dir<M_BF16>(trans, a, s);
    case M_F16: return dispatch_dir<M_F16>(trans, a, s);
    case M_BF16X3: return dispatch_dir<M_BF16X3>(trans, a, s);
  }
  return hipErrorInvalidValue;
}

}  // namespace pbq
