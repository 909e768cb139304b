// A-streaming products of PbP-QLP on gfx950 matrix cores.
//
// These are the passes that dominate the method's cost (Section IV-F: the
// cost is dominated by the multiplications of A and A^T with d-column
// matrices; 2q+2 of them):
//   K1  Y = A X      (eq. (c) for A^T, i.e. the sketch, and the A-side power step)
//   K2  Z = A^T X    (the A^T-side power step and the projection, eq. (D))
// A (m x n, row-major, FP32 or FP64) is read exactly once per pass; the
// l-column operand X is staged through LDS in the compute type and is read
// from L2.  Both kernels split the contraction over the grid's y dimension
// ("split-K") so small matrices still fill 256 CUs; the partial results are
// summed by splitk_reduce in a fixed order (deterministic).
//
// Modes: F64 (v_mfma_f64_16x16x4), F32 (v_mfma_f32_16x16x4), BF16 / FP16
// (v_mfma_f32_16x16x32_{bf16,f16}, FP32 accumulate; A converted in
// registers), BF16X3 (hi*hi + hi*lo + lo*hi of bfloat16 splits).
#include "common.h"
#include "kernels.h"

namespace pbq {

template <int MODE> struct Tr;
template <> struct Tr<M_F64> {
  typedef double TA; typedef double TC; typedef double TACC;
  static constexpr int V = 2, NSUB = 2, RT = 1, XN = 1;
};
template <> struct Tr<M_F32> {
  typedef float TA; typedef float TC; typedef float TACC;
  static constexpr int V = 4, NSUB = 4, RT = 2, XN = 1;
};
template <> struct Tr<M_BF16> {
  typedef float TA; typedef __bf16 TC; typedef float TACC;
  static constexpr int V = 8, NSUB = 1, RT = 2, XN = 1;
};
template <> struct Tr<M_F16> {
  typedef float TA; typedef _Float16 TC; typedef float TACC;
  static constexpr int V = 8, NSUB = 1, RT = 2, XN = 1;
};
template <> struct Tr<M_BF16X3> {
  typedef float TA; typedef __bf16 TC; typedef float TACC;
  static constexpr int V = 8, NSUB = 1, RT = 2, XN = 2;
};

// Every mode moves 128 bytes of compute-type operand per row per stage:
// KS = 4 V contraction indices per step, two steps per stage.
constexpr int kPitch = 128 + 16;  // LDS row pitch (bytes), padded against bank conflicts

// Load 16 bytes of A (row `row`, columns k..k+E-1) with bounds checks.
template <typename TA>
__device__ __forceinline__ u32x4 load_a16(const TA* __restrict__ A, int64_t lda, int64_t row,
                                          int64_t k, int64_t rend, int64_t kend, bool vec) {
  constexpr int E = 16 / sizeof(TA);
  if (vec && row < rend && k + E <= kend) return ld16(A + row * lda + k);
  union { u32x4 v; TA e[E]; } u;
#pragma unroll
  for (int i = 0; i < E; ++i) u.e[i] = (row < rend && k + i < kend) ? A[row * lda + k + i] : TA(0);
  return u.v;
}

__device__ __forceinline__ float u2f(uint32_t x) { return __uint_as_float(x); }

// Convert 8 FP32 values (two 16-byte loads) to the 16-bit compute type.
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

// acc += A_frag * B_frag for one 16-byte operand slice pair (one "step").
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

// Store one accumulator column slice: rows acc_row(g, r) of a 16-row tile
// starting at `tile_row`, i.e. out[col * ld + tile_row + acc_row(g, r)].
template <typename T, typename ACC>
__device__ __forceinline__ void store4(T* out, int64_t ld, int64_t col, int64_t tile_row, int g,
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

// ---------------------------------------------------------------------------
// K1: Ypart[s] (lp x m, column-major) = A[:, kslice(s)] * X[kslice(s), :]
// grid (ceil(m / (64 RT)), S); 4 waves, wave w owns rows 16 RT w .. +16 RT.
// ---------------------------------------------------------------------------
template <int MODE, int NT>
__global__ __launch_bounds__(256) void k1_ax(
    const typename Tr<MODE>::TA* __restrict__ A, int64_t lda, int64_t m, int64_t n,
    const typename Tr<MODE>::TC* __restrict__ Xc, const typename Tr<MODE>::TC* __restrict__ Xlo,
    int64_t ldx, int lp, typename Tr<MODE>::TACC* __restrict__ Ypart, int64_t ldy,
    int64_t split_stride, int64_t kchunk, double* __restrict__ normA, float a_scale,
    float out_scale, int vec_ok) {
  typedef Tr<MODE> TR;
  typedef typename TR::TA TA;
  typedef typename TR::TC TC;
  typedef typename TR::TACC TACC;
  typedef typename AccOf<TACC>::type ACC;
  constexpr int V = TR::V, KS = 4 * V, KC = 2 * KS, RT = TR::RT, XN = TR::XN;
  constexpr int NLA = (V * (int)sizeof(TA)) / 16;  // 16-byte A loads per lane per step
  constexpr int XCH = (NT * 16 * 8 + 255) / 256;   // 16-byte X chunks per thread per stage (max)
  __shared__ __attribute__((aligned(16))) char xs[XN][NT * 16 * kPitch];

  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63, li = lane & 15, lg = lane >> 4;
  const int T = lp >> 4;
  const int64_t row0 = (int64_t)blockIdx.x * (64 * RT) + wave * (16 * RT);
  const int64_t kb = (int64_t)blockIdx.y * kchunk;
  const int64_t ke = min(n, kb + kchunk);
  const bool vec = vec_ok != 0;
  const int nxch = lp * 8;  // 16-byte chunks of X per stage

  ACC acc[RT][NT];
#pragma unroll
  for (int r = 0; r < RT; ++r)
#pragma unroll
    for (int c = 0; c < NT; ++c) acc[r][c] = ACC{0, 0, 0, 0};

  u32x4 anext[RT][2][NLA];
  u32x4 xnext[XN][XCH];
  double nrm = 0.0;

  auto load_stage = [&](int64_t k0) {
#pragma unroll
    for (int rt = 0; rt < RT; ++rt)
#pragma unroll
      for (int st = 0; st < 2; ++st)
#pragma unroll
        for (int h = 0; h < NLA; ++h) {
          const int64_t kk = k0 + st * KS + lg * V + h * (16 / (int)sizeof(TA));
          anext[rt][st][h] = load_a16<TA>(A, lda, row0 + 16 * rt + li, kk, m, ke, vec);
        }
#pragma unroll
    for (int j = 0; j < XCH; ++j) {
      const int q = tid + 256 * j;
      if (q < nxch) {
        const int c = q >> 3, part = q & 7;
        const int64_t off = (int64_t)c * ldx + k0 + part * (16 / (int)sizeof(TC));
        xnext[0][j] = ld16(Xc + off);
        if constexpr (XN == 2) xnext[1][j] = ld16(Xlo + off);
      }
    }
  };

  if (kb < ke) load_stage(kb);
  for (int64_t k0 = kb; k0 < ke; k0 += KC) {
    lds_barrier();
#pragma unroll
    for (int j = 0; j < XCH; ++j) {
      const int q = tid + 256 * j;
      if (q < nxch) {
        const int c = q >> 3, part = q & 7;
#pragma unroll
        for (int x = 0; x < XN; ++x) st16(&xs[x][c * kPitch + part * 16], xnext[x][j]);
      }
    }
    lds_barrier();
    u32x4 acur[RT][2][NLA];
#pragma unroll
    for (int rt = 0; rt < RT; ++rt)
#pragma unroll
      for (int st = 0; st < 2; ++st)
#pragma unroll
        for (int h = 0; h < NLA; ++h) acur[rt][st][h] = anext[rt][st][h];
    if (k0 + KC < ke) load_stage(k0 + KC);

#pragma unroll
    for (int st = 0; st < 2; ++st) {
      u32x4 ahi[RT], alo[RT];
#pragma unroll
      for (int rt = 0; rt < RT; ++rt) {
        if (normA) {
#pragma unroll
          for (int h = 0; h < NLA; ++h) {
            if constexpr (sizeof(TA) == 8) {
              union { u32x4 v; double d[2]; } u;
              u.v = acur[rt][st][h];
              nrm += u.d[0] * u.d[0] + u.d[1] * u.d[1];
            } else {
              const u32x4 v = acur[rt][st][h];
              const double a0 = u2f(v.x), a1 = u2f(v.y), a2 = u2f(v.z), a3 = u2f(v.w);
              nrm += a0 * a0 + a1 * a1 + a2 * a2 + a3 * a3;
            }
          }
        }
        if constexpr (MODE == M_F64 || MODE == M_F32) {
          ahi[rt] = acur[rt][st][0];
        } else {
          to16<MODE>(acur[rt][st][0], acur[rt][st][1], a_scale, ahi[rt], alo[rt]);
        }
      }
#pragma unroll
      for (int ct = 0; ct < NT; ++ct) {
        if (ct < T) {
          const int boff = (16 * ct + li) * kPitch + st * 64 + lg * 16;
          const u32x4 bhi = *(const u32x4*)&xs[0][boff];
          u32x4 blo = bhi;
          if constexpr (XN == 2) blo = *(const u32x4*)&xs[XN - 1][boff];
#pragma unroll
          for (int rt = 0; rt < RT; ++rt) step_mma<MODE>(ahi[rt], alo[rt], bhi, blo, acc[rt][ct]);
        }
      }
    }
  }

  TACC* out = Ypart + (int64_t)blockIdx.y * split_stride;
#pragma unroll
  for (int rt = 0; rt < RT; ++rt)
#pragma unroll
    for (int ct = 0; ct < NT; ++ct)
      if (ct < T) store4<TACC>(out, ldy, 16 * ct + li, row0 + 16 * rt, lg, m, acc[rt][ct], out_scale);

  if (normA) {
    __shared__ double red[4];
    nrm = wave_sum(nrm);
    if (lane == 0) red[wave] = nrm;
    lds_barrier();
    if (tid == 0) normA[blockIdx.y * gridDim.x + blockIdx.x] = (red[0] + red[1]) + (red[2] + red[3]);
  }
}

// ---------------------------------------------------------------------------
// K2: Zpart[s] (lp x n, column-major) = A[rslice(s), :]^T * X[rslice(s), :]
// grid (ceil(n / (64 RT)), S); wave w owns A-columns 16 RT w .. +16 RT.
// A tiles are transposed into LDS in the compute type so both matrix-core
// operands read their contraction index (the rows of A) contiguously.
// ---------------------------------------------------------------------------
template <int MODE, int NT>
__global__ __launch_bounds__(256) void k2_atx(
    const typename Tr<MODE>::TA* __restrict__ A, int64_t lda, int64_t m, int64_t n,
    const typename Tr<MODE>::TC* __restrict__ Xc, const typename Tr<MODE>::TC* __restrict__ Xlo,
    int64_t ldx, int lp, typename Tr<MODE>::TACC* __restrict__ Zpart, int64_t ldz,
    int64_t split_stride, int64_t rchunk, float a_scale, float out_scale, int vec_ok) {
  typedef Tr<MODE> TR;
  typedef typename TR::TA TA;
  typedef typename TR::TC TC;
  typedef typename TR::TACC TACC;
  typedef typename AccOf<TACC>::type ACC;
  constexpr int V = TR::V, KS = 4 * V, KC = 2 * KS, JT = TR::RT, XN = TR::XN;
  constexpr int RB = 16 / sizeof(TC);   // A rows per thread (one 16-byte LDS chunk)
  constexpr int VA = 16 / sizeof(TA);   // A columns per 16-byte global load
  constexpr int XCH = (NT * 16 * 8 + 255) / 256;
  static_assert((KC / RB) * (64 * JT / VA) == 256, "A tile map must use all 256 threads");
  __shared__ __attribute__((aligned(16))) char xs[XN][NT * 16 * kPitch];
  __shared__ __attribute__((aligned(16))) char as[XN][64 * JT * kPitch];

  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63, li = lane & 15, lg = lane >> 4;
  const int T = lp >> 4;
  const int64_t j0 = (int64_t)blockIdx.x * (64 * JT);
  const int64_t ab = (int64_t)blockIdx.y * rchunk;
  const int64_t ae = min(m, ab + rchunk);
  const bool vec = vec_ok != 0;
  const int nxch = lp * 8;
  const int tu = tid >> 5, tv = tid & 31;  // A-tile loader: rows tu*RB.., columns tv*VA..

  ACC acc[JT][NT];
#pragma unroll
  for (int r = 0; r < JT; ++r)
#pragma unroll
    for (int c = 0; c < NT; ++c) acc[r][c] = ACC{0, 0, 0, 0};

  u32x4 anext[RB];
  u32x4 xnext[XN][XCH];

  auto load_stage = [&](int64_t a0) {
#pragma unroll
    for (int r = 0; r < RB; ++r)
      anext[r] = load_a16<TA>(A, lda, a0 + tu * RB + r, j0 + tv * VA, ae, n, vec);
#pragma unroll
    for (int j = 0; j < XCH; ++j) {
      const int q = tid + 256 * j;
      if (q < nxch) {
        const int c = q >> 3, part = q & 7;
        const int64_t off = (int64_t)c * ldx + a0 + part * (16 / (int)sizeof(TC));
        xnext[0][j] = ld16(Xc + off);
        if constexpr (XN == 2) xnext[1][j] = ld16(Xlo + off);
      }
    }
  };

  if (ab < ae) load_stage(ab);
  for (int64_t a0 = ab; a0 < ae; a0 += KC) {
    lds_barrier();
#pragma unroll
    for (int j = 0; j < XCH; ++j) {
      const int q = tid + 256 * j;
      if (q < nxch) {
        const int c = q >> 3, part = q & 7;
#pragma unroll
        for (int x = 0; x < XN; ++x) st16(&xs[x][c * kPitch + part * 16], xnext[x][j]);
      }
    }
    // transpose the A tile: column (tv*VA + e) gets rows tu*RB .. +RB
#pragma unroll
    for (int e = 0; e < VA; ++e) {
      u32x4 hi, lo;
      if constexpr (MODE == M_F64) {
        union { u32x4 v; double d[2]; } s0, s1, o;
        s0.v = anext[0]; s1.v = anext[1];
        o.d[0] = s0.d[e]; o.d[1] = s1.d[e];
        hi = o.v;
      } else if constexpr (MODE == M_F32) {
        union { u32x4 v; float f[4]; } s[4], o;
#pragma unroll
        for (int r = 0; r < 4; ++r) s[r].v = anext[r];
#pragma unroll
        for (int r = 0; r < 4; ++r) o.f[r] = s[r].f[e];
        hi = o.v;
      } else {
        union { u32x4 v; float f[4]; } s[8];
#pragma unroll
        for (int r = 0; r < 8; ++r) s[r].v = anext[r];
        const u32x4 p0 = {__float_as_uint(s[0].f[e]), __float_as_uint(s[1].f[e]),
                          __float_as_uint(s[2].f[e]), __float_as_uint(s[3].f[e])};
        const u32x4 p1 = {__float_as_uint(s[4].f[e]), __float_as_uint(s[5].f[e]),
                          __float_as_uint(s[6].f[e]), __float_as_uint(s[7].f[e])};
        to16<MODE>(p0, p1, a_scale, hi, lo);
      }
      const int off = (tv * VA + e) * kPitch + tu * 16;
      st16(&as[0][off], hi);
      if constexpr (XN == 2) st16(&as[1][off], lo);
    }
    lds_barrier();
    if (a0 + KC < ae) load_stage(a0 + KC);

#pragma unroll
    for (int st = 0; st < 2; ++st) {
      u32x4 ahi[JT], alo[JT];
#pragma unroll
      for (int jt = 0; jt < JT; ++jt) {
        const int aoff = (16 * JT * wave + 16 * jt + li) * kPitch + st * 64 + lg * 16;
        ahi[jt] = *(const u32x4*)&as[0][aoff];
        alo[jt] = ahi[jt];
        if constexpr (XN == 2) alo[jt] = *(const u32x4*)&as[XN - 1][aoff];
      }
#pragma unroll
      for (int ct = 0; ct < NT; ++ct) {
        if (ct < T) {
          const int boff = (16 * ct + li) * kPitch + st * 64 + lg * 16;
          const u32x4 bhi = *(const u32x4*)&xs[0][boff];
          u32x4 blo = bhi;
          if constexpr (XN == 2) blo = *(const u32x4*)&xs[XN - 1][boff];
#pragma unroll
          for (int jt = 0; jt < JT; ++jt) step_mma<MODE>(ahi[jt], alo[jt], bhi, blo, acc[jt][ct]);
        }
      }
    }
  }

  TACC* out = Zpart + (int64_t)blockIdx.y * split_stride;
#pragma unroll
  for (int jt = 0; jt < JT; ++jt)
#pragma unroll
    for (int ct = 0; ct < NT; ++ct)
      if (ct < T)
        store4<TACC>(out, ldz, 16 * ct + li, j0 + 16 * JT * wave + 16 * jt, lg, n, acc[jt][ct],
                     out_scale);
}

// ---------------------------------------------------------------------------
// Launchers
// ---------------------------------------------------------------------------
template <int MODE, int NT>
static hipError_t launch_k1_t(const StreamArgs& a, hipStream_t s) {
  typedef Tr<MODE> TR;
  const int rows = 64 * TR::RT;
  dim3 grid((unsigned)((a.m + rows - 1) / rows), (unsigned)a.splits);
  hipLaunchKernelGGL((k1_ax<MODE, NT>), grid, dim3(256), 0, s, (const typename TR::TA*)a.A, a.lda,
                     a.m, a.n, (const typename TR::TC*)a.X, (const typename TR::TC*)a.Xlo, a.ldx,
                     a.lp, (typename TR::TACC*)a.out, a.ldo, a.split_stride, a.chunk, a.normA,
                     a.a_scale, a.out_scale, a.vec_ok);
  return hipGetLastError();
}

template <int MODE, int NT>
static hipError_t launch_k2_t(const StreamArgs& a, hipStream_t s) {
  typedef Tr<MODE> TR;
  const int cols = 64 * TR::RT;
  dim3 grid((unsigned)((a.n + cols - 1) / cols), (unsigned)a.splits);
  hipLaunchKernelGGL((k2_atx<MODE, NT>), grid, dim3(256), 0, s, (const typename TR::TA*)a.A, a.lda,
                     a.m, a.n, (const typename TR::TC*)a.X, (const typename TR::TC*)a.Xlo, a.ldx,
                     a.lp, (typename TR::TACC*)a.out, a.ldo, a.split_stride, a.chunk, a.a_scale,
                     a.out_scale, a.vec_ok);
  return hipGetLastError();
}

template <int MODE>
static hipError_t dispatch_nt(bool trans, const StreamArgs& a, hipStream_t s) {
  const int T = a.lp / 16;
  if (T <= 2) return trans ? launch_k2_t<MODE, 2>(a, s) : launch_k1_t<MODE, 2>(a, s);
  if (T <= 4) return trans ? launch_k2_t<MODE, 4>(a, s) : launch_k1_t<MODE, 4>(a, s);
  if (T <= 8) return trans ? launch_k2_t<MODE, 8>(a, s) : launch_k1_t<MODE, 8>(a, s);
  if (T <= 16) return trans ? launch_k2_t<MODE, 16>(a, s) : launch_k1_t<MODE, 16>(a, s);
  return hipErrorInvalidValue;
}

int stream_rows_per_block(int mode) { return (mode == M_F64) ? 64 : 128; }
int stream_kc(int mode) { return mode == M_F64 ? 16 : (mode == M_F32 ? 32 : 64); }

hipError_t launch_stream(bool trans, int mode, const StreamArgs& a, hipStream_t s) {
  switch (mode) {
    case M_F64: return dispatch_nt<M_F64>(trans, a, s);
    case M_F32: return dispatch_nt<M_F32>(trans, a, s);
    case M_BF16: return dispatch_nt<M_BF16>(trans, a, s);
    case M_F16: return dispatch_nt<M_F16>(trans, a, s);
    case M_BF16X3: return dispatch_nt<M_BF16X3>(trans, a, s);
  }
  return hipErrorInvalidValue;
}

}  // namespace pbq
