// Tall-skinny kernels of PbP-QLP: the sketch generator, operand conversion,
// split-K reduction, and the two halves of a CholeskyQR sweep that touch the
// tall matrix (Gram accumulation and the triangular apply), plus the final
// right-multiplication Q Qt (Algorithm 1, last step: P := Pbar Pt).
//
// Column-major tall buffers: row c of a lp32 x ld buffer is column c of the
// tall matrix; every producer writes zeros in rows [l, lp) and in columns
// [len, ld) so consumers can read whole 64-element groups without checks.
#include "common.h"
#include "kernels.h"
#include "launch.h"
#include "../../include/pbpqlp.h"

namespace pbq {

// ---------------------------------------------------------------------------
// Sketch Omega (randn(n, l) of Algorithm 1, for A^T): element (i, c) is the
// normal of flat index t = i*l + c from Philox block t/4, slot t%4, rounded to
// bfloat16 and flushed below 2^-14.
// ---------------------------------------------------------------------------
__device__ __forceinline__ double omega_elem(int64_t i, int c, int l, uint64_t seed) {
  const uint64_t t = (uint64_t)i * (uint64_t)l + (uint64_t)c;
  return sketch_value(normal_at(t, 0u, 0u, seed));
}

struct OmegaP {
  int64_t n;
  int l, lp32;
  uint64_t seed;
  void* Ot;
  int64_t ld;
  PBQ_GRID;
};

// One block per kOmegaRows rows of Omega: every Philox block that touches those
// rows is generated once (four normals per call), staged row-major in LDS and
// written column-major with rows contiguous; padding rows and columns get 0.
constexpr int kOmegaRows = 32;

template <typename T, bool B>
__global__ __launch_bounds__(256) void omega_cm_kernel(const OmegaP* pb, OmegaP ps) {
  bool past;
  const OmegaP p = kparams<B>(pb, ps, past);
  if (past) return;
  __shared__ T tile[kOmegaRows * kMaxL];
  const int64_t i0 = (int64_t)blockIdx.x * kOmegaRows;
  if (i0 >= p.ld) return;
  const int64_t rows = min((int64_t)kOmegaRows, max((int64_t)0, p.n - i0));
  const uint64_t t0 = (uint64_t)i0 * (uint64_t)p.l;
  const uint64_t t1 = t0 + (uint64_t)rows * (uint64_t)p.l;   // flat indices [t0, t1)
  if (t1 > t0) {
    const uint64_t b0 = t0 >> 2, b1 = (t1 + 3) >> 2;
    for (uint64_t b = b0 + threadIdx.x; b < b1; b += blockDim.x) {
      double v[4];
      normals4_at(b, 0u, 0u, p.seed, v);
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const uint64_t t = 4 * b + e;
        if (t >= t0 && t < t1) tile[t - t0] = (T)sketch_value(v[e]);
      }
    }
  }
  __syncthreads();
  T* Ot = (T*)p.Ot;
  for (int q = threadIdx.x; q < p.lp32 * kOmegaRows; q += blockDim.x) {
    const int c = q / kOmegaRows, r = q % kOmegaRows;
    const int64_t i = i0 + r;
    if (i >= p.ld) continue;
    Ot[(int64_t)c * p.ld + i] = (c < p.l && r < rows) ? tile[r * p.l + c] : T(0);
  }
}

hipError_t launch_omega_cm(bool f64, int64_t n, int l, int lp32, uint64_t seed, void* Ot,
                           int64_t ld, hipStream_t s) {
  dim3 grid((unsigned)((ld + kOmegaRows - 1) / kOmegaRows));
  OmegaP p{n, l, lp32, seed, Ot, ld};
  if (f64) return launch_k(omega_cm_kernel<double, false>, omega_cm_kernel<double, true>, grid, dim3(256), s, p);
  return launch_k(omega_cm_kernel<float, false>, omega_cm_kernel<float, true>, grid, dim3(256), s, p);
}


// ---------------------------------------------------------------------------
// FP32 operand -> 16-bit compute type (hi, and lo = x - hi for BF16X3).
// ---------------------------------------------------------------------------
struct ConvertP {
  const float* X;
  int64_t ld, len;
  int l;
  float scale;
  void* hi;
  void* lo;
  PBQ_GRID;
};

template <int MODE, bool B>
__global__ void convert_kernel(const ConvertP* pb, ConvertP ps) {
  bool past;
  const ConvertP p = kparams<B>(pb, ps, past);
  if (past) return;
  const int c = blockIdx.y;
  const int64_t i0 = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) * 4;
  if (i0 >= p.ld) return;
  float v[4];
#pragma unroll
  for (int e = 0; e < 4; ++e) {
    const int64_t i = i0 + e;
    v[e] = (c < p.l && i < p.len) ? p.X[(int64_t)c * p.ld + i] * p.scale : 0.0f;
  }
  if constexpr (MODE == M_F16) {
    _Float16* hi = (_Float16*)p.hi;
    f16x4 h = {(_Float16)v[0], (_Float16)v[1], (_Float16)v[2], (_Float16)v[3]};
    *(f16x4*)(hi + (int64_t)c * p.ld + i0) = h;
  } else {
    __bf16* hi = (__bf16*)p.hi;
    bf16x4 h = {(__bf16)v[0], (__bf16)v[1], (__bf16)v[2], (__bf16)v[3]};
    *(bf16x4*)(hi + (int64_t)c * p.ld + i0) = h;
    if constexpr (MODE == M_BF16X3) {
      __bf16* lo = (__bf16*)p.lo;
      bf16x4 w = {(__bf16)(v[0] - (float)h[0]), (__bf16)(v[1] - (float)h[1]),
                  (__bf16)(v[2] - (float)h[2]), (__bf16)(v[3] - (float)h[3])};
      *(bf16x4*)(lo + (int64_t)c * p.ld + i0) = w;
    }
  }
}

hipError_t launch_convert(int mode, const float* X, int64_t ld, int64_t len, int l, int lp32,
                          float scale, void* hi, void* lo, hipStream_t s) {
  dim3 grid((unsigned)((ld / 4 + 255) / 256), (unsigned)lp32);
  ConvertP p{X, ld, len, l, scale, hi, lo};
  switch (mode) {
    case M_BF16: return launch_k(convert_kernel<M_BF16, false>, convert_kernel<M_BF16, true>, grid, dim3(256), s, p);
    case M_F16: return launch_k(convert_kernel<M_F16, false>, convert_kernel<M_F16, true>, grid, dim3(256), s, p);
    case M_BF16X3: return launch_k(convert_kernel<M_BF16X3, false>, convert_kernel<M_BF16X3, true>, grid, dim3(256), s, p);
  }
  return hipErrorInvalidValue;
}

// ---------------------------------------------------------------------------
// Split-K reduction in a fixed order (bitwise reproducible).
// ---------------------------------------------------------------------------
struct ReduceP {
  const void* part;
  int64_t stride;
  int S;
  int64_t ld, len;   // partials: leading dimension, rows summed (later rows are 0)
  void* out;
  int64_t ldo;
  int64_t wlen;      // rows written: len rounded to the buffer's padding, or one panel's rows
  PBQ_GRID;
};

template <typename T, bool B>
__global__ void splitk_reduce_kernel(const ReduceP* pb, ReduceP ps) {
  bool past;
  const ReduceP p = kparams<B>(pb, ps, past);
  if (past) return;
  const T* part = (const T*)p.part;
  T* out = (T*)p.out;
  const int c = blockIdx.y;
  const int64_t i0 = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) * 4;
  if (i0 >= p.wlen) return;
  T acc[4] = {0, 0, 0, 0};
  if (i0 + 3 < p.len) {
    for (int sp = 0; sp < p.S; ++sp) {
      const T* q = part + (int64_t)sp * p.stride + (int64_t)c * p.ld + i0;
#pragma unroll
      for (int e = 0; e < 4; ++e) acc[e] += q[e];
    }
  } else {
    for (int sp = 0; sp < p.S; ++sp) {
      const T* q = part + (int64_t)sp * p.stride + (int64_t)c * p.ld + i0;
#pragma unroll
      for (int e = 0; e < 4; ++e)
        if (i0 + e < p.len) acc[e] += q[e];
    }
  }
#pragma unroll
  for (int e = 0; e < 4; ++e)
    if (i0 + e < p.wlen) out[(int64_t)c * p.ldo + i0 + e] = acc[e];
}

hipError_t launch_splitk_reduce(bool f64, const void* part, int64_t stride, int S, int64_t ld,
                                int lp, int64_t len, void* out, int64_t ldo, hipStream_t s,
                                int64_t wlen) {
  if (wlen < 0) wlen = ldo;
  dim3 grid((unsigned)((wlen + 1023) / 1024), (unsigned)lp);
  ReduceP p{part, stride, S, ld, len, out, ldo, wlen};
  if (f64) return launch_k(splitk_reduce_kernel<double, false>, splitk_reduce_kernel<double, true>, grid, dim3(256), s, p);
  return launch_k(splitk_reduce_kernel<float, false>, splitk_reduce_kernel<float, true>, grid, dim3(256), s, p);
}

// ---------------------------------------------------------------------------
// Gram G = X X^T of a column-major lp x len operand, accumulated in FP64 on
// the FP64 matrix cores (FP32 inputs are exact in FP64).  Grid: (upper
// triangle of 32x32 blocks) x (contraction splits).  Each of the four waves
// computes the whole 32x32 block (four 16x16 tiles, three on the diagonal)
// over every fourth slice of the split, so one load of the two row panels
// feeds four products and the next two slices are in flight while the
// current one is multiplied; the waves' blocks are then summed through LDS in a fixed
// order.  Partials are summed by gram_reduce in a fixed order.
// ---------------------------------------------------------------------------
__host__ __device__ inline int npairs_of(int nb) { return nb * (nb + 1) / 2; }

int gram_splits(int64_t len, int lp, int target) {
  const int nb = (lp + 31) / 32;
  const int np = npairs_of(nb);
  int64_t S = (target + np - 1) / np;            // aim at ~target workgroups
  const int64_t maxS = (len + 255) / 256;        // at least 256 rows per split
  // from 8 splits up, a multiple of 8 (to the nearest) lets the kernel keep
  // each row range on one XCD
  if (S >= 8) {
    const int64_t S8 = (S + 4) / 8 * 8;
    if (S8 <= maxS) S = S8;
  }
  if (S > maxS) S = maxS;
  if (S < 1) S = 1;
  return (int)S;
}

size_t gram_partial_elems(int64_t len, int lp, int target) {
  const int nb = (lp + 31) / 32;
  return (size_t)gram_splits(len, lp, target) * npairs_of(nb) * 1024;
}

struct GramP {
  const void* X;
  int64_t ld, len;
  int lp;
  int64_t kchunk;
  double* part;
  PBQ_GRID;
};

template <typename T, bool B>
__global__ __launch_bounds__(256) void gram_partial_kernel(const GramP* pb, GramP ps) {
  bool past;
  const GramP prm = kparams<B>(pb, ps, past);
  if (past) return;
  const T* X = (const T*)prm.X;
  const int64_t ld = prm.ld, len = prm.len;
  const int lp = prm.lp;
  constexpr int VV = 16 / sizeof(T);
  constexpr int STEP = 4 * VV;  // contraction indices per slice (four lane groups)
  // block -> (pair p, row range sp).  Workgroups are dealt to the eight XCDs
  // round-robin by linear id; when the split count is a multiple of 8 the np
  // blocks of one row range go to the same XCD, whose L2 then serves their
  // repeated reads of those rows (each column block is read by nb blocks).
  int p = blockIdx.x, sp = blockIdx.y;
  if constexpr (!B) {
    if ((prm.gy & 7) == 0) {
      const int L = blockIdx.x + prm.gx * blockIdx.y;
      const int slot = L >> 3;
      p = slot % prm.gx;
      sp = (L & 7) + 8 * (slot / prm.gx);
    }
  }
  int bj = 0;
  while ((bj + 1) * (bj + 2) / 2 <= p) ++bj;
  const int bi = p - bj * (bj + 1) / 2;
  const bool dg = bi == bj;
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63, li = lane & 15, lg = lane >> 4;
  const int64_t kb = (int64_t)sp * prm.kchunk, ke = min(len, kb + prm.kchunk);
  const int r0 = 32 * bi + li, r1 = r0 + 16, c0 = 32 * bj + li, c1 = c0 + 16;
  const T* pI0 = X + (int64_t)r0 * ld;
  const T* pI1 = X + (int64_t)r1 * ld;
  const T* pJ0 = X + (int64_t)c0 * ld;
  const T* pJ1 = X + (int64_t)c1 * ld;
  const bool okI0 = r0 < lp, okI1 = r1 < lp, okJ0 = c0 < lp, okJ1 = c1 < lp;
  auto ld_slice = [&](const T* base, bool ok, int64_t k, T out[VV]) __attribute__((always_inline)) {
    if (ok && k + VV <= ke) {
      union { u32x4 v; T e[VV]; } u;
      u.v = ld16(base + k);
#pragma unroll
      for (int e = 0; e < VV; ++e) out[e] = u.e[e];
    } else {
#pragma unroll
      for (int e = 0; e < VV; ++e) out[e] = (ok && k + e < ke) ? base[k + e] : T(0);
    }
  };
  f64x4 a00 = {0, 0, 0, 0}, a01 = a00, a10 = a00, a11 = a00;
  // masked loads (any iteration)
  auto load4 = [&](int64_t at, T (*dst)[VV]) __attribute__((always_inline)) {
    const int64_t k = at + lg * VV;
    ld_slice(pI0, okI0, k, dst[0]);
    ld_slice(pI1, okI1, k, dst[1]);
    ld_slice(pJ0, okJ0, k, dst[2]);
    ld_slice(pJ1, okJ1, k, dst[3]);
  };
  // unconditional loads of an iteration that lies wholly in [kb, ke); a
  // padding column block (r1 or c1 >= lp, uniform) reads its partner column,
  // whose products are skipped
  const T* qI1 = okI1 ? pI1 : pI0;
  const T* qJ1 = okJ1 ? pJ1 : pJ0;
  auto load4f = [&](int64_t at, T (*dst)[VV]) __attribute__((always_inline)) {
    const int64_t k = at + lg * VV;
    union { u32x4 v; T e[VV]; } u0, u1, u2, u3;
    u0.v = ld16(pI0 + k);
    u1.v = ld16(qI1 + k);
    u2.v = ld16(pJ0 + k);
    u3.v = ld16(qJ1 + k);
#pragma unroll
    for (int e = 0; e < VV; ++e) {
      dst[0][e] = u0.e[e];
      dst[1][e] = u1.e[e];
      dst[2][e] = u2.e[e];
      dst[3][e] = u3.e[e];
    }
  };
  auto compute = [&](const T (*c)[VV]) __attribute__((always_inline)) {
#pragma unroll
    for (int e = 0; e < VV; ++e) {
      const double x0 = (double)c[0][e], x1 = (double)c[1][e];
      const double y0 = (double)c[2][e], y1 = (double)c[3][e];
      // tiles wholly in the padding columns (lp < 32 nb) stay zero: skipped
      // (block-uniform tests, lp is a multiple of 16)
      a00 = mma_f64(x0, y0, a00);
      if (okJ1) a01 = mma_f64(x0, y1, a01);
      if (!dg && okI1) a10 = mma_f64(x1, y0, a10);
      if (okI1 && okJ1) a11 = mma_f64(x1, y1, a11);
    }
  };
  // Wave-uniform iterations i = 0 .. nit-1 over the slices starting at
  // b0 + 4 STEP i; the first nfull lie wholly in [kb, ke).  For FP32, full
  // iterations run with unconditional loads two iterations ahead in three
  // rotating buffers (no masked load in the loop, so the wait before each
  // iteration's products covers only its own loads); the rest run with
  // masked loads.  FP64 keeps the masked loop throughout: on the wide
  // L2-bound Grams (thousands of block pairs) the deeper effective prefetch
  // made it slower (l = 7500: 14.6 -> 19.0 ms per launch).
  const int64_t b0 = kb + (int64_t)wave * STEP;
  const int nit = b0 < ke ? (int)((ke - b0 + 4 * STEP - 1) / (4 * STEP)) : 0;
  const int nfull = b0 + STEP <= ke ? (int)((ke - b0 - STEP) / (4 * STEP)) + 1 : 0;
  auto at = [&](int i) { return b0 + (int64_t)i * 4 * STEP; };
  T B0[4][VV], B1[4][VV], B2[4][VV];
  int it = 0;
  if (sizeof(T) == 4 && nfull >= 5) {
    load4f(at(0), B0);
    load4f(at(1), B1);
    do {
      load4f(at(it + 2), B2);
      compute(B0);
      load4f(at(it + 3), B0);
      compute(B1);
      load4f(at(it + 4), B1);
      compute(B2);
      it += 3;
    } while (it + 4 < nfull);
  } else {
    if (nit > 0) load4(at(0), B0);
    if (nit > 1) load4(at(1), B1);
  }
  // the remaining iterations: B0 holds iteration it, B1 iteration it + 1
  for (; it < nit; ++it) {
    if (it + 2 < nit) load4(at(it + 2), B2);
    compute(B0);
#pragma unroll
    for (int q = 0; q < 4; ++q)
#pragma unroll
      for (int e = 0; e < VV; ++e) {
        B0[q][e] = B1[q][e];
        B1[q][e] = B2[q][e];
      }
  }
  // sum the four waves' blocks in LDS (fixed order), write the 32x32 partial
  __shared__ double red[4][1024];
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const int row = acc_row<double>(lg, r);
    red[wave][row * 32 + li] = a00[r];
    red[wave][row * 32 + 16 + li] = a01[r];
    red[wave][(16 + row) * 32 + 16 + li] = a11[r];
    // on the diagonal block the lower-left tile is the transpose of the upper-right one
    red[wave][dg ? (16 + li) * 32 + row : (16 + row) * 32 + li] = dg ? a01[r] : a10[r];
  }
  __syncthreads();
  double* out = prm.part + ((int64_t)sp * prm.gx + p) * 1024;
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int e = tid + 256 * q;
    out[e] = (red[0][e] + red[1][e]) + (red[2][e] + red[3][e]);
  }
}

struct GramReduceP {
  const double* part;
  int S, np, lp;
  double* G;
  int64_t ldg;
  // optional identity test of a later CholeskyQR sweep: block (x, row i)
  // writes far[i gx + x] = 1 when some |G_ij - delta_ij| > tol (i, j < l)
  int* far;
  int l;
  double tol;
  PBQ_GRID;
};

template <bool B>
__global__ void gram_reduce_kernel(const GramReduceP* pb, GramReduceP ps) {
  bool past;
  const GramReduceP p = kparams<B>(pb, ps, past);
  if (past) return;
  const int i = blockIdx.y;
  const int j0 = blockIdx.x * blockDim.x + threadIdx.x;
  const int j = j0 < p.lp ? j0 : p.lp - 1;   // lanes past lp compute a valid entry, write nothing
  int bi = i >> 5, bj = j >> 5, ii = i & 31, jj = j & 31;
  if (bi > bj) {
    int t = bi; bi = bj; bj = t;
    t = ii; ii = jj; jj = t;
  }
  const int pr = bj * (bj + 1) / 2 + bi;
  const double* src = p.part + (int64_t)pr * 1024 + ii * 32 + jj;
  const int64_t stride = (int64_t)p.np * 1024;
  // four independent partial sums keep several loads in flight; the order is fixed
  double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0;
  int sp = 0;
  for (; sp + 4 <= p.S; sp += 4) {
    s0 += src[(int64_t)(sp + 0) * stride];
    s1 += src[(int64_t)(sp + 1) * stride];
    s2 += src[(int64_t)(sp + 2) * stride];
    s3 += src[(int64_t)(sp + 3) * stride];
  }
  for (; sp < p.S; ++sp) s0 += src[(int64_t)sp * stride];
  const double g = (s0 + s1) + (s2 + s3);
  if (j0 < p.lp) p.G[(int64_t)i * p.ldg + j] = g;
  if (p.far) {
    const bool far = j0 < p.l && i < p.l && !(fabs(g - (i == j ? 1.0 : 0.0)) <= p.tol);
    const uint64_t bal = __builtin_amdgcn_ballot_w64(far);
    if (threadIdx.x == 0) p.far[(int64_t)i * p.gx + blockIdx.x] = bal != 0;
  }
}

hipError_t launch_gram(bool f64, const void* X, int64_t ld, int64_t len, int lp, double* part,
                       double* G, int64_t ldg, int target, hipStream_t s, int* far, int l, double tol) {
  const int nb = (lp + 31) / 32;
  const int np = npairs_of(nb);
  const int S = gram_splits(len, lp, target);
  int64_t kchunk = (len + S - 1) / S;
  kchunk = (kchunk + 15) / 16 * 16;
  dim3 grid((unsigned)np, (unsigned)S);
  GramP p{X, ld, len, lp, kchunk, part};
  hipError_t e = f64 ? launch_k(gram_partial_kernel<double, false>, gram_partial_kernel<double, true>, grid, dim3(256), s, p)
                     : launch_k(gram_partial_kernel<float, false>, gram_partial_kernel<float, true>, grid, dim3(256), s, p);
  if (e != hipSuccess) return e;
  GramReduceP r{part, S, np, lp, G, ldg, far, l, tol};
  return launch_k(gram_reduce_kernel<false>, gram_reduce_kernel<true>, dim3((unsigned)((lp + 63) / 64), (unsigned)lp),
                  dim3(64), s, r);
}

// ---------------------------------------------------------------------------
// Layout conversions between the caller's row-major tall matrices and the
// internal column-major buffers (32 x 32 tiles through LDS).
// ---------------------------------------------------------------------------
template <typename T>
__global__ void rm_to_cm_kernel(const T* __restrict__ X, int64_t ldx, int64_t len, int l,
                                int lp32, T* __restrict__ Xt, int64_t ldt) {
  __shared__ T tile[32][33];
  const int64_t i0 = (int64_t)blockIdx.x * 32;   // tall index
  const int c0 = blockIdx.y * 32;                 // column index
  const int tx = threadIdx.x, ty = threadIdx.y;   // 32 x 8
  for (int r = ty; r < 32; r += 8) {
    const int64_t i = i0 + r;
    const int c = c0 + tx;
    tile[r][tx] = (i < len && c < l) ? X[i * ldx + c] : T(0);
  }
  __syncthreads();
  for (int r = ty; r < 32; r += 8) {
    const int c = c0 + r;
    const int64_t i = i0 + tx;
    if (c < lp32 && i < ldt) Xt[(int64_t)c * ldt + i] = tile[tx][r];
  }
}

template <typename T>
__global__ void cm_to_rm_kernel(const T* __restrict__ Xt, int64_t ldt, int64_t len, int l,
                                T* __restrict__ X, int64_t ldx) {
  __shared__ T tile[32][33];
  const int64_t i0 = (int64_t)blockIdx.x * 32;
  const int c0 = blockIdx.y * 32;
  const int tx = threadIdx.x, ty = threadIdx.y;
  for (int r = ty; r < 32; r += 8) {
    const int c = c0 + r;
    const int64_t i = i0 + tx;
    tile[r][tx] = (c < l && i < len) ? Xt[(int64_t)c * ldt + i] : T(0);
  }
  __syncthreads();
  for (int r = ty; r < 32; r += 8) {
    const int64_t i = i0 + r;
    const int c = c0 + tx;
    if (i < len && c < l) X[i * ldx + c] = tile[tx][r];
  }
}

hipError_t launch_rm_to_cm(bool f64, const void* X, int64_t ldx, int64_t len, int l, int lp32,
                           void* Xt, int64_t ldt, hipStream_t s) {
  dim3 grid((unsigned)((ldt + 31) / 32), (unsigned)((lp32 + 31) / 32));
  if (f64)
    hipLaunchKernelGGL(rm_to_cm_kernel<double>, grid, dim3(32, 8), 0, s, (const double*)X, ldx,
                       len, l, lp32, (double*)Xt, ldt);
  else
    hipLaunchKernelGGL(rm_to_cm_kernel<float>, grid, dim3(32, 8), 0, s, (const float*)X, ldx, len,
                       l, lp32, (float*)Xt, ldt);
  return hipGetLastError();
}

hipError_t launch_cm_to_rm(bool f64, const void* Xt, int64_t ldt, int64_t len, int l, void* X,
                           int64_t ldx, hipStream_t s) {
  dim3 grid((unsigned)((len + 31) / 32), (unsigned)((l + 31) / 32));
  if (f64)
    hipLaunchKernelGGL(cm_to_rm_kernel<double>, grid, dim3(32, 8), 0, s, (const double*)Xt, ldt,
                       len, l, (double*)X, ldx);
  else
    hipLaunchKernelGGL(cm_to_rm_kernel<float>, grid, dim3(32, 8), 0, s, (const float*)Xt, ldt, len,
                       l, (float*)X, ldx);
  return hipGetLastError();
}

}  // namespace pbq
