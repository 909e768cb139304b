// Kernels of the wide-sketch path (l > 256: the sample sizes d = 0.2 n and
// 0.3 n of the paper's runtime experiments, Section V-A).  The single-block
// kernels of the narrow path keep an l x l operand in one workgroup; past
// 256 columns the l x l stages are blocked by 256 and their products run
// here: a general matrix-core product with arbitrary strides (trailing
// updates of the blocked Cholesky, the block updates of the triangular
// apply, R2 R1, Q Qt), the sketch generator without the LDS row stage, and
// small helpers of the blocked Cholesky.
#include "common.h"
#include "kernels.h"
#include "launch.h"

namespace pbq {

// ---------------------------------------------------------------------------
// Sketch Omega (column-major lp32 x ld) for any width: one thread per
// element, each from its own Philox block (the same flat index i l + c and
// the same normal as the row-staged generator).
// ---------------------------------------------------------------------------
struct OmegaBigP {
  int64_t n, ld;
  int l, lp32;
  uint64_t seed;
  void* Ot;
  PBQ_GRID;
};

template <typename T, bool B>
__global__ __launch_bounds__(256) void omega_big_kernel(const OmegaBigP* pb, OmegaBigP ps) {
  bool past;
  const OmegaBigP p = kparams<B>(pb, ps, past);
  if (past) return;
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int c = blockIdx.y;
  if (i >= p.ld) return;
  double v = 0.0;
  if (c < p.l && i < p.n) {
    const uint64_t t = (uint64_t)i * (uint64_t)p.l + (uint64_t)c;
    v = sketch_value(normal_at(t, 0u, 0u, p.seed));
  }
  ((T*)p.Ot)[(int64_t)c * p.ld + i] = (T)v;
}

hipError_t launch_omega_big(bool f64, int64_t n, int l, int lp32, uint64_t seed, void* Ot, int64_t ld,
                            hipStream_t s) {
  dim3 grid((unsigned)((ld + 255) / 256), (unsigned)lp32);
  OmegaBigP p{n, ld, l, lp32, seed, Ot};
  if (f64) return launch_k(omega_big_kernel<double, false>, omega_big_kernel<double, true>, grid, dim3(256), s, p);
  return launch_k(omega_big_kernel<float, false>, omega_big_kernel<float, true>, grid, dim3(256), s, p);
}

// ---------------------------------------------------------------------------
// Cout(i, j) = beta Cin(i, j) + alpha sum_k A(i, k) B(k, j),  i < M, j < N,
// with A(i, k) = A[i sai + k sak], B(k, j) = B[k sbk + j sbj],
// C(i, j) = C[i sci + j scj] (Cin and Cout may be the same matrix).
// 64 x 64 output tile per workgroup of four waves (32 x 32 each, four 16 x 16
// matrix-core tiles); the k loop stages 16-deep slices of A and B in LDS in
// the accumulation type, the next slice's global loads in flight while the
// current one is multiplied.  TA/TB/TC: storage types; ACC: float (FP32
// matrix core) or double (FP64 matrix core).  upper: skip the output tiles
// that lie wholly below the diagonal (the trailing update of a symmetric
// matrix of which only the upper triangle is read).
// ---------------------------------------------------------------------------
struct GemmGP {
  int64_t M, N, K;
  const void* A;
  int64_t sai, sak;
  const void* B;
  int64_t sbk, sbj;
  const void* Cin;
  void* Cout;
  int64_t sci, scj;
  double alpha, beta;
  int upper;
  PBQ_GRID;
};

constexpr int kGB = 64, kGK = 16;

template <typename TA, typename TB, typename TC, typename ACC, bool B>
__global__ __launch_bounds__(256) void gemm_kernel(const GemmGP* pb, GemmGP ps) {
  bool past;
  const GemmGP p = kparams<B>(pb, ps, past);
  if (past) return;
  const int64_t i0 = (int64_t)blockIdx.y * kGB, j0 = (int64_t)blockIdx.x * kGB;
  if (p.upper && i0 >= j0 + kGB) return;   // wholly below the diagonal
  typedef typename Vec4<ACC>::type V4;
  __shared__ ACC As[2][kGK][kGB + 4];
  __shared__ ACC Bs[2][kGK][kGB + 4];
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63, li = lane & 15, lg = lane >> 4;
  const TA* A = (const TA*)p.A;
  const TB* Bm = (const TB*)p.B;
  // load maps: 4 elements per thread for each tile, along the unit stride
  const bool a_i = p.sai == 1, b_j = p.sbj == 1;
  int ai[4], ak[4], bk[4], bj[4];
#pragma unroll
  for (int e = 0; e < 4; ++e) {
    if (a_i) { ak[e] = tid >> 4; ai[e] = (tid & 15) * 4 + e; }
    else { ai[e] = tid >> 2; ak[e] = (tid & 3) * 4 + e; }
    if (b_j) { bk[e] = tid >> 4; bj[e] = (tid & 15) * 4 + e; }
    else { bj[e] = tid >> 2; bk[e] = (tid & 3) * 4 + e; }
  }
  ACC ra[4], rb[4];
  auto gload = [&](int64_t k0) __attribute__((always_inline)) {
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const int64_t gi = i0 + ai[e], gk = k0 + ak[e];
      ra[e] = (gi < p.M && gk < p.K) ? (ACC)A[gi * p.sai + gk * p.sak] : ACC(0);
      const int64_t hk = k0 + bk[e], hj = j0 + bj[e];
      rb[e] = (hk < p.K && hj < p.N) ? (ACC)Bm[hk * p.sbk + hj * p.sbj] : ACC(0);
    }
  };
  auto sstore = [&](int buf) __attribute__((always_inline)) {
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      As[buf][ak[e]][ai[e]] = ra[e];
      Bs[buf][bk[e]][bj[e]] = rb[e];
    }
  };
  V4 acc[2][2];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
      for (int r = 0; r < 4; ++r) acc[a][b][r] = ACC(0);
  const int wi = (wave >> 1) * 32, wj = (wave & 1) * 32;
  const int nk = (int)((p.K + kGK - 1) / kGK);
  gload(0);
  sstore(0);
  __syncthreads();
  for (int kt = 0; kt < nk; ++kt) {
    const int buf = kt & 1;
    if (kt + 1 < nk) gload((int64_t)(kt + 1) * kGK);
#pragma unroll
    for (int kk = 0; kk < kGK / 4; ++kk) {
      const int k = kk * 4 + lg;
      const ACC a0 = As[buf][k][wi + li], a1 = As[buf][k][wi + 16 + li];
      const ACC b0 = Bs[buf][k][wj + li], b1 = Bs[buf][k][wj + 16 + li];
      acc[0][0] = mma_native(a0, b0, acc[0][0]);
      acc[0][1] = mma_native(a0, b1, acc[0][1]);
      acc[1][0] = mma_native(a1, b0, acc[1][0]);
      acc[1][1] = mma_native(a1, b1, acc[1][1]);
    }
    if (kt + 1 < nk) sstore(buf ^ 1);
    __syncthreads();
  }
  const TC* Cin = (const TC*)p.Cin;
  TC* Cout = (TC*)p.Cout;
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int64_t i = i0 + wi + 16 * a + acc_row<ACC>(lg, r), j = j0 + wj + 16 * b + li;
        if (i < p.M && j < p.N) {
          const int64_t off = i * p.sci + j * p.scj;
          double v = p.alpha * (double)acc[a][b][r];
          if (p.beta != 0.0) v += p.beta * (double)Cin[off];
          Cout[off] = (TC)v;
        }
      }
}

// dt: 0 = float storage with FP32 accumulation, 1 = double storage and FP64
// accumulation, 2 = float A and B with FP64 accumulation into double C,
// 3 = float A and C, double B, FP32 accumulation.
hipError_t launch_gemm(int dt, int64_t M, int64_t N, int64_t K, const void* A, int64_t sai, int64_t sak,
                       const void* B, int64_t sbk, int64_t sbj, const void* Cin, void* Cout, int64_t sci,
                       int64_t scj, double alpha, double beta, bool upper, hipStream_t s) {
  if (M <= 0 || N <= 0) return hipSuccess;
  if ((M + kGB - 1) / kGB > 65535) return hipErrorInvalidValue;
  dim3 grid((unsigned)((N + kGB - 1) / kGB), (unsigned)((M + kGB - 1) / kGB));
  GemmGP p{M, N, K, A, sai, sak, B, sbk, sbj, Cin ? Cin : Cout, Cout, sci, scj, alpha, Cin ? beta : 0.0,
           upper ? 1 : 0};
  switch (dt) {
    case 0:
      return launch_k(gemm_kernel<float, float, float, float, false>, gemm_kernel<float, float, float, float, true>,
                      grid, dim3(256), s, p);
    case 1:
      return launch_k(gemm_kernel<double, double, double, double, false>,
                      gemm_kernel<double, double, double, double, true>, grid, dim3(256), s, p);
    case 2:
      return launch_k(gemm_kernel<float, float, double, double, false>,
                      gemm_kernel<float, float, double, double, true>, grid, dim3(256), s, p);
    case 3:
      return launch_k(gemm_kernel<float, double, float, float, false>,
                      gemm_kernel<float, double, float, float, true>, grid, dim3(256), s, p);
  }
  return hipErrorInvalidValue;
}

// ---------------------------------------------------------------------------
// Helpers of the blocked Cholesky.
// ---------------------------------------------------------------------------
struct DiagP {
  const double* G;
  int64_t ldg;
  int l, lp;
  double* d;
  PBQ_GRID;
};

// d[i] = G[i][i] for i < l, 0 for l <= i < lp (the unmodified diagonal that
// every block's dependence test is measured against)
template <bool B>
__global__ void save_diag_kernel(const DiagP* pb, DiagP ps) {
  bool past;
  const DiagP p = kparams<B>(pb, ps, past);
  if (past) return;
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < p.lp) p.d[i] = i < p.l ? p.G[(int64_t)i * p.ldg + i] : 0.0;
}

hipError_t launch_save_diag(const double* G, int64_t ldg, int l, int lp, double* d, hipStream_t s) {
  DiagP p{G, ldg, l, lp, d};
  return launch_k(save_diag_kernel<false>, save_diag_kernel<true>, dim3((unsigned)((lp + 255) / 256)), dim3(256), s, p);
}

struct DepRowsP {
  double* R;
  int64_t ldr;
  int rows;
  int64_t cols;
  const int* dep;
  PBQ_GRID;
};

// Row i (< rows) of R (cols wide) becomes 0 where dep[i] is set: a column
// that carries no new direction has a zero row in the true factor.
template <bool B>
__global__ void zero_dep_rows_kernel(const DepRowsP* pb, DepRowsP ps) {
  bool past;
  const DepRowsP p = kparams<B>(pb, ps, past);
  if (past) return;
  if (p.dep[p.rows] == 0) return;   // count of dependent columns of this block
  const int i = blockIdx.y;
  if (!p.dep[i]) return;
  for (int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; j < p.cols; j += (int64_t)p.gx * blockDim.x)
    p.R[(int64_t)i * p.ldr + j] = 0.0;
}

hipError_t launch_zero_dep_rows(double* R, int64_t ldr, int rows, int64_t cols, const int* dep, hipStream_t s) {
  if (cols <= 0) return hipSuccess;
  DepRowsP p{R, ldr, rows, cols, dep};
  return launch_k(zero_dep_rows_kernel<false>, zero_dep_rows_kernel<true>,
                  dim3((unsigned)((cols + 255) / 256 < 64 ? (cols + 255) / 256 : 64), (unsigned)rows), dim3(256), s, p);
}

struct CastP {
  const double* in;
  float* out;
  int64_t count;
  PBQ_GRID;
};

template <bool B>
__global__ void cast_f32_kernel(const CastP* pb, CastP ps) {
  bool past;
  const CastP p = kparams<B>(pb, ps, past);
  if (past) return;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < p.count; i += (int64_t)p.gx * blockDim.x)
    p.out[i] = (float)p.in[i];
}

hipError_t launch_cast_f32(const double* in, float* out, int64_t count, hipStream_t s) {
  if (count <= 0) return hipSuccess;
  CastP p{in, out, count};
  const int64_t g = (count + 255) / 256;
  return launch_k(cast_f32_kernel<false>, cast_f32_kernel<true>, dim3((unsigned)(g < 1024 ? g : 1024)), dim3(256), s, p);
}

}  // namespace pbq
