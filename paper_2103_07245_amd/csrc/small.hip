// l x l stages of PbP-QLP in FP64: the Cholesky factor of a Gram matrix (the
// small half of a CholeskyQR sweep, i.e. of orth()/qr() in Algorithm 1),
// small products (R2 R1, U2 U1) and the result record.
#include "common.h"
#include "kernels.h"
#include "../../include/pbpqlp.h"

namespace pbq {

// ---------------------------------------------------------------------------
// Upper Cholesky G = R^T R of an lp x lp Gram (only the first l columns are
// live; the rest is padding), one workgroup of 512 threads, blocked by 16.
// The upper triangle lives in registers as 16x16 tiles in the FP64
// matrix-core accumulator layout: wave w owns tile rows w and 15 - w
// (17 tiles for every wave), so every register index is a compile-time
// constant.  For each 16-column panel J:
//   A. the owner of tile (J,J) factors it in one wave (diag_factor), forms
//      the "apply" form of R_JJ and its inverse W_J;
//   B. the owner of row J solves R_JK = W_J^T G_JK on the FP64 matrix core;
//   C. every owner applies the rank-16 update G_IK -= R_JI^T R_JK (I,K > J).
// Two barriers per panel; no global memory inside the panel loop.
//
// Dependent columns: if the pivot satisfies !(d_k > eps * G_kk) (this also
// catches d_k <= 0, G_kk = 0 and NaN), column k carries no new direction.
// The "true" factor Rt gets a zero diagonal and a zero row k; the "apply"
// factor Ra gets an identity row and column k, so the triangular apply
// replaces column k of the tall matrix by a seeded random vector (a new
// orthonormal direction after the next sweep) while Y = Q Rt still holds.
// Padding columns (>= l) get 0 in Rt and identity in Ra and are not flagged.
// Outputs: Rt (FP64, ldr), Ra (T, ld lp), Dinv (T, W_J for every panel),
// dep[c] in {0,1}, status bits in info.
// ---------------------------------------------------------------------------
constexpr int kCholThreads = 512;

struct CholShared {
  double gd[kMaxL];
  int sdep[kMaxL];
  double dgt[16][17];         // diagonal tile: residual in, true R_JJ out
  double raj[16][17];         // apply form of R_JJ
  double winv[16][17];        // W_J = inverse of the apply form
  double pnl[16][kMaxL + 1];  // panel row R_J,:
  int sflag;
};

__device__ __forceinline__ void wave_lds_fence() {
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront", "local");
}

__device__ __forceinline__ double bcast_f64(double v, int lane) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_readlane((int)(b & 0xffffffffll), lane);
  const int hi = __builtin_amdgcn_readlane((int)(b >> 32), lane);
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

// Factor the 16x16 residual diagonal tile held in sh.dgt (executed by the
// tile's owner wave; lane c < 16 owns column c and pivots / row entries are
// broadcast with readlane), writing the true factor back to sh.dgt, the
// apply form to sh.raj, its inverse to sh.winv and the flags to sh.sdep.
__device__ __forceinline__ void diag_factor(CholShared& sh, int J, int l, double eps) {
  const int lane = threadIdx.x & 63, c = lane & 15;
  const bool act = lane < 16;
  double cv[16];
#pragma unroll
  for (int i = 0; i < 16; ++i) cv[i] = sh.dgt[i][c];
  bool zc = false;
  double rdiag[16];   // reciprocal of the apply-form diagonal
#pragma unroll
  for (int k = 0; k < 16; ++k) {
    const int kg = 16 * J + k;
    const double piv = bcast_f64(cv[k], k);
    const bool pad = kg >= l;
    const bool isdep = !pad && !(piv > eps * sh.gd[kg]);
    const bool zero = pad || isdep;
    const double rkk = zero ? 0.0 : sqrt(piv);
    const double rsc = zero ? 0.0 : 1.0 / rkk;
    rdiag[k] = zero ? 1.0 : rsc;
    if (c == k) zc = zero;
    if (lane == 0) sh.sdep[kg] = isdep ? 1 : 0;
    // row k of R: r_kc = g_kc / r_kk (c > k), r_kk on the diagonal
    cv[k] = (c == k) ? rkk : ((c > k) ? cv[k] * rsc : cv[k]);
#pragma unroll
    for (int i = 0; i < 16; ++i) {
      if (i > k) {
        const double rki = bcast_f64(cv[k], i);
        if (c >= i) cv[i] -= rki * cv[k];
      }
    }
  }
  if (act) {
#pragma unroll
    for (int i = 0; i < 16; ++i) {
      const double t = (i <= c) ? cv[i] : 0.0;
      sh.dgt[i][c] = t;
      sh.raj[i][c] = (i == c) ? (zc ? 1.0 : t) : ((i < c && !zc) ? t : 0.0);
    }
  }
  wave_lds_fence();
  // W = inverse of the apply form: column c by back substitution, no divisions
  if (act) {
    double x[16];
#pragma unroll
    for (int i = 15; i >= 0; --i) {
      double sum = 0.0;
#pragma unroll
      for (int j = 0; j < 16; ++j)
        if (j > i) sum += sh.raj[i][j] * x[j];
      x[i] = (i > c) ? 0.0 : ((i == c) ? rdiag[i] : -sum * rdiag[i]);
    }
#pragma unroll
    for (int i = 0; i < 16; ++i) sh.winv[i][c] = x[i];
  }
}

template <typename T>
__global__ __launch_bounds__(kCholThreads) void chol_kernel(const double* __restrict__ G, int64_t ldg,
                                                            int l, int lp, double eps,
                                                            double* __restrict__ Rt, int64_t ldr,
                                                            T* __restrict__ Ra, T* __restrict__ Dinv,
                                                            int* __restrict__ dep, pbpqlp_info* info) {
  __shared__ CholShared sh;
  const int tid = threadIdx.x, lane = tid & 63, li = lane & 15, lg = lane >> 4;
  if (tid < kMaxL) {
    sh.gd[tid] = (tid < l) ? G[(int64_t)tid * ldg + tid] : 0.0;
    sh.sdep[tid] = 0;
  }
  if (tid == 0) sh.sflag = 0;
  __syncthreads();
  if (tid < l && !isfinite(sh.gd[tid])) atomicOr(&sh.sflag, 1);

  // wave w owns tile rows RA = w and RB = 15 - w: slots 0..15 hold (RA, RA..15)
  // followed by (RB, RB+1..15); slot 16 holds the diagonal tile (RB, RB).
  const int w = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int RA = w, RB = 15 - w, NA = 16 - w;
  const int Tn = lp >> 4;
  constexpr int NS = 17;
  f64x4 t[NS];
  auto tile_i = [&](int j) { return j == 16 ? RB : (j < NA ? RA : RB); };
  auto tile_k = [&](int j) { return j == 16 ? RB : (j < NA ? RA + j : RB + 1 + (j - NA)); };
#pragma unroll
  for (int j = 0; j < NS; ++j) {
    const int I = tile_i(j), K = tile_k(j);
#pragma unroll
    for (int r = 0; r < 4; ++r)
      t[j][r] = (K < Tn) ? G[(int64_t)(16 * I + acc_row<double>(lg, r)) * ldg + 16 * K + li] : 0.0;
  }

  for (int J = 0; J < Tn; ++J) {
    // Re-derive the wave's tile coordinates each step from an opaque scalar
    // copy of w: hoisted out of the loop they would hold 34 VGPRs of LDS
    // offsets; recomputed they cost a few scalar instructions.
    int wl;
    asm volatile("s_mov_b32 %0, %1" : "=s"(wl) : "s"(w));
    const int RA = wl, RB = 15 - wl, NA = 16 - wl;
    auto tile_i = [&](int j) { return j == 16 ? RB : (j < NA ? RA : RB); };
    auto tile_k = [&](int j) { return j == 16 ? RB : (j < NA ? RA + j : RB + 1 + (j - NA)); };
    // ---- A: the owner factors the diagonal tile (staged through LDS)
    if (J == RA || J == RB) {
      const bool a = J == RA;
#pragma unroll
      for (int r = 0; r < 4; ++r) sh.dgt[acc_row<double>(lg, r)][li] = a ? t[0][r] : t[16][r];
      wave_lds_fence();
      diag_factor(sh, J, l, eps);
      wave_lds_fence();
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const double v = sh.dgt[acc_row<double>(lg, r)][li];
        if (a) t[0][r] = v; else t[16][r] = v;
      }
      if (lane < 16) {
#pragma unroll
        for (int i = 0; i < 16; ++i) Dinv[J * 256 + i * 16 + li] = (T)sh.winv[i][li];
      }
    }
    lds_barrier();
    // ---- B: panel row R_JK = W_J^T G_JK (dependent rows zero), K > J
    if (J == RA || J == RB) {
#pragma unroll
      for (int j = 0; j < 16; ++j) {
        const int I = tile_i(j), K = tile_k(j);
        if (I == J && K > J && K < Tn) {
          f64x4 acc = {0, 0, 0, 0};
#pragma unroll
          for (int s4 = 0; s4 < 4; ++s4)
            acc = mma_f64(sh.winv[acc_row<double>(lg, s4)][li], t[j][s4], acc);
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            const int row = acc_row<double>(lg, r);
            const double v = sh.sdep[16 * J + row] ? 0.0 : acc[r];
            t[j][r] = v;
            sh.pnl[row][16 * K + li] = v;
          }
        }
      }
    }
    lds_barrier();
    // ---- C: trailing update G_IK -= R_JI^T R_JK for J < I <= K
#pragma unroll
    for (int j = 0; j < NS; ++j) {
      const int I = tile_i(j), K = tile_k(j);
      if (I > J && K < Tn) {
#pragma unroll
        for (int s4 = 0; s4 < 4; ++s4) {
          const int kk = acc_row<double>(lg, s4);
          t[j] = mma_f64(-sh.pnl[kk][16 * I + li], sh.pnl[kk][16 * K + li], t[j]);
        }
      }
    }
  }
  __syncthreads();
  // write Rt (true factor) and Ra (apply factor); mirror tiles below the diagonal are zero
#pragma unroll
  for (int j = 0; j < NS; ++j) {
    const int I = tile_i(j), K = tile_k(j);
    if (K < Tn) {
      const int c = 16 * K + li;
      const bool zc = c >= l || sh.sdep[c];
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int i = 16 * I + acc_row<double>(lg, r);
        const double v = (i <= c) ? t[j][r] : 0.0;
        Rt[(int64_t)i * ldr + c] = v;
        const double a = (i == c) ? (zc ? 1.0 : v) : ((i < c && !zc) ? v : 0.0);
        Ra[i * lp + c] = (T)a;
        if (I != K) {
          Rt[(int64_t)c * ldr + i] = 0.0;
          Ra[c * lp + i] = T(0);
        }
      }
    }
  }
  if (tid < lp) dep[tid] = sh.sdep[tid];
  if (tid == 0 && info) {
    int nd = 0;
    for (int k = 0; k < l; ++k) nd += sh.sdep[k];
    if (nd) {
      atomicAdd(&info->n_dependent, nd);
      atomicOr(&info->status_flags, PBPQLP_FLAG_DEPENDENT);
    }
    if (sh.sflag) atomicOr(&info->status_flags, PBPQLP_FLAG_NONFINITE);
  }
}

hipError_t launch_chol(bool f64, const double* G, int64_t ldg, int l, int lp, double eps_dep,
                       double* Rt, int64_t ldr, void* Ra, void* Dinv, int* dep, void* info,
                       hipStream_t s) {
  if (lp > kMaxL || (lp & 15)) return hipErrorInvalidValue;
  if (f64)
    hipLaunchKernelGGL(chol_kernel<double>, dim3(1), dim3(kCholThreads), 0, s, G, ldg, l, lp, eps_dep, Rt,
                       ldr, (double*)Ra, (double*)Dinv, dep, (pbpqlp_info*)info);
  else
    hipLaunchKernelGGL(chol_kernel<float>, dim3(1), dim3(kCholThreads), 0, s, G, ldg, l, lp, eps_dep, Rt,
                       ldr, (float*)Ra, (float*)Dinv, dep, (pbpqlp_info*)info);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Small FP64 products C = op(A) op(B) (one thread per output element).
// ---------------------------------------------------------------------------
__global__ void small_gemm_kernel(int M, int N, int K, const double* __restrict__ A, int64_t lda,
                                  int ta, const double* __restrict__ B, int64_t ldb, int tb,
                                  double* __restrict__ C, int64_t ldc, int tc) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  const int i = blockIdx.y;
  if (j >= N || i >= M) return;
  double s = 0.0;
  for (int k = 0; k < K; ++k) {
    const double a = ta ? A[(int64_t)k * lda + i] : A[(int64_t)i * lda + k];
    const double b = tb ? B[(int64_t)j * ldb + k] : B[(int64_t)k * ldb + j];
    s = fma(a, b, s);
  }
  if (tc) C[(int64_t)j * ldc + i] = s;
  else C[(int64_t)i * ldc + j] = s;
}

hipError_t launch_small_gemm(int M, int N, int K, const double* A, int64_t lda, int ta,
                             const double* B, int64_t ldb, int tb, double* C, int64_t ldc, int tc,
                             hipStream_t s) {
  dim3 grid((unsigned)((N + 63) / 64), (unsigned)M);
  hipLaunchKernelGGL(small_gemm_kernel, grid, dim3(64), 0, s, M, N, K, A, lda, ta, B, ldb, tb, C,
                     ldc, tc);
  return hipGetLastError();
}

__global__ void cast_kernel(const double* __restrict__ in, int64_t n, float* __restrict__ out) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) out[i] = (float)in[i];
}

hipError_t launch_cast_f64_to_f32(const double* in, int64_t n, float* out, hipStream_t s) {
  hipLaunchKernelGGL(cast_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, in, n, out);
  return hipGetLastError();
}

// L = U^T (lower triangle, zero above) with one block per row i; the block
// also leaves sum_j L[i][j]^2 in rowsq[i] for the result record.
__global__ void write_lower_t_kernel(const double* __restrict__ U, int64_t ldu, int l,
                                     double* __restrict__ L, int64_t ldl, double* __restrict__ rowsq) {
  __shared__ double red[256];
  const int i = blockIdx.x, t = threadIdx.x;
  double s = 0.0;
  for (int j = t; j < l; j += 256) {
    const double v = (j <= i) ? U[(int64_t)j * ldu + i] : 0.0;
    L[(int64_t)i * ldl + j] = v;
    s += v * v;
  }
  red[t] = s;
  __syncthreads();
  for (int off = 128; off > 0; off >>= 1) {
    if (t < off) red[t] += red[t + off];
    __syncthreads();
  }
  if (t == 0 && rowsq) rowsq[i] = red[0];
}

hipError_t launch_write_lower_t(const double* U, int64_t ldu, int l, double* L, int64_t ldl,
                                double* rowsq, hipStream_t s) {
  hipLaunchKernelGGL(write_lower_t_kernel, dim3((unsigned)l), dim3(256), 0, s, U, ldu, l, L, ldl,
                     rowsq);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Result record: zeroed at the start of a call; at the end ||A||_F^2 (summed
// in a fixed order from the first pass's per-block partials), ||L||_F^2 and
// the a-posteriori residual sqrt(||A||^2 - ||L||^2) / ||A|| (for an
// orthogonal projection Q Q^T A the two norms differ by the residual's).
// ---------------------------------------------------------------------------
__global__ void info_init_kernel(pbpqlp_info* info, int l, int q) {
  if (threadIdx.x == 0) {
    info->status_flags = 0;
    info->n_dependent = 0;
    info->l = l;
    info->q = q;
    info->norm_a_fro2 = 0.0;
    info->norm_l_fro2 = 0.0;
    info->resid_rel_est = 0.0;
    info->reserved[0] = 0.0;
    info->reserved[1] = 0.0;
  }
}

hipError_t launch_info_init(void* info, int l, int q, hipStream_t s) {
  hipLaunchKernelGGL(info_init_kernel, dim3(1), dim3(64), 0, s, (pbpqlp_info*)info, l, q);
  return hipGetLastError();
}

__global__ void info_finalize_kernel(pbpqlp_info* info, const double* __restrict__ parts,
                                     int nparts, const double* __restrict__ rowsq, int l) {
  __shared__ double ra[256], rl[256];
  const int t = threadIdx.x;
  double a0 = 0.0, a1 = 0.0;
  int i = t;
  for (; i + 256 < nparts; i += 512) {
    a0 += parts[i];
    a1 += parts[i + 256];
  }
  if (i < nparts) a0 += parts[i];
  ra[t] = a0 + a1;
  rl[t] = (t < l) ? rowsq[t] : 0.0;
  __syncthreads();
  for (int off = 128; off > 0; off >>= 1) {
    if (t < off) {
      ra[t] += ra[t + off];
      rl[t] += rl[t + off];
    }
    __syncthreads();
  }
  if (t == 0) {
    info->norm_a_fro2 = ra[0];
    info->norm_l_fro2 = rl[0];
    const double d = ra[0] - rl[0];
    info->resid_rel_est = ra[0] > 0.0 ? sqrt((d > 0.0 ? d : 0.0) / ra[0]) : 0.0;
  }
}

hipError_t launch_info_finalize(void* info, const double* normA_part, int nparts,
                                const double* rowsq, int l, hipStream_t s) {
  hipLaunchKernelGGL(info_finalize_kernel, dim3(1), dim3(256), 0, s, (pbpqlp_info*)info,
                     normA_part, nparts, rowsq, l);
  return hipGetLastError();
}

__global__ void fill_zero_kernel(uint32_t* p, size_t nwords) {
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < nwords) p[i] = 0u;
}

hipError_t launch_fill_zero(void* p, size_t bytes, hipStream_t s) {
  const size_t nw = bytes / 4;
  if (nw == 0) return hipSuccess;
  hipLaunchKernelGGL(fill_zero_kernel, dim3((unsigned)((nw + 255) / 256)), dim3(256), 0, s,
                     (uint32_t*)p, nw);
  return hipGetLastError();
}

}  // namespace pbq

namespace pbq {

__global__ void copy_mat_kernel(const double* __restrict__ in, int64_t ldi, int rows, int cols,
                                double* __restrict__ out, int64_t ldo, int upper_only) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  const int i = blockIdx.y;
  if (j >= cols || i >= rows) return;
  const double v = in[(int64_t)i * ldi + j];
  out[(int64_t)i * ldo + j] = (upper_only && j < i) ? 0.0 : v;
}

hipError_t launch_copy_mat(const double* in, int64_t ldi, int rows, int cols, double* out,
                           int64_t ldo, int upper_only, hipStream_t s) {
  dim3 grid((unsigned)((cols + 63) / 64), (unsigned)rows);
  hipLaunchKernelGGL(copy_mat_kernel, grid, dim3(64), 0, s, in, ldi, rows, cols, out, ldo,
                     upper_only);
  return hipGetLastError();
}

}  // namespace pbq
