// l x l stages of PbP-QLP in FP64: the Cholesky factor of a Gram matrix (the
// small half of a CholeskyQR sweep, i.e. of orth()/qr() in Algorithm 1),
// small products (R2 R1, U2 U1) and the result record.
#include "common.h"
#include "kernels.h"
#include "../../include/pbpqlp.h"

namespace pbq {

// ---------------------------------------------------------------------------
// Upper Cholesky G = R^T R of an lp x lp Gram (only the first l columns are
// live; the rest is padding), one workgroup of 1024 threads.  The upper
// triangle is held in registers as 16x16 tiles (tile (I,K), I <= K, owned by
// wave (K(K+1)/2 + I) mod 16, lane layout of the matrix-core accumulator);
// each column step broadcasts the pivot row through LDS and updates the
// trailing tiles in place.
//
// Dependent columns: if the pivot satisfies !(d_k > eps * G_kk) (this also
// catches d_k <= 0, G_kk = 0 and NaN), column k carries no new direction.
// The "true" factor Rt gets a zero diagonal and a zero row k; the "apply"
// factor Ra gets an identity row and column k, so the triangular apply
// replaces column k of the tall matrix by a seeded random vector (a new
// orthonormal direction after the next sweep) while Y = Q Rt still holds.
// Outputs: Rt (FP64, ldr), Ra (T, ld lp), Dinv (T, inverse of each 16x16
// diagonal block of Ra), dep[c] in {0,1}, status bits in info.
// ---------------------------------------------------------------------------
template <typename T>
__global__ __launch_bounds__(1024) void chol_kernel(const double* __restrict__ G, int64_t ldg,
                                                    int l, int lp, double eps,
                                                    double* __restrict__ Rt, int64_t ldr,
                                                    T* __restrict__ Ra, T* __restrict__ Dinv,
                                                    int* __restrict__ dep, pbpqlp_info* info) {
  constexpr int SLOTS = 9;  // ceil(136 tiles / 16 waves) for lp = 256
  __shared__ double rowbuf[2][kMaxL];
  __shared__ double gd[kMaxL];
  __shared__ double dblk[kMaxL][17];
  __shared__ int sflag[2];
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63, li = lane & 15, lg = lane >> 4;
  const int Tn = lp >> 4;
  const int ntiles = Tn * (Tn + 1) / 2;

  for (int e = tid; e < lp * lp; e += 1024) {
    const int i = e / lp, j = e - (e / lp) * lp;
    Rt[(int64_t)i * ldr + j] = 0.0;
    Ra[e] = T(0);
  }
  for (int e = tid; e < lp * 17; e += 1024) dblk[e / 17][e % 17] = 0.0;
  if (tid < lp) gd[tid] = (tid < l) ? G[(int64_t)tid * ldg + tid] : 0.0;
  if (tid < 2) sflag[tid] = 0;
  __syncthreads();
  if (tid < l && !isfinite(gd[tid])) atomicOr(&sflag[1], 1);

  f64x4 tile[SLOTS];
  int tI[SLOTS], tK[SLOTS];
  bool tv[SLOTS];
#pragma unroll
  for (int s = 0; s < SLOTS; ++s) {
    const int idx = s * 16 + wave;
    tv[s] = idx < ntiles;
    int K = 0;
    while ((K + 1) * (K + 2) / 2 <= idx) ++K;
    tK[s] = tv[s] ? K : 0;                 // unused slots point at tile (0,0)
    tI[s] = tv[s] ? idx - K * (K + 1) / 2 : 0;
#pragma unroll
    for (int r = 0; r < 4; ++r)
      tile[s][r] = tv[s] ? G[(int64_t)(16 * tI[s] + 4 * lg + r) * ldg + 16 * tK[s] + li] : 0.0;
  }

  int ndep = 0;
  for (int k = 0; k < l; ++k) {
    const int kb = k >> 4, kk = k & 15;
    double* buf = rowbuf[k & 1];
#pragma unroll
    for (int s = 0; s < SLOTS; ++s) {
      if (tv[s] && tI[s] == kb && lg == (kk >> 2)) {
        const int c = 16 * tK[s] + li;
        const int r = kk & 3;
        if (c >= k) buf[c] = tile[s][r];
      }
    }
    __syncthreads();
    const double piv = buf[k];
    const bool isdep = !(piv > eps * gd[k]);
    const double rinv = isdep ? 0.0 : 1.0 / piv;
    const double rkk = isdep ? 0.0 : sqrt(piv);
    if (tid < lp) {
      const int c = tid;
      if (c == k) {
        Rt[(int64_t)k * ldr + k] = rkk;
        Ra[k * lp + k] = isdep ? T(1) : (T)rkk;
        dblk[k][k & 15] = isdep ? 1.0 : rkk;
      } else if (c > k) {
        const double r = isdep ? 0.0 : buf[c] / rkk;
        Rt[(int64_t)k * ldr + c] = r;
        Ra[k * lp + c] = (T)r;
        if ((c >> 4) == kb) dblk[k][c & 15] = r;
      } else if (isdep) {
        Ra[c * lp + k] = T(0);
        if ((c >> 4) == kb) dblk[c][k & 15] = 0.0;
      }
    }
    if (tid == 0) dep[k] = isdep ? 1 : 0;
    ndep += isdep ? 1 : 0;
#pragma unroll
    for (int s = 0; s < SLOTS; ++s) {
      if (tv[s] && tI[s] >= kb) {
        const int c = 16 * tK[s] + li;
        const double bc = buf[c] * rinv;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int i = 16 * tI[s] + 4 * lg + r;
          if (i > k && c >= i) tile[s][r] -= buf[i] * bc;
        }
      }
    }
  }
  __syncthreads();
  // padding columns: identity in Ra, zero in Rt, never dependent
  for (int c = l + tid; c < lp; c += 1024) {
    Ra[c * lp + c] = T(1);
    dblk[c][c & 15] = 1.0;
    dep[c] = 0;
  }
  __syncthreads();
  // inverses of the 16x16 diagonal blocks of Ra (column c by back substitution)
  if (wave < Tn && lg == 0) {
    const int w = wave, c = li;
    double x[16];
#pragma unroll
    for (int i = 15; i >= 0; --i) {
      double s = 0.0;
#pragma unroll
      for (int j = i + 1; j < 16; ++j) s += dblk[16 * w + i][j] * x[j];
      const double d = dblk[16 * w + i][i];
      x[i] = (i > c) ? 0.0 : ((i == c) ? 1.0 / d : -s / d);
    }
#pragma unroll
    for (int i = 0; i < 16; ++i) Dinv[w * 256 + i * 16 + c] = (T)x[i];
  }
  if (tid == 0 && info) {
    if (ndep) {
      atomicAdd(&info->n_dependent, ndep);
      atomicOr(&info->status_flags, PBPQLP_FLAG_DEPENDENT);
    }
    if (sflag[1]) atomicOr(&info->status_flags, PBPQLP_FLAG_NONFINITE);
  }
}

hipError_t launch_chol(bool f64, const double* G, int64_t ldg, int l, int lp, double eps_dep,
                       double* Rt, int64_t ldr, void* Ra, void* Dinv, int* dep, void* info,
                       hipStream_t s) {
  if (lp > kMaxL || (lp & 15)) return hipErrorInvalidValue;
  if (f64)
    hipLaunchKernelGGL(chol_kernel<double>, dim3(1), dim3(1024), 0, s, G, ldg, l, lp, eps_dep, Rt,
                       ldr, (double*)Ra, (double*)Dinv, dep, (pbpqlp_info*)info);
  else
    hipLaunchKernelGGL(chol_kernel<float>, dim3(1), dim3(1024), 0, s, G, ldg, l, lp, eps_dep, Rt,
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

__global__ void write_lower_t_kernel(const double* __restrict__ U, int64_t ldu, int l,
                                     double* __restrict__ L, int64_t ldl) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  const int i = blockIdx.y;
  if (j >= l) return;
  L[(int64_t)i * ldl + j] = (j <= i) ? U[(int64_t)j * ldu + i] : 0.0;
}

hipError_t launch_write_lower_t(const double* U, int64_t ldu, int l, double* L, int64_t ldl,
                                hipStream_t s) {
  dim3 grid((unsigned)((l + 63) / 64), (unsigned)l);
  hipLaunchKernelGGL(write_lower_t_kernel, grid, dim3(64), 0, s, U, ldu, l, L, ldl);
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
                                     int nparts, const double* __restrict__ L, int64_t ldl, int l) {
  __shared__ double ra[256], rl[256];
  const int t = threadIdx.x;
  double a = 0.0, b = 0.0;
  for (int i = t; i < nparts; i += 256) a += parts[i];
  for (int e = t; e < l * l; e += 256) {
    const int i = e / l, j = e - (e / l) * l;
    const double v = L[(int64_t)i * ldl + j];
    b += v * v;
  }
  ra[t] = a;
  rl[t] = b;
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

hipError_t launch_info_finalize(void* info, const double* normA_part, int nparts, const double* L,
                                int64_t ldl, int l, hipStream_t s) {
  hipLaunchKernelGGL(info_finalize_kernel, dim3(1), dim3(256), 0, s, (pbpqlp_info*)info,
                     normA_part, nparts, L, ldl, l);
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
