// The factorization's approximation A_hat = Q L^T P^T (eq. (Ahat) of the paper
// for A^T) and its explicit relative residual ||A - A_hat||_F / ||A||_F.
//
// W = P L (n x l) is formed first (an FP64 product of the small factor with
// the tall one), so that A_hat = Q W^T has both operands with the contraction
// index contiguous in memory.  The tile kernel computes 64 x 64 output tiles
// on the matrix cores from slices of Q and W staged in LDS; the residual
// variant never writes A_hat: it subtracts each tile from A and accumulates
// squares in FP64, one partial per block, summed afterwards in a fixed order.
// A is read once; the 2 m n l products dominate for l >= 16.
#include <hip/hip_runtime.h>

#include "../../include/pbpqlp.h"
#include "common.h"

namespace {

constexpr int TB = 64;   // output tile

// W (n x l, row-major, ldw) = P (n x l) L (l x l lower triangular, FP64).
template <typename T>
__global__ void pl_kernel(const T* __restrict__ P, int64_t ldp, const double* __restrict__ L,
                          int64_t ldl, int64_t n, int l, T* __restrict__ W, int64_t ldw) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.y + threadIdx.y;
  const int c = blockIdx.y * blockDim.x + threadIdx.x;
  if (i >= n || c >= l) return;
  double s = 0.0;
  for (int j = c; j < l; ++j) s += (double)P[i * ldp + j] * L[(int64_t)j * ldl + c];
  W[i * ldw + c] = (T)s;
}

// Tile (i0.., j0..) of Q W^T on the matrix cores (v_mfma_{f32,f64}_16x16x4):
// four waves, each a 32 x 32 quarter as 2 x 2 MFMA tiles; Q and W slices of
// KC contraction indices are staged in LDS.  MODE 0 writes A_hat, MODE 1
// accumulates ||A - A_hat||^2 and ||A||^2 of the tile into part[2 * block].
constexpr int KC = 32;

template <typename T, int MODE>
__global__ __launch_bounds__(256) void tile_kernel(const T* __restrict__ Q, int64_t ldq,
                                                   const T* __restrict__ W, int64_t ldw, int64_t m,
                                                   int64_t n, int l, const T* __restrict__ A,
                                                   int64_t lda, T* __restrict__ Ah, int64_t ldh,
                                                   double* __restrict__ part) {
  typedef typename pbq::Vec4<T>::type V4;
  __shared__ T qs[TB][KC + 1];
  __shared__ T ws[TB][KC + 1];
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6, li = lane & 15, lg = lane >> 4;
  const int64_t i0 = (int64_t)blockIdx.y * TB, j0 = (int64_t)blockIdx.x * TB;
  const int wr = (wv >> 1) * 32, wc = (wv & 1) * 32;
  V4 acc[2][2];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b) acc[a][b] = V4{0, 0, 0, 0};
  for (int k0 = 0; k0 < l; k0 += KC) {
    for (int e = tid; e < TB * KC; e += 256) {
      const int r = e / KC, c = e % KC;
      const int k = k0 + c;
      qs[r][c] = (i0 + r < m && k < l) ? Q[(i0 + r) * ldq + k] : T(0);
      ws[r][c] = (j0 + r < n && k < l) ? W[(j0 + r) * ldw + k] : T(0);
    }
    __syncthreads();
#pragma unroll
    for (int k4 = 0; k4 < KC; k4 += 4) {
      T av[2], bv[2];
#pragma unroll
      for (int u = 0; u < 2; ++u) {
        av[u] = qs[wr + 16 * u + li][k4 + lg];
        bv[u] = ws[wc + 16 * u + li][k4 + lg];
      }
#pragma unroll
      for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b) acc[a][b] = pbq::mma_native(av[a], bv[b], acc[a][b]);
    }
    __syncthreads();
  }
  double d2 = 0.0, a2 = 0.0;
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int64_t i = i0 + wr + 16 * a + pbq::acc_row<T>(lg, r);
        const int64_t j = j0 + wc + 16 * b + li;
        if (i >= m || j >= n) continue;
        if (MODE == 0) {
          Ah[i * ldh + j] = acc[a][b][r];
        } else {
          const double x = (double)A[i * lda + j];
          const double d = x - (double)acc[a][b][r];
          d2 += d * d;
          a2 += x * x;
        }
      }
  if (MODE == 1) {
    __shared__ double red[2][256];
    red[0][tid] = d2;
    red[1][tid] = a2;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
      if (tid < w) {
        red[0][tid] += red[0][tid + w];
        red[1][tid] += red[1][tid + w];
      }
      __syncthreads();
    }
    if (tid == 0) {
      const int64_t bb = (int64_t)blockIdx.y * gridDim.x + blockIdx.x;
      part[2 * bb] = red[0][0];
      part[2 * bb + 1] = red[1][0];
    }
  }
}

// r = sqrt(sum d2 / sum a2) over nb block partials (one thread per stride,
// then a fixed-order tree).
__global__ __launch_bounds__(256) void resid_final_kernel(const double* __restrict__ part, int64_t nb,
                                                          double* __restrict__ r) {
  __shared__ double red[2][256];
  const int tid = threadIdx.x;
  double d2 = 0.0, a2 = 0.0;
  for (int64_t b = tid; b < nb; b += 256) {
    d2 += part[2 * b];
    a2 += part[2 * b + 1];
  }
  red[0][tid] = d2;
  red[1][tid] = a2;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (tid < w) {
      red[0][tid] += red[0][tid + w];
      red[1][tid] += red[1][tid + w];
    }
    __syncthreads();
  }
  if (tid == 0) r[0] = red[1][0] > 0.0 ? sqrt(red[0][0] / red[1][0]) : 0.0;
}

template <typename T>
pbpqlp_status run(const void* A, int64_t lda, const void* Q, int64_t ldq, const double* L, int64_t ldl,
                  const void* P, int64_t ldp, int64_t m, int64_t n, int l, void* Ah, int64_t ldh,
                  double* d_r, hipStream_t st) {
  const dim3 grid((unsigned)((n + TB - 1) / TB), (unsigned)((m + TB - 1) / TB));
  const int64_t nb = (int64_t)grid.x * grid.y;
  const size_t wbytes = ((size_t)n * l * sizeof(T) + 255) / 256 * 256;
  const size_t bytes = wbytes + (d_r ? (size_t)nb * 2 * sizeof(double) : 0);
  char* buf = nullptr;
  if (hipMallocAsync((void**)&buf, bytes, st) != hipSuccess) return PBPQLP_ENOMEM;
  T* W = (T*)buf;
  double* part = (double*)(buf + wbytes);
  hipLaunchKernelGGL(pl_kernel<T>, dim3((unsigned)((n + 7) / 8), (unsigned)((l + 31) / 32)), dim3(32, 8), 0,
                     st, (const T*)P, ldp, L, ldl, n, l, W, (int64_t)l);
  hipError_t e = hipGetLastError();
  if (e == hipSuccess) {
    if (d_r) {
      hipLaunchKernelGGL((tile_kernel<T, 1>), grid, dim3(256), 0, st, (const T*)Q, ldq, (const T*)W,
                         (int64_t)l, m, n, l, (const T*)A, lda, (T*)nullptr, (int64_t)0, part);
      e = hipGetLastError();
      if (e == hipSuccess) {
        hipLaunchKernelGGL(resid_final_kernel, dim3(1), dim3(256), 0, st, (const double*)part, nb, d_r);
        e = hipGetLastError();
      }
    } else {
      hipLaunchKernelGGL((tile_kernel<T, 0>), grid, dim3(256), 0, st, (const T*)Q, ldq, (const T*)W,
                         (int64_t)l, m, n, l, (const T*)nullptr, (int64_t)0, (T*)Ah, ldh, (double*)nullptr);
      e = hipGetLastError();
    }
  }
  (void)hipFreeAsync(buf, st);
  return e == hipSuccess ? PBPQLP_OK : PBPQLP_EHIP;
}

bool check(const void* Q, int64_t ldq, const double* L, int64_t ldl, const void* P, int64_t ldp,
           int64_t m, int64_t n, int l, pbpqlp_dtype dt) {
  if (!Q || !L || !P || m < 1 || n < 1 || l < 1 || l > m || l > n) return false;
  if (ldq < l || ldl < l || ldp < l) return false;
  return dt == PBPQLP_F64 || dt == PBPQLP_F32;
}

}  // namespace

extern "C" {

pbpqlp_status pbpqlp_reconstruct(const void* Q, int64_t ldq, const double* L, int64_t ldl, const void* P,
                                 int64_t ldp, int64_t m, int64_t n, int l, pbpqlp_dtype dt, void* Ahat,
                                 int64_t ldh, void* stream) {
  if (!check(Q, ldq, L, ldl, P, ldp, m, n, l, dt) || !Ahat || ldh < n) return PBPQLP_EINVAL;
  hipStream_t st = (hipStream_t)stream;
  if (dt == PBPQLP_F64)
    return run<double>(nullptr, 0, Q, ldq, L, ldl, P, ldp, m, n, l, Ahat, ldh, nullptr, st);
  return run<float>(nullptr, 0, Q, ldq, L, ldl, P, ldp, m, n, l, Ahat, ldh, nullptr, st);
}

pbpqlp_status pbpqlp_residual(const void* A, int64_t lda, const void* Q, int64_t ldq, const double* L,
                              int64_t ldl, const void* P, int64_t ldp, int64_t m, int64_t n, int l,
                              pbpqlp_dtype dt, double* d_r, void* stream) {
  if (!check(Q, ldq, L, ldl, P, ldp, m, n, l, dt) || !A || !d_r || lda < n) return PBPQLP_EINVAL;
  hipStream_t st = (hipStream_t)stream;
  if (dt == PBPQLP_F64)
    return run<double>(A, lda, Q, ldq, L, ldl, P, ldp, m, n, l, nullptr, 0, d_r, st);
  return run<float>(A, lda, Q, ldq, L, ldl, P, ldp, m, n, l, nullptr, 0, d_r, st);
}

}  // extern "C"
