// Sparse A (Section IV-E: for a sparse A the products with A and A^T cost
// O(z d) for z nonzeros).  A is given in CSR (row pointers int64, column
// indices int32, values FP32/FP64).  Both products of the method become
// row-gather products Y = M X for a CSR matrix M: M = A for A X, and M = the
// CSR of A^T for A^T X, built once per factorization by a stable counting
// sort of the column indices (entries of each row of A^T in increasing row
// order of A), so every output entry is a sum in one fixed order and results
// are deterministic.  The orthonormalization stack is the dense path's.
#include "common.h"
#include "kernels.h"
#include "launch.h"
#include "../../include/pbpqlp.h"

namespace pbq {

constexpr int64_t kSpmmChunk = 256;   // nonzeros per wave of the balanced product

// Bounds of row i's entries, clamped to [0, nnz] and ordered.
__device__ __forceinline__ void row_range(const int64_t* rowptr, int64_t i, int64_t nnz, int64_t& e0,
                                          int64_t& e1) {
  e0 = rowptr[i];
  e1 = rowptr[i + 1];
  e0 = e0 < 0 ? 0 : (e0 > nnz ? nnz : e0);
  e1 = e1 < e0 ? e0 : (e1 > nnz ? nnz : e1);
}

// ---------------------------------------------------------------------------
// Stable transpose of the structure, step 1: row block b (rows [b R, b R + R))
// counts its entries per column into cnt[b n + j]; column indices outside
// [0, n) and row pointers out of order are flagged (PBPQLP_FLAG_BADINPUT into *bad) and such
// entries are skipped everywhere.
// ---------------------------------------------------------------------------
struct CsrCountP {
  const int64_t* rowptr;
  const int32_t* colind;
  int64_t m, n, nnz, R;
  int* cnt;
  int* bad;
  PBQ_GRID;
};

template <bool B>
__global__ __launch_bounds__(256) void csr_count_kernel(const CsrCountP* pb, CsrCountP ps) {
  bool past;
  const CsrCountP p = kparams<B>(pb, ps, past);
  if (past) return;
  const int64_t b = blockIdx.x;
  const int64_t r0 = b * p.R, r1 = r0 + p.R < p.m ? r0 + p.R : p.m;
  int* cnt = p.cnt + b * p.n;
  for (int64_t i = r0; i < r1; ++i) {
    const int64_t a0 = p.rowptr[i], a1 = p.rowptr[i + 1];
    if (threadIdx.x == 0 && (a0 < 0 || a1 < a0 || a1 > p.nnz)) atomicOr(p.bad, PBPQLP_FLAG_BADINPUT);
    int64_t e0, e1;
    row_range(p.rowptr, i, p.nnz, e0, e1);
    for (int64_t e = e0 + threadIdx.x; e < e1; e += blockDim.x) {
      const int j = p.colind[e];
      if (j < 0 || j >= p.n) {
        atomicOr(p.bad, PBPQLP_FLAG_BADINPUT);
        continue;
      }
      atomicAdd(&cnt[j], 1);
    }
  }
}

// Step 2: per column j, the entries of the row blocks before b
// (cnt[b n + j] becomes that exclusive prefix) and the column's total.
struct ColPrefixP {
  int* cnt;
  int64_t n;
  int nb;
  int64_t* colcnt;
  PBQ_GRID;
};

template <bool B>
__global__ void col_prefix_kernel(const ColPrefixP* pb, ColPrefixP ps) {
  bool past;
  const ColPrefixP p = kparams<B>(pb, ps, past);
  if (past) return;
  const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= p.n) return;
  int64_t s = 0;
  for (int b = 0; b < p.nb; ++b) {
    const int t = p.cnt[(int64_t)b * p.n + j];
    p.cnt[(int64_t)b * p.n + j] = (int)s;
    s += t;
  }
  p.colcnt[j] = s;
}

// Step 3: ptr[0] = 0, ptr[j + 1] = ptr[j] + cnt[j] (one workgroup, 1024
// entries per round with a running carry).
struct ScanP {
  const int64_t* cnt;
  int64_t n;
  int64_t* ptr;
  PBQ_GRID;
};

template <bool B>
__global__ __launch_bounds__(1024) void scan_kernel(const ScanP* pb, ScanP ps) {
  bool past;
  const ScanP p = kparams<B>(pb, ps, past);
  if (past) return;
  __shared__ int64_t s[1024];
  __shared__ int64_t carry;
  const int t = threadIdx.x;
  if (t == 0) {
    carry = 0;
    p.ptr[0] = 0;
  }
  __syncthreads();
  for (int64_t base = 0; base < p.n; base += 1024) {
    const int64_t j = base + t;
    s[t] = j < p.n ? p.cnt[j] : 0;
    __syncthreads();
    for (int off = 1; off < 1024; off <<= 1) {   // inclusive Hillis-Steele scan
      const int64_t v = t >= off ? s[t - off] : 0;
      __syncthreads();
      s[t] += v;
      __syncthreads();
    }
    if (j < p.n) p.ptr[j + 1] = carry + s[t];
    __syncthreads();
    if (t == 1023) carry += s[1023];
    __syncthreads();
  }
}

// Step 4: row block b places its entries row by row (rows in order, a
// barrier between rows), entry (i, j) at ptr[j] + (entries of column j in
// earlier rows): the CSR of A^T with each row's entries in increasing order of
// i.  Within one row every column appears once, so the slot counters see at
// most one increment per column between barriers.
struct PlaceP {
  const int64_t* rowptr;
  const int32_t* colind;
  const void* vals;
  int64_t m, n, nnz, R;
  const int64_t* ptr;
  int* cnt;
  int32_t* idx_t;
  void* vals_t;
  PBQ_GRID;
};

template <typename T, bool B>
__global__ __launch_bounds__(256) void csr_place_kernel(const PlaceP* pb, PlaceP ps) {
  bool past;
  const PlaceP p = kparams<B>(pb, ps, past);
  if (past) return;
  const int64_t b = blockIdx.x;
  const int64_t r0 = b * p.R, r1 = r0 + p.R < p.m ? r0 + p.R : p.m;
  int* cnt = p.cnt + b * p.n;
  const T* vals = (const T*)p.vals;
  T* vt = (T*)p.vals_t;
  for (int64_t i = r0; i < r1; ++i) {
    int64_t e0, e1;
    row_range(p.rowptr, i, p.nnz, e0, e1);
    for (int64_t e = e0 + threadIdx.x; e < e1; e += blockDim.x) {
      const int j = p.colind[e];
      if (j < 0 || j >= p.n) continue;
      const int64_t pos = p.ptr[j] + atomicAdd(&cnt[j], 1);
      p.idx_t[pos] = (int32_t)i;
      vt[pos] = vals[e];
    }
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------
// ||A||_F^2 partials: block b sums the squares of its slice of the values in
// FP64 (summed in a fixed order by the result record).
// ---------------------------------------------------------------------------
struct SqP {
  const void* vals;
  int64_t nnz, per;
  double* part;
  PBQ_GRID;
};

template <typename T, bool B>
__global__ __launch_bounds__(256) void sumsq_kernel(const SqP* pb, SqP ps) {
  bool past;
  const SqP p = kparams<B>(pb, ps, past);
  if (past) return;
  const T* v = (const T*)p.vals;
  const int64_t e0 = (int64_t)blockIdx.x * p.per, e1 = e0 + p.per < p.nnz ? e0 + p.per : p.nnz;
  double s = 0.0;
  for (int64_t e = e0 + threadIdx.x; e < e1; e += blockDim.x) {
    const double x = (double)v[e];
    s += x * x;
  }
  __shared__ double red[256];
  red[threadIdx.x] = s;
  __syncthreads();
  for (int off = 128; off > 0; off >>= 1) {
    if ((int)threadIdx.x < off) red[threadIdx.x] += red[threadIdx.x + off];
    __syncthreads();
  }
  if (threadIdx.x == 0) p.part[blockIdx.x] = red[0];
}

// ---------------------------------------------------------------------------
// Y = M X for a CSR matrix M (rows x cols) and a row-major operand X (cols x
// ldx, columns [c0, c0 + w) used, w <= 256), balanced by nonzeros: wave t
// takes the entries [t C, t C + C) in order, whatever rows they belong to,
// with each lane holding four columns of the running row sum (one gathered
// row of X per nonzero, eight nonzeros' gathers in flight).  A row that lies
// wholly inside the chunk is written to the row-major result Yrm; a row cut
// by a chunk boundary leaves its partial sum in slot 0 (the chunk's first
// row) or 1 (its last row) of the chunk's partials, and the fix-up kernel
// sums a cut row's partials in chunk order.  Every output is thus one fixed
// sum order, however skewed the row lengths.
// ---------------------------------------------------------------------------
struct SpmmP {
  const int64_t* rowptr;
  const int32_t* idx;
  const void* vals;
  int64_t rows, cols, nnz;
  const void* X;
  int64_t ldx;
  int c0, w;
  void* Y;          // row-major rows x ldy, zero before the call
  int64_t ldy;
  void* part;       // T x 2 x ldy partial rows
  int64_t C, T;
  PBQ_GRID;
};

// rowptr[i] clamped to [0, nnz]
__device__ __forceinline__ int64_t rp(const int64_t* rowptr, int64_t i, int64_t nnz) {
  const int64_t v = rowptr[i];
  return v < 0 ? 0 : (v > nnz ? nnz : v);
}

// The row holding entry e: the last r < rows with rowptr[r] <= e.
__device__ __forceinline__ int64_t row_of(const int64_t* rowptr, int64_t rows, int64_t nnz, int64_t e) {
  int64_t lo = 0, hi = rows - 1;
  while (lo < hi) {
    const int64_t mid = (lo + hi + 1) >> 1;
    if (rp(rowptr, mid, nnz) <= e) lo = mid; else hi = mid - 1;
  }
  return lo;
}

template <typename T, bool B>
__global__ __launch_bounds__(256) void spmm_kernel(const SpmmP* pb, SpmmP ps) {
  bool past;
  const SpmmP p = kparams<B>(pb, ps, past);
  if (past) return;
  const int lane = threadIdx.x & 63;
  const int64_t t = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (t >= p.T) return;
  const int64_t e0 = t * p.C, e1 = e0 + p.C < p.nnz ? e0 + p.C : p.nnz;
  const T* X = (const T*)p.X + p.c0;
  const T* vals = (const T*)p.vals;
  T* Y = (T*)p.Y;
  T* part = (T*)p.part;
  int64_t r = row_of(p.rowptr, p.rows, p.nnz, e0);
  const int64_t first = r;
  int64_t rs = rp(p.rowptr, r, p.nnz), re = rp(p.rowptr, r + 1, p.nnz);
  T acc[4] = {T(0), T(0), T(0), T(0)};
  auto flush = [&]() __attribute__((always_inline)) {
    T* dst;
    if (rs >= e0 && re <= e1) dst = Y + r * p.ldy;
    else dst = part + (t * 2 + (r == first ? 0 : 1)) * p.ldy;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int c = lane + 64 * q;
      if (c < p.w) dst[c] = acc[q];
      acc[q] = T(0);
    }
  };
  for (int64_t g = e0; g < e1; g += 8) {
    // eight entries: indices and values (lanes 0..7 load, all lanes read)
    const int64_t el = g + (lane & 7);
    int jl = -1;
    T al = T(0);
    if (el < e1) {
      jl = p.idx[el];
      al = vals[el];
    }
    int jv[8];
    T av[8];
    T xv[8][4];
#pragma unroll
    for (int k = 0; k < 8; ++k) {
      jv[k] = __shfl(jl, k);
      av[k] = __shfl(al, k);
    }
#pragma unroll
    for (int k = 0; k < 8; ++k) {
      const bool ok = jv[k] >= 0 && jv[k] < p.cols;
      const T* xr = X + (int64_t)(ok ? jv[k] : 0) * p.ldx;
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int c = lane + 64 * q;
        xv[k][q] = (ok && c < p.w) ? xr[c] : T(0);
      }
    }
#pragma unroll
    for (int k = 0; k < 8; ++k) {
      const int64_t e = g + k;
      if (e >= e1) break;
      while (e >= re && r + 1 < p.rows) {   // the next row (empty rows are written as 0)
        flush();
        ++r;
        rs = re;
        re = rp(p.rowptr, r + 1, p.nnz);
        if (re < rs) re = rs;
      }
#pragma unroll
      for (int q = 0; q < 4; ++q) acc[q] = fma(av[k], xv[k][q], acc[q]);
    }
  }
  flush();
}

// The rows cut by chunk boundaries: the wave of boundary t (t = 1 .. T - 1)
// sums the partials of the row holding entry t C when that row starts in
// chunk t - 1 (so each cut row is summed once), in chunk order.
template <typename T, bool B>
__global__ __launch_bounds__(256) void spmm_fix_kernel(const SpmmP* pb, SpmmP ps) {
  bool past;
  const SpmmP p = kparams<B>(pb, ps, past);
  if (past) return;
  const int lane = threadIdx.x & 63;
  const int64_t t = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6) + 1;
  if (t >= p.T) return;
  const int64_t b = t * p.C;
  const int64_t r = row_of(p.rowptr, p.rows, p.nnz, b);
  const int64_t rs = rp(p.rowptr, r, p.nnz);
  int64_t re = rp(p.rowptr, r + 1, p.nnz);
  if (!(rs < b && rs >= b - p.C && re > b)) return;
  const int64_t t0 = t - 1, t1 = (re - 1) / p.C;
  const T* part = (const T*)p.part;
  T s[4];
  const T* first = part + (t0 * 2 + (rs == t0 * p.C ? 0 : 1)) * p.ldy;
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int c = lane + 64 * q;
    s[q] = c < p.w ? first[c] : T(0);
  }
  for (int64_t u = t0 + 1; u <= t1 && u < p.T; ++u) {
    const T* pu = part + (u * 2) * p.ldy;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int c = lane + 64 * q;
      if (c < p.w) s[q] += pu[c];
    }
  }
  T* Y = (T*)p.Y + r * p.ldy;
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int c = lane + 64 * q;
    if (c < p.w) Y[c] = s[q];
  }
}

hipError_t launch_csr_transpose(bool f64, const int64_t* rowptr, const int32_t* colind, const void* vals,
                                int64_t m, int64_t n, int64_t nnz, int nb, int* cnt, int64_t* colcnt,
                                int64_t* ptr_t, int32_t* idx_t, void* vals_t, int* bad, hipStream_t s) {
  const int64_t R = (m + nb - 1) / nb;
  hipError_t e = launch_fill_zero(cnt, (size_t)nb * n * sizeof(int), s);
  if (e != hipSuccess) return e;
  CsrCountP cp{rowptr, colind, m, n, nnz, R, cnt, bad};
  e = launch_k(csr_count_kernel<false>, csr_count_kernel<true>, dim3((unsigned)nb), dim3(256), s, cp);
  if (e != hipSuccess) return e;
  ColPrefixP pp{cnt, n, nb, colcnt};
  e = launch_k(col_prefix_kernel<false>, col_prefix_kernel<true>, dim3((unsigned)((n + 255) / 256)), dim3(256), s, pp);
  if (e != hipSuccess) return e;
  ScanP sp{colcnt, n, ptr_t};
  e = launch_k(scan_kernel<false>, scan_kernel<true>, dim3(1), dim3(1024), s, sp);
  if (e != hipSuccess) return e;
  PlaceP lp{rowptr, colind, vals, m, n, nnz, R, ptr_t, cnt, idx_t, vals_t};
  if (f64) return launch_k(csr_place_kernel<double, false>, csr_place_kernel<double, true>, dim3((unsigned)nb), dim3(256), s, lp);
  return launch_k(csr_place_kernel<float, false>, csr_place_kernel<float, true>, dim3((unsigned)nb), dim3(256), s, lp);
}

hipError_t launch_sumsq(bool f64, const void* vals, int64_t nnz, int nparts, double* part, hipStream_t s) {
  const int64_t per = nnz > 0 ? (nnz + nparts - 1) / nparts : 1;
  SqP p{vals, nnz, per, part};
  if (f64) return launch_k(sumsq_kernel<double, false>, sumsq_kernel<double, true>, dim3((unsigned)nparts), dim3(256), s, p);
  return launch_k(sumsq_kernel<float, false>, sumsq_kernel<float, true>, dim3((unsigned)nparts), dim3(256), s, p);
}

int64_t spmm_chunks(int64_t nnz) { return (nnz + kSpmmChunk - 1) / kSpmmChunk; }

hipError_t launch_spmm(bool f64, const int64_t* rowptr, const int32_t* idx, const void* vals, int64_t rows,
                       int64_t cols, int64_t nnz, const void* X, int64_t ldx, int c0, int w, void* Yrm,
                       int64_t ldy, void* part, void* out, int64_t ldo, hipStream_t s) {
  if (w < 1 || w > 256 || ldy < w) return hipErrorInvalidValue;
  const size_t el = f64 ? 8 : 4;
  hipError_t e = launch_fill_zero(Yrm, (size_t)rows * ldy * el, s);
  if (e != hipSuccess) return e;
  const int64_t T = spmm_chunks(nnz);
  if (T > 0) {
    SpmmP p{rowptr, idx, vals, rows, cols, nnz, X, ldx, c0, w, Yrm, ldy, part, kSpmmChunk, T};
    const dim3 grid((unsigned)((T + 3) / 4));
    e = f64 ? launch_k(spmm_kernel<double, false>, spmm_kernel<double, true>, grid, dim3(256), s, p)
            : launch_k(spmm_kernel<float, false>, spmm_kernel<float, true>, grid, dim3(256), s, p);
    if (e != hipSuccess) return e;
    if (T > 1) {
      const dim3 gf((unsigned)((T - 1 + 3) / 4));
      e = f64 ? launch_k(spmm_fix_kernel<double, false>, spmm_fix_kernel<double, true>, gf, dim3(256), s, p)
              : launch_k(spmm_fix_kernel<float, false>, spmm_fix_kernel<float, true>, gf, dim3(256), s, p);
      if (e != hipSuccess) return e;
    }
  }
  // column-major result, padding rows and columns 0
  return launch_rm_to_cm(f64, Yrm, ldy, rows, w, w, out, ldo, s);
}

}  // namespace pbq
