// Sparse A (Section IV-E: for a sparse A the products with A and A^T cost
// O(z d) for z nonzeros).  A is given in CSR (row pointers int64, column
// indices int32, values FP32/FP64).  Both products of the method become
// row-gather products Y = M X for a CSR matrix M: M = A for A X, and M = the
// CSR of A^T for A^T X, built once per factorization by a stable radix sort
// of the column indices (entries of each row of A^T in increasing row
// order of A), so every output entry is a sum in one fixed order and results
// are deterministic.  The orthonormalization stack is the dense path's.
#include "common.h"
#include "kernels.h"
#include "launch.h"
#include "../../include/pbpqlp.h"

namespace pbq {

constexpr int64_t kSpmmChunk = 256;   // nonzeros per wave of the balanced product
constexpr int64_t kFixGroup = 64;     // chunks per head sum of the rows cut by chunk boundaries

// ---------------------------------------------------------------------------
// CSR of A^T by a stable LSD radix sort of the column indices (8 bits per
// pass) carrying each entry's position: entries keep A's order (increasing
// row) within each column.  An entry whose column index lies outside [0, n)
// gets key n, sorts after every valid one and is left out of A^T; such
// indices and row pointers out of order or range raise PBPQLP_FLAG_BADINPUT.
// One pass over tiles of 4096 entries:
//   histogram  per tile and digit (digit-major table H[d T + t]);
//   scan       exclusive prefix of H: where tile t's digit-d entries start;
//   scatter    16 rounds of 256 entries in order; each entry's rank among the
//              round's equal digits comes from eight ballots (its wave) and
//              per-wave counts in LDS (earlier waves), plus the tile's running
//              count of the digit from earlier rounds.
// ---------------------------------------------------------------------------
constexpr int kRsTile = 4096;

struct NarrowP {
  const int64_t* in;
  int32_t* out;
  int64_t n;
  PBQ_GRID;
};

template <bool B>
__global__ void narrow_kernel(const NarrowP* pb, NarrowP ps) {
  bool past;
  const NarrowP p = kparams<B>(pb, ps, past);
  if (past) return;
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < p.n) p.out[i] = (int32_t)p.in[i];
}

hipError_t launch_narrow(const int64_t* in, int32_t* out, int64_t n, hipStream_t s) {
  NarrowP p{in, out, n};
  return launch_k(narrow_kernel<false>, narrow_kernel<true>, dim3((unsigned)((n + 255) / 256)), dim3(256), s, p);
}

struct KeyInitP {
  const int32_t* colind;
  int64_t nnz, n;
  int32_t* key;
  int32_t* perm;
  int* bad;
  PBQ_GRID;
};

template <bool B>
__global__ void key_init_kernel(const KeyInitP* pb, KeyInitP ps) {
  bool past;
  const KeyInitP p = kparams<B>(pb, ps, past);
  if (past) return;
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= p.nnz) return;
  const int j = p.colind[e];
  const bool ok = j >= 0 && j < p.n;
  if (!ok) atomicOr(p.bad, PBPQLP_FLAG_BADINPUT);
  p.key[e] = ok ? j : (int32_t)p.n;
  p.perm[e] = (int32_t)e;
}

struct RowCheckP {
  const int64_t* rowptr;
  int64_t m, nnz;
  int* bad;
  int* rpbad;   // the transpose's own record of invalid row pointers
  PBQ_GRID;
};

template <bool B>
__global__ void rowptr_check_kernel(const RowCheckP* pb, RowCheckP ps) {
  bool past;
  const RowCheckP p = kparams<B>(pb, ps, past);
  if (past) return;
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i > p.m) return;
  const int64_t v = p.rowptr[i];
  bool badv = v < 0 || v > p.nnz || (i == 0 && v != 0) || (i == p.m && v != p.nnz);
  if (i < p.m && p.rowptr[i + 1] < v) badv = true;
  if (badv) {
    atomicOr(p.bad, PBPQLP_FLAG_BADINPUT);
    atomicOr(p.rpbad, 1);
  }
}

struct RsP {
  const int32_t* kin;
  const int32_t* pin;
  int32_t* kout;
  int32_t* pout;
  int64_t nnz, T;
  int shift;
  int* H;   // 256 x T: counts, then (after the scan) start positions
  PBQ_GRID;
};

template <bool B>
__global__ __launch_bounds__(256) void rs_hist_kernel(const RsP* pb, RsP ps) {
  bool past;
  const RsP p = kparams<B>(pb, ps, past);
  if (past) return;
  __shared__ int h[256];
  const int tid = threadIdx.x;
  h[tid] = 0;
  __syncthreads();
  const int64_t base = (int64_t)blockIdx.x * kRsTile;
  for (int r = 0; r < kRsTile / 256; ++r) {
    const int64_t e = base + r * 256 + tid;
    if (e < p.nnz) atomicAdd(&h[(p.kin[e] >> p.shift) & 255], 1);
  }
  __syncthreads();
  p.H[(int64_t)tid * p.T + blockIdx.x] = h[tid];
}

template <bool B>
__global__ __launch_bounds__(256) void rs_scatter_kernel(const RsP* pb, RsP ps) {
  bool past;
  const RsP p = kparams<B>(pb, ps, past);
  if (past) return;
  __shared__ int run[256];
  __shared__ int wc[4][256];
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  run[tid] = p.H[(int64_t)tid * p.T + blockIdx.x];   // start of this tile's digit-tid entries
  const uint64_t below = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
  const int64_t base = (int64_t)blockIdx.x * kRsTile;
  for (int r = 0; r < kRsTile / 256; ++r) {
    wc[0][tid] = 0;
    wc[1][tid] = 0;
    wc[2][tid] = 0;
    wc[3][tid] = 0;
    __syncthreads();
    const int64_t e = base + r * 256 + tid;
    const bool valid = e < p.nnz;
    int key = 0, d = 0;
    int32_t pv = 0;
    if (valid) {
      key = p.kin[e];
      pv = p.pin[e];
      d = (key >> p.shift) & 255;
    }
    uint64_t mask = __builtin_amdgcn_ballot_w64(valid);
#pragma unroll
    for (int bit = 0; bit < 8; ++bit) {
      const bool on = (d >> bit) & 1;
      const uint64_t bb = __builtin_amdgcn_ballot_w64(on);
      mask &= on ? bb : ~bb;
    }
    const int rank = __popcll(mask & below);
    if (valid && rank == 0) wc[wave][d] = __popcll(mask);
    __syncthreads();
    if (valid) {
      int off = run[d] + rank;
      for (int w = 0; w < wave; ++w) off += wc[w][d];
      p.kout[off] = key;
      p.pout[off] = pv;
    }
    __syncthreads();
    run[tid] += wc[0][tid] + wc[1][tid] + wc[2][tid] + wc[3][tid];
  }
}

// Exclusive scan of n int32 counts into int64 (out[0 .. n], out[n] = total),
// 4096 per block: local scan, block totals scanned by a recursive call,
// offsets added.
struct ScanLP {
  const int32_t* in;
  const int64_t* in64;
  int64_t n;
  int64_t* out;
  int64_t* bsum;
  PBQ_GRID;
};

template <bool B>
__global__ __launch_bounds__(1024) void scan_local_kernel(const ScanLP* pb, ScanLP ps) {
  bool past;
  const ScanLP p = kparams<B>(pb, ps, past);
  if (past) return;
  __shared__ int64_t s[1024];
  const int t = threadIdx.x;
  const int64_t base = (int64_t)blockIdx.x * 4096 + (int64_t)t * 4;
  int64_t v[4], acc = 0;
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    const int64_t i = base + k;
    v[k] = i < p.n ? (p.in ? (int64_t)p.in[i] : p.in64[i]) : 0;
    acc += v[k];
  }
  s[t] = acc;
  __syncthreads();
  for (int off = 1; off < 1024; off <<= 1) {
    const int64_t x = t >= off ? s[t - off] : 0;
    __syncthreads();
    s[t] += x;
    __syncthreads();
  }
  int64_t run = s[t] - acc;   // exclusive prefix of this thread's four
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    const int64_t i = base + k;
    if (i < p.n) p.out[i] = run;
    run += v[k];
  }
  if (t == 1023) p.bsum[blockIdx.x] = s[1023];
}

struct ScanAddP {
  int64_t* out;
  int64_t n;
  const int64_t* boff;
  PBQ_GRID;
};

template <bool B>
__global__ void scan_add_kernel(const ScanAddP* pb, ScanAddP ps) {
  bool past;
  const ScanAddP p = kparams<B>(pb, ps, past);
  if (past) return;
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < p.n) p.out[i] += p.boff[i / 4096];
}

struct TotalP {
  int64_t* out;
  int64_t n;
  const int64_t* boff;
  const int64_t* bsum;
  int64_t nb;
  PBQ_GRID;
};

template <bool B>
__global__ void scan_total_kernel(const TotalP* pb, TotalP ps) {
  bool past;
  const TotalP p = kparams<B>(pb, ps, past);
  if (past) return;
  if (threadIdx.x == 0) p.out[p.n] = p.boff[p.nb - 1] + p.bsum[p.nb - 1];
}

// scratch for a scan of n elements: its block totals and their own scan, recursively
size_t scan_scratch_elems(int64_t n) {
  const int64_t nb = (n + 4095) / 4096;
  return nb <= 1 ? 2 : (size_t)(2 * nb + 1) + scan_scratch_elems(nb);
}

hipError_t launch_scan(const int32_t* in, const int64_t* in64, int64_t n, int64_t* out, int64_t* scratch,
                       hipStream_t s) {
  const int64_t nb = (n + 4095) / 4096 > 0 ? (n + 4095) / 4096 : 1;
  int64_t* bsum = scratch;
  int64_t* boff = scratch + nb;
  ScanLP lp{in, in64, n, out, bsum};
  hipError_t e = launch_k(scan_local_kernel<false>, scan_local_kernel<true>, dim3((unsigned)nb), dim3(1024), s, lp);
  if (e != hipSuccess) return e;
  if (nb > 1) {
    e = launch_scan(nullptr, bsum, nb, boff, scratch + 2 * nb + 1, s);
    if (e != hipSuccess) return e;
    ScanAddP ap{out, n, boff};
    e = launch_k(scan_add_kernel<false>, scan_add_kernel<true>, dim3((unsigned)((n + 255) / 256)), dim3(256), s, ap);
    if (e != hipSuccess) return e;
  } else {
    e = launch_fill_zero(boff, sizeof(int64_t), s);
    if (e != hipSuccess) return e;
  }
  TotalP tp{out, n, boff, bsum, nb};
  return launch_k(scan_total_kernel<false>, scan_total_kernel<true>, dim3(1), dim3(64), s, tp);
}

// Row of every entry of A: thread r writes r over its row's entries.  Run
// only when the row pointers passed their check (then they rise from 0 to nnz
// and the threads write nnz entries in all); with invalid row pointers the
// finish kernel searches them per entry instead.
struct RowIdP {
  const int64_t* rowptr;
  int64_t m;
  const int* rpbad;
  int32_t* rowid;
  PBQ_GRID;
};

template <bool B>
__global__ void rowid_kernel(const RowIdP* pb, RowIdP ps) {
  bool past;
  const RowIdP p = kparams<B>(pb, ps, past);
  if (past) return;
  const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= p.m) return;
  if (__hip_atomic_load(p.rpbad, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) return;
  const int64_t e1 = p.rowptr[r + 1];
  for (int64_t e = p.rowptr[r]; e < e1; ++e) p.rowid[e] = (int32_t)r;
}

// Column counts of the valid entries (from the sorted keys: the last entry of
// each run of equal keys knows its count) and the entries of A^T.
struct FinishP {
  const int32_t* key;   // sorted
  const int32_t* perm;
  const int32_t* rowid; // row of each entry of A (rowid_kernel)
  const int64_t* rowptr;
  const int* rpbad;     // set: row pointers invalid, rowid not written
  const void* vals;
  int64_t m, n, nnz;
  int32_t* colcnt;
  int32_t* idx_t;
  void* vals_t;
  PBQ_GRID;
};

template <typename T, bool B>
__global__ void csr_finish_kernel(const FinishP* pb, FinishP ps) {
  bool past;
  const FinishP p = kparams<B>(pb, ps, past);
  if (past) return;
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= p.nnz) return;
  const int k = p.key[i];
  if (k >= p.n) return;   // invalid entries sort last and are left out
  const int64_t e = p.perm[i];
  int64_t r;
  if (!__hip_atomic_load(p.rpbad, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) {
    r = p.rowid[e];
  } else {
    // row of entry e: the last r with rowptr[r] <= e
    int64_t lo = 0, hi = p.m - 1;
    while (lo < hi) {
      const int64_t mid = (lo + hi + 1) >> 1;
      if (p.rowptr[mid] <= e) lo = mid; else hi = mid - 1;
    }
    r = lo;
  }
  p.idx_t[i] = (int32_t)r;
  ((T*)p.vals_t)[i] = ((const T*)p.vals)[e];
  if (i + 1 == p.nnz || p.key[i + 1] != k) {
    // the run of key k ends here; it started after the previous key's run
    int64_t a = 0, b = i;
    while (a < b) {   // first index with key == k (sorted keys)
      const int64_t mid = (a + b) >> 1;
      if (p.key[mid] < k) a = mid + 1; else b = mid;
    }
    p.colcnt[k] = (int32_t)(i + 1 - a);
  }
}

size_t csr_transpose_scratch_bytes(int64_t nnz, int64_t n) {
  const int64_t T = (nnz + kRsTile - 1) / kRsTile > 0 ? (nnz + kRsTile - 1) / kRsTile : 1;
  size_t b = 0;
  auto take = [&](size_t x) { b += (x + 255) / 256 * 256; };
  take(4 * (size_t)nnz * sizeof(int32_t));         // keys and positions, two of each
  take((size_t)256 * T * sizeof(int32_t));          // H
  take(((size_t)256 * T + 1) * sizeof(int64_t));    // its scan
  take((size_t)n * sizeof(int32_t));                // column counts
  take(sizeof(int32_t));                            // invalid row pointers
  const int64_t big = 256 * T > n ? 256 * T : n;
  take(scan_scratch_elems(big) * sizeof(int64_t));
  return b + 256;
}

hipError_t launch_csr_transpose(bool f64, const int64_t* rowptr, const int32_t* colind, const void* vals,
                                int64_t m, int64_t n, int64_t nnz, void* scratch, int64_t* ptr_t,
                                int32_t* idx_t, void* vals_t, int* bad, hipStream_t s) {
  const int64_t T = (nnz + kRsTile - 1) / kRsTile > 0 ? (nnz + kRsTile - 1) / kRsTile : 1;
  char* sp = (char*)(((uintptr_t)scratch + 255) & ~(uintptr_t)255);
  auto take = [&](size_t x) { char* r = sp; sp += (x + 255) / 256 * 256; return (void*)r; };
  int32_t* ka = (int32_t*)take((size_t)nnz * 4);
  int32_t* kb = (int32_t*)take((size_t)nnz * 4);
  int32_t* pa = (int32_t*)take((size_t)nnz * 4);
  int32_t* pbm = (int32_t*)take((size_t)nnz * 4);
  int32_t* H = (int32_t*)take((size_t)256 * T * 4);
  int64_t* Hs = (int64_t*)take(((size_t)256 * T + 1) * 8);
  int32_t* colcnt = (int32_t*)take((size_t)n * 4);
  int* rpbad = (int*)take(4);
  int64_t* ss = (int64_t*)sp;
  hipError_t e;
  {
    e = launch_fill_zero(rpbad, 4, s);
    if (e != hipSuccess) return e;
    RowCheckP rc{rowptr, m, nnz, bad, rpbad};
    e = launch_k(rowptr_check_kernel<false>, rowptr_check_kernel<true>, dim3((unsigned)((m + 1 + 255) / 256)),
                 dim3(256), s, rc);
    if (e != hipSuccess) return e;
  }
  if (nnz > 0) {
    KeyInitP kp{colind, nnz, n, ka, pa, bad};
    e = launch_k(key_init_kernel<false>, key_init_kernel<true>, dim3((unsigned)((nnz + 255) / 256)), dim3(256), s, kp);
    if (e != hipSuccess) return e;
    int bits = 1;
    while (bits < 31 && ((int64_t)1 << bits) <= n) ++bits;   // keys lie in [0, n]
    int32_t *kin = ka, *kout = kb, *pin = pa, *pout = pbm;
    for (int shift = 0; shift < bits; shift += 8) {
      RsP rp{kin, pin, kout, pout, nnz, T, shift, H};
      e = launch_k(rs_hist_kernel<false>, rs_hist_kernel<true>, dim3((unsigned)T), dim3(256), s, rp);
      if (e != hipSuccess) return e;
      e = launch_scan(H, nullptr, 256 * T, Hs, ss, s);
      if (e != hipSuccess) return e;
      // start positions back into H (they fit in int32: nnz < 2^31)
      e = launch_narrow(Hs, H, 256 * T, s);
      if (e != hipSuccess) return e;
      e = launch_k(rs_scatter_kernel<false>, rs_scatter_kernel<true>, dim3((unsigned)T), dim3(256), s, rp);
      if (e != hipSuccess) return e;
      int32_t* t1 = kin; kin = kout; kout = t1;
      int32_t* t2 = pin; pin = pout; pout = t2;
    }
    e = launch_fill_zero(colcnt, (size_t)n * 4, s);
    if (e != hipSuccess) return e;
    // the last pass's input keys are free: the row of every entry goes there
    RowIdP ri{rowptr, m, rpbad, kout};
    e = launch_k(rowid_kernel<false>, rowid_kernel<true>, dim3((unsigned)((m + 255) / 256)), dim3(256), s, ri);
    if (e != hipSuccess) return e;
    FinishP fp{kin, pin, kout, rowptr, rpbad, vals, m, n, nnz, colcnt, idx_t, vals_t};
    e = f64 ? launch_k(csr_finish_kernel<double, false>, csr_finish_kernel<double, true>,
                       dim3((unsigned)((nnz + 255) / 256)), dim3(256), s, fp)
            : launch_k(csr_finish_kernel<float, false>, csr_finish_kernel<float, true>,
                       dim3((unsigned)((nnz + 255) / 256)), dim3(256), s, fp);
    if (e != hipSuccess) return e;
  } else {
    e = launch_fill_zero(colcnt, (size_t)n * 4, s);
    if (e != hipSuccess) return e;
  }
  return launch_scan(colcnt, nullptr, n, ptr_t, ss, s);
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
  void* part;       // T x 2 x ldy partial rows, then ceil(T / kFixGroup) x ldy head sums
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

// The rows cut by chunk boundaries.  A cut row r starts in chunk t0 (its
// partial there is slot 0 of t0 when r begins the chunk, else slot 1) and
// continues through chunks t0 + 1 .. t1 (slot 0 of each).  Its sum runs in a
// fixed order: the first partial, the continuation chunks before the first
// group start (a multiple of kFixGroup), then the head sums of the groups
// that start inside the row, each the sum in chunk order of the row's
// continuation chunks in that group (spmm_head_kernel).  A row of a million
// nonzeros is then a few hundred additions instead of thousands.
//
// spmm_head_kernel: the wave of group j sums slot 0 of the chunks
// jG .. min(jG + G - 1, t1) when chunk jG continues a row that started earlier.
template <typename T, bool B>
__global__ __launch_bounds__(256) void spmm_head_kernel(const SpmmP* pb, SpmmP ps) {
  bool past;
  const SpmmP p = kparams<B>(pb, ps, past);
  if (past) return;
  const int lane = threadIdx.x & 63;
  const int64_t NG = (p.T + kFixGroup - 1) / kFixGroup;
  const int64_t j = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (j >= NG || j == 0) return;
  const int64_t u0 = j * kFixGroup, b = u0 * p.C;
  const int64_t r = row_of(p.rowptr, p.rows, p.nnz, b);
  const int64_t rs = rp(p.rowptr, r, p.nnz), re = rp(p.rowptr, r + 1, p.nnz);
  if (!(rs < b && re > b)) return;
  int64_t u1 = (re - 1) / p.C;
  if (u1 > u0 + kFixGroup - 1) u1 = u0 + kFixGroup - 1;
  if (u1 > p.T - 1) u1 = p.T - 1;
  const T* part = (const T*)p.part;
  T s[4] = {T(0), T(0), T(0), T(0)};
  for (int64_t u = u0; u <= u1; ++u) {
    const T* pu = part + (u * 2) * p.ldy;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int c = lane + 64 * q;
      if (c < p.w) s[q] += pu[c];
    }
  }
  T* h = (T*)p.part + (2 * p.T + j) * p.ldy;
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int c = lane + 64 * q;
    if (c < p.w) h[c] = s[q];
  }
}

// The wave of boundary t (t = 1 .. T - 1) sums the row holding entry t C when
// that row starts in chunk t - 1 (so each cut row is summed once).
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
  const int64_t t0 = t - 1;
  int64_t t1 = (re - 1) / p.C;
  if (t1 > p.T - 1) t1 = p.T - 1;
  const T* part = (const T*)p.part;
  T s[4];
  const T* first = part + (t0 * 2 + (rs == t0 * p.C ? 0 : 1)) * p.ldy;
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int c = lane + 64 * q;
    s[q] = c < p.w ? first[c] : T(0);
  }
  auto add_chunks = [&](int64_t ua, int64_t ub) {   // slot 0 of chunks ua .. ub - 1, in order
    for (int64_t u = ua; u < ub; ++u) {
      const T* pu = part + (u * 2) * p.ldy;
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int c = lane + 64 * q;
        if (c < p.w) s[q] += pu[c];
      }
    }
  };
  const int64_t ga = (t0 + kFixGroup) / kFixGroup, gb = t1 / kFixGroup;  // groups starting in t0 + 1 .. t1
  if (ga <= gb) {
    add_chunks(t0 + 1, ga * kFixGroup);
    for (int64_t j = ga; j <= gb; ++j) {
      const T* h = part + (2 * p.T + j) * p.ldy;
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int c = lane + 64 * q;
        if (c < p.w) s[q] += h[c];
      }
    }
  } else {
    add_chunks(t0 + 1, t1 + 1);
  }
  T* Y = (T*)p.Y + r * p.ldy;
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int c = lane + 64 * q;
    if (c < p.w) Y[c] = s[q];
  }
}

hipError_t launch_sumsq(bool f64, const void* vals, int64_t nnz, int nparts, double* part, hipStream_t s) {
  const int64_t per = nnz > 0 ? (nnz + nparts - 1) / nparts : 1;
  SqP p{vals, nnz, per, part};
  if (f64) return launch_k(sumsq_kernel<double, false>, sumsq_kernel<double, true>, dim3((unsigned)nparts), dim3(256), s, p);
  return launch_k(sumsq_kernel<float, false>, sumsq_kernel<float, true>, dim3((unsigned)nparts), dim3(256), s, p);
}

int64_t spmm_chunks(int64_t nnz) { return (nnz + kSpmmChunk - 1) / kSpmmChunk; }
int64_t spmm_part_rows(int64_t nnz) {
  const int64_t T = spmm_chunks(nnz) > 0 ? spmm_chunks(nnz) : 1;
  return 2 * T + (T + kFixGroup - 1) / kFixGroup;
}

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
      const int64_t NG = (T + kFixGroup - 1) / kFixGroup;
      if (NG > 1) {
        const dim3 gh((unsigned)((NG + 3) / 4));
        e = f64 ? launch_k(spmm_head_kernel<double, false>, spmm_head_kernel<double, true>, gh, dim3(256), s, p)
                : launch_k(spmm_head_kernel<float, false>, spmm_head_kernel<float, true>, gh, dim3(256), s, p);
        if (e != hipSuccess) return e;
      }
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
