// Host-side launchers of the PbP-QLP kernels (implemented in the .hip files).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

struct pbpqlp_info_dev;  // layout-compatible with pbpqlp_info (include/pbpqlp.h)

namespace pbq {

// Arguments of one A-streaming pass (K1: out = A X, K2: out = A^T X).
struct StreamArgs {
  const void* A;
  int64_t lda, m, n;
  const void* X;        // compute-type operand, column-major lp32 x ldx
  const void* Xlo;      // low bfloat16 part (BF16X3 only)
  int64_t ldx;
  int lp;               // l rounded up to 16: output columns stored
  int lp32;             // l rounded up to 32: X columns (zero padded) multiplied
  void* out;            // split partials, column-major lp x ldo each
  int64_t ldo;
  int64_t split_stride; // elements between consecutive split partials
  int splits;
  int64_t chunk;        // contraction indices per split (multiple of 64)
  double* normA;        // per-block partial ||A||_F^2 (K1 only), or null
  float a_scale, out_scale;
};

hipError_t launch_stream(bool trans, int mode, const StreamArgs& a, hipStream_t s);
// rows (A X) or columns (A^T X) of A one block of a streaming pass covers
int stream_span(int mode, bool trans);
// compute units of the current device (queried once per device)
int device_cus();
// K1 (Y = A X) workgroups along the rows of A for `rows` rows and `splits`
// contraction splits (the ||A||^2 partials of one launch: this times splits)
int64_t stream_k1_grid(int mode, int64_t rows, int splits);

// sketch: Omega^T (column-major lp32 x ld) in FP32 or FP64; zero padding
hipError_t launch_omega_cm(bool f64, int64_t n, int l, int lp32, uint64_t seed, void* Ot,
                           int64_t ld, hipStream_t s);
// Omega row-major n x l (ldo)

// FP32 column-major operand -> compute type (mode BF16/FP16/BF16X3), zero padded
hipError_t launch_convert(int mode, const float* X, int64_t ld, int64_t len, int l, int lp32,
                          float scale, void* hi, void* lo, hipStream_t s);
// out[c][i] = sum of the S partials for i < len, 0 for len <= i < wlen (wlen < 0: ldo)
hipError_t launch_splitk_reduce(bool f64, const void* part, int64_t stride, int S, int64_t ld,
                                int lp, int64_t len, void* out, int64_t ldo, hipStream_t s,
                                int64_t wlen = -1);
// Gram partials and reduction: G (lp x lp, FP64, row-major, ldg) = X X^T over len
// `target`: workgroups to aim at (contraction splits x block pairs)
int gram_splits(int64_t len, int lp, int target);
size_t gram_partial_elems(int64_t len, int lp, int target);
// far (optional): per (row, 64-column block) flags of |G_ij - delta_ij| > tol
// for i, j < l, the identity test of a later sweep (gram_far_cols(lp) per row)
hipError_t launch_gram(bool f64, const void* X, int64_t ld, int64_t len, int lp, double* part,
                       double* G, int64_t ldg, int target, hipStream_t s, int* far = nullptr, int l = 0,
                       double tol = 0.0);
inline int gram_far_cols(int lp) { return (lp + 63) / 64; }
// Cholesky of the Gram with dependent-column detection (single workgroup,
// lp <= 256); gdiag (optional): the diagonal the dependence test measures
// against, when G is a trailing block already updated by earlier panels
// ident (optional, later sweeps): when G is the identity to ident_tol the
// factor is the identity and *ident = 1 (the sweep's apply then copies)
hipError_t launch_chol(bool f64, const double* G, int64_t ldg, int l, int lp, double eps_dep,
                       double* Rt, int64_t ldr, void* Ra, void* Dinv, int* dep, void* info,
                       hipStream_t s, const double* gdiag = nullptr, int* ident = nullptr,
                       const int* far = nullptr);
// Q = Y Ra^-1 by blocked substitution (column-major in/out), optional row-major copy;
// Qcm rows [0, wq) are written (wq < 0: ldq, the padding rows zeroed)
// 16-bit copies of an apply's output for the next pass (mode 0: none)
struct Emit16 {
  void* hi = nullptr;
  void* lo = nullptr;
  int mode = 0;
  float xs = 1.0f;
};
hipError_t launch_apply(bool f64, const void* Y, int64_t ldy, int64_t len, int lp, int l,
                        const void* Ra, const void* Dinv, const int* dep, uint64_t seed,
                        void* Qcm, int64_t ldq, void* Qrm, int64_t ldqr, hipStream_t s,
                        int64_t wq = -1, const int* ident = nullptr, const Emit16& em = Emit16());
// Out = In M with M dense l x l given row-major (Mr[k*ldm + j] = M[k][j])
hipError_t launch_right_mul(bool f64, const void* In, int64_t ldi, int64_t len, int lp, int l,
                            const void* Mr, int64_t ldm, void* Ocm, int64_t ldo, void* Orm,
                            int64_t ldor, hipStream_t s);
// out[k * ldo + j] = in[j * ldi + k] for k < rows, j < cols (FP64 in; FP64 or FP32 out)
hipError_t launch_transpose_cast(bool f64_out, const double* in, int64_t ldi, int rows, int cols,
                                 void* out, int64_t ldo, hipStream_t s);
// layout conversions
hipError_t launch_rm_to_cm(bool f64, const void* X, int64_t ldx, int64_t len, int l, int lp32,
                           void* Xt, int64_t ldt, hipStream_t s);
hipError_t launch_cm_to_rm(bool f64, const void* Xt, int64_t ldt, int64_t len, int l, void* X,
                           int64_t ldx, hipStream_t s);
// small FP64 products: C = op(A) op(B) (lp x lp), optional transposed store
// ident (optional): when *ident is set, A is the identity and C = op(B) is copied
hipError_t launch_small_gemm(int M, int N, int K, const double* A, int64_t lda, int ta,
                             const double* B, int64_t ldb, int tb, double* C, int64_t ldc, int tc,
                             hipStream_t s, const int* ident = nullptr);
// write L = U^T (lower) from upper U, zero elsewhere; rowsq[i] = sum_j L[i][j]^2 (or null)
hipError_t launch_write_lower_t(const double* U, int64_t ldu, int l, double* L, int64_t ldl,
                                double* rowsq, hipStream_t s);
// number of leading L_ii > tol * L_11 (L row-major FP64) into *out (device)
hipError_t launch_rank_estimate(const double* L, int64_t ldl, int l, double tol, int* out, hipStream_t s);
hipError_t launch_info_init(void* info, int l, int q, hipStream_t s);
hipError_t launch_info_finalize(void* info, const double* normA_part, int nparts,
                                const double* rowsq, int l, hipStream_t s);
hipError_t launch_fill_zero(void* p, size_t bytes, hipStream_t s);
hipError_t launch_copy_mat(const double* in, int64_t ldi, int rows, int cols, double* out,
                           int64_t ldo, int upper_only, hipStream_t s);

// ---- wide sketches (l > 256) ----
// Omega for any width (column-major lp32 x ld, same values as launch_omega_cm)
hipError_t launch_omega_big(bool f64, int64_t n, int l, int lp32, uint64_t seed, void* Ot, int64_t ld,
                            hipStream_t s);
// Cout = beta Cin + alpha A B with element strides; dt 0: FP32, 1: FP64,
// 2: FP32 operands accumulated in FP64 into an FP64 C, 3: FP32 A and C with
// an FP64 B (FP32 accumulation); upper: skip output tiles wholly below the
// diagonal
hipError_t launch_gemm(int dt, int64_t M, int64_t N, int64_t K, const void* A, int64_t sai, int64_t sak,
                       const void* B, int64_t sbk, int64_t sbj, const void* Cin, void* Cout, int64_t sci,
                       int64_t scj, double alpha, double beta, bool upper, hipStream_t s);
hipError_t launch_save_diag(const double* G, int64_t ldg, int l, int lp, double* d, hipStream_t s);
hipError_t launch_zero_dep_rows(double* R, int64_t ldr, int rows, int64_t cols, const int* dep, hipStream_t s);
hipError_t launch_cast_f32(const double* in, float* out, int64_t count, hipStream_t s);

// ---- sparse A (CSR) ----
// CSR of A^T (ptr_t n + 1, idx_t / vals_t nnz) by a stable radix sort of the
// column indices; scratch of csr_transpose_scratch_bytes; *bad |= FLAG_BADINPUT
// for invalid structure
size_t csr_transpose_scratch_bytes(int64_t nnz, int64_t n);
hipError_t launch_csr_transpose(bool f64, const int64_t* rowptr, const int32_t* colind, const void* vals,
                                int64_t m, int64_t n, int64_t nnz, void* scratch, int64_t* ptr_t,
                                int32_t* idx_t, void* vals_t, int* bad, hipStream_t s);
// part[b] = sum of squares of values slice b (nparts slices)
hipError_t launch_sumsq(bool f64, const void* vals, int64_t nnz, int nparts, double* part, hipStream_t s);
// out (column-major, ldo, padding 0) = M X[:, c0:c0+w] for CSR M (rows x cols)
// and row-major X (ldx), balanced by nonzeros; Yrm (rows x ldy) and part
// (spmm_part_rows(nnz) x ldy) are scratch
int64_t spmm_chunks(int64_t nnz);
int64_t spmm_part_rows(int64_t nnz);
hipError_t launch_spmm(bool f64, const int64_t* rowptr, const int32_t* idx, const void* vals, int64_t rows,
                       int64_t cols, int64_t nnz, const void* X, int64_t ldx, int c0, int w, void* Yrm,
                       int64_t ldy, void* part, void* out, int64_t ldo, hipStream_t s);

}  // namespace pbq
