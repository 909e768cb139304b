/*
 * pbpqlp.h -- C ABI of the MI355X (gfx950) PbP-QLP library, libpbpqlp.so.
 *
 * Projection-based Partial QLP (Kaloorazi & Chen, IEEE TSP 2021,
 * arXiv 2103.07245).  Given an m x n matrix A and 1 <= k <= l = k + p, the
 * method (Section III, Algorithm 1, here applied to A^T so that Omega has n
 * rows) computes
 *     Omega = randn(n, l)            Y = A Omega            Q = orth(Y)
 *     q times:  Z = A^T Q,  P^ = orth(Z),  Y = A P^,  Q = orth(Y)
 *     B^T = A^T Q = P R              (unpivoted QR, eqs. (D), (DQR))
 *     R^T = Qt L^T                   (unpivoted QR, eq. (R^T = Pt Rt))
 * and returns Q Qt (m x l), the lower-triangular L (l x l) and P (n x l) with
 *     A ~= (Q Qt) L^T P^T                                 (eq. (Ahat) for A^T)
 * where diag(L) approximates the leading singular values of A.  orth() and
 * both QRs are upper-triangular (nested-span) factorizations with a
 * non-negative diagonal, so every output is unique whenever the sketch has
 * full rank.
 *
 * Conventions for every entry point:
 *   - All matrix arguments are DEVICE pointers, row-major, with a leading
 *     dimension (elements between consecutive rows) >= the row length, and
 *     aligned to their element type (EINVAL otherwise).
 *   - The caller owns every buffer; the library never frees caller memory
 *     and keeps no pointer after the call returns.
 *   - Work is enqueued on `stream` (a hipStream_t passed as void*; NULL is
 *     the default stream) and the call returns without synchronizing.
 *     Argument errors are reported synchronously by the return code before
 *     anything is enqueued; numerical conditions (dependent columns that had
 *     to be completed, non-finite input) are reported asynchronously in the
 *     device-resident pbpqlp_info, which is valid once the stream reaches the
 *     end of the call.
 *   - Outputs must not alias inputs.  No C++ exception crosses this ABI.
 */
#ifndef PBPQLP_H
#define PBPQLP_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  PBPQLP_OK = 0,
  PBPQLP_EINVAL = 1,       /* an argument breaks the rules stated below            */
  PBPQLP_ENOMEM = 2,       /* caller workspace too small, or device allocation failed */
  PBPQLP_EHIP = 3,         /* a HIP runtime call or kernel launch failed           */
  PBPQLP_EUNSUPPORTED = 4  /* valid input outside the library's limits (l > 256, ...) */
} pbpqlp_status;

/* Storage type of A and of the tall outputs Q and P. */
typedef enum { PBPQLP_F64 = 0, PBPQLP_F32 = 1 } pbpqlp_dtype;

/* Arithmetic of one A-streaming pass (products with A or A^T).
 *   NATIVE : the storage type (FP64 or FP32 matrix cores).
 *   BF16   : A and the l-column operand rounded to bfloat16 (RNE), FP32 accumulate.
 *   FP16   : the same in IEEE half; A is multiplied by opts.fp16_scale_a (a power
 *            of two) before rounding, so the caller keeps |A| inside half range.
 *   BF16X3 : split products hi*hi + hi*lo + lo*hi of bfloat16 pieces
 *            (hi = bf16(x), lo = bf16(x - hi)), FP32 accumulate: close to FP32.
 * The reduced precisions apply to PBPQLP_F32 storage only.  Grams, Cholesky
 * factors, triangular solves and the l x l QR always run in FP64 / FP32. */
typedef enum {
  PBPQLP_PREC_NATIVE = 0,
  PBPQLP_PREC_BF16 = 1,
  PBPQLP_PREC_FP16 = 2,
  PBPQLP_PREC_BF16X3 = 3
} pbpqlp_prec;

typedef struct {
  int sketch_prec;          /* pass Y = A Omega                                   */
  int power_prec;           /* the 2q passes of the power iterations              */
  int proj_prec;            /* pass B^T = A^T Q                                   */
  int split_k;              /* contraction splits of each A-streaming pass:
                               0 = automatic (the autotuned plan of the problem's
                               shape class if one is cached, else the built-in
                               heuristic), -1 = the built-in heuristic, > 0 forced */
  int gram_workgroups;      /* workgroups each Gram aims at (contraction splits x
                               column-block pairs): 0 = automatic (cached plan,
                               else 256; in a batch a count-based default), > 0 forced */
  double fp16_scale_a;      /* power of two applied to A in FP16 passes (0 -> 1)  */
  void* workspace;          /* device memory owned by the caller, or NULL: then the
                               library allocates stream-ordered and frees it after */
  size_t workspace_bytes;
} pbpqlp_opts;

/* Device-resident result record of one factorization. */
typedef struct {
  int status_flags;         /* PBPQLP_FLAG_* bits                                  */
  int n_dependent;          /* columns completed over all orthonormalizations     */
  int l;                    /* sketch width used                                   */
  int q;                    /* power iterations used                               */
  double norm_a_fro2;       /* ||A||_F^2, FP64, accumulated during the first pass */
  double norm_l_fro2;       /* ||L||_F^2                                           */
  double resid_rel_est;     /* sqrt(max(||A||^2 - ||L||^2, 0)) / ||A||_F: equals
                               ||A - Q L^T P^T||_F / ||A||_F when Q, P are orthonormal */
  double reserved[2];
} pbpqlp_info;

#define PBPQLP_FLAG_DEPENDENT 1  /* a Cholesky pivot fell below the dependence threshold:
                                    that column was replaced by a seeded random vector,
                                    its R row/diagonal is 0 (rank-deficient sketch)   */
#define PBPQLP_FLAG_NONFINITE 2  /* a Gram matrix held NaN or Inf (non-finite input)   */
#define PBPQLP_FLAG_INTERNAL 4   /* a bounded wait inside a kernel gave up (should never
                                    happen): the results of that call are not valid   */
#define PBPQLP_FLAG_BADINPUT 8   /* sparse input: a row pointer out of order or range, or
                                    a column index outside [0, n); such entries are
                                    skipped                                           */

/* Human-readable name of a status code (static storage). */
const char* pbpqlp_status_string(pbpqlp_status s);

/* Version of this ABI, 100 * major + minor. */
int pbpqlp_version(void);

/* Default options: every pass NATIVE, automatic split, library-owned workspace. */
void pbpqlp_default_opts(pbpqlp_opts* opts);

/* Bytes of device workspace pbpqlp_factor (and pbpqlp_factor_rr in either
 * orientation) needs for this problem.
 * Errors: EINVAL for arguments pbpqlp_factor would reject; EUNSUPPORTED for l > 256. */
pbpqlp_status pbpqlp_workspace_size(int64_t m, int64_t n, int k, int p, pbpqlp_dtype dt,
                                    const pbpqlp_opts* opts, size_t* bytes);

/* Full factorization (Algorithm 1 for A^T; Section III-A when q = 0).
 *   A     : m x n, dtype dt, lda >= n.  Read only.
 *   k, p  : 1 <= k, 0 <= p, l = k + p <= min(m, n), l <= 256.
 *   q     : number of power iterations, 0 <= q <= 16.
 *   seed  : selects Omega (Philox4x32-10 + Box-Muller, rounded to bfloat16),
 *           identical for every precision choice.
 *   Q     : m x l, dtype dt, ldq >= l: written with Q Qt (orthonormal columns).
 *   L     : l x l FP64, ldl >= l: lower triangular, upper part written 0,
 *           diagonal >= 0 (approximate singular values).
 *   P     : n x l, dtype dt, ldp >= l: orthonormal columns.
 *   opts  : may be NULL (defaults).  d_info: device pointer or NULL.
 * A == 0 returns OK with L = 0 and orthonormal (seeded) Q and P. */
pbpqlp_status pbpqlp_factor(const void* A, int64_t m, int64_t n, int64_t lda, pbpqlp_dtype dt,
                            int k, int p, int q, uint64_t seed,
                            void* Q, int64_t ldq, double* L, int64_t ldl, void* P, int64_t ldp,
                            const pbpqlp_opts* opts, pbpqlp_info* d_info, void* stream);

/* The same factorization with a caller-supplied sketch matrix in place of the
 * generated one (eq. (c) with Phi given; Algorithm 1 from its first product):
 *   Omega : n x l, dtype dt, row-major, ldo >= l, device; read only.
 * Everything else as pbpqlp_factor.  Passing the P of an earlier factorization
 * of the same A as Omega continues its power iterations: the earlier
 * projection A^T Q is the first half of the next iteration, so
 * pbpqlp_factor_sketch(Omega = P of a q-iteration run, q = j) spans the same
 * subspaces as pbpqlp_factor with q + 1 + j iterations, at 2 + 2 j more passes
 * over A.  Errors: as pbpqlp_factor; EINVAL for a NULL, misaligned or aliased
 * Omega or ldo < l. */
pbpqlp_status pbpqlp_factor_sketch(const void* A, int64_t m, int64_t n, int64_t lda,
                                   pbpqlp_dtype dt, const void* Omega, int64_t ldo, int k, int p,
                                   int q, void* Q, int64_t ldq, double* L, int64_t ldl, void* P,
                                   int64_t ldp, const pbpqlp_opts* opts, pbpqlp_info* d_info,
                                   void* stream);

/* ---- orientation and rank-revealing outputs ----
 *
 * The paper states the method for an n1 x n2 matrix with n1 >= n2 and a
 * sketch A^T Phi, Phi n1 x d (Algorithm 1), and returns A ~= Q L P^T.
 * pbpqlp_factor runs that algorithm on A^T (sketch A Omega, Omega n x l), so
 * its outputs satisfy A ~= Q L^T P^T.  pbpqlp_factor_rr offers both, and the
 * parts of the factorization that reveal the numerical rank (Section IV-A:
 * the partition of R, eqs. (Rparti), (sigmak_R11), (2normR22); Section IV-C:
 * the partition of L, eq. (Lparti), and the Mathias-Stewart inequalities
 * sigma_min(L11) >= sigma_min(R11), sigma_1(L22) <= sigma_1(R22)).
 *
 *   PBPQLP_ORIENT_AT   : A ~= Q L^T P^T, Algorithm 1 applied to A^T (the form
 *                        of pbpqlp_factor, bit for bit).
 *   PBPQLP_ORIENT_A    : A ~= Q L P^T, Algorithm 1 as stated: Phi is m x l
 *                        (element (i, j) from flat index i l + j, the same
 *                        generator), the power passes alternate A^T and A,
 *                        the last QR is that of D = A Pbar (eq. (DQR)).  It is
 *                        the ORIENT_AT factorization of A^T with the roles of
 *                        Q and P exchanged.
 *   PBPQLP_ORIENT_AUTO : ORIENT_A when m >= n, else ORIENT_AT, i.e. the
 *                        algorithm runs on whichever of A, A^T has at least as
 *                        many rows as columns, as the paper assumes.
 * The rank-k pieces need no copy: with row-major storage Q[:, :k], P[:, :k]
 * and L11 = L[:k, :k] are the same pointers with the same leading dimensions,
 * and Q1 L11 P1^T (ORIENT_A) or Q1 L11^T P1^T (ORIENT_AT) is the rank-k
 * approximation Q1 Q1^T A of the paper's Section IV-B. */
#define PBPQLP_ORIENT_AT 0
#define PBPQLP_ORIENT_A 1
#define PBPQLP_ORIENT_AUTO 2

typedef struct {
  int orientation;          /* in: PBPQLP_ORIENT_*                                 */
  int orientation_used;     /* out (host, written on success): AT or A             */
  double* R;                /* out, optional (NULL): l x l FP64 device matrix,
                               row-major, ldr >= l: the upper-triangular R of the
                               last QR (eq. (DQR)), lower part written 0; its
                               diagonal holds the R-values                         */
  int64_t ldr;
  double rank_tol;          /* in, >= 0: threshold of the rank estimate            */
  int* d_rank;              /* out, optional device int: the numerical rank
                               estimated from the L-values, the number of leading
                               L_ii > rank_tol * L_11 before the first that is not
                               (0 for A = 0, l if none drops)                      */
} pbpqlp_rr;

/* pbpqlp_factor in the orientation rr->orientation, with the optional R and
 * rank outputs of rr (same stream semantics: R and *d_rank are valid once the
 * stream reaches the end of the call).  Arguments as pbpqlp_factor; in both
 * orientations Q is m x l and P is n x l.  Errors: as pbpqlp_factor; EINVAL
 * for rr == NULL, an unknown orientation, ldr < l, a misaligned or aliased R,
 * rank_tol < 0 or NaN. */
pbpqlp_status pbpqlp_factor_rr(const void* A, int64_t m, int64_t n, int64_t lda, pbpqlp_dtype dt,
                               int k, int p, int q, uint64_t seed, void* Q, int64_t ldq, double* L,
                               int64_t ldl, void* P, int64_t ldp, const pbpqlp_opts* opts,
                               pbpqlp_rr* rr, pbpqlp_info* d_info, void* stream);

/* ---- A in host memory (Section IV-E: when A is stored externally the method
 * needs 2q + 2 passes over it) ----
 *
 * pbpqlp_factor for an A that stays in host memory: every product with A or
 * A^T streams A once from the host in row panels of panel_rows rows (0: about
 * 256 MiB of rows; rounded up to a multiple of 256), copied on a copy stream
 * of the library's own into two device staging buffers in turn, so copies
 * overlap the kernels of the previous panel.  The same kernels as
 * pbpqlp_factor run on each panel: A X panel by panel; A^T X as a sum over
 * panels, every panel's partials kept and summed in a fixed order at the end
 * (deterministic).  With one panel (panel_rows >= m) the results equal
 * pbpqlp_factor's bit for bit for the same options; with several, the A^T X
 * sums run in another order (FP32/FP64 rounding differences only).
 *   A_host     : m x n row-major in host memory (lda >= n), dtype dt; memory
 *                from hipHostMalloc lets the copies run at full PCIe rate,
 *                pageable memory also works (the runtime stages it).  Read only.
 *   Q, L, P    : device outputs as in pbpqlp_factor (A ~= Q L^T P^T).
 * The call returns once the last panel has been copied (the caller may then
 * reuse A_host); the remaining kernels complete in order on `stream`.  Not
 * capturable in a HIP graph.  The workspace (pbpqlp_workspace_size_host)
 * includes the two staging buffers.  Errors: as pbpqlp_factor (ldq, ldl,
 * ldp, alignment, shapes); EINVAL for panel_rows < 0; EHIP when the copy
 * stream or its events cannot be created. */
pbpqlp_status pbpqlp_workspace_size_host(int64_t m, int64_t n, int64_t lda, int k, int p,
                                         pbpqlp_dtype dt, int64_t panel_rows,
                                         const pbpqlp_opts* opts, size_t* bytes);
pbpqlp_status pbpqlp_factor_host(const void* A_host, int64_t m, int64_t n, int64_t lda,
                                 pbpqlp_dtype dt, int k, int p, int q, uint64_t seed,
                                 int64_t panel_rows, void* Q, int64_t ldq, double* L, int64_t ldl,
                                 void* P, int64_t ldp, const pbpqlp_opts* opts, pbpqlp_info* d_info,
                                 void* stream);

/* ---- sparse A (Section IV-E: for a sparse A with z nonzeros each product with
 * A or A^T costs O(z d)) ----
 *
 * pbpqlp_factor for A given in CSR on the device:
 *   rowptr : m + 1 int64 (rowptr[0] = 0, nondecreasing, rowptr[m] = nnz);
 *   colind : nnz int32 in [0, n), distinct within a row (any order);
 *   vals   : nnz values of dtype dt.  All three are read only.
 * The sketch and power passes and the projection are row-gather products with
 * A's CSR (A X) and with the CSR of A^T (A^T X), which the call builds first
 * by a stable radix sort (each row of A^T in increasing row order of A), so
 * every output entry is summed in one fixed order: results are deterministic.
 * The orthonormalization stack (Grams, Cholesky, apply, the l x l QR) is the
 * dense path's; the outputs are those of pbpqlp_factor on the dense A up to
 * rounding (A ~= Q L^T P^T).  Only the native precision of dt is supported
 * (every opts precision NATIVE; the gathers are not matrix-core products):
 * EUNSUPPORTED otherwise.  Invalid structure (row pointers out of order or
 * range, column indices outside [0, n)) is not read out of bounds: such
 * entries are skipped and PBPQLP_FLAG_BADINPUT is set in d_info.
 * Errors: as pbpqlp_factor; EINVAL for nnz < 0, nnz, m or n of 2^31 - 1 or
 * more, null or misaligned arrays. */
pbpqlp_status pbpqlp_workspace_size_csr(int64_t m, int64_t n, int64_t nnz, int k, int p, pbpqlp_dtype dt,
                                        const pbpqlp_opts* opts, size_t* bytes);
pbpqlp_status pbpqlp_factor_csr(const int64_t* rowptr, const int32_t* colind, const void* vals, int64_t m,
                                int64_t n, int64_t nnz, pbpqlp_dtype dt, int k, int p, int q, uint64_t seed,
                                void* Q, int64_t ldq, double* L, int64_t ldl, void* P, int64_t ldp,
                                const pbpqlp_opts* opts, pbpqlp_info* d_info, void* stream);

/* ---- allocation-free variant ----
 *
 * For callers that cannot allocate device memory: code recorded under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc.
 * pbpqlp_factor_noalloc is pbpqlp_factor (same arguments, rules, kernels,
 * results bit for bit for the same options) with its workspace taken from a
 * static device array of PBPQLP_NOALLOC_SCRATCH_BYTES that the library holds
 * on every GPU it runs on until the process ends; opts.workspace is ignored.
 * It calls no hipMalloc, hipFree or other allocating routine and creates no
 * trace events.  All calls on one GPU share that GPU's array, which keeps the
 * last call's contents: calls that overlap on one GPU (different streams or
 * threads without ordering between them) race and give undefined results.
 * The device is the calling thread's current HIP device.
 * Errors: as pbpqlp_factor; EUNSUPPORTED when the problem's workspace
 * (pbpqlp_workspace_size) exceeds PBPQLP_NOALLOC_SCRATCH_BYTES (checked before
 * anything touches the device); EHIP if the array's address cannot be
 * obtained. */
#define PBPQLP_NOALLOC_SCRATCH_BYTES (64ull << 20)
pbpqlp_status pbpqlp_factor_noalloc(const void* A, int64_t m, int64_t n, int64_t lda,
                                    pbpqlp_dtype dt, int k, int p, int q, uint64_t seed, void* Q,
                                    int64_t ldq, double* L, int64_t ldl, void* P, int64_t ldp,
                                    const pbpqlp_opts* opts, pbpqlp_info* d_info, void* stream);

/* The approximation A_hat = Q L^T P^T (eq. (Ahat), for A^T) of a factorization:
 *   Q (m x l), P (n x l) in dtype dt, L (l x l FP64, lower triangular), all
 *   device, row-major; Ahat (m x n, dt, ldh >= n) is written.
 * Forms W = P L in FP64 (stored in dt), then the m x n product in tiles with
 * accumulation in dt.  Errors: EINVAL; ENOMEM (stream-ordered scratch). */
pbpqlp_status pbpqlp_reconstruct(const void* Q, int64_t ldq, const double* L, int64_t ldl, const void* P,
                                 int64_t ldp, int64_t m, int64_t n, int l, pbpqlp_dtype dt, void* Ahat,
                                 int64_t ldh, void* stream);
/* Explicit relative residual ||A - Q L^T P^T||_F / ||A||_F (one pass over A,
 * A_hat never stored): squares summed in FP64 per tile, tiles summed in a
 * fixed order; the product itself accumulates in dt, so for FP32 the result
 * is meaningful down to about 1e-6.  d_r: device, one double.  Cross-checks
 * the estimate of pbpqlp_info (sqrt(||A||^2 - ||L||^2) / ||A||), which needs
 * orthonormal Q and P.  Errors: EINVAL; ENOMEM. */
pbpqlp_status pbpqlp_residual(const void* A, int64_t lda, const void* Q, int64_t ldq, const double* L,
                              int64_t ldl, const void* P, int64_t ldp, int64_t m, int64_t n, int l,
                              pbpqlp_dtype dt, double* d_r, void* stream);

/* ---- single steps of the method, for validation against the oracle ---- */

/* The sketch matrix of eq. (c) / Algorithm 1 (randn): Omega (n x l, row-major,
 * ldo >= l) in dtype dt; element (i, j) is the Box-Muller normal of flat index
 * i*l + j under `seed`, rounded to bfloat16 with |x| < 2^-14 flushed to 0.
 * Runs the factorization's own generator (into stream-ordered scratch) and
 * copies it out.  Errors: EINVAL; EUNSUPPORTED for l > 256; ENOMEM. */
pbpqlp_status pbpqlp_omega(int64_t n, int l, uint64_t seed, pbpqlp_dtype dt,
                           void* Omega, int64_t ldo, void* stream);

/* One A-streaming pass (eq. (c) or (D) and the power-iteration products):
 *   trans == 0:  Y (m x l) = A X,   X is n x l;
 *   trans == 1:  Y (n x l) = A^T X, X is m x l.
 * All row-major in dtype dt; prec as in pbpqlp_prec (reduced precisions need
 * PBPQLP_F32).  fp16_scale_a as in pbpqlp_opts.  l <= 256. */
pbpqlp_status pbpqlp_matmul(int trans, const void* A, int64_t m, int64_t n, int64_t lda,
                            pbpqlp_dtype dt, const void* X, int64_t ldx, int l, int prec,
                            double fp16_scale_a, void* Y, int64_t ldy, void* stream);

/* orth()/qr() of a tall matrix (eqs. (Pbar), (DQR)): Y (rows x l, dtype dt,
 * row-major) = Q R with Q orthonormal (rows x l, dtype dt) and R upper
 * triangular l x l FP64 (ldr >= l, lower part written 0, diag >= 0), by
 * `passes` (1 or 2) CholeskyQR sweeps with FP64 Grams; passes = 2 gives an
 * orthonormal Q to working precision.  The second sweep is decided on the
 * device: when the first sweep's Q^T Q is already within 4 u32 (FP32) or
 * 2e-14 (FP64) of the identity in every entry, it takes the identity factor
 * and Q and R are those of the first sweep, bit for bit.  R may be NULL.
 * l <= rows, l <= 256. */
pbpqlp_status pbpqlp_orth(const void* Y, int64_t rows, int l, int64_t ldy, pbpqlp_dtype dt,
                          int passes, void* Q, int64_t ldq, double* R, int64_t ldr,
                          pbpqlp_info* d_info, void* stream);

/* The l x l stage (eq. (R^T = Pt Rt)): R^T = Qt L^T for an upper-triangular
 * FP64 R (l x l, ldr >= l): writes Qt (l x l, orthogonal, FP64, ldqt >= l)
 * and L (l x l lower triangular, diag >= 0, FP64, ldl >= l). */
pbpqlp_status pbpqlp_small_qr(const double* R, int l, int64_t ldr, double* Qt, int64_t ldqt,
                              double* L, int64_t ldl, pbpqlp_info* d_info, void* stream);

/* ---- batches of independent problems (many uneven sizes, one plan) ----
 *
 * One problem of a batch: the arguments of pbpqlp_factor for one matrix, with
 * the same meaning, layout and rules; `info` is that problem's device result
 * record or NULL.  All pointers are DEVICE pointers owned by the caller. */
typedef struct {
  const void* A;
  int64_t m, n, lda;
  int k, p, q;
  uint64_t seed;
  void* Q;
  int64_t ldq;
  double* L;
  int64_t ldl;
  void* P;
  int64_t ldp;
  pbpqlp_info* info;
} pbpqlp_problem;

typedef struct pbpqlp_batch pbpqlp_batch;  /* opaque plan */

/* Plan a batch (a project extension of the method: the same factorization as
 * pbpqlp_factor for every problem, Algorithm 1 for A^T each).  The plan owns a
 * device workspace for all problems (sized here, allocated with hipMalloc) and
 * a HIP graph with one kernel launch per stage of the method and per shape
 * class (problems whose tile counts or alignment differ use different kernel
 * instances), the per-problem parameters in a device table.  Problems with
 * different q form separate launch sequences inside the same graph.
 * opts: precision plan as for pbpqlp_factor; split_k and workspace are
 * ignored (every pass runs unsplit).  The problem list is copied; the caller's
 * buffers must stay valid while the plan is used.  Synchronous: returns after
 * the plan is ready.  Errors: EINVAL/EUNSUPPORTED as pbpqlp_factor would give
 * for any problem, ENOMEM if the workspace cannot be allocated, EHIP if graph
 * capture fails. */
pbpqlp_status pbpqlp_batch_create(int count, const pbpqlp_problem* problems, pbpqlp_dtype dt,
                                  const pbpqlp_opts* opts, pbpqlp_batch** out);
/* Factorize every problem of the plan: one graph launch on `stream`
 * (asynchronous; results and records valid when the stream reaches it). */
pbpqlp_status pbpqlp_batch_run(pbpqlp_batch* b, void* stream);
/* Run the same grouped launches without the graph (0) or through it (1, default). */
pbpqlp_status pbpqlp_batch_set_graph(pbpqlp_batch* b, int use_graph);
/* Kernel launches per run and workspace bytes of a plan. */
pbpqlp_status pbpqlp_batch_stats(const pbpqlp_batch* b, int* launches, size_t* workspace_bytes);
/* The per-problem plan the batch chose for problem i (0 <= i < count): its
 * contraction split count (always 1) and Gram workgroup target.  pbpqlp_factor
 * called with these two values in opts launches the same kernels with the same
 * parameters, so it gives the batch's results bit for bit.  EINVAL for a bad i. */
pbpqlp_status pbpqlp_batch_problem_plan(const pbpqlp_batch* b, int i, int* split_k,
                                        int* gram_workgroups);
/* Release a plan (its work must be complete). */
void pbpqlp_batch_destroy(pbpqlp_batch* b);
/* create + run + synchronize `stream` + destroy. */
pbpqlp_status pbpqlp_factor_batched(int count, const pbpqlp_problem* problems, pbpqlp_dtype dt,
                                    const pbpqlp_opts* opts, void* stream);

/* ---- autotuning of the launch plan per shape class ----
 * A shape class is (dtype, the three pass precisions, l rounded up to 32,
 * ceil(log2 m), ceil(log2 n), batched or not); its plan is the contraction
 * split of the A-streaming passes and the Gram workgroup target.  The tuners
 * time candidate plans on `stream` (one warm-up and the median of three runs
 * each, HIP events), synchronize, and store the fastest in a process-wide
 * cache that calls with automatic options consult.  Workspace sizes depend on
 * the plan: query pbpqlp_workspace_size after tuning. */
typedef struct {
  int split_k;              /* -1 = the built-in heuristic, else the forced split     */
  int gram_workgroups;
  double ms;                /* measured time of the plan (one call or one batch run) */
} pbpqlp_tune_plan;

/* Tune one problem's class by factorizing A (read only) with each of the
 * candidate plans (split: heuristic, 1, 2, 4, 8, 16; Gram target: 512, 64,
 * 256, 1024) into library-allocated outputs.  opts: precision plan (its split
 * and Gram fields are ignored).  out may be NULL.  Errors: as pbpqlp_factor. */
pbpqlp_status pbpqlp_tune_factor(const void* A, int64_t m, int64_t n, int64_t lda, pbpqlp_dtype dt,
                                 int k, int p, int q, uint64_t seed, const pbpqlp_opts* opts,
                                 pbpqlp_tune_plan* out, void* stream);
/* Tune the Gram target of a batch (candidates 4, 16, 64, 256 workgroups per
 * problem; the split is always 1) by creating and running a plan for each;
 * the problems' outputs are overwritten.  The choice is stored for the class
 * of problems[0], marked batched.  Errors: as pbpqlp_batch_create. */
pbpqlp_status pbpqlp_tune_batch(int count, const pbpqlp_problem* problems, pbpqlp_dtype dt,
                                const pbpqlp_opts* opts, pbpqlp_tune_plan* out, void* stream);
/* The cached plan of a class (batched = 0 or 1); EINVAL if none is cached. */
pbpqlp_status pbpqlp_tune_lookup(int64_t m, int64_t n, int k, int p, pbpqlp_dtype dt,
                                 const pbpqlp_opts* opts, int batched, pbpqlp_tune_plan* out);
/* Forget every cached plan. */
void pbpqlp_tune_clear(void);
/* Write the cache as text: a header line "# pbpqlp autotune v1 ...", then one
 * line per class: dt sketch power proj lp32 log2m log2n batched split_k
 * gram_workgroups ms.  Errors: EINVAL if the file cannot be written. */
pbpqlp_status pbpqlp_tune_save(const char* path);
/* Merge a file written by pbpqlp_tune_save into the cache (all or nothing).
 * Errors: EINVAL if the file cannot be read or a line does not parse. */
pbpqlp_status pbpqlp_tune_load(const char* path);

/* ---- learned choice of q and k (project extension; the paper has none) ----
 *
 * A q = 0 probe with l = 64 gives L whose diagonal tracks the leading singular
 * values of A (Section III-A, eq. (Ahat), and the diagonal bounds of Theorems
 * 3-5).  Its 64 features
 *     f_i = clip(ln(L_ii / L_11) / ln(1e6), -1, 1)   (-1 where the ratio is not
 *           above 1e-6, not finite, or L_11 <= 0)
 * feed an FP32 network 64 -> 128 (ReLU) -> 128 (ReLU) -> 6 whose outputs are
 * five logits for the power-iteration count q in {0..4} (Section III-B,
 * Algorithm 1) and a regression output for ln k.
 *
 * Parameters are one FP32 vector of PBPQLP_MLP_PARAMS values in the order
 * W1 (128 x 64, row-major: row j holds the weights into hidden unit j), b1 (128),
 * W2 (128 x 128), b2 (128), W3 (6 x 128), b3 (6).  Training minimizes, over a
 * batch of B samples, the mean softmax cross-entropy of the five logits
 * against the label q* plus the mean of (output_6 - ln k*)^2, with Adam
 * (Kingma and Ba 2015, beta1 0.9, beta2 0.999, eps 1e-8, bias-corrected). */
#define PBPQLP_MLP_IN 64
#define PBPQLP_MLP_HIDDEN 128
#define PBPQLP_MLP_OUT 6
#define PBPQLP_MLP_PARAMS 25606
#define PBPQLP_PROBE_K 56          /* probe: k = 56, p = 8, q = 0 (l = 64) */
#define PBPQLP_PROBE_P 8

typedef struct pbpqlp_model pbpqlp_model;   /* device parameters + Adam state */

/* New model with the given parameters (host array of PBPQLP_MLP_PARAMS
 * floats; NULL = all zero) and zero Adam state.  Allocates device memory.
 * Errors: EINVAL (out NULL), ENOMEM, EHIP. */
pbpqlp_status pbpqlp_model_create(const float* h_params, pbpqlp_model** out);
/* Load a model file written by pbpqlp_model_save (parameters, Adam moments and
 * step count: training resumes where it stopped).  Errors: EINVAL if the file
 * cannot be read or is not a model file of these dimensions; ENOMEM; EHIP. */
pbpqlp_status pbpqlp_model_load(const char* path, pbpqlp_model** out);
/* Write the model (synchronizes with the device).  File layout, little-endian:
 * 8-byte magic "PBQMLP01", int32 in, hidden, out, int32 reserved (0), int64
 * Adam step count, then parameters, first moments and second moments, each
 * PBPQLP_MLP_PARAMS float32.  Errors: EINVAL (cannot write), EHIP. */
pbpqlp_status pbpqlp_model_save(const pbpqlp_model* model, const char* path);
/* Copy the parameters to a host array of PBPQLP_MLP_PARAMS floats (synchronous). */
pbpqlp_status pbpqlp_model_get_params(const pbpqlp_model* model, float* h_params);
/* Adam steps taken so far. */
int64_t pbpqlp_model_steps(const pbpqlp_model* model);
/* Release a model (no work may still use it). */
void pbpqlp_model_free(pbpqlp_model* model);

/* Probe features from the diagonal of L (device, FP64, row-major, ldl >= 64,
 * at least 64 x 64) into f (device, 64 floats).  Errors: EINVAL. */
pbpqlp_status pbpqlp_probe_features(const double* L, int64_t ldl, float* f, void* stream);

/* Network outputs for `batch` feature rows: X (device, batch x 64 FP32,
 * row-major, ldx >= 64) -> Z (device, batch x 6 FP32, row-major, ldz >= 6).
 * Errors: EINVAL (batch < 1, bad leading dimensions, NULL). */
pbpqlp_status pbpqlp_mlp_forward(const pbpqlp_model* model, const float* X, int64_t ldx, int batch,
                                 float* Z, int64_t ldz, void* stream);
/* Loss of a batch and its gradient.  X as above; q (device, batch int32 in
 * 0..4), logk (device, batch floats).  Writes the loss to d_loss (device, one
 * float, may be NULL) and the gradient (PBPQLP_MLP_PARAMS floats, the same
 * order as the parameters) to the model's gradient buffer and, if d_grad is
 * not NULL, to d_grad (device).  The model's activation buffers grow to the
 * largest batch seen (device allocation, synchronous).  Calls on one model
 * must not overlap.  Errors: EINVAL, ENOMEM, EHIP. */
pbpqlp_status pbpqlp_mlp_loss_grad(pbpqlp_model* model, const float* X, int64_t ldx,
                                   const int* q, const float* logk, int batch, float* d_loss,
                                   float* d_grad, void* stream);
/* One Adam step on the gradient held in the model (from the last
 * pbpqlp_mlp_loss_grad), learning rate lr > 0.  Errors: EINVAL, EHIP. */
pbpqlp_status pbpqlp_mlp_adam_step(pbpqlp_model* model, float lr, void* stream);
/* pbpqlp_mlp_loss_grad followed by pbpqlp_mlp_adam_step. */
pbpqlp_status pbpqlp_mlp_train_step(pbpqlp_model* model, const float* X, int64_t ldx,
                                    const int* q, const float* logk, int batch, float lr,
                                    float* d_loss, void* stream);

/* What pbpqlp_factor_auto chose and measured (host struct). */
typedef struct {
  int q_pred, k_pred;        /* the network's choice                                   */
  int q_used, k_used;        /* what the returned factorization used                   */
  int fell_back;             /* 1: the predicted run's residual was above tau          */
  int passes;                /* passes over A in total, the probe's two included       */
  double resid_first;        /* residual estimate of the predicted choice              */
  double resid_final;        /* residual estimate of the returned factorization        */
} pbpqlp_auto_result;

/* Learned factorization.  The probe (k = 56, p = 8, q = 0, l = 64) is also the
 * first stage of the answer:
 *   probe -> features -> network -> q_hat = argmax of the logits (lowest index
 *   on ties), k_hat = exp(output_6) rounded to the nearest integer, clamped
 *   to [1, k_max];
 *   if q_hat > 0 the probe's power iterations are continued to q_hat
 *   (pbpqlp_factor_sketch with Omega = the current P), 2 passes per iteration;
 *   the answer is the rank-(k_hat + p) leading part of the l = 64
 *   factorization: Q and P cut to their first k_hat + p columns and L to its
 *   leading block (A ~= Q' L'^T P'^T);
 *   its residual is checked against tau by the estimate
 *   sqrt(||A||^2 - ||L'||^2) / ||A|| (exact for orthonormal factors, since
 *   Q'^T A P' = L'^T); for FP32, whose estimate carries an error of order
 *   1e-3, an estimate closer to tau than its error bound (2 sqrt(m + n) FP32
 *   units on r^2) is replaced by the explicit pbpqlp_residual pass; with any
 *   BF16 or FP16 pass in opts, whose rounding lies far above that band, every
 *   check is the explicit pass;
 *   if it exceeds tau (or a non-finite input was flagged) the fallback
 *   continues to q = 3 (when q_hat < 3) and returns k = k_max.
 * A plain run with q iterations costs 2 q + 2 passes; this path costs
 * 2 q_used + 2, the probe included, plus one pass per explicit check.
 *   A, dt, lda, seed, opts as for pbpqlp_factor (opts.workspace is ignored);
 *   requires min(m, n) >= 64, 1 <= k_max and k_max + p <= 64.
 *   Q (m x (k_used + p), ldq >= k_max + p), L ((k_used + p)^2, ldl >= k_max + p),
 *   P (n x (k_used + p), ldp >= k_max + p) as pbpqlp_factor writes them;
 *   d_info (may be NULL) describes the returned factorization (l = k_used + p).
 * Synchronizes `stream` (it reads the prediction and the residual on the
 * host), so it cannot be captured in a graph; its buffers are allocated and
 * freed stream-ordered.  Errors: as pbpqlp_factor, and EINVAL for a NULL
 * model, tau <= 0, or k_max, p outside the limits above. */
pbpqlp_status pbpqlp_factor_auto(const pbpqlp_model* model, const void* A, int64_t m, int64_t n,
                                 int64_t lda, pbpqlp_dtype dt, int p, uint64_t seed, int k_max,
                                 double tau, void* Q, int64_t ldq, double* L, int64_t ldl,
                                 void* P, int64_t ldp, const pbpqlp_opts* opts,
                                 pbpqlp_info* d_info, pbpqlp_auto_result* result, void* stream);

/* ---- instrumentation (benchmarking and profiling) ----
 * With level >= 1, every later call records a pair of HIP events on its
 * stream around each A-streaming product; with level >= 2 also around the
 * Gram, Cholesky and apply kernels.  Records accumulate in a process-wide
 * list until pbpqlp_trace_reset().  Reading a record's time is valid only
 * once its stream has completed the call.  Level 0 (the default) records
 * nothing; each record adds two event markers to the stream. */
void pbpqlp_trace_enable(int level);
void pbpqlp_trace_reset(void);
int pbpqlp_trace_count(void);
/* Record i: kernel class name (e.g. "k2_bf16", "gram", "chol"), its
 * algorithmic bytes (the operands read once and the result written once) and
 * flops, and the elapsed milliseconds between its two events.
 * Errors: EINVAL for i out of range; EHIP if the events are not complete. */
pbpqlp_status pbpqlp_trace_get(int i, char* name, int name_len, double* bytes, double* flops,
                               float* ms);

#ifdef __cplusplus
}
#endif
#endif /* PBPQLP_H */
