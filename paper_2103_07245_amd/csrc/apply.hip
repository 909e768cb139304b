// Products of a tall column-major matrix with an l x l operand, the last two
// steps of each orth()/qr() sweep and of the method:
//   apply      Q = Y Ra^-1      (CholeskyQR: triangular solve with the factor)
//   right_mul  Out = In M       (Q Qt of eq. (Ahat))
// One wave owns 16 rows and keeps their lp columns in registers as 16 x 16
// tiles in the matrix-core accumulator layout; the accumulator layout of a
// finished tile is also the B-operand layout of the next product, so tiles
// flow between products without leaving registers.  The l x l operand is
// staged in LDS by the block's four waves (one block per CU), in as few
// phases as its size allows; the tile count is a template parameter, so
// every loop bound and phase boundary is a compile-time constant and the
// scheduler sees one basic block per phase.
#include "common.h"
#include "kernels.h"
#include "launch.h"

namespace pbq {

constexpr int kOpLdsBytes = 144 * 1024;  // LDS for the staged operand
constexpr int kTile = 16 * 17;           // padded 16 x 16 tile in LDS

// ---------------------------------------------------------------------------
// Dependent columns (flagged by the Cholesky, count in dep[lp]) are replaced
// in place by the seeded unit-variance vector w_c / sqrt(len) before the
// solve; Ra has an identity row and column there, so the solve passes them
// through.  Blocks exit at once when no column is dependent.
// ---------------------------------------------------------------------------
struct CompleteP {
  void* Y;
  int64_t ldy, len;
  int l, lp;
  const int* dep;
  uint64_t seed;
  PBQ_GRID;
};

template <typename T, bool B>
__global__ __launch_bounds__(256) void complete_kernel(const CompleteP* pb, CompleteP ps) {
  bool past;
  const CompleteP p = kparams<B>(pb, ps, past);
  if (past) return;
  if (p.dep[p.lp] == 0) return;
  __shared__ int sd[kMaxL];
  for (int c = threadIdx.x; c < p.lp; c += blockDim.x) sd[c] = p.dep[c];
  __syncthreads();
  const int64_t row = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (row >= p.len) return;
  T* Y = (T*)p.Y;
  const double sc = 1.0 / sqrt((double)p.len);
#pragma nounroll
  for (int c = 0; c < p.l; ++c)
    if (sd[c]) Y[(int64_t)c * p.ldy + row] = (T)(normal_at((uint64_t)row, 1u, (uint32_t)c, p.seed) * sc);
}

// Row blocks of Ra staged per phase: row block J needs NT - J tiles (W_J and
// -Ra_JK for K > J); a phase holds consecutive row blocks up to MAXT tiles.
template <int NT, int MAXT> struct ApplyPhases {
  int n = 0;
  int j0[NT + 1] = {}, j1[NT + 1] = {};
  constexpr ApplyPhases() {
    int J = 0;
    while (J < NT) {
      int J1 = J, nt = 0;
      while (J1 < NT && nt + (NT - J1) <= MAXT) { nt += NT - J1; ++J1; }
      j0[n] = J;
      j1[n] = J1;
      ++n;
      J = J1;
    }
  }
};

template <int NT, int MAXT> inline constexpr ApplyPhases<NT, MAXT> kApplyPhases{};

// Tiles of LDS a triangular operand of NT tile rows needs: all NT (NT + 1) / 2
// upper tiles, or the MAXT of the largest phase.
template <int NT, int MAXT>
inline constexpr int kOpTiles = NT * (NT + 1) / 2 < MAXT ? NT * (NT + 1) / 2 : MAXT;

// Row-major output of one wave's 16 rows (lane li: row arow; columns < l).
// An FP32 accumulator register r of lane group g holds column 4 g + r of the
// tile, so a lane's four registers are four consecutive columns of its row:
// one 16-byte store where the row is 16-byte aligned and the four columns
// are live, else one store per element.
template <typename T, int NT>
__device__ __forceinline__ void store_rows(T* __restrict__ O, int64_t ldo, int64_t arow, bool in, int l, int lg,
                                           const typename Vec4<T>::type (&v)[NT]) {
  if constexpr (sizeof(T) == 4) {
    const bool vec = (ldo & 3) == 0 && ((uintptr_t)O & 15) == 0;  // uniform
#pragma unroll
    for (int J = 0; J < NT; ++J) {
      const int c0 = 16 * J + 4 * lg;
      if (vec && in && c0 + 3 < l) {
        *(typename Vec4<T>::type*)(O + arow * ldo + c0) = v[J];
      } else {
#pragma unroll
        for (int r = 0; r < 4; ++r)
          if (in && c0 + r < l) O[arow * ldo + c0 + r] = v[J][r];
      }
    }
  } else {
#pragma unroll
    for (int J = 0; J < NT; ++J)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int c = 16 * J + acc_row<T>(lg, r);
        if (in && c < l) O[arow * ldo + c] = v[J][r];
      }
  }
}

// Staging of phase P (row blocks J0 .. J1-1 of the operand) into LDS: one
// element of each tile per thread.
template <typename T, int NT, int MAXT, int P>
__device__ __forceinline__ void apply_stage(T* ops, const T* __restrict__ Ra, const T* __restrict__ Dinv, int lp,
                                            int tid) {
  constexpr auto& PH = kApplyPhases<NT, MAXT>;
  constexpr int J0 = PH.j0[P], J1 = PH.j1[P];
  const int si = tid >> 4, sc = tid & 15;
  int t = 0;
#pragma unroll
  for (int J = J0; J < J1; ++J)
#pragma unroll
    for (int K = J; K < NT; ++K, ++t)
      ops[t * kTile + si * 17 + sc] =
          (K == J) ? Dinv[J * 256 + si * 16 + sc] : -Ra[(int64_t)(16 * J + si) * lp + 16 * K + sc];
}

// The products of phase P on one wave's 16 rows (the operand staged).
template <typename T, int NT, int MAXT, int P>
__device__ __forceinline__ void apply_compute(typename Vec4<T>::type (&y)[NT], const T* ops, int li, int lg) {
  typedef typename Vec4<T>::type ACC;
  constexpr auto& PH = kApplyPhases<NT, MAXT>;
  constexpr int J0 = PH.j0[P], J1 = PH.j1[P];
  if constexpr (NT >= (sizeof(T) == 8 ? 8 : 7)) {
    // One wave per SIMD at these widths: the four operand values of tile
    // t + 1 are read from LDS before the products of tile t (left to itself
    // the scheduler waited out one LDS read per pair of products).  Narrower
    // operands run several waves per SIMD, which hide that latency, and the
    // extra operand registers would cost one of them.
    int nt = 0;
#pragma unroll
    for (int J = J0; J < J1; ++J) nt += NT - J;
    T a[2][4];
    auto fetch = [&](int tt) __attribute__((always_inline)) {
#pragma unroll
      for (int s4 = 0; s4 < 4; ++s4) a[tt & 1][s4] = ops[tt * kTile + acc_row<T>(lg, s4) * 17 + li];
    };
    fetch(0);
    int t = 0;
#pragma unroll
    for (int J = J0; J < J1; ++J) {
      if (t + 1 < nt) fetch(t + 1);
      __builtin_amdgcn_sched_barrier(0);
      ACC q = {0, 0, 0, 0};
#pragma unroll
      for (int s4 = 0; s4 < 4; ++s4) q = mma_native(a[t & 1][s4], y[J][s4], q);
      y[J] = q;
      ++t;
#pragma unroll
      for (int K = J + 1; K < NT; ++K, ++t) {
        if (t + 1 < nt) fetch(t + 1);
        __builtin_amdgcn_sched_barrier(0);
#pragma unroll
        for (int s4 = 0; s4 < 4; ++s4) y[K] = mma_native(a[t & 1][s4], q[s4], y[K]);
      }
    }
  } else {
    int t = 0;
#pragma unroll
    for (int J = J0; J < J1; ++J) {
      ACC q = {0, 0, 0, 0};
#pragma unroll
      for (int s4 = 0; s4 < 4; ++s4) q = mma_native(ops[t * kTile + acc_row<T>(lg, s4) * 17 + li], y[J][s4], q);
      y[J] = q;
      ++t;
#pragma unroll
      for (int K = J + 1; K < NT; ++K, ++t)
#pragma unroll
        for (int s4 = 0; s4 < 4; ++s4) y[K] = mma_native(ops[t * kTile + acc_row<T>(lg, s4) * 17 + li], q[s4], y[K]);
    }
  }
}

// One staging phase P of the substitution (row blocks J0 .. J1-1), then the next.
template <typename T, int NT, int MAXT, int P>
__device__ __forceinline__ void apply_phase(typename Vec4<T>::type (&y)[NT], T* ops,
                                            const T* __restrict__ Ra, const T* __restrict__ Dinv,
                                            int lp, int tid, int li, int lg) {
  constexpr auto& PH = kApplyPhases<NT, MAXT>;
  if constexpr (P < PH.n) {
    if constexpr (P > 0) lds_barrier();  // every wave is done with the previous phase
    apply_stage<T, NT, MAXT, P>(ops, Ra, Dinv, lp, tid);
    lds_barrier();
    apply_compute<T, NT, MAXT, P>(y, ops, li, lg);
    apply_phase<T, NT, MAXT, P + 1>(y, ops, Ra, Dinv, lp, tid, li, lg);
  }
}

// Right-looking blocked substitution: for J = 0, 1, ... the wave forms
// Q_J = Y_J W_J (W_J the inverse of the diagonal block) in place of Y_J and
// removes Q_J Ra_JK from every later tile K (independent chains).
struct ApplyP {
  const void* Y;
  int64_t ldy, len;
  int l, lp;
  const void* Ra;
  const void* Dinv;
  void* Qcm;
  int64_t ldq;
  void* Qrm;
  int64_t ldqr;
  int64_t wq;     // rows of Qcm written (padding rows up to ldq, or only len for a sub-matrix)
  const int* ident;  // set by the Cholesky of a later sweep whose factor is the identity: copy
  // optional 16-bit copy of Qcm (x xs) for the next A-streaming pass (same
  // layout, ld ldq): BF16 or FP16 in hi, and for split-BF16x3 the low BF16
  // part of x xs - hi in lo; emode 0 = none
  void* hi;
  void* lo;
  int emode;
  float xs;
  int rtiles;     // 64-row tiles per block (1 unless the operand is staged in one phase)
  PBQ_GRID;
};

// The 16-bit copies of one stored value (the conversion of a separate pass,
// done where the value is produced).
template <typename T>
__device__ __forceinline__ void store16(const ApplyP& p, int64_t off, T y) {
  if constexpr (sizeof(T) == 4) {
    const float v = (float)y * p.xs;
    if (p.emode == M_F16) {
      ((_Float16*)p.hi)[off] = (_Float16)v;
    } else {
      const __bf16 h = (__bf16)v;
      ((__bf16*)p.hi)[off] = h;
      if (p.emode == M_BF16X3) ((__bf16*)p.lo)[off] = (__bf16)(v - (float)h);
    }
  }
}

template <typename T, int NT, bool B>
__global__ __launch_bounds__(256) void apply_kernel(const ApplyP* pb, ApplyP ps) {
  bool past;
  const ApplyP prm = kparams<B>(pb, ps, past);
  if (past) return;
  const T* __restrict__ Y = (const T*)prm.Y;
  const int64_t ldy = prm.ldy, len = prm.len, ldq = prm.ldq, ldqr = prm.ldqr;
  const int l = prm.l, lp = prm.lp;
  const T* __restrict__ Ra = (const T*)prm.Ra;
  const T* __restrict__ Dinv = (const T*)prm.Dinv;
  T* __restrict__ Qcm = (T*)prm.Qcm;
  T* __restrict__ Qrm = (T*)prm.Qrm;
  typedef typename Vec4<T>::type ACC;
  constexpr int MAXT = kOpLdsBytes / (kTile * (int)sizeof(T));
  static_assert(MAXT >= NT, "a phase must hold one full row block");
  // LDS for the operand's upper tiles, or for one phase of them: narrow
  // operands leave room for several blocks per CU
  __shared__ T ops[kOpTiles<NT, MAXT> * kTile];
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63, li = lane & 15, lg = lane >> 4;
  // the identity factor of a later sweep leaves Y as it is (block-uniform test)
  const bool ident = prm.ident && *prm.ident;
  // an operand staged in one phase serves every row tile of the block
  constexpr bool single = kApplyPhases<NT, MAXT>.n == 1;
  const int rtiles = single ? prm.rtiles : 1;
  if (single && !ident) {
    apply_stage<T, NT, MAXT, 0>(ops, Ra, Dinv, lp, tid);
    lds_barrier();
  }
  auto finish = [&](int rt, ACC (&y)[NT]) __attribute__((always_inline)) {
    const int64_t arow = (((int64_t)blockIdx.x * rtiles + rt) * 4 + wave) * 16 + li;
    const bool in = arow < len;
    if (!ident) {
      if constexpr (single)
        apply_compute<T, NT, MAXT, 0>(y, ops, li, lg);
      else
        apply_phase<T, NT, MAXT, 0>(y, ops, Ra, Dinv, lp, tid, li, lg);
    }
#pragma unroll
    for (int J = 0; J < NT; ++J)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int c = 16 * J + acc_row<T>(lg, r);
        if (Qcm && arow < prm.wq) {
          Qcm[(int64_t)c * ldq + arow] = y[J][r];
          if (prm.emode) store16<T>(prm, (int64_t)c * ldq + arow, y[J][r]);
        }
        if (Qrm && in && c < l) Qrm[arow * ldqr + c] = y[J][r];
      }
  };
  if constexpr (single && NT * sizeof(T) <= 32) {
    // Narrow operands, several row tiles per block: the next tile's rows are
    // requested before the current tile's products.  The loads take no
    // branch (rows past len read row len - 1, whose values are replaced by
    // zeros), so the wait before a tile's products covers only its own loads.
    auto load_tile = [&](int rt, ACC (&dst)[NT]) __attribute__((always_inline)) {
      const int64_t arow = (((int64_t)blockIdx.x * rtiles + rt) * 4 + wave) * 16 + li;
      const bool in = arow < len;
      const int64_t rc = in ? arow : len - 1;
#pragma unroll
      for (int K = 0; K < NT; ++K)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const T v = Y[(int64_t)(16 * K + acc_row<T>(lg, r)) * ldy + rc];
          dst[K][r] = in ? v : T(0);
        }
    };
    ACC ya[NT], yb[NT];
    load_tile(0, ya);
    for (int rt = 0; rt < rtiles; rt += 2) {
      load_tile(rt + 1 < rtiles ? rt + 1 : rt, yb);
      finish(rt, ya);
      if (rt + 1 < rtiles) {
        load_tile(rt + 2 < rtiles ? rt + 2 : rt + 1, ya);
        finish(rt + 1, yb);
      }
    }
  } else {
    for (int rt = 0; rt < rtiles; ++rt) {
      const int64_t arow = (((int64_t)blockIdx.x * rtiles + rt) * 4 + wave) * 16 + li;
      const bool in = arow < len;
      ACC y[NT];
#pragma unroll
      for (int K = 0; K < NT; ++K)
#pragma unroll
        for (int r = 0; r < 4; ++r)
          y[K][r] = in ? Y[(int64_t)(16 * K + acc_row<T>(lg, r)) * ldy + arow] : T(0);
      finish(rt, y);
    }
  }
}

// Short tall matrices (the l x l stages, len <= 256 rows): one block per
// 16-row panel, its four waves splitting the column tiles (wave w owns
// K = w, w + 4, ...).  At step J the owner of column J forms Q_J = Y_J W_J
// and hands it to the others through LDS; every wave then removes Q_J Ra_JK
// from its own tiles K > J.  Each tile sees the same products in the same
// order as in apply_kernel, so the results agree bit for bit; the chain per
// step is one product, the hand-over and a barrier instead of a whole row
// of products in one wave.
template <typename T, int NT, int MAXT, int P>
__device__ __forceinline__ void apply_cols_phase(typename Vec4<T>::type (&y)[(NT + 3) / 4], T* ops, T (*qb)[16 * 17],
                                                 const T* __restrict__ Ra, const T* __restrict__ Dinv, int lp,
                                                 int tid, int wave, int li, int lg) {
  typedef typename Vec4<T>::type ACC;
  constexpr auto& PH = kApplyPhases<NT, MAXT>;
  if constexpr (P < PH.n) {
    constexpr int J0 = PH.j0[P], J1 = PH.j1[P];
    if constexpr (P > 0) lds_barrier();  // every wave is done with the previous phase
    const int si = tid >> 4, sc = tid & 15;
    {
      int t = 0;
#pragma unroll
      for (int J = J0; J < J1; ++J)
#pragma unroll
        for (int K = J; K < NT; ++K, ++t)
          ops[t * kTile + si * 17 + sc] =
              (K == J) ? Dinv[J * 256 + si * 16 + sc] : -Ra[(int64_t)(16 * J + si) * lp + 16 * K + sc];
    }
    lds_barrier();
    int t = 0;  // tile index of W_J in this phase; (J, K) follows at t + K - J
#pragma unroll
    for (int J = J0; J < J1; ++J) {
      if (wave == J % 4) {
        ACC q = {0, 0, 0, 0};
#pragma unroll
        for (int s4 = 0; s4 < 4; ++s4) q = mma_native(ops[t * kTile + acc_row<T>(lg, s4) * 17 + li], y[J / 4][s4], q);
        y[J / 4] = q;
#pragma unroll
        for (int r = 0; r < 4; ++r) qb[J & 1][acc_row<T>(lg, r) * 17 + li] = q[r];
      }
      lds_barrier();
      ACC q;
#pragma unroll
      for (int s4 = 0; s4 < 4; ++s4) q[s4] = qb[J & 1][acc_row<T>(lg, s4) * 17 + li];
#pragma unroll
      for (int sl = 0; sl < (NT + 3) / 4; ++sl) {
        const int K = wave + 4 * sl;
        if (K > J && K < NT) {
          const int tk = t + K - J;
#pragma unroll
          for (int s4 = 0; s4 < 4; ++s4) y[sl] = mma_native(ops[tk * kTile + acc_row<T>(lg, s4) * 17 + li], q[s4], y[sl]);
        }
      }
      t += NT - J;
    }
    apply_cols_phase<T, NT, MAXT, P + 1>(y, ops, qb, Ra, Dinv, lp, tid, wave, li, lg);
  }
}

template <typename T, int NT, bool B>
__global__ __launch_bounds__(256) void apply_cols_kernel(const ApplyP* pb, ApplyP ps) {
  bool past;
  const ApplyP prm = kparams<B>(pb, ps, past);
  if (past) return;
  const T* __restrict__ Y = (const T*)prm.Y;
  const int64_t ldy = prm.ldy, len = prm.len, ldq = prm.ldq, ldqr = prm.ldqr;
  const int l = prm.l, lp = prm.lp;
  T* __restrict__ Qcm = (T*)prm.Qcm;
  T* __restrict__ Qrm = (T*)prm.Qrm;
  typedef typename Vec4<T>::type ACC;
  constexpr int MAXT = kOpLdsBytes / (kTile * (int)sizeof(T));
  constexpr int NS = (NT + 3) / 4;
  static_assert(MAXT >= NT, "a phase must hold one full row block");
  __shared__ T ops[kOpTiles<NT, MAXT> * kTile];
  __shared__ T qb[2][16 * 17];
  const int tid = threadIdx.x, lane = tid & 63, li = lane & 15, lg = lane >> 4;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int64_t arow = (int64_t)blockIdx.x * 16 + li;
  const bool in = arow < len;
  ACC y[NS];
#pragma unroll
  for (int sl = 0; sl < NS; ++sl) {
    const int K = wave + 4 * sl;
#pragma unroll
    for (int r = 0; r < 4; ++r)
      y[sl][r] = (in && K < NT) ? Y[(int64_t)(16 * K + acc_row<T>(lg, r)) * ldy + arow] : T(0);
  }
  if (!(prm.ident && *prm.ident))
    apply_cols_phase<T, NT, MAXT, 0>(y, ops, qb, (const T*)prm.Ra, (const T*)prm.Dinv, lp, tid, wave, li, lg);
#pragma unroll
  for (int sl = 0; sl < NS; ++sl) {
    const int K = wave + 4 * sl;
    if (K < NT) {
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int c = 16 * K + acc_row<T>(lg, r);
        if (Qcm && arow < prm.wq) {
          Qcm[(int64_t)c * ldq + arow] = y[sl][r];
          if (prm.emode) store16<T>(prm, (int64_t)c * ldq + arow, y[sl][r]);
        }
        if (Qrm && in && c < l) Qrm[arow * ldqr + c] = y[sl][r];
      }
    }
  }
}

// Out = In M for a dense lp x lp M given row-major (Mr[k*ldm + j] = M[k][j]):
// all output tiles accumulate at once while row blocks I of M stream
// through LDS, MAXT / NT of them per phase.
struct RightMulP {
  const void* In;
  int64_t ldi, len;
  int l;
  const void* Mr;
  int64_t ldm;
  void* Ocm;
  int64_t ldo;
  void* Orm;
  int64_t ldor;
  PBQ_GRID;
};

template <typename T, int NT, bool B>
__global__ __launch_bounds__(256) void right_mul_kernel(const RightMulP* pb, RightMulP ps) {
  bool past;
  const RightMulP prm = kparams<B>(pb, ps, past);
  if (past) return;
  const T* __restrict__ In = (const T*)prm.In;
  const int64_t ldi = prm.ldi, len = prm.len, ldm = prm.ldm, ldo = prm.ldo, ldor = prm.ldor;
  const int l = prm.l;
  const T* __restrict__ Mr = (const T*)prm.Mr;
  T* __restrict__ Ocm = (T*)prm.Ocm;
  T* __restrict__ Orm = (T*)prm.Orm;
  typedef typename Vec4<T>::type ACC;
  constexpr int MAXT = kOpLdsBytes / (kTile * (int)sizeof(T));
  constexpr int RPP = MAXT / NT < NT ? MAXT / NT : NT;  // row blocks of M per phase
  static_assert(RPP >= 1, "a phase must hold one row block");
  __shared__ T ops[RPP * NT * kTile];
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63, li = lane & 15, lg = lane >> 4;
  const int64_t arow = ((int64_t)blockIdx.x * 4 + wave) * 16 + li;
  const bool in = arow < len;
  ACC x[NT], acc[NT];
#pragma unroll
  for (int I = 0; I < NT; ++I) {
    acc[I] = ACC{0, 0, 0, 0};
#pragma unroll
    for (int r = 0; r < 4; ++r)
      x[I][r] = in ? In[(int64_t)(16 * I + acc_row<T>(lg, r)) * ldi + arow] : T(0);
  }
  const int si = tid >> 4, sc = tid & 15;
#pragma unroll
  for (int I0 = 0; I0 < NT; I0 += RPP) {
    if (I0 > 0) lds_barrier();
#pragma unroll
    for (int I = I0; I < I0 + RPP && I < NT; ++I) {
#pragma unroll
      for (int J = 0; J < NT; ++J)
        ops[((I - I0) * NT + J) * kTile + si * 17 + sc] = Mr[(int64_t)(16 * I + si) * ldm + 16 * J + sc];
      __builtin_amdgcn_sched_barrier(0);  // at most one row block of loads in flight
    }
    lds_barrier();
    if constexpr (NT >= (sizeof(T) == 8 ? 8 : 7) && (sizeof(T) == 8 || NT < 16)) {
      // one wave per SIMD: tile t + 1's operands are read before tile t's
      // products (as in apply_compute; FP32 at 16 tiles already spills)
      const int I1 = I0 + RPP < NT ? I0 + RPP : NT;
      const int nt = (I1 - I0) * NT;
      T a[2][4];
      auto fetch = [&](int tt) __attribute__((always_inline)) {
#pragma unroll
        for (int s4 = 0; s4 < 4; ++s4) a[tt & 1][s4] = ops[tt * kTile + acc_row<T>(lg, s4) * 17 + li];
      };
      fetch(0);
#pragma unroll
      for (int t = 0; t < nt; ++t) {
        if (t + 1 < nt) fetch(t + 1);
        __builtin_amdgcn_sched_barrier(0);
        const int I = I0 + t / NT, J = t % NT;
#pragma unroll
        for (int s4 = 0; s4 < 4; ++s4) acc[J] = mma_native(a[t & 1][s4], x[I][s4], acc[J]);
      }
    } else {
#pragma unroll
      for (int I = I0; I < I0 + RPP && I < NT; ++I) {
#pragma unroll
        for (int J = 0; J < NT; ++J)
#pragma unroll
          for (int s4 = 0; s4 < 4; ++s4)
            acc[J] = mma_native(ops[((I - I0) * NT + J) * kTile + acc_row<T>(lg, s4) * 17 + li], x[I][s4], acc[J]);
        // bound the LDS operands in flight to one row block
        __builtin_amdgcn_sched_barrier(0);
      }
    }
  }
#pragma unroll
  for (int J = 0; J < NT; ++J)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int c = 16 * J + acc_row<T>(lg, r);
      if (Ocm && arow < ldo) Ocm[(int64_t)c * ldo + arow] = acc[J][r];
    }
  if (Orm) store_rows<T, NT>(Orm, ldor, arow, in, l, lg, acc);
}

// ---------------------------------------------------------------------------
// Launchers (tile count dispatched to the exact template)
// ---------------------------------------------------------------------------
template <typename T, int NT>
static hipError_t apply_launch(const void* Y, int64_t ldy, int64_t len, int lp, int l, const void* Ra,
                               const void* Dinv, const int* dep, uint64_t seed, void* Qcm, int64_t ldq,
                               void* Qrm, int64_t ldqr, hipStream_t s, int64_t wq, const int* ident,
                               const Emit16& em) {
  if (len < 1) return hipErrorInvalidValue;  // the row-tile loads assume a first row
  CompleteP c{(void*)Y, ldy, len, l, lp, dep, seed};
  hipError_t e = launch_k(complete_kernel<T, false>, complete_kernel<T, true>, dim3((unsigned)((len + 255) / 256)),
                          dim3(256), s, c);
  if (e != hipSuccess) return e;
  if (wq < 0) wq = ldq;
  const int64_t rows = Qcm ? (wq > len ? wq : len) : len;
  ApplyP p{Y, ldy, len, l, lp, Ra, Dinv, Qcm, ldq, Qrm, ldqr, wq, ident, em.hi, em.lo, em.mode, em.xs, 1};
  if constexpr (sizeof(T) == 8) {
    if (rows <= 256)  // the FP64 l x l stages: four waves per row panel
      return launch_k(apply_cols_kernel<T, NT, false>, apply_cols_kernel<T, NT, true>,
                      dim3((unsigned)((rows + 15) / 16)), dim3(256), s, p);
  }
  // Several 64-row tiles per block share one staging of the operand: in a
  // batch (the problems fill the chip together) and where the row tiles make
  // more than two rounds of the CUs.
  const int64_t tiles = (rows + 63) / 64;
  constexpr int MAXT = kOpLdsBytes / (kTile * (int)sizeof(T));
  if (kApplyPhases<NT, MAXT>.n == 1) {
    const int64_t cus = device_cus();
    const int64_t want = current_recorder() ? 4 : tiles / (2 * cus);
    p.rtiles = (int)(want < 1 ? 1 : (want > 4 ? 4 : want));
  }
  return launch_k(apply_kernel<T, NT, false>, apply_kernel<T, NT, true>,
                  dim3((unsigned)((tiles + p.rtiles - 1) / p.rtiles)), dim3(256), s, p);
}

template <typename T, int NT>
static hipError_t right_mul_launch(const void* In, int64_t ldi, int64_t len, int l, const void* Mr,
                                   int64_t ldm, void* Ocm, int64_t ldo, void* Orm, int64_t ldor,
                                   hipStream_t s) {
  const int64_t rows = Ocm ? (ldo > len ? ldo : len) : len;
  RightMulP p{In, ldi, len, l, Mr, ldm, Ocm, ldo, Orm, ldor};
  return launch_k(right_mul_kernel<T, NT, false>, right_mul_kernel<T, NT, true>, dim3((unsigned)((rows + 63) / 64)),
                  dim3(256), s, p);
}

#define PBQ_TILES(X) X(1) X(2) X(3) X(4) X(5) X(6) X(7) X(8) X(9) X(10) X(11) X(12) X(13) X(14) X(15) X(16)

hipError_t launch_apply(bool f64, const void* Y, int64_t ldy, int64_t len, int lp, int l,
                        const void* Ra, const void* Dinv, const int* dep, uint64_t seed, void* Qcm,
                        int64_t ldq, void* Qrm, int64_t ldqr, hipStream_t s, int64_t wq, const int* ident,
                        const Emit16& em) {
  if (lp % 16 || lp < 16 || lp > kMaxL) return hipErrorInvalidValue;
  switch (lp / 16) {
#define PBQ_CASE(N)                                                                                             \
  case N:                                                                                                       \
    return f64 ? apply_launch<double, N>(Y, ldy, len, lp, l, Ra, Dinv, dep, seed, Qcm, ldq, Qrm, ldqr, s, wq,   \
                                         ident, em)                                                           \
               : apply_launch<float, N>(Y, ldy, len, lp, l, Ra, Dinv, dep, seed, Qcm, ldq, Qrm, ldqr, s, wq, ident, \
                                        em);
    PBQ_TILES(PBQ_CASE)
#undef PBQ_CASE
  }
  return hipErrorInvalidValue;
}

hipError_t launch_right_mul(bool f64, const void* In, int64_t ldi, int64_t len, int lp, int l,
                            const void* Mr, int64_t ldm, void* Ocm, int64_t ldo, void* Orm,
                            int64_t ldor, hipStream_t s) {
  if (lp % 16 || lp < 16 || lp > kMaxL) return hipErrorInvalidValue;
  switch (lp / 16) {
#define PBQ_CASE(N)                                                                               \
  case N:                                                                                         \
    return f64 ? right_mul_launch<double, N>(In, ldi, len, l, Mr, ldm, Ocm, ldo, Orm, ldor, s)    \
               : right_mul_launch<float, N>(In, ldi, len, l, Mr, ldm, Ocm, ldo, Orm, ldor, s);
    PBQ_TILES(PBQ_CASE)
#undef PBQ_CASE
  }
  return hipErrorInvalidValue;
}

}  // namespace pbq
