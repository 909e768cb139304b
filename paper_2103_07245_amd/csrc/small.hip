// l x l stages of PbP-QLP in FP64: the Cholesky factor of a Gram matrix (the
// small half of a CholeskyQR sweep, i.e. of orth()/qr() in Algorithm 1),
// small products (R2 R1, U2 U1) and the result record.
#include "common.h"
#include "kernels.h"
#include "launch.h"
#include "../../include/pbpqlp.h"

namespace pbq {

// ---------------------------------------------------------------------------
// Upper Cholesky G = R^T R of an lp x lp Gram (only the first l columns are
// live; the rest is padding), one workgroup of 512 threads, blocked by 16.
// The upper triangle lives in registers as 16x16 tiles in the FP64
// matrix-core accumulator layout: wave w owns tile rows w and 15 - w
// (17 tiles for every wave), so every register index is a compile-time
// constant.  Panel J (16 columns) goes through
//   A. the owner of row J factors the (updated) diagonal tile in one wave
//      (diag_factor) and stages the rest of row J, as updated through panel
//      J - 2, in LDS;
//   B. all waves share the tiles K > J of row J: apply panel J - 1's update
//      G_JK -= R_{J-1,J}^T R_{J-1,K}, then R_JK = W_J^T G_JK on the FP64
//      matrix core (W_J = inverse of the apply form of R_JJ);
//   C. the owners of rows I > J + 1 apply the rank-16 update
//      G_IK -= R_JI^T R_JK.
// Step A of panel J+1 runs inside step C of panel J (lookahead): its owner
// only updates the diagonal tile with panel J before factoring it.  Two
// barriers per panel; no global memory inside the panel loop except W_J.
//
// Dependent columns: if the pivot satisfies !(d_k > eps * G_kk) (this also
// catches d_k <= 0, G_kk = 0 and NaN), column k carries no new direction.
// The "true" factor Rt gets a zero diagonal and a zero row k; the "apply"
// factor Ra gets an identity row and column k, so the triangular apply
// replaces column k of the tall matrix by a seeded random vector (a new
// orthonormal direction after the next sweep) while Y = Q Rt still holds.
// Padding columns (>= l) get 0 in Rt and identity in Ra and are not flagged.
// Outputs: Rt (FP64, ldr), Ra (T, ld lp), Dinv (T, W_J for every panel),
// dep[c] in {0,1} for c < lp and their count dep[lp], status bits in info.
// ---------------------------------------------------------------------------
constexpr int kCholThreads = 512;

struct CholShared {
  double gd[kMaxL];
  int sdep[kMaxL];
  double dgt[16][17];            // diagonal tile: residual in, true R_JJ out
  double winv[16][17];           // W_J = inverse of the apply form of R_JJ
  double pnl[2][16][kMaxL + 1];  // panel rows, double buffered: raw G_J,: in, R_J,: out
  int sflag;
  int sflag2;
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

// Lanes 16..31 (and 48..63) receive lanes 0..15 (32..47); the even rows keep
// their values (v_permlane16_swap of a register with itself).
__device__ __forceinline__ double dup_even_rows(double v) {
  const unsigned long long b = __double_as_longlong(v);
  const unsigned lo = (unsigned)b, hi = (unsigned)(b >> 32);
  const auto rl = __builtin_amdgcn_permlane16_swap(lo, lo, false, false);
  const auto rh = __builtin_amdgcn_permlane16_swap(hi, hi, false, false);
  return __longlong_as_double(((unsigned long long)rh[0] << 32) | rl[0]);
}

// x -= s[lane I of the lane row] * v in one instruction: the 64-bit FMA takes
// its first operand through a DPP row broadcast (v_fmac_f64 with
// row_newbcast).  The caller orders the definition of s at least two wait
// states before the first such read (the assembler block is opaque to the
// compiler's hazard tracking).
template <int I> __device__ __forceinline__ void fma_bcast(double& x, double s, double v) {
  asm("v_fmac_f64_dpp %0, -%1, %2 row_newbcast:%3 row_mask:0xf bank_mask:0xf"
      : "+v"(x)
      : "v"(s), "v"(v), "n"(I));
}

// One wave factors the 16x16 residual diagonal tile.  Lane row 0 (lanes
// 0..15) holds the tile's columns, lane row 1 (lanes 16..31) the columns of
// an identity; the same row operations (scale row k by 1/r_kk, subtract
// r_ki times row k from row i) run on both, so lane row 1 ends with
// M = R^-T of the apply form and W_J = M^T.  After each pivot the scaled
// row k of the tile is copied into lane row 1 (one permlane swap), so one
// broadcast FMA per row serves both halves.  A dependent or padding pivot zeroes row k of the tile and resets
// row k of M to e_k (M is then the inverse transpose of the apply form).
// Entries below the diagonal of the tile are updated too and never read.
//
// The pivot chain runs on uniform scalars, apart from the row updates: with
// a = T[k][k+1] and b = T[k+1][k+1] as updated through pivot k - 1 (read
// from lane k + 1 once those two rows are updated), pivot k + 1 is
// b - (a / r_kk)^2, so each step of the chain is a multiply, an FMA and the
// reciprocal square root, while the fifteen row updates of a step overlap it.
// The diagonal of the scaled tile row is T[k][k] / r_kk, i.e. r_kk to a
// rounding.  The dependence test of all sixteen columns is one compare and
// a ballot, so the step needs no lane reads for it.
struct DiagState {
  double x[16];
  double thr;  // eps * G_cc of the lane's column
  int c, live;
  bool tile_lane;
  uint32_t depm;
};

// 1/sqrt(x) for x > 0 to about one rounding unit: hardware estimate, then
// two Newton steps y <- y (3/2 - (x/2) y^2).  Non-positive x gives a
// non-finite y, which the caller never uses (such a pivot is dependent).
__device__ __forceinline__ double rsqrt_nr(double x) {
  double y = __builtin_amdgcn_rsq(x);
  const double hx = 0.5 * x;
#pragma unroll
  for (int it = 0; it < 2; ++it) {
    const double r = __builtin_fma(-(hx * y), y, 0.5);
    y = __builtin_fma(y, r, y);
  }
  return y;
}

template <int I, int K>
__device__ __forceinline__ void diag_rest(DiagState& d, double s, double v) {
  if constexpr (I < 16) {
    fma_bcast<I>(d.x[I], s, v);
    diag_rest<I + 1, K>(d, s, v);
  }
}

// step K: pivot value p (uniform) with its 1/sqrt y, and the two entries
// a = T[K][K+1], b = T[K+1][K+1] for the next pivot
template <int K>
__device__ __forceinline__ void diag_steps(DiagState& d, double p, double y, double a, double b) {
  if constexpr (K < 16) {
    // dependence test of every lane's column at once; bit K decides
    const uint64_t dm = __builtin_amdgcn_ballot_w64(!(p > d.thr));
    const bool zero = K >= d.live || ((dm >> K) & 1);
    double ys = y;
    double v = d.x[K] * y;
    if (zero) {
      d.depm |= K < d.live ? (1u << K) : 0u;
      ys = 0.0;
      v = (!d.tile_lane && d.c == K) ? 1.0 : 0.0;
    }
    d.x[K] = v;
    double s = dup_even_rows(v);  // the scaled tile row K, in both lane rows
    asm volatile("s_nop 4" : "+v"(s));
    if constexpr (K + 1 < 16) {
      // the chain: next pivot from a and b
      const double t = a * ys;
      const double pn = __builtin_fma(-t, t, b);
      const double yn = rsqrt_nr(pn);
      double an = 0.0, bn = 0.0;
      fma_bcast<K + 1>(d.x[K + 1], s, v);
      if constexpr (K + 2 < 16) {
        fma_bcast<K + 2>(d.x[K + 2], s, v);
        asm volatile("s_nop 1" : "+v"(d.x[K + 1]), "+v"(d.x[K + 2]));
        an = bcast_f64(d.x[K + 1], K + 2);
        bn = bcast_f64(d.x[K + 2], K + 2);
        diag_rest<K + 3, K>(d, s, v);
      }
      diag_steps<K + 1>(d, pn, yn, an, bn);
    }
  }
}

// Factor diagonal tile J (tin, 16 x 17) into R_JJ (rout, upper triangle,
// zeros below) and W_J (wout[c][i]); flags of its dependent columns go to
// sdep[16 J + c].  rout may alias tin.
__device__ __forceinline__ void diag_factor(const double (*tin)[17], double (*rout)[17], double (*wout)[17],
                                            const double* gd, int* sdep, int J, int l, double eps) {
  const int lane = threadIdx.x & 63;
  DiagState d;
  d.c = lane & 15;
  d.tile_lane = lane < 16;
  const bool ml = lane >= 16 && lane < 32;
#pragma unroll
  for (int i = 0; i < 16; ++i) d.x[i] = d.tile_lane ? tin[i][d.c] : ((i == d.c) ? 1.0 : 0.0);
  d.thr = eps * gd[16 * J + d.c];
  d.live = l - 16 * J;
  d.depm = 0;
  asm volatile("s_nop 4" : "+v"(d.x[0]), "+v"(d.x[1]), "+v"(d.x[2]));
  const double p0 = bcast_f64(d.x[0], 0);
  const double y0 = rsqrt_nr(p0);
  diag_steps<0>(d, p0, y0, bcast_f64(d.x[0], 1), bcast_f64(d.x[1], 1));
  if (d.tile_lane) {
#pragma unroll
    for (int i = 0; i < 16; ++i) rout[i][d.c] = (i <= d.c) ? d.x[i] : 0.0;
    sdep[16 * J + d.c] = (d.depm >> d.c) & 1u;
  } else if (ml) {
#pragma unroll
    for (int i = 0; i < 16; ++i) wout[d.c][i] = d.x[i];
  }
}

struct CholP {
  const double* G;
  int64_t ldg;
  int l, lp;
  double eps;
  double* Rt;
  int64_t ldr;
  void* Ra;
  void* Dinv;
  int* dep;
  pbpqlp_info* info;
  const double* gdiag;  // dependence reference diagonal, or null (G's own)
  int* ident;           // later sweep: set to 1 when G is the identity to the Gram
  const int* far;       // reduction's tolerance (far: its per-row flags), else 0
  PBQ_GRID;
};

// A later CholeskyQR sweep: the Gram reduction flagged, per row and 64-column
// block, any |G_ij - delta_ij| above the tolerance (i, j < l; NaN counts).
// With no flag the sweep's input is already orthonormal to that tolerance:
// the factor is the identity (the sweep's apply copies, R2 R1 copies R1), no
// column is dependent, *ident = 1 and the caller returns; else *ident = 0 and
// the factorization proceeds.  Nothing else is written on the identity path.
template <typename T>
__device__ __forceinline__ bool chol_identity(const CholP& prm, int* sflag2) {
  const int tid = threadIdx.x, l = prm.l, lp = prm.lp;
  const int nf = l * ((lp + 63) / 64);
  if (tid == 0) *sflag2 = 0;
  __syncthreads();
  bool far = false;
  for (int e = tid; e < nf; e += kCholThreads) far = far || prm.far[e] != 0;
  if (far) atomicOr(sflag2, 1);
  __syncthreads();
  const bool id = *sflag2 == 0;
  if (id)
    for (int e = tid; e <= lp; e += kCholThreads) prm.dep[e] = 0;
  if (tid == 0) *prm.ident = id ? 1 : 0;
  return id;
}

template <typename T, bool B>
__global__ __launch_bounds__(kCholThreads) void chol_kernel(const CholP* pb, CholP ps) {
  bool past;
  const CholP prm = kparams<B>(pb, ps, past);
  if (past) return;
  const double* __restrict__ G = prm.G;
  const int64_t ldg = prm.ldg;
  const int l = prm.l, lp = prm.lp;
  const double eps = prm.eps;
  double* __restrict__ Rt = prm.Rt;
  const int64_t ldr = prm.ldr;
  T* __restrict__ Ra = (T*)prm.Ra;
  T* __restrict__ Dinv = (T*)prm.Dinv;
  int* __restrict__ dep = prm.dep;
  pbpqlp_info* info = prm.info;
  __shared__ CholShared sh;
  const int tid = threadIdx.x, lane = tid & 63, li = lane & 15, lg = lane >> 4;
  if (tid < kMaxL) {
    sh.gd[tid] = (tid < l) ? (prm.gdiag ? prm.gdiag[tid] : G[(int64_t)tid * ldg + tid]) : 0.0;
    sh.sdep[tid] = 0;
  }
  if (tid == 0) sh.sflag = 0;
  __syncthreads();
  if (prm.ident && chol_identity<T>(prm, &sh.sflag2)) return;
  if (tid < l && !isfinite(sh.gd[tid])) atomicOr(&sh.sflag, 1);

  // wave w owns tile rows RA = w and RB = 15 - w: slots 0..NA-1 hold
  // (RA, RA + j), slots NA..15 hold (RB, j) and slot 16 the diagonal (RB, RB).
  const int w = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int Tn = lp >> 4;
  constexpr int NS = 17;
  f64x4 t[NS];
  {
    const int RA = w, RB = 15 - w, NA = 16 - w;
#pragma unroll
    for (int j = 0; j < NS; ++j) {
      const int I = j == 16 ? RB : (j < NA ? RA : RB);
      const int K = j == 16 ? RB : (j < NA ? RA + j : j);
#pragma unroll
      for (int r = 0; r < 4; ++r)
        t[j][r] = (K < Tn) ? G[(int64_t)(16 * I + acc_row<double>(lg, r)) * ldg + 16 * K + li] : 0.0;
    }
  }

  // Step A for panel J by its owner: factor the diagonal tile (slot 0 if
  // J == RA, else slot 16), stage the rest of row J in pnl[J & 1], emit W_J.
  auto step_a = [&](int J, int RA, int NA) {
    const bool a = J == RA;
#pragma unroll
    for (int r = 0; r < 4; ++r) sh.dgt[acc_row<double>(lg, r)][li] = a ? t[0][r] : t[16][r];
    wave_lds_fence();
    diag_factor(sh.dgt, sh.dgt, sh.winv, sh.gd, sh.sdep, J, l, eps);
    wave_lds_fence();
    // value selects only: a store through a selected tile address would force
    // the tile array into scratch memory
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const double v = sh.dgt[acc_row<double>(lg, r)][li];
      t[0][r] = a ? v : t[0][r];
      t[16][r] = a ? t[16][r] : v;
    }
    double(*pn)[kMaxL + 1] = sh.pnl[J & 1];
#pragma unroll
    for (int j = 0; j < 16; ++j) {
      const int I = j < NA ? RA : 15 - RA;
      const int K = j < NA ? RA + j : j;
      if (I == J && K > J && K < Tn) {
#pragma unroll
        for (int r = 0; r < 4; ++r) pn[acc_row<double>(lg, r)][16 * K + li] = t[j][r];
      }
    }
    if (lane < 16) {
#pragma unroll
      for (int i = 0; i < 16; ++i) Dinv[J * 256 + i * 16 + li] = (T)sh.winv[i][li];
    }
  };
  // G_IK -= R_JI^T R_JK for slot j (panel J in pnl[J & 1])
  auto update = [&](int j, int J, int I, int K) {
    double(*pn)[kMaxL + 1] = sh.pnl[J & 1];
    // all eight operands requested before the first product
    double xa[4], xb[4];
#pragma unroll
    for (int s4 = 0; s4 < 4; ++s4) {
      const int kk = acc_row<double>(lg, s4);
      xa[s4] = pn[kk][16 * I + li];
      xb[s4] = pn[kk][16 * K + li];
    }
    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int s4 = 0; s4 < 4; ++s4) t[j] = mma_f64(-xa[s4], xb[s4], t[j]);
  };

  if (w == 0) step_a(0, 0, 16);  // panel 0 belongs to wave 0 (RA = 0)
  lds_barrier();

  for (int J = 0; J < Tn; ++J) {
    // Re-derive the wave's tile coordinates each step from an opaque scalar
    // copy of w: hoisted out of the loop they would hold 34 VGPRs of LDS
    // offsets; recomputed they cost a few scalar instructions.
    int wl;
    asm volatile("s_mov_b32 %0, %1" : "=s"(wl) : "s"(w));
    const int RA = wl, RB = 15 - wl, NA = 16 - wl;
    auto tile_i = [&](int j) { return j == 16 ? RB : (j < NA ? RA : RB); };
    auto tile_k = [&](int j) { return j == 16 ? RB : (j < NA ? RA + j : j); };
    double(*pn)[kMaxL + 1] = sh.pnl[J & 1];
    double(*pp)[kMaxL + 1] = sh.pnl[(J + 1) & 1];  // panel J - 1

    // ---- B: K = J + 1 + wl, J + 9 + wl
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const int K = J + 1 + wl + 8 * h;
      if (K < Tn) {
        f64x4 g;
#pragma unroll
        for (int r = 0; r < 4; ++r) g[r] = pn[acc_row<double>(lg, r)][16 * K + li];
        if (J > 0) {
#pragma unroll
          for (int s4 = 0; s4 < 4; ++s4) {
            const int kk = acc_row<double>(lg, s4);
            g = mma_f64(-pp[kk][16 * J + li], pp[kk][16 * K + li], g);
          }
        }
        // the updated tile is the B operand as it stands: accumulator
        // register r of lane group g holds row g + 4 r, which is the
        // contraction index that lane group takes in step r
        f64x4 acc = {0, 0, 0, 0};
#pragma unroll
        for (int s4 = 0; s4 < 4; ++s4) acc = mma_f64(sh.winv[acc_row<double>(lg, s4)][li], g[s4], acc);
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int row = acc_row<double>(lg, r);
          pn[row][16 * K + li] = sh.sdep[16 * J + row] ? 0.0 : acc[r];
        }
      }
    }
    lds_barrier();
    // the owner of row J keeps R_J,: in its registers (the factor's output)
    if (J == RA || J == RB) {
#pragma unroll
      for (int j = 0; j < 16; ++j) {
        const int I = tile_i(j), K = tile_k(j);
        if (I == J && K > J && K < Tn) {
#pragma unroll
          for (int r = 0; r < 4; ++r) t[j][r] = pn[acc_row<double>(lg, r)][16 * K + li];
        }
      }
    }
    // ---- C with lookahead: the owner of row J + 1 updates its diagonal tile
    // and factors it first (raised priority: it is the critical path)
    const int J1 = J + 1;
    if (J1 < Tn && (J1 == RA || J1 == RB)) {
      __builtin_amdgcn_s_setprio(3);
      if (J1 == RA) update(0, J, RA, RA); else update(16, J, RB, RB);
      step_a(J1, RA, NA);
      __builtin_amdgcn_s_setprio(0);
    }
#pragma unroll
    for (int j = 0; j < NS; ++j) {
      const int I = tile_i(j), K = tile_k(j);
      if (I > J1 && K < Tn) update(j, J, I, K);
      // bound the LDS operands in flight (the tiles already hold 136 VGPRs)
      if (j % 2 == 1) __builtin_amdgcn_sched_barrier(0);
    }
    lds_barrier();
  }
  __syncthreads();
  // write Rt (true factor) and Ra (apply factor); mirror tiles below the diagonal are zero
  {
    const int RA = w, RB = 15 - w, NA = 16 - w;
#pragma unroll
    for (int j = 0; j < NS; ++j) {
      const int I = j == 16 ? RB : (j < NA ? RA : RB);
      const int K = j == 16 ? RB : (j < NA ? RA + j : j);
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
  }
  if (tid < lp) dep[tid] = sh.sdep[tid];
  if (tid == 0) {
    int nd = 0;
    for (int k = 0; k < l; ++k) nd += sh.sdep[k];
    dep[lp] = nd;  // count of dependent columns: the completion pass skips when 0
    if (nd && info) {
      atomicAdd(&info->n_dependent, nd);
      atomicOr(&info->status_flags, PBPQLP_FLAG_DEPENDENT);
    }
    if (sh.sflag && info) atomicOr(&info->status_flags, PBPQLP_FLAG_NONFINITE);
  }
}

// ---------------------------------------------------------------------------
// The same factorization for lp <= 224 (at most 14 tile rows) with the
// diagonal tiles factored by a wave of their own.  Waves 0..6 own tile rows
// w and 13 - w (15 tiles each); wave 7 owns no tile.  Panel J:
//   wave 7: R_{J,J+1} = W_J^T (G_{J,J+1} - R_{J-1,J}^T R_{J-1,J+1}) (B for
//      one tile), then diagonal tile J + 1 as its owner left it (updated
//      through panel J - 1) gets panel J's update G -= R_{J,J+1}^T R_{J,J+1}
//      and is factored (R_{J+1,J+1} and W_{J+1} into LDS);
//   waves 0..6: B for the tiles K >= J + 2 of row J, a meeting of these
//      seven waves on an LDS counter (wave 7 does not wait for it), then the
//      rank-16 updates of rows I > J + 1; the owner of row J + 2 hands its
//      diagonal tile (updated through panel J) to wave 7 for the next panel
//      and the owner of row J + 1 stages that row for the next B.
// The chain of diagonal factors is thus one B tile, the diagonal update and
// the factor per panel, with one workgroup barrier at the panel's end.
// The updates of rows I > J + 1 never read R_{J,J+1}; its row owner picks it
// up in the next panel.  W_J of every panel stays in LDS and is written out
// at the end.
// ---------------------------------------------------------------------------
constexpr int kDwRows = 14;

struct CholSharedDW {
  double gd[kMaxL];
  int sdep[kMaxL];
  double dgt[16][17];             // diagonal tile being factored
  double dbuf[2][16][17];         // diagonal tile J from its owner (through panel J - 2)
  double rjj[2][16][17];          // R_JJ for its owner
  double wall[kDwRows][16][17];   // W_J of every panel
  double pnl[2][16][kMaxL + 1];   // panel rows, double buffered: raw G_J,: in, R_J,: out
  int sflag;
  int sflag2;
  int bcnt;                       // B tiles done: 7 per panel, one per tile wave
};

// Spin until *p >= target (LDS, workgroup scope).  The wait is bounded: after
// about 2^22 polls it gives up and returns false (the caller flags it).
__device__ __forceinline__ bool lds_wait_geq(int* p, int target) {
  for (int it = 0; it < (1 << 22); ++it) {
    if (__hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP) >= target) return true;
    __builtin_amdgcn_s_sleep(1);
  }
  return false;
}

template <typename T, bool B>
__global__ __launch_bounds__(kCholThreads) void chol_dw_kernel(const CholP* pb, CholP ps) {
  bool past;
  const CholP prm = kparams<B>(pb, ps, past);
  if (past) return;
  const double* __restrict__ G = prm.G;
  const int64_t ldg = prm.ldg;
  const int l = prm.l, lp = prm.lp;
  const double eps = prm.eps;
  double* __restrict__ Rt = prm.Rt;
  const int64_t ldr = prm.ldr;
  T* __restrict__ Ra = (T*)prm.Ra;
  T* __restrict__ Dinv = (T*)prm.Dinv;
  int* __restrict__ dep = prm.dep;
  pbpqlp_info* info = prm.info;
  __shared__ CholSharedDW sh;
  const int tid = threadIdx.x, lane = tid & 63, li = lane & 15, lg = lane >> 4;
  if (tid < kMaxL) {
    sh.gd[tid] = (tid < l) ? (prm.gdiag ? prm.gdiag[tid] : G[(int64_t)tid * ldg + tid]) : 0.0;
    sh.sdep[tid] = 0;
  }
  if (tid == 0) {
    sh.sflag = 0;
    sh.bcnt = 0;
  }
  __syncthreads();
  if (prm.ident && chol_identity<T>(prm, &sh.sflag2)) return;
  if (tid < l && !isfinite(sh.gd[tid])) atomicOr(&sh.sflag, 1);

  // tile wave w owns rows RA = w and RB = 13 - w: slots 0..NA-1 hold
  // (RA, RA + j), slots NA..13 hold (RB, j) and slot 14 the diagonal (RB, RB)
  const int w = __builtin_amdgcn_readfirstlane(tid >> 6);
  const bool dw = w == 7;
  const int Tn = lp >> 4;
  constexpr int NS = 15;
  f64x4 t[NS];
  {
    const int RA = w, RB = 13 - w, NA = 14 - w;
#pragma unroll
    for (int j = 0; j < NS; ++j) {
      const int I = j == 14 ? RB : (j < NA ? RA : RB);
      const int K = j == 14 ? RB : (j < NA ? RA + j : j);
#pragma unroll
      for (int r = 0; r < 4; ++r)
        t[j][r] = (!dw && K < Tn) ? G[(int64_t)(16 * I + acc_row<double>(lg, r)) * ldg + 16 * K + li] : 0.0;
    }
  }
  // the owner's tile slot of diagonal tile R (R == RA or R == RB)
  auto put_diag = [&](int R, int RA, double (*dst)[17]) {
#pragma unroll
    for (int r = 0; r < 4; ++r) dst[acc_row<double>(lg, r)][li] = R == RA ? t[0][r] : t[14][r];
  };
  // stage the tiles K > R of row R (R == RA or R == RB) into pn
  auto stage_row = [&](int R, int RA, int NA, double (*pn)[kMaxL + 1]) {
#pragma unroll
    for (int j = 0; j < NS - 1; ++j) {
      const int I = j < NA ? RA : 13 - RA;
      const int K = j < NA ? RA + j : j;
      if (I == R && K > R && K < Tn) {
#pragma unroll
        for (int r = 0; r < 4; ++r) pn[acc_row<double>(lg, r)][16 * K + li] = t[j][r];
      }
    }
  };

  if (!dw) {
    if (w == 0) {  // row 0: diagonal tile and panel 0
      put_diag(0, 0, sh.dbuf[0]);
      stage_row(0, 0, 14, sh.pnl[0]);
    }
    if (w == 1 && Tn > 1) put_diag(1, 1, sh.dbuf[1]);
  }
  lds_barrier();
  if (dw) {
    __builtin_amdgcn_s_setprio(3);
    diag_factor(sh.dbuf[0], sh.rjj[0], sh.wall[0], sh.gd, sh.sdep, 0, l, eps);
  }
  lds_barrier();

  for (int J = 0; J < Tn; ++J) {
    // tile coordinates re-derived each panel from an opaque scalar copy of w
    int wl;
    asm volatile("s_mov_b32 %0, %1" : "=s"(wl) : "s"(w));
    const int RA = wl, RB = 13 - wl, NA = 14 - wl;
    auto tile_i = [&](int j) { return j == 14 ? RB : (j < NA ? RA : RB); };
    auto tile_k = [&](int j) { return j == 14 ? RB : (j < NA ? RA + j : j); };
    double(*pn)[kMaxL + 1] = sh.pnl[J & 1];
    double(*pp)[kMaxL + 1] = sh.pnl[(J + 1) & 1];  // panel J - 1
    const int J1 = J + 1, J2 = J + 2;
    if (dw) {
      // ---- the diagonal wave: B for K = J + 1, panel J's update of diagonal
      // tile J + 1, its factor
      if (J1 < Tn) {
        f64x4 g, dd;
        double ar[4], bq[4], wv[4];
        int dm[4];
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int kk = acc_row<double>(lg, r);
          g[r] = pn[kk][16 * J1 + li];
          ar[r] = -pp[kk][16 * J + li];
          bq[r] = pp[kk][16 * J1 + li];
          wv[r] = sh.wall[J][kk][li];
          dm[r] = sh.sdep[16 * J + kk];
          dd[r] = sh.dbuf[J1 & 1][kk][li];
        }
        __builtin_amdgcn_sched_barrier(0);
        if (J > 0) {
#pragma unroll
          for (int s4 = 0; s4 < 4; ++s4) g = mma_f64(ar[s4], bq[s4], g);
        }
        f64x4 c = {0, 0, 0, 0};
#pragma unroll
        for (int s4 = 0; s4 < 4; ++s4) c = mma_f64(wv[s4], g[s4], c);
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          c[r] = dm[r] ? 0.0 : c[r];
          pn[acc_row<double>(lg, r)][16 * J1 + li] = c[r];  // R_{J,J+1} for the owner of row J
        }
        // accumulator register s of R_{J,J+1} is the operand of step s
#pragma unroll
        for (int s4 = 0; s4 < 4; ++s4) dd = mma_f64(-c[s4], c[s4], dd);
#pragma unroll
        for (int r = 0; r < 4; ++r) sh.dgt[acc_row<double>(lg, r)][li] = dd[r];
        wave_lds_fence();
        diag_factor(sh.dgt, sh.rjj[J1 & 1], sh.wall[J1], sh.gd, sh.sdep, J1, l, eps);
      }
    } else {
      // the owner of row J - 1 takes R_{J-1,J}, the diagonal wave's B tile
      if (J > 0 && (J - 1 == RA || J - 1 == RB)) {
#pragma unroll
        for (int j = 0; j < NS; ++j) {
          if (tile_i(j) == J - 1 && tile_k(j) == J) {
#pragma unroll
            for (int r = 0; r < 4; ++r) t[j][r] = pp[acc_row<double>(lg, r)][16 * J + li];
          }
        }
      }
      // ---- B: K = J + 2 + wl, J + 9 + wl (the operands are read up front;
      // no scheduling barrier: the resident tiles leave too few registers)
      {
        const int K0 = J + 2 + wl, K1 = K0 + 7;
        const bool v0 = K0 < Tn, v1 = K1 < Tn;
        const int C0 = min(K0, Tn - 1), C1 = min(K1, Tn - 1);  // clamped: in bounds, unused
        f64x4 g0, g1;
        double ar[4], b0[4], b1[4], wv[4];
        int dm[4];
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int kk = acc_row<double>(lg, r);
          g0[r] = pn[kk][16 * C0 + li];
          g1[r] = pn[kk][16 * C1 + li];
          ar[r] = -pp[kk][16 * J + li];
          b0[r] = pp[kk][16 * C0 + li];
          b1[r] = pp[kk][16 * C1 + li];
          wv[r] = sh.wall[J][kk][li];
          dm[r] = sh.sdep[16 * J + kk];
        }
        // the updated tile is the B operand as it stands: accumulator
        // register r of lane group g holds row g + 4 r, the contraction index
        // that lane group takes in step r
        f64x4 c0 = {0, 0, 0, 0}, c1 = {0, 0, 0, 0};
        if (v1) {  // two tiles, chains interleaved
          if (J > 0) {
#pragma unroll
            for (int s4 = 0; s4 < 4; ++s4) {
              g0 = mma_f64(ar[s4], b0[s4], g0);
              g1 = mma_f64(ar[s4], b1[s4], g1);
            }
          }
#pragma unroll
          for (int s4 = 0; s4 < 4; ++s4) {
            c0 = mma_f64(wv[s4], g0[s4], c0);
            c1 = mma_f64(wv[s4], g1[s4], c1);
          }
        } else if (v0) {
          if (J > 0) {
#pragma unroll
            for (int s4 = 0; s4 < 4; ++s4) g0 = mma_f64(ar[s4], b0[s4], g0);
          }
#pragma unroll
          for (int s4 = 0; s4 < 4; ++s4) c0 = mma_f64(wv[s4], g0[s4], c0);
        }
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int kk = acc_row<double>(lg, r);
          if (v0) pn[kk][16 * K0 + li] = dm[r] ? 0.0 : c0[r];
          if (v1) pn[kk][16 * K1 + li] = dm[r] ? 0.0 : c1[r];
        }
      }
      // the seven tile waves meet (the diagonal wave does not wait for them)
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
      if (lane == 0) atomicAdd(&sh.bcnt, 1);
      if (!lds_wait_geq(&sh.bcnt, 7 * (J + 1)) && lane == 0) atomicOr(&sh.sflag, 4);
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
      // the owner of row J keeps R_J,: in its registers (the factor's output)
      if (J == RA || J == RB) {
#pragma unroll
        for (int j = 0; j < NS; ++j) {
          const int I = tile_i(j), K = tile_k(j);
          if (I == J && K > J1 && K < Tn) {
#pragma unroll
            for (int r = 0; r < 4; ++r) t[j][r] = pn[acc_row<double>(lg, r)][16 * K + li];
          }
        }
        // R_JJ from the diagonal wave (value selects keep the tiles in registers)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const double v = sh.rjj[J & 1][acc_row<double>(lg, r)][li];
          t[0][r] = J == RA ? v : t[0][r];
          t[14][r] = J == RA ? t[14][r] : v;
        }
      }
      // ---- C, tile waves: G_IK -= R_JI^T R_JK for rows I > J + 1
#pragma unroll
      for (int j = 0; j < NS; ++j) {
        const int I = tile_i(j), K = tile_k(j);
        if (I > J1 && K < Tn) {
          // all eight operands are requested before the first product (left
          // to itself the scheduler waits out one LDS read per product)
          double xa[4], xb[4];
#pragma unroll
          for (int s4 = 0; s4 < 4; ++s4) {
            const int kk = acc_row<double>(lg, s4);
            xa[s4] = pn[kk][16 * I + li];
            xb[s4] = pn[kk][16 * K + li];
          }
          __builtin_amdgcn_sched_barrier(0);
#pragma unroll
          for (int s4 = 0; s4 < 4; ++s4) t[j] = mma_f64(-xa[s4], xb[s4], t[j]);
        }
        if (j % 2 == 1) __builtin_amdgcn_sched_barrier(0);
      }
      // hand-offs for the next panel (the staged columns K > J + 2 of pp are
      // disjoint from the two the diagonal wave reads there next panel)
      if (J2 < Tn && (J2 == RA || J2 == RB)) put_diag(J2, RA, sh.dbuf[J2 & 1]);
      if (J1 < Tn && (J1 == RA || J1 == RB)) stage_row(J1, RA, NA, pp);
    }
    lds_barrier();
  }
  __syncthreads();
  // write Rt (true factor) and Ra (apply factor); mirror tiles below the diagonal are zero
  if (!dw) {
    const int RA = w, RB = 13 - w, NA = 14 - w;
#pragma unroll
    for (int j = 0; j < NS; ++j) {
      const int I = j == 14 ? RB : (j < NA ? RA : RB);
      const int K = j == 14 ? RB : (j < NA ? RA + j : j);
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
  }
  for (int e = tid; e < Tn * 256; e += kCholThreads) {
    const int J = e >> 8, i = (e >> 4) & 15, c = e & 15;
    Dinv[e] = (T)sh.wall[J][i][c];
  }
  if (tid < lp) dep[tid] = sh.sdep[tid];
  if (tid == 0) {
    int nd = 0;
    for (int k = 0; k < l; ++k) nd += sh.sdep[k];
    dep[lp] = nd;
    if (nd && info) {
      atomicAdd(&info->n_dependent, nd);
      atomicOr(&info->status_flags, PBPQLP_FLAG_DEPENDENT);
    }
    if ((sh.sflag & 1) && info) atomicOr(&info->status_flags, PBPQLP_FLAG_NONFINITE);
    if ((sh.sflag & 4) && info) atomicOr(&info->status_flags, PBPQLP_FLAG_INTERNAL);
  }
}

hipError_t launch_chol(bool f64, const double* G, int64_t ldg, int l, int lp, double eps_dep,
                       double* Rt, int64_t ldr, void* Ra, void* Dinv, int* dep, void* info,
                       hipStream_t s, const double* gdiag, int* ident, const int* far) {
  if (lp > kMaxL || (lp & 15)) return hipErrorInvalidValue;
  if ((ident != nullptr) != (far != nullptr)) return hipErrorInvalidValue;
  CholP p{G, ldg, l, lp, eps_dep, Rt, ldr, Ra, Dinv, dep, (pbpqlp_info*)info, gdiag, ident, far};
  if (lp <= 16 * kDwRows) {
    if (f64) return launch_k(chol_dw_kernel<double, false>, chol_dw_kernel<double, true>, dim3(1), dim3(kCholThreads), s, p);
    return launch_k(chol_dw_kernel<float, false>, chol_dw_kernel<float, true>, dim3(1), dim3(kCholThreads), s, p);
  }
  if (f64) return launch_k(chol_kernel<double, false>, chol_kernel<double, true>, dim3(1), dim3(kCholThreads), s, p);
  return launch_k(chol_kernel<float, false>, chol_kernel<float, true>, dim3(1), dim3(kCholThreads), s, p);
}

// ---------------------------------------------------------------------------
// Small FP64 products C = op(A) op(B): one wave per 16 x 16 tile of C on the
// FP64 matrix core (M, N, K multiples of 16).
// ---------------------------------------------------------------------------
struct GemmP {
  int M, N, K;
  const double* A;
  int64_t lda;
  int ta;
  const double* Bm;
  int64_t ldb;
  int tb;
  double* C;
  int64_t ldc;
  int tc;
  const int* ident;
  PBQ_GRID;
};

template <bool B>
__global__ __launch_bounds__(64) void small_gemm_kernel(const GemmP* pb, GemmP ps) {
  bool past;
  const GemmP p = kparams<B>(pb, ps, past);
  if (past) return;
  const int lane = threadIdx.x, li = lane & 15, lg = lane >> 4;
  const int i0 = blockIdx.y * 16, j0 = blockIdx.x * 16;
  f64x4 acc = {0, 0, 0, 0};
  if (p.ident && *p.ident) {   // A is the identity: C = op(B)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int k = i0 + acc_row<double>(lg, r);
      acc[r] = p.tb ? p.Bm[(int64_t)(j0 + li) * p.ldb + k] : p.Bm[(int64_t)k * p.ldb + j0 + li];
    }
  } else
  for (int k0 = 0; k0 < p.K; k0 += 16) {
#pragma unroll
    for (int s4 = 0; s4 < 4; ++s4) {
      const int k = k0 + acc_row<double>(lg, s4);
      const double a = p.ta ? p.A[(int64_t)k * p.lda + i0 + li] : p.A[(int64_t)(i0 + li) * p.lda + k];
      const double b = p.tb ? p.Bm[(int64_t)(j0 + li) * p.ldb + k] : p.Bm[(int64_t)k * p.ldb + j0 + li];
      acc = mma_f64(a, b, acc);
    }
  }
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const int i = i0 + acc_row<double>(lg, r), j = j0 + li;
    if (p.tc) p.C[(int64_t)j * p.ldc + i] = acc[r];
    else p.C[(int64_t)i * p.ldc + j] = acc[r];
  }
}

hipError_t launch_small_gemm(int M, int N, int K, const double* A, int64_t lda, int ta,
                             const double* B, int64_t ldb, int tb, double* C, int64_t ldc, int tc,
                             hipStream_t s, const int* ident) {
  if ((M | N | K) & 15) return hipErrorInvalidValue;
  GemmP p{M, N, K, A, lda, ta, B, ldb, tb, C, ldc, tc, ident};
  return launch_k(small_gemm_kernel<false>, small_gemm_kernel<true>, dim3((unsigned)(N / 16), (unsigned)(M / 16)),
                  dim3(64), s, p);
}

// out[k * ldo + j] = in[j * ldi + k] (k < rows, j < cols), FP64 in, FP64 or FP32 out
struct TransposeP {
  const double* in;
  int64_t ldi;
  int rows, cols;
  void* out;
  int64_t ldo;
  PBQ_GRID;
};

template <typename T, bool B>
__global__ void transpose_cast_kernel(const TransposeP* pb, TransposeP ps) {
  bool past;
  const TransposeP p = kparams<B>(pb, ps, past);
  if (past) return;
  __shared__ double tile[16][17];
  const int tx = threadIdx.x & 15, ty = threadIdx.x >> 4;
  const int k0 = blockIdx.x * 16, j0 = blockIdx.y * 16;
  if (j0 + ty < p.cols && k0 + tx < p.rows) tile[ty][tx] = p.in[(int64_t)(j0 + ty) * p.ldi + k0 + tx];
  __syncthreads();
  if (k0 + ty < p.rows && j0 + tx < p.cols) ((T*)p.out)[(int64_t)(k0 + ty) * p.ldo + j0 + tx] = (T)tile[tx][ty];
}

hipError_t launch_transpose_cast(bool f64_out, const double* in, int64_t ldi, int rows, int cols,
                                 void* out, int64_t ldo, hipStream_t s) {
  dim3 grid((unsigned)((rows + 15) / 16), (unsigned)((cols + 15) / 16));
  TransposeP p{in, ldi, rows, cols, out, ldo};
  if (f64_out) return launch_k(transpose_cast_kernel<double, false>, transpose_cast_kernel<double, true>, grid, dim3(256), s, p);
  return launch_k(transpose_cast_kernel<float, false>, transpose_cast_kernel<float, true>, grid, dim3(256), s, p);
}

// L = U^T (lower triangle, zero above) with one block per row i; the block
// also leaves sum_j L[i][j]^2 in rowsq[i] for the result record.
struct LowerP {
  const double* U;
  int64_t ldu;
  int l;
  double* L;
  int64_t ldl;
  double* rowsq;
  PBQ_GRID;
};

template <bool B>
__global__ void write_lower_t_kernel(const LowerP* pb, LowerP ps) {
  bool past;
  const LowerP p = kparams<B>(pb, ps, past);
  if (past) return;
  __shared__ double red[256];
  const int i = blockIdx.x, t = threadIdx.x;
  double s = 0.0;
  for (int j = t; j < p.l; j += 256) {
    const double v = (j <= i) ? p.U[(int64_t)j * p.ldu + i] : 0.0;
    p.L[(int64_t)i * p.ldl + j] = v;
    s += v * v;
  }
  red[t] = s;
  __syncthreads();
  for (int off = 128; off > 0; off >>= 1) {
    if (t < off) red[t] += red[t + off];
    __syncthreads();
  }
  if (t == 0 && p.rowsq) p.rowsq[i] = red[0];
}

hipError_t launch_write_lower_t(const double* U, int64_t ldu, int l, double* L, int64_t ldl,
                                double* rowsq, hipStream_t s) {
  LowerP p{U, ldu, l, L, ldl, rowsq};
  return launch_k(write_lower_t_kernel<false>, write_lower_t_kernel<true>, dim3((unsigned)l), dim3(256), s, p);
}

// ---------------------------------------------------------------------------
// Result record: zeroed at the start of a call; at the end ||A||_F^2 (summed
// in a fixed order from the first pass's per-block partials), ||L||_F^2 and
// the a-posteriori residual sqrt(||A||^2 - ||L||^2) / ||A|| (for an
// orthogonal projection Q Q^T A the two norms differ by the residual's).
// ---------------------------------------------------------------------------
struct InfoInitP {
  pbpqlp_info* info;
  int l, q;
  PBQ_GRID;
};

template <bool B>
__global__ void info_init_kernel(const InfoInitP* pb, InfoInitP ps) {
  bool past;
  const InfoInitP p = kparams<B>(pb, ps, past);
  if (past) return;
  if (threadIdx.x == 0) {
    pbpqlp_info* info = p.info;
    info->status_flags = 0;
    info->n_dependent = 0;
    info->l = p.l;
    info->q = p.q;
    info->norm_a_fro2 = 0.0;
    info->norm_l_fro2 = 0.0;
    info->resid_rel_est = 0.0;
    info->reserved[0] = 0.0;
    info->reserved[1] = 0.0;
  }
}

hipError_t launch_info_init(void* info, int l, int q, hipStream_t s) {
  InfoInitP p{(pbpqlp_info*)info, l, q};
  return launch_k(info_init_kernel<false>, info_init_kernel<true>, dim3(1), dim3(64), s, p);
}

struct InfoFinP {
  pbpqlp_info* info;
  const double* parts;
  int nparts;
  const double* rowsq;
  int l;
  PBQ_GRID;
};

template <bool B>
__global__ void info_finalize_kernel(const InfoFinP* pb, InfoFinP ps) {
  bool past;
  const InfoFinP p = kparams<B>(pb, ps, past);
  if (past) return;
  __shared__ double ra[256], rl[256];
  const int t = threadIdx.x;
  double a0 = 0.0, a1 = 0.0;
  int i = t;
  for (; i + 256 < p.nparts; i += 512) {
    a0 += p.parts[i];
    a1 += p.parts[i + 256];
  }
  if (i < p.nparts) a0 += p.parts[i];
  ra[t] = a0 + a1;
  double sl = 0.0;
  for (int r = t; r < p.l; r += 256) sl += p.rowsq[r];
  rl[t] = sl;
  __syncthreads();
  for (int off = 128; off > 0; off >>= 1) {
    if (t < off) {
      ra[t] += ra[t + off];
      rl[t] += rl[t + off];
    }
    __syncthreads();
  }
  if (t == 0) {
    p.info->norm_a_fro2 = ra[0];
    p.info->norm_l_fro2 = rl[0];
    const double d = ra[0] - rl[0];
    p.info->resid_rel_est = ra[0] > 0.0 ? sqrt((d > 0.0 ? d : 0.0) / ra[0]) : 0.0;
  }
}

hipError_t launch_info_finalize(void* info, const double* normA_part, int nparts,
                                const double* rowsq, int l, hipStream_t s) {
  InfoFinP p{(pbpqlp_info*)info, normA_part, nparts, rowsq, l};
  return launch_k(info_finalize_kernel<false>, info_finalize_kernel<true>, dim3(1), dim3(256), s, p);
}

// ---------------------------------------------------------------------------
// Numerical rank from the L-values (Section III-A: the leading k x k block of
// L reveals the numerical rank): the number of leading diagonal entries with
// L_ii > tol * L_11 before the first one that is not (NaN counts as not).
// One wave scans the diagonal 64 entries at a time.
// ---------------------------------------------------------------------------
struct RankP {
  const double* L;
  int64_t ldl;
  int l;
  double tol;
  int* out;
  PBQ_GRID;
};

template <bool B>
__global__ void rank_estimate_kernel(const RankP* pb, RankP ps) {
  bool past;
  const RankP p = kparams<B>(pb, ps, past);
  if (past) return;
  const int lane = threadIdx.x;
  const double thr = p.tol * p.L[0];
  int rank = p.l;
  for (int i0 = 0; i0 < p.l; i0 += 64) {
    const int i = i0 + lane;
    const bool fail = i < p.l && !(p.L[(int64_t)i * p.ldl + i] > thr);
    const uint64_t m = __builtin_amdgcn_ballot_w64(fail);
    if (m) {
      rank = i0 + (int)__builtin_ctzll(m);
      break;
    }
  }
  if (lane == 0) *p.out = rank;
}

hipError_t launch_rank_estimate(const double* L, int64_t ldl, int l, double tol, int* out, hipStream_t s) {
  RankP p{L, ldl, l, tol, out};
  return launch_k(rank_estimate_kernel<false>, rank_estimate_kernel<true>, dim3(1), dim3(64), s, p);
}

struct FillP {
  uint32_t* p;
  size_t nwords;
  PBQ_GRID;
};

template <bool B>
__global__ void fill_zero_kernel(const FillP* pb, FillP ps) {
  bool past;
  const FillP p = kparams<B>(pb, ps, past);
  if (past) return;
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < p.nwords) p.p[i] = 0u;
}

hipError_t launch_fill_zero(void* p, size_t bytes, hipStream_t s) {
  const size_t nw = bytes / 4;
  if (nw == 0) return hipSuccess;
  FillP f{(uint32_t*)p, nw};
  return launch_k(fill_zero_kernel<false>, fill_zero_kernel<true>, dim3((unsigned)((nw + 255) / 256)), dim3(256), s, f);
}

struct CopyP {
  const double* in;
  int64_t ldi;
  int rows, cols;
  double* out;
  int64_t ldo;
  int upper_only;
  PBQ_GRID;
};

template <bool B>
__global__ void copy_mat_kernel(const CopyP* pb, CopyP ps) {
  bool past;
  const CopyP p = kparams<B>(pb, ps, past);
  if (past) return;
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  const int i = blockIdx.y;
  if (j >= p.cols || i >= p.rows) return;
  const double v = p.in[(int64_t)i * p.ldi + j];
  p.out[(int64_t)i * p.ldo + j] = (p.upper_only && j < i) ? 0.0 : v;
}

hipError_t launch_copy_mat(const double* in, int64_t ldi, int rows, int cols, double* out,
                           int64_t ldo, int upper_only, hipStream_t s) {
  CopyP p{in, ldi, rows, cols, out, ldo, upper_only};
  return launch_k(copy_mat_kernel<false>, copy_mat_kernel<true>, dim3((unsigned)((cols + 63) / 64), (unsigned)rows),
                  dim3(64), s, p);
}

}  // namespace pbq
