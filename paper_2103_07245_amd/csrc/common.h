// Device-side building blocks shared by the PbP-QLP kernels (gfx950 / CDNA4).
//
// Tall-skinny operands (the sketch Omega, the bases Q and P^, the sketches Y,
// Z) are kept "column-major": row c of a buffer of shape lp32 x ld holds
// column c of the n x l (or m x l) matrix, so every matrix-core operand reads
// its contraction index contiguously.  lp = l rounded up to 16, lp32 = l
// rounded up to 32; rows in [l, lp32) are kept zero.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace pbq {

typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef double f64x4 __attribute__((ext_vector_type(4)));
typedef float f32x2 __attribute__((ext_vector_type(2)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x4 __attribute__((ext_vector_type(4)));
typedef _Float16 f16x8 __attribute__((ext_vector_type(8)));
typedef _Float16 f16x4 __attribute__((ext_vector_type(4)));

// Arithmetic of an A-streaming pass.
enum Mode { M_F64 = 0, M_F32 = 1, M_BF16 = 2, M_F16 = 3, M_BF16X3 = 4 };

constexpr int kMaxL = 256;

// ---------------------------------------------------------------------------
// Philox4x32-10 (Salmon et al., SC'11) and Box-Muller normals.
// ---------------------------------------------------------------------------
__device__ __forceinline__ void philox4x32_10(uint32_t& c0, uint32_t& c1, uint32_t& c2,
                                              uint32_t& c3, uint32_t k0, uint32_t k1) {
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    const uint32_t lo0 = 0xD2511F53u * c0;
    const uint32_t hi0 = __umulhi(0xD2511F53u, c0);
    const uint32_t lo1 = 0xCD9E8D57u * c2;
    const uint32_t hi1 = __umulhi(0xCD9E8D57u, c2);
    const uint32_t n0 = hi1 ^ c1 ^ k0;
    const uint32_t n2 = hi0 ^ c3 ^ k1;
    c0 = n0;
    c1 = lo1;
    c2 = n2;
    c3 = lo0;
    k0 += 0x9E3779B9u;
    k1 += 0xBB67AE85u;
  }
}

// The standard normal of flat index t in stream (s2, s3): Philox block t/4
// gives words x0..x3; slots 0,1 use the Box-Muller pair (x0, x1) and slots
// 2,3 the pair (x2, x3), with u = (x + 1/2) 2^-32, r = sqrt(-2 ln u_a),
// theta = 2 pi u_b, and cos for even slots, sin for odd ones.
__device__ __forceinline__ double normal_at(uint64_t t, uint32_t s2, uint32_t s3, uint64_t seed) {
  const uint64_t blk = t >> 2;
  uint32_t c0 = (uint32_t)blk, c1 = (uint32_t)(blk >> 32), c2 = s2, c3 = s3;
  philox4x32_10(c0, c1, c2, c3, (uint32_t)seed, (uint32_t)(seed >> 32));
  const int e = (int)(t & 3);
  const uint32_t xa = (e < 2) ? c0 : c2;
  const uint32_t xb = (e < 2) ? c1 : c3;
  const double s = 2.3283064365386962890625e-10;  // 2^-32
  const double ua = ((double)xa + 0.5) * s, ub = ((double)xb + 0.5) * s;
  const double r = sqrt(-2.0 * log(ua));
  const double th = 6.283185307179586 * ub;
  return (e & 1) ? r * sin(th) : r * cos(th);
}

// All four normals of Philox block `blk` in stream (s2, s3): the same values
// normal_at gives for t = 4 blk + e, e = 0..3, with one generator call and one
// logarithm and square root per Box-Muller pair.
__device__ __forceinline__ void normals4_at(uint64_t blk, uint32_t s2, uint32_t s3, uint64_t seed,
                                            double out[4]) {
  uint32_t c0 = (uint32_t)blk, c1 = (uint32_t)(blk >> 32), c2 = s2, c3 = s3;
  philox4x32_10(c0, c1, c2, c3, (uint32_t)seed, (uint32_t)(seed >> 32));
  const double s = 2.3283064365386962890625e-10;  // 2^-32
  const uint32_t xa[2] = {c0, c2}, xb[2] = {c1, c3};
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    const double ua = ((double)xa[h] + 0.5) * s, ub = ((double)xb[h] + 0.5) * s;
    const double r = sqrt(-2.0 * log(ua));
    const double th = 6.283185307179586 * ub;
    out[2 * h] = r * cos(th);
    out[2 * h + 1] = r * sin(th);
  }
}

// Round a double to the nearest bfloat16 value (ties to even), kept as double.
__device__ __forceinline__ double bf16_rne_f64(double x) {
  uint64_t b = (uint64_t)__double_as_longlong(x);
  const uint64_t lsb = (b >> 45) & 1ull;
  b += 0x00000FFFFFFFFFFFull + lsb;
  b &= ~((1ull << 45) - 1ull);
  return __longlong_as_double((long long)b);
}

__device__ __forceinline__ double sketch_value(double z) {
  double v = bf16_rne_f64(z);
  return (fabs(v) < 6.103515625e-05) ? 0.0 : v;  // flush below 2^-14
}

// ---------------------------------------------------------------------------
// Matrix-core wrappers (16 x 16 output tile per wave).
// Operand layout for all of them: lane t supplies row (t % 16) of the A tile
// and column (t % 16) of the B tile; lane group g = t / 16 supplies the
// contraction slice g.  The 4-register accumulator of lane t holds column
// t % 16, rows acc_row<T>(g, r) (r = 0..3).
// ---------------------------------------------------------------------------
__device__ __forceinline__ f32x4 mma_f32(float a, float b, f32x4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}
__device__ __forceinline__ f64x4 mma_f64(double a, double b, f64x4 c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}
__device__ __forceinline__ f32x4 mma_bf16(bf16x8 a, bf16x8 b, f32x4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
}
__device__ __forceinline__ f32x4 mma_f16(f16x8 a, f16x8 b, f32x4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x32_f16(a, b, c, 0, 0, 0);
}

// Row (within the 16x16 tile) held by accumulator register r of lane group
// g.  FP32 tiles put rows 4g..4g+3 in one lane group; the FP64 matrix core
// interleaves them (row g + 4r), as measured on gfx950.  Operand layouts are
// the same for both: lane t supplies A[t % 16][t / 16] and B[t / 16][t % 16].
template <typename T> __device__ __forceinline__ constexpr int acc_row(int g, int r) {
  return sizeof(T) == 8 ? g + 4 * r : 4 * g + r;
}

template <typename T> struct Vec4;
template <> struct Vec4<float> { typedef f32x4 type; };
template <> struct Vec4<double> { typedef f64x4 type; };

__device__ __forceinline__ f32x4 mma_native(float a, float b, f32x4 c) { return mma_f32(a, b, c); }
__device__ __forceinline__ f64x4 mma_native(double a, double b, f64x4 c) { return mma_f64(a, b, c); }

// 16-byte vector of raw bits, used to move operands between global memory,
// registers and LDS without caring about the element type.
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ u32x4 ld16(const void* p) { return *(const u32x4*)p; }
__device__ __forceinline__ void st16(void* p, u32x4 v) { *(u32x4*)p = v; }

// Workgroup barrier that orders LDS only: outstanding global loads and
// stores (prefetches, result writes) stay in flight across it.
__device__ __forceinline__ void lds_barrier() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
  __builtin_amdgcn_s_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

template <typename T>
__device__ __forceinline__ T wave_sum(T v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
  return v;
}

}  // namespace pbq
