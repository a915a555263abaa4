// Shared device-side definitions of the single-pass PCA library (gfx950 / CDNA4 only).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace sk {

typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef double f64x4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef int i32x8 __attribute__((ext_vector_type(8)));
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));

// Compute modes; the numeric values are those of sketch_dtype.
enum Mode { M_F64 = 0, M_F32 = 1, M_BF16 = 2, M_BF16X2 = 3, M_FP8 = 4 };

// Matrix-core tile: 16 x 16 outputs per wave; lane L supplies row/column L % 16 of the A/B operand
// and the k-group L / 16.  Accumulator element i of lane L holds output row
//   4 * (L / 16) + i   for the FP32-accumulating instructions, and
//   L / 16 + 4 * i     for the FP64 instruction,
// in output column L % 16 (both verified on gfx950 hardware with integer-valued operands).
template <typename AccT> __device__ __forceinline__ int acc_row(int g, int i);
template <> __device__ __forceinline__ int acc_row<float>(int g, int i) { return 4 * g + i; }
template <> __device__ __forceinline__ int acc_row<double>(int g, int i) { return g + 4 * i; }

__device__ __forceinline__ f32x4 mma_f32(float a, float b, f32x4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}
__device__ __forceinline__ f64x4 mma_f64(double a, double b, f64x4 c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}
__device__ __forceinline__ f32x4 mma_bf16(bf16x8 a, bf16x8 b, f32x4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
}
// E4M3 x E4M3, 16x16x128; block-scale exponents 127 (= 2^0) on both operands.
__device__ __forceinline__ f32x4 mma_fp8(i32x8 a, i32x8 b, f32x4 c) {
  return __builtin_amdgcn_mfma_scale_f32_16x16x128_f8f6f4(a, b, c, 0, 0, 0, 127, 0, 127);
}

__device__ __forceinline__ __bf16 to_bf16(float x) { return (__bf16)x; }   // RNE on gfx950
__device__ __forceinline__ float from_bf16(__bf16 x) { return (float)x; }

// Two FP32 values to two E4M3 bytes (round to nearest even); callers keep |x| <= 448.
__device__ __forceinline__ uint32_t pack_fp8x2(float a, float b) {
  return (uint32_t)__builtin_amdgcn_cvt_pk_fp8_f32(a, b, 0, false) & 0xffffu;
}
// Exact E4M3 -> FP32 decode (bias 7, subnormal step 2^-9); 0x7f/0xff never occur after scaling.
__device__ __forceinline__ float fp8_to_f32(uint32_t v) {
  const uint32_t s = (v >> 7) & 1u, e = (v >> 3) & 15u, m = v & 7u;
  float r = e ? __uint_as_float(((e + 120u) << 23) | (m << 20)) : (float)m * 0.001953125f;
  return s ? -r : r;
}

__device__ __forceinline__ float wave_sum(float v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

template <typename T> __host__ __device__ constexpr T cdiv(T a, T b) { return (a + b - 1) / b; }
template <typename T> __host__ __device__ constexpr T rup(T a, T b) { return cdiv(a, b) * b; }

// Control block of the finalize loop, in device memory.
struct Ctrl {
  double r0;          // first diagonal entry of the first combined R (rank-guard reference)
  int last_iter;      // last column-block iteration that runs (t-1 unless the guard stopped it)
  int keep_last;      // columns kept by iteration last_iter
  int l_eff;          // basis vectors kept in total
  int nonfinite;      // set when a block produced a non-finite sketch row
  int pad[4];
};

}  // namespace sk
