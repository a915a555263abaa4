// Shared device-side definitions of the single-pass PCA library (gfx950 / CDNA4 only).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace sk {

typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef double f64x4 __attribute__((ext_vector_type(4)));
typedef double f64x2 __attribute__((ext_vector_type(2)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef int i32x8 __attribute__((ext_vector_type(8)));
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
typedef uint32_t u32x2 __attribute__((ext_vector_type(2)));

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
// Wait states between the last matrix-core instruction of a chain and the first VALU read of its
// accumulators.  On gfx950 the FP64 16x16x4 instruction runs at half the rate of gfx942's, and the
// compiler's hazard padding (18 wait states) is too short for it: without this drain the last
// accumulator element can be read before it is written (observed on hardware for a single
// dependent FP64 chain).  The scheduling barriers keep the padding between the two.  Kernels with
// FP64 chains in a loop drain inside the loop body, after each step's products, so that the
// accumulator copies the compiler places at loop edges also come after the padding.
__device__ __forceinline__ void mfma_drain() {
  __builtin_amdgcn_sched_barrier(0);
  asm volatile("s_nop 15\n\ts_nop 15\n\ts_nop 15\n\ts_nop 15" ::: "memory");
  __builtin_amdgcn_sched_barrier(0);
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

// Cross-lane sums without LDS round trips: DPP moves inside each 16-lane row (quad_perm [1,0,3,2]
// and [2,3,0,1], then row_half_mirror and row_mirror, which pair each lane with one whose partial
// covers the other half of its 8- and 16-lane group), then readlane of the four row totals.
namespace dpp {
constexpr int kXor1 = 0xB1, kXor2 = 0x4E, kHalfMirror = 0x141, kMirror = 0x140;
// Every pattern used here reads a valid lane for every lane (all rows and banks enabled), so no
// old value is needed and none is materialised.
template <int CTRL> __device__ __forceinline__ float mov(float v) {
  return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), CTRL, 0xF, 0xF, true));
}
template <int CTRL> __device__ __forceinline__ double mov(double v) {
  const uint64_t u = (uint64_t)__double_as_longlong(v);
  const int lo = __builtin_amdgcn_mov_dpp((int)(uint32_t)u, CTRL, 0xF, 0xF, true);
  const int hi = __builtin_amdgcn_mov_dpp((int)(uint32_t)(u >> 32), CTRL, 0xF, 0xF, true);
  return __longlong_as_double((long long)(((uint64_t)(uint32_t)hi << 32) | (uint32_t)lo));
}
__device__ __forceinline__ float lane(float v, int l) {
  return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), l));
}
__device__ __forceinline__ double lane(double v, int l) {
  const uint64_t u = (uint64_t)__double_as_longlong(v);
  const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)u, l);
  const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(u >> 32), l);
  return __longlong_as_double((long long)(((uint64_t)hi << 32) | lo));
}
}  // namespace dpp

// Sum over each 16-lane row; every lane of the row gets its row's total.
template <typename T> __device__ __forceinline__ T row16_sum(T v) {
  v += dpp::mov<dpp::kXor1>(v);
  v += dpp::mov<dpp::kXor2>(v);
  v += dpp::mov<dpp::kHalfMirror>(v);
  v += dpp::mov<dpp::kMirror>(v);
  return v;
}
// Sum over the whole 64-lane wave (all lanes active); every lane gets the total.
template <typename T> __device__ __forceinline__ T wave_sum(T v) {
  v = row16_sum(v);
  return (dpp::lane(v, 0) + dpp::lane(v, 16)) + (dpp::lane(v, 32) + dpp::lane(v, 48));
}

// Workgroup barrier that waits only for the wave's LDS operations: global loads issued for later
// steps stay in flight across it (a plain __syncthreads also waits for them).
__device__ __forceinline__ void lds_barrier() {
  asm volatile("s_waitcnt lgkmcnt(0)\n\ts_barrier" ::: "memory");
}

// Pointers the compiler must treat as global memory.  Pointers read from a descriptor in memory
// are generic, which makes every access a FLAT instruction; FLAT loads also count against the LDS
// wait counter, so each LDS wait would drain all outstanding global prefetches.
#define SK_GLOBAL __attribute__((address_space(1)))
template <typename T> __device__ __forceinline__ SK_GLOBAL T* gptr(T* p) {
  return (SK_GLOBAL T*)(p);
}
template <typename T> __device__ __forceinline__ const SK_GLOBAL T* gptr(const T* p) {
  return (const SK_GLOBAL T*)(p);
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
