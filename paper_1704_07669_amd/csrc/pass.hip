// The streaming pass of Algorithm 4 (steps 5-7): for each row block a of A,
//   g = a Omega,  G = [G; g]    (split over k = columns of a, partials reduced in a fixed order)
//   H = H + a^T g               (Eq. 10; each workgroup owns a strip of columns of a, i.e. of
//                                rows of H, so H is updated without atomics and deterministically)
// on the gfx950 matrix cores.  Operands are converted from the block's storage format to the
// compute mode's operand format as they are loaded (no extra pass over a), except in FP8 mode where
// the per-block power-of-two scale needs the block's amax first.
//
// Layouts: a is row-major (rows contiguous along n).  Omega', G and H are column-major: each of the
// LP sketch columns is contiguous, along n for Omega' and H and along the rows for G.  That makes
// every matrix-core operand a run of consecutive k values per lane:
//   g = a Omega : k = column of a; A operand = a rows, B operand = Omega' columns (staged in LDS).
//   a^T g       : k = row of a;    A operand = G columns (the transposed G), B operand = a columns.
#include "common.hpp"
#include "kernels.hpp"

namespace sk {
namespace {

// ---------------------------------------------------------------- per-mode tile parameters
template <int MODE> struct PT;
template <> struct PT<M_F64> {
  using op_t = double; using acc_t = double; using accv = f64x4;
  static constexpr int V1 = 4, KC = 64, V2 = 4, VC = 2;
};
template <> struct PT<M_F32> {
  using op_t = float; using acc_t = float; using accv = f32x4;
  static constexpr int V1 = 8, KC = 128, V2 = 4, VC = 4;
};
template <> struct PT<M_BF16> {
  using op_t = __bf16; using acc_t = float; using accv = f32x4;
  static constexpr int V1 = 8, KC = 256, V2 = 8, VC = 4;
};
template <> struct PT<M_BF16X2> : PT<M_BF16> {};
template <> struct PT<M_FP8> {
  using op_t = uint8_t; using acc_t = float; using accv = f32x4;
  static constexpr int V1 = 32, KC = 512, V2 = 8, VC = 4;
};
constexpr int RSUB = 2;      // 16-row sub-tiles per wave in g = a Omega
constexpr int WAVES = 4;     // waves per workgroup in both products
constexpr int ROW_TILE = WAVES * 16 * RSUB;

// ---------------------------------------------------------------- operand fragments
template <int MODE> struct Frag;
template <> struct Frag<M_F64> { double v[4]; };
template <> struct Frag<M_F32> { float v[8]; };
template <> struct Frag<M_BF16> { bf16x8 v; };
template <> struct Frag<M_BF16X2> { bf16x8 hi, lo; };
template <> struct Frag<M_FP8> { i32x8 v; };

template <typename Src> __device__ __forceinline__ float src_to_f32(Src x) { return (float)x; }
template <> __device__ __forceinline__ float src_to_f32<__bf16>(__bf16 x) { return from_bf16(x); }
template <> __device__ __forceinline__ float src_to_f32<uint8_t>(uint8_t x) { return fp8_to_f32(x); }

// V consecutive elements of one row of a, starting at column k (zeros outside the block).
// Vector loads need a 16-byte aligned block base and row pitch (vec_ok, uniform per launch).
template <typename Src, int V>
__device__ __forceinline__ void load_run(const Src* __restrict__ A, int64_t lda, int row, int nrows,
                                         int64_t k, int64_t n, bool vec_ok, Src (&buf)[V]) {
  static_assert((V * sizeof(Src)) % 16 == 0, "runs are whole 16-byte vectors");
  if (vec_ok && row < nrows && k + V <= n) {
    const u32x4* p = reinterpret_cast<const u32x4*>(A + (int64_t)row * lda + k);
    u32x4 tmp[V * sizeof(Src) / 16];
#pragma unroll
    for (int i = 0; i < (int)(V * sizeof(Src) / 16); ++i) tmp[i] = p[i];
    __builtin_memcpy(buf, tmp, sizeof(buf));
  } else {
#pragma unroll
    for (int e = 0; e < V; ++e)
      buf[e] = (row < nrows && k + e < n) ? A[(int64_t)row * lda + k + e] : Src(0);
  }
}

template <int MODE, typename Src, int V> struct MakeA;
template <typename Src> struct MakeA<M_F64, Src, 4> {
  static __device__ __forceinline__ Frag<M_F64> f(const Src (&b)[4]) {
    Frag<M_F64> r;
#pragma unroll
    for (int e = 0; e < 4; ++e) r.v[e] = (double)b[e];
    return r;
  }
};
template <typename Src> struct MakeA<M_F32, Src, 8> {
  static __device__ __forceinline__ Frag<M_F32> f(const Src (&b)[8]) {
    Frag<M_F32> r;
#pragma unroll
    for (int e = 0; e < 8; ++e) r.v[e] = (float)b[e];
    return r;
  }
};
template <typename Src> struct MakeA<M_BF16, Src, 8> {
  static __device__ __forceinline__ Frag<M_BF16> f(const Src (&b)[8]) {
    Frag<M_BF16> r;
#pragma unroll
    for (int e = 0; e < 8; ++e) r.v[e] = to_bf16(src_to_f32(b[e]));
    return r;
  }
};
template <> struct MakeA<M_BF16, __bf16, 8> {
  static __device__ __forceinline__ Frag<M_BF16> f(const __bf16 (&b)[8]) {
    Frag<M_BF16> r;
#pragma unroll
    for (int e = 0; e < 8; ++e) r.v[e] = b[e];
    return r;
  }
};
template <typename Src> struct MakeA<M_BF16X2, Src, 8> {
  static __device__ __forceinline__ Frag<M_BF16X2> f(const Src (&b)[8]) {
    Frag<M_BF16X2> r;
#pragma unroll
    for (int e = 0; e < 8; ++e) {
      const float x = src_to_f32(b[e]);
      const __bf16 h = to_bf16(x);
      r.hi[e] = h;
      r.lo[e] = to_bf16(x - from_bf16(h));
    }
    return r;
  }
};
template <> struct MakeA<M_FP8, uint8_t, 32> {
  static __device__ __forceinline__ Frag<M_FP8> f(const uint8_t (&b)[32]) {
    Frag<M_FP8> r;
    __builtin_memcpy(&r.v, b, 32);
    return r;
  }
};

// Omega' fragment from LDS (V consecutive k of one Omega' column).
template <int MODE> struct BFrag { using type = Frag<MODE>; };
template <> struct BFrag<M_BF16X2> { using type = Frag<M_BF16>; };

template <int MODE>
__device__ __forceinline__ typename BFrag<MODE>::type lds_frag(const uint8_t* p) {
  typename BFrag<MODE>::type r;
  __builtin_memcpy(&r, p, sizeof(r));
  return r;
}

__device__ __forceinline__ f64x4 mma(const Frag<M_F64>& a, const Frag<M_F64>& b, f64x4 c) {
#pragma unroll
  for (int j = 0; j < 4; ++j) c = mma_f64(a.v[j], b.v[j], c);
  return c;
}
__device__ __forceinline__ f32x4 mma(const Frag<M_F32>& a, const Frag<M_F32>& b, f32x4 c) {
#pragma unroll
  for (int j = 0; j < 8; ++j) c = mma_f32(a.v[j], b.v[j], c);
  return c;
}
__device__ __forceinline__ f32x4 mma(const Frag<M_BF16>& a, const Frag<M_BF16>& b, f32x4 c) {
  return mma_bf16(a.v, b.v, c);
}
__device__ __forceinline__ f32x4 mma(const Frag<M_BF16X2>& a, const Frag<M_BF16>& b, f32x4 c) {
  c = mma_bf16(a.hi, b.v, c);
  return mma_bf16(a.lo, b.v, c);
}
__device__ __forceinline__ f32x4 mma(const Frag<M_FP8>& a, const Frag<M_FP8>& b, f32x4 c) {
  return mma_fp8(a.v, b.v, c);
}

// ---------------------------------------------------------------- g = a Omega, split over k
// Grid: x = row tiles of ROW_TILE rows, y = k splits of `kchunk` columns.  Each wave owns 16*RSUB
// rows and all NT sketch-column tiles; the k-chunk of Omega' (NT*16 columns x KC) is staged in
// LDS once per workgroup and shared by its waves.
template <typename Src, int MODE, int NT>
__global__ __launch_bounds__(WAVES * 64) void k_gemm1(
    const Src* __restrict__ A, int64_t lda, int nrows, int64_t n,
    const typename PT<MODE>::op_t* __restrict__ omc, int64_t NP, int64_t kchunk,
    typename PT<MODE>::acc_t* __restrict__ P, int64_t ldp, int LP, int vec_ok) {
  using T = PT<MODE>;
  using op_t = typename T::op_t;
  using acc_t = typename T::acc_t;
  using accv = typename T::accv;
  constexpr int V = T::V1, KSS = 4 * V, KC = T::KC;
  constexpr int ROW_BYTES = KC * (int)sizeof(op_t) + 16;   // +16 B: conflict-free 16-lane reads
  constexpr int PIECES = KC * (int)sizeof(op_t) / 16;
  __shared__ __attribute__((aligned(16))) uint8_t lds[NT * 16 * ROW_BYTES];

  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6, g = lane >> 4, r16 = lane & 15;
  const int row_base = blockIdx.x * ROW_TILE + wave * 16 * RSUB;
  const int64_t k_begin = (int64_t)blockIdx.y * kchunk;
  const int64_t k_end = min(n, k_begin + kchunk);

  accv acc[RSUB][NT];
#pragma unroll
  for (int rs = 0; rs < RSUB; ++rs)
#pragma unroll
    for (int nt = 0; nt < NT; ++nt) acc[rs][nt] = accv{0, 0, 0, 0};

  for (int64_t kc = k_begin; kc < k_end; kc += KC) {
    __syncthreads();
    for (int p = tid; p < NT * 16 * PIECES; p += WAVES * 64) {
      const int c = p / PIECES, pc = p - c * PIECES;
      const u32x4 v = *reinterpret_cast<const u32x4*>(
          reinterpret_cast<const uint8_t*>(omc + (int64_t)c * NP + kc) + pc * 16);
      *reinterpret_cast<u32x4*>(lds + c * ROW_BYTES + pc * 16) = v;
    }
    __syncthreads();
    const int kspan = (int)min<int64_t>(KC, k_end - kc);
    for (int ks = 0; ks < kspan; ks += KSS) {
      const int64_t k = kc + ks + V * g;
      Frag<MODE> a[RSUB];
#pragma unroll
      for (int rs = 0; rs < RSUB; ++rs) {
        Src buf[V];
        load_run<Src, V>(A, lda, row_base + rs * 16 + r16, nrows, k, n, vec_ok != 0, buf);
        a[rs] = MakeA<MODE, Src, V>::f(buf);
      }
#pragma unroll
      for (int nt = 0; nt < NT; ++nt) {
        const auto b = lds_frag<MODE>(lds + (nt * 16 + r16) * ROW_BYTES +
                                      (ks + V * g) * (int)sizeof(op_t));
#pragma unroll
        for (int rs = 0; rs < RSUB; ++rs) acc[rs][nt] = mma(a[rs], b, acc[rs][nt]);
      }
    }
  }

  const int64_t pbase = (int64_t)blockIdx.y * LP;
#pragma unroll
  for (int rs = 0; rs < RSUB; ++rs)
#pragma unroll
    for (int nt = 0; nt < NT; ++nt)
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int row = row_base + rs * 16 + acc_row<acc_t>(g, i);
        if (row < nrows) P[(pbase + nt * 16 + r16) * ldp + row] = acc[rs][nt][i];
      }
}

// G rows of this block = sum of the k-split partials in split order, times the FP8 scale.
template <typename acc_t>
__global__ void k_reduce1(const acc_t* __restrict__ P, int64_t ldp, int splits, int LP, int nrows,
                          acc_t* __restrict__ G, int64_t ldg, int64_t g_row0,
                          const int* __restrict__ fp8_exp, Ctrl* __restrict__ ctrl) {
  const acc_t scale = fp8_exp ? (acc_t)ldexp(1.0, -(*fp8_exp) - 5) : (acc_t)1;
  const int64_t total = (int64_t)LP * nrows;
  bool bad = false;
  for (int64_t q = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; q < total;
       q += (int64_t)gridDim.x * blockDim.x) {
    const int c = (int)(q / nrows);
    const int r = (int)(q - (int64_t)c * nrows);
    acc_t s = 0;
    for (int sp = 0; sp < splits; ++sp) s += P[((int64_t)sp * LP + c) * ldp + r];
    s *= scale;
    bad |= !isfinite(s);
    G[(int64_t)c * ldg + g_row0 + r] = s;
  }
  if (bad) ctrl->nonfinite = 1;
}

// ---------------------------------------------------------------- H += a^T g
template <int MODE> struct GT { using type = float; };
template <> struct GT<M_F64> { using type = double; };

template <int MODE> struct GFrag;
template <> struct GFrag<M_F64> { double v[4]; };
template <> struct GFrag<M_F32> { float v[4]; };
template <> struct GFrag<M_BF16> { bf16x8 hi, lo; };
template <> struct GFrag<M_BF16X2> : GFrag<M_BF16> {};
template <> struct GFrag<M_FP8> : GFrag<M_BF16> {};

template <int MODE> struct AFrag2 { float v[4]; };                 // F32: 4 rows, one column
template <> struct AFrag2<M_F64> { double v[4]; };
template <> struct AFrag2<M_BF16> { bf16x8 v; };
template <> struct AFrag2<M_FP8> { bf16x8 v; };
template <> struct AFrag2<M_BF16X2> { bf16x8 hi, lo; };

__device__ __forceinline__ f64x4 mma2(const GFrag<M_F64>& gq, const AFrag2<M_F64>& a, f64x4 c) {
#pragma unroll
  for (int e = 0; e < 4; ++e) c = mma_f64(gq.v[e], a.v[e], c);
  return c;
}
__device__ __forceinline__ f32x4 mma2(const GFrag<M_F32>& gq, const AFrag2<M_F32>& a, f32x4 c) {
#pragma unroll
  for (int e = 0; e < 4; ++e) c = mma_f32(gq.v[e], a.v[e], c);
  return c;
}
__device__ __forceinline__ f32x4 mma2(const GFrag<M_BF16>& gq, const AFrag2<M_BF16>& a, f32x4 c) {
  c = mma_bf16(gq.hi, a.v, c);
  return mma_bf16(gq.lo, a.v, c);
}
__device__ __forceinline__ f32x4 mma2(const GFrag<M_BF16>& gq, const AFrag2<M_FP8>& a, f32x4 c) {
  c = mma_bf16(gq.hi, a.v, c);
  return mma_bf16(gq.lo, a.v, c);
}
__device__ __forceinline__ f32x4 mma2(const GFrag<M_BF16>& gq, const AFrag2<M_BF16X2>& a,
                                      f32x4 c) {
  c = mma_bf16(gq.hi, a.hi, c);
  c = mma_bf16(gq.lo, a.hi, c);
  return mma_bf16(gq.hi, a.lo, c);
}

// VC consecutive columns of one row of a (zeros outside the block).
template <typename Src, int VC>
__device__ __forceinline__ void load_cols(const Src* __restrict__ A, int64_t lda, int row,
                                          int nrows, int64_t col, int64_t n, bool vec_ok,
                                          Src (&buf)[VC]) {
  if (vec_ok && row < nrows && col + VC <= n) {
    __builtin_memcpy(buf, A + (int64_t)row * lda + col, sizeof(buf));
  } else {
#pragma unroll
    for (int j = 0; j < VC; ++j)
      buf[j] = (row < nrows && col + j < n) ? A[(int64_t)row * lda + col + j] : Src(0);
  }
}

template <int MODE, typename Src, int V2, int VC>
__device__ __forceinline__ AFrag2<MODE> make_a2(const Src (&a)[V2][VC], int j) {
  AFrag2<MODE> r;
  if constexpr (MODE == M_F64 || MODE == M_F32) {
#pragma unroll
    for (int e = 0; e < V2; ++e) r.v[e] = a[e][j];
  } else if constexpr (MODE == M_BF16X2) {
#pragma unroll
    for (int e = 0; e < V2; ++e) {
      const float x = src_to_f32(a[e][j]);
      const __bf16 h = to_bf16(x);
      r.hi[e] = h;
      r.lo[e] = to_bf16(x - from_bf16(h));
    }
  } else {
#pragma unroll
    for (int e = 0; e < V2; ++e) r.v[e] = to_bf16(src_to_f32(a[e][j]));
  }
  return r;
}

template <int MODE, int V2>
__device__ __forceinline__ GFrag<MODE> load_gfrag(const typename GT<MODE>::type* __restrict__ gp,
                                                  int r0, int nrows, bool aligned) {
  using gt = typename GT<MODE>::type;
  gt v[V2];
  if (aligned && r0 + V2 <= nrows) {
    __builtin_memcpy(v, gp, sizeof(v));
  } else {
#pragma unroll
    for (int e = 0; e < V2; ++e) v[e] = (r0 + e < nrows) ? gp[e] : gt(0);
  }
  GFrag<MODE> f;
  if constexpr (MODE == M_F64 || MODE == M_F32) {
#pragma unroll
    for (int e = 0; e < V2; ++e) f.v[e] = v[e];
  } else {
#pragma unroll
    for (int e = 0; e < V2; ++e) {
      const __bf16 h = to_bf16(v[e]);
      f.hi[e] = h;
      f.lo[e] = to_bf16(v[e] - from_bf16(h));
    }
  }
  return f;
}

// Grid: x = strips of 16*VC columns of a.  The WAVES waves of a workgroup take interleaved
// super-steps of 4*V2 rows; their partial sums are added in wave order through LDS and the FP64
// sum is added into the workgroup's own rows of H.
template <typename Src, int MODE, int NT>
__global__ __launch_bounds__(WAVES * 64) void k_gemm2(
    const Src* __restrict__ A, int64_t lda, int nrows, int64_t n,
    const typename GT<MODE>::type* __restrict__ G, int64_t ldg, int64_t g_row0,
    double* __restrict__ H, int64_t ldh, const int* __restrict__ fp8_exp, int vec_ok) {
  using T = PT<MODE>;
  using acc_t = typename T::acc_t;
  using accv = typename T::accv;
  constexpr int V2 = T::V2, VC = T::VC, KR = 4 * V2;
  __shared__ acc_t red[(WAVES - 1) * VC * 4 * 64];

  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6, g = lane >> 4, r16 = lane & 15;
  const int64_t col = (int64_t)blockIdx.x * 16 * VC + VC * r16;
  const bool galigned = ((g_row0 % V2) == 0) && ((ldg % V2) == 0);

  accv acc[NT][VC];
#pragma unroll
  for (int mt = 0; mt < NT; ++mt)
#pragma unroll
    for (int j = 0; j < VC; ++j) acc[mt][j] = accv{0, 0, 0, 0};

  for (int kr = wave * KR; kr < nrows; kr += WAVES * KR) {
    Src a[V2][VC];
#pragma unroll
    for (int e = 0; e < V2; ++e)
      load_cols<Src, VC>(A, lda, kr + V2 * g + e, nrows, col, n, vec_ok != 0, a[e]);
    AFrag2<MODE> af[VC];
#pragma unroll
    for (int j = 0; j < VC; ++j) af[j] = make_a2<MODE, Src, V2, VC>(a, j);
    const int r0 = kr + V2 * g;
#pragma unroll
    for (int mt = 0; mt < NT; ++mt) {
      const auto gq = load_gfrag<MODE, V2>(G + (int64_t)(mt * 16 + r16) * ldg + g_row0 + r0, r0,
                                           nrows, galigned);
#pragma unroll
      for (int j = 0; j < VC; ++j) acc[mt][j] = mma2(gq, af[j], acc[mt][j]);
    }
  }

  const double scale = fp8_exp ? ldexp(1.0, -(*fp8_exp)) : 1.0;
#pragma unroll
  for (int mt = 0; mt < NT; ++mt) {
    __syncthreads();
    if (wave > 0) {
#pragma unroll
      for (int j = 0; j < VC; ++j)
#pragma unroll
        for (int i = 0; i < 4; ++i) red[(((wave - 1) * VC + j) * 4 + i) * 64 + lane] = acc[mt][j][i];
    }
    __syncthreads();
    if (wave == 0) {
#pragma unroll
      for (int j = 0; j < VC; ++j) {
        if (col + j >= n) continue;
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          acc_t s = acc[mt][j][i];
          for (int w = 1; w < WAVES; ++w) s += red[(((w - 1) * VC + j) * 4 + i) * 64 + lane];
          const int lidx = mt * 16 + acc_row<acc_t>(g, i);
          double* h = H + (int64_t)lidx * ldh + col + j;
          *h += scale * (double)s;
        }
      }
    }
  }
}

// ---------------------------------------------------------------- FP8 block quantisation
__global__ void k_amax(const float* __restrict__ A, int64_t lda, int nrows, int64_t n,
                       uint32_t* __restrict__ amax) {
  float m = 0.f;
  const int64_t total = (int64_t)nrows * n;
  for (int64_t q = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; q < total;
       q += (int64_t)gridDim.x * blockDim.x) {
    const int64_t r = q / n, c = q - r * n;
    const float x = fabsf(A[r * lda + c]);
    m = (x > m || x != x) ? x : m;
  }
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    const float y = __shfl_xor(m, o, 64);
    m = (y > m || y != y) ? y : m;
  }
  if ((threadIdx.x & 63) == 0) atomicMax(amax, __float_as_uint(m));
}

__device__ __forceinline__ int fp8_exponent(uint32_t amax_bits) {
  const float a = __uint_as_float(amax_bits);
  if (!(a > 0.f) || !isfinite(a)) return 0;
  int ex;
  const float f = frexpf(a, &ex);   // a = f 2^ex, f in [0.5, 1)
  return (f <= 0.875f) ? (9 - ex) : (8 - ex);
}

__global__ void k_quant_fp8(const float* __restrict__ A, int64_t lda, int nrows, int64_t n,
                            const uint32_t* __restrict__ amax, uint8_t* __restrict__ q,
                            int64_t ldq, int* __restrict__ exp_out) {
  const int e = fp8_exponent(*amax);
  if (blockIdx.x == 0 && threadIdx.x == 0) *exp_out = e;
  const float sc = ldexpf(1.0f, e);
  const int64_t per_row = ldq / 4;
  const int64_t total = (int64_t)nrows * per_row;
  for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < total;
       t += (int64_t)gridDim.x * blockDim.x) {
    const int64_t r = t / per_row, c = (t - r * per_row) * 4;
    float x[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const float v = (c + j < n) ? A[r * lda + c + j] * sc : 0.f;
      x[j] = fminf(fmaxf(v, -448.f), 448.f);
    }
    const uint32_t w = pack_fp8x2(x[0], x[1]) | (pack_fp8x2(x[2], x[3]) << 16);
    *reinterpret_cast<uint32_t*>(q + r * ldq + c) = w;
  }
}

inline int grid_for(int64_t work, int block = 256, int cap = 65536) {
  int64_t g = cdiv<int64_t>(work, block);
  return (int)(g < 1 ? 1 : (g > cap ? cap : g));
}

// ---------------------------------------------------------------- dispatch
inline int vec_ok(const PassArgs& a, int es) {
  return (((uintptr_t)a.A) % 16 == 0) && ((a.lda * es) % 16 == 0);
}

template <typename Src, int MODE, int NT>
hipError_t gemm1_t(const PassArgs& a, hipStream_t s) {
  const dim3 grid(cdiv<int64_t>(a.nrows, ROW_TILE), a.splits);
  hipLaunchKernelGGL((k_gemm1<Src, MODE, NT>), grid, dim3(WAVES * 64), 0, s, (const Src*)a.A,
                     a.lda, a.nrows, a.n, (const typename PT<MODE>::op_t*)a.omc, a.NP, a.kchunk,
                     (typename PT<MODE>::acc_t*)a.P1, a.ldp, a.LP, vec_ok(a, sizeof(Src)));
  return hipGetLastError();
}
template <typename Src, int MODE, int NT>
hipError_t gemm2_t(const PassArgs& a, hipStream_t s) {
  const dim3 grid(cdiv<int64_t>(a.n, 16 * PT<MODE>::VC));
  hipLaunchKernelGGL((k_gemm2<Src, MODE, NT>), grid, dim3(WAVES * 64), 0, s, (const Src*)a.A,
                     a.lda, a.nrows, a.n, (const typename GT<MODE>::type*)a.G, a.ldg, a.g_row0,
                     a.H, a.ldh, a.fp8_exp, vec_ok(a, sizeof(Src)));
  return hipGetLastError();
}

template <template <typename, int, int> class F, typename Src, int MODE>
struct NTDispatch;

#define SK_NT_SWITCH(FN, SRC, MODE)                              \
  switch (a.NT) {                                                \
    case 1: return FN<SRC, MODE, 1>(a, s);                       \
    case 2: return FN<SRC, MODE, 2>(a, s);                       \
    case 3: return FN<SRC, MODE, 3>(a, s);                       \
    case 4: return FN<SRC, MODE, 4>(a, s);                       \
    case 5: return FN<SRC, MODE, 5>(a, s);                       \
    case 6: return FN<SRC, MODE, 6>(a, s);                       \
    case 7: return FN<SRC, MODE, 7>(a, s);                       \
    case 8: return FN<SRC, MODE, 8>(a, s);                       \
    default: return hipErrorInvalidValue;                        \
  }

// sketch_dtype codes of the storage format read by the kernels.
enum { S_F64 = 0, S_F32 = 1, S_BF16 = 2, S_FP8 = 4 };

#define SK_MODE_SWITCH(FN)                                                      \
  switch (a.mode) {                                                             \
    case M_F64:                                                                 \
      if (a.src == S_F64) { SK_NT_SWITCH(FN, double, M_F64) }                   \
      if (a.src == S_F32) { SK_NT_SWITCH(FN, float, M_F64) }                    \
      break;                                                                    \
    case M_F32:                                                                 \
      if (a.src == S_F32) { SK_NT_SWITCH(FN, float, M_F32) }                    \
      break;                                                                    \
    case M_BF16:                                                                \
      if (a.src == S_F32) { SK_NT_SWITCH(FN, float, M_BF16) }                   \
      if (a.src == S_BF16) { SK_NT_SWITCH(FN, __bf16, M_BF16) }                 \
      break;                                                                    \
    case M_BF16X2:                                                              \
      if (a.src == S_F32) { SK_NT_SWITCH(FN, float, M_BF16X2) }                 \
      break;                                                                    \
    case M_FP8:                                                                 \
      if (a.src == S_FP8) { SK_NT_SWITCH(FN, uint8_t, M_FP8) }                  \
      break;                                                                    \
  }                                                                             \
  return hipErrorInvalidValue;

}  // namespace

int gemm1_row_tile(int) { return ROW_TILE; }

hipError_t launch_gemm1(const PassArgs& a, hipStream_t s) { SK_MODE_SWITCH(gemm1_t) }
hipError_t launch_gemm2(const PassArgs& a, hipStream_t s) { SK_MODE_SWITCH(gemm2_t) }

hipError_t launch_reduce1(const PassArgs& a, hipStream_t s) {
  const dim3 grid(grid_for((int64_t)a.LP * a.nrows)), block(256);
  if (a.mode == M_F64) {
    hipLaunchKernelGGL(k_reduce1<double>, grid, block, 0, s, (const double*)a.P1, a.ldp, a.splits,
                       a.LP, a.nrows, (double*)a.G, a.ldg, a.g_row0, a.fp8_exp, a.ctrl);
  } else {
    hipLaunchKernelGGL(k_reduce1<float>, grid, block, 0, s, (const float*)a.P1, a.ldp, a.splits,
                       a.LP, a.nrows, (float*)a.G, a.ldg, a.g_row0, a.fp8_exp, a.ctrl);
  }
  return hipGetLastError();
}

hipError_t launch_fp8_quantize(const float* A, int64_t lda, int nrows, int64_t n, uint32_t* amax,
                               uint8_t* q, int64_t ldq, int* exp_out, hipStream_t s) {
  hipError_t e = launch_fill_u32(amax, 1, 0u, s);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_amax, dim3(grid_for((int64_t)nrows * n, 256, 4096)), dim3(256), 0, s, A,
                     lda, nrows, n, amax);
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_quant_fp8, dim3(grid_for((int64_t)nrows * (ldq / 4), 256, 16384)),
                     dim3(256), 0, s, A, lda, nrows, n, amax, q, ldq, exp_out);
  return hipGetLastError();
}

}  // namespace sk
