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
#include <algorithm>
#include <type_traits>

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

// The item of workgroup b in a (possibly grouped) grid: the last item whose first workgroup,
// selected by `first`, is <= b.  Uniform per workgroup.
__device__ __forceinline__ PassItem item_of(const PassItem& one, const PassItem* __restrict__ grp,
                                            int count, int b, int32_t PassItem::*first) {
  if (count == 1) return one;
  int i = count - 1;
  while (i > 0 && grp[i].*first > b) --i;
  return grp[i];
}


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
// LDS once per workgroup and shared by its waves.  Row loads are issued one super-step ahead of
// the matrix-core work (two register buffers).  A wave whose rows and super-step lie inside the
// block takes unconditional 16-byte loads; only tails take per-element masked loads.
template <typename Src, int V, int RS>
__device__ __forceinline__ void fetch_rows(const SK_GLOBAL Src* __restrict__ A, int64_t lda, int row0,
                                           int r16, int nrows, int64_t kbase, int g, int64_t n,
                                           bool rows_full, Src (&buf)[RS][V]) {
  const int64_t k = kbase + V * g;
  if (rows_full && kbase + 4 * V <= n) {
#pragma unroll
    for (int rs = 0; rs < RS; ++rs) {
      const SK_GLOBAL u32x4* p =
          reinterpret_cast<const SK_GLOBAL u32x4*>(A + (int64_t)(row0 + rs * 16 + r16) * lda + k);
      u32x4 tmp[V * sizeof(Src) / 16];
#pragma unroll
      for (int i = 0; i < (int)(V * sizeof(Src) / 16); ++i) tmp[i] = p[i];
      __builtin_memcpy(buf[rs], tmp, sizeof(buf[rs]));
    }
  } else {
#pragma unroll
    for (int rs = 0; rs < RS; ++rs) {
      const int row = row0 + rs * 16 + r16;
#pragma unroll
      for (int e = 0; e < V; ++e)
        buf[rs][e] = (row < nrows && k + e < n) ? A[(int64_t)row * lda + k + e] : Src(0);
    }
  }
}

template <typename Src, int MODE, int NT, int RS>
__device__ __forceinline__ void gemm1_step(const Src (&buf)[RS][PT<MODE>::V1], const uint8_t* lds,
                                           int row_bytes, int koff_bytes, int r16,
                                           typename PT<MODE>::accv (&acc)[RS][NT]) {
  Frag<MODE> a[RS];
#pragma unroll
  for (int rs = 0; rs < RS; ++rs) a[rs] = MakeA<MODE, Src, PT<MODE>::V1>::f(buf[rs]);
#pragma unroll
  for (int nt = 0; nt < NT; ++nt) {
    const auto b = lds_frag<MODE>(lds + (nt * 16 + r16) * row_bytes + koff_bytes);
#pragma unroll
    for (int rs = 0; rs < RS; ++rs) acc[rs][nt] = mma(a[rs], b, acc[rs][nt]);
  }
  // FP64: the wait states once per step, inside the step, so that any copy of an accumulator the
  // compiler places after it (loop edges) comes after them
  if constexpr (MODE == M_F64) mfma_drain();
}

// Omega' chunks of g = a Omega: 256 bytes of each Omega' column (32 FP64 .. 256 FP8 values) per
// LDS buffer, rows padded by 16 bytes so 16-lane reads are conflict free.
template <int MODE> struct G1C {
  using op_t = typename PT<MODE>::op_t;
  static constexpr int KC = 256 / (int)sizeof(op_t);          // columns of a per chunk
  static constexpr int KSS = 4 * PT<MODE>::V1;                 // columns of a per step
  static constexpr int SPC = KC / KSS;                         // steps per chunk
  static constexpr int ROWB = 256 + 16;
};

// A rows row0 + rs*16 + r16 (rs < RSUB), columns k .. k+V-1, at clamped addresses: rows past the
// block repeat its last row (their g rows are never written), and a window at or past kmax (the
// readable columns of a row, a multiple of V) reads column 0 instead: it meets zero rows of
// Omega', which is zero-padded past n.
template <typename Src, int V, int RS>
__device__ __forceinline__ void fetch_rows_clamped(const SK_GLOBAL Src* __restrict__ A, int64_t lda,
                                                   int row0, int r16, int nrows, int64_t k,
                                                   int64_t kmax, Src (&buf)[RS][V]) {
  const int64_t kc = (k < kmax) ? k : 0;
#pragma unroll
  for (int rs = 0; rs < RS; ++rs) {
    const int row = min(row0 + rs * 16 + r16, nrows - 1);
    const SK_GLOBAL u32x4* p = reinterpret_cast<const SK_GLOBAL u32x4*>(A + (int64_t)row * lda + kc);
    u32x4 tmp[V * sizeof(Src) / 16];
#pragma unroll
    for (int i = 0; i < (int)(V * sizeof(Src) / 16); ++i) tmp[i] = p[i];
    __builtin_memcpy(buf[rs], tmp, sizeof(buf[rs]));
  }
}

// The step loop of k_gemm1.  Step t covers columns k_begin + t KSS .. + KSS - 1; chunk c (SPC
// steps) reads Omega' buffer c & 1 of LDS.  a of step t + DEPTH is issued right after step t's
// matrix-core work (past the last step it re-reads the last one, unused); the next chunk of
// Omega' is loaded into registers one chunk ahead and stored to the idle buffer at the end of the
// chunk, followed by the chunk's only barrier (an LDS-count wait, so a loads stay in flight).
template <typename Src, int MODE, int NT, int DEPTH, bool VEC>
__device__ __forceinline__ void g1_steps(const SK_GLOBAL Src* __restrict__ A, int64_t lda, int nrows,
                                         int64_t n, int64_t kmax,
                                         const SK_GLOBAL typename PT<MODE>::op_t* __restrict__ omc,
                                         int64_t NP, int64_t k_begin, int64_t k_end, int row0,
                                         int tid, int g, int r16, uint8_t* lds,
                                         typename PT<MODE>::accv (&acc)[RSUB][NT]) {
  using op_t = typename PT<MODE>::op_t;
  constexpr int V = PT<MODE>::V1, KSS = G1C<MODE>::KSS, KC = G1C<MODE>::KC;
  constexpr int SPC = G1C<MODE>::SPC, ROWB = G1C<MODE>::ROWB, BUF = NT * 16 * ROWB;
  static_assert(SPC % DEPTH == 0, "the a ring must divide the steps of a chunk");
  const int T = (int)((k_end - k_begin + KSS - 1) / KSS);
  const int C = (T + SPC - 1) / SPC;
  Src ab[DEPTH][RSUB][V];
  u32x4 om[NT];                         // NT*16 rows x 16 pieces = NT pieces per thread
  auto load_a = [&](int t, int d) {
    const int tc = min(t, T - 1);
    const int64_t kb = k_begin + (int64_t)tc * KSS;
    if constexpr (VEC)
      fetch_rows_clamped<Src, V, RSUB>(A, lda, row0, r16, nrows, kb + V * g, kmax, ab[d]);
    else
      fetch_rows<Src, V, RSUB>(A, lda, row0, r16, nrows, kb, g, n, false, ab[d]);
  };
  auto load_om = [&](int c) {
    const int64_t kc = k_begin + (int64_t)min(c, C - 1) * KC;
#pragma unroll
    for (int i = 0; i < NT; ++i) {
      const int p = tid + i * 256, row = p >> 4, pc = p & 15;
      om[i] = *reinterpret_cast<const SK_GLOBAL u32x4*>(
          reinterpret_cast<const SK_GLOBAL uint8_t*>(omc + (int64_t)row * NP + kc) + pc * 16);
    }
  };
  auto store_om = [&](int b) {
#pragma unroll
    for (int i = 0; i < NT; ++i) {
      const int p = tid + i * 256, row = p >> 4, pc = p & 15;
      *reinterpret_cast<u32x4*>(lds + b * BUF + row * ROWB + pc * 16) = om[i];
    }
  };
  load_om(0);
#pragma unroll
  for (int d = 0; d < DEPTH; ++d) load_a(d, d);
  store_om(0);
  lds_barrier();
  load_om(1);
  for (int c = 0; c < C; ++c) {
    const uint8_t* buf = lds + (c & 1) * BUF;
#pragma unroll
    for (int j = 0; j < SPC; ++j) {
      const int t = c * SPC + j;
      if (t < T)
        gemm1_step<Src, MODE, NT, RSUB>(ab[j % DEPTH], buf, ROWB,
                                        (j * KSS + V * g) * (int)sizeof(op_t), r16, acc);
      load_a(t + DEPTH, j % DEPTH);
    }
    if (c + 1 < C) store_om((c + 1) & 1);
    lds_barrier();
    load_om(c + 2);
  }
}

// Tiles of an item are (row tile, split) pairs, numbered split-major and spread so that the
// workgroups of one split, which share one k-chunk of Omega', land on the same XCD (workgroups are
// dealt to the 8 XCDs round-robin; item offsets are multiples of 8).
template <typename Src, int MODE, int NT>
__global__ __launch_bounds__(WAVES * 64) void k_gemm1(const PassItem one,
                                                      const PassItem* __restrict__ grp, int count) {
  using T = PT<MODE>;
  using op_t = typename T::op_t;
  using acc_t = typename T::acc_t;
  using accv = typename T::accv;
  constexpr int V = T::V1, LP = NT * 16;
  constexpr int DEPTH = 2;
  __shared__ __attribute__((aligned(16))) uint8_t lds[2 * NT * 16 * G1C<MODE>::ROWB];

  const PassItem it = item_of(one, grp, count, blockIdx.x, &PassItem::wg1);
  const int ntile = it.row_tiles * it.splits;
  const int u = blockIdx.x - it.wg1;
  const int tile = (u & 7) * ((ntile + 7) >> 3) + (u >> 3);
  if (tile >= ntile) return;
  const int split = tile / it.row_tiles, rtile = tile - split * it.row_tiles;
  const SK_GLOBAL Src* __restrict__ A = gptr(reinterpret_cast<const Src*>(it.A));
  const int64_t lda = it.lda, n = it.n, NP = it.NP, ldp = it.ldp;
  const int nrows = it.nrows;
  const SK_GLOBAL op_t* __restrict__ omc = gptr(reinterpret_cast<const op_t*>(it.omc));
  SK_GLOBAL acc_t* __restrict__ P = gptr(reinterpret_cast<acc_t*>(it.P1));

  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6, g = lane >> 4, r16 = lane & 15;
  const int row0 = rtile * ROW_TILE + wave * 16 * RSUB;
  const int64_t k_begin = (int64_t)split * it.kchunk;
  const int64_t k_end = min(n, k_begin + it.kchunk);
  // readable columns of a row: n, or the zero-padded staging width of pre-quantised FP8 rows
  const int64_t kmax = (sizeof(Src) == 1) ? lda : n;

  accv acc[RSUB][NT];
#pragma unroll
  for (int rs = 0; rs < RSUB; ++rs)
#pragma unroll
    for (int nt = 0; nt < NT; ++nt) acc[rs][nt] = accv{0, 0, 0, 0};

  if (it.vec_ok && (kmax % V) == 0)
    g1_steps<Src, MODE, NT, DEPTH, true>(A, lda, nrows, n, kmax, omc, NP, k_begin, k_end, row0, tid,
                                         g, r16, lds, acc);
  else
    g1_steps<Src, MODE, NT, DEPTH, false>(A, lda, nrows, n, kmax, omc, NP, k_begin, k_end, row0,
                                          tid, g, r16, lds, acc);

  mfma_drain();
  const int64_t pbase = (int64_t)split * LP;
#pragma unroll
  for (int rs = 0; rs < RSUB; ++rs)
#pragma unroll
    for (int nt = 0; nt < NT; ++nt)
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int row = row0 + rs * 16 + acc_row<acc_t>(g, i);
        if (row < nrows) P[(pbase + nt * 16 + r16) * ldp + row] = acc[rs][nt][i];
      }
}

// G rows of this block = sum of the k-split partials in split order, times the FP8 scale.  Also
// writes the block-local operand copy read by a^T g: FP64 / FP32 as is, or, in the BF16-operand
// modes, the pair hi = bf16(g), lo = bf16(g - hi) (two LP x ldp BF16 arrays).
template <typename acc_t, bool HILO>
__global__ void k_reduce1(const PassItem one, const PassItem* __restrict__ grp, int count, int LP) {
  const PassItem it = item_of(one, grp, count, blockIdx.x, &PassItem::wgr);
  const SK_GLOBAL acc_t* __restrict__ P = gptr(reinterpret_cast<const acc_t*>(it.P1));
  SK_GLOBAL acc_t* __restrict__ G = gptr(reinterpret_cast<acc_t*>(it.G));
  SK_GLOBAL uint8_t* __restrict__ gop = gptr(reinterpret_cast<uint8_t*>(it.Gop));
  const int64_t ldp = it.ldp, ldg = it.ldg, g_row0 = it.g_row0;
  const int splits = it.splits, nrows = it.nrows;
  const acc_t scale = it.fp8_exp ? (acc_t)ldexp(1.0, -(*gptr(it.fp8_exp)) - 5) : (acc_t)1;
  const int64_t total = (int64_t)LP * nrows;
  bool bad = false;
  for (int64_t q = (int64_t)(blockIdx.x - it.wgr) * blockDim.x + threadIdx.x; q < total;
       q += (int64_t)it.red_wgs * blockDim.x) {
    const int c = (int)(q / nrows);
    const int r = (int)(q - (int64_t)c * nrows);
    // the split partials in split order, eight loads in flight per batch (clamped to the last
    // split, whose repeats are not added)
    acc_t s = 0;
    for (int sp0 = 0; sp0 < splits; sp0 += 8) {
      acc_t v[8];
#pragma unroll
      for (int u = 0; u < 8; ++u)
        v[u] = P[((int64_t)min(sp0 + u, splits - 1) * LP + c) * ldp + r];
#pragma unroll
      for (int u = 0; u < 8; ++u)
        if (sp0 + u < splits) s += v[u];
    }
    s *= scale;
    bad |= !isfinite(s);
    G[(int64_t)c * ldg + g_row0 + r] = s;
    // the operand of a^T g; the column-sum column (centring) is all ones
    const acc_t so = (it.sum_col != 0 && c == it.sum_col) ? (acc_t)1 : s;
    if constexpr (HILO) {
      SK_GLOBAL __bf16* hi = reinterpret_cast<SK_GLOBAL __bf16*>(gop);
      SK_GLOBAL __bf16* lo = hi + (int64_t)LP * ldp;
      const __bf16 h = to_bf16((float)so);
      hi[(int64_t)c * ldp + r] = h;
      lo[(int64_t)c * ldp + r] = to_bf16((float)so - from_bf16(h));
    } else {
      reinterpret_cast<SK_GLOBAL acc_t*>(gop)[(int64_t)c * ldp + r] = so;
    }
  }
  if (bad) {
    gptr(it.ctrl)->nonfinite = 1;
    if (it.nf_host) *it.nf_host = 1;
  }
}

// ---------------------------------------------------------------- H += a^T g
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

// V2 rows x VC columns of a (rows kr + V2*g + e, columns col .. col+VC-1).
template <typename Src, int V2, int VC>
__device__ __forceinline__ void fetch_cols(const SK_GLOBAL Src* __restrict__ A, int64_t lda, int kr, int g,
                                           int nrows, int64_t col, int64_t n, bool cols_full,
                                           Src (&a)[V2][VC]) {
  const int r0 = kr + V2 * g;
  if (cols_full && kr + 4 * V2 <= nrows) {
#pragma unroll
    for (int e = 0; e < V2; ++e) {
      const SK_GLOBAL Src* p = A + (int64_t)(r0 + e) * lda + col;
      if constexpr (VC * sizeof(Src) == 16) {
        const u32x4 v = *reinterpret_cast<const SK_GLOBAL u32x4*>(p);
        __builtin_memcpy(a[e], &v, 16);
      } else if constexpr (VC * sizeof(Src) == 8) {
        const u32x2 v = *reinterpret_cast<const SK_GLOBAL u32x2*>(p);
        __builtin_memcpy(a[e], &v, 8);
      } else {
        const uint32_t v = *reinterpret_cast<const SK_GLOBAL uint32_t*>(p);
        __builtin_memcpy(a[e], &v, 4);
      }
    }
  } else {
#pragma unroll
    for (int e = 0; e < V2; ++e)
#pragma unroll
      for (int j = 0; j < VC; ++j)
        a[e][j] = (r0 + e < nrows && col + j < n) ? A[(int64_t)(r0 + e) * lda + col + j] : Src(0);
  }
}

// G fragment of column m: V2 consecutive block rows r0 .. r0+V2-1 of the block-local operand copy
// (rows past the block are zero).
template <int MODE, int V2>
__device__ __forceinline__ GFrag<MODE> fetch_g(const SK_GLOBAL uint8_t* __restrict__ gop, int64_t ldp, int LP,
                                               int m, int r0, int nrows) {
  GFrag<MODE> f;
  if constexpr (MODE == M_F64 || MODE == M_F32) {
    using gt = typename std::conditional<MODE == M_F64, double, float>::type;
    const SK_GLOBAL gt* p = reinterpret_cast<const SK_GLOBAL gt*>(gop) + (int64_t)m * ldp + r0;
    if (r0 + V2 <= nrows) {
#pragma unroll
      for (int e = 0; e < V2; ++e) f.v[e] = p[e];
    } else {
#pragma unroll
      for (int e = 0; e < V2; ++e) f.v[e] = (r0 + e < nrows) ? p[e] : gt(0);
    }
  } else {
    const SK_GLOBAL __bf16* hi = reinterpret_cast<const SK_GLOBAL __bf16*>(gop) + (int64_t)m * ldp + r0;
    const SK_GLOBAL __bf16* lo = hi + (int64_t)LP * ldp;
    if (r0 + V2 <= nrows) {
      const u32x4 vh = *reinterpret_cast<const SK_GLOBAL u32x4*>(hi);
      const u32x4 vl = *reinterpret_cast<const SK_GLOBAL u32x4*>(lo);
      __builtin_memcpy(&f.hi, &vh, 16);
      __builtin_memcpy(&f.lo, &vl, 16);
    } else {
#pragma unroll
      for (int e = 0; e < V2; ++e) {
        f.hi[e] = (r0 + e < nrows) ? hi[e] : (__bf16)0.0f;
        f.lo[e] = (r0 + e < nrows) ? lo[e] : (__bf16)0.0f;
      }
    }
  }
  return f;
}

template <int MODE, int NT>
__device__ __forceinline__ void fetch_gall(const SK_GLOBAL uint8_t* __restrict__ gop, int64_t ldp, int LP,
                                           int r16, int r0, int nrows, GFrag<MODE> (&gq)[NT]) {
#pragma unroll
  for (int mt = 0; mt < NT; ++mt) gq[mt] = fetch_g<MODE, PT<MODE>::V2>(gop, ldp, LP, mt * 16 + r16, r0, nrows);
}

template <typename Src, int MODE, int NT>
__device__ __forceinline__ void gemm2_step(const Src (&a)[PT<MODE>::V2][PT<MODE>::VC],
                                           const GFrag<MODE> (&gq)[NT],
                                           typename PT<MODE>::accv (&acc)[NT][PT<MODE>::VC]) {
  constexpr int V2 = PT<MODE>::V2, VC = PT<MODE>::VC;
  AFrag2<MODE> af[VC];
#pragma unroll
  for (int j = 0; j < VC; ++j) af[j] = make_a2<MODE, Src, V2, VC>(a, j);
#pragma unroll
  for (int mt = 0; mt < NT; ++mt)
#pragma unroll
    for (int j = 0; j < VC; ++j) acc[mt][j] = mma2(gq[mt], af[j], acc[mt][j]);
  if constexpr (MODE == M_F64) mfma_drain();   // as in gemm1_step
}

// Grid: x = strips of 16*VC columns of a.  The WAVES waves of a workgroup take interleaved
// super-steps of 4*V2 rows (loads issued one super-step ahead); their partial sums are added in
// wave order through LDS and the FP64 sum is added into the workgroup's own rows of H.
template <typename Src, int MODE, int NT>
__global__ __launch_bounds__(WAVES * 64) void k_gemm2(const PassItem one,
                                                      const PassItem* __restrict__ grp, int count) {
  using T = PT<MODE>;
  using acc_t = typename T::acc_t;
  using accv = typename T::accv;
  constexpr int V2 = T::V2, VC = T::VC, KR = 4 * V2, LP = NT * 16;
  __shared__ acc_t red[(WAVES - 1) * VC * 4 * 64];

  const PassItem it = item_of(one, grp, count, blockIdx.x, &PassItem::wg2);
  const int tile = blockIdx.x - it.wg2;
  const int64_t strip = tile % it.strips;
  const int rs = tile / it.strips, rsplit = it.rsplit;
  const SK_GLOBAL Src* __restrict__ A = gptr(reinterpret_cast<const Src*>(it.A));
  const SK_GLOBAL uint8_t* __restrict__ gop = gptr(reinterpret_cast<const uint8_t*>(it.Gop));
  const int64_t lda = it.lda, n = it.n, ldp = it.ldp, ldh = it.ldh;
  SK_GLOBAL double* __restrict__ H = gptr(it.H);
  SK_GLOBAL acc_t* __restrict__ part = gptr(reinterpret_cast<acc_t*>(it.P2));
  unsigned* __restrict__ counters = it.counters;
  int nrows = it.nrows;

  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6, g = lane >> 4, r16 = lane & 15;
  const int64_t c0 = strip * 16 * VC;
  const int64_t col = c0 + VC * r16;
  const bool cols_full = it.vec_ok && (c0 + 16 * VC <= n);

  accv acc[NT][VC];
#pragma unroll
  for (int mt = 0; mt < NT; ++mt)
#pragma unroll
    for (int j = 0; j < VC; ++j) acc[mt][j] = accv{0, 0, 0, 0};

  // this workgroup's row range (split rs of rsplit), rows relative to the block
  const int row_lo = rs * it.rchunk;
  const int row_hi = min(nrows, row_lo + it.rchunk);

  // A and G of the next super-step are fetched before the matrix-core work of the current one
  Src a0[V2][VC], a1[V2][VC];
  GFrag<MODE> g0[NT], g1[NT];
  constexpr int STRIDE = WAVES * KR;
  int kr = row_lo + wave * KR;
  nrows = row_hi;
  if (kr < nrows) {
    fetch_cols<Src, V2, VC>(A, lda, kr, g, nrows, col, n, cols_full, a0);
    fetch_gall<MODE, NT>(gop, ldp, LP, r16, kr + V2 * g, nrows, g0);
  }
  for (; kr < nrows; kr += 2 * STRIDE) {
    const bool has1 = kr + STRIDE < nrows;
    if (has1) {
      fetch_cols<Src, V2, VC>(A, lda, kr + STRIDE, g, nrows, col, n, cols_full, a1);
      fetch_gall<MODE, NT>(gop, ldp, LP, r16, kr + STRIDE + V2 * g, nrows, g1);
    }
    gemm2_step<Src, MODE, NT>(a0, g0, acc);
    if (kr + 2 * STRIDE < nrows) {
      fetch_cols<Src, V2, VC>(A, lda, kr + 2 * STRIDE, g, nrows, col, n, cols_full, a0);
      fetch_gall<MODE, NT>(gop, ldp, LP, r16, kr + 2 * STRIDE + V2 * g, nrows, g0);
    }
    if (has1) gemm2_step<Src, MODE, NT>(a1, g1, acc);
  }

  mfma_drain();
  const double scale = it.fp8_exp ? ldexp(1.0, -(*gptr(it.fp8_exp))) : 1.0;
  // Row-split partials: every workgroup of a strip writes its (wave-ordered) FP32 sum; the last
  // one to finish, found with a per-strip counter, adds the rsplit partials in split order into
  // the FP64 rows of H and resets the counter.  No workgroup waits on another.
  const int64_t pstride = (int64_t)LP * 16 * VC;          // one partial tile
  SK_GLOBAL acc_t* mine = part + (strip * rsplit + rs) * pstride;
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
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          acc_t sm = acc[mt][j][i];
#pragma unroll
          for (int w = 1; w < WAVES; ++w) sm += red[(((w - 1) * VC + j) * 4 + i) * 64 + lane];
          const int lidx = mt * 16 + acc_row<acc_t>(g, i);
          if (rsplit == 1) {
            if (col + j < n) H[(int64_t)lidx * ldh + col + j] += scale * (double)sm;
          } else {
            mine[(int64_t)lidx * 16 * VC + VC * r16 + j] = sm;
          }
        }
      }
    }
  }
  if (rsplit == 1) return;
  __shared__ unsigned last;
  __threadfence();
  __syncthreads();
  if (tid == 0) last = (atomicAdd(counters + strip, 1u) == (unsigned)(rsplit - 1));
  __syncthreads();
  if (!last) return;
  __threadfence();
  const SK_GLOBAL acc_t* base = part + strip * rsplit * pstride;
  for (int e = tid; e < pstride; e += blockDim.x) {
    const int lidx = e / (16 * VC), cc = e - lidx * 16 * VC;
    if (c0 + cc >= n) continue;
    double sm = 0.0;
    for (int t = 0; t < rsplit; ++t) sm += (double)base[t * pstride + e];
    H[(int64_t)lidx * ldh + c0 + cc] += scale * sm;
  }
  if (tid == 0) counters[strip] = 0u;
}

// ---------------------------------------------------------------- H += a^T g, wide strips
// Matrix-core modes with FP32 accumulation.  Each workgroup owns a strip of 256 columns of a (its
// four waves take 64 columns each, all l_p sketch columns) and one range of the block's rows.
// Per step of KR = 4 V2 rows, the G operand of those rows (BF16 hi and lo, or FP32) is loaded
// once into LDS in lane order and read by the four waves; rows of a go straight to registers,
// DEPTH steps ahead of the matrix-core work.  The step loop synchronises with a bare barrier
// after an LDS-count wait only, so the a loads of later steps stay in flight across it.
template <int MODE> struct G2W { static constexpr int HALVES = (MODE == M_F32) ? 1 : 2; };


// The 16-byte G pieces of one step (rows kr .. kr+KR-1) in lane order.  Every thread issues GPT
// loads (indices past the last piece repeat it) at clamped, always valid addresses, so every step
// issues the same loads with no branch; rows at or past row_hi read as zero.
template <int MODE, int NT, int GPT>
__device__ __forceinline__ void fetch_gstep(const SK_GLOBAL uint8_t* __restrict__ gop, int64_t ldp, int tid,
                                           int kr, int row_hi, u32x4 (&gr)[GPT]) {
  constexpr int V2 = PT<MODE>::V2, HALVES = G2W<MODE>::HALVES;
  constexpr int ES = (MODE == M_F32) ? 4 : 2;
  constexpr int PIECES = HALVES * NT * 64;
  constexpr int LP = NT * 16;
#pragma unroll
  for (int i = 0; i < GPT; ++i) {
    const int p = min(tid + i * 256, PIECES - 1);
    const int r16 = p & 15, g = (p >> 4) & 3, th = p >> 6;       // th = h * NT + t
    const int h = th / NT, t = th - h * NT;
    const int r0 = kr + V2 * g;
    const int rc = min(r0, (int)ldp - V2);                       // rows past ldp are past row_hi
    const SK_GLOBAL uint8_t* src =
        gop + ((int64_t)h * LP * ldp + (int64_t)(t * 16 + r16) * ldp + rc) * ES;
    gr[i] = *reinterpret_cast<const SK_GLOBAL u32x4*>(src);
  }
}

// Stores the G pieces of the step at row kr into an LDS half, zeroing rows at or past row_hi.
template <int MODE, int NT, int GPT>
__device__ __forceinline__ void store_gstep(u32x4* dst, const u32x4 (&gr)[GPT], int tid, int kr,
                                           int row_hi) {
  constexpr int V2 = PT<MODE>::V2, HALVES = G2W<MODE>::HALVES;
  constexpr int ES = (MODE == M_F32) ? 4 : 2;
  constexpr int PIECES = HALVES * NT * 64, KRS = 4 * V2;
  const bool full = kr + KRS <= row_hi;
#pragma unroll
  for (int i = 0; i < GPT; ++i) {
    const int p = tid + i * 256;
    if (p < PIECES) {
      u32x4 v = gr[i];
      if (!full) {
        const int r0 = kr + V2 * ((p >> 4) & 3);
        uint32_t w[4] = {v[0], v[1], v[2], v[3]};
#pragma unroll
        for (int e = 0; e < V2; ++e) {
          if (r0 + e >= row_hi) {
            if constexpr (ES == 4) w[e] = 0u;
            else w[e >> 1] &= (e & 1) ? 0x0000ffffu : 0xffff0000u;
          }
        }
        v = u32x4{w[0], w[1], w[2], w[3]};
      }
      dst[p] = v;
    }
  }
}

// V2 rows x VC columns of a at clamped addresses (rows past row_hi repeat row row_hi - 1, columns
// start at most at n - VC): always valid, no branch.  Repeated rows meet zero G rows; clamped
// columns only feed outputs past n, which are discarded.
template <typename Src, int V2, int VC>
__device__ __forceinline__ void fetch_cols_clamped(const SK_GLOBAL Src* __restrict__ A, int64_t lda,
                                                   int kr, int g, int row_hi, int64_t colc,
                                                   Src (&a)[V2][VC]) {
  const int r0 = kr + V2 * g;
#pragma unroll
  for (int e = 0; e < V2; ++e) {
    const int r = min(r0 + e, row_hi - 1);
    const SK_GLOBAL Src* p = A + (int64_t)r * lda + colc;
    if constexpr (VC * sizeof(Src) == 16) {
      const u32x4 v = *reinterpret_cast<const SK_GLOBAL u32x4*>(p);
      __builtin_memcpy(a[e], &v, 16);
    } else if constexpr (VC * sizeof(Src) == 8) {
      const u32x2 v = *reinterpret_cast<const SK_GLOBAL u32x2*>(p);
      __builtin_memcpy(a[e], &v, 8);
    } else {
      const uint32_t v = *reinterpret_cast<const SK_GLOBAL uint32_t*>(p);
      __builtin_memcpy(a[e], &v, 4);
    }
  }
}

template <int MODE>
__device__ __forceinline__ GFrag<MODE> lds_gfrag(const u32x4* gl, int NTt, int t, int g, int r16) {
  GFrag<MODE> f;
  if constexpr (MODE == M_F32) {
    const u32x4 v = gl[(t * 4 + g) * 16 + r16];
    __builtin_memcpy(f.v, &v, 16);
  } else {
    const u32x4 vh = gl[(t * 4 + g) * 16 + r16];
    const u32x4 vl = gl[((NTt + t) * 4 + g) * 16 + r16];
    __builtin_memcpy(&f.hi, &vh, 16);
    __builtin_memcpy(&f.lo, &vl, 16);
  }
  return f;
}

// The step loop of k_gemm2w.  Steps s of KR rows: a(s) sits in registers ab[s % DEPTH] and G(s)
// in gr[s % DEPTH] until it is stored to LDS half s & 1 at the end of step s - 1.  a and G of step
// s + DEPTH are issued together (past the last step they re-read it, unused), so every step issues
// the same loads and waiting for G(s + 1) leaves the loads of DEPTH - 1 later steps in flight.
// Where a(s) is converted to BF16 operands, they are issued as soon as it has been, before step
// s's matrix-core work, which then runs with DEPTH steps in flight; FP32 operands are a(s)'s own
// registers, so there they follow the matrix-core work (issued earlier they cost registers and
// time).  VEC: aligned rows, n a multiple of 4; otherwise the masked element loads serve.
template <typename Src, int MODE, int NT, int DEPTH, bool VEC>
__device__ __forceinline__ void g2w_steps(const SK_GLOBAL Src* __restrict__ A, int64_t lda,
                                          int64_t n, const SK_GLOBAL uint8_t* __restrict__ gop,
                                          int64_t ldp, int row_lo, int row_hi, int nsteps, int tid,
                                          int g, int r16, int64_t col, u32x4* gl,
                                          f32x4 (&acc)[NT][4]) {
  using T = PT<MODE>;
  constexpr int V2 = T::V2, VC = 4, KR = 4 * V2;
  constexpr int PIECES = G2W<MODE>::HALVES * NT * 64;
  constexpr int GPT = (PIECES + 255) / 256;
  const int64_t colc = VEC ? min(col, n - VC) : col;
  constexpr bool kEarly = (MODE != M_F32);
  Src ab[DEPTH][V2][VC];
  u32x4 gr[DEPTH][GPT];
  auto load_step = [&](int s, int d) {
    const int sc = min(s, nsteps - 1);
    if constexpr (VEC)
      fetch_cols_clamped<Src, V2, VC>(A, lda, row_lo + sc * KR, g, row_hi, colc, ab[d]);
    else
      fetch_cols<Src, V2, VC>(A, lda, row_lo + sc * KR, g, row_hi, col, n, false, ab[d]);
    fetch_gstep<MODE, NT, GPT>(gop, ldp, tid, row_lo + sc * KR, row_hi, gr[d]);
  };
#pragma unroll
  for (int d = 0; d < DEPTH; ++d) load_step(d, d);
  store_gstep<MODE, NT, GPT>(gl, gr[0], tid, row_lo, row_hi);
  lds_barrier();

  for (int s0 = 0; s0 < nsteps; s0 += DEPTH) {
#pragma unroll
    for (int d = 0; d < DEPTH; ++d) {
      const int s = s0 + d;
      const u32x4* gb = gl + (s & 1) * PIECES;
      if (s < nsteps) {
        AFrag2<MODE> af[VC];
#pragma unroll
        for (int j = 0; j < VC; ++j) af[j] = make_a2<MODE, Src, V2, VC>(ab[d], j);
        if constexpr (kEarly) load_step(s + DEPTH, d);
#pragma unroll
        for (int t = 0; t < NT; ++t) {
          const GFrag<MODE> gq = lds_gfrag<MODE>(gb, NT, t, g, r16);
#pragma unroll
          for (int j = 0; j < VC; ++j) acc[t][j] = mma2(gq, af[j], acc[t][j]);
        }
      }
      if (!kEarly || s >= nsteps) load_step(s + DEPTH, d);
      if (s + 1 < nsteps)
        store_gstep<MODE, NT, GPT>(gl + ((s + 1) & 1) * PIECES, gr[(d + 1) % DEPTH], tid,
                                   row_lo + (s + 1) * KR, row_hi);
      lds_barrier();
    }
  }
}

template <typename Src, int MODE, int NT, int DEPTH>
__global__ __launch_bounds__(256) void k_gemm2w(const PassItem one,
                                                const PassItem* __restrict__ grp, int count) {
  using T = PT<MODE>;
  constexpr int V2 = T::V2, VC = 4, KR = 4 * V2, LP = NT * 16, SW = 256;
  constexpr int PIECES = G2W<MODE>::HALVES * NT * 64;
  constexpr int GPT = (PIECES + 255) / 256;
  __shared__ u32x4 gl[2 * PIECES];

  const PassItem it = item_of(one, grp, count, blockIdx.x, &PassItem::wg2);
  const int tile = blockIdx.x - it.wg2;
  const int64_t strip = tile % it.strips;
  const int rs = tile / it.strips, rsplit = it.rsplit;
  const SK_GLOBAL Src* __restrict__ A = gptr(reinterpret_cast<const Src*>(it.A));
  const SK_GLOBAL uint8_t* __restrict__ gop = gptr(reinterpret_cast<const uint8_t*>(it.Gop));
  const int64_t lda = it.lda, n = it.n, ldp = it.ldp, ldh = it.ldh;

  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6, g = lane >> 4, r16 = lane & 15;
  const int64_t c0 = strip * SW + wave * 64;
  const int64_t col = c0 + VC * r16;
  const int row_lo = rs * it.rchunk;
  const int row_hi = min(it.nrows, row_lo + it.rchunk);
  const int nsteps = (row_hi - row_lo + KR - 1) / KR;

  f32x4 acc[NT][VC];
#pragma unroll
  for (int t = 0; t < NT; ++t)
#pragma unroll
    for (int j = 0; j < VC; ++j) acc[t][j] = f32x4{0, 0, 0, 0};

  if (it.vec_ok && (n % VC) == 0 && n >= VC)
    g2w_steps<Src, MODE, NT, DEPTH, true>(A, lda, n, gop, ldp, row_lo, row_hi, nsteps, tid, g, r16,
                                          col, gl, acc);
  else
    g2w_steps<Src, MODE, NT, DEPTH, false>(A, lda, n, gop, ldp, row_lo, row_hi, nsteps, tid, g,
                                           r16, col, gl, acc);

  const double scale = it.fp8_exp ? ldexp(1.0, -(*gptr(it.fp8_exp))) : 1.0;
  SK_GLOBAL double* __restrict__ H = gptr(it.H);
  if (rsplit == 1) {
    // H rows of one sketch tile at a time: all 16 loads (4 rows x 4 columns per lane) are issued
    // before any store, so each tile costs one memory round trip
    const bool cfull = col + VC <= n;
#pragma unroll
    for (int t = 0; t < NT; ++t) {
      double h[4][VC];
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        SK_GLOBAL double* hp = H + (int64_t)(t * 16 + acc_row<float>(g, i)) * ldh + col;
#pragma unroll
        for (int j = 0; j < VC; ++j) h[i][j] = (cfull || col + j < n) ? hp[j] : 0.0;
      }
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        SK_GLOBAL double* hp = H + (int64_t)(t * 16 + acc_row<float>(g, i)) * ldh + col;
#pragma unroll
        for (int j = 0; j < VC; ++j)
          if (cfull || col + j < n) hp[j] = h[i][j] + scale * (double)acc[t][j][i];
      }
    }
    return;
  }
  // row splits: every workgroup writes its FP32 partial (strip-major, LP rows of 256 columns);
  // k_hsum adds them in split order into H
  SK_GLOBAL float* __restrict__ part = gptr(reinterpret_cast<float*>(it.P2));
  const int64_t pstride = (int64_t)LP * SW;
  SK_GLOBAL float* mine = part + (strip * rsplit + rs) * pstride;
#pragma unroll
  for (int t = 0; t < NT; ++t)
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int lidx = t * 16 + acc_row<float>(g, i);
      const f32x4 v = {acc[t][0][i], acc[t][1][i], acc[t][2][i], acc[t][3][i]};
      *reinterpret_cast<SK_GLOBAL f32x4*>(mine + (int64_t)lidx * SW + wave * 64 + VC * r16) = v;
    }
}

// H += scale * (sum over row splits, in split order, of the FP32 partials), in FP64.  One thread
// per 4 consecutive columns of one sketch row of one strip.  The H loads and the partial loads of
// up to four splits are issued together, so a thread waits for memory once per four splits.
__global__ __launch_bounds__(256) void k_hsum(const PassItem one, const PassItem* __restrict__ grp,
                                              int count, int LP) {
  const PassItem it = item_of(one, grp, count, blockIdx.x, &PassItem::wgh);
  if (it.rsplit <= 1) return;
  constexpr int SW = 256, U = 4;
  const int64_t q = (int64_t)(blockIdx.x - it.wgh) * 256 + threadIdx.x;   // group of 4 columns
  const int64_t per_strip = (int64_t)LP * (SW / 4);
  if (q >= per_strip * it.strips) return;
  const int64_t strip = q / per_strip;
  const int64_t w = q - strip * per_strip;
  const int lidx = (int)(w / (SW / 4));
  const int cc = (int)(w - (int64_t)lidx * (SW / 4)) * 4;
  const int64_t col = strip * SW + cc;
  if (col >= it.n) return;
  const int64_t pstride = (int64_t)LP * SW;
  const int rsplit = it.rsplit;
  const SK_GLOBAL float* base = gptr(reinterpret_cast<const float*>(it.P2)) +
                                strip * rsplit * pstride + (int64_t)lidx * SW + cc;
  SK_GLOBAL double* h = gptr(it.H) + (int64_t)lidx * it.ldh + col;
  const bool full = (col + 4 <= it.n) && ((reinterpret_cast<uintptr_t>(h) & 15) == 0);
  double hv[4];
  if (full) {
    const SK_GLOBAL f64x2* h2 = reinterpret_cast<const SK_GLOBAL f64x2*>(h);
    const f64x2 x0 = h2[0], x1 = h2[1];
    hv[0] = x0[0]; hv[1] = x0[1]; hv[2] = x1[0]; hv[3] = x1[1];
  } else {
#pragma unroll
    for (int j = 0; j < 4; ++j) hv[j] = (col + j < it.n) ? h[j] : 0.0;
  }
  double sm[4] = {0.0, 0.0, 0.0, 0.0};
  for (int r0 = 0; r0 < rsplit; r0 += U) {
    f32x4 v[U];
#pragma unroll
    for (int u = 0; u < U; ++u)   // clamped: splits past the last re-read it and are not added
      v[u] = *reinterpret_cast<const SK_GLOBAL f32x4*>(base + min(r0 + u, rsplit - 1) * pstride);
#pragma unroll
    for (int u = 0; u < U; ++u)
      if (r0 + u < rsplit)
#pragma unroll
        for (int j = 0; j < 4; ++j) sm[j] += (double)v[u][j];
  }
  const double scale = it.fp8_exp ? ldexp(1.0, -(*gptr(it.fp8_exp))) : 1.0;
  if (full) {
    SK_GLOBAL f64x2* h2 = reinterpret_cast<SK_GLOBAL f64x2*>(h);
    h2[0] = f64x2{hv[0] + scale * sm[0], hv[1] + scale * sm[1]};
    h2[1] = f64x2{hv[2] + scale * sm[2], hv[3] + scale * sm[3]};
  } else {
#pragma unroll
    for (int j = 0; j < 4; ++j)
      if (col + j < it.n) h[j] = hv[j] + scale * sm[j];
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

// A NaN or Inf anywhere in the block makes amax (the largest |x| as bits; NaN and Inf order above
// every finite value) non-finite: the block is flagged, since no scale could represent it.
__global__ void k_quant_fp8(const float* __restrict__ A, int64_t lda, int nrows, int64_t n,
                            const uint32_t* __restrict__ amax, uint8_t* __restrict__ q,
                            int64_t ldq, int* __restrict__ exp_out, int* __restrict__ nonfinite,
                            int* __restrict__ nf_host) {
  const uint32_t abits = *amax;
  const int e = fp8_exponent(abits);
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    *exp_out = e;
    if (abits >= 0x7f800000u) {
      *nonfinite = 1;
      if (nf_host) *nf_host = 1;
    }
  }
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

// ---------------------------------------------------------------- dispatch
template <typename Src, int MODE, int NT>
hipError_t gemm1_t(const PassGroup& a, hipStream_t s) {
  hipLaunchKernelGGL((k_gemm1<Src, MODE, NT>), dim3((unsigned)a.wg1_total), dim3(WAVES * 64), 0, s,
                     a.one, a.dev, a.count);
  return hipGetLastError();
}
// a steps in flight per wave in the wide-strip product (2 and 3 measured alike on the FP32-resident
// 100000 x 20000 workload; 2 needs fewer registers)
constexpr int kG2Depth = 2;
template <typename Src, int MODE, int NT>
hipError_t gemm2_t(const PassGroup& a, hipStream_t s) {
  if constexpr (MODE == M_F64) {
    hipLaunchKernelGGL((k_gemm2<Src, MODE, NT>), dim3((unsigned)a.wg2_total), dim3(WAVES * 64), 0,
                       s, a.one, a.dev, a.count);
  } else {
    hipLaunchKernelGGL((k_gemm2w<Src, MODE, NT, kG2Depth>), dim3((unsigned)a.wg2_total), dim3(256),
                       0, s, a.one, a.dev, a.count);
  }
  return hipGetLastError();
}

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

// Per-mode tile shape of a^T g: columns per lane (VC) and rows per lane per step (V2).
struct G2Shape { int VC, V2; };
G2Shape g2_shape(int mode) {
  switch (mode) {
    case M_F64: return {PT<M_F64>::VC, PT<M_F64>::V2};
    case M_F32: return {PT<M_F32>::VC, PT<M_F32>::V2};
    case M_FP8: return {PT<M_FP8>::VC, PT<M_FP8>::V2};
    default: return {PT<M_BF16>::VC, PT<M_BF16>::V2};
  }
}
int src_bytes(int src) { return src == S_F64 ? 8 : src == S_F32 ? 4 : src == S_BF16 ? 2 : 1; }
// workgroups the wide-strip product aims at for one block: one per CU (its register footprint
// allows one four-wave workgroup per CU)
constexpr int64_t kG2TargetWgs = 256;
constexpr int64_t kG1Wgs = 256;       // workgroups of g = a Omega per item: one per CU
constexpr int64_t kG1KAlign = 256;    // split granularity in columns (a multiple of every KC)
int64_t g2_target() { return kG2TargetWgs; }

}  // namespace

int64_t gemm2_strip_width(int mode) { return mode == M_F64 ? 16 * g2_shape(mode).VC : 256; }
int64_t gemm2_strips(int64_t n, int mode) { return cdiv<int64_t>(n, gemm2_strip_width(mode)); }
// Precision modes (FP32 and BF16X2, whose operands carry 24 and 16 bits) bound the length of
// their FP32 accumulation chains: at most kPrecRows rows of a per row-split partial of a^T g
// and at most kPrecCols columns per k split of g = a Omega.  The partials are summed in FP64
// (H) or in a fixed order (G).  Alg. 4 amplifies a relative sketch error by (sigma_1 /
// sigma_j)^2 (Eq. 9), so the chain length shows in the result: on sigma_j = j^-2, 250000 x 10000,
// l = 100, 8192-row blocks, the FP32 mode's relative sigma_k error against FP64 is 1.6e-3 with
// the throughput shape's 1366-row partials and 9e-6 with 512-row ones.
bool prec_mode(int mode) { return mode == M_F32 || mode == M_BF16X2; }
int64_t gemm2_partial_tiles_max() { return std::max<int64_t>(g2_target(), 1024 / WAVES); }
int64_t gemm2_partial_tiles_bound(int64_t n, int64_t rows, int mode) {
  int64_t t = gemm2_partial_tiles_max();
  if (prec_mode(mode))
    t = std::max<int64_t>(t, gemm2_strips(n, mode) *
                                 std::min<int64_t>(kGemm2MaxSplits, cdiv<int64_t>(rows, kPrecRows)));
  return t;
}

// Launch shape of one item.
//   g = a Omega: row tiles of 128 rows times k splits, as many splits as keep the launch within
//     one workgroup per CU (256): a second, partly filled round of workgroups leaves the CUs that
//     run two of them setting the pace.  Each split is a multiple of 256 columns (the widest
//     Omega' chunk).
//   a^T g: one four-wave workgroup per strip of 16 VC columns; narrow matrices also split the
//     rows across workgroups so that about half of the chip's 1024 wave slots are busy.
void plan_item(PassItem& it, int mode, int src, int splits_max) {
  const int es = src_bytes(src);
  it.vec_ok = ((((uintptr_t)it.A) % 16) == 0) && ((it.lda * es) % 16 == 0);
  it.row_tiles = (int)cdiv<int64_t>(it.nrows, ROW_TILE);
  int splits = (int)std::max<int64_t>(1, std::min<int64_t>(splits_max, kG1Wgs / it.row_tiles));
  if (prec_mode(mode))
    splits = (int)std::max<int64_t>(splits, std::min<int64_t>(splits_max, cdiv<int64_t>(it.n, kPrecCols)));
  it.kchunk = rup<int64_t>(cdiv<int64_t>(it.n, splits), kG1KAlign);
  it.splits = (int)cdiv<int64_t>(it.n, it.kchunk);
  const G2Shape sh = g2_shape(mode);
  const int KR = 4 * sh.V2;
  const int64_t steps = cdiv<int64_t>(it.nrows, KR);
  if (mode == M_F64) {
    constexpr int64_t kSlots = 1024;
    const int64_t strips = cdiv<int64_t>(it.n, 16 * sh.VC);
    int rsplit = 1;
    if (strips * WAVES < kSlots / 2) {
      rsplit = (int)std::max<int64_t>(1, std::min<int64_t>({(int64_t)kGemm2MaxSplits,
                                                             kSlots / (strips * WAVES),
                                                             steps / (2 * WAVES) + 1}));
    }
    it.rchunk = (int)rup<int64_t>(cdiv<int64_t>(it.nrows, rsplit), (int64_t)WAVES * KR);
    it.rsplit = (int)cdiv<int64_t>(it.nrows, it.rchunk);
    it.strips = (int)strips;
  } else {
    // wide strips: at most one workgroup per CU in total (row splits rounded down), each with at
    // least 8 steps of rows
    const int64_t strips = cdiv<int64_t>(it.n, 256);
    const int64_t want = g2_target() / strips;
    int rsplit = (int)std::max<int64_t>(1, std::min<int64_t>({(int64_t)kGemm2MaxSplits, want,
                                                              steps / 8}));
    if (prec_mode(mode))
      rsplit = (int)std::max<int64_t>(rsplit, std::min<int64_t>(kGemm2MaxSplits,
                                                               cdiv<int64_t>(it.nrows, kPrecRows)));
    it.rchunk = (int)rup<int64_t>(cdiv<int64_t>(it.nrows, rsplit), (int64_t)KR);
    it.rsplit = (int)cdiv<int64_t>(it.nrows, it.rchunk);
    it.strips = (int)strips;
  }
}

void plan_group(PassGroup& g, PassItem* items, int count) {
  int64_t w1 = 0, w2 = 0, wr = 0, wh = 0;
  for (int i = 0; i < count; ++i) {
    PassItem& it = items[i];
    it.red_wgs = (int)std::max<int64_t>(1, std::min<int64_t>(4096, cdiv<int64_t>((int64_t)g.LP * it.nrows, 256)));
    it.hsum_wgs = (g.mode != M_F64 && it.rsplit > 1)
                      ? (int)cdiv<int64_t>((int64_t)it.strips * g.LP * 64, 256) : 0;
    it.wg1 = (int)w1;
    it.wg2 = (int)w2;
    it.wgr = (int)wr;
    it.wgh = (int)wh;
    w1 += rup<int64_t>((int64_t)it.row_tiles * it.splits, 8);
    w2 += (int64_t)it.strips * it.rsplit;
    wr += it.red_wgs;
    wh += it.hsum_wgs;
  }
  g.count = count;
  g.wg1_total = w1;
  g.wg2_total = w2;
  g.wgr_total = wr;
  g.wgh_total = wh;
  if (count == 1) g.one = items[0];
}

hipError_t launch_gemm1(const PassGroup& a, hipStream_t s) { SK_MODE_SWITCH(gemm1_t) }
hipError_t launch_gemm2_main(const PassGroup& a, hipStream_t s) { SK_MODE_SWITCH(gemm2_t) }
hipError_t launch_gemm2(const PassGroup& a, hipStream_t s) {
  hipError_t e = launch_gemm2_main(a, s);
  if (e != hipSuccess || a.wgh_total == 0) return e;
  hipLaunchKernelGGL(k_hsum, dim3((unsigned)a.wgh_total), dim3(256), 0, s, a.one, a.dev, a.count,
                     a.LP);
  return hipGetLastError();
}

hipError_t launch_reduce1(const PassGroup& a, hipStream_t s) {
  const dim3 grid((unsigned)a.wgr_total), block(256);
  if (a.mode == M_F64) {
    hipLaunchKernelGGL((k_reduce1<double, false>), grid, block, 0, s, a.one, a.dev, a.count, a.LP);
  } else if (a.mode == M_F32) {
    hipLaunchKernelGGL((k_reduce1<float, false>), grid, block, 0, s, a.one, a.dev, a.count, a.LP);
  } else {
    hipLaunchKernelGGL((k_reduce1<float, true>), grid, block, 0, s, a.one, a.dev, a.count, a.LP);
  }
  return hipGetLastError();
}

// ---------------------------------------------------------------- FP8 quantisation launcher
namespace {
inline int grid_for(int64_t work, int block = 256, int cap = 65536) {
  int64_t g = cdiv<int64_t>(work, block);
  return (int)(g < 1 ? 1 : (g > cap ? cap : g));
}
}  // namespace

hipError_t launch_fp8_quantize(const float* A, int64_t lda, int nrows, int64_t n, uint32_t* amax,
                               uint8_t* q, int64_t ldq, int* exp_out, int* nonfinite, int* nf_host,
                               hipStream_t s) {
  hipError_t e = launch_fill_u32(amax, 1, 0u, s);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_amax, dim3(grid_for((int64_t)nrows * n, 256, 4096)), dim3(256), 0, s, A,
                     lda, nrows, n, amax);
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_quant_fp8, dim3(grid_for((int64_t)nrows * (ldq / 4), 256, 16384)),
                     dim3(256), 0, s, A, lda, nrows, n, amax, q, ldq, exp_out, nonfinite,
                     nf_host);
  return hipGetLastError();
}

}  // namespace sk
