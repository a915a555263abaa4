// After the pass: the column-block loop of Algorithm 4 (steps 9-15, re-orthogonalised as in
// Sec. 3.2, Eqs. 7-9) and the SVD of B with U = Q U~ (steps 16-19), all in FP64.
//
// Per iteration i (columns c = ib .. ib+b-1, p = ib earlier basis vectors):
//   W  = B Omega_i                 (p x b; reduction over n)
//   Y  = G(:,c) - Q W              (m x b)
//   T  = Q^T Y                     (p x b; Y_i^T Q = T^T, needed by the numerator of Eq. 9)
//   [Q_i, R_i] = qr(Y)             (tall-skinny QR, Householder on row chunks + reduction tree)
//   C  = Q^T Q_i; Z = Q_i - Q C    (Eq. 7)
//   [Q_i, R~_i] = qr(Z);  R_i = R~_i R_i
//   rank guard on diag(R_i)
//   N  = H(:,c) - B^T (T + W)      (= the transpose of H(:,c)^T - Y_i^T Q B - Omega_i^T B^T B)
//   B_i^T = N R_i^{-1}             (row-wise triangular solve)
// The two terms Y_i^T Q B and Omega_i^T B^T B of Eq. 9 share the factor B and are formed as one
// product (T + W)^T B.  B is kept transposed (B^T, n x l) so that every tall operand is a
// column-major array whose columns are contiguous.
//
// SVD of B: B^T = Q_B R_B by the same block Gram-Schmidt-with-re-orthogonalisation + TSQR scheme,
// then a one-sided (Hestenes) Jacobi SVD of R_B^T in one workgroup: R_B^T J = W with orthogonal
// columns, so B = (W S^-1) S (Q_B J)^T, i.e. U~ = W S^-1, V = Q_B J, U = Q U~.
#include <mutex>
#include <vector>

#include "common.hpp"
#include "kernels.hpp"

namespace sk {
namespace {

constexpr double kGuardTau = 1e-10;
constexpr int TPB = 256;
constexpr int JMAX = 128;       // largest l (the small SVD holds an l x l matrix in one workgroup)

inline int grid_for(int64_t work, int block = TPB, int cap = 65536) {
  int64_t g = cdiv<int64_t>(work, block);
  return (int)(g < 1 ? 1 : (g > cap ? cap : g));
}

__device__ __forceinline__ bool skip_iter(const Ctrl* ctrl, int iter) {
  return ctrl != nullptr && iter > ctrl->last_iter;
}

// 1/x and 1/sqrt(x) in FP64 from the hardware estimates, each refined by two Newton steps (the
// estimates are good to about 2^-23, so two steps reach full FP64 precision).
__device__ __forceinline__ double rcp_nr(double x) {
  double y = __builtin_amdgcn_rcp(x);
  y = y * fma(-x, y, 2.0);
  y = y * fma(-x, y, 2.0);
  return y;
}
__device__ __forceinline__ double rsq_nr(double x) {
  double y = __builtin_amdgcn_rsq(x);
  const double hx = 0.5 * x;
  y = y * fma(-hx * y, y, 1.5);
  y = y * fma(-hx * y, y, 1.5);
  return y;
}

// Sum of `cnt` per-thread values across a 256-thread block; result broadcast in out[0..cnt).
template <int CMAX>
__device__ __forceinline__ void block_sum(double (&v)[CMAX], int cnt, double* red, double* out) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
  for (int c = 0; c < CMAX; ++c) {
    if (c < cnt) {
      const double s = wave_sum(v[c]);
      if (lane == 0) red[wave * CMAX + c] = s;
    }
  }
  __syncthreads();
  if (threadIdx.x < cnt) {
    double s = 0;
    for (int w = 0; w < TPB / 64; ++w) s += red[w * CMAX + threadIdx.x];
    out[threadIdx.x] = s;
  }
  __syncthreads();
}

// Sum over the block of v[c] for c in [C0, C1) (compile-time range); result in out[c].
template <int C0, int C1, int CMAX>
__device__ __forceinline__ void block_sum_range(const double (&v)[CMAX], double* red, double* out) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
  for (int c = C0; c < C1; ++c) {
    const double s = wave_sum(v[c]);
    if (lane == 0) red[wave * CMAX + c] = s;
  }
  __syncthreads();
  if (threadIdx.x >= C0 && threadIdx.x < C1) {
    double s = 0;
    for (int w = 0; w < TPB / 64; ++w) s += red[w * CMAX + threadIdx.x];
    out[threadIdx.x] = s;
  }
  __syncthreads();
}

// Copies count values into shared memory with nthr threads, D loads in flight per thread (eight by
// default): each batch issues all of its loads (load(i), i < count) before any of its stores
// (store(i, v)), so a batch costs one memory latency instead of D.
template <int D = 8, typename LoadF, typename StoreF>
__device__ __forceinline__ void stage8(int count, int tid, int nthr, LoadF load, StoreF store) {
  for (int base = 0; base < count; base += D * nthr) {
    double v[D];
#pragma unroll
    for (int u = 0; u < D; ++u) {
      const int i = base + tid + u * nthr;
      v[u] = load(i < count ? i : count - 1);
    }
#pragma unroll
    for (int u = 0; u < D; ++u) {
      const int i = base + tid + u * nthr;
      if (i < count) store(i, v[u]);
    }
  }
}

// ------------------------------------------------------------------------------------------------
// Reductions over rows on the FP64 matrix cores: part[chunk][a][c] = sum_{r in chunk} X[a][r] Y[c][r].
// The MFMA k index is the row: lane L supplies rows r0 + 4(L/16) .. +3 of column a = 16 mt + L%16
// of X and of column c = 16 nt + L%16 of Y (32 contiguous bytes each), one 16x16x4 MFMA per row.
// The waves of a workgroup take interleaved 16-row steps (next step's operands fetched first) and
// are summed in wave order through LDS.
template <int MT, int NQ>
__device__ __forceinline__ void tn_fetch(const double* __restrict__ X, int64_t ldx,
                                         const double* __restrict__ Y, int64_t ldy, int p, int q,
                                         int64_t rr, int64_t r_end, int r16, bool full,
                                         double (&xa)[MT][4], double (&yb)[NQ][4]) {
#pragma unroll
  for (int mt = 0; mt < MT; ++mt) {
    const int a = mt * 16 + r16;
    const double* px = X + (int64_t)(a < p ? a : 0) * ldx + rr;
    if (full) {
      const f64x4 v = *reinterpret_cast<const f64x4*>(px);
#pragma unroll
      for (int j = 0; j < 4; ++j) xa[mt][j] = (a < p) ? v[j] : 0.0;
    } else {
#pragma unroll
      for (int j = 0; j < 4; ++j) xa[mt][j] = (a < p && rr + j < r_end) ? px[j] : 0.0;
    }
  }
#pragma unroll
  for (int nt = 0; nt < NQ; ++nt) {
    const int c = nt * 16 + r16;
    const double* py = Y + (int64_t)(c < q ? c : 0) * ldy + rr;
    if (full) {
      const f64x4 v = *reinterpret_cast<const f64x4*>(py);
#pragma unroll
      for (int j = 0; j < 4; ++j) yb[nt][j] = (c < q) ? v[j] : 0.0;
    } else {
#pragma unroll
      for (int j = 0; j < 4; ++j) yb[nt][j] = (c < q && rr + j < r_end) ? py[j] : 0.0;
    }
  }
}

//
// Column slices (qtot > 0): workgroup row y = blockIdx.y takes columns y q .. of Y (qtot in all),
// only the rows a < (y + 1) q of X (the upper triangle of a Gram matrix X = Y), and writes its
// partials to the slice's own region part + y * gridDim.x * p * q in the same layout.
template <int MT, int NQ>
__global__ __launch_bounds__(TPB) void k_tn_mfma(const double* __restrict__ X, int64_t ldx,
                                                 const double* __restrict__ Y, int64_t ldy, int p,
                                                 int q, int64_t rows, int RCH,
                                                 double* __restrict__ part,
                                                 const Ctrl* __restrict__ ctrl, int iter,
                                                 int qtot = 0) {
  __shared__ double red[(TPB / 64 - 1) * MT * NQ * 4 * 64];
  const int P = p, Q = q;                                    // layout of the partials
  if (qtot > 0) {
    const int y = blockIdx.y;
    Y += (int64_t)y * q * ldy;
    part += (int64_t)y * gridDim.x * p * q;
    p = min(p, (y + 1) * q);
    q = min(q, qtot - y * q);
  }
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, g = lane >> 4, r16 = lane & 15;
  const int64_t r_begin = (int64_t)blockIdx.x * RCH;
  const int64_t r_end = min<int64_t>(rows, r_begin + RCH);
  const bool aligned = ((ldx | ldy) % 4) == 0;
  f64x4 acc[MT][NQ];
#pragma unroll
  for (int mt = 0; mt < MT; ++mt)
#pragma unroll
    for (int nt = 0; nt < NQ; ++nt) acc[mt][nt] = f64x4{0, 0, 0, 0};
  double xa0[MT][4], yb0[NQ][4], xa1[MT][4], yb1[NQ][4];
  constexpr int STEP = (TPB / 64) * 16;
  int64_t r0 = r_begin + wave * 16;
  if (r0 < r_end)
    tn_fetch<MT, NQ>(X, ldx, Y, ldy, p, q, r0 + 4 * g, r_end, r16, aligned && r0 + 16 <= r_end,
                     xa0, yb0);
  // the iteration check after the first loads are in flight, so its latency overlaps theirs
  if (skip_iter(ctrl, iter)) return;
  for (; r0 < r_end; r0 += 2 * STEP) {
    const int64_t r1 = r0 + STEP, r2 = r0 + 2 * STEP;
    if (r1 < r_end)
      tn_fetch<MT, NQ>(X, ldx, Y, ldy, p, q, r1 + 4 * g, r_end, r16, aligned && r1 + 16 <= r_end,
                       xa1, yb1);
#pragma unroll
    for (int mt = 0; mt < MT; ++mt)
      if (mt * 16 < p)                            // uniform: tiles past p only in a slice
#pragma unroll
        for (int nt = 0; nt < NQ; ++nt)
#pragma unroll
          for (int j = 0; j < 4; ++j) acc[mt][nt] = mma_f64(xa0[mt][j], yb0[nt][j], acc[mt][nt]);
    mfma_drain();
    if (r2 < r_end)
      tn_fetch<MT, NQ>(X, ldx, Y, ldy, p, q, r2 + 4 * g, r_end, r16, aligned && r2 + 16 <= r_end,
                       xa0, yb0);
    if (r1 < r_end) {
#pragma unroll
      for (int mt = 0; mt < MT; ++mt)
        if (mt * 16 < p)
#pragma unroll
          for (int nt = 0; nt < NQ; ++nt)
#pragma unroll
            for (int j = 0; j < 4; ++j)
              acc[mt][nt] = mma_f64(xa1[mt][j], yb1[nt][j], acc[mt][nt]);
      mfma_drain();
    }
  }
  mfma_drain();
  if (wave > 0) {
#pragma unroll
    for (int mt = 0; mt < MT; ++mt)
#pragma unroll
      for (int nt = 0; nt < NQ; ++nt)
#pragma unroll
        for (int i = 0; i < 4; ++i)
          red[((((wave - 1) * MT + mt) * NQ + nt) * 4 + i) * 64 + lane] = acc[mt][nt][i];
  }
  __syncthreads();
  if (wave == 0) {
#pragma unroll
    for (int mt = 0; mt < MT; ++mt)
#pragma unroll
      for (int nt = 0; nt < NQ; ++nt)
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          double s = acc[mt][nt][i];
          for (int w = 1; w < TPB / 64; ++w) s += red[((((w - 1) * MT + mt) * NQ + nt) * 4 + i) * 64 + lane];
          const int a = mt * 16 + acc_row<double>(g, i), c = nt * 16 + r16;
          if (a < p && c < q) part[((int64_t)blockIdx.x * P + a) * Q + c] = s;
        }
  }
}

// The Gram matrix X^T X of the first L <= 16 MT columns of X over row chunks, each workgroup
// reading its rows of X once: the 16 x 16 tiles (mt, nt) with mt <= nt accumulate on the FP64
// matrix cores (the operand of tile nt's columns is that of tile nt's rows), and the partials go
// out in k_tn_mfma's slice layout (column slices of 32, rows a < 32 (y + 1) of slice y), so
// k_tn_final_gram sums them unchanged; the slice rows below the diagonal tiles, which nothing
// reads, are written as zeros.  The layout of the waves over rows and tiles is given with
// k_gram_mfma below.
__host__ __device__ constexpr int gram_tile_count(int MT) { return MT * (MT + 1) / 2; }

template <typename XT, int MT>
__device__ __forceinline__ void gram_fetch(const XT* __restrict__ X, int64_t ldx, int L,
                                           int64_t rr, int64_t r_end, int r16, bool full,
                                           double (&xa)[MT][4]) {
  using V4 = typename std::conditional<std::is_same<XT, double>::value, f64x4, f32x4>::type;
#pragma unroll
  for (int mt = 0; mt < MT; ++mt) {
    const int a = mt * 16 + r16;
    const XT* px = X + (int64_t)(a < L ? a : 0) * ldx + rr;
    if (full) {
      const V4 v = *reinterpret_cast<const V4*>(px);
#pragma unroll
      for (int j = 0; j < 4; ++j) xa[mt][j] = (a < L) ? (double)v[j] : 0.0;
    } else {
#pragma unroll
      for (int j = 0; j < 4; ++j) xa[mt][j] = (a < L && rr + j < r_end) ? (double)px[j] : 0.0;
    }
  }
}

// Eight waves: wave 2 r + h takes rows 16 r, 16 r + 64, ... of the chunk and half h of the upper
// tiles (two waves per SIMD, so that one loads while the other multiplies, and half the
// accumulators each); the four row groups of a half are summed through LDS in rounds.
constexpr int kGramMfmaThreads = 512;
constexpr int kGramGroups = kGramMfmaThreads / 128;   // row groups
constexpr int kGramRound2 = 7;                     // tiles per LDS round

template <int MT> struct GramHalves {
  static constexpr int N = gram_tile_count(MT), H0 = (N + 1) / 2, H1 = N - H0;
  static constexpr int first(int h) { return h ? H0 : 0; }
  static constexpr int count(int h) { return h ? H1 : H0; }
};

template <int MT, int HALF>
__device__ __forceinline__ void gram_half_mma(const double (&xa)[MT][4],
                                              f64x4 (&acc)[GramHalves<MT>::H0]) {
  constexpr int T0 = GramHalves<MT>::first(HALF), T1 = T0 + GramHalves<MT>::count(HALF);
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    int t = 0;
#pragma unroll
    for (int nt = 0; nt < MT; ++nt)
#pragma unroll
      for (int mt = 0; mt <= nt; ++mt) {
        if (t >= T0 && t < T1) acc[t - T0] = mma_f64(xa[mt][j], xa[nt][j], acc[t - T0]);
        ++t;
      }
  }
}

// Round u0 of the LDS sum: row groups 1.. store their tiles u0 .. u0 + kGramRound2 - 1 of the
// half (STORE), or row group 0 adds them to its own and writes the chunk partials (!STORE).
template <int MT, int HALF, bool STORE>
__device__ __forceinline__ void gram_half_round(int u0, const f64x4 (&acc)[GramHalves<MT>::H0],
                                                double* red, int rgp, int lane, int g, int r16,
                                                int L, double* mine, int64_t per_slice) {
  constexpr int T0 = GramHalves<MT>::first(HALF), T1 = T0 + GramHalves<MT>::count(HALF);
  int t = 0;
#pragma unroll
  for (int nt = 0; nt < MT; ++nt)
#pragma unroll
    for (int mt = 0; mt <= nt; ++mt) {
      const int u = t - T0;
      if (t >= T0 && t < T1 && u >= u0 && u < u0 + kGramRound2) {
        if constexpr (STORE) {
#pragma unroll
          for (int i = 0; i < 4; ++i)
            red[((((HALF * (kGramGroups - 1)) + rgp - 1) * kGramRound2 + (u - u0)) * 4 + i) * 64 +
                lane] = acc[u][i];
        } else {
#pragma unroll
          for (int i = 0; i < 4; ++i) {
            double sm = acc[u][i];
            for (int w = 1; w < kGramGroups; ++w)
              sm += red[((((HALF * (kGramGroups - 1)) + w - 1) * kGramRound2 + (u - u0)) * 4 + i) *
                            64 + lane];
            const int a = mt * 16 + acc_row<double>(g, i), c = nt * 16 + r16;
            if (a < L && c < L) mine[(c >> 5) * per_slice + (int64_t)a * 32 + (c & 31)] = sm;
          }
        }
      }
      ++t;
    }
}

template <typename XT, int MT>
__global__ __launch_bounds__(kGramMfmaThreads) void k_gram_mfma(const XT* __restrict__ X, int64_t ldx,
                                                            int L, int64_t rows, int RCH,
                                                            double* __restrict__ part) {
  using GH = GramHalves<MT>;
  __shared__ double red[2 * (kGramGroups - 1) * kGramRound2 * 4 * 64];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, g = lane >> 4, r16 = lane & 15;
  const int half = wave & 1, rgp = wave >> 1;
  const int64_t r_begin = (int64_t)blockIdx.x * RCH;
  const int64_t r_end = min<int64_t>(rows, r_begin + RCH);
  const bool aligned = (ldx % 4) == 0;
  f64x4 acc[GH::H0];
#pragma unroll
  for (int t = 0; t < GH::H0; ++t) acc[t] = f64x4{0, 0, 0, 0};
  double xa[MT][4];
  constexpr int STEP = kGramGroups * 16;
  for (int64_t r0 = r_begin + rgp * 16; r0 < r_end; r0 += STEP) {
    gram_fetch<XT, MT>(X, ldx, L, r0 + 4 * g, r_end, r16, aligned && r0 + 16 <= r_end, xa);
    if (half == 0) gram_half_mma<MT, 0>(xa, acc);
    else gram_half_mma<MT, 1>(xa, acc);
    mfma_drain();
  }
  const int64_t per_slice = (int64_t)gridDim.x * L * 32;
  double* mine = part + (int64_t)blockIdx.x * L * 32;
#pragma unroll
  for (int u0 = 0; u0 < GH::H0; u0 += kGramRound2) {
    __syncthreads();
    if (rgp > 0) {
      if (half == 0) gram_half_round<MT, 0, true>(u0, acc, red, rgp, lane, g, r16, L, mine, per_slice);
      else gram_half_round<MT, 1, true>(u0, acc, red, rgp, lane, g, r16, L, mine, per_slice);
    }
    __syncthreads();
    if (rgp == 0) {
      if (half == 0) gram_half_round<MT, 0, false>(u0, acc, red, rgp, lane, g, r16, L, mine, per_slice);
      else gram_half_round<MT, 1, false>(u0, acc, red, rgp, lane, g, r16, L, mine, per_slice);
    }
  }
  // the tiles (nt + 1, nt) of even nt: rows of slice nt / 2 below its diagonal tile
  if (wave == 2) {
#pragma unroll
    for (int nt = 0; nt + 1 < MT; nt += 2)
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int a = (nt + 1) * 16 + acc_row<double>(g, i), c = nt * 16 + r16;
        if (a < L && c < L) mine[(c >> 5) * per_slice + (int64_t)a * 32 + (c & 31)] = 0.0;
      }
  }
}

// Y = X W for the rows x L column-major X and the upper triangular L x L W (row-major, leading
// dimension ldw), L <= 16 MT, on the FP64 matrix cores, reading X once: every workgroup stages W,
// zero-padded to 16 MT, in LDS, and its waves take 16-row blocks of its row range.  The MFMA k
// index is the column a of X (lane (r16, g) supplies X[r0 + r16][4 s + g]); output tile nt only
// meets k < 16 (nt + 1), W being upper triangular.  Eight waves, two per SIMD, each with one
// row buffer: one wave's loads overlap the other's matrix-core work.  Rows past `rows` are read
// clamped and not written.
template <typename XT, int MT>
__device__ __forceinline__ void rmul_fetch(const XT* __restrict__ X, int64_t ldx, int L,
                                           int64_t row, int g, double (&xa)[MT][4]) {
#pragma unroll
  for (int t = 0; t < MT; ++t)
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int a = 16 * t + 4 * j + g;
      const double v = (double)X[(int64_t)(a < L ? a : L - 1) * ldx + row];
      xa[t][j] = a < L ? v : 0.0;
    }
}

constexpr int kRmulThreads = 512;   // two waves per SIMD: one loads its rows while the other multiplies
constexpr size_t rmul_lds_bytes(int MT) { return (size_t)(16 * MT) * (16 * MT + 1) * sizeof(double); }

template <typename XT, int MT>
__global__ __launch_bounds__(kRmulThreads) void k_rmul_mfma(double* __restrict__ Y, int64_t ldy,
                                                   const XT* __restrict__ X, int64_t ldx,
                                                   int64_t rows, int L,
                                                   const double* __restrict__ W, int ldw,
                                                   int RCH) {
  extern __shared__ double ws[];
  constexpr int LP = 16 * MT, WS = LP + 1;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, g = lane >> 4, r16 = lane & 15;
  stage8<25>(LP * LP, threadIdx.x, kRmulThreads,
         [&](int idx) {
           const int a = idx / LP, c = idx - a * LP;
           return (a < L && c < L && c >= a) ? W[(int64_t)a * ldw + c] : 0.0;
         },
         [&](int idx, double v) {
           const int a = idx / LP, c = idx - a * LP;
           ws[a * WS + c] = v;
         });
  __syncthreads();
  const int64_t r_begin = (int64_t)blockIdx.x * RCH;
  const int64_t r_end = min<int64_t>(rows, r_begin + RCH);
  double xa[MT][4];
  auto block = [&](const double (&xb)[MT][4], int64_t r0) {
    f64x4 acc[MT];
#pragma unroll
    for (int nt = 0; nt < MT; ++nt) acc[nt] = f64x4{0, 0, 0, 0};
#pragma unroll
    for (int nt = 0; nt < MT; ++nt)
#pragma unroll
      for (int t = 0; t <= nt; ++t)
#pragma unroll
        for (int j = 0; j < 4; ++j)
          acc[nt] = mma_f64(xb[t][j], ws[(16 * t + 4 * j + g) * WS + nt * 16 + r16], acc[nt]);
    mfma_drain();
#pragma unroll
    for (int nt = 0; nt < MT; ++nt)
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int64_t r = r0 + acc_row<double>(g, i);
        const int c = nt * 16 + r16;
        if (r < r_end && c < L) Y[(int64_t)c * ldy + r] = acc[nt][i];
      }
  };
  constexpr int SUB = (kRmulThreads / 64) * 16;
  for (int64_t r0 = r_begin + wave * 16; r0 < r_end; r0 += SUB) {
    rmul_fetch<XT, MT>(X, ldx, L, min<int64_t>(r0 + r16, rows - 1), g, xa);
    block(xa, r0);
  }
}

// Sum of the chunk partials (chunk stride pq entries) for the entries e0 .. e0 + ecount - 1, entry
// e = a q + c going to out[a * ldo + c] (row-major, leading dimension ldo).  A workgroup owns 64
// entries (one per lane, consecutive in part, so the loads coalesce); its 16 waves take the
// chunks in interleaved order and their partial sums are added in wave order through LDS, so the
// summation order is fixed.
constexpr int kTnFinalThreads = 1024;

// This lane's sum over the chunks of wave `wave` (chunks wave, wave + NW, ...) for entry ec: eight
// chunks per batch, all loads issued before the adds (clamped to the wave's first chunk, whose
// value is then dropped), so a wave pays one memory latency per eight chunks.
template <int NW>
__device__ __forceinline__ double chunk_sum(const double* __restrict__ part, int nchunks,
                                            int64_t pq, int64_t ec, int wave) {
  double s = 0;
  for (int ch0 = wave; ch0 < nchunks; ch0 += 8 * NW) {
    double v[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int ch = ch0 + u * NW;
      v[u] = part[(int64_t)(ch < nchunks ? ch : ch0) * pq + ec];
    }
#pragma unroll
    for (int u = 0; u < 8; ++u)
      if (ch0 + u * NW < nchunks) s += v[u];
  }
  return s;
}

__global__ __launch_bounds__(kTnFinalThreads) void k_tn_final(const double* __restrict__ part,
                                                              int nchunks, int64_t pq, int64_t e0,
                                                              int64_t ecount, int q,
                                                              double* __restrict__ out, int ldo,
                                                              const Ctrl* __restrict__ ctrl,
                                                              int iter) {
  constexpr int NW = kTnFinalThreads / 64;
  __shared__ double sm[NW * 64];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int64_t i = (int64_t)blockIdx.x * 64 + lane;
  const bool live = i < ecount;
  const double s = chunk_sum<NW>(part, nchunks, pq, e0 + (live ? i : 0), wave);
  if (skip_iter(ctrl, iter)) return;      // after the loads (uniform over the workgroup)
  sm[wave * 64 + lane] = s;
  __syncthreads();
  if (wave == 0 && live) {
    double t = sm[lane];
    for (int w = 1; w < NW; ++w) t += sm[w * 64 + lane];
    const int64_t e = e0 + i;
    out[(e / q) * ldo + e % q] = t;
  }
}

// The upper triangle of an L x L Gram matrix from the column-sliced chunk partials of k_tn_mfma
// (slices of 32 columns, ny of them): out[a * ldo + 32 y + c] for a < min(L, 32 (y + 1)).
__global__ __launch_bounds__(kTnFinalThreads) void k_tn_final_gram(const double* __restrict__ part,
                                                                   int nchunks, int L, int ny,
                                                                   double* __restrict__ out,
                                                                   int ldo) {
  constexpr int NW = kTnFinalThreads / 64;
  __shared__ double sm[NW * 64];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int64_t per = (int64_t)L * 32;
  const int64_t i = (int64_t)blockIdx.x * 64 + lane;
  const bool live = i < per * ny;
  const int64_t ic = live ? i : 0;
  const int y = (int)(ic / per);
  const int64_t rem = ic - y * per;
  const double s = chunk_sum<NW>(part + (int64_t)y * nchunks * per, nchunks, per, rem, wave);
  sm[wave * 64 + lane] = s;
  __syncthreads();
  if (wave == 0 && live) {
    double t = sm[lane];
    for (int w = 1; w < NW; ++w) t += sm[w * 64 + lane];
    const int a = (int)(rem / 32), c = 32 * y + (int)(rem % 32);
    if (a < min(L, 32 * (y + 1)) && c < L) out[a * ldo + c] = t;
  }
}

// out[c][r] = base[c][r] + alpha * sum_a X[a][r] W[a][c]  (W row-major p x q, ldw); base may be
// null (taken as 0) and may alias out.  One lane per row, kNnThreads rows per workgroup.  W is
// staged in LDS, zero-padded to QMAX >= q columns and to whole chunks of rows; each lane reads its
// row of X in chunks of kNnChunk entries, all loads of a chunk in flight together, and accumulates
// the QMAX columns in registers (rows a >= p of a chunk read X's last row and count as zero).  The
// first chunk and the base entries are fetched before the iteration check and the staging stores,
// so their latencies overlap; Rs, the same for every lane, is staged in LDS with W.
//
// With Rs non-null (q x q upper triangular, row-major, leading dimension q) each row v of the
// result is replaced by the solution x of x Rs = v (forward substitution) before it is written, and
// only the first `keep` entries are solved (keep = ctrl->keep_last on the iteration the rank guard
// stopped at, q otherwise); the others are written as zero.
constexpr int kNnChunk = 32;
constexpr int kNnThreads = 128;

template <typename BT, int QMAX>
__global__ __launch_bounds__(kNnThreads) void k_nn_update(double* __restrict__ out, int64_t ldo,
                                                          const BT* base, int64_t ldb,
                                                          const double* __restrict__ X,
                                                          int64_t ldx, int p,
                                                          const double* __restrict__ W, int ldw,
                                                          int q, int64_t rows, double alpha,
                                                          const Ctrl* __restrict__ ctrl, int iter,
                                                          const double* __restrict__ Rs = nullptr,
                                                          int qtot = 0, int tri = 1) {
  if (qtot > 0) {
    // column slices: workgroup row y = blockIdx.y takes output columns y q .. (qtot in all), with
    // the rows a < (y + 1) q of W only when W is upper triangular (tri)
    const int y = blockIdx.y;
    out += (int64_t)y * q * ldo;
    W += y * q;
    if (tri) p = min(p, (y + 1) * q);
    q = min(q, qtot - y * q);
  }
  constexpr int CH = kNnChunk;
  constexpr int FILL = (JMAX * QMAX + kNnThreads - 1) / kNnThreads;
  constexpr int RFILL = (QMAX * QMAX + kNnThreads - 1) / kNnThreads;
  __shared__ double ws[JMAX * QMAX];           // W, rows rounded up to whole chunks
  __shared__ double rsh[QMAX * QMAX];          // Rs (zero-padded), when given
  const int tid = threadIdx.x;
  const int64_t r = (int64_t)blockIdx.x * kNnThreads + tid;
  const int64_t rc = r < rows ? r : rows - 1;
  const int qc = q - 1, plast = p > 0 ? p - 1 : 0;
  const int nw = ((p + CH - 1) / CH) * CH * QMAX;   // staged entries
  double x[CH];
  auto load_chunk = [&](int a0) {
#pragma unroll
    for (int s = 0; s < CH; ++s) {
      const int a = a0 + s;
      const double v = X[(int64_t)(a < p ? a : plast) * ldx + rc];
      x[s] = a < p ? v : 0.0;
    }
  };
  // all loads first (W clamped to W[0], which always exists), then the check and the LDS stores
  double wv[FILL];
#pragma unroll
  for (int u = 0; u < FILL; ++u) {
    const int idx = tid + u * kNnThreads, a = idx / QMAX, c = idx % QMAX;
    const bool in = a < p && c < q;
    const double v = W[in ? a * ldw + c : 0];
    wv[u] = in ? v : 0.0;
  }
  double rv[RFILL];
  if (Rs != nullptr) {
#pragma unroll
    for (int u = 0; u < RFILL; ++u) {
      const int idx = tid + u * kNnThreads, a = idx / QMAX, c = idx % QMAX;
      const double v = Rs[min(a, qc) * q + min(c, qc)];
      rv[u] = (a < q && c < q) ? v : 0.0;
    }
  }
  if (p > 0) load_chunk(0);
  double bv[QMAX];
#pragma unroll
  for (int c = 0; c < QMAX; ++c)
    bv[c] = base ? (double)base[(int64_t)(c < q ? c : qc) * ldb + rc] : 0.0;
  if (skip_iter(ctrl, iter)) return;
#pragma unroll
  for (int u = 0; u < FILL; ++u) {
    const int idx = tid + u * kNnThreads;
    if (idx < nw) ws[idx] = wv[u];
  }
  if (Rs != nullptr) {
#pragma unroll
    for (int u = 0; u < RFILL; ++u) {
      const int idx = tid + u * kNnThreads;
      if (idx < QMAX * QMAX) rsh[idx] = rv[u];
    }
  }
  __syncthreads();
  double acc[QMAX];
#pragma unroll
  for (int c = 0; c < QMAX; ++c) acc[c] = 0.0;
  for (int a0 = 0; a0 < p; a0 += CH) {
    if (a0 > 0) load_chunk(a0);
    const double* w = ws + a0 * QMAX;
#pragma unroll
    for (int s = 0; s < CH; ++s)
#pragma unroll
      for (int c = 0; c < QMAX; ++c) acc[c] = fma(x[s], w[s * QMAX + c], acc[c]);
  }
  if (r >= rows) return;
  if (Rs == nullptr) {
#pragma unroll
    for (int c = 0; c < QMAX; ++c)
      if (c < q) out[c * ldo + r] = bv[c] + alpha * acc[c];
  } else {
    const int keep = (ctrl != nullptr && iter == ctrl->last_iter) ? ctrl->keep_last : q;
    double xs[QMAX];
#pragma unroll
    for (int c = 0; c < QMAX; ++c) {
      double v = 0.0;
      if (c < q) {
        v = bv[c] + alpha * acc[c];
#pragma unroll
        for (int k = 0; k < c; ++k) v = fma(-xs[k], rsh[k * QMAX + c], v);
        v = (c < keep) ? v / rsh[c * QMAX + c] : 0.0;
      }
      xs[c] = v;
      if (c < q) out[c * ldo + r] = v;
    }
  }
}

// ------------------------------------------------------------------------------------------------
// Tall-skinny QR.  Level arrays are column-major (rows x b).  Each chunk of CR rows is factored by
// Householder reflections (the LAPACK dlarfg convention) with RPT rows per thread held in
// registers; its b x b R goes to the next level's stacked array.  The Q factor is then formed from
// the root down by applying each chunk's reflectors to its b x b block of the level above.
// One column step of the Householder factorisation (J compile-time): with s_c = sum_{i>J} x_iJ x_ic,
// the reflector of column J (LAPACK dlarfg: beta = -sign(alpha) sqrt(alpha^2 + s_J),
// tau = (beta - alpha) / beta, v_i = x_iJ / (alpha - beta), v_J = 1) gives
// w_c = v^T x_c = x_Jc + s_c / (alpha - beta) from a single block reduction.
template <int J, int B, int RPT>
__device__ __forceinline__ void house_col(double (&x)[RPT][B], int b, double* red, double* sc,
                                          double* rowj, double* tau_out) {
  double part[B];
#pragma unroll
  for (int c = 0; c < B; ++c) part[c] = 0.0;
#pragma unroll
  for (int t = 0; t < RPT; ++t) {
    const int i = threadIdx.x + t * TPB;
    if (i > J) {
#pragma unroll
      for (int c = J; c < B; ++c) part[c] = fma(x[t][J], x[t][c], part[c]);
    }
  }
  if (threadIdx.x == J) {
#pragma unroll
    for (int c = J; c < B; ++c) rowj[c] = x[0][c];
  }
  block_sum_range<J, B, B>(part, red, sc);
  const double alpha = rowj[J], xn2 = sc[J];
  double tj, beta, scal;
  if (xn2 == 0.0) {
    tj = 0.0; beta = alpha; scal = 0.0;
  } else {
    beta = -copysign(sqrt(alpha * alpha + xn2), alpha);
    tj = (beta - alpha) / beta;
    scal = 1.0 / (alpha - beta);
  }
  if (threadIdx.x == 0 && J < b) tau_out[J] = tj;
  double w[B];
#pragma unroll
  for (int c = J + 1; c < B; ++c) w[c] = tj * (rowj[c] + scal * sc[c]);
#pragma unroll
  for (int t = 0; t < RPT; ++t) {
    const int i = threadIdx.x + t * TPB;
    if (i > J) {
      const double vi = x[t][J] * scal;
#pragma unroll
      for (int c = J + 1; c < B; ++c) x[t][c] = fma(-vi, w[c], x[t][c]);
      x[t][J] = vi;
    } else if (i == J) {
#pragma unroll
      for (int c = J + 1; c < B; ++c) x[t][c] -= w[c];
      x[t][J] = beta;
    }
  }
  __syncthreads();   // rowj / sc are rewritten by the next column
}

template <int J, int B, int RPT>
struct HouseCols {
  static __device__ __forceinline__ void run(double (&x)[RPT][B], int b, double* red, double* sc,
                                             double* rowj, double* tau_out) {
    house_col<J, B, RPT>(x, b, red, sc, rowj, tau_out);
    HouseCols<J + 1, B, RPT>::run(x, b, red, sc, rowj, tau_out);
  }
};
template <int B, int RPT>
struct HouseCols<B, B, RPT> {
  static __device__ __forceinline__ void run(double (&)[RPT][B], int, double*, double*, double*,
                                             double*) {}
};

// Chunk factorisation; B >= b is the compile-time width (columns b..B-1 are zero padding).
template <int B, int RPT>
__global__ __launch_bounds__(TPB) void k_house_factor(double* __restrict__ X, int64_t ldx,
                                                      int64_t rows, int b, int CR,
                                                      double* __restrict__ tau,
                                                      double* __restrict__ Rnext, int64_t ldr,
                                                      const Ctrl* __restrict__ ctrl, int iter) {
  if (skip_iter(ctrl, iter)) return;
  __shared__ double red[(TPB / 64) * B];
  __shared__ double sc[B];
  __shared__ double rowj[B];
  const int64_t r0 = (int64_t)blockIdx.x * CR;
  const int cnt = (int)min<int64_t>(CR, rows - r0);
  double x[RPT][B];
#pragma unroll
  for (int t = 0; t < RPT; ++t) {
    const int i = threadIdx.x + t * TPB;
#pragma unroll
    for (int c = 0; c < B; ++c) x[t][c] = (c < b && i < cnt) ? X[c * ldx + r0 + i] : 0.0;
  }
  HouseCols<0, B, RPT>::run(x, b, red, sc, rowj, tau + (int64_t)blockIdx.x * b);
  // reflectors back in place (rows < cnt), R (upper triangle, zero below) to the next level
#pragma unroll
  for (int t = 0; t < RPT; ++t) {
    const int i = threadIdx.x + t * TPB;
#pragma unroll
    for (int c = 0; c < B; ++c) {
      if (c < b) {
        if (i < cnt) X[c * ldx + r0 + i] = x[t][c];
        if (i < b) Rnext[c * ldr + (int64_t)blockIdx.x * b + i] = (i <= c) ? x[t][c] : 0.0;
      }
    }
  }
}

// Explicit Q of each chunk: Y = H_0 H_1 ... H_{b-1} [Qabove(chunk rows); 0], written over the
// chunk's reflectors.  At the root (Qabove == null) the start is D = diag(sign(R_jj)) with R the
// root's stacked rows, so the final R = D R has a nonnegative diagonal; the root also writes that
// R (row-major b x b) to Rout.
template <int J, int B, int RPT>
struct FormCols {   // applies H_J, then H_{J-1}, ..., H_0
  static __device__ __forceinline__ void run(const double (&v)[RPT][B], double (&y)[RPT][B], int b,
                                             const double* tau, double* red, double* bc) {
    if (J < b) {
      const double tj = tau[J];
      if (tj != 0.0) {
        double w[B];
#pragma unroll
        for (int c = 0; c < B; ++c) w[c] = 0.0;
#pragma unroll
        for (int t = 0; t < RPT; ++t) {
          const int i = threadIdx.x + t * TPB;
          const double vi = (i > J) ? v[t][J] : (i == J ? 1.0 : 0.0);
#pragma unroll
          for (int c = 0; c < B; ++c) w[c] = fma(vi, y[t][c], w[c]);
        }
        block_sum_range<0, B, B>(w, red, bc);
#pragma unroll
        for (int t = 0; t < RPT; ++t) {
          const int i = threadIdx.x + t * TPB;
          const double vi = (i > J) ? v[t][J] : (i == J ? 1.0 : 0.0);
#pragma unroll
          for (int c = 0; c < B; ++c) y[t][c] = fma(-tj * vi, bc[c], y[t][c]);
        }
        __syncthreads();
      }
    }
    FormCols<J - 1, B, RPT>::run(v, y, b, tau, red, bc);
  }
};
template <int B, int RPT>
struct FormCols<-1, B, RPT> {
  static __device__ __forceinline__ void run(const double (&)[RPT][B], double (&)[RPT][B], int,
                                             const double*, double*, double*) {}
};

// Explicit Q of each chunk: Y = H_0 H_1 ... H_{b-1} [Qabove(chunk rows); 0], written over the
// chunk's reflectors.  At the root (Qabove == null) the start is D = diag(sign(R_jj)) with R the
// root's stacked rows, so the final R = D R has a nonnegative diagonal; the root also writes that
// R (row-major b x b) to Rout.
template <int B, int RPT>
__global__ __launch_bounds__(TPB) void k_house_form(double* __restrict__ X, int64_t ldx,
                                                    int64_t rows, int b, int CR,
                                                    const double* __restrict__ tau,
                                                    const double* __restrict__ Qabove,
                                                    int64_t lda, const double* __restrict__ Rroot,
                                                    int64_t ldr, double* __restrict__ Rout,
                                                    const Ctrl* __restrict__ ctrl, int iter) {
  if (skip_iter(ctrl, iter)) return;
  __shared__ double red[(TPB / 64) * B];
  __shared__ double bc[B];
  __shared__ double d[B];
  const int64_t r0 = (int64_t)blockIdx.x * CR;
  const int cnt = (int)min<int64_t>(CR, rows - r0);
  if (Qabove == nullptr && threadIdx.x < b) {
    const double rjj = Rroot[threadIdx.x * ldr + threadIdx.x];
    d[threadIdx.x] = (rjj < 0.0) ? -1.0 : 1.0;
  }
  __syncthreads();
  if (Qabove == nullptr && Rout != nullptr) {
    for (int idx = threadIdx.x; idx < b * b; idx += TPB) {
      const int i = idx / b, c = idx % b;
      Rout[idx] = (c >= i) ? d[i] * Rroot[c * ldr + i] : 0.0;
    }
  }
  double v[RPT][B], y[RPT][B];
#pragma unroll
  for (int t = 0; t < RPT; ++t) {
    const int i = threadIdx.x + t * TPB;
#pragma unroll
    for (int c = 0; c < B; ++c) {
      v[t][c] = (c < b && i < cnt) ? X[c * ldx + r0 + i] : 0.0;
      double y0 = 0.0;
      if (c < b && i < b) {
        if (Qabove) y0 = Qabove[c * lda + (int64_t)blockIdx.x * b + i];
        else y0 = (i == c) ? d[c] : 0.0;
      }
      y[t][c] = y0;
    }
  }
  FormCols<B - 1, B, RPT>::run(v, y, b, tau + (int64_t)blockIdx.x * b, red, bc);
#pragma unroll
  for (int t = 0; t < RPT; ++t) {
    const int i = threadIdx.x + t * TPB;
    if (i < cnt) {
#pragma unroll
      for (int c = 0; c < B; ++c)
        if (c < b) X[c * ldx + r0 + i] = y[t][c];
    }
  }
}

// ------------------------------------------------------------------------------------------------
// Small b x b / p x b kernels (one workgroup).

// R = R2 R1 (upper triangular), then the rank guard of the column-block loop.
// Rank guard on the combined R_i (b x b, row-major): the leading columns whose diagonal exceeds
// kGuardTau r0 are kept (r0 = R_0[0][0]); the first iteration that keeps fewer than b is the last.
__device__ void guard_store(int keep, int b, int iter, Ctrl* ctrl) {
  if (keep < b) {
    ctrl->last_iter = iter;
    ctrl->keep_last = keep;
    ctrl->l_eff = iter * b + keep;
  } else {
    ctrl->l_eff = (iter + 1) * b;
    ctrl->keep_last = b;
  }
}
__device__ void guard_apply(const double* R, int b, int iter, Ctrl* ctrl) {
  if (iter == 0) ctrl->r0 = R[0];
  const double thr = kGuardTau * ctrl->r0;
  int keep = 0;
  while (keep < b && fabs(R[keep * b + keep]) > thr) ++keep;
  guard_store(keep, b, iter, ctrl);
}

__global__ void k_guard(const double* __restrict__ R1, const double* __restrict__ R2,
                        double* __restrict__ R, int b, int iter, int t, Ctrl* __restrict__ ctrl) {
  if (skip_iter(ctrl, iter)) return;
  for (int idx = threadIdx.x; idx < b * b; idx += blockDim.x) {
    const int i = idx / b, c = idx % b;
    double s = 0.0;
    for (int q = i; q <= c; ++q) s = fma(R2[i * b + q], R1[q * b + c], s);
    R[idx] = (c >= i) ? s : 0.0;
  }
  __syncthreads();
  if (threadIdx.x == 0) guard_apply(R, b, iter, ctrl);
}

// ------------------------------------------------------------------------------------------------
// Cholesky QR of one column block (the panels of the loop above, b <= 32 columns): with the block
// Gram matrix G = Y^T Y = R^T R, Y R^-1 has orthonormal columns up to O(u cond(Y)^2).  The loop
// uses one such step on Y and two on the projected Z = Q_i - Q C (Eq. 7), which brings Z to
// orthonormality at working precision whenever cond(Z) is below about 1/sqrt(u); R_i is the
// product of the three factors.  A block whose Gram matrix has a pivot below kCholQrPivot G_jj
// (its columns are too close to dependent for the Gram matrix to resolve) or a non-finite pivot is
// flagged in ctrl->pad[0], and the host repeats the whole loop with Householder TSQR.
constexpr double kCholQrPivot = 1e-10;

// The Gram matrix G = Y^T Y of a column block (b x b, entries e0 .. e0 + b^2 - 1 of the row
// reduction's chunk partials, chunk stride pq) and its Cholesky factor, once, in one workgroup:
// the 16 waves sum the chunks (fixed order, as k_tn_final), then wave 0 factors G in registers:
// lane c holds column c of G (then of R, then of X = R^-1), takes the entries of other columns by
// lane broadcasts, and G is padded with the identity to BMAX columns so that no loop tests a
// bound (the padded factor is diag(R, I)).  Writes X (b x b, row-major) and Rout = R Rprev
// (Rprev null: identity).  On the last step of a block (`last` set) it also applies the rank guard
// to R Rprev and forms Wn = T + W (p x b, the combined weights of the numerator of Eq. 9).  A pivot
// below kCholQrPivot G_jj, or a non-finite one, marks the block (ctrl->pad[0] = 1) instead.
constexpr int kGramThreads = 512;     // the factoring wave needs up to 256 registers
template <int BMAX>
__global__ __launch_bounds__(kGramThreads) void k_gram_chol(
    const double* __restrict__ part, int nchunks, int64_t pq, int64_t e0, int b,
    const double* __restrict__ Rprev, double* __restrict__ Rout, double* __restrict__ Xout,
    int last, const double* __restrict__ T, const double* __restrict__ Wt,
    double* __restrict__ Wn, int p, Ctrl* __restrict__ ctrl, int iter) {
  constexpr int NW = kGramThreads / 64;
  __shared__ double sm[NW * 64];
  __shared__ double gram[BMAX * BMAX];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int bb = b * b;
  for (int og = 0; og < bb; og += 64) {                      // uniform
    const int idx = og + lane;
    const bool live = idx < bb;
    const double s = chunk_sum<NW>(part, nchunks, pq, e0 + (live ? idx : 0), wave);
    sm[wave * 64 + lane] = s;
    __syncthreads();
    if (wave == 0 && live) {
      double t = sm[lane];
      for (int w = 1; w < NW; ++w) t += sm[w * 64 + lane];
      gram[idx] = t;
    }
    __syncthreads();
  }
  if (skip_iter(ctrl, iter)) return;                         // uniform, after the loads
  if (last)
    for (int idx = threadIdx.x; idx < p * b; idx += kGramThreads) Wn[idx] = T[idx] + Wt[idx];
  if (wave != 0) return;
  const bool lcol = lane < b;
  double a[BMAX], rpc[BMAX];
#pragma unroll
  for (int i = 0; i < BMAX; ++i) a[i] = (i < b && lcol) ? gram[i * b + lane] : (i == lane ? 1.0 : 0.0);
  const double gdg = lcol ? gram[lane * b + lane] : 1.0;
#pragma unroll
  for (int k = 0; k < BMAX; ++k)                             // column of Rprev, or of I
    rpc[k] = (Rprev != nullptr && k < b && lcol) ? Rprev[k * b + lane] : (k == lane ? 1.0 : 0.0);
  // right-looking Cholesky, G = R^T R: lane c ends with R[i][c] (i <= c) in a[i]
  bool bad = false;
  double rinv[BMAX];                                         // 1 / R[j][j]
#pragma unroll
  for (int j = 0; j < BMAX; ++j) {
    const double d = dpp::lane(a[j], j);
    bad |= !(d > kCholQrPivot * dpp::lane(gdg, j)) || !(d < INFINITY);
    // 1/sqrt(d) from the refined hardware estimate; R[j][j] = d / sqrt(d)
    const double inv = rsq_nr(d), rj = d * inv;
    rinv[j] = inv;
    a[j] = (lane == j) ? rj : (lane > j ? a[j] * inv : a[j]);
#pragma unroll
    for (int i = j + 1; i < BMAX; ++i) {
      const double rji = dpp::lane(a[j], i);                 // R[j][i]
      a[i] = (lane >= i) ? fma(-rji, a[j], a[i]) : a[i];
    }
  }
  if (bad) {
    if (lane == 0) ctrl->pad[0] = 1;
    return;
  }
  // X = R^-1 by columns: lane c solves R x = e_c from the bottom, x[i] = X[i][c]
  double x[BMAX];
#pragma unroll
  for (int i = BMAX - 1; i >= 0; --i) {
    double acc = 0.0;
#pragma unroll
    for (int k = i + 1; k < BMAX; ++k) {
      const double rik = dpp::lane(a[i], k);                 // R[i][k]
      acc = (lane >= k) ? fma(rik, x[k], acc) : acc;
    }
    x[i] = (lane == i) ? rinv[i] : ((lane > i) ? -rinv[i] * acc : 0.0);
  }
  // Rout = R Rprev (upper triangular) and X: lane c writes column c
#pragma unroll
  for (int i = 0; i < BMAX; ++i) {
    double s = 0.0;
#pragma unroll
    for (int k = i; k < BMAX; ++k) s = (lane >= k) ? fma(dpp::lane(a[i], k), rpc[k], s) : s;
    if (i < b && lcol) {
      Rout[i * b + lane] = s;
      Xout[i * b + lane] = x[i];
    }
  }
  if (last) {
    // the rank guard on diag(R Rprev) = diag(R) diag(Rprev)
    const double r00 = dpp::lane(a[0], 0) * dpp::lane(rpc[0], 0);
    const double thr = kGuardTau * (iter == 0 ? r00 : ctrl->r0);
    int keep = b;
#pragma unroll
    for (int j = BMAX - 1; j >= 0; --j) {
      const double djj = dpp::lane(a[j], j) * dpp::lane(rpc[j], j);
      if (j < b && !(fabs(djj) > thr)) keep = j;             // first column at or below the threshold
    }
    if (lane == 0) {
      if (iter == 0) ctrl->r0 = r00;
      guard_store(keep, b, iter, ctrl);
    }
  }
}

// One Cholesky QR step for narrow blocks (b <= B <= 12): every lane factors the b x b Gram matrix
// G (row-major, leading dimension b, upper triangle read, padded with the identity to B) in its own
// registers, a few hundred FP64 operations with no communication, then solves x R = y for its
// own row y of Y by forward substitution and writes x back (Y <- Y R^-1).  Workgroup 0 also writes
// Rout = R Rprev (Rprev null: identity); on the last step (`last` set) every lane takes the rank
// guard's decision from diag(R) diag(Rprev) and writes zeros in place of the dropped columns, and
// workgroup 0 records the decision and forms Wn = T + W (p x b, the combined weights of the
// numerator of Eq. 9).  A pivot below kCholQrPivot G_jj, or a non-finite one, marks the block
// (ctrl->pad[0] = 1) and leaves Y as it was.
template <int B>
__host__ __device__ constexpr int upk(int i, int c) { return i * B - i * (i - 1) / 2 + (c - i); }

constexpr int kLaneCholThreads = 256;
template <int B>
__global__ __launch_bounds__(kLaneCholThreads) void k_cholqr_lane(
    double* __restrict__ Y, int64_t ldy, int64_t rows, const double* __restrict__ G, int b,
    const double* __restrict__ Rprev, double* __restrict__ Rout, int last,
    const double* __restrict__ T, const double* __restrict__ Wt, double* __restrict__ Wn, int p,
    Ctrl* __restrict__ ctrl, int iter) {
  constexpr int NU = B * (B + 1) / 2;
  __shared__ double rs[B * B], rpv[B * B];
  const int tid = threadIdx.x;
  const int64_t r = (int64_t)blockIdx.x * kLaneCholThreads + tid;
  const int64_t rc = r < rows ? r : 0;
  __shared__ double gsh[B * B + B];   // G identity-padded to B x B, then the Rprev diagonal
  double y[B], R[NU], gd[B], pd[B];
  // the Gram matrix is the same for every lane: one entry per thread into LDS (issued before the
  // row loads, so waiting for it leaves them in flight), then read back by every lane
  // (every thread loads at a clamped address, without branches, so the row loads follow at once)
  const int bl = b - 1;
  const int gi = min(tid / B, B - 1), gc = tid % B, gj = min(max(tid - B * B, 0), B - 1);
  const double* rpd = (Rprev != nullptr) ? Rprev : G;
  const double* gp = (tid < B * B) ? G + min(gi, bl) * b + min(gc, bl) : rpd + min(gj, bl) * (b + 1);
  const double gv = *gp;
#pragma unroll
  for (int c = 0; c < B; ++c) {
    const double v = Y[(c < b ? c : 0) * ldy + rc];
    y[c] = (c < b) ? v : 0.0;
  }
  if (tid < B * B)
    gsh[tid] = (gi < b && gc < b) ? gv : (gi == gc ? 1.0 : 0.0);
  else if (tid < B * B + B)
    gsh[tid] = (gj < b && Rprev != nullptr) ? gv : 1.0;
  lds_barrier();
#pragma unroll
  for (int i = 0; i < B; ++i)
#pragma unroll
    for (int c = i; c < B; ++c) R[upk<B>(i, c)] = gsh[i * B + c];
#pragma unroll
  for (int j = 0; j < B; ++j) {
    gd[j] = R[upk<B>(j, j)];
    pd[j] = gsh[B * B + j];
  }
  if (skip_iter(ctrl, iter)) return;
  // right-looking Cholesky in place, G = R^T R
  bool bad = false;
  double rinv[B];
#pragma unroll
  for (int j = 0; j < B; ++j) {
    const double d = R[upk<B>(j, j)];
    bad |= !(d > kCholQrPivot * gd[j]) || !(d < INFINITY);
    const double inv = rsq_nr(d);                     // refined 1/sqrt(d); R[j][j] = d / sqrt(d)
    rinv[j] = inv;
    R[upk<B>(j, j)] = d * inv;
#pragma unroll
    for (int c = j + 1; c < B; ++c) R[upk<B>(j, c)] *= inv;
#pragma unroll
    for (int i = j + 1; i < B; ++i)
#pragma unroll
      for (int c = i; c < B; ++c)
        R[upk<B>(i, c)] = fma(-R[upk<B>(j, i)], R[upk<B>(j, c)], R[upk<B>(i, c)]);
  }
  if (bad) {
    if (blockIdx.x == 0 && tid == 0) ctrl->pad[0] = 1;
    return;
  }
  // the rank guard's decision: diag(R Rprev) = diag(R) diag(Rprev)
  const double r00 = R[upk<B>(0, 0)] * pd[0];
  int keep = b;
  if (last) {
    const double thr = kGuardTau * (iter == 0 ? r00 : ctrl->r0);
#pragma unroll
    for (int j = B - 1; j >= 0; --j)
      if (j < b && !(fabs(R[upk<B>(j, j)] * pd[j]) > thr)) keep = j;
  }
  // x R = y, forward substitution over the columns
  if (r < rows) {
    double x[B];
#pragma unroll
    for (int c = 0; c < B; ++c) {
      double v = y[c];
#pragma unroll
      for (int k = 0; k < c; ++k) v = fma(-x[k], R[upk<B>(k, c)], v);
      x[c] = v * rinv[c];
    }
#pragma unroll
    for (int c = 0; c < B; ++c)
      if (c < b) Y[c * ldy + r] = (c < keep) ? x[c] : 0.0;
  }
  if (blockIdx.x != 0) return;
  if (tid < b * b) rpv[tid] = (Rprev != nullptr) ? Rprev[tid] : 0.0;
  if (tid == 0) {
#pragma unroll
    for (int i = 0; i < B; ++i)
#pragma unroll
      for (int c = 0; c < B; ++c) rs[i * B + c] = (c >= i) ? R[upk<B>(i, c)] : 0.0;
  }
  __syncthreads();
  for (int idx = tid; idx < b * b; idx += kLaneCholThreads) {
    const int i = idx / b, c = idx % b;
    double s = 0.0;
    if (c >= i) {
      if (Rprev == nullptr) s = rs[i * B + c];
      else
        for (int k = i; k <= c; ++k) s = fma(rs[i * B + k], rpv[k * b + c], s);
    }
    Rout[idx] = s;
  }
  if (!last) return;
  for (int idx = tid; idx < p * b; idx += kLaneCholThreads) Wn[idx] = T[idx] + Wt[idx];
  if (tid == 0) {
    if (iter == 0) ctrl->r0 = r00;
    guard_store(keep, b, iter, ctrl);
  }
}

// Y <- Y X in place (X = R^-1 from k_gram_chol, b x b row-major, staged in LDS zero-padded to
// BMAX).  On the last step of a block the columns the rank guard dropped are written as zeros.
constexpr int kApplyThreads = 256;
template <int BMAX>
__global__ __launch_bounds__(kApplyThreads) void k_cholqr_apply(
    double* __restrict__ Y, int64_t ldy, int64_t rows, const double* __restrict__ X, int b,
    int last, const Ctrl* __restrict__ ctrl, int iter) {
  __shared__ double xs[BMAX * BMAX];
  const int tid = threadIdx.x;
  const int64_t r = (int64_t)blockIdx.x * kApplyThreads + tid;
  const int64_t rc = r < rows ? r : 0;
  double y[BMAX];
#pragma unroll
  for (int c = 0; c < BMAX; ++c) {
    const double v = Y[(c < b ? c : 0) * ldy + rc];
    y[c] = (c < b) ? v : 0.0;
  }
  stage8(BMAX * BMAX, tid, kApplyThreads,
         [&](int idx) {
           const int k = idx / BMAX, c = idx % BMAX;
           return (k < b && c < b) ? X[k * b + c] : 0.0;
         },
         [&](int idx, double v) { xs[idx] = v; });
  if (skip_iter(ctrl, iter)) return;
  const int keep = (last && ctrl != nullptr && iter == ctrl->last_iter) ? ctrl->keep_last : b;
  __syncthreads();
  if (r >= rows) return;
#pragma unroll
  for (int c = 0; c < BMAX; ++c) {
    double s = 0.0;
#pragma unroll
    for (int k = 0; k <= c; ++k) s = fma(y[k], xs[k * BMAX + c], s);
    if (c < b) Y[c * ldy + r] = (c < keep) ? s : 0.0;
  }
}

// out = A + B (p x q, row-major with leading dimension q)
__global__ void k_add_small(const double* __restrict__ A, const double* __restrict__ B,
                            double* __restrict__ out, int count, const Ctrl* __restrict__ ctrl,
                            int iter) {
  if (skip_iter(ctrl, iter)) return;
  for (int i = threadIdx.x; i < count; i += blockDim.x) out[i] = A[i] + B[i];
}

__global__ void k_zero_cols(double* __restrict__ Q, int64_t ldq, int64_t rows, int c0, int b,
                            const Ctrl* __restrict__ ctrl, int iter) {
  if (skip_iter(ctrl, iter) || iter != ctrl->last_iter) return;
  const int keep = ctrl->keep_last;
  const int64_t total = (int64_t)(b - keep) * rows;
  for (int64_t q = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; q < total;
       q += (int64_t)gridDim.x * blockDim.x) {
    const int c = (int)(q / rows);
    Q[(c0 + keep + c) * ldq + (q - (int64_t)c * rows)] = 0.0;
  }
}

// R_B blocks of one panel (row-major R_B, leading dimension ldr):
//   R_B[0:c0, panel] = C1 + C2 R1,  R_B[panel, panel] = R2 R1.
__global__ void k_rb_assemble(const double* __restrict__ C1, const double* __restrict__ C2,
                              const double* __restrict__ R1, const double* __restrict__ R2,
                              double* __restrict__ RB, int ldr, int c0, int w) {
  for (int idx = threadIdx.x; idx < (c0 + w) * w; idx += blockDim.x) {
    const int i = idx / w, c = idx % w;
    double s = 0.0;
    if (i < c0) {
      s = C1[i * w + c];
      for (int q = 0; q <= c; ++q) s = fma(C2[i * w + q], R1[q * w + c], s);
    } else {
      const int ii = i - c0;
      for (int q = ii; q <= c; ++q) s = fma(R2[ii * w + q], R1[q * w + c], s);
    }
    RB[i * ldr + c0 + c] = s;
  }
}

// ------------------------------------------------------------------------------------------------
// Cholesky QR of B^T (shifted Cholesky QR3: Fukaya, Kannan, Nakatsukasa, Zhang, Yamamoto, SIAM J.
// Sci. Comput. 42(1), 2020).  Only R_B is needed downstream (V is formed from B^T itself), and R_B
// is a Cholesky factor of the L x L Gram matrix B B^T.  One Cholesky of the Gram matrix squares
// the condition number, so three passes are made: the first on B B^T + s I with the shift
// s = 11 (n L + L (L + 1)) u tr(B B^T) (u = 2^-53; the trace bounds ||B||_2^2), which keeps the
// factorisation defined for cond(B) up to about 1/u and gives Q1 = B^T R1^-1 with a moderate
// condition number; then Cholesky QR twice on Q1.  R_B = R3 R2 R1.  A pivot that is not positive
// and finite in any pass sends the host to the Gram-Schmidt + TSQR path.
// Gm (upper triangle read, row-major, leading dimension ldg) + s I = R^T R with R upper triangular
// with a positive diagonal; s = shift_rel tr(Gm) when shift_rel > 0, else 0.  Writes R and, when
// Rinv is non-null, R^-1 (row-major, leading dimension ldr, zeros below the diagonal).  A pivot that
// is not positive and finite sets *fail (left as it was otherwise) and writes identity factors.
// Conditioning tests, each setting *ill: ill_rel > 0, a pivot below ill_rel times the diagonal
// entry of Gm it started from; dev_rel > 0, an entry of R farther than dev_rel from the identity.
// The outputs of a failed factorisation: identity factors, so that the kernels that consume them
// before the host reads the failure flag work on defined, finite values.
__device__ __forceinline__ void chol_write_identity(double* __restrict__ R,
                                                    double* __restrict__ Rinv, int ldr, int L,
                                                    int tid) {
  for (int idx = tid; idx < L * L; idx += blockDim.x) {
    const int i = idx / L, c = idx % L;
    R[(int64_t)i * ldr + c] = (i == c) ? 1.0 : 0.0;
    if (Rinv != nullptr) Rinv[(int64_t)i * ldr + c] = (i == c) ? 1.0 : 0.0;
  }
}

// The factorisation (k_chol_blk), in 16 x 16 blocks of the matrix padded with the
// identity to LP = 16 MT rows: per block column, wave 0 factors the diagonal block (one pivot at a
// time, its lanes in step through LDS, which orders one wave's accesses), one thread per column
// solves the block row to its right (R_kk^T Y = A_k), and the waves update the trailing upper
// tiles on the FP64 matrix cores (A_ij -= R_ki^T R_kj, 16 x 16 x 4 products over the 16 rows of
// the block row).  R^-1 by blocks: every diagonal block inverted by its own wave (right-looking
// back substitution, one lane per column), Y_it = X_ii R_it in place of R_it, then the blocks at
// distance s = j - i from the diagonal, X_ij = -sum_{t = i+1..j} Y_it X_tj, one wave per block;
// R^-1 is kept transposed in the strictly lower triangle (X[k][c] at [c][k]) and its diagonal in
// ri.  Three barriers per block column and one per distance.
constexpr int kCholBlkThreads = 512;

size_t cholb_lds_bytes(int L) {
  const size_t LP = (size_t)rup(L, 16);
  return (LP * (LP + 1) + 3 * LP) * sizeof(double);
}

__device__ __forceinline__ void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

__global__ __launch_bounds__(kCholBlkThreads) void k_chol_blk(const double* __restrict__ Gm,
                                                              int ldg, int L, double shift_rel,
                                                              double* __restrict__ R,
                                                              double* __restrict__ Rinv, int ldr,
                                                              int* __restrict__ fail,
                                                              double ill_rel, double dev_rel,
                                                              int* __restrict__ ill,
                                                              int force_fail) {
  extern __shared__ double a[];
  const int MT = (L + 15) >> 4, LP = 16 * MT, LS = LP + 1;
  double* rd = a + (int64_t)LP * LS;     // diagonal of R
  double* ri = rd + LP;                  // its inverse (the diagonal of R^-1)
  double* g0 = ri + LP;                  // the diagonal the factorisation started from
  __shared__ int bad;
  __shared__ double shs;
  __shared__ double prow[32];            // the current two pivot rows of a diagonal block
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6, g = lane >> 4, r16 = lane & 15;
  // the upper triangle of Gm, zeros below it, the identity on the padding (all 112^2 entries in
  // one batch of loads at the largest size)
  stage8<25>(LP * LP, tid, kCholBlkThreads,
         [&](int idx) {
           const int i = idx / LP, c = idx - i * LP;
           return (i < L && c < L) ? (c >= i ? Gm[(int64_t)i * ldg + c] : 0.0)
                                   : (i == c ? 1.0 : 0.0);
         },
         [&](int idx, double v) {
           const int i = idx / LP, c = idx - i * LP;
           a[i * LS + c] = v;
         });
  if (tid == 0) { bad = 0; shs = 0.0; }
  __syncthreads();
  if (shift_rel > 0.0) {
    if (tid < 64) {
      double t = 0.0;
      for (int i = tid; i < L; i += 64) t += a[i * LS + i];
      t = wave_sum(t);
      if (tid == 0) shs = t * shift_rel;
    }
    __syncthreads();
    for (int i = tid; i < L; i += kCholBlkThreads) a[i * LS + i] += shs;
    __syncthreads();
  }
  for (int i = tid; i < LP; i += kCholBlkThreads) g0[i] = a[i * LS + i];
  __syncthreads();

  for (int kb = 0; kb < MT; ++kb) {
    const int k0 = 16 * kb;
    // (a) the diagonal block, by wave 0 in registers: lane c < 16 holds column c (rows 0..15),
    // takes the pivot row through LDS, and ends with R's rows in its column.  The scalings and
    // updates are not masked to the upper triangle: an entry on or above the diagonal only ever
    // meets entries on or above it (its own column's pivot-row entry and the pivot row), and the
    // entries below it, which they also change, are neither read nor written back.
    if (wave == 0) {
      const int c = lane;
      double col[16];
#pragma unroll
      for (int i = 0; i < 16; ++i) col[i] = c < 16 ? a[(k0 + i) * LS + k0 + c] : 0.0;
      bool fl = false;
      double piv[16];                            // the pivots, for the conditioning test after
#pragma unroll
      for (int p = 0; p < 16; ++p) piv[p] = 1.0;
      // two pivots per step: P = k0 + p and P + 1.  R[P][P+1] and the second pivot come from lane
      // broadcasts, both rows of R go through LDS together, and the trailing entries take both
      // updates in pivot order (the same operations as one pivot at a time, so the same bits)
#pragma unroll
      for (int p = 0; p < 16; p += 2) {
        const int P = k0 + p;
        const double d0 = dpp::lane(col[p], p);       // A[P][P], the same in every lane
        piv[p] = d0;
        if (P < L && ((force_fail && P == 0) || !(d0 > 0.0) || !(d0 < INFINITY))) fl = true;
        if (fl) break;
        const double e = dpp::lane(col[p], p + 1);    // A[P][P+1]
        const double d1 = dpp::lane(col[p + 1], p + 1);
        const double r0 = rsq_nr(d0), rp0 = d0 * r0;  // refined 1/sqrt(d); R[P][P] = d / sqrt(d)
        const double r01 = e * r0;                    // R[P][P+1]
        const double d1u = fma(-r01, r01, d1);        // the second pivot after the first's update
        piv[p + 1] = d1u;
        if (P + 1 < L && (!(d1u > 0.0) || !(d1u < INFINITY))) fl = true;
        if (fl) break;
        const double r1 = rsq_nr(d1u), rp1 = d1u * r1;
        if (lane == 0) { rd[P] = rp0; ri[P] = r0; rd[P + 1] = rp1; ri[P + 1] = r1; }
        col[p] = (c == p) ? rp0 : col[p] * r0;                                   // row P of R
        col[p + 1] = (c == p + 1) ? rp1 : fma(-r01, col[p], col[p + 1]) * r1;  // row P + 1
        // both rows to every lane through LDS (one wave's LDS accesses execute in order)
        if (c < 16) { prow[c] = col[p]; prow[16 + c] = col[p + 1]; }
        __builtin_amdgcn_wave_barrier();
#pragma unroll
        for (int i = p + 2; i < 16; ++i)
          col[i] = fma(-prow[16 + i], col[p + 1], fma(-prow[i], col[p], col[i]));
        __builtin_amdgcn_wave_barrier();
      }
      if (c < 16)
#pragma unroll
        for (int i = 0; i < 16; ++i)
          if (i <= c) a[(k0 + i) * LS + k0 + c] = col[i];
      if (lane == 0 && ill_rel > 0.0 && !fl) {
        bool low = false;
#pragma unroll
        for (int p = 0; p < 16; ++p) low |= (k0 + p < L) && !(piv[p] >= ill_rel * g0[k0 + p]);
        if (low) *ill = 1;
      }
      if (fl && lane == 0) bad = 1;
    }
    __syncthreads();
    if (bad) {
      if (tid == 0) *fail = 1;
      chol_write_identity(R, Rinv, ldr, L, tid);
      return;
    }
    // (b) the block row to the right: column c of R_k solves R_kk^T y = A_k(:, c)
    if (tid < LP - k0 - 16) {
      const int c = k0 + 16 + tid;
      double y[16];
#pragma unroll
      for (int p = 0; p < 16; ++p) y[p] = a[(k0 + p) * LS + c];
#pragma unroll
      for (int p = 0; p < 16; ++p) {
        y[p] *= ri[k0 + p];
#pragma unroll
        for (int q = p + 1; q < 16; ++q) y[q] = fma(-a[(k0 + p) * LS + k0 + q], y[p], y[q]);
      }
#pragma unroll
      for (int p = 0; p < 16; ++p) a[(k0 + p) * LS + c] = y[p];
    }
    __syncthreads();
    // (c) trailing tiles (mi, nc), kb < mi <= nc < MT, one wave per tile
    const int nb = MT - kb - 1;
    for (int tt = wave; tt < nb * (nb + 1) / 2; tt += kCholBlkThreads / 64) {
      int nc = 0;
      while ((nc + 1) * (nc + 2) / 2 <= tt) ++nc;
      const int mi = tt - nc * (nc + 1) / 2;
      const int i0 = k0 + 16 + 16 * mi, c0 = k0 + 16 + 16 * nc;
      f64x4 acc = f64x4{0, 0, 0, 0};
#pragma unroll
      for (int s = 0; s < 4; ++s) {
        const int kr = k0 + 4 * s + g;
        acc = mma_f64(a[kr * LS + i0 + r16], a[kr * LS + c0 + r16], acc);
      }
      mfma_drain();
#pragma unroll
      for (int i = 0; i < 4; ++i) a[(i0 + acc_row<double>(g, i)) * LS + c0 + r16] -= acc[i];
    }
    __syncthreads();
  }
  bool dev = false;
  for (int idx = tid; idx < L * L; idx += kCholBlkThreads) {
    const int i = idx / L, c = idx - i * L;
    const double v = c > i ? a[i * LS + c] : (c == i ? rd[i] : 0.0);
    R[(int64_t)i * ldr + c] = v;
    dev |= dev_rel > 0.0 && !(fabs(v - (c == i ? 1.0 : 0.0)) <= dev_rel);
  }
  if (dev) *ill = 1;                             // every writer stores the same value
  if (Rinv == nullptr) return;
  __syncthreads();
  // (d1) X_ii = R_ii^-1, wave i, lane c owning column c (q from the bottom: x_q = rhs_q / R_qq,
  // then rhs_t -= R_tq x_q for t < q)
  if (wave < MT && lane < 16) {
    const int k0 = 16 * wave, c = lane;
    double x[16];
#pragma unroll
    for (int q = 0; q < 16; ++q) x[q] = (q == c) ? 1.0 : 0.0;
#pragma unroll
    for (int q = 15; q >= 0; --q) {
      if (q <= c) {
        x[q] *= ri[k0 + q];
#pragma unroll
        for (int t = 0; t < q; ++t) x[t] = fma(-a[(k0 + t) * LS + k0 + q], x[q], x[t]);
      }
    }
#pragma unroll
    for (int q = 0; q < 16; ++q)
      if (q < c) a[(k0 + c) * LS + k0 + q] = x[q];
  }
  __syncthreads();
  // (d2) Y_it = X_ii R_it in place of R_it (i < t), one thread per column of a block
  for (int w = tid; w < 16 * MT * (MT - 1) / 2; w += kCholBlkThreads) {
    const int col = w & 15, bp = w >> 4;
    int t = 1;
    while (t * (t + 1) / 2 <= bp) ++t;
    const int i = bp - t * (t - 1) / 2;        // block pair (i, t), i < t
    const int k0 = 16 * i, c = 16 * t + col;
    double y[16], o[16];
#pragma unroll
    for (int r = 0; r < 16; ++r) y[r] = a[(k0 + r) * LS + c];
#pragma unroll
    for (int q = 0; q < 16; ++q) {
      double sacc = ri[k0 + q] * y[q];
#pragma unroll
      for (int r = q + 1; r < 16; ++r) sacc = fma(a[(k0 + r) * LS + k0 + q], y[r], sacc);
      o[q] = sacc;
    }
#pragma unroll
    for (int q = 0; q < 16; ++q) a[(k0 + q) * LS + c] = o[q];
  }
  __syncthreads();
  // (d3) X_ij = -sum_{t=i+1..j} Y_it X_tj at distance s = j - i, one wave per block
  for (int s = 1; s < MT; ++s) {
    for (int i = wave; i < MT - s; i += kCholBlkThreads / 64) {
      const int j = i + s, qi = 16 * i, cj = 16 * j;
      f64x4 acc = f64x4{0, 0, 0, 0};
      for (int t = i + 1; t <= j; ++t) {
#pragma unroll
        for (int kk = 0; kk < 4; ++kk) {
          const int r = 4 * kk + g;                // row r of block t
          const double av = a[(qi + r16) * LS + 16 * t + r];
          double bv;
          if (t < j) bv = a[(cj + r16) * LS + 16 * t + r];
          else bv = (r < r16) ? a[(cj + r16) * LS + cj + r] : (r == r16 ? ri[cj + r16] : 0.0);
          acc = mma_f64(av, bv, acc);
        }
      }
      mfma_drain();
#pragma unroll
      for (int k = 0; k < 4; ++k) a[(cj + r16) * LS + qi + acc_row<double>(g, k)] = -acc[k];
    }
    __syncthreads();
  }
  for (int idx = tid; idx < L * L; idx += kCholBlkThreads) {
    const int i = idx / L, c = idx - i * L;
    Rinv[(int64_t)i * ldr + c] = c > i ? a[c * LS + i] : (c == i ? ri[i] : 0.0);
  }
}

// out = X Y for upper triangular L x L X and Y (row-major, leading dimension L); out must not
// alias X or Y.  One workgroup per row i (row i of X staged in LDS), one thread per column; the
// loads of Y are issued eight at a time.
__global__ __launch_bounds__(JMAX) void k_trmm_upper(const double* __restrict__ X,
                                                     const double* __restrict__ Y,
                                                     double* __restrict__ out, int L) {
  __shared__ double xs[JMAX];
  const int i = blockIdx.x, c = threadIdx.x;
  if (c < L) xs[c] = X[i * L + c];
  __syncthreads();
  if (c >= L) return;
  double s = 0.0;
  for (int k0 = i; k0 <= c; k0 += 8) {
    double y[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) y[u] = Y[(k0 + u <= c ? k0 + u : c) * L + c];
#pragma unroll
    for (int u = 0; u < 8; ++u)
      if (k0 + u <= c) s = fma(xs[k0 + u], y[u], s);
  }
  out[i * L + c] = s;
}

// Both products of k_trmm_upper in one launch (blockIdx.y picks the pair), the first also
// writing its diagonal to diag0.
__global__ __launch_bounds__(JMAX) void k_trmm_upper2(const double* __restrict__ X0,
                                                      const double* __restrict__ Y0,
                                                      double* __restrict__ out0,
                                                      const double* __restrict__ X1,
                                                      const double* __restrict__ Y1,
                                                      double* __restrict__ out1, int L,
                                                      double* __restrict__ diag0) {
  __shared__ double xs[JMAX];
  const bool second = blockIdx.y != 0;
  const double* __restrict__ X = second ? X1 : X0;
  const double* __restrict__ Y = second ? Y1 : Y0;
  double* __restrict__ out = second ? out1 : out0;
  const int i = blockIdx.x, c = threadIdx.x;
  if (c < L) xs[c] = X[i * L + c];
  __syncthreads();
  if (c >= L) return;
  double s = 0.0;
  for (int k0 = i; k0 <= c; k0 += 8) {
    double y[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) y[u] = Y[(k0 + u <= c ? k0 + u : c) * L + c];
#pragma unroll
    for (int u = 0; u < 8; ++u)
      if (k0 + u <= c) s = fma(xs[k0 + u], y[u], s);
  }
  out[i * L + c] = s;
  if (!second && c == i) diag0[i] = s;
}

__global__ void k_set_int(int* p, int v) {
  if (threadIdx.x == 0) *p = v;
}
__global__ void k_set_int2(int* p, int* q, int v) {
  if (threadIdx.x == 0) { *p = v; *q = v; }
}


// ------------------------------------------------------------------------------------------------
// One-sided Jacobi on M = R_B^T (L x L, L = l_eff): columns of M are the rows of R_B.  Outputs:
// sig (descending), perm, W = M J (column perm[j] holds sigma_j u_j).  Each sweep meets every
// column pair once, in rounds of disjoint pairs rotated in parallel.
constexpr int JSWEEPS = 40;
constexpr int kJacobiGroups = 64;      // lane groups (one pair each per round); N / 2 <= 64

// Rounds of a sweep over n columns in the home / visitor order below: h = ceil(n / 2) rounds,
// then the two halves of size h in parallel.
__host__ __device__ constexpr int jacobi_rounds(int n) {
  int r = 0;
  while (n > 1) { const int h = (n + 1) >> 1; r += h; n = h; }
  return r;
}

// The pair of lane group k in round r of a sweep over N (even) columns, as (home, visitor), or
// 255 for both when the group idles.  The order: the n columns of a level (padded to 2h with an
// empty column when n is odd) split into homes 0..h-1 and visitors h..2h-1; in round r < h group
// j pairs home j with visitor h + (j + r) mod h, so every home meets every visitor; then the
// homes and the visitors each repeat the scheme on their own, at the next level, the homes on
// the first half of the level's groups (so every home stays with its group) and the visitors on
// the second half.  A group's level-d range spans 64 >> d groups, which holds the h <= 64 >> d
// pairs of that level.  Between two rounds a group thus changes only its visitor, except where
// a level ends.
__host__ __device__ __forceinline__ void jacobi_pair(int N, int r, int k, int& p, int& q) {
  int n = N, base = 0, span = kJacobiGroups, depth = 0;
  int off[8], pn[8];
  p = q = 255;
  while (depth < 8) {
    const int h = (n + 1) >> 1;
    if (r < h) {
      const int j = k - base;
      if (j < 0 || j >= h) return;
      int v = j + r;
      if (v >= h) v -= h;
      int pos[2] = {j, h + v};
#pragma unroll
      for (int s = 0; s < 2; ++s) {
        if (pos[s] >= n) return;                   // the padding column of this level
        for (int d = depth - 1; d >= 0; --d) {
          pos[s] += off[d];
          if (pos[s] >= pn[d]) return;             // the padding column of an enclosing level
        }
      }
      p = pos[0];
      q = pos[1];
      return;
    }
    r -= h;
    const int half = span >> 1;
    const bool second = (k - base) >= half;
    off[depth] = second ? h : 0;
    pn[depth] = n;
    ++depth;
    if (second) base += half;
    n = h;
    span = half;
  }
}

// 1/x from the hardware estimate and one Newton step (about 2^-46 relative): enough for a
// rotation angle, which only steers convergence.
__device__ __forceinline__ double rcp_nr1(double x) {
  const double y = __builtin_amdgcn_rcp(x);
  return y * fma(-x, y, 2.0);
}
__device__ __forceinline__ double rsq_nr1(double x) {
  const double y = __builtin_amdgcn_rsq(x);
  return y * fma(-0.5 * x * y, y, 1.5);
}

// M (N columns, each padded to LPAD = 8 EPL rows, zero beyond L) lives in LDS with column stride
// CS (LPAD, plus 8 when LPAD / 8 is even, so that the 8 pairs a wave touches spread over the LDS
// banks); the pair table is built once.  Eight lanes per pair, lane gl holding rows gl + 8 e: the
// inner product is reduced within the 8 lanes.  A group keeps its home column in registers while
// the home stays (it is written back only when it changes, and at the end of each sweep, if it was
// rotated) and moves only the visitor through LDS.  The right factor is not accumulated: with
// M J = W (orthogonal columns, norms sigma), B^T = Q_B R_B and M = R_B^T, B^T W = Q_B J S^2, so
// V = B^T W S^-2 (see run_finalize).
constexpr int kJacobiLds = 160 * 1024 - 4096;   // dynamic LDS limit of k_jacobi (static: norms)
constexpr int kJacobiLpp = 8;                   // lanes per pair (the 8-lane reduction below)
constexpr int kJacobiThreads = kJacobiGroups * kJacobiLpp;
// rows per lane (EPL) the kernel is built for: LPAD = kJacobiLpp EPL covers every L <= JMAX
#define SK_JACOBI_EPLS(X) X(2) X(4) X(8) X(12) X(13) X(14) X(16)

__host__ __device__ constexpr int jacobi_cs(int lpad) {
  return ((lpad / kJacobiLpp) % 2 == 0) ? lpad + kJacobiLpp : lpad;
}

template <int EPL>
__global__ __launch_bounds__(kJacobiThreads) void k_jacobi(const double* __restrict__ RB, int ldr,
                                                           int L, double* __restrict__ W, int ldw,
                                                           int* __restrict__ info,
                                                           double* __restrict__ sig,
                                                           int* __restrict__ perm,
                                                           double* __restrict__ nrm) {
  extern __shared__ double M[];           // N columns x CS, then the pair table
  __shared__ int rotated, large;
  __shared__ double nrm2[JMAX];           // squared column norms
  constexpr int LPP = kJacobiLpp, LPAD = LPP * EPL, CS = jacobi_cs(LPAD);
  const int N = (L + 1) & ~1;
  const int RN = jacobi_rounds(N);
  uint8_t* pairs = reinterpret_cast<uint8_t*>(M + (int64_t)N * CS);   // RN x 64 x {home, visitor}
  const double tol = (double)L * 2.220446049250313e-16;
  const double tol2 = tol * tol;
  // Convergence is quadratic at the end: once every pair of a sweep starts with a relative
  // inner product |g| / sqrt(a b) <= sqrt(tol) / 8, the rotations of a further sweep would move
  // the columns by about N (sqrt(tol) / 8)^2 <= tol relative, the stopping threshold itself, so
  // that sweep (which would only confirm convergence) is skipped.
  const double stop2 = tol / 64.0;
  const int grp = threadIdx.x / LPP, gl = threadIdx.x % LPP;
  stage8<21>(N * LPAD, threadIdx.x, kJacobiThreads,                    // M(:, col) = R_B(col, :)^T
         [&](int idx) {
           const int col = idx / LPAD, i = idx % LPAD;
           return (col < L && i < L) ? RB[col * ldr + i] : 0.0;
         },
         [&](int idx, double v) { M[(idx / LPAD) * CS + idx % LPAD] = v; });
  for (int idx = threadIdx.x; idx < RN * kJacobiGroups; idx += kJacobiThreads) {
    int p, q;
    jacobi_pair(N, idx / kJacobiGroups, idx % kJacobiGroups, p, q);
    pairs[2 * idx] = (uint8_t)p;
    pairs[2 * idx + 1] = (uint8_t)q;
  }
  __syncthreads();
  int sweep = 0;
  for (; sweep < JSWEEPS && N > 1; ++sweep) {
    // squared column norms, recomputed each sweep and carried through its rotations by
    // a' = a - t g, b' = b + t g (exact for the rotation that zeroes g)
    for (int col = grp; col < N; col += kJacobiGroups) {
      const double* mc = M + col * CS + gl;
      double s0 = 0, s1 = 0;
#pragma unroll
      for (int e = 0; e < EPL; e += 2) {
        s0 = fma(mc[LPP * e], mc[LPP * e], s0);
        if (e + 1 < EPL) s1 = fma(mc[LPP * (e + 1)], mc[LPP * (e + 1)], s1);
      }
      double v = s0 + s1;
      v += dpp::mov<dpp::kXor1>(v);
      v += dpp::mov<dpp::kXor2>(v);
      v += dpp::mov<dpp::kHalfMirror>(v);
      if (gl == 0) nrm2[col] = v;
    }
    if (threadIdx.x == 0) { rotated = 0; large = 0; }
    __syncthreads();
    int p = pairs[2 * grp], q = pairs[2 * grp + 1];
    int held = -1;                       // the home column held in xp (-1: none)
    bool dirty = false;                  // xp rotated since it was loaded
    double xp[EPL];
#pragma unroll
    for (int e = 0; e < EPL; ++e) xp[e] = 0.0;
    for (int r = 0; r < RN; ++r) {
      // the next round's pair (the table never changes), fetched behind this round's loads
      int pn = 255, qn = 255;
      if (r + 1 < RN) {
        const int pi = 2 * ((r + 1) * kJacobiGroups + grp);
        pn = pairs[pi]; qn = pairs[pi + 1];
      }
      if (p != 255) {
        if (p != held) {
#pragma unroll
          for (int e = 0; e < EPL; ++e) xp[e] = M[p * CS + gl + LPP * e];
          held = p;
          dirty = false;
        }
        double* mq = M + q * CS + gl;
        double xq[EPL];
#pragma unroll
        for (int e = 0; e < EPL; ++e) xq[e] = mq[LPP * e];
        const double a = nrm2[p], bb = nrm2[q];
        double g0 = 0, g1 = 0;
#pragma unroll
        for (int e = 0; e < EPL; e += 2) {
          g0 = fma(xp[e], xq[e], g0);
          if (e + 1 < EPL) g1 = fma(xp[e + 1], xq[e + 1], g1);
        }
        double g = g0 + g1;
        g += dpp::mov<dpp::kXor1>(g);
        g += dpp::mov<dpp::kXor2>(g);
        g += dpp::mov<dpp::kHalfMirror>(g);
        // rotate unless the pair is orthogonal to working precision (L eps relative)
        if ((g != 0.0) && (g * g > tol2 * (a * bb))) {
          // zeta = (bb - a) / 2g, t = sign(zeta) / (|zeta| + sqrt(1 + zeta^2)): the angle from
          // one-step refined estimates; c = 1/sqrt(1+t^2) to full precision and s = c t, so
          // c^2 + s^2 = 1 to working precision whatever the accuracy of t
          const double zeta = fmin(fmax((bb - a) * rcp_nr1(2.0 * g), -1e150), 1e150);
          const double z2 = fma(zeta, zeta, 1.0);
          const double t = copysign(1.0, zeta) * rcp_nr1(fma(z2, rsq_nr1(z2), fabs(zeta)));
          const double c = rsq_nr(fma(t, t, 1.0));
          const double s = c * t;
#pragma unroll
          for (int e = 0; e < EPL; ++e) {
            const double np = c * xp[e] - s * xq[e];
            mq[LPP * e] = s * xp[e] + c * xq[e];
            xp[e] = np;
          }
          dirty = true;
          if (gl == 0) {
            nrm2[p] = fmax(fma(-t, g, a), 0.0);
            nrm2[q] = fma(t, g, bb);
            rotated = 1;
            if (g * g > stop2 * (a * bb)) large = 1;
          }
        }
      }
      // the home goes back to LDS when the next round gives the group another one (and after
      // the last round, so that the sweep ends with every column in LDS)
      if (held >= 0 && pn != held) {
        if (dirty) {
#pragma unroll
          for (int e = 0; e < EPL; ++e) M[held * CS + gl + LPP * e] = xp[e];
        }
        held = -1;
        dirty = false;
      }
      p = pn; q = qn;
      __syncthreads();
    }
    if (!rotated || !large) { ++sweep; break; }
    __syncthreads();
  }
  if (threadIdx.x == 0) info[0] = sweep;
  for (int col = threadIdx.x; col < L; col += kJacobiThreads) {
    double s = 0;
    for (int i = 0; i < L; ++i) s = fma(M[col * CS + i], M[col * CS + i], s);
    nrm[col] = sqrt(s);
  }
  __syncthreads();
  // descending order with ties by index; a NaN norm (a non-finite R_B) ranks below every number,
  // so the ranks stay a permutation whatever the input
  for (int col = threadIdx.x; col < L; col += kJacobiThreads) {
    const double kc = (nrm[col] == nrm[col]) ? nrm[col] : -1.0;
    int rank = 0;
    for (int o = 0; o < L; ++o) {
      const double ko = (nrm[o] == nrm[o]) ? nrm[o] : -1.0;
      rank += (ko > kc) || (ko == kc && o < col);
    }
    sig[rank] = nrm[col];
    perm[rank] = col;
  }
  for (int idx = threadIdx.x; idx < L * L; idx += kJacobiThreads) {
    const int col = idx / L, i = idx % L;
    W[i * ldw + col] = M[col * CS + i];   // W row-major L x L
  }
}

// EPL (rows per lane) for L: the smallest built one with kJacobiLpp EPL >= L.
inline int jacobi_epl(int L) {
  const int need = cdiv(L, kJacobiLpp);
#define SK_EPL_PICK(E) if (need <= (E)) return (E);
  SK_JACOBI_EPLS(SK_EPL_PICK)
#undef SK_EPL_PICK
  return 16;
}
size_t jacobi_lds_bytes(int L) {
  const int N = (L + 1) & ~1, CS = jacobi_cs(kJacobiLpp * jacobi_epl(L));
  return (size_t)N * CS * sizeof(double) + (size_t)jacobi_rounds(N) * kJacobiGroups * 2 + 16;
}

// Gather the k leading factors: Wk = W(:, perm[0:kk]) / sig (U = Q Wk) and
// Wv = W(:, perm[0:kk]) / sig^2 (V = B^T Wv); the first workgroup also writes S (k values, zero
// past kk).
__global__ void k_gather(const double* __restrict__ W, int ld, int L, const int* __restrict__ perm,
                         const double* __restrict__ sig, int kk, double* __restrict__ Wv,
                         double* __restrict__ Wk, int k, double* __restrict__ S) {
  if (blockIdx.x == 0)
    for (int j = threadIdx.x; j < k; j += blockDim.x) S[j] = (j < kk) ? sig[j] : 0.0;
  for (int idx = blockIdx.x * blockDim.x + threadIdx.x; idx < L * kk; idx += gridDim.x * blockDim.x) {
    const int i = idx / kk, j = idx % kk;
    const int pc = perm[j];
    const int col = pc < 0 ? 0 : (pc >= L ? L - 1 : pc);
    const double sj = sig[j];
    Wk[idx] = sj > 0.0 ? W[i * ld + col] / sj : 0.0;
    Wv[idx] = sj > 0.0 ? W[i * ld + col] / (sj * sj) : 0.0;
  }
}

// Sign of each column j < kk of V (column-major, ld): + if its largest-magnitude entry (lowest
// index on ties) is positive.  One workgroup per column.
__global__ __launch_bounds__(TPB) void k_signs(const double* __restrict__ V, int64_t ldv,
                                               int64_t n, double* __restrict__ sgn) {
  __shared__ double bv[TPB];
  __shared__ int64_t bi[TPB];
  const int j = blockIdx.x;
  double best = -1.0;
  int64_t bidx = 0;
  // eight loads in flight per batch (at clamped addresses; rows past n are not compared), then
  // the comparisons in row order, so ties keep the first index as before
  for (int64_t r0 = threadIdx.x; r0 < n; r0 += 8 * TPB) {
    double a[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int64_t r = r0 + (int64_t)u * TPB;
      a[u] = fabs(V[j * ldv + (r < n ? r : n - 1)]);
    }
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int64_t r = r0 + (int64_t)u * TPB;
      if (r < n && a[u] > best) { best = a[u]; bidx = r; }
    }
  }
  bv[threadIdx.x] = best;
  bi[threadIdx.x] = bidx;
  __syncthreads();
  for (int o = TPB / 2; o > 0; o >>= 1) {
    if (threadIdx.x < o) {
      const double a = bv[threadIdx.x + o];
      const int64_t ia = bi[threadIdx.x + o];
      if (a > bv[threadIdx.x] || (a == bv[threadIdx.x] && ia < bi[threadIdx.x])) {
        bv[threadIdx.x] = a;
        bi[threadIdx.x] = ia;
      }
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) sgn[j] = (V[j * ldv + bi[0]] < 0.0) ? -1.0 : 1.0;
}

// out = sign_j * (X Wk)(r, j) for j < kk, 0 for kk <= j < k; row-major (out[r*ld + j]) or, with
// colmajor, out[j*ld + r].  sgn may be null (all +1).  Grid: x = row blocks, y = 16-column slabs.
__global__ __launch_bounds__(TPB) void k_write_rows(const double* __restrict__ X, int64_t ldx,
                                                    int L, const double* __restrict__ Wk, int kk,
                                                    int k, const double* __restrict__ sgn,
                                                    int64_t rows, double* __restrict__ out,
                                                    int64_t ld, int colmajor) {
  extern __shared__ double ws[];
  const int j0 = blockIdx.y * 16;
  stage8(L * 16, threadIdx.x, TPB,
         [&](int idx) {
           const int a = idx / 16, j = idx % 16;
           return (j0 + j < kk) ? Wk[a * kk + j0 + j] : 0.0;
         },
         [&](int idx, double v) { ws[idx] = v; });
  __syncthreads();
  for (int64_t r = blockIdx.x * (int64_t)TPB + threadIdx.x; r < rows;
       r += (int64_t)gridDim.x * TPB) {
    double acc[16];
#pragma unroll
    for (int j = 0; j < 16; ++j) acc[j] = 0.0;
    int a = 0;
    for (; a + 16 <= L; a += 16) {            // sixteen loads in flight per batch
      double x[16];
#pragma unroll
      for (int u = 0; u < 16; ++u) x[u] = X[(a + u) * ldx + r];
#pragma unroll
      for (int u = 0; u < 16; ++u)
#pragma unroll
        for (int j = 0; j < 16; ++j) acc[j] = fma(x[u], ws[(a + u) * 16 + j], acc[j]);
    }
    for (; a < L; ++a) {
      const double x = X[a * ldx + r];
#pragma unroll
      for (int j = 0; j < 16; ++j) acc[j] = fma(x, ws[a * 16 + j], acc[j]);
    }
#pragma unroll
    for (int j = 0; j < 16; ++j) {
      if (j0 + j < k) {
        const double v = (j0 + j < kk) ? (sgn ? sgn[j0 + j] : 1.0) * acc[j] : 0.0;
        if (colmajor) out[(int64_t)(j0 + j) * ld + r] = v;
        else out[r * ld + j0 + j] = v;
      }
    }
  }
}

// out (row-major rows x k, ld) = sign_j * Vt(:, j) (column-major, ldv) for j < kk, 0 beyond.
__global__ void k_signed_transpose(const double* __restrict__ Vt, int64_t ldv, int kk, int k,
                                   const double* __restrict__ sgn, int64_t rows,
                                   double* __restrict__ out, int64_t ld) {
  for (int64_t q = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; q < rows * k;
       q += (int64_t)gridDim.x * blockDim.x) {
    const int64_t r = q / k;
    const int j = (int)(q - r * k);
    out[r * ld + j] = (j < kk) ? sgn[j] * Vt[(int64_t)j * ldv + r] : 0.0;
  }
}

__global__ void k_init_ctrl(Ctrl* ctrl, int t, int l, int* zero0, int* zero1) {
  if (threadIdx.x == 0) {
    if (zero0 != nullptr) *zero0 = 0;
    if (zero1 != nullptr) *zero1 = 0;
    const int nf = ctrl->nonfinite;
    ctrl->r0 = 0.0;
    ctrl->last_iter = t - 1;
    ctrl->keep_last = 0;
    ctrl->l_eff = l;
    ctrl->nonfinite = nf;
    ctrl->pad[0] = 0;          // set by a Cholesky QR step that cannot be trusted
  }
}

// ------------------------------------------------------------------------------------------------
// Host orchestration.
struct Ctx {
  hipStream_t s;
  hipError_t err = hipSuccess;
  bool ok() const { return err == hipSuccess; }
  void chk() { if (err == hipSuccess) err = hipGetLastError(); }
};

// Row reductions: chunks of a multiple of 16 rows, at most kTnChunks of them (enough workgroups
// to fill the chip; the partials stay small next to the rows read).
constexpr int kTnChunks = 512;
constexpr int kGramWgs = 256;   // workgroups of one l x l Gram matrix launch

inline int tn_rows_per_chunk(int64_t rows) {
  const int64_t r = rup<int64_t>(cdiv<int64_t>(rows, kTnChunks), 16);
  return (int)(r < 64 ? 64 : r);
}

template <int MT>
void tn_launch(Ctx& cx, int nq, dim3 grid, const double* X, int64_t ldx, const double* Y,
               int64_t ldy, int p, int q, int64_t rows, int rch, double* part, const Ctrl* ctrl,
               int iter, int qtot = 0) {
  if (nq == 1)
    hipLaunchKernelGGL((k_tn_mfma<MT, 1>), grid, dim3(TPB), 0, cx.s, X, ldx, Y, ldy, p, q, rows,
                       rch, part, ctrl, iter, qtot);
  else
    hipLaunchKernelGGL((k_tn_mfma<MT, 2>), grid, dim3(TPB), 0, cx.s, X, ldx, Y, ldy, p, q, rows,
                       rch, part, ctrl, iter, qtot);
}

// Chunk partials of X[:, 0:p]^T Y[:, 0:q] over `rows` rows (p <= 128, q <= 32) into `part`;
// returns the number of chunks.
int tn_partials(Ctx& cx, const double* X, int64_t ldx, const double* Y, int64_t ldy, int p, int q,
                int64_t rows, double* part, const Ctrl* ctrl, int iter) {
  if (!cx.ok() || p == 0 || q == 0) return 0;
  const int rch = tn_rows_per_chunk(rows);
  const int nch = (int)cdiv<int64_t>(rows, rch);
  const int mt = cdiv(p, 16), nq = cdiv(q, 16);
  const dim3 grid(nch);
  switch (mt) {
    case 1: tn_launch<1>(cx, nq, grid, X, ldx, Y, ldy, p, q, rows, rch, part, ctrl, iter); break;
    case 2: tn_launch<2>(cx, nq, grid, X, ldx, Y, ldy, p, q, rows, rch, part, ctrl, iter); break;
    case 3: tn_launch<3>(cx, nq, grid, X, ldx, Y, ldy, p, q, rows, rch, part, ctrl, iter); break;
    case 4: tn_launch<4>(cx, nq, grid, X, ldx, Y, ldy, p, q, rows, rch, part, ctrl, iter); break;
    case 5: tn_launch<5>(cx, nq, grid, X, ldx, Y, ldy, p, q, rows, rch, part, ctrl, iter); break;
    case 6: tn_launch<6>(cx, nq, grid, X, ldx, Y, ldy, p, q, rows, rch, part, ctrl, iter); break;
    case 7: tn_launch<7>(cx, nq, grid, X, ldx, Y, ldy, p, q, rows, rch, part, ctrl, iter); break;
    default: tn_launch<8>(cx, nq, grid, X, ldx, Y, ldy, p, q, rows, rch, part, ctrl, iter); break;
  }
  cx.chk();
  return nch;
}

// Entries e0 .. e0 + ecount - 1 of the p x q product from its chunk partials, into out.
void tn_final(Ctx& cx, const double* part, int nch, int p, int q, int64_t e0, int64_t ecount,
              double* out, int ldo, const Ctrl* ctrl, int iter) {
  if (!cx.ok() || ecount <= 0) return;
  hipLaunchKernelGGL(k_tn_final, dim3((unsigned)cdiv<int64_t>(ecount, 64)), dim3(kTnFinalThreads),
                     0, cx.s, part, nch, (int64_t)p * q, e0, ecount, q, out, ldo, ctrl, iter);
  cx.chk();
}

// out (p x q row-major, ldo) = X[:, 0:p]^T Y[:, 0:q] over `rows` rows (p <= 128, q <= 32).
void tn(Ctx& cx, const double* X, int64_t ldx, const double* Y, int64_t ldy, int p, int q,
        int64_t rows, double* part, double* out, int ldo, const Ctrl* ctrl, int iter) {
  const int nch = tn_partials(cx, X, ldx, Y, ldy, p, q, rows, part, ctrl, iter);
  if (nch > 0) tn_final(cx, part, nch, p, q, 0, (int64_t)p * q, out, ldo, ctrl, iter);
}

template <typename BT>
void nn(Ctx& cx, double* out, int64_t ldo, const BT* base, int64_t ldb, const double* X,
        int64_t ldx, int p, const double* W, int ldw, int q, int64_t rows, double alpha,
        const Ctrl* ctrl, int iter, const double* Rs = nullptr) {
  if (!cx.ok() || q == 0 || rows == 0) return;
  const dim3 g((unsigned)cdiv<int64_t>(rows, kNnThreads)), blk(kNnThreads);
#define SK_NN_LAUNCH(QM)                                                                        \
  hipLaunchKernelGGL((k_nn_update<BT, QM>), g, blk, 0, cx.s, out, ldo, base, ldb, X, ldx, p, W, \
                     ldw, q, rows, alpha, ctrl, iter, Rs, 0)
  if (q <= 8) SK_NN_LAUNCH(8);
  else if (q <= 10) SK_NN_LAUNCH(10);
  else if (q <= 12) SK_NN_LAUNCH(12);
  else if (q <= 16) SK_NN_LAUNCH(16);
  else SK_NN_LAUNCH(32);
#undef SK_NN_LAUNCH
  cx.chk();
}

struct Level {
  double* X; int64_t ld; int64_t rows; int nch; int CR; double* tau;
};

template <int BMAX, int RPT>
void tsqr_t(Ctx& cx, double* X, int64_t ldx, int64_t rows, int b, double* ws, double* Rout,
            const Ctrl* ctrl, int iter) {
  constexpr int CR0 = TPB * RPT;
  Level lv[16];
  int L = 0;
  double* cur = ws;
  lv[0] = {X, ldx, rows, 0, 0, nullptr};
  for (;;) {
    Level& v = lv[L];
    v.nch = (int)cdiv<int64_t>(v.rows, CR0);
    v.CR = (int)cdiv<int64_t>(v.rows, v.nch);
    v.tau = cur;
    cur += rup<int64_t>((int64_t)v.nch * b, 32);
    // the next level holds the stacked R factors (also used for the root's raw R)
    Level& nx = lv[L + 1];
    nx.rows = (int64_t)v.nch * b;
    nx.ld = nx.rows;
    nx.X = cur;
    cur += rup<int64_t>(nx.rows * b, 32);
    if (v.nch == 1) break;
    ++L;
  }
  // factor levels 0..L; level L is the root (one chunk) and writes its raw R into lv[L+1].X
  for (int k = 0; k <= L && cx.ok(); ++k) {
    hipLaunchKernelGGL((k_house_factor<BMAX, RPT>), dim3(lv[k].nch), dim3(TPB), 0, cx.s, lv[k].X,
                       lv[k].ld, lv[k].rows, b, lv[k].CR, lv[k].tau, lv[k + 1].X, lv[k + 1].ld,
                       ctrl, iter);
    cx.chk();
  }
  // form Q from the root down
  for (int k = L; k >= 0 && cx.ok(); --k) {
    const bool root = (k == L);
    hipLaunchKernelGGL((k_house_form<BMAX, RPT>), dim3(lv[k].nch), dim3(TPB), 0, cx.s, lv[k].X,
                       lv[k].ld, lv[k].rows, b, lv[k].CR, lv[k].tau,
                       root ? (const double*)nullptr : lv[k + 1].X, lv[k + 1].ld, lv[L + 1].X,
                       lv[L + 1].ld, root ? Rout : (double*)nullptr, ctrl, iter);
    cx.chk();
  }
}

void tsqr(Ctx& cx, double* X, int64_t ldx, int64_t rows, int b, double* ws, double* Rout,
          const Ctrl* ctrl, int iter) {
  if (!cx.ok()) return;
  // exact widths for the common b; others run in the next wider instantiation with zero padding
  if (b <= 1) tsqr_t<1, 4>(cx, X, ldx, rows, b, ws, Rout, ctrl, iter);
  else if (b <= 2) tsqr_t<2, 4>(cx, X, ldx, rows, b, ws, Rout, ctrl, iter);
  else if (b <= 4) tsqr_t<4, 4>(cx, X, ldx, rows, b, ws, Rout, ctrl, iter);
  else if (b <= 5) tsqr_t<5, 4>(cx, X, ldx, rows, b, ws, Rout, ctrl, iter);
  else if (b <= 8) tsqr_t<8, 4>(cx, X, ldx, rows, b, ws, Rout, ctrl, iter);
  else if (b <= 10) tsqr_t<10, 4>(cx, X, ldx, rows, b, ws, Rout, ctrl, iter);
  else if (b <= 16) tsqr_t<16, 4>(cx, X, ldx, rows, b, ws, Rout, ctrl, iter);
  else if (b <= 20) tsqr_t<20, 2>(cx, X, ldx, rows, b, ws, Rout, ctrl, iter);
  else tsqr_t<32, 2>(cx, X, ldx, rows, b, ws, Rout, ctrl, iter);
}

// Small-buffer layout (doubles), see finalize_small_elems.
struct Small {
  double *W, *T, *C, *Wn, *R1, *R2, *R, *X, *RB, *C1, *C2, *Jm, *Wm, *sig, *Jk, *Wk, *sgn;
  double *sG, *wc;   // centring: s_G = G^T 1 and w = Omega'^T mu
  double *Rg, *Rgi;  // one column block: R of G and its inverse
  int* perm; int* info;
};
// Flags in sm.info: [0] Jacobi sweeps, [1] and [2] the R_B Cholesky QR2 tests, [kObFail] and
// [kObIll] the one-block Cholesky QR2 tests.
constexpr int kObFail = 4, kObIll = 5;

Small carve_small(double* base, int l, int b) {
  const int P = l * 32;   // p x b blocks with p <= l, b <= 32
  Small sm;
  double* c = base;
  auto take = [&](int64_t cnt) { double* r = c; c += rup<int64_t>(cnt, 32); return r; };
  sm.W = take(P); sm.T = take(P); sm.C = take(P); sm.Wn = take(P);
  sm.R1 = take(32 * 32); sm.R2 = take(32 * 32); sm.R = take(32 * 32); sm.X = take(32 * 32);
  sm.RB = take((int64_t)l * l); sm.C1 = take(P); sm.C2 = take(P);
  sm.Jm = take((int64_t)l * l + l); sm.Wm = take((int64_t)l * l); sm.sig = take(l);
  sm.Jk = take((int64_t)l * l); sm.Wk = take((int64_t)l * l); sm.sgn = take(l);
  sm.perm = reinterpret_cast<int*>(take(l));
  sm.info = reinterpret_cast<int*>(take(4));
  sm.sG = take(l); sm.wc = take(l);
  sm.Rg = take((int64_t)l * l); sm.Rgi = take((int64_t)l * l);
  return sm;
}

// One Cholesky QR step of the column block Y (rows x b, in place): the Gram matrix from the row
// reduction's chunk partials (entries e0 .. e0 + b^2 - 1, chunk stride pq) and its factor in one
// workgroup (k_gram_chol), then Y <- Y R^-1 (k_cholqr_apply).
void cholqr(Ctx& cx, double* Y, int64_t ldy, int64_t rows, const double* part, int nch,
            int64_t pq, int64_t e0, int b, const double* Rprev, double* Rout, bool last,
            const Small& sm, int p, Ctrl* ctrl, int iter) {
  if (!cx.ok()) return;
  const dim3 g1(1), b1(kGramThreads);
  const dim3 g((unsigned)cdiv<int64_t>(rows, kApplyThreads)), blk(kApplyThreads);
  const int lf = last ? 1 : 0;
  if (b <= 8) {
    hipLaunchKernelGGL(k_gram_chol<8>, g1, b1, 0, cx.s, part, nch, pq, e0, b, Rprev, Rout, sm.X,
                       lf, sm.T, sm.W, sm.Wn, p, ctrl, iter);
    cx.chk();
    if (cx.ok())
      hipLaunchKernelGGL(k_cholqr_apply<8>, g, blk, 0, cx.s, Y, ldy, rows, sm.X, b, lf, ctrl, iter);
  } else if (b <= 16) {
    hipLaunchKernelGGL(k_gram_chol<16>, g1, b1, 0, cx.s, part, nch, pq, e0, b, Rprev, Rout, sm.X,
                       lf, sm.T, sm.W, sm.Wn, p, ctrl, iter);
    cx.chk();
    if (cx.ok())
      hipLaunchKernelGGL(k_cholqr_apply<16>, g, blk, 0, cx.s, Y, ldy, rows, sm.X, b, lf, ctrl, iter);
  } else {
    hipLaunchKernelGGL(k_gram_chol<32>, g1, b1, 0, cx.s, part, nch, pq, e0, b, Rprev, Rout, sm.X,
                       lf, sm.T, sm.W, sm.Wn, p, ctrl, iter);
    cx.chk();
    if (cx.ok())
      hipLaunchKernelGGL(k_cholqr_apply<32>, g, blk, 0, cx.s, Y, ldy, rows, sm.X, b, lf, ctrl, iter);
  }
  cx.chk();
}

// Blocks of at most this many columns take the per-lane factorisation (k_cholqr_lane).
constexpr int kLaneCholMax = 12;

// One Cholesky QR step of a narrow column block (b <= kLaneCholMax) from its Gram matrix G.
void cholqr_lane(Ctx& cx, double* Y, int64_t ldy, int64_t rows, const double* G, int b,
                 const double* Rprev, double* Rout, bool last, const Small& sm, int p, Ctrl* ctrl,
                 int iter) {
  if (!cx.ok()) return;
  const dim3 g((unsigned)cdiv<int64_t>(rows, kLaneCholThreads)), blk(kLaneCholThreads);
  const int lf = last ? 1 : 0;
  if (b <= 4)
    hipLaunchKernelGGL(k_cholqr_lane<4>, g, blk, 0, cx.s, Y, ldy, rows, G, b, Rprev, Rout, lf, sm.T,
                       sm.W, sm.Wn, p, ctrl, iter);
  else if (b <= 8)
    hipLaunchKernelGGL(k_cholqr_lane<8>, g, blk, 0, cx.s, Y, ldy, rows, G, b, Rprev, Rout, lf, sm.T,
                       sm.W, sm.Wn, p, ctrl, iter);
  else if (b <= 10)
    hipLaunchKernelGGL(k_cholqr_lane<10>, g, blk, 0, cx.s, Y, ldy, rows, G, b, Rprev, Rout, lf,
                       sm.T, sm.W, sm.Wn, p, ctrl, iter);
  else
    hipLaunchKernelGGL(k_cholqr_lane<12>, g, blk, 0, cx.s, Y, ldy, rows, G, b, Rprev, Rout, lf,
                       sm.T, sm.W, sm.Wn, p, ctrl, iter);
  cx.chk();
}

// Gram matrix X^T X (L x L, upper triangle, row-major, leading dimension L) of the n x L
// column-major X, in column slices of at most 32.
template <typename XT>
void gram_upper(Ctx& cx, const XT* X, int64_t ldx, int64_t rows, int L, double* red_ws,
                double* Gm) {
  if (!cx.ok() || L <= 0) return;
  // about one workgroup per CU over all slices: a workgroup's share of the matrix-core work then
  // outweighs its partial sums and their reduction, and the partials stay small
  const int ny = cdiv(L, 32), mt = cdiv(L, 16);
  const int64_t want = std::max<int64_t>(1, kGramWgs / ny);
  // (chunks of at least 64 rows and at most kTnChunks of them, as the workspace is sized for)
  const int rch = (int)std::max<int64_t>(
      tn_rows_per_chunk(rows), rup<int64_t>(cdiv<int64_t>(rows, want), 16));
  const int nch = (int)cdiv<int64_t>(rows, rch);
  const dim3 grid(nch, ny);
  // one read of X for the whole upper triangle (l <= 112); the slice launch otherwise
  const int nch1 = (int)cdiv<int64_t>(rows, std::max<int64_t>(tn_rows_per_chunk(rows),
                                                              rup<int64_t>(cdiv<int64_t>(rows, kGramWgs), 16)));
  const int rch1 = (int)std::max<int64_t>(tn_rows_per_chunk(rows),
                                          rup<int64_t>(cdiv<int64_t>(rows, kGramWgs), 16));
  if (mt <= 7) {
    const dim3 g1(nch1);
    switch (mt) {
      case 1: hipLaunchKernelGGL((k_gram_mfma<XT, 1>), g1, dim3(kGramMfmaThreads), 0, cx.s, X, ldx, L, rows, rch1, red_ws); break;
      case 2: hipLaunchKernelGGL((k_gram_mfma<XT, 2>), g1, dim3(kGramMfmaThreads), 0, cx.s, X, ldx, L, rows, rch1, red_ws); break;
      case 3: hipLaunchKernelGGL((k_gram_mfma<XT, 3>), g1, dim3(kGramMfmaThreads), 0, cx.s, X, ldx, L, rows, rch1, red_ws); break;
      case 4: hipLaunchKernelGGL((k_gram_mfma<XT, 4>), g1, dim3(kGramMfmaThreads), 0, cx.s, X, ldx, L, rows, rch1, red_ws); break;
      case 5: hipLaunchKernelGGL((k_gram_mfma<XT, 5>), g1, dim3(kGramMfmaThreads), 0, cx.s, X, ldx, L, rows, rch1, red_ws); break;
      case 6: hipLaunchKernelGGL((k_gram_mfma<XT, 6>), g1, dim3(kGramMfmaThreads), 0, cx.s, X, ldx, L, rows, rch1, red_ws); break;
      default: hipLaunchKernelGGL((k_gram_mfma<XT, 7>), g1, dim3(kGramMfmaThreads), 0, cx.s, X, ldx, L, rows, rch1, red_ws); break;
    }
    cx.chk();
    if (!cx.ok()) return;
    hipLaunchKernelGGL(k_tn_final_gram, dim3((unsigned)cdiv<int64_t>((int64_t)ny * L * 32, 64)),
                       dim3(kTnFinalThreads), 0, cx.s, red_ws, nch1, L, ny, Gm, L);
    cx.chk();
    return;
  }
  if constexpr (!std::is_same<XT, double>::value) {
    cx.err = hipErrorInvalidValue;             // FP32 columns are read directly only for l <= 112
    return;
  } else {
  switch (mt) {
    case 1: tn_launch<1>(cx, 2, grid, X, ldx, X, ldx, L, 32, rows, rch, red_ws, nullptr, 0, L); break;
    case 2: tn_launch<2>(cx, 2, grid, X, ldx, X, ldx, L, 32, rows, rch, red_ws, nullptr, 0, L); break;
    case 3: tn_launch<3>(cx, 2, grid, X, ldx, X, ldx, L, 32, rows, rch, red_ws, nullptr, 0, L); break;
    case 4: tn_launch<4>(cx, 2, grid, X, ldx, X, ldx, L, 32, rows, rch, red_ws, nullptr, 0, L); break;
    case 5: tn_launch<5>(cx, 2, grid, X, ldx, X, ldx, L, 32, rows, rch, red_ws, nullptr, 0, L); break;
    case 6: tn_launch<6>(cx, 2, grid, X, ldx, X, ldx, L, 32, rows, rch, red_ws, nullptr, 0, L); break;
    case 7: tn_launch<7>(cx, 2, grid, X, ldx, X, ldx, L, 32, rows, rch, red_ws, nullptr, 0, L); break;
    default: tn_launch<8>(cx, 2, grid, X, ldx, X, ldx, L, 32, rows, rch, red_ws, nullptr, 0, L); break;
  }
  cx.chk();
  if (!cx.ok()) return;
  hipLaunchKernelGGL(k_tn_final_gram, dim3((unsigned)cdiv<int64_t>((int64_t)ny * L * 32, 64)),
                     dim3(kTnFinalThreads), 0, cx.s, red_ws, nch, L, ny, Gm, L);
  cx.chk();
  }
}

// Y = X R^-1 for the n x L column-major X and upper triangular R^-1 (row-major, leading dimension
// L), in column slices of at most 16 (slice c0..c0+w-1 only needs rows 0..c0+w-1 of R^-1).
template <typename XT>
void right_trmul(Ctx& cx, double* Y, int64_t ldy, const XT* X, int64_t ldx, int64_t rows,
                 int L, const double* Rinv, int ldr = 0) {
  if (!cx.ok() || L <= 0 || rows <= 0) return;
  const int mt = cdiv(L, 16);
  if (mt <= 7 && (const void*)Y != (const void*)X) {
    // one read of X on the matrix cores, one workgroup per CU (W takes most of the LDS)
    const int rch = (int)std::max<int64_t>(64, rup<int64_t>(cdiv<int64_t>(rows, 256), 16));
    const dim3 g1((unsigned)cdiv<int64_t>(rows, rch));
    const int lw = ldr > 0 ? ldr : L;
    switch (mt) {
#define SK_RMUL(M)                                                                                \
      case M:                                                                                     \
        hipLaunchKernelGGL((k_rmul_mfma<XT, M>), g1, dim3(kRmulThreads), rmul_lds_bytes(M), cx.s, Y, ldy, X, ldx, \
                           rows, L, Rinv, lw, rch);                                               \
        break;
      SK_RMUL(1) SK_RMUL(2) SK_RMUL(3) SK_RMUL(4) SK_RMUL(5) SK_RMUL(6) SK_RMUL(7)
#undef SK_RMUL
      default: break;
    }
    cx.chk();
    return;
  }
  if constexpr (!std::is_same<XT, double>::value) {
    cx.err = hipErrorInvalidValue;             // FP32 columns are read directly only for l <= 112
    return;
  } else {
  const int ny = cdiv(L, 16);
  const dim3 g((unsigned)cdiv<int64_t>(rows, kNnThreads), ny), blk(kNnThreads);
  hipLaunchKernelGGL((k_nn_update<double, 16>), g, blk, 0, cx.s, Y, ldy, (const double*)nullptr,
                     0, X, ldx, L, Rinv, ldr > 0 ? ldr : L, 16, rows, 1.0, (const Ctrl*)nullptr,
                     0, (const double*)nullptr, L);
  cx.chk();
  }
}

void chol(Ctx& cx, const double* Gm, int L, double shift_rel, double* R, double* Rinv, int* fail,
          double ill_rel = 0.0, double dev_rel = 0.0, int* ill = nullptr, int force_fail = 0) {
  if (!cx.ok()) return;
  hipLaunchKernelGGL(k_chol_blk, dim3(1), dim3(kCholBlkThreads), cholb_lds_bytes(L), cx.s, Gm, L,
                     L, shift_rel, R, Rinv, L, fail, ill_rel, dev_rel, ill, force_fail);
  cx.chk();
}

// R_B of B^T = Q_B R_B by Cholesky QR: two unshifted passes when B is well enough conditioned for
// them (tested on the device, read back with the one wait this needs), else shifted Cholesky QR3
// (see the shifted Cholesky QR3 note above k_chol_blk).  Returns the device matrix holding R_B (row-major L x L), or nullptr when a pivot
// failed (then the caller factors B^T another way).  Q1 goes to the Q_B storage and Q2 to the H
// storage (H is no longer needed at this point).
const double* chol_qr3_shifted(Ctx& cx, const FinalizeArgs& f, const Small& sm, int L);

void chol_qr2(Ctx& cx, const FinalizeArgs& f, const Small& sm, int L, int force_fail) {
  const int64_t n = f.n;
  double* Gm = sm.Jm;
  double* Rs = sm.Wm;
  double* Ri = sm.Jk;
  double* Racc = sm.Wk;
  int* fail = sm.info + 1;
  int* ill = sm.info + 2;
  // Cholesky QR2 without a shift: accurate when no pivot of B B^T falls below 1e-8 of its
  // diagonal entry (cond(B) up to about 1e4) and the second factor is within 1e-6 of I (Q1 was
  // orthonormal to about 1e-6, so Q2 is to working precision).  R_B goes to sm.RB; the two tests
  // leave nonzero flags at sm.info[1] (a pivot failed) and sm.info[2] (a test failed), which the
  // caller reads later.  force_fail (a test hook) makes the first factorisation take its
  // failed-pivot exit at the first step.
  hipLaunchKernelGGL(k_set_int2, dim3(1), dim3(64), 0, cx.s, fail, ill, 0);
  cx.chk();
  gram_upper(cx, f.Bt, f.ldb, n, L, f.red_ws, Gm);
  chol(cx, Gm, L, 0.0, Racc, Ri, fail, 1e-8, 0.0, ill, force_fail);
  right_trmul(cx, f.Qb, f.ldb, f.Bt, f.ldb, n, L, Ri);
  gram_upper(cx, f.Qb, f.ldb, n, L, f.red_ws, Gm);
  chol(cx, Gm, L, 0.0, Rs, nullptr, fail, 0.0, 1e-6, ill);
  if (!cx.ok()) return;
  hipLaunchKernelGGL(k_trmm_upper, dim3(L), dim3(JMAX), 0, cx.s, Rs, Racc, sm.RB, L);
  cx.chk();
}

// Shifted Cholesky QR3 of B^T (see k_chol_blk); R_B as chol_qr, or nullptr when a pivot failed.
const double* chol_qr3_shifted(Ctx& cx, const FinalizeArgs& f, const Small& sm, int L) {
  const int64_t n = f.n;
  double* Gm = sm.Jm;
  double* Rs = sm.Wm;
  double* Ri = sm.Jk;
  double* Racc = sm.Wk;
  double* Q2 = const_cast<double*>(f.H);
  int* fail = sm.info + 1;
  const double u = 1.1102230246251565e-16;     // 2^-53
  const double shift_rel = 11.0 * ((double)n * L + (double)L * (L + 1)) * u;
  // shifted Cholesky QR3
  hipLaunchKernelGGL(k_set_int, dim3(1), dim3(64), 0, cx.s, fail, 0);
  cx.chk();
  // pass 1: B^T = Q1 R1 (shifted)
  gram_upper(cx, f.Bt, f.ldb, n, L, f.red_ws, Gm);
  chol(cx, Gm, L, shift_rel, Racc, Ri, fail);
  right_trmul(cx, f.Qb, f.ldb, f.Bt, f.ldb, n, L, Ri);
  // pass 2: Q1 = Q2 R2
  gram_upper(cx, f.Qb, f.ldb, n, L, f.red_ws, Gm);
  chol(cx, Gm, L, 0.0, Rs, Ri, fail);
  right_trmul(cx, Q2, f.ldh, f.Qb, f.ldb, n, L, Ri);
  if (!cx.ok()) return nullptr;
  hipLaunchKernelGGL(k_trmm_upper, dim3(L), dim3(JMAX), 0, cx.s, Rs, Racc, sm.RB, L);
  cx.chk();
  // pass 3: Q2 = Q3 R3; R_B = R3 R2 R1
  gram_upper(cx, Q2, f.ldh, n, L, f.red_ws, Gm);
  chol(cx, Gm, L, 0.0, Rs, nullptr, fail);
  if (!cx.ok()) return nullptr;
  hipLaunchKernelGGL(k_trmm_upper, dim3(L), dim3(JMAX), 0, cx.s, Rs, sm.RB, Racc, L);
  cx.chk();
  int hfail = 1;
  if (cx.ok()) cx.err = read_back(&hfail, fail, sizeof(int), cx.s, f.host_pin, f.host_ev);
  if (!cx.ok() || hfail != 0) return nullptr;
  return Racc;
}

}  // namespace

// The pair table of one Jacobi sweep over n columns (n rounded up to even), as k_jacobi builds
// it: rounds x 64 lane groups x {home, visitor}, 255 for an idle group.  Returns the number of
// rounds, or -1 when n is outside 0..JMAX or `cap` bytes cannot hold the table.
int jacobi_schedule(int n, uint8_t* out, int64_t cap) {
  if (n < 0 || n > JMAX) return -1;
  const int N = (n + 1) & ~1, RN = jacobi_rounds(N);
  if (out == nullptr || cap < (int64_t)RN * kJacobiGroups * 2) return -1;
  for (int r = 0; r < RN; ++r)
    for (int k = 0; k < kJacobiGroups; ++k) {
      int p, q;
      jacobi_pair(N, r, k, p, q);
      out[2 * (r * kJacobiGroups + k)] = (uint8_t)p;
      out[2 * (r * kJacobiGroups + k) + 1] = (uint8_t)q;
    }
  return RN;
}

// Raises the dynamic LDS limits of the kernels that need more than the default, once per device
// (the attribute belongs to the device the call runs on), safely from any number of threads.
hipError_t finalize_prepare() {
  static std::mutex mu;
  static bool done[kMaxDevices] = {};
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(mu);
  if (done[dev]) return hipSuccess;
#define SK_EPL_FN(E) (const void*)k_jacobi<E>,
  for (const void* kj : {SK_JACOBI_EPLS(SK_EPL_FN)})
#undef SK_EPL_FN
    if (e == hipSuccess)
      e = hipFuncSetAttribute(kj, hipFuncAttributeMaxDynamicSharedMemorySize, kJacobiLds);
  if (e == hipSuccess)
    e = hipFuncSetAttribute((const void*)k_chol_blk, hipFuncAttributeMaxDynamicSharedMemorySize,
                            (int)cholb_lds_bytes(JMAX));
#define SK_RMUL_ATTR(M)                                                                        \
  if (e == hipSuccess)                                                                         \
    e = hipFuncSetAttribute((const void*)k_rmul_mfma<double, M>,                               \
                            hipFuncAttributeMaxDynamicSharedMemorySize, (int)rmul_lds_bytes(M)); \
  if (e == hipSuccess)                                                                         \
    e = hipFuncSetAttribute((const void*)k_rmul_mfma<float, M>,                                \
                            hipFuncAttributeMaxDynamicSharedMemorySize, (int)rmul_lds_bytes(M));
  SK_RMUL_ATTR(1) SK_RMUL_ATTR(2) SK_RMUL_ATTR(3) SK_RMUL_ATTR(4) SK_RMUL_ATTR(5) SK_RMUL_ATTR(6)
  SK_RMUL_ATTR(7)
#undef SK_RMUL_ATTR
  if (e == hipSuccess) done[dev] = true;
  return e;
}

size_t finalize_small_elems(int l, int b) {
  (void)b;
  const int64_t P = (int64_t)l * 32;
  int64_t e = 6 * rup<int64_t>(P, 32) + 4 * 1024 + 7 * rup<int64_t>((int64_t)l * l + l, 32) +
              5 * rup<int64_t>(l, 32) + 32;
  return (size_t)e + 1024;
}

size_t tsqr_workspace_elems(int64_t rows, int b) {
  const int RPT = 2;   // the smallest rows-per-thread of any instantiation: most chunks
  const int64_t CR0 = TPB * RPT;
  int64_t total = 0, r = rows;
  for (int guard = 0; guard < 16; ++guard) {
    const int64_t nch = cdiv<int64_t>(r, CR0);
    total += rup<int64_t>(nch * b, 32) + rup<int64_t>(nch * b * b, 32);
    if (nch == 1) break;
    r = nch * b;
  }
  return (size_t)total + 64;
}

size_t reduce_workspace_elems(int64_t rows, int p, int q) {
  (void)q;
  // any row count up to `rows` splits into at most this many chunks (chunks hold >= 64 rows); the
  // p x p Gram matrices take cdiv(p, 32) column slices of 32
  const int64_t c64 = cdiv<int64_t>(rows, 64);
  const int64_t nch = c64 < kTnChunks ? c64 : kTnChunks;
  return (size_t)(nch * p * 32 * cdiv(p, 32)) + 64;
}

// ---------------------------------------------------------------- implicit column centring
// PCA of the column-centred A_c = A - 1 mu^T, mu = s_A / m, from the sketch of A (the method
// assumes centred data, Sec. 2.1).  The pass accumulated s_A = A^T 1 as sketch column l of H (its
// operand column of g is all ones); here s_G = G^T 1 and w = Omega'^T mu give
//   G_c = G - 1 w^T,   H_c = H - mu s_G^T
// (the A^T 1 w^T and m mu w^T terms of A_c^T G_c cancel), written over G and H.
template <typename GT>
__global__ __launch_bounds__(TPB) void k_col_sums(const GT* __restrict__ X, int64_t ldx,
                                                  int64_t rows, double* __restrict__ out) {
  __shared__ double red[TPB / 64];
  const int c = blockIdx.x;
  double acc = 0.0;
  for (int64_t r = threadIdx.x; r < rows; r += TPB) acc += (double)X[c * ldx + r];
  acc = wave_sum(acc);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = acc;
  __syncthreads();
  if (threadIdx.x == 0) {
    double t = 0.0;
    for (int w = 0; w < TPB / 64; ++w) t += red[w];
    out[c] = t;
  }
}

// mu = s_A / m from column l of H; w[c] = sum_r Omega'(r, c) mu_r, one workgroup per column
__global__ __launch_bounds__(TPB) void k_centre_w(const double* __restrict__ H, int64_t ldh,
                                                  const double* __restrict__ om, int64_t ldo,
                                                  int64_t n, int l, double inv_m,
                                                  double* __restrict__ mu,
                                                  double* __restrict__ w) {
  __shared__ double red[TPB / 64];
  const int c = blockIdx.x;
  const double* sA = H + (int64_t)l * ldh;
  double acc = 0.0;
  for (int64_t r = threadIdx.x; r < n; r += TPB) {
    const double m_r = sA[r] * inv_m;
    if (c == 0) mu[r] = m_r;
    acc += om[c * ldo + r] * m_r;
  }
  acc = wave_sum(acc);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = acc;
  __syncthreads();
  if (threadIdx.x == 0) {
    double t = 0.0;
    for (int v = 0; v < TPB / 64; ++v) t += red[v];
    w[c] = t;
  }
}

template <typename GT>
__global__ void k_centre_G(GT* __restrict__ G, int64_t ldg, int64_t rows, int l,
                           const double* __restrict__ w) {
  for (int64_t q = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; q < rows * l;
       q += (int64_t)gridDim.x * blockDim.x) {
    const int64_t c = q / rows, r = q - c * rows;
    G[c * ldg + r] = (GT)((double)G[c * ldg + r] - w[c]);
  }
}

__global__ void k_centre_H(double* __restrict__ H, int64_t ldh, int64_t n, int l,
                           const double* __restrict__ mu, const double* __restrict__ sG) {
  for (int64_t q = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; q < n * l;
       q += (int64_t)gridDim.x * blockDim.x) {
    const int64_t c = q / n, r = q - c * n;
    H[c * ldh + r] -= mu[r] * sG[c];
  }
}

hipError_t centre_sketch(int mode, void* G, int64_t ldg, int64_t m, double* H, int64_t ldh,
                         int64_t n, int l, const double* om64, int64_t ldo, double* mu,
                         double* small, int b, hipStream_t stream) {
  Ctx cx{stream};
  Small sm = carve_small(small, l, b);
  if (mode == M_F64)
    hipLaunchKernelGGL(k_col_sums<double>, dim3(l), dim3(TPB), 0, stream, (const double*)G, ldg, m,
                       sm.sG);
  else
    hipLaunchKernelGGL(k_col_sums<float>, dim3(l), dim3(TPB), 0, stream, (const float*)G, ldg, m,
                       sm.sG);
  cx.chk();
  if (cx.ok())
    hipLaunchKernelGGL(k_centre_w, dim3(l), dim3(TPB), 0, stream, H, ldh, om64, ldo, n, l,
                       1.0 / (double)m, mu, sm.wc);
  cx.chk();
  if (cx.ok()) {
    if (mode == M_F64)
      hipLaunchKernelGGL(k_centre_G<double>, dim3(grid_for(m * l)), dim3(TPB), 0, stream,
                         (double*)G, ldg, m, l, sm.wc);
    else
      hipLaunchKernelGGL(k_centre_G<float>, dim3(grid_for(m * l)), dim3(TPB), 0, stream,
                         (float*)G, ldg, m, l, sm.wc);
  }
  cx.chk();
  if (cx.ok())
    hipLaunchKernelGGL(k_centre_H, dim3(grid_for(n * l)), dim3(TPB), 0, stream, H, ldh, n, l, mu,
                       sm.sG);
  cx.chk();
  return cx.err;
}

// ---------------------------------------------------------------- one column block (b = l)
// Alg. 4 steps 9-15 with t = 1: Y_1 = G, [Q, R] = qr(G) with the re-orthogonalisation of Sec. 3.2
// (here: Cholesky QR applied twice), the rank guard on R's diagonal, and B = R^{-T} H^T, which is
// Eq. 9 with Q and B still empty.  Every step is a tall product or reduction over all rows at
// once instead of t = l / b dependent rounds of them.  Nothing here waits for the device: B^T is
// formed for all l columns, and Cholesky QR2's tests (flags at sm.info[4] and [5]: a pivot below
// 1e-8 of its diagonal entry, or a second factor more than 1e-6 from I) and R's diagonal (sm.sG,
// for the rank guard) are read with the finalize's last wait.  If the tests reject G the caller
// then runs the blocked loop, whose Householder TSQR fallback handles any G; if the rank guard
// keeps fewer columns it forms the SVD again from the leading ones (B^T's leading columns do not
// depend on the later ones, R^-1 being upper triangular).
template <typename GT>
__global__ void k_widen(const GT* __restrict__ G, int64_t ldg, int64_t rows, int l,
                        double* __restrict__ X, int64_t ldx) {
  for (int64_t q = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; q < rows * l;
       q += (int64_t)gridDim.x * blockDim.x) {
    const int64_t c = q / rows, r = q - c * rows;
    X[c * ldx + r] = (double)G[c * ldg + r];
  }
}

bool one_block(Ctx& cx, FinalizeArgs& f, const Small& sm, Ctrl& hc) {
  const int l = f.l;
  const int64_t m = f.m, n = f.n;
  hipStream_t stream = cx.s;
  double* X = f.Q2;                       // G in FP64 where it is widened; the basis Q
  int* fail = sm.info + kObFail;
  int* ill = sm.info + kObIll;
  // up to l = 112 the Gram and product kernels read G (FP32 or FP64) themselves
  const bool direct = l <= 112;
  if (!direct) {
    if (f.mode == M_F64)
      hipLaunchKernelGGL(k_widen<double>, dim3(grid_for(m * l)), dim3(TPB), 0, stream,
                         (const double*)f.G, f.ldg, m, l, X, f.ldq);
    else
      hipLaunchKernelGGL(k_widen<float>, dim3(grid_for(m * l)), dim3(TPB), 0, stream,
                         (const float*)f.G, f.ldg, m, l, X, f.ldq);
  }
  // (the flags at fail and ill were zeroed by the control-block initialisation)
  // Q1 = G R1^-1 with R1 = chol(G^T G); Q = Q1 R2^-1 with R2 = chol(Q1^T Q1)
  if (!direct) {
    gram_upper(cx, (const double*)X, f.ldq, m, l, f.red_ws, sm.Jm);
  } else if (f.mode == M_F64) {
    gram_upper(cx, (const double*)f.G, f.ldg, m, l, f.red_ws, sm.Jm);
  } else {
    gram_upper(cx, (const float*)f.G, f.ldg, m, l, f.red_ws, sm.Jm);
  }
  chol(cx, sm.Jm, l, 0.0, sm.Wk, sm.Jk, fail, 1e-8, 0.0, ill);
  if (!direct) {
    right_trmul(cx, f.Q, f.ldq, (const double*)X, f.ldq, m, l, sm.Jk);
  } else if (f.mode == M_F64) {
    right_trmul(cx, f.Q, f.ldq, (const double*)f.G, f.ldg, m, l, sm.Jk);
  } else {
    right_trmul(cx, f.Q, f.ldq, (const float*)f.G, f.ldg, m, l, sm.Jk);
  }
  gram_upper(cx, f.Q, f.ldq, m, l, f.red_ws, sm.Jm);
  chol(cx, sm.Jm, l, 0.0, sm.Wm, sm.RB, fail, 0.0, 1e-6, ill);
  if (f.U != nullptr) right_trmul(cx, X, f.ldq, f.Q, f.ldq, m, l, sm.RB);   // Q only feeds U
  // R = R2 R1 and R^-1 = R1^-1 R2^-1 (upper triangular; the products write the zero lower parts
  // too), and the diagonal of R to sm.sG
  if (cx.ok()) {
    hipLaunchKernelGGL(k_trmm_upper2, dim3(l, 2), dim3(JMAX), 0, stream, sm.Wm, sm.Wk, sm.Rg,
                       sm.Jk, sm.RB, sm.Rgi, l, sm.sG);
    cx.chk();
  }
  // B^T = H R^-1 over all l columns (ctrl->l_eff = l from the control-block initialisation)
  right_trmul(cx, f.Bt, f.ldb, f.H, f.ldh, n, l, sm.Rgi, l);
  f.Q = X;
  hc.l_eff = l;
  f.path_loop = 2;
  return cx.ok();
}

// The rank guard of the one-block path: the leading columns whose R diagonal exceeds tau R_00.
int one_block_keep(const double* diag, int l) {
  const double r0 = diag[0];
  if (!(r0 > 0.0)) return 0;
  int keep = 0;
  while (keep < l && fabs(diag[keep]) > kGuardTau * r0) ++keep;
  return keep;
}

hipError_t run_finalize(FinalizeArgs& f, hipStream_t stream) {
  Ctx cx{stream};
  const int l = f.l;
  int b = f.b;
  const int64_t m = f.m, n = f.n;
  Small sm = carve_small(f.small, l, b <= 32 ? b : 32);
  Ctrl* ctrl = f.ctrl;
  if (f.centre) {
    hipError_t e = centre_sketch(f.mode, const_cast<void*>(f.G), f.ldg, m,
                                 const_cast<double*>(f.H), f.ldh, n, l, f.om64, f.ldo, f.mu,
                                 f.small, b, stream);
    if (e != hipSuccess) return e;
  }

  // ---------------- one column block when b = l (see one_block)
  Ctrl hc{};
  bool done = false;
  bool verify = false;                    // one_block's tests and rank guard not yet read
  double* const q_loop = f.Q;             // the blocked loop's basis storage
  if (b == l && f.Q2 != nullptr && !f.force_loop) {
    hipLaunchKernelGGL(k_init_ctrl, dim3(1), dim3(64), 0, stream, ctrl, 1, l, sm.info + kObFail,
                       sm.info + kObIll);
    cx.chk();
    done = cx.ok() && one_block(cx, f, sm, hc);
    if (!cx.ok()) return cx.err;
    verify = done;
  }
  // the blocked loop works on blocks of at most 32 columns: a wider b (b = l) that one_block did
  // not take runs as the widest divisor of l that fits
  if (b > 32) {
    int d = 32;
    while (l % d != 0) --d;
    b = d;
  }
  const int t = l / b;

  // ---------------- column-block loop (Alg. 4 steps 9-15).  Cholesky QR of the blocks first; if a
  // block was flagged as too ill-conditioned for it, the loop is repeated with Householder TSQR.
  auto blocked_loop = [&]() {
    for (int attempt = f.force_loop ? 1 : 0; attempt < 2 && cx.ok(); ++attempt) {
      const bool chol = (attempt == 0);
      hipLaunchKernelGGL(k_init_ctrl, dim3(1), dim3(64), 0, stream, ctrl, t, l, (int*)nullptr,
                         (int*)nullptr);
      cx.chk();
      for (int i = 0; i < t && cx.ok(); ++i) {
        const int c0 = i * b, p = c0;
        double* Qi = f.Q + (int64_t)c0 * f.ldq;
        // W = B Omega_i  (B^T is n x p)
        tn(cx, f.Bt, f.ldb, f.om64 + (int64_t)c0 * f.ldo, f.ldo, p, b, n, f.red_ws, sm.W, b, ctrl, i);
        // Y = G(:, c) - Q W, formed in the basis slot of Q_i
        if (f.mode == M_F64)
          nn<double>(cx, Qi, f.ldq, (const double*)f.G + (int64_t)c0 * f.ldg, f.ldg, f.Q, f.ldq, p,
                     sm.W, b, b, m, -1.0, ctrl, i);
        else
          nn<float>(cx, Qi, f.ldq, (const float*)f.G + (int64_t)c0 * f.ldg, f.ldg, f.Q, f.ldq, p,
                    sm.W, b, b, m, -1.0, ctrl, i);
        if (chol) {
          // [T; Y^T Y] = [Q, Y]^T Y in one row reduction (Q and the slot of Q_i are adjacent): T
          // from the first p b entries, the Gram matrix of Y from the last b^2
          int nch = tn_partials(cx, f.Q, f.ldq, Qi, f.ldq, p + b, b, m, f.red_ws, ctrl, i);
          if (b <= kLaneCholMax) {
            // narrow blocks: the Gram matrices in full, each factored by every lane of the apply
            tn_final(cx, f.red_ws, nch, p + b, b, 0, (int64_t)(p + b) * b, sm.T, b, ctrl, i);
            cholqr_lane(cx, Qi, f.ldq, m, sm.T + (int64_t)p * b, b, nullptr, sm.R1, false, sm, p,
                        ctrl, i);
            // C = Q^T Q_i; Z = Q_i - Q C; two Cholesky QR steps on Z
            tn(cx, f.Q, f.ldq, Qi, f.ldq, p, b, m, f.red_ws, sm.C, b, ctrl, i);
            if (p > 0)   // (with p = 0 the projection leaves Z = Q_i)
              nn<double>(cx, Qi, f.ldq, Qi, f.ldq, f.Q, f.ldq, p, sm.C, b, b, m, -1.0, ctrl, i);
            tn(cx, Qi, f.ldq, Qi, f.ldq, b, b, m, f.red_ws, sm.C1, b, ctrl, i);
            cholqr_lane(cx, Qi, f.ldq, m, sm.C1, b, sm.R1, sm.R2, false, sm, p, ctrl, i);
            tn(cx, Qi, f.ldq, Qi, f.ldq, b, b, m, f.red_ws, sm.C2, b, ctrl, i);
            cholqr_lane(cx, Qi, f.ldq, m, sm.C2, b, sm.R2, sm.R, true, sm, p, ctrl, i);
          } else {
            // wider blocks: the Gram matrix and its factor once, in one workgroup
            tn_final(cx, f.red_ws, nch, p + b, b, 0, (int64_t)p * b, sm.T, b, ctrl, i);
            cholqr(cx, Qi, f.ldq, m, f.red_ws, nch, (int64_t)(p + b) * b, (int64_t)p * b, b,
                   nullptr, sm.R1, false, sm, p, ctrl, i);
            tn(cx, f.Q, f.ldq, Qi, f.ldq, p, b, m, f.red_ws, sm.C, b, ctrl, i);
            if (p > 0)
              nn<double>(cx, Qi, f.ldq, Qi, f.ldq, f.Q, f.ldq, p, sm.C, b, b, m, -1.0, ctrl, i);
            nch = tn_partials(cx, Qi, f.ldq, Qi, f.ldq, b, b, m, f.red_ws, ctrl, i);
            cholqr(cx, Qi, f.ldq, m, f.red_ws, nch, (int64_t)b * b, 0, b, sm.R1, sm.R2, false, sm,
                   p, ctrl, i);
            nch = tn_partials(cx, Qi, f.ldq, Qi, f.ldq, b, b, m, f.red_ws, ctrl, i);
            cholqr(cx, Qi, f.ldq, m, f.red_ws, nch, (int64_t)b * b, 0, b, sm.R2, sm.R, true, sm, p,
                   ctrl, i);
          }
          if (!cx.ok()) break;
        } else {
          // T = Q^T Y
          tn(cx, f.Q, f.ldq, Qi, f.ldq, p, b, m, f.red_ws, sm.T, b, ctrl, i);
          // [Q_i, R_i] = qr(Y), in place
          tsqr(cx, Qi, f.ldq, m, b, f.tsqr_ws, sm.R1, ctrl, i);
          // C = Q^T Q_i; Q_i <- Q_i - Q C; [Q_i, R~_i] = qr(Q_i)
          tn(cx, f.Q, f.ldq, Qi, f.ldq, p, b, m, f.red_ws, sm.C, b, ctrl, i);
          nn<double>(cx, Qi, f.ldq, Qi, f.ldq, f.Q, f.ldq, p, sm.C, b, b, m, -1.0, ctrl, i);
          tsqr(cx, Qi, f.ldq, m, b, f.tsqr_ws, sm.R2, ctrl, i);
          if (!cx.ok()) break;
          // R_i = R~_i R_i and the rank guard
          hipLaunchKernelGGL(k_guard, dim3(1), dim3(256), 0, stream, sm.R1, sm.R2, sm.R, b, i, t,
                             ctrl);
          cx.chk();
          if (p > 0) {
            hipLaunchKernelGGL(k_add_small, dim3(1), dim3(256), 0, stream, sm.T, sm.W, sm.Wn, p * b,
                               ctrl, i);
            cx.chk();
          }
        }
        if (!chol) {
          hipLaunchKernelGGL(k_zero_cols, dim3(grid_for((int64_t)b * m)), dim3(TPB), 0, stream, f.Q,
                             f.ldq, m, c0, b, ctrl, i);
          cx.chk();
        }
        // N = H(:, c) - B^T (T + W);  B_i^T = N R_i^{-1} (row-wise solve in the same kernel)
        nn<double>(cx, f.Bt + (int64_t)c0 * f.ldb, f.ldb, f.H + (int64_t)c0 * f.ldh, f.ldh, f.Bt,
                   f.ldb, p, sm.Wn, b, b, n, -1.0, ctrl, i, sm.R);
      }
      f.path_loop = chol ? 0 : 1;
      if (!cx.ok()) break;
      // one wait per loop: the rank decided on the device (it sizes the rest) and the Cholesky QR
      // flag (pad[0]), which sends the loop round again with Householder TSQR
      cx.err = read_back(&hc, ctrl, sizeof(Ctrl), stream, f.host_pin, f.host_ev);
      if (!chol || !cx.ok() || hc.pad[0] == 0) break;
    }
  };
  if (!done) blocked_loop();
  if (!cx.ok()) return cx.err;
  int L = hc.l_eff;
  bool fresh = false;   // the last wait also read the control block, and no work followed it
  // The one-block path's only wait: its Cholesky QR2 tests, R's diagonal (the rank guard) and the
  // R_B tests, read together (sm.sG follows sm.info in the small matrices).  Returns 1 when the
  // tests rejected G, 2 when the guard keeps fewer than L columns (L is then cut), else 0 with
  // the R_B tests in rbf.
  auto check_one_block = [&](int* rbf) -> int {
    const int64_t dofs = sm.sG - reinterpret_cast<const double*>(sm.info);
    std::vector<double> rbuf((size_t)(dofs + l));
    cx.err = read_back2(rbuf.data(), sm.info, rbuf.size() * sizeof(double), f.ctrl_host, ctrl,
                        f.ctrl_host ? sizeof(Ctrl) : 0, stream, f.host_pin, f.host_ev);
    if (!cx.ok()) return 0;
    fresh = true;
    verify = false;
    const int* fl = reinterpret_cast<const int*>(rbuf.data());
    if (fl[kObFail] != 0 || fl[kObIll] != 0) return 1;
    const int keep = one_block_keep(rbuf.data() + dofs, l);
    if (keep < L) { L = keep; return 2; }
    rbf[0] = fl[1];
    rbf[1] = fl[2];
    return 0;
  };
  for (;;) {
    const int kk = (f.k < L) ? f.k : L;
    int redo = 0;   // after the one-block check: 1 its tests rejected G, 2 the rank guard cut L

    // ---------------- R_B, then the Jacobi SVD and the outputs.  Cholesky QR2 first (rb_mode 0): its
    // acceptance tests are read with the final wait, the SVD and the outputs being formed from its
    // R_B meanwhile; in the rare case it is not accepted, all of it is formed again from shifted
    // Cholesky QR3 (rb_mode 2), or from Gram-Schmidt + TSQR (rb_mode 1) if a pivot of that fails.
    for (int rb_mode = (f.force_rb >= 3) ? 0 : f.force_rb; L > 0;) {
      if (verify && rb_mode == 2) {
        // shifted Cholesky QR3 takes the H storage as scratch: settle the one-block path first
        int rbf[2];
        redo = check_one_block(rbf);
        if (!cx.ok()) return cx.err;
        if (redo != 0) break;
      }
      fresh = false;
      const double* RBp = nullptr;
      if (rb_mode == 0) {
        chol_qr2(cx, f, sm, L, f.force_rb == 4 ? 1 : 0);
        RBp = sm.RB;
      } else if (rb_mode == 2) {
        RBp = chol_qr3_shifted(cx, f, sm, L);
      }
      if (!cx.ok()) return cx.err;
      f.path_rb = (rb_mode == 0) ? 0 : (RBp == nullptr ? 1 : 2);
      if (RBp == nullptr) {
        RBp = sm.RB;
        cx.err = launch_fill_f64(sm.RB, (int64_t)L * L, 0.0, stream);
        for (int c0 = 0; c0 < L && cx.ok(); c0 += b) {
          const int w = (L - c0 < b) ? (L - c0) : b;
          double* Qp = f.Qb + (int64_t)c0 * f.ldb;
          const double* Bp = f.Bt + (int64_t)c0 * f.ldb;
          tn(cx, f.Qb, f.ldb, Bp, f.ldb, c0, w, n, f.red_ws, sm.C1, w, nullptr, 0);
          nn<double>(cx, Qp, f.ldb, Bp, f.ldb, f.Qb, f.ldb, c0, sm.C1, w, w, n, -1.0, nullptr, 0);
          tsqr(cx, Qp, f.ldb, n, w, f.tsqr_ws, sm.R1, nullptr, 0);
          tn(cx, f.Qb, f.ldb, Qp, f.ldb, c0, w, n, f.red_ws, sm.C2, w, nullptr, 0);
          nn<double>(cx, Qp, f.ldb, Qp, f.ldb, f.Qb, f.ldb, c0, sm.C2, w, w, n, -1.0, nullptr, 0);
          tsqr(cx, Qp, f.ldb, n, w, f.tsqr_ws, sm.R2, nullptr, 0);
          if (!cx.ok()) break;
          hipLaunchKernelGGL(k_rb_assemble, dim3(1), dim3(256), 0, stream, sm.C1, sm.C2, sm.R1,
                             sm.R2, sm.RB, L, c0, w);
          cx.chk();
        }
        if (!cx.ok()) return cx.err;
      }
      // ---------------- Jacobi SVD of R_B^T
      {
        const size_t jshm = jacobi_lds_bytes(L);
        if (jshm > (size_t)kJacobiLds) return hipErrorInvalidValue;   // l <= JMAX keeps it inside
        const dim3 g1(1), bj(kJacobiThreads);
        switch (jacobi_epl(L)) {
  #define SK_EPL_CASE(E)                                                                        \
          case E:                                                                               \
            hipLaunchKernelGGL(k_jacobi<E>, g1, bj, jshm, stream, RBp, L, L, sm.Wm, L, sm.info, \
                               sm.sig, sm.perm, sm.Jm);                                         \
            break;
          SK_JACOBI_EPLS(SK_EPL_CASE)
  #undef SK_EPL_CASE
          default: break;
        }
      }
      cx.chk();
      if (!cx.ok()) return cx.err;
      hipLaunchKernelGGL(k_gather, dim3(cdiv(L * kk, 256)), dim3(256), 0, stream, sm.Wm, L, L,
                         sm.perm, sm.sig, kk, sm.Jk, sm.Wk, f.k, f.S);
      cx.chk();
      // V (column-major temp in the Q_B storage, free once R_B is formed; H stays intact for a
      // blocked loop that may still have to run) = B^T W S^-2 in column slices of 16, its signs,
      // then the row-major outputs
      double* Vt = f.Qb;
      const dim3 gv((unsigned)cdiv<int64_t>(n, kNnThreads), cdiv(kk, 16));
      hipLaunchKernelGGL((k_nn_update<double, 16>), gv, dim3(kNnThreads), 0, stream, Vt, f.ldb,
                         (const double*)nullptr, 0, f.Bt, f.ldb, L, sm.Jk, kk, 16, n, 1.0,
                         (const Ctrl*)nullptr, 0, (const double*)nullptr, kk, 0);
      cx.chk();
      if (!cx.ok()) return cx.err;
      hipLaunchKernelGGL(k_signs, dim3(kk), dim3(TPB), 0, stream, Vt, f.ldb, n, sm.sgn);
      cx.chk();
      if (!cx.ok()) return cx.err;
      hipLaunchKernelGGL(k_signed_transpose, dim3(grid_for(n * f.k)), dim3(TPB), 0, stream, Vt,
                         f.ldb, kk, f.k, sm.sgn, n, f.V, f.ldv);
      cx.chk();
      if (f.U && cx.ok()) {
        const dim3 gu(grid_for(m, TPB, 4096), cdiv(f.k, 16));
        hipLaunchKernelGGL(k_write_rows, gu, dim3(TPB), (size_t)L * 16 * sizeof(double), stream,
                           f.Q, f.ldq, L, sm.Wk, kk, f.k, sm.sgn, m, f.U, f.ldu, 0);
        cx.chk();
      }
      if (!cx.ok()) return cx.err;
      int hflags[2] = {1, 1};
      if (verify) {
        redo = check_one_block(hflags);
        if (!cx.ok()) return cx.err;
        if (redo != 0) break;
      } else {
        if (rb_mode != 0) break;
        cx.err = read_back2(hflags, sm.info + 1, 2 * sizeof(int), f.ctrl_host, ctrl,
                            f.ctrl_host ? sizeof(Ctrl) : 0, stream, f.host_pin, f.host_ev);
        if (!cx.ok()) return cx.err;
        fresh = true;
      }
      if (rb_mode != 0) break;
      if (hflags[0] == 0 && hflags[1] == 0 && f.force_rb != 3) break;
      rb_mode = 2;
    }
    if (redo != 0) fresh = false;
    if (redo == 1) {
      // G is too ill-conditioned for Cholesky QR2: the blocked loop, and its SVD
      f.Q = q_loop;
      blocked_loop();
      if (!cx.ok()) return cx.err;
      L = hc.l_eff;
      continue;
    }
    if (redo == 2) {
      // fewer columns pass the rank guard: the SVD of the leading ones
      hipLaunchKernelGGL(k_set_int, dim3(1), dim3(64), 0, stream, &ctrl->l_eff, L);
      cx.chk();
      if (!cx.ok()) return cx.err;
      continue;
    }
    break;
  }
  if (L <= 0) {
    fresh = false;
    // rank 0: all outputs zero
    double zero_s = 0.0;
    (void)zero_s;
    cx.err = launch_fill_f64(f.S, f.k, 0.0, stream);
    for (int64_t r = 0; r < 1 && cx.ok(); ++r) {
      hipLaunchKernelGGL(k_write_rows, dim3(grid_for(n, TPB, 4096), cdiv(f.k, 16)), dim3(TPB), 8,
                         stream, f.Qb, f.ldb, 0, sm.Jk, 0, f.k, sm.sgn, n, f.V, f.ldv, 0);
      cx.chk();
      if (f.U && cx.ok()) {
        hipLaunchKernelGGL(k_write_rows, dim3(grid_for(m, TPB, 4096), cdiv(f.k, 16)), dim3(TPB),
                           8, stream, f.Q, f.ldq, 0, sm.Wk, 0, f.k, sm.sgn, m, f.U, f.ldu, 0);
        cx.chk();
      }
    }
  }
  // the caller reads the control block with a wait of its own unless the last wait read it
  f.ctrl_read = fresh && f.ctrl_host != nullptr && cx.ok();
  return cx.err;
}

// ---------------------------------------------------------------- power scheme, P = 1
// Omega_2 = sqrt(n) orth(H) for the second pass (Sec. 2.2 and the remark closing Sec. 3.3: the
// loop runs again with Omega replaced by H after orth; Sec. 4.2 measures it).  orth is the Q
// factor of H by Cholesky QR2 when its tests accept it (as for R_B: no pivot below 1e-8 of its
// diagonal entry, second factor within 1e-6 of I), else shifted Cholesky QR3, else block
// Gram-Schmidt with Householder TSQR.  H's columns all lean towards v_1 (they are A^T A omega_j),
// so H is as ill-conditioned as (sigma_1 / sigma_l)^2 and the later routes are taken more often
// than for R_B.  The sqrt(n) scale keeps the entries near the unit variance of the Gaussian
// Omega (which the FP8 operand format needs); Alg. 4 depends on Omega only through its span.
__global__ void k_scale_cols(double* __restrict__ X, int64_t ldx, int64_t rows, int cols,
                             double a) {
  for (int64_t q = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; q < rows * cols;
       q += (int64_t)gridDim.x * blockDim.x) {
    const int64_t c = q / rows, r = q - c * rows;
    X[c * ldx + r] *= a;
  }
}

hipError_t run_power_omega(PowerArgs& p, hipStream_t stream) {
  Ctx cx{stream};
  const int L = p.l, b = p.b <= 32 ? p.b : 32;   // Householder TSQR blocks of at most 32 columns
  const int64_t n = p.n;
  Small sm = carve_small(p.small, p.l, p.b);
  int* fail = sm.info + 1;
  int* ill = sm.info + 2;
  const double u = 1.1102230246251565e-16;     // 2^-53
  int route = p.route;
  for (;;) {
    if (route == 0) {
      hipLaunchKernelGGL(k_set_int2, dim3(1), dim3(64), 0, stream, fail, ill, 0);
      cx.chk();
      gram_upper(cx, p.H, p.ldh, n, L, p.red_ws, sm.Jm);
      chol(cx, sm.Jm, L, 0.0, sm.Wk, sm.Jk, fail, 1e-8, 0.0, ill);
      right_trmul(cx, p.W1, p.ldw, p.H, p.ldh, n, L, sm.Jk);
      gram_upper(cx, p.W1, p.ldw, n, L, p.red_ws, sm.Jm);
      chol(cx, sm.Jm, L, 0.0, sm.Wm, sm.Jk, fail, 0.0, 1e-6, ill);
      right_trmul(cx, p.om64, p.ldo, p.W1, p.ldw, n, L, sm.Jk);
    } else if (route == 2) {
      const double shift_rel = 11.0 * ((double)n * L + (double)L * (L + 1)) * u;
      hipLaunchKernelGGL(k_set_int2, dim3(1), dim3(64), 0, stream, fail, ill, 0);
      cx.chk();
      gram_upper(cx, p.H, p.ldh, n, L, p.red_ws, sm.Jm);
      chol(cx, sm.Jm, L, shift_rel, sm.Wk, sm.Jk, fail);
      right_trmul(cx, p.W1, p.ldw, p.H, p.ldh, n, L, sm.Jk);
      gram_upper(cx, p.W1, p.ldw, n, L, p.red_ws, sm.Jm);
      chol(cx, sm.Jm, L, 0.0, sm.Wk, sm.Jk, fail);
      right_trmul(cx, p.W2, p.ldw, p.W1, p.ldw, n, L, sm.Jk);
      gram_upper(cx, p.W2, p.ldw, n, L, p.red_ws, sm.Jm);
      chol(cx, sm.Jm, L, 0.0, sm.Wk, sm.Jk, fail);
      right_trmul(cx, p.om64, p.ldo, p.W2, p.ldw, n, L, sm.Jk);
    } else {
      // block Gram-Schmidt with two Householder TSQR passes per block, on a copy of H
      if (cx.ok())
        cx.err = hipMemcpy2DAsync(p.W1, p.ldw * 8, p.H, p.ldh * 8, n * 8, L,
                                  hipMemcpyDeviceToDevice, stream);
      for (int c0 = 0; c0 < L && cx.ok(); c0 += b) {
        const int w = (L - c0 < b) ? (L - c0) : b;
        double* Qp = p.W2 + (int64_t)c0 * p.ldw;
        const double* Bp = p.W1 + (int64_t)c0 * p.ldw;
        tn(cx, p.W2, p.ldw, Bp, p.ldw, c0, w, n, p.red_ws, sm.C1, w, nullptr, 0);
        nn<double>(cx, Qp, p.ldw, Bp, p.ldw, p.W2, p.ldw, c0, sm.C1, w, w, n, -1.0, nullptr, 0);
        tsqr(cx, Qp, p.ldw, n, w, p.tsqr_ws, sm.R1, nullptr, 0);
        tn(cx, p.W2, p.ldw, Qp, p.ldw, c0, w, n, p.red_ws, sm.C2, w, nullptr, 0);
        nn<double>(cx, Qp, p.ldw, Qp, p.ldw, p.W2, p.ldw, c0, sm.C2, w, w, n, -1.0, nullptr, 0);
        tsqr(cx, Qp, p.ldw, n, w, p.tsqr_ws, sm.R2, nullptr, 0);
      }
      if (cx.ok())
        cx.err = hipMemcpy2DAsync(p.om64, p.ldo * 8, p.W2, p.ldw * 8, n * 8, L,
                                  hipMemcpyDeviceToDevice, stream);
      if (!cx.ok()) return cx.err;
      p.route_used = 1;
      break;
    }
    if (!cx.ok()) return cx.err;
    int hflags[2] = {1, 1};
    cx.err = read_back(hflags, sm.info + 1, 2 * sizeof(int), stream, p.host_pin, p.host_ev);
    if (!cx.ok()) return cx.err;
    if (hflags[0] == 0 && (route == 2 || hflags[1] == 0)) {
      p.route_used = route;
      break;
    }
    route = (route == 0) ? 2 : 1;
  }
  hipLaunchKernelGGL(k_scale_cols, dim3(grid_for(n * L)), dim3(TPB), 0, stream, p.om64, p.ldo, n,
                     L, sqrt((double)n));
  cx.chk();
  return cx.err;
}

}  // namespace sk
