// Gaussian test matrix Omega = randn(n, l) (Algorithm 4, step 3) and its operand copies.
//
// Generator (the paper only says "randn"): Philox-4x64-10 of Salmon et al. (SC'11) with key
// (seed, 0); word w is lane w % 4 of the block at counter (w / 4, 0, 0, 0).  Entry (r, c), with
// q = r*l + c, uses words 2q and 2q+1: u1 = (w0 >> 11) 2^-53, u2 = (w1 >> 11) 2^-53 and the
// Box-Muller value sqrt(-2 ln(1 - u1)) cos(2 pi u2).  Omega is stored column-major (each of the l
// columns contiguous along n), which is the K-contiguous layout the streaming product reads.
#include "common.hpp"
#include "kernels.hpp"

namespace sk {

namespace {
constexpr uint64_t PH_M0 = 0xD2E7470EE14C6C93ull, PH_M1 = 0xCA5A826395121157ull;
constexpr uint64_t PH_W0 = 0x9E3779B97F4A7C15ull, PH_W1 = 0xBB67AE8584CAA73Bull;

__device__ __forceinline__ void philox_block(uint64_t c0, uint64_t key0, uint64_t out[4]) {
  uint64_t x0 = c0, x1 = 0, x2 = 0, x3 = 0, k0 = key0, k1 = 0;
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    const uint64_t lo0 = PH_M0 * x0, hi0 = __umul64hi(PH_M0, x0);
    const uint64_t lo1 = PH_M1 * x2, hi1 = __umul64hi(PH_M1, x2);
    const uint64_t y0 = hi1 ^ x1 ^ k0, y2 = hi0 ^ x3 ^ k1;
    x0 = y0; x1 = lo1; x2 = y2; x3 = lo0;
    k0 += PH_W0; k1 += PH_W1;
  }
  out[0] = x0; out[1] = x1; out[2] = x2; out[3] = x3;
}

__device__ __forceinline__ double box_muller(uint64_t w0, uint64_t w1) {
  const double u1 = (double)(w0 >> 11) * 0x1.0p-53;
  const double u2 = (double)(w1 >> 11) * 0x1.0p-53;
  return sqrt(-2.0 * log1p(-u1)) * cos(2.0 * 3.141592653589793 * u2);
}

// One thread per Philox block = two consecutive entries q = 2p, 2p + 1.
__global__ void k_omega_philox(uint64_t seed, int64_t n, int l, double* __restrict__ om,
                               int64_t ldo) {
  const int64_t total = n * (int64_t)l;
  const int64_t npairs = (total + 1) / 2;
  for (int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; p < npairs;
       p += (int64_t)gridDim.x * blockDim.x) {
    uint64_t w[4];
    philox_block((uint64_t)p, seed, w);
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const int64_t q = 2 * p + h;
      if (q < total) {
        const int64_t r = q / l;
        const int c = (int)(q - r * l);
        om[c * ldo + r] = box_muller(w[2 * h], w[2 * h + 1]);
      }
    }
  }
}

__global__ void k_philox_words(uint64_t seed, uint64_t first, int64_t count,
                               uint64_t* __restrict__ out) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < count;
       i += (int64_t)gridDim.x * blockDim.x) {
    const uint64_t w = first + (uint64_t)i;
    uint64_t b[4];
    philox_block(w >> 2, seed, b);
    out[i] = b[w & 3];
  }
}

__global__ void k_omega_user(const double* __restrict__ src, int64_t ld, int64_t n, int l,
                             double* __restrict__ om, int64_t ldo) {
  const int64_t total = n * (int64_t)l;
  for (int64_t q = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; q < total;
       q += (int64_t)gridDim.x * blockDim.x) {
    const int c = (int)(q / n);
    const int64_t r = q - (int64_t)c * n;
    om[c * ldo + r] = src[r * ld + c];
  }
}

// Omega' in the operand format; padding rows (>= n) and columns (>= l) are zero.
template <int MODE, typename OpT>
__global__ void k_omega_quantize(int64_t n, int64_t NP, int l, int LP, double* __restrict__ om64,
                                 OpT* __restrict__ omc) {
  const int64_t total = NP * (int64_t)LP;
  for (int64_t q = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; q < total;
       q += (int64_t)gridDim.x * blockDim.x) {
    const int c = (int)(q / NP);
    const int64_t r = q - (int64_t)c * NP;
    const bool in = (r < n) && (c < l);
    const double x = in ? om64[q] : 0.0;
    double xq;
    OpT v;
    if constexpr (MODE == M_F64) {
      xq = x; v = x;
    } else if constexpr (MODE == M_F32) {
      const float w = (float)x; xq = w; v = w;
    } else if constexpr (MODE == M_BF16 || MODE == M_BF16X2) {
      // one rounding from FP64 to the BF16 grid (8 significant bits, nearest even) on the bit
      // pattern, then an exact conversion; values below 2^-126 (BF16 subnormals) go through FP32
      double r = x;
      if (fabs(x) >= 0x1p-126 && fabs(x) < 0x1p127) {
        uint64_t u = (uint64_t)__double_as_longlong(x);
        u += 0xFFFFFFFFFFFull + ((u >> 45) & 1ull);
        u &= ~0x1FFFFFFFFFFFull;
        r = __longlong_as_double((long long)u);
      }
      const __bf16 h = to_bf16((float)r); xq = (double)from_bf16(h); v = h;
    } else {
      const float sx = fminf(fmaxf((float)x * 32.0f, -448.0f), 448.0f);
      const uint32_t byte = pack_fp8x2(sx, 0.0f) & 0xffu;
      xq = (double)fp8_to_f32(byte) / 32.0; v = (OpT)byte;
    }
    om64[q] = in ? xq : 0.0;
    omc[q] = v;
  }
}

inline int grid_for(int64_t work, int block = 256) {
  int64_t g = cdiv<int64_t>(work, block);
  return (int)(g < 1 ? 1 : (g > 65536 ? 65536 : g));
}
}  // namespace

hipError_t launch_omega_philox(uint64_t seed, int64_t n, int l, double* om64, int64_t ldo,
                               hipStream_t s) {
  const int64_t npairs = (n * l + 1) / 2;
  hipLaunchKernelGGL(k_omega_philox, dim3(grid_for(npairs)), dim3(256), 0, s, seed, n, l, om64,
                     ldo);
  return hipGetLastError();
}

hipError_t launch_philox_words(uint64_t seed, uint64_t first, int64_t count, uint64_t* out,
                               hipStream_t s) {
  hipLaunchKernelGGL(k_philox_words, dim3(grid_for(count)), dim3(256), 0, s, seed, first, count,
                     out);
  return hipGetLastError();
}

hipError_t launch_omega_user(const double* src, int64_t ld, int64_t n, int l, double* om64,
                             int64_t ldo, hipStream_t s) {
  hipLaunchKernelGGL(k_omega_user, dim3(grid_for(n * l)), dim3(256), 0, s, src, ld, n, l, om64,
                     ldo);
  return hipGetLastError();
}

hipError_t launch_omega_quantize(int mode, int64_t n, int64_t NP, int l, int LP, double* om64,
                                 void* omc, hipStream_t s) {
  const dim3 grid(grid_for(NP * LP)), block(256);
  switch (mode) {
    case M_F64:
      hipLaunchKernelGGL((k_omega_quantize<M_F64, double>), grid, block, 0, s, n, NP, l, LP, om64,
                         (double*)omc);
      break;
    case M_F32:
      hipLaunchKernelGGL((k_omega_quantize<M_F32, float>), grid, block, 0, s, n, NP, l, LP, om64,
                         (float*)omc);
      break;
    case M_BF16:
    case M_BF16X2:
      hipLaunchKernelGGL((k_omega_quantize<M_BF16, __bf16>), grid, block, 0, s, n, NP, l, LP,
                         om64, (__bf16*)omc);
      break;
    case M_FP8:
      hipLaunchKernelGGL((k_omega_quantize<M_FP8, uint8_t>), grid, block, 0, s, n, NP, l, LP,
                         om64, (uint8_t*)omc);
      break;
    default:
      return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

}  // namespace sk
