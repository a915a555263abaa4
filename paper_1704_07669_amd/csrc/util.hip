// Small device helpers: fills (kernel-based, so the library issues no memset nodes) and copies of
// internal column-major state to the caller's row-major FP64 buffers.
#include <cstring>

#include "common.hpp"
#include "kernels.hpp"

namespace sk {
namespace {

template <typename T>
__global__ void k_fill(T* __restrict__ p, int64_t count, T v) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < count;
       i += (int64_t)gridDim.x * blockDim.x)
    p[i] = v;
}

template <typename GT>
__global__ void k_copy_state(const GT* __restrict__ G, int64_t ldg, int64_t rows,
                             const double* __restrict__ H, int64_t ldh, int64_t n, int l,
                             double* __restrict__ Gout, double* __restrict__ Hout) {
  const int64_t tg = Gout ? rows * l : 0, th = Hout ? n * l : 0;
  for (int64_t q = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; q < tg + th;
       q += (int64_t)gridDim.x * blockDim.x) {
    if (q < tg) {
      const int64_t r = q / l;
      const int c = (int)(q - r * l);
      Gout[q] = (double)G[c * ldg + r];
    } else {
      const int64_t qq = q - tg, r = qq / l;
      const int c = (int)(qq - r * l);
      Hout[qq] = H[c * ldh + r];
    }
  }
}

__global__ void k_copy_omega(const double* __restrict__ om, int64_t ldo, int64_t n, int l,
                             double* __restrict__ out, int64_t ld) {
  for (int64_t q = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; q < n * l;
       q += (int64_t)gridDim.x * blockDim.x) {
    const int64_t r = q / l;
    const int c = (int)(q - r * l);
    out[r * ld + c] = om[c * ldo + r];
  }
}

__global__ void k_fill_rows(double* __restrict__ p, int64_t rows, int cols, int64_t ld, double v) {
  for (int64_t q = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; q < rows * cols;
       q += (int64_t)gridDim.x * blockDim.x) {
    const int64_t r = q / cols;
    p[r * ld + (q - r * cols)] = v;
  }
}

__global__ void k_scale(double* __restrict__ p, int64_t count, double a) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < count;
       i += (int64_t)gridDim.x * blockDim.x)
    p[i] *= a;
}

// a[c * lda + r] += b[c * ldb + r] for r < rows, c < cols (column-major FP64)
__global__ void k_add_cols(double* __restrict__ a, int64_t lda, const double* __restrict__ b,
                           int64_t ldb, int64_t rows, int cols) {
  for (int64_t q = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; q < rows * cols;
       q += (int64_t)gridDim.x * blockDim.x) {
    const int64_t c = q / rows, r = q - c * rows;
    a[c * lda + r] += b[c * ldb + r];
  }
}

// *diff = number of (r, c) with the bit patterns of a and b differing (column-major FP64)
__global__ void k_count_diff(const double* __restrict__ a, int64_t lda,
                             const double* __restrict__ b, int64_t ldb, int64_t rows, int cols,
                             unsigned* __restrict__ diff) {
  unsigned d = 0;
  for (int64_t q = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; q < rows * cols;
       q += (int64_t)gridDim.x * blockDim.x) {
    const int64_t c = q / rows, r = q - c * rows;
    d += (__double_as_longlong(a[c * lda + r]) != __double_as_longlong(b[c * ldb + r])) ? 1u : 0u;
  }
  if (d) atomicAdd(diff, d);
}

inline int grid_for(int64_t work) {
  int64_t g = cdiv<int64_t>(work, 256);
  return (int)(g < 1 ? 1 : (g > 65536 ? 65536 : g));
}
}  // namespace

hipError_t read_back(void* dst, const void* src, size_t bytes, hipStream_t s, void* pin,
                     hipEvent_t ev) {
  if (pin == nullptr || ev == nullptr || bytes > kHostPinBytes) {
    hipError_t e = bytes ? hipMemcpyAsync(dst, src, bytes, hipMemcpyDeviceToHost, s) : hipSuccess;
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    return e;
  }
  hipError_t e = bytes ? hipMemcpyAsync(pin, src, bytes, hipMemcpyDeviceToHost, s) : hipSuccess;
  if (e == hipSuccess) e = hipEventRecord(ev, s);
  if (e == hipSuccess) {
    while ((e = hipEventQuery(ev)) == hipErrorNotReady) {
    }
    // the polls leave "not ready" as the runtime's last error; the launch checks that follow
    // read it, so it is cleared once the event has completed
    if (e == hipSuccess) (void)hipGetLastError();
  }
  if (e == hipSuccess && bytes) memcpy(dst, pin, bytes);
  return e;
}

hipError_t read_back2(void* dst1, const void* src1, size_t bytes1, void* dst2, const void* src2,
                      size_t bytes2, hipStream_t s, void* pin, hipEvent_t ev) {
  const size_t off = (bytes1 + 63) & ~(size_t)63;
  if (pin == nullptr || ev == nullptr || off + bytes2 > kHostPinBytes) {
    hipError_t e = read_back(dst1, src1, bytes1, s, nullptr, nullptr);
    if (e == hipSuccess) e = read_back(dst2, src2, bytes2, s, nullptr, nullptr);
    return e;
  }
  uint8_t* p = static_cast<uint8_t*>(pin);
  hipError_t e = bytes1 ? hipMemcpyAsync(p, src1, bytes1, hipMemcpyDeviceToHost, s) : hipSuccess;
  if (e == hipSuccess && bytes2)
    e = hipMemcpyAsync(p + off, src2, bytes2, hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipEventRecord(ev, s);
  if (e == hipSuccess) {
    while ((e = hipEventQuery(ev)) == hipErrorNotReady) {
    }
    if (e == hipSuccess) (void)hipGetLastError();   // (as in read_back)
  }
  if (e == hipSuccess && bytes1) memcpy(dst1, p, bytes1);
  if (e == hipSuccess && bytes2) memcpy(dst2, p + off, bytes2);
  return e;
}

hipError_t launch_fill_f64(double* p, int64_t count, double v, hipStream_t s) {
  if (count <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_fill<double>, dim3(grid_for(count)), dim3(256), 0, s, p, count, v);
  return hipGetLastError();
}

hipError_t launch_fill_rows(double* p, int64_t rows, int cols, int64_t ld, double v,
                            hipStream_t s) {
  if (rows <= 0 || cols <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_fill_rows, dim3(grid_for(rows * cols)), dim3(256), 0, s, p, rows, cols, ld,
                     v);
  return hipGetLastError();
}

hipError_t launch_fill_u32(uint32_t* p, int64_t count, uint32_t v, hipStream_t s) {
  if (count <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_fill<uint32_t>, dim3(grid_for(count)), dim3(256), 0, s, p, count, v);
  return hipGetLastError();
}

hipError_t launch_copy_state(int mode, const void* G, int64_t ldg, int64_t rows, const double* H,
                             int64_t ldh, int64_t n, int l, double* Gout, double* Hout,
                             hipStream_t s) {
  const int64_t work = (Gout ? rows * l : 0) + (Hout ? n * l : 0);
  if (work == 0) return hipSuccess;
  if (mode == M_F64)
    hipLaunchKernelGGL(k_copy_state<double>, dim3(grid_for(work)), dim3(256), 0, s,
                       (const double*)G, ldg, rows, H, ldh, n, l, Gout, Hout);
  else
    hipLaunchKernelGGL(k_copy_state<float>, dim3(grid_for(work)), dim3(256), 0, s,
                       (const float*)G, ldg, rows, H, ldh, n, l, Gout, Hout);
  return hipGetLastError();
}

hipError_t launch_copy_omega_out(const double* om64, int64_t ldo, int64_t n, int l, double* out,
                                 int64_t ld, hipStream_t s) {
  hipLaunchKernelGGL(k_copy_omega, dim3(grid_for(n * l)), dim3(256), 0, s, om64, ldo, n, l, out,
                     ld);
  return hipGetLastError();
}

hipError_t launch_scale_f64(double* p, int64_t count, double a, hipStream_t s) {
  if (count <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_scale, dim3(grid_for(count)), dim3(256), 0, s, p, count, a);
  return hipGetLastError();
}

hipError_t launch_add_cols(double* a, int64_t lda, const double* b, int64_t ldb, int64_t rows,
                           int cols, hipStream_t s) {
  if (rows <= 0 || cols <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_add_cols, dim3(grid_for(rows * cols)), dim3(256), 0, s, a, lda, b, ldb, rows,
                     cols);
  return hipGetLastError();
}

hipError_t launch_count_diff(const double* a, int64_t lda, const double* b, int64_t ldb,
                             int64_t rows, int cols, unsigned* diff, hipStream_t s) {
  if (rows <= 0 || cols <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_count_diff, dim3(grid_for(rows * cols)), dim3(256), 0, s, a, lda, b, ldb,
                     rows, cols, diff);
  return hipGetLastError();
}

}  // namespace sk
