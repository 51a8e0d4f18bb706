// Small utility kernels: max |x| over an array (facet sizing) and fills.
// Fills are kernels rather than hipMemsetAsync so that a captured graph
// holds only kernel nodes.
#include "rlf_internal.h"

namespace rlf {

namespace {

__global__ __launch_bounds__(256) void k_absmax(const double *x, int64_t n, double *out2, int slot) {
  __shared__ double sh[4];
  double m = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    m = fmax(m, fabs(x[i]));
#pragma unroll
  for (int d = 32; d > 0; d >>= 1) m = fmax(m, __shfl_xor(m, d));
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = m;
  __syncthreads();
  if (threadIdx.x == 0) {
    m = fmax(fmax(sh[0], sh[1]), fmax(sh[2], sh[3]));
    // non-negative doubles order like their bit patterns
    atomicMax(reinterpret_cast<unsigned long long *>(out2 + slot), (unsigned long long)__double_as_longlong(m));
  }
}

__global__ __launch_bounds__(256) void k_fill_u32(uint32_t *p, int64_t n, uint32_t v) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) p[i] = v;
}

// dst[idx[i]] = src[i] (| bits for the 32-bit form), i < n; idx in range by
// construction of the caller.
__global__ __launch_bounds__(256) void k_scatter_f64(const double *src, const int32_t *idx, int64_t n, double *dst) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    dst[idx[i]] = src[i];
}

__global__ __launch_bounds__(256) void k_scatter_u32(const uint32_t *src, const int32_t *idx, int64_t n, uint32_t bits,
                                                     uint32_t *dst) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    dst[idx[i]] = src[i] | bits;
}

unsigned grid_for(int64_t n) {
  const int64_t b = (n + 255) / 256;
  return (unsigned)(b < 8192 ? (b > 0 ? b : 1) : 8192);
}

}  // namespace

hipError_t launch_absmax(const double *x, int64_t n, double *out2, int slot, hipStream_t st) {
  hipLaunchKernelGGL(k_absmax, dim3(grid_for(n)), dim3(256), 0, st, x, n, out2, slot);
  return hipGetLastError();
}

hipError_t launch_scatter_f64(const double *src, const int32_t *idx, int64_t n, double *dst, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_scatter_f64, dim3(grid_for(n)), dim3(256), 0, st, src, idx, n, dst);
  return hipGetLastError();
}

hipError_t launch_scatter_u32(const uint32_t *src, const int32_t *idx, int64_t n, uint32_t bits, uint32_t *dst,
                              hipStream_t st) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_scatter_u32, dim3(grid_for(n)), dim3(256), 0, st, src, idx, n, bits, dst);
  return hipGetLastError();
}

hipError_t launch_fill_u32(uint32_t *p, int64_t n, uint32_t v, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_fill_u32, dim3(grid_for(n)), dim3(256), 0, st, p, n, v);
  return hipGetLastError();
}

}  // namespace rlf
