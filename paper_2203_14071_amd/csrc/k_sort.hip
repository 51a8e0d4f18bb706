// uv-sorted visibility layout of a facet object.
//
// Every visibility (row, channel) is a point (u, v) in wavelengths.  Points
// are ordered along a Morton (Z-order) curve over a 2^16 x 2^16 grid
// covering [-max|u|, max|u|] x [-max|v|, max|v|].  A facet cell is a square
// of side 1/theta in the same plane, so along the curve each source's cells
// are entered only a few times and visited in long runs: the extraction
// accumulates runs in registers and touches global memory once per run.
// The order depends only on the geometry, so it is built once per facet
// object (a radix sort of 32-bit keys), then reused by every extraction.
#include <cstring>

#include <rocprim/device/device_radix_sort.hpp>

#include "rlf_internal.h"

namespace rlf {

namespace {

__device__ __forceinline__ uint32_t spread16(uint32_t x) {
  x &= 0xffffu;
  x = (x | (x << 8)) & 0x00ff00ffu;
  x = (x | (x << 4)) & 0x0f0f0f0fu;
  x = (x | (x << 2)) & 0x33333333u;
  x = (x | (x << 1)) & 0x55555555u;
  return x;
}

__device__ __forceinline__ uint32_t quant16(double t) {
  // t in [-1/2, 1/2] -> [0, 65535]
  double q = floor((t + 0.5) * 65536.0);
  q = fmin(fmax(q, 0.0), 65535.0);
  return (uint32_t)q;
}

__global__ __launch_bounds__(256) void k_uv_keys(SortKeyArgs a) {
  const int64_t n = a.n_rows * a.n_chan;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    const int64_t row = i / a.n_chan;
    const int c = (int)(i - row * a.n_chan);
    const double sc = a.chan->scale[c];
    const double u = a.u_m[row] * sc, v = a.v_m[row] * sc;
    a.keys[i] = spread16(quant16(u * a.inv_span_u)) | (spread16(quant16(v * a.inv_span_v)) << 1);
    a.vals[i] = (uint32_t)i;
  }
}

// Static per-visibility data in sorted order: coordinates in wavelengths
// (exactly fl(u_m nu/c)), the channel's spectral factor, and the profile's
// quadratic terms u^2, u v, v^2 (FP64, or FP32 from the FP32-rounded
// coordinates for the mixed form), which are uniform across a wave in the
// extraction and so are computed once here.
__global__ __launch_bounds__(256) void k_sorted_static(Sorted sv, const double *u_m, const double *v_m,
                                                       const double *w_m, int32_t n_chan, const ChanTable *chan,
                                                       int mixed) {
  for (int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; j < sv.n_vis; j += (int64_t)gridDim.x * blockDim.x) {
    const int64_t i = sv.order[j];
    const int64_t row = i / n_chan;
    const int c = (int)(i - row * n_chan);
    const double sc = chan->scale[c];
    const double u = __dmul_rn(u_m[row], sc), v = __dmul_rn(v_m[row], sc);
    const double spec = chan->spec[c];
    sv.geo[j] = make_double4(u, v, __dmul_rn(w_m[row], sc), spec);
    if (mixed) {
      const float uf = (float)u, vf = (float)v;
      reinterpret_cast<float4 *>(sv.quad)[j] = make_float4(uf * uf, uf * vf, vf * vf, (float)spec);
    } else {
      reinterpret_cast<double4 *>(sv.quad)[j] = make_double4(__dmul_rn(u, u), __dmul_rn(u, v), __dmul_rn(v, v), 0.0);
    }
  }
}

unsigned grid_for(int64_t n) {
  const int64_t b = (n + 255) / 256;
  return (unsigned)(b < 16384 ? (b > 0 ? b : 1) : 16384);
}

}  // namespace

hipError_t launch_sort_keys(const SortKeyArgs &a, hipStream_t st) {
  hipLaunchKernelGGL(k_uv_keys, dim3(grid_for(a.n_rows * a.n_chan)), dim3(256), 0, st, a);
  return hipGetLastError();
}

hipError_t sort_pairs_u32(void *tmp, size_t &tmp_bytes, const uint32_t *kin, uint32_t *kout, const uint32_t *vin,
                          uint32_t *vout, int64_t n, hipStream_t st) {
  return rocprim::radix_sort_pairs(tmp, tmp_bytes, kin, kout, vin, vout, (size_t)n, 0, 32, st);
}

hipError_t launch_sorted_static(const Sorted &sv, const double *u_m, const double *v_m, const double *w_m,
                                int32_t n_chan, const ChanTable *chan, int mixed, hipStream_t st) {
  hipLaunchKernelGGL(k_sorted_static, dim3(grid_for(sv.n_vis)), dim3(256), 0, st, sv, u_m, v_m, w_m, n_chan, chan,
                     mixed);
  return hipGetLastError();
}

}  // namespace rlf
