// Facet compaction (Sec. 2.3): keep the cells of each source's dense block
// that received at least one visibility, in memory order of the block, which
// is (iy, ix) order.  Vbar = Z / W; the cell centre is (ix, iy) / theta.
// Three steps: count per source, scan over sources, write; the write step
// also clears the dense block for the next extraction.
#include "rlf_internal.h"

namespace rlf {

namespace {

__device__ __forceinline__ int block_sum_int(int x, int *sh) {
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
#pragma unroll
  for (int d = 32; d > 0; d >>= 1) x += __shfl_xor(x, d);
  if (lane == 0) sh[wid] = x;
  __syncthreads();
  int t = 0;
  for (int k = 0; k < (int)(blockDim.x >> 6); ++k) t += sh[k];
  __syncthreads();
  return t;
}

__global__ __launch_bounds__(256) void k_count(CompactArgs a) {
  __shared__ int sh[4];
  const int s = blockIdx.x;
  const SrcGeom g = a.geom[s];
  const int64_t n = (int64_t)g.side * g.side;
  int local = 0;
  for (int64_t k = threadIdx.x; k < n; k += blockDim.x) local += a.acc.cell[g.base + k].w > 0.0;
  const int t = block_sum_int(local, sh);
  if (threadIdx.x == 0) a.cells.n_nonempty[s] = t;
}

// Exclusive scan over sources (one block).
__global__ __launch_bounds__(1024) void k_scan(CompactArgs a) {
  __shared__ int64_t sh[1024];
  const int n = a.n_src;
  const int per = (n + 1023) / 1024;
  const int lo = min(n, (int)threadIdx.x * per), hi = min(n, lo + per);
  int64_t local = 0;
  for (int k = lo; k < hi; ++k) local += a.cells.n_nonempty[k];
  sh[threadIdx.x] = local;
  __syncthreads();
  for (int d = 1; d < 1024; d <<= 1) {               // Hillis-Steele inclusive scan
    const int64_t o = threadIdx.x >= (unsigned)d ? sh[threadIdx.x - d] : 0;
    __syncthreads();
    sh[threadIdx.x] += o;
    __syncthreads();
  }
  int64_t run = sh[threadIdx.x] - local;
  for (int k = lo; k < hi; ++k) {
    a.cells.offsets[k] = run;
    run += a.cells.n_nonempty[k];
  }
  if (threadIdx.x == 1023) a.cells.offsets[n] = sh[1023];
}

template <bool kMixed>
__global__ __launch_bounds__(256) void k_write(CompactArgs a) {
  __shared__ int wsum[4];
  const int s = blockIdx.x;
  const SrcGeom g = a.geom[s];
  const double theta = a.src[s].theta;
  const int64_t n = (int64_t)g.side * g.side;
  int64_t out = a.cells.offsets[s];
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  for (int64_t k0 = 0; k0 < n; k0 += blockDim.x) {
    const int64_t k = k0 + threadIdx.x;
    uint32_t cnt = 0u;
    double W = 0.0, zr = 0.0, zi = 0.0;
    if (k < n) {
      const int64_t d = g.base + k;
      const double4 c = a.acc.cell[d];
      cnt = (uint32_t)c.w;                       // an exact integer sum
      if (cnt) {
        W = c.x;
        zr = c.y;
        zi = c.z;
        a.acc.cell[d] = make_double4(0.0, 0.0, 0.0, 0.0);
      }
    }
    const bool keep = cnt > 0u;
    const uint64_t m = __ballot(keep);
    const int before = __popcll(m & ((1ull << lane) - 1ull));
    if (lane == 0) wsum[wid] = __popcll(m);
    __syncthreads();
    int wave_off = 0, total = 0;
    for (int q = 0; q < 4; ++q) {
      wave_off += q < wid ? wsum[q] : 0;
      total += wsum[q];
    }
    __syncthreads();
    if (keep) {
      const int64_t o = out + wave_off + before;
      const int ix = (int)(k % g.side) - g.half;
      const int iy = (int)(k / g.side) - g.half;
      const double vr = zr / W, vi = zi / W;
      a.cells.ix[o] = ix;
      a.cells.iy[o] = iy;
      a.cells.count[o] = (int32_t)cnt;
      a.cells.wsum[o] = W;
      a.cells.vre[o] = vr;
      a.cells.vim[o] = vi;
      // likelihood records with sqrt(W) carried by the profile: with
      // c = W^{-1/3}, sqrt(W) f(x) = (c x)^{-3/2} and c x = c + s_k |A^{-T} k'|^2
      // for the cell centre k' = W^{-1/6} (uc, vc), so a knot's terms are
      // h = (c + s_k q')^{-3/2}, D += (sqrt(W) Re Vbar) h, M += h h
      const double uc = (double)ix / theta, vc = (double)iy / theta;
      const double cw = 1.0 / cbrt(W), rw = sqrt(cw), b = sqrt(W) * vr;
      // the mixed form's fit runs on the FP32 records; its estimator
      // rechecks the points at its decisions on the FP64 ones
      if (kMixed) a.cells.fit32[o] = make_float4((float)(uc * rw), (float)(vc * rw), (float)cw, (float)b);
      a.cells.fit64[o] = make_double4(uc * rw, vc * rw, cw, b);
    }
    out += total;
  }
}

}  // namespace

hipError_t launch_compact(const CompactArgs &a, int mixed, hipStream_t st) {
  hipLaunchKernelGGL(k_count, dim3(a.n_src), dim3(256), 0, st, a);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_scan, dim3(1), dim3(1024), 0, st, a);
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  if (mixed)
    hipLaunchKernelGGL(k_write<true>, dim3(a.n_src), dim3(256), 0, st, a);
  else
    hipLaunchKernelGGL(k_write<false>, dim3(a.n_src), dim3(256), 0, st, a);
  return hipGetLastError();
}

}  // namespace rlf
