// Adaptive refinement of the shape estimate (Sec. 2.4: sample around the
// maximum until NP_MAX samples lie above the 5 % threshold or the resolution
// E_RES is reached).  Nested grids: level L holds e = k * e_step / 2^L (k
// integer).  A source whose thresholded set at level L - 1 has fewer than
// np_max points is evaluated at level L on the set's bounding box (in level-L
// indices 2 kmin - 2 .. 2 kmax + 2, i.e. widened by one level-(L-1) step),
// at most max_side points per axis (else max_side points centred on twice
// the maximum's index).  Every decision is on integers or on the same FP64
// values as the estimator, so a reference computes the same windows.
//
// k_refine_start scans the full-grid surface (level 0); k_refine_estimate
// takes the level's window values, writes the estimate (flag REFINED, the
// bad-variance flag from the refined widths) and the next window.  One
// block per source.
#include "rlf_internal.h"

namespace rlf {

namespace {

constexpr int kThreads = 256;

__device__ __forceinline__ double block_sum(double x, double *sh) {
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
#pragma unroll
  for (int d = 32; d > 0; d >>= 1) x += __shfl_xor(x, d);
  if (lane == 0) sh[wid] = x;
  __syncthreads();
  const double t = (sh[0] + sh[1]) + (sh[2] + sh[3]);
  __syncthreads();
  return t;
}

__device__ __forceinline__ int block_min(int x, int *sh) {
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
#pragma unroll
  for (int d = 32; d > 0; d >>= 1) x = min(x, __shfl_xor(x, d));
  if (lane == 0) sh[wid] = x;
  __syncthreads();
  const int t = min(min(sh[0], sh[1]), min(sh[2], sh[3]));
  __syncthreads();
  return t;
}

// Maximum over the block with the smallest index on ties.
__device__ __forceinline__ void block_argmax(double &best, int &bi, double *shv, int *shi) {
#pragma unroll
  for (int d = 32; d > 0; d >>= 1) {
    const double ov = __shfl_xor(best, d);
    const int oi = __shfl_xor(bi, d);
    if (ov > best || (ov == best && oi < bi)) {
      best = ov;
      bi = oi;
    }
  }
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  if (lane == 0) {
    shv[wid] = best;
    shi[wid] = bi;
  }
  __syncthreads();
  best = shv[0];
  bi = shi[0];
  for (int q = 1; q < 4; ++q)
    if (shv[q] > best || (shv[q] == best && shi[q] < bi)) {
      best = shv[q];
      bi = shi[q];
    }
  __syncthreads();
}

// Next window along one axis (see the file comment).
__device__ __forceinline__ void next_range(int kmin, int kmax, int karg, int max_side, int &lo, int &n) {
  lo = 2 * kmin - 2;
  int hi = 2 * kmax + 2;
  if (hi - lo + 1 > max_side) {
    lo = 2 * karg - (max_side - 1) / 2;
    hi = lo + max_side - 1;
  }
  n = hi - lo + 1;
}

__global__ __launch_bounds__(kThreads) void k_refine_start(RefineArgs r) {
  __shared__ double shv[4];
  __shared__ int shi[4];
  __shared__ double shd[4];
  __shared__ int shm[4];
  const int s = blockIdx.x;
  int32_t *w = r.win + (int64_t)s * 5;
  if (r.offsets[s + 1] == r.offsets[s]) {                 // empty facet
    if (threadIdx.x == 0) w[0] = 0;
    return;
  }
  const double *L = r.lsurf + (int64_t)s * r.n_valid;
  const int ctr = (r.n_e - 1) / 2;
  double best = -INFINITY;
  int bi = 0x7fffffff;
  for (int j = threadIdx.x; j < r.n_valid; j += kThreads) {
    const double v = L[j];
    if (v > best) {
      best = v;
      bi = j;
    }
  }
  block_argmax(best, bi, shv, shi);
  const double thr = best + r.log_frac;
  double cnt = 0.0;
  int k1min = 1 << 30, k2min = 1 << 30, k1nmax = 1 << 30, k2nmax = 1 << 30;   // -max as a min
  for (int j = threadIdx.x; j < r.n_valid; j += kThreads) {
    if (L[j] >= thr) {
      const int f = r.epts[j];
      const int k1 = f / r.n_e - ctr, k2 = f - (f / r.n_e) * r.n_e - ctr;
      cnt += 1.0;
      k1min = min(k1min, k1);
      k2min = min(k2min, k2);
      k1nmax = min(k1nmax, -k1);
      k2nmax = min(k2nmax, -k2);
    }
  }
  cnt = block_sum(cnt, shd);
  k1min = block_min(k1min, shm);
  k2min = block_min(k2min, shm);
  k1nmax = block_min(k1nmax, shm);
  k2nmax = block_min(k2nmax, shm);
  if (threadIdx.x == 0) {
    if (!(best > -INFINITY) || cnt >= (double)r.np_max || r.last_level < 1) {
      w[0] = 0;
      return;
    }
    const int f = r.epts[bi];
    int lo1, n1, lo2, n2;
    next_range(k1min, -k1nmax, f / r.n_e - ctr, r.max_side, lo1, n1);
    next_range(k2min, -k2nmax, f - (f / r.n_e) * r.n_e - ctr, r.max_side, lo2, n2);
    w[0] = 1;
    w[1] = lo1;
    w[2] = lo2;
    w[3] = n1;
    w[4] = n2;
  }
}

__global__ __launch_bounds__(kThreads) void k_refine_estimate(RefineArgs r) {
  __shared__ double shv[4];
  __shared__ int shi[4];
  __shared__ double shd[4];
  __shared__ int shm[4];
  const int s = blockIdx.x;
  int32_t *w = r.win + (int64_t)s * 5;
  if (!w[0]) return;
  const int lo1 = w[1], lo2 = w[2], n1 = w[3], n2 = w[4];
  const int np = n1 * n2;
  const double *L = r.lloc + (int64_t)s * r.max_side * r.max_side;
  const double res = r.e_step / (double)(1 << r.level);
  double best = -INFINITY;
  int bi = 0x7fffffff;
  for (int t = threadIdx.x; t < np; t += kThreads) {
    const double v = L[t];
    if (v > best) {
      best = v;
      bi = t;
    }
  }
  block_argmax(best, bi, shv, shi);
  if (!(best > -INFINITY)) {                                // no valid point: keep the previous estimate
    __syncthreads();
    if (threadIdx.x == 0) w[0] = 0;
    return;
  }
  const double thr = best + r.log_frac;
  double sw = 0.0, s1 = 0.0, s2 = 0.0, cnt = 0.0;
  int k1min = 1 << 30, k2min = 1 << 30, k1nmax = 1 << 30, k2nmax = 1 << 30;
  for (int t = threadIdx.x; t < np; t += kThreads) {
    const double v = L[t];
    if (v >= thr) {
      const int k1 = lo1 + t / n2, k2 = lo2 + t % n2;
      const double wt = exp(v - best);
      sw += wt;
      s1 += wt * ((double)k1 * res);
      s2 += wt * ((double)k2 * res);
      cnt += 1.0;
      k1min = min(k1min, k1);
      k2min = min(k2min, k2);
      k1nmax = min(k1nmax, -k1);
      k2nmax = min(k2nmax, -k2);
    }
  }
  sw = block_sum(sw, shd);
  s1 = block_sum(s1, shd);
  s2 = block_sum(s2, shd);
  cnt = block_sum(cnt, shd);
  k1min = block_min(k1min, shm);
  k2min = block_min(k2min, shm);
  k1nmax = block_min(k1nmax, shm);
  k2nmax = block_min(k2nmax, shm);
  const double m1 = s1 / sw, m2 = s2 / sw;
  double c11 = 0.0, c22 = 0.0, c12 = 0.0;
  for (int t = threadIdx.x; t < np; t += kThreads) {
    const double v = L[t];
    if (v >= thr) {
      const double wt = exp(v - best);
      const double d1 = (double)(lo1 + t / n2) * res - m1, d2 = (double)(lo2 + t % n2) * res - m2;
      c11 += wt * d1 * d1;
      c22 += wt * d2 * d2;
      c12 += wt * d1 * d2;
    }
  }
  c11 = block_sum(c11, shd) / sw;
  c22 = block_sum(c22, shd) / sw;
  c12 = block_sum(c12, shd) / sw;
  if (threadIdx.x == 0) {
    const double sd1 = sqrt(c11), sd2 = sqrt(c22);
    const double det = c11 * c22 - c12 * c12;
    const double sqd = det > 0.0 ? sqrt(det) : 0.0;
    const bool bad = sd1 <= r.bad_sigma || sd2 <= r.bad_sigma || sqd <= r.bad_sqrtdet;
    if (r.e1) r.e1[s] = m1;
    if (r.e2) r.e2[s] = m2;
    if (r.s1) r.s1[s] = sd1;
    if (r.s2) r.s2[s] = sd2;
    if (r.c12) r.c12[s] = c12;
    if (r.lmax) r.lmax[s] = best;
    if (r.n_above) r.n_above[s] = (int32_t)cnt;
    r.flags[s] = (r.flags[s] & ~(uint32_t)RLF_FLAG_BAD_VAR) | (bad ? (uint32_t)RLF_FLAG_BAD_VAR : 0u) |
                 (uint32_t)RLF_FLAG_REFINED;
    if (cnt >= (double)r.np_max || r.level >= r.last_level) {
      w[0] = 0;
    } else {
      int nlo1, nn1, nlo2, nn2;
      next_range(k1min, -k1nmax, lo1 + bi / n2, r.max_side, nlo1, nn1);
      next_range(k2min, -k2nmax, lo2 + bi % n2, r.max_side, nlo2, nn2);
      w[1] = nlo1;
      w[2] = nlo2;
      w[3] = nn1;
      w[4] = nn2;
    }
  }
}

}  // namespace

hipError_t launch_refine_start(const RefineArgs &r, hipStream_t st) {
  hipLaunchKernelGGL(k_refine_start, dim3(r.n_src), dim3(kThreads), 0, st, r);
  return hipGetLastError();
}

hipError_t launch_refine_estimate(const RefineArgs &r, hipStream_t st) {
  hipLaunchKernelGGL(k_refine_estimate, dim3(r.n_src), dim3(kThreads), 0, st, r);
  return hipGetLastError();
}

}  // namespace rlf
