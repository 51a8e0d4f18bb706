// Shape estimate (Sec. 2.4, 4.1): per source, the maximum of ln L(e) over
// the evaluated grid points (smallest flat index on ties), the set
// {ln L >= ln Lmax + ln frac}, its likelihood-weighted mean and population
// covariance (weights exp(ln L - ln Lmax)), and the flags: bad variance,
// empty facet, maximum on an edge of the evaluated region.  One block per
// source; three passes over the source's grid values with block reductions.
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

__device__ __forceinline__ bool grid_valid(int i1, int i2, int n_e, int r2) {
  const int c = (n_e - 1) / 2;
  if (i1 < 0 || i2 < 0 || i1 >= n_e || i2 >= n_e) return false;
  return (i1 - c) * (i1 - c) + (i2 - c) * (i2 - c) < r2;
}

__device__ __forceinline__ bool in_box(const int32_t *win, int s, int i1, int i2) {
  if (!win) return true;
  const int4 b = reinterpret_cast<const int4 *>(win)[s];
  return i1 >= b.x && i1 <= b.y && i2 >= b.z && i2 <= b.w;
}

__global__ __launch_bounds__(kThreads) void k_estimate(EstimateArgs a) {
  __shared__ double shd[4];
  __shared__ double shv[4];
  __shared__ int shi[4];
  __shared__ int touch;
  const int s = blockIdx.x;
  if (a.redo && !a.redo[s]) return;
  const double *L = a.lsurf + (int64_t)s * a.n_valid;
  const int64_t n_cells = a.offsets[s + 1] - a.offsets[s];
  const uint32_t extra = a.redo ? (uint32_t)RLF_FLAG_FALLBACK : 0u;
  const int ctr = (a.n_e - 1) / 2;

  if (a.surface) {
    double *S = a.surface + (int64_t)s * a.n_e * a.n_e;
    for (int f = threadIdx.x; f < a.n_e * a.n_e; f += kThreads) {
      const int i1 = f / a.n_e, i2 = f - i1 * a.n_e;
      if (!grid_valid(i1, i2, a.n_e, a.half_r2)) S[f] = -INFINITY;
    }
    for (int j = threadIdx.x; j < a.n_valid; j += kThreads) {
      const int f = a.epts[j];
      const int i1 = f / a.n_e, i2 = f - i1 * a.n_e;
      S[f] = (n_cells > 0 && in_box(a.window, s, i1, i2)) ? L[j] : -INFINITY;
    }
  }

  // pass 1: maximum, smallest index on ties (each thread scans increasing j)
  double best = -INFINITY;
  int bi = 0x7fffffff;
  if (n_cells > 0) {
    for (int j = threadIdx.x; j < a.n_valid; j += kThreads) {
      const double v = L[j];
      if (a.window) {
        const int f = a.epts[j];
        const int i1 = f / a.n_e, i2 = f - i1 * a.n_e;
        if (!in_box(a.window, s, i1, i2)) continue;
      }
      if (v > best) {
        best = v;
        bi = j;
      }
    }
  }
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

  if (!(best > -INFINITY)) {                   // empty facet or nothing evaluated
    if (threadIdx.x == 0) {
      const double nan = NAN;
      if (a.e1) a.e1[s] = nan;
      if (a.e2) a.e2[s] = nan;
      if (a.s1) a.s1[s] = nan;
      if (a.s2) a.s2[s] = nan;
      if (a.c12) a.c12[s] = nan;
      if (a.lmax) a.lmax[s] = nan;
      if (a.argmax) a.argmax[s] = -1;
      if (a.n_above) a.n_above[s] = 0;
      a.flags[s] = (uint32_t)RLF_FLAG_EMPTY | extra;
      // a window holding no valid grid point of a non-empty facet is refitted
      if (a.redo_out) a.redo_out[s] = n_cells > 0 ? 1 : 0;
    }
    return;
  }

  // pass 2: weight, first moments, count over the thresholded set; with a
  // window, also whether any member has a grid neighbour outside the window
  // (the set may continue beyond it: the narrowed result is not trusted) or
  // an evaluated lattice point outside the window reaches the set
  const double thr = best + a.log_frac;
  double sw = 0.0, s1 = 0.0, s2 = 0.0, cnt = 0.0;
  if (threadIdx.x == 0) touch = 0;
  __syncthreads();
  for (int j = threadIdx.x; j < a.n_valid; j += kThreads) {
    const double v = L[j];
    if (v >= thr) {
      const int f = a.epts[j];
      const int i1 = f / a.n_e, i2 = f - i1 * a.n_e;
      if (!in_box(a.window, s, i1, i2)) {
        // a lattice point outside the window reaching the set: refit
        if (a.redo_out && a.check_stride > 0 && (i1 - ctr) % a.check_stride == 0 &&
            (i2 - ctr) % a.check_stride == 0)
          atomicOr(&touch, 1);
        continue;
      }
      if (a.window && a.redo_out) {
        const int nb[4][2] = {{1, 0}, {-1, 0}, {0, 1}, {0, -1}};
        for (int q = 0; q < 4; ++q) {
          const int j1 = i1 + nb[q][0], j2 = i2 + nb[q][1];
          if (grid_valid(j1, j2, a.n_e, a.half_r2) && !in_box(a.window, s, j1, j2)) atomicOr(&touch, 1);
        }
      }
      const double w = exp(v - best);
      const double x1 = (double)(i1 - ctr) * a.e_step, x2 = (double)(i2 - ctr) * a.e_step;
      sw += w;
      s1 += w * x1;
      s2 += w * x2;
      cnt += 1.0;
    }
  }
  sw = block_sum(sw, shd);
  s1 = block_sum(s1, shd);
  s2 = block_sum(s2, shd);
  cnt = block_sum(cnt, shd);
  const double m1 = s1 / sw, m2 = s2 / sw;

  // pass 3: central second moments
  double c11 = 0.0, c22 = 0.0, c12 = 0.0;
  for (int j = threadIdx.x; j < a.n_valid; j += kThreads) {
    const double v = L[j];
    if (v >= thr) {
      const int f = a.epts[j];
      const int i1 = f / a.n_e, i2 = f - i1 * a.n_e;
      if (!in_box(a.window, s, i1, i2)) continue;
      const double w = exp(v - best);
      const double d1 = (double)(i1 - ctr) * a.e_step - m1, d2 = (double)(i2 - ctr) * a.e_step - m2;
      c11 += w * d1 * d1;
      c22 += w * d2 * d2;
      c12 += w * d1 * d2;
    }
  }
  c11 = block_sum(c11, shd) / sw;
  c22 = block_sum(c22, shd) / sw;
  c12 = block_sum(c12, shd) / sw;

  if (threadIdx.x == 0) {
    const double sd1 = sqrt(c11), sd2 = sqrt(c22);
    const double det = c11 * c22 - c12 * c12;
    const double sqd = det > 0.0 ? sqrt(det) : 0.0;
    uint32_t fl = extra;
    if (sd1 <= a.bad_sigma || sd2 <= a.bad_sigma || sqd <= a.bad_sqrtdet) fl |= RLF_FLAG_BAD_VAR;
    const int f = a.epts[bi];
    const int i1 = f / a.n_e, i2 = f - i1 * a.n_e;
    bool edge = i1 == 0 || i2 == 0 || i1 == a.n_e - 1 || i2 == a.n_e - 1;
    bool inner_edge = false;
    const int nb[4][2] = {{1, 0}, {-1, 0}, {0, 1}, {0, -1}};
    for (int q = 0; q < 4; ++q) {
      const int j1 = i1 + nb[q][0], j2 = i2 + nb[q][1];
      const bool gv = grid_valid(j1, j2, a.n_e, a.half_r2);
      const bool inw = in_box(a.window, s, j1, j2);
      if (!(gv && inw)) edge = true;
      if (gv && !inw) inner_edge = true;
    }
    if (edge) fl |= RLF_FLAG_EDGE;
    if (a.e1) a.e1[s] = m1;
    if (a.e2) a.e2[s] = m2;
    if (a.s1) a.s1[s] = sd1;
    if (a.s2) a.s2[s] = sd2;
    if (a.c12) a.c12[s] = c12;
    if (a.lmax) a.lmax[s] = best;
    if (a.argmax) a.argmax[s] = f;
    if (a.n_above) a.n_above[s] = (int32_t)cnt;
    a.flags[s] = fl;
    if (a.redo_out) a.redo_out[s] = (inner_edge || touch) ? 1 : 0;
  }
}

}  // namespace

hipError_t launch_estimate(const EstimateArgs &a, hipStream_t st) {
  hipLaunchKernelGGL(k_estimate, dim3(a.n_src), dim3(kThreads), 0, st, a);
  return hipGetLastError();
}

}  // namespace rlf
