// Shape estimate (Sec. 2.4, 4.1): per source, the maximum of ln L(e) over
// the evaluated grid points (smallest flat index on ties), the set
// {ln L >= ln Lmax + ln frac}, its likelihood-weighted mean and population
// covariance (weights exp(ln L - ln Lmax)), and the flags: bad variance,
// empty facet, maximum on an edge of the evaluated region.  One block per
// source; three passes over the source's grid values with block reductions.
//
// The set is cut at a threshold and the maximum is a comparison, so the
// estimate is discontinuous in ln L: a point within the arithmetic error of
// the threshold can go either way.  In the mixed form (ln L summed in FP32,
// error bounded by delta) every point within 2 delta of the threshold or
// below the maximum is evaluated again in FP64 first, so both decisions are
// those of FP64 arithmetic on the same facet; the weights of the other
// points keep their FP32-summed values.
#include "rlf_devmath.h"
#include "rlf_internal.h"

namespace rlf {

namespace {

constexpr int kThreads = 256;
constexpr double kLnPowM32Scale = 0.40546510810816438198;   // ln(3/2)

// ln L(e) of source s at (e1, e2) in FP64, evaluated by one whole wave (all
// 64 lanes, uniform arguments): the lanes split the source's cells, knots in
// groups of four; per knot D and M are summed per lane and then across the
// wave, and ln L(e) = ln sum_k w_k L(e, alpha_k) as in the FP64 fit (the
// same terms, summed in another order).  Every lane returns the same value.
__device__ double loglike_f64_wave(const EstimateArgs &a, int s, double e1, double e2) {
  const int lane = threadIdx.x & 63;
  const double det = 1.0 - e1 * e1 - e2 * e2;
  const double g = 1.0 / (det * det);
  const double a11 = 1.0 + e1, a12 = e2, a22 = 1.0 - e1;
  const int64_t c0 = a.offsets[s], c1 = a.offsets[s + 1];
  const double *lw = a.logw + (int64_t)s * a.num_r;
  double mx = -INFINITY, acc = 0.0;
  for (int k0 = 0; k0 < a.num_r; k0 += 4) {
    double D[4], M[4], sk[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      D[k] = M[k] = 0.0;
      sk[k] = k0 + k < a.num_r ? a.sk[k0 + k] * g : 0.0;
    }
    for (int64_t c = c0 + lane; c < c1; c += 64) {
      const double4 cl = a.fit64[c];
      const double ku = fma(a11, cl.x, a12 * cl.y);
      const double kv = fma(a12, cl.x, a22 * cl.y);
      const double q = fma(ku, ku, kv * kv);
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        const double h = pow_m32_f64(fma(sk[k], q, cl.z));        // (2/3) sqrt(W) f_c
        D[k] = fma(cl.w, h, D[k]);
        M[k] = fma(h, h, M[k]);
      }
    }
#pragma unroll
    for (int k = 0; k < 4; ++k) {
#pragma unroll
      for (int d = 32; d > 0; d >>= 1) {
        D[k] += __shfl_xor(D[k], d);
        M[k] += __shfl_xor(M[k], d);
      }
    }
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      if (k0 + k < a.num_r) {
        // D and M carry (2/3) and (4/9) of their values: ln M is off by -2 ln(3/2)
        const double v = lw[k0 + k] + (D[k] * D[k] / (2.0 * M[k]) - 0.5 * log(M[k]) - kLnPowM32Scale);
        const double nm = fmax(mx, v);
        acc = (mx > -INFINITY ? acc * exp(mx - nm) : 0.0) + exp(v - nm);
        mx = nm;
      }
    }
  }
  return mx + log(acc);
}

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
  double *L = a.lsurf + (int64_t)s * a.n_valid;
  const int64_t n_cells = a.offsets[s + 1] - a.offsets[s];
  const uint32_t extra = a.redo ? (uint32_t)RLF_FLAG_FALLBACK : 0u;
  const int ctr = (a.n_e - 1) / 2;
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;

  // pass 1: maximum, smallest index on ties (each thread scans increasing j)
  double best;
  int bi;
  auto find_max = [&]() {
    best = -INFINITY;
    bi = 0x7fffffff;
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
  };
  find_max();

  // FP64 recheck (mixed form): the points that can decide the maximum or sit
  // at the threshold, each evaluated by a whole wave; the waves own disjoint
  // points, and every read of a point's FP32-summed value precedes its write
  if (a.fit64 && best > -INFINITY) {
    const double delta = a.recheck_rel * (fabs(best) + a.recheck_abs);
    const double lo = best - 2.0 * delta, thr0 = best + a.log_frac;
    const bool lat_out = a.redo_out && a.check_stride > 0;
    for (int j0 = wid * 64; j0 < a.n_valid; j0 += kThreads) {
      const int j = j0 + lane;
      bool cand = false;
      if (j < a.n_valid) {
        const double v = L[j];
        const int f = a.epts[j];
        const int i1 = f / a.n_e, i2 = f - i1 * a.n_e;
        if (in_box(a.window, s, i1, i2))
          cand = v >= lo || fabs(v - thr0) <= 2.0 * delta;
        else if (lat_out && (i1 - ctr) % a.check_stride == 0 && (i2 - ctr) % a.check_stride == 0)
          cand = fabs(v - thr0) <= 2.0 * delta;
      }
      uint64_t m = __ballot(cand);
      while (m) {
        const int b = __ffsll((unsigned long long)m) - 1;
        m &= m - 1;
        const int f = a.epts[j0 + b];
        const int i1 = f / a.n_e, i2 = f - i1 * a.n_e;
        const double v = loglike_f64_wave(a, s, (double)(i1 - ctr) * a.e_step, (double)(i2 - ctr) * a.e_step);
        if (lane == 0) L[j0 + b] = v;
      }
    }
    __threadfence_block();
    __syncthreads();
    find_max();
  }

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
