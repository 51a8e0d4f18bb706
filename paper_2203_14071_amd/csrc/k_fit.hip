// Likelihood grid (Sec. 2.4): for each source, ellipticity grid point e and
// scale-length knot alpha_k,
//   f_c = (1 + s_k q_c(e))^{-3/2},  q_c(e) = |A_e^{-T} k_c|^2,  s_k = 4 pi^2 alpha_k^2,
//   D_k = sum_c W_c f_c Re Vbar_c,  M_k = sum_c W_c f_c^2,
//   ln L(e, alpha_k) = D_k^2 / (2 M_k) - ln(M_k) / 2            (flux marginalised)
//   ln L(e) = m + ln sum_k exp(ln w_k + ln L(e, alpha_k) - m)   (scale marginalised)
//
// One thread per grid point, all knots of that point in registers (D_k, M_k),
// a uniform loop over the source's cells: each cell (uc, vc, W, W Re Vbar)
// comes in through one scalar load shared by the wave.  Per (cell, point)
// the quadratic form costs 7 ops and is reused by all knots; per
// (cell, point, knot) the work is 1 FMA, rsqrt, 2 MUL, 3 FMA/MUL.
#include "rlf_internal.h"

namespace rlf {

namespace {

__device__ __forceinline__ bool in_window(const int32_t *win, int s, int i1, int i2) {
  if (!win) return true;
  const int4 b = reinterpret_cast<const int4 *>(win)[s];
  return i1 >= b.x && i1 <= b.y && i2 >= b.z && i2 <= b.w;
}

template <int R, bool kExact>
__global__ __launch_bounds__(256) void k_fit_f64(FitArgs a, int num_r_arg) {
  const int num_r = kExact ? R : num_r_arg;
  const int s = blockIdx.y;
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= a.n_valid) return;
  double *out = a.lsurf + (int64_t)s * a.n_valid + j;
  if (a.redo && !a.redo[s]) return;
  const int idx = a.epts[j];
  const int i1 = idx / a.n_e, i2 = idx - (idx / a.n_e) * a.n_e;
  const int ctr = (a.n_e - 1) / 2;
  if (!in_window(a.window, s, i1, i2)) {
    *out = -INFINITY;
    return;
  }
  const double e1 = (double)(i1 - ctr) * a.e_step;
  const double e2 = (double)(i2 - ctr) * a.e_step;
  const double det = 1.0 - e1 * e1 - e2 * e2;
  const double g = 1.0 / (det * det);
  const double a11 = 1.0 + e1, a12 = e2, a22 = 1.0 - e1;

  double sk[R];
#pragma unroll
  for (int k = 0; k < R; ++k) sk[k] = k < num_r ? a.sk[k] * g : 0.0;
  double D[R], M[R];
#pragma unroll
  for (int k = 0; k < R; ++k) D[k] = M[k] = 0.0;

  const int64_t c0 = a.offsets[s], c1 = a.offsets[s + 1];
  const double4 *__restrict__ cells = a.fit64;
  for (int64_t c = c0; c < c1; ++c) {
    const double4 cl = cells[c];
    const double ku = fma(a11, cl.x, a12 * cl.y);
    const double kv = fma(a12, cl.x, a22 * cl.y);
    const double q = fma(ku, ku, kv * kv);
#pragma unroll
    for (int k = 0; k < R; ++k) {
      if (k < num_r) {
        const double x = fma(sk[k], q, 1.0);
        const double r = rsqrt(x);
        const double f = r * r * r;
        D[k] = fma(cl.w, f, D[k]);
        M[k] = fma(cl.z * f, f, M[k]);
      }
    }
  }
  if (c1 == c0) {
    *out = NAN;
    return;
  }
  const double *lw = a.logw + (int64_t)s * a.num_r;
  double L[R];
  double m = -INFINITY;
#pragma unroll
  for (int k = 0; k < R; ++k) {
    if (k < num_r) {
      L[k] = D[k] * D[k] / (2.0 * M[k]) - 0.5 * log(M[k]);
      m = fmax(m, L[k]);
    }
  }
  double acc = 0.0;
#pragma unroll
  for (int k = 0; k < R; ++k)
    if (k < num_r) acc += exp(lw[k] + L[k] - m);
  *out = m + log(acc);
}

}  // namespace

hipError_t launch_fit_f64(const FitArgs &a, hipStream_t st) {
  const dim3 grid((a.n_valid + 255) / 256, a.n_src);
  if (a.num_r == 20)
    hipLaunchKernelGGL((k_fit_f64<20, true>), grid, dim3(256), 0, st, a, 20);
  else if (a.num_r == 23)
    hipLaunchKernelGGL((k_fit_f64<23, true>), grid, dim3(256), 0, st, a, 23);
  else if (a.num_r <= 8)
    hipLaunchKernelGGL((k_fit_f64<8, false>), grid, dim3(256), 0, st, a, a.num_r);
  else
    hipLaunchKernelGGL((k_fit_f64<kMaxKnots, false>), grid, dim3(256), 0, st, a, a.num_r);
  return hipGetLastError();
}

}  // namespace rlf
