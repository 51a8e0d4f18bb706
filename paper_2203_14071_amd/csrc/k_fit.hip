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
// the quadratic form costs 7 ops and serves all knots; per (cell, point,
// knot): 1 FMA, rsqrt, 2 MUL, 1 FMA, 1 MUL + 1 FMA.
//   FP64 form:  v_rsq_f64 + one second-order refinement.
//   Mixed form: FP32 cell data and arithmetic (v_rsq_f32), partial sums of
//               each block of kBlock cells folded into FP64 totals, so the
//               FP32 rounding error grows with kBlock, not with the cell count.
// The epilogue (logs, exps, log-sum-exp over knots) is FP64 in both forms.
#include "rlf_devmath.h"
#include "rlf_internal.h"

namespace rlf {

namespace {

constexpr int kBlock = 32;

__device__ __forceinline__ bool in_window(const int32_t *win, int s, int i1, int i2) {
  if (!win) return true;
  const int4 b = reinterpret_cast<const int4 *>(win)[s];
  return i1 >= b.x && i1 <= b.y && i2 >= b.z && i2 <= b.w;
}

template <int R, bool kExact, bool kMixed>
__global__ __launch_bounds__(256) void k_fit(FitArgs a, int num_r_arg) {
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
  const int64_t c0 = a.offsets[s], c1 = a.offsets[s + 1];
  double D[R], M[R];
#pragma unroll
  for (int k = 0; k < R; ++k) D[k] = M[k] = 0.0;

  if (!kMixed) {
    const double a11 = 1.0 + e1, a12 = e2, a22 = 1.0 - e1;
    double sk[R];
#pragma unroll
    for (int k = 0; k < R; ++k) sk[k] = k < num_r ? a.sk[k] * g : 0.0;
    const double4 *__restrict__ cells = a.fit64;
    for (int64_t c = c0; c < c1; ++c) {
      const double4 cl = cells[c];
      const double ku = fma(a11, cl.x, a12 * cl.y);
      const double kv = fma(a12, cl.x, a22 * cl.y);
      const double q = fma(ku, ku, kv * kv);
#pragma unroll
      for (int k = 0; k < R; ++k) {
        if (k < num_r) {
          const double r = rsqrt_f64(fma(sk[k], q, 1.0));
          const double f = r * r * r;
          D[k] = fma(cl.w, f, D[k]);
          M[k] = fma(cl.z * f, f, M[k]);
        }
      }
    }
  } else {
    const float a11 = (float)(1.0 + e1), a12 = (float)e2, a22 = (float)(1.0 - e1);
    float sk[R];
#pragma unroll
    for (int k = 0; k < R; ++k) sk[k] = k < num_r ? (float)(a.sk[k] * g) : 0.0f;
    const float4 *__restrict__ cells = a.fit32;
    auto block = [&](int64_t cb, int n) {
      float d[R], m[R];
#pragma unroll
      for (int k = 0; k < R; ++k) d[k] = m[k] = 0.0f;
      for (int t = 0; t < n; ++t) {
        const float4 cl = cells[cb + t];
        const float ku = fmaf(a11, cl.x, a12 * cl.y);
        const float kv = fmaf(a12, cl.x, a22 * cl.y);
        const float q = fmaf(ku, ku, kv * kv);
#pragma unroll
        for (int k = 0; k < R; ++k) {
          if (k < num_r) {
            const float r = __builtin_amdgcn_rsqf(fmaf(sk[k], q, 1.0f));
            const float f = r * r * r;
            d[k] = fmaf(cl.w, f, d[k]);
            m[k] = fmaf(cl.z * f, f, m[k]);
          }
        }
      }
#pragma unroll
      for (int k = 0; k < R; ++k) {
        D[k] += (double)d[k];
        M[k] += (double)m[k];
      }
    };
    int64_t cb = c0;
#pragma clang loop unroll(disable)
    for (; cb + kBlock <= c1; cb += kBlock) block(cb, kBlock);
    if (cb < c1) block(cb, (int)(c1 - cb));
  }
  if (c1 == c0) {
    *out = NAN;
    return;
  }
  const double *lw = a.logw + (int64_t)s * a.num_r;
  double L[R];
  double mx = -INFINITY;
#pragma unroll
  for (int k = 0; k < R; ++k) {
    if (k < num_r) {
      L[k] = D[k] * D[k] / (2.0 * M[k]) - 0.5 * log(M[k]);
      mx = fmax(mx, L[k]);
    }
  }
  double acc = 0.0;
#pragma unroll
  for (int k = 0; k < R; ++k)
    if (k < num_r) acc += exp(lw[k] + L[k] - mx);
  *out = mx + log(acc);
}

template <bool kMixed>
hipError_t launch(const FitArgs &a, hipStream_t st) {
  const dim3 grid((a.n_valid + 255) / 256, a.n_src);
  if (a.num_r == 20)
    hipLaunchKernelGGL((k_fit<20, true, kMixed>), grid, dim3(256), 0, st, a, 20);
  else if (a.num_r == 23)
    hipLaunchKernelGGL((k_fit<23, true, kMixed>), grid, dim3(256), 0, st, a, 23);
  else if (a.num_r <= 8)
    hipLaunchKernelGGL((k_fit<8, false, kMixed>), grid, dim3(256), 0, st, a, a.num_r);
  else
    hipLaunchKernelGGL((k_fit<kMaxKnots, false, kMixed>), grid, dim3(256), 0, st, a, a.num_r);
  return hipGetLastError();
}

}  // namespace

hipError_t launch_fit_f64(const FitArgs &a, hipStream_t st) { return launch<false>(a, st); }
hipError_t launch_fit_mixed(const FitArgs &a, hipStream_t st) { return launch<true>(a, st); }

}  // namespace rlf
