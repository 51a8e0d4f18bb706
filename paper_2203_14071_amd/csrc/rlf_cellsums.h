// Per-grid-point sums of the likelihood (Sec. 2.4) over a range of facet
// cells, for KP scale-length knots held in registers:
//   D_k += W Re(Vbar) f,  M_k += W f^2,  f = (1 + s_k q)^{-3/2},  q = |A^{-T} k_c|^2.
// The cell records carry sqrt(W) in the profile's scale: a record is
// (u', v', c, b) = (W^{-1/6} uc, W^{-1/6} vc, W^{-1/3}, sqrt(W) Re Vbar), and
// with q' = |A^{-T} (u', v')|^2 = c q the term h = (c + s_k q')^{-3/2} equals
// sqrt(W) f, so D_k += b h and M_k += h h (two FMAs per knot, where W f f
// needs a multiplication more).
// The cells are wave-uniform (one scalar load per cell, shared by the wave);
// each lane is one ellipticity grid point.  Shared by the likelihood kernels
// and by the issue-rate probe that measures these loops on their own.
//   cell_sums_f64: FP64 records, h as (2/3) sqrt(W) f_c from the corrected
//                  v_rsq_f64 cube (pow_m32_f64).
//   cell_sums_f32: FP32 records and arithmetic (v_rsq_f32 cubed); the sums of
//                  each block of kCellBlock cells are formed in FP32 and then
//                  added into the FP64 totals, so the FP32 rounding error
//                  grows with the block length, not with the cell count.
#pragma once

#include "rlf_devmath.h"

namespace rlf {

constexpr int kCellBlock = 32;

// The first n_use of the KP knots are summed; s_k in sk[], which the caller
// may hold wave-uniform.
template <int KP>
__device__ __forceinline__ void cell_sums_f64(const double4 *__restrict__ cells, int64_t cb, int64_t ce, double a11,
                                              double a12, double a22, const double *sk, int n_use, double *D,
                                              double *M) {
  for (int64_t c = cb; c < ce; ++c) {
    const double4 cl = cells[c];
    const double ku = fma(a11, cl.x, a12 * cl.y);
    const double kv = fma(a12, cl.x, a22 * cl.y);
    const double q = fma(ku, ku, kv * kv);
#pragma unroll
    for (int k = 0; k < KP; ++k) {
      if (k < n_use) {
        const double h = pow_m32_f64(fma(sk[k], q, cl.z));          // (2/3) sqrt(W) f_c
        D[k] = fma(cl.w, h, D[k]);
        M[k] = fma(h, h, M[k]);
      }
    }
  }
}

template <int KP>
__device__ __forceinline__ void cell_sums_f32(const float4 *__restrict__ cells, int64_t cb, int64_t ce, float a11,
                                              float a12, float a22, const float *sk, int n_use, double *D,
                                              double *M) {
  auto block = [&](int64_t b, int n) {
    float d[KP], m[KP];
#pragma unroll
    for (int k = 0; k < KP; ++k) d[k] = m[k] = 0.0f;
    for (int t = 0; t < n; ++t) {
      const float4 cl = cells[b + t];
      const float ku = fmaf(a11, cl.x, a12 * cl.y);
      const float kv = fmaf(a12, cl.x, a22 * cl.y);
      const float q = fmaf(ku, ku, kv * kv);
#pragma unroll
      for (int k = 0; k < KP; ++k) {
        if (k < n_use) {
          const float r = __builtin_amdgcn_rsqf(fmaf(sk[k], q, cl.z));
          const float h = r * r * r;                                  // sqrt(W) f_c
          d[k] = fmaf(cl.w, h, d[k]);
          m[k] = fmaf(h, h, m[k]);
        }
      }
    }
#pragma unroll
    for (int k = 0; k < KP; ++k) {
      D[k] += (double)d[k];
      M[k] += (double)m[k];
    }
  };
  int64_t c = cb;
#pragma clang loop unroll(disable)
  for (; c + kCellBlock <= ce; c += kCellBlock) block(c, kCellBlock);
  if (c < ce) block(c, (int)(ce - c));
}

}  // namespace rlf
