// Device math used by the kernels.
//
// cis2pi_f64: exp(2 pi i phi) in FP64 for phase arguments of thousands of
// turns.  Reduction is exact: r = phi - rint(phi) in [-1/2, 1/2] (the
// difference is a multiple of ulp(phi) no larger than 1/2, so it is
// representable), k = rint(256 r), d = r - k/256 in [-1/512, 1/512] (again
// exact).  exp(2 pi i r) = T[k] * exp(2 pi i d) with T[k] = exp(2 pi i k/256)
// from a 257-entry table in LDS, and exp(i x), |x| <= pi/256 < 0.0123, from
// its Taylor series: cos to x^6 (truncation < x^8/8! < 6e-21) and sin to x^7
// (truncation < x^9/9! < 2e-23).  About 19 VALU operations against ~40 for a
// general-range sincospi.
//
// rsqrt_f64: v_rsq_f64 refined by one second-order step,
// y = y0 (1 + e/2 + 3 e^2 / 8) with e = 1 - x y0^2; arguments here are finite
// and >= 1, so no special-case handling is needed.
#pragma once

#include <hip/hip_runtime.h>

namespace rlf {

constexpr int kCisTable = 256;                  // table steps per turn

// Fill the block's LDS table (257 entries, k = -128..128).  Call from every
// thread of the block, followed by __syncthreads().
__device__ __forceinline__ void cis_table_init(double2 *tab) {
  for (int k = threadIdx.x; k <= kCisTable; k += blockDim.x) {
    double s, c;
    sincospi((double)(k - kCisTable / 2) * (2.0 / kCisTable), &s, &c);
    tab[k] = make_double2(c, s);
  }
}

// (cos 2 pi phi, sin 2 pi phi) with the table above.
__device__ __forceinline__ double2 cis2pi_f64(double phi, const double2 *tab) {
  const double r = phi - rint(phi);
  const double kf = rint(r * (double)kCisTable);
  const double d = fma(kf, -1.0 / kCisTable, r);
  const double x = d * 6.283185307179586476925286766559;   // 2 pi
  const double x2 = x * x;
  // cos x = 1 - x^2/2 + x^4/24 - x^6/720
  const double cx = fma(x2, fma(x2, fma(x2, -1.0 / 720.0, 1.0 / 24.0), -0.5), 1.0);
  // sin x = x (1 - x^2/6 + x^4/120 - x^6/5040)
  const double sx = x * fma(x2, fma(x2, fma(x2, -1.0 / 5040.0, 1.0 / 120.0), -1.0 / 6.0), 1.0);
  const double2 t = tab[(int)kf + kCisTable / 2];
  return make_double2(fma(t.x, cx, -(t.y * sx)), fma(t.x, sx, t.y * cx));
}

__device__ __forceinline__ double rsqrt_f64(double x) {
  const double y0 = __builtin_amdgcn_rsq(x);
  const double e = fma(-x * y0, y0, 1.0);
  return fma(y0 * e, fma(e, 0.375, 0.5), y0);
}

}  // namespace rlf
