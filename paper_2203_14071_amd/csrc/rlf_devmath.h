// Device math used by the kernels.
//
// cis2pi_f64: exp(2 pi i phi) in FP64 for phase arguments of thousands of
// turns.  Reduction is exact: m = phi + 1.5 * 2^42 rounds phi to the
// nearest multiple k / 1024 of 1/1024 turn (ties to even) for
// |phi| < 2^41, k / 1024 = m - 1.5 * 2^42 and d = phi - k / 1024 in
// [-1/2048, 1/2048] are exact, and k mod 1024 is the low ten bits of m's
// mantissa.  Then exp(2 pi i phi) = T[k mod 1024] * exp(i x), x = 2 pi d,
// with T[j] = exp(2 pi i j / 1024) from a 1024-entry table in LDS (16 KB),
// and exp(i x), x = 2 pi d, |x| <= pi/1024 < 3.1e-3, from its Taylor series
// written in powers of d (the factors of 2 pi folded into the
// coefficients): cos to x^4 (truncation < x^6/6! < 1.2e-18) and sin to x^5
// (truncation < x^7/7! < 4.3e-22).  Fifteen VALU operations (two of them
// form the table index) and one LDS read; the index is in range whatever
// phi is.
//
// pow_m32_f64: (2/3) x^(-3/2) for x >= 1 from v_rsq_f64 (relative error
// ~2^-24) with one correction: with y = rsq(x), x^(-3/2) = y^3 (1 + 3e/2 +
// O(e^2)) where e = 1 - x y^2, and y^3 (1 + 3e/2) = (3/2) y^3 (5/3 - x y^2).
// The returned y^3 (5/3 - x y^2) has relative error ~ (15/8) e^2 < 3e-14;
// five VALU operations.  The constant 2/3 is left to the callers (it
// multiplies every profile value: a flux scale, or a constant offset of the
// log-likelihood).
#pragma once

#include <hip/hip_runtime.h>

namespace rlf {

constexpr int kCisTable = 1024;                 // table steps per turn (the default table)

// Fill the block's LDS table (T entries, T a power of two).  Call from every
// thread of the block, followed by __syncthreads().
template <int T = kCisTable>
__device__ __forceinline__ void cis_table_init(double2 *tab) {
  for (int k = threadIdx.x; k < T; k += blockDim.x) {
    double s, c;
    sincospi((double)k * (2.0 / T), &s, &c);
    tab[k] = make_double2(c, s);
  }
}

// 1.5 * 2^52 / T: adding it rounds phi to a multiple of 1/T turn
template <int T>
constexpr double turn_magic() { return 1.5 * 4503599627370496.0 / T; }
constexpr double kTurnMagic = turn_magic<kCisTable>();

// Taylor coefficients of cos(2 pi d) and sin(2 pi d) in powers of d (turns):
// -(2 pi)^2 / 2, (2 pi)^4 / 24; 2 pi, -(2 pi)^3 / 6, (2 pi)^5 / 120.
constexpr double kCos2 = -19.739208802178716, kCos4 = 64.9393940226683;
constexpr double kSin1 = 6.283185307179586, kSin3 = -41.34170224039976, kSin5 = 81.60524927607506;

// a * b + c as one VOP3 FMA with the addend c from an SGPR.  For an FMA
// whose multiplier and addend are both constants the compiler keeps one of
// them in a VGPR and copies it into the destination every time (a
// two-address FMA); here the multiplier constant stays in a VGPR and the
// addend is read as a scalar operand, one instruction instead of two.
__device__ __forceinline__ double fma_vvs(double a, double b, double c) {
  double r;
  asm("v_fma_f64 %0, %1, %2, %3" : "=v"(r) : "v"(a), "v"(b), "s"(c));
  return r;
}

// (cos 2 pi phi, sin 2 pi phi) with a T-entry table.  T = 1024: |x| <= pi/1024
// as described above.  T = 2048: |x| <= pi/2048 < 1.54e-3, and sin's x^5
// term (< 7.2e-17) is dropped: sin to x^3 (truncation < x^5/5! < 7.2e-17,
// below half an ulp of 1), cos to x^4 as before; fourteen VALU operations.
template <int T = kCisTable>
__device__ __forceinline__ double2 cis2pi_f64(double phi, const double2 *tab) {
  static_assert(T == 1024 || T == 2048, "table sizes with a derived truncation bound");
  constexpr double magic = turn_magic<T>();
  const double m = phi + magic;
  const double d = phi - (m - magic);            // turns, |d| <= 1/(2T)
  const double d2 = d * d;
  const double cx = fma(d2, fma_vvs(d2, kCos4, kCos2), 1.0);
  double sx;
  if constexpr (T == 1024)
    sx = d * fma_vvs(d2, fma_vvs(d2, kSin5, kSin3), kSin1);
  else
    sx = d * fma_vvs(d2, kSin3, kSin1);
  const double2 tv = tab[(uint32_t)__double2loint(m) & (uint32_t)(T - 1)];
  return make_double2(fma(tv.x, cx, -(tv.y * sx)), fma(tv.x, sx, tv.y * cx));
}

// (2/3) x^(-3/2), x >= 1 and finite.
__device__ __forceinline__ double pow_m32_f64(double x) {
  const double y = __builtin_amdgcn_rsq(x);
  const double y2 = y * y;
  const double h = fma(-x, y2, 5.0 / 3.0);
  return (y2 * y) * h;
}

constexpr double kPowM32Scale = 1.5;              // x^(-3/2) = kPowM32Scale * pow_m32_f64(x)

}  // namespace rlf
