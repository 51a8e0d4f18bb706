// Sky-model sums (Sec. 2.2, Eq. 1) at one visibility over a range of
// sources whose records are uniform across the wave (scalar loads), shared
// by the kernels that form or update a residual so that every path adds the
// same terms in the same order.
//   sum_f64:   FP64 phase, exact reduction + table exp (cis2pi_f64), the
//              profile by the corrected rsqrt cube; returns the sum of
//              S exp(2 pi i phi) / x^{3/2} (without the spectral factor).
//   sum_mixed: FP64 phase and fractional part, FP32 sin/cos, profile, sum.
// The flux stays a multiplication: folded into the profile argument (as the
// FP64 extraction does with per-lane sources) the innermost FMA would take
// two wave-uniform scalar operands, which one VOP3 instruction cannot read,
// and the compiler's move to a VGPR costs what the multiplication saved.
#pragma once

#include "rlf_devmath.h"
#include "rlf_internal.h"

namespace rlf {

// T: entries of the exp table tab (1024 or 2048).
template <int T = kCisTable>
__device__ __forceinline__ double2 sum_f64(double u, double v, double w, const SrcModel *__restrict__ src, int b,
                                           int e, const double2 *tab) {
  const double uu = u * u, uv = u * v, vv = v * v;
  double ar = 0.0, ai = 0.0;
  auto term = [&](const SrcModel &p) {
    const double ph = fma(u, p.l, fma(v, p.m, w * p.n1));
    const double2 cs = cis2pi_f64<T>(ph, tab);
    const double x = fma(p.q11, uu, fma(p.q12x2, uv, fma(p.q22, vv, 1.0)));
    const double amp = p.flux * pow_m32_f64(x);             // (2/3) of the term's amplitude
    ar = fma(amp, cs.x, ar);
    ai = fma(amp, cs.y, ai);
  };
  // two source records per step: both scalar loads are in flight together
  struct Two {
    SrcModel p0, p1;
  };
  int s = b;
  for (; s + 1 < e; s += 2) {
    const Two t = *reinterpret_cast<const Two *>(src + s);
    term(t.p0);
    term(t.p1);
  }
  if (s < e) term(src[s]);
  return make_double2(kPowM32Scale * ar, kPowM32Scale * ai);
}

__device__ __forceinline__ float2 sum_mixed(double u, double v, double w, const SrcMixed *__restrict__ src, int b,
                                            int e) {
  const float uf = (float)u, vf = (float)v;
  const float uu = uf * uf, uv = uf * vf, vv = vf * vf;
  float ar = 0.0f, ai = 0.0f;
  auto term = [&](const SrcMixed &p) {
    const double ph = fma(u, p.l, fma(v, p.m, w * p.n1));
    const float t = (float)__builtin_amdgcn_fract(ph);      // turns, in [0, 1]
    const float sn = __builtin_amdgcn_sinf(t), cs = __builtin_amdgcn_cosf(t);
    const float x = fmaf(p.q11, uu, fmaf(p.q12x2, uv, fmaf(p.q22, vv, 1.0f)));
    const float r = __builtin_amdgcn_rsqf(x);
    const float amp = p.flux * (r * r * r);
    ar = fmaf(amp, cs, ar);
    ai = fmaf(amp, sn, ai);
  };
  struct Two {
    SrcMixed p0, p1;
  };
  int s = b;
  for (; s + 1 < e; s += 2) {
    const Two t = *reinterpret_cast<const Two *>(src + s);
    term(t.p0);
    term(t.p1);
  }
  if (s < e) term(src[s]);
  return make_float2(ar, ai);
}

}  // namespace rlf
