// Sky-model DFT (Sec. 2.2, Eq. 1): every visibility accumulates the model of
// every catalogue source in [s_begin, s_end).
//
// One thread per visibility; the source loop is uniform across the wave, so
// the 64-byte source record comes in through one scalar load and feeds all
// 64 lanes from SGPRs.  The work per (visibility, source) pair is the FP64
// phase (3 FMA), sincospi of that phase, the quadratic form of the sheared
// profile (3 FMA), x^{-3/2} through rsqrt, and two FMAs into the sum.
#include "rlf_internal.h"

namespace rlf {

namespace {

__device__ __forceinline__ double shape_factor(double x) {
  const double r = rsqrt(x);
  return r * r * r;
}

__global__ __launch_bounds__(256) void k_model_f64(ModelArgs a) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t n_vis = a.n_rows * a.n_chan;
  if (i >= n_vis) return;
  int64_t row = i;
  int c = 0;
  if (a.n_chan > 1) {
    row = i / a.n_chan;
    c = (int)(i - row * a.n_chan);
  }
  const double sc = a.chan->scale[c];
  const double u = __dmul_rn(a.u_m[row], sc);
  const double v = __dmul_rn(a.v_m[row], sc);
  const double w = __dmul_rn(a.w_m[row], sc);
  const double uu = u * u, uv = u * v, vv = v * v;
  double acc_r = 0.0, acc_i = 0.0;
  const SrcModel *__restrict__ src = a.src;
  for (int s = a.s_begin; s < a.s_end; ++s) {
    const SrcModel p = src[s];
    const double ph = fma(u, p.l, fma(v, p.m, w * p.n1));
    double sn, cs;
    sincospi(ph + ph, &sn, &cs);
    const double x = fma(p.q11, uu, fma(p.q12x2, uv, fma(p.q22, vv, 1.0)));
    const double amp = p.flux * shape_factor(x);
    acc_r = fma(amp, cs, acc_r);
    acc_i = fma(amp, sn, acc_i);
  }
  const double spec = a.chan->spec[c];
  double2 *out = reinterpret_cast<double2 *>(a.out);
  double2 r;
  if (a.mode == 0) {
    r = make_double2(spec * acc_r, spec * acc_i);
  } else if (a.mode == 1) {
    const double2 o = out[i];
    r = make_double2(fma(spec, acc_r, o.x), fma(spec, acc_i, o.y));
  } else {
    const double2 o = reinterpret_cast<const double2 *>(a.vis_in)[i];
    r = make_double2(fma(-spec, acc_r, o.x), fma(-spec, acc_i, o.y));
  }
  out[i] = r;
}

}  // namespace

hipError_t launch_model_f64(const ModelArgs &a, hipStream_t st) {
  const int64_t n = a.n_rows * a.n_chan;
  const int64_t blocks = (n + 255) / 256;
  hipLaunchKernelGGL(k_model_f64, dim3((unsigned)blocks), dim3(256), 0, st, a);
  return hipGetLastError();
}

}  // namespace rlf
