// Sky-model DFT (Sec. 2.2, Eq. 1): every visibility accumulates the model of
// every catalogue source.
//
// One thread per visibility and a uniform loop over sources: the source
// records come in two at a time through scalar loads shared by the wave.  Work per
// (visibility, source) pair:
//   FP64 form:  phase (3 FMA), exp(2 pi i phase) by exact reduction + LDS
//               table + short polynomials (14 ops), profile
//               (3 FMA + corrected rsqrt cube, 5 ops, + 1 MUL), 2 FMA into the
//               sum (the profile's constant 3/2 is applied once at the end);
//   mixed form: phase and its fractional part (v_fract_f64, exact, in
//               [0, 1) turns) in FP64, rounded to FP32 for v_sin/v_cos
//               (argument in turns), profile and sum in FP32.
// Two entry kernels: visibilities in caller order (rlf_model_vis), and the
// residual in the facet object's uv-sorted order (extraction input).  Their
// FP64 forms take a 2048-entry table (32 KB of LDS; sin's x^5 term drops,
// one FMA per pair) in blocks of 512 threads, so that four blocks per CU
// keep eight waves per SIMD in 128 KB of LDS; both form the sky sum with the
// same table, so the two orders give the same residual values.
#include "rlf_devmath.h"
#include "rlf_internal.h"
#include "rlf_sky.h"

namespace rlf {

namespace {

constexpr int kModelTable = 2048;                 // FP64 k_model's table entries

template <bool kMixed>
constexpr int model_threads() { return kMixed ? 256 : 512; }

template <bool kMixed>
__global__ __launch_bounds__(model_threads<kMixed>()) void k_model(ModelArgs a) {
  __shared__ double2 tab[kMixed ? 1 : kModelTable];
  if (!kMixed) {
    cis_table_init<kModelTable>(tab);
    __syncthreads();
  }
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
  const double spec = a.chan->spec[c];
  if (!kMixed) {
    const double2 acc = sum_f64<kModelTable>(u, v, w, a.src, a.s_begin, a.s_end, tab);
    double2 *out = reinterpret_cast<double2 *>(a.out);
    double2 r;
    if (a.mode == 0) {
      r = make_double2(spec * acc.x, spec * acc.y);
    } else if (a.mode == 1) {
      const double2 o = out[i];
      r = make_double2(fma(spec, acc.x, o.x), fma(spec, acc.y, o.y));
    } else {
      const double2 o = reinterpret_cast<const double2 *>(a.vis_in)[i];
      r = make_double2(fma(-spec, acc.x, o.x), fma(-spec, acc.y, o.y));
    }
    out[i] = r;
  } else {
    const float2 acc = sum_mixed(u, v, w, a.src32, a.s_begin, a.s_end);
    const float sp = (float)spec;
    float2 *out = reinterpret_cast<float2 *>(a.out);
    float2 r;
    if (a.mode == 0) {
      r = make_float2(sp * acc.x, sp * acc.y);
    } else if (a.mode == 1) {
      const float2 o = out[i];
      r = make_float2(fmaf(sp, acc.x, o.x), fmaf(sp, acc.y, o.y));
    } else {
      const float2 o = reinterpret_cast<const float2 *>(a.vis_in)[i];
      r = make_float2(fmaf(-sp, acc.x, o.x), fmaf(-sp, acc.y, o.y));
    }
    out[i] = r;
  }
}

// Residual (or a plain gather) into the uv-sorted order, plus the weights;
// the FP64 form stores w R and w spec, the products its extraction uses.
template <bool kMixed>
__global__ __launch_bounds__(model_threads<kMixed>(), kMixed ? 1 : 8) void k_residual_sorted(ResidualArgs a) {
  __shared__ double2 tab[kMixed ? 1 : kModelTable];
  if (!kMixed && a.subtract) {
    cis_table_init<kModelTable>(tab);
    __syncthreads();
  }
  const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= a.sv.n_vis) return;
  const int64_t i = a.sv.order[j];
  const double4 g = a.sv.geo[j];
  // The source loop comes before any store: loads that no store of this
  // kernel can have clobbered stay scalar (one s_load per source per wave).
  const double w = kMixed ? (double)reinterpret_cast<const float *>(a.weight)[i]
                          : reinterpret_cast<const double *>(a.weight)[i];
  const double wpos = w > 0.0 ? w : 0.0;
  if (!kMixed) {
    double2 r = reinterpret_cast<const double2 *>(a.vis)[i];
    if (a.subtract) {
      const double2 acc = sum_f64<kModelTable>(g.x, g.y, g.z, a.src, 0, a.n_src, tab);
      r = make_double2(fma(-g.w, acc.x, r.x), fma(-g.w, acc.y, r.y));
    }
    // FP64 form: the weighted residual, and the weight times the spectral
    // factor in the fourth slot of the quadratic terms
    reinterpret_cast<double2 *>(a.sv.res)[j] = make_double2(wpos * r.x, wpos * r.y);
    reinterpret_cast<double4 *>(a.sv.quad)[j].w = wpos * g.w;
    if (a.rs) a.rs[j] = r;
  } else {
    float2 r = reinterpret_cast<const float2 *>(a.vis)[i];
    if (a.subtract) {
      const float spec = (float)g.w;
      const float2 acc = sum_mixed(g.x, g.y, g.z, a.src32, 0, a.n_src);
      r = make_float2(fmaf(-spec, acc.x, r.x), fmaf(-spec, acc.y, r.y));
    }
    reinterpret_cast<float2 *>(a.sv.res)[j] = r;
  }
  // flagged weights (<= 0 or NaN) are stored as +0: the extraction tests bits
  a.sv.wt[j] = wpos;
}

// Residual kept in sorted order, updated for changed source models: the
// old models' sum is added and the new models' sum subtracted with the
// arithmetic of k_model's accumulate and residual modes, so the result is
// the one those two passes and a gather would give.
template <bool kMixed>
__global__ __launch_bounds__(256) void k_update_sorted(UpdateArgs a) {
  __shared__ double2 tab[kMixed ? 1 : kCisTable];
  if (!kMixed) {
    cis_table_init(tab);
    __syncthreads();
  }
  const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= a.sv.n_vis) return;
  const double4 g = a.sv.geo[j];
  if (!kMixed) {
    const double2 ao = sum_f64(g.x, g.y, g.z, a.old64, 0, a.n_old, tab);
    const double2 an = sum_f64(g.x, g.y, g.z, a.new64, 0, a.n_new, tab);
    double2 r = a.rs[j];
    r = make_double2(fma(g.w, ao.x, r.x), fma(g.w, ao.y, r.y));
    r = make_double2(fma(-g.w, an.x, r.x), fma(-g.w, an.y, r.y));
    a.rs[j] = r;
    const double wpos = a.sv.wt[j];
    reinterpret_cast<double2 *>(a.sv.res)[j] = make_double2(wpos * r.x, wpos * r.y);
  } else {
    const float2 ao = sum_mixed(g.x, g.y, g.z, a.old32, 0, a.n_old);
    const float2 an = sum_mixed(g.x, g.y, g.z, a.new32, 0, a.n_new);
    const float sp = (float)g.w;
    float2 *res = reinterpret_cast<float2 *>(a.sv.res);
    float2 r = res[j];
    r = make_float2(fmaf(sp, ao.x, r.x), fmaf(sp, ao.y, r.y));
    r = make_float2(fmaf(-sp, an.x, r.x), fmaf(-sp, an.y, r.y));
    res[j] = r;
  }
}

}  // namespace

hipError_t launch_update_sorted(const UpdateArgs &a, int mixed, hipStream_t st) {
  const int64_t blocks = (a.sv.n_vis + 255) / 256;
  if (blocks == 0) return hipSuccess;
  if (mixed)
    hipLaunchKernelGGL(k_update_sorted<true>, dim3((unsigned)blocks), dim3(256), 0, st, a);
  else
    hipLaunchKernelGGL(k_update_sorted<false>, dim3((unsigned)blocks), dim3(256), 0, st, a);
  return hipGetLastError();
}

hipError_t launch_model(const ModelArgs &a, int mixed, hipStream_t st) {
  const int64_t n = a.n_rows * a.n_chan;
  if (mixed) {
    constexpr int t = model_threads<true>();
    hipLaunchKernelGGL(k_model<true>, dim3((unsigned)((n + t - 1) / t)), dim3(t), 0, st, a);
  } else {
    constexpr int t = model_threads<false>();
    hipLaunchKernelGGL(k_model<false>, dim3((unsigned)((n + t - 1) / t)), dim3(t), 0, st, a);
  }
  return hipGetLastError();
}

hipError_t launch_residual_sorted(const ResidualArgs &a, int mixed, hipStream_t st) {
  const int64_t n = a.sv.n_vis;
  if (mixed) {
    constexpr int t = model_threads<true>();
    hipLaunchKernelGGL(k_residual_sorted<true>, dim3((unsigned)((n + t - 1) / t)), dim3(t), 0, st, a);
  } else {
    constexpr int t = model_threads<false>();
    hipLaunchKernelGGL(k_residual_sorted<false>, dim3((unsigned)((n + t - 1) / t)), dim3(t), 0, st, a);
  }
  return hipGetLastError();
}

}  // namespace rlf
